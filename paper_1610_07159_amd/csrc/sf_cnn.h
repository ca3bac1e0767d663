// Internal interface of the learned coarse-level initialiser (sf_cnn.hip).
#pragma once

#include <hip/hip_runtime.h>

#define SF_CNN_LAYERS 6
#define SF_CNN_INPUT_LEVEL 4  // the network sees the 1/16-resolution level
#define SF_CNN_CHUNK 1024     // pixels per weight-gradient partial sum

// Channel counts and offsets of every layer: in the flat parameter vector
// (per layer the weights (c_out, c_in, ky, kx) then the biases), in the
// device weight buffers (bf16 [coutp][9][cinp], padded to 16 channels) and
// in the device bias buffer (float [coutp]).
struct CnnLayout {
    int cin[SF_CNN_LAYERS], cout[SF_CNN_LAYERS];
    int cinp[SF_CNN_LAYERS], coutp[SF_CNN_LAYERS];
    int flat_off[SF_CNN_LAYERS], w_off[SF_CNN_LAYERS], b_off[SF_CNN_LAYERS];
    int n_params, dev_w_total, dev_b_total;
};

// Device weights: forward layout, flipped transpose for the input
// gradient, biases.
struct CnnWeights {
    unsigned short *wf;
    unsigned short *wd;
    float *bias;
};

CnnLayout cnn_layout();
int cnn_chunks(long P);
int cnn_l1_blocks(long P);
void launch_cnn_pack(hipStream_t st, const CnnLayout &L, const float *flat, unsigned short *wf,
                     unsigned short *wd, float *bias);
void launch_cnn_input(hipStream_t st, const float *src, long img_stride, long batch_stride,
                      unsigned short *x, int B, int H, int W);
void launch_cnn_input_tex(hipStream_t st, const float4 *tex, unsigned short *x, int N);
void launch_cnn_forward(hipStream_t st, const CnnLayout &L, const CnnWeights &wts,
                        const unsigned short *x, unsigned short *const acts[SF_CNN_LAYERS - 1],
                        float *out, int B, int H, int W);
void launch_cnn_backward(hipStream_t st, const CnnLayout &L, const CnnWeights &wts,
                         const unsigned short *x, unsigned short *const acts[SF_CNN_LAYERS - 1],
                         unsigned short *dout, unsigned short *const dpre[SF_CNN_LAYERS - 1],
                         float *wpart, float *bpart, float *grad, int B, int H, int W);
void launch_cnn_l1(hipStream_t st, const float *out, const float *tgt, unsigned short *dout,
                   float *part, int B, int H, int W);
void launch_cnn_adam(hipStream_t st, float *w, float *m, float *v, const float *g, int n,
                     float lr, float beta1, float beta2, float eps, float c1, float c2);
