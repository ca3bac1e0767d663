// gfx950 kernels of the learned coarse-level initialiser: a six-layer 3x3
// convolutional network (4 -> 32 -> 32 -> 32 -> 32 -> 32 -> 6 channels,
// ReLU after the first five) that predicts the coarsest-level flows from the
// 1/16-resolution images (the smarter initialisation the paper's Sec. 7
// names as future work), trained with an L1 loss and Adam.
//
// Tensors are NHWC bfloat16 with the channel count padded to a multiple of
// 16 (input 4 -> 16, output 6 -> 16); accumulation is float32 on the matrix
// cores with gfx950's 16 x 16 x 32 bf16 product (v_mfma_f32_16x16x32_bf16,
// eight K values per lane).  Every convolution is an implicit GEMM: a
// wavefront owns 16 consecutive pixels of one image row (the M rows of the
// tile) and all output channels (N), and runs K over the 9 taps times the
// input channels (32 channels: one tap per product; 16 channels: two taps
// per product), with the layer's weights staged in LDS once per workgroup.
// The weight gradient is a GEMM over pixels (32 per product) split into
// fixed chunks whose partial sums are reduced in a fixed order.
#include <math.h>

#include "sf_cnn.h"

namespace {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
    // round to nearest even (inputs are finite)
    const unsigned u = __builtin_bit_cast(unsigned, f);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
    return __builtin_bit_cast(float, (unsigned)h << 16);
}

// MFMA 16x16x32 operand layouts (lane l, r = l % 16, q = l / 16):
//   A (16 x 32, rows x k): row r, k = 8q .. 8q + 7
//   B (32 x 16, k x cols): col r, k = 8q .. 8q + 7
//   D (16 x 16):           col r, rows 4q .. 4q + 3
__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

__device__ __forceinline__ v8s load8(const unsigned short *p) {
    return *reinterpret_cast<const v8s *>(p);
}

enum { CONV_RELU = 0, CONV_LINEAR = 1, CONV_DGRAD = 2 };

// One 3x3 convolution over B images of H x W.  in: NHWC bf16 with CIN
// channels; wt: bf16 [COUT][9][CIN] (tap = 3 ky + kx); bias: float [COUT]
// (CONV_RELU, CONV_LINEAR).  Outputs:
//   CONV_RELU    out_bf NHWC COUT: bf16(max(acc + bias, 0))
//   CONV_LINEAR  out_f [B][n_out][H][W] float: acc + bias, channels < n_out
//   CONV_DGRAD   out_bf NHWC COUT: bf16(acc) where mask (NHWC COUT) > 0,
//                else 0 (the gradient through the ReLU of the layer below)
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(const unsigned short *__restrict__ in,
                                              const unsigned short *__restrict__ wt,
                                              const float *__restrict__ bias,
                                              const unsigned short *__restrict__ mask,
                                              unsigned short *__restrict__ out_bf,
                                              float *__restrict__ out_f, int n_out, int B,
                                              int H, int W) {
    static_assert(CIN == 16 || CIN == 32, "input channels");
    constexpr int NB = COUT / 16;
    constexpr int NW = COUT * 9 * CIN;  // weights of the layer
    __shared__ __attribute__((aligned(16))) unsigned short wl[NW];
    for (int e = threadIdx.x * 8; e < NW; e += 256 * 8)
        *reinterpret_cast<v8s *>(wl + e) = load8(wt + e);
    __syncthreads();
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int xs = (W + 15) / 16;
    const int seg = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (seg >= B * H * xs) return;  // uniform per wavefront, after the barrier
    const int b = seg / (H * xs), rem = seg % (H * xs);
    const int y = rem / xs, x0 = (rem % xs) * 16;
    const int px = x0 + r;
    v4f acc[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
    // K step: 32 channels of one tap, or 16 channels of two taps (lanes
    // q = 0, 1 the even tap, q = 2, 3 the odd one; the tenth tap is zero)
    constexpr int STEPS = CIN == 32 ? 9 : 5;
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        const int tap = CIN == 32 ? s : 2 * s + (q >> 1);
        const int ch = CIN == 32 ? 8 * q : 8 * (q & 1);
        const int yy = y + tap / 3 - 1, xx = px + tap % 3 - 1;
        const bool ok = tap < 9 && px < W && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const unsigned short *src = in + ((long)(b * H + (ok ? yy : 0)) * W + (ok ? xx : 0)) * CIN;
        const v8s a = ok ? load8(src + ch) : v8s{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const v8s w = tap < 9 ? *reinterpret_cast<const v8s *>(
                                        wl + ((n * 16 + r) * 9 + tap) * CIN + ch)
                                  : v8s{0, 0, 0, 0, 0, 0, 0, 0};
            acc[n] = mfma32(a, w, acc[n]);
        }
    }
#pragma unroll
    for (int n = 0; n < NB; ++n) {
        const int co = n * 16 + r;
        const float bv = MODE == CONV_DGRAD ? 0.f : bias[co];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int xo = x0 + 4 * q + i;
            if (xo >= W) continue;
            const long p = (long)(b * H + y) * W + xo;
            const float v = acc[n][i] + bv;
            if (MODE == CONV_RELU) {
                out_bf[p * COUT + co] = f2bf(fmaxf(v, 0.f));
            } else if (MODE == CONV_LINEAR) {
                if (co < n_out) out_f[((long)(b * n_out + co) * H + y) * W + xo] = v;
            } else {
                out_bf[p * COUT + co] = bf2f(mask[p * COUT + co]) > 0.f ? f2bf(v) : (unsigned short)0;
            }
        }
    }
}

// Weight-gradient partials of one layer: for pixel chunk c, output-channel
// block m, tap and input-channel block n, the 16 x 16 tile
//   sum over the chunk's pixels p of dpre[p][co] x[p + off(tap)][ci].
// part: [chunks][COUT][9][CIN] float.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(const unsigned short *__restrict__ dpre,
                                               const unsigned short *__restrict__ x,
                                               float *__restrict__ part, int B, int H, int W,
                                               int chunk) {
    constexpr int MB = COUT / 16, NBK = CIN / 16, TILES = MB * 9 * NBK;
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const long P = (long)B * H * W;
    const int nchunks = (int)((P + chunk - 1) / chunk);
    if (w >= nchunks * TILES) return;  // uniform per wavefront
    const int c = w / TILES, t = w % TILES;
    const int mb = t / (9 * NBK), tap = (t / NBK) % 9, nb = t % NBK;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int co = mb * 16 + r, ci = nb * 16 + r;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const long p_end = min(P, (long)(c + 1) * chunk);
    for (long p0 = (long)c * chunk; p0 < p_end; p0 += 32) {
        v8s a, bv;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const long p = p0 + 8 * q + i;
            short av = 0, xv = 0;
            if (p < p_end) {
                av = (short)dpre[p * COUT + co];
                const int b = (int)(p / ((long)H * W));
                const int rem = (int)(p % ((long)H * W));
                const int yy = rem / W + dy, xx = rem % W + dx;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    xv = (short)x[((long)(b * H + yy) * W + xx) * CIN + ci];
            }
            a[i] = av;
            bv[i] = xv;
        }
        acc = mfma32(a, bv, acc);
    }
    // D rows = output channels mb*16 + 4q + i, column = input channel ci
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = mb * 16 + 4 * q + i;
        part[(((long)c * COUT + o) * 9 + tap) * CIN + ci] = acc[i];
    }
}

// Bias-gradient partials: part[c][co] = sum over chunk c of dpre[p][co].
template <int COUT>
__global__ __launch_bounds__(256) void k_bgrad(const unsigned short *__restrict__ dpre,
                                               float *__restrict__ part, long P, int chunk) {
    const int c = blockIdx.x;
    const int co = threadIdx.x % COUT, sub = threadIdx.x / COUT;
    constexpr int SUBS = 256 / COUT;
    __shared__ float red[256];
    float acc = 0.f;
    const long p_end = min(P, (long)(c + 1) * chunk);
    for (long p = (long)c * chunk + sub; p < p_end; p += SUBS) acc += bf2f(dpre[p * COUT + co]);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (sub == 0) {
        float s = 0.f;
        for (int k = 0; k < SUBS; ++k) s += red[k * COUT + co];
        part[(long)c * COUT + co] = s;
    }
}

// Sums the chunk partials in chunk order into the flat gradient vector
// (layout of sf_cnn.h: per layer the weights (c_out, c_in, ky, kx) of the
// real channels, then the biases).
__global__ __launch_bounds__(256) void k_grad_reduce(const float *__restrict__ wpart,
                                                     const float *__restrict__ bpart,
                                                     float *__restrict__ grad, int nchunks,
                                                     int cin, int cout, int cinp, int coutp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * 9;
    if (k >= nw + cout) return;
    double s = 0.0;
    if (k < nw) {
        const int co = k / (cin * 9), ci = (k / 9) % cin, tap = k % 9;
        for (int c = 0; c < nchunks; ++c)
            s += (double)wpart[(((long)c * coutp + co) * 9 + tap) * cinp + ci];
    } else {
        const int co = k - nw;
        for (int c = 0; c < nchunks; ++c) s += (double)bpart[(long)c * coutp + co];
    }
    grad[k] = (float)s;
}

// Network input: bf16(I - 0.5) in channels 0..3, zero in 4..15.
// src: [B][4][H][W] float (stride between images of one sample: img_stride).
__global__ __launch_bounds__(256) void k_input(const float *__restrict__ src, long img_stride,
                                               long batch_stride, unsigned short *__restrict__ x,
                                               int B, int H, int W) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long)B * H * W) return;
    const int b = (int)(p / ((long)H * W));
    const long hw = p % ((long)H * W);
    unsigned short v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = f2bf(src[b * batch_stride + c * img_stride + hw] - 0.5f);
    uint4 *o = reinterpret_cast<uint4 *>(x + p * 16);
    const unsigned *u = reinterpret_cast<const unsigned *>(v);
    o[0] = make_uint4(u[0], u[1], u[2], u[3]);
    o[1] = make_uint4(u[4], u[5], u[6], u[7]);
}

// The same from the solver's level texture (float4 (I, Gx, Gy, 0) per
// pixel, four images of N pixels).
__global__ __launch_bounds__(256) void k_input_tex(const float4 *__restrict__ tex,
                                                   unsigned short *__restrict__ x, int N) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    unsigned short v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = f2bf(tex[(long)c * N + p].x - 0.5f);
    uint4 *o = reinterpret_cast<uint4 *>(x + (long)p * 16);
    const unsigned *u = reinterpret_cast<const unsigned *>(v);
    o[0] = make_uint4(u[0], u[1], u[2], u[3]);
    o[1] = make_uint4(u[4], u[5], u[6], u[7]);
}

// L1 loss: per-workgroup partial sums of |out - target| and the gradient
// bf16(sign(out - target) / count) into NHWC with 16 channels (6 real).
__global__ __launch_bounds__(256) void k_l1(const float *__restrict__ out,
                                            const float *__restrict__ tgt,
                                            unsigned short *__restrict__ dout,
                                            float *__restrict__ part, int B, int H, int W) {
    __shared__ float red[256];
    const long P = (long)B * H * W;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const float inv = 1.f / (float)(P * 6);
    float acc = 0.f;
    if (p < P) {
        const int b = (int)(p / ((long)H * W));
        const long hw = p % ((long)H * W);
        unsigned short v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const long k = ((long)b * 6 + c) * H * W + hw;
            const float d = out[k] - tgt[k];
            acc += fabsf(d);
            v[c] = f2bf(d > 0.f ? inv : (d < 0.f ? -inv : 0.f));
        }
        uint4 *o = reinterpret_cast<uint4 *>(dout + p * 16);
        const unsigned *u = reinterpret_cast<const unsigned *>(v);
        o[0] = make_uint4(u[0], u[1], u[2], u[3]);
        o[1] = make_uint4(u[4], u[5], u[6], u[7]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam (Kingma and Ba, 2015, Algorithm 1) on the flat float32 master
// weights; step t counted from 1; bias corrections in double on the host.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, float *__restrict__ m,
                                              float *__restrict__ v, const float *__restrict__ g,
                                              int n, float lr, float beta1, float beta2,
                                              float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = beta1 * m[k] + (1.f - beta1) * gk;
    const float vk = beta2 * v[k] + (1.f - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Device weights of all layers from the flat float vector: bf16 [coutp][9]
// [cinp] for the forward pass, the flipped transpose bf16 [cinp][9][coutp]
// for the input gradient, and float biases (padding zero).
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ flat, CnnLayout L,
                                              unsigned short *__restrict__ wf,
                                              unsigned short *__restrict__ wd,
                                              float *__restrict__ bias) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L.dev_w_total + L.dev_b_total) return;
    if (k >= L.dev_w_total) {
        const int j = k - L.dev_w_total;
        int l = 0;
        while (l + 1 < SF_CNN_LAYERS && j >= L.b_off[l + 1]) ++l;
        const int co = j - L.b_off[l];
        bias[j] = co < L.cout[l] ? flat[L.flat_off[l] + L.cout[l] * L.cin[l] * 9 + co] : 0.f;
        return;
    }
    int l = 0;
    while (l + 1 < SF_CNN_LAYERS && k >= L.w_off[l + 1]) ++l;
    const int j = k - L.w_off[l];
    const int cinp = L.cinp[l], coutp = L.coutp[l];
    const int co = j / (9 * cinp), tap = (j / cinp) % 9, ci = j % cinp;
    float val = 0.f;
    if (co < L.cout[l] && ci < L.cin[l])
        val = flat[L.flat_off[l] + (co * L.cin[l] + ci) * 9 + tap];
    const unsigned short h = f2bf(val);
    wf[k] = h;
    // flipped transpose: [ci][8 - tap][co]
    wd[L.w_off[l] + ((long)ci * 9 + (8 - tap)) * coutp + co] = h;
}

}  // namespace

// ---- launchers ----------------------------------------------------------------

CnnLayout cnn_layout() {
    CnnLayout L;
    const int cin[SF_CNN_LAYERS] = {4, 32, 32, 32, 32, 32};
    const int cout[SF_CNN_LAYERS] = {32, 32, 32, 32, 32, 6};
    int fo = 0, wo = 0, bo = 0;
    for (int l = 0; l < SF_CNN_LAYERS; ++l) {
        L.cin[l] = cin[l];
        L.cout[l] = cout[l];
        L.cinp[l] = (cin[l] + 15) / 16 * 16;
        L.coutp[l] = (cout[l] + 15) / 16 * 16;
        L.flat_off[l] = fo;
        L.w_off[l] = wo;
        L.b_off[l] = bo;
        fo += cout[l] * cin[l] * 9 + cout[l];
        wo += L.coutp[l] * 9 * L.cinp[l];
        bo += L.coutp[l];
    }
    L.n_params = fo;
    L.dev_w_total = wo;
    L.dev_b_total = bo;
    return L;
}

void launch_cnn_pack(hipStream_t st, const CnnLayout &L, const float *flat, unsigned short *wf,
                     unsigned short *wd, float *bias) {
    const int n = L.dev_w_total + L.dev_b_total;
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, st, flat, L, wf, wd, bias);
}

void launch_cnn_input(hipStream_t st, const float *src, long img_stride, long batch_stride,
                      unsigned short *x, int B, int H, int W) {
    const long P = (long)B * H * W;
    hipLaunchKernelGGL(k_input, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, src,
                       img_stride, batch_stride, x, B, H, W);
}

void launch_cnn_input_tex(hipStream_t st, const float4 *tex, unsigned short *x, int N) {
    hipLaunchKernelGGL(k_input_tex, dim3((N + 255) / 256), dim3(256), 0, st, tex, x, N);
}

static unsigned conv_blocks(int B, int H, int W) {
    return (unsigned)(((long)B * H * ((W + 15) / 16) + 3) / 4);
}

void launch_cnn_forward(hipStream_t st, const CnnLayout &L, const CnnWeights &wts,
                        const unsigned short *x, unsigned short *const acts[SF_CNN_LAYERS - 1],
                        float *out, int B, int H, int W) {
    const dim3 g(conv_blocks(B, H, W)), blk(256);
    const unsigned short *in = x;
    for (int l = 0; l < SF_CNN_LAYERS; ++l) {
        const unsigned short *w = wts.wf + L.w_off[l];
        const float *b = wts.bias + L.b_off[l];
        if (l == 0)
            hipLaunchKernelGGL((k_conv<16, 32, CONV_RELU>), g, blk, 0, st, in, w, b, nullptr,
                               acts[0], nullptr, 0, B, H, W);
        else if (l < SF_CNN_LAYERS - 1)
            hipLaunchKernelGGL((k_conv<32, 32, CONV_RELU>), g, blk, 0, st, in, w, b, nullptr,
                               acts[l], nullptr, 0, B, H, W);
        else
            hipLaunchKernelGGL((k_conv<32, 16, CONV_LINEAR>), g, blk, 0, st, in, w, b, nullptr,
                               nullptr, out, L.cout[l], B, H, W);
        if (l < SF_CNN_LAYERS - 1) in = acts[l];
    }
}

int cnn_chunks(long P) { return (int)((P + SF_CNN_CHUNK - 1) / SF_CNN_CHUNK); }

void launch_cnn_backward(hipStream_t st, const CnnLayout &L, const CnnWeights &wts,
                         const unsigned short *x, unsigned short *const acts[SF_CNN_LAYERS - 1],
                         unsigned short *dout, unsigned short *const dpre[SF_CNN_LAYERS - 1],
                         float *wpart, float *bpart, float *grad, int B, int H, int W) {
    const long P = (long)B * H * W;
    const int nch = cnn_chunks(P);
    const dim3 g(conv_blocks(B, H, W)), blk(256);
    // dpre of layer l (l = 5: dout, no ReLU on the output layer)
    for (int l = SF_CNN_LAYERS - 1; l >= 0; --l) {
        const unsigned short *d = l == SF_CNN_LAYERS - 1 ? dout : dpre[l];
        const unsigned short *xin = l == 0 ? x : acts[l - 1];
        const int cinp = L.cinp[l], coutp = L.coutp[l];
        const int tiles = (coutp / 16) * 9 * (cinp / 16);
        const dim3 gw((unsigned)(((long)nch * tiles + 3) / 4));
        if (l == 0)
            hipLaunchKernelGGL((k_wgrad<16, 32>), gw, blk, 0, st, d, xin, wpart, B, H, W, SF_CNN_CHUNK);
        else if (l < SF_CNN_LAYERS - 1)
            hipLaunchKernelGGL((k_wgrad<32, 32>), gw, blk, 0, st, d, xin, wpart, B, H, W, SF_CNN_CHUNK);
        else
            hipLaunchKernelGGL((k_wgrad<32, 16>), gw, blk, 0, st, d, xin, wpart, B, H, W, SF_CNN_CHUNK);
        if (coutp == 32)
            hipLaunchKernelGGL(k_bgrad<32>, dim3(nch), blk, 0, st, d, bpart, P, SF_CNN_CHUNK);
        else
            hipLaunchKernelGGL(k_bgrad<16>, dim3(nch), blk, 0, st, d, bpart, P, SF_CNN_CHUNK);
        const int ng = L.cout[l] * L.cin[l] * 9 + L.cout[l];
        hipLaunchKernelGGL(k_grad_reduce, dim3((ng + 255) / 256), blk, 0, st, wpart, bpart,
                           grad + L.flat_off[l], nch, L.cin[l], L.cout[l], cinp, coutp);
        if (l == 0) break;
        // gradient w.r.t. this layer's input, through the ReLU below
        const unsigned short *wd = wts.wd + L.w_off[l];
        if (l == SF_CNN_LAYERS - 1)
            hipLaunchKernelGGL((k_conv<16, 32, CONV_DGRAD>), g, blk, 0, st, d, wd, nullptr,
                               acts[l - 1], dpre[l - 1], nullptr, 0, B, H, W);
        else
            hipLaunchKernelGGL((k_conv<32, 32, CONV_DGRAD>), g, blk, 0, st, d, wd, nullptr,
                               acts[l - 1], dpre[l - 1], nullptr, 0, B, H, W);
    }
}

int cnn_l1_blocks(long P) { return (int)((P + 255) / 256); }

void launch_cnn_l1(hipStream_t st, const float *out, const float *tgt, unsigned short *dout,
                   float *part, int B, int H, int W) {
    const long P = (long)B * H * W;
    hipLaunchKernelGGL(k_l1, dim3(cnn_l1_blocks(P)), dim3(256), 0, st, out, tgt, dout, part, B,
                       H, W);
}

void launch_cnn_adam(hipStream_t st, float *w, float *m, float *v, const float *g, int n,
                     float lr, float beta1, float beta2, float eps, float c1, float c2) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, m, v, g, n, lr,
                       beta1, beta2, eps, c1, c2);
}
