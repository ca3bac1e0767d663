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

// Weight-gradient partials of one layer, one workgroup per chunk of `chunk`
// pixels (flattened over the batch):
//   part[c][co][tap][ci] = sum over the chunk's pixels p of
//                          dpre[p][co] x[p + off(tap)][ci]
// (x zero where the tap leaves the image).  The contraction runs over
// pixels, which NHWC stores apart, so each slice of WG_SLICE pixels is
// staged transposed in LDS: the output gradient once (dT[co][p]), then per
// tap the shifted inputs (xT[ci][p]).  An MFMA operand is then eight
// consecutive pixels of one channel, one 16-byte LDS read (rows padded by
// 16 bytes so that the 16 channels of a read fall on different banks).
// Wavefront w takes tile w mod T of the (co block, ci block) grid and every
// (4 / T)-th 32-pixel step of each slice; the partial tiles of a K split are
// added in wavefront order at the end.  The bias-gradient partial
// bpart[c][co] = sum over the chunk of dpre[p][co] comes from the same
// staged rows: thread t sums its share (co = t mod COUT) of each slice, and
// the shares are added in thread order.
#define WG_SLICE 256
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(const unsigned short *__restrict__ dpre,
                                               const unsigned short *__restrict__ x,
                                               float *__restrict__ part,
                                               float *__restrict__ bpart, int B, int H, int W,
                                               int chunk) {
    constexpr int MB = COUT / 16, NB = CIN / 16, T = MB * NB, KP = 4 / T;
    static_assert(T == 1 || T == 2 || T == 4, "tiles per tap");
    constexpr int ROW = WG_SLICE + 8;  // shorts per LDS row
    __shared__ __attribute__((aligned(16))) unsigned short dT[COUT * ROW];
    __shared__ __attribute__((aligned(16))) unsigned short xT[CIN * ROW];
    __shared__ __attribute__((aligned(16))) float comb[KP > 1 ? (KP - 1) * T : 1][9][64][4];
    __shared__ float bred[256];
    constexpr int BPARTS = 256 / COUT, BSEG = WG_SLICE / BPARTS;
    static_assert(BSEG % 8 == 0, "16-byte bias reads");
    float bacc = 0.f;
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int wv = threadIdx.x >> 6, t = wv % T, kp = wv / T;
    const int mb = t / NB, nb = t % NB;
    const long P = (long)B * H * W;
    const long HW = (long)H * W;
    const int c = blockIdx.x;
    const long p_begin = (long)c * chunk, p_end = min(P, p_begin + chunk);
    v4f acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
    for (long p0 = p_begin; p0 < p_end; p0 += WG_SLICE) {
        // this thread's pixel of the slice, its image and position
        const long p = p0 + threadIdx.x;
        const bool in = p < p_end;
        const int b = in ? (int)(p / HW) : 0;
        const int rem = in ? (int)(p % HW) : 0;
        const int py = rem / W, px = rem % W;
        {
            unsigned short v[COUT];
            if (in) {
                const uint4 *src = reinterpret_cast<const uint4 *>(dpre + p * COUT);
#pragma unroll
                for (int k = 0; k < COUT / 8; ++k) {
                    const uint4 u = src[k];
                    const unsigned w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[8 * k + 2 * j] = (unsigned short)(w4[j] & 0xFFFFu);
                        v[8 * k + 2 * j + 1] = (unsigned short)(w4[j] >> 16);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < COUT; ++k) v[k] = 0;
            }
#pragma unroll
            for (int k = 0; k < COUT; ++k) dT[k * ROW + threadIdx.x] = v[k];
        }
#pragma unroll 1
        for (int tap = 0; tap < 9; ++tap) {
            const int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
            const bool ok = in && yy >= 0 && yy < H && xx >= 0 && xx < W;
            unsigned short v[CIN];
            if (ok) {
                const uint4 *src =
                    reinterpret_cast<const uint4 *>(x + ((long)(b * H + yy) * W + xx) * CIN);
#pragma unroll
                for (int k = 0; k < CIN / 8; ++k) {
                    const uint4 u = src[k];
                    const unsigned w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[8 * k + 2 * j] = (unsigned short)(w4[j] & 0xFFFFu);
                        v[8 * k + 2 * j + 1] = (unsigned short)(w4[j] >> 16);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < CIN; ++k) v[k] = 0;
            }
            __syncthreads();  // the previous tap's products are done with xT
#pragma unroll
            for (int k = 0; k < CIN; ++k) xT[k * ROW + threadIdx.x] = v[k];
            __syncthreads();
            if (tap == 0) {
                // this thread's share of the slice's bias gradient
                const unsigned short *row =
                    dT + (threadIdx.x % COUT) * ROW + (threadIdx.x / COUT) * BSEG;
#pragma unroll
                for (int k = 0; k < BSEG; k += 8) {
                    const v8s v = load8(row + k);
#pragma unroll
                    for (int j = 0; j < 8; ++j) bacc += bf2f((unsigned short)v[j]);
                }
            }
#pragma unroll
            for (int kk = kp; kk < WG_SLICE / 32; kk += KP) {
                const v8s av = load8(dT + (mb * 16 + r) * ROW + 32 * kk + 8 * q);
                const v8s bv = load8(xT + (nb * 16 + r) * ROW + 32 * kk + 8 * q);
                acc[tap] = mfma32(av, bv, acc[tap]);
            }
        }
        __syncthreads();  // dT and xT are rewritten by the next slice
    }
    // the bias partial: the threads' shares in thread order
    bred[threadIdx.x] = bacc;
    __syncthreads();
    if (threadIdx.x < COUT) {
        float t = 0.f;
        for (int k = 0; k < BPARTS; ++k) t += bred[k * COUT + threadIdx.x];
        bpart[(long)c * COUT + threadIdx.x] = t;
    }
    // the K split's partial tiles, added in wavefront order
    if (KP > 1) {
        if (kp > 0)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int i = 0; i < 4; ++i) comb[(kp - 1) * T + t][tap][lane][i] = acc[tap][i];
        __syncthreads();
        if (kp > 0) return;
#pragma unroll
        for (int k = 1; k < KP; ++k)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[tap][i] += comb[(k - 1) * T + t][tap][lane][i];
    }
    // D rows = output channels mb*16 + 4q + i, column = input channel ci
    const int ci = nb * 16 + r;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = mb * 16 + 4 * q + i;
            part[(((long)c * COUT + o) * 9 + tap) * CIN + ci] = acc[tap][i];
        }
}

// Sums the chunk partials into the flat gradient vector (layout of
// sf_cnn.h: per layer the weights (c_out, c_in, ky, kx) of the real
// channels, then the biases).  A workgroup takes 64 consecutive partial
// entries (coalesced loads) in 4 chunk groups: group g sums chunks g, g + 4,
// ... in order, and the group sums are added in group order, so the result
// does not depend on scheduling.
__global__ __launch_bounds__(256) void k_grad_reduce(const float *__restrict__ wpart,
                                                     const float *__restrict__ bpart,
                                                     float *__restrict__ grad, int nchunks,
                                                     int cin, int cout, int cinp, int coutp) {
    __shared__ double red[4][64];
    const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + l;
    const int nwp = coutp * 9 * cinp, ne = nwp + coutp;
    double s = 0.0;
    if (e < ne) {
        if (e < nwp) {
#pragma unroll 8
            for (int c = g; c < nchunks; c += 4) s += (double)wpart[(long)c * nwp + e];
        } else {
            for (int c = g; c < nchunks; c += 4) s += (double)bpart[(long)c * coutp + (e - nwp)];
        }
    }
    red[g][l] = s;
    __syncthreads();
    if (g != 0 || e >= ne) return;
    const double tot = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
    if (e < nwp) {
        const int co = e / (9 * cinp), tap = (e / cinp) % 9, ci = e % cinp;
        if (co < cout && ci < cin) grad[(co * cin + ci) * 9 + tap] = (float)tot;
    } else {
        const int co = e - nwp;
        if (co < cout) grad[cout * cin * 9 + co] = (float)tot;
    }
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
        const dim3 gw((unsigned)nch);
        if (l == 0)
            hipLaunchKernelGGL((k_wgrad<16, 32>), gw, blk, 0, st, d, xin, wpart, bpart, B, H, W,
                               SF_CNN_CHUNK);
        else if (l < SF_CNN_LAYERS - 1)
            hipLaunchKernelGGL((k_wgrad<32, 32>), gw, blk, 0, st, d, xin, wpart, bpart, B, H, W,
                               SF_CNN_CHUNK);
        else
            hipLaunchKernelGGL((k_wgrad<32, 16>), gw, blk, 0, st, d, xin, wpart, bpart, B, H, W,
                               SF_CNN_CHUNK);
        const int nge = coutp * 9 * cinp + coutp;
        hipLaunchKernelGGL(k_grad_reduce, dim3((nge + 63) / 64), blk, 0, st, wpart, bpart,
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
