// gfx950 kernels of the halfway-domain scene-flow solve.
//
// Per level the work splits into
//   * pixel kernels (16x16-pixel workgroups): residuals of the six
//     consistency checks and the gradient-constancy term with their
//     reweighted Gauss-Newton records (Sec. 3.2, Sec. 4.1-4.2, Eqs. (1)-(6),
//     (11)-(13), (19)-(24));
//   * node-tile kernels (TX x TY warp nodes per workgroup): the transpose of
//     the bilinear warp-grid interpolation (Eq. (7)) that accumulates
//     per-pixel quantities onto nodes, done as a deterministic two-pass
//     separable reduction in LDS, plus the regularisers of Eqs. (14)-(18);
//   * node-wise kernels for the PCG vector updates and step control.
// Every cross-workgroup sum is deterministic and needs no atomics or
// device-scope fences: each workgroup writes a partial, and the kernels
// that consume the sum add all partials in a fixed order in double
// precision (every consuming workgroup obtaining the same value).
#include <math.h>
#include <stdlib.h>

#include "sf_cnn.h"
#include "sf_internal.h"

// Node-tile shape per grid stride S and variant V: tx x ty nodes, tpn
// threads per node (tpn >= 2S so one thread sums one support row),
// NT = tx ty tpn threads and at most PPT region pixels per thread.
// Variant 0 (every kernel): 256 threads where the register budget allows
// more than one workgroup per CU, 512 for the largest strides.  Variants 1
// and 2 (the PCG kernels at strides 2, 4, 8, chosen by the autotuner):
// twice the nodes per tile (fewer re-read halo pixels, 512 threads) and a
// smaller tile (more workgroups for small levels).
template <int S, int V>
struct TileShape {
    static constexpr int TX = S <= 2 ? 16 : (S <= 4 ? 8 : 4);
    static constexpr int TY = S == 1 ? 8 : (S == 2 ? 4 : (S <= 4 ? 4 : 2));
    static constexpr int TPN = S == 1 ? 2 : (S == 2 ? 4 : (S <= 4 ? 8 : (S <= 6 ? 32 : 64)));
};
template <> struct TileShape<2, 1> { static constexpr int TX = 16, TY = 8, TPN = 4; };
template <> struct TileShape<2, 2> { static constexpr int TX = 8, TY = 4, TPN = 8; };
template <> struct TileShape<4, 1> { static constexpr int TX = 8, TY = 8, TPN = 8; };
template <> struct TileShape<4, 2> { static constexpr int TX = 4, TY = 4, TPN = 16; };
template <> struct TileShape<8, 1> { static constexpr int TX = 2, TY = 4, TPN = 64; };
template <> struct TileShape<8, 2> { static constexpr int TX = 2, TY = 2, TPN = 64; };
// S = 0: the node-block apply mode (any stride): 8 x 8 nodes, four threads
// per node share its nine block products.
template <> struct TileShape<0, 0> { static constexpr int TX = 8, TY = 8, TPN = 4; };
template <> struct TileShape<0, 1> { static constexpr int TX = 16, TY = 8, TPN = 4; };
template <> struct TileShape<0, 2> { static constexpr int TX = 8, TY = 4, TPN = 4; };
template <> struct TileShape<0, 3> { static constexpr int TX = 4, TY = 4, TPN = 4; };

template <int S, int V = 0>
struct TileTraits {
    static constexpr int TX = TileShape<S, V>::TX;
    static constexpr int TY = TileShape<S, V>::TY;
    static constexpr int TPN = TileShape<S, V>::TPN;
    static constexpr int NT = TX * TY * TPN;
    static constexpr int MAXPX = ((TX + 1) * S + (S & 1)) * ((TY + 1) * S + (S & 1));
    static constexpr int PPT = S == 0 ? 1 : (MAXPX + NT - 1) / NT;
    static_assert(TPN >= 2 * S && TPN <= 64, "one support row per thread, one wave per node");
    static_assert(NT == 256 || NT == 512 || (S == 0 && (NT == 128 || NT == 64)), "block size");
    static_assert(NT <= 512 || PPT <= 2, "registers");
    static_assert(PPT <= 3, "pixels per thread");
};

namespace {

// sign of (s, m, d) in the sample position of camera L0, R0, L1, R1
// (Eqs. (1)-(6) and (16)-(17))
__device__ __forceinline__ float sgn(int cam, int f) {
    // rows: L0 (-,-,+), R0 (+,-,-), L1 (-,+,-), R1 (+,+,+)
    const int t[4][3] = {{-1, -1, 1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, 1}};
    return (float)t[cam][f];
}
// d_k = I_a(P_a) - I_b(P_b): stereo (R0,L0), (R1,L1); motion (L1,L0),
// (R1,R0); cross (R1,L0), (L1,R0)
__device__ __forceinline__ int pair_a(int k) {
    const int t[6] = {1, 3, 2, 3, 3, 2};
    return t[k];
}
__device__ __forceinline__ int pair_b(int k) {
    const int t[6] = {0, 2, 0, 1, 0, 1};
    return t[k];
}

// upper-triangular index of (i, j), i <= j, in a 6x6 symmetric block
__device__ __forceinline__ int tri(int i, int j) {
    return i * 6 - (i * (i - 1)) / 2 + (j - i);
}

// Bilinear bracket of coordinate x on a lattice of G nodes at stride s with
// nodes at cell centres: u = (x + 1/2)/s - 1/2 = (2x + 1 - s) / (2s),
// clamped to [0, G-1]; evaluated in integers so the bracket is exact.
struct Bracket {
    int i0, i1;
    float w0, w1;
};
__device__ __forceinline__ Bracket bracket(int x, int s, int G) {
    Bracket b;
    if (G == 1) {
        b.i0 = 0; b.i1 = 0; b.w0 = 1.f; b.w1 = 0.f;
        return b;
    }
    const int num = 2 * x + 1 - s;
    const int den = 2 * s;
    if (num <= 0) {
        b.i0 = 0; b.i1 = 1; b.w0 = 1.f; b.w1 = 0.f;
        return b;
    }
    const int c = num / den;
    if (c >= G - 1) {
        b.i0 = G - 2; b.i1 = G - 1; b.w0 = 0.f; b.w1 = 1.f;
        return b;
    }
    const float f = (float)(num - c * den) / (float)den;
    b.i0 = c; b.i1 = c + 1; b.w0 = 1.f - f; b.w1 = f;
    return b;
}
// First / last pixel where node i has a nonzero bilinear weight (pixels
// clamped beyond the last node weigh only on node G-1, those before the
// first node only on node 0).
__device__ __forceinline__ int sup_lo(int i, int s) {
    return i == 0 ? 0 : ((2 * i - 1) * s) / 2;
}
__device__ __forceinline__ int sup_hi(int i, int s, int G, int W) {
    return i >= G - 1 ? W - 1 : min(W - 1, ((2 * i + 3) * s) / 2 - 1);
}

// ---- reductions ----------------------------------------------------------

// Lane sums with DPP (data-parallel primitives fused into the add): within a
// row of 16 lanes by quad permutations and mirrors, across rows with
// readlane.  `width` (a power of two, uniform) is the size of the groups of
// consecutive lanes summed; every lane of a group receives the group's sum.
// Must be called with all lanes of the wavefront active.
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float readlane_f(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T dpp_step(T v, int ctrl_id);
template <>
__device__ __forceinline__ float dpp_step<float>(float v, int c) {
    return c == 0 ? dppf<0xB1>(v) : c == 1 ? dppf<0x4E>(v) : c == 2 ? dppf<0x141>(v) : dppf<0x140>(v);
}
template <>
__device__ __forceinline__ double dpp_step<double>(double v, int c) {
    return c == 0 ? dppd<0xB1>(v) : c == 1 ? dppd<0x4E>(v) : c == 2 ? dppd<0x141>(v) : dppd<0x140>(v);
}
__device__ __forceinline__ float rl(float v, int l) { return readlane_f(v, l); }
__device__ __forceinline__ double rl(double v, int l) { return readlane_d(v, l); }

template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
    if (width >= 2) v += dpp_step<T>(v, 0);   // quad_perm [1,0,3,2]: lane ^ 1
    if (width >= 4) v += dpp_step<T>(v, 1);   // quad_perm [2,3,0,1]: lane ^ 2
    if (width >= 8) v += dpp_step<T>(v, 2);   // row_half_mirror
    if (width >= 16) v += dpp_step<T>(v, 3);  // row_mirror
    if (width >= 32) {
        const T r0 = rl(v, 0), r1 = rl(v, 16), r2 = rl(v, 32), r3 = rl(v, 48);
        if (width == 32) v = (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
        else v = (r0 + r1) + (r2 + r3);
    }
    return v;
}
__device__ __forceinline__ float wave_sum(float v) { return group_sum<float>(v, 64); }
__device__ __forceinline__ double wave_sum_d(double v) { return group_sum<double>(v, 64); }

// Sums K per-thread values over the (256-thread) block; the result is valid
// in thread 0.  Fixed order, so bitwise reproducible.
// REUSE: a second barrier lets the caller reuse the reduction buffer (a
// later call); at the end of a kernel it is not needed.
template <int K, bool REUSE = true>
__device__ void block_sum(float (&v)[K], float (&out)[K]) {
    __shared__ float red[16][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float s = wave_sum(v[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float acc = red[0][k];
            for (int w = 1; w < nw; ++w) acc += red[w][k];
            out[k] = acc;
        }
    }
    if (REUSE) __syncthreads();
}

// Sum in double of n partials by the whole block; result valid in every
// thread.  Fixed order, so bitwise reproducible.
// acc[k] += get(k, i) for i = first, first + step, ... < n, in that order,
// with the loads of U indices issued together (an index past n reads entry
// 0 and adds +0), so a long stride loop costs one memory round trip per U
// steps instead of one per step.
template <int K, int U, class Get>
__device__ __forceinline__ void strided_sums(int first, int step, int n, Get get,
                                             double (&acc)[K]) {
    for (int i0 = first; i0 < n; i0 += U * step) {
        float v[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * step;
            const bool ok = i < n;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float t = get(k, ok ? i : 0);
                v[u][k] = ok ? t : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += (double)v[u][k];
    }
}

// K planes at once (plane(k) gives plane k): every load is issued before
// the first barrier, and each plane is summed in the same order as by
// block_sum_partials.
template <int K, class PlaneFn>
__device__ void block_sum_planes(PlaneFn plane, int n, double (&out)[K]) {
    __shared__ double red[16][K];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    strided_sums<K, 8>(threadIdx.x, blockDim.x, n, [&](int k, int i) { return plane(k)[i]; }, acc);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = wave_sum_d(acc[k]);
        if (lane == 0) red[wv][k] = acc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double r = red[0][k];
        for (int w = 1; w < nw; ++w) r += red[w][k];
        out[k] = r;
    }
    __syncthreads();
}

__device__ double block_sum_partials(const float *part, int n) {
    __shared__ double red[16];
    double a1[1] = {0.0};
    strided_sums<1, 8>(threadIdx.x, blockDim.x, n, [&](int, int i) { return part[i]; }, a1);
    double acc = a1[0];
    acc = wave_sum_d(acc);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < nw; ++w) r += red[w];
    __syncthreads();
    return r;
}


// ---- frame binding ---------------------------------------------------------
//
// Every kernel exists in a single-frame form, which takes the frame's
// LevelArgs by value, and a batched form, which takes a FrameMap: the
// workgroup finds its frame in the map's block prefix (uniform scalar
// compares), loads that frame's arguments from the device table and works
// on its block index within the frame.  Per-frame partial sums,
// scalars and logs keep every reduction segmented by frame.
template <bool B>
using KArg = typename std::conditional<B, FrameMap, LevelArgs>::type;

// XCD-aware block order of single-frame launches.  The dispatcher hands
// workgroup b of a launch to XCD b mod 8, and each XCD has its own L2; this
// bijection gives every XCD one contiguous range of logical blocks (XCD x
// takes the ceil/floor(n/8) indices after those of XCDs 0..x-1), so
// neighbouring tiles, whose halos overlap, run on the same XCD and share
// its L2 (at 640x480 the level-0 PCG iteration fetches 30 % fewer bytes and
// runs 6 % faster).  Batched launches keep the hardware order: there the
// same remap, or one in chunks of 32 or 128 blocks, cut the fetched bytes
// too but made the level-0 iteration 2-3 % slower.  Results do not depend
// on which physical workgroup runs a logical block.
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ void bind(const LevelArgs &ka, LevelArgs &a, int &bid, int &nblk) {
    a = ka;
    bid = xcd_block(blockIdx.x, gridDim.x);
    nblk = gridDim.x;
}
__device__ __forceinline__ void bind(const FrameMap &m, LevelArgs &a, int &bid, int &nblk) {
    const int b = blockIdx.x;
    int f = 0;
    for (int k = 1; k < m.nf; ++k) f += b >= m.first[k] ? 1 : 0;
    a = m.tab[f];
    bid = b - m.first[f];
    nblk = m.first[f + 1] - m.first[f];
}
// ---- node vectors ------------------------------------------------------------
//
// A node vector holds one packed 6-float record per node (s_x, s_y, m_x,
// m_y, d_x, d_y; 24 bytes, so a run of nodes moves no padding), moved as
// three 8-byte accesses; vector v of the level starts at
// nodes + v * SF_NREC * G_0.
__device__ __forceinline__ float *nvec(const LevelArgs &a, int v) {
    return a.nodes + (size_t)v * SF_NREC * a.G0;
}
__device__ __forceinline__ void ld6(const float *vec, long n, float (&x)[6]) {
    const float2 *p = reinterpret_cast<const float2 *>(vec + n * SF_NREC);
    const float2 a = p[0], b = p[1], c = p[2];
    x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y; x[4] = c.x; x[5] = c.y;
}
__device__ __forceinline__ void st6(float *vec, long n, const float (&x)[6]) {
    float2 *p = reinterpret_cast<float2 *>(vec + n * SF_NREC);
    p[0] = make_float2(x[0], x[1]);
    p[1] = make_float2(x[2], x[3]);
    p[2] = make_float2(x[4], x[5]);
}

#define SF_BIND(ka)              \
    LevelArgs a;                 \
    int bid, nblk;               \
    bind(ka, a, bid, nblk);      \
    (void)nblk

// ---- bilinear sampling of (I, Gx, Gy) ------------------------------------

// A sample coordinate x + dlt (x the integer pixel, dlt the displacement
// of Eqs. (1)-(6)) taken apart into its bilinear cell and fraction without
// forming x + dlt in float32: the fraction keeps the precision of the
// displacement (2^-20 px for |dlt| < 16) instead of that of the absolute
// coordinate (2^-14 px beyond 512 px), so cell choices at the interpolant's
// kinks and the weights follow the exact position far more closely.
// `in` is the exact test 0 <= x + dlt <= n - 1; outside, the coordinate is
// clamped to the nearest end (fraction 0 at 0, 1 in cell n - 2 at n - 1).
// A NaN or huge displacement clamps to the low end, outside.
struct AxisPos {
    int i0;     // cell: samples i0 and i0 + 1
    float fr;   // fraction in [0, 1]
    bool in;
};
__device__ __forceinline__ AxisPos axis_pos(int x, float dlt, int n) {
    constexpr float LIM = 1.0e7f;
    float k = floorf(dlt);
    float fr = dlt - k;  // exact: dlt and k share the exponent range, fr in [0, 1)
    if (!(fabsf(dlt) < LIM)) {
        k = dlt > 0.f ? LIM : -LIM;
        fr = 0.f;
    }
    const long xi = (long)x + (long)k;
    AxisPos a;
    a.in = xi >= 0 && (xi < n - 1 || (xi == n - 1 && fr == 0.f));
    if (xi < 0) {
        a.i0 = 0;
        a.fr = 0.f;
    } else if (xi >= n - 1) {
        a.i0 = n - 2;
        a.fr = 1.f;
    } else {
        a.i0 = (int)xi;
        a.fr = fr;
    }
    return a;
}

// Displacement of camera cam's position from the halfway pixel (Eqs.
// (1)-(6)): signs of s, m, d per camera, x and y components.
__device__ __forceinline__ float cam_dx(int cam, const float (&f)[6]) {
    return (sgn(cam, 0) * f[0] + sgn(cam, 1) * f[2]) + sgn(cam, 2) * f[4];
}
__device__ __forceinline__ float cam_dy(int cam, const float (&f)[6]) {
    return (sgn(cam, 0) * f[1] + sgn(cam, 1) * f[3]) + sgn(cam, 2) * f[5];
}

// Value of the three channels at a sample position and the derivatives of
// their bilinear interpolants; clamp-to-edge coordinates, zero derivative
// in a clamped direction.  All accesses stay inside the W x H image.
struct Samp {
    float v[3];   // I, Gx, Gy
    float dx[3];  // d/dpx
    float dy[3];  // d/dpy
};
__device__ __forceinline__ void sample3(const float4 *__restrict__ img, int W,
                                        const AxisPos &px, const AxisPos &py, Samp &o) {
    const int x0 = px.i0, y0 = py.i0;
    const float fx = px.fr, fy = py.fr;
    const float4 a = img[y0 * W + x0];
    const float4 b = img[y0 * W + x0 + 1];
    const float4 c = img[(y0 + 1) * W + x0];
    const float4 d = img[(y0 + 1) * W + x0 + 1];
    const float ta[3] = {a.x, a.y, a.z}, tb[3] = {b.x, b.y, b.z};
    const float tc[3] = {c.x, c.y, c.z}, td[3] = {d.x, d.y, d.z};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        o.v[ch] = (1.f - fy) * ((1.f - fx) * ta[ch] + fx * tb[ch]) +
                  fy * ((1.f - fx) * tc[ch] + fx * td[ch]);
        o.dx[ch] = px.in ? ((1.f - fy) * (tb[ch] - ta[ch]) + fy * (td[ch] - tc[ch])) : 0.f;
        o.dy[ch] = py.in ? ((1.f - fx) * (tc[ch] - ta[ch]) + fx * (td[ch] - tb[ch])) : 0.f;
    }
}

// ---- pyramid --------------------------------------------------------------

struct Img4 {
    const float *p[4];
};

// Pyramid workgroups cover 64 x 4 texels of one image.
__host__ __device__ inline int tex_blocks_x(int W) { return (W + 63) / 64; }
__host__ __device__ inline int tex_blocks(int W, int H) { return tex_blocks_x(W) * ((H + 3) / 4) * 4; }

// Level 0: texel = (I, Gx, Gy, 0) with central-difference gradients
// (one-sided at the borders).  Images come from the argument (single
// frame) or the frame's caller buffers (batched).
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_tex0(KArg<B> ka, Img4 in) {
    SF_BIND(ka);
    const int W = a.d.W, H = a.d.H;
    const int bx = tex_blocks_x(W), per = bx * ((H + 3) / 4);
    const int c = bid / per, r = bid % per;
    const int x = (r % bx) * 64 + (threadIdx.x & 63);
    const int y = (r / bx) * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    float4 *tex = const_cast<float4 *>(a.tex);
    const float *I = B ? a.io->img[c] : in.p[c];
    const float v = I[y * W + x];
    float gx, gy;
    if (x == 0) gx = I[y * W + 1] - I[y * W];
    else if (x == W - 1) gx = I[y * W + W - 1] - I[y * W + W - 2];
    else gx = 0.5f * (I[y * W + x + 1] - I[y * W + x - 1]);
    if (y == 0) gy = I[W + x] - I[x];
    else if (y == H - 1) gy = I[(H - 1) * W + x] - I[(H - 2) * W + x];
    else gy = 0.5f * (I[(y + 1) * W + x] - I[(y - 1) * W + x]);
    tex[(long)c * W * H + y * W + x] = make_float4(v, gx, gy, 0.f);
}

// 2x2 box (mip-map) value of the coarser level at (x, y) from the finer
// level's intensities.
__device__ __forceinline__ float box(const float4 *src, int Ws, int x, int y) {
    const float a = src[(2 * y) * Ws + 2 * x].x;
    const float b = src[(2 * y) * Ws + 2 * x + 1].x;
    const float c = src[(2 * y + 1) * Ws + 2 * x].x;
    const float d = src[(2 * y + 1) * Ws + 2 * x + 1].x;
    return 0.25f * (((a + b) + c) + d);
}

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_texl(KArg<B> ka) {
    SF_BIND(ka);
    const int W = a.d.W, H = a.d.H, Ws = a.Wf, Hs = a.Hf;
    const int bx = tex_blocks_x(W), per = bx * ((H + 3) / 4);
    const int c = bid / per, r = bid % per;
    const int x = (r % bx) * 64 + (threadIdx.x & 63);
    const int y = (r / bx) * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    float4 *dst = const_cast<float4 *>(a.tex);
    const float4 *S = a.tex_fine + (long)c * Ws * Hs;
    const float v = box(S, Ws, x, y);
    float gx, gy;
    if (x == 0) gx = box(S, Ws, 1, y) - v;
    else if (x == W - 1) gx = v - box(S, Ws, W - 2, y);
    else gx = 0.5f * (box(S, Ws, x + 1, y) - box(S, Ws, x - 1, y));
    if (y == 0) gy = box(S, Ws, x, 1) - v;
    else if (y == H - 1) gy = v - box(S, Ws, x, H - 2);
    else gy = 0.5f * (box(S, Ws, x, y + 1) - box(S, Ws, x, y - 1));
    dst[(long)c * W * H + y * W + x] = make_float4(v, gx, gy, 0.f);
}

// ---- per-pixel evaluation -------------------------------------------------

#define TILE_PX 16       // pixel tile edge of the pixel kernels
#define TILE_NODES 20    // max nodes per axis a pixel tile touches (s >= 1)

// Workgroup counts of one frame's launches.
__host__ __device__ inline int pixel_tiles(const LevelDims &d) {
    return ((d.W + TILE_PX - 1) / TILE_PX) * ((d.H + TILE_PX - 1) / TILE_PX);
}
__host__ __device__ inline int node_blocks(const LevelDims &d) {
    return (d.G + SF_BLOCK - 1) / SF_BLOCK;
}
__host__ __device__ inline int energy_blocks_of(const LevelDims &d) {
    return pixel_tiles(d) + node_blocks(d);
}
__host__ __device__ inline int tiles_x_of(const LevelDims &d, const TileCfg &t) {
    return (d.Gx + t.tx - 1) / t.tx;
}
__host__ __device__ inline int node_tiles_of(const LevelDims &d, const TileCfg &t) {
    return tiles_x_of(d, t) * ((d.Gy + t.ty - 1) / t.ty);
}

// Node totals (base + delta + tau dx) of the nodes a pixel tile touches,
// staged in LDS.
struct NodeStage {
    float t[6][TILE_NODES][TILE_NODES];
    int nx0, ny0;
};

__device__ void stage_nodes(const LevelArgs &a, int x0, int y0, float tau,
                            NodeStage &S) {
    const LevelDims &d = a.d;
    const int x1 = min(x0 + TILE_PX - 1, d.W - 1);
    const int y1 = min(y0 + TILE_PX - 1, d.H - 1);
    const Bracket bx0 = bracket(x0, a.s, d.Gx), bx1 = bracket(x1, a.s, d.Gx);
    const Bracket by0 = bracket(y0, a.s, d.Gy), by1 = bracket(y1, a.s, d.Gy);
    const int nx0 = bx0.i0, nx1 = bx1.i1, ny0 = by0.i0, ny1 = by1.i1;
    const int cw = nx1 - nx0 + 1, ch = ny1 - ny0 + 1;
    if (threadIdx.x == 0) { S.nx0 = nx0; S.ny0 = ny0; }
    const float *base = nvec(a, NV_BASE);
    const float *delta = nvec(a, NV_DELTA);
    const float *dx = nvec(a, NV_X);
    for (int t = threadIdx.x; t < cw * ch; t += blockDim.x) {
        const int j = t / cw, i = t % cw;
        const long n = (long)(ny0 + j) * d.Gx + (nx0 + i);
        float b[6], dl[6], x[6];
        ld6(base, n, b);
        ld6(delta, n, dl);
        if (tau != 0.f) ld6(dx, n, x);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            float v = dl[q];
            if (tau != 0.f) v = v + tau * x[q];
            S.t[q][j][i] = b[q] + v;
        }
    }
}

// Node values of one vector that a pixel tile touches, staged
// in LDS like stage_nodes.
__device__ void stage_vector(const LevelArgs &a, int x0, int y0, const float *vec,
                             NodeStage &S) {
    const LevelDims &d = a.d;
    const int x1 = min(x0 + TILE_PX - 1, d.W - 1);
    const int y1 = min(y0 + TILE_PX - 1, d.H - 1);
    const Bracket bx0 = bracket(x0, a.s, d.Gx), bx1 = bracket(x1, a.s, d.Gx);
    const Bracket by0 = bracket(y0, a.s, d.Gy), by1 = bracket(y1, a.s, d.Gy);
    const int nx0 = bx0.i0, nx1 = bx1.i1, ny0 = by0.i0, ny1 = by1.i1;
    const int cw = nx1 - nx0 + 1, ch = ny1 - ny0 + 1;
    if (threadIdx.x == 0) { S.nx0 = nx0; S.ny0 = ny0; }
    for (int t = threadIdx.x; t < cw * ch; t += blockDim.x) {
        const int j = t / cw, i = t % cw;
        float v[6];
        ld6(vec, (long)(ny0 + j) * d.Gx + (nx0 + i), v);
#pragma unroll
        for (int q = 0; q < 6; ++q) S.t[q][j][i] = v[q];
    }
}

struct PixelOut {
    float e_photo, e_grad;
    float grad[6];
    float gram[21];
};

// Residuals of pixel (x, y) given its six flows; energies (times the mask
// c) and, if LIN, the reweighted gradient and Gauss-Newton block.
template <bool LIN>
__device__ __forceinline__ void pixel_terms(const LevelArgs &a, int x, int y,
                                            const float (&f)[6], float c,
                                            PixelOut &o) {
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    Samp S[4];
#pragma unroll
    for (int cam = 0; cam < 4; ++cam) {
        const AxisPos px = axis_pos(x, cam_dx(cam, f), d.W);
        const AxisPos py = axis_pos(y, cam_dy(cam, f), d.H);
        sample3(a.tex + (long)cam * d.N, d.W, px, py, S[cam]);
    }
    if (a.illum) {
        // illumination correction of the right-camera samples
        const float cr = a.illum[(long)y * d.W + x];
        S[1].v[0] -= cr;
        S[3].v[0] -= cr;
    }
    const float eps2 = C.eps * C.eps;
    o.e_photo = 0.f;
    o.e_grad = 0.f;
    if (LIN) {
#pragma unroll
        for (int q = 0; q < 6; ++q) o.grad[q] = 0.f;
#pragma unroll
        for (int t = 0; t < 21; ++t) o.gram[t] = 0.f;
    }
    if (c == 0.f) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int A = pair_a(k), B = pair_b(k);
        const float dk = S[A].v[0] - S[B].v[0];
        const float g0 = S[A].v[1] - S[B].v[1];
        const float g1 = S[A].v[2] - S[B].v[2];
        const float ph = sqrtf(dk * dk + eps2);
        const float pg = sqrtf(g0 * g0 + g1 * g1 + eps2);
        o.e_photo += ph;
        o.e_grad += pg;
        if (LIN) {
            // flow-space Jacobian rows: photometric J_d and gradient J_g0, J_g1
            float jd[6], j0[6], j1[6];
#pragma unroll
            for (int ff = 0; ff < 3; ++ff) {
                const float sa = sgn(A, ff), sb = sgn(B, ff);
                jd[2 * ff] = sa * S[A].dx[0] - sb * S[B].dx[0];
                jd[2 * ff + 1] = sa * S[A].dy[0] - sb * S[B].dy[0];
                j0[2 * ff] = sa * S[A].dx[1] - sb * S[B].dx[1];
                j0[2 * ff + 1] = sa * S[A].dy[1] - sb * S[B].dy[1];
                j1[2 * ff] = sa * S[A].dx[2] - sb * S[B].dx[2];
                j1[2 * ff + 1] = sa * S[A].dy[2] - sb * S[B].dy[2];
            }
            const float wd = c * C.w_photo / ph;
            const float wg = c * C.w_grad / pg;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                o.grad[i] += wd * dk * jd[i] + wg * (g0 * j0[i] + g1 * j1[i]);
#pragma unroll
                for (int j = i; j < 6; ++j)
                    o.gram[tri(i, j)] += wd * jd[i] * jd[j] + wg * (j0[i] * j0[j] + j1[i] * j1[j]);
            }
        }
    }
    o.e_photo *= c;
    o.e_grad *= c;
}

__device__ __forceinline__ void pixel_flows(const LevelArgs &a, int x, int y,
                                            const NodeStage &S, float (&f)[6]) {
    const Bracket bx = bracket(x, a.s, a.d.Gx), by = bracket(y, a.s, a.d.Gy);
    const int ix0 = bx.i0 - S.nx0, ix1 = bx.i1 - S.nx0;
    const int iy0 = by.i0 - S.ny0, iy1 = by.i1 - S.ny0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        f[q] = by.w0 * (bx.w0 * S.t[q][iy0][ix0] + bx.w1 * S.t[q][iy0][ix1]) +
               by.w1 * (bx.w0 * S.t[q][iy1][ix0] + bx.w1 * S.t[q][iy1][ix1]);
}

// ---- regularisers on one node ---------------------------------------------

// Epipolar residuals e_t = l_t^T F r_t (t = 0, 1) at the node's total flows
// and their gradients w.r.t. the six node components, Eqs. (15)-(17).
__device__ __forceinline__ void epi_terms(const float *F, float gx, float gy,
                                          const float (&tot)[6], float (&e)[2],
                                          float (&J)[2][6]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int cl = t == 0 ? 0 : 2, cr = t == 0 ? 1 : 3;
        const float lx = ((gx + sgn(cl, 0) * tot[0]) + sgn(cl, 1) * tot[2]) + sgn(cl, 2) * tot[4];
        const float ly = ((gy + sgn(cl, 0) * tot[1]) + sgn(cl, 1) * tot[3]) + sgn(cl, 2) * tot[5];
        const float rx = ((gx + sgn(cr, 0) * tot[0]) + sgn(cr, 1) * tot[2]) + sgn(cr, 2) * tot[4];
        const float ry = ((gy + sgn(cr, 0) * tot[1]) + sgn(cr, 1) * tot[3]) + sgn(cr, 2) * tot[5];
        // F r and F^T l
        const float fr0 = F[0] * rx + F[1] * ry + F[2];
        const float fr1 = F[3] * rx + F[4] * ry + F[5];
        const float fr2 = F[6] * rx + F[7] * ry + F[8];
        const float fl0 = F[0] * lx + F[3] * ly + F[6];
        const float fl1 = F[1] * lx + F[4] * ly + F[7];
        e[t] = lx * fr0 + ly * fr1 + fr2;
#pragma unroll
        for (int ff = 0; ff < 3; ++ff) {
            J[t][2 * ff] = sgn(cl, ff) * fr0 + sgn(cr, ff) * fl0;
            J[t][2 * ff + 1] = sgn(cl, ff) * fr1 + sgn(cr, ff) * fl1;
        }
    }
}

__device__ __forceinline__ void node_xy(int i, int j, int s, float &gx, float &gy) {
    gx = (float)(2 * i + 1) * 0.5f * (float)s - 0.5f;
    gy = (float)(2 * j + 1) * 0.5f * (float)s - 0.5f;
}

// ---- energy / linearisation kernel -----------------------------------------

// Regulariser energies of node n at delta (+ tau dx): raw E_smooth, E_epi,
// E_mag contributions (Eqs. (14), (15), (18)).
__device__ void node_energy(const LevelArgs &a, int n, float tau, float (&part)[5]) {
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    const int i = n % d.Gx, j = n / d.Gx;
    const float *base = nvec(a, NV_BASE);
    const float *delta = nvec(a, NV_DELTA);
    const float *dx = nvec(a, NV_X);
    float dl[6], tot[6], b[6], x[6];
    ld6(delta, n, dl);
    ld6(base, n, b);
    if (tau != 0.f) ld6(dx, n, x);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (tau != 0.f) dl[q] = dl[q] + tau * x[q];
        tot[q] = b[q] + dl[q];
    }
    const float wi = a.wnode[n];
    float es = 0.f;
    const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ii = i + nb[k][0], jj = j + nb[k][1];
        if (ii < 0 || ii >= d.Gx || jj < 0 || jj >= d.Gy) continue;
        const int m = jj * d.Gx + ii;
        float dm[6], xm[6];
        ld6(delta, m, dm);
        if (tau != 0.f) ld6(dx, m, xm);
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            float v = dm[q];
            if (tau != 0.f) v = v + tau * xm[q];
            const float df = dl[q] - v;
            acc += C.wf[q] * df * df;
        }
        es += wi * acc;
    }
    float gx, gy;
    node_xy(i, j, a.s, gx, gy);
    float e[2], J[2][6];
    epi_terms(C.F[a.level], gx, gy, tot, e, J);
    float em = 0.f;
#pragma unroll
    for (int q = 0; q < 6; ++q) em += C.mf[q] * dl[q] * dl[q];
    part[2] = es;
    part[3] = e[0] * e[0] + e[1] * e[1];
    part[4] = em;
}

// Energy grid: blocks [0, n_pix) are 16x16 pixel tiles, blocks
// [n_pix, grid) 256 nodes each for the regulariser energies, at
// delta + tau dx.  With LIN also the per-pixel records (tau = 0: the
// linearisation at delta; tau = 1: the speculative one at delta + dx, whose
// energy is also the step control's tau = 1 trial); the right-hand-side
// kernel sums the energy.  Otherwise a trial energy (summed by the step
// control).

// Energy terms of one energy-grid workgroup's share at step length tau:
// pixel tile `tile` (16 x 16 pixels; with LIN also its Gauss-Newton
// records) or, past the pixel tiles, a block of nodes (regularisers).
// Uses S for the tile's node totals and ends with a barrier, so a caller
// may stage the next tile into S right away.
template <bool LIN>
__device__ void energy_tile(const LevelArgs &a, int tile, float tau, NodeStage &S,
                            float (&part)[5]) {
    const LevelDims &d = a.d;
    const int n_pix = pixel_tiles(d);
    if (tile < n_pix) {
        const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
        const int x0 = (tile % tiles_x) * TILE_PX, y0 = (tile / tiles_x) * TILE_PX;
        stage_nodes(a, x0, y0, tau, S);
        __syncthreads();
        const int x = x0 + (threadIdx.x & (TILE_PX - 1));
        const int y = y0 + (threadIdx.x / TILE_PX);
        if (x < d.W && y < d.H) {
            float f[6];
            pixel_flows(a, x, y, S, f);
            const int pix = y * d.W + x;
            const float c = a.cmask[pix] ? 1.f : 0.f;
            PixelOut o;
            pixel_terms<LIN>(a, x, y, f, c, o);
            part[0] += o.e_photo;
            part[1] += o.e_grad;
            if (LIN) {
                float g24[SF_GRAM_STRIDE];
#pragma unroll
                for (int i = 0; i < 6; ++i)
#pragma unroll
                    for (int j = i; j < 6; ++j) g24[gram_index(i, j)] = o.gram[tri(i, j)];
                g24[21] = g24[22] = g24[23] = 0.f;
                float4 *gp = reinterpret_cast<float4 *>(a.gram + (long)pix * SF_GRAM_STRIDE);
#pragma unroll
                for (int v = 0; v < 6; ++v)
                    gp[v] = make_float4(g24[4 * v], g24[4 * v + 1], g24[4 * v + 2], g24[4 * v + 3]);
                float4 *rp = reinterpret_cast<float4 *>(a.grad + (long)pix * SF_GRAD_STRIDE);
                rp[0] = make_float4(o.grad[0], o.grad[1], o.grad[2], o.grad[3]);
                rp[1] = make_float4(o.grad[4], o.grad[5], 0.f, 0.f);
            }
        }
        __syncthreads();
    } else {
        const int n = (tile - n_pix) * SF_BLOCK + threadIdx.x;
        if (n < d.G) {
            float pn[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            node_energy(a, n, tau, pn);
#pragma unroll
            for (int k = 0; k < 5; ++k) part[k] += pn[k];
        }
    }
}

// The energy grid: one workgroup per pixel tile and per node block, each
// writing its five partial sums to the planes PS_E (the linearisation, or
// the full step tau = 1 of the step control).  The consumers reduce them.
template <bool B, bool LIN>
__global__ __launch_bounds__(SF_BLOCK) void k_energy(KArg<B> ka, float tau) {
    SF_BIND(ka);
    (void)nblk;
    __shared__ NodeStage S;
    float part[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    energy_tile<LIN>(a, bid, tau, S, part);
    float tot5[5];
    block_sum<5, false>(part, tot5);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) a.partials[(long)(PS_E + k) * a.max_blocks + bid] = tot5[k];
    }
}

// Energy terms of a trial from its five partial planes (n entries from
// plane `base`), summed by one wavefront in a fixed order, and the total
// E (the weights of Eqs. (8)-(10)).  Every caller obtains the same values.
__device__ void trial_energy_wave(const LevelArgs &a, int base, int n, double (&e)[6]) {
    const int lane = threadIdx.x & 63;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const float *p0 = a.partials + (long)base * a.max_blocks;
    strided_sums<5, 8>(lane, 64, n, [&](int k, int b) { return p0[(long)k * a.max_blocks + b]; },
                       acc);
#pragma unroll
    for (int k = 0; k < 5; ++k) e[k] = wave_sum_d(acc[k]);
    const DevConst &C = *a.cst;
    e[5] = (double)C.w_photo * e[0] + (double)C.w_grad * e[1] +
           (double)C.w_reg * ((double)C.w_smooth * e[2] + (double)C.w_epi * e[3] +
                              (double)C.w_mag * e[4]);
}

// Workgroups of the shorter-step trials of a frame (a fixed, small grid
// that strides over the energy tiles).
__host__ __device__ inline int rest_blocks_of(const LevelDims &d) {
    const int n = energy_blocks_of(d);
    return n < 128 ? n : 128;
}

// The first shorter step tau = 2^-t (t = 1 .. n_trials - 1) whose energy
// does not exceed E(delta), from the shorter trials' partials, once tau = 1
// was rejected; -1 if none (delta stays).  e: that trial's terms.  One
// wavefront; every caller obtains the same result.
__device__ int rest_decision(const LevelArgs &a, int n_trials, double (&e)[6]) {
    const double e0 = a.sc->e_lin[5];
    int kacc = -1;
    for (int t = 1; t < n_trials && kacc < 0; ++t) {
        trial_energy_wave(a, PS_TRIAL + 5 * (t - 1), rest_blocks_of(a.d), e);
        if (e[5] <= e0) kacc = t;
    }
    return kacc;
}

// The log entry of a Gauss-Newton step (gn_iter >= 0) and the accepted
// trial's terms e (kacc >= 0), by one wavefront of one workgroup, before
// the next linearisation energy replaces e_lin.
__device__ void step_record(const LevelArgs &a, int gn_iter, int pcg_iters, int kacc,
                            const double (&e)[6]) {
    const int lane = threadIdx.x & 63;
    const int log_index = gn_iter >= 0 ? a.log_base + gn_iter : -1;
    const DevScalars *sc = a.sc;
    double rr = 0.0;
    if (log_index >= 0) {
        // ||r||^2 of the final PCG residual (node_blocks partials)
        const float *rrp = a.partials +
                           (long)(((pcg_iters & 1) ? PS_PCG1 : PS_PCG0) + 2) * a.max_blocks;
        double acc[1] = {0.0};
        strided_sums<1, 8>(lane, 64, node_blocks(a.d), [&](int, int b) { return rrp[b]; }, acc);
        rr = wave_sum_d(acc[0]);
    }
    if (lane != 0) return;
    const double e0 = sc->e_lin[5];
    if (kacc >= 0)
        for (int k = 0; k < 6; ++k) a.sc->e_trial[kacc][k] = e[k];
    if (log_index < 0) return;
    DevLog &Lg = a.log[log_index];
    Lg.level = a.level;
    Lg.gn_iter = gn_iter;
    Lg.energy = e0;
    Lg.e_photo = sc->e_lin[0];
    Lg.e_grad = sc->e_lin[1];
    Lg.e_smooth = sc->e_lin[2];
    Lg.e_epi = sc->e_lin[3];
    Lg.e_mag = sc->e_lin[4];
    Lg.energy_after = kacc >= 0 ? e[5] : e0;
    Lg.tau = kacc >= 0 ? ldexpf(1.f, -kacc) : 0.f;
    Lg.pcg_iters = pcg_iters;
    // an inactive last iteration left r unchanged
    const bool same = !sc->hist[pcg_iters].active && pcg_iters >= 2;
    Lg.pcg_res[pcg_iters - 1] = same ? Lg.pcg_res[pcg_iters - 2] : (float)sqrt(rr);
    Lg.n_valid = sc->n_valid;
}

// Trials tau = 1/2, 1/4, ... (n_rest of them), evaluated only if tau = 1
// was rejected: every workgroup first sums the tau = 1 partials itself and
// returns at once on acceptance.  Partials of trial t go to plane
// PS_TRIAL + 5 (t - 1).  spec (the tau = 1 energy came with the
// speculative linearisation at delta + dx): workgroup 0 records the
// verdict, and on acceptance the workgroups apply delta += dx (striding
// over the nodes) and workgroup 0 writes the step's log, which leaves the
// speculative records as the next step's linearisation.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_trials_rest(KArg<B> ka, int n_rest, int spec,
                                                          int gn_iter, int pcg_iters) {
    SF_BIND(ka);
    __shared__ NodeStage S;
    __shared__ int s_go;
    if (threadIdx.x < 64) {
        double e[6];
        trial_energy_wave(a, PS_E, energy_blocks_of(a.d), e);
        const int acc = e[5] <= a.sc->e_lin[5];
        if (threadIdx.x == 0) s_go = !acc;
        if (spec && bid == 0) {
            if (threadIdx.x == 0) a.sc->spec_acc = acc;
            if (acc) step_record(a, gn_iter, pcg_iters, 0, e);
        }
    }
    __syncthreads();
    if (!s_go) {
        if (spec) {
            float *delta = nvec(a, NV_DELTA);
            const float *dx = nvec(a, NV_X);
            for (long n = (long)bid * SF_BLOCK + threadIdx.x; n < a.d.G;
                 n += (long)nblk * SF_BLOCK) {
                float dl[6], x[6];
                ld6(delta, n, dl);
                ld6(dx, n, x);
#pragma unroll
                for (int q = 0; q < 6; ++q) dl[q] = dl[q] + x[q];
                st6(delta, n, dl);
            }
        }
        return;
    }
    const int n_tiles = energy_blocks_of(a.d);
    for (int t = 1; t <= n_rest; ++t) {
        const float tau = ldexpf(1.f, -t);
        float part[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        for (int tile = bid; tile < n_tiles; tile += nblk) energy_tile<false>(a, tile, tau, S, part);
        float tot5[5];
        block_sum<5>(part, tot5);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k)
                a.partials[(long)(PS_TRIAL + 5 * (t - 1) + k) * a.max_blocks + bid] = tot5[k];
        }
    }
}

// ---- node tiles ---------------------------------------------------------------
//
// A workgroup owns tx x ty warp nodes.  Its pixel region is every pixel whose
// bilinear bracket (Eq. (7)) contains one of its nodes.  Per-pixel values are
// staged in LDS; then the tpn threads of each node sum the node's support
// rows (weights alpha, or alpha^2 for diagonal entries) and combine their
// partial sums with fixed-order lane shuffles, so results are bitwise
// reproducible.  Neighbouring tiles recompute the shared border pixels.

struct TileGeom {
    int i0, j0, txa, tya;  // tile origin and clipped size
    int X0, X1, Y0, Y1;    // pixel region
    int RX, RY;
};

__device__ __forceinline__ TileGeom tile_geom(const LevelArgs &a, const TileCfg &t, int bid) {
    TileGeom g;
    const LevelDims &d = a.d;
    const int tx = tiles_x_of(d, t);
    g.i0 = (bid % tx) * t.tx;
    g.j0 = (bid / tx) * t.ty;
    g.txa = min(t.tx, d.Gx - g.i0);
    g.tya = min(t.ty, d.Gy - g.j0);
    g.X0 = sup_lo(g.i0, a.s);
    g.X1 = sup_hi(g.i0 + g.txa - 1, a.s, d.Gx, d.W);
    g.Y0 = sup_lo(g.j0, a.s);
    g.Y1 = sup_hi(g.j0 + g.tya - 1, a.s, d.Gy, d.H);
    g.RX = g.X1 - g.X0 + 1;
    g.RY = g.Y1 - g.Y0 + 1;
    return g;
}

// LDS carve-up of a node-tile kernel
// Records in LDS are whole 16-byte vectors so that a pixel's or a node's
// components move with one or two vector accesses (and rows of records
// spread over the banks): per-pixel values in records of KP floats (K
// rounded up to a multiple of 4), halo nodes in records of 8 floats, and
// each region column / row's bilinear bracket as one float4 (first node
// index as int bits, its weight, the next node's weight).
struct TileLds {
    float4 *bx, *by;  // brackets of region columns / rows
    int pitch;        // floats per row of records
    float *vals;      // RY rows of RX records of KP floats
    float *halo;      // (ty + 2) x (tx + 2) records of 8 floats
    float *ownd;      // 8 x tx x ty scratch per owned node (two partial
                      // products, then u of the previous iteration)
};

__host__ __device__ constexpr int rec_pad(int K) { return (K + 3) / 4 * 4; }
__host__ __device__ inline int tile_rxs(const TileCfg &t, int s) { return (t.tx + 1) * s + 2; }
__host__ __device__ inline int tile_rys(const TileCfg &t, int s) { return (t.ty + 1) * s + 2; }
// Row pitch (floats) of the per-pixel records: a multiple of 32 floats plus
// 4, so that the rows a node's threads read at one column fall on
// different 16-byte bank groups.
__host__ __device__ inline int tile_pitch(const TileCfg &t, int s, int K) {
    return (tile_rxs(t, s) * rec_pad(K) + 31) / 32 * 32 + 4;
}
__host__ __device__ inline size_t tile_lds_floats(const TileCfg &t, int s, int K) {
    const size_t RXs = tile_rxs(t, s), RYs = tile_rys(t, s);
    return 4 * RXs + 4 * RYs + (size_t)tile_pitch(t, s, K) * RYs +
           (size_t)8 * (t.tx + 2) * (t.ty + 2) + (size_t)8 * t.tx * t.ty;
}

__device__ TileLds tile_lds(float *lds, const TileCfg &t, int s, int K) {
    const int RXs = tile_rxs(t, s), RYs = tile_rys(t, s);
    TileLds L;
    L.bx = reinterpret_cast<float4 *>(lds);
    L.by = L.bx + RXs;
    L.pitch = tile_pitch(t, s, K);
    L.vals = reinterpret_cast<float *>(L.by + RYs);
    L.halo = L.vals + (size_t)L.pitch * RYs;
    L.ownd = L.halo + (size_t)8 * (t.tx + 2) * (t.ty + 2);
    return L;
}

// LDS of the block-assembly kernel: the bracket tables and, for each pixel
// of a tile's largest region ((n + 1) s pixels wide and high, one more for
// odd s), the 21 entries of its Gauss-Newton block (gram order) in a
// 22-float record of 8-byte pairs; the pixel's gradient stays in global
// memory.  Nothing else, so that more of its workgroups fit on a compute
// unit (four at stride 4).
#define BLK_REC 22
__host__ __device__ inline int blk_rxm(const TileCfg &t, int s) { return (t.tx + 1) * s + (s & 1); }
__host__ __device__ inline int blk_rym(const TileCfg &t, int s) { return (t.ty + 1) * s + (s & 1); }
__host__ __device__ inline int blk_pitch(const TileCfg &t, int s) {
    return (blk_rxm(t, s) * BLK_REC + 31) / 32 * 32 + 4;
}
__host__ __device__ inline size_t blk_lds_floats(const TileCfg &t, int s) {
    return 4 * (size_t)blk_rxm(t, s) + 4 * (size_t)blk_rym(t, s) +
           (size_t)blk_pitch(t, s) * blk_rym(t, s);
}
__device__ __forceinline__ void blk_rec_store(float *p, const float (&v)[21]) {
    float2 *p2 = reinterpret_cast<float2 *>(p);
#pragma unroll
    for (int m = 0; m < 10; ++m) p2[m] = make_float2(v[2 * m], v[2 * m + 1]);
    p[20] = v[20];
}
__device__ __forceinline__ void blk_rec_load(const float *p, float (&v)[21]) {
    const float2 *p2 = reinterpret_cast<const float2 *>(p);
#pragma unroll
    for (int m = 0; m < 10; ++m) {
        const float2 t2 = p2[m];
        v[2 * m] = t2.x;
        v[2 * m + 1] = t2.y;
    }
    v[20] = p[20];
}
__device__ TileLds blk_lds(float *lds, const TileCfg &t, int s) {
    TileLds L;
    L.bx = reinterpret_cast<float4 *>(lds);
    L.by = L.bx + blk_rxm(t, s);
    L.pitch = blk_pitch(t, s);
    L.vals = reinterpret_cast<float *>(L.by + blk_rym(t, s));
    L.halo = nullptr;
    L.ownd = nullptr;
    return L;
}

__device__ void tile_brackets(const LevelArgs &a, const TileGeom &g, const TileLds &L) {
    for (int u = threadIdx.x; u < g.RX; u += blockDim.x) {
        const Bracket b = bracket(g.X0 + u, a.s, a.d.Gx);
        L.bx[u] = make_float4(__int_as_float(b.i0), b.w0, b.w1, 0.f);
    }
    for (int u = threadIdx.x; u < g.RY; u += blockDim.x) {
        const Bracket b = bracket(g.Y0 + u, a.s, a.d.Gy);
        L.by[u] = make_float4(__int_as_float(b.i0), b.w0, b.w1, 0.f);
    }
}

// K floats of a record at p (16-byte aligned) / into a record
template <int K>
__device__ __forceinline__ void rec_load(const float *p, float (&v)[K]) {
    const float4 *p4 = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int m = 0; m < rec_pad(K) / 4; ++m) {
        const float4 t4 = p4[m];
        if (4 * m + 0 < K) v[4 * m + 0] = t4.x;
        if (4 * m + 1 < K) v[4 * m + 1] = t4.y;
        if (4 * m + 2 < K) v[4 * m + 2] = t4.z;
        if (4 * m + 3 < K) v[4 * m + 3] = t4.w;
    }
}
template <int K>
__device__ __forceinline__ void rec_store(float *p, const float (&v)[K]) {
    float4 *p4 = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int m = 0; m < rec_pad(K) / 4; ++m)
        p4[m] = make_float4(v[4 * m], 4 * m + 1 < K ? v[4 * m + 1] : 0.f,
                            4 * m + 2 < K ? v[4 * m + 2] : 0.f, 4 * m + 3 < K ? v[4 * m + 3] : 0.f);
}

// Block k of node n's record in the node-block layout (SF_BLK_STRIDE).
__device__ __forceinline__ void blk_load(const float *blk, long n, int k, float (&v)[21]) {
    const float *p = blk + n * SF_BLK_STRIDE;
    const float4 *p4 = reinterpret_cast<const float4 *>(p + 20 * k);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const float4 t4 = p4[m];
        v[4 * m] = t4.x;
        v[4 * m + 1] = t4.y;
        v[4 * m + 2] = t4.z;
        v[4 * m + 3] = t4.w;
    }
    v[20] = p[100 + k];
}
__device__ __forceinline__ void blk_store(float *blk, long n, int k, const float (&v)[21]) {
    float *p = blk + n * SF_BLK_STRIDE;
    float4 *p4 = reinterpret_cast<float4 *>(p + 20 * k);
#pragma unroll
    for (int m = 0; m < 5; ++m)
        p4[m] = make_float4(v[4 * m], v[4 * m + 1], v[4 * m + 2], v[4 * m + 3]);
    p[100 + k] = v[20];
}

// (unrolled so that the loads of several pixels are in flight together:
// one memory round trip per unrolled step instead of per pixel)
template <int K, class Fn>
__device__ __forceinline__ void pixels_to_lds(const TileGeom &g, const TileLds &L, Fn fn) {
    const int n = g.RX * g.RY;
    constexpr int U = K <= 12 ? 4 : 2;
    for (int u0 = threadIdx.x; u0 < n; u0 += U * blockDim.x) {
        float v[U][K];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            // past the region: reload its first pixel, not stored
            const int u = u0 + q * blockDim.x < n ? u0 + q * blockDim.x : 0;
            const int rx = u % g.RX, ry = u / g.RX;
            fn(g.X0 + rx, g.Y0 + ry, rx, ry, v[q]);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int u = u0 + q * blockDim.x;
            if (u < n) {
                const int rx = u % g.RX, ry = u / g.RX;
                rec_store<K>(L.vals + (size_t)ry * L.pitch + rx * rec_pad(K), v[q]);
            }
        }
    }
}

// weight of node i in a region column's / row's bracket
__device__ __forceinline__ float bweight(const float4 b, int i, int G) {
    if (G == 1) return b.y;
    const int i0 = __float_as_int(b.x);
    return (i0 == i ? b.y : 0.f) + (i0 + 1 == i ? b.z : 0.f);
}

// Sum over the support of this thread's node (valid in the thread with
// sub == 0 of each node group).  A node's support is at most 2S pixels wide
// and high, and tpn >= 2S, so every thread sums at most one support row,
// with the columns unrolled; the tpn row sums are combined with fixed-order
// lane shuffles.  TPN (= t.tpn) is a compile-time constant so that the
// shuffle sequence and the thread split fold to straight-line code.
template <int K, int S, int TPN>
__device__ __forceinline__ void lds_to_nodes(const LevelArgs &a, const TileCfg &t,
                                             const TileGeom &g, const TileLds &L,
                                             unsigned pow2, float (&acc)[K]) {
    (void)t;
    const int nl = threadIdx.x / TPN, sub = threadIdx.x % TPN;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.f;
    if (nl < g.txa * g.tya) {
        const int i = g.i0 + nl % g.txa, j = g.j0 + nl / g.txa;
        const int xa = max(sup_lo(i, S), g.X0) - g.X0;
        const int xb = min(sup_hi(i, S, a.d.Gx, a.d.W), g.X1) - g.X0;
        const int ya = max(sup_lo(j, S), g.Y0) - g.Y0;
        const int yb = min(sup_hi(j, S, a.d.Gy, a.d.H), g.Y1) - g.Y0;
        const int ry = ya + sub;
        if (ry <= yb) {
            const float wy = bweight(L.by[ry], j, a.d.Gy);
            const float *row = L.vals + (size_t)ry * L.pitch;
#pragma unroll
            for (int c = 0; c < 2 * S; ++c) {
                const int rx = xa + c;
                if (rx <= xb) {
                    const float w1 = bweight(L.bx[rx], i, a.d.Gx) * wy;
                    const float w2 = w1 * w1;
                    float v[K];
                    rec_load<K>(row + (size_t)rx * rec_pad(K), v);
#pragma unroll
                    for (int k = 0; k < K; ++k) acc[k] += (((pow2 >> k) & 1u) ? w2 : w1) * v[k];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = group_sum<float>(acc[k], TPN);
}

// Regulariser pieces of node (i, j).  The Gauss-Newton matrix of these
// least-squares terms is 2 J^T J:
//   smooth (Eq. (14), ordered 4-neighbour pairs on the deltas):
//     grad += 2 w_reg w_smooth w_f sum_j (w_i + w_j)(D_i - D_j)
//   epipolar (Eqs. (15)-(17), on totals): grad += 2 w_reg w_epi sum_t e_t de_t
//   magnitude (Eq. (18), on deltas): grad += 2 w_reg w_mag m_f D_i
// The right-hand-side kernel stores, per node, a 16-float record of the
// pieces the H-products need: the four smoothness coefficients
// 2 w_reg w_smooth (w_i + w_j) (0 without a neighbour) and the two epipolar
// gradients scaled by sqrt(2 w_reg w_epi), so that
//   (H_reg u)_i = sum_j c_j w_f (u_i - u_j) + sum_t J_t (J_t . u_i)
//                 + 2 w_reg w_mag m_f u_i.
#define REG_PLANES 16

__device__ __forceinline__ void nb_offset(int k, int &di, int &dj) {
    di = k == 0 ? 1 : (k == 1 ? -1 : 0);
    dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
}

// ---- right-hand side and diag(H) (node tiles) ----------------------------

// A node's own part of the right-hand-side kernels: its deltas, totals and
// neighbours (loaded before the pixel phase), then, from the data term's
// gradient and diagonal summed over its support, the regularisers, r, u,
// diag(H) and the regulariser record.
struct RhsNode {
    float dl[6], tot[6], dn[4][6], wn[4], wi = 0.f;
    int has[4];

    // delta + tau dx (tau != 0: a step the PCG's first kernel applies later)
    __device__ void load(const LevelArgs &a, int i, int j, long n, float tau = 0.f) {
        const LevelDims &d = a.d;
        const float *base = nvec(a, NV_BASE);
        const float *delta = nvec(a, NV_DELTA);
        const float *dx = nvec(a, NV_X);
        wi = a.wnode[n];
        float b[6];
        ld6(delta, n, dl);
        ld6(base, n, b);
        if (tau != 0.f) {
            float x[6];
            ld6(dx, n, x);
#pragma unroll
            for (int q = 0; q < 6; ++q) dl[q] = dl[q] + tau * x[q];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) tot[q] = b[q] + dl[q];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int di, dj;
            nb_offset(k, di, dj);
            has[k] = i + di >= 0 && i + di < d.Gx && j + dj >= 0 && j + dj < d.Gy;
            const long m = has[k] ? (long)(j + dj) * d.Gx + i + di : n;
            wn[k] = has[k] ? a.wnode[m] : 0.f;
            ld6(delta, m, dn[k]);
            if (tau != 0.f) {
                float x[6];
                ld6(dx, m, x);
#pragma unroll
                for (int q = 0; q < 6; ++q) dn[k][q] = dn[k][q] + tau * x[q];
            }
        }
    }

    // keep_x: the PCG solution still holds a deferred step (the PCG's first
    // kernel clears it)
    template <int S>
    __device__ void finish(const LevelArgs &a, int i, int j, long n, const float (&gdata)[6],
                           const float (&ddata)[6], bool keep_x = false) const {
        const DevConst &C = *a.cst;
        float grad[6], dg[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) { grad[q] = gdata[q]; dg[q] = ddata[q]; }
        const float cs = 2.f * C.w_reg * C.w_smooth;
        float cnb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cnb[k] = has[k] ? cs * (wi + wn[k]) : 0.f;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                grad[q] += cnb[k] * C.wf[q] * (dl[q] - dn[k][q]);
                dg[q] += cnb[k] * C.wf[q];
            }
        }
        float gx, gy;
        node_xy(i, j, S, gx, gy);
        float e[2], J[2][6];
        epi_terms(C.F[a.level], gx, gy, tot, e, J);
        const float ce = 2.f * C.w_reg * C.w_epi, cm = 2.f * C.w_reg * C.w_mag;
        const float se = sqrtf(ce);
        float rv[6], uv[6];
        const float zero[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            grad[q] += ce * (e[0] * J[0][q] + e[1] * J[1][q]) + cm * C.mf[q] * dl[q];
            dg[q] += ce * (J[0][q] * J[0][q] + J[1][q] * J[1][q]) + cm * C.mf[q];
            rv[q] = -grad[q];
            uv[q] = rv[q] / dg[q];
        }
        if (!keep_x) st6(nvec(a, NV_X), n, zero);
        st6(nvec(a, NV_R0), n, rv);
        st6(nvec(a, NV_U), n, uv);
        st6(nvec(a, NV_DIAG), n, dg);
        float4 *rg4 = reinterpret_cast<float4 *>(a.reg + n * REG_PLANES);
        rg4[0] = make_float4(cnb[0], cnb[1], cnb[2], cnb[3]);
        rg4[1] = make_float4(se * J[0][0], se * J[0][1], se * J[0][2], se * J[0][3]);
        rg4[2] = make_float4(se * J[0][4], se * J[0][5], se * J[1][0], se * J[1][1]);
        rg4[3] = make_float4(se * J[1][2], se * J[1][3], se * J[1][4], se * J[1][5]);
    }
};

// The energy at the linearisation point from n partials of plane PS_E
// (whole workgroup; valid after the call).
__device__ void lin_energy_scalars(const LevelArgs &a, int n) {
    const DevConst &C = *a.cst;
    double es[5];
    const float *p0 = a.partials + (long)PS_E * a.max_blocks;
    block_sum_planes<5>([&](int k) { return p0 + (long)k * a.max_blocks; }, n, es);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 5; ++k) a.sc->e_lin[k] = es[k];
        a.sc->e_lin[5] = (double)C.w_photo * es[0] + (double)C.w_grad * es[1] +
                         (double)C.w_reg * ((double)C.w_smooth * es[2] + (double)C.w_epi * es[3] +
                                            (double)C.w_mag * es[4]);
    }
}

// Workgroup 0 of a right-hand-side kernel: the energy at the linearisation
// point (the linearise kernel's partials; with_energy false: formed later,
// by the PCG's first kernel) and the PCG start state.
__device__ void rhs_level_scalars(const LevelArgs &a, bool with_energy = true) {
    if (with_energy) lin_energy_scalars(a, energy_blocks_of(a.d));
    if (threadIdx.x == 0) {
        PcgHist h0;
        h0.gamma = 0.0; h0.alpha = 0.f; h0.beta = 0.f; h0.active = 1; h0.pad = 0;
        a.sc->hist[0] = h0;
    }
}

template <bool B, int S>
__global__ __launch_bounds__(TileTraits<S>::NT) void k_rhs(KArg<B> ka, TileCfg t) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const TileGeom g = tile_geom(a, t, bid);
    const TileLds L = tile_lds(lds, t, S, 12);
    const int tid = threadIdx.x;
    constexpr int TPN = TileTraits<S>::TPN;
    const int nl = tid / TPN, sub = tid % TPN;
    const bool mine = sub == 0 && nl < g.txa * g.tya;
    const int i = g.i0 + (nl % max(g.txa, 1)), j = g.j0 + nl / max(g.txa, 1);
    const long n = (long)j * d.Gx + i;
    RhsNode nd;
    if (mine) nd.load(a, i, j, n);
    if (bid == 0) rhs_level_scalars(a);
    tile_brackets(a, g, L);
    pixels_to_lds<12>(g, L, [&](int x, int y, int, int, float (&v)[12]) {
        const long pix = (long)y * d.W + x;
        const float4 *rp = reinterpret_cast<const float4 *>(a.grad + pix * SF_GRAD_STRIDE);
        const float4 *gp = reinterpret_cast<const float4 *>(a.gram + pix * SF_GRAM_STRIDE);
        const float4 r0 = rp[0], r1 = rp[1], g0 = gp[0], g1 = gp[1];
        v[0] = r0.x; v[1] = r0.y; v[2] = r0.z; v[3] = r0.w; v[4] = r1.x; v[5] = r1.y;
        v[6] = g0.x; v[7] = g0.y; v[8] = g0.z; v[9] = g0.w; v[10] = g1.x; v[11] = g1.y;
    });
    __syncthreads();
    float acc[12];
    lds_to_nodes<12, S, TileTraits<S>::TPN>(a, t, g, L, 0xFC0u, acc);
    if (mine) {
        float gd[6], dd[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) { gd[q] = acc[q]; dd[q] = acc[6 + q]; }
        nd.finish<S>(a, i, j, n, gd, dd);
    }
}

// ---- per-node system-matrix blocks (node-block apply mode) -----------------
//
// The data term's Gauss-Newton matrix couples nodes that share a pixel's
// bilinear bracket (Eq. (7)): H_nm = sum_x a_n(x) a_m(x) G(x), symmetric
// since a_n a_m is a scalar and G(x) is symmetric, and H_mn = H_nm.  Node n
// stores the blocks of its pairs with itself and with the nodes E, S, SE
// and SW of it; the other four neighbours' blocks are the stored blocks of
// those neighbours.  The products a_n a_m are separable, so the thread of
// (node, support row r) sums the row's columns with the column weights
// bx_i bx_{i+di} for di = 0, +1, -1 and scales the three sums by the row
// weights by_j^2 (same row of nodes) and by_j by_{j+1} (next row).
// The same kernel forms the right-hand side: the data gradient is summed
// over the same support rows, and diag(H)'s data part is the diagonal of
// the self block.

// Assembly tile per stride: tx x ty nodes, tpn >= 2S threads per node, the
// pixel region's 27-float records (gradient, Gauss-Newton block) under
// 64 KB of LDS.
template <int S> struct BlkShape;
template <> struct BlkShape<1> { static constexpr int TX = 16, TY = 8, TPN = 2; };
template <> struct BlkShape<2> { static constexpr int TX = 16, TY = 4, TPN = 4; };
template <> struct BlkShape<3> { static constexpr int TX = 8, TY = 4, TPN = 8; };
template <> struct BlkShape<4> { static constexpr int TX = 8, TY = 2, TPN = 8; };
template <> struct BlkShape<5> { static constexpr int TX = 4, TY = 2, TPN = 16; };
template <> struct BlkShape<6> { static constexpr int TX = 2, TY = 2, TPN = 16; };
template <> struct BlkShape<7> { static constexpr int TX = 2, TY = 2, TPN = 16; };
template <> struct BlkShape<8> { static constexpr int TX = 2, TY = 1, TPN = 32; };
template <int S>
struct BlkTraits {
    static constexpr int NT = BlkShape<S>::TX * BlkShape<S>::TY * BlkShape<S>::TPN;
    static_assert(BlkShape<S>::TPN >= 2 * S && BlkShape<S>::TPN <= 64, "one support row per thread");
    static_assert(NT % 64 == 0 && NT <= 256, "whole wavefronts");
};

// partner offset of block type k (self, E, S, SE, SW)
__host__ __device__ inline void blk_offset(int k, int &di, int &dj) {
    di = (k == 1 || k == 3) ? 1 : (k == 4 ? -1 : 0);
    dj = k >= 2 ? 1 : 0;
}

// Pixel records of a node tile's region at delta + tau dx, formed in place
// of the linearisation kernel's (a rejected speculative step): the blocks
// into the tile's LDS, the gradients over the per-pixel gradient records
// in global memory (a pixel shared with a neighbouring tile gets the same
// value from both); and the energies of the pixels this tile owns: each
// pixel belongs to the tile of the node with the larger bilinear weight in
// each direction (the first on a tie), so every pixel is counted once.
template <int S>
__device__ void relin_pixels(const LevelArgs &a, const TileGeom &g, const TileLds &L, float tau,
                             float (&part)[5]) {
    const LevelDims &d = a.d;
    const float *base = nvec(a, NV_BASE);
    const float *delta = nvec(a, NV_DELTA);
    const float *dx = nvec(a, NV_X);
    const int n_px = g.RX * g.RY;
    for (int u = threadIdx.x; u < n_px; u += blockDim.x) {
        const int rx = u % g.RX, ry = u / g.RX;
        const int x = g.X0 + rx, y = g.Y0 + ry;
        const Bracket bx = bracket(x, S, d.Gx), by = bracket(y, S, d.Gy);
        float t[2][2][6];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const long m = (long)(cy ? by.i1 : by.i0) * d.Gx + (cx ? bx.i1 : bx.i0);
                float b[6], dl[6], xv[6];
                ld6(base, m, b);
                ld6(delta, m, dl);
                if (tau != 0.f) ld6(dx, m, xv);
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    float v = dl[q];
                    if (tau != 0.f) v = v + tau * xv[q];
                    t[cy][cx][q] = b[q] + v;
                }
            }
        float f[6];
#pragma unroll
        for (int q = 0; q < 6; ++q)
            f[q] = by.w0 * (bx.w0 * t[0][0][q] + bx.w1 * t[0][1][q]) +
                   by.w1 * (bx.w0 * t[1][0][q] + bx.w1 * t[1][1][q]);
        const long pix = (long)y * d.W + x;
        PixelOut o;
        pixel_terms<true>(a, x, y, f, a.cmask[pix] ? 1.f : 0.f, o);
        const int ox = bx.w1 > bx.w0 ? bx.i1 : bx.i0, oy = by.w1 > by.w0 ? by.i1 : by.i0;
        if (ox >= g.i0 && ox < g.i0 + g.txa && oy >= g.j0 && oy < g.j0 + g.tya) {
            part[0] += o.e_photo;
            part[1] += o.e_grad;
        }
        float v[21];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r; c < 6; ++c) v[gram_index(r, c)] = o.gram[tri(r, c)];
        blk_rec_store(L.vals + (size_t)ry * L.pitch + rx * BLK_REC, v);
        float4 *rp = reinterpret_cast<float4 *>(a.grad + pix * SF_GRAD_STRIDE);
        rp[0] = make_float4(o.grad[0], o.grad[1], o.grad[2], o.grad[3]);
        rp[1] = make_float4(o.grad[4], o.grad[5], 0.f, 0.f);
    }
}

// n_pend > 0: a speculative step precedes (the linearisation at
// delta + dx).  If its tau = 1 was accepted, delta has moved and the
// records are the ones to use.  Otherwise every workgroup chooses the step
// length from the shorter trials (as k_accept does), workgroup 0 writes
// that step's log (gn_prev), and the tile forms its records, the right-hand
// side and the energy partials at delta + tau dx itself; delta and the
// energy sum follow in the PCG's first kernel, which also clears dx.
template <bool B, int S>
__global__ __launch_bounds__(BlkTraits<S>::NT) void k_rhs_blocks(KArg<B> ka, TileCfg t,
                                                                 int n_pend, int gn_prev,
                                                                 int pcg_iters) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const TileGeom g = tile_geom(a, t, bid);
    const TileLds L = blk_lds(lds, t, S);
    constexpr int TPN = BlkShape<S>::TPN;
    const int nl = threadIdx.x / TPN, sub = threadIdx.x % TPN;
    const bool valid = nl < g.txa * g.tya;
    const bool mine = valid && sub == 0;
    const int i = g.i0 + nl % max(g.txa, 1), j = g.j0 + nl / max(g.txa, 1);
    const long n = (long)j * d.Gx + i;
    __shared__ int s_k;
    const bool redo = n_pend > 0 && !a.sc->spec_acc;
    float tau = 0.f;
    if (redo) {
        if (threadIdx.x < 64) {
            double e[6];
            const int kacc = rest_decision(a, n_pend, e);
            if (threadIdx.x == 0) s_k = kacc;
            if (bid == 0) step_record(a, gn_prev, pcg_iters, kacc, e);
        }
        __syncthreads();
        tau = s_k >= 0 ? ldexpf(1.f, -s_k) : 0.f;
        if (bid == 0 && threadIdx.x == 0) {
            a.sc->spec_tau = tau;
            a.sc->lin_n = nblk;
        }
    }
    RhsNode nd;
    if (mine && !redo) nd.load(a, i, j, n);
    if (bid == 0) rhs_level_scalars(a, !redo);
    tile_brackets(a, g, L);
    if (redo) {
        float part[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        relin_pixels<S>(a, g, L, tau, part);
        if (mine) {
            float pn[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            node_energy(a, (int)n, tau, pn);
#pragma unroll
            for (int k = 2; k < 5; ++k) part[k] += pn[k];
        }
        float tot5[5];
        block_sum<5>(part, tot5);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) a.partials[(long)(PS_E + k) * a.max_blocks + bid] = tot5[k];
        }
        if (mine) nd.load(a, i, j, n, tau);
    } else {
        // the region's blocks into LDS, two pixels in flight per thread
        const int n_px = g.RX * g.RY;
        for (int u0 = threadIdx.x; u0 < n_px; u0 += 2 * blockDim.x) {
            float v[2][21];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                // past the region: reload its first pixel, not stored
                const int u = u0 + q * blockDim.x < n_px ? u0 + q * blockDim.x : 0;
                const long pix = (long)(g.Y0 + u / g.RX) * d.W + g.X0 + u % g.RX;
                const float4 *gp = reinterpret_cast<const float4 *>(a.gram + pix * SF_GRAM_STRIDE);
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    const float4 t4 = gp[m];
                    v[q][4 * m] = t4.x; v[q][4 * m + 1] = t4.y;
                    v[q][4 * m + 2] = t4.z; v[q][4 * m + 3] = t4.w;
                }
                v[q][20] = gp[5].x;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int u = u0 + q * blockDim.x;
                if (u < n_px)
                    blk_rec_store(L.vals + (size_t)(u / g.RX) * L.pitch + (u % g.RX) * BLK_REC, v[q]);
            }
        }
    }
    // the redo's gradient stores are read back below by other wavefronts
    // of this workgroup
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    float gs[6], c0[21], cp[21], cm[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) gs[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 21; ++k) c0[k] = cp[k] = cm[k] = 0.f;
    float r_same = 0.f, r_next = 0.f;
    if (valid) {
        const int xa = max(sup_lo(i, S), g.X0) - g.X0;
        const int xb = min(sup_hi(i, S, d.Gx, d.W), g.X1) - g.X0;
        const int ya = max(sup_lo(j, S), g.Y0) - g.Y0;
        const int yb = min(sup_hi(j, S, d.Gy, d.H), g.Y1) - g.Y0;
        const int ry = ya + sub;
        if (ry <= yb) {
            const float4 byr = L.by[ry];
            const float vj = bweight(byr, j, d.Gy);
            const float vn = j + 1 < d.Gy ? bweight(byr, j + 1, d.Gy) : 0.f;
            r_same = vj * vj;
            r_next = vj * vn;
            const float *row = L.vals + (size_t)ry * L.pitch;
            const float4 *grow = reinterpret_cast<const float4 *>(
                a.grad + ((long)(g.Y0 + ry) * d.W + g.X0) * SF_GRAD_STRIDE);
#pragma unroll
            for (int c = 0; c < 2 * S; ++c) {
                const int rx = xa + c;
                if (rx <= xb) {
                    const float4 b = L.bx[rx];
                    const float wi = bweight(b, i, d.Gx);
                    const float wp = i + 1 < d.Gx ? bweight(b, i + 1, d.Gx) : 0.f;
                    const float wm = i >= 1 ? bweight(b, i - 1, d.Gx) : 0.f;
                    const float w1 = wi * vj;
                    const float a0 = wi * wi, ap = wi * wp, am = wi * wm;
                    const float4 g0 = grow[2 * rx], g1 = grow[2 * rx + 1];
                    const float gv[6] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y};
                    float v[21];
                    blk_rec_load(row + (size_t)rx * BLK_REC, v);
#pragma unroll
                    for (int k = 0; k < 6; ++k) gs[k] += w1 * gv[k];
#pragma unroll
                    for (int k = 0; k < 21; ++k) {
                        c0[k] += a0 * v[k];
                        cp[k] += ap * v[k];
                        cm[k] += am * v[k];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) gs[k] = group_sum<float>(gs[k], TPN);
    float sd[6];
#pragma unroll
    for (int kb = 0; kb < SF_BLK_TYPES; ++kb) {
        const float rw = kb < 2 ? r_same : r_next;
        float o[21];
#pragma unroll
        for (int k = 0; k < 21; ++k) {
            const float src = (kb == 0 || kb == 2) ? c0[k] : ((kb == 4) ? cm[k] : cp[k]);
            o[k] = group_sum<float>(rw * src, TPN);
        }
        if (kb == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q) sd[q] = o[gram_index(q, q)];
        }
        if (valid && sub == kb % TPN) blk_store(a.blk, n, kb, o);
    }
    if (mine) nd.finish<S>(a, i, j, n, gs, sd, redo);
}

// ---- preconditioned CG in single-reduction form --------------------------
//
// Iteration k (x_0 = 0, r_0 = b, u_0 = M^-1 r_0, w_0 = H u_0, M = diag H):
//   p_k = u_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}   (s_k = H p_k)
//   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k
//   u_{k+1} = M^-1 r_{k+1},  w_{k+1} = H u_{k+1}
//   gamma_k = r_k.u_k, delta_k = w_k.u_k (one fused reduction),
//   beta_k = gamma_k / gamma_{k-1},
//   alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
// which are the iterates of textbook PCG in exact arithmetic, with one
// H-product and one global reduction per iteration.  Kernel i (1 <= i < n)
// forms the scalars of iteration i-1 from kernel i-1's partial sums (every
// workgroup sums them in the same order), applies iteration i-1 and computes
// w_i; the first kernel computes w_0, the last one applies iteration n-1.
// Breakdown: once gamma <= 1e-30 or the curvature p.Hp <= 0 the remaining
// iterations change nothing.


// Per-lane strided sums of the previous iteration's three partial planes;
// every wavefront of every workgroup loads and sums all of them in the same
// order.
// Up to 512 workgroups, eight scalar loads per plane and lane take one
// memory round trip.  Beyond (the level-0 iteration at 640x480 has 600),
// each lane reads four consecutive partials at a time (the planes start on
// 16-byte boundaries: max_blocks is a multiple of 4): three 16-byte loads
// per plane and lane cover 768 workgroups in one round trip instead of two.
__device__ __forceinline__ void load_pcg_partials(const LevelArgs &a, int i, int nb_prev,
                                                  double (&acc)[3]) {
    const float *prev = a.partials + (long)(((i - 1) & 1) ? PS_PCG1 : PS_PCG0) * a.max_blocks;
    constexpr int U = 3;
    const int lane = threadIdx.x & 63;
    acc[0] = acc[1] = acc[2] = 0.0;
    if (nb_prev <= 64 * 8) {
        strided_sums<3, 8>(lane, 64, nb_prev,
                           [&](int k, int b) { return prev[(long)k * a.max_blocks + b]; }, acc);
        return;
    }
    const int nq = (nb_prev + 3) >> 2;  // float4 groups holding the nb_prev partials
    for (int j0 = lane; j0 < nq; j0 += 64 * U) {
        float4 v[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + 64 * u;
            const int jj = j < nq ? j : 0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                v[u][k] = reinterpret_cast<const float4 *>(prev + (long)k * a.max_blocks)[jj];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = 4 * (j0 + 64 * u);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc[k] += b < nb_prev ? (double)v[u][k].x : 0.0;
                acc[k] += b + 1 < nb_prev ? (double)v[u][k].y : 0.0;
                acc[k] += b + 2 < nb_prev ? (double)v[u][k].z : 0.0;
                acc[k] += b + 3 < nb_prev ? (double)v[u][k].w : 0.0;
            }
        }
    }
}

// The scalars of iteration i-1 from the lane sums: every wavefront reduces
// the same values in the same order and decides alike, so no workgroup
// barrier is needed.  `rec` and `rr` are recorded by workgroup 0 at the end
// of the kernel (record_decision), after its last barrier, so that no
// barrier waits for those stores.
__device__ void pcg_decide(int i, const double (&acc)[3], const PcgHist &h, int force,
                           float &alpha, float &beta, int &act, PcgHist &rec, double &rr) {
    const double gam = wave_sum_d(acc[0]), del = wave_sum_d(acc[1]);
    rr = wave_sum_d(acc[2]);
    double b = 0.0, pq = del;
    int ok = h.active;
    if (ok && i - 1 > 0) {
        b = gam / h.gamma;
        pq = del - b * gam / (double)h.alpha;
    }
    ok = ok && gam > 1e-30 && pq > 0.0 && isfinite(pq);
    float al = ok ? (float)(gam / pq) : 0.f;
    float be = ok ? (float)b : 0.f;
    if (force) { ok = 1; al = 1e-3f; be = 0.5f; }
    rec.gamma = gam; rec.alpha = al; rec.beta = be; rec.active = ok; rec.pad = 0;
    alpha = al;
    beta = be;
    act = ok;
}

__device__ __forceinline__ void record_decision(const LevelArgs &a, int i, int log_index,
                                                const PcgHist &rec, double rr) {
    a.sc->hist[i] = rec;
    if (log_index >= 0 && i >= 2) a.log[log_index].pcg_res[i - 2] = (float)sqrt(rr);
}

// Copies this workgroup's partials to the next slot (inactive iteration:
// r and u are unchanged).
__device__ void carry_partials(const LevelArgs &a, int bid, int i) {
    if (threadIdx.x < 3) {
        const long src = (long)(((i - 1) & 1) ? PS_PCG1 : PS_PCG0) * a.max_blocks;
        const long dst = (long)((i & 1) ? PS_PCG1 : PS_PCG0) * a.max_blocks;
        a.partials[dst + (long)threadIdx.x * a.max_blocks + bid] =
            a.partials[src + (long)threadIdx.x * a.max_blocks + bid];
    }
}

// Block products of a node in the node-block mode, split over its four
// threads: task q of thread `sub` is block type k (-1: none); with `own` it
// is the node's block of type k times u at the partner n + off(k), else the
// block of type k stored by n - off(k) (whose partner is n) times u there.
// Together: H_nn u_n + sum over the eight neighbours m of H_nm u_m.
__device__ __forceinline__ void nb_task(int sub, int q, int &k, bool &own) {
    if (q == 0) k = sub == 0 ? 0 : (sub == 2 ? 4 : 2);
    else if (q == 1) k = (sub & 1) ? 3 : 1;
    else k = sub == 3 ? 4 : -1;
    own = sub < 2 || (sub == 2 && q == 0);
}

// Every load of an iteration that does not depend on its scalars is issued
// before the partial sums are reduced, and constants are read once, so the
// workgroup waits for memory about once.
// Deferred step of a rejected speculative tau = 1 (see k_rhs_blocks), for
// the PCG's first kernel: delta += tau dx on node n with the step length
// the right-hand-side kernel chose.
__device__ __forceinline__ void deferred_step(const LevelArgs &a, long n, float tau) {
    if (tau == 0.f) return;
    float *delta = nvec(a, NV_DELTA);
    float dl[6], x[6];
    ld6(delta, n, dl);
    ld6(nvec(a, NV_X), n, x);
#pragma unroll
    for (int q = 0; q < 6; ++q) dl[q] = dl[q] + tau * x[q];
    st6(delta, n, dl);
}

// force: later iterations are applied even if inactive (kernel timing);
// in the first kernel (node-block form) it means that a speculative step
// precedes, whose deferred part (if tau = 1 was rejected) happens here.
// Single-frame iteration launches of more tiles than this reduce the
// previous iteration's partial sums in wavefront 0 (WD; batched launches
// always do).
#define SF_WD_TILES 256
// Single-frame node-block iteration launches of more threads than this
// (two wavefronts per SIMD of the device) load their operands where they
// are used (LATE; batched launches always do).
#define SF_LATE_THREADS (2 * 64 * 1024)

template <bool B, bool FIRST, int S, int V, bool WD, bool LATE>
__global__ __launch_bounds__((TileTraits<S, V>::NT)) void k_pcg(KArg<B> ka, TileCfg t, int i,
                                                              int gn, int force) {
    constexpr int NT_TILE = TileTraits<S, V>::NT;
    constexpr int PPT = TileTraits<S, V>::PPT;
    extern __shared__ __attribute__((aligned(16))) float lds[];
    SF_BIND(ka);
    const int nb_prev = nblk;  // the previous iteration ran on the same tiles
    const int log_index = gn >= 0 ? a.log_base + gn : -1;
    const LevelDims &d = a.d;
    const TileGeom g = tile_geom(a, t, bid);
    const TileLds L = tile_lds(lds, t, S, 6);
    const int tid = threadIdx.x;
    const float *Rp = nvec(a, ((i - 1) & 1) ? NV_R1 : NV_R0);
    float *Rc = nvec(a, (i & 1) ? NV_R1 : NV_R0);
    const float *Wp = nvec(a, ((i - 1) & 1) ? NV_W1 : NV_W0);
    float *Wc = nvec(a, (i & 1) ? NV_W1 : NV_W0);
    const float *Sp = nvec(a, ((i - 2) & 1) ? NV_S1 : NV_S0);
    float *Sc = nvec(a, ((i - 1) & 1) ? NV_S1 : NV_S0);
    float *U = nvec(a, NV_U);
    float *P = nvec(a, NV_P);
    float *X = nvec(a, NV_X);
    const float *D = nvec(a, NV_DIAG);
    const float *R0 = nvec(a, NV_R0);

    // ---- phase 0: loads --------------------------------------------------
    float wf[6], cm[6];
    {
        const DevConst *C = a.cst;
        const float c = 2.f * C->w_reg * C->w_mag;
#pragma unroll
        for (int q = 0; q < 6; ++q) { wf[q] = C->wf[q]; cm[q] = c * C->mf[q]; }
    }
    double pacc[3] = {0.0, 0.0, 0.0};
    PcgHist h;
    h.gamma = 0.0; h.alpha = 0.f; h.beta = 0.f; h.active = 1; h.pad = 0;
    // WD (many partial sums: batched launches, single-frame launches of more
    // than SF_WD_TILES tiles): wavefront 0 reduces them and decides, the
    // others read the scalars from LDS after a barrier, instead of every
    // wavefront loading every partial.  Few partials: each wavefront
    // decides itself, which spares the barrier.  Either way every thread
    // gets the same scalars.
    constexpr bool w0_decides = WD;
    if (!FIRST) {
        if (!w0_decides || tid < 64) load_pcg_partials(a, i, nb_prev, pacc);
        h = a.sc->hist[i - 1];
    }
    // owned node of this thread's node group
    const int HX = t.tx + 2;
    constexpr int TPN = TileTraits<S, V>::TPN;
    const int nl = tid / TPN, sub = tid % TPN;
    const bool mine = sub == 0 && nl < g.txa * g.tya;
    const int ti = nl % max(g.txa, 1), tj = nl / max(g.txa, 1);
    const int i_n = g.i0 + ti, j_n = g.j0 + tj;
    const long n_own = (long)j_n * d.Gx + i_n;
    if (FIRST && S == 0 && force && !a.sc->spec_acc) {
        if (mine) {
            deferred_step(a, n_own, a.sc->spec_tau);
            const float zero[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            st6(X, n_own, zero);
        }
        if (bid == 0) lin_energy_scalars(a, a.sc->lin_n);
    }
    // S > 0: Gram blocks of this thread's region pixels; S = 0: the node
    // blocks of this thread's share of its node's nine block products, and
    // the halo records of the u they multiply (-1: no such neighbour).
    // Small single-frame launches load the blocks here, with the other loads
    // that do not depend on the scalars (one memory round trip).  Batched
    // launches, whose speed follows how many workgroups fit on a CU, load
    // each block just before its product (and the regulariser record and
    // the owned node's vectors where they are used): 96 instead of 154
    // registers (93 instead of 120 for the first kernel), five wavefronts
    // per SIMD instead of three.  Large single-frame launches (LATE) load
    // the blocks and the regulariser record late: 106 instead of 158
    // registers, four wavefronts instead of three.
    constexpr bool late = B || LATE;
    const int npx = S > 0 ? g.RX * g.RY : 0;
    float Gm[PPT][SF_GRAM_STRIDE];
    float Bk[3][21];
    int bu[3] = {-1, -1, -1};
    long bo[3] = {0, 0, 0};  // batched: the owner of each task's block
    int bt[3] = {0, 0, 0};   // and its type
    if constexpr (S > 0) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int u = tid + k * NT_TILE;
            if (u < npx) {
                const long pix = (long)(g.Y0 + u / g.RX) * d.W + g.X0 + u % g.RX;
                const float4 *gp = reinterpret_cast<const float4 *>(a.gram + pix * SF_GRAM_STRIDE);
#pragma unroll
                for (int v = 0; v < 6; ++v) {
                    const float4 t4 = gp[v];
                    Gm[k][4 * v] = t4.x;
                    Gm[k][4 * v + 1] = t4.y;
                    Gm[k][4 * v + 2] = t4.z;
                    Gm[k][4 * v + 3] = t4.w;
                }
            }
        }
    } else {
        const bool valid = nl < g.txa * g.tya;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            int k, di, dj;
            bool own;
            nb_task(sub, q, k, own);
            blk_offset(k, di, dj);
            const int pi = own ? i_n + di : i_n - di, pj = own ? j_n + dj : j_n - dj;
            if (valid && k >= 0 && pi >= 0 && pi < d.Gx && pj >= 0 && pj < d.Gy) {
                bu[q] = (tj + 1 + pj - j_n) * HX + (ti + 1 + pi - i_n);
                const long owner = own ? n_own : (long)pj * d.Gx + pi;
                if (late) {
                    bo[q] = owner;
                    bt[q] = k;
                } else {
                    blk_load(a.blk, owner, k, Bk[q]);
                }
            }
        }
    }
    // halo node of this thread: the vectors u_i is formed from
    const int hx0 = max(g.i0 - 1, 0), hx1 = min(g.i0 + g.txa, d.Gx - 1);
    const int hy0 = max(g.j0 - 1, 0), hy1 = min(g.j0 + g.tya, d.Gy - 1);
    const int hw = hx1 - hx0 + 1, hh = hy1 - hy0 + 1;
    const bool hal = tid < hw * hh;
    const int hni = hx0 + tid % max(hw, 1), hnj = hy0 + tid / max(hw, 1);
    const long hn = (long)hnj * d.Gx + hni;
    const bool hown = hal && hni >= g.i0 && hni < g.i0 + g.txa && hnj >= g.j0 && hnj < g.j0 + g.tya;
    float hv0[6], hv1[6], hv2[6], hv3[6];
    if (hal) {
        if (FIRST) {
            ld6(U, hn, hv0);
            ld6(R0, hn, hv1);
        } else {
            ld6(Rp, hn, hv0);
            ld6(Wp, hn, hv1);
            if (i > 1) {
                ld6(Sp, hn, hv2);
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q) hv2[q] = 0.f;
            }
            ld6(D, hn, hv3);
        }
    }
    // the owned node's regulariser record (batched launches: where it is
    // used, as their blocks)
    float rg[REG_PLANES];
    auto load_rg = [&]() {
#pragma unroll
        for (int k = 0; k < REG_PLANES / 4; ++k) {
            const float4 t4 = reinterpret_cast<const float4 *>(a.reg + n_own * REG_PLANES)[k];
            rg[4 * k] = t4.x;
            rg[4 * k + 1] = t4.y;
            rg[4 * k + 2] = t4.z;
            rg[4 * k + 3] = t4.w;
        }
    };
    if (mine && !late) load_rg();
    // the owned node's u, p and x: read here in single-frame launches (one
    // fewer dependent memory round trip, same occupancy); batched launches,
    // which stream from HBM, read them just before the final reduction to
    // keep the register count (and occupancy) lower
    // (u of iteration i-1: read here in single-frame launches; batched
    // launches, which stream from HBM, rebuild it as r / diag from the halo
    // records they read anyway, bitwise the same value, and neither read
    // nor write the u vector)
    float uo[6], po[6], xo[6];
    auto load_own = [&]() {
        if (mine && !FIRST) {
            if (!B) ld6(U, n_own, uo);
            ld6(X, n_own, xo);
            if (i > 1) {
                ld6(P, n_own, po);
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q) po[q] = 0.f;
            }
        }
    };
    if (!B) load_own();

    // ---- phase 1: scalars of iteration i-1 ---------------------------------
    if constexpr (S > 0) tile_brackets(a, g, L);
    float alpha = 0.f, beta = 0.f;
    int act = 1;
    PcgHist rec;
    double rr_prev = 0.0;
    if (!FIRST) {
        if (w0_decides) {
            __shared__ float s_ab[2];
            __shared__ int s_act;
            if (tid < 64) {
                pcg_decide(i, pacc, h, force, alpha, beta, act, rec, rr_prev);
                if (tid == 0) {
                    s_ab[0] = alpha;
                    s_ab[1] = beta;
                    s_act = act;
                }
            }
            __syncthreads();
            alpha = s_ab[0];
            beta = s_ab[1];
            act = s_act;
        } else {
            pcg_decide(i, pacc, h, force, alpha, beta, act, rec, rr_prev);
        }
        if (!act) {
            carry_partials(a, bid, i);
            if (bid == 0 && tid == 0) record_decision(a, i, log_index, rec, rr_prev);
            return;
        }
    }

    // ---- phase 2: u_i on the tile and its halo -----------------------------
    float ru = 0.f, rr = 0.f, sv6[6], rn6[6], uh[6];
    if (hal) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            float uu, rn;
            if (FIRST) {
                uu = hv0[q];
                rn = hv1[q];
            } else {
                sv6[q] = i > 1 ? hv1[q] + beta * hv2[q] : hv1[q];
                rn = hv0[q] - alpha * sv6[q];
                uu = rn / hv3[q];
            }
            rn6[q] = rn;
            uh[q] = uu;
            ru += rn * uu;
            rr += rn * rn;
        }
        rec_store<6>(L.halo + (size_t)((hnj - g.j0 + 1) * HX + (hni - g.i0 + 1)) * 8, uh);
        if (hown) {
            const int o = (hnj - g.j0) * t.tx + (hni - g.i0);
            L.ownd[o] = ru;
            L.ownd[t.tx * t.ty + o] = rr;
            if (B && !FIRST) {
                // u of iteration i-1 of this owned node, r / diag as the
                // previous kernel formed it (bitwise), for its p update
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    L.ownd[(2 + q) * t.tx * t.ty + o] = hv0[q] / hv3[q];
            }
        }
    }
    __syncthreads();

    // ---- phase 3: per-pixel block times the interpolated u_i ---------------
    if constexpr (S > 0) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int u = tid + k * NT_TILE;
        if (u < npx) {
            const int rx = u % g.RX, ry = u / g.RX;
            const float4 bxr = L.bx[rx], byr = L.by[ry];
            const int bx0 = __float_as_int(bxr.x), by0 = __float_as_int(byr.x);
            const float wx0 = bxr.y, wx1 = bxr.z, wy0 = byr.y, wy1 = byr.z;
            const int lx0 = bx0 - g.i0 + 1, lx1 = (d.Gx == 1 ? bx0 : bx0 + 1) - g.i0 + 1;
            const int ly0 = by0 - g.j0 + 1, ly1 = (d.Gy == 1 ? by0 : by0 + 1) - g.j0 + 1;
            float c00[6], c01[6], c10[6], c11[6];
            rec_load<6>(L.halo + (size_t)(ly0 * HX + lx0) * 8, c00);
            rec_load<6>(L.halo + (size_t)(ly0 * HX + lx1) * 8, c01);
            rec_load<6>(L.halo + (size_t)(ly1 * HX + lx0) * 8, c10);
            rec_load<6>(L.halo + (size_t)(ly1 * HX + lx1) * 8, c11);
            float pv[6];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                pv[q] = wy0 * (wx0 * c00[q] + wx1 * c01[q]) + wy1 * (wx0 * c10[q] + wx1 * c11[q]);
            float hv[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                float acc = 0.f;
#pragma unroll
                for (int c = 0; c < 6; ++c) acc += Gm[k][gram_index(r, c)] * pv[c];
                hv[r] = acc;
            }
            rec_store<6>(L.vals + (size_t)ry * L.pitch + rx * 8, hv);
        }
    }
    __syncthreads();
    }

    // ---- phase 4: sums onto nodes, regularisers ----------------------------
    float acc[6];
    if constexpr (S > 0) {
        lds_to_nodes<6, S, TileTraits<S, V>::TPN>(a, t, g, L, 0u, acc);
    } else {
        // the node's block products, summed over its threads in fixed order
#pragma unroll
        for (int r = 0; r < 6; ++r) acc[r] = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (bu[q] >= 0) {
                float un[6];
                if (late) blk_load(a.blk, bo[q], bt[q], Bk[q]);
                rec_load<6>(L.halo + (size_t)bu[q] * 8, un);
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = 0; c < 6; ++c) acc[r] += Bk[q][gram_index(r, c)] * un[c];
            }
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) acc[r] = group_sum<float>(acc[r], TileTraits<S, V>::TPN);
    }
    float prt[3] = {0.f, 0.f, 0.f};
    float w6[6], uv[6];
    if (mine) {
        if (late) load_rg();
        rec_load<6>(L.halo + (size_t)((tj + 1) * HX + ti + 1) * 8, uv);
        float jp0 = 0.f, jp1 = 0.f;
#pragma unroll
        for (int q = 0; q < 6; ++q) { jp0 += rg[4 + q] * uv[q]; jp1 += rg[10 + q] * uv[q]; }
        float sm[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // neighbours outside the grid have coefficient 0 and no halo
        // record: they read the node's own record (adding exactly 0), so
        // the four loads issue together
        float un[4][6];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int di, dj;
            nb_offset(k, di, dj);
            if (rg[k] == 0.f) di = dj = 0;
            rec_load<6>(L.halo + (size_t)((tj + 1 + dj) * HX + ti + 1 + di) * 8, un[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 6; ++q) sm[q] += rg[k] * (uv[q] - un[k][q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            w6[q] = acc[q] + wf[q] * sm[q] + rg[4 + q] * jp0 + rg[10 + q] * jp1 + cm[q] * uv[q];
            prt[1] += w6[q] * uv[q];
        }
        const int o = tj * t.tx + ti;
        prt[0] = L.ownd[o];
        prt[2] = L.ownd[t.tx * t.ty + o];
    }
    float tot3[3];
    if (B) load_own();
    if (B && mine && !FIRST) {
        const int o = tj * t.tx + ti;
#pragma unroll
        for (int q = 0; q < 6; ++q) uo[q] = L.ownd[(2 + q) * t.tx * t.ty + o];
    }
    block_sum<3, false>(prt, tot3);

    // ---- stores ---------------------------------------------------------------
    if (hown && !FIRST) {
        st6(Sc, hn, sv6);
        st6(Rc, hn, rn6);
    }
    if (mine) {
        st6(Wc, n_own, w6);
        if (!FIRST) {
            float pn[6], xn[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                pn[q] = i > 1 ? uo[q] + beta * po[q] : uo[q];
                xn[q] = xo[q] + alpha * pn[q];
            }
            st6(P, n_own, pn);
            st6(X, n_own, xn);
            if (!B) st6(U, n_own, uv);
        }
    }
    if (tid == 0) {
        const long dst = (long)((i & 1) ? PS_PCG1 : PS_PCG0) * a.max_blocks;
        for (int k = 0; k < 3; ++k) a.partials[dst + (long)k * a.max_blocks + bid] = tot3[k];
        if (!FIRST && bid == 0) record_decision(a, i, log_index, rec, rr_prev);
    }
}

// Applies iteration n-1 (no H-product) and leaves ||r_n||^2 partials.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_pcg_last(KArg<B> ka, TileCfg t, int n_it,
                                                       int gn, int force) {
    SF_BIND(ka);
    const int nb_prev = node_tiles_of(a.d, t);
    const int log_index = gn >= 0 ? a.log_base + gn : -1;
    const int i = n_it;
    const float *Rp = nvec(a, ((i - 1) & 1) ? NV_R1 : NV_R0);
    float *Rc = nvec(a, (i & 1) ? NV_R1 : NV_R0);
    const float *Wp = nvec(a, ((i - 1) & 1) ? NV_W1 : NV_W0);
    const float *Sp = nvec(a, ((i - 2) & 1) ? NV_S1 : NV_S0);
    const float *D = nvec(a, NV_DIAG);
    float *P = nvec(a, NV_P);
    float *X = nvec(a, NV_X);
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    const bool in = n < a.d.G;
    double pacc[3];
    load_pcg_partials(a, i, nb_prev, pacc);
    const PcgHist h = a.sc->hist[i - 1];
    float rp[6], wp[6], sp[6], up[6], pp[6], xp[6];
    if (in) {
        ld6(Rp, n, rp);
        ld6(Wp, n, wp);
        // u of iteration n-1 (batched: r / diag, bitwise as the iteration
        // kernel formed it, which does not store u there)
        if (B) {
            float dg[6];
            ld6(D, n, dg);
#pragma unroll
            for (int q = 0; q < 6; ++q) up[q] = rp[q] / dg[q];
        } else {
            ld6(nvec(a, NV_U), n, up);
        }
        ld6(X, n, xp);
        if (i > 1) {
            ld6(Sp, n, sp);
            ld6(P, n, pp);
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) sp[q] = pp[q] = 0.f;
        }
    }
    float alpha, beta;
    int act;
    PcgHist rec;
    double rr_prev;
    pcg_decide(i, pacc, h, force, alpha, beta, act, rec, rr_prev);
    float prt[1] = {0.f};
    if (in) {
        float rn[6], pn[6], xn[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            rn[q] = rp[q];
            if (act) {
                const float sv = i > 1 ? wp[q] + beta * sp[q] : wp[q];
                pn[q] = i > 1 ? up[q] + beta * pp[q] : up[q];
                xn[q] = xp[q] + alpha * pn[q];
                rn[q] = rn[q] - alpha * sv;
            }
            prt[0] += rn[q] * rn[q];
        }
        if (act) {
            st6(P, n, pn);
            st6(X, n, xn);
        }
        st6(Rc, n, rn);
    }
    float tot1[1];
    block_sum<1, false>(prt, tot1);
    if (threadIdx.x == 0) {
        a.partials[(long)(((i & 1) ? PS_PCG1 : PS_PCG0) + 2) * a.max_blocks + bid] = tot1[0];
        if (bid == 0) record_decision(a, i, log_index, rec, rr_prev);
    }
}

#define SMALL_NT 1024
#define SMALL_NPW 21  // nodes per wavefront, three lanes each
static_assert(SMALL_NT / 64 * SMALL_NPW == SF_SMALL_G, "small-level capacity");

// ---- whole PCG of a small level in one workgroup (node blocks) ------------
//
// For levels with at most SF_SMALL_G nodes the n PCG iterations of a
// Gauss-Newton step run in one workgroup per frame: three lanes per node
// (21 nodes per wavefront), each holding three of the node's nine blocks in
// registers and two of its six components of x, r, p, s, w and diag(H); u
// is exchanged through LDS records and the three inner products through a
// fixed-order workgroup reduction, so every iteration costs two barriers
// instead of a kernel launch and a round trip through memory.  The
// iterates, history entries, logged residual norms and the final partial
// sum read by the step control are those of the multi-kernel form.

// A value every lane holds the same copy of, moved to scalar registers.
__device__ __forceinline__ double uniform_d(double v) {
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float uniform_f(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

// Block products of a node's three lanes: task q of lane `sub` is block
// type k, the node's own (partner n + off(k)) or the one stored by
// n - off(k) (whose partner is n).
__device__ __forceinline__ void small_task(int sub, int q, int &k, bool &own) {
    if (sub == 0) { k = q; own = true; }                   // self, E, S
    else if (sub == 1) { k = q == 2 ? 1 : 3 + q; own = q < 2; }  // SE, SW, E of W
    else { k = 2 + q; own = false; }                        // S of N, SE of NW, SW of NE
}

template <bool B>
__global__ __launch_bounds__(SMALL_NT) void k_pcg_small(KArg<B> ka, int n_it, int gn, int pend) {
    __shared__ __attribute__((aligned(16))) float su[SF_SMALL_G * 8];
    // each lane's third block (registers hold the first two)
    __shared__ __attribute__((aligned(16))) float sb[SMALL_NT * SF_GRAM_STRIDE];
    // per lane: its block products (6) and epipolar pair sums (2); two spare
    // records for the idle last lane of a wavefront, which reads past it
    __shared__ __attribute__((aligned(16))) float sx[(SMALL_NT + 2) * 8];
    __shared__ float red[SMALL_NT / 64][3];
    // decisions and logged residual norms, written out after the loop
    __shared__ PcgHist shist[SF_MAX_PCG + 1];
    __shared__ double sres[SF_MAX_PCG];
    SF_BIND(ka);
    (void)nblk;
    const LevelDims &d = a.d;
    if (d.G > SF_SMALL_G) return;  // the host never launches such a level
    if (pend && !a.sc->spec_acc) {
        // the deferred step of a rejected speculative tau = 1 (k_rhs_blocks)
        const float tau = a.sc->spec_tau;
        for (int m = threadIdx.x; m < d.G; m += blockDim.x) deferred_step(a, m, tau);
        lin_energy_scalars(a, a.sc->lin_n);
    }
    const int log_index = gn >= 0 ? a.log_base + gn : -1;
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int sub = lane % 3;
    const int n = wv * SMALL_NPW + lane / 3;
    const bool valid = lane < 3 * SMALL_NPW && n < d.G;
    const int i_n = valid ? n % d.Gx : 0, j_n = valid ? n / d.Gx : 0;
    const int c0 = 2 * sub;  // this lane's two components
    // A missing partner gets a zero block and the node's own u record, so
    // that every lane issues the same loads and products (adding +0 leaves
    // the sums unchanged).
    float Bk[2][21];
    int pn[3];
    float *myb = sb + threadIdx.x * SF_GRAM_STRIDE;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int k, di, dj;
        bool own;
        small_task(sub, q, k, own);
        blk_offset(k, di, dj);
        const int pi = own ? i_n + di : i_n - di, pj = own ? j_n + dj : j_n - dj;
        const bool has = valid && pi >= 0 && pi < d.Gx && pj >= 0 && pj < d.Gy;
        pn[q] = has ? pj * d.Gx + pi : (valid ? n : 0);
        float t[21];
#pragma unroll
        for (int e = 0; e < 21; ++e) t[e] = 0.f;
        if (has) {
            const long owner = own ? (long)n : (long)pn[q];
            blk_load(a.blk, owner, k, t);
        }
        if (q < 2) {
#pragma unroll
            for (int e = 0; e < 21; ++e) Bk[q][e] = t[e];
        } else {
            rec_store<21>(myb, t);
        }
    }
    float cnb[4] = {0.f, 0.f, 0.f, 0.f}, J0o[2] = {0.f, 0.f}, J1o[2] = {0.f, 0.f};
    int nbr[4];
    float r2[2] = {0.f, 0.f}, u2[2] = {0.f, 0.f}, D2[2] = {1.f, 1.f};
    float x2[2] = {0.f, 0.f}, p2[2] = {0.f, 0.f}, s2[2] = {0.f, 0.f}, w2[2] = {0.f, 0.f};
    float wf2[2], cm2[2];
    {
        const DevConst *C = a.cst;
        const float c = 2.f * C->w_reg * C->w_mag;
        wf2[0] = C->wf[c0]; wf2[1] = C->wf[c0 + 1];
        cm2[0] = c * C->mf[c0]; cm2[1] = c * C->mf[c0 + 1];
    }
    if (valid) {
        const float2 rv = *reinterpret_cast<const float2 *>(nvec(a, NV_R0) + (long)n * SF_NREC + c0);
        const float2 uv = *reinterpret_cast<const float2 *>(nvec(a, NV_U) + (long)n * SF_NREC + c0);
        const float2 dv = *reinterpret_cast<const float2 *>(nvec(a, NV_DIAG) + (long)n * SF_NREC + c0);
        r2[0] = rv.x; r2[1] = rv.y; u2[0] = uv.x; u2[1] = uv.y; D2[0] = dv.x; D2[1] = dv.y;
        float rg[REG_PLANES];
        rec_load<REG_PLANES>(a.reg + (long)n * REG_PLANES, rg);
#pragma unroll
        for (int k = 0; k < 4; ++k) cnb[k] = rg[k];
        // this lane's components of the two epipolar rows
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            J0o[j] = sub == 0 ? rg[4 + j] : (sub == 1 ? rg[6 + j] : rg[8 + j]);
            J1o[j] = sub == 0 ? rg[10 + j] : (sub == 1 ? rg[12 + j] : rg[14 + j]);
        }
    }
    // neighbours without a smoothness coefficient read the node's own u
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int di, dj;
        nb_offset(k, di, dj);
        nbr[k] = valid && cnb[k] != 0.f ? (j_n + dj) * d.Gx + i_n + di : (valid ? n : 0);
    }

    // The PCG scalars are reduced and decided by wavefront 0 at the end of
    // each pass and handed to every thread through LDS: one more barrier,
    // but the double-precision decision runs once instead of in every
    // wavefront.
    __shared__ float s_dec[2];
    __shared__ int s_act;
    double rsum = 0.0;         // (wavefront 0) r.r of the last pass
    double hg = 0.0;           // (wavefront 0) gamma of the previous pass
    float ha = 0.f;            // (wavefront 0) alpha of the previous pass
    float al = 0.f, be = 0.f;  // scalars of iteration i-1
    int act = 1;
    for (int i = 0; i <= n_it; ++i) {
        if (i > 0) {
            if (!act) break;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                s2[j] = i > 1 ? w2[j] + be * s2[j] : w2[j];
                p2[j] = i > 1 ? u2[j] + be * p2[j] : u2[j];
                x2[j] = x2[j] + al * p2[j];
                r2[j] = r2[j] - al * s2[j];
                u2[j] = r2[j] / D2[j];
            }
            if (i == n_it) break;  // ||r_n||^2 below
        }
        // u_i into LDS; w_i = H u_i
        if (valid) *reinterpret_cast<float2 *>(su + n * 8 + c0) = make_float2(u2[0], u2[1]);
        __syncthreads();
        float y[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        {
            float un[3][6];
#pragma unroll
            for (int q = 0; q < 3; ++q) rec_load<6>(su + pn[q] * 8, un[q]);
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = 0; c < 6; ++c) y[r] += Bk[q][gram_index(r, c)] * un[q][c];
            float b2[21];
            rec_load<21>(myb, b2);
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = 0; c < 6; ++c) y[r] += b2[gram_index(r, c)] * un[2][c];
        }
        // the node's sums over its three lanes in lane order, and the
        // epipolar projections J_t . u from the lanes' component pairs,
        // exchanged through LDS records (the three lanes share a wavefront,
        // whose LDS accesses are performed in order)
        {
            const float e0 = J0o[0] * u2[0] + J0o[1] * u2[1];
            const float e1 = J1o[0] * u2[0] + J1o[1] * u2[1];
            float4 *mx = reinterpret_cast<float4 *>(sx + threadIdx.x * 8);
            mx[0] = make_float4(y[0], y[1], y[2], y[3]);
            mx[1] = make_float4(y[4], y[5], e0, e1);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float w2s[2] = {0.f, 0.f}, jp0 = 0.f, jp1 = 0.f;
        const float *gx = sx + (threadIdx.x - sub) * 8;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const float2 yc = *reinterpret_cast<const float2 *>(gx + t * 8 + c0);
            const float2 ee = *reinterpret_cast<const float2 *>(gx + t * 8 + 6);
            w2s[0] += yc.x;
            w2s[1] += yc.y;
            jp0 += ee.x;
            jp1 += ee.y;
        }
        float ru = 0.f, wu = 0.f, rr = 0.f;
        if (valid) {
            float sm[2] = {0.f, 0.f};
            float2 un[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) un[k] = *reinterpret_cast<const float2 *>(su + nbr[k] * 8 + c0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sm[0] += cnb[k] * (u2[0] - un[k].x);
                sm[1] += cnb[k] * (u2[1] - un[k].y);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                w2[j] = w2s[j] + wf2[j] * sm[j] + J0o[j] * jp0 + J1o[j] * jp1 + cm2[j] * u2[j];
                ru += r2[j] * u2[j];
                wu += w2[j] * u2[j];
                rr += r2[j] * r2[j];
            }
        }
        // wavefront sums in float (as a workgroup's partial in the
        // multi-kernel form), the wavefronts' sums in double: every
        // 16-lane row adds them in the same order
        const float t0 = wave_sum(ru), t1 = wave_sum(wu), t2 = wave_sum(rr);
        if (lane == 0) { red[wv][0] = t0; red[wv][1] = t1; red[wv][2] = t2; }
        __syncthreads();
        if (wv == 0) {
            // scalars of iteration i from this pass's sums
            const int rw = lane & 15;
            const double gsum = uniform_d(group_sum<double>(rw < nw ? (double)red[rw][0] : 0.0, 16));
            const double dsum = uniform_d(group_sum<double>(rw < nw ? (double)red[rw][1] : 0.0, 16));
            rsum = uniform_d(group_sum<double>(rw < nw ? (double)red[rw][2] : 0.0, 16));
            double b = 0.0, pq = dsum;
            if (i > 0) {
                b = gsum / hg;
                pq = dsum - b * gsum / (double)ha;
            }
            const int ok = gsum > 1e-30 && pq > 0.0 && isfinite(pq);
            const float aln = ok ? (float)(gsum / pq) : 0.f;
            const float ben = ok ? (float)b : 0.f;
            if (lane == 0) {
                // an inactive iteration leaves every later one inactive with
                // the same sums (the multi-kernel form carries its partials)
                for (int m = i + 1; m <= (ok ? i + 1 : n_it); ++m) {
                    PcgHist o;
                    o.gamma = gsum; o.alpha = aln; o.beta = ben; o.active = ok; o.pad = 0;
                    shist[m] = o;
                    if (m >= 2) sres[m - 2] = rsum;
                }
                s_dec[0] = aln;
                s_dec[1] = ben;
                s_act = ok;
            }
            hg = gsum;
            ha = aln;
        }
        __syncthreads();
        al = uniform_f(s_dec[0]);
        be = uniform_f(s_dec[1]);
        act = __builtin_amdgcn_readfirstlane(s_act);
    }
    if (act) {
        // ||r_n||^2 for the step control's log
        const float rr = valid ? r2[0] * r2[0] + r2[1] * r2[1] : 0.f;
        const float t2 = wave_sum(rr);
        __syncthreads();
        if (lane == 0) red[wv][2] = t2;
        __syncthreads();
        const int rw = lane & 15;
        rsum = group_sum<double>(rw < nw ? (double)red[rw][2] : 0.0, 16);
    }
    if (valid) *reinterpret_cast<float2 *>(nvec(a, NV_X) + (long)n * SF_NREC + c0) = make_float2(x2[0], x2[1]);
    __syncthreads();
    for (int m = threadIdx.x + 1; m <= n_it; m += blockDim.x) {
        a.sc->hist[m] = shist[m];
        if (log_index >= 0 && m >= 2) a.log[log_index].pcg_res[m - 2] = (float)sqrt(sres[m - 2]);
    }
    if (threadIdx.x < node_blocks(d)) {
        a.partials[(long)(((n_it & 1) ? PS_PCG1 : PS_PCG0) + 2) * a.max_blocks + threadIdx.x] =
            threadIdx.x == 0 ? (float)rsum : 0.f;
    }
}

// ---- PCG of a level in co-resident tiles, tagged exchange --------------------
//
// apply_mode 3, single frames: a level with more than SF_SMALL_G nodes whose
// tiles all fit on the device at once runs all PCG iterations of a
// Gauss-Newton step in one launch, one workgroup per tile of SF_PT_TW x
// SF_PT_TH nodes (four wavefronts, three lanes per node as in the
// one-workgroup kernel).  Each lane keeps its three block products'
// blocks in registers for all iterations.  Between passes the tiles
// exchange only what the next pass needs: their three partial sums and,
// for the nodes on the tile border, r, w and s of the pass, from which a
// neighbour rebuilds the u of its halo (as the multi-kernel form does).
// Every value travels as one 64-bit word, the float and a tag (the
// launch's epoch and the pass), stored and loaded with relaxed agent-scope
// atomics: a reader polls until the tag it expects is there, so no fence,
// counter or barrier is needed.  Two parity slots per pass suffice: a tile
// that writes pass p + 2 has read every tile's pass p + 1 sums, so each
// reader of pass p has finished.  The epoch advances by one per launch
// (tile 0 moves it once every tile has published its last word, so every
// tile has read it); a word a launch waits for was last written by an
// earlier launch of the same level, whose tags differ unless 2^24 launches
// lie between them.  Every wait is bounded, and a tile that
// gives up raises the sticky flag the host reports.  The iterates are those
// of the single-reduction PCG (the partial sums are reduced per tile).

#define PT_N (SF_PT_TW * SF_PT_TH)
#define PT_NT (64 * (PT_N / SMALL_NPW))
#define PT_HX (SF_PT_TW + 2)
#define PT_HY (SF_PT_TH + 2)
#define PT_PER_LANE (SF_PT_MAXWG / 64)
static_assert(PT_N % SMALL_NPW == 0, "whole wavefronts of three-lane nodes");
static_assert(SF_PT_MAXWG % 64 == 0, "lane-strided partial slots");
static_assert(2 * (SF_PT_TW + 2) + 2 * SF_PT_TH <= 64, "halo nodes in wavefront 0");

// Tagged words: the float in the high half, the tag in the low half.
__device__ __forceinline__ void tag_store(unsigned long long *p, float v, unsigned tag) {
    const unsigned long long w = ((unsigned long long)__float_as_uint(v) << 32) | tag;
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long tag_load(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float tag_value(unsigned long long w) {
    return __uint_as_float((unsigned)(w >> 32));
}
__device__ __forceinline__ bool wave_any(bool p) {
    return __builtin_amdgcn_readfirstlane((unsigned)(__ballot(p) != 0ull)) != 0u;
}
// A give-up: raise the flag; true if this wait (or another tile) gave up.
__device__ __forceinline__ bool wait_over(DevScalars *sc, int &spins, int spin_limit) {
    if (++spins > spin_limit ||
        __hip_atomic_load(&sc->mid_fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        atomicExch(&sc->mid_fail, 1);
        return true;
    }
    return false;
}

// Exchange-buffer layout (64-bit words): the partial sums of each parity
// (3 planes) and the final ||r||^2 partials, each in PT_REP replicas (a
// tile reads replica wg % PT_REP, so that the tiles' polls spread over
// several lines instead of all meeting on one), then per parity and node
// the 18 words r, w, s of its border record.
#define PT_REP 8
__device__ __forceinline__ unsigned long long *pt_part(const LevelArgs &a, int par, int k,
                                                      int rep) {
    return a.xtag + (((size_t)par * 3 + k) * PT_REP + rep) * SF_PT_MAXWG;
}
__device__ __forceinline__ unsigned long long *pt_final(const LevelArgs &a, int rep) {
    return a.xtag + ((size_t)6 * PT_REP + rep) * SF_PT_MAXWG;
}
__device__ __forceinline__ unsigned long long *pt_rec(const LevelArgs &a, int par, long n) {
    return a.xtag + (size_t)7 * PT_REP * SF_PT_MAXWG + ((size_t)par * a.G0 + n) * 18;
}

// One wavefront's poll: the K planes' sums over the P tiles (lane-strided
// loads, polled until every tag matches, summed in double in a fixed
// order: the same in every tile) and, in lanes with a halo node (rec not
// null), the record words `need_h` of that node, all issued together in
// each round; false if a wait gave up (alike in every lane).
template <int K>
__device__ bool pt_poll(const LevelArgs &a, unsigned long long *const (&src)[K], int P,
                        unsigned tag, const unsigned long long *rec, unsigned need_h,
                        float (&hv)[18], int spin_limit, double (&out)[K]) {
    const int lane = threadIdx.x & 63;
    float v[PT_PER_LANE][K];
    unsigned need = 0;
#pragma unroll
    for (int u = 0; u < PT_PER_LANE; ++u)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            v[u][q] = 0.f;
            if (lane + 64 * u < P) need |= 1u << (u * K + q);
        }
    if (!rec) need_h = 0;
    int spins = 0;
    while (true) {
#pragma unroll
        for (int u = 0; u < PT_PER_LANE; ++u)
#pragma unroll
            for (int q = 0; q < K; ++q) {
                if (need & (1u << (u * K + q))) {
                    const unsigned long long w = tag_load(src[q] + lane + 64 * u);
                    if ((unsigned)w == tag) {
                        v[u][q] = tag_value(w);
                        need &= ~(1u << (u * K + q));
                    }
                }
            }
#pragma unroll
        for (int q = 0; q < 18; ++q) {
            if (need_h & (1u << q)) {
                const unsigned long long w = tag_load(rec + q);
                if ((unsigned)w == tag) {
                    hv[q] = tag_value(w);
                    need_h &= ~(1u << q);
                }
            }
        }
        if (!wave_any(need != 0 || need_h != 0)) break;
        if (__builtin_amdgcn_readfirstlane(wait_over(a.sc, spins, spin_limit) ? 1u : 0u))
            return false;
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < PT_PER_LANE; ++u) acc += (double)v[u][q];
        out[q] = uniform_d(group_sum<double>(acc, 64));
    }
    return true;
}

__global__ __launch_bounds__(PT_NT) void k_pcg_tile(LevelArgs a, int n_it, int gn,
                                                    int spin_limit, int pend) {
    __shared__ __attribute__((aligned(16))) float su[PT_HX * PT_HY * 8];
    __shared__ __attribute__((aligned(16))) float sx[(PT_NT + 2) * 8];
    __shared__ float red[PT_NT / 64][3];
    __shared__ double s_sum[3];
    const LevelDims &d = a.d;
    const int tiles_x = (d.Gx + SF_PT_TW - 1) / SF_PT_TW;
    const int P = gridDim.x, wg = blockIdx.x;
    const int i0 = (wg % tiles_x) * SF_PT_TW, j0 = (wg / tiles_x) * SF_PT_TH;
    const int tw = min(SF_PT_TW, d.Gx - i0), th = min(SF_PT_TH, d.Gy - j0);
    const unsigned epoch = a.sc->pt_epoch;
    // tags: pass p of this launch (p = 200: the final ||r||^2); never 0, the
    // word of a cleared buffer
    auto tag = [epoch](int p) { return (epoch << 8) | (unsigned)(p + 1); };
    const int log_index = gn >= 0 ? a.log_base + gn : -1;
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane % 3;
    const int t = wv * SMALL_NPW + lane / 3;
    const bool valid = lane < 3 * SMALL_NPW && t < tw * th;
    const int i_n = i0 + (valid ? t % tw : 0), j_n = j0 + (valid ? t / tw : 0);
    const long n = (long)j_n * d.Gx + i_n;
    const int c0 = 2 * sub;
    // LDS record of node (i, j) of the tile or its halo ring
    auto loc = [i0, j0](int i, int j) { return (j - j0 + 1) * PT_HX + (i - i0 + 1); };
    const int n_loc = loc(i_n, j_n);
    if (pend && !a.sc->spec_acc) {
        // the deferred step of a rejected speculative tau = 1 (k_rhs_blocks)
        if (valid && sub == 0) deferred_step(a, n, a.sc->spec_tau);
        if (wg == 0) lin_energy_scalars(a, a.sc->lin_n);
    }
    // this lane's three blocks, partners at their LDS records
    float Bk[3][21];
    int pn[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int k, di, dj;
        bool own;
        small_task(sub, q, k, own);
        blk_offset(k, di, dj);
        const int pi = own ? i_n + di : i_n - di, pj = own ? j_n + dj : j_n - dj;
        const bool has = valid && pi >= 0 && pi < d.Gx && pj >= 0 && pj < d.Gy;
        pn[q] = has ? loc(pi, pj) : n_loc;
#pragma unroll
        for (int e = 0; e < 21; ++e) Bk[q][e] = 0.f;
        if (has) {
            const long owner = own ? n : (long)pj * d.Gx + pi;
            blk_load(a.blk, owner, k, Bk[q]);
        }
    }
    float cnb[4] = {0.f, 0.f, 0.f, 0.f}, J0o[2] = {0.f, 0.f}, J1o[2] = {0.f, 0.f};
    int nbr[4];
    float r2[2] = {0.f, 0.f}, u2[2] = {0.f, 0.f}, D2[2] = {1.f, 1.f};
    float x2[2] = {0.f, 0.f}, p2[2] = {0.f, 0.f}, s2[2] = {0.f, 0.f}, w2[2] = {0.f, 0.f};
    float wf2[2], cm2[2];
    {
        const DevConst *C = a.cst;
        const float c = 2.f * C->w_reg * C->w_mag;
        wf2[0] = C->wf[c0]; wf2[1] = C->wf[c0 + 1];
        cm2[0] = c * C->mf[c0]; cm2[1] = c * C->mf[c0 + 1];
    }
    if (valid) {
        const float2 rv = *reinterpret_cast<const float2 *>(nvec(a, NV_R0) + n * SF_NREC + c0);
        const float2 uv = *reinterpret_cast<const float2 *>(nvec(a, NV_U) + n * SF_NREC + c0);
        const float2 dv = *reinterpret_cast<const float2 *>(nvec(a, NV_DIAG) + n * SF_NREC + c0);
        r2[0] = rv.x; r2[1] = rv.y; u2[0] = uv.x; u2[1] = uv.y; D2[0] = dv.x; D2[1] = dv.y;
        float rg[REG_PLANES];
        rec_load<REG_PLANES>(a.reg + n * REG_PLANES, rg);
#pragma unroll
        for (int k = 0; k < 4; ++k) cnb[k] = rg[k];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            J0o[j] = sub == 0 ? rg[4 + j] : (sub == 1 ? rg[6 + j] : rg[8 + j]);
            J1o[j] = sub == 0 ? rg[10 + j] : (sub == 1 ? rg[12 + j] : rg[14 + j]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int di, dj;
        nb_offset(k, di, dj);
        nbr[k] = valid && cnb[k] != 0.f ? loc(i_n + di, j_n + dj) : n_loc;
    }
    // the border nodes publish their records; the halo ring's nodes (one
    // thread each) are rebuilt from their owners' records
    const bool border = valid && (i_n == i0 || i_n == i0 + tw - 1 || j_n == j0 || j_n == j0 + th - 1);
    const int hw = tw + 2, hh = th + 2, n_ring = 2 * hw + 2 * (hh - 2);
    int hi = -1, hj = -1;
    if ((int)threadIdx.x < n_ring) {
        const int r = threadIdx.x;
        if (r < hw) { hi = i0 - 1 + r; hj = j0 - 1; }
        else if (r < 2 * hw) { hi = i0 - 1 + (r - hw); hj = j0 + th; }
        else { const int q = r - 2 * hw; hi = (q & 1) ? i0 + tw : i0 - 1; hj = j0 + (q >> 1); }
    }
    const bool halo = hi >= 0 && hi < d.Gx && hj >= 0 && hj < d.Gy;
    const long hn = halo ? (long)hj * d.Gx + hi : 0;
    float hdg[6] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
    if (halo) ld6(nvec(a, NV_DIAG), hn, hdg);

    double hg = 0.0;           // gamma of the previous decision
    float ha = 0.f;            // alpha of the previous decision
    float al = 0.f, be = 0.f;  // scalars of iteration i-1
    int act = 1;
    for (int i = 0; i <= n_it; ++i) {
        if (i > 0) {
            // wavefront 0 polls every tile's sums of pass i-1 and, in the
            // lanes of halo nodes, their owners' records of pass i-1, all
            // in the same rounds; the workgroup goes on only if every wait
            // succeeded
            float hv[18];
            bool ok_w = true;
            if (wv == 0) {
                const int par = (i - 1) & 1, rep = wg % PT_REP;
                unsigned long long *const src[3] = {pt_part(a, par, 0, rep),
                                                    pt_part(a, par, 1, rep),
                                                    pt_part(a, par, 2, rep)};
                const bool hpoll = halo && i < n_it;
#pragma unroll
                for (int q = 0; q < 18; ++q) hv[q] = 0.f;
                double s3w[3];
                ok_w = pt_poll<3>(a, src, P, tag(i - 1), hpoll ? pt_rec(a, par, hn) : nullptr,
                                  i > 1 ? 0x3FFFFu : 0xFFFu, hv, spin_limit, s3w);
                if (lane == 0) { s_sum[0] = s3w[0]; s_sum[1] = s3w[1]; s_sum[2] = s3w[2]; }
            }
            if (!__syncthreads_and(ok_w)) return;
            const double s3[3] = {s_sum[0], s_sum[1], s_sum[2]};
            // iteration i-1 from those sums (alike in every wavefront)
            const double gam = s3[0], del = s3[1], rsum = s3[2];
            double b = 0.0, pq = del;
            if (i - 1 > 0) {
                b = gam / hg;
                pq = del - b * gam / (double)ha;
            }
            const int ok = act && gam > 1e-30 && pq > 0.0 && isfinite(pq);
            al = ok ? (float)(gam / pq) : 0.f;
            be = ok ? (float)b : 0.f;
            if (wg == 0 && threadIdx.x == 0) {
                // an inactive iteration leaves every later one inactive with
                // the same sums
                for (int m = i; m <= (ok ? i : n_it); ++m) {
                    PcgHist o;
                    o.gamma = gam; o.alpha = al; o.beta = be; o.active = ok; o.pad = 0;
                    a.sc->hist[m] = o;
                    if (log_index >= 0 && m >= 2) a.log[log_index].pcg_res[m - 2] = (float)sqrt(rsum);
                }
            }
            hg = gam;
            ha = al;
            act = ok;
            if (!act) break;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                s2[j] = i > 1 ? w2[j] + be * s2[j] : w2[j];
                p2[j] = i > 1 ? u2[j] + be * p2[j] : u2[j];
                x2[j] = x2[j] + al * p2[j];
                r2[j] = r2[j] - al * s2[j];
                u2[j] = r2[j] / D2[j];
            }
            if (i == n_it) break;
            // halo u_i
            if (halo) {
                float uh[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const float sv = i > 1 ? hv[6 + q] + be * hv[12 + q] : hv[6 + q];
                    const float rn = hv[q] - al * sv;
                    uh[q] = rn / hdg[q];
                }
                rec_store<6>(su + (size_t)loc(hi, hj) * 8, uh);
            }
        } else {
            // u_0 of the halo as the right-hand-side kernel stored it
            if (halo) {
                float uh[6];
                ld6(nvec(a, NV_U), hn, uh);
                rec_store<6>(su + (size_t)loc(hi, hj) * 8, uh);
            }
        }
        // u_i of the own nodes; w_i = H u_i
        if (valid) *reinterpret_cast<float2 *>(su + n_loc * 8 + c0) = make_float2(u2[0], u2[1]);
        __syncthreads();
        float y[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        {
            float un[3][6];
#pragma unroll
            for (int q = 0; q < 3; ++q) rec_load<6>(su + pn[q] * 8, un[q]);
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = 0; c < 6; ++c) y[r] += Bk[q][gram_index(r, c)] * un[q][c];
        }
        {
            const float e0 = J0o[0] * u2[0] + J0o[1] * u2[1];
            const float e1 = J1o[0] * u2[0] + J1o[1] * u2[1];
            float4 *mx = reinterpret_cast<float4 *>(sx + threadIdx.x * 8);
            mx[0] = make_float4(y[0], y[1], y[2], y[3]);
            mx[1] = make_float4(y[4], y[5], e0, e1);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float w2s[2] = {0.f, 0.f}, jp0 = 0.f, jp1 = 0.f;
        const float *gx = sx + (threadIdx.x - sub) * 8;
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) {
            const float2 yc = *reinterpret_cast<const float2 *>(gx + tt * 8 + c0);
            const float2 ee = *reinterpret_cast<const float2 *>(gx + tt * 8 + 6);
            w2s[0] += yc.x;
            w2s[1] += yc.y;
            jp0 += ee.x;
            jp1 += ee.y;
        }
        float ru = 0.f, wu = 0.f, rr = 0.f;
        if (valid) {
            float sm[2] = {0.f, 0.f};
            float2 un[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) un[k] = *reinterpret_cast<const float2 *>(su + nbr[k] * 8 + c0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sm[0] += cnb[k] * (u2[0] - un[k].x);
                sm[1] += cnb[k] * (u2[1] - un[k].y);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                w2[j] = w2s[j] + wf2[j] * sm[j] + J0o[j] * jp0 + J1o[j] * jp1 + cm2[j] * u2[j];
                ru += r2[j] * u2[j];
                wu += w2[j] * u2[j];
                rr += r2[j] * r2[j];
            }
        }
        // the border records of pass i (s of pass i-1, as the halo rebuild
        // of pass i+1 needs it), then this tile's sums
        if (border) {
            unsigned long long *rec = pt_rec(a, i & 1, n);
            const unsigned tg = tag(i);
            tag_store(rec + c0, r2[0], tg);
            tag_store(rec + c0 + 1, r2[1], tg);
            tag_store(rec + 6 + c0, w2[0], tg);
            tag_store(rec + 6 + c0 + 1, w2[1], tg);
            tag_store(rec + 12 + c0, s2[0], tg);
            tag_store(rec + 12 + c0 + 1, s2[1], tg);
        }
        const float t0 = wave_sum(ru), t1 = wave_sum(wu), t2 = wave_sum(rr);
        if (lane == 0) { red[wv][0] = t0; red[wv][1] = t1; red[wv][2] = t2; }
        __syncthreads();
        if (threadIdx.x < 3 * PT_REP) {
            const int k = threadIdx.x % 3;
            double tsum = 0.0;
            for (int w = 0; w < nw; ++w) tsum += (double)red[w][k];
            tag_store(pt_part(a, i & 1, k, threadIdx.x / 3) + wg, (float)tsum, tag(i));
        }
    }
    // the solution, and ||r_n||^2 for the step control's log: tile 0 sums
    // every tile's final partial and leaves it as the one nonzero partial
    if (valid) *reinterpret_cast<float2 *>(nvec(a, NV_X) + n * SF_NREC + c0) = make_float2(x2[0], x2[1]);
    const float rrf = valid ? r2[0] * r2[0] + r2[1] * r2[1] : 0.f;
    const float tr = wave_sum(rrf);
    __syncthreads();
    if (lane == 0) red[wv][2] = tr;
    __syncthreads();
    if (threadIdx.x < PT_REP) {
        double tsum = 0.0;
        for (int w = 0; w < nw; ++w) tsum += (double)red[w][2];
        tag_store(pt_final(a, threadIdx.x) + wg, (float)tsum, tag(200));
    }
    if (wg == 0 && wv == 0) {
        unsigned long long *const src[1] = {pt_final(a, 0)};
        double fr[1];
        float unused[18];
        if (!pt_poll<1>(a, src, P, tag(200), nullptr, 0u, unused, spin_limit, fr)) return;
        float *rrp = a.partials + (long)(((n_it & 1) ? PS_PCG1 : PS_PCG0) + 2) * a.max_blocks;
        for (int b = lane; b < node_blocks(d); b += 64) rrp[b] = b == 0 ? (float)fr[0] : 0.f;
        // every tile has read the epoch (each published its final partial):
        // the next launch takes a fresh one
        if (lane == 0) a.sc->pt_epoch = epoch + 1u;
    }
}

// ---- step control: accept the first tau with E_trial <= E ------------------

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_accept(KArg<B> ka, int n_trials, int gn_iter,
                                                     int pcg_iters) {
    SF_BIND(ka);
    __shared__ int s_k;
    const double e0 = a.sc->e_lin[5];
    if (threadIdx.x < 64) {
        // the first trial with E_trial <= E, from the trial kernels' partials
        double e[6];
        trial_energy_wave(a, PS_E, energy_blocks_of(a.d), e);
        int kacc = e[5] <= e0 ? 0 : -1;
        if (kacc < 0) kacc = rest_decision(a, n_trials, e);
        if (threadIdx.x == 0) s_k = kacc;
        if (bid == 0) step_record(a, gn_iter, pcg_iters, kacc, e);
    }
    __syncthreads();
    const int kacc = s_k;
    const float tau = kacc >= 0 ? ldexpf(1.f, -kacc) : 0.f;
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (kacc >= 0 && n < a.d.G) {
        float *delta = nvec(a, NV_DELTA);
        float dl[6], x[6];
        ld6(delta, n, dl);
        ld6(nvec(a, NV_X), n, x);
#pragma unroll
        for (int q = 0; q < 6; ++q) dl[q] = dl[q] + tau * x[q];
        st6(delta, n, dl);
    }
}

// ---- level start: prolongation, masks, smoothness weights -------------------

// ---- learned initialisation of the coarsest level --------------------------

// Candidate node flows: the network output (level-4 pixels) sampled at the
// coarsest level's nodes; node position p maps to 2^(l - 4) (p + 1/2) - 1/2
// in level-4 pixels (pixel-centre convention), clamp-to-edge bilinear, and
// flows scale by 2^(4 - l).  Stored in the P vector (free at level start).
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_cnn_nodes(KArg<B> ka) {
    SF_BIND(ka);
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= a.d.G) return;
    const int i = (int)(n % a.d.Gx), j = (int)(n / a.d.Gx);
    float gx, gy;
    node_xy(i, j, a.s, gx, gy);
    const float r = ldexpf(1.f, a.level - SF_CNN_INPUT_LEVEL);
    const int W4 = a.W4, H4 = a.H4;
    const float u = fminf(fmaxf(r * (gx + 0.5f) - 0.5f, 0.f), (float)(W4 - 1));
    const float v = fminf(fmaxf(r * (gy + 0.5f) - 0.5f, 0.f), (float)(H4 - 1));
    const int x0 = min((int)floorf(u), max(W4 - 2, 0)), y0 = min((int)floorf(v), max(H4 - 2, 0));
    const int x1 = min(x0 + 1, W4 - 1), y1 = min(y0 + 1, H4 - 1);
    const float fx = u - (float)x0, fy = v - (float)y0;
    const long N4 = (long)W4 * H4;
    float cand[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float *o = a.cnn_out + q * N4;
        const float val = (1.f - fy) * ((1.f - fx) * o[y0 * W4 + x0] + fx * o[y0 * W4 + x1]) +
                          fy * ((1.f - fx) * o[y1 * W4 + x0] + fx * o[y1 * W4 + x1]);
        cand[q] = val / r;
    }
    st6(nvec(a, NV_P), n, cand);
}

// Energies of Eq. (8) at zero deltas for the candidate (P vector) and for
// the zero initialisation, with the same visibility mask for both (all
// four positions inside the image under the candidate; the zero flow keeps
// every position inside) and no colour pruning.  Per-workgroup partials of
// both totals in the first two energy planes.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_fallback(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    const int n_pix = pixel_tiles(d);
    __shared__ NodeStage S;
    float part[2] = {0.f, 0.f};
    if (bid < n_pix) {
        const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
        const int x0 = (bid % tiles_x) * TILE_PX, y0 = (bid / tiles_x) * TILE_PX;
        stage_vector(a, x0, y0, nvec(a, NV_P), S);
        __syncthreads();
        const int x = x0 + (threadIdx.x & (TILE_PX - 1));
        const int y = y0 + (threadIdx.x / TILE_PX);
        if (x < d.W && y < d.H) {
            float f[6];
            pixel_flows(a, x, y, S, f);
            bool V = true;
#pragma unroll
            for (int cam = 0; cam < 4; ++cam)
                V = V && axis_pos(x, cam_dx(cam, f), d.W).in && axis_pos(y, cam_dy(cam, f), d.H).in;
            const float c = V ? 1.f : 0.f;
            const float z[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            PixelOut o;
            pixel_terms<false>(a, x, y, f, c, o);
            part[0] = C.w_photo * o.e_photo + C.w_grad * o.e_grad;
            pixel_terms<false>(a, x, y, z, c, o);
            part[1] = C.w_photo * o.e_photo + C.w_grad * o.e_grad;
        }
    } else {
        const long n = (long)(bid - n_pix) * SF_BLOCK + threadIdx.x;
        if (n < d.G) {
            const int i = (int)(n % d.Gx), j = (int)(n / d.Gx);
            float gx, gy;
            node_xy(i, j, a.s, gx, gy);
            float tot[6], zero[6], e[2], J[2][6];
            ld6(nvec(a, NV_P), n, tot);
#pragma unroll
            for (int q = 0; q < 6; ++q) zero[q] = 0.f;
            const float ce = C.w_reg * C.w_epi;
            epi_terms(C.F[a.level], gx, gy, tot, e, J);
            part[0] = ce * (e[0] * e[0] + e[1] * e[1]);
            epi_terms(C.F[a.level], gx, gy, zero, e, J);
            part[1] = ce * (e[0] * e[0] + e[1] * e[1]);
        }
    }
    float tot2[2];
    block_sum<2>(part, tot2);
    if (threadIdx.x == 0) {
        a.partials[(long)PS_E * a.max_blocks + bid] = tot2[0];
        a.partials[(long)(PS_E + 1) * a.max_blocks + bid] = tot2[1];
    }
}

// Bilinear sample of a level's node records at level-pixel position (x, y):
// node coordinate (x + 1/2) / s - 1/2, clamped to the grid.
__device__ __forceinline__ void sample_node_records(const float *rec, const LevelDims &d, int s,
                                                    float x, float y, float (&out)[6]) {
    const float u = fminf(fmaxf((x + 0.5f) / (float)s - 0.5f, 0.f), (float)(d.Gx - 1));
    const float v = fminf(fmaxf((y + 0.5f) / (float)s - 0.5f, 0.f), (float)(d.Gy - 1));
    const int i0 = min((int)floorf(u), max(d.Gx - 2, 0)), i1 = min(i0 + 1, d.Gx - 1);
    const int j0 = min((int)floorf(v), max(d.Gy - 2, 0)), j1 = min(j0 + 1, d.Gy - 1);
    const float fx = u - (float)i0, fy = v - (float)j0;
    float f00[6], f01[6], f10[6], f11[6];
    ld6(rec, (long)j0 * d.Gx + i0, f00);
    ld6(rec, (long)j0 * d.Gx + i1, f01);
    ld6(rec, (long)j1 * d.Gx + i0, f10);
    ld6(rec, (long)j1 * d.Gx + i1, f11);
#pragma unroll
    for (int q = 0; q < 6; ++q)
        out[q] = (1.f - fy) * ((1.f - fx) * f00[q] + fx * f01[q]) +
                 fy * ((1.f - fx) * f10[q] + fx * f11[q]);
}

// base_l = 2 bilerp(total_{l+1}) at coarse-node coordinate i/2 - 1/4
// (Sec. 5.3); at the coarsest level zero, or the network's candidate if the
// fallback energies favour it (ties keep zero).  delta = 0, or with the
// temporal initialisation (Sec. 5.3, constant velocity) the previous
// solve's delta of this level at y - 2 m(y), m the motion components of the
// previous total at node y.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_prolong(KArg<B> ka) {
    SF_BIND(ka);
    const int Gxc = a.Gxc, Gyc = a.Gyc, coarsest = a.coarsest;
    int use_cnn = 0;
    if (coarsest && a.learned) {
        const int nb = energy_blocks_of(a.d);
        double e2[2];
        const float *p0 = a.partials + (long)PS_E * a.max_blocks;
        block_sum_planes<2>([&](int k) { return p0 + (long)k * a.max_blocks; }, nb, e2);
        const double ec = e2[0], ez = e2[1];
        use_cnn = ec < ez ? 1 : 0;
        if (bid == 0 && threadIdx.x == 0) {
            a.sc->e_init[0] = ec;
            a.sc->e_init[1] = ez;
            a.sc->init_used = use_cnn;
        }
    }
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= a.d.G) return;
    const float *tp = nvec(a, NV_TPREV);
    const int i = (int)(n % a.d.Gx), j = (int)(n / a.d.Gx);
    float v[6];
    const float zero[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (coarsest) {
        if (use_cnn) {
            ld6(nvec(a, NV_P), n, v);
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] = 0.f;
        }
    } else {
        // fine node i has coarse coordinate (2i - 1)/4: the bracket rule
        // with stride 2
        const Bracket bx = bracket(i, 2, Gxc), by = bracket(j, 2, Gyc);
        float t00[6], t01[6], t10[6], t11[6];
        ld6(tp, by.i0 * Gxc + bx.i0, t00);
        ld6(tp, by.i0 * Gxc + bx.i1, t01);
        ld6(tp, by.i1 * Gxc + bx.i0, t10);
        ld6(tp, by.i1 * Gxc + bx.i1, t11);
#pragma unroll
        for (int q = 0; q < 6; ++q)
            v[q] = 2.f * (by.w0 * (bx.w0 * t00[q] + bx.w1 * t01[q]) +
                          by.w1 * (bx.w0 * t10[q] + bx.w1 * t11[q]));
    }
    st6(nvec(a, NV_BASE), n, v);
    if (a.temporal && a.sc->have_prev) {
        const LevelDims &d = a.d;
        float tp[6], dl[6];
        ld6(a.prev + (long)8 * d.G, n, tp);
        float gx, gy;
        node_xy(i, j, a.s, gx, gy);
        sample_node_records(a.prev, d, a.s, gx - 2.f * tp[2], gy - 2.f * tp[3], dl);
        st6(nvec(a, NV_DELTA), n, dl);
    } else {
        st6(nvec(a, NV_DELTA), n, zero);
    }
}

// V(x): all four positions inside the level image; W(x): max_k |d_k| <
// eps_p (Sec. 4.1); both at the level-start flow.  Also stores the mean of
// the four warped images for the smoothness weights.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_masks(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    __shared__ NodeStage S;
    const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
    const int x0 = (bid % tiles_x) * TILE_PX, y0 = (bid / tiles_x) * TILE_PX;
    stage_nodes(a, x0, y0, 0.f, S);
    __syncthreads();
    const int x = x0 + (threadIdx.x & (TILE_PX - 1));
    const int y = y0 + (threadIdx.x / TILE_PX);
    float cnt[1] = {0.f};
    if (x < d.W && y < d.H) {
        float f[6];
        pixel_flows(a, x, y, S, f);
        bool V = true;
        float I[4];
#pragma unroll
        for (int cam = 0; cam < 4; ++cam) {
            const AxisPos px = axis_pos(x, cam_dx(cam, f), d.W);
            const AxisPos py = axis_pos(y, cam_dy(cam, f), d.H);
            V = V && px.in && py.in;
            Samp sm;
            sample3(a.tex + (long)cam * d.N, d.W, px, py, sm);
            I[cam] = sm.v[0];
        }
        if (a.occ && !a.occ[(long)y * d.W + x]) V = false;
        float Ic[4] = {I[0], I[1], I[2], I[3]};
        if (a.illum) {
            const float cr = a.illum[(long)y * d.W + x];
            Ic[1] -= cr;
            Ic[3] -= cr;
        }
        float dmax = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) dmax = fmaxf(dmax, fabsf(Ic[pair_a(k)] - Ic[pair_b(k)]));
        const bool Wm = dmax < C.eps_p;
        const int pix = y * d.W + x;
        a.cmask[pix] = (V && Wm) ? 1 : 0;
        a.grad[(long)pix * SF_GRAD_STRIDE + SF_GRAD_IBAR] = 0.25f * (((I[0] + I[1]) + I[2]) + I[3]);
        cnt[0] = (V && Wm) ? 1.f : 0.f;
    }
    float tot1[1];
    block_sum<1>(cnt, tot1);
    if (threadIdx.x == 0) a.partials[(long)PS_MASK * a.max_blocks + bid] = tot1[0];
}

// w_i = 1 + gamma exp(-lambda_min / tau_l) of the structure tensor of the
// mean warped image over a 3x3 window at the node's rounded position.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_node_weights(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const int n_mask_blocks = pixel_tiles(d);
    if (bid == 0) {
        const double c = block_sum_partials(a.partials + (long)PS_MASK * a.max_blocks, n_mask_blocks);
        if (threadIdx.x == 0) a.sc->n_valid = (int)c;
    }
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= d.G) return;
    const DevConst &C = *a.cst;
    const int i = (int)(n % d.Gx), j = (int)(n / d.Gx);
    // mean warped image of pixel (x, y), stored by the mask kernel
    auto Ib = [&](int x, int y) { return a.grad[((long)y * d.W + x) * SF_GRAD_STRIDE + SF_GRAD_IBAR]; };
    const int cx = min(((2 * i + 1) * a.s) / 2, d.W - 1);
    const int cy = min(((2 * j + 1) * a.s) / 2, d.H - 1);
    float A = 0.f, Bt = 0.f, Cc = 0.f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = min(max(cx + dx, 0), d.W - 1);
            const int yy = min(max(cy + dy, 0), d.H - 1);
            float gx, gy;
            if (xx == 0) gx = Ib(1, yy) - Ib(0, yy);
            else if (xx == d.W - 1) gx = Ib(xx, yy) - Ib(xx - 1, yy);
            else gx = 0.5f * (Ib(xx + 1, yy) - Ib(xx - 1, yy));
            if (yy == 0) gy = Ib(xx, 1) - Ib(xx, 0);
            else if (yy == d.H - 1) gy = Ib(xx, yy) - Ib(xx, yy - 1);
            else gy = 0.5f * (Ib(xx, yy + 1) - Ib(xx, yy - 1));
            A += gx * gx;
            Bt += gx * gy;
            Cc += gy * gy;
        }
    const float h = 0.5f * (A - Cc);
    const float lmin = 0.5f * (A + Cc) - sqrtf(h * h + Bt * Bt);
    const float tau = C.st_tau * ldexpf(1.f, 2 * a.level);
    a.wnode[n] = 1.f + C.st_gamma * expf(-fmaxf(lmin, 0.f) / tau);
}

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_finish_level(KArg<B> ka) {
    SF_BIND(ka);
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= a.d.G) return;
    float b[6], dl[6];
    ld6(nvec(a, NV_BASE), n, b);
    ld6(nvec(a, NV_DELTA), n, dl);
#pragma unroll
    for (int q = 0; q < 6; ++q) b[q] = b[q] + dl[q];
    st6(nvec(a, NV_TPREV), n, b);
    if (a.temporal) {
        // this level's state for the next solve (read only by the next
        // solve's level start)
        st6(a.prev, n, dl);
        st6(a.prev + (long)8 * a.d.G, n, b);
        if (a.level == 0 && n == 0) a.sc->have_prev = 1;
    }
}

// ---- illumination correction (Sec. 5.3) ----------------------------------------
//
// After a level: the stereo residual of the raw images at the final flow,
// ((I_R0 - I_L0) + (I_R1 - I_L1)) / 2 per halfway pixel (0 where a position
// leaves its image), low-passed by a separable Gaussian (sigma 3.2 px, 10
// taps a side, clamped borders) and box-upsampled to the next finer level,
// whose right-camera samples it corrects.

#define ILLUM_SIGMA 3.2f
#define ILLUM_R 10  // ceil(3 sigma)

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_illum_resid(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    __shared__ NodeStage S;
    const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
    const int x0 = (bid % tiles_x) * TILE_PX, y0 = (bid / tiles_x) * TILE_PX;
    stage_nodes(a, x0, y0, 0.f, S);
    __syncthreads();
    const int x = x0 + (threadIdx.x & (TILE_PX - 1));
    const int y = y0 + (threadIdx.x / TILE_PX);
    if (x < d.W && y < d.H) {
        float f[6];
        pixel_flows(a, x, y, S, f);
        bool V = true;
        float I[4];
#pragma unroll
        for (int cam = 0; cam < 4; ++cam) {
            const AxisPos px = axis_pos(x, cam_dx(cam, f), d.W);
            const AxisPos py = axis_pos(y, cam_dy(cam, f), d.H);
            V = V && px.in && py.in;
            Samp sm;
            sample3(a.tex + (long)cam * d.N, d.W, px, py, sm);
            I[cam] = sm.v[0];
        }
        a.ill_e[(long)y * d.W + x] = V ? 0.5f * ((I[1] - I[0]) + (I[3] - I[2])) : 0.f;
    }
}

__device__ __forceinline__ float illum_weight(int k) {
    return expf(-(float)(k * k) / (2.f * ILLUM_SIGMA * ILLUM_SIGMA));
}

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_illum_blur_x(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= d.N) return;
    const int x = (int)(n % d.W), y = (int)(n / d.W);
    float acc = 0.f, ws = 0.f;
    for (int k = -ILLUM_R; k <= ILLUM_R; ++k) {
        const float w = illum_weight(k);
        acc += w * a.ill_e[(long)y * d.W + min(max(x + k, 0), d.W - 1)];
        ws += w;
    }
    a.ill_t[n] = acc / ws;
}

// one thread per pixel of the next finer level (Wf x Hf)
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_illum_up(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= (long)a.Wf * a.Hf) return;
    const int xf = (int)(n % a.Wf), yf = (int)(n / a.Wf);
    const int xc = min(xf / 2, d.W - 1), yc = min(yf / 2, d.H - 1);
    float acc = 0.f, ws = 0.f;
    for (int k = -ILLUM_R; k <= ILLUM_R; ++k) {
        const float w = illum_weight(k);
        acc += w * a.ill_t[(long)min(max(yc + k, 0), d.H - 1) * d.W + xc];
        ws += w;
    }
    a.illum[n] = acc / ws;
}

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_illum_zero(KArg<B> ka) {
    SF_BIND(ka);
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n < a.d.N) a.illum[n] = 0.f;
}

// ---- occlusion maps (Sec. 5.3) ---------------------------------------------
//
// After a level (but the finest) the halfway pixel grid, triangulated (each
// quad (x, y), (x+1, y), (x, y+1), (x+1, y+1) split along its
// (x+1, y)-(x, y+1) diagonal), is rendered into the four views with a
// z-buffer of stereo disparity D_t = P_Lt.x - P_Rt.x (larger = nearer).
// A triangle is skipped if one of its edges is longer than OCC_EDGE px in
// the view (it spans a depth discontinuity), a vertex has D_t <= 0 or its
// area is zero; the pixel centres on or inside it take its barycentric
// D_t and the largest value wins (atomic max on the float bits: exact for
// positive floats and independent of the order).  A halfway pixel is
// occluded if, in some view, its nearest pixel centre lies in the image and
// 0 < D_t < (1 - OCC_TOL) z there.  The map is box-upsampled (fine pixel
// (x, y) takes coarse (x/2, y/2), clamped) and removes the occluded pixels
// from the next finer level's V(x).

#define OCC_TOL 0.02f
#define OCC_EDGE 2.0f

// Positions of every pixel in the four views and its two disparities:
// planes 2c, 2c + 1 = P_c.x, P_c.y; 8 = D_0; 9 = D_1.  Also clears the
// four z-buffers.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_occ_pos(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    __shared__ NodeStage S;
    const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
    const int x0 = (bid % tiles_x) * TILE_PX, y0 = (bid / tiles_x) * TILE_PX;
    stage_nodes(a, x0, y0, 0.f, S);
    __syncthreads();
    const int x = x0 + (threadIdx.x & (TILE_PX - 1));
    const int y = y0 + (threadIdx.x / TILE_PX);
    if (x < d.W && y < d.H) {
        float f[6];
        pixel_flows(a, x, y, S, f);
        const long n = (long)y * d.W + x;
        float P[8];
#pragma unroll
        for (int cam = 0; cam < 4; ++cam) {
            P[2 * cam] = (((float)x + sgn(cam, 0) * f[0]) + sgn(cam, 1) * f[2]) + sgn(cam, 2) * f[4];
            P[2 * cam + 1] = (((float)y + sgn(cam, 0) * f[1]) + sgn(cam, 1) * f[3]) + sgn(cam, 2) * f[5];
            a.occ_pos[(long)(2 * cam) * d.N + n] = P[2 * cam];
            a.occ_pos[(long)(2 * cam + 1) * d.N + n] = P[2 * cam + 1];
            a.occ_zb[(long)cam * d.N + n] = 0u;
        }
        a.occ_pos[8L * d.N + n] = P[0] - P[2];  // L0.x - R0.x
        a.occ_pos[9L * d.N + n] = P[4] - P[6];  // L1.x - R1.x
    }
}

__device__ __forceinline__ float occ_edge(float ax, float ay, float bx, float by, float qx,
                                          float qy) {
    return (bx - ax) * (qy - ay) - (by - ay) * (qx - ax);
}

// Renders one triangle into the z-buffer `zb` (W x H).  The edge test also
// rejects NaN coordinates; after it the bounding box spans at most three
// pixel centres per axis.
__device__ __forceinline__ void occ_triangle(int W, int H, unsigned *zb, float ax, float ay,
                                             float ad, float bx, float by, float bd, float cx,
                                             float cy, float cd) {
    const float e2 = OCC_EDGE * OCC_EDGE;
    const float lab = (bx - ax) * (bx - ax) + (by - ay) * (by - ay);
    const float lbc = (cx - bx) * (cx - bx) + (cy - by) * (cy - by);
    const float lca = (ax - cx) * (ax - cx) + (ay - cy) * (ay - cy);
    if (!(lab <= e2 && lbc <= e2 && lca <= e2)) return;
    if (!(ad > 0.f && bd > 0.f && cd > 0.f)) return;
    const float area = occ_edge(ax, ay, bx, by, cx, cy);
    if (area == 0.f) return;
    const float sg = area < 0.f ? -1.f : 1.f;
    const float lo_x = fminf(fminf(ax, bx), cx), hi_x = fmaxf(fmaxf(ax, bx), cx);
    const float lo_y = fminf(fminf(ay, by), cy), hi_y = fmaxf(fmaxf(ay, by), cy);
    if (hi_x < 0.f || hi_y < 0.f || lo_x > (float)(W - 1) || lo_y > (float)(H - 1)) return;
    const int qx0 = max((int)ceilf(lo_x), 0), qx1 = min((int)floorf(hi_x), W - 1);
    const int qy0 = max((int)ceilf(lo_y), 0), qy1 = min((int)floorf(hi_y), H - 1);
    for (int qy = qy0; qy <= qy1; ++qy) {
        for (int qx = qx0; qx <= qx1; ++qx) {
            const float fx = (float)qx, fy = (float)qy;
            const float e_bc = occ_edge(bx, by, cx, cy, fx, fy);
            const float e_ca = occ_edge(cx, cy, ax, ay, fx, fy);
            const float e_ab = occ_edge(ax, ay, bx, by, fx, fy);
            if (sg * e_bc >= 0.f && sg * e_ca >= 0.f && sg * e_ab >= 0.f) {
                // barycentric weights: the area opposite a vertex over the whole
                const float z = (e_bc * ad + e_ca * bd + e_ab * cd) / area;
                if (z > 0.f) atomicMax(zb + (long)qy * W + qx, __float_as_uint(z));
            }
        }
    }
}

// One thread per (view, quad): the quad's two triangles in that view.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_occ_raster(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const long nq = (long)(d.W - 1) * (d.H - 1);
    const long t = (long)bid * SF_BLOCK + threadIdx.x;
    if (t >= 4 * nq) return;
    const int cam = (int)(t / nq);
    const long q = t % nq;
    const int x = (int)(q % (d.W - 1)), y = (int)(q / (d.W - 1));
    const float *X = a.occ_pos + (long)(2 * cam) * d.N;
    const float *Y = X + d.N;
    const float *D = a.occ_pos + (long)(8 + (cam >> 1)) * d.N;
    const long ia = (long)y * d.W + x, ib = ia + 1, ic = ia + d.W, id = ic + 1;
    unsigned *zb = a.occ_zb + (long)cam * d.N;
    occ_triangle(d.W, d.H, zb, X[ia], Y[ia], D[ia], X[ib], Y[ib], D[ib], X[ic], Y[ic], D[ic]);
    occ_triangle(d.W, d.H, zb, X[ib], Y[ib], D[ib], X[id], Y[id], D[id], X[ic], Y[ic], D[ic]);
}

// One thread per pixel of this level: the z-buffer test in the four views,
// written to the fine pixels that box upsampling assigns to it.
template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_occ_test(KArg<B> ka) {
    SF_BIND(ka);
    const LevelDims &d = a.d;
    const long n = (long)bid * SF_BLOCK + threadIdx.x;
    if (n >= d.N) return;
    const int x = (int)(n % d.W), y = (int)(n / d.W);
    bool vis = true;
#pragma unroll
    for (int cam = 0; cam < 4; ++cam) {
        const float X = a.occ_pos[(long)(2 * cam) * d.N + n];
        const float Y = a.occ_pos[(long)(2 * cam + 1) * d.N + n];
        const float D = a.occ_pos[(long)(8 + (cam >> 1)) * d.N + n];
        const float nx = floorf(X + 0.5f), ny = floorf(Y + 0.5f);
        if (nx >= 0.f && nx <= (float)(d.W - 1) && ny >= 0.f && ny <= (float)(d.H - 1) &&
            D > 0.f) {
            const float z =
                __uint_as_float(a.occ_zb[(long)cam * d.N + (long)ny * d.W + (long)nx]);
            if (D < (1.f - OCC_TOL) * z) vis = false;
        }
    }
    // fine pixels (xf, yf) with (min(xf / 2, W - 1), min(yf / 2, H - 1)) = (x, y);
    // the finer level is at most 2 W + 1 by 2 H + 1 pixels
    const int xa = 2 * x, xb = min(x == d.W - 1 ? a.Wf - 1 : 2 * x + 1, a.Wf - 1);
    const int ya = 2 * y, yb = min(y == d.H - 1 ? a.Hf - 1 : 2 * y + 1, a.Hf - 1);
    for (int yf = ya; yf <= yb; ++yf)
        for (int xf = xa; xf <= xb; ++xf) a.occ_next[(long)yf * a.Wf + xf] = vis ? 1 : 0;
}

// ---- output: depth and 3D flow at level 0 -----------------------------------

template <bool B>
__global__ __launch_bounds__(SF_BLOCK) void k_output(KArg<B> ka, float *depth,
                                                     float *flow3d, float *flows) {
    SF_BIND(ka);
    if (B) {
        depth = a.io->depth;
        flow3d = a.io->flow3d;
        flows = a.io->flows;
    }
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    __shared__ NodeStage S;
    const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
    const int x0 = (bid % tiles_x) * TILE_PX, y0 = (bid / tiles_x) * TILE_PX;
    stage_nodes(a, x0, y0, 0.f, S);
    __syncthreads();
    const int x = x0 + (threadIdx.x & (TILE_PX - 1));
    const int y = y0 + (threadIdx.x / TILE_PX);
    if (x >= d.W || y >= d.H) return;
    float f[6];
    pixel_flows(a, x, y, S, f);
    const long pix = (long)y * d.W + x;
    const long N = d.N;
    float X[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int cl = t == 0 ? 0 : 2, cr = t == 0 ? 1 : 3;
        // the pixel coordinate cancels in the disparity and is taken
        // relative to the principal point first, so neither rounds at the
        // scale of the image size
        const float dl = cam_dx(cl, f), dr = cam_dx(cr, f);
        const float disp = dl - dr;
        const float Z = disp > 0.f ? C.fx * C.baseline / disp : __builtin_nanf("");
        X[t][0] = (((float)x - C.cx) + dl) * Z / C.fx;
        X[t][1] = (((float)y - C.cy) + cam_dy(cl, f)) * Z / C.fy;
        X[t][2] = Z;
    }
    depth[pix] = X[0][2];
#pragma unroll
    for (int k = 0; k < 3; ++k) flow3d[k * N + pix] = X[1][k] - X[0][k];
    if (flows) {
#pragma unroll
        for (int q = 0; q < 6; ++q) flows[q * N + pix] = f[q];
    }
}

}  // namespace

// ---- launchers ----------------------------------------------------------------

// Launches the single-frame instantiation `ks` with the frame's arguments by
// value, or the batched instantiation `kb` over all frames of L with a
// block map; `blocks(a)` is one frame's workgroup count.
template <class Blocks, class KB, class KS, class... Args>
static void go(hipStream_t st, const Launch &L, Blocks blocks, KB kb, KS ks, int threads,
               size_t lds, Args... args) {
    if (!L.batched) {
        const int nb = blocks(L.host[0]);
        if (nb > 0) hipLaunchKernelGGL(ks, dim3(nb), dim3(threads), lds, st, L.host[0], args...);
        return;
    }
    FrameMap m;
    m.tab = L.dev;
    m.nf = L.nf;
    int acc = 0;
    for (int f = 0; f < L.nf; ++f) {
        m.first[f] = acc;
        acc += blocks(L.host[f]);
    }
    for (int f = L.nf; f <= SF_MAX_BATCH; ++f) m.first[f] = acc;
    if (acc > 0) hipLaunchKernelGGL(kb, dim3(acc), dim3(threads), lds, st, m, args...);
}

// The node-tile kernels are instantiated per grid stride (1..8).
#define SF_STRIDE_SWITCH(s, CALL) \
    switch (s) {                  \
        case 1: CALL(1); break;   \
        case 2: CALL(2); break;   \
        case 3: CALL(3); break;   \
        case 4: CALL(4); break;   \
        case 5: CALL(5); break;   \
        case 6: CALL(6); break;   \
        case 7: CALL(7); break;   \
        default: CALL(8); break;  \
    }


// Node tile per grid stride: a pixel region of roughly 20-40 px a side, the
// 256 threads split evenly over the tile's nodes.
template <int S, int V = 0>
static TileCfg tile_of() {
    TileCfg t;
    t.tx = TileTraits<S, V>::TX;
    t.ty = TileTraits<S, V>::TY;
    t.tpn = TileTraits<S, V>::TPN;
    t.v = V;
    return t;
}

TileCfg pick_tile(int s) {
#define TILE(S) return tile_of<S>()
    SF_STRIDE_SWITCH(s, TILE)
#undef TILE
    return tile_of<8>();
}

int tile_variants(int s) { return s == 2 || s == 4 || s == 8 ? 3 : 1; }

TileCfg pick_pcg_tile(int s, int v) {
    if (v <= 0 || v >= tile_variants(s)) return pick_tile(s);
    if (s == 2) return v == 1 ? tile_of<2, 1>() : tile_of<2, 2>();
    if (s == 4) return v == 1 ? tile_of<4, 1>() : tile_of<4, 2>();
    return v == 1 ? tile_of<8, 1>() : tile_of<8, 2>();
}

TileCfg pick_nb_tile(int v) {
    if (v < 0 || v >= SF_NB_VARIANTS) v = 0;
    TileCfg t = v == 1 ? tile_of<0, 1>()
                       : (v == 2 ? tile_of<0, 2>() : (v == 3 ? tile_of<0, 3>() : tile_of<0, 0>()));
    t.v = SF_TILE_NB + v;
    return t;
}

template <int S>
static TileCfg blk_tile_of() {
    TileCfg t;
    t.tx = BlkShape<S>::TX;
    t.ty = BlkShape<S>::TY;
    t.tpn = BlkShape<S>::TPN;
    t.v = 0;
    return t;
}

TileCfg pick_blk_tile(int s) {
#define BTILE(S) return blk_tile_of<S>()
    SF_STRIDE_SWITCH(s, BTILE)
#undef BTILE
    return blk_tile_of<8>();
}

size_t blk_tile_lds_bytes(int s) { return blk_lds_floats(pick_blk_tile(s), s) * sizeof(float); }

int tile_threads(const TileCfg &t) { return t.tx * t.ty * t.tpn; }

int tile_threads(int s) { return tile_threads(pick_tile(s)); }

// Largest pixel region of a tile: (n + 1) s columns for even s, one more
// for odd s (floor rounding of the support bounds).
int tile_max_pixels(const TileCfg &t, int s) {
    const int ex = (s & 1) ? 1 : 0;
    return ((t.tx + 1) * s + ex) * ((t.ty + 1) * s + ex);
}

int tile_ppt(int s) {
#define PPTS(S) return TileTraits<S>::PPT
    SF_STRIDE_SWITCH(s, PPTS)
#undef PPTS
    return TileTraits<8>::PPT;
}

int tile_ppt(int s, int v) {
    if (v <= 0 || v >= tile_variants(s)) return tile_ppt(s);
    if (s == 2) return v == 1 ? TileTraits<2, 1>::PPT : TileTraits<2, 2>::PPT;
    if (s == 4) return v == 1 ? TileTraits<4, 1>::PPT : TileTraits<4, 2>::PPT;
    return v == 1 ? TileTraits<8, 1>::PPT : TileTraits<8, 2>::PPT;
}

size_t node_tile_lds_bytes(const TileCfg &t, int s, int K) {
    return tile_lds_floats(t, s, K) * sizeof(float);
}

int energy_blocks(const LevelDims &d) { return energy_blocks_of(d); }

int node_tile_blocks(const LevelDims &d, const TileCfg &t) { return node_tiles_of(d, t); }

static auto px_blocks = [](const LevelArgs &a) { return pixel_tiles(a.d); };
static auto nd_blocks = [](const LevelArgs &a) { return node_blocks(a.d); };
static auto en_blocks = [](const LevelArgs &a) { return energy_blocks_of(a.d); };
static auto tx_blocks = [](const LevelArgs &a) { return tex_blocks(a.d.W, a.d.H); };

void launch_tex_level0(hipStream_t st, const Launch &L, const float *const img[4]) {
    Img4 in;
    for (int c = 0; c < 4; ++c) in.p[c] = img ? img[c] : nullptr;
    go(st, L, tx_blocks, k_tex0<true>, k_tex0<false>, SF_BLOCK, 0, in);
}

void launch_downsample(hipStream_t st, const Launch &L) {
    go(st, L, tx_blocks, k_texl<true>, k_texl<false>, SF_BLOCK, 0);
}

// Only the frames whose coarsest level is initialised by the network get
// workgroups (a batch may mix them with frames that start from zero).
void launch_cnn_candidate(hipStream_t st, const Launch &L) {
    auto nd = [](const LevelArgs &a) { return a.learned ? node_blocks(a.d) : 0; };
    auto en = [](const LevelArgs &a) { return a.learned ? energy_blocks_of(a.d) : 0; };
    go(st, L, nd, k_cnn_nodes<true>, k_cnn_nodes<false>, SF_BLOCK, 0);
    go(st, L, en, k_fallback<true>, k_fallback<false>, SF_BLOCK, 0);
}

void launch_level_masks(hipStream_t st, const Launch &L) {
    go(st, L, px_blocks, k_masks<true>, k_masks<false>, SF_BLOCK, 0);
    go(st, L, nd_blocks, k_node_weights<true>, k_node_weights<false>, SF_BLOCK, 0);
}

void launch_level_init(hipStream_t st, const Launch &L) {
    go(st, L, nd_blocks, k_prolong<true>, k_prolong<false>, SF_BLOCK, 0);
    launch_level_masks(st, L);
}

void launch_linearize(hipStream_t st, const Launch &L) {
    go(st, L, en_blocks, k_energy<true, true>, k_energy<false, true>, SF_BLOCK, 0, 0.f);
}

void launch_spec_linearize(hipStream_t st, const Launch &L) {
    go(st, L, en_blocks, k_energy<true, true>, k_energy<false, true>, SF_BLOCK, 0, 1.f);
}

void launch_trial0(hipStream_t st, const Launch &L) {
    go(st, L, en_blocks, k_energy<true, false>, k_energy<false, false>, SF_BLOCK, 0, 1.f);
}

void launch_trials_rest(hipStream_t st, const Launch &L, int n_rest, bool spec, int gn,
                        int pcg_iters) {
    auto nb = [](const LevelArgs &a) { return rest_blocks_of(a.d); };
    go(st, L, nb, k_trials_rest<true>, k_trials_rest<false>, SF_BLOCK, 0, n_rest, spec ? 1 : 0,
       gn, pcg_iters);
}

void launch_rhs(hipStream_t st, const Launch &L, const TileCfg &t) {
    auto nb = [t](const LevelArgs &a) { return node_tiles_of(a.d, t); };
    const int s = L.host[0].s;
#define RHS(S)                                                                           \
    go(st, L, nb, k_rhs<true, S>, k_rhs<false, S>, TileTraits<S>::NT,                    \
       node_tile_lds_bytes(t, S, 12), t)
    SF_STRIDE_SWITCH(s, RHS)
#undef RHS
}

// The PCG kernels per (stride, variant): the tile in t says which.
#define SF_PCG_SWITCH(s, v, CALL)                          \
    if ((v) == SF_TILE_NB) { CALL(0, 0); }                 \
    else if ((v) == SF_TILE_NB + 1) { CALL(0, 1); }        \
    else if ((v) == SF_TILE_NB + 2) { CALL(0, 2); }        \
    else if ((v) == SF_TILE_NB + 3) { CALL(0, 3); }        \
    else if ((s) == 2 && (v) == 1) { CALL(2, 1); }         \
    else if ((s) == 2 && (v) == 2) { CALL(2, 2); }         \
    else if ((s) == 4 && (v) == 1) { CALL(4, 1); }         \
    else if ((s) == 4 && (v) == 2) { CALL(4, 2); }         \
    else if ((s) == 8 && (v) == 1) { CALL(8, 1); }         \
    else if ((s) == 8 && (v) == 2) { CALL(8, 2); }         \
    else {                                                 \
        switch (s) {                                       \
            case 1: CALL(1, 0); break;                     \
            case 2: CALL(2, 0); break;                     \
            case 3: CALL(3, 0); break;                     \
            case 4: CALL(4, 0); break;                     \
            case 5: CALL(5, 0); break;                     \
            case 6: CALL(6, 0); break;                     \
            case 7: CALL(7, 0); break;                     \
            default: CALL(8, 0); break;                    \
        }                                                  \
    }

// Frames with at most SF_SMALL_G nodes are skipped by the multi-kernel PCG
// when `skip_small` (their PCG runs in launch_pcg_small).
static bool small_frame(const LevelArgs &a) { return a.d.G <= SF_SMALL_G; }

void launch_pcg_first(hipStream_t st, const Launch &L, const TileCfg &t, bool skip_small,
                      bool pend) {
    auto nb = [t, skip_small](const LevelArgs &a) {
        return skip_small && small_frame(a) ? 0 : node_tiles_of(a.d, t);
    };
    const int s = L.host[0].s;
#define PCG0(S, V)                                                                         \
    go(st, L, nb, k_pcg<true, true, S, V, true, false>, k_pcg<false, true, S, V, false, false>, \
       TileTraits<S, V>::NT, node_tile_lds_bytes(t, S, 6), t, 0, -1, pend ? 1 : 0)
    SF_PCG_SWITCH(s, t.v, PCG0)
#undef PCG0
}

void launch_pcg_iter(hipStream_t st, const Launch &L, const TileCfg &t, int iter, int gn,
                     int force, bool skip_small) {
    auto nb = [t, skip_small](const LevelArgs &a) {
        return skip_small && small_frame(a) ? 0 : node_tiles_of(a.d, t);
    };
    const int s = L.host[0].s;
    // the single-frame variant by the number of partial sums it reduces
    // (the previous iteration ran on the same tiles) and, node-block
    // products only, by its size
    const int nt1 = L.batched ? 0 : nb(L.host[0]);
    const bool wd = nt1 > SF_WD_TILES;
#define PCGI(S, V)                                                                            \
    {                                                                                         \
        auto kb = k_pcg<true, false, S, V, true, false>;                                      \
        const int nth = TileTraits<S, V>::NT;                                                 \
        const size_t lb = node_tile_lds_bytes(t, S, 6);                                       \
        if constexpr (S == 0) {                                                               \
            if ((long)nt1 * nth > SF_LATE_THREADS)                                            \
                go(st, L, nb, kb, k_pcg<false, false, S, V, true, true>, nth, lb, t, iter, gn, force); \
            else if (wd)                                                                      \
                go(st, L, nb, kb, k_pcg<false, false, S, V, true, false>, nth, lb, t, iter, gn, force); \
            else                                                                              \
                go(st, L, nb, kb, k_pcg<false, false, S, V, false, false>, nth, lb, t, iter, gn, force); \
        } else {                                                                              \
            if (wd)                                                                           \
                go(st, L, nb, kb, k_pcg<false, false, S, V, true, false>, nth, lb, t, iter, gn, force); \
            else                                                                              \
                go(st, L, nb, kb, k_pcg<false, false, S, V, false, false>, nth, lb, t, iter, gn, force); \
        }                                                                                     \
    }
    SF_PCG_SWITCH(s, t.v, PCGI)
#undef PCGI
}

void launch_rhs_blocks(hipStream_t st, const Launch &L, int n_pend, int gn_prev, int pcg_iters) {
    const int s = L.host[0].s;
    const TileCfg t = pick_blk_tile(s);
    auto nb = [t](const LevelArgs &a) { return node_tiles_of(a.d, t); };
#define BLK(S)                                                                            \
    go(st, L, nb, k_rhs_blocks<true, S>, k_rhs_blocks<false, S>, BlkTraits<S>::NT,        \
       blk_tile_lds_bytes(S), t, n_pend, gn_prev, pcg_iters)
    SF_STRIDE_SWITCH(s, BLK)
#undef BLK
}

// One workgroup per small frame with a wavefront per 21 of its nodes (the
// largest small frame of the launch sets the count).
void launch_pcg_small(hipStream_t st, const Launch &L, int n_it, int gn, bool pend) {
    auto one = [](const LevelArgs &a) { return small_frame(a) ? 1 : 0; };
    int gmax = 0;
    for (int f = 0; f < L.nf; ++f)
        if (small_frame(L.host[f])) gmax = gmax > L.host[f].d.G ? gmax : L.host[f].d.G;
    if (gmax == 0) return;
    const int threads = 64 * ((gmax + SMALL_NPW - 1) / SMALL_NPW);
    go(st, L, one, k_pcg_small<true>, k_pcg_small<false>, threads, 0, n_it, gn, pend ? 1 : 0);
}

int pt_tiles(const LevelDims &d) {
    return ((d.Gx + SF_PT_TW - 1) / SF_PT_TW) * ((d.Gy + SF_PT_TH - 1) / SF_PT_TH);
}

int pt_capacity() {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pcg_tile, PT_NT, 0) != hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

size_t pt_xtag_words(long G0) { return (size_t)7 * PT_REP * SF_PT_MAXWG + (size_t)2 * 18 * G0; }

void launch_pcg_tile(hipStream_t st, const Launch &L, int n_it, int gn, bool pend) {
    const LevelArgs &a = L.host[0];
    // about a second of polling before a wait gives up; SF_MID_SPIN_LIMIT
    // overrides it (tests force the give-up path with a tiny limit)
    int spin_limit = 1 << 20;
    if (const char *e = getenv("SF_MID_SPIN_LIMIT")) spin_limit = atoi(e);
    hipLaunchKernelGGL(k_pcg_tile, dim3(pt_tiles(a.d)), dim3(PT_NT), 0, st, a, n_it, gn,
                       spin_limit, pend ? 1 : 0);
}

void launch_pcg_last(hipStream_t st, const Launch &L, const TileCfg &t, int iter, int gn,
                     int force, bool skip_small) {
    auto nb = [skip_small](const LevelArgs &a) {
        return skip_small && small_frame(a) ? 0 : node_blocks(a.d);
    };
    go(st, L, nb, k_pcg_last<true>, k_pcg_last<false>, SF_BLOCK, 0, t, iter, gn, force);
}

void launch_accept(hipStream_t st, const Launch &L, int n_trials, int gn, int pcg_iters) {
    go(st, L, nd_blocks, k_accept<true>, k_accept<false>, SF_BLOCK, 0, n_trials, gn, pcg_iters);
}

void launch_illum_zero(hipStream_t st, const Launch &L) {
    auto nb = [](const LevelArgs &a) {
        return a.illum && a.coarsest ? (a.d.N + SF_BLOCK - 1) / SF_BLOCK : 0;
    };
    go(st, L, nb, k_illum_zero<true>, k_illum_zero<false>, SF_BLOCK, 0);
}

void launch_illum_next(hipStream_t st, const Launch &L) {
    auto on = [](const LevelArgs &a) { return a.illum && a.level > 0; };
    auto nr = [on](const LevelArgs &a) { return on(a) ? pixel_tiles(a.d) : 0; };
    auto nx = [on](const LevelArgs &a) { return on(a) ? (a.d.N + SF_BLOCK - 1) / SF_BLOCK : 0; };
    auto nu = [on](const LevelArgs &a) {
        return on(a) ? (int)(((long)a.Wf * a.Hf + SF_BLOCK - 1) / SF_BLOCK) : 0;
    };
    go(st, L, nr, k_illum_resid<true>, k_illum_resid<false>, SF_BLOCK, 0);
    go(st, L, nx, k_illum_blur_x<true>, k_illum_blur_x<false>, SF_BLOCK, 0);
    go(st, L, nu, k_illum_up<true>, k_illum_up<false>, SF_BLOCK, 0);
}

void launch_occ_next(hipStream_t st, const Launch &L) {
    auto on = [](const LevelArgs &a) { return a.occ_next != nullptr; };
    auto np = [on](const LevelArgs &a) { return on(a) ? pixel_tiles(a.d) : 0; };
    auto nq = [on](const LevelArgs &a) {
        const long q = 4L * (a.d.W - 1) * (a.d.H - 1);
        return on(a) && q > 0 ? (int)((q + SF_BLOCK - 1) / SF_BLOCK) : 0;
    };
    auto nt = [on](const LevelArgs &a) { return on(a) ? (a.d.N + SF_BLOCK - 1) / SF_BLOCK : 0; };
    go(st, L, np, k_occ_pos<true>, k_occ_pos<false>, SF_BLOCK, 0);
    go(st, L, nq, k_occ_raster<true>, k_occ_raster<false>, SF_BLOCK, 0);
    go(st, L, nt, k_occ_test<true>, k_occ_test<false>, SF_BLOCK, 0);
}

void launch_finish_level(hipStream_t st, const Launch &L) {
    go(st, L, nd_blocks, k_finish_level<true>, k_finish_level<false>, SF_BLOCK, 0);
}

// Workspace clearing and per-call constants of solves that bring their own
// workspace (no memset or host-to-device copy: both are plain kernels, so
// the launches can also be captured).
__global__ __launch_bounds__(SF_BLOCK) void k_fill_zero(uint4 *p, long n16) {
    const uint4 z = {0u, 0u, 0u, 0u};
    for (long i = (long)blockIdx.x * SF_BLOCK + threadIdx.x; i < n16;
         i += (long)gridDim.x * SF_BLOCK)
        p[i] = z;
}

__global__ __launch_bounds__(64) void k_store_const(DevConst k, DevConst *dst) {
    if (threadIdx.x == 0) *dst = k;
}

void launch_fill_zero(hipStream_t st, void *p, size_t bytes) {
    const long n16 = (long)(bytes / 16);
    if (n16 <= 0) return;
    const long want = (n16 + SF_BLOCK - 1) / SF_BLOCK;
    const int nb = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(SF_BLOCK), 0, st, (uint4 *)p, n16);
}

void launch_store_const(hipStream_t st, const DevConst &k, DevConst *dst) {
    hipLaunchKernelGGL(k_store_const, dim3(1), dim3(64), 0, st, k, dst);
}

void launch_output(hipStream_t st, const Launch &L, float *depth, float *flow3d,
                   float *flows) {
    go(st, L, px_blocks, k_output<true>, k_output<false>, SF_BLOCK, 0, depth, flow3d, flows);
}
