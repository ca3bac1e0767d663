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
// Every cross-workgroup sum is deterministic: each workgroup writes a
// partial, and the last workgroup to arrive sums all partials in a fixed
// order in double precision.
#include <math.h>

#include "sf_internal.h"

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
// first / last pixel whose bracket contains node i
__device__ __forceinline__ int sup_lo(int i, int s) {
    return i <= 1 ? 0 : ((2 * i - 1) * s) / 2;
}
__device__ __forceinline__ int sup_hi(int i, int s, int G, int W) {
    return i >= G - 2 ? W - 1 : min(W - 1, ((2 * i + 3) * s) / 2 - 1);
}

// ---- reductions ----------------------------------------------------------

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums K per-thread values over the (256-thread) block; the result is valid
// in thread 0.  Fixed order, so bitwise reproducible.
template <int K>
__device__ void block_sum(float (&v)[K], float (&out)[K]) {
    __shared__ float red[4][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float s = wave_sum(v[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
    __syncthreads();
}

// Sum in double of n partials (plane `plane` of the partial buffer) by the
// whole block; result valid in thread 0.
__device__ double block_sum_partials(const float *part, int n) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += (double)part[i];
    acc = wave_sum_d(acc);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    double r = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return r;
}

// Arrival at a device-wide counter: true in every thread of the last
// workgroup of the grid to arrive, which then sees all partials.
__device__ bool last_block(unsigned int *counter) {
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int total = gridDim.x * gridDim.y * gridDim.z;
        const unsigned int prev = atomicAdd(counter, 1u);
        s_last = (prev == total - 1) ? 1 : 0;
        if (s_last) atomicExch(counter, 0u);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

__device__ __forceinline__ int block_linear() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// ---- bilinear sampling of (I, Gx, Gy) ------------------------------------

// Value of the three channels at (px, py) and the derivatives of their
// bilinear interpolants; clamp-to-edge coordinates, zero derivative in a
// clamped direction.  All accesses stay inside the W x H image for any
// input, NaN included.
struct Samp {
    float v[3];   // I, Gx, Gy
    float dx[3];  // d/dpx
    float dy[3];  // d/dpy
};
__device__ __forceinline__ void sample3(const float4 *__restrict__ img, int W,
                                        int H, float px, float py, Samp &o) {
    const bool inx = (px >= 0.f) && (px <= (float)(W - 1));
    const bool iny = (py >= 0.f) && (py <= (float)(H - 1));
    const float cx = fminf(fmaxf(px, 0.f), (float)(W - 1));
    const float cy = fminf(fmaxf(py, 0.f), (float)(H - 1));
    const int x0 = min((int)floorf(cx), W - 2);
    const int y0 = min((int)floorf(cy), H - 2);
    const float fx = cx - (float)x0, fy = cy - (float)y0;
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
        o.dx[ch] = inx ? ((1.f - fy) * (tb[ch] - ta[ch]) + fy * (td[ch] - tc[ch])) : 0.f;
        o.dy[ch] = iny ? ((1.f - fx) * (tc[ch] - ta[ch]) + fx * (td[ch] - tb[ch])) : 0.f;
    }
}

// ---- pyramid --------------------------------------------------------------

struct Img4 {
    const float *p[4];
};

// Level 0: texel = (I, Gx, Gy, 0) with central-difference gradients
// (one-sided at the borders).
__global__ __launch_bounds__(SF_BLOCK) void k_tex0(Img4 in, float4 *tex, int W,
                                                   int H) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int c = blockIdx.z;
    if (x >= W || y >= H) return;
    const float *I = in.p[c];
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

__global__ __launch_bounds__(SF_BLOCK) void k_texl(const float4 *src, int Ws,
                                                   int Hs, float4 *dst, int W,
                                                   int H) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int c = blockIdx.z;
    if (x >= W || y >= H) return;
    const float4 *S = src + (long)c * Ws * Hs;
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
    const float *base = a.nodes + (long)NV_BASE * 6 * a.G0;
    const float *delta = a.nodes + (long)NV_DELTA * 6 * a.G0;
    const float *dx = a.nodes + (long)NV_DX * 6 * a.G0;
    for (int t = threadIdx.x; t < 6 * cw * ch; t += blockDim.x) {
        const int q = t / (cw * ch), r = t % (cw * ch);
        const int j = r / cw, i = r % cw;
        const long n = (long)(ny0 + j) * d.Gx + (nx0 + i);
        float dl = delta[q * a.G0 + n];
        if (tau != 0.f) dl = dl + tau * dx[q * a.G0 + n];
        S.t[q][j][i] = base[q * a.G0 + n] + dl;
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
        const float px = (((float)x + sgn(cam, 0) * f[0]) + sgn(cam, 1) * f[2]) + sgn(cam, 2) * f[4];
        const float py = (((float)y + sgn(cam, 0) * f[1]) + sgn(cam, 1) * f[3]) + sgn(cam, 2) * f[5];
        sample3(a.tex + (long)cam * d.N, d.W, d.H, px, py, S[cam]);
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

// blocks [0, n_pix): 16x16 pixel tiles; blocks [n_pix, grid): 256 nodes each
// for the regulariser energies.  mode 0 = linearise (records + E at delta),
// mode 1 = trial energy at delta + tau dx (skipped if an earlier trial of
// this step was accepted).
template <bool LIN>
__global__ __launch_bounds__(SF_BLOCK) void k_energy(LevelArgs a, int trial,
                                                     float tau, int n_before,
                                                     int n_pix) {
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    if (!LIN) {
        const double e0 = a.sc->e_lin[5];
        for (int k = 0; k < n_before; ++k)
            if (a.sc->e_trial[k][5] <= e0) return;  // uniform over the grid
    }
    __shared__ NodeStage S;
    float part[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const int bid = blockIdx.x;
    if (bid < n_pix) {
        const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
        const int x0 = (bid % tiles_x) * TILE_PX, y0 = (bid / tiles_x) * TILE_PX;
        stage_nodes(a, x0, y0, LIN ? 0.f : tau, S);
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
            part[0] = o.e_photo;
            part[1] = o.e_grad;
            if (LIN) {
#pragma unroll
                for (int q = 0; q < 6; ++q) a.rec[(long)q * a.N0 + pix] = o.grad[q];
#pragma unroll
                for (int t = 0; t < 21; ++t) a.rec[(long)(6 + t) * a.N0 + pix] = o.gram[t];
            }
        }
    } else {
        const int n = (bid - n_pix) * SF_BLOCK + threadIdx.x;
        if (n < d.G) {
            const int i = n % d.Gx, j = n / d.Gx;
            const float *base = a.nodes + (long)NV_BASE * 6 * a.G0;
            const float *delta = a.nodes + (long)NV_DELTA * 6 * a.G0;
            const float *dx = a.nodes + (long)NV_DX * 6 * a.G0;
            const float tt = LIN ? 0.f : tau;
            float dl[6], tot[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                dl[q] = delta[q * a.G0 + n];
                if (tt != 0.f) dl[q] = dl[q] + tt * dx[q * a.G0 + n];
                tot[q] = base[q * a.G0 + n] + dl[q];
            }
            const float wi = a.wnode[n];
            float es = 0.f;
            const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ii = i + nb[k][0], jj = j + nb[k][1];
                if (ii < 0 || ii >= d.Gx || jj < 0 || jj >= d.Gy) continue;
                const int m = jj * d.Gx + ii;
                float acc = 0.f;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    float dm = delta[q * a.G0 + m];
                    if (tt != 0.f) dm = dm + tt * dx[q * a.G0 + m];
                    const float df = dl[q] - dm;
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
    }
    float tot5[5];
    block_sum<5>(part, tot5);
    const int nb = gridDim.x;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) a.partials[(long)k * a.max_blocks + bid] = tot5[k];
    }
    if (last_block(&a.sc->counter[0])) {
        double s[5];
        for (int k = 0; k < 5; ++k) s[k] = block_sum_partials(a.partials + (long)k * a.max_blocks, nb);
        if (threadIdx.x == 0) {
            const double E = (double)C.w_photo * s[0] + (double)C.w_grad * s[1] +
                             (double)C.w_reg * ((double)C.w_smooth * s[2] +
                                                (double)C.w_epi * s[3] +
                                                (double)C.w_mag * s[4]);
            double *dst = LIN ? a.sc->e_lin : a.sc->e_trial[trial];
            for (int k = 0; k < 5; ++k) dst[k] = s[k];
            dst[5] = E;
        }
    }
}

// ---- node-tile reduction ---------------------------------------------------

// Accumulates K per-pixel values onto the nodes of a TX x TY tile through the
// bilinear weights of Eq. (7): value k is weighted by alpha (or alpha^2 if
// bit k of pow2 is set).  Pass 1 sums each pixel row onto node columns, pass
// 2 sums rows onto node rows; both in a fixed order.  Result in
// nodeAcc[(k * TY + tj) * TX + ti].
struct TileGeom {
    int i0, j0, txa, tya;  // tile origin and clipped size
    int X0, X1, Y0, Y1;    // pixel region
};

template <int K, class Fn>
__device__ void tile_reduce(const LevelArgs &a, const TileCfg &t,
                            const TileGeom &g, unsigned pow2, float *lds,
                            float *nodeAcc, Fn fn) {
    const int s = a.s;
    const LevelDims &d = a.d;
    const int RX = g.X1 - g.X0 + 1, RY = g.Y1 - g.Y0 + 1;
    const int RXs = (t.tx + 1) * s + 2, RYs = (t.ty + 1) * s + 2;
    float *vals = lds;                                    // K x RB x RXs
    float *accx = vals + K * t.rb * RXs;                  // K x TX x RYs
    // brackets of region columns / rows
    int *bxi = (int *)(accx + K * t.tx * RYs);            // RXs
    float *bxw0 = (float *)(bxi + RXs);
    float *bxw1 = bxw0 + RXs;
    int *byi = (int *)(bxw1 + RXs);                       // RYs
    float *byw0 = (float *)(byi + RYs);
    float *byw1 = byw0 + RYs;
    for (int u = threadIdx.x; u < RX; u += blockDim.x) {
        const Bracket b = bracket(g.X0 + u, s, d.Gx);
        bxi[u] = b.i0; bxw0[u] = b.w0; bxw1[u] = b.w1;
    }
    for (int u = threadIdx.x; u < RY; u += blockDim.x) {
        const Bracket b = bracket(g.Y0 + u, s, d.Gy);
        byi[u] = b.i0; byw0[u] = b.w0; byw1[u] = b.w1;
    }
    __syncthreads();
    for (int yb = g.Y0; yb <= g.Y1; yb += t.rb) {
        const int nr = min(t.rb, g.Y1 - yb + 1);
        for (int u = threadIdx.x; u < nr * RX; u += blockDim.x) {
            const int ry = u / RX, rx = u % RX;
            float v[K];
            fn(g.X0 + rx, yb + ry, rx, yb + ry - g.Y0, v);
#pragma unroll
            for (int k = 0; k < K; ++k) vals[(k * t.rb + ry) * RXs + rx] = v[k];
        }
        __syncthreads();
        for (int u = threadIdx.x; u < K * g.txa * nr; u += blockDim.x) {
            const int k = u / (g.txa * nr), rem = u % (g.txa * nr);
            const int ti = rem / nr, ry = rem % nr;
            const int i = g.i0 + ti;
            const int xa = max(sup_lo(i, s), g.X0) - g.X0;
            const int xb = min(sup_hi(i, s, d.Gx, d.W), g.X1) - g.X0;
            const bool sq = (pow2 >> k) & 1u;
            float acc = 0.f;
            for (int rx = xa; rx <= xb; ++rx) {
                float w = (bxi[rx] == i ? bxw0[rx] : 0.f) + (bxi[rx] + 1 == i ? bxw1[rx] : 0.f);
                if (d.Gx == 1) w = bxw0[rx];
                if (sq) w = w * w;
                acc += w * vals[(k * t.rb + ry) * RXs + rx];
            }
            accx[(k * t.tx + ti) * RYs + (yb - g.Y0 + ry)] = acc;
        }
        __syncthreads();
    }
    for (int u = threadIdx.x; u < K * g.txa * g.tya; u += blockDim.x) {
        const int k = u / (g.txa * g.tya), rem = u % (g.txa * g.tya);
        const int tj = rem / g.txa, ti = rem % g.txa;
        const int j = g.j0 + tj;
        const int ya = max(sup_lo(j, s), g.Y0) - g.Y0;
        const int yb = min(sup_hi(j, s, d.Gy, d.H), g.Y1) - g.Y0;
        const bool sq = (pow2 >> k) & 1u;
        float acc = 0.f;
        for (int ry = ya; ry <= yb; ++ry) {
            float w = (byi[ry] == j ? byw0[ry] : 0.f) + (byi[ry] + 1 == j ? byw1[ry] : 0.f);
            if (d.Gy == 1) w = byw0[ry];
            if (sq) w = w * w;
            acc += w * accx[(k * t.tx + ti) * RYs + ry];
        }
        nodeAcc[(k * t.ty + tj) * t.tx + ti] = acc;
    }
    __syncthreads();
}

__device__ __forceinline__ TileGeom tile_geom(const LevelArgs &a, const TileCfg &t) {
    TileGeom g;
    const LevelDims &d = a.d;
    g.i0 = blockIdx.x * t.tx;
    g.j0 = blockIdx.y * t.ty;
    g.txa = min(t.tx, d.Gx - g.i0);
    g.tya = min(t.ty, d.Gy - g.j0);
    g.X0 = sup_lo(g.i0, a.s);
    g.X1 = sup_hi(g.i0 + g.txa - 1, a.s, d.Gx, d.W);
    g.Y0 = sup_lo(g.j0, a.s);
    g.Y1 = sup_hi(g.j0 + g.tya - 1, a.s, d.Gy, d.H);
    return g;
}

// Shared-memory layout sizes (floats) of a node-tile kernel.
__host__ __device__ inline size_t tile_lds_floats(const TileCfg &t, int s, int K) {
    const size_t RXs = (size_t)(t.tx + 1) * s + 2, RYs = (size_t)(t.ty + 1) * s + 2;
    return (size_t)K * t.rb * RXs + (size_t)K * t.tx * RYs + 3 * RXs + 3 * RYs +
           (size_t)K * t.tx * t.ty;
}

// Regulariser gradient / diagonal / product on one node.
//   smooth (Eq. (14), ordered 4-neighbour pairs on the deltas):
//     grad += 2 w_reg w_smooth w_f sum_j (w_i + w_j)(D_i - D_j)
//   epipolar (Eqs. (15)-(17), on totals): grad += 2 w_reg w_epi sum_t e_t de_t
//   magnitude (Eq. (18), on deltas): grad += 2 w_reg w_mag m_f D_i
// The Gauss-Newton matrix of these least-squares terms is 2 J^T J.

// ---- right-hand side and PCG start (node tiles) ----------------------------

__global__ __launch_bounds__(SF_BLOCK) void k_node_rhs(LevelArgs a, TileCfg t) {
    extern __shared__ float lds[];
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    const TileGeom g = tile_geom(a, t);
    float *nodeAcc = lds + (tile_lds_floats(t, a.s, 12) - (size_t)12 * t.tx * t.ty);
    const float *rec = a.rec;
    const long N0 = a.N0;
    tile_reduce<12>(a, t, g, 0xFC0u, lds, nodeAcc,
                    [&](int x, int y, int, int, float (&v)[12]) {
                        const long pix = (long)y * d.W + x;
#pragma unroll
                        for (int q = 0; q < 6; ++q) v[q] = rec[q * N0 + pix];
#pragma unroll
                        for (int q = 0; q < 6; ++q) {
                            const int tq = q * 6 - (q * (q - 1)) / 2;  // tri(q, q)
                            v[6 + q] = rec[(6 + tq) * N0 + pix];
                        }
                    });
    float prt[2] = {0.f, 0.f};
    const int nt = g.txa * g.tya;
    if ((int)threadIdx.x < nt) {
        const int ti = threadIdx.x % g.txa, tj = threadIdx.x / g.txa;
        const int i = g.i0 + ti, j = g.j0 + tj;
        const long n = (long)j * d.Gx + i;
        const long G0 = a.G0;
        float *base = a.nodes + (long)NV_BASE * 6 * G0;
        float *delta = a.nodes + (long)NV_DELTA * 6 * G0;
        float grad[6], dg[6], dl[6], tot[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            grad[q] = nodeAcc[(q * t.ty + tj) * t.tx + ti];
            dg[q] = nodeAcc[((6 + q) * t.ty + tj) * t.tx + ti];
            dl[q] = delta[q * G0 + n];
            tot[q] = base[q * G0 + n] + dl[q];
        }
        const float wi = a.wnode[n];
        const float cs = 2.f * C.w_reg * C.w_smooth;
        const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ii = i + nb[k][0], jj = j + nb[k][1];
            if (ii < 0 || ii >= d.Gx || jj < 0 || jj >= d.Gy) continue;
            const long m = (long)jj * d.Gx + ii;
            const float wsum = wi + a.wnode[m];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                grad[q] += cs * C.wf[q] * wsum * (dl[q] - delta[q * G0 + m]);
                dg[q] += cs * C.wf[q] * wsum;
            }
        }
        float gx, gy;
        node_xy(i, j, a.s, gx, gy);
        float e[2], J[2][6];
        epi_terms(C.F[a.level], gx, gy, tot, e, J);
        const float ce = 2.f * C.w_reg * C.w_epi, cm = 2.f * C.w_reg * C.w_mag;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            grad[q] += ce * (e[0] * J[0][q] + e[1] * J[1][q]);
            dg[q] += ce * (J[0][q] * J[0][q] + J[1][q] * J[1][q]);
            grad[q] += cm * C.mf[q] * dl[q];
            dg[q] += cm * C.mf[q];
        }
        float *X = a.nodes + (long)NV_DX * 6 * G0;
        float *R = a.nodes + (long)NV_R * 6 * G0;
        float *Z = a.nodes + (long)NV_Z * 6 * G0;
        float *D = a.nodes + (long)NV_DIAG * 6 * G0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float r = -grad[q];
            const float z = r / dg[q];
            X[q * G0 + n] = 0.f;
            R[q * G0 + n] = r;
            Z[q * G0 + n] = z;
            D[q * G0 + n] = dg[q];
            prt[0] += r * z;
            prt[1] += r * r;
        }
    }
    float tot2[2];
    block_sum<2>(prt, tot2);
    const int bid = block_linear();
    const int nb = gridDim.x * gridDim.y;
    if (threadIdx.x == 0) {
        a.partials[bid] = tot2[0];
        a.partials[(long)a.max_blocks + bid] = tot2[1];
    }
    if (last_block(&a.sc->counter[1])) {
        const double rz = block_sum_partials(a.partials, nb);
        const double rr = block_sum_partials(a.partials + a.max_blocks, nb);
        if (threadIdx.x == 0) {
            a.sc->rz = rz;
            a.sc->rr = rr;
            a.sc->active = rz > 1e-30 ? 1 : 0;
            a.sc->first = 1;
            a.sc->beta = 0.f;
        }
    }
}

// ---- q = H p (node tiles) --------------------------------------------------

__global__ __launch_bounds__(SF_BLOCK) void k_apply(LevelArgs a, TileCfg t,
                                                    int iter) {
    extern __shared__ float lds[];
    DevScalars *sc = a.sc;
    if (!sc->active) return;  // uniform over the grid
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    const TileGeom g = tile_geom(a, t);
    const long G0 = a.G0;
    const int first = sc->first;
    const float beta = sc->beta;
    const size_t base_f = tile_lds_floats(t, a.s, 6);
    float *nodeAcc = lds + (base_f - (size_t)6 * t.tx * t.ty);
    float *pS = lds + base_f;  // 6 x (TY+2) x (TX+2), halo of one node
    const int HX = t.tx + 2, HY = t.ty + 2;
    const float *Z = a.nodes + (long)NV_Z * 6 * G0;
    float *Pc = a.nodes + (long)((iter & 1) ? NV_P1 : NV_P0) * 6 * G0;
    const float *Po = a.nodes + (long)((iter & 1) ? NV_P0 : NV_P1) * 6 * G0;
    // p = z + beta p_old on the tile and its halo; owned nodes stored
    const int hx0 = max(g.i0 - 1, 0), hx1 = min(g.i0 + g.txa, d.Gx - 1);
    const int hy0 = max(g.j0 - 1, 0), hy1 = min(g.j0 + g.tya, d.Gy - 1);
    const int hw = hx1 - hx0 + 1, hh = hy1 - hy0 + 1;
    for (int u = threadIdx.x; u < hw * hh; u += blockDim.x) {
        const int ni = hx0 + u % hw, nj = hy0 + u / hw;
        const long n = (long)nj * d.Gx + ni;
        const bool own = ni >= g.i0 && ni < g.i0 + g.txa && nj >= g.j0 && nj < g.j0 + g.tya;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            float p = Z[q * G0 + n];
            if (!first) p = p + beta * Po[q * G0 + n];
            pS[(q * HY + (nj - g.j0 + 1)) * HX + (ni - g.i0 + 1)] = p;
            if (own) Pc[q * G0 + n] = p;
        }
    }
    __syncthreads();
    const float *rec = a.rec + 6 * (long)a.N0;
    const long N0 = a.N0;
    const int s = a.s;
    tile_reduce<6>(a, t, g, 0u, lds, nodeAcc,
                   [&](int x, int y, int, int, float (&v)[6]) {
                       const Bracket bx = bracket(x, s, d.Gx), by = bracket(y, s, d.Gy);
                       const int lx0 = bx.i0 - g.i0 + 1, lx1 = bx.i1 - g.i0 + 1;
                       const int ly0 = by.i0 - g.j0 + 1, ly1 = by.i1 - g.j0 + 1;
                       float pv[6];
#pragma unroll
                       for (int q = 0; q < 6; ++q) {
                           const float *P = pS + q * HY * HX;
                           pv[q] = by.w0 * (bx.w0 * P[ly0 * HX + lx0] + bx.w1 * P[ly0 * HX + lx1]) +
                                   by.w1 * (bx.w0 * P[ly1 * HX + lx0] + bx.w1 * P[ly1 * HX + lx1]);
                       }
                       const long pix = (long)y * d.W + x;
                       float G[21];
#pragma unroll
                       for (int k = 0; k < 21; ++k) G[k] = rec[k * N0 + pix];
#pragma unroll
                       for (int i = 0; i < 6; ++i) {
                           float acc = 0.f;
#pragma unroll
                           for (int j = 0; j < 6; ++j)
                               acc += G[i <= j ? tri(i, j) : tri(j, i)] * pv[j];
                           v[i] = acc;
                       }
                   });
    float prt[2] = {0.f, 0.f};
    const int nt = g.txa * g.tya;
    if ((int)threadIdx.x < nt) {
        const int ti = threadIdx.x % g.txa, tj = threadIdx.x / g.txa;
        const int i = g.i0 + ti, j = g.j0 + tj;
        const long n = (long)j * d.Gx + i;
        const float *base = a.nodes + (long)NV_BASE * 6 * G0;
        const float *delta = a.nodes + (long)NV_DELTA * 6 * G0;
        float p[6], q6[6], tot[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            p[q] = pS[(q * HY + tj + 1) * HX + ti + 1];
            q6[q] = nodeAcc[(q * t.ty + tj) * t.tx + ti];
            tot[q] = base[q * G0 + n] + delta[q * G0 + n];
        }
        const float wi = a.wnode[n];
        const float cs = 2.f * C.w_reg * C.w_smooth;
        const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ii = i + nb[k][0], jj = j + nb[k][1];
            if (ii < 0 || ii >= d.Gx || jj < 0 || jj >= d.Gy) continue;
            const float wsum = wi + a.wnode[(long)jj * d.Gx + ii];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                q6[q] += cs * C.wf[q] * wsum * (p[q] - pS[(q * HY + tj + 1 + nb[k][1]) * HX + ti + 1 + nb[k][0]]);
        }
        float gx, gy;
        node_xy(i, j, a.s, gx, gy);
        float e[2], J[2][6];
        epi_terms(C.F[a.level], gx, gy, tot, e, J);
        float jp0 = 0.f, jp1 = 0.f;
#pragma unroll
        for (int q = 0; q < 6; ++q) { jp0 += J[0][q] * p[q]; jp1 += J[1][q] * p[q]; }
        const float ce = 2.f * C.w_reg * C.w_epi, cm = 2.f * C.w_reg * C.w_mag;
        float *Q = a.nodes + (long)NV_Q * 6 * G0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            q6[q] += ce * (J[0][q] * jp0 + J[1][q] * jp1) + cm * C.mf[q] * p[q];
            Q[q * G0 + n] = q6[q];
            prt[0] += p[q] * q6[q];
            prt[1] += p[q] * p[q];
        }
    }
    float tot2[2];
    block_sum<2>(prt, tot2);
    const int bid = block_linear();
    const int nb = gridDim.x * gridDim.y;
    if (threadIdx.x == 0) {
        a.partials[bid] = tot2[0];
        a.partials[(long)a.max_blocks + bid] = tot2[1];
    }
    if (last_block(&sc->counter[1])) {
        const double pq = block_sum_partials(a.partials, nb);
        const double pp = block_sum_partials(a.partials + a.max_blocks, nb);
        if (threadIdx.x == 0) {
            sc->pq = pq;
            sc->pp = pp;
            const int act = pq > 1e-30 * pp ? 1 : 0;
            sc->active = act;
            sc->alpha = act ? (float)(sc->rz / pq) : 0.f;
        }
    }
}

// ---- x += alpha p, r -= alpha q, z = r / diag ------------------------------

__global__ __launch_bounds__(SF_BLOCK) void k_update(LevelArgs a, int iter,
                                                     int log_index) {
    DevScalars *sc = a.sc;
    if (!sc->active) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && log_index >= 0)
            a.log[log_index].pcg_res[iter] = (float)sqrt(sc->rr);
        return;
    }
    const long G0 = a.G0;
    const float alpha = sc->alpha;
    float *X = a.nodes + (long)NV_DX * 6 * G0;
    float *R = a.nodes + (long)NV_R * 6 * G0;
    float *Z = a.nodes + (long)NV_Z * 6 * G0;
    const float *Pc = a.nodes + (long)((iter & 1) ? NV_P1 : NV_P0) * 6 * G0;
    const float *Q = a.nodes + (long)NV_Q * 6 * G0;
    const float *D = a.nodes + (long)NV_DIAG * 6 * G0;
    float prt[2] = {0.f, 0.f};
    const long n = (long)blockIdx.x * SF_BLOCK + threadIdx.x;
    if (n < a.d.G) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const long k = q * G0 + n;
            X[k] = X[k] + alpha * Pc[k];
            const float r = R[k] - alpha * Q[k];
            const float z = r / D[k];
            R[k] = r;
            Z[k] = z;
            prt[0] += r * z;
            prt[1] += r * r;
        }
    }
    float tot2[2];
    block_sum<2>(prt, tot2);
    if (threadIdx.x == 0) {
        a.partials[blockIdx.x] = tot2[0];
        a.partials[(long)a.max_blocks + blockIdx.x] = tot2[1];
    }
    if (last_block(&sc->counter[1])) {
        const double rz = block_sum_partials(a.partials, gridDim.x);
        const double rr = block_sum_partials(a.partials + a.max_blocks, gridDim.x);
        if (threadIdx.x == 0) {
            sc->rr = rr;
            if (log_index >= 0) a.log[log_index].pcg_res[iter] = (float)sqrt(rr);
            if (rz > 1e-30) {
                sc->beta = (float)(rz / sc->rz);
                sc->rz = rz;
                sc->first = 0;
            } else {
                sc->active = 0;
            }
        }
    }
}

// ---- step control: accept the first tau with E_trial <= E ------------------

__global__ __launch_bounds__(SF_BLOCK) void k_accept(LevelArgs a, int n_trials,
                                                     int log_index, int gn_iter,
                                                     int pcg_iters) {
    const DevScalars *sc = a.sc;
    const double e0 = sc->e_lin[5];
    int kacc = -1;
    for (int k = 0; k < n_trials; ++k)
        if (sc->e_trial[k][5] <= e0) { kacc = k; break; }
    const float tau = kacc >= 0 ? ldexpf(1.f, -kacc) : 0.f;
    const long G0 = a.G0;
    const long n = (long)blockIdx.x * SF_BLOCK + threadIdx.x;
    if (kacc >= 0 && n < a.d.G) {
        float *delta = a.nodes + (long)NV_DELTA * 6 * G0;
        const float *X = a.nodes + (long)NV_DX * 6 * G0;
#pragma unroll
        for (int q = 0; q < 6; ++q) delta[q * G0 + n] = delta[q * G0 + n] + tau * X[q * G0 + n];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && log_index >= 0) {
        DevLog &L = a.log[log_index];
        L.level = a.level;
        L.gn_iter = gn_iter;
        L.energy = e0;
        L.e_photo = sc->e_lin[0];
        L.e_grad = sc->e_lin[1];
        L.e_smooth = sc->e_lin[2];
        L.e_epi = sc->e_lin[3];
        L.e_mag = sc->e_lin[4];
        L.energy_after = kacc >= 0 ? sc->e_trial[kacc][5] : e0;
        L.tau = tau;
        L.pcg_iters = pcg_iters;
        L.n_valid = sc->n_valid;
    }
}

// ---- level start: prolongation, masks, smoothness weights -------------------

// base_l = 2 bilerp(total_{l+1}) at coarse-node coordinate i/2 - 1/4
// (Sec. 5.3), or zero at the coarsest level; delta = 0.
__global__ __launch_bounds__(SF_BLOCK) void k_prolong(LevelArgs a, int Gxc, int Gyc,
                                                      int coarsest) {
    const long n = (long)blockIdx.x * SF_BLOCK + threadIdx.x;
    if (n >= a.d.G) return;
    const long G0 = a.G0;
    float *base = a.nodes + (long)NV_BASE * 6 * G0;
    float *delta = a.nodes + (long)NV_DELTA * 6 * G0;
    const float *tp = a.nodes + (long)NV_TPREV * 6 * G0;
    const int i = (int)(n % a.d.Gx), j = (int)(n / a.d.Gx);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        float v = 0.f;
        if (!coarsest) {
            // fine node i has coarse coordinate (2i - 1)/4: the bracket rule
            // with stride 2
            const Bracket bx = bracket(i, 2, Gxc), by = bracket(j, 2, Gyc);
            const float *T = tp + q * G0;
            v = 2.f * (by.w0 * (bx.w0 * T[by.i0 * Gxc + bx.i0] + bx.w1 * T[by.i0 * Gxc + bx.i1]) +
                       by.w1 * (bx.w0 * T[by.i1 * Gxc + bx.i0] + bx.w1 * T[by.i1 * Gxc + bx.i1]));
        }
        base[q * G0 + n] = v;
        delta[q * G0 + n] = 0.f;
    }
}

// V(x): all four positions inside the level image; W(x): max_k |d_k| <
// eps_p (Sec. 4.1); both at the level-start flow.  Also stores the mean of
// the four warped images for the smoothness weights.
__global__ __launch_bounds__(SF_BLOCK) void k_masks(LevelArgs a, int n_pix) {
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    __shared__ NodeStage S;
    const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
    const int bid = blockIdx.x;
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
            const float px = (((float)x + sgn(cam, 0) * f[0]) + sgn(cam, 1) * f[2]) + sgn(cam, 2) * f[4];
            const float py = (((float)y + sgn(cam, 0) * f[1]) + sgn(cam, 1) * f[3]) + sgn(cam, 2) * f[5];
            V = V && px >= 0.f && px <= (float)(d.W - 1) && py >= 0.f && py <= (float)(d.H - 1);
            Samp sm;
            sample3(a.tex + (long)cam * d.N, d.W, d.H, px, py, sm);
            I[cam] = sm.v[0];
        }
        float dmax = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) dmax = fmaxf(dmax, fabsf(I[pair_a(k)] - I[pair_b(k)]));
        const bool Wm = dmax < C.eps_p;
        const int pix = y * d.W + x;
        a.cmask[pix] = (V && Wm) ? 1 : 0;
        a.rec[pix] = 0.25f * (((I[0] + I[1]) + I[2]) + I[3]);
        cnt[0] = (V && Wm) ? 1.f : 0.f;
    }
    float tot1[1];
    block_sum<1>(cnt, tot1);
    if (threadIdx.x == 0) a.partials[bid] = tot1[0];
    if (last_block(&a.sc->counter[2])) {
        const double c = block_sum_partials(a.partials, gridDim.x);
        if (threadIdx.x == 0) a.sc->n_valid = (int)c;
    }
}

// w_i = 1 + gamma exp(-lambda_min / tau_l) of the structure tensor of the
// mean warped image over a 3x3 window at the node's rounded position.
__global__ __launch_bounds__(SF_BLOCK) void k_node_weights(LevelArgs a) {
    const long n = (long)blockIdx.x * SF_BLOCK + threadIdx.x;
    const LevelDims &d = a.d;
    if (n >= d.G) return;
    const DevConst &C = *a.cst;
    const int i = (int)(n % d.Gx), j = (int)(n / d.Gx);
    const float *Ib = a.rec;
    const int cx = min(((2 * i + 1) * a.s) / 2, d.W - 1);
    const int cy = min(((2 * j + 1) * a.s) / 2, d.H - 1);
    float A = 0.f, B = 0.f, Cc = 0.f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = min(max(cx + dx, 0), d.W - 1);
            const int yy = min(max(cy + dy, 0), d.H - 1);
            float gx, gy;
            if (xx == 0) gx = Ib[yy * d.W + 1] - Ib[yy * d.W];
            else if (xx == d.W - 1) gx = Ib[yy * d.W + xx] - Ib[yy * d.W + xx - 1];
            else gx = 0.5f * (Ib[yy * d.W + xx + 1] - Ib[yy * d.W + xx - 1]);
            if (yy == 0) gy = Ib[d.W + xx] - Ib[xx];
            else if (yy == d.H - 1) gy = Ib[yy * d.W + xx] - Ib[(yy - 1) * d.W + xx];
            else gy = 0.5f * (Ib[(yy + 1) * d.W + xx] - Ib[(yy - 1) * d.W + xx]);
            A += gx * gx;
            B += gx * gy;
            Cc += gy * gy;
        }
    const float h = 0.5f * (A - Cc);
    const float lmin = 0.5f * (A + Cc) - sqrtf(h * h + B * B);
    const float tau = C.st_tau * ldexpf(1.f, 2 * a.level);
    a.wnode[n] = 1.f + C.st_gamma * expf(-fmaxf(lmin, 0.f) / tau);
}

__global__ __launch_bounds__(SF_BLOCK) void k_finish_level(LevelArgs a) {
    const long n = (long)blockIdx.x * SF_BLOCK + threadIdx.x;
    if (n >= a.d.G) return;
    const long G0 = a.G0;
    const float *base = a.nodes + (long)NV_BASE * 6 * G0;
    const float *delta = a.nodes + (long)NV_DELTA * 6 * G0;
    float *tp = a.nodes + (long)NV_TPREV * 6 * G0;
#pragma unroll
    for (int q = 0; q < 6; ++q) tp[q * G0 + n] = base[q * G0 + n] + delta[q * G0 + n];
}

// ---- output: depth and 3D flow at level 0 -----------------------------------

__global__ __launch_bounds__(SF_BLOCK) void k_output(LevelArgs a, float *depth,
                                                     float *flow3d, float *flows) {
    const LevelDims &d = a.d;
    const DevConst &C = *a.cst;
    __shared__ NodeStage S;
    const int tiles_x = (d.W + TILE_PX - 1) / TILE_PX;
    const int bid = blockIdx.x;
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
        const float lx = (((float)x + sgn(cl, 0) * f[0]) + sgn(cl, 1) * f[2]) + sgn(cl, 2) * f[4];
        const float ly = (((float)y + sgn(cl, 0) * f[1]) + sgn(cl, 1) * f[3]) + sgn(cl, 2) * f[5];
        const float rx = (((float)x + sgn(cr, 0) * f[0]) + sgn(cr, 1) * f[2]) + sgn(cr, 2) * f[4];
        const float disp = lx - rx;
        const float Z = disp > 0.f ? C.fx * C.baseline / disp : __builtin_nanf("");
        X[t][0] = (lx - C.cx) * Z / C.fx;
        X[t][1] = (ly - C.cy) * Z / C.fy;
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

__global__ void k_set_apply_state(DevScalars *sc) {
    if (threadIdx.x == 0) {
        sc->active = 1;
        sc->first = 1;
        sc->beta = 0.f;
    }
}

// A mid-solve PCG state for timing: active, not the first iteration, so
// every launch does the full work (p = z + beta p_old, all updates).
__global__ void k_set_pcg_state(DevScalars *sc) {
    if (threadIdx.x == 0) {
        sc->active = 1;
        sc->first = 0;
        sc->beta = 0.5f;
        sc->alpha = 0.f;
        sc->rz = 1.0;
    }
}

}  // namespace

// ---- launchers ----------------------------------------------------------------

size_t node_tile_lds_bytes(const TileCfg &t, int s, int K) {
    size_t f = tile_lds_floats(t, s, K);
    if (K == 6) f += (size_t)6 * (t.tx + 2) * (t.ty + 2);
    return f * sizeof(float);
}

static int pixel_tiles(const LevelDims &d) {
    return ((d.W + TILE_PX - 1) / TILE_PX) * ((d.H + TILE_PX - 1) / TILE_PX);
}

int energy_blocks(const LevelDims &d) {
    return pixel_tiles(d) + (d.G + SF_BLOCK - 1) / SF_BLOCK;
}

int node_tile_blocks(const LevelDims &d, const TileCfg &t) {
    return ((d.Gx + t.tx - 1) / t.tx) * ((d.Gy + t.ty - 1) / t.ty);
}

void launch_tex_level0(hipStream_t st, const float *const img[4], float4 *tex,
                       int W, int H) {
    Img4 in;
    for (int c = 0; c < 4; ++c) in.p[c] = img[c];
    dim3 grid((W + 63) / 64, (H + 3) / 4, 4);
    hipLaunchKernelGGL(k_tex0, grid, dim3(SF_BLOCK), 0, st, in, tex, W, H);
}

void launch_downsample(hipStream_t st, const float4 *src, int Ws, int Hs,
                       float4 *dst, int Wd, int Hd) {
    dim3 grid((Wd + 63) / 64, (Hd + 3) / 4, 4);
    hipLaunchKernelGGL(k_texl, grid, dim3(SF_BLOCK), 0, st, src, Ws, Hs, dst, Wd, Hd);
}

void launch_level_init(hipStream_t st, const LevelArgs &a,
                       const LevelDims *coarse, bool coarsest) {
    const int gn = (a.d.G + SF_BLOCK - 1) / SF_BLOCK;
    hipLaunchKernelGGL(k_prolong, dim3(gn), dim3(SF_BLOCK), 0, st, a,
                       coarse ? coarse->Gx : 1, coarse ? coarse->Gy : 1,
                       coarsest ? 1 : 0);
    const int np = pixel_tiles(a.d);
    hipLaunchKernelGGL(k_masks, dim3(np), dim3(SF_BLOCK), 0, st, a, np);
    hipLaunchKernelGGL(k_node_weights, dim3(gn), dim3(SF_BLOCK), 0, st, a);
}

void launch_energy(hipStream_t st, const LevelArgs &a, int mode, int trial,
                   float tau, int n_before) {
    const int np = pixel_tiles(a.d);
    const int nb = energy_blocks(a.d);
    if (mode == 0)
        hipLaunchKernelGGL(k_energy<true>, dim3(nb), dim3(SF_BLOCK), 0, st, a, trial, tau, n_before, np);
    else
        hipLaunchKernelGGL(k_energy<false>, dim3(nb), dim3(SF_BLOCK), 0, st, a, trial, tau, n_before, np);
}

void launch_node_rhs(hipStream_t st, const LevelArgs &a, const TileCfg &t) {
    dim3 grid((a.d.Gx + t.tx - 1) / t.tx, (a.d.Gy + t.ty - 1) / t.ty);
    hipLaunchKernelGGL(k_node_rhs, grid, dim3(SF_BLOCK), node_tile_lds_bytes(t, a.s, 12), st, a, t);
}

void launch_apply(hipStream_t st, const LevelArgs &a, const TileCfg &t, int iter,
                  int) {
    dim3 grid((a.d.Gx + t.tx - 1) / t.tx, (a.d.Gy + t.ty - 1) / t.ty);
    hipLaunchKernelGGL(k_apply, grid, dim3(SF_BLOCK), node_tile_lds_bytes(t, a.s, 6), st, a, t, iter);
}

void launch_update(hipStream_t st, const LevelArgs &a, int iter, int log_index) {
    const int gn = (a.d.G + SF_BLOCK - 1) / SF_BLOCK;
    hipLaunchKernelGGL(k_update, dim3(gn), dim3(SF_BLOCK), 0, st, a, iter, log_index);
}

void launch_accept(hipStream_t st, const LevelArgs &a, int n_trials,
                   int log_index, int gn_iter, int pcg_iters) {
    const int gn = (a.d.G + SF_BLOCK - 1) / SF_BLOCK;
    hipLaunchKernelGGL(k_accept, dim3(gn), dim3(SF_BLOCK), 0, st, a, n_trials, log_index,
                       gn_iter, pcg_iters);
}

void launch_finish_level(hipStream_t st, const LevelArgs &a) {
    const int gn = (a.d.G + SF_BLOCK - 1) / SF_BLOCK;
    hipLaunchKernelGGL(k_finish_level, dim3(gn), dim3(SF_BLOCK), 0, st, a);
}

void launch_output(hipStream_t st, const LevelArgs &a, float *depth,
                   float *flow3d, float *flows) {
    hipLaunchKernelGGL(k_output, dim3(pixel_tiles(a.d)), dim3(SF_BLOCK), 0, st, a,
                       depth, flow3d, flows);
}

void launch_set_apply_state(hipStream_t st, DevScalars *sc) {
    hipLaunchKernelGGL(k_set_apply_state, dim3(1), dim3(64), 0, st, sc);
}

void launch_set_pcg_state(hipStream_t st, DevScalars *sc) {
    hipLaunchKernelGGL(k_set_pcg_state, dim3(1), dim3(64), 0, st, sc);
}
