// Internal types shared by the host orchestration and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sf.h"

#define SF_MAX_LEVELS 12
#define SF_MAX_TRIALS 8
#define SF_MAX_PCG 64
#define SF_BLOCK 256

// Number of per-pixel record planes: 6 gradient components of the pixel's
// energy w.r.t. its six flow components, then the 21 upper-triangular
// entries of its reweighted Gauss-Newton block J^T Omega J.
#define SF_REC_GRAD 6
#define SF_REC_GRAM 21
#define SF_REC_PLANES 27

// Node vectors (each 6 planes of G_0 floats).
enum {
    NV_BASE = 0,
    NV_DELTA,
    NV_DX,
    NV_R,
    NV_Z,
    NV_P0,
    NV_P1,
    NV_Q,
    NV_DIAG,
    NV_TPREV,
    NV_COUNT
};

// Sizes of one pyramid level.
struct LevelDims {
    int W, H;      // pixels
    int Gx, Gy;    // warp-grid nodes
    int N, G;      // W*H, Gx*Gy
    long tex_off;  // offset of this level's texels (float4 units)
};

// Weights, calibration and per-level fundamental matrices, kept in device
// memory so that a captured graph picks up new values on replay.
struct DevConst {
    float w_reg, w_photo, w_grad, w_epi, w_smooth, w_mag;
    float wf[6];  // w_s, w_s, w_m, w_m, w_d, w_d
    float mf[6];  // m_s, m_s, m_m, m_m, m_d, m_d
    float eps, eps_p, st_gamma, st_tau;
    float fx, fy, cx, cy, baseline;
    float F[SF_MAX_LEVELS][9];  // fundamental matrix in level pixels
};

// Device-resident scalars of the solve.  Each is written by the last
// workgroup of the kernel that reduces it and read by later kernels only.
struct DevScalars {
    unsigned int counter[4];          // arrival counters (reset by the last)
    double e_lin[6];                  // photo, grad, smooth, epi, mag, total
    double e_trial[SF_MAX_TRIALS][6]; // same for each trial step length
    double rz, rr, pq, pp;            // PCG inner products
    float alpha, beta;
    int active, first;
    int n_valid;
    int pad;
};

// Device log record (mirrors sf_iter_log).
struct DevLog {
    int level, gn_iter;
    double energy, e_photo, e_grad, e_smooth, e_epi, e_mag, energy_after;
    float tau;
    int pcg_iters;
    float pcg_res[SF_MAX_PCG];
    int n_valid;
};

// Launch geometry of the node-tile kernels.
struct TileCfg {
    int tx, ty;    // nodes per workgroup
    int rb;        // pixel rows per strip of the pixel->node reduction
};

// Everything a kernel needs about the current level, by value.
struct LevelArgs {
    LevelDims d;
    int level;
    int s;                 // grid stride
    int N0, G0;            // plane strides of records / node vectors
    const float4 *tex;     // this level's 4 images (image-major)
    float *nodes;          // base of all node vectors
    float *rec;            // per-pixel records
    unsigned char *cmask;  // V(x) W(x)
    float *wnode;          // smoothness weights
    float *partials;       // per-workgroup partial sums
    int max_blocks;        // stride of the partial-sum planes
    const DevConst *cst;
    DevScalars *sc;
    DevLog *log;
};

// Kernel launchers (sf_kernels.hip).
void launch_tex_level0(hipStream_t st, const float *const img[4], float4 *tex,
                       int W, int H);
void launch_downsample(hipStream_t st, const float4 *src, int Ws, int Hs,
                       float4 *dst, int Wd, int Hd);
void launch_level_init(hipStream_t st, const LevelArgs &a,
                       const LevelDims *coarse, bool coarsest);
void launch_energy(hipStream_t st, const LevelArgs &a, int mode, int trial,
                   float tau, int n_trials_before);
void launch_node_rhs(hipStream_t st, const LevelArgs &a, const TileCfg &t);
void launch_apply(hipStream_t st, const LevelArgs &a, const TileCfg &t,
                  int iter, int log_index);
void launch_update(hipStream_t st, const LevelArgs &a, int iter,
                   int log_index);
void launch_accept(hipStream_t st, const LevelArgs &a, int n_trials,
                   int log_index, int gn_iter, int pcg_iters);
void launch_finish_level(hipStream_t st, const LevelArgs &a);
void launch_output(hipStream_t st, const LevelArgs &a, float *depth,
                   float *flow3d, float *flows);
void launch_set_apply_state(hipStream_t st, DevScalars *sc);
void launch_set_pcg_state(hipStream_t st, DevScalars *sc);
size_t node_tile_lds_bytes(const TileCfg &t, int s, int K);
int energy_blocks(const LevelDims &d);
int node_tile_blocks(const LevelDims &d, const TileCfg &t);
