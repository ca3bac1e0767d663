// Internal types shared by the host orchestration and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sf.h"

#define SF_MAX_LEVELS 12
#define SF_MAX_TRIALS 8
#define SF_MAX_PCG 64
#define SF_BLOCK 256
#define SF_MAX_BATCH 64

// Per-pixel linearisation records, one aligned record per pixel so that a
// pixel is read with whole 16-byte loads:
//  gram: 24 floats, the reweighted Gauss-Newton block J^T Omega J of the
//        pixel's six flow components: its diagonal (6), the upper
//        off-diagonal entries row by row (15), padding (3);
//  grad: 8 floats, the gradient of the pixel's energy w.r.t. its flows (6);
//        slot 6 holds the mean warped image from level start until the
//        first linearisation; slot 7 is padding.
#define SF_GRAM_STRIDE 24
#define SF_GRAD_STRIDE 8
#define SF_GRAD_IBAR 6
// Per-node system-matrix blocks (the node-block apply mode): for each node
// n = (i, j) the symmetric 6x6 blocks H_nm = sum_x a_n(x) a_m(x) G(x) of its
// pairs with m = n, (i+1, j), (i, j+1), (i+1, j+1), (i-1, j+1), in that
// order, each as the 21 entries of a gram record: the first 20 of block k
// at floats 20 k .. 20 k + 19 of the node's record (five aligned float4),
// its last at float 100 + k, then 3 floats of padding (432 bytes a node).
#define SF_BLK_TYPES 5
#define SF_BLK_STRIDE (SF_BLK_TYPES * 20 + 8)
// the test interface's plane layout: 6 gradient planes, then the 21
// upper-triangular entries of the block row by row
#define SF_REC_PLANES 27

// Slot of entry (i, j) of a pixel's symmetric block in its gram record.
__host__ __device__ inline int gram_index(int i, int j) {
    if (i > j) {
        const int t = i;
        i = j;
        j = t;
    }
    return i == j ? i : 6 + i * 5 - (i * (i - 1)) / 2 + (j - i - 1);
}

// Node vectors (each G_0 records of SF_NREC = 6 floats: s_x, s_y, m_x, m_y,
// d_x, d_y, packed, so that a run of nodes moves no padding).  The PCG runs
// in the
// single-reduction form: r, w = H u and s = H p alternate between two
// buffers by iteration parity because neighbouring tiles read them.
#define SF_NREC 6
enum {
    NV_BASE = 0,
    NV_DELTA,
    NV_X,      // PCG solution (the Gauss-Newton step)
    NV_R0,
    NV_R1,
    NV_U,      // preconditioned residual
    NV_W0,
    NV_W1,
    NV_S0,
    NV_S1,
    NV_P,
    NV_DIAG,
    NV_TPREV,  // total of the level just solved (for prolongation)
    NV_COUNT
};

// Partial-sum planes (each max_blocks floats).
enum {
    PS_E = 0,        // 5 planes: energy terms per workgroup
    PS_PCG0 = 5,     // 3 planes: r.u, w.u, r.r (even iterations)
    PS_PCG1 = 8,     // 3 planes: odd iterations
    PS_MASK = 11,    // 1 plane: valid-pixel counts
    PS_TRIAL = 12,   // 5 planes per further trial of a multi-trial launch
    PS_COUNT = PS_TRIAL + 5 * (SF_MAX_TRIALS - 1)
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

// Scalars of one PCG iteration k, stored in slot k + 1 (slot 0 is the
// state before the first iteration).
struct PcgHist {
    double gamma;   // r_k . u_k
    float alpha, beta;
    int active;     // iteration k was applied
    int pad;
};

// Device-resident scalars of the solve.  Every slot is written by exactly
// one workgroup and read only by later kernels.
struct DevScalars {
    double e_lin[6];                  // photo, grad, smooth, epi, mag, total
    double e_trial[SF_MAX_TRIALS][6]; // the accepted trial's terms
    PcgHist hist[SF_MAX_PCG + 2];
    double e_init[2];  // fallback energies: learned, zero initialisation
    int init_used;     // the learned initialisation was kept
    int n_valid;
    int have_prev;     // the temporal state holds a finished solve
    unsigned pt_epoch;   // launches of the co-resident tiled PCG (its tags)
    int mid_fail;        // a co-resident PCG gave up waiting (sticky)
    // speculative steps: tau = 1 was accepted (the shorter-trial kernel's
    // verdict); otherwise the step length the right-hand-side kernel chose
    // and the number of energy partials it left
    int spec_acc;
    float spec_tau;
    int lin_n;
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

// Launch geometry of the node-tile kernels: tx x ty nodes per workgroup,
// tpn threads per node (the workgroup has tx * ty * tpn threads).
struct TileCfg {
    int tx, ty, tpn;
    int v;  // shape variant (PCG kernels)
};

// Caller buffers of one frame of a batch (device pointers, rewritten on
// every batch call).
struct FrameIO {
    const float *img[4];
    float *depth, *flow3d, *flows;
};

// Everything a kernel needs about one frame at the current level.  Passed
// by value for single-frame launches; batched launches read it from a
// device table (see FrameMap).
struct LevelArgs {
    LevelDims d;
    int level;
    int s;                 // grid stride
    int N0, G0;            // plane strides of records / node vectors
    int coarsest;          // this is the frame's coarsest level
    int Gxc, Gyc;          // node grid of the next coarser level
    int log_base;          // log slot of this level's first Gauss-Newton step
    int Wf, Hf;            // size of the next finer level (pyramid)
    int learned;           // coarsest level initialised by the network
    int temporal;          // initialise the deltas from the previous solve
    float *illum;          // illumination correction of this level's pixels
                           // (nullptr: none); the next finer level's is
                           // written into the same buffer after this level
    float *ill_e, *ill_t;  // its scratch: residual and horizontal blur
    const unsigned char *occ;  // occlusion map of this level's pixels, 1 =
                               // visible (nullptr: none)
    unsigned char *occ_next;   // the next finer level's map, written after
                               // this level (nullptr: none)
    float *occ_pos;            // scratch: 10 planes of N (positions, disparities)
    unsigned *occ_zb;          // scratch: 4 z-buffers of N (float bits)
    float *prev;           // temporal state of this level: G records of the
                           // previous solve's delta, then G of its total
    int W4, H4;            // size of the network's output (level 4)
    const float *cnn_out;  // network output, 6 planes of W4 x H4
    const float4 *tex;     // this level's 4 images (image-major)
    const float4 *tex_fine;  // the next finer level's images
    const FrameIO *io;     // caller buffers (batched launches)
    float *nodes;          // base of all node vectors
    float *gram;           // per-pixel Gauss-Newton blocks (SF_GRAM_STRIDE)
    float *grad;           // per-pixel gradients (SF_GRAD_STRIDE)
    unsigned char *cmask;  // V(x) W(x)
    float *wnode;          // smoothness weights
    float *reg;            // per-node regulariser record, 16 floats per node
    float *blk;            // per-node blocks (SF_BLK_STRIDE), node-block mode
    float *partials;       // per-workgroup partial sums
    int max_blocks;        // stride of the partial-sum planes
    unsigned long long *xtag;  // tagged exchange of the co-resident tiled PCG
                               // (nullptr: not used)
    const DevConst *cst;
    DevScalars *sc;
    DevLog *log;
};

// Kernel argument of a launch over several frames: the workgroups of frame
// f are [first[f], first[f + 1]) and its arguments are tab[f].
struct FrameMap {
    const LevelArgs *tab;
    int nf;
    int first[SF_MAX_BATCH + 1];
};

// One launch target: a single frame (arguments by value) or nf frames
// (host copies for launch geometry, device table for the kernels).
struct Launch {
    int nf;
    const LevelArgs *host;  // nf entries
    const LevelArgs *dev;   // device table, used when batched
    bool batched;
};

// Kernel launchers (sf_kernels.hip).  `gn` is the Gauss-Newton step within
// the level (log slot log_base + gn), or -1 for no logging.
void launch_tex_level0(hipStream_t st, const Launch &L, const float *const img[4]);
void launch_downsample(hipStream_t st, const Launch &L);
void launch_level_init(hipStream_t st, const Launch &L);
// masks and smoothness weights at the current base (part of level init)
void launch_level_masks(hipStream_t st, const Launch &L);
// network candidate for the coarsest level and the fallback energies
// (before launch_level_init)
void launch_cnn_candidate(hipStream_t st, const Launch &L);
void launch_linearize(hipStream_t st, const Launch &L);
// speculative step (node-block modes, every Gauss-Newton step of a level
// but its last): the linearisation at delta + dx, whose energy is also the
// step control's tau = 1 trial
void launch_spec_linearize(hipStream_t st, const Launch &L);
// step control: the energy at tau = 1, then (each workgroup returning at
// once if tau = 1 was accepted) the n_rest shorter steps 2^-1 .. 2^-n_rest.
// spec: the tau = 1 energy came from launch_spec_linearize; the kernel then
// records its verdict, and on acceptance applies delta += dx and writes the
// step's log (gn, pcg_iters as for launch_accept)
void launch_trial0(hipStream_t st, const Launch &L);
void launch_trials_rest(hipStream_t st, const Launch &L, int n_rest, bool spec = false,
                        int gn = -1, int pcg_iters = 0);
void launch_rhs(hipStream_t st, const Launch &L, const TileCfg &t);
// right-hand side, diag(H) and the per-node blocks from the pixel records
// (node-block apply mode; replaces launch_rhs after launch_linearize).
// n_pend > 0 (= the step control's trial count): a speculative step
// precedes; where tau = 1 was rejected the kernel chooses the step length,
// forms the pixel records at delta + tau dx itself and writes the previous
// step's log (gn_prev, pcg_iters); delta itself moves in the PCG's first
// kernel
void launch_rhs_blocks(hipStream_t st, const Launch &L, int n_pend = 0, int gn_prev = -1,
                       int pcg_iters = 0);
// skip_small: frames with at most SF_SMALL_G nodes are left out (their PCG
// runs in launch_pcg_small); pend: a speculative step precedes (the
// deferred delta update of a rejected tau = 1 happens here)
void launch_pcg_first(hipStream_t st, const Launch &L, const TileCfg &t,
                      bool skip_small = false, bool pend = false);
void launch_pcg_iter(hipStream_t st, const Launch &L, const TileCfg &t,
                     int iter, int gn, int force, bool skip_small = false);
void launch_pcg_last(hipStream_t st, const Launch &L, const TileCfg &t,
                     int iter, int gn, int force, bool skip_small = false);
// all pcg_iters iterations of a level in one workgroup per frame, for the
// frames with at most SF_SMALL_G nodes (node-block mode; replaces first /
// iter / last for them)
#define SF_SMALL_G 336
void launch_pcg_small(hipStream_t st, const Launch &L, int n_it, int gn, bool pend = false);
// all pcg_iters iterations of a single frame's level in one launch of
// co-resident tiles of SF_PT_TW x SF_PT_TH nodes that exchange tagged
// partial sums and border records (apply_mode 3; levels with more than
// SF_SMALL_G nodes and at most min(SF_PT_MAXWG, the device's co-resident
// capacity) tiles)
#define SF_PT_TW 12
#define SF_PT_TH 7
#define SF_PT_MAXWG 256
int pt_tiles(const LevelDims &d);
// tiles of k_pcg_tile the current device holds at once
int pt_capacity();
// 64-bit words of a frame's exchange buffer (G0 nodes at level 0)
size_t pt_xtag_words(long G0);
void launch_pcg_tile(hipStream_t st, const Launch &L, int n_it, int gn, bool pend = false);
void launch_accept(hipStream_t st, const Launch &L, int n_trials, int gn,
                   int pcg_iters);
void launch_finish_level(hipStream_t st, const Launch &L);
// illumination correction: zero map at each frame's coarsest level start;
// after a level (not the finest) the next finer level's map
void launch_illum_zero(hipStream_t st, const Launch &L);
void launch_illum_next(hipStream_t st, const Launch &L);
// occlusion map of the next finer level from this level's final flow
void launch_occ_next(hipStream_t st, const Launch &L);
// Clears bytes (a multiple of 16, 16-byte aligned) at p; stores the
// per-call constants through a kernel argument.
void launch_fill_zero(hipStream_t st, void *p, size_t bytes);
void launch_store_const(hipStream_t st, const DevConst &k, DevConst *dst);
void launch_output(hipStream_t st, const Launch &L, float *depth,
                   float *flow3d, float *flows);
TileCfg pick_tile(int s);
// PCG tile shapes: tile_variants(s) shapes per stride, variant 0 = pick_tile
int tile_variants(int s);
TileCfg pick_pcg_tile(int s, int v);
// PCG tiles of the node-block apply modes (any stride): SF_NB_VARIANTS
// shapes, 8 x 8 (default), 16 x 8, 8 x 4 and 4 x 4 nodes, 4 threads per
// node; TileCfg.v = SF_TILE_NB + variant
#define SF_TILE_NB 3
#define SF_NB_VARIANTS 4
TileCfg pick_nb_tile(int v = 0);
// block-assembly tile per stride and its LDS bytes
TileCfg pick_blk_tile(int s);
size_t blk_tile_lds_bytes(int s);
int tile_threads(int s);
int tile_threads(const TileCfg &t);
int tile_max_pixels(const TileCfg &t, int s);
int tile_ppt(int s);
int tile_ppt(int s, int v);
size_t node_tile_lds_bytes(const TileCfg &t, int s, int K);
int energy_blocks(const LevelDims &d);
int node_tile_blocks(const LevelDims &d, const TileCfg &t);
