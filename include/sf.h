/*
 * sf.h - C ABI of the halfway-domain scene-flow solver for MI355X (gfx950).
 *
 * The library computes dense geometry and 3D motion from two synchronized,
 * pre-calibrated monochrome stereo pairs (left/right camera at time t and
 * t+1; paper Sec. 3), by minimising the halfway-domain energy of Sec. 4
 * (Eqs. (8)-(18)) over a coarse warp grid (Sec. 3.3, Eq. (7)) with
 * data-parallel Gauss-Newton and preconditioned conjugate gradients
 * (Sec. 5.1, Eqs. (19)-(24)) inside the delta hierarchy of Sec. 5.3.
 *
 * Conventions shared by every entry point:
 *  - Images are float32, row-major, H x W, nominally in [0, 1]; pixel (x, y)
 *    has integer coordinates at its centre.
 *  - "device" pointers are HIP device memory owned by the caller (for
 *    example torch tensors); they must stay valid until the work enqueued on
 *    the context's stream has completed.  All compute runs on the GPU.
 *  - Every function returns sf_status; arguments are validated on the host
 *    before anything is enqueued, so a failed call enqueues nothing.
 *  - A context is bound to one HIP stream and one device; it is not
 *    thread-safe (use one context per host thread / stream).
 *  - No C++ types or exceptions cross this boundary.
 */
#ifndef SF_H
#define SF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SF_OK = 0,
    SF_ERR_INVALID_ARG = -1, /* null pointer, bad enum, weight < 0, ...     */
    SF_ERR_SIZE = -2,        /* image too small for the requested levels    */
    SF_ERR_HIP = -3,         /* a HIP runtime call failed                   */
    SF_ERR_OOM = -4,         /* device allocation failed                    */
    SF_ERR_NUMERIC = -5,     /* NaN/Inf energy (reported through the log)   */
    SF_ERR_STATE = -6        /* call not valid in the context's state       */
} sf_status;

/* Opaque solver context: owns all device workspace (pyramid, node vectors,
 * per-pixel linearisation records, reduction scratch, log, HIP graph). */
typedef struct sf_ctx sf_ctx;

/* Rectified pinhole stereo pair (Sec. 3): focal lengths and principal point
 * in level-0 pixels, baseline in metres, and the fundamental matrix F
 * (row-major) with x_L^T F x_R = 0 for corresponding homogeneous pixels,
 * used by the epipolar term, Eqs. (15)-(17).  For a rectified rig normalise
 * F = [[0,0,0],[0,0,-1],[0,1,0]], so the residual is r_y - l_y in pixels. */
typedef struct {
    float fx, fy, cx, cy, baseline;
    float F[9];
} sf_calib;

/* Energy weights (Eqs. (8)-(10), (14), (18); Appendix A) and schedule.
 *  levels          pyramid levels (coarse-to-fine hierarchy, Sec. 5.3)
 *  grid_stride     warp-grid step in pixels at every level (Sec. 3.3), 1..8
 *  gn_iters        Gauss-Newton steps per level
 *  gn_fine         if > 0, Gauss-Newton steps on the two finest levels
 *                  instead (the paper's real-time schedule, Sec. 6.2: 2 on
 *                  the two finest levels, 5 on the others); 0 = gn_iters
 *  pcg_iters       PCG iterations per Gauss-Newton step (1..64)
 *  max_backtracks  step-length halvings after tau = 1 (0..7)
 *  init_mode       0 = zero initialisation of the coarsest level; 1 = the
 *                  learned initialiser (needs weights from
 *                  sf_set_initializer and, in single-frame contexts,
 *                  levels >= 5; batch frames with fewer levels start from
 *                  zero; see below)
 *  exec_mode       0 = replay a captured HIP graph, 1 = enqueue kernels
 *  tile_mode       node-tile shape of the PCG kernels: 0 = default per
 *                  stride; 1 = autotuned (each candidate shape is timed on
 *                  the first solve of a frame size or batch shape and the
 *                  fastest is cached per device, stride and level sizes, in
 *                  the process and, if the environment variable
 *                  SF_TUNE_CACHE names a file, in that file); 2, 3 = the
 *                  alternative shapes (strides 2, 4, 8; others use the
 *                  default); with apply_mode 1, 2 the same choice among
 *                  the node-block tiles (8 x 8 nodes; 16 x 8; 8 x 4;
 *                  4 = 4 x 4, which the matrix-free mode treats as 0)
 *  apply_mode      how the PCG kernels form H u (Sec. 5.2): 0 = matrix-free
 *                  from the per-pixel Gauss-Newton records (the transpose
 *                  of the bilinear interpolation, Eq. (7), applied on every
 *                  product); 1 = from per-node 6x6 blocks
 *                  H_nm = sum_x a_n(x) a_m(x) J^T Omega J (x) of each node
 *                  and its eight neighbours, assembled once per
 *                  Gauss-Newton step (the paper's precomputed per-node
 *                  blocks; 120 floats of extra workspace per node); 2 = as
 *                  1, and levels with at most 336 nodes run all PCG
 *                  iterations of a Gauss-Newton step in one workgroup;
 *                  3 = as 2, and in single-frame solves every level with
 *                  more than 336 nodes whose 12 x 7-node tiles (at most
 *                  256) the device holds at once runs all PCG iterations
 *                  of a Gauss-Newton step in one launch, one workgroup
 *                  per tile, its blocks in registers, the tiles
 *                  exchanging tagged partial sums and border records
 *                  (bounded waits: if a wait gives up, sf_get_log reports
 *                  SF_ERR_STATE, the solve is undefined and the context
 *                  falls back to per-iteration kernels); other levels and
 *                  batches run as in mode 2
 *  temporal        1 = video mode (Sec. 5.3): every sf_solve after the first
 *                  starts each level's delta from the previous sf_solve of
 *                  the context, transferred by its motion flow under
 *                  constant velocity (node y takes the previous delta at
 *                  y - 2 m(y), m the motion components of the previous
 *                  level total at y, bilinear on the node grid, clamped;
 *                  masks and weights are then taken at base + delta).  The
 *                  first solve after sf_create or sf_reset_sequence starts
 *                  from zero.  Single-frame solves with init_mode 0 only
 *                  (sf_solve_batch rejects it); 32 floats of state per node
 *                  and level.
 *  illum           1 = illumination correction (Sec. 5.3): after each level
 *                  the stereo residual ((I_R0 - I_L0) + (I_R1 - I_L1)) / 2
 *                  of the raw images at the final flow (0 where a position
 *                  leaves its image) is low-passed (Gaussian, sigma 3.2 px,
 *                  10 taps a side, clamped borders), box-upsampled to the
 *                  next finer level and subtracted there from both
 *                  right-camera samples (masks and energies); the coarsest
 *                  level has none.  3 floats of workspace per pixel.
 *  occlusion       1 = occlusion maps (Sec. 5.3): after each level but the
 *                  finest the mesh that triangulates the halfway pixel grid
 *                  is rendered into the four views with a z-buffer of
 *                  stereo disparity (triangles with an edge longer than
 *                  2 px in a view, a vertex of disparity <= 0 or zero area
 *                  are skipped; pixel centres on or inside a triangle take
 *                  its barycentric disparity; the largest value is kept); a
 *                  halfway pixel is occluded if, in some view, its nearest
 *                  pixel centre is in the image and its own disparity is
 *                  positive and below 0.98 times the z-buffer there.  The
 *                  map is box-upsampled to the next finer level and removes
 *                  occluded pixels from its V(x) (the coarsest level has
 *                  none).  About 17 bytes of workspace per pixel.
 *  w_*, m_*        weights of the energy terms; m_s, m_m, m_d must be > 0
 *  eps             pseudo-Huber parameter of Eq. (12)
 *  eps_p           colour-pruning threshold of Sec. 4.1
 *  st_gamma,st_tau smoothness-weight map w_i = 1 + st_gamma exp(-l / tau_l),
 *                  tau_l = st_tau 4^level, l = smaller eigenvalue of the
 *                  3x3-window structure tensor (Sec. 4.3 names only the
 *                  eigenvalue analysis; this map is the library's reading). */
typedef struct {
    int levels, grid_stride, gn_iters, pcg_iters, max_backtracks, init_mode;
    int exec_mode, tile_mode, apply_mode, temporal, illum, occlusion, gn_fine;
    float w_reg, w_photo, w_grad, w_epi, w_smooth, w_mag;
    float w_s, w_m, w_d, m_s, m_m, m_d;
    float eps, eps_p, st_gamma, st_tau;
} sf_params;

/* Fills *out with the paper's "Figures 5, 6, 8" parameter column
 * (Appendix A), w_smooth = w_mag = 1, eps = 0.001, eps_p = 0.2, the
 * schedule levels 3, stride 8, 5 GN x 10 PCG, 4 backtracks, and the
 * node-block products with one-workgroup PCG at small levels
 * (apply_mode 2). */
sf_status sf_params_default(sf_params *out);

/* Creates a context for width x height frames on the current HIP device,
 * allocating all workspace up front.  hip_stream is a hipStream_t (NULL for
 * the null stream).  Errors: SF_ERR_INVALID_ARG (null out/p, bad params),
 * SF_ERR_SIZE (a level would be smaller than 8 x 8 pixels), SF_ERR_OOM,
 * SF_ERR_HIP.  On error *out is set to NULL. */
sf_status sf_create(sf_ctx **out, int width, int height, const sf_params *p,
                    void *hip_stream);

/* Solves one frame.  Inputs: the four device images of the context's size
 * (left t, right t, left t+1, right t+1; Sec. 3.1), calibration, and
 * optional params (NULL = creation-time params; a non-NULL p may change
 * weights but must keep levels, grid_stride, gn_iters, gn_fine, pcg_iters and
 * max_backtracks, else SF_ERR_STATE).  Outputs (device, caller-owned):
 *  depth   H x W: depth Z_t of each halfway-domain pixel at time t in the
 *          left camera (metres), NaN where the disparity is <= 0;
 *  flow3d  3 x H x W: X_{t+1} - X_t in the left-camera frame (metres);
 *  flows   6 x H x W (may be NULL): per-pixel s_x, s_y, m_x, m_y, d_x, d_y
 *          of the finest level in pixels.
 * Asynchronous on the context's stream; allocates nothing. */
sf_status sf_solve(sf_ctx *ctx, const float *I_left_t, const float *I_right_t,
                   const float *I_left_t1, const float *I_right_t1,
                   const sf_calib *calib, const sf_params *p, float *depth,
                   float *flow3d, float *flows);

/* One record per (level, Gauss-Newton step), coarsest level first. */
typedef struct {
    int level, gn_iter;
    double energy;            /* E of Eq. (8) before the step                */
    double e_photo, e_grad;   /* raw E_photo, E_grad (Eqs. (11), (13))       */
    double e_smooth, e_epi, e_mag; /* raw regularisers (Eqs. (14),(15),(18)) */
    double energy_after;      /* E after the accepted step                   */
    float tau;                /* accepted step length (0 = rejected)         */
    int pcg_iters;
    float pcg_res[64];        /* ||r|| after each PCG iteration              */
    int n_valid;              /* pixels with V(x) W(x) = 1 at this level     */
} sf_iter_log;

/* Copies the log of the last solve into out (at most cap records) and sets
 * *n_written.  Synchronises the context's stream.  Returns SF_ERR_NUMERIC
 * if any logged energy is NaN or Inf (the records are still written). */
sf_status sf_get_log(sf_ctx *ctx, sf_iter_log *out, int cap, int *n_written);

/* ---- batches of frames ------------------------------------------------
 * A batch solves up to 64 independent frames of any sizes together: every
 * kernel of the hierarchy runs once per step for all frames (each workgroup
 * serves one frame; reductions stay per frame), and the whole batch
 * (pyramids, all levels, outputs) replays as one captured HIP graph.  Each
 * frame gets the same result as a single-frame solve with the same
 * parameters and level count. */
typedef struct {
    const float *img[4];  /* device H x W float32: left t, right t, left t+1,
                             right t+1 (Sec. 3.1)                           */
    int width, height;
    sf_calib calib;
    float *depth;         /* device H x W, as in sf_solve                   */
    float *flow3d;        /* device 3 x H x W, as in sf_solve               */
    float *flows;         /* device 6 x H x W or NULL                       */
} sf_frame;

/* Pyramid levels a batch uses for a width x height frame: the largest
 * L <= max_levels with W / 2^(L-1) >= 40 px (at least 1), reduced until the
 * coarsest level is at least 8 x 8. */
int sf_batch_levels(int width, int height, int max_levels);

/* Solves n frames (1..64).  p: as in sf_solve, except that the schedule may
 * differ from the context's (the batch workspace is rebuilt when the
 * schedule or the list of frame sizes changes: the first call for a batch
 * shape allocates, later calls with the same shape allocate nothing).
 * frames[i] needs four images, depth and flow3d, width and height >= 16 and
 * a valid calibration, else SF_ERR_INVALID_ARG / SF_ERR_SIZE before
 * anything is enqueued.  Asynchronous on the context's stream. */
sf_status sf_solve_batch(sf_ctx *ctx, int n, const sf_frame *frames,
                         const sf_params *p);

/* Log of frame `frame` of the last batch solve, as sf_get_log. */
sf_status sf_get_batch_log(sf_ctx *ctx, int frame, sf_iter_log *out, int cap,
                           int *n_written);

/* ---- learned coarse-level initialiser ---------------------------------
 * The paper (Sec. 7) names a smarter initialisation of the coarsest level
 * as future work.  With init_mode = 1 the solver runs a six-layer 3x3
 * convolutional network (4 -> 32 -> 32 -> 32 -> 32 -> 32 -> 6 channels,
 * zero padding, ReLU after the first five; bfloat16 weights and
 * activations, float32 accumulation on the matrix cores) on the four
 * level-4 (1/16-resolution) images minus 0.5.  Its output, per pixel
 * (s_x, s_y, m_x, m_y, d_x, d_y) in level-4 pixels, is sampled bilinearly
 * (clamp-to-edge) at the coarsest level's warp nodes and converted to that
 * level's pixels.  Fallback: E of Eq. (8) at zero deltas is evaluated for
 * the prediction and for the zero initialisation with one common
 * visibility mask (all four positions inside the image under both) and no
 * colour pruning; the prediction is used only if its energy is strictly
 * lower.  Masks and smoothness weights are then taken at the chosen
 * initialisation as usual.
 *
 * Parameter vector (SF_CNN_PARAMS values): per layer the weights in
 * row-major (c_out, c_in, ky, kx) order followed by the c_out biases. */
#define SF_CNN_PARAMS 39910

/* Copies the initialiser's parameters: SF_CNN_PARAMS bfloat16 values
 * (uint16 bit patterns, host memory), bytes = 2 * SF_CNN_PARAMS.  Takes
 * effect for the following solves, also in a captured graph.  A context of
 * either init_mode accepts them (the first call allocates the weight
 * buffers); they serve its single-frame solves and its batches alike.
 * SF_ERR_SIZE for another byte count, SF_ERR_INVALID_ARG for a non-finite
 * value. */
sf_status sf_set_initializer(sf_ctx *ctx, const void *weights, size_t bytes);

/* Outcome of the fallback at the last solve with init_mode = 1: *used = 1
 * if the prediction was kept, and both energies.  Synchronises the stream;
 * SF_ERR_STATE if no such solve ran. */
sf_status sf_get_init_result(sf_ctx *ctx, int *used, double *e_pred, double *e_zero);

/* Batches with init_mode = 1: every frame with at least 5 levels (so that
 * it has a level 4 for the network's input) is initialised as above, with
 * its own fallback decision; frames of one level-4 size share one forward
 * pass.  Frames with fewer levels start from zero.  Each frame gets the
 * result of its single-frame solve with the same parameters and level
 * count.  sf_solve_batch returns SF_ERR_STATE if init_mode = 1 and no
 * weights were set.
 *
 * Outcome of the fallback for frame `frame` of the last batch: as
 * sf_get_init_result; *used = -1 (energies NaN) for a frame with fewer than
 * 5 levels.  Synchronises the stream; SF_ERR_STATE if the last batch did
 * not run with init_mode = 1, SF_ERR_INVALID_ARG for a frame index outside
 * it. */
sf_status sf_get_batch_init_result(sf_ctx *ctx, int frame, int *used, double *e_pred,
                                   double *e_zero);

/* Trainer of the initialiser: batches of B level-4 image quadruples
 * (device float32 [B][4][H][W], left t, right t, left t+1, right t+1) with
 * targets (device float32 [B][6][H][W], flows in level-4 pixels).  One
 * step = forward, L1 loss (mean absolute error over all B 6 H W values),
 * backpropagation and one Adam update (beta1 0.9, beta2 0.999, eps 1e-8)
 * of the float32 master parameters; the network itself runs on bfloat16
 * copies.  Deterministic: fixed-order reductions only. */
typedef struct sf_trainer sf_trainer;
sf_status sf_trainer_create(sf_trainer **out, int max_batch, int height, int width,
                            void *hip_stream);
/* Sets the float32 master parameters (host, n = SF_CNN_PARAMS) and resets
 * the Adam state; synchronises. */
sf_status sf_trainer_set_params(sf_trainer *t, const float *host, size_t n);
sf_status sf_trainer_get_params(sf_trainer *t, float *host, size_t n);
/* Network output for `batch` samples into out (device [batch][6][H][W]). */
sf_status sf_trainer_forward(sf_trainer *t, const float *x, int batch, float *out);
/* One training step with learning rate lr (lr = 0 computes the gradient
 * and leaves the parameters unchanged).  loss (host, may be NULL): the
 * mean absolute error before the update; non-NULL synchronises. */
sf_status sf_trainer_step(sf_trainer *t, const float *x, const float *target, int batch,
                          float lr, float *loss);
/* Test access to the last batch: network input (bf16 NHWC, 16 channels),
 * post-ReLU activations of layers 0..4 (bf16 NHWC, 32 channels), output
 * (float [B][6][H][W]), loss gradient (bf16 NHWC, 16 channels), the
 * gradients w.r.t. the pre-activations of layers 0..4 (bf16 NHWC, 32) and
 * the parameter gradient (float, SF_CNN_PARAMS). */
enum {
    SF_TR_INPUT = 0,
    SF_TR_ACT = 1,
    SF_TR_OUT = 2,
    SF_TR_DOUT = 3,
    SF_TR_DPRE = 4,
    SF_TR_GRAD = 5
};
size_t sf_trainer_size(sf_trainer *t, int what, int layer);
sf_status sf_trainer_read(sf_trainer *t, int what, int layer, void *host, size_t bytes);
void sf_trainer_destroy(sf_trainer *t);

/* Human-readable name of a status code (static string). */
const char *sf_status_string(sf_status s);

/* The HIP call behind the calling thread's last SF_ERR_HIP / SF_ERR_OOM,
 * with HIP's error string ("" if none); valid until the thread's next
 * failing call. */
const char *sf_last_error(void);

/* Frees the context and all its device memory; NULL-safe.  Synchronises the
 * context's stream first. */
void sf_destroy(sf_ctx *ctx);

/* Video mode (sf_params.temporal = 1): forgets the previous solve, so the
 * next sf_solve starts from zero (a new sequence).  Synchronises the
 * context's stream.  Errors: SF_ERR_INVALID_ARG, SF_ERR_HIP. */
sf_status sf_reset_sequence(sf_ctx *ctx);

/* ---- solving without allocation ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * sf_solve_noalloc is sf_create + sf_solve in one call without a context:
 * the same inputs, parameters and outputs as sf_solve (p is required), run
 * with direct launches (exec_mode is ignored) and the default tile shapes
 * (tile_mode 1, autotuning, is treated as 0), giving bitwise the outputs of
 * a context created with those parameters.  It allocates nothing: the
 * whole workspace lives in the library's static device array of
 * SF_NOALLOC_SCRATCH_BYTES, which every GPU the library runs on holds until
 * the process ends; per-call constants travel as kernel arguments and the
 * array is cleared by a kernel, so every step is a kernel launch on
 * hip_stream (a hipStream_t, NULL for the null stream).  The first call on
 * a device looks up the array's address there.
 *
 * Limits: the frame's workspace must fit the array (at stride 4 with 4
 * levels, frames up to 320 x 240 pixels), else SF_ERR_SIZE with the needed
 * size in sf_last_error; init_mode and temporal must be 0, else
 * SF_ERR_INVALID_ARG.  Every call on a device uses that device's one
 * array, and each call starts by clearing it: calls whose GPU work overlaps
 * on one device (different streams, or host threads enqueueing at once)
 * race on it and give undefined results.  Other errors as sf_create and
 * sf_solve.  There is no log (sf_get_log needs a context). */
#define SF_NOALLOC_SCRATCH_BYTES (32u << 20)
sf_status sf_solve_noalloc(int width, int height, const float *I_left_t,
                           const float *I_right_t, const float *I_left_t1,
                           const float *I_right_t1, const sf_calib *calib,
                           const sf_params *p, float *depth, float *flow3d,
                           float *flows, void *hip_stream);

/* ---- test support: per-stage access to intermediates --------------------
 * These entry points exist so that tests can compare each stage with an
 * independent implementation.  They synchronise the stream.  host_dst /
 * host_src are host pointers of exactly `bytes` bytes; the expected size
 * for (what, level) is returned by sf_debug_size. */
enum {
    SF_DBG_TEX = 0,     /* 4 x N_l float4: (I, G_x, G_y, 0) per image, with
                           G the central-difference gradient images       */
    SF_DBG_CMASK = 1,   /* N_l uint8: V(x) W(x)                              */
    SF_DBG_WNODE = 2,   /* G_l float: smoothness weights w_i                 */
    SF_DBG_BASE = 3,    /* 6 x G_l float: prolongated total of the level     */
    SF_DBG_DELTA = 4,   /* 6 x G_l float: delta unknowns                     */
    SF_DBG_DX = 5,      /* 6 x G_l float: PCG solution (GN step)             */
    SF_DBG_R = 6,       /* 6 x G_l float: PCG residual (initially -grad E)   */
    SF_DBG_Z = 7,       /* 6 x G_l float: preconditioned residual u =
                           diag(H)^-1 r at the PCG's start (the vector
                           SF_STAGE_APPLY multiplies)                       */
    SF_DBG_Q = 8,       /* 6 x G_l float: H u of the first PCG product        */
    SF_DBG_DIAG = 9,    /* 6 x G_l float: diag(H)                            */
    SF_DBG_REC = 10,    /* 27 x N_l float: per-pixel gradient (6) and
                           upper-triangular Gauss-Newton block (21)          */
    SF_DBG_P = 11,      /* 6 x G_l float: the vector the first product used  */
    SF_DBG_ENERGY = 12, /* 6 double: photo, grad, smooth, epi, mag, total
                           at the last linearisation                         */
    SF_DBG_OCC = 13     /* N_l uint8: the occlusion map level l reads, 1 =
                           visible (written by SF_STAGE_OCC at level l + 1;
                           occlusion = 1 only)                               */
};
size_t sf_debug_size(sf_ctx *ctx, int what, int level);
sf_status sf_debug_read(sf_ctx *ctx, int what, int level, void *host_dst,
                        size_t bytes);
sf_status sf_debug_write(sf_ctx *ctx, int what, int level,
                         const void *host_src, size_t bytes);

/* Builds the image pyramid from four device images and stores the
 * calibration, without solving. */
sf_status sf_debug_set_images(sf_ctx *ctx, const float *I_left_t,
                              const float *I_right_t, const float *I_left_t1,
                              const float *I_right_t1, const sf_calib *calib);

/* Runs one stage at `level` on the current state:
 *  SF_STAGE_LEVEL_INIT   prolongate (zero at the coarsest level), zero the
 *                        delta, compute masks and smoothness weights
 *  SF_STAGE_LINEARIZE    per-pixel records, energy, gradient and diag(H)
 *  SF_STAGE_APPLY        q = H p with p = the current SF_DBG_Z vector
 *  SF_STAGE_PCG          pcg_iters PCG iterations from x = 0
 *  SF_STAGE_GN           one full Gauss-Newton step with step control
 *  SF_STAGE_FINISH       store base + delta as the level's total
 *  SF_STAGE_MASKS        masks and smoothness weights at the current base
 *                        (the level set-up without the prolongation)
 *  SF_STAGE_STEP         the step control alone (the library's reading;
 *                        the paper states none): delta +=
 *                        tau dx with dx = the current SF_DBG_DX and tau the
 *                        first of 1, 1/2, ..., 2^-max_backtracks whose
 *                        energy does not exceed E at the last
 *                        SF_STAGE_LINEARIZE (delta unchanged if none)
 *  SF_STAGE_OCC          the occlusion map of level - 1 from this level's
 *                        base + delta (level >= 1, occlusion = 1)
 *  SF_STAGE_SPEC_STEP    the same step control in the solve's speculative
 *                        form (apply_mode >= 1; every Gauss-Newton step of
 *                        a level but its last): the linearisation at
 *                        delta + dx, the shorter trials, then the next
 *                        step's right-hand side and PCG.  Afterwards delta
 *                        is moved as by SF_STAGE_STEP, the energy
 *                        (SF_DBG_ENERGY) and diag(H) are those at the new
 *                        delta, and dx is the new PCG solution         */
enum {
    SF_STAGE_LEVEL_INIT = 0,
    SF_STAGE_LINEARIZE = 1,
    SF_STAGE_APPLY = 2,
    SF_STAGE_PCG = 3,
    SF_STAGE_GN = 4,
    SF_STAGE_FINISH = 5,
    SF_STAGE_MASKS = 6,
    SF_STAGE_STEP = 7,
    SF_STAGE_OCC = 8,
    SF_STAGE_SPEC_STEP = 9
};
sf_status sf_debug_run(sf_ctx *ctx, int stage, int level);

/* ---- measurement support ---------------------------------------------------
 * Launches one solver kernel `reps` times back to back on the context's
 * stream at `level`, on the state left by the last solve (its last
 * linearisation), between two HIP events recorded on that same stream, and
 * writes the average duration per launch in milliseconds to *avg_ms.
 * Synchronises the stream.  The kernel's outputs are scratch afterwards.
 *  SF_KERNEL_APPLY      one PCG iteration: vector updates + w = H u
 *                       (matrix-free, node tiles)
 *  SF_KERNEL_LINEARIZE  per-pixel records and energy
 *  SF_KERNEL_UPDATE     the last PCG iteration's vector update
 *  SF_KERNEL_RHS        right-hand side and diag(H) (node tiles; with
 *                       apply_mode >= 1 together with the per-node blocks)
 *  SF_KERNEL_BLOCKS     right-hand side and per-node blocks (apply_mode >= 1
 *                       only; the same kernel as SF_KERNEL_RHS there)
 *  SF_KERNEL_PCG_TILE   all pcg_iters iterations of the level in the
 *                       co-resident tiled PCG (apply_mode 3, levels it
 *                       takes; as in the solve, not forced active)
 * The per-iteration PCG kernels run forced active with fixed step
 * lengths. 
 * Errors: SF_ERR_STATE before the first solve, SF_ERR_INVALID_ARG. */
enum {
    SF_KERNEL_APPLY = 0,
    SF_KERNEL_LINEARIZE = 1,
    SF_KERNEL_UPDATE = 2,
    SF_KERNEL_RHS = 3,
    SF_KERNEL_BLOCKS = 4,
    SF_KERNEL_PCG_TILE = 5
};
sf_status sf_time_kernel(sf_ctx *ctx, int kernel, int level, int reps,
                         float *avg_ms);

/* The same for the batch workspace: one launch covers every frame of the
 * last batch that has a level `level`. */
sf_status sf_time_batch_kernel(sf_ctx *ctx, int kernel, int level, int reps,
                               float *avg_ms);

/* The tile shape of the PCG iteration kernel at `level` that the last solve
 * (batched = 0) or batch (batched = 1) used, as chosen by tile_mode and the
 * autotuner: *variant = V of k_pcg<B, FIRST, S, V> (node-block modes: 8 x 8,
 * 16 x 8, 8 x 4, 4 x 4 nodes for 0..3).  Lets measurements name the kernel
 * they report.  Errors: SF_ERR_STATE before the first solve / batch,
 * SF_ERR_INVALID_ARG. */
sf_status sf_tile_variant(sf_ctx *ctx, int batched, int level, int *variant);

#ifdef __cplusplus
}
#endif

#endif /* SF_H */
