// Host side of the C ABI declared in include/sf.h: argument validation,
// workspace allocation, the coarse-to-fine level loop (Algorithm 1 without
// the occlusion and illumination map updates; Sec. 5.3), HIP graph capture
// and replay, batches of frames, logging and test access to intermediates.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sf_cnn.h"
#include "sf_internal.h"

namespace {

// Device buffers of one frame (SF_FRAME_BUFS sub-allocations of the pool).
#define SF_FRAME_BUFS 17
struct FrameBuf {
    int W = 0, H = 0, L = 0;
    LevelDims lv[SF_MAX_LEVELS]{};
    long N0 = 0, G0 = 0, tex_len = 0;
    int max_blocks = 0;
    int nlog = 0;
    float4 *tex = nullptr;
    unsigned char *cmask = nullptr;
    float *wnode = nullptr, *reg = nullptr, *nodes = nullptr;
    float *gram = nullptr, *grad = nullptr;
    float *blk = nullptr;   // node-block apply mode only
    float *prev = nullptr;  // temporal state (16 floats per node of every level)
    float *illum = nullptr; // illumination map and its two scratch planes (3 x N0)
    unsigned char *occ = nullptr;  // occlusion map of the level being solved (N0)
    float *occ_pos = nullptr;      // its scratch: 10 planes of N_1 ...
    unsigned *occ_zb = nullptr;    // ... and 4 z-buffers of N_1
    unsigned long long *xtag = nullptr;  // co-resident tiled PCG exchange
    float *partials = nullptr;
    DevConst *cst = nullptr;
    DevScalars *sc = nullptr;
    DevLog *log = nullptr;
    FrameIO *io = nullptr;
};

// Network weights of a context (sf_set_initializer): the float32
// parameters and the bf16 device copies the kernels read.
struct CnnNet {
    bool have_weights = false;
    CnnLayout L{};
    float *flat = nullptr;
    CnnWeights w{};
    char *pool = nullptr;
};

// Learned-initialiser workspace of a plan (init_mode = 1).  Frames with a
// level 4 are grouped by its size, and one forward pass per group serves
// all of its frames: per group their bf16 input quadruples, hidden
// activations and float outputs, frame by frame.  Frames with fewer levels
// start from zero.
struct CnnGroup {
    int W4 = 0, H4 = 0;
    std::vector<int> frames;
    unsigned short *x = nullptr;
    unsigned short *acts[SF_CNN_LAYERS - 1]{};
    float *out = nullptr;
};
struct CnnRun {
    bool on = false;
    std::vector<CnnGroup> groups;
    std::vector<bool> slot_has;   // level slot holds a network-initialised coarsest level
    char *pool = nullptr;
};

// A set of frames solved together: their buffers (one device allocation),
// per-level kernel arguments, staging of per-call constants and the
// captured graph.  Level slot l holds the frames that have a level l.
struct Plan {
    int nf = 0;
    bool batched = false;
    int Lmax = 0;
    sf_params prm{};
    TileCfg tile{};                    // right-hand-side kernel
    TileCfg ptile[SF_MAX_LEVELS]{};    // PCG kernels, per level slot
    bool tuned = false;
    std::vector<FrameBuf> fr;
    std::vector<std::vector<LevelArgs>> host;  // [slot] -> args of its frames
    std::vector<long> slot_off;                // offset of each slot in dtab
    LevelArgs *dtab = nullptr;
    char *pool = nullptr;
    DevConst *dcst = nullptr;  // nf DevConst, then nf FrameIO (one upload)
    FrameIO *dio = nullptr;
    char *stage = nullptr;     // pinned copy of the same
    size_t stage_bytes = 0;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    bool have_inputs = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> shape;  // W, H per frame (batch cache key)
    CnnRun cnn;              // learned initialiser
    const CnnNet *net = nullptr;
    bool no_mid = false;     // co-resident PCG switched off after a failed wait
    int pt_cap = 0;          // co-resident tiles the device holds (0: not used)
    bool external = false;   // pool is caller-provided workspace (not freed)
    size_t pool_bytes = 0;
};

// Caller-provided device workspace for a plan: the plan is carved from it
// instead of an allocation, with no staging buffer and no host copies.
struct ExtPool {
    char *base = nullptr;
    size_t cap = 0;
};

}  // namespace

struct sf_ctx {
    int W = 0, H = 0, device = 0;
    sf_params prm{};
    hipStream_t stream = nullptr;      // caller's stream
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    Plan single;
    Plan *batch = nullptr;
    CnnNet net;
};

namespace {

// Description of the last failed HIP call of this thread (sf_last_error).
thread_local char g_err[256] = "";

void note_hip_error(const char *what, hipError_t e) {
    snprintf(g_err, sizeof(g_err), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(x)                                   \
    do {                                             \
        const hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) {                      \
            note_hip_error(#x, e_);                  \
            return SF_ERR_HIP;                       \
        }                                            \
    } while (0)

sf_status check_params(const sf_params *p) {
    if (!p) return SF_ERR_INVALID_ARG;
    if (p->levels < 1 || p->levels > SF_MAX_LEVELS) return SF_ERR_INVALID_ARG;
    if (p->grid_stride < 1 || p->grid_stride > 8) return SF_ERR_INVALID_ARG;
    if (p->gn_iters < 1 || p->gn_iters > 1000) return SF_ERR_INVALID_ARG;
    if (p->gn_fine < 0 || p->gn_fine > 1000) return SF_ERR_INVALID_ARG;
    if (p->pcg_iters < 1 || p->pcg_iters > SF_MAX_PCG) return SF_ERR_INVALID_ARG;
    if (p->max_backtracks < 0 || p->max_backtracks > SF_MAX_TRIALS - 1) return SF_ERR_INVALID_ARG;
    if (p->init_mode != 0 && p->init_mode != 1) return SF_ERR_INVALID_ARG;
    if (p->init_mode == 1 && p->levels <= SF_CNN_INPUT_LEVEL) return SF_ERR_INVALID_ARG;
    if (p->exec_mode != 0 && p->exec_mode != 1) return SF_ERR_INVALID_ARG;
    if (p->tile_mode < 0 || p->tile_mode > 4) return SF_ERR_INVALID_ARG;
    if (p->apply_mode < 0 || p->apply_mode > 3) return SF_ERR_INVALID_ARG;
    if (p->temporal != 0 && p->temporal != 1) return SF_ERR_INVALID_ARG;
    if (p->temporal == 1 && p->init_mode != 0) return SF_ERR_INVALID_ARG;
    if (p->illum != 0 && p->illum != 1) return SF_ERR_INVALID_ARG;
    if (p->occlusion != 0 && p->occlusion != 1) return SF_ERR_INVALID_ARG;
    const float w[] = {p->w_reg, p->w_photo, p->w_grad, p->w_epi, p->w_smooth,
                       p->w_mag, p->w_s, p->w_m, p->w_d, p->st_gamma};
    for (float v : w)
        if (!(v >= 0.f) || !isfinite(v)) return SF_ERR_INVALID_ARG;
    const float pos[] = {p->m_s, p->m_m, p->m_d, p->eps, p->eps_p, p->st_tau};
    for (float v : pos)
        if (!(v > 0.f) || !isfinite(v)) return SF_ERR_INVALID_ARG;
    if (!(p->w_reg > 0.f && p->w_mag > 0.f)) return SF_ERR_INVALID_ARG;  // keeps H SPD
    return SF_OK;
}

bool same_schedule(const sf_params &a, const sf_params &b) {
    return a.levels == b.levels && a.grid_stride == b.grid_stride &&
           a.gn_iters == b.gn_iters && a.gn_fine == b.gn_fine && a.pcg_iters == b.pcg_iters &&
           a.max_backtracks == b.max_backtracks && a.init_mode == b.init_mode &&
           a.tile_mode == b.tile_mode && a.apply_mode == b.apply_mode &&
           a.temporal == b.temporal && a.illum == b.illum && a.occlusion == b.occlusion;
}

// Gauss-Newton steps at level l: gn_fine on the two finest levels if set.
int gn_at(const sf_params &p, int l) { return (p.gn_fine > 0 && l < 2) ? p.gn_fine : p.gn_iters; }

sf_status check_calib(const sf_calib *cal) {
    if (!cal) return SF_ERR_INVALID_ARG;
    const float v[] = {cal->fx, cal->fy, cal->cx, cal->cy, cal->baseline};
    for (float x : v)
        if (!isfinite(x)) return SF_ERR_INVALID_ARG;
    if (!(cal->fx > 0.f) || !(cal->fy > 0.f) || !(cal->baseline > 0.f)) return SF_ERR_INVALID_ARG;
    for (int i = 0; i < 9; ++i)
        if (!isfinite(cal->F[i])) return SF_ERR_INVALID_ARG;
    return SF_OK;
}

void fill_const(int L, const sf_params &p, const sf_calib &cal, DevConst &k) {
    memset(&k, 0, sizeof(k));
    k.w_reg = p.w_reg; k.w_photo = p.w_photo; k.w_grad = p.w_grad;
    k.w_epi = p.w_epi; k.w_smooth = p.w_smooth; k.w_mag = p.w_mag;
    const float wf[6] = {p.w_s, p.w_s, p.w_m, p.w_m, p.w_d, p.w_d};
    const float mf[6] = {p.m_s, p.m_s, p.m_m, p.m_m, p.m_d, p.m_d};
    for (int q = 0; q < 6; ++q) { k.wf[q] = wf[q]; k.mf[q] = mf[q]; }
    k.eps = p.eps; k.eps_p = p.eps_p; k.st_gamma = p.st_gamma; k.st_tau = p.st_tau;
    k.fx = cal.fx; k.fy = cal.fy; k.cx = cal.cx; k.cy = cal.cy; k.baseline = cal.baseline;
    // level-l pixel p_l maps to level-0 pixel 2^l p_l + (2^l - 1)/2; the
    // level fundamental matrix A^T F A / 2^l keeps residuals in level pixels
    for (int l = 0; l < L; ++l) {
        const double s = ldexp(1.0, l), o = (s - 1.0) / 2.0;
        const double A[9] = {s, 0, o, 0, s, o, 0, 0, 1};
        double T[9], R[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += (double)cal.F[i * 3 + m] * A[m * 3 + j];
                T[i * 3 + j] = acc;  // F A
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += A[m * 3 + i] * T[m * 3 + j];
                R[i * 3 + j] = acc / s;  // A^T F A / 2^l
            }
        for (int q = 0; q < 9; ++q) k.F[l][q] = (float)R[q];
    }
}

// ---- plans -------------------------------------------------------------------

// Level sizes of a W x H frame with L levels; false if a level would be
// smaller than 8 x 8.
bool frame_dims(FrameBuf &f, int W, int H, int L, int st) {
    f.W = W;
    f.H = H;
    f.L = L;
    long tex_off = 0;
    for (int l = 0; l < L; ++l) {
        LevelDims &d = f.lv[l];
        d.W = W >> l;
        d.H = H >> l;
        if (d.W < 8 || d.H < 8) return false;
        d.Gx = (d.W + st - 1) / st;
        d.Gy = (d.H + st - 1) / st;
        d.N = d.W * d.H;
        d.G = d.Gx * d.Gy;
        d.tex_off = tex_off;
        tex_off += 4L * d.N;
    }
    f.tex_len = tex_off;
    f.N0 = f.lv[0].N;
    f.G0 = f.lv[0].G;
    return true;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

void free_plan(Plan &P) {
    // best-effort release: errors here cannot be reported to anyone
    if (P.gexec) (void)hipGraphExecDestroy(P.gexec);
    if (P.graph) (void)hipGraphDestroy(P.graph);
    if (P.pool && !P.external) (void)hipFree(P.pool);
    if (P.cnn.pool) (void)hipFree(P.cnn.pool);
    if (P.stage) (void)hipHostFree(P.stage);
    if (P.stage_ev) (void)hipEventDestroy(P.stage_ev);
    P = Plan();
}

// Allocates and initialises the workspace of frames of the given sizes and
// level counts.
sf_status build_plan(Plan &P, const sf_params &prm, const std::vector<int> &shape,
                     const std::vector<int> &levels, bool batched, const CnnNet *net,
                     const ExtPool *ext = nullptr) {
    P.prm = prm;
    P.net = net;
    P.batched = batched;
    // tiles of the co-resident PCG the device holds at once (apply_mode 3,
    // single frames), checked once per plan
    P.pt_cap = prm.apply_mode == 3 && !batched ? pt_capacity() : 0;
    P.nf = (int)levels.size();
    P.shape = shape;
    const int st = prm.grid_stride;
    P.tile = pick_tile(st);
    if (node_tile_lds_bytes(P.tile, st, 12) > 64 * 1024 ||
        tile_max_pixels(P.tile, st) > tile_ppt(st) * tile_threads(st))
        return SF_ERR_INVALID_ARG;
    for (int v = 0; v < tile_variants(st); ++v) {
        const TileCfg t = pick_pcg_tile(st, v);
        if (node_tile_lds_bytes(t, st, 6) > 64 * 1024 ||
            tile_max_pixels(t, st) > tile_ppt(st, v) * tile_threads(t))
            return SF_ERR_INVALID_ARG;
    }
    const bool nb = prm.apply_mode >= 1;
    if (nb && blk_tile_lds_bytes(st) > 64 * 1024) return SF_ERR_INVALID_ARG;
    const int forced = prm.tile_mode >= 2 ? prm.tile_mode - 1 : 0;
    for (int l = 0; l < SF_MAX_LEVELS; ++l)
        P.ptile[l] = nb ? pick_nb_tile(forced) : pick_pcg_tile(st, forced);
    P.tuned = prm.tile_mode != 1;
    P.fr.resize(P.nf);
    P.Lmax = 0;
    // sizes, then one allocation carved in 256-byte aligned pieces
    size_t off = 0;
    std::vector<size_t> o(P.nf * SF_FRAME_BUFS);
    for (int f = 0; f < P.nf; ++f) {
        FrameBuf &F = P.fr[f];
        if (!frame_dims(F, shape[2 * f], shape[2 * f + 1], levels[f], st)) return SF_ERR_SIZE;
        P.Lmax = P.Lmax > F.L ? P.Lmax : F.L;
        int mb = 1;
        for (int l = 0; l < F.L; ++l) {
            const LevelDims &d = F.lv[l];
            mb = mb > energy_blocks(d) ? mb : energy_blocks(d);
            for (int v = 0; v < tile_variants(st); ++v) {
                const int nt = node_tile_blocks(d, pick_pcg_tile(st, v));
                mb = mb > nt ? mb : nt;
            }
            mb = mb > node_tile_blocks(d, P.tile) ? mb : node_tile_blocks(d, P.tile);
            // the block-assembly tiles (their energy partials, when they
            // re-linearise after a rejected speculative step)
            const int bt = node_tile_blocks(d, pick_blk_tile(st));
            mb = mb > bt ? mb : bt;
            for (int v = 0; v < SF_NB_VARIANTS; ++v) {
                const int nbt = node_tile_blocks(d, pick_nb_tile(v));
                mb = mb > nbt ? mb : nbt;
            }
            const int gb = (d.G + SF_BLOCK - 1) / SF_BLOCK;
            mb = mb > gb ? mb : gb;
        }
        // a multiple of 4: every partial-sum plane starts on 16 bytes
        F.max_blocks = (mb + 3) & ~3;
        F.nlog = 0;
        for (int l = 0; l < F.L; ++l) F.nlog += gn_at(prm, l);
        long g_all = 0;
        for (int l = 0; l < F.L; ++l) g_all += F.lv[l].G;
        const size_t n1 = F.L > 1 ? (size_t)F.lv[1].N : 0;
        const bool occ = prm.occlusion && F.L > 1;
        const size_t sz[SF_FRAME_BUFS] = {sizeof(float4) * (size_t)F.tex_len,
                               (size_t)F.N0,
                               sizeof(float) * (size_t)F.G0,
                               sizeof(float) * 16 * (size_t)F.G0,
                               sizeof(float) * NV_COUNT * SF_NREC * (size_t)F.G0,
                               sizeof(float) * SF_GRAM_STRIDE * (size_t)F.N0,
                               sizeof(float) * PS_COUNT * (size_t)F.max_blocks,
                               sizeof(DevScalars),
                               sizeof(DevLog) * (size_t)F.nlog,
                               sizeof(float) * SF_GRAD_STRIDE * (size_t)F.N0,
                               nb ? sizeof(float) * SF_BLK_STRIDE * (size_t)F.G0 : 0,
                               prm.temporal ? sizeof(float) * 16 * (size_t)g_all : 0,
                               prm.illum ? sizeof(float) * 3 * (size_t)F.N0 : 0,
                               occ ? (size_t)F.N0 : 0,
                               occ ? sizeof(float) * 10 * n1 : 0,
                               occ ? sizeof(unsigned) * 4 * n1 : 0,
                               P.pt_cap > 0 ? 8 * pt_xtag_words(F.G0) : 0};
        for (int k = 0; k < SF_FRAME_BUFS; ++k) {
            o[f * SF_FRAME_BUFS + k] = off;
            off += align_up(sz[k]);
        }
    }
    const size_t cst_off = off;
    off += align_up(sizeof(DevConst) * P.nf);
    const size_t io_off = off;
    off += align_up(sizeof(FrameIO) * P.nf);
    const size_t stage_len = off - cst_off;
    const size_t tab_off = off;
    long ntab = 0;
    P.slot_off.assign(P.Lmax, 0);
    for (int l = 0; l < P.Lmax; ++l) {
        P.slot_off[l] = ntab;
        for (int f = 0; f < P.nf; ++f) ntab += P.fr[f].L > l ? 1 : 0;
    }
    off += align_up(sizeof(LevelArgs) * (size_t)ntab);
    P.pool_bytes = off;
    hipError_t e = hipSuccess;
    if (ext) {
        if (off > ext->cap) {
            snprintf(g_err, sizeof(g_err),
                     "workspace of %zu bytes exceeds the %zu bytes available", off, ext->cap);
            return SF_ERR_SIZE;
        }
        P.pool = ext->base;
        P.external = true;
    } else {
        e = hipMalloc(&P.pool, off);
        if (e != hipSuccess) {
            note_hip_error("hipMalloc(workspace)", e);
            P.pool = nullptr;
            return SF_ERR_OOM;
        }
        e = hipHostMalloc(&P.stage, stage_len, hipHostMallocDefault);
        if (e != hipSuccess) {
            note_hip_error("hipHostMalloc(staging)", e);
            P.stage = nullptr;
            return SF_ERR_OOM;
        }
        memset(P.stage, 0, stage_len);
        P.stage_bytes = stage_len;
        HIP_TRY(hipEventCreateWithFlags(&P.stage_ev, hipEventDisableTiming));
    }
    P.dcst = (DevConst *)(P.pool + cst_off);
    P.dio = (FrameIO *)(P.pool + io_off);
    P.dtab = (LevelArgs *)(P.pool + tab_off);
    for (int f = 0; f < P.nf; ++f) {
        FrameBuf &F = P.fr[f];
        F.tex = (float4 *)(P.pool + o[f * SF_FRAME_BUFS + 0]);
        F.cmask = (unsigned char *)(P.pool + o[f * SF_FRAME_BUFS + 1]);
        F.wnode = (float *)(P.pool + o[f * SF_FRAME_BUFS + 2]);
        F.reg = (float *)(P.pool + o[f * SF_FRAME_BUFS + 3]);
        F.nodes = (float *)(P.pool + o[f * SF_FRAME_BUFS + 4]);
        F.gram = (float *)(P.pool + o[f * SF_FRAME_BUFS + 5]);
        F.grad = (float *)(P.pool + o[f * SF_FRAME_BUFS + 9]);
        F.blk = nb ? (float *)(P.pool + o[f * SF_FRAME_BUFS + 10]) : nullptr;
        F.prev = prm.temporal ? (float *)(P.pool + o[f * SF_FRAME_BUFS + 11]) : nullptr;
        F.illum = prm.illum ? (float *)(P.pool + o[f * SF_FRAME_BUFS + 12]) : nullptr;
        if (prm.occlusion && F.L > 1) {
            F.occ = (unsigned char *)(P.pool + o[f * SF_FRAME_BUFS + 13]);
            F.occ_pos = (float *)(P.pool + o[f * SF_FRAME_BUFS + 14]);
            F.occ_zb = (unsigned *)(P.pool + o[f * SF_FRAME_BUFS + 15]);
        }
        F.partials = (float *)(P.pool + o[f * SF_FRAME_BUFS + 6]);
        F.xtag = P.pt_cap > 0 ? (unsigned long long *)(P.pool + o[f * SF_FRAME_BUFS + 16])
                              : nullptr;
        F.sc = (DevScalars *)(P.pool + o[f * SF_FRAME_BUFS + 7]);
        F.log = (DevLog *)(P.pool + o[f * SF_FRAME_BUFS + 8]);
        F.cst = P.dcst + f;
        F.io = P.dio + f;
    }
    // zeroed workspace (a caller-provided one is cleared by its caller)
    if (!ext) HIP_TRY(hipMemset(P.pool, 0, off));
    // learned initialiser: frames with a level 4, grouped by its size
    std::vector<const float *> cnn_out(P.nf, nullptr);
    if (prm.init_mode == 1 && !ext) {
        CnnRun &R = P.cnn;
        for (int f = 0; f < P.nf; ++f) {
            const FrameBuf &F = P.fr[f];
            if (F.L <= SF_CNN_INPUT_LEVEL) continue;
            const int W4 = F.lv[SF_CNN_INPUT_LEVEL].W, H4 = F.lv[SF_CNN_INPUT_LEVEL].H;
            CnnGroup *g = nullptr;
            for (CnnGroup &q : R.groups)
                if (q.W4 == W4 && q.H4 == H4) g = &q;
            if (!g) {
                R.groups.emplace_back();
                g = &R.groups.back();
                g->W4 = W4;
                g->H4 = H4;
            }
            g->frames.push_back(f);
        }
        size_t tot = 0;
        std::vector<size_t> goff;
        for (const CnnGroup &g : R.groups) {
            const size_t n = (size_t)g.W4 * g.H4 * g.frames.size();
            goff.push_back(tot);
            tot += align_up(2 * 16 * n) + align_up(2 * 32 * n * (SF_CNN_LAYERS - 1)) +
                   align_up(sizeof(float) * 6 * n);
        }
        if (tot > 0) {
            e = hipMalloc(&R.pool, tot);
            if (e != hipSuccess) {
                note_hip_error("hipMalloc(initialiser)", e);
                R.pool = nullptr;
                return SF_ERR_OOM;
            }
            HIP_TRY(hipMemset(R.pool, 0, tot));
        }
        R.slot_has.assign(P.Lmax, false);
        for (size_t k = 0; k < R.groups.size(); ++k) {
            CnnGroup &g = R.groups[k];
            const size_t n4 = (size_t)g.W4 * g.H4, n = n4 * g.frames.size();
            char *b = R.pool + goff[k];
            g.x = (unsigned short *)b;
            b += align_up(2 * 16 * n);
            for (int l = 0; l < SF_CNN_LAYERS - 1; ++l)
                g.acts[l] = (unsigned short *)b + (size_t)l * 32 * n;
            b += align_up(2 * 32 * n * (SF_CNN_LAYERS - 1));
            g.out = (float *)b;
            for (size_t i = 0; i < g.frames.size(); ++i) {
                cnn_out[g.frames[i]] = g.out + 6 * n4 * i;
                R.slot_has[P.fr[g.frames[i]].L - 1] = true;
            }
        }
        R.on = !R.groups.empty();
    }
    // per-slot kernel arguments
    P.host.assign(P.Lmax, {});
    std::vector<LevelArgs> flat;
    for (int l = 0; l < P.Lmax; ++l) {
        for (int f = 0; f < P.nf; ++f) {
            FrameBuf &F = P.fr[f];
            if (F.L <= l) continue;
            LevelArgs a;
            memset(&a, 0, sizeof(a));
            a.d = F.lv[l];
            a.level = l;
            a.s = st;
            a.N0 = (int)F.N0;
            a.G0 = (int)F.G0;
            a.coarsest = l == F.L - 1;
            a.Gxc = l + 1 < F.L ? F.lv[l + 1].Gx : 1;
            a.Gyc = l + 1 < F.L ? F.lv[l + 1].Gy : 1;
            a.log_base = 0;  // coarsest level first
            for (int k = l + 1; k < F.L; ++k) a.log_base += gn_at(prm, k);
            a.Wf = l > 0 ? F.lv[l - 1].W : 0;
            a.Hf = l > 0 ? F.lv[l - 1].H : 0;
            a.tex = F.tex + F.lv[l].tex_off;
            a.tex_fine = l > 0 ? F.tex + F.lv[l - 1].tex_off : nullptr;
            a.io = F.io;
            a.nodes = F.nodes;
            a.gram = F.gram;
            a.grad = F.grad;
            a.cmask = F.cmask;
            a.wnode = F.wnode;
            a.reg = F.reg;
            a.blk = F.blk;
            a.temporal = prm.temporal;
            a.illum = F.illum;
            a.ill_e = F.illum ? F.illum + F.N0 : nullptr;
            a.ill_t = F.illum ? F.illum + 2 * F.N0 : nullptr;
            // the map a level reads is written after the next coarser one
            a.occ = F.occ && l < F.L - 1 ? F.occ : nullptr;
            a.occ_next = F.occ && l > 0 ? F.occ : nullptr;
            a.occ_pos = F.occ_pos;
            a.occ_zb = F.occ_zb;
            a.prev = nullptr;
            if (prm.temporal) {
                long goff = 0;
                for (int k = 0; k < l; ++k) goff += F.lv[k].G;
                a.prev = F.prev + 16 * goff;
            }
            a.partials = F.partials;
            a.max_blocks = F.max_blocks;
            a.xtag = F.xtag;
            a.cst = F.cst;
            a.sc = F.sc;
            a.log = F.log;
            if (cnn_out[f] && l == F.L - 1) {
                a.learned = 1;
                a.W4 = F.lv[SF_CNN_INPUT_LEVEL].W;
                a.H4 = F.lv[SF_CNN_INPUT_LEVEL].H;
                a.cnn_out = cnn_out[f];
            }
            P.host[l].push_back(a);
            flat.push_back(a);
        }
    }
    if (ext) return SF_OK;  // single frames take their arguments by value
    if (!flat.empty())
        HIP_TRY(hipMemcpy(P.dtab, flat.data(), sizeof(LevelArgs) * flat.size(),
                          hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    return SF_OK;
}

Launch slot(const Plan &P, int l) {
    Launch L;
    L.nf = (int)P.host[l].size();
    L.host = P.host[l].data();
    L.dev = P.dtab + P.slot_off[l];
    L.batched = P.batched;
    return L;
}

// Uploads per-frame constants (and, for batches, caller buffers) through
// the pinned staging copy; the previous upload must have landed first.
sf_status upload(Plan &P, hipStream_t st, const sf_params &prm, const sf_calib *const *cal,
                 const FrameIO *io) {
    if (P.stage_pending) {
        HIP_TRY(hipEventSynchronize(P.stage_ev));
        P.stage_pending = false;
    }
    DevConst *hc = (DevConst *)P.stage;
    FrameIO *hio = (FrameIO *)(P.stage + ((char *)P.dio - (char *)P.dcst));
    bool changed = !P.have_inputs;
    for (int f = 0; f < P.nf; ++f) {
        DevConst k;
        fill_const(P.fr[f].L, prm, *cal[f], k);
        if (memcmp(&k, hc + f, sizeof(k)) != 0) {
            hc[f] = k;
            changed = true;
        }
        if (io && memcmp(&io[f], hio + f, sizeof(FrameIO)) != 0) {
            hio[f] = io[f];
            changed = true;
        }
    }
    if (!changed) return SF_OK;
    HIP_TRY(hipMemcpyAsync(P.dcst, P.stage, P.stage_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(P.stage_ev, st));
    P.stage_pending = true;
    return SF_OK;
}

// ---- the level loop ----------------------------------------------------------

void enqueue_pyramid(const Plan &P, hipStream_t st, const float *const img[4]) {
    launch_tex_level0(st, slot(P, 0), img);
    for (int l = 1; l < P.Lmax; ++l) launch_downsample(st, slot(P, l));
}

void enqueue_linearize(const Plan &P, hipStream_t st, int l) {
    const Launch L = slot(P, l);
    launch_linearize(st, L);
    if (P.prm.apply_mode >= 1)
        launch_rhs_blocks(st, L);
    else
        launch_rhs(st, L, P.tile);
}

// Levels of a single frame that the co-resident tiled PCG takes (apply_mode
// 3): more nodes than the one-workgroup kernel, and tiles the device holds
// at once.
bool pt_level(const Plan &P, int l) {
    if (P.prm.apply_mode != 3 || P.pt_cap <= 0 || P.no_mid || P.batched) return false;
    const LevelDims &d = P.fr[0].lv[l];
    const int cap = P.pt_cap < SF_PT_MAXWG ? P.pt_cap : SF_PT_MAXWG;
    return d.G > SF_SMALL_G && pt_tiles(d) <= cap;
}

// With apply_mode 2 the frames of a slot with at most SF_SMALL_G nodes run
// their PCG in one workgroup each and the others in the multi-kernel form,
// so a frame takes the same path alone or in any batch.  apply_mode 3
// (single frames; batches run it as 2) also gives mid-size levels their
// PCG in a few co-resident workgroups.
void enqueue_pcg(const Plan &P, hipStream_t st, int l, int gn, bool pend = false) {
    const Launch L = slot(P, l);
    const int n = P.prm.pcg_iters;
    if (pt_level(P, l)) {
        launch_pcg_tile(st, L, n, gn, pend);
        return;
    }
    const bool sm = P.prm.apply_mode >= 2;
    if (sm) launch_pcg_small(st, L, n, gn, pend);
    const TileCfg &t = P.ptile[l];
    launch_pcg_first(st, L, t, sm, pend);
    for (int i = 1; i < n; ++i) launch_pcg_iter(st, L, t, i, gn, 0, sm);
    launch_pcg_last(st, L, t, n, gn, 0, sm);
}

// Step control with the PCG solution in x: tau = 1 alone (usually
// accepted), then the shorter steps together, then the update of delta.
void enqueue_step(const Plan &P, hipStream_t st, int l, int g) {
    const Launch L = slot(P, l);
    const int T = P.prm.max_backtracks + 1;
    launch_trial0(st, L);
    if (T > 1) launch_trials_rest(st, L, T - 1);
    launch_accept(st, L, T, g, P.prm.pcg_iters);
}

void enqueue_gn(const Plan &P, hipStream_t st, int l, int g, bool log) {
    enqueue_linearize(P, st, l);
    enqueue_pcg(P, st, l, log ? g : -1);
    enqueue_step(P, st, l, log ? g : -1);
}

// The Gauss-Newton steps of level l.  In the node-block modes every step
// but the level's last ends speculatively: the linearisation at delta + dx
// (its energy is the tau = 1 trial), then the shorter-trial kernel, which
// on acceptance moves delta, so that the next step starts at its
// right-hand side.  A rejected tau = 1 is finished by the next step's
// right-hand-side and first PCG kernels (step length, records at the
// chosen point, delta).  Either way every iterate is that of the plain
// sequence (linearise, PCG, trials, accept), with three launches per step
// instead of five.
void enqueue_gn_steps(const Plan &P, hipStream_t st, int l) {
    const int n = gn_at(P.prm, l);
    const bool spec = P.prm.apply_mode >= 1;
    const int T = P.prm.max_backtracks + 1;
    const Launch L = slot(P, l);
    for (int g = 0; g < n; ++g) {
        const bool pend = spec && g > 0;
        if (pend)
            launch_rhs_blocks(st, L, T, g - 1, P.prm.pcg_iters);
        else
            enqueue_linearize(P, st, l);
        enqueue_pcg(P, st, l, g, pend);
        if (spec && g + 1 < n) {
            launch_spec_linearize(st, L);
            launch_trials_rest(st, L, T - 1, true, g, P.prm.pcg_iters);
        } else {
            enqueue_step(P, st, l, g);
        }
    }
}

// The network on the level-4 images of every frame that uses it: each
// frame's texels to the bf16 input, then one forward pass per size group.
void enqueue_cnn_forward(const Plan &P, hipStream_t st) {
    for (const CnnGroup &g : P.cnn.groups) {
        const int n4 = g.W4 * g.H4;
        for (size_t i = 0; i < g.frames.size(); ++i) {
            const FrameBuf &F = P.fr[g.frames[i]];
            launch_cnn_input_tex(st, F.tex + F.lv[SF_CNN_INPUT_LEVEL].tex_off,
                                 g.x + (size_t)16 * n4 * i, n4);
        }
        launch_cnn_forward(st, P.net->L, P.net->w, g.x, g.acts, g.out, (int)g.frames.size(),
                           g.H4, g.W4);
    }
}

void enqueue_levels(const Plan &P, hipStream_t st) {
    for (int l = P.Lmax - 1; l >= 0; --l) {
        if (P.prm.illum) launch_illum_zero(st, slot(P, l));
        if (P.cnn.on && l == P.Lmax - 1) enqueue_cnn_forward(P, st);
        // candidates and fallback energies of the frames whose coarsest
        // level this is
        if (P.cnn.on && P.cnn.slot_has[l]) launch_cnn_candidate(st, slot(P, l));
        launch_level_init(st, slot(P, l));
        enqueue_gn_steps(P, st, l);
        launch_finish_level(st, slot(P, l));
        if (P.prm.illum) launch_illum_next(st, slot(P, l));
        if (P.prm.occlusion) launch_occ_next(st, slot(P, l));
    }
}

// Everything after the inputs are staged: single frames replay the level
// loop (pyramid and output take the caller's pointers as arguments);
// batches also run pyramid and output inside the graph, reading the
// caller's pointers from the uploaded table.
void enqueue_body(const Plan &P, hipStream_t st) {
    if (P.batched) enqueue_pyramid(P, st, nullptr);
    enqueue_levels(P, st);
    if (P.batched) launch_output(st, slot(P, 0), nullptr, nullptr, nullptr);
}

sf_status ensure_graph(Plan &P, hipStream_t cap) {
    if (P.gexec) return SF_OK;
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    enqueue_body(P, cap);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(cap, &g));
    if (!g) return SF_ERR_HIP;
    hipGraphExec_t e = nullptr;
    const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        note_hip_error("hipGraphInstantiate", ie);
        (void)hipGraphDestroy(g);
        return SF_ERR_HIP;
    }
    P.graph = g;
    P.gexec = e;
    return SF_OK;
}

// ---- PCG tile autotuner --------------------------------------------------------
//
// Per level slot, every candidate shape of the PCG iteration kernel is timed
// (forced active, as graph replays timed with HIP events) on the plan's own
// buffers before the first solve, and the fastest is kept.  Choices are
// cached per (device architecture, stride, sizes of the slot's frames) in
// the process and, if SF_TUNE_CACHE names a file, in that file (one
// "key variant" line per entry).

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const Plan &P, int l, int device) {
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    std::string k = arch + "/s" + std::to_string(P.prm.grid_stride) +
                    (P.prm.apply_mode >= 1 ? "/nb/" : "/");
    for (const LevelArgs &a : P.host[l]) k += std::to_string(a.d.W) + "x" + std::to_string(a.d.H) + ",";
    return k;
}

void tune_cache_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("SF_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[1024];
    int v;
    while (fscanf(f, "%1023s %d", key, &v) == 2) g_tune[key] = v;
    fclose(f);
}

void tune_cache_store(const std::string &key, int v) {
    g_tune[key] = v;
    const char *path = getenv("SF_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d\n", key.c_str(), v);
    fclose(f);
}

sf_status autotune(sf_ctx *c, Plan &P) {
    const int st = P.prm.grid_stride;
    const bool nb = P.prm.apply_mode >= 1;
    const int nv = nb ? SF_NB_VARIANTS : tile_variants(st);
    auto pick = [&](int v) { return nb ? pick_nb_tile(v) : pick_pcg_tile(st, v); };
    hipStream_t s = c->stream;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_cache_load();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    sf_status rc = SF_OK;
    for (int l = 0; l < P.Lmax && rc == SF_OK; ++l) {
        const std::string key = tune_key(P, l, c->device);
        auto it = g_tune.find(key);
        if (it != g_tune.end() && it->second >= 0 && it->second < nv) {
            P.ptile[l] = pick(it->second);
            continue;
        }
        const Launch L = slot(P, l);
        // Each candidate's forced iterations are captured into a graph and
        // timed as graph replays (as the solve runs them; direct launches
        // would time the host's launch rate), in three rounds over the
        // candidates keeping each one's best, so that clock ramp-up and
        // noise do not favour a position.
        const int reps = 20;
        float best_v[SF_NB_VARIANTS > 3 ? SF_NB_VARIANTS : 3];
        hipGraph_t gv[SF_NB_VARIANTS > 3 ? SF_NB_VARIANTS : 3] = {};
        hipGraphExec_t ev[SF_NB_VARIANTS > 3 ? SF_NB_VARIANTS : 3] = {};
        for (int v = 0; v < nv; ++v) best_v[v] = 1e30f;
        for (int v = 0; v < nv && rc == SF_OK; ++v) {
            const TileCfg t = pick(v);
            if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                rc = SF_ERR_HIP;
                break;
            }
            for (int i = 0; i < reps; ++i) launch_pcg_iter(c->cap_stream, L, t, 2 + (i & 1), -1, 1);
            if (hipStreamEndCapture(c->cap_stream, &gv[v]) != hipSuccess || !gv[v] ||
                hipGraphInstantiate(&ev[v], gv[v], nullptr, nullptr, 0) != hipSuccess)
                rc = SF_ERR_HIP;
        }
        for (int round = 0; round < 4 && rc == SF_OK; ++round) {
            for (int v = 0; v < nv && rc == SF_OK; ++v) {
                float ms = 0.f;
                if (hipGraphLaunch(ev[v], s) != hipSuccess || hipEventRecord(e0, s) != hipSuccess ||
                    hipGraphLaunch(ev[v], s) != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    rc = SF_ERR_HIP;
                if (rc == SF_OK && ms < best_v[v]) best_v[v] = ms;
            }
        }
        for (int v = 0; v < nv; ++v) {
            if (ev[v]) (void)hipGraphExecDestroy(ev[v]);
            if (gv[v]) (void)hipGraphDestroy(gv[v]);
        }
        int best = 0;
        for (int v = 1; v < nv; ++v)
            if (best_v[v] < best_v[best]) best = v;
        if (rc == SF_OK) {
            P.ptile[l] = pick(best);
            tune_cache_store(key, best);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SF_OK && hipGetLastError() != hipSuccess) rc = SF_ERR_HIP;
    if (rc == SF_OK) P.tuned = true;
    return rc;
}

sf_status run_body(sf_ctx *c, Plan &P) {
    if (!P.tuned) {
        sf_status s = autotune(c, P);
        if (s != SF_OK) return s;
    }
    if (P.prm.exec_mode == 0) {
        sf_status s = ensure_graph(P, c->cap_stream);
        if (s != SF_OK) return s;
        HIP_TRY(hipGraphLaunch(P.gexec, c->stream));
    } else {
        enqueue_body(P, c->stream);
    }
    return SF_OK;
}

sf_status prepare_frame(sf_ctx *c, const float *const img[4], const sf_calib *cal,
                        const sf_params *p) {
    for (int k = 0; k < 4; ++k)
        if (!img[k]) return SF_ERR_INVALID_ARG;
    sf_status s = check_calib(cal);
    if (s != SF_OK) return s;
    if (p) {
        s = check_params(p);
        if (s != SF_OK) return s;
        if (!same_schedule(*p, c->prm)) return SF_ERR_STATE;
        c->prm = *p;
        c->single.prm = *p;
    }
    HIP_TRY(hipSetDevice(c->device));
    const sf_calib *cals[1] = {cal};
    s = upload(c->single, c->stream, c->prm, cals, nullptr);
    if (s != SF_OK) return s;
    enqueue_pyramid(c->single, c->stream, img);
    c->single.have_inputs = true;
    return SF_OK;
}

sf_status copy_log(hipStream_t st, const FrameBuf &F, sf_iter_log *out, int cap,
                   int *n_written) {
    HIP_TRY(hipStreamSynchronize(st));
    const int n = cap < F.nlog ? cap : F.nlog;
    std::vector<DevLog> tmp(F.nlog > 0 ? F.nlog : 1);
    HIP_TRY(hipMemcpy(tmp.data(), F.log, sizeof(DevLog) * F.nlog, hipMemcpyDeviceToHost));
    bool bad = false;
    for (int i = 0; i < n; ++i) {
        sf_iter_log &o = out[i];
        const DevLog &d = tmp[i];
        o.level = d.level;
        o.gn_iter = d.gn_iter;
        o.energy = d.energy;
        o.e_photo = d.e_photo;
        o.e_grad = d.e_grad;
        o.e_smooth = d.e_smooth;
        o.e_epi = d.e_epi;
        o.e_mag = d.e_mag;
        o.energy_after = d.energy_after;
        o.tau = d.tau;
        o.pcg_iters = d.pcg_iters;
        for (int k = 0; k < 64; ++k) o.pcg_res[k] = k < SF_MAX_PCG ? d.pcg_res[k] : 0.f;
        o.n_valid = d.n_valid;
        if (!isfinite(d.energy) || !isfinite(d.energy_after)) bad = true;
    }
    *n_written = n;
    return bad ? SF_ERR_NUMERIC : SF_OK;
}

sf_status time_kernel(hipStream_t st, const Plan &P, int kernel, int level, int reps,
                      float *avg_ms) {
    const Launch L = slot(P, level);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SF_ERR_HIP;
    }
    sf_status s = SF_OK;
    auto one = [&](int i) {
        switch (kernel) {
            case SF_KERNEL_APPLY: launch_pcg_iter(st, L, P.ptile[level], 2 + (i & 1), -1, 1); break;
            case SF_KERNEL_LINEARIZE: launch_linearize(st, L); break;
            case SF_KERNEL_UPDATE: launch_pcg_last(st, L, P.ptile[level], 2 + (i & 1), -1, 1); break;
            case SF_KERNEL_RHS:
                if (P.prm.apply_mode >= 1)
                    launch_rhs_blocks(st, L);
                else
                    launch_rhs(st, L, P.tile);
                break;
            case SF_KERNEL_BLOCKS: launch_rhs_blocks(st, L); break;
            case SF_KERNEL_PCG_TILE: launch_pcg_tile(st, L, P.prm.pcg_iters, -1); break;
        }
    };
    if (kernel < SF_KERNEL_APPLY || kernel > SF_KERNEL_PCG_TILE ||
        (kernel == SF_KERNEL_BLOCKS && P.prm.apply_mode < 1) ||
        (kernel == SF_KERNEL_PCG_TILE && !pt_level(P, level))) {
        s = SF_ERR_INVALID_ARG;
    } else {
        // the PCG kernels are forced active with fixed step lengths so that
        // every launch does the full work; the state is scratch afterwards
        one(0);  // warm-up
        if (hipEventRecord(e0, st) != hipSuccess) s = SF_ERR_HIP;
        for (int i = 0; i < reps && s == SF_OK; ++i) one(i);
        if (s == SF_OK && hipEventRecord(e1, st) != hipSuccess) s = SF_ERR_HIP;
        if (s == SF_OK && hipGetLastError() != hipSuccess) s = SF_ERR_HIP;
        if (s == SF_OK && hipEventSynchronize(e1) != hipSuccess) s = SF_ERR_HIP;
        float ms = 0.f;
        if (s == SF_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = SF_ERR_HIP;
        if (s == SF_OK) *avg_ms = ms / (float)reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

int batch_levels(int W, int H, int max_levels) {
    int L = 1;
    while (L < max_levels && (W >> L) >= 40) ++L;
    while (L > 1 && ((W >> (L - 1)) < 8 || (H >> (L - 1)) < 8)) --L;
    return L;
}

// Allocates the context's network weight buffers (once).
sf_status ensure_net(sf_ctx *c) {
    CnnNet &N = c->net;
    if (N.pool) return SF_OK;
    N.L = cnn_layout();
    const size_t sz[] = {sizeof(float) * N.L.n_params, 2 * (size_t)N.L.dev_w_total,
                         2 * (size_t)N.L.dev_w_total, sizeof(float) * N.L.dev_b_total};
    size_t off[4], tot = 0;
    for (int k = 0; k < 4; ++k) {
        off[k] = tot;
        tot += align_up(sz[k]);
    }
    const hipError_t e = hipMalloc(&N.pool, tot);
    if (e != hipSuccess) {
        note_hip_error("hipMalloc(initialiser weights)", e);
        N.pool = nullptr;
        return SF_ERR_OOM;
    }
    HIP_TRY(hipMemset(N.pool, 0, tot));
    N.flat = (float *)(N.pool + off[0]);
    N.w.wf = (unsigned short *)(N.pool + off[1]);
    N.w.wd = (unsigned short *)(N.pool + off[2]);
    N.w.bias = (float *)(N.pool + off[3]);
    return SF_OK;
}

}  // namespace

extern "C" {

sf_status sf_params_default(sf_params *out) {
    if (!out) return SF_ERR_INVALID_ARG;
    memset(out, 0, sizeof(*out));
    out->levels = 3;
    out->grid_stride = 8;
    out->gn_iters = 5;
    out->pcg_iters = 10;
    out->max_backtracks = 4;
    out->init_mode = 0;
    out->exec_mode = 0;
    out->apply_mode = 2;
    out->w_reg = 0.5f;
    out->w_photo = 0.5f;
    out->w_grad = 5.0f;
    out->w_epi = 0.5f;
    out->w_smooth = 1.0f;
    out->w_mag = 1.0f;
    out->w_s = 0.75f;
    out->w_m = 0.5f;
    out->w_d = 0.01f;
    out->m_s = 0.5f;
    out->m_m = 10.0f;
    out->m_d = 100.0f;
    out->eps = 0.001f;
    out->eps_p = 0.2f;
    out->st_gamma = 4.0f;
    out->st_tau = 1e-3f;
    return SF_OK;
}

sf_status sf_create(sf_ctx **out, int width, int height, const sf_params *p,
                    void *hip_stream) {
    if (!out) return SF_ERR_INVALID_ARG;
    *out = nullptr;
    sf_status s = check_params(p);
    if (s != SF_OK) return s;
    if (width < 8 || height < 8) return SF_ERR_SIZE;
    // every level must be at least 8 x 8
    if ((width >> (p->levels - 1)) < 8 || (height >> (p->levels - 1)) < 8) return SF_ERR_SIZE;
    sf_ctx *c = new (std::nothrow) sf_ctx();
    if (!c) return SF_ERR_OOM;
    c->W = width;
    c->H = height;
    c->prm = *p;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        note_hip_error("sf_create: device / capture stream", e);
        delete c;
        return SF_ERR_HIP;
    }
    if (p->init_mode == 1) s = ensure_net(c);
    if (s == SF_OK) s = build_plan(c->single, *p, {width, height}, {p->levels}, false, &c->net);
    if (s != SF_OK) {
        if (c->net.pool) (void)hipFree(c->net.pool);
        free_plan(c->single);
        (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return s;
    }
    *out = c;
    return SF_OK;
}

sf_status sf_solve(sf_ctx *c, const float *I_left_t, const float *I_right_t,
                   const float *I_left_t1, const float *I_right_t1,
                   const sf_calib *calib, const sf_params *p, float *depth,
                   float *flow3d, float *flows) {
    if (!c || !depth || !flow3d) return SF_ERR_INVALID_ARG;
    const float *img[4] = {I_left_t, I_right_t, I_left_t1, I_right_t1};
    sf_status s = prepare_frame(c, img, calib, p);
    if (s != SF_OK) return s;
    if (c->single.cnn.on && !c->net.have_weights) return SF_ERR_STATE;
    s = run_body(c, c->single);
    if (s != SF_OK) return s;
    launch_output(c->stream, slot(c->single, 0), depth, flow3d, flows);
    HIP_TRY(hipGetLastError());
    return SF_OK;
}

int sf_batch_levels(int width, int height, int max_levels) {
    if (width < 8 || height < 8 || max_levels < 1) return 0;
    return batch_levels(width, height, max_levels < SF_MAX_LEVELS ? max_levels : SF_MAX_LEVELS);
}

sf_status sf_solve_batch(sf_ctx *c, int n, const sf_frame *frames, const sf_params *p) {
    if (!c || !frames || n < 1 || n > SF_MAX_BATCH) return SF_ERR_INVALID_ARG;
    const sf_params prm = p ? *p : c->prm;
    sf_status s = check_params(&prm);
    if (s != SF_OK) return s;
    // batches keep no temporal state; the learned initialisation needs the
    // context's network
    if (prm.temporal != 0) return SF_ERR_INVALID_ARG;
    if (prm.init_mode == 1 && !c->net.have_weights) return SF_ERR_STATE;
    std::vector<int> shape(2 * n), levels(n);
    std::vector<const sf_calib *> cals(n);
    std::vector<FrameIO> io(n);
    for (int f = 0; f < n; ++f) {
        const sf_frame &F = frames[f];
        for (int k = 0; k < 4; ++k)
            if (!F.img[k]) return SF_ERR_INVALID_ARG;
        if (!F.depth || !F.flow3d) return SF_ERR_INVALID_ARG;
        if (F.width < 16 || F.height < 16) return SF_ERR_SIZE;
        s = check_calib(&F.calib);
        if (s != SF_OK) return s;
        shape[2 * f] = F.width;
        shape[2 * f + 1] = F.height;
        levels[f] = batch_levels(F.width, F.height, prm.levels);
        cals[f] = &F.calib;
        for (int k = 0; k < 4; ++k) io[f].img[k] = F.img[k];
        io[f].depth = F.depth;
        io[f].flow3d = F.flow3d;
        io[f].flows = F.flows;
    }
    HIP_TRY(hipSetDevice(c->device));
    Plan *P = c->batch;
    if (P && (P->shape != shape || !same_schedule(P->prm, prm) ||
              P->prm.exec_mode != prm.exec_mode)) {
        // a different batch shape: the old workspace may still be in use
        HIP_TRY(hipStreamSynchronize(c->stream));
        free_plan(*P);
        delete P;
        c->batch = P = nullptr;
    }
    if (!P) {
        P = new (std::nothrow) Plan();
        if (!P) return SF_ERR_OOM;
        s = build_plan(*P, prm, shape, levels, true, &c->net);
        if (s != SF_OK) {
            free_plan(*P);
            delete P;
            return s;
        }
        c->batch = P;
    }
    P->prm = prm;
    s = upload(*P, c->stream, prm, cals.data(), io.data());
    if (s != SF_OK) return s;
    P->have_inputs = true;
    s = run_body(c, *P);
    if (s != SF_OK) return s;
    HIP_TRY(hipGetLastError());
    return SF_OK;
}

sf_status sf_get_log(sf_ctx *c, sf_iter_log *out, int cap, int *n_written) {
    if (!c || !n_written || (cap > 0 && !out) || cap < 0) return SF_ERR_INVALID_ARG;
    sf_status s = copy_log(c->stream, c->single.fr[0], out, cap, n_written);
    if (s != SF_OK && s != SF_ERR_NUMERIC) return s;
    // a co-resident PCG that gave up waiting leaves the solve undefined:
    // report it, clear the flag and use the per-iteration kernels from now on
    Plan &P = c->single;
    if (P.prm.apply_mode == 3) {
        int fail = 0;
        HIP_TRY(hipMemcpy(&fail, &P.fr[0].sc->mid_fail, sizeof(int), hipMemcpyDeviceToHost));
        if (fail) {
            const int zero = 0;
            HIP_TRY(hipMemcpy(&P.fr[0].sc->mid_fail, &zero, sizeof(int), hipMemcpyHostToDevice));
            P.no_mid = true;
            if (P.gexec) (void)hipGraphExecDestroy(P.gexec);
            if (P.graph) (void)hipGraphDestroy(P.graph);
            P.gexec = nullptr;
            P.graph = nullptr;
            snprintf(g_err, sizeof(g_err),
                     "co-resident PCG workgroups gave up waiting for each other: the last "
                     "solve is undefined; later solves use the per-iteration kernels");
            return SF_ERR_STATE;
        }
    }
    return s;
}

sf_status sf_get_batch_log(sf_ctx *c, int frame, sf_iter_log *out, int cap, int *n_written) {
    if (!c || !n_written || (cap > 0 && !out) || cap < 0) return SF_ERR_INVALID_ARG;
    if (!c->batch || !c->batch->have_inputs) return SF_ERR_STATE;
    if (frame < 0 || frame >= c->batch->nf) return SF_ERR_INVALID_ARG;
    return copy_log(c->stream, c->batch->fr[frame], out, cap, n_written);
}

sf_status sf_set_initializer(sf_ctx *c, const void *weights, size_t bytes) {
    if (!c || !weights) return SF_ERR_INVALID_ARG;
    if (bytes != 2 * (size_t)cnn_layout().n_params) return SF_ERR_SIZE;
    const int n = cnn_layout().n_params;
    const unsigned short *h = (const unsigned short *)weights;
    std::vector<float> f(n);
    for (int k = 0; k < n; ++k) {
        const unsigned u = (unsigned)h[k] << 16;
        float v;
        memcpy(&v, &u, 4);
        if (!isfinite(v)) return SF_ERR_INVALID_ARG;
        f[k] = v;
    }
    HIP_TRY(hipSetDevice(c->device));
    sf_status s = ensure_net(c);
    if (s != SF_OK) return s;
    CnnNet &N = c->net;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(N.flat, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice));
    launch_cnn_pack(c->stream, N.L, N.flat, N.w.wf, N.w.wd, N.w.bias);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    N.have_weights = true;
    return SF_OK;
}

namespace {
sf_status init_result(sf_ctx *c, const Plan &P, int frame, int *used, double *e_pred,
                      double *e_zero) {
    const FrameBuf &F = P.fr[frame];
    if (F.L <= SF_CNN_INPUT_LEVEL) {
        *used = -1;
        *e_pred = *e_zero = nan("");
        return SF_OK;
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    DevScalars sc;
    HIP_TRY(hipMemcpy(&sc, F.sc, sizeof(sc), hipMemcpyDeviceToHost));
    *used = sc.init_used;
    *e_pred = sc.e_init[0];
    *e_zero = sc.e_init[1];
    return SF_OK;
}
}  // namespace

sf_status sf_get_init_result(sf_ctx *c, int *used, double *e_pred, double *e_zero) {
    if (!c || !used || !e_pred || !e_zero) return SF_ERR_INVALID_ARG;
    if (!c->single.cnn.on || !c->single.have_inputs) return SF_ERR_STATE;
    return init_result(c, c->single, 0, used, e_pred, e_zero);
}

sf_status sf_get_batch_init_result(sf_ctx *c, int frame, int *used, double *e_pred,
                                   double *e_zero) {
    if (!c || !used || !e_pred || !e_zero) return SF_ERR_INVALID_ARG;
    const Plan *P = c->batch;
    if (!P || !P->have_inputs || P->prm.init_mode != 1) return SF_ERR_STATE;
    if (frame < 0 || frame >= P->nf) return SF_ERR_INVALID_ARG;
    return init_result(c, *P, frame, used, e_pred, e_zero);
}

// ---- solves without allocation ------------------------------------------
//
// The workspace of sf_solve_noalloc lives in this library's static device
// array, SF_NOALLOC_SCRATCH_BYTES per device for the life of the process.
// In host code `scratch` only names the symbol: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is handed to kernels.

}  // extern "C"

static __device__ __align__(256) char scratch[SF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SF_NOALLOC_DEVICES = 64;
struct NoAllocState {
    std::mutex mu;
    char *ptr = nullptr;  // device address of this device's `scratch`
    Plan plan;            // host-side layout of the last call's frame
    bool have_plan = false;
    int W = 0, H = 0;
};
NoAllocState g_noalloc[SF_NOALLOC_DEVICES];
}  // namespace

extern "C" {

sf_status sf_solve_noalloc(int width, int height, const float *I_left_t, const float *I_right_t,
                           const float *I_left_t1, const float *I_right_t1,
                           const sf_calib *calib, const sf_params *p, float *depth,
                           float *flow3d, float *flows, void *hip_stream) {
    if (!depth || !flow3d) return SF_ERR_INVALID_ARG;
    const float *img[4] = {I_left_t, I_right_t, I_left_t1, I_right_t1};
    for (int k = 0; k < 4; ++k)
        if (!img[k]) return SF_ERR_INVALID_ARG;
    sf_status s = check_params(p);
    if (s != SF_OK) return s;
    // no network weights and no state between calls
    if (p->init_mode != 0 || p->temporal != 0) return SF_ERR_INVALID_ARG;
    s = check_calib(calib);
    if (s != SF_OK) return s;
    if (width < 8 || height < 8) return SF_ERR_SIZE;
    if ((width >> (p->levels - 1)) < 8 || (height >> (p->levels - 1)) < 8) return SF_ERR_SIZE;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= SF_NOALLOC_DEVICES) return SF_ERR_INVALID_ARG;
    NoAllocState &S = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    if (!S.ptr) {
        void *q = nullptr;
        HIP_TRY(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
        if (!q) return SF_ERR_HIP;
        S.ptr = (char *)q;
    }
    // direct launches with the default (or a forced) tile shape: autotuning
    // and graph capture would allocate
    sf_params prm = *p;
    prm.exec_mode = 1;
    if (prm.tile_mode == 1) prm.tile_mode = 0;
    if (!S.have_plan || S.W != width || S.H != height || !same_schedule(S.plan.prm, prm)) {
        S.have_plan = false;
        free_plan(S.plan);
        ExtPool ext;
        ext.base = S.ptr;
        ext.cap = SF_NOALLOC_SCRATCH_BYTES;
        s = build_plan(S.plan, prm, {width, height}, {prm.levels}, false, nullptr, &ext);
        if (s != SF_OK) {
            free_plan(S.plan);
            return s;
        }
        S.have_plan = true;
        S.W = width;
        S.H = height;
    }
    Plan &P = S.plan;
    P.prm = prm;
    hipStream_t st = (hipStream_t)hip_stream;
    // the previous call's contents: cleared, then this call's constants
    launch_fill_zero(st, S.ptr, P.pool_bytes);
    DevConst k;
    fill_const(P.fr[0].L, prm, *calib, k);
    launch_store_const(st, k, P.fr[0].cst);
    enqueue_pyramid(P, st, img);
    enqueue_body(P, st);
    launch_output(st, slot(P, 0), depth, flow3d, flows);
    HIP_TRY(hipGetLastError());
    return SF_OK;
}

const char *sf_last_error(void) { return g_err; }

const char *sf_status_string(sf_status s) {
    switch (s) {
        case SF_OK: return "ok";
        case SF_ERR_INVALID_ARG: return "invalid argument";
        case SF_ERR_SIZE: return "image size not supported for the requested levels";
        case SF_ERR_HIP: return "HIP runtime error";
        case SF_ERR_OOM: return "out of device memory";
        case SF_ERR_NUMERIC: return "non-finite energy";
        case SF_ERR_STATE: return "call not valid in the context's state";
    }
    return "unknown status";
}

sf_status sf_reset_sequence(sf_ctx *c) {
    if (!c) return SF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->device));
    for (FrameBuf &F : c->single.fr)
        HIP_TRY(hipMemsetAsync(&F.sc->have_prev, 0, sizeof(int), c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SF_OK;
}

void sf_destroy(sf_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->batch) {
        free_plan(*c->batch);
        delete c->batch;
    }
    free_plan(c->single);
    if (c->net.pool) (void)hipFree(c->net.pool);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

// ---- test support ---------------------------------------------------------

size_t sf_debug_size(sf_ctx *c, int what, int level) {
    if (!c || level < 0 || level >= c->single.fr[0].L) return 0;
    const LevelDims &d = c->single.fr[0].lv[level];
    switch (what) {
        case SF_DBG_TEX: return sizeof(float4) * 4 * (size_t)d.N;
        case SF_DBG_CMASK: return (size_t)d.N;
        case SF_DBG_WNODE: return sizeof(float) * (size_t)d.G;
        case SF_DBG_BASE: case SF_DBG_DELTA: case SF_DBG_DX: case SF_DBG_R:
        case SF_DBG_Z: case SF_DBG_Q: case SF_DBG_DIAG: case SF_DBG_P:
            return sizeof(float) * 6 * (size_t)d.G;
        case SF_DBG_REC: return sizeof(float) * SF_REC_PLANES * (size_t)d.N;
        case SF_DBG_ENERGY: return sizeof(double) * 6;
        case SF_DBG_OCC: return c->single.fr[0].occ ? (size_t)d.N : 0;
    }
    return 0;
}

static int node_vec_of(int what) {
    switch (what) {
        case SF_DBG_BASE: return NV_BASE;
        case SF_DBG_DELTA: return NV_DELTA;
        case SF_DBG_DX: return NV_X;
        case SF_DBG_R: return NV_R0;
        case SF_DBG_Z: return NV_U;
        case SF_DBG_Q: return NV_W0;
        case SF_DBG_DIAG: return NV_DIAG;
        case SF_DBG_P: return NV_U;
    }
    return -1;
}

static sf_status debug_copy(sf_ctx *c, int what, int level, void *host, size_t bytes,
                            bool to_device) {
    if (!c || !host) return SF_ERR_INVALID_ARG;
    const size_t need = sf_debug_size(c, what, level);
    if (need == 0) return SF_ERR_INVALID_ARG;
    if (bytes != need) return SF_ERR_SIZE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const FrameBuf &F = c->single.fr[0];
    const LevelDims &d = F.lv[level];
    const hipMemcpyKind kind = to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
    char *h = (char *)host;
    auto cp = [&](void *dev, size_t off, size_t n) -> bool {
        return to_device ? hipMemcpy((char *)dev, h + off, n, kind) == hipSuccess
                         : hipMemcpy(h + off, (char *)dev, n, kind) == hipSuccess;
    };
    bool ok = true;
    switch (what) {
        case SF_DBG_TEX: ok = cp(F.tex + d.tex_off, 0, bytes); break;
        case SF_DBG_CMASK: ok = cp(F.cmask, 0, bytes); break;
        case SF_DBG_OCC: ok = cp(F.occ, 0, bytes); break;
        case SF_DBG_WNODE: ok = cp(F.wnode, 0, bytes); break;
        case SF_DBG_REC: {
            // records are per pixel on the device, planes at the interface
            std::vector<float> g((size_t)SF_GRAM_STRIDE * d.N), r((size_t)SF_GRAD_STRIDE * d.N);
            float *hp = (float *)host;
            if (to_device) {
                for (long p = 0; p < d.N; ++p) {
                    for (int q = 0; q < 6; ++q) r[p * SF_GRAD_STRIDE + q] = hp[(size_t)q * d.N + p];
                    for (int i = 0, t = 0; i < 6; ++i)
                        for (int j = i; j < 6; ++j, ++t)
                            g[p * SF_GRAM_STRIDE + gram_index(i, j)] = hp[(size_t)(6 + t) * d.N + p];
                }
                ok = hipMemcpy(F.gram, g.data(), g.size() * sizeof(float), kind) == hipSuccess &&
                     hipMemcpy(F.grad, r.data(), r.size() * sizeof(float), kind) == hipSuccess;
            } else {
                ok = hipMemcpy(g.data(), F.gram, g.size() * sizeof(float), kind) == hipSuccess &&
                     hipMemcpy(r.data(), F.grad, r.size() * sizeof(float), kind) == hipSuccess;
                for (long p = 0; ok && p < d.N; ++p) {
                    for (int q = 0; q < 6; ++q) hp[(size_t)q * d.N + p] = r[p * SF_GRAD_STRIDE + q];
                    for (int i = 0, t = 0; i < 6; ++i)
                        for (int j = i; j < 6; ++j, ++t)
                            hp[(size_t)(6 + t) * d.N + p] = g[p * SF_GRAM_STRIDE + gram_index(i, j)];
                }
            }
            break;
        }
        case SF_DBG_ENERGY:
            if (to_device) return SF_ERR_INVALID_ARG;
            ok = cp(&F.sc->e_lin[0], 0, bytes);
            break;
        default: {
            // node records on the device, six planes at the interface
            const int v = node_vec_of(what);
            if (v < 0) return SF_ERR_INVALID_ARG;
            float *base = F.nodes + (size_t)v * SF_NREC * F.G0;
            std::vector<float> rec((size_t)SF_NREC * d.G, 0.f);
            float *hp = (float *)host;
            if (to_device) {
                ok = hipMemcpy(rec.data(), base, rec.size() * sizeof(float),
                               hipMemcpyDeviceToHost) == hipSuccess;
                for (long n = 0; ok && n < d.G; ++n)
                    for (int q = 0; q < 6; ++q) rec[n * SF_NREC + q] = hp[(size_t)q * d.G + n];
                ok = ok && hipMemcpy(base, rec.data(), rec.size() * sizeof(float), kind) == hipSuccess;
            } else {
                ok = hipMemcpy(rec.data(), base, rec.size() * sizeof(float), kind) == hipSuccess;
                for (long n = 0; ok && n < d.G; ++n)
                    for (int q = 0; q < 6; ++q) hp[(size_t)q * d.G + n] = rec[n * SF_NREC + q];
            }
        }
    }
    return ok ? SF_OK : SF_ERR_HIP;
}

sf_status sf_debug_read(sf_ctx *c, int what, int level, void *host_dst, size_t bytes) {
    return debug_copy(c, what, level, host_dst, bytes, false);
}

sf_status sf_debug_write(sf_ctx *c, int what, int level, const void *host_src,
                         size_t bytes) {
    return debug_copy(c, what, level, (void *)host_src, bytes, true);
}

sf_status sf_debug_set_images(sf_ctx *c, const float *I_left_t, const float *I_right_t,
                              const float *I_left_t1, const float *I_right_t1,
                              const sf_calib *calib) {
    if (!c) return SF_ERR_INVALID_ARG;
    const float *img[4] = {I_left_t, I_right_t, I_left_t1, I_right_t1};
    sf_status s = prepare_frame(c, img, calib, nullptr);
    if (s != SF_OK) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SF_OK;
}

sf_status sf_debug_run(sf_ctx *c, int stage, int level) {
    if (!c || level < 0 || level >= c->single.fr[0].L) return SF_ERR_INVALID_ARG;
    if (!c->single.have_inputs) return SF_ERR_STATE;
    hipStream_t st = c->stream;
    const Plan &P = c->single;
    const Launch L = slot(P, level);
    switch (stage) {
        case SF_STAGE_LEVEL_INIT: launch_level_init(st, L); break;
        case SF_STAGE_LINEARIZE: enqueue_linearize(P, st, level); break;
        case SF_STAGE_APPLY: launch_pcg_first(st, L, P.ptile[level]); break;
        case SF_STAGE_PCG: enqueue_pcg(P, st, level, -1); break;
        case SF_STAGE_GN: enqueue_gn(P, st, level, 0, false); break;
        case SF_STAGE_FINISH: launch_finish_level(st, L); break;
        case SF_STAGE_MASKS: launch_level_masks(st, L); break;
        case SF_STAGE_STEP: enqueue_step(P, st, level, -1); break;
        case SF_STAGE_OCC:
            if (level == 0 || !P.fr[0].occ) return SF_ERR_INVALID_ARG;
            launch_occ_next(st, L);
            break;
        case SF_STAGE_SPEC_STEP: {
            if (P.prm.apply_mode < 1) return SF_ERR_INVALID_ARG;
            const int T = P.prm.max_backtracks + 1;
            launch_spec_linearize(st, L);
            launch_trials_rest(st, L, T - 1, true, -1, P.prm.pcg_iters);
            launch_rhs_blocks(st, L, T, -1, P.prm.pcg_iters);
            enqueue_pcg(P, st, level, -1, true);
            break;
        }
        default: return SF_ERR_INVALID_ARG;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return SF_OK;
}

sf_status sf_time_kernel(sf_ctx *c, int kernel, int level, int reps, float *avg_ms) {
    if (!c || !avg_ms || level < 0 || level >= c->single.fr[0].L || reps < 1)
        return SF_ERR_INVALID_ARG;
    if (!c->single.have_inputs) return SF_ERR_STATE;
    return time_kernel(c->stream, c->single, kernel, level, reps, avg_ms);
}

sf_status sf_time_batch_kernel(sf_ctx *c, int kernel, int level, int reps, float *avg_ms) {
    if (!c || !avg_ms || reps < 1) return SF_ERR_INVALID_ARG;
    if (!c->batch || !c->batch->have_inputs) return SF_ERR_STATE;
    if (level < 0 || level >= c->batch->Lmax) return SF_ERR_INVALID_ARG;
    return time_kernel(c->stream, *c->batch, kernel, level, reps, avg_ms);
}

sf_status sf_tile_variant(sf_ctx *c, int batched, int level, int *variant) {
    if (!c || !variant) return SF_ERR_INVALID_ARG;
    const Plan *P = batched ? c->batch : &c->single;
    if (!P || !P->have_inputs) return SF_ERR_STATE;
    if (level < 0 || level >= P->Lmax) return SF_ERR_INVALID_ARG;
    // node-block tiles carry SF_TILE_NB + their shape index
    const int v = P->ptile[level].v;
    *variant = v >= SF_TILE_NB ? v - SF_TILE_NB : v;
    return SF_OK;
}

}  // extern "C"
