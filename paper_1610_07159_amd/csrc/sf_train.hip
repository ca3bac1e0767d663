// C ABI of the initialiser's trainer (include/sf.h): workspace for batches
// of level-4 image quadruples, forward, L1 loss, backward and Adam on the
// GPU, float32 master weights with bfloat16 working copies.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "sf.h"
#include "sf_cnn.h"

struct sf_trainer {
    int maxB = 0, H = 0, W = 0, lastB = 0;
    hipStream_t stream = nullptr;
    CnnLayout L{};
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    CnnWeights w{};
    unsigned short *x = nullptr, *dout = nullptr;
    unsigned short *acts[SF_CNN_LAYERS - 1]{};
    unsigned short *dpre[SF_CNN_LAYERS - 1]{};
    float *out = nullptr, *wpart = nullptr, *bpart = nullptr, *lpart = nullptr;
    int step = 0;
    bool have_params = false;
    std::vector<void *> allocs;
};

namespace {

sf_status tr_alloc(sf_trainer *t, void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return SF_ERR_OOM;
    }
    t->allocs.push_back(*p);
    return SF_OK;
}

void tr_free(sf_trainer *t) {
    for (void *p : t->allocs) (void)hipFree(p);
    t->allocs.clear();
}

sf_status run_forward(sf_trainer *t, const float *x, int B) {
    const long HW = (long)t->H * t->W;
    launch_cnn_input(t->stream, x, HW, 4 * HW, t->x, B, t->H, t->W);
    launch_cnn_forward(t->stream, t->L, t->w, t->x, t->acts, t->out, B, t->H, t->W);
    t->lastB = B;
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

}  // namespace

extern "C" {

sf_status sf_trainer_create(sf_trainer **out, int max_batch, int height, int width,
                            void *hip_stream) {
    if (!out) return SF_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_batch < 1 || height < 1 || width < 1) return SF_ERR_INVALID_ARG;
    if ((long)max_batch * height * width > (1L << 26)) return SF_ERR_SIZE;
    sf_trainer *t = new (std::nothrow) sf_trainer();
    if (!t) return SF_ERR_OOM;
    t->maxB = max_batch;
    t->H = height;
    t->W = width;
    t->stream = (hipStream_t)hip_stream;
    t->L = cnn_layout();
    const long P = (long)max_batch * height * width;
    const int n = t->L.n_params;
    const int nch = cnn_chunks(P);
    sf_status s = SF_OK;
    auto A = [&](void **p, size_t bytes) {
        if (s == SF_OK) s = tr_alloc(t, p, bytes);
    };
    A((void **)&t->master, sizeof(float) * n);
    A((void **)&t->m, sizeof(float) * n);
    A((void **)&t->v, sizeof(float) * n);
    A((void **)&t->grad, sizeof(float) * n);
    A((void **)&t->w.wf, 2 * (size_t)t->L.dev_w_total);
    A((void **)&t->w.wd, 2 * (size_t)t->L.dev_w_total);
    A((void **)&t->w.bias, sizeof(float) * t->L.dev_b_total);
    A((void **)&t->x, 2 * 16 * (size_t)P);
    A((void **)&t->dout, 2 * 16 * (size_t)P);
    for (int l = 0; l < SF_CNN_LAYERS - 1; ++l) {
        A((void **)&t->acts[l], 2 * 32 * (size_t)P);
        A((void **)&t->dpre[l], 2 * 32 * (size_t)P);
    }
    A((void **)&t->out, sizeof(float) * 6 * (size_t)P);
    A((void **)&t->wpart, sizeof(float) * (size_t)nch * 32 * 9 * 32);
    A((void **)&t->bpart, sizeof(float) * (size_t)nch * 32);
    A((void **)&t->lpart, sizeof(float) * (size_t)cnn_l1_blocks(P));
    if (s != SF_OK) {
        tr_free(t);
        delete t;
        return s;
    }
    *out = t;
    return SF_OK;
}

sf_status sf_trainer_set_params(sf_trainer *t, const float *host, size_t n) {
    if (!t || !host) return SF_ERR_INVALID_ARG;
    if (n != (size_t)t->L.n_params) return SF_ERR_SIZE;
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(host[k])) return SF_ERR_INVALID_ARG;
    if (hipMemcpyAsync(t->master, host, sizeof(float) * n, hipMemcpyHostToDevice, t->stream) !=
            hipSuccess ||
        hipMemsetAsync(t->m, 0, sizeof(float) * n, t->stream) != hipSuccess ||
        hipMemsetAsync(t->v, 0, sizeof(float) * n, t->stream) != hipSuccess)
        return SF_ERR_HIP;
    launch_cnn_pack(t->stream, t->L, t->master, t->w.wf, t->w.wd, t->w.bias);
    if (hipStreamSynchronize(t->stream) != hipSuccess) return SF_ERR_HIP;
    t->step = 0;
    t->have_params = true;
    return SF_OK;
}

sf_status sf_trainer_get_params(sf_trainer *t, float *host, size_t n) {
    if (!t || !host) return SF_ERR_INVALID_ARG;
    if (n != (size_t)t->L.n_params) return SF_ERR_SIZE;
    if (!t->have_params) return SF_ERR_STATE;
    if (hipStreamSynchronize(t->stream) != hipSuccess ||
        hipMemcpy(host, t->master, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess)
        return SF_ERR_HIP;
    return SF_OK;
}

sf_status sf_trainer_forward(sf_trainer *t, const float *x, int batch, float *out) {
    if (!t || !x || !out) return SF_ERR_INVALID_ARG;
    if (batch < 1 || batch > t->maxB) return SF_ERR_SIZE;
    if (!t->have_params) return SF_ERR_STATE;
    sf_status s = run_forward(t, x, batch);
    if (s != SF_OK) return s;
    const size_t bytes = sizeof(float) * 6 * (size_t)batch * t->H * t->W;
    if (hipMemcpyAsync(out, t->out, bytes, hipMemcpyDeviceToDevice, t->stream) != hipSuccess)
        return SF_ERR_HIP;
    return SF_OK;
}

sf_status sf_trainer_step(sf_trainer *t, const float *x, const float *target, int batch,
                          float lr, float *loss) {
    if (!t || !x || !target) return SF_ERR_INVALID_ARG;
    if (batch < 1 || batch > t->maxB) return SF_ERR_SIZE;
    if (!(lr >= 0.f) || !isfinite(lr)) return SF_ERR_INVALID_ARG;
    if (!t->have_params) return SF_ERR_STATE;
    sf_status s = run_forward(t, x, batch);
    if (s != SF_OK) return s;
    const int B = batch, H = t->H, W = t->W;
    launch_cnn_l1(t->stream, t->out, target, t->dout, t->lpart, B, H, W);
    launch_cnn_backward(t->stream, t->L, t->w, t->x, t->acts, t->dout, t->dpre, t->wpart,
                        t->bpart, t->grad, B, H, W);
    t->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, t->step)), c2 = (float)(1.0 - pow(b2, t->step));
    launch_cnn_adam(t->stream, t->master, t->m, t->v, t->grad, t->L.n_params, lr, (float)b1,
                    (float)b2, 1e-8f, c1, c2);
    launch_cnn_pack(t->stream, t->L, t->master, t->w.wf, t->w.wd, t->w.bias);
    if (hipGetLastError() != hipSuccess) return SF_ERR_HIP;
    if (loss) {
        const long P = (long)B * H * W;
        std::vector<float> part(cnn_l1_blocks(P));
        if (hipStreamSynchronize(t->stream) != hipSuccess ||
            hipMemcpy(part.data(), t->lpart, sizeof(float) * part.size(),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return SF_ERR_HIP;
        double acc = 0.0;
        for (float f : part) acc += f;
        *loss = (float)(acc / (double)(P * 6));
    }
    return SF_OK;
}

size_t sf_trainer_size(sf_trainer *t, int what, int layer) {
    if (!t || t->lastB < 1) return 0;
    const size_t P = (size_t)t->lastB * t->H * t->W;
    switch (what) {
        case SF_TR_INPUT: return 2 * 16 * P;
        case SF_TR_ACT: return layer >= 0 && layer < SF_CNN_LAYERS - 1 ? 2 * 32 * P : 0;
        case SF_TR_OUT: return sizeof(float) * 6 * P;
        case SF_TR_DOUT: return 2 * 16 * P;
        case SF_TR_DPRE: return layer >= 0 && layer < SF_CNN_LAYERS - 1 ? 2 * 32 * P : 0;
        case SF_TR_GRAD: return sizeof(float) * (size_t)t->L.n_params;
    }
    return 0;
}

sf_status sf_trainer_read(sf_trainer *t, int what, int layer, void *host, size_t bytes) {
    if (!t || !host) return SF_ERR_INVALID_ARG;
    const size_t need = sf_trainer_size(t, what, layer);
    if (need == 0) return SF_ERR_INVALID_ARG;
    if (bytes != need) return SF_ERR_SIZE;
    const void *src = nullptr;
    switch (what) {
        case SF_TR_INPUT: src = t->x; break;
        case SF_TR_ACT: src = t->acts[layer]; break;
        case SF_TR_OUT: src = t->out; break;
        case SF_TR_DOUT: src = t->dout; break;
        case SF_TR_DPRE: src = t->dpre[layer]; break;
        case SF_TR_GRAD: src = t->grad; break;
    }
    if (hipStreamSynchronize(t->stream) != hipSuccess ||
        hipMemcpy(host, src, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return SF_ERR_HIP;
    return SF_OK;
}

void sf_trainer_destroy(sf_trainer *t) {
    if (!t) return;
    (void)hipStreamSynchronize(t->stream);
    tr_free(t);
    delete t;
}

}  // extern "C"
