// Learned warm start (host side) and checkpoint files.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "ctx.h"

namespace fepic {

int mlp_grad_blocks(int64_t n);
void mlp_launch_grad(hipStream_t s, const float* X, const float* T, int64_t n, int64_t n_all, uint64_t seed,
                     const float* P, float* part, double* loss_part, int blocks);
void mlp_launch_reduce_adam(hipStream_t s, const float* part, int blocks, float* grad, float* P, float* m, float* v,
                            int adam, float lr, float b1, float b2, float eps, float bc1, float bc2);
void mlp_launch_loss_sum(hipStream_t s, const double* loss_part, int blocks, double inv_n, double* loss);

constexpr int kNP = FEPIC_MLP_N_PARAMS;
constexpr double kMaxTargetRms = 10.0;   // recorded steps: RMS of (e^{n+1} - e^n) / s_d at most this
constexpr int kMaxGradBlocks = 512;

// ---- scratch of the allocation-free gradient (fepic_mlp_grad_noalloc)
// The per-workgroup partial gradients (kNP floats each) and partial squared errors of
// k_mlp_grad, for at most kNoAllocBlocks workgroups: mlp_grad_blocks(n) <= 128 exactly
// when n <= FEPIC_MLP_NOALLOC_MAX_ROWS, so the allocation-free call launches the same grid
// as fepic_mlp_grad and sums in the same order.  Every workgroup overwrites its whole
// slice, so nothing needs clearing between calls.  One copy per GPU, for the life of the
// process.
constexpr int kNoAllocBlocks = 128;
constexpr size_t kScratchGradBytes = sizeof(float) * (size_t)kNP * kNoAllocBlocks;
constexpr size_t kScratchBytes = kScratchGradBytes + sizeof(double) * kNoAllocBlocks;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of scratch on each GPU (the array's name is only a host-side handle).
constexpr int kMaxScratchDevices = 64;
static void* g_scratch_addr[kMaxScratchDevices] = {};
static hipError_t g_scratch_err[kMaxScratchDevices] = {};
static std::mutex g_scratch_mu;

// Called by fepic_create with the context's device current: looks the array's address up
// once per device.
void mlp_noalloc_setup(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_addr[device] = p;
    else g_scratch_err[device] = (e == hipSuccess ? hipErrorInvalidSymbol : e);
}

static_assert(FEPIC_MLP_NOALLOC_MAX_ROWS == 32 * 16 * kNoAllocBlocks, "grid of the allocation-free gradient");

struct MlpState {
    float* P = nullptr;      // FP32 master weights
    float* m = nullptr;      // Adam moments
    float* v = nullptr;
    float* grad = nullptr;
    float* part = nullptr;   // [kMaxGradBlocks][kNP]
    double* loss_part = nullptr;
    double* scales = nullptr;  // s_d, s_g, line step, target RMS, s_e of the current step
    float* Xcur = nullptr;   // features of the current step [n_int][4]
    float* ycur = nullptr;
    // recording ring: each snapshot keeps rows r0, r0 + stride, ... of the interior edges
    // (n_rec of them), r0 cycling through 0..stride-1 over the snapshots taken
    float* Xrec = nullptr;   // [cap][n_rec][4]
    float* Trec = nullptr;   // [cap][n_rec]
    int64_t cap = 0, count = 0, head = 0;
    int64_t stride = 1, n_rec = 0, taken = 0;
    int64_t adam_t = 0;
    bool have_weights = false;
    // scratch for host batches
    float* Xh = nullptr;
    float* Th = nullptr;
    int64_t h_cap = 0;
};

static int ensure_mlp(fepic_ctx* c) {
    if (c->host_only) return fail(c, FEPIC_E_NO_DEVICE, "host-only context");
    if (!c->have_mesh) return fail(c, FEPIC_E_STATE, "no mesh uploaded");
    if (c->mlp) return FEPIC_OK;
    MlpState* s = new MlpState();
    const int64_t ni = std::max<int64_t>(c->mesh.n_int_edges, 1);
    s->P = (float*)dmalloc(c, sizeof(float) * kNP);
    s->m = (float*)dmalloc(c, sizeof(float) * kNP);
    s->v = (float*)dmalloc(c, sizeof(float) * kNP);
    s->grad = (float*)dmalloc(c, sizeof(float) * kNP);
    s->part = (float*)dmalloc(c, sizeof(float) * kNP * kMaxGradBlocks);
    s->loss_part = (double*)dmalloc(c, sizeof(double) * std::max(kMaxGradBlocks, 3 * 256));   // also the RMS partials
    s->scales = (double*)dmalloc(c, sizeof(double) * 5);  // s_d, s_g, line step, target RMS, s_e
    s->Xcur = (float*)dmalloc(c, sizeof(float) * 4 * ni);
    s->ycur = (float*)dmalloc(c, sizeof(float) * ni);
    c->mlp = s;
    if (!s->P || !s->m || !s->v || !s->grad || !s->part || !s->loss_part || !s->scales || !s->Xcur || !s->ycur)
        return fail(c, FEPIC_E_OOM, "device allocation failed");
    return FEPIC_OK;
}

// He-uniform weights (scaled output layer), zero biases; Adam state cleared.
static int init_weights(fepic_ctx* c, uint64_t seed) {
    std::vector<float> w(kNP, 0.f);
    std::mt19937_64 gen(seed);
    auto fill = [&](int off, int n, int fan_in, float scale) {
        std::uniform_real_distribution<float> U(-std::sqrt(6.f / fan_in), std::sqrt(6.f / fan_in));
        for (int i = 0; i < n; ++i) w[off + i] = scale * U(gen);
    };
    fill(0, 256, 4, 1.f);
    fill(320, 4096, 64, 1.f);
    fill(4480, 64, 64, 0.1f);
    MlpState* s = c->mlp;
    if (hipMemcpy(s->P, w.data(), sizeof(float) * kNP, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->m, 0, sizeof(float) * kNP) != hipSuccess || hipMemset(s->v, 0, sizeof(float) * kNP) != hipSuccess)
        return fail(c, FEPIC_E_HIP, "weight upload failed");
    s->adam_t = 0;
    s->have_weights = true;
    return FEPIC_OK;
}

// Scales and features of the current step (e^n, e^n - e^{n-1}, e^{n-1} - e^{n-2}, dG^{n+1},
// formed in FP64) into dst.
static void features_into(fepic_ctx* c, float* dst) {
    MlpState* s = c->mlp;
    const int64_t ni = c->mesh.n_int_edges;
    mlp_launch_rms(c->stream, ni, c->d_int_edges, c->d_e, c->d_ep, c->d_dgn, s->loss_part, s->scales);
    mlp_launch_features(c->stream, ni, c->d_int_edges, c->d_e, c->d_ep, c->d_ep2, c->d_dgn, s->scales, dst);
}

int mlp_warm_start(fepic_ctx* c, bool direct) {
    int rc = ensure_mlp(c);
    if (rc) return rc;
    MlpState* s = c->mlp;
    const int64_t ni = c->mesh.n_int_edges;
    features_into(c, s->Xcur);
    hipEvent_t* ev = timer_pair(c, FAM_MLP_FWD);
    if (ev) (void)hipEventRecord(ev[0], c->stream);
    mlp_launch_forward(c->stream, ni, s->Xcur, s->P, s->ycur);
    if (ev) (void)hipEventRecord(ev[1], c->stream);
    // the predicted increment d = s_d y; the line-step form moves along it to the
    // energy-norm-optimal x0 = e^n + theta d (never worse than x0 = e^n in the A-norm), the
    // direct form takes x0 = e^n + d
    double* d = c->d_Me;  // work vector, free during the solve
    launch_fill(c->stream, d, c->mesh.n_edges, 0.0);
    mlp_launch_direction(c->stream, ni, c->d_int_edges, s->ycur, s->scales, d);
    if (direct)
        launch_axpby(c->stream, c->d_x, c->d_e, 1.0, d, 1.0, c->mesh.n_edges);
    else
        launch_line_start(c->stream, c->mesh.n_edges, c->d_sp, c->d_col, c->d_A, c->d_rhs, c->d_e, d, c->d_partial,
                          s->scales + 2, c->d_x);
    return FEPIC_OK;
}

int mlp_record_features(fepic_ctx* c) {
    int rc = ensure_mlp(c);
    if (rc) return rc;
    MlpState* s = c->mlp;
    if (s->cap == 0) return FEPIC_OK;
    float* dst = s->Xrec + (size_t)s->head * s->n_rec * 4;
    const bool have = (c->opt.warm_start == FEPIC_WS_MLP || c->opt.warm_start == FEPIC_WS_MLP_DIRECT) && c->mlp_ready;
    if (!have) features_into(c, s->Xcur);
    mlp_launch_pick(c->stream, s->Xcur, s->taken % s->stride, s->stride, s->n_rec, dst);
    return FEPIC_OK;
}

int mlp_record_target(fepic_ctx* c) {
    MlpState* s = c->mlp;
    if (!s || s->cap == 0) return FEPIC_OK;
    // work: d_Me is free after the solve (the diagnostics recompute it); n_rec <= n_edges
    mlp_launch_target(c->stream, s->n_rec, s->taken % s->stride, s->stride, c->d_int_edges, c->d_x, c->d_e, c->d_Me,
                      s->loss_part, s->scales, s->Trec + (size_t)s->head * s->n_rec);
    s->taken++;
    // a step whose increment dwarfs e^n (e^n near zero: a neutral start) would teach the
    // network nothing but outliers; its slot is reused by the next snapshot
    double ratio = 0.0;
    HIPCHK_RET(c, hipMemcpyAsync(&ratio, s->scales + 3, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    if (!(ratio <= kMaxTargetRms)) return FEPIC_OK;
    s->head = (s->head + 1) % s->cap;
    s->count = std::min(s->count + 1, s->cap);
    return FEPIC_OK;
}

// Device buffers of the state are owned by the context's allocation list.
void mlp_destroy(fepic_ctx* c) {
    delete c->mlp;
    c->mlp = nullptr;
}

int mlp_save(fepic_ctx* c, std::FILE* f) {
    const int32_t have = (c->mlp && c->mlp->have_weights) ? 1 : 0;
    if (std::fwrite(&have, 4, 1, f) != 1) return FEPIC_E_IO;
    if (!have) return FEPIC_OK;
    std::vector<float> w(3 * kNP);
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    HIPCHK_RET(c, hipMemcpy(w.data(), c->mlp->P, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    HIPCHK_RET(c, hipMemcpy(w.data() + kNP, c->mlp->m, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    HIPCHK_RET(c, hipMemcpy(w.data() + 2 * kNP, c->mlp->v, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    const int64_t t = c->mlp->adam_t;
    const int32_t ready = c->mlp_ready ? 1 : 0;
    if (std::fwrite(w.data(), sizeof(float), w.size(), f) != w.size() || std::fwrite(&t, 8, 1, f) != 1 ||
        std::fwrite(&ready, 4, 1, f) != 1)
        return FEPIC_E_IO;
    return FEPIC_OK;
}

int mlp_load(fepic_ctx* c, std::FILE* f) {
    int32_t have = 0;
    if (std::fread(&have, 4, 1, f) != 1) return FEPIC_E_IO;
    if (!have) return FEPIC_OK;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    std::vector<float> w(3 * kNP);
    int64_t t = 0;
    int32_t ready = 0;
    if (std::fread(w.data(), sizeof(float), w.size(), f) != w.size() || std::fread(&t, 8, 1, f) != 1 ||
        std::fread(&ready, 4, 1, f) != 1)
        return FEPIC_E_IO;
    HIPCHK_RET(c, hipMemcpy(c->mlp->P, w.data(), sizeof(float) * kNP, hipMemcpyHostToDevice));
    HIPCHK_RET(c, hipMemcpy(c->mlp->m, w.data() + kNP, sizeof(float) * kNP, hipMemcpyHostToDevice));
    HIPCHK_RET(c, hipMemcpy(c->mlp->v, w.data() + 2 * kNP, sizeof(float) * kNP, hipMemcpyHostToDevice));
    c->mlp->adam_t = t;
    c->mlp->have_weights = true;
    c->mlp_ready = ready != 0;
    return FEPIC_OK;
}

// Loss of the current weights on explicit device rows (mean squared error).
static int eval_loss(fepic_ctx* c, const float* X, const float* T, int64_t n, double* loss) {
    MlpState* s = c->mlp;
    if (n <= 0) {
        *loss = 0.0;
        return FEPIC_OK;
    }
    const int blocks = std::min(mlp_grad_blocks(n), kMaxGradBlocks);
    mlp_launch_grad(c->stream, X, T, n, 0, 0, s->P, s->part, s->loss_part, blocks);
    std::vector<double> lp(blocks);
    HIPCHK_RET(c, hipMemcpyAsync(lp.data(), s->loss_part, sizeof(double) * blocks, hipMemcpyDeviceToHost, c->stream));
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    double a = 0.0;
    for (double v : lp) a += v;
    *loss = a / (double)n;
    return FEPIC_OK;
}

static int host_batch(fepic_ctx* c, int64_t n, const float* X, const float* T) {
    MlpState* s = c->mlp;
    if (n > s->h_cap) {
        dfree(c, s->Xh);
        dfree(c, s->Th);
        s->Xh = (float*)dmalloc(c, sizeof(float) * 4 * n);
        s->Th = (float*)dmalloc(c, sizeof(float) * n);
        if (!s->Xh || !s->Th) return fail(c, FEPIC_E_OOM, "device allocation failed");
        s->h_cap = n;
    }
    HIPCHK_RET(c, hipMemcpy(s->Xh, X, sizeof(float) * 4 * n, hipMemcpyHostToDevice));
    if (T) HIPCHK_RET(c, hipMemcpy(s->Th, T, sizeof(float) * n, hipMemcpyHostToDevice));
    return FEPIC_OK;
}

}  // namespace fepic

using namespace fepic;

extern "C" {

int fepic_ws_record(fepic_ctx* c, int on, int64_t max_snapshots) {
    if (!c || on < 0) return FEPIC_E_ARG;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    MlpState* s = c->mlp;
    const int64_t ni = c->mesh.n_int_edges;
    if (on > ni) return fail(c, FEPIC_E_ARG, "row stride above the number of interior edges");
    if (on && max_snapshots > 0 && (max_snapshots != s->cap || on != s->stride)) {
        const int64_t n_rec = ni / on;
        dfree(c, s->Xrec);
        dfree(c, s->Trec);
        s->Xrec = (float*)dmalloc(c, sizeof(float) * 4 * n_rec * max_snapshots);
        s->Trec = (float*)dmalloc(c, sizeof(float) * n_rec * max_snapshots);
        if (!s->Xrec || !s->Trec) {
            s->cap = 0;
            return fail(c, FEPIC_E_OOM, "recording buffer allocation failed");
        }
        s->cap = max_snapshots;
        s->stride = on;
        s->n_rec = n_rec;
        s->count = s->head = s->taken = 0;
    }
    if (on && s->cap == 0) return fail(c, FEPIC_E_ARG, "recording needs max_snapshots > 0");
    c->recording = on != 0;
    return FEPIC_OK;
}

int fepic_ws_num_snapshots(fepic_ctx* c, int64_t* n) {
    if (!c || !n) return FEPIC_E_ARG;
    *n = c->mlp ? c->mlp->count : 0;
    return FEPIC_OK;
}

int fepic_ws_train(fepic_ctx* c, const fepic_train_opts* o, fepic_train_stats* out) {
    if (!c || !o) return FEPIC_E_ARG;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    MlpState* s = c->mlp;
    const int64_t ni = s->n_rec;   // rows per snapshot
    if (s->count < 1 || ni == 0) return fail(c, FEPIC_E_STATE, "no recorded snapshots");
    if (o->epochs < 1 || o->batch < 64 || !(o->lr > 0)) return fail(c, FEPIC_E_ARG, "bad training options");
    const auto t0 = std::chrono::steady_clock::now();
    if (!s->have_weights && (rc = init_weights(c, o->seed))) return rc;
    // the ring's oldest snapshots train, the newest val_fraction validate
    int64_t n_val_snap = (int64_t)std::floor(o->val_fraction * (double)s->count);
    if (s->count > 1) n_val_snap = std::max<int64_t>(std::min(n_val_snap, s->count - 1), o->val_fraction > 0 ? 1 : 0);
    else n_val_snap = 0;
    const int64_t n_tr_snap = s->count - n_val_snap;
    // make the ring contiguous in time order: rotate so the oldest snapshot is first
    if (s->count == s->cap && s->head != 0) {
        std::vector<float> tmpX((size_t)4 * ni * s->cap), tmpT((size_t)ni * s->cap);
        HIPCHK_RET(c, hipStreamSynchronize(c->stream));
        HIPCHK_RET(c, hipMemcpy(tmpX.data(), s->Xrec, sizeof(float) * tmpX.size(), hipMemcpyDeviceToHost));
        HIPCHK_RET(c, hipMemcpy(tmpT.data(), s->Trec, sizeof(float) * tmpT.size(), hipMemcpyDeviceToHost));
        std::rotate(tmpX.begin(), tmpX.begin() + (size_t)4 * ni * s->head, tmpX.end());
        std::rotate(tmpT.begin(), tmpT.begin() + (size_t)ni * s->head, tmpT.end());
        HIPCHK_RET(c, hipMemcpy(s->Xrec, tmpX.data(), sizeof(float) * tmpX.size(), hipMemcpyHostToDevice));
        HIPCHK_RET(c, hipMemcpy(s->Trec, tmpT.data(), sizeof(float) * tmpT.size(), hipMemcpyHostToDevice));
        s->head = 0;
    }
    const int64_t n_tr = n_tr_snap * ni, n_val = n_val_snap * ni;
    const float* Xtr = s->Xrec;
    const float* Ttr = s->Trec;
    const float* Xva = s->Xrec + (size_t)4 * n_tr;
    const float* Tva = s->Trec + (size_t)n_tr;
    const int64_t batch = (o->batch / 64) * 64;
    const int64_t steps_per_epoch = std::max<int64_t>(1, n_tr / batch);
    const int blocks = std::min(mlp_grad_blocks(batch), kMaxGradBlocks);
    const float b1 = (float)(o->beta1 > 0 ? o->beta1 : 0.9), b2 = (float)(o->beta2 > 0 ? o->beta2 : 0.999);
    const float eps = (float)(o->eps > 0 ? o->eps : 1e-8);
    int64_t steps = 0;
    for (int ep = 0; ep < o->epochs; ++ep) {
        for (int64_t k = 0; k < steps_per_epoch; ++k) {
            s->adam_t++;
            const uint64_t seed = o->seed * 0x9E3779B97F4A7C15ull + (uint64_t)s->adam_t * 0xBF58476D1CE4E5B9ull;
            mlp_launch_grad(c->stream, Xtr, Ttr, batch, n_tr, seed, s->P, s->part, s->loss_part, blocks);
            // bias corrections in FP64: 1 - b^t cancels badly in FP32 for b near 1
            const float bc1 = (float)(1.0 - std::pow((double)b1, (double)s->adam_t)),
                        bc2 = (float)(1.0 - std::pow((double)b2, (double)s->adam_t));
            mlp_launch_reduce_adam(c->stream, s->part, blocks, nullptr, s->P, s->m, s->v, 1, (float)o->lr, b1, b2, eps,
                                   bc1, bc2);
            ++steps;
        }
    }
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    HIPCHK_RET(c, hipGetLastError());
    double tl = 0.0, vl = 0.0;
    // training loss on (at most) the first 1M training rows, validation on all held-out rows
    if ((rc = eval_loss(c, Xtr, Ttr, std::min<int64_t>(n_tr, 1 << 20), &tl))) return rc;
    if ((rc = eval_loss(c, Xva, Tva, n_val, &vl))) return rc;
    c->mlp_ready = true;
    if (out) {
        out->train_loss = tl;
        out->val_loss = n_val ? vl : -1.0;
        out->n_train_rows = n_tr;
        out->n_val_rows = n_val;
        out->n_steps = steps;
        out->ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return FEPIC_OK;
}

int fepic_ws_get_weights(fepic_ctx* c, float* w, int64_t cap, int64_t* n) {
    if (!c || !w || !n) return FEPIC_E_ARG;
    if (!c->mlp || !c->mlp->have_weights) return fail(c, FEPIC_E_STATE, "no weights");
    if (cap < kNP) return fail(c, FEPIC_E_ARG, "buffer too small");
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    HIPCHK_RET(c, hipMemcpy(w, c->mlp->P, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    *n = kNP;
    return FEPIC_OK;
}

int fepic_ws_set_weights(fepic_ctx* c, const float* w, int64_t n) {
    if (!c || !w || n != kNP) return FEPIC_E_ARG;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    HIPCHK_RET(c, hipMemcpy(c->mlp->P, w, sizeof(float) * kNP, hipMemcpyHostToDevice));
    HIPCHK_RET(c, hipMemset(c->mlp->m, 0, sizeof(float) * kNP));
    HIPCHK_RET(c, hipMemset(c->mlp->v, 0, sizeof(float) * kNP));
    c->mlp->adam_t = 0;
    c->mlp->have_weights = true;
    c->mlp_ready = true;
    return FEPIC_OK;
}

int fepic_set_warm_start(fepic_ctx* c, int mode) {
    if (!c || mode < FEPIC_WS_PREV || mode > FEPIC_WS_MLP_DIRECT) return FEPIC_E_ARG;
    if ((mode == FEPIC_WS_MLP || mode == FEPIC_WS_MLP_DIRECT) && c->opt.deterministic)
        return fail(c, FEPIC_E_STATE, "the deterministic mode does not take the learned start");
    c->opt.warm_start = mode;
    return FEPIC_OK;
}

int fepic_mlp_forward(fepic_ctx* c, int64_t n, const float* X, float* y) {
    if (!c || n < 0 || (n > 0 && (!X || !y))) return FEPIC_E_ARG;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    if (!c->mlp->have_weights) return fail(c, FEPIC_E_STATE, "no weights");
    if (n == 0) return FEPIC_OK;
    if ((rc = host_batch(c, n, X, nullptr))) return rc;
    float* dy = (float*)dmalloc(c, sizeof(float) * n);
    if (!dy) return fail(c, FEPIC_E_OOM, "device allocation failed");
    mlp_launch_forward(c->stream, n, c->mlp->Xh, c->mlp->P, dy);
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    HIPCHK_RET(c, hipMemcpy(y, dy, sizeof(float) * n, hipMemcpyDeviceToHost));
    dfree(c, dy);
    return FEPIC_OK;
}

int fepic_mlp_adam_step(fepic_ctx* c, const float* grad, double lr, double beta1, double beta2, double eps) {
    if (!c || !grad || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return c ? fail(c, FEPIC_E_ARG, "fepic_mlp_adam_step: bad arguments") : FEPIC_E_ARG;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    MlpState* s = c->mlp;
    if (!s->have_weights) return fail(c, FEPIC_E_STATE, "no weights");
    // the gradient as the single "partial sum" of the reduce-and-update kernel training uses
    HIPCHK_RET(c, hipMemcpyAsync(s->part, grad, sizeof(float) * kNP, hipMemcpyHostToDevice, c->stream));
    s->adam_t++;
    const float b1 = (float)beta1, b2 = (float)beta2;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)s->adam_t)),
                bc2 = (float)(1.0 - std::pow((double)b2, (double)s->adam_t));
    mlp_launch_reduce_adam(c->stream, s->part, 1, nullptr, s->P, s->m, s->v, 1, (float)lr, b1, b2, (float)eps, bc1,
                           bc2);
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    return FEPIC_OK;
}

int fepic_mlp_grad_noalloc(fepic_ctx* c, int64_t n, const float* X, const float* t, float* grad, double* loss) {
    if (!c) return FEPIC_E_ARG;
    if (c->host_only) return fail(c, FEPIC_E_NO_DEVICE, "host-only context");
    if (n <= 0 || !X || !t || !grad || !loss) return fail(c, FEPIC_E_ARG, "fepic_mlp_grad_noalloc: bad arguments");
    if (n > FEPIC_MLP_NOALLOC_MAX_ROWS)
        return fail(c, FEPIC_E_ARG,
                    "fepic_mlp_grad_noalloc: n = " + std::to_string(n) + " rows exceeds FEPIC_MLP_NOALLOC_MAX_ROWS = " +
                        std::to_string(FEPIC_MLP_NOALLOC_MAX_ROWS));
    if (!c->mlp || !c->mlp->have_weights)
        return fail(c, FEPIC_E_STATE, "fepic_mlp_grad_noalloc: no network weights (set or train them first)");
    const int dev = c->opt.device;
    void* base = (dev >= 0 && dev < kMaxScratchDevices) ? g_scratch_addr[dev] : nullptr;
    if (!base) {
        const hipError_t e = (dev >= 0 && dev < kMaxScratchDevices) ? g_scratch_err[dev] : hipErrorInvalidDevice;
        return hip_fail(c, e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
    }
    const int blocks = mlp_grad_blocks(n);
    if (blocks > kNoAllocBlocks) return fail(c, FEPIC_E_ARG, "fepic_mlp_grad_noalloc: grid exceeds the scratch");
    float* part = (float*)base;
    double* loss_part = (double*)((unsigned char*)base + kScratchGradBytes);
    mlp_launch_grad(c->stream, X, t, n, 0, 0, c->mlp->P, part, loss_part, blocks);
    mlp_launch_reduce_adam(c->stream, part, blocks, grad, nullptr, nullptr, nullptr, 0, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f);
    mlp_launch_loss_sum(c->stream, loss_part, blocks, 1.0 / (double)n, loss);
    HIPCHK_RET(c, hipGetLastError());
    return FEPIC_OK;
}

int fepic_mlp_grad(fepic_ctx* c, int64_t n, const float* X, const float* t, float* grad, double* loss) {
    if (!c || n <= 0 || !X || !t || !grad) return FEPIC_E_ARG;
    int rc = ensure_mlp(c);
    if (rc) return rc;
    if (!c->mlp->have_weights) return fail(c, FEPIC_E_STATE, "no weights");
    if ((rc = host_batch(c, n, X, t))) return rc;
    MlpState* s = c->mlp;
    const int blocks = std::min(mlp_grad_blocks(n), kMaxGradBlocks);
    mlp_launch_grad(c->stream, s->Xh, s->Th, n, 0, 0, s->P, s->part, s->loss_part, blocks);
    mlp_launch_reduce_adam(c->stream, s->part, blocks, s->grad, s->P, s->m, s->v, 0, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f);
    std::vector<double> lp(blocks);
    HIPCHK_RET(c, hipStreamSynchronize(c->stream));
    HIPCHK_RET(c, hipMemcpy(grad, s->grad, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    HIPCHK_RET(c, hipMemcpy(lp.data(), s->loss_part, sizeof(double) * blocks, hipMemcpyDeviceToHost));
    if (loss) {
        double a = 0.0;
        for (double v : lp) a += v;
        *loss = a / (double)n;
    }
    return FEPIC_OK;
}

}  // extern "C"
