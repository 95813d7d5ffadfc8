// libfepic C ABI: context, device state, the step, read-out (see include/fepic.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ctx.h"

using namespace fepic;

namespace fepic {

const char* kFamilies[] = {"push", "stage", "sort", "rhs", "cg_iter", "faraday", "mlp_fwd"};

int hip_fail(fepic_ctx* c, hipError_t e, const char* what) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return FEPIC_E_HIP;
}

int fail(fepic_ctx* c, int code, const std::string& msg) {
    c->err = msg;
    return code;
}

void* dmalloc(fepic_ctx* c, size_t bytes) {
    if (bytes == 0) bytes = 8;
    void* p = nullptr;
    if (c->ualloc) {
        p = c->ualloc(bytes, c->uarg);
        if (!p) return nullptr;
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        return nullptr;
    }
    c->allocs.push_back(p);
    return p;
}

// Returns one device allocation to whichever allocator made it.  A caller's allocator may
// hand the memory to other work at once, so the context's stream is drained first.
static void release(fepic_ctx* c, void* p) {
    if (c->ufree) {
        (void)hipStreamSynchronize(c->stream);
        c->ufree(p, c->uarg);
    } else {
        (void)hipFree(p);
    }
}

void dfree(fepic_ctx* c, void* p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    release(c, p);
}

hipEvent_t* timer_pair(fepic_ctx* c, int fam, int64_t n_launches) {
    if (fam < 0 || !c->timers[fam].on) return nullptr;
    KernelTimer& k = c->timers[fam];
    k.launches += n_launches;
    if (k.used + 2 > (int64_t)k.ev.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            k.ev.push_back(e);
        }
    }
    hipEvent_t* p = &k.ev[k.used];
    k.used += 2;
    return p;
}

}  // namespace fepic

#define HIPCHK(c, expr)                                            \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return fepic::hip_fail(c, e_, #expr); \
    } while (0)

#define NEED_DEV(c)                                                                                   \
    do {                                                                                              \
        if (!(c)) return FEPIC_E_ARG;                                                                 \
        if ((c)->host_only) return fepic::fail(c, FEPIC_E_NO_DEVICE, "host-only context");           \
        if (!(c)->have_mesh) return fepic::fail(c, FEPIC_E_STATE, "no mesh uploaded");               \
    } while (0)

namespace {

template <typename T>
T* dalloc(fepic_ctx* c, int64_t n) {
    return (T*)dmalloc(c, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

template <typename T>
int upload(fepic_ctx* c, T** dst, const std::vector<T>& src) {
    *dst = dalloc<T>(c, (int64_t)src.size());
    if (!*dst) return fail(c, FEPIC_E_OOM, "device allocation failed");
    if (!src.empty()) HIPCHK(c, hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return FEPIC_OK;
}

// Array a (0..7) of the species' current state.
void* cur_arr(Species& s, int a) { return s.buf[a == 7 ? s.idcur : s.cur][a]; }

template <typename T>
PArrays<T> parr(Species& s, int which) {
    PArrays<T> p;
    p.tet = (int32_t*)s.buf[which][0];
    p.l1 = (T*)s.buf[which][1];
    p.l2 = (T*)s.buf[which][2];
    p.l3 = (T*)s.buf[which][3];
    p.u0 = (T*)s.buf[which][4];
    p.u1 = (T*)s.buf[which][5];
    p.u2 = (T*)s.buf[which][6];
    p.id = (int64_t*)s.buf[which == s.cur ? s.idcur : 1 - s.idcur][7];
    return p;
}

// The arrays of parr() from slot `off` on.
template <typename T>
PArrays<T> parr_off(Species& s, int which, int64_t off) {
    PArrays<T> p = parr<T>(s, which);
    p.tet += off;
    p.l1 += off;
    p.l2 += off;
    p.l3 += off;
    p.u0 += off;
    p.u1 += off;
    p.u2 += off;
    p.id += off;
    return p;
}

size_t field_size(const fepic_ctx* c) { return c->opt.precision == FEPIC_ALL_FP64 ? 8 : 4; }

size_t array_bytes(const fepic_ctx* c, int a, int64_t n) {
    if (a == 0) return 4 * (size_t)n;
    if (a == 7) return 8 * (size_t)n;
    return field_size(c) * (size_t)n;
}

// Makes an existing Adams-Bashforth history match the species' particle capacity, keeping
// the history of slots [0, n) (one 2-D copy per array: the component stride changes).
int ab_fit(fepic_ctx* c, Species& s) {
    if (!s.d_abh[0] || s.abh_cap == s.cap) return FEPIC_OK;
    double* nh[2] = {dalloc<double>(c, s.cap * kAbStride), dalloc<double>(c, s.cap * kAbStride)};
    int32_t* nm[2] = {dalloc<int32_t>(c, s.cap), dalloc<int32_t>(c, s.cap)};
    if (!nh[0] || !nh[1] || !nm[0] || !nm[1]) return fail(c, FEPIC_E_OOM, "history allocation failed");
    if (!s.ab_reset && s.n > 0) {
        HIPCHK(c, hipMemcpy2DAsync(nh[0], 8 * s.cap, s.d_abh[s.abh_cur], 8 * s.abh_cap, 8 * s.n, kAbStride,
                                   hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(nm[0], s.d_abm[s.abm_cur], 4 * s.n, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int w = 0; w < 2; ++w) {
        dfree(c, s.d_abh[w]);
        dfree(c, s.d_abm[w]);
        s.d_abh[w] = nh[w];
        s.d_abm[w] = nm[w];
    }
    s.abh_cur = s.abm_cur = 0;
    s.abh_cap = s.cap;
    return FEPIC_OK;
}

int ensure_capacity(fepic_ctx* c, Species& s, int64_t need) {
    if (need <= s.cap) return FEPIC_OK;
    const int64_t cap = std::max<int64_t>({need, s.cap + s.cap / 4, 1024});
    void* nb[2][8] = {};
    for (int w = 0; w < 2; ++w)
        for (int a = 0; a < 8; ++a) {
            nb[w][a] = dmalloc(c, array_bytes(c, a, cap));
            if (!nb[w][a]) return fail(c, FEPIC_E_OOM, "particle buffer allocation failed");
        }
    for (int a = 0; a < 8; ++a)
        if (s.n > 0) HIPCHK(c, hipMemcpyAsync(nb[0][a], cur_arr(s, a), array_bytes(c, a, s.n), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int w = 0; w < 2; ++w)
        for (int a = 0; a < 8; ++a) {
            dfree(c, s.buf[w][a]);
            s.buf[w][a] = nb[w][a];
        }
    s.cur = 0;
    s.idcur = 0;
    s.cap = cap;
    return ab_fit(c, s);
}

bool ab_carry(const fepic_ctx* c, const Species& s) {
    return c->opt.pusher == FEPIC_PUSHER_AB && s.d_abh[0] && !s.ab_reset;
}

// Slots appended since the last Adams-Bashforth step have no history yet (AbMeta -1).
void ab_mark_new(fepic_ctx* c, Species& s) {
    if (ab_carry(c, s) && s.ab_fill_from < s.n)
        launch_fill_i32(c->stream, s.d_abm[s.abm_cur] + s.ab_fill_from, s.n - s.ab_fill_from, -1);
    s.ab_fill_from = INT64_MAX;
}

template <typename T>
void sort_species(fepic_ctx* c, Species& s) {
    hipEvent_t* ev = timer_pair(c, FAM_SORT);
    if (ev) (void)hipEventRecord(ev[0], c->stream);
    AbHistIo ab;
    const bool carry = ab_carry(c, s);
    if (carry) {   // the Adams-Bashforth history moves with the particles
        ab_mark_new(c, s);
        ab.hin = s.d_abh[s.abh_cur];
        ab.hout = s.d_abh[1 - s.abh_cur];
        ab.stride = s.abh_cap;
        ab.min = s.d_abm[s.abm_cur];
        ab.mout = s.d_abm[1 - s.abm_cur];
    }
    launch_sort<T>(c->stream, parr<T>(s, s.cur), parr<T>(s, 1 - s.cur), s.n, c->mesh.n_tets, c->d_count, c->d_offset,
                   c->d_bsums, s.d_nlive, ab);
    if (ev) (void)hipEventRecord(ev[1], c->stream);
    s.cur = 1 - s.cur;
    s.idcur = 1 - s.idcur;
    if (carry) {
        s.abh_cur = 1 - s.abh_cur;
        s.abm_cur = 1 - s.abm_cur;
    } else {
        s.ab_reset = true;
    }
    s.sorted_pending = true;
    s.moved = 0;
    s.added = false;
}

// Species that left the sorted order by at least this share of their particles (face
// crossings and losses since the last re-binning) are re-binned under FEPIC_SORT_AUTO.
constexpr int64_t kResortDivisor = 64;

// The sorts of a step: every species, or under FEPIC_SORT_AUTO those that need it.
void sort_all(fepic_ctx* c) {
    for (auto& s : c->species) {
        if (c->opt.sort_period == FEPIC_SORT_AUTO && !s.added && s.moved * kResortDivisor < s.n) continue;
        if (c->opt.precision == FEPIC_ALL_FP64) sort_species<double>(c, s);
        else sort_species<float>(c, s);
    }
}

// Reads the live counts written by the last sorts (stream must be synchronized).
void settle_counts(fepic_ctx* c) {
    for (auto& s : c->species)
        if (s.sorted_pending) {
            s.n = *s.h_nlive;
            s.sorted_pending = false;
        }
}

int sync_counts(fepic_ctx* c) {
    bool any = false;
    for (auto& s : c->species)
        if (s.sorted_pending) {
            HIPCHK(c, hipMemcpyAsync(s.h_nlive, s.d_nlive, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            any = true;
        }
    if (!any) return FEPIC_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    settle_counts(c);
    return FEPIC_OK;
}

// Deterministic mode: the accumulators (2 words per edge or node, cleared), and the unit of
// the fixed-point sums: the power of two at or above the largest |q w| (a piece's current
// on an edge and a particle's charge on a node are at most |q w|).
unsigned long long* fix_buffer(fepic_ctx* c) {
    if (!c->opt.deterministic) return nullptr;
    if (!c->d_fix) {
        const int64_t n = 2 * std::max(c->mesh.n_edges, c->mesh.n_nodes);
        c->d_fix = dalloc<unsigned long long>(c, n);
        if (!c->d_fix) return nullptr;
        launch_fill(c->stream, reinterpret_cast<double*>(c->d_fix), n, 0.0);   // all-zero bits
    }
    return c->d_fix;
}

double fix_scale(const fepic_ctx* c) {
    double q = 0.0;
    for (const auto& s : c->species) q = std::max(q, std::fabs(s.q * s.w));
    if (!(q > 0.0)) return 1.0;
    return std::ldexp(1.0, std::ilogb(q) + 1);
}

template <typename T>
void compute_rho_T(fepic_ctx* c, double* rho) {
    unsigned long long* fix = fix_buffer(c);
    const double scale = fix_scale(c);
    if (!fix) launch_fill(c->stream, rho, c->mesh.n_nodes, 0.0);
    for (auto& s : c->species)
        launch_rho<T>(c->stream, parr<T>(s, s.cur), s.n, c->d_tets, s.q * s.w, rho, fix, 1.0 / scale);
    if (fix) launch_fix_out(c->stream, fix, c->mesh.n_nodes, scale, rho);
}

void compute_rho(fepic_ctx* c, double* rho) {
    if (c->opt.precision == FEPIC_ALL_FP64) compute_rho_T<double>(c, rho);
    else compute_rho_T<float>(c, rho);
}

void ev_mark(fepic_ctx* c, int i) {
    if (c->opt.timing) (void)hipEventRecord(c->phase_ev[i], c->stream);
}

// Crossing queue of the particle step: room for one slot per particle of the largest
// species (rounded up to whole 256-particle workgroups), carved into the CrossQueue arrays.
constexpr int64_t kQueueSlotBytes = 5 * 8 + 3 * 8 + 3 * 4;   // l0..l3, frac; dx (as FP64 at most); ids

int ensure_queue(fepic_ctx* c) {
    int64_t need = 0;
    for (const auto& s : c->species) need = std::max(need, (s.n + 255) / 256 * 256);
    if (need <= c->cq_cap) return FEPIC_OK;
    const int64_t cap = std::max<int64_t>(need, (c->cq_cap + c->cq_cap / 4 + 255) / 256 * 256);
    unsigned char* p = (unsigned char*)dmalloc(c, (size_t)cap * kQueueSlotBytes + (size_t)(cap / 256) * 4 + 256);
    if (!p) return fail(c, FEPIC_E_OOM, "crossing queue allocation failed");
    dfree(c, c->d_cq);
    c->d_cq = p;
    c->cq_cap = cap;
    return FEPIC_OK;
}

template <typename T>
CrossQueue<T> cqueue(fepic_ctx* c) {
    CrossQueue<T> q;
    const int64_t n = c->cq_cap;
    double* d = (double*)c->d_cq;
    q.l0 = d;
    q.l1 = d + n;
    q.l2 = d + 2 * n;
    q.l3 = d + 3 * n;
    q.frac = d + 4 * n;
    T* t = (T*)(d + 5 * n);
    q.dx0 = t;
    q.dx1 = t + n;
    q.dx2 = t + 2 * n;
    int32_t* i = (int32_t*)(d + 8 * n);
    q.idx = i;
    q.tet = i + n;
    q.entry = i + 2 * n;
    q.wg_count = i + 3 * n;
    return q;
}

// The injectors' particles of this step, drawn on the device and appended after the sort
// (the push moves them with the rest, their charge joins rho^n when diagnostics run);
// inject_undo drops them again when the step is not committed.
template <typename T>
int inject_phase(fepic_ctx* c) {
    bool any = false;
    for (const auto& s : c->species) any = any || (s.inj_on && s.inj.per_step > 0);
    if (!any) return FEPIC_OK;
    int rc = sync_counts(c);
    if (rc != FEPIC_OK) return rc;
    for (auto& s : c->species) {
        s.inj_undo_n = -1;
        if (!s.inj_on || s.inj.per_step <= 0) continue;
        const int64_t m = s.inj.per_step;
        if (s.n + m >= ((int64_t)1 << 31)) return fail(c, FEPIC_E_ARG, "too many particles for one species");
        if ((rc = ensure_capacity(c, s, s.n + m)) != FEPIC_OK) return rc;
        if (c->inj_cap < m) {
            dfree(c, c->d_inj);
            c->d_inj = dalloc<double>(c, 6 * m);
            if (!c->d_inj) return fail(c, FEPIC_E_OOM, "injection staging allocation failed");
            c->inj_cap = m;
        }
        InjectorSpec sp = s.inj;
        sp.relativistic_u = c->opt.pusher == FEPIC_PUSHER_AB ? 0 : 1;
        launch_inject_disk(c->stream, sp, s.inj_k, c->d_inj, c->d_inj + 3 * m);
        const double* g = c->d_grid;
        launch_locate<T>(c->stream, m, c->d_inj, c->d_inj + 3 * m, nullptr, s.next_id, parr<T>(s, s.cur), s.n,
                         c->d_grad64, c->d_r0, c->d_cell_start, c->d_cell_tets, g, g + 3, c->d_grid_n, c->d_cnt);
        if (c->opt.diagnostics && c->rho_valid)
            launch_rho<T>(c->stream, parr_off<T>(s, s.cur, s.n), m, c->d_tets, s.q * s.w, c->d_rho);
        s.inj_undo_n = s.n;
        s.ab_fill_from = std::min(s.ab_fill_from, s.n);
        s.next_id += m;
        s.n += m;
        s.added = true;
    }
    return FEPIC_OK;
}

void inject_undo(fepic_ctx* c) {
    for (auto& s : c->species)
        if (s.inj_undo_n >= 0) {
            s.n = s.inj_undo_n;
            s.next_id -= s.inj.per_step;
            s.inj_undo_n = -1;
            c->rho_valid = false;
        }
}

int64_t inject_commit(fepic_ctx* c) {
    int64_t n = 0;
    for (auto& s : c->species)
        if (s.inj_undo_n >= 0) {
            n += s.inj.per_step;
            s.inj_k++;
            s.inj_undo_n = -1;
        }
    return n;
}

// Particle half: optional sort, staging, gather/push/track/deposit into d_dgn and the
// alternate particle buffers.  Nothing is committed here.
template <typename T>
void particle_phase_T(fepic_ctx* c, double dt, bool do_sort) {
    ev_mark(c, 0);
    if (do_sort) sort_all(c);
    {
        const int rc = inject_phase<T>(c);
        if (rc != FEPIC_OK) {
            c->deferred_err = rc;
            return;
        }
    }
    ev_mark(c, 1);
    {
        hipEvent_t* ev = timer_pair(c, FAM_STAGE);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        launch_stage<T>(c->stream, c->mesh.n_tets, (TetBlock<T>*)c->d_blk, c->d_e, c->d_b, c->d_grad64,
                        c->d_tet_edges, c->d_tet_faces);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
    }
    ev_mark(c, 2);
    launch_fill(c->stream, c->d_dgn, c->mesh.n_edges, 0.0);
    if (ensure_queue(c) != FEPIC_OK) {
        c->deferred_err = FEPIC_E_OOM;
        return;
    }
    unsigned long long* fix = fix_buffer(c);
    if (c->opt.deterministic && !fix) {
        c->deferred_err = FEPIC_E_OOM;
        return;
    }
    const double scale = fix_scale(c);
    for (auto& s : c->species) {
        if (s.n == 0) continue;
        PushParams pp;
        pp.dt = dt;
        pp.qm_half_dt = s.q * dt / (2.0 * s.m);
        pp.qw = s.q * s.w;
        pp.cap = c->opt.crossing_cap;
        pp.fix = fix;
        pp.fix_inv = 1.0 / scale;
        hipEvent_t* ev = timer_pair(c, FAM_PUSH);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        launch_push<T>(c->stream, parr<T>(s, s.cur), parr<T>(s, 1 - s.cur), s.n, (const TetBlock<T>*)c->d_blk,
                       c->d_dgn, pp, c->d_cnt_slots, s.sorted_pending ? s.d_nlive : nullptr, cqueue<T>(c),
                       c->cross_share, s.own_share, c->opt.walk);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
        s.n_pushed = s.n;
        launch_cnt_crossings(c->stream, c->d_cnt_slots, s.d_xcum);
        const hipError_t xe = hipMemcpyAsync(s.h_xcum, s.d_xcum, 2 * sizeof(unsigned long long),
                                             hipMemcpyDeviceToHost, c->stream);
        if (xe != hipSuccess) {
            c->deferred_err = hip_fail(c, xe, "hipMemcpyAsync(crossing count)");
            return;
        }
    }
    if (fix) launch_fix_out(c->stream, fix, c->mesh.n_edges, scale, c->d_dgn);
    launch_cnt_finish(c->stream, c->d_cnt_slots, c->d_cnt);
    ev_mark(c, 3);
}

void ab_tables(AbParams& ap);

// Sizes the species' Adams-Bashforth history and marks the slots whose history is missing or
// stale (dt changed: the coefficients assume equally spaced levels) to restart at order 1.
int ab_prepare(fepic_ctx* c, Species& s, double dt) {
    if (!s.d_abh[0]) {
        for (int w = 0; w < 2; ++w) {
            s.d_abh[w] = dalloc<double>(c, s.cap * kAbStride);
            s.d_abm[w] = dalloc<int32_t>(c, s.cap);
            if (!s.d_abh[w] || !s.d_abm[w]) return fail(c, FEPIC_E_OOM, "history allocation failed");
        }
        s.abh_cap = s.cap;
        s.abh_cur = s.abm_cur = 0;
        s.ab_reset = true;
    }
    int rc = ab_fit(c, s);
    if (rc != FEPIC_OK) return rc;
    if (s.ab_reset || s.ab_dt != dt) {
        launch_fill_i32(c->stream, s.d_abm[s.abm_cur], s.n, -1);
        s.ab_reset = false;
        s.ab_fill_from = INT64_MAX;
        s.ab_dt = dt;
    } else {
        ab_mark_new(c, s);
    }
    return FEPIC_OK;
}

// The Adams-Bashforth particle phase (all-FP64): the sort carries the histories; one
// k_push_ab per species into d_dgn, the alternate particle buffers and the alternate AbMeta.
// Nothing is committed here.
void particle_phase_ab(fepic_ctx* c, double dt, bool do_sort) {
    for (auto& s : c->species) {
        const int rc = ab_prepare(c, s, dt);
        if (rc != FEPIC_OK) {
            c->deferred_err = rc;
            return;
        }
    }
    ev_mark(c, 0);
    if (do_sort) sort_all(c);
    {
        int rc = inject_phase<double>(c);
        if (rc == FEPIC_OK)
            for (auto& s : c->species) {   // injected slots start at order 1
                rc = ab_fit(c, s);
                if (rc != FEPIC_OK) break;
                ab_mark_new(c, s);
            }
        if (rc != FEPIC_OK) {
            c->deferred_err = rc;
            return;
        }
    }
    ev_mark(c, 1);
    {
        hipEvent_t* ev = timer_pair(c, FAM_STAGE);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        launch_stage<double>(c->stream, c->mesh.n_tets, (TetBlock<double>*)c->d_blk, c->d_e, c->d_b, c->d_grad64,
                             c->d_tet_edges, c->d_tet_faces);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
    }
    ev_mark(c, 2);
    launch_fill(c->stream, c->d_dgn, c->mesh.n_edges, 0.0);
    AbParams ap;
    ab_tables(ap);
    ap.dt = dt;
    ap.k = c->opt.ab_order;
    ap.cap = c->opt.crossing_cap;
    unsigned long long* fix = fix_buffer(c);
    if (c->opt.deterministic && !fix) {
        c->deferred_err = FEPIC_E_OOM;
        return;
    }
    const double scale = fix_scale(c);
    ap.fix = fix;
    ap.fix_inv = 1.0 / scale;
    for (auto& s : c->species) {
        if (s.n == 0) continue;
        ap.qm = s.q / s.m;
        ap.qw = s.q * s.w;
        hipEvent_t* ev = timer_pair(c, FAM_PUSH);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        launch_push_ab(c->stream, parr<double>(s, s.cur), parr<double>(s, 1 - s.cur), s.n,
                       (const TetBlock<double>*)c->d_blk, c->d_r0, s.d_abh[s.abh_cur], s.abh_cap, s.d_abm[s.abm_cur],
                       s.d_abm[1 - s.abm_cur], c->d_dgn, ap, c->d_cnt_slots, s.sorted_pending ? s.d_nlive : nullptr);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
        s.n_pushed = s.n;
        launch_cnt_crossings(c->stream, c->d_cnt_slots, s.d_xcum);
        const hipError_t xe = hipMemcpyAsync(s.h_xcum, s.d_xcum, 2 * sizeof(unsigned long long),
                                             hipMemcpyDeviceToHost, c->stream);
        if (xe != hipSuccess) {
            c->deferred_err = hip_fail(c, xe, "hipMemcpyAsync(crossing count)");
            return;
        }
    }
    if (fix) launch_fix_out(c->stream, fix, c->mesh.n_edges, scale, c->d_dgn);
    launch_cnt_finish(c->stream, c->d_cnt_slots, c->d_cnt);
    ev_mark(c, 3);
}

void particle_phase(fepic_ctx* c, double dt, bool do_sort) {
    if (c->opt.pusher == FEPIC_PUSHER_AB) particle_phase_ab(c, dt, do_sort);
    else if (c->opt.precision == FEPIC_ALL_FP64) particle_phase_T<double>(c, dt, do_sort);
    else particle_phase_T<float>(c, dt, do_sort);
}

// Admittance of free space, 1 / (mu0 c): the first-order absorbing condition's damping
// matrix is this times the boundary matrix K.
constexpr double kY0 = 1.0 / (kMu0 * kC);

void ensure_operator(fepic_ctx* c, double dt, double beta, double gamma = 0.5) {
    const double cA = beta * dt * dt, cK = c->abc_on ? gamma * dt * kY0 : 0.0;
    c->aux.n_far = c->opt.aux_far_levels >= 0 ? std::min(c->opt.aux_far_levels, kAuxFarLevels)
                                              : aux_far_auto(cA * c->s_over_m, c->aux.n_aux);
    if (c->A_scale == cA && c->A_scale_K == cK && c->A_valid) return;
    launch_scale_A(c->stream, c->mesh.mat, c->d_sp, c->d_col, c->d_M, c->d_S, c->d_A, c->d_dinv, c->d_bedge, cA,
                   c->abc_on ? c->d_K : nullptr, cK);
    launch_aux_scale(c->stream, c->aux, c->d_sp, c->d_col, c->d_A);
    c->A_scale = cA;
    c->A_scale_K = cK;
    c->A_valid = true;
    c->A32_valid = false;
}

// The FP32 state of the mixed-precision solve: allocated on first use, the operator's
// copies refreshed whenever A changed.
int ensure_operator_f32(fepic_ctx* c) {
    const int64_t ne = c->mesh.n_edges, nnz = c->mesh.mat.slice_ptr.back(), na = c->aux.n_aux;
    if (!c->d_A32) {
        AuxSpace& g = c->aux;
        c->d_A32 = dalloc<float>(c, nnz);
        c->d_dinv32 = dalloc<float>(c, ne);
        c->d_x32 = dalloc<float>(c, ne);
        c->d_rq32 = dalloc<float>(c, 2 * ne);
        for (float2*& p : c->d_zp32) p = dalloc<float2>(c, ne);
        g.scale_f = dalloc<float4>(c, na);
        g.scale8_f = dalloc<float4>(c, (na + 7) / 8);
        g.scale64_f = dalloc<float4>(c, (na + 63) / 64);
        g.Y_f = dalloc<float4>(c, na + 1);
        bool ok = c->d_A32 && c->d_dinv32 && c->d_x32 && c->d_rq32 && c->d_zp32[0] && c->d_zp32[1] && g.scale_f &&
                  g.scale8_f && g.scale64_f && g.Y_f;
        for (int L = 0; L < kAuxFarLevels; ++L) {
            g.far_scale_f[L] = dalloc<float4>(c, aux_far_count(na, L));
            ok = ok && g.far_scale_f[L];
        }
        if (!ok) return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemsetAsync(g.Y_f, 0, sizeof(float4) * (na + 1), c->stream));   // entry n_aux stays zero
        HIPCHK(c, hipMemsetAsync(c->d_rq32, 0, sizeof(float) * 2 * ne, c->stream));
        for (float2* p : c->d_zp32) HIPCHK(c, hipMemsetAsync(p, 0, sizeof(float2) * ne, c->stream));
    }
    if (!c->A32_valid) {
        launch_operator_f32(c->stream, nnz, c->d_A, c->d_A32, ne, c->d_dinv, c->d_dinv32, c->aux);
        c->A32_valid = true;
    }
    return FEPIC_OK;
}

// SELL-64 layout of variable-length rows: slice s of 64 rows has the width of its longest
// row; entry k of row r sits at sp[s] + 64 k + (r mod 64); shorter rows are padded with
// `pad` (column) and zero values.
template <typename V>
void sell_pack(const std::vector<int64_t>& row_ptr, const std::vector<int32_t>& cols, const std::vector<V>& vals,
               bool pad_self, int32_t pad, std::vector<int64_t>& sp, std::vector<int32_t>& out_col,
               std::vector<V>& out_val) {
    const int64_t n = (int64_t)row_ptr.size() - 1, ns = (n + kSell - 1) / kSell;
    sp.assign(ns + 1, 0);
    for (int64_t sl = 0; sl < ns; ++sl) {
        int64_t w = 0;
        for (int64_t r = sl * kSell; r < std::min(n, (sl + 1) * kSell); ++r) w = std::max(w, row_ptr[r + 1] - row_ptr[r]);
        sp[sl + 1] = sp[sl] + w * kSell;
    }
    out_col.assign(sp[ns], pad);
    out_val.assign(sp[ns], V(0));
    for (int64_t sl = 0; sl < ns; ++sl)
        for (int64_t l = 0; l < kSell; ++l) {
            const int64_t r = sl * kSell + l;
            const int64_t w = (sp[sl + 1] - sp[sl]) / kSell;
            for (int64_t k = 0; k < w; ++k) {
                const int64_t at = sp[sl] + k * kSell + l;
                if (r < n && row_ptr[r] + k < row_ptr[r + 1]) {
                    out_col[at] = cols[row_ptr[r] + k];
                    out_val[at] = vals[row_ptr[r] + k];
                } else if (pad_self) {
                    out_col[at] = (int32_t)std::min<int64_t>(r, n - 1);
                }
            }
        }
}

// The operators of the mixed (b, e) updates, built once on the host: the Whitney-2 mass
// Mf = [*mu0^-1] over faces, element by element from the field's vertex values (the
// field of face (i, j, l) is 2 grad l_j x grad l_l at vertex i, and so on, zero at the
// opposite vertex; int lambda_v lambda_w = V (1 + delta_vw) / 20), and each edge's list of
// incident faces with the sign of C (face (i, j, k): +(i, j), +(j, k), -(i, k)).
int ensure_mfem(fepic_ctx* c) {
    if (c->mfem_ready) return FEPIC_OK;
    const HostMesh& m = c->mesh;
    const int64_t nt = m.n_tets, nf = m.n_faces, ne = m.n_edges;
    constexpr int kLFv[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    std::vector<int8_t> cnt(nf, 0);
    std::vector<int32_t> cc(7 * nf, -1);
    std::vector<double> cv(7 * nf, 0.0);
    auto add = [&](int64_t f, int32_t g, double v) {
        for (int k = 0; k < cnt[f]; ++k)
            if (cc[7 * f + k] == g) {
                cv[7 * f + k] += v;
                return;
            }
        cc[7 * f + cnt[f]] = g;
        cv[7 * f + cnt[f]] = v;
        ++cnt[f];
    };
    for (int64_t t = 0; t < nt; ++t) {
        double g[4][3];
        for (int k = 1; k < 4; ++k)
            for (int d = 0; d < 3; ++d) g[k][d] = m.grad[9 * t + 3 * (k - 1) + d];
        for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        double w[4][4][3] = {};   // w[face][vertex]
        auto cr = [](const double* a, const double* b, double* o) {
            o[0] = 2.0 * (a[1] * b[2] - a[2] * b[1]);
            o[1] = 2.0 * (a[2] * b[0] - a[0] * b[2]);
            o[2] = 2.0 * (a[0] * b[1] - a[1] * b[0]);
        };
        for (int k = 0; k < 4; ++k) {
            const int i = kLFv[k][0], j = kLFv[k][1], l = kLFv[k][2];
            cr(g[j], g[l], w[k][i]);
            cr(g[l], g[i], w[k][j]);
            cr(g[i], g[j], w[k][l]);
        }
        const double f0 = m.vol[t] / (20.0 * kMu0);
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l) {
                double sv = 0.0, sk[3] = {0, 0, 0}, sl[3] = {0, 0, 0};
                for (int v = 0; v < 4; ++v)
                    for (int d = 0; d < 3; ++d) {
                        sv += w[k][v][d] * w[l][v][d];
                        sk[d] += w[k][v][d];
                        sl[d] += w[l][v][d];
                    }
                add(m.tet_faces[4 * t + k], m.tet_faces[4 * t + l], f0 * (sv + sk[0] * sl[0] + sk[1] * sl[1] + sk[2] * sl[2]));
            }
    }
    std::vector<int64_t> rp(nf + 1, 0);
    for (int64_t f = 0; f < nf; ++f) rp[f + 1] = rp[f] + cnt[f];
    std::vector<int32_t> cols(rp[nf]);
    std::vector<double> vals(rp[nf]);
    for (int64_t f = 0; f < nf; ++f)
        for (int k = 0; k < cnt[f]; ++k) {
            cols[rp[f] + k] = cc[7 * f + k];
            vals[rp[f] + k] = cv[7 * f + k];
        }
    std::vector<int64_t> msp, esp;
    std::vector<int32_t> mcol, einc;
    std::vector<double> mval;
    sell_pack(rp, cols, vals, true, 0, msp, mcol, mval);
    // edge rows (device order): incident faces with the sign of C
    std::vector<int64_t> erp(ne + 1, 0);
    for (int64_t f = 0; f < nf; ++f)
        for (int j = 0; j < 3; ++j) ++erp[m.dev_face_edges[3 * f + j] + 1];
    for (int64_t e = 0; e < ne; ++e) erp[e + 1] += erp[e];
    std::vector<int32_t> ecode(erp[ne]);
    std::vector<int64_t> fill(erp.begin(), erp.end() - 1);
    for (int64_t f = 0; f < nf; ++f)
        for (int j = 0; j < 3; ++j) ecode[fill[m.dev_face_edges[3 * f + j]]++] = (int32_t)((f << 1) | (j == 2 ? 1 : 0));
    std::vector<int32_t> dummy_val(erp[ne], 0), dummy_out;
    sell_pack(erp, ecode, dummy_val, false, -1, esp, einc, dummy_out);
    int rc;
    if ((rc = upload(c, &c->d_mf_sp, msp)) || (rc = upload(c, &c->d_mf_col, mcol)) ||
        (rc = upload(c, &c->d_mf_val, mval)) || (rc = upload(c, &c->d_ef_sp, esp)) || (rc = upload(c, &c->d_ef_inc, einc)))
        return rc;
    c->d_h = dalloc<double>(c, nf);
    if (!c->d_h) return fail(c, FEPIC_E_OOM, "device allocation failed");
    c->mfem_ready = true;
    return FEPIC_OK;
}

constexpr int kMaxRestarts = 3;

// The learned start's guard on its squared residual rr0 against ||b||^2: with the line
// step (never worse than e^n in the A-norm) a start worse than x0 = 0 means broken
// weights; the direct prediction is judged like an extrapolation, which may raise the
// residual, so only a non-finite or absurd one (above 1e4 ||b||) is refused.
bool mlp_start_rejected(int mode, double rr0, double bb) {
    if (mode == FEPIC_WS_MLP) return !std::isfinite(rr0) || rr0 > bb;
    if (mode == FEPIC_WS_MLP_DIRECT) return !std::isfinite(rr0) || rr0 > 1e8 * bb;
    return false;
}

// Field half: RHS, warm start, PCG, true residual, Faraday into d_bn.  Returns the
// iteration count via the host scalars (stream synchronized at return).
int field_phase(fepic_ctx* c, double dt, double beta, double gamma) {
    const int64_t ne = c->mesh.n_edges;
    const int fs = c->opt.field_solver;
    if (fs != FEPIC_FIELD_WAVE) {
        const int rc = ensure_mfem(c);
        if (rc != FEPIC_OK) return rc;
    }
    // the mixed updates solve with the wave operator's form: M + dt^2/4 S (NM), M + dt^2 S (BD)
    ensure_operator(c, dt, fs == FEPIC_FIELD_NM_MFEM ? 0.25 : fs == FEPIC_FIELD_BD_MFEM ? 1.0 : beta, gamma);
    ev_mark(c, 4);
    {
        hipEvent_t* ev = timer_pair(c, FAM_RHS);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        const int64_t nf = c->mesh.n_faces;
        if (fs == FEPIC_FIELD_NM_MFEM)
            launch_mfem_rhs(c->stream, ne, nf, c->d_sp, c->d_col, c->d_M, c->d_S, c->d_e, c->d_ep, c->d_dgn, c->d_dg,
                            c->d_bedge, c->d_mf_sp, c->d_mf_col, c->d_mf_val, c->d_b, 1.0, c->d_bp, 1.0, c->d_ef_sp,
                            c->d_ef_inc, c->d_h, dt, 0.0, 1.0, -0.5, -0.25, 1.0, 1.0, c->d_rhs, c->d_partial);
        else if (fs == FEPIC_FIELD_BD_MFEM)
            launch_mfem_rhs(c->stream, ne, nf, c->d_sp, c->d_col, c->d_M, c->d_S, c->d_e, c->d_ep, c->d_dgn, c->d_dg,
                            c->d_bedge, c->d_mf_sp, c->d_mf_col, c->d_mf_val, c->d_b, 1.0, c->d_bp, 0.0, c->d_ef_sp,
                            c->d_ef_inc, c->d_h, dt, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, c->d_rhs, c->d_partial);
        else
            launch_rhs(c->stream, ne, c->d_sp, c->d_col, c->d_M, c->d_S, c->d_e, c->d_ep, c->d_dgn, c->d_dg,
                       c->d_bedge, dt * dt, 0.5 - 2.0 * beta + gamma, 0.5 + beta - gamma,
                       c->abc_on ? c->d_K : nullptr, -(1.0 - 2.0 * gamma) * dt * kY0, (1.0 - gamma) * dt * kY0,
                       c->d_rhs, c->d_partial);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
    }
    ev_mark(c, 5);
    int mode = c->opt.warm_start;
    const bool learned = mode == FEPIC_WS_MLP || mode == FEPIC_WS_MLP_DIRECT;
    if (learned && !c->mlp_ready) mode = FEPIC_WS_PREV;
    if (mode == FEPIC_WS_MLP || mode == FEPIC_WS_MLP_DIRECT) {
        int rc = mlp_warm_start(c, mode == FEPIC_WS_MLP_DIRECT);
        if (rc != FEPIC_OK) return rc;
    } else {
        launch_warm(c->stream, mode, ne, c->d_e, c->d_ep, c->d_ep2, c->d_x);
    }
    if (c->recording) {
        int rc = mlp_record_features(c);
        if (rc != FEPIC_OK) return rc;
    }
    if (c->keep_start && !c->d_x0keep && !(c->d_x0keep = dalloc<double>(c, ne)))
        return fail(c, FEPIC_E_OOM, "allocation failed");
    // the start the solve uses (after the learned start's guard), kept on request
    auto keep_x0 = [&]() -> int {
        if (c->keep_start)
            HIPCHK(c, hipMemcpyAsync(c->d_x0keep, c->d_x, sizeof(double) * ne, hipMemcpyDeviceToDevice, c->stream));
        return FEPIC_OK;
    };
    ev_mark(c, 6);
    CgVec* const V[2] = {c->d_cgv[0], c->d_cgv[1]};
    double2* const ZP[2] = {c->d_zp[0], c->d_zp[1]};
    const bool aux = c->opt.preconditioner == FEPIC_PC_AUX;
    const bool mixed = aux && c->opt.solve_precision == FEPIC_SOLVE_MIXED;
    if (mixed) {
        int rc = ensure_operator_f32(c);
        if (rc != FEPIC_OK) return rc;
    }
    auto cg_init = [&]() {
        if (aux)
            launch_pcg_init(c->stream, ne, c->d_sp, c->d_col, c->d_A, c->d_dinv, c->d_rhs, c->d_x, c->aux, ZP[0],
                            c->d_rq, c->d_partial, c->d_sc, c->opt.cg_tol);
        else
            launch_cg_init(c->stream, ne, c->d_sp, c->d_col, c->d_A, c->d_dinv, c->d_rhs, c->d_x, V[0], c->d_partial,
                           c->d_sc, c->opt.cg_tol, c->opt.deterministic != 0);
    };
    auto true_resid = [&]() -> int {
        launch_cg_resid(c->stream, ne, c->d_sp, c->d_col, c->d_A, c->d_rhs, c->d_x, c->d_rt, c->d_partial, c->d_sc);
        HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return FEPIC_OK;
    };
    const int maxit = c->opt.cg_max_iters;
    const int batch = std::max(1, c->opt.cg_check_every);
    int total = 0;
    double rr0_first = -1.0;
    c->cg_restarts = 0;
    c->cg_passes = 0;
    // Iterations are launched in batches; after each batch the host reads the device's
    // convergence flag and sizes the next batch from the recent contraction of ||r||
    // (never more than doubling what has been launched).  The first batch is the last
    // solve's count (of the same pass) plus two: counts vary little from step to step, and
    // launches after convergence return at once, which costs less than another round trip
    // to the host.  iter(i) launches iteration i.
    auto iterate = [&](int first, auto&& iter) -> int {
        int launched = 0, last_done = -1;
        double last_rr = 0.0;
        const int budget = maxit - total;
        int todo = first;
        for (;;) {
            // the launch after the budget only checks (and is discarded on failure)
            todo = std::min(todo, budget + 1 - launched);
            hipEvent_t* ev = timer_pair(c, FAM_CG_ITER, todo);
            if (ev) (void)hipEventRecord(ev[0], c->stream);
            for (int k = 0; k < todo; ++k) iter(launched + k);
            if (ev) (void)hipEventRecord(ev[1], c->stream);
            launched += todo;
            HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            const CgScalars& h = *c->h_sc;
            if (h.converged || launched > budget) break;
            const int done = h.iters;
            if (last_done < 0 && done > 0 && h.rr0 > 0) {   // contraction since the start
                last_done = 0;
                last_rr = h.rr0;
            }
            todo = launched;
            if (last_done >= 0 && done > last_done && h.rr > 0 && last_rr > h.rr && h.tol2_bb > 0) {
                const double rate = std::log(h.rr / last_rr) / (done - last_done);
                const double need = std::log(h.tol2_bb / h.rr) / rate;
                if (std::isfinite(need)) todo = (int)std::ceil(0.85 * need) - (launched - 1 - done);
            }
            todo = std::max(batch, std::min(todo, launched));
            last_done = done;
            last_rr = h.rr;
        }
        return FEPIC_OK;
    };
    if (mixed) {
        // Iterative refinement: the FP64 residual of x, an FP32 PCG for the correction
        // from zero, x += d in FP64.  The inner solves overwrite the device's ||b||^2 and
        // tolerance; the outer ones are kept here.
        launch_pcg_rhs_norm(c->stream, ne, c->d_partial, c->d_sc, c->opt.cg_tol);
        float2* const ZP32[2] = {c->d_zp32[0], c->d_zp32[1]};
        constexpr int kMaxPasses = 8;
        double bb = 0.0, tol2 = 0.0;
        for (int pass = 0;; ++pass) {
            int rc = true_resid();
            if (rc != FEPIC_OK) return rc;
            const CgScalars h = *c->h_sc;
            if (pass == 0) {
                bb = h.bb;
                tol2 = h.tol2_bb;
                if (mlp_start_rejected(mode, h.rr_true, bb)) {
                    // guard: a non-finite or implausible start falls back to e^n
                    c->mlp_fallbacks++;
                    mode = FEPIC_WS_PREV;
                    launch_warm(c->stream, FEPIC_WS_PREV, ne, c->d_e, c->d_ep, c->d_ep2, c->d_x);
                    --pass;
                    continue;
                }
                rr0_first = h.rr_true;
                if ((rc = keep_x0()) != FEPIC_OK) return rc;
            }
            if (!(h.rr_true > tol2) || !std::isfinite(h.rr_true) || pass >= kMaxPasses || total >= maxit) break;
            // the pass ends when its own residual has fallen by mixed_inner_tol, or below half
            // the outer target
            const double tol_in = std::max(c->opt.mixed_inner_tol, 0.5 * std::sqrt(tol2 / h.rr_true));
            launch_pcg_init_f32(c->stream, ne, c->d_sp, c->d_col, c->d_A32, c->d_dinv32, c->d_rt, c->d_x32, c->aux,
                                ZP32[0], c->d_rq32, c->d_partial, c->d_sc, tol_in);
            const int first = c->last_pass_iters[pass] > 0 ? std::max(batch, c->last_pass_iters[pass] + 2) : batch;
            rc = iterate(first, [&](int i) {
                launch_pcg_iter_f32(c->stream, i, ne, c->d_sp, c->d_col, c->d_A32, c->d_dinv32, c->d_x32, c->aux,
                                    ZP32, c->d_rq32, c->d_partial, c->d_sc);
            });
            if (rc != FEPIC_OK) return rc;
            c->last_pass_iters[pass] = c->h_sc->iters;
            total += c->h_sc->iters;
            c->cg_passes = pass + 1;
            launch_add_f32(c->stream, c->d_x, c->d_x32, ne);
        }
        c->h_sc->bb = bb;
        c->h_sc->tol2_bb = tol2;
    } else {
        for (int restart = 0;; ++restart) {
            cg_init();
            if (restart == 0 && (mode == FEPIC_WS_MLP || mode == FEPIC_WS_MLP_DIRECT)) {
                // guard: a non-finite or implausible start falls back to e^n
                if (aux) launch_pcg_rr0(c->stream, c->d_partial, c->d_sc);
                else launch_cg_rr0(c->stream, ne, c->d_partial, c->d_sc);
                HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                if (mlp_start_rejected(mode, c->h_sc->rr0, c->h_sc->bb)) {
                    c->mlp_fallbacks++;
                    launch_warm(c->stream, FEPIC_WS_PREV, ne, c->d_e, c->d_ep, c->d_ep2, c->d_x);
                    cg_init();
                }
            }
            if (restart == 0) {
                const int rk = keep_x0();
                if (rk != FEPIC_OK) return rk;
            }
            const int first = (restart == 0 && c->last_cg_iters > 0) ? std::max(batch, c->last_cg_iters + 2) : batch;
            int rc = iterate(first, [&](int i) {
                if (aux)
                    launch_pcg_iter(c->stream, i, ne, c->d_sp, c->d_col, c->d_A, c->d_dinv, c->d_x, c->aux, ZP,
                                    c->d_rq, c->d_partial, c->d_sc);
                else
                    launch_cg_iter(c->stream, i, ne, c->d_sp, c->d_col, c->d_A, c->d_dinv, c->d_x, V, c->d_partial,
                                   c->d_sc, c->opt.deterministic != 0);
            });
            if (rc != FEPIC_OK) return rc;
            if (restart == 0) rr0_first = c->h_sc->rr0;
            total += c->h_sc->iters;
            // The stopping rule is on the true residual.  If the recurrences drifted from it,
            // or broke down (converged == 2: a non-positive or non-finite step), restart from
            // the current iterate, up to kMaxRestarts times within the iteration budget.
            rc = true_resid();
            if (rc != FEPIC_OK) return rc;
            const CgScalars& h = *c->h_sc;
            if (h.rr_true <= h.tol2_bb || restart >= kMaxRestarts || total >= maxit || h.converged == 0) break;
            c->cg_restarts++;
        }
    }
    c->h_sc->iters = total;
    c->h_sc->rr0 = rr0_first;
    // success only when the true residual meets the tolerance
    c->h_sc->converged = (c->h_sc->rr_true <= c->h_sc->tol2_bb) ? 1 : 0;
    if (c->h_sc->converged) c->last_cg_iters = total;
    ev_mark(c, 7);
    {
        hipEvent_t* ev = timer_pair(c, FAM_FARADAY);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        if (fs == FEPIC_FIELD_NM_MFEM)
            launch_mfem_faraday(c->stream, c->mesh.n_faces, c->d_face_edges, c->d_bp, c->d_e, c->d_ep, c->d_x, dt,
                                1.0, 0.5, 0.5, c->d_bn);
        else if (fs == FEPIC_FIELD_BD_MFEM)
            launch_mfem_faraday(c->stream, c->mesh.n_faces, c->d_face_edges, c->d_b, c->d_e, c->d_ep, c->d_x, dt,
                                0.0, 0.0, 1.0, c->d_bn);
        else
            launch_faraday(c->stream, c->mesh.n_faces, c->d_face_edges, c->d_b, c->d_x, c->d_e, dt, gamma, c->d_bn);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
    }
    ev_mark(c, 8);
    return FEPIC_OK;
}

void fill_phase_times(fepic_ctx* c, fepic_step_stats* st, bool field) {
    if (!c->opt.timing || !st) return;
    float ms[8] = {0};
    const int last = field ? 8 : 3;
    for (int i = 0; i < last; ++i) (void)hipEventElapsedTime(&ms[i], c->phase_ev[i], c->phase_ev[i + 1]);
    st->ms_sort = ms[0];
    st->ms_stage = ms[1];
    st->ms_particles = ms[2];
    if (field) {
        st->ms_rhs = ms[4];
        st->ms_warm = ms[5];
        st->ms_cg = ms[6];
        st->ms_faraday = ms[7];
    }
}

double max_abs_qw(const fepic_ctx* c) {
    double q = 0.0;
    for (const auto& s : c->species) q = std::max(q, std::fabs(s.q * s.w));
    return q > 0 ? q : 1.0;
}

// Conservation diagnostics after a committed step.  have_step: continuity/drift apply.
int run_diagnostics(fepic_ctx* c, fepic_step_stats* st, bool have_step, bool have_solve) {
    const int64_t nn = c->mesh.n_nodes, ne = c->mesh.n_edges;
    const hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(c->d_acc, 0, sizeof(DiagAcc), s));
    compute_rho(c, c->d_rho_new);
    launch_fill(s, c->d_n1, nn, 0.0);
    launch_DT(s, ne, c->d_edges, c->d_dg, c->d_n1);                   // D^T dG
    launch_sell_spmv(s, ne, c->d_sp, c->d_col, c->d_M, c->d_e, c->d_Me);
    launch_fill(s, c->d_n2, nn, 0.0);
    launch_DT(s, ne, c->d_edges, c->d_Me, c->d_n2);                   // D^T M e
    launch_fill(s, c->d_n3, nn, 0.0);
    if (have_solve) launch_DT(s, ne, c->d_edges, c->d_rt, c->d_n3);   // D^T r_cg
    const int have_hist = (have_step && have_solve && c->rG_levels >= 2) ? 1 : 0;
    double* rG_new = c->d_rG[c->rG_head];
    const double* rG1 = c->d_rG[(c->rG_head + 2) % 3];
    const double* rG2 = c->d_rG[(c->rG_head + 1) % 3];
    // the Gauss residual's recurrence follows the field update's stencil (r^{n+1} + c1 r^n +
    // c2 r^{n-1} = D^T r_cg): wave (-2, 1), NM-MFEM (0, -1), BD-MFEM (-1, 0)
    const double gc1 = c->opt.field_solver == FEPIC_FIELD_WAVE ? -2.0 : c->opt.field_solver == FEPIC_FIELD_BD_MFEM ? -1.0 : 0.0;
    const double gc2 = c->opt.field_solver == FEPIC_FIELD_BD_MFEM ? 0.0 : c->opt.field_solver == FEPIC_FIELD_NM_MFEM ? -1.0 : 1.0;
    launch_diag_nodes(s, nn, c->d_inode, c->d_rho_new, c->rho_valid ? c->d_rho : c->d_rho_new, c->d_n1, c->d_n2, rG1,
                      rG2, c->d_n3, have_hist, gc1, gc2, rG_new, c->d_acc);
    launch_divb(s, c->mesh.n_tets, c->d_tet_faces, c->d_b, c->d_acc);
    launch_dot(s, ne, c->d_e, c->d_Me, c->d_partial, &c->d_acc->energy);
    launch_magnetic(s, c->mesh.n_tets, c->d_b, c->d_grad64, c->d_tet_faces, &c->d_acc->magnetic);
    for (auto& sp : c->species) {
        const double wmc2 = sp.w * sp.m * kC * kC;
        if (c->opt.precision == FEPIC_ALL_FP64)
            launch_kinetic<double>(s, parr<double>(sp, sp.cur), sp.n, wmc2, &c->d_acc->kinetic);
        else
            launch_kinetic<float>(s, parr<float>(sp, sp.cur), sp.n, wmc2, &c->d_acc->kinetic);
    }
    HIPCHK(c, hipMemcpyAsync(c->h_acc, c->d_acc, sizeof(DiagAcc), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    auto dbl = [](unsigned long long v) {
        double d;
        std::memcpy(&d, &v, 8);
        return d;
    };
    const double scale = std::max(dbl(c->h_acc->rho_max), max_abs_qw(c));
    if (st) {
        st->cont_resid_rel = (have_step && c->rho_valid) ? dbl(c->h_acc->cont_max) / scale : -1.0;
        st->gauss_resid_rel = dbl(c->h_acc->gauss_max) / scale;
        st->gauss_drift_check_rel = have_hist ? dbl(c->h_acc->drift_max) / scale : -1.0;
        st->divb_max = dbl(c->h_acc->divb_max);
        st->field_energy = 0.5 * c->h_acc->energy;
        st->magnetic_energy = c->h_acc->magnetic;
        st->kinetic_energy = c->h_acc->kinetic;
    }
    // rotate: the new charge becomes the current one; Gauss residual history
    std::swap(c->d_rho, c->d_rho_new);
    c->rho_valid = true;
    if (have_step && have_solve) {
        c->rG_head = (c->rG_head + 1) % 3;
        c->rG_levels = std::min(c->rG_levels + 1, 3);
    } else {
        c->rG_levels = 0;
    }
    return FEPIC_OK;
}

// A Boris step or a checkpoint load leaves the Adams-Bashforth histories stale: the next AB
// step restarts every particle from its current state (order 1 first).
void ab_history_stale(fepic_ctx* c) {
    for (auto& s : c->species) s.ab_reset = true;
}

// Adams-Bashforth coefficients of orders 1..kAbMax: the integrals over s in [0, 1] of the
// Lagrange basis on the nodes s = 0, -1, ..., -(m - 1); Gauss-Legendre rules of 2..kAbMax+1
// points (Newton on the Legendre polynomial from the usual cosine guesses).
void ab_tables(AbParams& ap) {
    for (int m = 1; m <= kAbMax; ++m)
        for (int j = 0; j < kAbMax; ++j) {
            if (j >= m) {
                ap.beta[m - 1][j] = 0.0;
                continue;
            }
            long double poly[kAbMax + 1] = {1.0L};   // coefficients, lowest degree first
            long double den = 1.0L;
            int deg = 0;
            for (int q = 0; q < m; ++q) {
                if (q == j) continue;
                const long double node = -(long double)q;
                for (int i = deg + 1; i >= 1; --i) poly[i] = poly[i - 1] - node * poly[i];
                poly[0] = -node * poly[0];
                ++deg;
                den *= (-(long double)j) - node;
            }
            long double integral = 0.0L;
            for (int i = 0; i <= deg; ++i) integral += poly[i] / (i + 1);
            ap.beta[m - 1][j] = (double)(integral / den);
        }
    for (int n = 0; n < kAbMax + 2; ++n)
        for (int q = 0; q < kAbMax + 2; ++q) ap.gl_x[n][q] = ap.gl_w[n][q] = 0.0;
    for (int n = 1; n < kAbMax + 2; ++n) {
        for (int q = 0; q < n; ++q) {
            long double x = std::cos(3.14159265358979323846L * (q + 0.75L) / (n + 0.5L)), dp = 1.0L;
            for (int it = 0; it < 100; ++it) {
                long double p0 = 1.0L, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (x * p1 - p0) / (x * x - 1.0L);
                const long double dx = p1 / dp;
                x -= dx;
                if (std::fabs((double)dx) < 1e-19) break;
            }
            // ascending order of nodes
            ap.gl_x[n][n - 1 - q] = (double)x;
            ap.gl_w[n][n - 1 - q] = (double)(2.0L / ((1.0L - x * x) * dp * dp));
        }
    }
}

int do_step(fepic_ctx* c, double dt, double beta, double gamma, fepic_step_stats* out, bool solve) {
    NEED_DEV(c);
    if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(beta) || !std::isfinite(gamma))
        return fail(c, FEPIC_E_ARG, "bad step parameters");
    fepic_step_stats st;
    std::memset(&st, 0, sizeof(st));
    st.gauss_drift_check_rel = st.cont_resid_rel = st.gauss_resid_rel = -1.0;
    st.pc_far_levels = -1;
    if (c->opt.diagnostics && !c->rho_valid) {
        compute_rho(c, c->d_rho);
        c->rho_valid = true;
    }
    const bool do_sort = c->opt.sort_period == FEPIC_SORT_AUTO ||
                         ((c->opt.sort_period > 0) && (c->step_count % c->opt.sort_period == 0));
    // particles injected by this step are dropped again on any failure below
    struct InjectGuard {
        fepic_ctx* c;
        bool committed = false;
        ~InjectGuard() {
            if (!committed) inject_undo(c);
        }
    } guard{c};
    particle_phase(c, dt, do_sort);
    if (c->deferred_err) {
        int rc = c->deferred_err;
        c->deferred_err = 0;
        return rc;
    }
    if (solve) {
        int rc = field_phase(c, dt, beta, gamma);
        if (rc != FEPIC_OK) return rc;
    }
    HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(PushCounters), hipMemcpyDeviceToHost, c->stream));
    int rc = sync_counts(c);
    if (rc != FEPIC_OK) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    st.n_crossings = (int64_t)c->h_cnt->n_crossings;
    {
        int64_t n_all = 0;
        for (const auto& sp : c->species) n_all += sp.n;
        c->cross_share = n_all > 0 ? (double)st.n_crossings / (double)n_all : 1.0;
        // each species' own crossings and losses: the running counts read after each
        // species' kernels, differenced in push order (a species without particles keeps
        // its last share); its crossings per particle choose its crossing-walk form at the
        // next step, and crossings plus losses count towards its re-binning
        unsigned long long prev = 0, prev_gone = 0;
        for (auto& sp : c->species) {
            if (sp.n_pushed <= 0) continue;
            const unsigned long long cum = sp.h_xcum[0], gone = sp.h_xcum[1];
            const unsigned long long own = cum >= prev ? cum - prev : 0, own_gone = gone >= prev_gone ? gone - prev_gone : 0;
            sp.own_share = (double)own / (double)sp.n_pushed;
            sp.moved += (int64_t)(own + own_gone);
            prev = cum;
            prev_gone = gone;
            sp.n_pushed = 0;
        }
    }
    st.max_crossings = (int)c->h_cnt->max_crossings;
    st.n_absorbed = c->h_cnt->n_absorbed;
    st.n_cap_exceeded = (int)c->h_cnt->n_cap;
    if (solve) {
        const CgScalars& sc = *c->h_sc;
        st.cg_iters = sc.iters;
        st.cg_rel_resid = sc.bb > 0 ? std::sqrt(sc.rr_true / sc.bb) : 0.0;
        st.cg_rel_resid0 = sc.bb > 0 ? std::sqrt(sc.rr0 / sc.bb) : 0.0;
        st.pc_far_levels = c->opt.preconditioner == FEPIC_PC_AUX ? c->aux.n_far : -1;
        st.cg_passes = c->cg_passes;
    }
    fill_phase_times(c, &st, solve);
    // failure: leave the state as it was before the call (the sort is a pure reorder)
    if (st.n_cap_exceeded) {
        if (out) *out = st;
        return fail(c, FEPIC_E_CROSSING_CAP, "a particle path exceeded the crossing cap; step not committed");
    }
    if (solve && !c->h_sc->converged) {
        if (out) *out = st;
        return fail(c, FEPIC_E_CG_NOT_CONVERGED, "PCG did not reach the tolerance; step not committed");
    }
    if (solve && c->recording) {
        rc = mlp_record_target(c);
        if (rc != FEPIC_OK) return rc;
    }
    // commit
    guard.committed = true;
    st.n_injected = inject_commit(c);
    for (auto& s : c->species) s.cur = 1 - s.cur;
    if (c->opt.pusher == FEPIC_PUSHER_AB)
        for (auto& s : c->species) s.abm_cur = 1 - s.abm_cur;
    else
        ab_history_stale(c);
    std::swap(c->d_dg, c->d_dgn);
    launch_axpby(c->stream, c->d_G, c->d_G, 1.0, c->d_dg, 1.0, c->mesh.n_edges);
    if (solve) {
        double* old_ep2 = c->d_ep2;
        c->d_ep2 = c->d_ep;
        c->d_ep = c->d_e;
        c->d_e = c->d_x;
        c->d_x = old_ep2;
        double* old_bp = c->d_bp;   // b^{n-1} <- b^n <- b^{n+1}
        c->d_bp = c->d_b;
        c->d_b = c->d_bn;
        c->d_bn = old_bp;
    }
    c->step_count++;
    c->time += dt;
    // one more sort bookkeeping: dead particles are compacted at the next sort
    int64_t live = 0;
    for (auto& s : c->species) live += s.n;
    st.n_particles = live - st.n_absorbed;
    if (c->opt.diagnostics) {
        rc = run_diagnostics(c, &st, true, solve);
        if (rc != FEPIC_OK) return rc;
    } else {
        c->rho_valid = false;
    }
    st.step = c->step_count;
    st.t = c->time;
    if (out) *out = st;
    return FEPIC_OK;
}

}  // namespace

namespace fepic {

// Electrostatic start: -D^T M (-D phi) = rho on interior nodes.  D^T M D is the P1
// (Whitney-0) stiffness eps0 int grad l_i . grad l_j, assembled here in closed form and
// solved by Jacobi-PCG on the host (set-up only), then e^0 = e^{-1} = -D phi.
int init_electrostatic(fepic_ctx* c, double tol, int* iters) {
    NEED_DEV(c);
    if (!(tol > 0)) return fail(c, FEPIC_E_ARG, "bad tolerance");
    int rc = sync_counts(c);
    if (rc) return rc;
    const HostMesh& m = c->mesh;
    const int64_t nn = m.n_nodes;
    compute_rho(c, c->d_n1);
    std::vector<double> rho(nn);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(rho.data(), c->d_n1, 8 * nn, hipMemcpyDeviceToHost));
    std::vector<int64_t> idx(nn, -1);
    int64_t ni = 0;
    for (int64_t v = 0; v < nn; ++v)
        if (!m.bnode[v]) idx[v] = ni++;
    std::vector<double> bvec(ni);
    double bn = 0.0;
    for (int64_t v = 0; v < nn; ++v)
        if (idx[v] >= 0) {
            bvec[idx[v]] = rho[v];
            bn += rho[v] * rho[v];
        }
    bn = std::sqrt(bn);
    std::vector<double> phi(ni, 0.0);
    int it = 0;
    if (bn > 0) {
        struct Trip { int64_t r, c; double v; };
        std::vector<Trip> tr;
        tr.reserve(16 * m.n_tets);
        for (int64_t t = 0; t < m.n_tets; ++t) {
            double g[4][3];
            for (int k = 1; k < 4; ++k)
                for (int d = 0; d < 3; ++d) g[k][d] = m.grad[9 * t + 3 * (k - 1) + d];
            for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
            for (int a = 0; a < 4; ++a) {
                const int64_t ra = idx[m.tets[4 * t + a]];
                if (ra < 0) continue;
                for (int b = 0; b < 4; ++b) {
                    const int64_t rb = idx[m.tets[4 * t + b]];
                    if (rb < 0) continue;
                    tr.push_back({ra, rb, kEps0 * m.vol[t] * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2])});
                }
            }
        }
        std::sort(tr.begin(), tr.end(), [](const Trip& x, const Trip& y) { return x.r != y.r ? x.r < y.r : x.c < y.c; });
        std::vector<int64_t> rp(ni + 1, 0), ci;
        std::vector<double> vv;
        for (size_t k = 0; k < tr.size(); ++k) {
            if (k > 0 && tr[k].r == tr[k - 1].r && tr[k].c == tr[k - 1].c) {
                vv.back() += tr[k].v;
                continue;
            }
            ci.push_back(tr[k].c);
            vv.push_back(tr[k].v);
            rp[tr[k].r + 1]++;
        }
        for (int64_t r = 0; r < ni; ++r) rp[r + 1] += rp[r];
        std::vector<double> dinv(ni), r(bvec), z(ni), p(ni), q(ni);
        for (int64_t i = 0; i < ni; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] == i) dinv[i] = 1.0 / vv[k];
        auto spmv = [&](const std::vector<double>& x, std::vector<double>& y) {
            for (int64_t i = 0; i < ni; ++i) {
                double a = 0.0;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) a += vv[k] * x[ci[k]];
                y[i] = a;
            }
        };
        double rz = 0.0;
        for (int64_t i = 0; i < ni; ++i) {
            z[i] = dinv[i] * r[i];
            p[i] = z[i];
            rz += r[i] * z[i];
        }
        for (it = 0; it < 100000; ++it) {
            spmv(p, q);
            double pq = 0.0;
            for (int64_t i = 0; i < ni; ++i) pq += p[i] * q[i];
            const double al = rz / pq;
            double rr = 0.0, rzn = 0.0;
            for (int64_t i = 0; i < ni; ++i) {
                phi[i] += al * p[i];
                r[i] -= al * q[i];
                rr += r[i] * r[i];
            }
            if (std::sqrt(rr) <= tol * bn) {
                ++it;
                break;
            }
            for (int64_t i = 0; i < ni; ++i) {
                z[i] = dinv[i] * r[i];
                rzn += r[i] * z[i];
            }
            const double be = rzn / rz;
            rz = rzn;
            for (int64_t i = 0; i < ni; ++i) p[i] = z[i] + be * p[i];
        }
    }
    std::vector<double> e(m.n_edges, 0.0);  // device order
    for (int64_t k = 0; k < m.n_edges; ++k) {
        const int64_t a = idx[m.edges[2 * k]], b = idx[m.edges[2 * k + 1]];
        const double pa = a >= 0 ? phi[a] : 0.0, pb = b >= 0 ? phi[b] : 0.0;
        e[m.eperm[k]] = m.bedge[k] ? 0.0 : -(pb - pa);
    }
    for (double* d : {c->d_e, c->d_ep, c->d_ep2}) HIPCHK(c, hipMemcpy(d, e.data(), 8 * m.n_edges, hipMemcpyHostToDevice));
    c->rG_levels = 0;
    if (iters) *iters = it;
    return FEPIC_OK;
}

}  // namespace fepic

// =============================================================================== C ABI
extern "C" {

int fepic_abi_version(void) { return FEPIC_ABI_VERSION; }

void fepic_default_options(fepic_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->precision = FEPIC_FP32_PUSH_FP64_ACC;
    o->cg_tol = 1e-10;
    o->cg_max_iters = 10000;
    o->cg_check_every = 8;
    o->sort_period = 1;
    o->crossing_cap = 64;
    o->warm_start = FEPIC_WS_PREV;
    o->diagnostics = 0;
    o->timing = 0;
    o->preconditioner = FEPIC_PC_AUX;
    o->aux_far_levels = -1;
    o->walk = FEPIC_WALK_AUTO;
    o->solve_precision = FEPIC_SOLVE_FP64;
    o->mixed_inner_tol = 1e-4;
    o->pusher = FEPIC_PUSHER_BORIS;
    o->ab_order = 4;
    o->field_solver = FEPIC_FIELD_WAVE;
    o->deterministic = 0;
}

const char* fepic_error_string(int code) {
    switch (code) {
        case FEPIC_OK: return "ok";
        case FEPIC_E_ARG: return "bad argument";
        case FEPIC_E_MESH: return "bad mesh";
        case FEPIC_E_STATE: return "bad call order";
        case FEPIC_E_OOM: return "out of memory";
        case FEPIC_E_HIP: return "HIP error";
        case FEPIC_E_CG_NOT_CONVERGED: return "PCG did not converge";
        case FEPIC_E_CROSSING_CAP: return "crossing cap exceeded";
        case FEPIC_E_IO: return "I/O error";
        case FEPIC_E_NO_DEVICE: return "no device in this context";
        default: return "unknown error";
    }
}

const char* fepic_last_error(const fepic_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fepic_create(const fepic_options* opts, fepic_ctx** out) {
    if (!out) return FEPIC_E_ARG;
    *out = nullptr;
    fepic_options o;
    fepic_default_options(&o);
    if (opts) o = *opts;
    if (o.precision != FEPIC_FP32_PUSH_FP64_ACC && o.precision != FEPIC_ALL_FP64) return FEPIC_E_ARG;
    if (!(o.cg_tol > 0) || o.cg_max_iters < 1 || o.crossing_cap < 1 ||
        (o.sort_period < 0 && o.sort_period != FEPIC_SORT_AUTO))
        return FEPIC_E_ARG;
    if (o.warm_start < FEPIC_WS_PREV || o.warm_start > FEPIC_WS_MLP_DIRECT) return FEPIC_E_ARG;
    if (o.preconditioner != FEPIC_PC_JACOBI && o.preconditioner != FEPIC_PC_AUX) return FEPIC_E_ARG;
    if (o.aux_far_levels < -1 || o.aux_far_levels > kAuxFarLevels) return FEPIC_E_ARG;
    if (o.walk < FEPIC_WALK_AUTO || o.walk > FEPIC_WALK_FUSED) return FEPIC_E_ARG;
    if (o.solve_precision != FEPIC_SOLVE_FP64 && o.solve_precision != FEPIC_SOLVE_MIXED) return FEPIC_E_ARG;
    if (o.solve_precision == FEPIC_SOLVE_MIXED && o.preconditioner != FEPIC_PC_AUX) return FEPIC_E_ARG;
    if (!(o.mixed_inner_tol > 0.0 && o.mixed_inner_tol < 1.0)) return FEPIC_E_ARG;
    if (o.pusher != FEPIC_PUSHER_BORIS && o.pusher != FEPIC_PUSHER_AB) return FEPIC_E_ARG;
    if (o.ab_order < 1 || o.ab_order > kAbMax) return FEPIC_E_ARG;
    if (o.pusher == FEPIC_PUSHER_AB && o.precision != FEPIC_ALL_FP64) return FEPIC_E_ARG;
    if (o.field_solver < FEPIC_FIELD_WAVE || o.field_solver > FEPIC_FIELD_BD_MFEM) return FEPIC_E_ARG;
    if (o.deterministic != 0 && o.deterministic != 1) return FEPIC_E_ARG;
    if (o.deterministic && (o.preconditioner != FEPIC_PC_JACOBI || o.solve_precision != FEPIC_SOLVE_FP64 ||
                            o.warm_start == FEPIC_WS_MLP || o.warm_start == FEPIC_WS_MLP_DIRECT))
        return FEPIC_E_ARG;
    if (o.cg_check_every < 1) o.cg_check_every = 8;
    fepic_ctx* c = new fepic_ctx();
    c->opt = o;
    c->host_only = (o.device < 0);
    if (!c->host_only) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) {
            delete c;
            return FEPIC_E_NO_DEVICE;
        }
        if (hipSetDevice(o.device) != hipSuccess || hipStreamCreate(&c->own_stream) != hipSuccess) {
            delete c;
            return FEPIC_E_HIP;
        }
        c->stream = c->own_stream;
        if (hipHostMalloc((void**)&c->h_sc, sizeof(CgScalars)) != hipSuccess ||
            hipHostMalloc((void**)&c->h_cnt, sizeof(PushCounters)) != hipSuccess ||
            hipHostMalloc((void**)&c->h_acc, sizeof(DiagAcc)) != hipSuccess) {
            delete c;
            return FEPIC_E_OOM;
        }
        for (auto& e : c->phase_ev) (void)hipEventCreate(&e);
        mlp_noalloc_setup(o.device);
    }
    *out = c;
    return FEPIC_OK;
}

int fepic_destroy(fepic_ctx* c) {
    if (!c) return FEPIC_E_ARG;
    if (!c->host_only) {
        (void)hipSetDevice(c->opt.device);
        (void)hipStreamSynchronize(c->stream);
        for (void* p : c->allocs) release(c, p);
        for (auto& s : c->species) {
            if (s.h_nlive) (void)hipHostFree(s.h_nlive);
            if (s.h_xcum) (void)hipHostFree(s.h_xcum);
        }
        for (auto& t : c->timers)
            for (auto e : t.ev) (void)hipEventDestroy(e);
        for (auto e : c->phase_ev) (void)hipEventDestroy(e);
        if (c->h_sc) (void)hipHostFree(c->h_sc);
        if (c->h_cnt) (void)hipHostFree(c->h_cnt);
        if (c->h_acc) (void)hipHostFree(c->h_acc);
        if (c->h_stage) (void)hipHostFree(c->h_stage);
        if (c->stage_event_valid) (void)hipEventDestroy(c->stage_event);
        if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    }
    mlp_destroy(c);
    delete c;
    return FEPIC_OK;
}

int fepic_set_allocator(fepic_ctx* c, void* (*alloc)(size_t bytes, void* user), void (*free_)(void* ptr, void* user),
                        void* user) {
    if (!c) return FEPIC_E_ARG;
    if (c->host_only) return fail(c, FEPIC_E_NO_DEVICE, "host-only context");
    if (c->have_mesh || !c->allocs.empty()) return fail(c, FEPIC_E_STATE, "set the allocator before the mesh upload");
    if ((alloc == nullptr) != (free_ == nullptr)) return fail(c, FEPIC_E_ARG, "give both functions or neither");
    c->ualloc = alloc;
    c->ufree = free_;
    c->uarg = user;
    return FEPIC_OK;
}

int fepic_set_preconditioner(fepic_ctx* c, int pc) {
    if (!c || (pc != FEPIC_PC_JACOBI && pc != FEPIC_PC_AUX)) return FEPIC_E_ARG;
    if (pc == FEPIC_PC_JACOBI && c->opt.solve_precision == FEPIC_SOLVE_MIXED)
        return fail(c, FEPIC_E_ARG, "the mixed-precision solve needs the auxiliary-space preconditioner");
    if (pc == FEPIC_PC_AUX && c->abc_on)
        return fail(c, FEPIC_E_STATE, "absorbing faces need the Jacobi preconditioner");
    if (pc == FEPIC_PC_AUX && c->opt.deterministic)
        return fail(c, FEPIC_E_STATE, "the deterministic mode needs the Jacobi preconditioner");
    if (c->opt.preconditioner != pc) c->last_cg_iters = 0;   // batch sizing starts afresh
    c->opt.preconditioner = pc;
    return FEPIC_OK;
}

int fepic_set_solve_precision(fepic_ctx* c, int sp) {
    if (!c || (sp != FEPIC_SOLVE_FP64 && sp != FEPIC_SOLVE_MIXED)) return FEPIC_E_ARG;
    if (sp == FEPIC_SOLVE_MIXED && c->opt.preconditioner != FEPIC_PC_AUX)
        return fail(c, FEPIC_E_ARG, "the mixed-precision solve needs the auxiliary-space preconditioner");
    if (c->opt.solve_precision != sp) {
        c->last_cg_iters = 0;
        for (int& n : c->last_pass_iters) n = 0;
    }
    c->opt.solve_precision = sp;
    return FEPIC_OK;
}

int fepic_set_field_solver(fepic_ctx* c, int solver) {
    if (!c) return FEPIC_E_ARG;
    if (solver < FEPIC_FIELD_WAVE || solver > FEPIC_FIELD_BD_MFEM) return fail(c, FEPIC_E_ARG, "bad field solver");
    if (solver != FEPIC_FIELD_WAVE && c->abc_on)
        return fail(c, FEPIC_E_STATE, "absorbing faces work with the wave-equation update only");
    if (solver != c->opt.field_solver) c->rG_levels = 0;   // the Gauss recurrence changes with it
    c->opt.field_solver = solver;
    return FEPIC_OK;
}

int fepic_set_absorbing_faces(fepic_ctx* c, int64_t n, const int32_t* faces) {
    if (!c) return FEPIC_E_ARG;
    if (!c->have_mesh) return fail(c, FEPIC_E_STATE, "no mesh uploaded");
    if (c->abc_on) return fail(c, FEPIC_E_STATE, "absorbing faces already set");
    if (c->step_count > 0) return fail(c, FEPIC_E_STATE, "absorbing faces are set before the first step");
    if (c->opt.field_solver != FEPIC_FIELD_WAVE)
        return fail(c, FEPIC_E_STATE, "absorbing faces work with the wave-equation update only");
    if (c->opt.preconditioner != FEPIC_PC_JACOBI || c->opt.solve_precision != FEPIC_SOLVE_FP64)
        return fail(c, FEPIC_E_STATE, "absorbing faces need the Jacobi preconditioner and the FP64 solve");
    HostMesh& m = c->mesh;
    // a face is on the wall when its tet instance has no neighbour across it
    std::vector<uint8_t> wall(m.n_faces, 0);
    for (int64_t j = 0; j < 4 * m.n_tets; ++j)
        if (m.nbr[j] < 0) wall[m.tet_faces[j]] = 1;
    std::vector<uint8_t> abc(m.n_faces, 0);
    if (!faces) {
        abc = wall;
    } else {
        if (n <= 0) return fail(c, FEPIC_E_ARG, "no faces given");
        for (int64_t i = 0; i < n; ++i) {
            const int32_t f = faces[i];
            if (f < 0 || f >= m.n_faces || !wall[f])
                return fail(c, FEPIC_E_ARG, "face " + std::to_string(f) + " is not a wall face");
            abc[f] = 1;
        }
    }
    // fixed edges: those on a PEC (non-absorbing) wall face
    std::vector<uint8_t> fixed(m.n_edges, 0);
    for (int64_t f = 0; f < m.n_faces; ++f)
        if (wall[f] && !abc[f])
            for (int j = 0; j < 3; ++j) fixed[m.dev_face_edges[3 * f + j]] = 1;
    HostMesh trial = m;   // assemble aside: on failure the context keeps its PEC matrices
    int rc = assemble_edge_matrices(trial, fixed, abc, c->err);
    if (rc != FEPIC_OK) return rc;
    if (!c->host_only) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int64_t* sp = nullptr;
        int32_t* col = nullptr;
        uint8_t* fx = nullptr;
        double *M = nullptr, *S = nullptr, *K = nullptr, *A = nullptr;
        const int64_t nnz = trial.mat.slice_ptr.back();
        if ((rc = upload(c, &sp, trial.mat.slice_ptr)) || (rc = upload(c, &col, trial.mat.col)) ||
            (rc = upload(c, &M, trial.mat.M)) || (rc = upload(c, &S, trial.mat.S)) || (rc = upload(c, &K, trial.mat.K)) ||
            (rc = upload(c, &fx, fixed)) || !(A = dalloc<double>(c, nnz))) {
            for (void* p : {(void*)sp, (void*)col, (void*)M, (void*)S, (void*)K, (void*)fx}) dfree(c, p);
            return rc ? rc : fail(c, FEPIC_E_OOM, "device allocation failed");
        }
        for (void* p : {(void*)c->d_sp, (void*)c->d_col, (void*)c->d_M, (void*)c->d_S, (void*)c->d_A,
                        (void*)c->d_bedge})
            dfree(c, p);
        c->d_sp = sp;
        c->d_col = col;
        c->d_M = M;
        c->d_S = S;
        c->d_K = K;
        c->d_A = A;
        c->d_bedge = fx;
        c->A_valid = false;
        c->A32_valid = false;
    }
    m.mat = std::move(trial.mat);
    m.dev_fixed = std::move(fixed);
    m.abc_face = std::move(abc);
    c->abc_on = true;
    return FEPIC_OK;
}

int fepic_set_pusher(fepic_ctx* c, int pusher, int ab_order) {
    if (!c) return FEPIC_E_ARG;
    if (pusher != FEPIC_PUSHER_BORIS && pusher != FEPIC_PUSHER_AB)
        return fail(c, FEPIC_E_ARG, "pusher must be FEPIC_PUSHER_BORIS or FEPIC_PUSHER_AB");
    if (ab_order < 1 || ab_order > kAbMax) return fail(c, FEPIC_E_ARG, "ab_order must be 1..5");
    if (pusher == FEPIC_PUSHER_AB && c->opt.precision != FEPIC_ALL_FP64)
        return fail(c, FEPIC_E_ARG, "the Adams-Bashforth pusher needs the all-FP64 particle path");
    if (pusher != c->opt.pusher) ab_history_stale(c);
    c->opt.pusher = pusher;
    c->opt.ab_order = ab_order;
    return FEPIC_OK;
}

int fepic_set_stream(fepic_ctx* c, void* stream) {
    if (!c) return FEPIC_E_ARG;
    if (c->host_only) return fail(c, FEPIC_E_NO_DEVICE, "host-only context");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->stream = stream ? (hipStream_t)stream : c->own_stream;
    return FEPIC_OK;
}

int fepic_upload_mesh(fepic_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets) {
    if (!c) return FEPIC_E_ARG;
    if (c->have_mesh) return fail(c, FEPIC_E_STATE, "mesh already uploaded");
    int rc = build_host_mesh(c->mesh, n_nodes, xyz, n_tets, tets, c->err);
    if (rc != FEPIC_OK) return rc;
    c->have_mesh = true;
    if (c->host_only) return FEPIC_OK;
    HostMesh& m = c->mesh;
    const int64_t ne = m.n_edges, nf = m.n_faces, nn = m.n_nodes, nt = m.n_tets;
    std::vector<uint8_t> inode(nn);
    for (int64_t v = 0; v < nn; ++v) inode[v] = !m.bnode[v];
    std::vector<double> r0(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int d = 0; d < 3; ++d) r0[3 * t + d] = m.xyz[3 * m.tets[4 * t] + d];
    if ((rc = upload(c, &c->d_tets, m.tets)) || (rc = upload(c, &c->d_edges, m.dev_edges)) ||
        (rc = upload(c, &c->d_tet_edges, m.dev_tet_edges)) || (rc = upload(c, &c->d_tet_faces, m.tet_faces)) ||
        (rc = upload(c, &c->d_face_edges, m.dev_face_edges)) || (rc = upload(c, &c->d_bedge, m.dev_fixed)) ||
        (rc = upload(c, &c->d_inode, inode)) || (rc = upload(c, &c->d_grad64, m.grad)) ||
        (rc = upload(c, &c->d_r0, r0)) || (rc = upload(c, &c->d_sp, m.mat.slice_ptr)) ||
        (rc = upload(c, &c->d_col, m.mat.col)) || (rc = upload(c, &c->d_M, m.mat.M)) ||
        (rc = upload(c, &c->d_S, m.mat.S)) || (rc = upload(c, &c->d_cell_start, m.cell_start)) ||
        (rc = upload(c, &c->d_cell_tets, m.cell_tets)) || (rc = upload(c, &c->d_int_edges, m.dev_int_edges)))
        return rc;
    std::vector<double> g3 = {m.grid_lo[0], m.grid_lo[1], m.grid_lo[2], m.grid_inv_h[0], m.grid_inv_h[1], m.grid_inv_h[2]};
    std::vector<int32_t> gn = {m.grid_n[0], m.grid_n[1], m.grid_n[2]};
    if ((rc = upload(c, &c->d_grid, g3)) || (rc = upload(c, &c->d_grid_n, gn))) return rc;
    // per-tet records with the static geometry filled in
    const bool f64 = c->opt.precision == FEPIC_ALL_FP64;
    const size_t bsz = f64 ? sizeof(TetBlock<double>) : sizeof(TetBlock<float>);
    std::vector<unsigned char> blk(bsz * nt, 0);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t nbr[4], ed[6];
        for (int k = 0; k < 4; ++k) nbr[k] = m.nbr[4 * t + k] < 0 ? -1 : (m.nbr[4 * t + k] << 2) | m.nbr_far[4 * t + k];
        for (int i = 0; i < 6; ++i) ed[i] = m.dev_tet_edges[6 * t + i];
        if (f64) {
            auto* b = (TetBlock<double>*)(blk.data() + bsz * t);
            for (int i = 0; i < 9; ++i) b->gl[i] = m.grad[9 * t + i];
            std::memcpy(b->nbr, nbr, sizeof(nbr));
            std::memcpy(b->edge, ed, sizeof(ed));
        } else {
            auto* b = (TetBlock<float>*)(blk.data() + bsz * t);
            for (int i = 0; i < 9; ++i) b->gl[i] = (float)m.grad[9 * t + i];
            std::memcpy(b->nbr, nbr, sizeof(nbr));
            std::memcpy(b->edge, ed, sizeof(ed));
        }
    }
    if ((rc = upload(c, (unsigned char**)&c->d_blk, blk))) return rc;
    const int64_t nnz = m.mat.slice_ptr.back();
    c->d_A = dalloc<double>(c, nnz);
    c->d_dinv = dalloc<double>(c, ne);
    double** ev[] = {&c->d_e, &c->d_ep, &c->d_ep2, &c->d_x, &c->d_dg, &c->d_dgn, &c->d_G, &c->d_rhs, &c->d_rt,
                     &c->d_Me};
    for (double** p : ev) {
        *p = dalloc<double>(c, ne);
        if (!*p) return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemset(*p, 0, sizeof(double) * ne));
    }
    for (CgVec*& p : c->d_cgv) {
        p = dalloc<CgVec>(c, ne);
        if (!p) return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemset(p, 0, sizeof(CgVec) * ne));
    }
    // nodal auxiliary space of the preconditioner
    {
        double sum = 0.0;
        int64_t cnt = 0;
        for (int64_t r = 0; r < ne; ++r) {
            if (m.dev_fixed[r]) continue;
            const int64_t k = m.mat.slice_ptr[r / kSell] + r % kSell;   // the diagonal slot
            if (m.mat.M[k] > 0) {
                sum += m.mat.S[k] / m.mat.M[k];
                ++cnt;
            }
        }
        c->s_over_m = cnt ? sum / (double)cnt : 0.0;
        int64_t *asp = nullptr;
        int32_t *ainc = nullptr, *aends = nullptr;
        EdgeVec* ath = nullptr;
        if ((rc = upload(c, &asp, m.aux_sp)) || (rc = upload(c, &ainc, m.aux_inc)) ||
            (rc = upload(c, &ath, m.aux_th)) || (rc = upload(c, &aends, m.aux_ends)))
            return rc;
        c->aux.n_aux = m.n_aux;
        c->aux.sp = asp;
        c->aux.inc = ainc;
        c->aux.th = ath;
        c->aux.ends = reinterpret_cast<const int2*>(aends);
        c->aux.scale = dalloc<double4>(c, m.n_aux);
        c->aux.scale8 = dalloc<double4>(c, (m.n_aux + 7) / 8);
        c->aux.scale64 = dalloc<double4>(c, (m.n_aux + 63) / 64);
        c->aux.Y = dalloc<double4>(c, m.n_aux + 1);
        for (int L = 0; L < kAuxFarLevels; ++L) {
            c->aux.far_scale[L] = dalloc<double4>(c, aux_far_count(m.n_aux, L));
            if (!c->aux.far_scale[L]) return fail(c, FEPIC_E_OOM, "device allocation failed");
        }
        const int64_t nf0 = aux_far_count(m.n_aux, 0);
        c->aux.far_acc = dalloc<double4>(c, 8 * nf0);
        if (!c->aux.far_acc) return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemset(c->aux.far_acc, 0, sizeof(double4) * std::max<int64_t>(8 * nf0, 1)));
        c->d_rq = dalloc<double2>(c, ne);
        for (double2*& p : c->d_zp) p = dalloc<double2>(c, ne);
        if (!c->aux.scale || !c->aux.scale8 || !c->aux.scale64 || !c->aux.Y || !c->d_rq || !c->d_zp[0] ||
            !c->d_zp[1])
            return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemset(c->aux.Y, 0, sizeof(double4) * (m.n_aux + 1)));   // entry n_aux stays zero
        HIPCHK(c, hipMemset(c->aux.scale, 0, sizeof(double4) * std::max<int64_t>(m.n_aux, 1)));
        HIPCHK(c, hipMemset(c->d_rq, 0, sizeof(double2) * ne));
        for (double2* p : c->d_zp) HIPCHK(c, hipMemset(p, 0, sizeof(double2) * ne));
    }
    double** fv[] = {&c->d_b, &c->d_bn, &c->d_bp};
    for (double** p : fv) {
        *p = dalloc<double>(c, nf);
        if (!*p) return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemset(*p, 0, sizeof(double) * nf));
    }
    double** nv[] = {&c->d_rho, &c->d_rho_new, &c->d_n1, &c->d_n2, &c->d_n3, &c->d_rG[0], &c->d_rG[1], &c->d_rG[2]};
    for (double** p : nv) {
        *p = dalloc<double>(c, nn);
        if (!*p) return fail(c, FEPIC_E_OOM, "device allocation failed");
        HIPCHK(c, hipMemset(*p, 0, sizeof(double) * nn));
    }
    c->d_partial = dalloc<double>(c, (int64_t)partial_buffer_doubles());
    c->d_sc = dalloc<CgScalars>(c, 1);
    c->d_cnt = dalloc<PushCounters>(c, 1);
    c->d_cnt_slots = dalloc<PushCounters>(c, kCntSlots);
    if (c->d_cnt_slots) HIPCHK(c, hipMemset(c->d_cnt_slots, 0, sizeof(PushCounters) * kCntSlots));
    c->d_acc = dalloc<DiagAcc>(c, 1);
    c->d_dotc = dalloc<unsigned int>(c, 1);
    c->d_live = dalloc<double>(c, 1);
    c->d_count = dalloc<int32_t>(c, nt);
    c->d_offset = dalloc<int32_t>(c, nt);
    c->d_bsums = dalloc<int32_t>(c, nt / 1024 + 2);
    if (!c->d_A || !c->d_dinv || !c->d_partial || !c->d_sc || !c->d_cnt || !c->d_cnt_slots || !c->d_acc || !c->d_count ||
        !c->d_offset || !c->d_bsums || !c->d_dotc || !c->d_live)
        return fail(c, FEPIC_E_OOM, "device allocation failed");
    HIPCHK(c, hipMemset(c->d_sc, 0, sizeof(CgScalars)));
    HIPCHK(c, hipMemset(c->d_dotc, 0, sizeof(unsigned int)));
    HIPCHK(c, hipDeviceSynchronize());
    return FEPIC_OK;
}

int fepic_get_topology_sizes(fepic_ctx* c, int64_t* n_edges, int64_t* n_faces, int64_t* n_int_edges,
                             int64_t* n_int_nodes, int64_t* euler) {
    if (!c) return FEPIC_E_ARG;
    if (!c->have_mesh) return fail(c, FEPIC_E_STATE, "no mesh uploaded");
    const HostMesh& m = c->mesh;
    if (n_edges) *n_edges = m.n_edges;
    if (n_faces) *n_faces = m.n_faces;
    if (n_int_edges) *n_int_edges = m.n_int_edges;
    if (n_int_nodes) *n_int_nodes = m.n_int_nodes;
    if (euler) *euler = m.n_nodes - m.n_edges + m.n_faces - m.n_tets;
    return FEPIC_OK;
}

int fepic_get_topology(fepic_ctx* c, int32_t* tets_sorted, int32_t* edges, int32_t* faces, int32_t* tet_edges,
                       int32_t* tet_faces, int32_t* nbr) {
    if (!c) return FEPIC_E_ARG;
    if (!c->have_mesh) return fail(c, FEPIC_E_STATE, "no mesh uploaded");
    const HostMesh& m = c->mesh;
    if (tets_sorted) std::copy(m.tets.begin(), m.tets.end(), tets_sorted);
    if (edges) std::copy(m.edges.begin(), m.edges.end(), edges);
    if (faces) std::copy(m.faces.begin(), m.faces.end(), faces);
    if (tet_edges) std::copy(m.tet_edges.begin(), m.tet_edges.end(), tet_edges);
    if (tet_faces) std::copy(m.tet_faces.begin(), m.tet_faces.end(), tet_faces);
    if (nbr) std::copy(m.nbr.begin(), m.nbr.end(), nbr);
    return FEPIC_OK;
}

int fepic_get_matrix(fepic_ctx* c, int which, int64_t cap, int64_t* nnz, int64_t* row, int64_t* col, double* val) {
    if (!c || !nnz || which < 0 || which > 2) return FEPIC_E_ARG;
    if (!c->have_mesh) return fail(c, FEPIC_E_STATE, "no mesh uploaded");
    const HostMesh& m = c->mesh;
    const SellMatrix& A = m.mat;
    if (which == 2 && A.K.empty()) return fail(c, FEPIC_E_STATE, "no absorbing faces set");
    const std::vector<double>& v = which == 0 ? A.M : which == 1 ? A.S : A.K;
    int64_t n = 0;
    for (int64_t s = 0; s < A.n_slices; ++s) {
        const int64_t w = (A.slice_ptr[s + 1] - A.slice_ptr[s]) / kSell;
        for (int l = 0; l < kSell; ++l) {
            const int64_t r = s * kSell + l;
            if (r >= A.n_rows || m.dev_fixed[r]) continue;
            for (int64_t k = 0; k < w; ++k) {
                const int64_t p = A.slice_ptr[s] + k * kSell + l;
                if (k > 0 && A.col[p] == r) continue;  // padding
                if (row && n < cap) {
                    row[n] = m.eiperm[r];
                    col[n] = m.eiperm[A.col[p]];
                    val[n] = v[p];
                }
                ++n;
            }
        }
    }
    *nnz = n;
    return (row && n > cap) ? FEPIC_E_ARG : FEPIC_OK;
}

int fepic_set_fields(fepic_ctx* c, const double* e, const double* e_prev, const double* b) {
    NEED_DEV(c);
    const HostMesh& m = c->mesh;
    auto put_e = [&](double* dst, const double* src) -> int {
        std::vector<double> v(m.n_edges);
        for (int64_t i = 0; i < m.n_edges; ++i) v[m.eperm[i]] = m.dev_fixed[m.eperm[i]] ? 0.0 : src[i];
        HIPCHK(c, hipMemcpy(dst, v.data(), sizeof(double) * m.n_edges, hipMemcpyHostToDevice));
        return FEPIC_OK;
    };
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc;
    if (e && (rc = put_e(c->d_e, e))) return rc;
    if (e_prev && (rc = put_e(c->d_ep, e_prev))) return rc;
    if (e_prev && (rc = put_e(c->d_ep2, e_prev))) return rc;
    if (b) {
        HIPCHK(c, hipMemcpy(c->d_b, b, sizeof(double) * m.n_faces, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_bp, b, sizeof(double) * m.n_faces, hipMemcpyHostToDevice));
    }
    c->rG_levels = 0;
    return FEPIC_OK;
}

int fepic_set_uniform_B(fepic_ctx* c, const double B0[3]) {
    NEED_DEV(c);
    if (!B0) return FEPIC_E_ARG;
    std::vector<double> av;
    face_area_vectors(c->mesh, av);
    std::vector<double> b(c->mesh.n_faces);
    for (int64_t f = 0; f < c->mesh.n_faces; ++f) b[f] = B0[0] * av[3 * f] + B0[1] * av[3 * f + 1] + B0[2] * av[3 * f + 2];
    return fepic_set_fields(c, nullptr, nullptr, b.data());
}

int fepic_add_species(fepic_ctx* c, double q, double m, double w, int* out) {
    NEED_DEV(c);
    if (!(m > 0) || !std::isfinite(q) || !std::isfinite(w)) return fail(c, FEPIC_E_ARG, "bad species parameters");
    Species s;
    s.q = q;
    s.m = m;
    s.w = w;
    s.d_nlive = dalloc<int32_t>(c, 1);
    s.d_xcum = dalloc<unsigned long long>(c, 2);
    if (!s.d_nlive || !s.d_xcum || hipHostMalloc((void**)&s.h_nlive, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void**)&s.h_xcum, 2 * sizeof(unsigned long long)) != hipSuccess)
        return fail(c, FEPIC_E_OOM, "allocation failed");
    s.h_xcum[0] = s.h_xcum[1] = 0;
    c->species.push_back(s);
    if (out) *out = (int)c->species.size() - 1;
    return FEPIC_OK;
}

int fepic_set_injector(fepic_ctx* c, int species, const fepic_injector* spec) {
    NEED_DEV(c);
    if (species < 0 || species >= (int)c->species.size()) return fail(c, FEPIC_E_ARG, "bad species");
    Species& s = c->species[species];
    if (!spec) {
        s.inj_on = false;
        return FEPIC_OK;
    }
    const double nn = std::sqrt(spec->normal[0] * spec->normal[0] + spec->normal[1] * spec->normal[1] +
                                spec->normal[2] * spec->normal[2]);
    bool ok = std::isfinite(nn) && nn > 0 && spec->radius > 0 && std::isfinite(spec->radius) &&
              spec->kinetic_eV >= 0 && std::isfinite(spec->kinetic_eV) && spec->thermal_eV >= 0 &&
              std::isfinite(spec->thermal_eV) && spec->per_step >= 0 && spec->per_step < ((int64_t)1 << 30);
    for (int d = 0; d < 3; ++d) ok = ok && std::isfinite(spec->center[d]);
    if (!ok) return fail(c, FEPIC_E_ARG, "bad injector parameters");
    InjectorSpec& sp = s.inj;
    for (int d = 0; d < 3; ++d) {
        sp.c[d] = spec->center[d];
        sp.n[d] = spec->normal[d] / nn;
    }
    // in-plane basis: e1 = unit(n x a), a the x axis unless n is within 26 degrees of it
    const double a[3] = {std::fabs(sp.n[0]) < 0.9 ? 1.0 : 0.0, std::fabs(sp.n[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    double e1[3] = {sp.n[1] * a[2] - sp.n[2] * a[1], sp.n[2] * a[0] - sp.n[0] * a[2], sp.n[0] * a[1] - sp.n[1] * a[0]};
    const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int d = 0; d < 3; ++d) sp.e1[d] = e1[d] / l1;
    sp.e2[0] = sp.n[1] * sp.e1[2] - sp.n[2] * sp.e1[1];
    sp.e2[1] = sp.n[2] * sp.e1[0] - sp.n[0] * sp.e1[2];
    sp.e2[2] = sp.n[0] * sp.e1[1] - sp.n[1] * sp.e1[0];
    sp.radius = spec->radius;
    const double g0 = 1.0 + spec->kinetic_eV * kQe / (s.m * kC * kC);
    sp.v0 = kC * std::sqrt(1.0 - 1.0 / (g0 * g0));
    sp.sigma = std::sqrt(spec->thermal_eV * kQe / s.m);
    sp.per_step = spec->per_step;
    sp.seed = spec->seed;
    sp.species = species;
    s.inj_on = true;
    s.inj_k = 0;
    return FEPIC_OK;
}

// Locates n particles read from device memory, appends them to species s, sorts the
// species and reads back the rejected count (synchronizes the stream).
static int upload_located(fepic_ctx* c, Species& s, int64_t n, const int64_t* did, const double* dx,
                          const double* du, int64_t* n_rejected) {
    HIPCHK(c, hipMemsetAsync(c->d_cnt, 0, sizeof(PushCounters), c->stream));
    const double* g = c->d_grid;
    if (c->opt.precision == FEPIC_ALL_FP64)
        launch_locate<double>(c->stream, n, dx, du, did, s.next_id, parr<double>(s, s.cur), s.n, c->d_grad64, c->d_r0,
                              c->d_cell_start, c->d_cell_tets, g, g + 3, c->d_grid_n, c->d_cnt);
    else
        launch_locate<float>(c->stream, n, dx, du, did, s.next_id, parr<float>(s, s.cur), s.n, c->d_grad64, c->d_r0,
                             c->d_cell_start, c->d_cell_tets, g, g + 3, c->d_grid_n, c->d_cnt);
    s.next_id += n;
    s.ab_fill_from = std::min(s.ab_fill_from, s.n);
    s.n += n;
    if (c->opt.precision == FEPIC_ALL_FP64) sort_species<double>(c, s);
    else sort_species<float>(c, s);
    HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(PushCounters), hipMemcpyDeviceToHost, c->stream));
    int rc = sync_counts(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    if (n_rejected) *n_rejected = c->h_cnt->n_rejected;
    c->rho_valid = false;
    c->rG_levels = 0;
    return FEPIC_OK;
}

static int check_upload(fepic_ctx* c, int species, int64_t n, const double* x, const double* u) {
    if (species < 0 || species >= (int)c->species.size() || n < 0 || (n > 0 && (!x || !u)))
        return fail(c, FEPIC_E_ARG, "bad particle upload arguments");
    if (n == 0) return FEPIC_OK;
    Species& s = c->species[species];
    int rc = sync_counts(c);
    if (rc) return rc;
    if (s.n + n >= ((int64_t)1 << 31)) return fail(c, FEPIC_E_ARG, "too many particles for one species");
    return ensure_capacity(c, s, s.n + n);
}

int fepic_upload_particles(fepic_ctx* c, int species, int64_t n, const int64_t* id, const double* x,
                           const double* u, int64_t* n_rejected) {
    NEED_DEV(c);
    if (n_rejected) *n_rejected = 0;
    int rc = check_upload(c, species, n, x, u);
    if (rc || n == 0) return rc;
    Species& s = c->species[species];
    double* dx = dalloc<double>(c, 3 * n);
    double* du = dalloc<double>(c, 3 * n);
    int64_t* did = id ? dalloc<int64_t>(c, n) : nullptr;
    if (!dx || !du || (id && !did)) {
        dfree(c, dx);
        dfree(c, du);
        dfree(c, did);
        return fail(c, FEPIC_E_OOM, "device allocation failed");
    }
    hipError_t e = hipMemcpyAsync(dx, x, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(du, u, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && id) e = hipMemcpyAsync(did, id, sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream);
    rc = (e == hipSuccess) ? upload_located(c, s, n, did, dx, du, n_rejected) : hip_fail(c, e, "particle upload copy");
    (void)hipStreamSynchronize(c->stream);
    dfree(c, dx);
    dfree(c, du);
    dfree(c, did);
    return rc;
}

int fepic_upload_particles_device(fepic_ctx* c, int species, int64_t n, const int64_t* id, const double* x,
                                  const double* u, int64_t* n_rejected) {
    NEED_DEV(c);
    if (n_rejected) *n_rejected = 0;
    int rc = check_upload(c, species, n, x, u);
    if (rc || n == 0) return rc;
    return upload_located(c, c->species[species], n, id, x, u, n_rejected);
}

static int inject_located(fepic_ctx* c, Species& s, int64_t n, const int64_t* did, const double* dx,
                          const double* du);

int fepic_inject_particles(fepic_ctx* c, int species, int64_t n, const int64_t* id, const double* x,
                           const double* u) {
    NEED_DEV(c);
    if (species < 0 || species >= (int)c->species.size() || n < 0 || (n > 0 && (!x || !u)))
        return fail(c, FEPIC_E_ARG, "bad injection arguments");
    if (n == 0) return FEPIC_OK;
    Species& s = c->species[species];
    int rc = sync_counts(c);
    if (rc) return rc;
    if (s.n + n >= ((int64_t)1 << 31)) return fail(c, FEPIC_E_ARG, "too many particles for one species");
    if ((rc = ensure_capacity(c, s, s.n + n))) return rc;
    const size_t per = 7 * sizeof(double);  // x[3], u[3], id
    if (n > c->stage_cap) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->h_stage) (void)hipHostFree(c->h_stage);
        dfree(c, c->d_stage);
        const int64_t cap = std::max<int64_t>(n, 4096);
        if (hipHostMalloc(&c->h_stage, per * cap) != hipSuccess) return fail(c, FEPIC_E_OOM, "pinned allocation");
        c->d_stage = dmalloc(c, per * cap);
        if (!c->d_stage) return fail(c, FEPIC_E_OOM, "device allocation failed");
        c->stage_cap = cap;
    }
    // the previous injection's copy must be done before the pinned buffer is reused
    if (c->stage_event_valid) HIPCHK(c, hipEventSynchronize(c->stage_event));
    double* hx = (double*)c->h_stage;
    double* hu = hx + 3 * n;
    int64_t* hid = (int64_t*)(hu + 3 * n);
    std::memcpy(hx, x, 24 * n);
    std::memcpy(hu, u, 24 * n);
    if (id) std::memcpy(hid, id, 8 * n);
    HIPCHK(c, hipMemcpyAsync(c->d_stage, c->h_stage, (id ? 7 : 6) * 8 * n, hipMemcpyHostToDevice, c->stream));
    if (!c->stage_event_valid) {
        HIPCHK(c, hipEventCreateWithFlags(&c->stage_event, hipEventDisableTiming));
        c->stage_event_valid = true;
    }
    HIPCHK(c, hipEventRecord(c->stage_event, c->stream));
    const double* dx = (const double*)c->d_stage;
    const double* du = dx + 3 * n;
    const int64_t* did = id ? (const int64_t*)(du + 3 * n) : nullptr;
    return inject_located(c, s, n, did, dx, du);
}

// Appends n particles read from device memory (x, u [n][3] FP64, id [n] or null) to
// species s: located on the device in stream order, sorted by the next step.
static int inject_located(fepic_ctx* c, Species& s, int64_t n, const int64_t* did, const double* dx,
                          const double* du) {
    const double* g = c->d_grid;
    if (c->opt.precision == FEPIC_ALL_FP64)
        launch_locate<double>(c->stream, n, dx, du, did, s.next_id, parr<double>(s, s.cur), s.n, c->d_grad64, c->d_r0,
                              c->d_cell_start, c->d_cell_tets, g, g + 3, c->d_grid_n, c->d_cnt);
    else
        launch_locate<float>(c->stream, n, dx, du, did, s.next_id, parr<float>(s, s.cur), s.n, c->d_grad64, c->d_r0,
                             c->d_cell_start, c->d_cell_tets, g, g + 3, c->d_grid_n, c->d_cnt);
    s.next_id += n;
    s.ab_fill_from = std::min(s.ab_fill_from, s.n);
    s.n += n;
    s.added = true;
    c->rho_valid = false;
    c->rG_levels = 0;
    return FEPIC_OK;
}

int fepic_inject_particles_device(fepic_ctx* c, int species, int64_t n, const int64_t* id, const double* x,
                                  const double* u) {
    NEED_DEV(c);
    if (species < 0 || species >= (int)c->species.size() || n < 0 || (n > 0 && (!x || !u)))
        return fail(c, FEPIC_E_ARG, "bad injection arguments");
    if (n == 0) return FEPIC_OK;
    Species& s = c->species[species];
    int rc = sync_counts(c);
    if (rc) return rc;
    if (s.n + n >= ((int64_t)1 << 31)) return fail(c, FEPIC_E_ARG, "too many particles for one species");
    if ((rc = ensure_capacity(c, s, s.n + n))) return rc;
    return inject_located(c, s, n, id, x, u);
}

int fepic_num_particles(fepic_ctx* c, int species, int64_t* n) {
    NEED_DEV(c);
    if (species < 0 || species >= (int)c->species.size() || !n) return FEPIC_E_ARG;
    int rc = sync_counts(c);
    if (rc) return rc;
    // count live entries on the device (dead ones stay until the next sort)
    Species& s = c->species[species];
    double live = 0.0;
    if (s.n) {
        launch_fill(c->stream, c->d_live, 1, 0.0);
        launch_count_live(c->stream, (const int32_t*)s.buf[s.cur][0], s.n, c->d_live);
        HIPCHK(c, hipMemcpyAsync(&live, c->d_live, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n = (int64_t)live;
    return FEPIC_OK;
}

int fepic_get_particles(fepic_ctx* c, int species, int64_t cap, int64_t* n, int64_t* id, double* x, double* u,
                        int32_t* tet, double* lambda) {
    NEED_DEV(c);
    if (species < 0 || species >= (int)c->species.size() || !n) return FEPIC_E_ARG;
    int rc = sync_counts(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Species& s = c->species[species];
    const int64_t N = s.n;
    std::vector<int32_t> ht(N);
    std::vector<int64_t> hid(N);
    std::vector<double> hv[6];
    for (auto& v : hv) v.resize(N);
    if (N) {
        HIPCHK(c, hipMemcpy(ht.data(), s.buf[s.cur][0], 4 * N, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hid.data(), cur_arr(s, 7), 8 * N, hipMemcpyDeviceToHost));
        for (int a = 1; a < 7; ++a) {
            if (c->opt.precision == FEPIC_ALL_FP64) {
                HIPCHK(c, hipMemcpy(hv[a - 1].data(), s.buf[s.cur][a], 8 * N, hipMemcpyDeviceToHost));
            } else {
                std::vector<float> f(N);
                HIPCHK(c, hipMemcpy(f.data(), s.buf[s.cur][a], 4 * N, hipMemcpyDeviceToHost));
                for (int64_t i = 0; i < N; ++i) hv[a - 1][i] = f[i];
            }
        }
    }
    const HostMesh& m = c->mesh;
    int64_t k = 0;
    for (int64_t i = 0; i < N && k < cap; ++i) {
        const int t = ht[i];
        if (t < 0) continue;
        const double l[4] = {1.0 - hv[0][i] - hv[1][i] - hv[2][i], hv[0][i], hv[1][i], hv[2][i]};
        if (id) id[k] = hid[i];
        if (tet) tet[k] = t;
        if (lambda)
            for (int j = 0; j < 4; ++j) lambda[4 * k + j] = l[j];
        if (u)
            for (int d = 0; d < 3; ++d) u[3 * k + d] = hv[3 + d][i];
        if (x)
            for (int d = 0; d < 3; ++d) {
                double v = 0.0;
                for (int j = 0; j < 4; ++j) v += l[j] * m.xyz[3 * m.tets[4 * t + j] + d];
                x[3 * k + d] = v;
            }
        ++k;
    }
    *n = k;
    return FEPIC_OK;
}

int fepic_init_electrostatic(fepic_ctx* c, double tol, int* iters) { return fepic::init_electrostatic(c, tol, iters); }

int fepic_step(fepic_ctx* c, double dt, double beta, double gamma, fepic_step_stats* out) {
    return do_step(c, dt, beta, gamma, out, true);
}

int fepic_push_particles(fepic_ctx* c, double dt, fepic_step_stats* out) { return do_step(c, dt, 0.25, 0.5, out, false); }


// Device edge vector -> caller's array in canonical edge order.
static int edge_out(fepic_ctx* c, const double* d, double* out) {
    const HostMesh& m = c->mesh;
    std::vector<double> v(m.n_edges);
    HIPCHK(c, hipMemcpy(v.data(), d, 8 * m.n_edges, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m.n_edges; ++i) out[i] = v[m.eperm[i]];
    return FEPIC_OK;
}

int fepic_get_fields(fepic_ctx* c, double* e, double* e_prev, double* b) {
    NEED_DEV(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc;
    if (e && (rc = edge_out(c, c->d_e, e))) return rc;
    if (e_prev && (rc = edge_out(c, c->d_ep, e_prev))) return rc;
    if (b) HIPCHK(c, hipMemcpy(b, c->d_b, 8 * c->mesh.n_faces, hipMemcpyDeviceToHost));
    return FEPIC_OK;
}

int fepic_keep_warm_start(fepic_ctx* c, int on) {
    NEED_DEV(c);
    c->keep_start = on != 0;
    return FEPIC_OK;
}

int fepic_get_warm_start(fepic_ctx* c, double* x0) {
    NEED_DEV(c);
    if (!x0) return fail(c, FEPIC_E_ARG, "null output");
    if (!c->d_x0keep) return fail(c, FEPIC_E_STATE, "no start kept (fepic_keep_warm_start, then a step)");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return edge_out(c, c->d_x0keep, x0);
}

int fepic_get_current(fepic_ctx* c, double* dG, double* G) {
    NEED_DEV(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc;
    if (dG && (rc = edge_out(c, c->d_dg, dG))) return rc;
    if (G && (rc = edge_out(c, c->d_G, G))) return rc;
    return FEPIC_OK;
}

int fepic_get_rho(fepic_ctx* c, double* rho) {
    NEED_DEV(c);
    if (!rho) return FEPIC_E_ARG;
    int rc = sync_counts(c);
    if (rc) return rc;
    compute_rho(c, c->d_n1);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(rho, c->d_n1, 8 * c->mesh.n_nodes, hipMemcpyDeviceToHost));
    return FEPIC_OK;
}

int fepic_diagnostics(fepic_ctx* c, fepic_step_stats* out) {
    NEED_DEV(c);
    int rc = sync_counts(c);
    if (rc) return rc;
    fepic_step_stats st;
    std::memset(&st, 0, sizeof(st));
    const bool keep = c->rho_valid;
    c->rho_valid = false;
    rc = run_diagnostics(c, &st, false, false);
    c->rho_valid = keep || c->rho_valid;
    st.step = c->step_count;
    st.t = c->time;
    if (out) *out = st;
    return rc;
}

// Checkpoint: "FEPICCK1", sizes, step/time, fields and histories, species and their
// particles (buffer in use, live entries only), then the warm-start network.
int fepic_save(fepic_ctx* c, const char* path) {
    NEED_DEV(c);
    if (!path) return FEPIC_E_ARG;
    int rc = sync_counts(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::FILE* f = std::fopen(path, "wb");
    if (!f) return fail(c, FEPIC_E_IO, std::string("cannot open ") + path);
    const HostMesh& m = c->mesh;
    bool ok = true;
    auto W = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
    W("FEPICCK2", 8);
    const int64_t hdr[6] = {m.n_nodes, m.n_tets, m.n_edges, m.n_faces, (int64_t)c->species.size(),
                            c->opt.precision};
    W(hdr, sizeof(hdr));
    W(&c->step_count, 8);
    W(&c->time, 8);
    std::vector<double> buf(std::max(m.n_edges, m.n_faces));
    auto dump = [&](const double* d, int64_t n) {
        if (hipMemcpy(buf.data(), d, 8 * n, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        W(buf.data(), 8 * n);
    };
    for (const double* d : {c->d_e, c->d_ep, c->d_ep2, c->d_dg, c->d_G}) dump(d, m.n_edges);
    dump(c->d_b, m.n_faces);
    dump(c->d_bp, m.n_faces);
    for (auto& s : c->species) {
        W(&s.q, 8);
        W(&s.m, 8);
        W(&s.w, 8);
        W(&s.n, 8);
        W(&s.next_id, 8);
        for (int a = 0; a < 8; ++a) {
            const size_t nb = array_bytes(c, a, s.n);
            std::vector<unsigned char> tmp(nb);
            if (nb && hipMemcpy(tmp.data(), cur_arr(s, a), nb, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
            W(tmp.data(), nb);
        }
    }
    if (ok) ok = mlp_save(c, f) == FEPIC_OK;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? FEPIC_OK : fail(c, FEPIC_E_IO, std::string("write failed: ") + path);
}

int fepic_load(fepic_ctx* c, const char* path) {
    NEED_DEV(c);
    ab_history_stale(c);
    if (!path) return FEPIC_E_ARG;
    int rc = sync_counts(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::FILE* f = std::fopen(path, "rb");
    if (!f) return fail(c, FEPIC_E_IO, std::string("cannot open ") + path);
    const HostMesh& m = c->mesh;
    bool ok = true;
    auto R = [&](void* p, size_t n) { ok = ok && std::fread(p, 1, n, f) == n; };
    char magic[8];
    R(magic, 8);
    int64_t hdr[6];
    R(hdr, sizeof(hdr));
    if (!ok || std::memcmp(magic, "FEPICCK2", 8) || hdr[0] != m.n_nodes || hdr[1] != m.n_tets ||
        hdr[2] != m.n_edges || hdr[3] != m.n_faces || hdr[4] != (int64_t)c->species.size() ||
        hdr[5] != c->opt.precision) {
        std::fclose(f);
        return fail(c, FEPIC_E_IO, "checkpoint does not match this context (mesh, species or precision)");
    }
    R(&c->step_count, 8);
    R(&c->time, 8);
    std::vector<double> buf(std::max(m.n_edges, m.n_faces));
    auto fill = [&](double* d, int64_t n) {
        R(buf.data(), 8 * n);
        if (ok && hipMemcpy(d, buf.data(), 8 * n, hipMemcpyHostToDevice) != hipSuccess) ok = false;
    };
    for (double* d : {c->d_e, c->d_ep, c->d_ep2, c->d_dg, c->d_G}) fill(d, m.n_edges);
    fill(c->d_b, m.n_faces);
    fill(c->d_bp, m.n_faces);
    for (auto& s : c->species) {
        double q, mm, w;
        int64_t n, next_id;
        R(&q, 8);
        R(&mm, 8);
        R(&w, 8);
        R(&n, 8);
        R(&next_id, 8);
        if (!ok || q != s.q || mm != s.m || w != s.w || n < 0) {
            std::fclose(f);
            return fail(c, FEPIC_E_IO, "checkpoint species differ from this context's");
        }
        if ((rc = ensure_capacity(c, s, n))) {
            std::fclose(f);
            return rc;
        }
        for (int a = 0; a < 8; ++a) {
            const size_t nb = array_bytes(c, a, n);
            std::vector<unsigned char> tmp(nb);
            R(tmp.data(), nb);
            if (ok && nb && hipMemcpy(cur_arr(s, a), tmp.data(), nb, hipMemcpyHostToDevice) != hipSuccess) ok = false;
        }
        s.n = n;
        s.next_id = next_id;
        s.sorted_pending = false;
    }
    if (ok) ok = mlp_load(c, f) == FEPIC_OK;
    std::fclose(f);
    c->rho_valid = false;
    c->rG_levels = 0;
    return ok ? FEPIC_OK : fail(c, FEPIC_E_IO, std::string("read failed: ") + path);
}

int fepic_kernel_timing(fepic_ctx* c, const char* family, int enable) {
    if (!c || !family) return FEPIC_E_ARG;
    if (c->host_only) return fail(c, FEPIC_E_NO_DEVICE, "host-only context");
    for (int f = 0; f < FAM_COUNT; ++f)
        if (!std::strcmp(family, kFamilies[f])) {
            KernelTimer& k = c->timers[f];
            HIPCHK(c, hipStreamSynchronize(c->stream));
            k.on = enable != 0;
            k.used = 0;
            k.launches = 0;
            // pre-create events so the timed region does not create them
            while ((int64_t)k.ev.size() < 2 * (int64_t)std::max(enable, 0)) {
                hipEvent_t e;
                HIPCHK(c, hipEventCreate(&e));
                k.ev.push_back(e);
            }
            return FEPIC_OK;
        }
    return fail(c, FEPIC_E_ARG, std::string("unknown kernel family ") + family);
}

int fepic_kernel_time(fepic_ctx* c, const char* family, double* total_ms, int64_t* launches) {
    if (!c || !family) return FEPIC_E_ARG;
    if (c->host_only) return fail(c, FEPIC_E_NO_DEVICE, "host-only context");
    for (int f = 0; f < FAM_COUNT; ++f)
        if (!std::strcmp(family, kFamilies[f])) {
            KernelTimer& k = c->timers[f];
            HIPCHK(c, hipStreamSynchronize(c->stream));
            double tot = 0.0;
            for (int64_t i = 0; i + 1 < k.used; i += 2) {
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, k.ev[i], k.ev[i + 1]));
                tot += ms;
            }
            if (total_ms) *total_ms = tot;
            if (launches) *launches = k.launches;
            return FEPIC_OK;
        }
    return fail(c, FEPIC_E_ARG, std::string("unknown kernel family ") + family);
}

}  // extern "C"
