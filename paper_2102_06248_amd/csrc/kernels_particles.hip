// Particle-side kernels for gfx950: per-tet field staging, the particle step (gather ->
// relativistic Boris -> straight-path tracking -> Whitney-1 deposit) as one kernel, or as a
// first-piece kernel for every particle plus a kernel for the compacted face-crossing
// paths when few particles cross, point location, counting sort by tet, nodal charge,
// energies.
//
// Wave64 throughout; particles are kept sorted by tet so that lanes of a wave read the
// same 128-byte tet record and the current of their first path piece can be summed
// across the wave; per-workgroup LDS tables then merge the currents per edge before the
// FP64 atomics.
#include <algorithm>

#include "fepic_internal.h"
#include "fixed_point.h"

namespace fepic {

int grid_1d(int64_t n, int block) { return (int)((n + block - 1) / block); }

namespace {

constexpr int kBlock = 256;
constexpr int LE_A[6] = {0, 0, 0, 1, 1, 2};
constexpr int LE_B[6] = {1, 2, 3, 2, 3, 3};

// a / sqrt(x) and a / x: for FP32 particles by the hardware's reciprocal square root and
// reciprocal (about 1 ulp, no range scaling or refinement steps), for FP64 ones correctly
// rounded
template <typename T>
__device__ __forceinline__ T div_sqrt(T a, T x);
template <>
__device__ __forceinline__ float div_sqrt<float>(float a, float x) { return a * __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double div_sqrt<double>(double a, double x) { return a / __builtin_sqrt(x); }
template <typename T>
__device__ __forceinline__ T tdiv(T a, T x);
template <>
__device__ __forceinline__ float tdiv<float>(float a, float x) { return a * __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double tdiv<double>(double a, double x) { return a / x; }

__device__ __forceinline__ void atomic_add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// ------------------------------------------------------------------------- staging
// B in a tet from its four face fluxes: sum_k b_k W2_k evaluated at the centroid
// (lambda = 1/4), i.e. sum_k b_k * 1/2 (g_j x g_l + g_l x g_i + g_i x g_j) for face
// k = (i,j,l).  For a divergence-free flux the Whitney-2 field is constant in the tet.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stage(int64_t n_tets, TetBlock<T>* __restrict__ blk,
                                                   const double* __restrict__ e, const double* __restrict__ b,
                                                   const double* __restrict__ grad64,
                                                   const int32_t* __restrict__ tet_edges,
                                                   const int32_t* __restrict__ tet_faces) {
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_tets) return;
    TetBlock<T>* B = blk + t;
#pragma unroll
    for (int i = 0; i < 6; ++i) B->e[i] = (T)e[tet_edges[6 * t + i]];
    double g[4][3];
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = grad64[9 * t + 3 * (k - 1) + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    constexpr int F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    double Bv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double* gi = g[F[k][0]];
        const double* gj = g[F[k][1]];
        const double* gl = g[F[k][2]];
        double bf = 0.5 * b[tet_faces[4 * t + k]];
        Bv[0] += bf * ((gj[1] * gl[2] - gj[2] * gl[1]) + (gl[1] * gi[2] - gl[2] * gi[1]) + (gi[1] * gj[2] - gi[2] * gj[1]));
        Bv[1] += bf * ((gj[2] * gl[0] - gj[0] * gl[2]) + (gl[2] * gi[0] - gl[0] * gi[2]) + (gi[2] * gj[0] - gi[0] * gj[2]));
        Bv[2] += bf * ((gj[0] * gl[1] - gj[1] * gl[0]) + (gl[0] * gi[1] - gl[1] * gi[0]) + (gi[0] * gj[1] - gi[1] * gj[0]));
    }
    B->B[0] = (T)Bv[0];
    B->B[1] = (T)Bv[1];
    B->B[2] = (T)Bv[2];
}

// ------------------------------------------------------------------------- particle step
template <typename T>
__device__ __forceinline__ void load_grads(const TetBlock<T>* bp, T g[4][3]) {
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = bp->gl[3 * (k - 1) + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
}

// Whitney-1 path integral of one straight piece from barycentric point s to e inside a
// tet: for edge (a,b), int (lambda_a d lambda_b - lambda_b d lambda_a) = s_a e_b - e_a s_b
// (the integrand is constant along a line).
__device__ __forceinline__ void piece_current(double qw, const double s[4], const double e[4], double out[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) out[i] = qw * (s[LE_A[i]] * e[LE_B[i]] - e[LE_A[i]] * s[LE_B[i]]);
}

__device__ __forceinline__ double pick4(int idx, const double v[4]) {
    double r = v[3];
    r = (idx == 2) ? v[2] : r;
    r = (idx == 1) ? v[1] : r;
    r = (idx == 0) ? v[0] : r;
    return r;
}

// First exit of a straight piece from barycentric point ls along dl (d lambda over the
// rest of the step): the smallest ls_k / (-dl_k) over faces with dl_k < 0, other than the
// entry face; kb = -1 if the piece ends inside (t* >= 1).  Ties go to the smallest k.
// The candidates are compared as fractions with positive denominators, by cross products
// against the best so far (bn / bd, starting at 1 / 1), and only the winner's quotient is
// divided out: one FP64 division per exit instead of one per candidate face.
__device__ __forceinline__ void exit_search(const double ls[4], const double dl[4], int entry, double& best,
                                            int& kb) {
    double bn = 1.0, bd = 1.0;
    kb = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double d = -dl[k];
        if (k != entry && d > 0.0 && ls[k] * bd < bn * d) {
            bn = ls[k];
            bd = d;
            kb = k;
        }
    }
    best = 1.0;
    if (kb >= 0) best = bn / bd;
}

// Barycentric coordinates in the neighbour across the face opposite local kb, whose far
// vertex is its local q: shared vertices keep their relative order (both tets are sorted
// by node id), so new local k != q takes old local index r + (r >= kb), r = k - (k > q).
__device__ __forceinline__ void enter_neighbour(const double le[4], int kb, int q, double ln[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = k - (k > q ? 1 : 0);
        ln[k] = (k == q) ? 0.0 : pick4(r + (r >= kb ? 1 : 0), le);
    }
}

template <typename T>
__device__ __forceinline__ void path_step(const T g[4][3], const T dx[3], double frac, double dl[4]) {
#pragma unroll
    for (int k = 1; k < 4; ++k) dl[k] = frac * (double)(g[k][0] * dx[0] + g[k][1] * dx[1] + g[k][2] * dx[2]);
    dl[0] = -(dl[1] + dl[2] + dl[3]);
}

// End point of the last piece, rounded to storage precision (clamped at 0) before the
// piece's current is formed, so the stored state and the deposit agree exactly.
template <typename T>
__device__ __forceinline__ void end_point(const double ls[4], const double dl[4], T r[3], double le[4]) {
    r[0] = (T)fmax(ls[1] + dl[1], 0.0);
    r[1] = (T)fmax(ls[2] + dl[2], 0.0);
    r[2] = (T)fmax(ls[3] + dl[3], 0.0);
    le[1] = (double)r[0];
    le[2] = (double)r[1];
    le[3] = (double)r[2];
    le[0] = 1.0 - le[1] - le[2] - le[3];
}

// Counters: summed across the wave, then across the workgroup in LDS; one thread adds the
// workgroup's totals into one of kCntSlots slots (so no single address takes an atomic
// from every wave); k_cnt_finish folds the slots afterwards.  Every thread must call it.
template <int kB = kBlock>
__device__ __forceinline__ void add_counters(unsigned int sc, unsigned int mc, unsigned int na, unsigned int ncap,
                                             PushCounters* __restrict__ cnt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sc += __shfl_xor(sc, off);
        mc = max(mc, (unsigned int)__shfl_xor(mc, off));
        na += __shfl_xor(na, off);
        ncap += __shfl_xor(ncap, off);
    }
    __shared__ unsigned int s_cnt[kB / 64][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_cnt[w][0] = sc;
        s_cnt[w][1] = mc;
        s_cnt[w][2] = na;
        s_cnt[w][3] = ncap;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int tc = 0, tm = 0, ta = 0, tp = 0;
#pragma unroll
        for (int k = 0; k < kB / 64; ++k) {
            tc += s_cnt[k][0];
            tm = max(tm, s_cnt[k][1]);
            ta += s_cnt[k][2];
            tp += s_cnt[k][3];
        }
        PushCounters* slot = cnt + (blockIdx.x & (kCntSlots - 1));
        if (tc) atomicAdd(&slot->n_crossings, (unsigned long long)tc);
        if (tm) atomicMax(&slot->max_crossings, tm);
        if (ta) atomicAdd(&slot->n_absorbed, ta);
        if (tp) atomicAdd(&slot->n_cap, tp);
    }
}

// Per-workgroup accumulation of edge currents in LDS: an open-addressed table of 2^kBits
// slots keyed by edge id (linear probing, insertion by compare-and-swap), flushed with one
// FP64 global atomic per distinct edge.  An insert that finds no slot within kProbe steps
// goes to global memory directly.
constexpr int kProbe = 16;

// Kernels that walk paths keep their registers within what 6 waves per SIMD allow in FP32
// (80 VGPRs; the fused push needs 81 unconstrained, and 6 workgroups of it fit one CU's
// LDS): the exit searches and LDS round trips of a walk are latency bound, so the extra
// wave pays more than the registers it costs.  The FP64 forms (validation precision) hold
// 5, where they do not spill.
template <typename T>
constexpr int walk_waves() { return sizeof(T) == 4 ? 6 : 5; }

// The six edge currents of one piece: the first probe of all six keys is issued at once,
// so one LDS round trip serves the common case; keys whose first slot holds another edge
// probe on.  A slot's key is read before it is claimed: a slot, once claimed, keeps its
// key, and lanes of a wave that add to the same edges then share one broadcast read
// instead of serialising on compare-and-swaps of one address.
template <int kBits>
__device__ __forceinline__ void lds_add6(int* s_key, double* s_val, double* __restrict__ dg, const int32_t* e,
                                         const double v[6]) {
    int key[6], got[6];
    unsigned int h[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        key[c] = e[c];
        h[c] = ((unsigned int)key[c] * 2654435761u) >> (32 - kBits);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c)
        got[c] = (v[c] != 0.0) ? __hip_atomic_load(s_key + h[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : key[c];
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (got[c] == -1) got[c] = atomicCAS(s_key + h[c], -1, key[c]);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (v[c] == 0.0) continue;
        if (got[c] == -1 || got[c] == key[c]) {
            __hip_atomic_fetch_add(s_val + h[c], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            // probe on from the next slot
            unsigned int hh = (h[c] + 1) & ((1u << kBits) - 1u);
            bool placed = false;
            for (int p = 1; p < kProbe && !placed; ++p) {
                int k = __hip_atomic_load(s_key + hh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (k == -1) k = atomicCAS(s_key + hh, -1, key[c]);
                if (k == -1 || k == key[c]) {
                    __hip_atomic_fetch_add(s_val + hh, v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    placed = true;
                }
                hh = (hh + 1) & ((1u << kBits) - 1u);
            }
            if (!placed) atomic_add_f64(dg + key[c], v[c]);
        }
    }
}

constexpr int log2_const(int v) { return v <= 1 ? 0 : 1 + log2_const(v / 2); }

// Segmented inclusive sums across the wave of N doubles, a segment starting at every lane
// with f != 0 (lane 0 always starts one): after it, the last lane of each segment holds the
// segment's sum.  Steps of the Hillis-Steele scan by DPP moves: row shifts by 1, 2, 4 and 8
// inside each row of 16 lanes, then the rows' running sums carried across by broadcasting
// lane 15 (into rows 1 and 3) and lane 31 (into rows 2 and 3).  Lanes without a source
// receive zeros, which neither add nor end a segment.  VALU moves, where shuffles would
// be LDS permutes.  Every lane of the wave must take part.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xf, true);
}

template <int N, int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_step(double v[N], int& f) {
    double o[N];
#pragma unroll
    for (int c = 0; c < N; ++c)
        o[c] = __hiloint2double(dpp_i32<kCtrl, kRowMask>(__double2hiint(v[c])),
                                dpp_i32<kCtrl, kRowMask>(__double2loint(v[c])));
    const int fo = dpp_i32<kCtrl, kRowMask>(f);
    if (!f) {
#pragma unroll
        for (int c = 0; c < N; ++c) v[c] += o[c];
    }
    f |= fo;
}

template <int N>
__device__ __forceinline__ void seg_sum_wave(double v[N], int f) {
    seg_step<N, 0x111, 0xf>(v, f);   // row_shr:1
    seg_step<N, 0x112, 0xf>(v, f);   // row_shr:2
    seg_step<N, 0x114, 0xf>(v, f);   // row_shr:4
    seg_step<N, 0x118, 0xf>(v, f);   // row_shr:8
    seg_step<N, 0x142, 0xa>(v, f);   // row_bcast:15
    seg_step<N, 0x143, 0xc>(v, f);   // row_bcast:31
}

// The six edge currents of one piece into the deterministic mode's accumulators.
__device__ __forceinline__ void fix_add6(const PushParams& pp, const int32_t* e, const double v[6]) {
#pragma unroll
    for (int c = 0; c < 6; ++c) fix_add(pp.fix, e[c], v[c], pp.fix_inv);
}

// One FP64 atomic per occupied slot of the table (after a barrier).
template <int kSlots, int kB>
__device__ __forceinline__ void flush_table(const int* s_key, const double* s_val, double* __restrict__ dg) {
    for (int k = threadIdx.x; k < kSlots; k += kB)
        if (s_key[k] >= 0) atomic_add_f64(dg + s_key[k], s_val[k]);
}

// The rest of one particle's path after its first face crossing: from barycentric ls in
// tet t (entered through local face `entry`) with the remaining fraction frac of the
// displacement dx, tet by tet up to the end point or a wall, each piece's current into the
// workgroup's LDS table.  nc counts the particle's crossings (1 on entry); na and ncap
// count an absorption and a stop at the crossing cap.
template <typename T, int kBits, bool kDet = false>
__device__ __forceinline__ void walk_rest(PArrays<T>& out, int64_t i, int t, int entry, double ls[4], double frac,
                                          const T dx[3], const TetBlock<T>* __restrict__ blk, double* __restrict__ dg,
                                          const PushParams& pp, int* s_key, double* s_val, unsigned int& nc,
                                          unsigned int& na, unsigned int& ncap) {
    const TetBlock<T>* bp = blk + t;
    T g[4][3];
    load_grads(bp, g);
    double dl[4];
    path_step(g, dx, frac, dl);
    nc = 1;
    for (;;) {
        double best;
        int kb;
        exit_search(ls, dl, entry, best, kb);
        double le[4], cur[6];
        if (kb < 0) {
            T rr[3];
            end_point(ls, dl, rr, le);
            piece_current(pp.qw, ls, le, cur);
            if constexpr (kDet) fix_add6(pp, bp->edge, cur);
            else lds_add6<kBits>(s_key, s_val, dg, bp->edge, cur);
            out.tet[i] = t;
            out.l1[i] = rr[0];
            out.l2[i] = rr[1];
            out.l3[i] = rr[2];
            return;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) le[k] = (k == kb) ? 0.0 : ls[k] + best * dl[k];
        piece_current(pp.qw, ls, le, cur);
        if constexpr (kDet) fix_add6(pp, bp->edge, cur);
        else lds_add6<kBits>(s_key, s_val, dg, bp->edge, cur);
        const int nb = bp->nbr[kb];
        if (nb < 0) {
            ++na;
            out.tet[i] = -1;
            return;
        }
        if (++nc > (unsigned)pp.cap) {
            ++ncap;
            out.tet[i] = -1;
            return;
        }
        const int q = nb & 3;
        double ln[4];
        enter_neighbour(le, kb, q, ln);
        frac *= (1.0 - best);
        t = nb >> 2;
        bp = blk + t;
        load_grads(bp, g);
        path_step(g, dx, frac, dl);
#pragma unroll
        for (int k = 0; k < 4; ++k) ls[k] = ln[k];
        entry = q;
    }
}

// The particle step: gather E and B in the particle's tet, relativistic Boris, and the
// straight path up to its first face crossing (or its end).  With kFused the crossing
// paths are walked to their end here; otherwise they are compacted, per workgroup, into
// the crossing queue (slots blockIdx * kBlock + rank, count in wg_count) and finished by
// k_cross, their u and id being final here.  First-piece currents are summed over runs of
// lanes that share a tet (the particles are sorted by tet); in the fused form the run sums
// and walk pieces go through the workgroup's LDS table, flushed with one FP64 atomic per
// edge, in the queue form each run adds its six sums with FP64 atomics.  kDet (fused form
// only): every lane adds its own pieces to the fixed-point accumulators, no table.
template <typename T, bool kFused, int kPB, bool kDet = false>
__global__ __launch_bounds__(kPB) __attribute__((amdgpu_waves_per_eu(kFused ? walk_waves<T>() : 1, 8))) void k_push(PArrays<T> in, PArrays<T> out, int64_t n,
                                                  const TetBlock<T>* __restrict__ blk, double* __restrict__ dg,
                                                  PushParams pp, PushCounters* __restrict__ cnt,
                                                  const int32_t* __restrict__ n_live, CrossQueue<T> cq) {
    // the LDS table of the fused form (the queue form leaves it to k_cross: its 24 KB
    // would cost the first kernel occupancy)
    static_assert(kFused || kPB == kBlock, "the queue form fills regions of kBlock slots");
    static_assert(kFused || !kDet, "the deterministic form walks in place");
    constexpr bool kTable = kFused && !kDet;
    constexpr int kBits = log2_const(8 * kPB);
    constexpr int kSlots = kTable ? (1 << kBits) : 1;
    __shared__ int s_key[kSlots];
    __shared__ double s_val[kSlots];
    if (kTable) {
        for (int k = threadIdx.x; k < kSlots; k += kPB) {
            s_key[k] = -1;
            s_val[k] = 0.0;
        }
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (n_live) n = min(n, (int64_t)*n_live);
    // the particle's own words are loaded together with its tet index (one memory round
    // trip before the tet record's), whether or not the particle is live
    int t0 = -1;
    T l1 = T(0), l2 = T(0), l3 = T(0), u[3] = {T(0), T(0), T(0)};
    if (i < n) {
        t0 = in.tet[i];
        l1 = in.l1[i];
        l2 = in.l2[i];
        l3 = in.l3[i];
        u[0] = in.u0[i];
        u[1] = in.u1[i];
        u[2] = in.u2[i];
    }
    double first[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int status = 0;       // 1 absorbed, 2 crossing cap
    bool cross = false;   // continues in k_cross
    double ln[4] = {0.0, 0.0, 0.0, 0.0}, frac = 0.0;
    T dx[3] = {T(0), T(0), T(0)};
    int tn = 0, q = 0;
    int o_tet = -1;       // the slot's tet after this kernel
    if (t0 >= 0) {
        const TetBlock<T>* bp = blk + t0;
        T g[4][3];
        load_grads(bp, g);
        // gather: E = sum over edges e_ab (lambda_a grad l_b - lambda_b grad l_a)
        const T lam[4] = {T(1) - l1 - l2 - l3, l1, l2, l3};
        T E[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const T ek = bp->e[k];
            const int a = LE_A[k], b = LE_B[k];
#pragma unroll
            for (int d = 0; d < 3; ++d) E[d] += ek * (lam[a] * g[b][d] - lam[b] * g[a][d]);
        }
        const T Bv[3] = {bp->B[0], bp->B[1], bp->B[2]};
        // relativistic Boris: half kick, rotation, half kick
        const T h = (T)pp.qm_half_dt;
        const T ic2 = (T)(1.0 / (kC * kC));
        T um[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
        const T hg = div_sqrt<T>(h, T(1) + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]) * ic2);
        const T tv[3] = {hg * Bv[0], hg * Bv[1], hg * Bv[2]};
        const T s2 = tdiv<T>(T(2), T(1) + tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
        const T up[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]), um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                         um[2] + (um[0] * tv[1] - um[1] * tv[0])};
        u[0] = um[0] + s2 * (up[1] * tv[2] - up[2] * tv[1]) + h * E[0];
        u[1] = um[1] + s2 * (up[2] * tv[0] - up[0] * tv[2]) + h * E[1];
        u[2] = um[2] + s2 * (up[0] * tv[1] - up[1] * tv[0]) + h * E[2];
        const T ginv = div_sqrt<T>(T(1), T(1) + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * ic2);
        const T dtt = (T)pp.dt;
        dx[0] = dtt * u[0] * ginv;
        dx[1] = dtt * u[1] * ginv;
        dx[2] = dtt * u[2] * ginv;

        // path in barycentric coordinates of the tet; exit points kept in FP64
        const double ls[4] = {1.0 - (double)l1 - (double)l2 - (double)l3, (double)l1, (double)l2, (double)l3};
        double dl[4];
        path_step(g, dx, 1.0, dl);
        double best;
        int kb;
        exit_search(ls, dl, -1, best, kb);
        double le[4];
        if (kb < 0) {
            T r[3];
            end_point(ls, dl, r, le);
            piece_current(pp.qw, ls, le, first);
            o_tet = t0;
            l1 = r[0];
            l2 = r[1];
            l3 = r[2];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) le[k] = (k == kb) ? 0.0 : ls[k] + best * dl[k];
            piece_current(pp.qw, ls, le, first);
            const int nb = bp->nbr[kb];
            if (nb < 0) {           // wall: absorbed after depositing up to it
                status = 1;
            } else if (pp.cap < 1) {
                status = 2;
            } else {
                cross = true;
                tn = nb >> 2;
                q = nb & 3;
                enter_neighbour(le, kb, q, ln);
                frac = 1.0 - best;
                o_tet = tn;
            }
        }
    }
    // every lane writes all six words of its slot and its tet, so that each store covers
    // whole cache lines: a path that goes on into another tet has its end written later (in
    // k_cross, or by the walk below); an absorbed or dead particle's words other than its
    // tet (-1) are never read.  The slot's id is kept: ids are not copied.
    if (i < n) {
        out.tet[i] = o_tet;
        out.l1[i] = l1;
        out.l2[i] = l2;
        out.l3[i] = l3;
        out.u0[i] = u[0];
        out.u1[i] = u[1];
        out.u2[i] = u[2];
    }

    // first-piece currents: one sum per run of lanes sharing a tet, added by the run's last
    // lane (fused form: into the workgroup's LDS table, where runs of neighbouring tets and
    // the walks share edges; queue form: six FP64 atomics); deterministic form: each lane's
    // own, exactly
    if constexpr (kDet) {
        if (t0 >= 0) fix_add6(pp, blk[t0].edge, first);
    } else {
        const int key = t0;
        const int prev_key = __shfl_up(key, 1);
        seg_sum_wave<6>(first, (lane == 0) || (key != prev_key));
        const int next_key = __shfl_down(key, 1);
        if (key >= 0 && (lane == 63 || next_key != key)) {
            if (kTable) {
                lds_add6<kBits>(s_key, s_val, dg, blk[key].edge, first);
            } else {
                const TetBlock<T>* bk = blk + key;
#pragma unroll
                for (int c = 0; c < 6; ++c) atomic_add_f64(dg + bk->edge[c], first[c]);
            }
        }
    }

    if (kFused) {
        // the rest of every crossing path here, currents through the LDS table
        unsigned int nc = 0, na = 0, ncap = 0;
        if (cross) walk_rest<T, kBits, kDet>(out, i, tn, q, ln, frac, dx, blk, dg, pp, s_key, s_val, nc, na, ncap);
        if constexpr (!kDet) {
            __syncthreads();
            flush_table<kSlots, kPB>(s_key, s_val, dg);
        }
        const unsigned int c1 = (cross || status == 2) ? 1u : 0u;
        const unsigned int sc = cross ? nc : c1;
        add_counters<kPB>(sc, sc, (status == 1) + na, (status == 2) + ncap, cnt);
        return;
    }
    // compact the crossing lanes of the workgroup into its queue region; the counters here
    // are flags (a path crossed, was absorbed, stopped at the cap), counted by ballots and
    // summed over the workgroup's waves in the same LDS exchange as the queue offsets
    {
        __shared__ int s_wc[kBlock / 64][3];
        const int w = threadIdx.x >> 6;
        const unsigned long long m = __ballot(cross);
        const unsigned long long m_abs = __ballot(status == 1);
        const unsigned long long m_cap = __ballot(status == 2);
        if (lane == 0) {
            s_wc[w][0] = (int)__popcll(m);
            s_wc[w][1] = (int)__popcll(m_abs);
            s_wc[w][2] = (int)__popcll(m_cap);
        }
        __syncthreads();
        int base = 0, total = 0;
#pragma unroll
        for (int k = 0; k < kBlock / 64; ++k) {
            base += (k < w) ? s_wc[k][0] : 0;
            total += s_wc[k][0];
        }
        if (cross) {
            const int64_t slot =
                (int64_t)blockIdx.x * kBlock + base + (int)__popcll(m & ((1ull << lane) - 1ull));
            cq.l0[slot] = ln[0];
            cq.l1[slot] = ln[1];
            cq.l2[slot] = ln[2];
            cq.l3[slot] = ln[3];
            cq.frac[slot] = frac;
            cq.dx0[slot] = dx[0];
            cq.dx1[slot] = dx[1];
            cq.dx2[slot] = dx[2];
            cq.idx[slot] = (int32_t)i;
            cq.tet[slot] = tn;
            cq.entry[slot] = q;
        }
        if (threadIdx.x == 0) {
            cq.wg_count[blockIdx.x] = total;
            unsigned int ta = 0, tp = 0;
#pragma unroll
            for (int k = 0; k < kBlock / 64; ++k) {
                ta += s_wc[k][1];
                tp += s_wc[k][2];
            }
            // a refused crossing (the cap) counts as a crossing, as in k_cross
            const unsigned int tc = (unsigned int)total + tp;
            PushCounters* slot = cnt + (blockIdx.x & (kCntSlots - 1));
            if (tc) {
                atomicAdd(&slot->n_crossings, (unsigned long long)tc);
                atomicMax(&slot->max_crossings, 1u);
            }
            if (ta) atomicAdd(&slot->n_absorbed, ta);
            if (tp) atomicAdd(&slot->n_cap, tp);
        }
    }
}


// The rest of the paths that crossed a face in k_push: workgroup b takes the queue region
// of k_push workgroup b (up to 256 particles) with kB threads and walks each particle tet
// by tet, up to the end point or a wall.  Piece currents are summed per edge in an LDS
// table of 8 kB slots, then added to global memory once per edge.  kB is chosen from the
// expected share of crossing particles, so most threads have one particle.
template <typename T, int kB>
__global__ __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(walk_waves<T>(), 8))) void k_cross(PArrays<T> out, CrossQueue<T> cq, const TetBlock<T>* __restrict__ blk,
                                              double* __restrict__ dg, PushParams pp,
                                              PushCounters* __restrict__ cnt) {
    constexpr int kBits = log2_const(8 * kB);
    constexpr int kSlots = 1 << kBits;
    __shared__ int s_key[kSlots];
    __shared__ double s_val[kSlots];
    // an empty queue region (no path of the first kernel's workgroup crossed a face) has
    // nothing to walk, deposit or count: the whole workgroup leaves before the table
    const int total = cq.wg_count[blockIdx.x];
    if (total == 0) return;
    for (int k = threadIdx.x; k < kSlots; k += kB) {
        s_key[k] = -1;
        s_val[k] = 0.0;
    }
    __syncthreads();
    unsigned int sc = 0, mc = 0, na = 0, ncap = 0;
    for (int j = threadIdx.x; j < total; j += kB) {
        const int64_t slot = (int64_t)blockIdx.x * kBlock + j;
        const int64_t i = cq.idx[slot];
        double ls[4] = {cq.l0[slot], cq.l1[slot], cq.l2[slot], cq.l3[slot]};
        const T dx[3] = {cq.dx0[slot], cq.dx1[slot], cq.dx2[slot]};
        unsigned int nc = 0;
        walk_rest<T, kBits>(out, i, cq.tet[slot], cq.entry[slot], ls, cq.frac[slot], dx, blk, dg, pp, s_key, s_val, nc,
                            na, ncap);
        sc += nc - 1;
        mc = max(mc, nc);
    }
    __syncthreads();
    flush_table<kSlots, kB>(s_key, s_val, dg);
    add_counters<kB>(sc, mc, na, ncap, cnt);
}

// The same walks for a species whose paths rarely cross a face (most queue regions empty):
// a resident grid of one-wave workgroups, each taking a contiguous run of regions 64 at a
// time, one region per lane: a lane walks the paths of its region (none, mostly), so the
// few paths of 64 regions are walked side by side.  All go through one LDS table per
// workgroup, flushed at the end (a dispatch per region would cost more than the walks).
template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(walk_waves<T>(), 8))) void k_cross_sparse(
    PArrays<T> out, CrossQueue<T> cq, int64_t n_regions, const TetBlock<T>* __restrict__ blk, double* __restrict__ dg,
    PushParams pp, PushCounters* __restrict__ cnt) {
    constexpr int kB = 64;
    constexpr int kBits = log2_const(8 * kB);
    constexpr int kSlots = 1 << kBits;
    __shared__ int s_key[kSlots];
    __shared__ double s_val[kSlots];
    for (int k = threadIdx.x; k < kSlots; k += kB) {
        s_key[k] = -1;
        s_val[k] = 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x;
    const int64_t per = (n_regions + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n_regions, r0 + per);
    unsigned int sc = 0, mc = 0, na = 0, ncap = 0;
    for (int64_t base = r0; base < r1; base += kB) {
        const int64_t b = base + lane;
        const int total = b < r1 ? cq.wg_count[b] : 0;
        for (int j = 0; j < total; ++j) {
            const int64_t slot = b * kBlock + j;
            const int64_t i = cq.idx[slot];
            double ls[4] = {cq.l0[slot], cq.l1[slot], cq.l2[slot], cq.l3[slot]};
            const T dx[3] = {cq.dx0[slot], cq.dx1[slot], cq.dx2[slot]};
            unsigned int nc = 0;
            walk_rest<T, kBits>(out, i, cq.tet[slot], cq.entry[slot], ls, cq.frac[slot], dx, blk, dg, pp, s_key, s_val,
                                nc, na, ncap);
            sc += nc - 1;
            mc = max(mc, nc);
        }
    }
    __syncthreads();
    flush_table<kSlots, kB>(s_key, s_val, dg);
    add_counters<kB>(sc, mc, na, ncap, cnt);
}

// Resident one-wave workgroups of k_cross_sparse: what the walk's register budget keeps on
// the 256 CUs (walk_waves waves on each of four SIMDs).
template <typename T>
constexpr unsigned sparse_grid() { return 256u * 4u * (unsigned)walk_waves<T>(); }

// Face crossings counted so far in this step (the slots' running sum) into out[0], and the
// absorptions plus paths stopped at the crossing cap into out[1].
__global__ __launch_bounds__(kCntSlots) void k_cnt_crossings(const PushCounters* __restrict__ slots,
                                                             unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_c[kCntSlots], s_a[kCntSlots];
    const int t = threadIdx.x;
    s_c[t] = slots[t].n_crossings;
    s_a[t] = (unsigned long long)slots[t].n_absorbed + slots[t].n_cap;
    __syncthreads();
    for (int h = kCntSlots / 2; h > 0; h >>= 1) {
        if (t < h) {
            s_c[t] += s_c[t + h];
            s_a[t] += s_a[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = s_c[0];
        out[1] = s_a[0];
    }
}

// Folds the per-slot push counters into *out and clears the slots for the next step.
__global__ __launch_bounds__(kCntSlots) void k_cnt_finish(PushCounters* __restrict__ slots,
                                                          PushCounters* __restrict__ out) {
    __shared__ unsigned long long s_c[kCntSlots];
    __shared__ unsigned int s_m[kCntSlots], s_a[kCntSlots], s_p[kCntSlots];
    const int t = threadIdx.x;
    PushCounters v = slots[t];
    s_c[t] = v.n_crossings;
    s_m[t] = v.max_crossings;
    s_a[t] = v.n_absorbed;
    s_p[t] = v.n_cap;
    slots[t] = PushCounters{};
    __syncthreads();
    for (int h = kCntSlots / 2; h > 0; h >>= 1) {
        if (t < h) {
            s_c[t] += s_c[t + h];
            s_m[t] = max(s_m[t], s_m[t + h]);
            s_a[t] += s_a[t + h];
            s_p[t] += s_p[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        PushCounters r{};
        r.n_crossings = s_c[0];
        r.max_crossings = s_m[0];
        r.n_absorbed = s_a[0];
        r.n_cap = s_p[0];
        *out = r;
    }
}

// ------------------------------------------------------------------------- locate
// Point location through a uniform bucket grid: the tet among the bucket's candidates
// whose smallest barycentric coordinate is largest, accepted if >= -1e-12.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_locate(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ u, const int64_t* __restrict__ id,
                                                    int64_t id_base, PArrays<T> out, int64_t out_off,
                                                    const double* __restrict__ grad64, const double* __restrict__ r0,
                                                    const int32_t* __restrict__ cell_start,
                                                    const int32_t* __restrict__ cell_tets,
                                                    const double* __restrict__ lo, const double* __restrict__ inv_h,
                                                    const int32_t* __restrict__ gn, PushCounters* cnt) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double px = x[3 * i], py = x[3 * i + 1], pz = x[3 * i + 2];
    const double ux = u[3 * i], uy = u[3 * i + 1], uz = u[3 * i + 2];
    int best_t = -1;
    double best_s = -1e300, bl[3] = {0.0, 0.0, 0.0};
    const bool finite = isfinite(px) && isfinite(py) && isfinite(pz) && isfinite(ux) && isfinite(uy) && isfinite(uz);
    if (finite) {
        int c[3];
        const double p[3] = {px, py, pz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double f = (p[d] - lo[d]) * inv_h[d];
            int ci = (int)floor(f);
            c[d] = ci < 0 ? 0 : (ci >= gn[d] ? gn[d] - 1 : ci);
        }
        const int cell = c[0] + gn[0] * (c[1] + gn[1] * c[2]);
        for (int j = cell_start[cell]; j < cell_start[cell + 1]; ++j) {
            const int t = cell_tets[j];
            const double* g = grad64 + 9 * t;
            const double dxv = px - r0[3 * t], dyv = py - r0[3 * t + 1], dzv = pz - r0[3 * t + 2];
            const double a1 = g[0] * dxv + g[1] * dyv + g[2] * dzv;
            const double a2 = g[3] * dxv + g[4] * dyv + g[5] * dzv;
            const double a3 = g[6] * dxv + g[7] * dyv + g[8] * dzv;
            const double a0 = 1.0 - a1 - a2 - a3;
            const double s = fmin(fmin(a0, a1), fmin(a2, a3));
            if (s > best_s) {
                best_s = s;
                best_t = t;
                bl[0] = a1;
                bl[1] = a2;
                bl[2] = a3;
            }
        }
    }
    const int64_t o = out_off + i;
    if (best_t < 0 || best_s < -1e-12) {
        out.tet[o] = -1;
        atomicAdd(&cnt->n_rejected, 1u);
        return;
    }
    out.tet[o] = best_t;
    out.l1[o] = (T)fmax(bl[0], 0.0);
    out.l2[o] = (T)fmax(bl[1], 0.0);
    out.l3[o] = (T)fmax(bl[2], 0.0);
    out.u0[o] = (T)ux;
    out.u1[o] = (T)uy;
    out.u2[o] = (T)uz;
    out.id[o] = id ? id[i] : id_base + i;
}

// ------------------------------------------------------------------------- counting sort
__global__ __launch_bounds__(kBlock) void k_zero_i32(int32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Lanes of a wave grouped by key, in any order: for each lane with key >= 0 its group's
// leader (lowest lane), its rank among the group's lanes and the group's size; one pass
// per distinct key.  Between sorts the particles stay nearly sorted, but those that
// crossed a face break the runs of equal tets, so grouping by key needs about half the
// atomics that one per run would.
__device__ __forceinline__ void key_groups(int key, int lane, int& leader, int& rank, int& size) {
    unsigned long long todo = __ballot(key >= 0);
    leader = lane;
    rank = 0;
    size = 0;
    while (todo) {
        const int l = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, l);
        const unsigned long long m = __ballot(key == k) & todo;
        if (key == k) {
            leader = l;
            rank = __popcll(m & ((1ull << lane) - 1ull));
            size = __popcll(m);
        }
        todo &= ~m;
    }
}

// count[t] += number of particles in t; one atomic per distinct tet in a wave.
__global__ __launch_bounds__(kBlock) void k_hist(const int32_t* __restrict__ tet, int64_t n, int32_t* count) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int t = i < n ? tet[i] : -1;
    int leader, rank, size;
    key_groups(t, lane, leader, rank, size);
    if (t >= 0 && lane == leader) atomicAdd(count + t, size);
}

// Block-wide exclusive scan of one value per thread (256 threads = 4 waves).
__device__ __forceinline__ int block_excl_scan(int v, int* s_w, int& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) base += (k < w) ? s_w[k] : 0;
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return x - v + base;
}

constexpr int kScanItems = 4;  // per thread; 1024 per block

__global__ __launch_bounds__(kBlock) void k_scan_blocks(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                         int64_t n, int32_t* __restrict__ block_sums) {
    __shared__ int s_w[4];
    const int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        sum += v[k];
    }
    int total;
    int run = block_excl_scan(sum, s_w, total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single block: exclusive scan of the block sums in place; total -> *n_total.
__global__ __launch_bounds__(kBlock) void k_scan_top(int32_t* block_sums, int64_t nb, int32_t* n_total) {
    __shared__ int s_w[4];
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t b0 = threadIdx.x * per;
    int sum = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) sum += block_sums[b0 + k];
    int total;
    int run = block_excl_scan(sum, s_w, total);
    for (int64_t k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            const int v = block_sums[b0 + k];
            block_sums[b0 + k] = run;
            run += v;
        }
    }
    if (threadIdx.x == 0) *n_total = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                      const int32_t* __restrict__ block_sums) {
    const int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kScanItems;
    const int add = block_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) out[base + k] += add;
}

// Each live particle to its place in its tet's range (offset[t], the exclusive scan of the
// counts, advanced as places are taken): the lanes of a wave in one tet take consecutive
// places, in lane order, reserved by one atomic; absorbed particles (t < 0) are dropped.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter(PArrays<T> in, PArrays<T> out, int64_t n,
                                                     int32_t* __restrict__ offset, AbHistIo ab) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int t = i < n ? in.tet[i] : -1;
    int leader, rank, size;
    key_groups(t, lane, leader, rank, size);
    // the group's leader reserves its places in t's range; lanes keep their order
    int base = 0;
    if (t >= 0 && lane == leader) base = atomicAdd(offset + t, size);
    base = __shfl(base, leader);
    if (t < 0) return;
    const int pos = base + rank;
    out.tet[pos] = t;
    out.l1[pos] = in.l1[i];
    out.l2[pos] = in.l2[i];
    out.l3[pos] = in.l3[i];
    out.u0[pos] = in.u0[i];
    out.u1[pos] = in.u1[i];
    out.u2[pos] = in.u2[i];
    out.id[pos] = in.id[i];
    if (ab.hin) {   // the Adams-Bashforth history moves with its particle
        ab.mout[pos] = ab.min[i];
        for (int c = 0; c < kAbStride; ++c) ab.hout[c * ab.stride + pos] = ab.hin[c * ab.stride + i];
    }
}

// ------------------------------------------------------------------------- charge
// One value into the workgroup's LDS table under key (linear probing, the key read before
// the slot is claimed); to global memory directly if no slot is found within kProbe.
template <int kBits>
__device__ __forceinline__ void lds_add1(int* s_key, double* s_val, double* __restrict__ out, int key, double v) {
    if (v == 0.0) return;
    unsigned int h = ((unsigned int)key * 2654435761u) >> (32 - kBits);
    for (int p = 0; p < kProbe; ++p) {
        int k = __hip_atomic_load(s_key + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == -1) k = atomicCAS(s_key + h, -1, key);
        if (k == -1 || k == key) {
            __hip_atomic_fetch_add(s_val + h, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        h = (h + 1) & ((1u << kBits) - 1u);
    }
    atomic_add_f64(out + key, v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rho(PArrays<T> p, int64_t n, const int32_t* __restrict__ tets,
                                                 double qw, double* __restrict__ rho) {
    // qw lambda_k summed over runs of lanes in the same tet (particles are kept sorted by
    // tet, and a step moves few of them out of their run), then per node in the
    // workgroup's LDS table (neighbouring tets share most of their nodes), flushed with one
    // FP64 atomic per distinct node
    constexpr int kBits = log2_const(4 * kBlock);
    constexpr int kSlots = 1 << kBits;
    __shared__ int s_key[kSlots];
    __shared__ double s_val[kSlots];
    for (int k = threadIdx.x; k < kSlots; k += kBlock) {
        s_key[k] = -1;
        s_val[k] = 0.0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int key = -1;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        key = p.tet[i];
        if (key >= 0) {
            const double l1 = (double)p.l1[i], l2 = (double)p.l2[i], l3 = (double)p.l3[i];
            v[0] = qw * (1.0 - l1 - l2 - l3);
            v[1] = qw * l1;
            v[2] = qw * l2;
            v[3] = qw * l3;
        }
    }
    const int prev_key = __shfl_up(key, 1);   // every lane takes part in the shuffle
    seg_sum_wave<4>(v, (lane == 0) || (key != prev_key));
    const int next_key = __shfl_down(key, 1);
    if (key >= 0 && (lane == 63 || next_key != key)) {
#pragma unroll
        for (int c = 0; c < 4; ++c) lds_add1<kBits>(s_key, s_val, rho, tets[4 * key + c], v[c]);
    }
    __syncthreads();
    flush_table<kSlots, kBlock>(s_key, s_val, rho);
}

// Deterministic form: q w lambda_k of every particle into the fixed-point accumulators.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rho_fix(PArrays<T> p, int64_t n, const int32_t* __restrict__ tets,
                                                     double qw, unsigned long long* __restrict__ fix, double fix_inv) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int t = p.tet[i];
    if (t < 0) return;
    const double l1 = (double)p.l1[i], l2 = (double)p.l2[i], l3 = (double)p.l3[i];
    fix_add(fix, tets[4 * t], qw * (1.0 - l1 - l2 - l3), fix_inv);
    fix_add(fix, tets[4 * t + 1], qw * l1, fix_inv);
    fix_add(fix, tets[4 * t + 2], qw * l2, fix_inv);
    fix_add(fix, tets[4 * t + 3], qw * l3, fix_inv);
}

__global__ __launch_bounds__(kBlock) void k_fix_out(unsigned long long* __restrict__ acc, int64_t n, double scale,
                                                     double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = fix_value(acc[2 * i], acc[2 * i + 1], scale);
    acc[2 * i] = 0ull;
    acc[2 * i + 1] = 0ull;
}

}  // namespace

// ------------------------------------------------------------------------- energies
// Sum of v over the workgroup, then one atomic add into *out (diagnostics only).
__device__ __forceinline__ void block_add(double v, double* out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __shared__ double s_w[kBlock / 64];
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kBlock / 64; ++k) t += s_w[k];
        atomic_add_f64(out, t);
    }
}

// Magnetic energy 1/(2 mu0) int |B|^2: the Whitney-2 field of a divergence-free flux is
// constant in each tet, B = sum_k b_k W2_k, so each tet adds V |B|^2 / (2 mu0), with
// V = 1 / (6 |det(grad l1, grad l2, grad l3)|).
__global__ __launch_bounds__(kBlock) void k_magnetic(int64_t n_tets, const double* __restrict__ b,
                                                      const double* __restrict__ grad64,
                                                      const int32_t* __restrict__ tet_faces, double* out) {
    // The Whitney-2 field of the face fluxes is linear in a tet (constant when the tet's
    // fluxes are divergence-free): B = sum_v lambda_v B_v with B_v its value at vertex v,
    // and int lambda_v lambda_w = V (1 + delta_vw) / 20 gives
    // int |B|^2 = V / 20 (sum_v |B_v|^2 + |sum_v B_v|^2), exact for any fluxes.
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n_tets; t += (int64_t)gridDim.x * kBlock) {
        double g[4][3];
#pragma unroll
        for (int k = 1; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[k][d] = grad64[9 * t + 3 * (k - 1) + d];
#pragma unroll
        for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        constexpr int F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        double Bv[4][3] = {};
        auto cross_add = [&](double* out3, const double* a, const double* c, double f) {
            out3[0] += f * (a[1] * c[2] - a[2] * c[1]);
            out3[1] += f * (a[2] * c[0] - a[0] * c[2]);
            out3[2] += f * (a[0] * c[1] - a[1] * c[0]);
        };
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // W = 2 (lambda_i grad l_j x grad l_l + lambda_j grad l_l x grad l_i + lambda_l grad l_i x grad l_j)
            const int i = F[k][0], j = F[k][1], l = F[k][2];
            const double bf = 2.0 * b[tet_faces[4 * t + k]];
            cross_add(Bv[i], g[j], g[l], bf);
            cross_add(Bv[j], g[l], g[i], bf);
            cross_add(Bv[l], g[i], g[j], bf);
        }
        double sq = 0.0, sum[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                sq += Bv[v][d] * Bv[v][d];
                sum[d] += Bv[v][d];
            }
        sq += sum[0] * sum[0] + sum[1] * sum[1] + sum[2] * sum[2];
        const double det = g[1][0] * (g[2][1] * g[3][2] - g[2][2] * g[3][1]) -
                           g[1][1] * (g[2][0] * g[3][2] - g[2][2] * g[3][0]) +
                           g[1][2] * (g[2][0] * g[3][1] - g[2][1] * g[3][0]);
        const double vol = 1.0 / (6.0 * fabs(det));
        acc += vol / 20.0 * sq / (2.0 * kMu0);
    }
    block_add(acc, out);
}

// Kinetic energy sum_p w m c^2 (gamma - 1), with gamma - 1 = (u^2/c^2) / (gamma + 1).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kinetic(PArrays<T> p, int64_t n, double wmc2, double* out) {
    double acc = 0.0;
    const double ic2 = 1.0 / (kC * kC);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (p.tet[i] < 0) continue;
        const double u0 = p.u0[i], u1 = p.u1[i], u2 = p.u2[i];
        const double q = (u0 * u0 + u1 * u1 + u2 * u2) * ic2;
        acc += wmc2 * q / (sqrt(1.0 + q) + 1.0);
    }
    block_add(acc, out);
}

// Live particles (tet >= 0; absorbed ones stay until the next sort), summed into *out
// (exact in FP64 for any count that fits device memory).
__global__ __launch_bounds__(kBlock) void k_count_live(const int32_t* __restrict__ tet, int64_t n, double* out) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        acc += tet[i] >= 0 ? 1.0 : 0.0;
    block_add(acc, out);
}

// ------------------------------------------------------------------------- launchers
void launch_count_live(hipStream_t s, const int32_t* tet, int64_t n, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_count_live, dim3((unsigned)std::min<int64_t>(1024, grid_1d(n, kBlock))), dim3(kBlock), 0, s,
                       tet, n, out);
}

void launch_magnetic(hipStream_t s, int64_t n_tets, const double* b, const double* grad64, const int32_t* tet_faces,
                     double* out) {
    if (n_tets <= 0) return;
    hipLaunchKernelGGL(k_magnetic, dim3((unsigned)std::min<int64_t>(1024, grid_1d(n_tets, kBlock))), dim3(kBlock), 0,
                       s, n_tets, b, grad64, tet_faces, out);
}

template <typename T>
void launch_kinetic(hipStream_t s, PArrays<T> p, int64_t n, double wmc2, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_kinetic<T>, dim3((unsigned)std::min<int64_t>(1024, grid_1d(n, kBlock))), dim3(kBlock), 0, s,
                       p, n, wmc2, out);
}

void launch_cnt_finish(hipStream_t s, PushCounters* slots, PushCounters* out) {
    hipLaunchKernelGGL(k_cnt_finish, dim3(1), dim3(kCntSlots), 0, s, slots, out);
}

void launch_cnt_crossings(hipStream_t s, const PushCounters* slots, unsigned long long* out) {
    hipLaunchKernelGGL(k_cnt_crossings, dim3(1), dim3(kCntSlots), 0, s, slots, out);
}

template <typename T>
void launch_stage(hipStream_t s, int64_t n_tets, TetBlock<T>* blk, const double* e, const double* b,
                  const double* grad64, const int32_t* tet_edges, const int32_t* tet_faces) {
    if (n_tets <= 0) return;
    hipLaunchKernelGGL(k_stage<T>, dim3(grid_1d(n_tets, kBlock)), dim3(kBlock), 0, s, n_tets, blk, e, b, grad64,
                       tet_edges, tet_faces);
}

// Crossings per particle (last step) above which the particle step is one kernel, and that
// kernel's workgroup size.
constexpr double kFuseShare = 0.5;
constexpr int kFusedBlock = 256;
// A species' own crossings per particle (last step) below which its queue regions are
// visited by k_cross_sparse: fewer than four crossing paths per region of 256 on average.
constexpr double kSparseShare = 1.0 / 64.0;

template <typename T>
void launch_push(hipStream_t s, PArrays<T> in, PArrays<T> out, int64_t n, const TetBlock<T>* blk, double* dg,
                 PushParams pp, PushCounters* cnt, const int32_t* n_live, CrossQueue<T> cq, double cross_share,
                 double own_share, int walk) {
    if (n <= 0) return;
    const unsigned n_wg = (unsigned)grid_1d(n, kBlock);
    if (pp.fix) {
        hipLaunchKernelGGL((k_push<T, true, kFusedBlock, true>), dim3((unsigned)grid_1d(n, kFusedBlock)),
                           dim3(kFusedBlock), 0, s, in, out, n, blk, dg, pp, cnt, n_live, cq);
        return;
    }
    if (walk == FEPIC_WALK_FUSED || (walk == FEPIC_WALK_AUTO && cross_share > kFuseShare)) {
        // most paths cross: finishing them in place costs less idle lanes than the queue
        // costs bytes (64 B written and read back per crossing particle)
        hipLaunchKernelGGL((k_push<T, true, kFusedBlock>), dim3((unsigned)grid_1d(n, kFusedBlock)), dim3(kFusedBlock), 0,
                           s, in, out, n, blk, dg, pp, cnt, n_live, cq);
        return;
    }
    hipLaunchKernelGGL((k_push<T, false, kBlock>), dim3(n_wg), dim3(kBlock), 0, s, in, out, n, blk, dg, pp, cnt, n_live,
                       cq);
    // a species whose paths rarely cross: resident one-wave workgroups visit the few
    // non-empty queue regions; otherwise one k_cross workgroup per k_push workgroup, sized
    // for its expected queue length
    if (own_share < kSparseShare)
        hipLaunchKernelGGL((k_cross_sparse<T>), dim3(std::min<unsigned>(n_wg, sparse_grid<T>())), dim3(64), 0, s, out,
                           cq, (int64_t)n_wg, blk, dg, pp, cnt);
    else if (cross_share <= 0.25)
        hipLaunchKernelGGL((k_cross<T, 64>), dim3(n_wg), dim3(64), 0, s, out, cq, blk, dg, pp, cnt);
    else if (cross_share <= 0.5)
        hipLaunchKernelGGL((k_cross<T, 128>), dim3(n_wg), dim3(128), 0, s, out, cq, blk, dg, pp, cnt);
    else
        hipLaunchKernelGGL((k_cross<T, 256>), dim3(n_wg), dim3(256), 0, s, out, cq, blk, dg, pp, cnt);
}

template <typename T>
void launch_locate(hipStream_t s, int64_t n, const double* x, const double* u, const int64_t* id, int64_t id_base,
                   PArrays<T> out, int64_t out_off, const double* grad64, const double* r0, const int32_t* cell_start,
                   const int32_t* cell_tets, const double* grid_lo, const double* grid_inv_h, const int32_t* grid_n,
                   PushCounters* cnt) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_locate<T>, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, n, x, u, id, id_base, out,
                       out_off, grad64, r0, cell_start, cell_tets, grid_lo, grid_inv_h, grid_n, cnt);
}

template <typename T>
void launch_sort(hipStream_t s, PArrays<T> in, PArrays<T> out, int64_t n, int64_t n_tets, int32_t* count,
                 int32_t* offset, int32_t* block_sums, int32_t* n_live_dev, AbHistIo ab) {
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_1d(n_tets, kBlock)), dim3(kBlock), 0, s, count, n_tets);
    if (n > 0)
        hipLaunchKernelGGL(k_hist, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, in.tet, n, count);
    const int64_t per_block = (int64_t)kBlock * kScanItems;
    const int64_t nb = (n_tets + per_block - 1) / per_block;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kBlock), 0, s, count, offset, n_tets, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, block_sums, nb, n_live_dev);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, offset, n_tets, block_sums);
    if (n > 0)
        hipLaunchKernelGGL(k_scatter<T>, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, in, out, n, offset, ab);
}

template <typename T>
void launch_rho(hipStream_t s, PArrays<T> p, int64_t n, const int32_t* tets, double qw, double* rho,
                unsigned long long* fix, double fix_inv) {
    if (n <= 0) return;
    if (fix)
        hipLaunchKernelGGL(k_rho_fix<T>, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, p, n, tets, qw, fix, fix_inv);
    else
        hipLaunchKernelGGL(k_rho<T>, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, p, n, tets, qw, rho);
}

void launch_fix_out(hipStream_t s, unsigned long long* acc, int64_t n, double scale, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fix_out, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, acc, n, scale, out);
}

#define FEPIC_INSTANTIATE(T)                                                                                      \
    template void launch_stage<T>(hipStream_t, int64_t, TetBlock<T>*, const double*, const double*,             \
                                  const double*, const int32_t*, const int32_t*);                                \
    template void launch_push<T>(hipStream_t, PArrays<T>, PArrays<T>, int64_t, const TetBlock<T>*, double*,      \
                                 PushParams, PushCounters*, const int32_t*, CrossQueue<T>, double, double, int); \
    template void launch_locate<T>(hipStream_t, int64_t, const double*, const double*, const int64_t*, int64_t,  \
                                   PArrays<T>, int64_t, const double*, const double*, const int32_t*,            \
                                   const int32_t*, const double*, const double*, const int32_t*, PushCounters*); \
    template void launch_sort<T>(hipStream_t, PArrays<T>, PArrays<T>, int64_t, int64_t, int32_t*, int32_t*,      \
                                 int32_t*, int32_t*, AbHistIo);                                                  \
    template void launch_rho<T>(hipStream_t, PArrays<T>, int64_t, const int32_t*, double, double*,                 \
                                unsigned long long*, double);                                                     \
    template void launch_kinetic<T>(hipStream_t, PArrays<T>, int64_t, double, double*);

FEPIC_INSTANTIATE(float)
FEPIC_INSTANTIATE(double)

}  // namespace fepic
