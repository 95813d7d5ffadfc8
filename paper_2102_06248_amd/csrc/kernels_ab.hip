// kernels_ab.hip - the paper's Adams-Bashforth-k particle pusher (Sec. III-B) with its
// Lagrange-polynomial path, followed cell by cell (Sec. III-C, Alg. 1 and Alg. 2), and the
// Whitney-1 path integral of each curved piece by Gauss-Legendre quadrature.  All-FP64.
//
// One thread per particle.  The particle's past positions, velocities and accelerations
// live in a per-particle history (structure of arrays); the step:
//   a^n = (q/m)(E + v x B) from the staged tet record at the particle's barycentric point;
//   order m = min(k, levels of history + 1);
//   v^{n+1} = v^n + dt sum_j beta_j a^{n-j},  r^{n+1} = r^n + dt sum_j beta_j v^{n-j};
//   path r(s), s in [0, 1]: the Lagrange polynomial through r^{n+1} (s = 1), r^n (s = 0),
//   r^{n-1} (s = -1), ..., r^{n+1-m};
//   walk: in the current tet, the first of the remaining interval's m + 1 Gauss-Legendre
//   points (or its end) found outside brackets the exit with the piece's start, and
//   bisection (Alg. 2) narrows the bracket to 1e-15 of the step around where the smallest
//   barycentric coordinate reaches -eps; the exit face is the most negative barycentric
//   coordinate at the bracket's outer end; a wall face absorbs the particle.  (A faster
//   root finder, regula falsi, may settle on another root where the path grazes a face
//   between two sample points, and so on other pieces than Alg. 2's; bisection is kept.)
//   deposit: each piece adds q w int W_ab(r(s)) . r'(s) ds over its interval with m + 1
//   Gauss-Legendre points (exact: the integrand has degree 2m - 1), closed onto the face
//   it leaves by: the root lies near the face, not on it, so the piece adds the straight
//   segment from its end point to the face point P (the exit coordinate set to 0, its
//   value shared by the other three) and the next cell starts with the segment from P (the
//   same numbers on the shared vertices) to its own coordinates of the end point; then the
//   pieces telescope and D^T dG = q w (lambda_end - lambda_start) holds to round-off
//   (Sec. III-A).  Six adds per piece into the workgroup's LDS edge table, flushed to dG at
//   the end.
// Barycentric coordinates of a point x in tet t: lambda_k = grad lambda_k . (x - r_0(t)) for
// k = 1..3 (r_0 = the tet's local vertex 0), lambda_0 = 1 - the others.
#include "fepic_internal.h"
#include "fixed_point.h"

namespace fepic {
namespace {

constexpr int kBlock = 256;
constexpr int LE_A[6] = {0, 0, 0, 1, 1, 2};   // local edges (a, b), a < b
constexpr int LE_B[6] = {1, 2, 3, 2, 3, 3};

// Per-workgroup table of edge currents in LDS (open addressing from a multiplicative hash,
// linear probing).  A slot's key is read before it is claimed, so lanes adding to an edge
// that is already there share one broadcast read; a value that finds no slot within
// kProbe probes goes straight to the global vector.  Particles arrive sorted by tet, so a
// workgroup's pieces touch few edges and most adds stay in LDS; the table is flushed with
// one FP64 atomic per occupied slot.
constexpr int kTableBits = 10;
constexpr int kTableSlots = 1 << kTableBits;
constexpr int kProbe = 8;

struct EdgeTable {
    int* key;
    double* val;
    double* dg;
    unsigned long long* fix;   // deterministic mode: straight to the fixed-point accumulators
    double fix_inv;
    __device__ __forceinline__ void add(int e, double v) const {
        if (fix) {
            fix_add(fix, e, v, fix_inv);
            return;
        }
        unsigned int h = ((unsigned int)e * 2654435761u) >> (32 - kTableBits);
        for (int p = 0; p < kProbe; ++p) {
            int k = __hip_atomic_load(key + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == -1) k = atomicCAS(key + h, -1, e);
            if (k == -1 || k == e) {
                __hip_atomic_fetch_add(val + h, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
            h = (h + 1) & (kTableSlots - 1);
        }
        unsafeAtomicAdd(dg + e, v);
    }
};

__device__ __forceinline__ void lam_at(const TetBlock<double>* bp, const double* r0, const double x[3],
                                       double lam[4]) {
    const double d0 = x[0] - r0[0], d1 = x[1] - r0[1], d2 = x[2] - r0[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) lam[k + 1] = bp->gl[3 * k] * d0 + bp->gl[3 * k + 1] * d1 + bp->gl[3 * k + 2] * d2;
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
}

__device__ __forceinline__ double min4(const double l[4]) { return fmin(fmin(l[0], l[1]), fmin(l[2], l[3])); }

// The path of one step in Newton form on its nodes s_j = 1 - j (j = 0..M): r(s) =
// sum_k c_k prod_{i<k} (s - s_i), with c_k the divided differences of the points P[j] at
// s_j.  The nodes are unit-spaced, so each level of the table divides by -k.  Built once
// per particle and step; every evaluation is then a nested product, without divisions.
template <int M>
struct NewtonPath {
    double c[M + 1][3];
    __device__ __forceinline__ explicit NewtonPath(const double P[M + 1][3]) {
#pragma unroll
        for (int j = 0; j <= M; ++j)
#pragma unroll
            for (int d = 0; d < 3; ++d) c[j][d] = P[j][d];
#pragma unroll
        for (int k = 1; k <= M; ++k) {
            const double inv = -1.0 / (double)k;
#pragma unroll
            for (int j = M; j >= k; --j)
#pragma unroll
                for (int d = 0; d < 3; ++d) c[j][d] = (c[j][d] - c[j - 1][d]) * inv;
        }
    }
    __device__ __forceinline__ void at(double s, double r[3]) const {
#pragma unroll
        for (int d = 0; d < 3; ++d) r[d] = c[M][d];
#pragma unroll
        for (int k = M - 1; k >= 0; --k) {
            const double f = s - (1.0 - k);
#pragma unroll
            for (int d = 0; d < 3; ++d) r[d] = r[d] * f + c[k][d];
        }
    }
    __device__ __forceinline__ void at(double s, double r[3], double dr[3]) const {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            r[d] = c[M][d];
            dr[d] = 0.0;
        }
#pragma unroll
        for (int k = M - 1; k >= 0; --k) {
            const double f = s - (1.0 - k);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                dr[d] = dr[d] * f + r[d];
                r[d] = r[d] * f + c[k][d];
            }
        }
    }
};

template <int M>
__device__ __forceinline__ double min_lambda_at(const TetBlock<double>* bp, const double* r0, const NewtonPath<M>& path,
                                                double s) {
    double r[3], lam[4];
    path.at(s, r);
    lam_at(bp, r0, r, lam);
    return min4(lam);
}

template <int M>
__device__ __forceinline__ bool inside_at(const TetBlock<double>* bp, const double* r0, const NewtonPath<M>& path,
                                          double s) {
    return min_lambda_at(bp, r0, path, s) >= -kAbInsideEps;
}

// The straight segment from barycentric point A to B of one tet: its integrand W . dr is
// constant, so q w (m_a d_b - m_b d_a) with m = (A + B) / 2, d = B - A is exact.
__device__ __forceinline__ void deposit_segment(const TetBlock<double>* bp, const double A[4], const double B[4],
                                                const AbParams& ap, const EdgeTable& tab) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int a = LE_A[c], b = LE_B[c];
        const double v = 0.5 * ((A[a] + B[a]) * (B[b] - A[b]) - (A[b] + B[b]) * (B[a] - A[a]));
        if (v != 0.0) tab.add(bp->edge[c], ap.qw * v);
    }
}

// The piece [sa, sb] of the path in tet t: q w int W . r' ds into the table, with M + 1
// Gauss-Legendre points.
template <int M>
__device__ __forceinline__ void deposit_piece(const TetBlock<double>* bp, const double* r0,
                                              const NewtonPath<M>& path, double sa, double sb, const AbParams& ap,
                                              const EdgeTable& tab) {
    constexpr int ng = M + 1;
    const double half = 0.5 * (sb - sa);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int q = 0; q < ng; ++q) {
        const double s = sa + half * (ap.gl_x[ng][q] + 1.0);
        double r[3], dr[3], lam[4], dl[4];
        path.at(s, r, dr);
        lam_at(bp, r0, r, lam);
#pragma unroll
        for (int k = 0; k < 3; ++k) dl[k + 1] = bp->gl[3 * k] * dr[0] + bp->gl[3 * k + 1] * dr[1] + bp->gl[3 * k + 2] * dr[2];
        dl[0] = -(dl[1] + dl[2] + dl[3]);
        const double w = ap.gl_w[ng][q];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += w * (lam[LE_A[c]] * dl[LE_B[c]] - lam[LE_B[c]] * dl[LE_A[c]]);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) tab.add(bp->edge[c], ap.qw * half * acc[c]);
}

// Walks the order-M path of one step from tet t (Alg. 1 and 2) and deposits every piece
// with its face closures.  Returns the final tet, or -1 when a wall absorbed the particle
// or it passed the crossing cap (counted in na / ncap); nc counts the faces crossed.
template <int M>
__device__ __forceinline__ int walk_path(const TetBlock<double>* __restrict__ blk, const double* __restrict__ r0s, int t,
                                      const double P[M + 1][3], const AbParams& ap, const EdgeTable& tab,
                                      unsigned int& nc, unsigned int& na, unsigned int& ncap) {
    constexpr int ng = M + 1;
    const NewtonPath<M> path(P);
    const TetBlock<double>* bp = blk + t;
    double sa = 0.0;
    unsigned int crossed = 0;
    for (;;) {
        const double* r0 = r0s + 3 * t;
        double out = -1.0;
#pragma unroll 1
        for (int q = 0; q <= ng; ++q) {
            const double s = q < ng ? sa + (1.0 - sa) * 0.5 * (ap.gl_x[ng][q] + 1.0) : 1.0;
            if (!inside_at(bp, r0, path, s)) {
                out = s;
                break;
            }
        }
        if (out < 0.0) {
            deposit_piece(bp, r0, path, sa, 1.0, ap, tab);
            nc += crossed;
            return t;
        }
        // Alg. 2: halve [lo, hi], keeping lo inside and hi outside, to kAbRootTol of the step
        double lo = sa, hi = out;
#pragma unroll 1
        for (int it = 0; it < 64 && hi - lo > kAbRootTol; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (inside_at(bp, r0, path, mid)) lo = mid;
            else hi = mid;
        }
        const double sx = 0.5 * (lo + hi);
        deposit_piece(bp, r0, path, sa, sx, ap, tab);
        // exit face: the most negative coordinate at the bracket's outer end
        double r[3], L[4];
        path.at(hi, r);
        lam_at(bp, r0, r, L);
        int kf = 0;
#pragma unroll
        for (int k = 1; k < 4; ++k)
            if (L[k] < L[kf]) kf = k;
        // close the piece onto face kf from its end point r(sx)
        path.at(sx, r);
        lam_at(bp, r0, r, L);
        double Pf[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) Pf[k] = L[k] + L[kf] * (1.0 / 3.0);
        Pf[kf] = 0.0;
        deposit_segment(bp, L, Pf, ap, tab);
        const int nb = bp->nbr[kf];
        if (nb < 0) {
            nc += crossed;
            ++na;
            return -1;
        }
        if (++crossed > (unsigned)ap.cap) {
            nc += crossed;
            ++ncap;
            return -1;
        }
        // the face point in the neighbour's local order (shared vertices keep their order,
        // the far vertex gets 0), then the segment from it to the neighbour's coordinates of
        // the piece's end point
        const int far = nb & 3;
        double Pn[4];
        {
            int jt = 0;
#pragma unroll
            for (int jn = 0; jn < 4; ++jn) {
                if (jn == far) {
                    Pn[jn] = 0.0;
                    continue;
                }
                if (jt == kf) ++jt;
                Pn[jn] = Pf[jt];
                ++jt;
            }
        }
        t = nb >> 2;
        bp = blk + t;
        path.at(sx, r);
        double Ln[4];
        lam_at(bp, r0s + 3 * t, r, Ln);
        deposit_segment(bp, Pn, Ln, ap, tab);
        sa = sx;
    }
}

// One particle's history in the structure-of-arrays store: component c of particle i at
// hist[c * stride + i], so a wave's loads of one component are contiguous.
struct HistRef {
    double* base;
    int64_t stride;
    __device__ __forceinline__ double& operator[](int c) const { return base[c * stride]; }
};

// Slot of level j in a ring of kAbRing levels whose newest level sits at `head`.
__device__ __forceinline__ int ring(int head, int j) {
    const int s = head + j;
    return s >= kAbRing ? s - kAbRing : s;
}

template <int M>
__device__ __forceinline__ int walk_m(const TetBlock<double>* __restrict__ blk, const double* __restrict__ r0s, int t,
                                      const double rn[3], const HistRef& H, int head, const AbParams& ap,
                                      const EdgeTable& tab, unsigned int& nc, unsigned int& na, unsigned int& ncap) {
    double P[M + 1][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) P[0][d] = rn[d];
#pragma unroll
    for (int j = 1; j <= M; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) P[j][d] = H[3 * ring(head, j - 1) + d];
    return walk_path<M>(blk, r0s, t, P, ap, tab, nc, na, ncap);
}

// Cartesian point of barycentric (l1, l2, l3) in a tet: r_0 + G^-1 (l1, l2, l3), G the rows
// grad lambda_1..3.
__device__ __forceinline__ void point_of(const double* G, const double* r0, double l1, double l2, double l3,
                                         double x[3]) {
    const double a = G[0], b = G[1], c = G[2], d = G[3], e = G[4], f = G[5], g = G[6], h = G[7], k = G[8];
    const double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
    const double inv[9] = {(e * k - f * h) / det, (c * h - b * k) / det, (b * f - c * e) / det,
                           (f * g - d * k) / det, (a * k - c * g) / det, (c * d - a * f) / det,
                           (d * h - e * g) / det, (b * g - a * h) / det, (a * e - b * d) / det};
#pragma unroll
    for (int r = 0; r < 3; ++r) x[r] = r0[r] + inv[3 * r] * l1 + inv[3 * r + 1] * l2 + inv[3 * r + 2] * l3;
}

// History of one particle (kAbStride components): three rings of kAbRing levels that share
// one head h: r^{n-j} at 3 ring(h, j), v^{n-j} at 18 + 3 ring(h, j) and a^{n-1-j} at
// 36 + 3 ring(h, j); the levels held and h are in the slot's AbMeta.  A step reads at most
// kAbMax levels of each ring and writes its new level into the slot before the head (the
// one no level of the current state uses), so a step that is not committed leaves the
// history as it was.  A particle without history (AbMeta -1) takes r^n from its
// barycentric position and v^n = u, and writes them at slot 0 first.
__global__ __launch_bounds__(kBlock) void k_push_ab(PArrays<double> in, PArrays<double> out, int64_t n,
                                                     const TetBlock<double>* __restrict__ blk,
                                                     const double* __restrict__ r0s, double* __restrict__ hist,
                                                     int64_t hstride, const int32_t* __restrict__ meta_in,
                                                     int32_t* __restrict__ meta_out, double* __restrict__ dg,
                                                     AbParams ap, PushCounters* __restrict__ slots,
                                                     const int32_t* __restrict__ n_live) {
    __shared__ int s_key[kTableSlots];
    __shared__ double s_val[kTableSlots];
    for (int k = threadIdx.x; k < kTableSlots; k += kBlock) {
        s_key[k] = -1;
        s_val[k] = 0.0;
    }
    __syncthreads();
    const EdgeTable tab{s_key, s_val, dg, ap.fix, ap.fix_inv};
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned int nc = 0, na = 0, ncap = 0;
    // after a sort in the same step only the first *n_live slots hold particles
    const int64_t n_in = n_live ? (int64_t)*n_live : n;
    if (i < n && (i >= n_in || in.tet[i] < 0)) {
        out.tet[i] = -1;
        meta_out[i] = -1;
    } else if (i < n) {
        const HistRef H{hist + i, hstride};
        int t = in.tet[i];
        const TetBlock<double>* bp = blk + t;
        // gather at the particle's barycentric point
        const double l1 = in.l1[i], l2 = in.l2[i], l3 = in.l3[i];
        const double lam[4] = {1.0 - l1 - l2 - l3, l1, l2, l3};
        double g[4][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g[1][d] = bp->gl[d];
            g[2][d] = bp->gl[3 + d];
            g[3][d] = bp->gl[6 + d];
            g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        }
        double E[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const int a = LE_A[c], b = LE_B[c];
#pragma unroll
            for (int d = 0; d < 3; ++d) E[d] += bp->e[c] * (lam[a] * g[b][d] - lam[b] * g[a][d]);
        }
        const double v[3] = {in.u0[i], in.u1[i], in.u2[i]};
        const double acc[3] = {ap.qm * (E[0] + v[1] * bp->B[2] - v[2] * bp->B[1]),
                               ap.qm * (E[1] + v[2] * bp->B[0] - v[0] * bp->B[2]),
                               ap.qm * (E[2] + v[0] * bp->B[1] - v[1] * bp->B[0])};
        const int meta = meta_in[i];
        int held = meta & 0xff, head = meta >> 8;
        if (meta < 0) {
            // no history: r^n from the barycentric position, v^n = u, at slot 0
            double x[3];
            point_of(bp->gl, r0s + 3 * t, l1, l2, l3, x);
            held = 0;
            head = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                H[d] = x[d];
                H[18 + d] = v[d];
            }
        }
        const int m = min(ap.k, held + 1);
        const double* beta = ap.beta[m - 1];
        double vn[3], rn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double dv = beta[0] * acc[d], dr = beta[0] * v[d];
            for (int j = 1; j < m; ++j) {
                dv += beta[j] * H[36 + 3 * ring(head, j - 1) + d];
                dr += beta[j] * H[18 + 3 * ring(head, j) + d];
            }
            vn[d] = v[d] + ap.dt * dv;
            rn[d] = H[3 * head + d] + ap.dt * dr;
        }
        // the path through r^{n+1}, r^n, ..., r^{n+1-m}, walked with the order in use
        switch (m) {
            case 1: t = walk_m<1>(blk, r0s, t, rn, H, head, ap, tab, nc, na, ncap); break;
            case 2: t = walk_m<2>(blk, r0s, t, rn, H, head, ap, tab, nc, na, ncap); break;
            case 3: t = walk_m<3>(blk, r0s, t, rn, H, head, ap, tab, nc, na, ncap); break;
            case 4: t = walk_m<4>(blk, r0s, t, rn, H, head, ap, tab, nc, na, ncap); break;
            default: t = walk_m<5>(blk, r0s, t, rn, H, head, ap, tab, nc, na, ncap); break;
        }
        if (t < 0) {
            out.tet[i] = -1;
            meta_out[i] = -1;
        } else {
            bp = blk + t;
            double lf[4];
            lam_at(bp, r0s + 3 * t, rn, lf);
            out.tet[i] = t;
            out.l1[i] = lf[1];
            out.l2[i] = lf[2];
            out.l3[i] = lf[3];
            out.u0[i] = vn[0];
            out.u1[i] = vn[1];
            out.u2[i] = vn[2];
            // the new level goes into the slot before the head
            const int nh = ring(head, kAbRing - 1);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                H[3 * nh + d] = rn[d];
                H[18 + 3 * nh + d] = vn[d];
                H[36 + 3 * nh + d] = acc[d];
            }
            meta_out[i] = ab_meta(min(held + 1, kAbMax - 1), nh);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kTableSlots; k += kBlock)
        if (s_key[k] >= 0) unsafeAtomicAdd(dg + s_key[k], s_val[k]);
    // counters: per wave, then one add per wave into the workgroup's slot
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        nc += __shfl_xor(nc, off);
        na += __shfl_xor(na, off);
        ncap += __shfl_xor(ncap, off);
    }
    if ((threadIdx.x & 63) == 0 && (nc | na | ncap)) {
        PushCounters* s = slots + (blockIdx.x & (kCntSlots - 1));
        atomicAdd(&s->n_crossings, (unsigned long long)nc);
        atomicAdd(&s->n_absorbed, na);
        atomicAdd(&s->n_cap, ncap);
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* __restrict__ x, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}

}  // namespace

void launch_push_ab(hipStream_t s, PArrays<double> in, PArrays<double> out, int64_t n,
                    const TetBlock<double>* blk, const double* r0, double* hist, int64_t hstride,
                    const int32_t* meta_in, int32_t* meta_out, double* dg, const AbParams& ap, PushCounters* slots,
                    const int32_t* n_live) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_push_ab, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, in, out, n, blk, r0, hist, hstride,
                       meta_in, meta_out, dg, ap, slots, n_live);
}

void launch_fill_i32(hipStream_t s, int32_t* x, int64_t n, int32_t v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, x, n, v);
}

}  // namespace fepic
