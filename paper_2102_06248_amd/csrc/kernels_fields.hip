// Field-side kernels for gfx950: Newmark right-hand side, Jacobi-PCG on a sliced-ELLPACK
// matrix (slice height 64 = one wavefront, coalesced column loads), Faraday update and
// the conservation diagnostics.  All arithmetic FP64.
//
// Row blocks are mapped XCD-contiguously: the hardware hands workgroup b to XCD b % 8,
// so logical block (b % 8) * ceil(nb / 8) + b / 8 gives each XCD's L2 one contiguous
// stretch of rows (and of the vector entries their columns mostly touch).
//
// Global reductions use per-block partials plus a last-block-done ticket: the block that
// arrives last sums the partials in index order (deterministic) and publishes the
// scalar, so a PCG iteration is two kernels and no host round trip.
#include "fepic_internal.h"

namespace fepic {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t xcd_block(int64_t nb_real) {
    const int64_t per = (nb_real + 7) / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

inline unsigned xcd_grid(int64_t nb_real) { return (unsigned)(((nb_real + 7) / 8) * 8); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sums NV values over the block; thread 0 gets the totals in out[].
template <int NV>
__device__ __forceinline__ void block_sum(const double v[NV], double out[NV]) {
    __shared__ double s[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double x = wave_sum(v[j]);
        if (lane == 0) s[j][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) out[j] = s[j][0] + s[j][1] + s[j][2] + s[j][3];
    }
    __syncthreads();
}

// Writes this block's partials, then returns true in the block that arrived last, which
// then sees every partial.  The ticket counter is reset by that block.
template <int NV>
__device__ __forceinline__ bool publish_partials(const double v[NV], double* partial, unsigned int* counter) {
    double tot[NV];
    block_sum<NV>(v, tot);
    __shared__ bool last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) partial[(size_t)j * gridDim.x + blockIdx.x] = tot[j];
        __threadfence();
        const unsigned int ticket = atomicAdd(counter, 1u);
        last = (ticket == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// In the last block: totals[j] = sum of partial[j][*] in a fixed order.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* partial, double tot[NV]) {
    double v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double a = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock)
            a += __builtin_nontemporal_load(partial + (size_t)j * gridDim.x + b);
        v[j] = a;
    }
    block_sum<NV>(v, tot);
}

// Row r of a sliced-ELLPACK matrix times x.
__device__ __forceinline__ double sell_dot(const int64_t* __restrict__ sp, const int32_t* __restrict__ col,
                                           const double* __restrict__ val, const double* __restrict__ x,
                                           int64_t r) {
    const int64_t s = r >> 6;
    const int lane = (int)(r & 63);
    const int64_t b = sp[s], e = sp[s + 1];
    double acc = 0.0;
    for (int64_t k = b + lane; k < e; k += 64) acc += val[k] * x[col[k]];
    return acc;
}

__global__ __launch_bounds__(kBlock) void k_fill(double* x, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_axpby(double* y, const double* a, double alpha, const double* b,
                                                   double beta, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = alpha * a[i] + beta * b[i];
}

// A = M + c S; boundary rows (PEC) become identity rows.  The diagonal is slot 0 of every
// row (the host orders it first), so dinv = 1 / A(slot 0).
__global__ __launch_bounds__(kBlock) void k_scale_A(int64_t n_rows, const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ col, const double* __restrict__ M,
                                                     const double* __restrict__ S, double* __restrict__ A,
                                                     double* __restrict__ dinv, const uint8_t* __restrict__ bmask,
                                                     double c) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t s = r >> 6;
    const int lane = (int)(r & 63);
    if ((s << 6) >= n_rows) return;
    const int64_t b = sp[s], e = sp[s + 1];
    const bool real = r < n_rows;
    const bool bnd = real && bmask[r];
    for (int64_t k = b + lane; k < e; k += 64) {
        double a = M[k] + c * S[k];
        if (bnd) a = (k == b + lane) ? 1.0 : 0.0;
        if (!real) a = 0.0;
        A[k] = a;
    }
    if (real) dinv[r] = 1.0 / A[b + lane];
}

__global__ __launch_bounds__(kBlock) void k_spmv(int64_t n_rows, const int64_t* __restrict__ sp,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ x, double* __restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if ((r >> 6) << 6 >= n_rows) return;
    const double v = sell_dot(sp, col, val, x, r);
    if (r < n_rows) y[r] = v;
}

// b = M (2 e - ep) - dt^2 S (c1 e + c2 ep) - (dg_new - dg_old), zero on boundary rows.
__global__ __launch_bounds__(kBlock) void k_rhs(int64_t n_rows, int64_t nb_real, const int64_t* __restrict__ sp,
                                                 const int32_t* __restrict__ col, const double* __restrict__ M,
                                                 const double* __restrict__ S, const double* __restrict__ e,
                                                 const double* __restrict__ ep, const double* __restrict__ dgn,
                                                 const double* __restrict__ dgo, const uint8_t* __restrict__ bmask,
                                                 double dt2, double c1, double c2, double* __restrict__ bvec,
                                                 double* partial, CgScalars* sc, double tol) {
    const int64_t lb = xcd_block(nb_real);
    const int64_t r = lb * kBlock + threadIdx.x;
    double bb = 0.0;
    if (lb < nb_real && ((r >> 6) << 6) < n_rows) {
        const int64_t s = r >> 6;
        const int lane = (int)(r & 63);
        const int64_t k0 = sp[s], k1 = sp[s + 1];
        double am = 0.0, as = 0.0;
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            const int c = col[k];
            const double ec = e[c], epc = ep[c];
            am += M[k] * (2.0 * ec - epc);
            as += S[k] * (c1 * ec + c2 * epc);
        }
        if (r < n_rows) {
            double v = am - dt2 * as - (dgn[r] - dgo[r]);
            if (bmask[r]) v = 0.0;
            bvec[r] = v;
            bb = v * v;
        }
    }
    const double pv[1] = {bb};
    if (publish_partials<1>(pv, partial, &sc->counter[0])) {
        double tot[1];
        reduce_partials<1>(partial, tot);
        if (threadIdx.x == 0) {
            sc->bb = tot[0];
            sc->tol2_bb = tol * tol * tot[0];
            sc->counter[0] = 0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_warm(int mode, int64_t n, const double* __restrict__ e,
                                                  const double* __restrict__ ep, const double* __restrict__ ep2,
                                                  double* __restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double v = e[i];
    if (mode == FEPIC_WS_EXTRAP1) v = 2.0 * e[i] - ep[i];
    if (mode == FEPIC_WS_EXTRAP2) v = 3.0 * e[i] - 3.0 * ep[i] + ep2[i];
    x[i] = v;
}

// r = b - A x, z = D^-1 r, p_old = 0; rz, rr.
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t n_rows, int64_t nb_real, const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ col, const double* __restrict__ A,
                                                     const double* __restrict__ dinv, const double* __restrict__ b,
                                                     const double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ z, double* __restrict__ p,
                                                     double* partial, CgScalars* sc) {
    const int64_t lb = xcd_block(nb_real);
    const int64_t row = lb * kBlock + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (lb < nb_real && ((row >> 6) << 6) < n_rows) {
        const double ax = sell_dot(sp, col, A, x, row);
        if (row < n_rows) {
            const double rv = b[row] - ax;
            const double zv = dinv[row] * rv;
            r[row] = rv;
            z[row] = zv;
            p[row] = 0.0;
            rz = rv * zv;
            rr = rv * rv;
        }
    }
    const double pv[2] = {rz, rr};
    if (publish_partials<2>(pv, partial, &sc->counter[1])) {
        double tot[2];
        reduce_partials<2>(partial, tot);
        if (threadIdx.x == 0) {
            sc->rz = tot[0];
            sc->rr = tot[1];
            sc->rr0 = tot[1];
            sc->beta = 0.0;
            sc->iters = 0;
            sc->converged = (tot[1] <= sc->tol2_bb) ? 1 : 0;
            sc->counter[1] = 0;
        }
    }
}

// p_new = z + beta p_old (formed on the fly for the neighbours as well), q = A p_new,
// p.q; the last block sets alpha = rz / pq.
__global__ __launch_bounds__(kBlock) void k_cg_spmv(int64_t n_rows, int64_t nb_real, const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ col, const double* __restrict__ A,
                                                     const double* __restrict__ z, const double* __restrict__ p_old,
                                                     double* __restrict__ p_new, double* __restrict__ q,
                                                     double* partial, CgScalars* sc) {
    if (sc->converged) return;
    const double beta = sc->beta;
    const int64_t lb = xcd_block(nb_real);
    const int64_t row = lb * kBlock + threadIdx.x;
    double pq = 0.0;
    if (lb < nb_real && ((row >> 6) << 6) < n_rows) {
        const int64_t s = row >> 6;
        const int lane = (int)(row & 63);
        const int64_t k0 = sp[s], k1 = sp[s + 1];
        double acc = 0.0;
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            const int c = col[k];
            acc += A[k] * (z[c] + beta * p_old[c]);
        }
        if (row < n_rows) {
            const double pn = z[row] + beta * p_old[row];
            p_new[row] = pn;
            q[row] = acc;
            pq = pn * acc;
        }
    }
    const double pv[1] = {pq};
    if (publish_partials<1>(pv, partial, &sc->counter[2])) {
        double tot[1];
        reduce_partials<1>(partial, tot);
        if (threadIdx.x == 0) {
            if (tot[0] > 0.0) {
                sc->alpha = sc->rz / tot[0];
            } else {
                sc->alpha = 0.0;
                sc->converged = 2;  // breakdown: p = 0
            }
            sc->pq = tot[0];
            sc->counter[2] = 0;
        }
    }
}

// x += alpha p, r -= alpha q, z = D^-1 r; rz, rr; the last block sets beta and tests
// ||r||^2 <= tol^2 ||b||^2.
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n_rows, int64_t nb_real, const double* __restrict__ dinv,
                                                       double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ z, const double* __restrict__ p,
                                                       const double* __restrict__ q, double* partial, CgScalars* sc) {
    if (sc->converged) return;
    const double alpha = sc->alpha;
    const int64_t lb = xcd_block(nb_real);
    const int64_t row = lb * kBlock + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (lb < nb_real && row < n_rows) {
        x[row] += alpha * p[row];
        const double rv = r[row] - alpha * q[row];
        const double zv = dinv[row] * rv;
        r[row] = rv;
        z[row] = zv;
        rz = rv * zv;
        rr = rv * rv;
    }
    const double pv[2] = {rz, rr};
    if (publish_partials<2>(pv, partial, &sc->counter[3])) {
        double tot[2];
        reduce_partials<2>(partial, tot);
        if (threadIdx.x == 0) {
            sc->beta = tot[0] / sc->rz;
            sc->rz = tot[0];
            sc->rr = tot[1];
            sc->iters += 1;
            if (tot[1] <= sc->tol2_bb) sc->converged = 1;
            sc->counter[3] = 0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_if_b_zero(double* x, int64_t n, const CgScalars* sc) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && sc->bb == 0.0) x[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_cg_resid(int64_t n_rows, int64_t nb_real, const int64_t* __restrict__ sp,
                                                      const int32_t* __restrict__ col, const double* __restrict__ A,
                                                      const double* __restrict__ b, const double* __restrict__ x,
                                                      double* __restrict__ rt, double* partial, CgScalars* sc) {
    const int64_t lb = xcd_block(nb_real);
    const int64_t row = lb * kBlock + threadIdx.x;
    double rr = 0.0;
    if (lb < nb_real && ((row >> 6) << 6) < n_rows) {
        const double ax = sell_dot(sp, col, A, x, row);
        if (row < n_rows) {
            const double v = b[row] - ax;
            rt[row] = v;
            rr = v * v;
        }
    }
    const double pv[1] = {rr};
    if (publish_partials<1>(pv, partial, &sc->counter[0])) {
        double tot[1];
        reduce_partials<1>(partial, tot);
        if (threadIdx.x == 0) {
            sc->rr_true = tot[0];
            sc->counter[0] = 0;
        }
    }
}

// b_new = b_old - dt C (gamma e_new + (1 - gamma) e_old); face (i,j,k) has edges
// (i,j) +1, (j,k) +1, (i,k) -1.
__global__ __launch_bounds__(kBlock) void k_faraday(int64_t n_faces, const int32_t* __restrict__ fe,
                                                     const double* __restrict__ b_old,
                                                     const double* __restrict__ e_new,
                                                     const double* __restrict__ e_old, double dt, double gamma,
                                                     double* __restrict__ b_new) {
    int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= n_faces) return;
    const int a = fe[3 * f], b = fe[3 * f + 1], c = fe[3 * f + 2];
    const double ea = gamma * e_new[a] + (1.0 - gamma) * e_old[a];
    const double eb = gamma * e_new[b] + (1.0 - gamma) * e_old[b];
    const double ec = gamma * e_new[c] + (1.0 - gamma) * e_old[c];
    b_new[f] = b_old[f] - dt * (ea + eb - ec);
}

// out[node] += D^T v: +v at the head, -v at the tail of every edge.
__global__ __launch_bounds__(kBlock) void k_DT(int64_t n_edges, const int32_t* __restrict__ edges,
                                                const double* __restrict__ v, double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_edges) return;
    const double x = v[i];
    if (x != 0.0) {
        unsafeAtomicAdd(out + edges[2 * i + 1], x);
        unsafeAtomicAdd(out + edges[2 * i], -x);
    }
}

__device__ __forceinline__ void atomic_max_abs(unsigned long long* p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(fabs(v)));
}

__global__ __launch_bounds__(kBlock) void k_diag_nodes(int64_t n_nodes, const uint8_t* __restrict__ interior,
                                                        const double* __restrict__ rho_new,
                                                        const double* __restrict__ rho_old,
                                                        const double* __restrict__ dtdg,
                                                        const double* __restrict__ dtMe,
                                                        const double* __restrict__ rG1, const double* __restrict__ rG2,
                                                        const double* __restrict__ dtrcg, int have_hist,
                                                        double* __restrict__ rG_out, DiagAcc* acc) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_nodes) return;
    if (!interior[k]) {
        rG_out[k] = 0.0;
        return;
    }
    const double rc = (rho_new[k] - rho_old[k]) - dtdg[k];
    const double rg = -dtMe[k] - rho_new[k];
    rG_out[k] = rg;
    atomic_max_abs(&acc->cont_max, rc);
    atomic_max_abs(&acc->gauss_max, rg);
    atomic_max_abs(&acc->rho_max, rho_new[k]);
    if (have_hist) atomic_max_abs(&acc->drift_max, (rg - 2.0 * rG1[k] + rG2[k]) - dtrcg[k]);
}

__global__ __launch_bounds__(kBlock) void k_divb(int64_t n_tets, const int32_t* __restrict__ tf,
                                                  const double* __restrict__ b, DiagAcc* acc) {
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_tets) return;
    const double d = b[tf[4 * t]] - b[tf[4 * t + 1]] + b[tf[4 * t + 2]] - b[tf[4 * t + 3]];
    atomic_max_abs(&acc->divb_max, d);
}

__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                 double* partial, double* out, unsigned int* counter) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double pv[1] = {i < n ? a[i] * b[i] : 0.0};
    if (publish_partials<1>(pv, partial, counter)) {
        double tot[1];
        reduce_partials<1>(partial, tot);
        if (threadIdx.x == 0) {
            *out = tot[0];
            *counter = 0;
        }
    }
}

}  // namespace

// ------------------------------------------------------------------------- launchers
void launch_fill(hipStream_t s, double* x, int64_t n, double v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, x, n, v);
}

void launch_axpby(hipStream_t s, double* y, const double* a, double alpha, const double* b, double beta, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, y, a, alpha, b, beta, n);
}

static int64_t row_blocks(int64_t n_rows) { return (n_rows + kBlock - 1) / kBlock; }

void launch_scale_A(hipStream_t s, const SellMatrix& shape, const int64_t* sp, const int32_t* col, const double* M,
                    const double* S, double* A, double* dinv, const uint8_t* bmask, double c) {
    hipLaunchKernelGGL(k_scale_A, dim3((unsigned)row_blocks(shape.n_slices * kSell)), dim3(kBlock), 0, s,
                       shape.n_rows, sp, col, M, S, A, dinv, bmask, c);
}

void launch_sell_spmv(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* val,
                      const double* x, double* y) {
    hipLaunchKernelGGL(k_spmv, dim3((unsigned)row_blocks(n_rows)), dim3(kBlock), 0, s, n_rows, sp, col, val, x, y);
}

void launch_rhs(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* M,
                const double* S, const double* e, const double* ep, const double* dg_new, const double* dg_old,
                const uint8_t* bmask, double dt2, double c1, double c2, double* b, double* partial, CgScalars* sc,
                double tol) {
    const int64_t nb = row_blocks(n_rows);
    hipLaunchKernelGGL(k_rhs, dim3(xcd_grid(nb)), dim3(kBlock), 0, s, n_rows, nb, sp, col, M, S, e, ep, dg_new,
                       dg_old, bmask, dt2, c1, c2, b, partial, sc, tol);
}

void launch_warm(hipStream_t s, int mode, int64_t n, const double* e, const double* ep, const double* ep2, double* x) {
    hipLaunchKernelGGL(k_warm, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, mode, n, e, ep, ep2, x);
}

void launch_cg_init(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                    const double* dinv, const double* b, const double* x, double* r, double* z, double* p,
                    double* partial, CgScalars* sc) {
    const int64_t nb = row_blocks(n_rows);
    hipLaunchKernelGGL(k_cg_init, dim3(xcd_grid(nb)), dim3(kBlock), 0, s, n_rows, nb, sp, col, A, dinv, b, x, r, z,
                       p, partial, sc);
}

void launch_cg_iter(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                    const double* dinv, double* x, double* r, double* z, const double* p_old, double* p_new,
                    double* q, double* partial, CgScalars* sc, hipEvent_t* ev_spmv, hipEvent_t* ev_upd) {
    const int64_t nb = row_blocks(n_rows);
    if (ev_spmv) (void)hipEventRecord(ev_spmv[0], s);
    hipLaunchKernelGGL(k_cg_spmv, dim3(xcd_grid(nb)), dim3(kBlock), 0, s, n_rows, nb, sp, col, A, z, p_old, p_new, q,
                       partial, sc);
    if (ev_spmv) (void)hipEventRecord(ev_spmv[1], s);
    if (ev_upd) (void)hipEventRecord(ev_upd[0], s);
    hipLaunchKernelGGL(k_cg_update, dim3(xcd_grid(nb)), dim3(kBlock), 0, s, n_rows, nb, dinv, x, r, z, p_new, q,
                       partial, sc);
    if (ev_upd) (void)hipEventRecord(ev_upd[1], s);
}

void launch_cg_resid(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                     const double* b, double* x, double* r_true, double* partial, CgScalars* sc) {
    hipLaunchKernelGGL(k_zero_if_b_zero, dim3(grid_1d(n_rows, kBlock)), dim3(kBlock), 0, s, x, n_rows, sc);
    const int64_t nb = row_blocks(n_rows);
    hipLaunchKernelGGL(k_cg_resid, dim3(xcd_grid(nb)), dim3(kBlock), 0, s, n_rows, nb, sp, col, A, b, x, r_true,
                       partial, sc);
}

void launch_faraday(hipStream_t s, int64_t n_faces, const int32_t* face_edges, const double* b_old,
                    const double* e_new, const double* e_old, double dt, double gamma, double* b_new) {
    if (n_faces <= 0) return;
    hipLaunchKernelGGL(k_faraday, dim3(grid_1d(n_faces, kBlock)), dim3(kBlock), 0, s, n_faces, face_edges, b_old,
                       e_new, e_old, dt, gamma, b_new);
}

void launch_DT(hipStream_t s, int64_t n_edges, const int32_t* edges, const double* v, double* out_nodes) {
    hipLaunchKernelGGL(k_DT, dim3(grid_1d(n_edges, kBlock)), dim3(kBlock), 0, s, n_edges, edges, v, out_nodes);
}

void launch_diag_nodes(hipStream_t s, int64_t n_nodes, const uint8_t* interior_node, const double* rho_new,
                       const double* rho_old, const double* dtdg, const double* dtMe, const double* rG1,
                       const double* rG2, const double* dtrcg, int have_hist, double* rG_out, DiagAcc* acc) {
    hipLaunchKernelGGL(k_diag_nodes, dim3(grid_1d(n_nodes, kBlock)), dim3(kBlock), 0, s, n_nodes, interior_node,
                       rho_new, rho_old, dtdg, dtMe, rG1, rG2, dtrcg, have_hist, rG_out, acc);
}

void launch_divb(hipStream_t s, int64_t n_tets, const int32_t* tet_faces, const double* b, DiagAcc* acc) {
    hipLaunchKernelGGL(k_divb, dim3(grid_1d(n_tets, kBlock)), dim3(kBlock), 0, s, n_tets, tet_faces, b, acc);
}

void launch_dot(hipStream_t s, int64_t n, const double* a, const double* b, double* partial, double* out,
                unsigned int* counter) {
    hipLaunchKernelGGL(k_dot, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, n, a, b, partial, out, counter);
}

}  // namespace fepic
