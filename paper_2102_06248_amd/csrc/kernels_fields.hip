// Field-side kernels for gfx950: Newmark right-hand side, PCG on a sliced-ELLPACK matrix
// (slice height 64 = one wavefront, coalesced column loads) with the nodal auxiliary-space
// preconditioner or with Jacobi, Faraday update and the conservation diagnostics.  Field
// vectors, residuals, dot products and the diagnostics are FP64; the PCG kernels are
// templated on their storage type, and the FP32 instances (matrix values, inverse
// diagonals and iteration vectors rounded to FP32, dot products and step lengths still
// FP64) run the inner passes of the mixed-precision solve.
//
// Grids are XCD-contiguous: the hardware hands workgroup b to XCD b % 8, so workgroup b
// walks the row blocks of the b % 8-th eighth of the rows, giving each XCD's L2 one
// contiguous stretch of rows and of the vector entries their columns mostly touch.
//
// Global dot products never communicate between workgroups inside a kernel: the
// once-per-solve reductions write one partial per workgroup that the next kernel sums
// (every workgroup, redundantly, in the same fixed order, so all reach the same bits);
// the iteration dots go through FP64-atomic slots that the next kernel sums the same way.
// Kernel boundaries give the visibility; no device-scope fences are issued.
#include <algorithm>

#include "fepic_internal.h"

namespace fepic {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxGrid = 1024;  // 4 workgroups per CU on 256 CUs

struct RowGrid {
    int64_t nb;      // row blocks of kBlock rows
    int64_t per;     // row blocks per XCD
    int g;           // workgroups per XCD
    unsigned grid;   // 8 * g
};

inline RowGrid row_grid(int64_t n_rows, int max_grid = kMaxGrid) {
    RowGrid r;
    r.nb = (n_rows + kBlock - 1) / kBlock;
    r.per = (r.nb + 7) / 8;
    r.g = (int)std::min<int64_t>(r.per, max_grid / 8);
    if (r.g < 1) r.g = 1;
    r.grid = 8u * (unsigned)r.g;
    return r;
}

__device__ __forceinline__ int64_t rg_first(const RowGrid& rg) {
    return (int64_t)(blockIdx.x % 8) * rg.per + blockIdx.x / 8;
}
__device__ __forceinline__ int64_t rg_end(const RowGrid& rg) {
    const int64_t e = (int64_t)(blockIdx.x % 8 + 1) * rg.per;
    return e < rg.nb ? e : rg.nb;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Block-wide sums of NV values over a block of BS threads; every thread receives the
// totals (summed in a fixed order).
template <int NV, int BS = kBlock>
__device__ __forceinline__ void block_sum_all(double v[NV]) {
    constexpr int NW = BS / 64;
    __shared__ double s[NV][NW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double x = wave_sum(v[j]);
        if (lane == 0) s[j][w] = x;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) a += s[j][q];
        v[j] = a;
    }
    __syncthreads();
}

// Workgroup totals -> partial[j * gridDim.x + blockIdx.x].
template <int NV, int BS = kBlock>
__device__ __forceinline__ void write_partials(double v[NV], double* partial) {
    block_sum_all<NV, BS>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) partial[(size_t)j * gridDim.x + blockIdx.x] = v[j];
    }
}

// Sum of the partials a previous kernel of n_src workgroups wrote (fixed order).
template <int NV, int BS = kBlock>
__device__ __forceinline__ void read_partials(const double* partial, int n_src, double tot[NV]) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double a = 0.0;
        for (int b = threadIdx.x; b < n_src; b += BS) a += partial[(size_t)j * n_src + b];
        tot[j] = a;
    }
    block_sum_all<NV, BS>(tot);
}

// Sum over the row's slots of A(j,c) * f(c), four slots in flight at a time so the column
// and gather loads of a wavefront overlap (one thread per row, one wave per slice).
template <typename GatherFn>
__device__ __forceinline__ double sell_row(const int64_t* __restrict__ sp, const int32_t* __restrict__ col,
                                           const double* __restrict__ A, int64_t row, GatherFn f) {
    const int64_t sl = row >> 6;
    const int lane = (int)(row & 63);
    const int64_t k1 = sp[sl + 1];
    int64_t k = sp[sl] + lane;
    double acc0 = 0.0, acc1 = 0.0;
    for (; k + 3 * 64 < k1; k += 4 * 64) {
        const int c0 = col[k], c1 = col[k + 64], c2 = col[k + 128], c3 = col[k + 192];
        const double a0 = A[k], a1 = A[k + 64], a2 = A[k + 128], a3 = A[k + 192];
        const double u0 = f(c0), u1 = f(c1), u2 = f(c2), u3 = f(c3);
        acc0 += a0 * u0 + a2 * u2;
        acc1 += a1 * u1 + a3 * u3;
    }
    for (; k < k1; k += 64) acc0 += A[k] * f(col[k]);
    return acc0 + acc1;
}

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

// A = M + c S (+ cK K with absorbing faces); fixed (PEC) rows become identity rows.  The
// diagonal is slot 0 of every row (the host orders it first), so dinv = 1 / A(slot 0).
__global__ __launch_bounds__(kBlock) void k_scale_A(int64_t n_rows, const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ col, const double* __restrict__ M,
                                                     const double* __restrict__ S, double* __restrict__ A,
                                                     double* __restrict__ dinv, const uint8_t* __restrict__ bmask,
                                                     double c, const double* __restrict__ K, double cK) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t s = r >> 6;
    const int lane = (int)(r & 63);
    if ((s << 6) >= n_rows) return;
    const int64_t b = sp[s], e = sp[s + 1];
    const bool real = r < n_rows;
    const bool bnd = real && bmask[r];
    for (int64_t k = b + lane; k < e; k += 64) {
        double a = M[k] + c * S[k];
        if (K) a += cK * K[k];
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

// b = M (2 e - ep) - dt^2 S (c1 e + c2 ep) - (dg_new - dg_old), zero on fixed rows;
// partials of ||b||^2.  With absorbing faces (kAbc) also + K (kc1 e + kc2 ep), the damping
// terms of the Newmark recurrence.
template <bool kAbc>
__global__ __launch_bounds__(kBlock) void k_rhs(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                 const int32_t* __restrict__ col, const double* __restrict__ M,
                                                 const double* __restrict__ S, const double* __restrict__ e,
                                                 const double* __restrict__ ep, const double* __restrict__ dgn,
                                                 const double* __restrict__ dgo, const uint8_t* __restrict__ bmask,
                                                 double dt2, double c1, double c2, const double* __restrict__ K,
                                                 double kc1, double kc2, double* __restrict__ bvec,
                                                 double* __restrict__ partial) {
    double bb[1] = {0.0};
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t r = lb * kBlock + threadIdx.x;
        if (((r >> 6) << 6) >= n_rows) continue;
        const int64_t s = r >> 6;
        const int lane = (int)(r & 63);
        const int64_t k0 = sp[s], k1 = sp[s + 1];
        double am = 0.0, as = 0.0, ak = 0.0;
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            const int c = col[k];
            const double ec = e[c], epc = ep[c];
            am += M[k] * (2.0 * ec - epc);
            as += S[k] * (c1 * ec + c2 * epc);
            if constexpr (kAbc) ak += K[k] * (kc1 * ec + kc2 * epc);
        }
        if (r < n_rows) {
            double v = am - dt2 * as - (dgn[r] - dgo[r]);
            if constexpr (kAbc) v += ak;
            if (bmask[r]) v = 0.0;
            bvec[r] = v;
            bb[0] += v * v;
        }
    }
    write_partials<1>(bb, partial);
}

// The mixed (b, e) updates (FEPIC_FIELD_NM_MFEM, FEPIC_FIELD_BD_MFEM) with b^{n+1}
// eliminated: h = Mf (c1 b^n + c2 b^{n-1}) on face rows (Whitney-2 mass, SELL-64), then on
// edge rows
//   rhs = M (a0 e^n + a1 e^{n-1}) + dt^2 S (s0 e^n + s1 e^{n-1}) + dt sum_f C_fe h_f
//         - (g0 dG^{n+1} + g1 dG^n),
// C_fe from each edge's list of faces ((f << 1) | 1 for -1; -1 pads); wall rows 0.  The
// partials of ||rhs||^2 go where k_rhs puts them, for the solve that follows.
__global__ __launch_bounds__(kBlock) void k_face_spmv(int64_t n_faces, const int64_t* __restrict__ sp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ b1, double c1,
                                                       const double* __restrict__ b2, double c2,
                                                       double* __restrict__ h) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (((r >> 6) << 6) >= n_faces) return;
    const int64_t sl = r >> 6;
    const int lane = (int)(r & 63);
    double acc = 0.0;
    for (int64_t k = sp[sl] + lane; k < sp[sl + 1]; k += 64) {
        const int c = col[k];
        acc += val[k] * (c1 * b1[c] + c2 * b2[c]);
    }
    if (r < n_faces) h[r] = acc;
}

struct MfemCoef {
    double a0, a1, s0, s1, g0, g1;
};

__global__ __launch_bounds__(kBlock) void k_mfem_rhs(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                      const int32_t* __restrict__ col, const double* __restrict__ M,
                                                      const double* __restrict__ S, const double* __restrict__ e,
                                                      const double* __restrict__ ep, const double* __restrict__ dgn,
                                                      const double* __restrict__ dgo, const uint8_t* __restrict__ bmask,
                                                      const int64_t* __restrict__ esp, const int32_t* __restrict__ einc,
                                                      const double* __restrict__ h, double dt, MfemCoef k,
                                                      double* __restrict__ bvec, double* __restrict__ partial) {
    double bb[1] = {0.0};
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t r = lb * kBlock + threadIdx.x;
        if (((r >> 6) << 6) >= n_rows) continue;
        const int64_t s = r >> 6;
        const int lane = (int)(r & 63);
        double am = 0.0, as = 0.0, ac = 0.0;
        for (int64_t q = sp[s] + lane; q < sp[s + 1]; q += 64) {
            const int c = col[q];
            const double ec = e[c], epc = ep[c];
            am += M[q] * (k.a0 * ec + k.a1 * epc);
            as += S[q] * (k.s0 * ec + k.s1 * epc);
        }
        for (int64_t q = esp[s] + lane; q < esp[s + 1]; q += 64) {
            const int code = einc[q];
            if (code < 0) continue;
            const double hf = h[code >> 1];
            ac += (code & 1) ? -hf : hf;
        }
        if (r < n_rows) {
            double v = am + dt * dt * as + dt * ac - (k.g0 * dgn[r] + k.g1 * dgo[r]);
            if (bmask[r]) v = 0.0;
            bvec[r] = v;
            bb[0] += v * v;
        }
    }
    write_partials<1>(bb, partial);
}

// b^{n+1} = b_base - dt C (cn e^n + cm e^{n-1} + cp e^{n+1}) (NM: b_base = b^{n-1},
// coefficients 1, 1/2, 1/2; BD: b_base = b^n, 0, 0, 1).
__global__ __launch_bounds__(kBlock) void k_mfem_faraday(int64_t n_faces, const int32_t* __restrict__ fe,
                                                          const double* __restrict__ b_base,
                                                          const double* __restrict__ e_n,
                                                          const double* __restrict__ e_nm1,
                                                          const double* __restrict__ e_np1, double dt, double cn,
                                                          double cm, double cp, double* __restrict__ b_new) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= n_faces) return;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int a = fe[3 * f + j];
        const double ea = cn * e_n[a] + cm * e_nm1[a] + cp * e_np1[a];
        v += j == 2 ? -ea : ea;
    }
    b_new[f] = b_base[f] - dt * v;
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

// Jacobi-preconditioned CG in the single-reduction form of Chronopoulos and Gear (1989):
// with u = D^-1 r and w = A u kept by recurrence, one iteration needs the three dots
// (r,u), (u,w), (r,r) of the previous iterate only, so it is one kernel:
//   beta_i  = g_i / g_{i-1},   alpha_i = g_i / (d_i - beta_i g_i / alpha_{i-1})
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r' = r - alpha s,  u' = D^-1 r',
//   w' = A u' (the neighbours' u' formed on the fly from the previous r, w, s),
//   g_{i+1} = (r',u'), d_{i+1} = (u',w'), ||r'||^2.
// The kernel keeps r, w and s scaled by D^-1 (R = D^-1 r, W = D^-1 w, S = D^-1 s, D =
// diag A) so a neighbour's u' = R - alpha (W + beta S) needs three of its values; they
// are stored interleaved with the row's own p (CgVec, 32 bytes per row) so the three
// come from one sector.  The interleaved state is double buffered (neighbours read the
// previous values); x is touched by its own row only.

// Iteration partials: the three dots of each iteration are added with FP64 atomics into
// kCgSlots slots per value (workgroup b -> slot b mod kCgSlots), in three rotating
// buffers: iteration i reads buffer i mod 3 (filled by the previous kernel), adds into
// buffer (i + 1) mod 3 (cleared by the previous kernel) and clears buffer (i + 2) mod 3
// (read by the previous kernel).  Reading 3 x 64 values instead of one partial per
// workgroup lets the iteration kernel run one workgroup per row block at any size.
constexpr int kCgSlots = 64;
__device__ __forceinline__ double* cg_buf(double* base, int k) { return base + (size_t)(k % 3) * 3 * kCgSlots; }

// Workgroup totals v (already summed over the block) added into buffer slots.
__device__ __forceinline__ void cg_add(double* buf, const double v[3]) {
    if (threadIdx.x == 0) {
        const int s = blockIdx.x & (kCgSlots - 1);
#pragma unroll
        for (int j = 0; j < 3; ++j) unsafeAtomicAdd(buf + j * kCgSlots + s, v[j]);
    }
}

// ||b||^2 from the right-hand side's partials; R = D^-1 (b - A x); W = S = P = 0; clears
// iteration buffers 0 and 1.
__global__ __launch_bounds__(kBlock) void k_cg_init_a(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ A,
                                                       const double* __restrict__ dinv, const double* __restrict__ b,
                                                       const double* __restrict__ x, CgVec* __restrict__ V,
                                                       const double* __restrict__ part_rhs, int n_rhs_wg,
                                                       double* cg_slots, CgScalars* sc, double tol) {
    double bb[1];
    read_partials<1>(part_rhs, n_rhs_wg, bb);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            sc->bb = bb[0];
            sc->tol2_bb = tol * tol * bb[0];
            sc->converged = 0;
        }
        for (int k = threadIdx.x; k < 2 * 3 * kCgSlots; k += kBlock) cg_slots[k] = 0.0;
    }
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t row = lb * kBlock + threadIdx.x;
        if (((row >> 6) << 6) >= n_rows) continue;
        const double ax = sell_row(sp, col, A, row, [&](int c) { return x[c]; });
        if (row < n_rows) {
            double2* o = reinterpret_cast<double2*>(V + row);
            o[0] = make_double2(dinv[row] * (b[row] - ax), 0.0);
            o[1] = make_double2(0.0, 0.0);
        }
    }
}

// W = D^-1 A u with u = R (only R is gathered); partials of (r,u), (u,w), (r,r).
__global__ __launch_bounds__(kBlock) void k_cg_init_b(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ A,
                                                       const double* __restrict__ dinv, CgVec* __restrict__ V,
                                                       double* __restrict__ cg_slots) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t row = lb * kBlock + threadIdx.x;
        if (((row >> 6) << 6) >= n_rows) continue;
        const double acc = sell_row(sp, col, A, row, [&](int c) { return V[c].R; });
        if (row < n_rows) {
            const double dj = dinv[row], uv = V[row].R, rv = uv / dj;
            V[row].W = dj * acc;
            v[0] += rv * uv;
            v[1] += uv * acc;
            v[2] += rv * rv;
        }
    }
    block_sum_all<3>(v);
    cg_add(cg_buf(cg_slots, 0), v);
}

// The part of row j's product that does not depend on the iteration's scalars: the three
// sums sum_k A_jk R_k, sum_k A_jk W_k, sum_k A_jk S_k over the row's stored entries, and
// the row's own entries (1 / A_jj from the row's first slot).  A_j u' = sR - alpha sW
// - alpha beta sS, so the gathers of a row can be issued before the scalars of this
// iteration are known.
struct RowPart {
    double sR, sW, sS;
    double2 RW, SP;   // own R, W and S, P
    double x, dinv;
};

constexpr int kUnroll = 6;   // slots per batch of gathers (rows hold up to ~20 slots)

__device__ __forceinline__ void row_part(RowPart& P, const int64_t* __restrict__ sp, const int32_t* __restrict__ col,
                                         const double* __restrict__ A, const CgVec* __restrict__ V,
                                         const double* __restrict__ x, const double* __restrict__ dinv, int64_t row,
                                         bool real) {
    const int64_t sl = row >> 6;
    const int lane = (int)(row & 63);
    const int64_t k1 = sp[sl + 1];
    int64_t k = sp[sl] + lane;
    const int64_t r = real ? row : 0;
    const double2* own = reinterpret_cast<const double2*>(V + r);
    P.RW = own[0];
    P.SP = own[1];
    P.x = x[r];
    P.dinv = real ? 1.0 / A[sp[sl] + lane] : 1.0;   // the diagonal is slot 0 of the row
    double r0 = 0.0, w0 = 0.0, s0 = 0.0, r1 = 0.0, w1 = 0.0, s1 = 0.0;
    for (; k + (kUnroll - 1) * 64 < k1; k += kUnroll * 64) {
        int c[kUnroll];
        double a[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            c[q] = col[k + 64 * q];
            a[q] = A[k + 64 * q];
        }
        double2 rw[kUnroll];
        double sv[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            rw[q] = *reinterpret_cast<const double2*>(V + c[q]);
            sv[q] = V[c[q]].S;
        }
#pragma unroll
        for (int q = 0; q < kUnroll; q += 2) {
            r0 += a[q] * rw[q].x;
            w0 += a[q] * rw[q].y;
            s0 += a[q] * sv[q];
            r1 += a[q + 1] * rw[q + 1].x;
            w1 += a[q + 1] * rw[q + 1].y;
            s1 += a[q + 1] * sv[q + 1];
        }
    }
    for (; k < k1; k += 64) {
        const int c = col[k];
        const double a = A[k];
        const double2 rw = *reinterpret_cast<const double2*>(V + c);
        r0 += a * rw.x;
        w0 += a * rw.y;
        s0 += a * V[c].S;
    }
    P.sR = r0 + r1;
    P.sW = w0 + w1;
    P.sS = s0 + s1;
}

__global__ __launch_bounds__(kBlock) void k_cg_iter(int64_t n_rows, RowGrid rg, int i, const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ col, const double* __restrict__ A,
                                                     const double* __restrict__ dinv, double* __restrict__ x,
                                                     const CgVec* __restrict__ V, CgVec* __restrict__ V_new,
                                                     double* __restrict__ cg_slots, CgScalars* sc) {
    // The converged flag, the previous kernel's dot slots and this workgroup's first rows
    // are all in flight together; the flag (the same for every thread) is checked before
    // any write, so a launch after convergence changes nothing.
    const int conv = sc->converged;
    double t[3] = {0.0, 0.0, 0.0};
    {
        const double* in = cg_buf(cg_slots, i);
        if (threadIdx.x < kCgSlots) {
            t[0] = in[threadIdx.x];
            t[1] = in[kCgSlots + threadIdx.x];
            t[2] = in[2 * kCgSlots + threadIdx.x];
        }
    }
    int64_t lb = rg_first(rg);
    const int64_t le = rg_end(rg);
    RowPart P;
    int64_t row = lb * kBlock + threadIdx.x;
    bool active = lb < le && ((row >> 6) << 6) < n_rows;
    if (active) row_part(P, sp, col, A, V, x, dinv, row, row < n_rows);
    if (conv) return;
    block_sum_all<3>(t);
    const double g = t[0], d = t[1], rr = t[2];
    const bool done = !(rr > sc->tol2_bb) || sc->bb == 0.0;
    const double beta = (i == 0) ? 0.0 : g / sc->gam[(i - 1) & 1];
    const double alpha = (i == 0) ? g / d : g / (d - beta * g / sc->alpha[(i - 1) & 1]);
    const bool bad = !done && !(alpha > 0.0 && alpha < INFINITY && beta >= 0.0 && beta < INFINITY);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gam[i & 1] = g;
        sc->alpha[i & 1] = alpha;
        sc->rr = rr;
        sc->iters = i;
        if (i == 0) sc->rr0 = rr;
        if (done) sc->converged = 1;
        if (bad) sc->converged = 2;
    }
    if (done || bad) return;
    if (blockIdx.x == 0)   // read by the previous kernel; the next one adds into it
        for (int k = threadIdx.x; k < 3 * kCgSlots; k += kBlock) cg_buf(cg_slots, i + 2)[k] = 0.0;
    const double ab = alpha * beta;
    double v[3] = {0.0, 0.0, 0.0};
    while (lb < le) {
        if (active && row < n_rows) {
            const double acc = P.sR - alpha * P.sW - ab * P.sS;   // (A u')_j
            const double pj = P.RW.x + beta * P.SP.y;
            const double sj = P.RW.y + beta * P.SP.x;   // D^-1 s
            x[row] = P.x + alpha * pj;
            const double un = P.RW.x - alpha * sj;      // D^-1 r' = u'
            const double rn = un / P.dinv;
            const double wn = P.dinv * acc;
            double2* o = reinterpret_cast<double2*>(V_new + row);
            o[0] = make_double2(un, wn);
            o[1] = make_double2(sj, pj);
            v[0] += rn * un;
            v[1] += un * acc;
            v[2] += rn * rn;
        }
        lb += rg.g;
        row = lb * kBlock + threadIdx.x;
        active = lb < le && ((row >> 6) << 6) < n_rows;
        if (active) row_part(P, sp, col, A, V, x, dinv, row, row < n_rows);
    }
    block_sum_all<3>(v);
    cg_add(cg_buf(cg_slots, i + 1), v);
}

// ------------------------------------------------------------------------------------
// PCG with the nodal auxiliary-space preconditioner of Hiptmair and Xu (2007), additive,
// one Jacobi step in each space:  B r = D^-1 r + G D_G^-1 G^T r + Pi D_Pi^-1 Pi^T r,
// D = diag A, D_G = diag G^T A G, D_Pi = diag Pi^T A Pi, G the discrete gradient and Pi the
// vector nodal interpolation on interior edges and nodes, plus the same two corrections
// for piecewise-constant nodal fields on aggregates of 8, 64 (within a node slice) and
// 512, 4096, 32768 (far levels) Morton-consecutive nodes.  The slow components of
// Jacobi-PCG on the Newmark system are gradients (the kernel of S) and smooth curl
// fields; the nodal spaces reach both.  Plain (Hestenes-Stiefel) recurrences; an
// iteration is three kernels (four with far levels), because z = B r needs the nodal sums
// of the new residual before any edge can form it:
//   k_pcg_q(i):      beta = g_i / g_{i-1};  p = z + beta p;  q = A p (the neighbours' p
//                    formed on the fly from their gathered (z, p) pair);  dot (p, q)
//   k_pcg_nodes(i):  alpha = g_i / (p, q);  per interior node, G^T r' and Pi^T r' over its
//                    edges, r' = r - alpha q, scaled by D_G^-1 and D_Pi^-1, plus the
//                    aggregate levels of the node's slice; the finest far level's sums
//                    by atomics
//   k_pcg_fold(i):   with far levels, the coarser far levels' sums from the finest
//                    level's, then each node's Y += its far aggregates' sums times their
//                    scales (once per node, not at both ends of every edge)
//   k_pcg_update(i): p again (same operands, same bits);  x += alpha p;  r = r';
//                    z = D^-1 r + G y + Pi v (all levels);  dots (r, z), (r, r)
// Every kernel issues its loads before it sums the previous kernel's slots.  Reductions
// use the iteration slots in four rotating buffers: reduction k goes to buffer k mod 4;
// iteration i adds (p, q) as reduction 2i and (r, z), (r, r) as reduction 2i + 1; the
// start's dots are reduction -1.  k_pcg_nodes(i) clears buffer 2i + 1 and
// k_pcg_update(i) buffer 2i + 2, each after that buffer's last reader and before its next
// writer.
__device__ __forceinline__ double* red_buf(double* base, int k) {
    return base + (size_t)(((k % 4) + 4) % 4) * 3 * kCgSlots;
}

template <int NV>
__device__ __forceinline__ void slot_load(const double* buf, double t[NV]) {
#pragma unroll
    for (int j = 0; j < NV; ++j) t[j] = threadIdx.x < kCgSlots ? buf[j * kCgSlots + threadIdx.x] : 0.0;
}

template <int NV>
__device__ __forceinline__ void slot_add(double* buf, const double v[NV]) {
    if (threadIdx.x == 0) {
        const int s = blockIdx.x & (kCgSlots - 1);
#pragma unroll
        for (int j = 0; j < NV; ++j) unsafeAtomicAdd(buf + j * kCgSlots + s, v[j]);
    }
}

__device__ __forceinline__ void clear_buf(double* buf) {
    for (int k = threadIdx.x; k < 3 * kCgSlots; k += kBlock) buf[k] = 0.0;
}

__device__ __forceinline__ double3 edge_vec(const AuxSpace& g, int64_t e) {
    const EdgeVec t = g.th[e];
    return make_double3((double)(float)t.x, (double)(float)t.y, (double)(float)t.z);
}

// Per node: D_G^-1 and D_Pi^-1 from the rows of A.  The pair (e, f) of the node's edges
// contributes s_e A_ef s_f to diag G^T A G (s = +1 at an edge's head, -1 at its tail) and
// th_e,d A_ef th_f,d to component d of diag Pi^T A Pi; f runs over row e's stored columns
// and counts when the node is one of its ends.
__global__ __launch_bounds__(kBlock) void k_aux_scale(AuxSpace g, const int64_t* __restrict__ sp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ A) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.n_aux) return;
    const int64_t sl = n >> 6;
    const int lane = (int)(n & 63);
    double dg = 0.0, dp0 = 0.0, dp1 = 0.0, dp2 = 0.0;
    for (int64_t k = g.sp[sl] + lane; k < g.sp[sl + 1]; k += 64) {
        const int32_t c = g.inc[k];
        if (c == kAuxPad) continue;
        const int32_t e = c >= 0 ? c : ~c;
        const double se = c >= 0 ? 1.0 : -1.0;
        const double3 te = edge_vec(g, e);
        const int64_t esl = e >> 6;
        const int el = e & 63;
        for (int64_t kk = sp[esl] + el; kk < sp[esl + 1]; kk += 64) {
            const int32_t f = col[kk];
            const int2 ef = g.ends[f];
            const double sf = ef.y == n ? 1.0 : (ef.x == n ? -1.0 : 0.0);
            if (sf == 0.0) continue;
            const double a = A[kk];
            const double3 tf = edge_vec(g, f);
            dg += se * a * sf;
            dp0 += (double)te.x * a * (double)tf.x;
            dp1 += (double)te.y * a * (double)tf.y;
            dp2 += (double)te.z * a * (double)tf.z;
        }
    }
    g.scale[n] = make_double4(dg > 0.0 ? 1.0 / dg : 0.0, dp0 > 0.0 ? 1.0 / dp0 : 0.0, dp1 > 0.0 ? 1.0 / dp1 : 0.0,
                              dp2 > 0.0 ? 1.0 / dp2 : 0.0);
}

// Diagonals of the aggregate levels: for aggregate a (aux nodes [a L, (a + 1) L)) the
// G-level basis vector is phi_e = (head of e in a) - (tail of e in a) and the Pi-level one
// psi_e = th_e ((tail in a) + (head in a)); diag = phi^T A phi and psi_d^T A psi_d.  Each
// node adds the terms of its incident edges, an edge with both ends in the aggregate from
// its tail only, into the aggregate's accumulator (zeroed before).
template <int kLog>
__device__ __forceinline__ void coarse_terms(const AuxSpace& g, const int64_t* __restrict__ sp,
                                             const int32_t* __restrict__ col, const double* __restrict__ A,
                                             int64_t n, double out[4]) {
    const int64_t agg = n >> kLog;
    auto in_agg = [&](int32_t k) { return k < g.n_aux && ((int64_t)k >> kLog) == agg; };
    const int64_t sl = n >> 6;
    const int lane = (int)(n & 63);
    double dg = 0.0, dp0 = 0.0, dp1 = 0.0, dp2 = 0.0;
    for (int64_t k = g.sp[sl] + lane; k < g.sp[sl + 1]; k += 64) {
        const int32_t c = g.inc[k];
        if (c == kAuxPad) continue;
        const int32_t e = c >= 0 ? c : ~c;
        const int2 ee = g.ends[e];
        const bool t_in = in_agg(ee.x), h_in = in_agg(ee.y);
        if (c >= 0 && t_in) continue;   // head end of an edge inside the aggregate: its tail counts it
        const double phe = (h_in ? 1.0 : 0.0) - (t_in ? 1.0 : 0.0);
        const double pse = (t_in ? 1.0 : 0.0) + (h_in ? 1.0 : 0.0);
        const double3 te = edge_vec(g, e);
        const int64_t esl = e >> 6;
        const int el = e & 63;
        double rg = 0.0, r0 = 0.0, r1 = 0.0, r2 = 0.0;   // (A phi)_e, (A psi_d)_e
        for (int64_t kk = sp[esl] + el; kk < sp[esl + 1]; kk += 64) {
            const int32_t f = col[kk];
            const int2 ef = g.ends[f];
            const bool ft = in_agg(ef.x), fh = in_agg(ef.y);
            if (!ft && !fh) continue;
            const double a = A[kk];
            const double3 tf = edge_vec(g, f);
            const double phf = (fh ? 1.0 : 0.0) - (ft ? 1.0 : 0.0);
            const double psf = (ft ? 1.0 : 0.0) + (fh ? 1.0 : 0.0);
            rg += a * phf;
            r0 += a * psf * (double)tf.x;
            r1 += a * psf * (double)tf.y;
            r2 += a * psf * (double)tf.z;
        }
        dg += phe * rg;
        dp0 += pse * (double)te.x * r0;
        dp1 += pse * (double)te.y * r1;
        dp2 += pse * (double)te.z * r2;
    }
    out[0] = dg;
    out[1] = dp0;
    out[2] = dp1;
    out[3] = dp2;
}

__device__ __forceinline__ void add4(double4* acc, const double v[4]) {
    double* o = reinterpret_cast<double*>(acc);
#pragma unroll
    for (int k = 0; k < 4; ++k) unsafeAtomicAdd(o + k, v[k]);
}

// Aggregates of 8 and 64 nodes take one atomic per node; the far levels (whole
// workgroups of consecutive nodes per aggregate) one per workgroup.
__global__ __launch_bounds__(kBlock) void k_aux_coarse(AuxSpace g, const int64_t* __restrict__ sp,
                                                        const int32_t* __restrict__ col, const double* __restrict__ A) {
    static_assert(aux_far_log(0) >= 8, "a far aggregate holds whole workgroups");
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool real = n < g.n_aux;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (real) {
        coarse_terms<3>(g, sp, col, A, n, v);
        add4(g.scale8 + (n >> 3), v);
        coarse_terms<6>(g, sp, col, A, n, v);
        add4(g.scale64 + (n >> 6), v);
    }
#pragma unroll
    for (int L = 0; L < kAuxFarLevels; ++L) {
        if (real) {
            static_assert(kAuxFarLevels == 3, "one coarse_terms instance per far level");
            if (L == 0) coarse_terms<aux_far_log(0)>(g, sp, col, A, n, v);
            else if (L == 1) coarse_terms<aux_far_log(1)>(g, sp, col, A, n, v);
            else coarse_terms<aux_far_log(2)>(g, sp, col, A, n, v);
        } else {
            v[0] = v[1] = v[2] = v[3] = 0.0;
        }
        block_sum_all<4>(v);
        if (threadIdx.x == 0) add4(g.far_scale[L] + (((int64_t)blockIdx.x * kBlock) >> aux_far_log(L)), v);
    }
}

// diag -> 1 / diag in place (0 where the diagonal is not positive).
__global__ __launch_bounds__(kBlock) void k_invert_pos(double* v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = v[i] > 0.0 ? 1.0 / v[i] : 0.0;
}

// Zeroes the finest far level's accumulators, the only ones the node pass adds into (one
// workgroup).
__device__ __forceinline__ void clear_far(const AuxSpace& g) {
    if (g.n_far < 1) return;
    const int64_t nf = (g.n_aux + (1ll << aux_far_log(0)) - 1) >> aux_far_log(0);
    double* a = reinterpret_cast<double*>(g.far_acc);
    for (int64_t k = threadIdx.x; k < 4 * nf; k += kBlock) a[8 * k] = 0.0;
}

// The accumulator of component comp of the finest far level's aggregate a: one 64-byte
// line each.
__device__ __forceinline__ double* far_line(const AuxSpace& g, int64_t a, int comp) {
    return reinterpret_cast<double*>(g.far_acc) + 8 * (4 * a + comp);
}

// Storage of the iteration: FP64, or FP32 for the inner solves of the mixed-precision
// form (scalars and dot products stay FP64 either way).
template <typename S>
struct Vec;
template <>
struct Vec<double> {
    using t2 = double2;
    using t3 = double3;
    using t4 = double4;
    static __device__ __forceinline__ double2 two(double a, double b) { return make_double2(a, b); }
    static __device__ __forceinline__ double4 four(double a, double b, double c, double d) {
        return make_double4(a, b, c, d);
    }
};
template <>
struct Vec<float> {
    using t2 = float2;
    using t3 = float3;
    using t4 = float4;
    static __device__ __forceinline__ float2 two(float a, float b) { return make_float2(a, b); }
    static __device__ __forceinline__ float4 four(float a, float b, float c, float d) {
        return make_float4(a, b, c, d);
    }
};

// The FP64 or the FP32 copy of an auxiliary-space array.
template <typename S, typename D, typename F>
__device__ __forceinline__ auto pick(D d, F f) {
    if constexpr (sizeof(S) == 8)
        return d;
    else
        return f;
}

template <typename S>
__device__ __forceinline__ typename Vec<S>::t3 edge_vec_t(const AuxSpace& g, int64_t e) {
    const EdgeVec t = g.th[e];
    typename Vec<S>::t3 v;
    v.x = (S)(float)t.x;
    v.y = (S)(float)t.y;
    v.z = (S)(float)t.z;
    return v;
}

// ||b||^2 from the partials of the kernel that summed it (the right-hand side's, or the
// true residual's for an inner solve); r = b - A x, or with zero_x r = b and x = 0 (the
// inner solves start from zero); q = 0; clears the four reduction buffers and the far
// levels' accumulators.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_pcg_init(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                      const int32_t* __restrict__ col, const S* __restrict__ A,
                                                      const double* __restrict__ b, S* __restrict__ x, bool zero_x,
                                                      S* __restrict__ R, S* __restrict__ Q,
                                                      const double* __restrict__ part_b, double* cg_slots,
                                                      CgScalars* sc, double tol, AuxSpace g) {
    double bb[1];
    read_partials<1>(part_b, gridDim.x, bb);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            sc->bb = bb[0];
            sc->tol2_bb = tol * tol * bb[0];
            sc->converged = 0;
        }
        for (int k = threadIdx.x; k < 4 * 3 * kCgSlots; k += kBlock) cg_slots[k] = 0.0;
        clear_far(g);
    }
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t row = lb * kBlock + threadIdx.x;
        if (((row >> 6) << 6) >= n_rows) continue;
        if (zero_x) {
            if (row < n_rows) {
                R[row] = (S)b[row];
                Q[row] = S(0);
                x[row] = S(0);
            }
            continue;
        }
        if constexpr (sizeof(S) == 8) {
            const double ax = sell_row(sp, col, A, row, [&](int c) { return x[c]; });
            if (row < n_rows) {
                R[row] = b[row] - ax;
                Q[row] = 0.0;
            }
        }
    }
}

// Row j of A p split by the iteration's scalar: sum_k A_jk z_k and sum_k A_jk p_k over
// the stored entries, so the gathers are issued before beta is known; own (z, p).
template <typename S>
struct QPart {
    S sZ, sP;
    typename Vec<S>::t2 own;
};

template <typename S>
__device__ __forceinline__ void q_part(QPart<S>& P, const int64_t* __restrict__ sp, const int32_t* __restrict__ col,
                                       const S* __restrict__ A, const typename Vec<S>::t2* __restrict__ ZP,
                                       int64_t row, bool real) {
    const int64_t sl = row >> 6;
    const int lane = (int)(row & 63);
    const int64_t k1 = sp[sl + 1];
    int64_t k = sp[sl] + lane;
    P.own = ZP[real ? row : 0];
    S z0 = S(0), p0 = S(0), z1 = S(0), p1 = S(0);
    for (; k + (kUnroll - 1) * 64 < k1; k += kUnroll * 64) {
        int c[kUnroll];
        S a[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            c[q] = col[k + 64 * q];
            a[q] = A[k + 64 * q];
        }
        typename Vec<S>::t2 zp[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) zp[q] = ZP[c[q]];
#pragma unroll
        for (int q = 0; q < kUnroll; q += 2) {
            z0 += a[q] * zp[q].x;
            p0 += a[q] * zp[q].y;
            z1 += a[q + 1] * zp[q + 1].x;
            p1 += a[q + 1] * zp[q + 1].y;
        }
    }
    for (; k < k1; k += 64) {
        const S a = A[k];
        const typename Vec<S>::t2 zp = ZP[col[k]];
        z0 += a * zp.x;
        p0 += a * zp.y;
    }
    P.sZ = z0 + z1;
    P.sP = p0 + p1;
}

// The convergence test of iterate i (its (r, r) from reduction 2i - 1), beta, the new
// direction p = z + beta p and q = A p (only q is stored: the update kernel forms the same
// p from the same operands); (p, q) into reduction 2i.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_pcg_q(int64_t n_rows, RowGrid rg, int i, const int64_t* __restrict__ sp,
                                                   const int32_t* __restrict__ col, const S* __restrict__ A,
                                                   const typename Vec<S>::t2* __restrict__ ZP, S* __restrict__ Q,
                                                   double* __restrict__ cg_slots, CgScalars* sc, AuxSpace aux) {
    const int conv = sc->converged;
    double t[2];
    slot_load<2>(red_buf(cg_slots, 2 * i - 1), t);
    int64_t lb = rg_first(rg);
    const int64_t le = rg_end(rg);
    QPart<S> P;
    int64_t row = lb * kBlock + threadIdx.x;
    bool active = lb < le && ((row >> 6) << 6) < n_rows;
    if (active) q_part<S>(P, sp, col, A, ZP, row, row < n_rows);
    if (conv) return;
    block_sum_all<2>(t);
    const double g = t[0], rr = t[1];
    const bool done = !(rr > sc->tol2_bb) || sc->bb == 0.0;
    const double beta = (i == 0) ? 0.0 : g / sc->gam[(i - 1) & 1];
    const bool bad = !done && !(g > 0.0 && g < INFINITY && beta >= 0.0 && beta < INFINITY);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gam[i & 1] = g;
        sc->rr = rr;
        sc->iters = i;
        if (i == 0) sc->rr0 = rr;
        if (done) sc->converged = 1;
        if (bad) sc->converged = 2;
    }
    if (done || bad) return;
    if (blockIdx.x == 0) clear_far(aux);   // read by the previous update, added to by the next node pass
    const S bs = (S)beta;
    double v[1] = {0.0};
    while (lb < le) {
        if (active && row < n_rows) {
            const S p = P.own.x + bs * P.own.y;
            const S q = P.sZ + bs * P.sP;
            Q[row] = q;
            v[0] += (double)p * (double)q;
        }
        lb += rg.g;
        row = lb * kBlock + threadIdx.x;
        active = lb < le && ((row >> 6) << 6) < n_rows;
        if (active) q_part<S>(P, sp, col, A, ZP, row, row < n_rows);
    }
    block_sum_all<1>(v);
    slot_add<1>(red_buf(cg_slots, 2 * i), v);
}

// Sums over a node's edges of s_e r_e, s_e q_e, th_e r_e and th_e q_e (r' = r - alpha q is
// formed once alpha is known).  A workgroup takes one slice of 64 nodes: wave j sums
// slots j, j + 4, j + 8, ... of every node (coalesced loads of the slice's columns), and
// the four partial sums meet in LDS.  Padding entries read edge 0 and count zero.
constexpr int kNodePhases = kBlock / 64;

template <typename S>
__device__ __forceinline__ void node_part(S P[8], const AuxSpace& g, const S* __restrict__ R,
                                          const S* __restrict__ Q, int64_t sl, int lane, int j) {
    const int64_t k0 = g.sp[sl] + lane, k1 = g.sp[sl + 1];
#pragma unroll
    for (int v = 0; v < 8; ++v) P[v] = S(0);
    constexpr int U = 4;   // slots per thread in flight together (about all of a node's share)
    for (int64_t k = k0 + 64 * j; k < k1; k += U * kNodePhases * 64) {
        int32_t c[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t kk = k + (int64_t)q * kNodePhases * 64;
            c[q] = kk < k1 ? g.inc[kk] : kAuxPad;
        }
        S rv[U], qv[U];
        typename Vec<S>::t3 th[U];
        S s[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const bool ok = c[q] != kAuxPad;
            const int32_t e = ok ? (c[q] >= 0 ? c[q] : ~c[q]) : 0;
            s[q] = ok ? (c[q] >= 0 ? S(1) : S(-1)) : S(0);
            rv[q] = R[e];
            qv[q] = Q[e];
            th[q] = edge_vec_t<S>(g, e);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const S r = s[q] != S(0) ? rv[q] : S(0), qq = s[q] != S(0) ? qv[q] : S(0);
            P[0] += s[q] * r;
            P[1] += s[q] * qq;
            P[2] += th[q].x * r;
            P[3] += th[q].y * r;
            P[4] += th[q].z * r;
            P[5] += th[q].x * qq;
            P[6] += th[q].y * qq;
            P[7] += th[q].z * qq;
        }
    }
}

// alpha from reduction 2i (i = -1: the start, alpha = 0); Y = (D_G^-1 G^T r', D_Pi^-1 Pi^T r').
// rg runs over slices of 64 nodes.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_pcg_nodes(RowGrid rg, int i, AuxSpace g, const S* __restrict__ R,
                                                       const S* __restrict__ Q, double* __restrict__ cg_slots,
                                                       CgScalars* sc) {
    __shared__ S part[8][kNodePhases][64];
    const int conv = sc->converged;
    double t[1] = {0.0};
    if (i >= 0) slot_load<1>(red_buf(cg_slots, 2 * i), t);
    const int lane = threadIdx.x & 63, j = threadIdx.x >> 6;
    const int nl = threadIdx.x >> 2, comp = threadIdx.x & 3;   // output: node of the slice, component
    int64_t sl = rg_first(rg);
    const int64_t le = rg_end(rg);
    const S* scale = reinterpret_cast<const S*>(pick<S>(g.scale, g.scale_f));
    const S* scale8 = reinterpret_cast<const S*>(pick<S>(g.scale8, g.scale8_f));
    const S* scale64 = reinterpret_cast<const S*>(pick<S>(g.scale64, g.scale64_f));
    // the output's three scales, loaded with the slice's incidences (they depend on nothing
    // else, and would otherwise be a memory round trip of their own after the barrier)
    S d1 = S(0), d8 = S(0), d64 = S(0);
    auto load_scales = [&](int64_t s) {
        const int64_t node = s * 64 + nl;
        if (node < g.n_aux) {
            d1 = scale[4 * node + comp];
            d8 = scale8[4 * (node >> 3) + comp];
            d64 = scale64[4 * s + comp];
        }
    };
    S P[8];
    if (sl < le) {
        load_scales(sl);
        node_part<S>(P, g, R, Q, sl, lane, j);
    }
    if (conv) return;
    double alpha = 0.0;
    if (i >= 0) {
        block_sum_all<1>(t);
        alpha = sc->gam[i & 1] / t[0];
        if (!(alpha > 0.0 && alpha < INFINITY)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) sc->converged = 2;
            return;
        }
    }
    if (blockIdx.x == 0) clear_buf(red_buf(cg_slots, 2 * i + 1));
    const S as = (S)alpha;
    S* Y = reinterpret_cast<S*>(pick<S>(g.Y, g.Y_f));
    __shared__ S wsum[kNodePhases][4];
    // component comp of P^T r' at node nl: (sum of value va) - alpha (sum of value vb)
    const int va = comp == 0 ? 0 : 1 + comp, vb = comp == 0 ? 1 : 4 + comp;
    while (sl < le) {
#pragma unroll
        for (int v = 0; v < 8; ++v) part[v][j][lane] = P[v];
        __syncthreads();
        const int64_t node = sl * 64 + nl;
        S a = S(0), b = S(0);
#pragma unroll
        for (int q = 0; q < kNodePhases; ++q) {
            a += part[va][q][nl];
            b += part[vb][q][nl];
        }
        const S u = a - as * b;   // zero for the padding nodes of the last slice
        // the aggregate of 8 nodes: lanes 4 nl + comp with the same comp and nl >> 3
        S s8 = u;
        s8 += __shfl_xor(s8, 4);
        s8 += __shfl_xor(s8, 8);
        s8 += __shfl_xor(s8, 16);
        // the aggregate of 64 nodes (the slice): the wave's two groups, then the four waves
        S s16 = s8 + __shfl_xor(s8, 32);
        if (lane < 4) wsum[j][lane] = s16;
        __syncthreads();
        S s64 = S(0);
#pragma unroll
        for (int q = 0; q < kNodePhases; ++q) s64 += wsum[q][comp];
        if (node < g.n_aux) Y[4 * node + comp] = u * d1 + s8 * d8 + s64 * d64;
        // Far levels: the slice's sums added into its aggregate of the finest far level
        // (each component of an aggregate has its own 64-byte line, so eight workgroups add
        // into one line); the coarser far levels' sums are formed from those by the fold.
        if (threadIdx.x < 4 && g.n_far > 0)   // comp = threadIdx.x
            unsafeAtomicAdd(far_line(g, (sl * 64) >> aux_far_log(0), comp), (double)s64);
        __syncthreads();
        sl += rg.g;
        if (sl < le) {
            load_scales(sl);
            node_part<S>(P, g, R, Q, sl, lane, j);
        }
    }
}

// A row's own values for the update.
template <typename S>
struct UPart {
    S r, q;
    typename Vec<S>::t2 zp;
    S x, dinv;
    typename Vec<S>::t3 th;
    typename Vec<S>::t4 ya, yb;
};

template <typename S>
__device__ __forceinline__ void u_part(UPart<S>& P, const AuxSpace& g, const S* __restrict__ dinv,
                                       const S* __restrict__ x, const typename Vec<S>::t2* __restrict__ ZP,
                                       const S* __restrict__ R, const S* __restrict__ Q, int64_t row) {
    P.r = R[row];
    P.q = Q[row];
    P.zp = ZP[row];
    P.x = x[row];
    P.dinv = dinv[row];
    P.th = edge_vec_t<S>(g, row);
    const int2 en = g.ends[row];
    const typename Vec<S>::t4* Y = pick<S>(g.Y, g.Y_f);
    P.ya = Y[en.x];   // the far levels' corrections are already folded in (k_pcg_fold)
    P.yb = Y[en.y];
}

// The far levels' corrections folded into each node's Y once, after the node pass has
// summed the finest far level's aggregates and before the update reads Y at both ends of
// every edge: Y += (the aggregate's sum) * (its scale), level by level.  The coarser
// levels' sums are those of their eight (level 1) and 64 (level 2) finest aggregates: a
// workgroup's 256 nodes lie in one aggregate of each far level, so thread t loads
// component t & 3 of the (t >> 2)-th finest aggregate of its level-2 aggregate, groups of
// eight are summed across lanes and the groups in LDS.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_pcg_fold(AuxSpace g, const CgScalars* __restrict__ sc) {
    static_assert(kBlock == 256 && aux_far_log(0) >= 8 && aux_far_log(1) == aux_far_log(0) + 3 &&
                      aux_far_log(2) == aux_far_log(0) + 6 && kAuxFarLevels == 3,
                  "one workgroup's nodes in one aggregate per far level; 8 and 64 finest ones per coarser");
    if (sc->converged) return;   // a stopped solve's node pass left Y as it was (uniform)
    const int64_t n0 = (int64_t)blockIdx.x * kBlock, n = n0 + threadIdx.x;
    double c1[4] = {0.0, 0.0, 0.0, 0.0}, c2[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.n_far > 1) {
        __shared__ double grp[8][4];
        const int comp = threadIdx.x & 3, lane = threadIdx.x & 63;
        const int64_t nf0 = (g.n_aux + (1ll << aux_far_log(0)) - 1) >> aux_far_log(0);
        const int64_t a = ((n0 >> aux_far_log(2)) << 6) + (threadIdx.x >> 2);
        double v = a < nf0 ? *far_line(g, a, comp) : 0.0;
        v += __shfl_xor(v, 4);    // lanes 4k + comp: the eight consecutive k of one group
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 16);
        if ((lane & 28) == 0) grp[threadIdx.x >> 5][comp] = v;   // group (threadIdx.x >> 2) >> 3
        __syncthreads();
        const int q1 = (int)((n0 >> aux_far_log(1)) & 7);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            c1[c] = grp[q1][c];
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) t += grp[q][c];
            c2[c] = t;
        }
    }
    if (n >= g.n_aux) return;
    typename Vec<S>::t4* Y = pick<S>(g.Y, g.Y_f);
    typename Vec<S>::t4 y = Y[n];
#pragma unroll
    for (int L = 0; L < kAuxFarLevels; ++L) {
        if (L >= g.n_far) break;
        const typename Vec<S>::t4* fs = pick<S>(g.far_scale[L], g.far_scale_f[L]);
        const int64_t a = n >> aux_far_log(L);
        const typename Vec<S>::t4 d = fs[a];
        double f[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) f[c] = L == 0 ? *far_line(g, a, c) : (L == 1 ? c1[c] : c2[c]);
        y.x += (S)f[0] * d.x;
        y.y += (S)f[1] * d.y;
        y.z += (S)f[2] * d.z;
        y.w += (S)f[3] * d.w;
    }
    Y[n] = y;
}

// x += alpha p with p = z + beta p from the pair k_pcg_q(i) read (not at the start),
// r' = r - alpha q, z' = D^-1 r' + G y + Pi v; the pair (z', p) into the other buffer;
// (r', z') and (r', r') into reduction 2i + 1.  Each workgroup takes one block of kR
// consecutive groups of kBlock rows (the grid covers all rows), and each thread issues the
// loads of its kR rows together: the FP32 form, whose rows carry fewer bytes, takes two.
template <typename S, int kR>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int64_t n_rows, RowGrid rg, int i, AuxSpace g,
                                                        const S* __restrict__ dinv, S* __restrict__ x,
                                                        const typename Vec<S>::t2* __restrict__ ZP,
                                                        typename Vec<S>::t2* __restrict__ ZPn, S* __restrict__ R,
                                                        const S* __restrict__ Q, double* __restrict__ cg_slots,
                                                        CgScalars* sc) {
    const int conv = sc->converged;
    double t[1] = {0.0};
    if (i >= 0) slot_load<1>(red_buf(cg_slots, 2 * i), t);
    const int64_t lb = rg_first(rg);
    const int64_t le = rg_end(rg);
    UPart<S> P[kR];
    bool act[kR];
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        const int64_t row = (lb * kR + k) * kBlock + threadIdx.x;
        act[k] = lb < le && row < n_rows;
        if (act[k]) u_part<S>(P[k], g, dinv, x, ZP, R, Q, row);
    }
    if (conv) return;
    double alpha = 0.0;
    if (i >= 0) {
        block_sum_all<1>(t);
        alpha = sc->gam[i & 1] / t[0];
        if (!(alpha > 0.0 && alpha < INFINITY)) return;
    }
    // beta of this iteration, from the same operands as in k_pcg_q (the same bits)
    const double beta = (i <= 0) ? 0.0 : sc->gam[i & 1] / sc->gam[(i - 1) & 1];
    if (blockIdx.x == 0) clear_buf(red_buf(cg_slots, 2 * i + 2));
    const S as = (S)alpha, bs = (S)beta;
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        if (!act[k]) continue;
        const int64_t row = (lb * kR + k) * kBlock + threadIdx.x;
        const UPart<S>& U = P[k];
        const S r = U.r - as * U.q;
        const S p = i >= 0 ? U.zp.x + bs * U.zp.y : S(0);
        if (i >= 0) x[row] = U.x + as * p;
        const S z = U.dinv * r + (U.yb.x - U.ya.x) + U.th.x * (U.ya.y + U.yb.y) + U.th.y * (U.ya.z + U.yb.z) +
                    U.th.z * (U.ya.w + U.yb.w);
        R[row] = r;
        ZPn[row] = Vec<S>::two(z, p);
        v[0] += (double)r * (double)z;
        v[1] += (double)r * (double)r;
    }
    block_sum_all<2>(v);
    slot_add<2>(red_buf(cg_slots, 2 * i + 1), v);
}

// Rows per thread of the update kernel.
template <typename S>
constexpr int update_rows() { return sizeof(S) == 4 ? 2 : 1; }

// ||b||^2 and the tolerance from the right-hand side's partials (one workgroup).
__global__ __launch_bounds__(kBlock) void k_rhs_norm(const double* __restrict__ part_b, int n_src, CgScalars* sc,
                                                      double tol) {
    double bb[1];
    read_partials<1>(part_b, n_src, bb);
    if (threadIdx.x == 0) {
        sc->bb = bb[0];
        sc->tol2_bb = tol * tol * bb[0];
        sc->converged = 0;
    }
}

// FP32 copy of n values; x += d (FP64 from FP32).
__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ __launch_bounds__(kBlock) void k_add_f32(double* __restrict__ x, const float* __restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] += (double)d[i];
}

__global__ __launch_bounds__(kBlock) void k_zero_if_b_zero(double* x, int64_t n, const CgScalars* sc) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && sc->bb == 0.0) x[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_cg_resid(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                      const int32_t* __restrict__ col, const double* __restrict__ A,
                                                      const double* __restrict__ b, const double* __restrict__ x,
                                                      double* __restrict__ rt, double* __restrict__ partial) {
    double v[1] = {0.0};
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t row = lb * kBlock + threadIdx.x;
        if (((row >> 6) << 6) >= n_rows) continue;
        const double ax = sell_row(sp, col, A, row, [&](int c) { return x[c]; });
        if (row < n_rows) {
            const double d = b[row] - ax;
            rt[row] = d;
            v[0] += d * d;
        }
    }
    write_partials<1>(v, partial);
}

// One workgroup: sum n_src partials into *out.
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partial, int n_src, double* out) {
    double t[1];
    read_partials<1>(partial, n_src, t);
    if (threadIdx.x == 0) *out = t[0];
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

// Largest |v| over the workgroup (values as ordered bit patterns), then one atomicMax by
// thread 0: same-address atomics from every thread would serialize at the memory side.
template <int NV>
__device__ __forceinline__ void block_max_abs(const double v[NV], unsigned long long* const out[NV]) {
    __shared__ unsigned long long s[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        unsigned long long m = (unsigned long long)__double_as_longlong(fabs(v[j]));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(m, off);
            m = o > m ? o : m;
        }
        if (lane == 0) s[j][w] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            unsigned long long m = 0;
            for (int q = 0; q < kBlock / 64; ++q) m = s[j][q] > m ? s[j][q] : m;
            if (m) atomicMax(out[j], m);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_diag_nodes(int64_t n_nodes, const uint8_t* __restrict__ interior,
                                                        const double* __restrict__ rho_new,
                                                        const double* __restrict__ rho_old,
                                                        const double* __restrict__ dtdg,
                                                        const double* __restrict__ dtMe,
                                                        const double* __restrict__ rG1, const double* __restrict__ rG2,
                                                        const double* __restrict__ dtrcg, int have_hist,
                                                        double c1, double c2, double* __restrict__ rG_out,
                                                        DiagAcc* acc) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};   // continuity, Gauss, rho, drift
    if (k < n_nodes) {
        if (!interior[k]) {
            rG_out[k] = 0.0;
        } else {
            const double rc = (rho_new[k] - rho_old[k]) - dtdg[k];
            const double rg = -dtMe[k] - rho_new[k];
            rG_out[k] = rg;
            v[0] = rc;
            v[1] = rg;
            v[2] = rho_new[k];
            if (have_hist) v[3] = (rg + c1 * rG1[k] + c2 * rG2[k]) - dtrcg[k];
        }
    }
    unsigned long long* const out[4] = {&acc->cont_max, &acc->gauss_max, &acc->rho_max, &acc->drift_max};
    block_max_abs<4>(v, out);
}

__global__ __launch_bounds__(kBlock) void k_divb(int64_t n_tets, const int32_t* __restrict__ tf,
                                                  const double* __restrict__ b, DiagAcc* acc) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (t < n_tets) v[0] = b[tf[4 * t]] - b[tf[4 * t + 1]] + b[tf[4 * t + 2]] - b[tf[4 * t + 3]];
    unsigned long long* const out[1] = {&acc->divb_max};
    block_max_abs<1>(v, out);
}

__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, RowGrid rg, const double* __restrict__ a,
                                                 const double* __restrict__ b, double* __restrict__ partial) {
    double v[1] = {0.0};
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t i = lb * kBlock + threadIdx.x;
        if (i < n) v[0] += a[i] * b[i];
    }
    write_partials<1>(v, partial);
}

// Energy-norm step along a given direction d from e: x = e + theta d with
// theta = d.(b - A e) / d.A d = (b.d - e.(A d)) / (d.A d) (A symmetric), the minimiser of
// the A-norm error over the line, so x is never farther from the solution than e.
__global__ __launch_bounds__(kBlock) void k_line_dots(int64_t n_rows, RowGrid rg, const int64_t* __restrict__ sp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ A,
                                                       const double* __restrict__ b, const double* __restrict__ e,
                                                       const double* __restrict__ d, double* __restrict__ partial) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t lb = rg_first(rg), le = rg_end(rg); lb < le; lb += rg.g) {
        const int64_t row = lb * kBlock + threadIdx.x;
        if (((row >> 6) << 6) >= n_rows) continue;
        const double ad = sell_row(sp, col, A, row, [&](int c) { return d[c]; });
        if (row < n_rows) {
            v[0] += b[row] * d[row];
            v[1] += e[row] * ad;
            v[2] += d[row] * ad;
        }
    }
    write_partials<3>(v, partial);
}

__global__ __launch_bounds__(kBlock) void k_line_theta(const double* __restrict__ partial, int n_src,
                                                        double* __restrict__ theta) {
    double t[3];
    read_partials<3>(partial, n_src, t);
    if (threadIdx.x == 0) theta[0] = (t[2] > 0.0 && isfinite(t[0] - t[1])) ? (t[0] - t[1]) / t[2] : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_line_apply(int64_t n, const double* __restrict__ e,
                                                        const double* __restrict__ d,
                                                        const double* __restrict__ theta, double* __restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = e[i] + theta[0] * d[i];
}

// Partial-buffer slots (each holds up to 3 values per workgroup of the largest grid).
constexpr size_t kSlot = 4 * kMaxGrid;
enum { SLOT_RHS = 0, SLOT_CG, SLOT_RESID, SLOT_DOT, SLOT_COUNT };
static_assert(4 * 3 * kCgSlots <= kSlot, "iteration slots fit one partial region");

}  // namespace

size_t partial_buffer_doubles() { return SLOT_COUNT * kSlot; }

// ------------------------------------------------------------------------- launchers
void launch_fill(hipStream_t s, double* x, int64_t n, double v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, x, n, v);
}

void launch_axpby(hipStream_t s, double* y, const double* a, double alpha, const double* b, double beta, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, y, a, alpha, b, beta, n);
}

void launch_scale_A(hipStream_t s, const SellMatrix& shape, const int64_t* sp, const int32_t* col, const double* M,
                    const double* S, double* A, double* dinv, const uint8_t* bmask, double c, const double* K,
                    double cK) {
    const int64_t rows = shape.n_slices * kSell;
    hipLaunchKernelGGL(k_scale_A, dim3(grid_1d(rows, kBlock)), dim3(kBlock), 0, s, shape.n_rows, sp, col, M, S, A,
                       dinv, bmask, c, K, cK);
}

void launch_sell_spmv(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* val,
                      const double* x, double* y) {
    hipLaunchKernelGGL(k_spmv, dim3(grid_1d(n_rows, kBlock)), dim3(kBlock), 0, s, n_rows, sp, col, val, x, y);
}

void launch_rhs(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* M,
                const double* S, const double* e, const double* ep, const double* dg_new, const double* dg_old,
                const uint8_t* bmask, double dt2, double c1, double c2, const double* K, double k1, double k2,
                double* b, double* partial) {
    const RowGrid rg = row_grid(n_rows);
    if (K)
        hipLaunchKernelGGL(k_rhs<true>, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, M, S, e, ep, dg_new,
                           dg_old, bmask, dt2, c1, c2, K, k1, k2, b, partial + SLOT_RHS * kSlot);
    else
        hipLaunchKernelGGL(k_rhs<false>, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, M, S, e, ep, dg_new,
                           dg_old, bmask, dt2, c1, c2, K, k1, k2, b, partial + SLOT_RHS * kSlot);
}

void launch_mfem_rhs(hipStream_t s, int64_t n_rows, int64_t n_faces, const int64_t* sp, const int32_t* col,
                     const double* M, const double* S, const double* e, const double* ep, const double* dg_new,
                     const double* dg_old, const uint8_t* bmask, const int64_t* fsp, const int32_t* fcol,
                     const double* fval, const double* b1, double cb1, const double* b2, double cb2,
                     const int64_t* esp, const int32_t* einc, double* h, double dt, double a0, double a1, double s0,
                     double s1, double g0, double g1, double* bvec, double* partial) {
    hipLaunchKernelGGL(k_face_spmv, dim3(grid_1d((n_faces + 63) / 64 * 64, kBlock)), dim3(kBlock), 0, s, n_faces, fsp,
                       fcol, fval, b1, cb1, b2, cb2, h);
    const RowGrid rg = row_grid(n_rows);
    const MfemCoef k{a0, a1, s0, s1, g0, g1};
    hipLaunchKernelGGL(k_mfem_rhs, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, M, S, e, ep, dg_new, dg_old,
                       bmask, esp, einc, h, dt, k, bvec, partial + SLOT_RHS * kSlot);
}

void launch_mfem_faraday(hipStream_t s, int64_t n_faces, const int32_t* face_edges, const double* b_base,
                         const double* e_n, const double* e_nm1, const double* e_np1, double dt, double cn, double cm,
                         double cp, double* b_new) {
    hipLaunchKernelGGL(k_mfem_faraday, dim3(grid_1d(n_faces, kBlock)), dim3(kBlock), 0, s, n_faces, face_edges, b_base,
                       e_n, e_nm1, e_np1, dt, cn, cm, cp, b_new);
}

void launch_warm(hipStream_t s, int mode, int64_t n, const double* e, const double* ep, const double* ep2, double* x) {
    hipLaunchKernelGGL(k_warm, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, mode, n, e, ep, ep2, x);
}

void launch_cg_init(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                    const double* dinv, const double* b, const double* x, CgVec* v, double* partial, CgScalars* sc,
                    double tol, bool det) {
    const RowGrid rg = row_grid(n_rows, det ? kCgSlots : kMaxGrid);
    hipLaunchKernelGGL(k_cg_init_a, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, A, dinv, b, x, v,
                       partial + SLOT_RHS * kSlot, (int)row_grid(n_rows).grid, partial + SLOT_CG * kSlot, sc, tol);
    hipLaunchKernelGGL(k_cg_init_b, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, A, dinv, v,
                       partial + SLOT_CG * kSlot);
}

// One workgroup per block of kBlock rows (the iteration's partials do not grow with the
// grid), consecutive blocks on the same XCD.
inline RowGrid row_grid_full(int64_t n_rows) {
    RowGrid r;
    r.nb = (n_rows + kBlock - 1) / kBlock;
    r.per = (r.nb + 7) / 8;
    r.g = (int)std::max<int64_t>(1, r.per);
    r.grid = 8u * (unsigned)r.g;
    return r;
}

// Iteration i reads the interleaved state from buffer i & 1 and writes buffer (i + 1) & 1.
void launch_cg_iter(hipStream_t s, int i, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                    const double* dinv, double* x, CgVec* const v[2], double* partial, CgScalars* sc, bool det) {
    const RowGrid rg = det ? row_grid(n_rows, kCgSlots) : row_grid_full(n_rows);
    const int a = i & 1, b = 1 - a;
    hipLaunchKernelGGL(k_cg_iter, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, i, sp, col, A, dinv, x, v[a], v[b],
                       partial + SLOT_CG * kSlot, sc);
}

// One workgroup per slice of 64 auxiliary nodes, consecutive slices on the same XCD.
inline RowGrid node_grid(int64_t n_aux) {
    RowGrid r;
    r.nb = (n_aux + 63) / 64;
    r.per = (r.nb + 7) / 8;
    r.g = (int)std::max<int64_t>(1, r.per);
    r.grid = 8u * (unsigned)r.g;
    return r;
}

void launch_aux_scale(hipStream_t s, const AuxSpace& g, const int64_t* sp, const int32_t* col, const double* A) {
    if (g.n_aux <= 0) return;
    const int64_t n8 = 4 * ((g.n_aux + 7) / 8), n64 = 4 * ((g.n_aux + 63) / 64);
    hipLaunchKernelGGL(k_aux_scale, dim3(grid_1d(g.n_aux, kBlock)), dim3(kBlock), 0, s, g, sp, col, A);
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n8, kBlock)), dim3(kBlock), 0, s, reinterpret_cast<double*>(g.scale8), n8,
                       0.0);
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n64, kBlock)), dim3(kBlock), 0, s, reinterpret_cast<double*>(g.scale64),
                       n64, 0.0);
    for (int L = 0; L < kAuxFarLevels; ++L) {
        const int64_t nf = 4 * aux_far_count(g.n_aux, L);
        hipLaunchKernelGGL(k_fill, dim3(grid_1d(nf, kBlock)), dim3(kBlock), 0, s,
                           reinterpret_cast<double*>(g.far_scale[L]), nf, 0.0);
    }
    hipLaunchKernelGGL(k_aux_coarse, dim3(grid_1d(g.n_aux, kBlock)), dim3(kBlock), 0, s, g, sp, col, A);
    hipLaunchKernelGGL(k_invert_pos, dim3(grid_1d(n8, kBlock)), dim3(kBlock), 0, s, reinterpret_cast<double*>(g.scale8),
                       n8);
    hipLaunchKernelGGL(k_invert_pos, dim3(grid_1d(n64, kBlock)), dim3(kBlock), 0, s,
                       reinterpret_cast<double*>(g.scale64), n64);
    for (int L = 0; L < kAuxFarLevels; ++L) {
        const int64_t nf = 4 * aux_far_count(g.n_aux, L);
        hipLaunchKernelGGL(k_invert_pos, dim3(grid_1d(nf, kBlock)), dim3(kBlock), 0, s,
                           reinterpret_cast<double*>(g.far_scale[L]), nf);
    }
}

namespace {
template <typename S>
void pcg_start(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const S* A, const S* dinv,
               const double* b, S* x, bool zero_x, const AuxSpace& g, typename Vec<S>::t2* zp0, S* R, S* Q,
               const double* part_b, double* slots, CgScalars* sc, double tol) {
    const RowGrid rg = row_grid(n_rows);
    hipLaunchKernelGGL(k_pcg_init<S>, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, A, b, x, zero_x, R, Q,
                       part_b, slots, sc, tol, g);
    const RowGrid ng = node_grid(g.n_aux);
    hipLaunchKernelGGL(k_pcg_nodes<S>, dim3(ng.grid), dim3(kBlock), 0, s, ng, -1, g, (const S*)R, (const S*)Q, slots,
                       sc);
    if (g.n_far > 0)
        hipLaunchKernelGGL(k_pcg_fold<S>, dim3(grid_1d(g.n_aux, kBlock)), dim3(kBlock), 0, s, g, sc);
    constexpr int kR = update_rows<S>();
    const RowGrid ug = row_grid_full((n_rows + kR - 1) / kR);
    hipLaunchKernelGGL((k_pcg_update<S, kR>), dim3(ug.grid), dim3(kBlock), 0, s, n_rows, ug, -1, g, dinv, x,
                       (const typename Vec<S>::t2*)zp0, zp0, R, (const S*)Q, slots, sc);
}

template <typename S>
void pcg_iter(hipStream_t s, int i, int64_t n_rows, const int64_t* sp, const int32_t* col, const S* A, const S* dinv,
              S* x, const AuxSpace& g, typename Vec<S>::t2* const zp[2], S* R, S* Q, double* slots, CgScalars* sc) {
    const RowGrid rg = row_grid_full(n_rows);
    const RowGrid ng = node_grid(g.n_aux);
    const int a = i & 1, b = 1 - a;
    hipLaunchKernelGGL(k_pcg_q<S>, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, i, sp, col, A,
                       (const typename Vec<S>::t2*)zp[a], Q, slots, sc, g);
    hipLaunchKernelGGL(k_pcg_nodes<S>, dim3(ng.grid), dim3(kBlock), 0, s, ng, i, g, (const S*)R, (const S*)Q, slots,
                       sc);
    if (g.n_far > 0)
        hipLaunchKernelGGL(k_pcg_fold<S>, dim3(grid_1d(g.n_aux, kBlock)), dim3(kBlock), 0, s, g, sc);
    constexpr int kR = update_rows<S>();
    const RowGrid ug = row_grid_full((n_rows + kR - 1) / kR);
    hipLaunchKernelGGL((k_pcg_update<S, kR>), dim3(ug.grid), dim3(kBlock), 0, s, n_rows, ug, i, g, dinv, x,
                       (const typename Vec<S>::t2*)zp[a], zp[b], R, (const S*)Q, slots, sc);
}
}  // namespace

// The start: r = b - A x, then z = B r and the dots (r, z), (r, r) as reduction -1.
void launch_pcg_init(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                     const double* dinv, const double* b, const double* x, const AuxSpace& g, double2* zp0,
                     double2* rq, double* partial, CgScalars* sc, double tol) {
    double* R = reinterpret_cast<double*>(rq);
    pcg_start<double>(s, n_rows, sp, col, A, dinv, b, const_cast<double*>(x), false, g, zp0, R, R + n_rows,
                      partial + SLOT_RHS * kSlot, partial + SLOT_CG * kSlot, sc, tol);
}

// Iteration i: (z, p) pairs read from buffer i & 1, the new pair written to (i + 1) & 1;
// r in the first n_rows doubles of rq, q in the next n_rows.
void launch_pcg_iter(hipStream_t s, int i, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                     const double* dinv, double* x, const AuxSpace& g, double2* const zp[2], double2* rq,
                     double* partial, CgScalars* sc) {
    double* R = reinterpret_cast<double*>(rq);
    pcg_iter<double>(s, i, n_rows, sp, col, A, dinv, x, g, zp, R, R + n_rows, partial + SLOT_CG * kSlot, sc);
}

// The inner solve of the mixed-precision form: A d = r in FP32 from d = 0, r the FP64
// true residual that launch_cg_resid left in r_true (its norm from that kernel's partials).
void launch_pcg_init_f32(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const float* A32,
                         const float* dinv32, const double* r_true, float* d, const AuxSpace& g, float2* zp0,
                         float* rq, double* partial, CgScalars* sc, double tol) {
    pcg_start<float>(s, n_rows, sp, col, A32, dinv32, r_true, d, true, g, zp0, rq, rq + n_rows,
                     partial + SLOT_RESID * kSlot, partial + SLOT_CG * kSlot, sc, tol);
}

void launch_pcg_iter_f32(hipStream_t s, int i, int64_t n_rows, const int64_t* sp, const int32_t* col,
                         const float* A32, const float* dinv32, float* d, const AuxSpace& g, float2* const zp[2],
                         float* rq, double* partial, CgScalars* sc) {
    pcg_iter<float>(s, i, n_rows, sp, col, A32, dinv32, d, g, zp, rq, rq + n_rows, partial + SLOT_CG * kSlot, sc);
}

// FP32 copies of the operator for the inner solves: A (all nnz stored slots), D^-1, and the
// auxiliary space's inverse diagonals at every level.
void launch_operator_f32(hipStream_t s, int64_t nnz, const double* A, float* A32, int64_t n_rows, const double* dinv,
                         float* dinv32, const AuxSpace& g) {
    auto cvt = [&](const void* a, void* b, int64_t n) {
        if (n > 0)
            hipLaunchKernelGGL(k_to_f32, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s,
                               reinterpret_cast<const double*>(a), reinterpret_cast<float*>(b), n);
    };
    cvt(A, A32, nnz);
    cvt(dinv, dinv32, n_rows);
    cvt(g.scale, g.scale_f, 4 * g.n_aux);
    cvt(g.scale8, g.scale8_f, 4 * ((g.n_aux + 7) / 8));
    cvt(g.scale64, g.scale64_f, 4 * ((g.n_aux + 63) / 64));
    for (int L = 0; L < kAuxFarLevels; ++L) cvt(g.far_scale[L], g.far_scale_f[L], 4 * aux_far_count(g.n_aux, L));
}

void launch_pcg_rhs_norm(hipStream_t s, int64_t n_rows, double* partial, CgScalars* sc, double tol) {
    hipLaunchKernelGGL(k_rhs_norm, dim3(1), dim3(kBlock), 0, s, partial + SLOT_RHS * kSlot, (int)row_grid(n_rows).grid,
                       sc, tol);
}

void launch_add_f32(hipStream_t s, double* x, const float* d, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_add_f32, dim3(grid_1d(n, kBlock)), dim3(kBlock), 0, s, x, d, n);
}

void launch_pcg_rr0(hipStream_t s, double* partial, CgScalars* sc) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partial + SLOT_CG * kSlot + 3 * 3 * kCgSlots + kCgSlots,
                       kCgSlots, &sc->rr0);
}

void launch_cg_rr0(hipStream_t s, int64_t n_rows, double* partial, CgScalars* sc) {
    (void)n_rows;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partial + SLOT_CG * kSlot + 2 * kCgSlots, kCgSlots,
                       &sc->rr0);
}

void launch_cg_resid(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                     const double* b, double* x, double* r_true, double* partial, CgScalars* sc) {
    hipLaunchKernelGGL(k_zero_if_b_zero, dim3(grid_1d(n_rows, kBlock)), dim3(kBlock), 0, s, x, n_rows, sc);
    const RowGrid rg = row_grid(n_rows);
    hipLaunchKernelGGL(k_cg_resid, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, A, b, x, r_true,
                       partial + SLOT_RESID * kSlot);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partial + SLOT_RESID * kSlot, (int)rg.grid,
                       &sc->rr_true);
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
                       const double* rG2, const double* dtrcg, int have_hist, double c1, double c2, double* rG_out,
                       DiagAcc* acc) {
    hipLaunchKernelGGL(k_diag_nodes, dim3(grid_1d(n_nodes, kBlock)), dim3(kBlock), 0, s, n_nodes, interior_node,
                       rho_new, rho_old, dtdg, dtMe, rG1, rG2, dtrcg, have_hist, c1, c2, rG_out, acc);
}

void launch_divb(hipStream_t s, int64_t n_tets, const int32_t* tet_faces, const double* b, DiagAcc* acc) {
    hipLaunchKernelGGL(k_divb, dim3(grid_1d(n_tets, kBlock)), dim3(kBlock), 0, s, n_tets, tet_faces, b, acc);
}

void launch_line_start(hipStream_t s, int64_t n_rows, const int64_t* sp, const int32_t* col, const double* A,
                       const double* b, const double* e, const double* d, double* partial, double* theta, double* x) {
    const RowGrid rg = row_grid(n_rows);
    hipLaunchKernelGGL(k_line_dots, dim3(rg.grid), dim3(kBlock), 0, s, n_rows, rg, sp, col, A, b, e, d,
                       partial + SLOT_DOT * kSlot);
    hipLaunchKernelGGL(k_line_theta, dim3(1), dim3(kBlock), 0, s, partial + SLOT_DOT * kSlot, (int)rg.grid, theta);
    hipLaunchKernelGGL(k_line_apply, dim3(grid_1d(n_rows, kBlock)), dim3(kBlock), 0, s, n_rows, e, d, theta, x);
}

void launch_dot(hipStream_t s, int64_t n, const double* a, const double* b, double* partial, double* out) {
    const RowGrid rg = row_grid(n);
    hipLaunchKernelGGL(k_dot, dim3(rg.grid), dim3(kBlock), 0, s, n, rg, a, b, partial + SLOT_DOT * kSlot);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partial + SLOT_DOT * kSlot, (int)rg.grid, out);
}

}  // namespace fepic
