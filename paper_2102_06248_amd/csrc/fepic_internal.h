// Internal declarations shared by the host side and the HIP kernels of libfepic.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fepic.h"

namespace fepic {

// SI constants (CODATA 2018).
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kC = 299792458.0;
constexpr double kQe = 1.602176634e-19;   // elementary charge (exact); eV -> J

// Sliced-ELLPACK slice height: one 64-lane wavefront per slice of 64 consecutive rows,
// each of the slice's columns stored contiguously so a wave's loads coalesce.
constexpr int kSell = 64;

// Per-tet record read by the particle kernel: the staged field (edge DoFs, constant B)
// and the static geometry/topology, padded to a whole number of 64-byte lines.
template <typename T>
struct TetBlock {
    T e[6];           // edge unknowns of local edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
    T B[3];           // B inside the tet (Whitney-2 field of a div-free flux is constant)
    T gl[9];          // grad lambda_1..3 (grad lambda_0 = -sum)
    int32_t nbr[4];   // (neighbour tet << 2) | neighbour's local index of its far vertex;
                      // -1 = wall
    int32_t edge[6];  // global edge ids of the 6 local edges
    int32_t pad[sizeof(T) == 4 ? 4 : 2];
};
static_assert(sizeof(TetBlock<float>) == 128, "TetBlock<float> layout");
static_assert(sizeof(TetBlock<double>) == 192, "TetBlock<double> layout");

// Structure-of-arrays particle storage for one species (one buffer of a double buffer).
template <typename T>
struct PArrays {
    int32_t* tet;     // -1 = dead (absorbed or rejected)
    T* l1;
    T* l2;
    T* l3;            // barycentric coordinates 1..3 in the sorted tet (lambda_0 = 1 - sum)
    T* u0;
    T* u1;
    T* u2;            // gamma v
    int64_t* id;
};

// Particles whose path crosses a face in the first kernel of the particle step, queued
// for the second: SoA, slot blockIdx * 256 + rank within the first kernel's workgroup
// (capacity = its grid * 256), with the per-workgroup counts in wg_count.
template <typename T>
struct CrossQueue {
    double *l0, *l1, *l2, *l3;  // barycentric start in the entered tet
    double* frac;               // fraction of the step's displacement still to go
    T *dx0, *dx1, *dx2;         // the step's displacement
    int32_t *idx, *tet, *entry; // particle slot, entered tet, its local index of the entry face
    int32_t* wg_count;
};

struct PushParams {
    double dt;
    double qm_half_dt;   // q dt / (2 m)
    double qw;           // q w (deposit scale)
    int cap;             // crossing cap
    // deterministic mode: currents go to fixed-point accumulators (fixed_point.h) in units
    // of 1 / fix_inv instead of the FP64 vector; nullptr otherwise
    unsigned long long* fix = nullptr;
    double fix_inv = 0.0;
};

// The particle kernel adds its per-workgroup counts into kCntSlots copies of the counters
// (workgroup b -> slot b mod kCntSlots); launch_cnt_finish folds them into one.
constexpr int kCntSlots = 256;

// Adams-Bashforth pusher (all-FP64): orders 1..kAbMax, a history of kAbStride doubles per
// particle slot (rings of kAbRing levels of r, v and a), stored component-major: component c
// of slot i at c * capacity + i.  A step uses at most kAbMax levels of a ring and writes its
// new level into the one left over, so the levels of the state before the step survive
// until the step is committed.  Per slot an int32 AbMeta (double-buffered with the
// particle state) holds the levels held and the rings' head, or -1 for a particle without
// history (it starts at order 1 from its current state).
constexpr int kAbMax = 5;
constexpr int kAbRing = kAbMax + 1;
constexpr int kAbStride = 9 * kAbRing;
constexpr double kAbInsideEps = 1e-13;   // a point is in a tet when its smallest lambda >= -eps
constexpr double kAbRootTol = 1e-15;     // width of the final crossing bracket, in steps
__host__ __device__ constexpr int ab_meta(int held, int head) { return held | (head << 8); }
struct AbParams {
    double dt, qm, qw;
    int k, cap;
    unsigned long long* fix = nullptr;    // deterministic mode, as in PushParams
    double fix_inv = 0.0;
    double beta[kAbMax][kAbMax];          // beta[m - 1][j]: the order-m coefficients
    double gl_x[kAbMax + 2][kAbMax + 2];  // row n: the n Gauss-Legendre nodes on [-1, 1]
    double gl_w[kAbMax + 2][kAbMax + 2];  // and weights
};

struct PushCounters {
    unsigned long long n_crossings;
    unsigned int max_crossings;
    unsigned int n_absorbed;
    unsigned int n_cap;
    unsigned int n_rejected;
    unsigned int pad[2];
};

// Scalars of the PCG recurrence, kept on the device between kernels.
struct CgScalars {
    double bb;        // ||b||^2
    double tol2_bb;   // tol^2 ||b||^2
    double gam[2];    // (r,u) of iteration i (slot i & 1)
    double alpha[2];  // step length of iteration i
    double rr;        // r . r of the current iterate
    double rr0;       // ||b - A x0||^2
    double rr_true;   // ||b - A x||^2 at exit
    int converged;    // 1 = tolerance met, 2 = breakdown
    int iters;
};

// Per-row state of the PCG iteration, interleaved so that a neighbour's three gathered
// values (R, W, S) share one 32-byte sector: R = D^-1 r, W = D^-1 w, S = D^-1 s, and the
// row's own search direction P.
struct alignas(32) CgVec {
    double R, W, S, P;
};

// Half edge vector (r_head - r_tail) / 2 of the auxiliary space, divided by the mesh's
// largest such component and rounded to FP16 (a constant factor on Pi cancels in
// Pi diag(Pi^T A Pi)^-1 Pi^T, and every kernel uses the same rounded values).
struct alignas(8) EdgeVec {
    _Float16 x, y, z, w;
};

// Padding entry of the auxiliary space's node incidence lists (no edge).
constexpr int32_t kAuxPad = INT32_MIN;
// log2 of the aggregate sizes of the auxiliary space's levels beyond one node slice.
constexpr int kAuxFarLevels = 3;
__host__ __device__ constexpr int aux_far_log(int L) { return 9 + 3 * L; }   // 512, 4096, 32768 nodes
inline int64_t aux_far_count(int64_t n_aux, int L) { return (n_aux + (1ll << aux_far_log(L)) - 1) >> aux_far_log(L); }
// Far levels chosen from tau^2 = mean over interior rows of beta dt^2 S_jj / M_jj (how many
// cells a wave crosses in a step, squared): the level of 2^k nodes (about 2^(k/3) cells
// across) is used when tau >= 2 * 2^(k/3) and the mesh holds at least 16 such aggregates
// (fewer, nearly global ones add cost and no convergence).
inline int aux_far_auto(double tau2, int64_t n_aux) {
    int n = 0;
    while (n < kAuxFarLevels && tau2 >= 4.0 * std::exp2(2.0 * aux_far_log(n) / 3.0) &&
           n_aux >= (int64_t)16 << aux_far_log(n))
        ++n;
    return n;
}

// Device arrays of the nodal auxiliary space of the Newmark preconditioner
// B = diag(A)^-1 + G diag(G^T A G)^-1 G^T + Pi diag(Pi^T A Pi)^-1 Pi^T, with G the discrete
// gradient and Pi the vector nodal interpolation, both on interior edges and nodes.
struct AuxSpace {
    int64_t n_aux = 0;            // interior nodes
    const int64_t* sp = nullptr;  // SELL-64 slice offsets of the node incidence lists
    const int32_t* inc = nullptr; // device edge id (node is its head) or ~id (tail); kAuxPad
    const EdgeVec* th = nullptr;  // [n_edges] scaled (r_head - r_tail) / 2; zero on wall edges
    const int2* ends = nullptr;   // [n_edges] auxiliary index of tail, head (n_aux: zero entry)
    double4* scale = nullptr;     // [n_aux] 1/diag(G^T A G), 1/diag(Pi^T A Pi) for x, y, z
    // the same for the aggregates of 8 and of 64 consecutive auxiliary nodes (the coarser
    // levels: summed hat functions for G, constant vectors for Pi)
    double4* scale8 = nullptr;    // [ceil(n_aux / 8)]
    double4* scale64 = nullptr;   // [ceil(n_aux / 64)]
    // levels of 2^aux_far_log(L) nodes, which span several workgroups of the node pass: the
    // residual's sums per aggregate of the finest far level are accumulated with atomics
    // (far_acc: a 64-byte line per aggregate and component, the sum in its first double;
    // zeroed by the product kernel of each iteration); the coarser levels' sums are formed
    // from those, and all are folded into each node's Y once per iteration
    double4* far_scale[kAuxFarLevels] = {};
    double4* far_acc = nullptr;                 // [8 * count of level 0] double4
    int n_far = 0;                              // far levels in use (0 .. kAuxFarLevels)
    double4* Y = nullptr;         // [n_aux + 1] nodal corrections of the residual, all levels;
                                  // Y[n_aux] = 0
    // FP32 copies for the inner solves of the mixed-precision form (null until first used)
    float4* scale_f = nullptr;
    float4* scale8_f = nullptr;
    float4* scale64_f = nullptr;
    float4* far_scale_f[kAuxFarLevels] = {};
    float4* Y_f = nullptr;        // [n_aux + 1], Y_f[n_aux] = 0
};

// Device-side diagnostics accumulators (max-abs values stored as ordered bit patterns).
struct DiagAcc {
    unsigned long long cont_max, gauss_max, drift_max, rho_max, divb_max;
    double energy;            // e^T M e
    double magnetic, kinetic; // joules
    unsigned int counter;
    unsigned int pad;
};

struct SellMatrix {
    int64_t n_rows = 0;
    int64_t n_slices = 0;
    std::vector<int64_t> slice_ptr;  // [n_slices + 1], element offsets
    std::vector<int32_t> col;        // padded entries point at the row itself, value 0
    std::vector<double> M, S;        // edge mass and curl-curl values
    std::vector<double> K;           // boundary matrix of absorbing faces (empty: none)
};

// ----------------------------------------------------------------------------- launchers
// Particle kernels (kernels_particles.hip).
template <typename T>
void launch_stage(hipStream_t s, int64_t n_tets, TetBlock<T>* blk, const double* e, const double* b,
                  const double* grad64, const int32_t* tet_edges, const int32_t* tet_faces);
template <typename T>
void launch_push(hipStream_t s, PArrays<T> in, PArrays<T> out, int64_t n, const TetBlock<T>* blk, double* dg,
                 PushParams pp, PushCounters* cnt, const int32_t* n_live, CrossQueue<T> cq, double cross_share,
                 double own_share, int walk);
void launch_cnt_finish(hipStream_t s, PushCounters* slots, PushCounters* out);
// The face crossings the slots hold so far (summed over the slots) into out[0], the
// absorptions and paths stopped at the crossing cap into out[1].
void launch_cnt_crossings(hipStream_t s, const PushCounters* slots, unsigned long long* out);
template <typename T>
void launch_locate(hipStream_t s, int64_t n, const double* x, const double* u, const int64_t* id, int64_t id_base,
                   PArrays<T> out, int64_t out_off, const double* grad64, const double* r0, const int32_t* cell_start,
                   const int32_t* cell_tets, const double* grid_lo, const double* grid_inv_h, const int32_t* grid_n,
                   PushCounters* cnt);
// Seeded disk source (fepic_set_injector, kernels_inject.hip): centre, unit normal, the
// in-plane basis e1 = unit(n x a), e2 = n x e1, radius, drift speed, thermal spread.
struct InjectorSpec {
    double c[3], n[3], e1[3], e2[3];
    double radius, v0, sigma;
    int64_t per_step;
    uint64_t seed;
    int species;
    int relativistic_u;   // store gamma v (Boris) rather than v (Adams-Bashforth)
};
void launch_inject_disk(hipStream_t s, const InjectorSpec& spec, int64_t k, double* x, double* u);
// The Adams-Bashforth history moved by a sort with the particles it belongs to (hin ==
// nullptr: no history); both history buffers have `stride` slots per component.
struct AbHistIo {
    const double* hin = nullptr;
    double* hout = nullptr;
    int64_t stride = 0;
    const int32_t* min = nullptr;
    int32_t* mout = nullptr;
};
template <typename T>
void launch_sort(hipStream_t s, PArrays<T> in, PArrays<T> out, int64_t n, int64_t n_tets, int32_t* count,
                 int32_t* offset, int32_t* block_sums, int32_t* n_live_dev, AbHistIo ab = AbHistIo());
// rho += q w lambda per particle (FP64 atomics), or with fix into fixed-point accumulators
// in units of 1 / fix_inv (deterministic mode; rho untouched).
template <typename T>
void launch_rho(hipStream_t s, PArrays<T> p, int64_t n, const int32_t* tets, double qw, double* rho,
                unsigned long long* fix = nullptr, double fix_inv = 0.0);
// out[i] = accumulator i times scale, and the accumulators cleared (fixed_point.h).
void launch_fix_out(hipStream_t s, unsigned long long* acc, int64_t n, double scale, double* out);
void launch_magnetic(hipStream_t s, int64_t n_tets, const double* b, const double* grad64, const int32_t* tet_faces,
                     double* out);
template <typename T>
void launch_kinetic(hipStream_t s, PArrays<T> p, int64_t n, double wmc2, double* out);
void launch_count_live(hipStream_t s, const int32_t* tet, int64_t n, double* out);
// Adams-Bashforth pusher (kernels_ab.hip): state read from in, written to out, the new
// history level into the free ring slot of hist, the new AbMeta into meta_out.
void launch_push_ab(hipStream_t s, PArrays<double> in, PArrays<double> out, int64_t n,
                    const TetBlock<double>* blk, const double* r0, double* hist, int64_t hstride,
                    const int32_t* meta_in, int32_t* meta_out, double* dg, const AbParams& ap, PushCounters* slots,
                    const int32_t* n_live);
void launch_fill_i32(hipStream_t s, int32_t* x, int64_t n, int32_t v);

// Field kernels (kernels_fields.hip).
void launch_fill(hipStream_t s, double* x, int64_t n, double v);
void launch_axpby(hipStream_t s, double* y, const double* a, double alpha, const double* b, double beta, int64_t n);
void launch_scale_A(hipStream_t s, const SellMatrix& shape, const int64_t* slice_ptr, const int32_t* col,
                    const double* M, const double* S, double* A, double* dinv, const uint8_t* bmask, double c,
                    const double* K = nullptr, double cK = 0.0);
void launch_sell_spmv(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col,
                      const double* val, const double* x, double* y);
void launch_rhs(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col, const double* M,
                const double* S, const double* e, const double* ep, const double* dg_new, const double* dg_old,
                const uint8_t* bmask, double dt2, double c1, double c2, const double* K, double k1, double k2,
                double* b, double* partial);
void launch_warm(hipStream_t s, int mode, int64_t n, const double* e, const double* ep, const double* ep2, double* x);
void launch_cg_init(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col, const double* A,
                    const double* dinv, const double* b, const double* x, CgVec* v, double* partial, CgScalars* sc,
                    double tol, bool det = false);
// det: at most one workgroup per dot slot, so every slot takes a single add and the dots
// do not depend on the order of the workgroups (deterministic mode).
void launch_cg_iter(hipStream_t s, int i, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col,
                    const double* A, const double* dinv, double* x, CgVec* const v[2], double* partial,
                    CgScalars* sc, bool det = false);
void launch_cg_rr0(hipStream_t s, int64_t n_rows, double* partial, CgScalars* sc);
// PCG with the nodal auxiliary-space preconditioner: per row z = B r with the previous
// search direction p (zp, double buffered), and r and q = A p as two arrays of n_rows
// doubles in rq (r first; each written whole by one kernel).
void launch_aux_scale(hipStream_t s, const AuxSpace& g, const int64_t* slice_ptr, const int32_t* col,
                      const double* A);
void launch_pcg_init(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col, const double* A,
                     const double* dinv, const double* b, const double* x, const AuxSpace& g, double2* zp0,
                     double2* rq, double* partial, CgScalars* sc, double tol);
void launch_pcg_iter(hipStream_t s, int i, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col,
                     const double* A, const double* dinv, double* x, const AuxSpace& g, double2* const zp[2],
                     double2* rq, double* partial, CgScalars* sc);
void launch_pcg_init_f32(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col,
                         const float* A32, const float* dinv32, const double* r_true, float* d, const AuxSpace& g,
                         float2* zp0, float* rq, double* partial, CgScalars* sc, double tol);
void launch_pcg_iter_f32(hipStream_t s, int i, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col,
                         const float* A32, const float* dinv32, float* d, const AuxSpace& g, float2* const zp[2],
                         float* rq, double* partial, CgScalars* sc);
void launch_operator_f32(hipStream_t s, int64_t nnz, const double* A, float* A32, int64_t n_rows, const double* dinv,
                         float* dinv32, const AuxSpace& g);
void launch_add_f32(hipStream_t s, double* x, const float* d, int64_t n);
void launch_pcg_rhs_norm(hipStream_t s, int64_t n_rows, double* partial, CgScalars* sc, double tol);
void launch_pcg_rr0(hipStream_t s, double* partial, CgScalars* sc);
void launch_cg_resid(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col,
                     const double* A, const double* b, double* x, double* r_true, double* partial,
                     CgScalars* sc);
void launch_faraday(hipStream_t s, int64_t n_faces, const int32_t* face_edges, const double* b_old,
                    const double* e_new, const double* e_old, double dt, double gamma, double* b_new);
void launch_DT(hipStream_t s, int64_t n_edges, const int32_t* edges, const double* v, double* out_nodes);
void launch_diag_nodes(hipStream_t s, int64_t n_nodes, const uint8_t* interior_node, const double* rho_new,
                       const double* rho_old, const double* dtdg, const double* dtMe, const double* rG1,
                       const double* rG2, const double* dtrcg, int have_hist, double c1, double c2, double* rG_out,
                       DiagAcc* acc);
// Mixed (b, e) field updates: face-mass product then the eliminated right-hand side (see
// kernels_fields.hip), and the face flux update.
void launch_mfem_rhs(hipStream_t s, int64_t n_rows, int64_t n_faces, const int64_t* sp, const int32_t* col,
                     const double* M, const double* S, const double* e, const double* ep, const double* dg_new,
                     const double* dg_old, const uint8_t* bmask, const int64_t* fsp, const int32_t* fcol,
                     const double* fval, const double* b1, double cb1, const double* b2, double cb2,
                     const int64_t* esp, const int32_t* einc, double* h, double dt, double a0, double a1, double s0,
                     double s1, double g0, double g1, double* bvec, double* partial);
void launch_mfem_faraday(hipStream_t s, int64_t n_faces, const int32_t* face_edges, const double* b_base,
                         const double* e_n, const double* e_nm1, const double* e_np1, double dt, double cn, double cm,
                         double cp, double* b_new);
void launch_divb(hipStream_t s, int64_t n_tets, const int32_t* tet_faces, const double* b, DiagAcc* acc);
void launch_dot(hipStream_t s, int64_t n, const double* a, const double* b, double* partial, double* out);
size_t partial_buffer_doubles();
void launch_line_start(hipStream_t s, int64_t n_rows, const int64_t* slice_ptr, const int32_t* col, const double* A,
                       const double* b, const double* e, const double* d, double* partial, double* theta, double* x);

// Learned warm start (kernels_mlp.hip).
void mlp_launch_rms(hipStream_t s, int64_t n_int, const int32_t* int_edges, const double* e, const double* ep,
                    const double* dg, double* part, double* scales);
void mlp_launch_features(hipStream_t s, int64_t n_int, const int32_t* int_edges, const double* e,
                         const double* ep, const double* ep2, const double* dg, const double* scales, float* X);
void mlp_launch_forward(hipStream_t s, int64_t n, const float* X, const float* params_f32, float* y);
void mlp_launch_direction(hipStream_t s, int64_t n_int, const int32_t* int_edges, const float* y,
                          const double* scales, double* d);
// Training targets of interior edges r0, r0 + stride, ... (n rows): the increments
// (e_new - e) / scales[0] (s_d), their RMS into scales[3] (work: n doubles, part: 256 doubles of
// scratch); the same rows of a feature array [rows][4] picked into dst.
void mlp_launch_target(hipStream_t s, int64_t n, int64_t r0, int64_t stride, const int32_t* int_edges,
                       const double* e_new, const double* e, double* work, double* part, double* scales, float* t);
void mlp_launch_pick(hipStream_t s, const float* X, int64_t r0, int64_t stride, int64_t n, float* dst);

int grid_1d(int64_t n, int block);

}  // namespace fepic
