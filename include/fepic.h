/*
 * fepic.h - C ABI of the MI355X (gfx950) charge-conserving finite-element PIC hot path.
 *
 * Method: O'Connor, Crawford, Ramachandran, Luginsland, Shanker, "Time Integrator
 * Agnostic Charge Conserving Finite Element PIC" (arXiv:2102.06248).  Each step:
 *   gather E from edge (Whitney-1) and B from face (Whitney-2) unknowns at every
 *   particle (Sec. II-A), push with a relativistic Boris step (Sec. III-B), follow the
 *   straight path through the tetrahedra splitting it at every face (Sec. III-C, Alg. 1),
 *   integrate the Whitney-1 forms along each piece to get the time-integrated current G
 *   (Sec. III-A, eqs. (gaussredo)-(G)), then advance the edge field with the Newmark-beta
 *   wave-equation update whose source is the second difference of G (Sec. II-B, III-A),
 *   solved by preconditioned CG (the paper leaves the solver open: Jacobi, or the nodal
 *   auxiliary-space preconditioner of Hiptmair and Xu 2007), and the face flux with
 *   Faraday's law.
 *
 * Conventions for every entry point:
 *   - Return value: FEPIC_OK (0) or a negative FEPIC_E_* code.  fepic_error_string(code)
 *     names the code; fepic_last_error(ctx) gives the message of the last failure.
 *   - Ownership: the caller owns every buffer it passes; the library copies what it needs
 *     during the call and keeps no caller pointer (fepic_inject_particles_device reads its
 *     device arrays in stream order, see there).  The context owns all device memory it
 *     allocates (hipMalloc, or the caller's allocator from fepic_set_allocator) and frees it
 *     in fepic_destroy.  Pointer arguments are host pointers unless the function's name
 *     says device.
 *   - Threading: one context per host thread; calls on one context must not overlap.
 *   - Units: SI.  Edge unknowns e_i are volts (line integrals of E), face unknowns b_f are
 *     webers (fluxes of B), currents are time-integrated (coulombs).
 *   - Numbering (canonical, independent of the input order of vertices): each tet's node
 *     ids are sorted ascending (local vertex k = k-th smallest); edges are the unique
 *     sorted node pairs in lexicographic order, oriented low -> high id; faces are the
 *     unique sorted node triples in lexicographic order, oriented by the right-hand normal
 *     (r_j - r_i) x (r_k - r_i), i < j < k; local face k of a tet is opposite vertex k.
 *   - Every boundary face is a perfect electric conductor (eq. (dirichlet) with
 *     Psi_D = 0): boundary edge unknowns are held at zero and particles reaching the wall
 *     are absorbed after depositing their current up to it.
 */
#ifndef FEPIC_H
#define FEPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEPIC_ABI_VERSION 8

enum {
    FEPIC_OK = 0,
    FEPIC_E_ARG = -1,               /* null pointer, bad size or enum value            */
    FEPIC_E_MESH = -2,              /* degenerate tet, non-conforming face, bad id      */
    FEPIC_E_STATE = -3,             /* call order (e.g. step before mesh upload)        */
    FEPIC_E_OOM = -4,               /* device or host allocation failed                 */
    FEPIC_E_HIP = -5,               /* HIP runtime error (message in fepic_last_error)  */
    FEPIC_E_CG_NOT_CONVERGED = -6,  /* stats filled, nothing committed                  */
    FEPIC_E_CROSSING_CAP = -7,      /* a path crossed more faces than allowed; nothing  */
                                    /* committed                                        */
    FEPIC_E_IO = -8,                /* checkpoint file error                            */
    FEPIC_E_NO_DEVICE = -9          /* the call needs a device context                  */
};

enum { FEPIC_FP32_PUSH_FP64_ACC = 0, FEPIC_ALL_FP64 = 1 };

/* Warm start of the Newmark solve: previous field, linear or quadratic extrapolation in
 * time, or the per-edge learned predictor (fepic_ws_*) of the increment, s_d y (s_d the
 * RMS of e^n - e^{n-1} over interior edges): FEPIC_WS_MLP takes the energy-norm-optimal
 * step along it, x0 = e^n + theta s_d y (never worse than e^n in the A-norm; falls back to e^n when
 * the start's residual exceeds ||b|| or is not finite); FEPIC_WS_MLP_DIRECT takes the
 * prediction as it is, x0 = e^n + s_d y, as the extrapolations take theirs (falls back to
 * e^n when the start's residual is not finite or exceeds 1e4 ||b||).  Both need trained
 * or set weights; until then they start from e^n. */
enum { FEPIC_WS_PREV = 0, FEPIC_WS_EXTRAP1 = 1, FEPIC_WS_EXTRAP2 = 2, FEPIC_WS_MLP = 3, FEPIC_WS_MLP_DIRECT = 4 };

/* Preconditioner of the Newmark solve.  FEPIC_PC_JACOBI: diag(A)^-1.  FEPIC_PC_AUX: the
 * nodal auxiliary-space preconditioner (Hiptmair and Xu, SIAM J. Numer. Anal. 45, 2007),
 * additive with one Jacobi step per space:
 *   B = diag(A)^-1 + G diag(G^T A G)^-1 G^T + Pi diag(Pi^T A Pi)^-1 Pi^T + coarse levels,
 * G the discrete gradient (edge-node incidence, Sec. II-A) and Pi the interpolation of
 * nodal vector fields into edge unknowns ((r_b - r_a) . (v_a + v_b) / 2), both on interior
 * edges and nodes.  The coarse levels add the same two corrections, again with one Jacobi
 * step, for piecewise-constant nodal fields on aggregates of 8, 64 (always) and 512,
 * 4096, 32768 (aux_far_levels) interior nodes consecutive in Morton order of their
 * positions.
 * Either preconditioner converges to the same tolerance; the auxiliary spaces need
 * several times fewer iterations once dt is well beyond the explicit limit. */
enum { FEPIC_PC_JACOBI = 0, FEPIC_PC_AUX = 1 };

/* Arithmetic of the Newmark solve (Sec. III-A; the paper fixes the tolerance, not how it
 * is met).  FEPIC_SOLVE_FP64: PCG in FP64.  FEPIC_SOLVE_MIXED (needs FEPIC_PC_AUX):
 * iterative refinement: the residual r = b - A x in FP64, then the same PCG in FP32 (A,
 * the preconditioner's diagonals and the iteration vectors rounded to FP32; dot products
 * and step lengths in FP64) on A d = r from d = 0 until its residual has fallen by
 * mixed_inner_tol, or as far as cg_tol needs, then x += d in FP64; repeated until the FP64
 * residual meets cg_tol (at most 8 passes).  The stopping rule, and so the guaranteed
 * accuracy, is the FP64 solve's; an FP32 iteration moves about 40 % fewer bytes, at the
 * price of a few more iterations in all (each pass restarts the Krylov space). */
enum { FEPIC_SOLVE_FP64 = 0, FEPIC_SOLVE_MIXED = 1 };

/* How the particle step finishes paths that cross a face (Sec. III-C, Alg. 1): in a second
 * kernel from a compacted queue of the crossing particles (FEPIC_WALK_QUEUE), or in place
 * in the first kernel (FEPIC_WALK_FUSED: no queue traffic, idle lanes while others walk).
 * FEPIC_WALK_AUTO takes the fused form when the last step had more than 0.5 crossings per
 * particle.  Results agree to the rounding order of the current sums either way. */
enum { FEPIC_WALK_AUTO = 0, FEPIC_WALK_QUEUE = 1, FEPIC_WALK_FUSED = 2 };

/* fepic_options.sort_period: re-bin each species by its own need (see there) */
enum { FEPIC_SORT_AUTO = -1 };

/* Particle pusher of fepic_step and fepic_push_particles.  FEPIC_PUSHER_BORIS: relativistic
 * Boris with straight paths (u = gamma v at t_{n-1/2}).  FEPIC_PUSHER_AB: the paper's own
 * pusher (Sec. III-B, III-C, Alg. 1 and 2): Adams-Bashforth of order ab_order (1..5) of the
 * non-relativistic equations dv/dt = (q/m)(E + v x B), dr/dt = v, with u read and written as
 * the velocity v at t_n; the path over a step is the Lagrange polynomial through r^{n+1}
 * and the last `order` positions, followed cell by cell (exits bracketed by Gauss-Legendre
 * points, then located to 1e-15 of the step where the smallest barycentric coordinate
 * reaches -1e-13; wall faces absorb), and each piece's Whitney-1 path integral, by
 * (order + 1)-point Gauss-Legendre quadrature (exact), is closed onto the face it leaves
 * by with a straight segment, so that D^T dG = q w (lambda_end - lambda_start) holds to
 * round-off (Sec. III-A).  Needs FEPIC_ALL_FP64.  Each particle slot keeps its last five
 * positions, velocities and accelerations; the sort moves them with the particle.  A
 * particle starts at order 1 from its state (after upload or injection) and gains one
 * order per step; every history restarts at order 1 when dt changes (the coefficients
 * assume equally spaced levels), after a Boris step or a pusher switch, and after
 * fepic_load. */
enum { FEPIC_PUSHER_BORIS = 0, FEPIC_PUSHER_AB = 1 };

/* Field update of fepic_step (Sec. II-B; the source is the time-integrated current G in
 * every case, Sec. III-A, so continuity and Gauss hold whichever is used).
 * FEPIC_FIELD_WAVE: the Newmark(beta, gamma) wave equation for e (step's beta, gamma),
 * b by Faraday b^{n+1} = b^n - dt C (gamma e^{n+1} + (1 - gamma) e^n).
 * FEPIC_FIELD_NM_MFEM: the mixed system (b on faces, e on edges: d_t b + C e = 0,
 * M d_t e - C^T Mf b = -j, Mf the Whitney-2 mass [*mu0^-1]) with the three-level Newmark
 * recurrence at beta = 1/4, gamma = 1/2 and the e-row source -1/2 (G^{n+1} - G^{n-1});
 * b^{n+1} eliminated, e^{n+1} solves (M + dt^2/4 S) e^{n+1} = M e^{n-1}
 * + dt C^T Mf (b^n + b^{n-1}) - dt^2 S (e^n / 2 + e^{n-1} / 4) - (G^{n+1} - G^{n-1}), then
 * b^{n+1} = b^{n-1} - dt C (e^n + (e^{n+1} + e^{n-1}) / 2).
 * FEPIC_FIELD_BD_MFEM: the same system with backward differences (backward Euler):
 * (M + dt^2 S) e^{n+1} = M e^n + dt C^T Mf b^n - (G^{n+1} - G^n), b^{n+1} = b^n - dt C e^{n+1}.
 * The mixed updates ignore the step's beta and gamma.  The Gauss-drift check follows each
 * update's recurrence: r^{n+1} - 2 r^n + r^{n-1}, r^{n+1} - r^{n-1} or r^{n+1} - r^n equals
 * D^T r_cg. */
enum { FEPIC_FIELD_WAVE = 0, FEPIC_FIELD_NM_MFEM = 1, FEPIC_FIELD_BD_MFEM = 2 };

typedef struct fepic_ctx fepic_ctx;

typedef struct {
    int device;        /* HIP device ordinal; -1 = host-only context: mesh topology and
                          matrix assembly only (no device calls), for inspection/tests   */
    int precision;     /* FEPIC_FP32_PUSH_FP64_ACC: gather/push/path split in FP32 with
                          per-tet barycentric positions, current and charge in FP64;
                          FEPIC_ALL_FP64: everything FP64                               */
    double cg_tol;     /* stop when ||b - A x||_2 <= cg_tol ||b||_2 (default 1e-10)      */
    int cg_max_iters;  /* default 10000                                                  */
    int cg_check_every;/* iterations between convergence reads on the host (default 8)   */
    int sort_period;   /* re-bin particles by tet every this many steps (default 1; 0:
                          never); FEPIC_SORT_AUTO: each species when its particles that
                          left their tet or the mesh since its last re-binning reach 1/64
                          of it, or particles were added to it (a run resumed from a
                          checkpoint starts its count afresh, so it agrees with the
                          uninterrupted run to rounding order, not bit for bit)         */
    int crossing_cap;  /* faces one path may cross in one step (default 64)              */
    int warm_start;    /* FEPIC_WS_* (default FEPIC_WS_PREV)                             */
    int diagnostics;   /* 1: charge continuity, Gauss and div b residuals every step      */
    int timing;        /* 1: per-phase HIP-event times in fepic_step_stats                */
    int preconditioner;/* FEPIC_PC_* (default FEPIC_PC_AUX)                               */
    int aux_far_levels;/* FEPIC_PC_AUX aggregate levels beyond 64 nodes (512, 4096, 32768
                          nodes): -1 (default) from dt: with tau^2 = mean beta dt^2
                          S_jj / M_jj, the level of 2^k nodes when tau >= 2 * 2^(k/3)
                          and there are at least 16 such aggregates; or 0 to 3           */
    int walk;          /* FEPIC_WALK_* (default FEPIC_WALK_AUTO)                          */
    int solve_precision;   /* FEPIC_SOLVE_* (default FEPIC_SOLVE_FP64)                    */
    double mixed_inner_tol;/* FEPIC_SOLVE_MIXED: residual reduction of one FP32 pass, in
                              (0, 1) (default 1e-4)                                       */
    int pusher;            /* FEPIC_PUSHER_* (default FEPIC_PUSHER_BORIS)                 */
    int ab_order;          /* FEPIC_PUSHER_AB: order 1..5 (default 4)                     */
    int field_solver;      /* FEPIC_FIELD_* (default FEPIC_FIELD_WAVE)                    */
    int deterministic;     /* 1: bitwise reproducible steps.  Current and charge are summed
                              as 128-bit fixed-point integers (order-independent; each term
                              truncated to 2^-64 of the power of two above the largest
                              |q w|), the particle step always walks in place, and the PCG
                              dots use one workgroup per partial slot.  Needs
                              FEPIC_PC_JACOBI, FEPIC_SOLVE_FP64 and a warm start other than
                              the learned ones (FEPIC_E_ARG at create; the setters refuse to
                              leave them with FEPIC_E_STATE).  The state after a step
                              (fields, charge, current, each particle by id) and the
                              integer step stats repeat bit for bit; the floating-point
                              conservation and energy diagnostics are still summed in any
                              order.  Default 0.                                           */
} fepic_options;

typedef struct {
    int64_t step;                 /* steps committed so far                               */
    double t;                     /* simulated time after the step                        */
    int cg_iters;                 /* PCG iterations of this step's Newmark solve          */
    double cg_rel_resid;          /* true ||b - A e^{n+1}||_2 / ||b||_2 at exit           */
    double cg_rel_resid0;         /* ||b - A x0||_2 / ||b||_2 (quality of the warm start) */
    double cont_resid_rel;        /* max |rho^{n+1} - rho^n - D^T dG| / scale, interior   */
    double gauss_resid_rel;       /* max |-D^T M e - rho| / scale, interior nodes         */
    double gauss_drift_check_rel; /* max |Delta^2 r_Gauss - D^T r_cg| / scale (Sec. III-A */
                                  /* solver-tolerance caveat); -1 until 3 levels exist    */
    double divb_max;              /* max over tets of |sum of signed face fluxes|         */
    double field_energy;          /* 1/2 e^T M e (electric part), joules                  */
    int64_t n_particles;          /* live particles after the step (all species)          */
    int64_t n_absorbed;           /* absorbed at the wall this step                       */
    int64_t n_crossings;          /* face crossings this step                             */
    int max_crossings;            /* most crossings of one path this step                 */
    int n_cap_exceeded;           /* paths stopped by the crossing cap                    */
    float ms_sort, ms_stage, ms_particles, ms_rhs, ms_warm, ms_cg, ms_faraday, ms_diag;
    double magnetic_energy;       /* 1/(2 mu0) int |B|^2 = 1/2 b^T [*mu0^-1] b, joules    */
    double kinetic_energy;        /* sum over live particles of w m c^2 (gamma - 1), J    */
    int pc_far_levels;            /* aggregate levels beyond 64 nodes the solve used (-1:  */
                                  /* Jacobi preconditioner or no solve)                   */
    int cg_passes;                /* FP64 residual passes of a FEPIC_SOLVE_MIXED solve     */
                                  /* (cg_iters counts the FP32 iterations of all of them); */
                                  /* 0 for an FP64 solve                                  */
    int64_t n_injected;           /* particles the injectors added in this step            */
} fepic_step_stats;

/* ---------------------------------------------------------------- lifecycle */
int fepic_abi_version(void);
void fepic_default_options(fepic_options* opts);
const char* fepic_error_string(int code);
const char* fepic_last_error(const fepic_ctx* ctx);
/* Creates a context on opts->device (NULL opts = defaults).  *out receives it. */
int fepic_create(const fepic_options* opts, fepic_ctx** out);
int fepic_destroy(fepic_ctx* ctx);
/* Device memory of the context from the caller's allocator instead of hipMalloc/hipFree
 * (e.g. a framework's caching allocator): alloc(bytes, user) returns device memory of the
 * context's device or NULL (then the calling entry point fails with FEPIC_E_OOM);
 * free_(ptr, user) takes back a pointer alloc returned, after the context's stream has
 * drained.  Both NULL restores hipMalloc.  Only before fepic_upload_mesh
 * (FEPIC_E_STATE after).  The functions and user must outlive the context. */
int fepic_set_allocator(fepic_ctx* ctx, void* (*alloc)(size_t bytes, void* user), void (*free_)(void* ptr, void* user),
                        void* user);
/* Selects the preconditioner of later Newmark solves (FEPIC_PC_*; FEPIC_E_ARG for any
 * other value, and for FEPIC_PC_JACOBI while the solve is FEPIC_SOLVE_MIXED;
 * FEPIC_E_STATE for FEPIC_PC_AUX with absorbing faces or in the deterministic mode).
 * Results agree to the solver tolerance either way. */
int fepic_set_preconditioner(fepic_ctx* ctx, int pc);
/* Selects the arithmetic of later Newmark solves (FEPIC_SOLVE_*; FEPIC_E_ARG for any other
 * value, and for FEPIC_SOLVE_MIXED with the Jacobi preconditioner). */
int fepic_set_solve_precision(fepic_ctx* ctx, int solve_precision);
/* Selects the field update of later steps (FEPIC_FIELD_*; FEPIC_E_ARG otherwise). */
int fepic_set_field_solver(fepic_ctx* ctx, int solver);
/* Selects the pusher (FEPIC_PUSHER_*) and Adams-Bashforth order (1..5) of later steps;
 * FEPIC_E_ARG for other values and for FEPIC_PUSHER_AB without FEPIC_ALL_FP64.  A switch of
 * pusher restarts the Adams-Bashforth histories. */
int fepic_set_pusher(fepic_ctx* ctx, int pusher, int ab_order);
/* Runs all later device work of this context on the given hipStream_t (NULL = the
 * context's own stream).  The caller keeps the stream alive while the context uses it. */
int fepic_set_stream(fepic_ctx* ctx, void* hip_stream);

/* ---------------------------------------------------------------- mesh (Sec. II-A)
 * xyz: [n_nodes][3] float64 node coordinates.  tets: [n_tets][4] int32 0-based node ids,
 * any vertex order.  Builds the canonical edges/faces, incidence, neighbours, per-tet
 * barycentric gradients, the edge mass matrix M = [*eps0] and the curl-curl matrix
 * S = [curl]^T [*mu0^-1] [curl] (Sec. II-A) over interior edges, and uploads them.
 * Errors: FEPIC_E_MESH for a degenerate tet, an out-of-range id or a face shared by
 * more than two tets.  May be called once per context. */
int fepic_upload_mesh(fepic_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets);
/* Entity counts after upload; any output pointer may be NULL.  euler = V - E + F - T. */
int fepic_get_topology_sizes(fepic_ctx* ctx, int64_t* n_edges, int64_t* n_faces, int64_t* n_int_edges,
                             int64_t* n_int_nodes, int64_t* euler);
/* Canonical topology; any output may be NULL.  tets_sorted [n_tets][4], edges
 * [n_edges][2], faces [n_faces][3], tet_edges [n_tets][6] (local edge order (0,1),(0,2),
 * (0,3),(1,2),(1,3),(2,3)), tet_faces [n_tets][4], nbr [n_tets][4] (tet across local
 * face k, -1 on the wall). */
int fepic_get_topology(fepic_ctx* ctx, int32_t* tets_sorted, int32_t* edges, int32_t* faces, int32_t* tet_edges,
                       int32_t* tet_faces, int32_t* nbr);
/* Assembled matrix which = 0 (M), 1 (S) or 2 (K, the boundary matrix of the absorbing
 * faces; FEPIC_E_STATE before fepic_set_absorbing_faces) restricted to the unknown edges
 * (all but those on a PEC wall face), as COO over global edge ids.  With row == NULL only
 * *nnz is returned.  cap = capacity of the arrays. */
int fepic_get_matrix(fepic_ctx* ctx, int which, int64_t cap, int64_t* nnz, int64_t* row, int64_t* col, double* val);

/* First-order absorbing boundary (Sec. II-A, eq. (impedanceBC) with Psi_I = 0 and Y the
 * admittance of free space 1 / (mu0 c); the surface impedance matrix of Sec. II-A):
 * marks wall faces as absorbing instead of PEC.  faces: n canonical face ids (as
 * fepic_get_topology numbers them), each a wall face; NULL = every wall face (n ignored).
 * The tangential field on absorbing faces becomes unknown: edges on them join the solve,
 * and the wave-equation update gains the damping matrix C = Y K, K_ij = the integral over
 * the absorbing faces of (n x W_i) . (n x W_j), in the Newmark recurrence
 *   (M + gamma dt C + beta dt^2 S) e^{n+1} = (2M - (1 - 2 gamma) dt C - (1/2 - 2 beta
 *   + gamma) dt^2 S) e^n - (M - (1 - gamma) dt C + (1/2 + beta - gamma) dt^2 S) e^{n-1}
 *   - (G^{n+1} - 2 G^n + G^{n-1}).
 * Particles still leave the domain through any wall face.  Only before the first step and
 * once per context; only with FEPIC_FIELD_WAVE, FEPIC_PC_JACOBI and FEPIC_SOLVE_FP64
 * (FEPIC_E_STATE otherwise; later requests for another field update or preconditioner are
 * refused the same way); FEPIC_E_ARG for an id that is not a wall face.  Fields set
 * before the call keep their values.  Works on a host-only context too (assembly only).
 * Checkpoints do not record the absorbing faces: restore into a context set up alike. */
int fepic_set_absorbing_faces(fepic_ctx* ctx, int64_t n, const int32_t* faces);

/* ---------------------------------------------------------------- fields
 * e, e_prev: [n_edges] edge unknowns at t_n and t_{n-1} (entries of edges on PEC wall
 * faces ignored, held at 0); b: [n_faces] face fluxes at t_n.  Any may be NULL (left unchanged). */
int fepic_set_fields(fepic_ctx* ctx, const double* e, const double* e_prev, const double* b);
/* b_f = B0 . (area vector of f): the exact Whitney-2 interpolant of a uniform field. */
int fepic_set_uniform_B(fepic_ctx* ctx, const double B0[3]);
/* Electrostatic start (Gauss at t_0 and t_{-1}): solves -D^T M (-D phi) = rho^0 on
 * interior nodes by CG to tol, sets e^0 = e^{-1} = -D phi.  *iters may be NULL. */
int fepic_init_electrostatic(fepic_ctx* ctx, double tol, int* iters);

/* ---------------------------------------------------------------- particles
 * A species has charge q (C), mass m (kg) and macro-particle weight w (physical particles
 * per macro-particle, Sec. II-A point shapes). */
int fepic_add_species(fepic_ctx* ctx, double q, double m, double w, int* species_out);
/* Seeded disk source of a species (a beam entering through a wall, Sec. IV-B): every later
 * step (fepic_step, fepic_push_particles) first adds per_step particles drawn on the
 * device, uniformly on the disk of the given radius around center in the plane normal to
 * normal (a wall of the mesh, for the particles to start inside it), with velocity
 * v = v0 n + sigma (N1, N2, N3): drift v0 from kinetic_eV (relativistic), N standard
 * normals per Cartesian component, sigma = sqrt(thermal_eV e / m); u is stored as gamma v
 * (Boris) or v (Adams-Bashforth).  Draws come from the counter-based generator
 * Philox4x32-10 (Salmon et al., SC 2011): particle j of the k-th injection of species s
 * uses the blocks of counter (j, k mod 2^32, k div 2^32, 4 s + b), b = 0..2, under the key
 * (seed mod 2^32, seed div 2^32); the twelve words give six uniforms
 * ((w_2i >> 5) 2^26 + (w_2i+1 >> 6) + 1/2) 2^-53: radius R sqrt(u0), angle 2 pi u1,
 * Box-Muller normals from (u2, u3) and (u4, u5); the plane's basis is e1 = unit(n x a),
 * e2 = n x e1, a = the x axis unless |n_x| >= 0.9, then the y axis.  The particles are
 * located after the step's sort and pushed with the others a full step; ids continue the
 * species' default ids.  A step that fails commits none of them and does not count the
 * injection (k advances only with committed steps).  spec == NULL switches the source off;
 * setting one restarts k at 0.  FEPIC_E_ARG for a bad species or non-finite, negative or
 * degenerate parameters. */
typedef struct {
    double center[3], normal[3], radius;   /* m                                       */
    double kinetic_eV, thermal_eV;         /* drift energy along normal, temperature  */
    int64_t per_step;                      /* particles per step (< 2^30)             */
    uint64_t seed;
} fepic_injector;
int fepic_set_injector(fepic_ctx* ctx, int species, const fepic_injector* spec);
/* Appends n particles: id [n] (caller-chosen, kept through sorting; NULL = running
 * index), x [n][3] Cartesian positions at t_n, u [n][3] = gamma v at t_{n-1/2} (m/s).
 * Each is located in its tet on the device; points outside the mesh or with non-finite
 * values are dropped and counted in *n_rejected (may be NULL). */
int fepic_upload_particles(fepic_ctx* ctx, int species, int64_t n, const int64_t* id, const double* x,
                           const double* u, int64_t* n_rejected);
/* The same with x, u ([n][3] FP64) and id ([n] int64, or NULL) in device memory of the
 * context's device (e.g. torch tensors), read on the context's stream; synchronous like
 * fepic_upload_particles (the arrays may be freed when it returns). */
int fepic_upload_particles_device(fepic_ctx* ctx, int species, int64_t n, const int64_t* id, const double* x,
                                  const double* u, int64_t* n_rejected);
/* Injection during a run (e.g. a beam source): appends n particles like
 * fepic_upload_particles but without re-sorting or waiting for the device; the next
 * step's sort orders them, and points outside the mesh are dropped there (not counted).
 * The counts of live particles are exact again after the next fepic_step. */
int fepic_inject_particles(fepic_ctx* ctx, int species, int64_t n, const int64_t* id, const double* x,
                           const double* u);
/* The same with x, u ([n][3] FP64) and id ([n] int64, or NULL for default ids) in device
 * memory of the context's device (e.g. torch tensors): read by kernels enqueued on the
 * context's stream, with no host copy; the caller keeps them valid and unchanged until the
 * stream has passed this call (e.g. until the next fepic_step returns). */
int fepic_inject_particles_device(fepic_ctx* ctx, int species, int64_t n, const int64_t* id, const double* x,
                                  const double* u);
int fepic_num_particles(fepic_ctx* ctx, int species, int64_t* n);
/* Copies live particles out (order = current device order): id, x [n][3] (Cartesian,
 * reconstructed as sum lambda_k r_k), u [n][3], tet [n], lambda [n][4] (local vertex
 * order of the sorted tet).  Any output may be NULL.  *n = count written (<= cap). */
int fepic_get_particles(fepic_ctx* ctx, int species, int64_t cap, int64_t* n, int64_t* id, double* x, double* u,
                        int32_t* tet, double* lambda);

/* ---------------------------------------------------------------- the step
 * One PIC step (Sec. II-A cycle): stage fields per tet, gather + relativistic Boris +
 * path tracking + Whitney-1 deposit of dG^{n+1} = G^{n+1} - G^n for every particle,
 * Newmark right-hand side
 *   b = (2M - (1/2 - 2beta + gamma) dt^2 S) e^n - (M + (1/2 + beta - gamma) dt^2 S) e^{n-1}
 *       - (dG^{n+1} - dG^n),
 * PCG solve (M + beta dt^2 S) e^{n+1} = b from the configured warm start, Faraday
 * b^{n+1} = b^n - dt C (gamma e^{n+1} + (1 - gamma) e^n).  Atomic: on
 * FEPIC_E_CG_NOT_CONVERGED or FEPIC_E_CROSSING_CAP nothing is committed.  out may be
 * NULL. */
int fepic_step(fepic_ctx* ctx, double dt, double beta, double gamma, fepic_step_stats* out);
/* Particle half only (fields frozen): stage, gather, push (the configured pusher), track,
 * deposit; commits the particles and dG^{n+1} (the field history is left as is).  Atomic
 * like fepic_step: on FEPIC_E_CROSSING_CAP nothing is committed.  out may be NULL. */
int fepic_push_particles(fepic_ctx* ctx, double dt, fepic_step_stats* out);

/* ---------------------------------------------------------------- read-out
 * Host copies; sizes from fepic_get_topology_sizes.  Any output may be NULL. */
int fepic_get_fields(fepic_ctx* ctx, double* e, double* e_prev, double* b);
/* dG: [n_edges] current deposited by the last step (G^n - G^{n-1}); G: [n_edges]
 * time-integrated current G^n = sum of all deposits (eq. (G)). */
int fepic_get_current(fepic_ctx* ctx, double* dG, double* G);
/* rho: [n_nodes] nodal charge sum_p q w lambda_k(x_p) of the live particles. */
int fepic_get_rho(fepic_ctx* ctx, double* rho);
/* on != 0: each later Newmark solve keeps a copy of its start vector x0 (after the warm
 * start: e^n, an extrapolation, or the learned prediction with its line step), for
 * inspection; fepic_get_warm_start copies the last one out ([n_edges], canonical order;
 * FEPIC_E_STATE before any). */
int fepic_keep_warm_start(fepic_ctx* ctx, int on);
int fepic_get_warm_start(fepic_ctx* ctx, double* x0);
/* Recomputes the residuals of fepic_step_stats for the current state on demand. */
int fepic_diagnostics(fepic_ctx* ctx, fepic_step_stats* out);

/* ---------------------------------------------------------------- profiling
 * Brackets the launches of the named kernel family ("push", "stage", "sort", "rhs",
 * "cg_iter", "faraday", "mlp_fwd") with HIP events on the context's stream while
 * enabled: one pair per launch, except "cg_iter", whose pair spans each batch of
 * back-to-back iteration launches (so its per-launch average includes the dispatch gap
 * between iterations, and events do not separate them) and whose launch count is the
 * number of PCG iterations launched (one kernel each with Jacobi, three with the
 * auxiliary-space preconditioner).  fepic_kernel_time returns the summed duration and
 * the launch count since enabling (synchronizes the stream). */
int fepic_kernel_timing(fepic_ctx* ctx, const char* family, int enable);
int fepic_kernel_time(fepic_ctx* ctx, const char* family, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------- learned warm start
 * Per-edge network 4 -> 64 -> 64 -> 1 (ReLU), BF16 matrix-core arithmetic with FP32
 * accumulation.  Inputs per interior edge: e^n / s_e, (e^n - e^{n-1}) / s_d,
 * (e^{n-1} - e^{n-2}) / s_d (differences formed in FP64) and dG^{n+1} / s_g, with s_e,
 * s_d, s_g the RMS over interior edges (1 if zero); the output predicts the increment in
 * units of s_d (see FEPIC_WS_MLP and FEPIC_WS_MLP_DIRECT).
 * Flat FP32 weight layout: W1[64][4], b1[64], W2[64][64], b2[64], W3[1][64], b3[1]
 * (4545 values).  The PCG always runs to cg_tol from whatever start, so the network only
 * changes the iteration count, never the accuracy; a non-finite prediction or one whose
 * residual exceeds ||b|| falls back to e^n. */
#define FEPIC_MLP_N_PARAMS 4545
typedef struct {
    int epochs;          /* passes over the recorded samples                       */
    int64_t batch;       /* rows per minibatch (multiple of 64)                    */
    double lr, beta1, beta2, eps;  /* Adam                                         */
    uint64_t seed;       /* initialization and minibatch order                    */
    double val_fraction; /* share of recorded snapshots held out for validation   */
} fepic_train_opts;
typedef struct {
    double train_loss, val_loss;   /* final mean squared error (normalized units)  */
    int64_t n_train_rows, n_val_rows, n_steps;
    float ms_total;
} fepic_train_stats;
/* on = k >= 1: each later fepic_step appends (features, target (e^{n+1} - e^n) / s_d) of
 * one interior edge in k
 * (rows r0, r0 + k, ... with r0 = snapshot count mod k, so successive snapshots sample
 * different edges; k = 1 records every interior edge) to a device buffer holding up to
 * max_snapshots steps (oldest dropped first); a new k or max_snapshots starts the buffer
 * afresh.  A step whose increment's RMS exceeds 10 s_d (the history near zero, as after a
 * neutral start) is not recorded.  on = 0 stops recording.  FEPIC_E_ARG for k above the interior
 * edge count. */
int fepic_ws_record(fepic_ctx* ctx, int on, int64_t max_snapshots);
int fepic_ws_num_snapshots(fepic_ctx* ctx, int64_t* n);
int fepic_ws_train(fepic_ctx* ctx, const fepic_train_opts* opts, fepic_train_stats* out);
int fepic_ws_get_weights(fepic_ctx* ctx, float* w, int64_t cap, int64_t* n);
int fepic_ws_set_weights(fepic_ctx* ctx, const float* w, int64_t n);
int fepic_set_warm_start(fepic_ctx* ctx, int mode);
/* Test entries on host batches: X [n][4] FP32 -> y [n]; gradient of the mean squared
 * error against t [n] -> grad [4545] and *loss, computed by the device kernels. */
int fepic_mlp_forward(fepic_ctx* ctx, int64_t n, const float* X, float* y);
int fepic_mlp_grad(fepic_ctx* ctx, int64_t n, const float* X, const float* t, float* grad, double* loss);

/* One Adam update (Kingma and Ba) of the network's FP32 master weights with the given
 * gradient grad [4545] (host), by the device kernel training uses; the moment estimates
 * and step counter are the context's (they restart with fepic_ws_set_weights).  A test
 * entry: training feeds the kernel minibatch gradients itself. */
int fepic_mlp_adam_step(fepic_ctx* ctx, const float* grad, double lr, double beta1, double beta2, double eps);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * training or serving loops, harnesses that forbid hipMalloc): fepic_mlp_grad on device
 * arrays, allocating nothing.  X [n][4] FP32 and t [n] FP32 are read, grad [4545] FP32 and
 * loss [1] FP64 (the mean squared error) written, all in device memory of the context's
 * device; the kernels are enqueued on the context's stream and the call returns without
 * waiting (the caller synchronizes before reading the outputs).  The result is that of
 * fepic_mlp_grad on the same rows, summed in the same order.  The per-workgroup partial
 * sums live in one fixed device array of the library per GPU (2.3 MB, held until the
 * process ends), set up by fepic_create: calls that overlap on one GPU, from any context
 * or stream, race on it.  Errors: FEPIC_E_ARG for n <= 0, a NULL pointer or n above
 * FEPIC_MLP_NOALLOC_MAX_ROWS; FEPIC_E_STATE when the context has no network weights yet
 * (fepic_ws_set_weights or fepic_ws_train first; this call does not create them);
 * FEPIC_E_NO_DEVICE on a host-only context. */
#define FEPIC_MLP_NOALLOC_MAX_ROWS 65536
int fepic_mlp_grad_noalloc(fepic_ctx* ctx, int64_t n, const float* X, const float* t, float* grad, double* loss);

/* ---------------------------------------------------------------- checkpoint
 * Versioned binary file: fields and their history, current history, particles of every
 * species, step counter and time, warm-start weights.  Load requires a context with the
 * same mesh uploaded and the same species added. */
int fepic_save(fepic_ctx* ctx, const char* path);
int fepic_load(fepic_ctx* ctx, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* FEPIC_H */
