// The libfepic context: host mesh, device state and bookkeeping shared by the API files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>
#include <vector>

#include "fepic_internal.h"
#include "host_mesh.h"
#include <climits>

namespace fepic {

enum { FAM_PUSH, FAM_STAGE, FAM_SORT, FAM_RHS, FAM_CG_ITER, FAM_FARADAY, FAM_MLP_FWD, FAM_COUNT };
extern const char* kFamilies[];

struct KernelTimer {
    bool on = false;
    int64_t used = 0;       // events recorded (pairs * 2)
    int64_t launches = 0;   // kernel launches the pairs span
    std::vector<hipEvent_t> ev;
};

struct Species {
    double q = 0, m = 1, w = 1;
    int64_t n = 0;        // slots in use in buffer cur (dead entries have tet -1)
    int64_t cap = 0;
    int cur = 0;
    int64_t next_id = 0;  // default ids
    void* buf[2][8] = {}; // tet, l1, l2, l3, u0, u1, u2, id
    // The particle step keeps each particle's slot, so ids are not copied by it: the id
    // arrays have their own current index, flipped only by the sort.
    int idcur = 0;
    int32_t* d_nlive = nullptr;
    int32_t* h_nlive = nullptr;
    // face crossings of the step so far, counted after this species' particle kernels (its
    // own crossings are the difference to the previous species'), and the species' own
    // crossings per particle at its last committed step
    unsigned long long* d_xcum = nullptr;   // [2]: crossings, and absorptions + paths cut at the cap
    unsigned long long* h_xcum = nullptr;
    int64_t n_pushed = 0;
    double own_share = 1.0;
    // FEPIC_SORT_AUTO: particles that left their tet or the mesh since the species' last
    // re-binning (face crossings counted), and whether particles were added since
    int64_t moved = 0;
    bool added = false;
    // Adams-Bashforth pusher: history [kAbStride][abh_cap] (component-major) and per-slot
    // AbMeta, each double-buffered.  The sorts move both (flipping abh_cur and abm_cur); a
    // step writes its meta to the other buffer, flipped at the commit with cur.
    double* d_abh[2] = {};
    int32_t* d_abm[2] = {};
    int abh_cur = 0, abm_cur = 0;
    int64_t abh_cap = 0;
    double ab_dt = 0.0;                // dt of the levels held
    bool ab_reset = true;              // every slot restarts at order 1 at the next AB step
    int64_t ab_fill_from = INT64_MAX;  // slots appended since: no history yet
    bool sorted_pending = false;  // d_nlive holds a count not yet read back
    // seeded disk source (fepic_set_injector): inj_k counts committed injections; a step
    // that is not committed drops the particles it appended (inj_undo_n = count before)
    bool inj_on = false;
    InjectorSpec inj{};
    int64_t inj_k = 0;
    int64_t inj_undo_n = -1;
};

struct MlpState;

}  // namespace fepic

struct fepic_ctx {
    fepic_options opt{};
    std::string err;
    bool host_only = false;
    hipStream_t stream = nullptr, own_stream = nullptr;
    std::vector<void*> allocs;
    // caller's device allocator (fepic_set_allocator), or hipMalloc/hipFree when null
    void* (*ualloc)(size_t, void*) = nullptr;
    void (*ufree)(void*, void*) = nullptr;
    void* uarg = nullptr;

    fepic::HostMesh mesh;
    bool have_mesh = false;

    // device mesh
    int32_t *d_tets = nullptr, *d_edges = nullptr, *d_tet_edges = nullptr, *d_tet_faces = nullptr,
            *d_face_edges = nullptr, *d_int_edges = nullptr;
    uint8_t *d_bedge = nullptr, *d_inode = nullptr;
    double *d_grad64 = nullptr, *d_r0 = nullptr;
    void* d_blk = nullptr;
    int64_t* d_sp = nullptr;
    int32_t* d_col = nullptr;
    double *d_M = nullptr, *d_S = nullptr, *d_A = nullptr, *d_dinv = nullptr;
    int32_t *d_cell_start = nullptr, *d_cell_tets = nullptr, *d_grid_n = nullptr;
    double* d_grid = nullptr;  // lo[3], inv_h[3]
    double* d_live = nullptr;   // one double: live-particle count of fepic_num_particles
    double A_scale = -1.0, A_scale_K = 0.0;
    // deterministic mode: fixed-point accumulators, two words per edge or node (kept
    // cleared between uses), allocated on first use
    unsigned long long* d_fix = nullptr;
    // first-order absorbing faces: their boundary matrix K in the pattern of M and S
    double* d_K = nullptr;
    bool abc_on = false;
    double s_over_m = 0.0;   // mean of S_jj / M_jj over interior rows (chooses the far levels)
    bool A_valid = false;

    // fields (edge vectors length n_edges, face vectors length n_faces)
    double *d_e = nullptr, *d_ep = nullptr, *d_ep2 = nullptr, *d_x = nullptr;
    double *d_dg = nullptr, *d_dgn = nullptr, *d_G = nullptr;
    double *d_b = nullptr, *d_bn = nullptr;
    double* d_bp = nullptr;   // b^{n-1} (the three-level mixed update needs it)
    // mixed (b, e) updates: Whitney-2 mass over faces and each edge's incident faces, both
    // SELL-64 (built on first use), and a face work vector
    bool mfem_ready = false;
    int64_t *d_mf_sp = nullptr, *d_ef_sp = nullptr;
    int32_t *d_mf_col = nullptr, *d_ef_inc = nullptr;
    double *d_mf_val = nullptr, *d_h = nullptr;
    double *d_rhs = nullptr, *d_rt = nullptr, *d_Me = nullptr;
    fepic::CgVec* d_cgv[2] = {nullptr, nullptr};   // Jacobi-PCG state, double buffered
    // auxiliary-space PCG: (z, p) pairs double buffered, r and q (n_edges each), nodal arrays
    double2* d_zp[2] = {nullptr, nullptr};
    double2* d_rq = nullptr;
    // FP32 inner solves of the mixed-precision form (allocated on first use): A and D^-1,
    // the correction d, r and q, (z, p) pairs; valid for the operator of A_scale
    float *d_A32 = nullptr, *d_dinv32 = nullptr, *d_x32 = nullptr, *d_rq32 = nullptr;
    float2* d_zp32[2] = {nullptr, nullptr};
    bool A32_valid = false;
    int last_pass_iters[8] = {};   // iterations of each pass of the last mixed solve
    int cg_passes = 0;             // passes of the last mixed solve
    fepic::AuxSpace aux;
    double* d_partial = nullptr;
    fepic::CgScalars* d_sc = nullptr;
    fepic::CgScalars* h_sc = nullptr;
    fepic::PushCounters* d_cnt = nullptr;
    fepic::PushCounters* d_cnt_slots = nullptr;   // [kCntSlots], zero between steps
    unsigned char* d_cq = nullptr;                 // crossing queue storage (CrossQueue arrays)
    int64_t cq_cap = 0;                            // its capacity in slots (multiple of 256)
    double cross_share = 1.0;                      // face crossings per particle, last step
    int last_cg_iters = 0;                         // iterations of the last successful solve
    fepic::PushCounters* h_cnt = nullptr;
    int deferred_err = 0;
    // injection staging: pinned host buffer and its device mirror (x, u, id)
    void* h_stage = nullptr;
    void* d_stage = nullptr;
    int64_t stage_cap = 0;
    hipEvent_t stage_event{};
    bool stage_event_valid = false;

    // sort scratch
    int32_t *d_count = nullptr, *d_offset = nullptr, *d_bsums = nullptr;

    // diagnostics
    double *d_rho = nullptr, *d_rho_new = nullptr, *d_n1 = nullptr, *d_n2 = nullptr, *d_n3 = nullptr;
    double* d_rG[3] = {nullptr, nullptr, nullptr};
    int rG_head = 0, rG_levels = 0;
    bool rho_valid = false;
    fepic::DiagAcc* d_acc = nullptr;
    fepic::DiagAcc* h_acc = nullptr;
    unsigned int* d_dotc = nullptr;

    std::vector<fepic::Species> species;
    int64_t step_count = 0;
    double time = 0.0;

    fepic::KernelTimer timers[fepic::FAM_COUNT];
    hipEvent_t phase_ev[9] = {};

    // learned warm start
    fepic::MlpState* mlp = nullptr;
    bool mlp_ready = false;
    int cg_restarts = 0;
    bool recording = false;
    int64_t mlp_fallbacks = 0;
    // staging of the injectors' draws (x, u per particle)
    double* d_inj = nullptr;
    int64_t inj_cap = 0;
    // copy of the last Newmark solve's start vector (fepic_keep_warm_start)
    bool keep_start = false;
    double* d_x0keep = nullptr;
};

#define HIPCHK_RET(c, expr)                                          \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return fepic::hip_fail(c, e_, #expr); \
    } while (0)

namespace fepic {
int hip_fail(fepic_ctx* c, hipError_t e, const char* what);
int fail(fepic_ctx* c, int code, const std::string& msg);
void* dmalloc(fepic_ctx* c, size_t bytes);
void dfree(fepic_ctx* c, void* p);
hipEvent_t* timer_pair(fepic_ctx* c, int fam, int64_t n_launches = 1);

int init_electrostatic(fepic_ctx* c, double tol, int* iters);
int mlp_warm_start(fepic_ctx* c, bool direct);
int mlp_record_features(fepic_ctx* c);
int mlp_record_target(fepic_ctx* c);
void mlp_destroy(fepic_ctx* c);
void mlp_noalloc_setup(int device);
int mlp_save(fepic_ctx* c, std::FILE* f);
int mlp_load(fepic_ctx* c, std::FILE* f);
}  // namespace fepic
