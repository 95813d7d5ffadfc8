// Learned warm start: host side (placeholder until the MFMA kernels land).
#include "ctx.h"

namespace fepic {
int mlp_warm_start(fepic_ctx* c) { return fail(c, FEPIC_E_STATE, "learned warm start not built"); }
int mlp_record_features(fepic_ctx* c) { return fail(c, FEPIC_E_STATE, "recording not built"); }
int mlp_record_target(fepic_ctx* c) { return fail(c, FEPIC_E_STATE, "recording not built"); }
void mlp_destroy(fepic_ctx*) {}
}  // namespace fepic

extern "C" {
int fepic_ws_record(fepic_ctx* c, int, int64_t) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_ws_num_snapshots(fepic_ctx* c, int64_t* n) { if (n) *n = 0; return c ? FEPIC_OK : FEPIC_E_ARG; }
int fepic_ws_train(fepic_ctx* c, const fepic_train_opts*, fepic_train_stats*) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_ws_get_weights(fepic_ctx* c, float*, int64_t, int64_t*) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_ws_set_weights(fepic_ctx* c, const float*, int64_t) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_set_warm_start(fepic_ctx* c, int mode) {
    if (!c || mode < FEPIC_WS_PREV || mode > FEPIC_WS_MLP) return FEPIC_E_ARG;
    c->opt.warm_start = mode;
    return FEPIC_OK;
}
int fepic_mlp_forward(fepic_ctx* c, int64_t, const float*, float*) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_mlp_grad(fepic_ctx* c, int64_t, const float*, const float*, float*, double*) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_save(fepic_ctx* c, const char*) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
int fepic_load(fepic_ctx* c, const char*) { return c ? fepic::fail(c, FEPIC_E_STATE, "not built") : FEPIC_E_ARG; }
}
