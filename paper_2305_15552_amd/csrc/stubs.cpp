// Entry points whose implementation is not built yet: they fail cleanly.
#include "internal.h"

extern "C" {
hyeig_status hyeig_mlp_create(hyeig_ctx* ctx, const float*, hyeig_mlp** out) {
  if (out) *out = nullptr;
  return set_err(ctx, HYEIG_EUNSUPPORTED, "mlp: not built");
}
hyeig_status hyeig_mlp_get(hyeig_ctx* ctx, const hyeig_mlp*, float*) { return set_err(ctx, HYEIG_EUNSUPPORTED, "mlp: not built"); }
void hyeig_mlp_destroy(hyeig_mlp*) {}
hyeig_status hyeig_mlp_forward(hyeig_ctx* ctx, const hyeig_mlp*, int64_t, const float*, float*) {
  return set_err(ctx, HYEIG_EUNSUPPORTED, "mlp: not built");
}
hyeig_status hyeig_mlp_backward(hyeig_ctx* ctx, const hyeig_mlp*, int64_t, const float*, const float*, float*, double*) {
  return set_err(ctx, HYEIG_EUNSUPPORTED, "mlp: not built");
}
hyeig_status hyeig_mlp_train(hyeig_ctx* ctx, hyeig_mlp*, int64_t, const float*, const float*, const hyeig_train_params*,
                             double*) {
  return set_err(ctx, HYEIG_EUNSUPPORTED, "mlp: not built");
}
}
