// INLA entry points (placeholder until the model path is in place).
#include "../../include/adelia.h"
extern "C" {
int inla_model_create(adelia_ctx, const inla_model_desc*, inla_model*) { return ADELIA_E_UNSUPPORTED; }
int inla_model_destroy(inla_model) { return 0; }
int inla_model_dim(inla_model) { return 0; }
size_t inla_workspace_bytes(inla_model, int, int) { return 0; }
int inla_objective(inla_model, const double*, int32_t, double*, int32_t*, void*, size_t, int, void*) { return ADELIA_E_UNSUPPORTED; }
int inla_grad(inla_model, const double*, double*, double*, int32_t*, void*, size_t, int, void*) { return ADELIA_E_UNSUPPORTED; }
int inla_fd_grad(inla_model, const double*, double, int32_t, double*, double*, int32_t*, void*, size_t, void*) { return ADELIA_E_UNSUPPORTED; }
}
