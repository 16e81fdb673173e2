// Score network (learned column selection): placeholder until the kernels land.
#include "common.hpp"

namespace ffk {

ffk_mlp* mlp_create(int32_t D, int32_t H, uint64_t) {
  (void)D; (void)H;
  fail(FFK_ERR_ARG, "mlp: not available in this build");
}
void mlp_forward(const ffk_mlp*, const float*, int64_t, float*, int, hipStream_t) { fail(FFK_ERR_ARG, "mlp: not available"); }
void mlp_grad(ffk_mlp*, const float*, const float*, int64_t, float*, float*, hipStream_t) { fail(FFK_ERR_ARG, "mlp: not available"); }
void mlp_adam(ffk_mlp*, const float*, float, hipStream_t) { fail(FFK_ERR_ARG, "mlp: not available"); }
void mlp_scores(const ffk_mlp*, const ffk_system*, double*, hipStream_t) { fail(FFK_ERR_ARG, "mlp: not available"); }

}  // namespace ffk
