// Vector-Jacobian product of the residual with frozen switches.
#include "hfv_internal.hpp"

namespace hfv {

hfv_status run_vjp(hfv_ctx *ctx, const void *, const uint8_t *, const void *, void *, hipStream_t) {
  ctx->err = "residual VJP is not available in this build";
  return HFV_ERR_STATE;
}

}  // namespace hfv
