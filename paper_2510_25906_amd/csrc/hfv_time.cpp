// One stage of an explicit Runge-Kutta method in Shu-Osher form
// (Section 2.4: the paper advances the semi-discrete system with the
// strong-stability-preserving Runge-Kutta methods of Spiteri and Ruuth, whose
// stages are convex combinations of earlier stages and forward-Euler steps):
//   out = a U0 + b U1 + c R,
// elementwise over the conserved variables of every cell, in the context's
// precision, evaluated as (a U0 + b U1) + c R.  A term whose pointer is NULL is
// left out.  Any of U0, U1, R may alias `out` (each element is read before it
// is written, by the same thread).
#include <algorithm>
#include <cmath>

#include "hfv_internal.hpp"

namespace hfv {

template <typename T>
__global__ __launch_bounds__(256) void k_rk_stage(long n, T a, const T *U0, T b, const T *U1, T c, const T *R,
                                                  T *out) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    T v = U0 ? a * U0[i] : (T)0;
    if (U1) v += b * U1[i];
    if (R) v += c * R[i];
    out[i] = v;
  }
}

template <typename T>
static hfv_status rk_t(hfv_ctx *ctx, double a, const void *U0, double b, const void *U1, double c, const void *R,
                       void *out, hipStream_t s) {
  const long n = (long)ctx->nvar * ctx->N;
  const long blocks = std::min<long>((n + 255) / 256, 16L * ctx->n_cu);
  k_rk_stage<T><<<(unsigned)std::max<long>(blocks, 1), 256, 0, s>>>(n, (T)a, (const T *)U0, (T)b, (const T *)U1,
                                                                     (T)c, (const T *)R, (T *)out);
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

}  // namespace hfv

using namespace hfv;

extern "C" hfv_status hfv_rk_stage(hfv_ctx *ctx, double a, const void *U0, double b, const void *U1, double c,
                                   const void *R, void *out, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!out) return ctx->err = "NULL output pointer", HFV_ERR_PARAM;
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c))
    return ctx->err = "non-finite stage coefficient", HFV_ERR_PARAM;
  hipStream_t s = (hipStream_t)stream;
  return ctx->prec == 64 ? rk_t<double>(ctx, a, U0, b, U1, c, R, out, s)
                         : rk_t<float>(ctx, a, U0, b, U1, c, R, out, s);
}
