// Time integration support.
//
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

// Spectral radius of every cell's upwind update, (|u| + c) sum_f |S_f| / |V|
// (|S_f| = sum of the face's Gauss weights x Jacobians), in double, max-reduced:
// per block into part[blockIdx.x], then one block over the parts.  A cell
// whose state is not physical (rho or p not positive, or not finite) has rate
// +inf.  Fixed reduction order: no atomics.
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_rate_blocks(int N, const T *U, const double *vol, const int *cf_off,
                                                     const int *cf, const int *gp_off, const T *gpw, double gamma,
                                                     double *part) {
  constexpr int NV = DIM + 2;
  __shared__ double sm[256];
  double m = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
    const double rho = (double)U[c];
    double q2 = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const double mj = (double)U[(long)(1 + j) * N + c];
      q2 += mj * mj;
    }
    const double E = (double)U[(long)(NV - 1) * N + c];
    const double p = (gamma - 1.0) * (E - 0.5 * q2 / rho);
    double area = 0.0;
    for (int e = cf_off[c]; e < cf_off[c + 1]; ++e) {
      const int f = cf[e] & 0x7fffffff;
      for (int g = gp_off[f]; g < gp_off[f + 1]; ++g) area += (double)gpw[g];
    }
    double r = INFINITY;
    if (rho > 0.0 && p > 0.0 && rho < INFINITY && p < INFINITY)
      r = (sqrt(q2) / rho + sqrt(gamma * p / rho)) * area / vol[c];
    m = fmax(m, r);
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_rate_final(int nb, const double *part, double *out) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

template <typename T>
static hfv_status rate_t(hfv_ctx *ctx, Tables<T> &t, const void *U, double *out, hipStream_t s) {
  const int nb = (int)std::min<long>(((long)ctx->N + 255) / 256, RED_BLOCKS);
  const double *vol = ctx->geom + (size_t)ctx->dim * ctx->N;
  if (ctx->dim == 2)
    k_rate_blocks<2, T><<<nb, 256, 0, s>>>(ctx->N, (const T *)U, vol, t.cf_off, t.cf, t.gp_off, t.gpw,
                                           ctx->p.gamma, ctx->red);
  else
    k_rate_blocks<3, T><<<nb, 256, 0, s>>>(ctx->N, (const T *)U, vol, t.cf_off, t.cf, t.gp_off, t.gpw,
                                           ctx->p.gamma, ctx->red);
  HFV_HIP(hipGetLastError());
  k_rate_final<<<1, 256, 0, s>>>(nb, ctx->red, out);
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

}  // namespace hfv

using namespace hfv;

extern "C" hfv_status hfv_cfl_rate(hfv_ctx *ctx, const void *U, double *out, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !out) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  hipStream_t s = (hipStream_t)stream;
  return ctx->prec == 64 ? rate_t<double>(ctx, ctx->t64, U, out, s) : rate_t<float>(ctx, ctx->t32, U, out, s);
}

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
