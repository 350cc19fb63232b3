// Viscous fluxes of the Navier-Stokes equations (Section 2, Eqs. Terms1,
// sutherlandlaw, HeatConduct, Stresses; Section 2.4, Eq. viscous_jump).
//
//   k_keep_fits   the central least-squares fit of every cell, [K][NV][N],
//                 for the modes without a linear pass (the linear pass keeps
//                 it itself when the context is viscous)
//   k_slot_grads  FP64: per Gauss-point slot of a cell (one lane each, a
//                 cell's slots in neighbouring lanes, so they share its fit's
//                 loads), the gradient of the cell's kept fit there, grad U =
//                 (1/h_c) sum_k a_k grad_xi phi_k, stored cell-major
//                 [N][NGPC][DIM][NV] (a face reads each side's DIM x NV
//                 values from one line)
//   k_flux_visc   per face: at each Gauss point, both sides' gradients (the
//                 slot pass's in FP64, evaluated here in FP32) averaged with
//                 the penalty (alpha / L_int) (U_R - U_L) n; F_v . n at the
//                 mean state; w |S| F_v subtracted from the face's integrated
//                 flux, before the gather.
// (Evaluated in the face kernel, both sides at every point, the FP64
// gradients held so many registers that 3D r = 4 spilled 1988 B per lane; the
// slot pass holds one gradient at a time.)
//
// Temperature T = p / rho; viscosity by Sutherland's law; conduction
// (mu / Pr) gamma / (gamma - 1) grad T.  Velocity and temperature gradients
// follow from the conserved ones by the chain rule at the mean state:
//   grad u_i = (grad m_i - u_i grad rho) / rho,
//   grad p = (gamma - 1) (grad E - sum_i u_i grad m_i + |u|^2 grad rho / 2),
//   grad T = (grad p - T grad rho) / rho.
#include "hfv_device.hpp"

namespace hfv {

template <typename T>
struct ViscParams {
  T gamma, mu0, T0, S, prandtl, alpha;
};

// Large FP64 fits (K > 20) take one lane per (cell, variable): a lane then
// holds K coefficients instead of K nvar (3D r = 4: one thread per cell held
// 256 VGPRs, one wave per SIMD, 4.5 ms per pass on 64^3 cells); the same sums
// per variable, so the same fits.  Elsewhere one thread per cell, which loads
// each pseudo-inverse entry once for all variables, measured faster.
template <int DIM, int R, typename T>
constexpr bool keep_split() { return sizeof(T) == 8 && n_unknowns(DIM, R) > 20; }

template <int DIM, int R, typename T>
__global__ __launch_bounds__(256) void k_keep_fits(HotArgs<T> a) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R);
  if constexpr (keep_split<DIM, R, T>()) {
    Lane<NV> L(a.xcd);
    const int cell = L.item, v = L.sub;
    if (!L.ok || cell >= a.N) return;
    T u0[1] = {a.U[(long)v * a.N + cell]};
    T co[K][1];
    lsq_coeffs<DIM, R, 1, T>(a, cell, v, u0, co);
#pragma unroll
    for (int k = 0; k < K; ++k) a.coef[((long)k * NV + v) * a.N + cell] = co[k][0];
  } else {
    const int cell = (int)(block_id(a.xcd) * blockDim.x + threadIdx.x);
    if (cell >= a.N) return;
    T u0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u0[v] = a.U[(long)v * a.N + cell];
    T co[K][NV];
    lsq_coeffs<DIM, R, NV, T>(a, cell, 0, u0, co);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) a.coef[((long)k * NV + v) * a.N + cell] = co[k][v];
  }
}

// Gradient of the conserved variables of cell c at its slot g from its kept
// fit: d/dx_j = (1/h_c) sum_k a_k d(xi^alpha_k)/d xi_j.
template <int DIM, int R, typename T>
__device__ inline void fit_gradient(const T *coef, const T *gpxi, int N, int c, int g, T hinv,
                                    T (&grad)[DIM][DIM + 2]) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R);
  constexpr Exps<DIM, 1, R> E{};
  T xi[DIM], pw[DIM][R + 1];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    xi[j] = gpxi[((long)g * DIM + j) * N + c];
    pw[j][0] = (T)1;
#pragma unroll
    for (int p = 1; p <= R; ++p) pw[j][p] = pw[j][p - 1] * xi[j];
  }
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) grad[j][v] = (T)0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T d[DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      if (E.e[k][j] == 0) {
        d[j] = (T)0;
      } else {
        T m = (T)E.e[k][j] * pw[j][E.e[k][j] - 1];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
          if (i != j) m *= pw[i][E.e[k][i]];
        d[j] = m;
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T ak = coef[((long)k * NV + v) * N + c];
#pragma unroll
      for (int j = 0; j < DIM; ++j) grad[j][v] += ak * d[j];
    }
  }
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) grad[j][v] *= hinv;
}

template <int DIM, typename T>
__device__ inline void viscous_flux(const T (&qL)[DIM + 2], const T (&qR)[DIM + 2], const T (&gL)[DIM][DIM + 2],
                                    const T (&gR)[DIM][DIM + 2], const T (&n)[DIM], T il, const ViscParams<T> &vp,
                                    T (&F)[DIM + 2]) {
  constexpr int NV = DIM + 2;
  T Um[NV], G[DIM][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Um[v] = (T)0.5 * (qL[v] + qR[v]);
    const T jump = vp.alpha * il * (qR[v] - qL[v]);
#pragma unroll
    for (int j = 0; j < DIM; ++j) G[j][v] = (T)0.5 * (gL[j][v] + gR[j][v]) + jump * n[j];
  }
  const T rho = Um[0], ir = (T)1 / rho;
  T u[DIM], q2 = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    u[i] = Um[1 + i] * ir;
    q2 += u[i] * u[i];
  }
  const T gm1 = vp.gamma - (T)1;
  const T p = gm1 * (Um[NV - 1] - (T)0.5 * rho * q2);
  const T Tm = p * ir;
  T du[DIM][DIM], gT[DIM];   // du[i][j] = d u_i / d x_j
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    T um = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      du[i][j] = (G[j][1 + i] - u[i] * G[j][0]) * ir;
      um += u[i] * G[j][1 + i];
    }
    const T gp = gm1 * (G[j][NV - 1] - um + (T)0.5 * q2 * G[j][0]);
    gT[j] = (gp - Tm * G[j][0]) * ir;
  }
  const T tr = Tm / vp.T0;
  const T mu = vp.mu0 * tr * sqrt(tr) * (vp.T0 + vp.S) / (Tm + vp.S);
  T div = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) div += du[i][i];
  const T kc = mu / vp.prandtl * vp.gamma / gm1;
  F[0] = (T)0;
  T work = 0, cond = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const T tau = mu * (du[i][j] + du[j][i] - (i == j ? (T)(2.0 / 3.0) * div : (T)0));
      s += tau * n[j];
    }
    F[1 + i] = s;
    work += u[i] * s;
    cond += gT[i] * n[i];
  }
  F[NV - 1] = work + kc * cond;
}

// FP64 takes the slot pass (its face kernel with both gradients spilled:
// 3D r = 4, 1988 B per lane); FP32 evaluates the gradients in the face kernel
// (no spill there, and no gradient array to write and read back).
template <typename T>
constexpr bool visc_slots() { return sizeof(T) == 8; }

template <int DIM, int R, typename T>
__global__ __launch_bounds__(256) void k_slot_grads(int N, int NGPC, const T *coef, const T *gpxi,
                                                    const uint8_t *ngp, const T *hinv, T *vgrad) {
  constexpr int NV = DIM + 2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)N * NGPC) return;
  const int c = (int)(t / NGPC), g = (int)(t - (long)c * NGPC);
  if (g >= ngp[c]) return;
  T gr[DIM][NV];
  fit_gradient<DIM, R, T>(coef, gpxi, N, c, g, hinv[c], gr);
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) vgrad[(t * DIM + j) * NV + v] = gr[j][v];
}

// SLOTS: the gradients come from k_slot_grads; otherwise the face evaluates
// both sides' fits at each of its points itself.
template <int DIM, int R, typename T, bool SLOTS>
__global__ __launch_bounds__(256) void k_flux_visc(int NF, int N, int NGPC, const T *fs, const T *vgrad,
                                                   const T *coef, const T *gpxi, const T *hinv, const int *gp_off,
                                                   const int *fc, const int *fgb, const T *fn, const T *gpw,
                                                   const T *linv, ViscParams<T> vp, T *Ff, int xcd) {
  constexpr int NV = DIM + 2;
  const int f = (int)(block_id(xcd) * blockDim.x + threadIdx.x);
  if (f >= NF) return;
  T n[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) n[j] = fn[(long)j * NF + f];
  const int cL = fc[f], cR0 = fc[NF + f], cR = cR0 >= 0 ? cR0 : cL;
  const int code = fgb[f], sL = code & 255, sR = (code >> 8) & 255;
  const T il = linv[f];
  T acc[NV] = {};
  for (int g = gp_off[f], i = 0; g < gp_off[f + 1]; ++g, ++i) {
    T qL[NV], qR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qL[v] = fs[((long)(sL + i) * NV + v) * N + cL];
      qR[v] = fs[((long)(sR + i) * NV + v) * N + cR];
    }
    T gL[DIM][NV], gR[DIM][NV];
    if constexpr (SLOTS) {
#pragma unroll
      for (int j = 0; j < DIM; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          gL[j][v] = vgrad[(((long)cL * NGPC + sL + i) * DIM + j) * NV + v];
          gR[j][v] = vgrad[(((long)cR * NGPC + sR + i) * DIM + j) * NV + v];
        }
    } else {
      fit_gradient<DIM, R, T>(coef, gpxi, N, cL, sL + i, hinv[cL], gL);
      fit_gradient<DIM, R, T>(coef, gpxi, N, cR, sR + i, hinv[cR], gR);
    }
    T F[NV];
    viscous_flux<DIM, T>(qL, qR, gL, gR, n, il, vp, F);
    const T w = gpw[g];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += w * F[v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Ff[(long)v * NF + f] -= acc[v];
}

template <int DIM, int R, typename T>
static void launch_dr(hfv_ctx *ctx, Tables<T> &t, const void *fs, void *Ff, hipStream_t s) {
  const ViscParams<T> vp{(T)ctx->p.gamma, (T)ctx->p.mu0, (T)ctx->p.T0, (T)ctx->p.suth_S, (T)ctx->p.prandtl,
                         (T)ctx->p.visc_alpha};
  const unsigned gf = (ctx->NF + 255) / 256;
  if constexpr (visc_slots<T>()) {
    const long slots = (long)ctx->N * ctx->NGPC;
    k_slot_grads<DIM, R, T><<<(unsigned)((slots + 255) / 256), 256, 0, s>>>(
        ctx->N, ctx->NGPC, (const T *)ctx->coef, t.gpxi, t.ngp, t.hinv, (T *)ctx->vgrad);
    k_flux_visc<DIM, R, T, true><<<gf, 256, 0, s>>>(
        ctx->NF, ctx->N, ctx->NGPC, (const T *)fs, (const T *)ctx->vgrad, nullptr, nullptr, nullptr, t.gp_off,
        t.face_cells, t.fgb, t.fnormal, t.gpw, t.linv, vp, (T *)Ff, ctx->xcd_remap);
  } else {
    k_flux_visc<DIM, R, T, false><<<gf, 256, 0, s>>>(
        ctx->NF, ctx->N, ctx->NGPC, (const T *)fs, nullptr, (const T *)ctx->coef, t.gpxi, t.hinv, t.gp_off,
        t.face_cells, t.fgb, t.fnormal, t.gpw, t.linv, vp, (T *)Ff, ctx->xcd_remap);
  }
}

template <int DIM, int R, typename T>
static void keep_dr(hfv_ctx *ctx, Tables<T> &t, const void *U, hipStream_t s) {
  HotArgs<T> a{};
  a.N = ctx->N;
  a.NF = ctx->NF;
  a.U = (const T *)U;
  a.coef = (T *)ctx->coef;
  a.t = t;
  a.xcd = ctx->xcd_remap;
  constexpr int CPW = keep_split<DIM, R, T>() ? 64 / (DIM + 2) : 64;
  const long waves = ((long)ctx->N + CPW - 1) / CPW;
  k_keep_fits<DIM, R, T><<<(unsigned)((waves * 64 + 255) / 256), 256, 0, s>>>(a);
}

template <typename T>
static hfv_status visc_t(hfv_ctx *ctx, Tables<T> &t, const void *fs, void *Ff, hipStream_t s) {
#define F(D, R, TT) launch_dr<D, R, TT>(ctx, t, fs, Ff, s)
  switch (ctx->dim * 10 + ctx->r) {
    case 21: F(2, 1, T); break;
    case 22: F(2, 2, T); break;
    case 23: F(2, 3, T); break;
    case 24: F(2, 4, T); break;
    case 25: F(2, 5, T); break;
    case 26: F(2, 6, T); break;
    case 31: F(3, 1, T); break;
    case 32: F(3, 2, T); break;
    case 33: F(3, 3, T); break;
    case 34: F(3, 4, T); break;
    default: ctx->err = "unsupported (dim, order_r)"; return HFV_ERR_PARAM;
  }
#undef F
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

template <typename T>
static hfv_status keep_t(hfv_ctx *ctx, Tables<T> &t, const void *U, hipStream_t s) {
#define F(D, R, TT) keep_dr<D, R, TT>(ctx, t, U, s)
  switch (ctx->dim * 10 + ctx->r) {
    case 21: F(2, 1, T); break;
    case 22: F(2, 2, T); break;
    case 23: F(2, 3, T); break;
    case 24: F(2, 4, T); break;
    case 25: F(2, 5, T); break;
    case 26: F(2, 6, T); break;
    case 31: F(3, 1, T); break;
    case 32: F(3, 2, T); break;
    case 33: F(3, 3, T); break;
    case 34: F(3, 4, T); break;
    default: ctx->err = "unsupported (dim, order_r)"; return HFV_ERR_PARAM;
  }
#undef F
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

hfv_status run_viscous_flux(hfv_ctx *ctx, const void *fs, void *Ff, hipStream_t s) {
  if (ctx->prec == 64 && !ctx->vgrad) return ctx->err = "viscous gradient buffer missing", HFV_ERR_STATE;
  return ctx->prec == 64 ? visc_t<double>(ctx, ctx->t64, fs, Ff, s) : visc_t<float>(ctx, ctx->t32, fs, Ff, s);
}

hfv_status run_keep_fits(hfv_ctx *ctx, const void *U, hipStream_t s) {
  return ctx->prec == 64 ? keep_t<double>(ctx, ctx->t64, U, s) : keep_t<float>(ctx, ctx->t32, U, s);
}

}  // namespace hfv
