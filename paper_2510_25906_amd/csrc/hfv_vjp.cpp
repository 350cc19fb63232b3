// Vector-Jacobian product of the residual with the cell classes frozen.
//
// R(U) composes three maps: cell averages -> face Gauss-point states (the
// reconstruction of each cell's class), face states -> integrated face
// fluxes, face fluxes -> residual (Eq. EulerEquationsDetails).  The adjoint
// runs them backwards:
//   k_flux_vjp    dJ/dF from dJ/dR, then back through the Riemann solver at
//                 every Gauss point in hand-written reverse mode, branches
//                 (wave-speed choices, HLLC region) held at the primal values
//   k_recon_vjp   per cell and variable, back through the cell's frozen class:
//                 linear (Section 2.1), CWENOZ including its nonlinear weights
//                 (Section 2.3), MUSCL (Barth-Jespersen or Venkatakrishnan)
//                 through its limiting point and the neighbour that sets the
//                 bound (Section 2.2), or first order; contributions
//                 to each central-stencil slot are stored, not scattered
//   k_gather_vjp  each cell sums the slot contributions that refer to it
//                 through the transposed stencil, in a fixed order
// No floating-point atomics are used, so the result is deterministic.
#include "hfv_device.hpp"
#include "hfv_riemann_adj.hpp"

namespace hfv {

template <typename T>
struct VjpArgs {
  int N, form, limiter;
  const T *U;
  const uint8_t *cls;
  const int *lists;   // [3][N] class lists of the frozen forward recompute: CWENOZ, MUSCL, first order
  const int *counts;  // list lengths at 1 + list index
  const T *gfs;
  T *C;
  T *S;
  Tables<T> t;
  T lam1p, eps_w, b_w;
};

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_flux_vjp(int NF, int N, const T *fs, const int *gp_off, const int *fgb,
                                                  const T *fn, const T *gpw, const int *fc, const T *ivol,
                                                  const T *gR, T gamma, int hllc, T *gfs) {
  constexpr int NV = DIM + 2;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= NF) return;
  const int L = fc[f], Rc = fc[NF + f];
  const int code = fgb[f];
  const long oL = (long)(code & 255) * NV * N + L;
  const long oR = (long)((code >> 8) & 255) * NV * N + (Rc >= 0 ? Rc : L);
  T n[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) n[j] = fn[(long)j * NF + f];
  T gF[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    gF[v] = -gR[(long)v * N + L] * ivol[L] + (Rc >= 0 ? gR[(long)v * N + Rc] * ivol[Rc] : (T)0);
  for (int g = gp_off[f], i = 0; g < gp_off[f + 1]; ++g, ++i) {
    T qL[NV], qR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qL[v] = fs[oL + ((long)i * NV + v) * N];
      qR[v] = fs[oR + ((long)i * NV + v) * N];
    }
    const T w = gpw[g];
    T gl[NV], gr[NV];
    riemann_vjp<DIM, T>(qL, qR, n, gamma, hllc, gF, gl, gr);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      gl[v] *= w;
      gr[v] *= w;
    }
    // every cell slot belongs to exactly one face side, so each is written once
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (Rc < 0) {  // transmissive ghost: the right state is a copy of the left one
        gfs[oL + ((long)i * NV + v) * N] = gl[v] + gr[v];
      } else {
        gfs[oL + ((long)i * NV + v) * N] = gl[v];
        gfs[oR + ((long)i * NV + v) * N] = gr[v];
      }
    }
  }
}

__device__ inline double pow_safe(double x, double e) { return (x == 0.0 && e > 0.0) ? 0.0 : pow(x, e); }

// Reverse pass per (cell, variable) through the cell's class, one lane each.
// PASS 0 runs over every cell and takes the linear and first-order cells;
// PASS 1 and 2 run over the CWENOZ and MUSCL lists that the frozen forward
// recompute compacted, one list entry per lane group over a grid sized for
// every cell (a loop over entries would hold its registers across
// iterations).  PASS 0 and 2 compile only their classes' code, so they carry
// few registers; PASS 1 keeps the run-time switch over all classes (only
// CWENOZ cells reach it; at 3D r = 3 it needs fewer spill slots than a
// CWENOZ-only build, at equal occupancy).  The body stays in the kernel:
// moved into a device function (inlined or not), the CWENOZ path took 256
// VGPRs instead of 172 at 2D r = 3 FP64 and spilled to scratch at 3D r = 3.
template <int DIM, int R, typename T, int PASS>
__global__ __launch_bounds__(256) void k_recon_vjp(VjpArgs<T> a) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R), M = 2 * K, NFM = nf_max(DIM), MD = 2 * DIM;
  Lane<NV> L;
  if (!L.ok) return;
  int cell;
  if constexpr (PASS == 0) {
    if (L.item >= a.N) return;
    cell = L.item;
  } else {
    if (L.item >= a.counts[PASS]) return;
    cell = a.lists[(long)(PASS - 1) * a.N + L.item];
  }
  const int v = L.sub, N = a.N;
  const int cls = PASS == 2 ? (int)HFV_CLASS_MUSCL : (int)a.cls[cell];
  if (PASS == 0 && (cls == HFV_CLASS_CWENOZ || cls == HFV_CLASS_MUSCL)) return;
  const Tables<T> &t = a.t;
  const int ng = t.ngp[cell];
  const long MS = (long)NV * N;
  T *C = a.C + (long)cell * NV + v;  // [M][N][nvar]: slot m lives at C[m * MS]
  auto gq_at = [&](int g) -> T { return a.gfs[((long)g * NV + v) * N + cell]; };
  T gsum = 0;
  if (PASS != 2 && cls >= HFV_CLASS_FIRST_ORDER) {
    for (int g = 0; g < ng; ++g) gsum += gq_at(g);
    for (int m = 0; m < M; ++m) C[m * MS] = 0;
    a.S[(long)v * N + cell] = gsum;
    return;
  }
  const T u0 = a.U[(long)v * N + cell];
  T psb[K];
#pragma unroll
  for (int k = 0; k < K; ++k) psb[k] = t.psibar[(long)k * N + cell];
  auto xi_at = [&](int g, T(&xi)[DIM]) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) xi[j] = t.gpxi[((long)g * DIM + j) * N + cell];
  };

  if (PASS == 0 || (PASS == 1 && cls == HFV_CLASS_LINEAR)) {
    T b[K];
#pragma unroll
    for (int k = 0; k < K; ++k) b[k] = 0;
    for (int g = 0; g < ng; ++g) {
      const T gq = gq_at(g);
      gsum += gq;
      T xi[DIM], phi[K];
      xi_at(g, xi);
      basis_at<DIM, R, T>(xi, psb, phi);
#pragma unroll
      for (int k = 0; k < K; ++k) b[k] += phi[k] * gq;
    }
    T self = gsum;
    for (int m = 0; m < M; ++m) {
      T c = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) c += t.P[((long)k * M + m) * N + cell] * b[k];
      C[m * MS] = c;
      self -= c;
    }
    a.S[(long)v * N + cell] = self;
    return;
  }

  if (PASS == 1 && cls == HFV_CLASS_CWENOZ) {
    // ---- forward recompute (Section 2.3)
    T co[K];
#pragma unroll
    for (int k = 0; k < K; ++k) co[k] = 0;
    for (int m = 0; m < M; ++m) {
      const T du = a.U[(long)v * N + t.sten[(long)m * N + cell]] - u0;
#pragma unroll
      for (int k = 0; k < K; ++k) co[k] += t.P[((long)k * M + m) * N + cell] * du;
    }
    const int nd = t.ndir[cell];
    T ad[NFM][DIM];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) ad[s][j] = 0;
      if (s < nd) {
        for (int q = 0; q < MD; ++q) {
          const T du = a.U[(long)v * N + t.dsten[((long)s * MD + q) * N + cell]] - u0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) ad[s][j] += t.Pdir[(((long)s * DIM + j) * MD + q) * N + cell] * du;
        }
      }
    }
    const T lam1 = (T)1 - (T)1 / a.lam1p;
    const T lams = ((T)1 - lam1) / (T)nd;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T sdir = 0;
#pragma unroll
      for (int s = 0; s < NFM; ++s) sdir += ad[s][j];
      co[j] = co[j] - lams * sdir;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) co[k] /= lam1;  // co now holds p_1's coefficients
    double si1 = 0, sis[NFM];
#pragma unroll
    for (int s = 0; s < NFM; ++s) sis[s] = 0;
    {
      int p = 0;
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = k; q < K; ++q, ++p) {
          const double o = (double)t.OI[(long)p * N + cell] * (q == k ? 1.0 : 2.0);
          si1 += o * (double)co[k] * (double)co[q];
          if (q < DIM) {
#pragma unroll
            for (int s = 0; s < NFM; ++s) sis[s] += o * (double)ad[s][k] * (double)ad[s][q];
          }
        }
    }
    double tau = 0;
#pragma unroll
    for (int s = 0; s < NFM; ++s)
      if (s < nd) tau += fabs(sis[s] - si1);
    tau /= (double)nd;
    const double eps = (double)a.eps_w, b = (double)a.b_w, l1 = (double)lam1, ls = (double)lams;
    const bool zform = a.form == HFV_WENOZ_POW;
    double w1, ws[NFM], W;
    if (zform)
      w1 = l1 * (1.0 + pow_safe(tau / (eps + si1), b));
    else
      w1 = l1 * (1.0 + pow_safe(tau, b) / (eps + si1));
    W = w1;
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
      ws[s] = 0;
      if (s < nd)
        ws[s] = zform ? ls * (1.0 + pow_safe(tau / (eps + sis[s]), b)) : ls * (1.0 + pow_safe(tau, b) / (eps + sis[s]));
      W += ws[s];
    }
    const double om1 = w1 / W;
    double oms[NFM];
#pragma unroll
    for (int s = 0; s < NFM; ++s) oms[s] = ws[s] / W;
    // ---- backward
    T gb[K];  // d J / d (CWENOZ coefficients)
#pragma unroll
    for (int k = 0; k < K; ++k) gb[k] = 0;
    for (int g = 0; g < ng; ++g) {
      const T gq = gq_at(g);
      gsum += gq;
      T xi[DIM], phi[K];
      xi_at(g, xi);
      basis_at<DIM, R, T>(xi, psb, phi);
#pragma unroll
      for (int k = 0; k < K; ++k) gb[k] += phi[k] * gq;
    }
    double g_om1 = 0, g_oms[NFM];
#pragma unroll
    for (int k = 0; k < K; ++k) g_om1 += (double)gb[k] * (double)co[k];
    T gad[NFM][DIM];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
      g_oms[s] = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        g_oms[s] += (double)gb[j] * (double)ad[s][j];
        gad[s][j] = (T)oms[s] * gb[j];
      }
    }
    // gb becomes d J / d a_1
#pragma unroll
    for (int k = 0; k < K; ++k) gb[k] = (T)om1 * gb[k];
    double dot = g_om1 * om1;
#pragma unroll
    for (int s = 0; s < NFM; ++s) dot += g_oms[s] * oms[s];
    const double gw1 = (g_om1 - dot) / W;
    double gtau = 0, gsi1 = 0, gsis[NFM];
    {
      const double d1 = eps + si1;
      if (zform) {
        const double r1 = tau / d1;
        gtau += gw1 * l1 * b * pow_safe(r1, b - 1.0) / d1;
        gsi1 += -gw1 * l1 * b * pow_safe(r1, b) / d1;
      } else {
        gtau += gw1 * l1 * b * pow_safe(tau, b - 1.0) / d1;
        gsi1 += -gw1 * l1 * pow_safe(tau, b) / (d1 * d1);
      }
    }
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
      gsis[s] = 0;
      if (s < nd) {
        const double gws = (g_oms[s] - dot) / W;
        const double ds = eps + sis[s];
        if (zform) {
          const double rs = tau / ds;
          gtau += gws * ls * b * pow_safe(rs, b - 1.0) / ds;
          gsis[s] = -gws * ls * b * pow_safe(rs, b) / ds;
        } else {
          gtau += gws * ls * b * pow_safe(tau, b - 1.0) / ds;
          gsis[s] = -gws * ls * pow_safe(tau, b) / (ds * ds);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
      if (s < nd) {
        const double sg = (double)((sis[s] > si1) - (sis[s] < si1));
        gsis[s] += gtau * sg / (double)nd;
        gsi1 -= gtau * sg / (double)nd;
      }
    }
    // SI = a^T OI a  ->  d SI / d a = 2 OI a
    {
      int p = 0;
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = k; q < K; ++q, ++p) {
          const T o = t.OI[(long)p * N + cell];
          const T c1 = (T)(2.0 * gsi1) * o;
          gb[k] += c1 * co[q];
          if (q != k) gb[q] += c1 * co[k];
          if (q < DIM) {
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
              const T cs = (T)(2.0 * gsis[s]) * o;
              gad[s][k] += cs * ad[s][q];
              if (q != k) gad[s][q] += cs * ad[s][k];
            }
          }
        }
    }
    // a_1 = (a_opt - lambda_s sum_s a_s) / lambda_1
#pragma unroll
    for (int k = 0; k < K; ++k) gb[k] /= lam1;  // now d J / d a_opt
#pragma unroll
    for (int s = 0; s < NFM; ++s)
      if (s < nd) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) gad[s][j] -= lams * gb[j];
      }
    T self = gsum;
    for (int m = 0; m < M; ++m) {
      T c = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) c += t.P[((long)k * M + m) * N + cell] * gb[k];
      C[m * MS] = c;
      self -= c;
    }
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
      if (s < nd) {
        for (int q = 0; q < MD; ++q) {
          T x = 0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) x += t.Pdir[(((long)s * DIM + j) * MD + q) * N + cell] * gad[s][j];
          C[(long)t.dpos[((long)s * MD + q) * N + cell] * MS] += x;
          self -= x;
        }
      }
    }
    a.S[(long)v * N + cell] = self;
    return;
  }

  if (PASS != 0) {  // MUSCL with the Barth-Jespersen or Venkatakrishnan limiter (Sections 2.2, 3.2)
  for (int m = 0; m < M; ++m) C[m * MS] = 0;
  const int nm = t.nmus[cell];
  T gr[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) gr[j] = 0;
  for (int q = 0; q < nm; ++q) {
    const T du = a.U[(long)v * N + t.msten[(long)q * N + cell]] - u0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) gr[j] += t.Pmus[((long)j * NFM + q) * N + cell] * du;
  }
  T mn = u0, mx = u0;
  int imn = -1, imx = -1;
  const int nf = t.nfc[cell];
  for (int f = 0; f < nf; ++f) {
    const int j = t.nbr[(long)f * N + cell];
    if (j >= 0) {
      const T u = a.U[(long)v * N + j];
      if (u < mn) {
        mn = u;
        imn = f;
      }
      if (u > mx) {
        mx = u;
        imx = f;
      }
    }
  }
  // theta = min over the points of the limiter function, as in the forward pass
  const bool venkat = a.limiter == HFV_LIM_VENKAT;
  const T e2 = venkat ? t.veps2[cell] : (T)0;
  T th = 1, dstar = 0, dpstar = 0;
  int gstar = -1;
  for (int g = 0; g < ng; ++g) {
    T xi[DIM];
    xi_at(g, xi);
    T d = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) d += gr[j] * (xi[j] - psb[j]);
    T ratio = 1, dp = 0;
    if (d != 0) {
      dp = (d > 0 ? mx : mn) - u0;
      if (venkat)
        ratio = ((dp * dp + e2) * d + (T)2 * d * d * dp) / (d * (dp * dp + (T)2 * d * d + dp * d + e2));
      else
        ratio = fmin((T)1, dp / d);
    }
    if (ratio < th) {
      th = ratio;
      gstar = g;
      dstar = d;
      dpstar = dp;
    }
  }
  T gth = 0, gg[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) gg[j] = 0;
  for (int g = 0; g < ng; ++g) {
    const T gq = gq_at(g);
    gsum += gq;
    T xi[DIM];
    xi_at(g, xi);
    T d = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) d += gr[j] * (xi[j] - psb[j]);
    gth += gq * d;
#pragma unroll
    for (int j = 0; j < DIM; ++j) gg[j] += th * gq * (xi[j] - psb[j]);
  }
  T self = gsum;
  if (gstar >= 0) {
    // theta as a function of the room dp = bound - U_i and the increment d at
    // the limiting point: Barth-Jespersen dp / d; Venkatakrishnan
    // (dp^2 + 2 d dp + e2) / (dp^2 + 2 d^2 + d dp + e2)
    T th_dp, th_d;
    if (venkat) {
      const T num = dpstar * dpstar + (T)2 * dstar * dpstar + e2;
      const T den = dpstar * dpstar + (T)2 * dstar * dstar + dstar * dpstar + e2;
      th_dp = (((T)2 * dpstar + (T)2 * dstar) * den - num * ((T)2 * dpstar + dstar)) / (den * den);
      th_d = ((T)2 * dpstar * den - num * ((T)4 * dstar + dpstar)) / (den * den);
    } else {
      th_dp = (T)1 / dstar;
      th_d = -th / dstar;
    }
    const T ginv = gth * th_dp;
    self -= ginv;
    const int ib = dstar > 0 ? imx : imn;
    if (ib < 0)
      self += ginv;
    else
      C[(long)t.nbpos[(long)ib * N + cell] * MS] += ginv;
    T xi[DIM];
    xi_at(gstar, xi);
    const T gd = gth * th_d;
#pragma unroll
    for (int j = 0; j < DIM; ++j) gg[j] += gd * (xi[j] - psb[j]);
  }
  for (int q = 0; q < nm; ++q) {
    T x = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) x += t.Pmus[((long)j * NFM + q) * N + cell] * gg[j];
    C[(long)t.mpos[(long)q * N + cell] * MS] += x;
    self -= x;
  }
  a.S[(long)v * N + cell] = self;
  }
}

template <int NV, typename T>
__global__ __launch_bounds__(256) void k_gather_vjp(int N, const int *inv_off, const int *inv_idx, const T *C,
                                                    const T *S, T *gU) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  T acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = S[(long)v * N + j];
  // four entries at a time: their codes, then their contributions, requested
  // at once (a short last batch repeats its last entry, which is not added);
  // the sum keeps the entry order
  constexpr int EB = 4;
  const int e1 = inv_off[j + 1];
  for (int e0 = inv_off[j]; e0 < e1; e0 += EB) {
    int code[EB];
#pragma unroll
    for (int b = 0; b < EB; ++b) code[b] = inv_idx[min(e0 + b, e1 - 1)];
    T cv[EB][NV];
#pragma unroll
    for (int b = 0; b < EB; ++b) {
      const int m = code[b] / N, i = code[b] - m * N;
#pragma unroll
      for (int v = 0; v < NV; ++v) cv[b][v] = C[((long)m * N + i) * NV + v];  // one cache line per entry
    }
#pragma unroll
    for (int b = 0; b < EB; ++b)
      if (e0 + b < e1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += cv[b][v];
      }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) gU[(long)v * N + j] = acc[v];
}

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <int DIM, int R, typename T>
static hfv_status vjp_impl(hfv_ctx *ctx, Tables<T> &t, const void *U, const uint8_t *cls, const void *fs,
                           const void *gR, void *gU, hipStream_t s) {
  constexpr int NV = DIM + 2;
  // face states given: only the class lists are rebuilt; else the frozen
  // forward reconstruction recomputes the states (and builds the lists)
  hfv_status e = fs ? run_class_lists(ctx, cls, s) : run_reconstruct_frozen(ctx, U, ctx->fs_ws, cls, s);
  if (e != HFV_OK) return e;
  const T *fsu = (const T *)(fs ? fs : ctx->fs_ws);
  ProfScope ps(ctx, HFV_SLOT_VJP, s);
  k_flux_vjp<DIM, T><<<nblk(ctx->NF, 256), 256, 0, s>>>(ctx->NF, ctx->N, fsu, t.gp_off, t.fgb,
                                                         t.fnormal, t.gpw, t.face_cells, t.ivol, (const T *)gR,
                                                         (T)ctx->p.gamma, ctx->p.riemann == HFV_HLLC,
                                                         (T *)ctx->vjp_gfs);
  VjpArgs<T> a;
  a.N = ctx->N;
  a.form = ctx->p.form;
  a.limiter = ctx->p.limiter;
  a.U = (const T *)U;
  a.cls = cls;
  a.gfs = (const T *)ctx->vjp_gfs;
  a.C = (T *)ctx->vjp_C;
  a.S = (T *)ctx->vjp_S;
  a.t = t;
  a.lam1p = (T)ctx->p.lam1p;
  a.eps_w = (T)ctx->p.eps_w;
  a.b_w = (T)ctx->p.b_w;
  a.lists = ctx->lists;
  a.counts = ctx->counts;
  constexpr int CPW = 64 / NV;
  const long waves = ((long)ctx->N + CPW - 1) / CPW;
  const unsigned grid_cells = nblk(waves * 64, 256);
  k_recon_vjp<DIM, R, T, 0><<<grid_cells, 256, 0, s>>>(a);
  k_recon_vjp<DIM, R, T, 1><<<grid_cells, 256, 0, s>>>(a);
  k_recon_vjp<DIM, R, T, 2><<<grid_cells, 256, 0, s>>>(a);
  k_gather_vjp<NV, T><<<nblk(ctx->N, 256), 256, 0, s>>>(ctx->N, t.inv_off, t.inv_idx, (const T *)ctx->vjp_C,
                                                       (const T *)ctx->vjp_S, (T *)gU);
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

template <typename T>
static hfv_status vjp_t(hfv_ctx *ctx, Tables<T> &t, const void *U, const uint8_t *cls, const void *fs,
                        const void *gR, void *gU, hipStream_t s) {
  switch (ctx->dim * 10 + ctx->r) {
    case 21: return vjp_impl<2, 1, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 22: return vjp_impl<2, 2, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 23: return vjp_impl<2, 3, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 24: return vjp_impl<2, 4, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 31: return vjp_impl<3, 1, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 32: return vjp_impl<3, 2, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 33: return vjp_impl<3, 3, T>(ctx, t, U, cls, fs, gR, gU, s);
    case 34: return vjp_impl<3, 4, T>(ctx, t, U, cls, fs, gR, gU, s);
  }
  ctx->err = "the residual VJP is built for order_r <= 4";
  return HFV_ERR_PARAM;
}

hfv_status run_vjp(hfv_ctx *ctx, const void *U, const uint8_t *cls, const void *fs, const void *gR, void *gU,
                   hipStream_t s) {
  if (!ctx->vjp_ok) {
    ctx->err = "residual VJP unavailable for these stencils: " + ctx->vjp_why;
    return HFV_ERR_STATE;
  }
  if (ctx->p.cvars != HFV_CONSERVED) {
    ctx->err = "the residual VJP differentiates conserved-variable CWENOZ only";
    return HFV_ERR_STATE;
  }
  if (ctx->p.viscous) {
    ctx->err = "the residual VJP differentiates the inviscid residual only";
    return HFV_ERR_STATE;
  }
  return ctx->prec == 64 ? vjp_t<double>(ctx, ctx->t64, U, cls, fs, gR, gU, s)
                         : vjp_t<float>(ctx, ctx->t32, U, cls, fs, gR, gU, s);
}

}  // namespace hfv
