// Device code shared by the forward and adjoint kernels.
#pragma once

#include "hfv_internal.hpp"

namespace hfv {


template <typename T>
struct HotArgs {
  int N, NF, mode, form;
  int frozen;              // adjoint recompute: classes given, no NAD or Harten re-check
  const uint8_t *cls_in;   // given classes when frozen
  const T *U;
  T *fs;
  T *coef;                 // central fits kept for CWENOZ ([K][NV][N]), or null
  uint8_t *own;
  uint8_t *cls;
  int *lists;
  int *counts;
  Tables<T> t;
  T gamma, alpha_m, beta_m, alpha_w, beta_w, lam1p, eps_w, b_w, theta, tvd_eps;
  int ib_w;  // b_w when it is an integer in [1, 8] (powers by multiplication), else 0
  int xcd;   // block ids remapped so each XCD takes one contiguous range (block_id)
  int limiter;  // HFV_LIM_*
  T *margin;    // [N] near_margin output of the linear pass, or null
  int NGPC;     // Gauss-point slots per cell (row length of the cell-major gpxi copy)
};

// CWENOZ on characteristic variables (hfv_char.cpp) over the class-1 list,
// or over every cell when direct.
template <typename T>
hfv_status launch_cwenoz_char(hfv_ctx *ctx, const HotArgs<T> &a, int direct, hipStream_t s);

// Block id, optionally permuted.  The dispatcher hands workgroups to the 8
// XCDs in turn (block b to XCD b mod 8), and each XCD has its own L2.  With
// the remap, the blocks running on one XCD cover one contiguous range of
// items instead of every eighth block, so cells that gather the same
// neighbour values (nearby ids) meet in the same L2.  A permutation of the
// block ids: results do not change.
__device__ inline long block_id(int xcd) {
  const unsigned b = blockIdx.x, n = gridDim.x;
  if (!xcd || n < 16) return b;
  const unsigned x = b & 7u, k = b >> 3, per = n >> 3, rem = n & 7u;
  return (long)x * per + min(x, rem) + k;
}

// x^b for x >= 0: repeated products when b is a small integer, pow otherwise.
__device__ inline double powb(double x, double b, int ib) {
  if (ib > 0) {
    double r = x;
    for (int i = 1; i < ib; ++i) r *= x;
    return r;
  }
  return pow(x, b);
}

template <int G>
struct Lane {
  int item, sub, base;
  bool ok;
  __device__ explicit Lane(int xcd = 0) {
    constexpr int CPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const long wave = (block_id(xcd) * blockDim.x + threadIdx.x) >> 6;
    item = (int)(wave * CPW + lane / G);
    sub = lane % G;
    base = lane - sub;
    ok = lane < CPW * G;
  }
};

template <int G, typename V>
__device__ inline V group_sum(V x, int base) {
  if constexpr (G == 1) return x;
  V s = 0;
#pragma unroll
  for (int t = 0; t < G; ++t) s += __shfl(x, base + t);
  return s;
}
template <int G>
__device__ inline int group_max(int x, int base) {
  if constexpr (G == 1) return x;
  int s = x;
#pragma unroll
  for (int t = 0; t < G; ++t) s = max(s, __shfl(x, base + t));
  return s;
}
template <int G, typename V>
__device__ inline V group_min(V x, int base) {
  if constexpr (G == 1) return x;
  V s = x;
#pragma unroll
  for (int t = 0; t < G; ++t) s = fmin(s, __shfl(x, base + t));
  return s;
}
template <int G>
__device__ inline bool group_all(bool x, int base) {
  if constexpr (G == 1) return x;
  int s = 1;
#pragma unroll
  for (int t = 0; t < G; ++t) s &= __shfl((int)x, base + t);
  return s != 0;
}

// All NV values of a state whose variables are spread over the group.
template <int NV, int G, typename T>
__device__ inline void group_state(const T (&mine)[NV / G], T (&all)[NV], int base) {
  constexpr int VPL = NV / G;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if constexpr (G == 1)
      all[v] = mine[v];
    else
      all[v] = __shfl(mine[v % VPL], base + v / VPL);
  }
}

// Harten bound check at one point for density and pressure (Eq. harten_jump_fix).
template <int NV, typename T>
__device__ inline bool harten_point(const T (&q)[NV], T rho_b, T p_b, const HotArgs<T> &a) {
  const T rho = q[0];
  if (!(fabs(rho - rho_b) <= a.theta * fmax(fabs(rho_b), a.tvd_eps))) return false;
  T m2 = 0;
#pragma unroll
  for (int j = 1; j < NV - 1; ++j) m2 += q[j] * q[j];
  const T p = (a.gamma - (T)1) * (q[NV - 1] - (T)0.5 * m2 / rho);
  return fabs(p - p_b) <= a.theta * fmax(fabs(p_b), a.tvd_eps);
}

template <int NV, typename T>
__device__ inline T pressure(const T (&q)[NV], T gamma) {
  T m2 = 0;
#pragma unroll
  for (int j = 1; j < NV - 1; ++j) m2 += q[j] * q[j];
  return (gamma - (T)1) * (q[NV - 1] - (T)0.5 * m2 / q[0]);
}

// near_margin: how far a cell's class decisions are from their thresholds,
// each as a relative distance; the output is the smallest.
//   Harten (Eq. harten_jump_fix) at one point, density and pressure:
//     | |q - q_bar| - theta s | / s,  s = max(|q_bar|, eps)
template <int NV, typename T>
__device__ inline T harten_margin(const T (&q)[NV], T rho_b, T p_b, const HotArgs<T> &a) {
  const T sr = fmax(fabs(rho_b), a.tvd_eps), sp = fmax(fabs(p_b), a.tvd_eps);
  const T p = pressure<NV, T>(q, a.gamma);
  return fmin(fabs(fabs(q[0] - rho_b) - a.theta * sr) / sr, fabs(fabs(p - p_b) - a.theta * sp) / sp);
}
//   NAD (Eqs. NADMUSCL, NADCWENOZ, marginm, marginw) for one variable with
//   a non-zero range R = M - m: min(|d - delta_w|, |d - delta_m|) / S with
//   S = max(|m|, |M|, R); a variable with R = 0 has no threshold (+inf)
template <typename T>
__device__ inline T nad_margin(T exc, T mn, T mx, T dw, T dm) {
  const T Rg = mx - mn;
  if (!(Rg > (T)0)) return (T)INFINITY;
  const T S = fmax(fmax(fabs(mn), fabs(mx)), Rg);
  return fmin(fabs(exc - dw), fabs(exc - dm)) / S;
}
//   deactivation (Eq. NADDeactivatedCriteria): |dU - thr| / max(dU, thr)
//   (0 when both are 0: the strict test sits exactly at its threshold)
template <typename T>
__device__ inline T deact_margin(T dU, T thr) {
  const T den = fmax(dU, thr);
  return den > (T)0 ? fabs(dU - thr) / den : (T)0;
}

// phi_k(xi) = xi^alpha_k - psi_bar_k for the hierarchical monomial basis.
template <int DIM, int R, typename T>
__device__ inline void basis_at(const T (&xi)[DIM], const T (&psb)[n_unknowns(DIM, R)],
                                T (&phi)[n_unknowns(DIM, R)]) {
  constexpr Exps<DIM, 1, R> E{};
  constexpr int K = n_unknowns(DIM, R);
  T pw[DIM][R + 1];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    pw[j][0] = (T)1;
#pragma unroll
    for (int p = 1; p <= R; ++p) pw[j][p] = pw[j][p - 1] * xi[j];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T m = pw[0][E.e[k][0]];
#pragma unroll
    for (int j = 1; j < DIM; ++j) m *= pw[j][E.e[k][j]];
    phi[k] = m - psb[k];
  }
}

// The polynomial U_i + sum_k a_k (xi^alpha_k - psi_bar_k) regrouped as
// c0 + sum_k a_k xi^alpha_k with c0 = U_i - sum_k a_k psi_bar_k, so that the
// Gauss-point loop needs neither the basis means nor their K registers.
template <int DIM, int R, int VPL, typename T>
__device__ inline void poly_offset(const HotArgs<T> &a, int cell, const T (&u0)[VPL],
                                   const T (&co)[n_unknowns(DIM, R)][VPL], T (&c0)[VPL]) {
  constexpr int K = n_unknowns(DIM, R);
#pragma unroll
  for (int q = 0; q < VPL; ++q) c0[q] = u0[q];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const T pb = a.t.psibar[(long)k * a.N + cell];
#pragma unroll
    for (int q = 0; q < VPL; ++q) c0[q] -= co[k][q] * pb;
  }
}

template <int DIM, int R, int VPL, typename T>
__device__ inline void poly_at(const T (&xi)[DIM], const T (&co)[n_unknowns(DIM, R)][VPL], const T (&c0)[VPL],
                               T (&val)[VPL]) {
  constexpr Exps<DIM, 1, R> E{};
  constexpr int K = n_unknowns(DIM, R);
  T pw[DIM][R + 1];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    pw[j][0] = (T)1;
#pragma unroll
    for (int p = 1; p <= R; ++p) pw[j][p] = pw[j][p - 1] * xi[j];
  }
#pragma unroll
  for (int q = 0; q < VPL; ++q) val[q] = c0[q];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T m = pw[0][E.e[k][0]];
#pragma unroll
    for (int j = 1; j < DIM; ++j) m *= pw[j][E.e[k][j]];
#pragma unroll
    for (int q = 0; q < VPL; ++q) val[q] += co[k][q] * m;
  }
}

// a[k][q] = sum_m P[k][m] (U_{s_m} - U_i)   (Section 2.1, a = A^+ b)
template <int DIM, int R, int VPL, typename T>
__device__ inline void lsq_coeffs(const HotArgs<T> &a, int cell, int v0, const T (&u0)[VPL],
                                  T (&co)[n_unknowns(DIM, R)][VPL]) {
  constexpr int K = n_unknowns(DIM, R), M = 2 * K;
  const int N = a.N;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int q = 0; q < VPL; ++q) co[k][q] = (T)0;
  auto member = [&](int m) {
    const int j = a.t.sten[(long)m * N + cell];
    T du[VPL];
#pragma unroll
    for (int q = 0; q < VPL; ++q) du[q] = a.U[(long)(v0 + q) * N + j] - u0[q];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T p = a.t.P[((long)k * M + m) * N + cell];
#pragma unroll
      for (int q = 0; q < VPL; ++q) co[k][q] += p * du[q];
    }
  };
  // two members in flight for small K; one for large K, whose K loads per
  // member would otherwise exhaust the registers
  if constexpr (K > 20) {
#pragma unroll 1
    for (int m = 0; m < M; ++m) member(m);
  } else {
#pragma unroll 2
    for (int m = 0; m < M; ++m) member(m);
  }
}

// Gauss-point states are cell-major, [NGPC][NV][N]: slot g of a cell is its
// g-th face Gauss point in the cell's face order, so a wave's stores of one
// (slot, variable) pair are contiguous across its cells.
template <int NV, typename T>
__device__ inline void store(const HotArgs<T> &a, int g, int cell, int v, T val) {
  a.fs[((long)g * NV + v) * a.N + cell] = val;
}

// Frame coordinates of PB of a cell's Gauss-point slots, g0, g0 + step, ...;
// slots past its count ng (>= 1) repeat its last one, so every load is in
// bounds and unconditional.  A point loop that stores face states cannot have
// its later loads moved above those stores (the compiler cannot rule out that
// they alias), so it would wait for each point's coordinates in turn; loading
// PB points at once waits once per PB points.
constexpr int GP_BATCH = 4;
// CM: from the cell-major copy.
template <int PB, int DIM, typename T, bool CM = false>
__device__ inline void load_points(const HotArgs<T> &a, int cell, int g0, int step, int ng, T (&xs)[PB][DIM]) {
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int g = min(g0 + p * step, ng - 1);
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      xs[p][j] = CM ? a.t.gpxiC[((long)cell * a.NGPC + g) * DIM + j] : a.t.gpxi[((long)g * DIM + j) * a.N + cell];
  }
}

// Riemann fluxes (Section 2.4): HLLC and HLL with Davis wave-speed estimates.
template <int DIM, typename T>
__device__ inline void euler_flux(const T (&q)[DIM + 2], const T (&n)[DIM], T p, T un, T (&F)[DIM + 2]) {
  F[0] = q[0] * un;
#pragma unroll
  for (int j = 0; j < DIM; ++j) F[1 + j] = q[1 + j] * un + p * n[j];
  F[DIM + 1] = un * (q[DIM + 1] + p);
}

template <int DIM, typename T>
__device__ inline void riemann(const T (&qL)[DIM + 2], const T (&qR)[DIM + 2], const T (&n)[DIM], T gamma,
                               int hllc, T (&F)[DIM + 2]) {
  constexpr int NV = DIM + 2;
  const T rL = qL[0], rR = qR[0];
  T vL[DIM], vR[DIM], unL = T(0), unR = T(0), kL = T(0), kR = T(0);
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    vL[j] = qL[1 + j] / rL;
    vR[j] = qR[1 + j] / rR;
    unL += vL[j] * n[j];
    unR += vR[j] * n[j];
    kL += vL[j] * vL[j];
    kR += vR[j] * vR[j];
  }
  const T gm1 = gamma - (T)1, half = (T)0.5;
  const T pL = gm1 * (qL[NV - 1] - half * rL * kL);
  const T pR = gm1 * (qR[NV - 1] - half * rR * kR);
  const T cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
  const T SL = fmin(unL - cL, unR - cR), SR = fmax(unL + cL, unR + cR);
  T FL[NV], FR[NV];
  euler_flux<DIM, T>(qL, n, pL, unL, FL);
  euler_flux<DIM, T>(qR, n, pR, unR, FR);
  if (SL >= (T)0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = FL[v];
    return;
  }
  if (!hllc) {
    if (SR <= (T)0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = FR[v];
      return;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (qR[v] - qL[v])) / (SR - SL);
    return;
  }
  const T Ss = (pR - pL + rL * unL * (SL - unL) - rR * unR * (SR - unR)) / (rL * (SL - unL) - rR * (SR - unR));
  if (Ss >= (T)0) {
    const T fac = rL * (SL - unL) / (SL - Ss);
    F[0] = FL[0] + SL * (fac - qL[0]);
#pragma unroll
    for (int j = 0; j < DIM; ++j) F[1 + j] = FL[1 + j] + SL * (fac * (vL[j] + (Ss - unL) * n[j]) - qL[1 + j]);
    F[NV - 1] = FL[NV - 1] + SL * (fac * (qL[NV - 1] / rL + (Ss - unL) * (Ss + pL / (rL * (SL - unL)))) -
                                   qL[NV - 1]);
  } else if (SR > (T)0) {
    const T fac = rR * (SR - unR) / (SR - Ss);
    F[0] = FR[0] + SR * (fac - qR[0]);
#pragma unroll
    for (int j = 0; j < DIM; ++j) F[1 + j] = FR[1 + j] + SR * (fac * (vR[j] + (Ss - unR) * n[j]) - qR[1 + j]);
    F[NV - 1] = FR[NV - 1] + SR * (fac * (qR[NV - 1] / rR + (Ss - unR) * (Ss + pR / (rR * (SR - unR)))) -
                                   qR[NV - 1]);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = FR[v];
  }
}

}  // namespace hfv
