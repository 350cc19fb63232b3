// Hot path of the hybrid reconstruction (Section 2.5, Fig. HybridWENOFlowchart).
//
//   k_linear     linear least-squares candidate of every cell (Section 2.1),
//                its face Gauss-point states, the NAD class of the cell
//                (Eqs. DMP, NADMUSCL, NADCWENOZ, marginm, marginw, with the
//                deactivation of Eq. NADDeactivatedCriteria) and the Harten
//                check of the candidate (Eq. harten_jump_fix)
//   k_classify   tagging of the flagged cells' von Neumann neighbourhood and
//                wave-ballot / prefix compaction into per-class work lists
//   k_cwenoz     CWENOZ on the class-1 list (Section 2.3); with merged lists
//                also the two lists below, in the same launch
//   k_muscl      Barth-Jespersen limited MUSCL on the class-2 list (Section 2.2)
//                and first-order states on the cells that failed the Harten check
//   k_flux       HLLC / HLL flux integrated over each face's Gauss points
//   k_gather     residual of Eq. EulerEquationsDetails, fixed-order sums
//
// Work mapping: G lanes of a 64-wide wave share one cell, each lane owning
// NV/G conserved variables (per-variable reconstruction, Section 2.3).  The
// per-cell matrices are stored [row][cell] so a wave's loads of one matrix
// entry are contiguous across its cells.
#include "hfv_device.hpp"

namespace hfv {

// ---------------------------------------------------------------------------
// Central fit of a cell kept for the CWENOZ pass (the linear polynomial is
// CWENOZ's central candidate, Section 2.3).  Every cell's fit is kept so that
// the CWENOZ list stays one dense list in cell order.
template <int NV, typename T, int K, int VPL>
__device__ inline void keep_fit(const HotArgs<T> &a, int cell, int v0, const T (&co)[K][VPL]) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int q = 0; q < VPL; ++q) a.coef[((long)k * NV + v0 + q) * a.N + cell] = co[k][q];
}

// K1: linear candidate, face states, NAD own class, Harten flag.  MG: the
// near_margin output is computed (a variant of its own: its code, even
// unexecuted, was allocated registers that cost the plain kernel occupancy,
// 3D r = 4 FP64 five lanes 168 -> 204 VGPRs, 3 -> 2 waves/SIMD).
template <int DIM, int R, typename T, int G, bool MG>
__global__ __launch_bounds__(256) void k_linear(HotArgs<T> a) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R), VPL = NV / G, NFM = nf_max(DIM);
  if constexpr (!MG) a.margin = nullptr;
  if (blockIdx.x == 0 && threadIdx.x < 8) a.counts[threadIdx.x] = 0;
  Lane<G> L(a.xcd);
  const int cell = L.item;
  if (!L.ok || cell >= a.N) return;
  const int N = a.N, v0 = L.sub * VPL;
  T u0[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) u0[q] = a.U[(long)(v0 + q) * N + cell];
  T co[K][VPL];
  lsq_coeffs<DIM, R, VPL, T>(a, cell, v0, u0, co);

  // NAD bounds over the cell and its face neighbours; deactivation norms
  T mn[VPL], mx[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) mn[q] = mx[q] = u0[q];
  T dmax = -INFINITY, dmin = INFINITY;
  bool has_nb = false;
  // rows past the cell's face count hold -1, as do boundary faces: every
  // row is read without waiting for the count
#pragma unroll
  for (int f = 0; f < NFM; ++f) {
    const int j = a.t.nbr[(long)f * N + cell];
    if (j >= 0) {
      T s2 = 0;
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        const T u = a.U[(long)(v0 + q) * N + j];
        mn[q] = fmin(mn[q], u);
        mx[q] = fmax(mx[q], u);
        s2 += (u - u0[q]) * (u - u0[q]);
      }
      s2 = group_sum<G>(s2, L.base);
      const T nrm = sqrt(s2);
      dmax = fmax(dmax, nrm);
      dmin = fmin(dmin, nrm);
      has_nb = true;
    }
  }
  T all0[NV];
  group_state<NV, G, T>(u0, all0, L.base);
  const T rho_b = all0[0];
  const T p_b = pressure<NV, T>(all0, a.gamma);

  T c0[VPL];
  poly_offset<DIM, R, VPL, T>(a, cell, u0, co, c0);
  T exc[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) exc[q] = -INFINITY;
  bool hok = true;
  T mg = (T)INFINITY;  // near_margin (every lane sees the full state at each point)
  const int ng = a.t.ngp[cell];
  for (int g0 = 0; g0 < ng; g0 += GP_BATCH) {
    T xs[GP_BATCH][DIM];
    load_points<GP_BATCH, DIM, T>(a, cell, g0, 1, ng, xs);
#pragma unroll
    for (int p = 0; p < GP_BATCH; ++p) {
      const int g = g0 + p;
      if (g < ng) {
        T val[VPL];
        poly_at<DIM, R, VPL, T>(xs[p], co, c0, val);
#pragma unroll
        for (int q = 0; q < VPL; ++q) exc[q] = fmax(exc[q], fmax(mn[q] - val[q], val[q] - mx[q]));
        T all[NV];
        group_state<NV, G, T>(val, all, L.base);
        hok = hok && harten_point<NV, T>(all, rho_b, p_b, a);
        if (a.margin) mg = fmin(mg, harten_margin<NV, T>(all, rho_b, p_b, a));
#pragma unroll
        for (int q = 0; q < VPL; ++q) store<NV, T>(a, g, cell, v0 + q, val[q]);
      }
    }
  }
  int c = 0;
  if (a.mode == HFV_HYBRID) {
    T nm = (T)INFINITY;
#pragma unroll
    for (int q = 0; q < VPL; ++q) {
      const T Rg = mx[q] - mn[q];
      const T dm = fmax(a.alpha_m, a.beta_m * Rg);
      const T sgn = (T)((a.beta_w > 0) - (a.beta_w < 0));
      const T dw = sgn * fmax(a.alpha_w, fabs(a.beta_w * Rg));
      const int cq = exc[q] <= dw ? HFV_CLASS_LINEAR : (exc[q] >= dm ? HFV_CLASS_MUSCL : HFV_CLASS_CWENOZ);
      c = max(c, cq);
      nm = fmin(nm, nad_margin(exc[q], mn[q], mx[q], dw, dm));
    }
    c = group_max<G>(c, L.base);
    const T dU = has_nb ? dmax - dmin : (T)0;
    if (dU < a.t.thr[cell]) c = HFV_CLASS_LINEAR;
    if (a.margin) mg = fmin(fmin(mg, group_min<G>(nm, L.base)), deact_margin(dU, a.t.thr[cell]));
  }
  if (a.coef) keep_fit<NV>(a, cell, v0, co);
  if (L.sub == 0) {
    a.own[cell] = (uint8_t)(c | (hok ? 0 : 4));
    if (a.margin) a.margin[cell] = mg;
  }
}

// K1, member-split mapping: the G lanes of a cell's group each take every G-th
// stencil member (all variables), so one load instruction fetches G distinct
// rows of the cell's pseudo-inverse; a butterfly sum gives every lane the
// full coefficients.  The lanes then split the face neighbours and the Gauss
// points, and combine the NAD excursions and Harten flags.  Same results as
// k_linear up to the order of the sums.
template <int G, typename V>
__device__ inline V xor_sum(V x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x += __shfl_xor(x, off);
  return x;
}
template <int G, typename V>
__device__ inline V xor_max(V x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x = fmax(x, __shfl_xor(x, off));
  return x;
}
template <int G, typename V>
__device__ inline V xor_min(V x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x = fmin(x, __shfl_xor(x, off));
  return x;
}

template <int DIM, int R, typename T, int G, bool MG>
__global__ __launch_bounds__(256) void k_linear_ms(HotArgs<T> a) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R), M = 2 * K, NFM = nf_max(DIM);
  if constexpr (!MG) a.margin = nullptr;
  constexpr int MPL = (M + G - 1) / G;
  static_assert((G & (G - 1)) == 0 && 64 % G == 0, "group size must be a power of two");
  if (blockIdx.x == 0 && threadIdx.x < 8) a.counts[threadIdx.x] = 0;
  Lane<G> L(a.xcd);
  const int cell = L.item;
  if (!L.ok || cell >= a.N) return;  // whole groups leave together
  const int N = a.N, q = L.sub;
  T u0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u0[v] = a.U[(long)v * N + cell];
  T co[K][NV];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v) co[k][v] = (T)0;
#pragma unroll
  for (int t = 0; t < MPL; ++t) {
    const int m = q + t * G;
    if (m < M) {
      const int j = a.t.sten[(long)m * N + cell];
      T du[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) du[v] = a.U[(long)v * N + j] - u0[v];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T p = a.t.P[((long)k * M + m) * N + cell];
#pragma unroll
        for (int v = 0; v < NV; ++v) co[k][v] += p * du[v];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v) co[k][v] = xor_sum<G>(co[k][v]);

  T mn[NV], mx[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) mn[v] = mx[v] = u0[v];
  T dmax = -INFINITY, dmin = INFINITY;
#pragma unroll
  for (int f0 = 0; f0 < NFM; f0 += G) {
    const int f = f0 + q;
    if (f < NFM) {  // rows past the cell's face count hold -1
      const int j = a.t.nbr[(long)f * N + cell];
      if (j >= 0) {
        T s2 = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T u = a.U[(long)v * N + j];
          mn[v] = fmin(mn[v], u);
          mx[v] = fmax(mx[v], u);
          s2 += (u - u0[v]) * (u - u0[v]);
        }
        const T nrm = sqrt(s2);
        dmax = fmax(dmax, nrm);
        dmin = fmin(dmin, nrm);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    mn[v] = xor_min<G>(mn[v]);
    mx[v] = xor_max<G>(mx[v]);
  }
  dmax = xor_max<G>(dmax);
  dmin = xor_min<G>(dmin);
  const bool has_nb = dmax >= (T)0;
  const T rho_b = u0[0];
  const T p_b = pressure<NV, T>(u0, a.gamma);
  T c0[NV];
  poly_offset<DIM, R, NV, T>(a, cell, u0, co, c0);
  T exc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) exc[v] = -INFINITY;
  bool hok = true;
  T mg = (T)INFINITY;  // near_margin, this lane's points
  const int ng = a.t.ngp[cell];
  constexpr int PB = GP_BATCH / 2;
  for (int g0 = q; g0 < ng; g0 += PB * G) {
    T xs[PB][DIM];
    load_points<PB, DIM, T>(a, cell, g0, G, ng, xs);
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int g = g0 + p * G;
      if (g < ng) {
        T val[NV];
        poly_at<DIM, R, NV, T>(xs[p], co, c0, val);
#pragma unroll
        for (int v = 0; v < NV; ++v) exc[v] = fmax(exc[v], fmax(mn[v] - val[v], val[v] - mx[v]));
        hok = hok && harten_point<NV, T>(val, rho_b, p_b, a);
        if (a.margin) mg = fmin(mg, harten_margin<NV, T>(val, rho_b, p_b, a));
#pragma unroll
        for (int v = 0; v < NV; ++v) store<NV, T>(a, g, cell, v, val[v]);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) exc[v] = xor_max<G>(exc[v]);
  {
    int hv = hok ? 1 : 0;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) hv &= __shfl_xor(hv, off);
    hok = hv != 0;
  }
  if (a.margin) mg = xor_min<G>(mg);
  int c = 0;
  if (a.mode == HFV_HYBRID) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T Rg = mx[v] - mn[v];
      const T dm = fmax(a.alpha_m, a.beta_m * Rg);
      const T sgn = (T)((a.beta_w > 0) - (a.beta_w < 0));
      const T dw = sgn * fmax(a.alpha_w, fabs(a.beta_w * Rg));
      const int cv = exc[v] <= dw ? HFV_CLASS_LINEAR : (exc[v] >= dm ? HFV_CLASS_MUSCL : HFV_CLASS_CWENOZ);
      c = max(c, cv);
      if (a.margin) mg = fmin(mg, nad_margin(exc[v], mn[v], mx[v], dw, dm));
    }
    const T dU = has_nb ? dmax - dmin : (T)0;
    if (dU < a.t.thr[cell]) c = HFV_CLASS_LINEAR;
    if (a.margin) mg = fmin(mg, deact_margin(dU, a.t.thr[cell]));
  }
  if (a.coef) {  // every lane holds the full fit: split the stores
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if ((k * NV + v) % G == q) a.coef[((long)k * NV + v) * N + cell] = co[k][v];
  }
  if (q == 0) {
    a.own[cell] = (uint8_t)(c | (hok ? 0 : 4));
    if (a.margin) a.margin[cell] = mg;
  }
}

// K1, unknown-split mapping: lane q of a cell's group of G owns the unknowns
// k = q, q + G, q + 2G, ... for every variable, so the group streams each row
// of the cell's pseudo-inverse exactly once and a lane holds only K/G x NV
// coefficients.  Face Gauss points are taken G at a time: each lane forms the
// partial sums of its unknowns at the G points, and a butterfly
// reduce-scatter over the group leaves lane q with the full state at point q
// of the batch, which it checks (NAD excursion, Harten) and stores.
template <int DIM, int R, typename T, int G, bool MG>
__global__ __launch_bounds__(256) void k_linear_ks(HotArgs<T> a) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R), M = 2 * K, NFM = nf_max(DIM);
  if constexpr (!MG) a.margin = nullptr;
  constexpr int KPL = (K + G - 1) / G;
  constexpr Exps<DIM, 1, R> E{};
  static_assert((G & (G - 1)) == 0 && G >= 2 && 64 % G == 0, "group size must be a power of two");
  if (blockIdx.x == 0 && threadIdx.x < 8) a.counts[threadIdx.x] = 0;
  Lane<G> L(a.xcd);
  const int cell = L.item;
  if (!L.ok || cell >= a.N) return;  // whole groups leave together
  const int N = a.N, q = L.sub;
  T u0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u0[v] = a.U[(long)v * N + cell];
  T co[KPL][NV];
#pragma unroll
  for (int j = 0; j < KPL; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) co[j][v] = (T)0;
  // members in pairs (M = 2K is even), their stencil ids loaded one pair
  // ahead: a pair's averages are requested with its pseudo-inverse rows
  int jn0 = a.t.sten[cell], jn1 = a.t.sten[(long)N + cell];
#pragma unroll 1
  for (int m = 0; m < M; m += 2) {
    const int jp[2] = {jn0, jn1};
    jn0 = a.t.sten[(long)min(m + 2, M - 2) * N + cell];
    jn1 = a.t.sten[(long)min(m + 3, M - 1) * N + cell];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jc = jp[h];
      T du[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) du[v] = a.U[(long)v * N + jc] - u0[v];
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        const int k = q + j * G;
        if (j * G + G <= K || k < K) {
          const T p = a.t.P[((long)k * M + m + h) * N + cell];
#pragma unroll
          for (int v = 0; v < NV; ++v) co[j][v] += p * du[v];
        }
      }
    }
  }
  // NAD bounds and deactivation norms over the face neighbours, split over the group
  T mn[NV], mx[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) mn[v] = mx[v] = u0[v];
  T dmax = -INFINITY, dmin = INFINITY;
#pragma unroll
  for (int f0 = 0; f0 < NFM; f0 += G) {
    const int f = f0 + q;
    if (f < NFM) {  // rows past the cell's face count hold -1
      const int j = a.t.nbr[(long)f * N + cell];
      if (j >= 0) {
        T s2 = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T u = a.U[(long)v * N + j];
          mn[v] = fmin(mn[v], u);
          mx[v] = fmax(mx[v], u);
          s2 += (u - u0[v]) * (u - u0[v]);
        }
        const T nrm = sqrt(s2);
        dmax = fmax(dmax, nrm);
        dmin = fmin(dmin, nrm);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    mn[v] = xor_min<G>(mn[v]);
    mx[v] = xor_max<G>(mx[v]);
  }
  dmax = xor_max<G>(dmax);
  dmin = xor_min<G>(dmin);
  const bool has_nb = dmax >= (T)0;
  const T rho_b = u0[0];
  const T p_b = pressure<NV, T>(u0, a.gamma);
  // In FP64 this lane's share of sum_k a_k psi_bar_k leaves the Gauss-point
  // loop (raw monomials there, fewer live registers); in FP32 keeping the
  // basis means measured faster.
  constexpr bool FOLD = sizeof(T) == 8;
  T off[NV], psb[KPL];
#pragma unroll
  for (int v = 0; v < NV; ++v) off[v] = (T)0;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int k = q + j * G;
    const T pb = (k < K) ? a.t.psibar[(long)k * N + cell] : (T)0;
    if constexpr (FOLD) {
#pragma unroll
      for (int v = 0; v < NV; ++v) off[v] += co[j][v] * pb;
    } else {
      psb[j] = pb;
    }
  }
  T exc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) exc[v] = -INFINITY;
  bool hok = true;
  T mg = (T)INFINITY;  // near_margin, this lane's points
  const int ng = a.t.ngp[cell];
  for (int g0 = 0; g0 < ng; g0 += G) {
    T part[G][NV];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const int g = min(g0 + t, ng - 1);  // a short last batch repeats the cell's last point
      T pw[DIM][R + 1];
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const T x = a.t.gpxi[((long)g * DIM + j) * N + cell];
        pw[j][0] = (T)1;
#pragma unroll
        for (int p = 1; p <= R; ++p) pw[j][p] = pw[j][p - 1] * x;
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) part[t][v] = FOLD ? -off[v] : (T)0;
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        // this lane's unknown k = q + j G: pick its monomial among the G candidates
        T mono = (T)0;
#pragma unroll
        for (int s = 0; s < G; ++s) {
          const int k = j * G + s;
          if (k < K) {
            T m = pw[0][E.e[k][0]];
#pragma unroll
            for (int d = 1; d < DIM; ++d) m *= pw[d][E.e[k][d]];
            mono = (q == s) ? m : mono;
          }
        }
        if constexpr (!FOLD) mono -= psb[j];
#pragma unroll
        for (int v = 0; v < NV; ++v) part[t][v] += co[j][v] * mono;
      }
    }
    // reduce-scatter: halve the batch at each step, keeping the half picked by this lane's bit
    T full[NV];
    {
      T cur[G][NV];
#pragma unroll
      for (int t = 0; t < G; ++t)
#pragma unroll
        for (int v = 0; v < NV; ++v) cur[t][v] = part[t][v];
#pragma unroll
      for (int H = G / 2; H >= 1; H /= 2) {
        const bool hi = (q & H) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i)
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const T keep = hi ? cur[i + H][v] : cur[i][v];
            const T send = hi ? cur[i][v] : cur[i + H][v];
            cur[i][v] = keep + __shfl_xor(send, H);
          }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) full[v] = cur[0][v];
    }
    const int g = g0 + q;
    if (g < ng) {
      T val[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        val[v] = u0[v] + full[v];
        exc[v] = fmax(exc[v], fmax(mn[v] - val[v], val[v] - mx[v]));
      }
      hok = hok && harten_point<NV, T>(val, rho_b, p_b, a);
      if (a.margin) mg = fmin(mg, harten_margin<NV, T>(val, rho_b, p_b, a));
#pragma unroll
      for (int v = 0; v < NV; ++v) store<NV, T>(a, g, cell, v, val[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) exc[v] = xor_max<G>(exc[v]);
  {
    int hv = hok ? 1 : 0;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) hv &= __shfl_xor(hv, off);
    hok = hv != 0;
  }
  if (a.margin) mg = xor_min<G>(mg);
  int c = 0;
  if (a.mode == HFV_HYBRID) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T Rg = mx[v] - mn[v];
      const T dm = fmax(a.alpha_m, a.beta_m * Rg);
      const T sgn = (T)((a.beta_w > 0) - (a.beta_w < 0));
      const T dw = sgn * fmax(a.alpha_w, fabs(a.beta_w * Rg));
      const int cv = exc[v] <= dw ? HFV_CLASS_LINEAR : (exc[v] >= dm ? HFV_CLASS_MUSCL : HFV_CLASS_CWENOZ);
      c = max(c, cv);
      if (a.margin) mg = fmin(mg, nad_margin(exc[v], mn[v], mx[v], dw, dm));
    }
    const T dU = has_nb ? dmax - dmin : (T)0;
    if (dU < a.t.thr[cell]) c = HFV_CLASS_LINEAR;
    if (a.margin) mg = fmin(mg, deact_margin(dU, a.t.thr[cell]));
  }
  if (a.coef) {
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
      const int k = q + j * G;
      if (k < K) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.coef[((long)k * NV + v) * N + cell] = co[j][v];
      }
    }
  }
  if (q == 0) {
    a.own[cell] = (uint8_t)(c | (hok ? 0 : 4));
    if (a.margin) a.margin[cell] = mg;
  }
}

// K2: final class (dilation over face neighbours) and per-class lists.  The
// neighbour rows are read all at once (rows past a cell's face count hold
// -1, like boundary faces), not in a loop over the cell's count, whose loads
// would wait on one another.  Blocks of 1024: each block reserves its range
// of a list with one atomic on the list's length, and on the 1M-cell mixed
// box blocks of 256 made those atomics the bottleneck (24 -> 50 us).
constexpr int CLASSIFY_BLOCK = 1024;
template <typename T, int NFM>
__global__ __launch_bounds__(CLASSIFY_BLOCK) void k_classify(HotArgs<T> a) {
  const int cell = (int)(block_id(a.xcd) * blockDim.x + threadIdx.x);
  const bool valid = cell < a.N;
  int c = 0;
  if (valid && a.frozen) {
    c = min((int)a.cls_in[cell], (int)HFV_CLASS_FIRST_ORDER);  // larger values: first order
  } else if (valid) {
    const int o = a.own[cell];
    c = o & 3;
    if (a.mode == HFV_HYBRID) {
      int nb[NFM];
#pragma unroll
      for (int f = 0; f < NFM; ++f) nb[f] = a.t.nbr[(long)f * a.N + cell];
#pragma unroll
      for (int f = 0; f < NFM; ++f)
        if (nb[f] >= 0) c = max(c, a.own[nb[f]] & 3);
    } else {
      c = HFV_CLASS_LINEAR;
    }
    if (c == HFV_CLASS_LINEAR && (o & 4)) c = HFV_CLASS_FIRST_ORDER;
    a.cls[cell] = (uint8_t)c;
  }
  // List of the cell: CWENOZ (0), MUSCL (1), first order (2).
  const int li = c - 1;
  // Compaction: wave ballots give each lane its rank inside the wave; the
  // waves of the block combine their counts in LDS and the block reserves its
  // range of each list with one atomic per list.
  constexpr int NW = CLASSIFY_BLOCK / 64;
  __shared__ int wcount[3][NW];
  __shared__ int wbase[3][NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long masks[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    masks[k] = __ballot(valid && li == k);
    if (lane == 0) wcount[k][wave] = __popcll(masks[k]);
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    int tot = 0;
    for (int w = 0; w < NW; ++w) {
      wbase[k][w] = tot;
      tot += wcount[k][w];
    }
    const int start = tot ? atomicAdd(&a.counts[k + 1], tot) : 0;
    for (int w = 0; w < NW; ++w) wbase[k][w] += start;
  }
  __syncthreads();
  if (valid && li >= 0) a.lists[(long)li * a.N + wbase[li][wave] + __popcll(masks[li] & lt)] = cell;
}

// K4: one cell of the MUSCL list: gradient by least squares over the face
// neighbours, Barth-Jespersen (or Venkatakrishnan) limiter, Harten check.
template <int DIM, int R, typename T, int G, bool CM = false>
__device__ __forceinline__ void muscl_cell(const HotArgs<T> &a, int cell, const Lane<G> &L) {
  constexpr int NV = DIM + 2, VPL = NV / G, NFM = nf_max(DIM);
  const int N = a.N, v0 = L.sub * VPL;
  T u0[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) u0[q] = a.U[(long)(v0 + q) * N + cell];
  T gr[DIM][VPL];
#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int q = 0; q < VPL; ++q) gr[j][q] = 0;
  // members past the cell's count are padded with the cell itself and zero
  // weights (exact zeros), neighbour rows past its face count with -1
#pragma unroll
  for (int m = 0; m < NFM; ++m) {
    const int jc = CM ? a.t.mstenC[(long)cell * NFM + m] : a.t.msten[(long)m * N + cell];
    T du[VPL];
#pragma unroll
    for (int q = 0; q < VPL; ++q) du[q] = a.U[(long)(v0 + q) * N + jc] - u0[q];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const T p = CM ? a.t.PmusC[((long)cell * DIM + j) * NFM + m] : a.t.Pmus[((long)j * NFM + m) * N + cell];
#pragma unroll
      for (int q = 0; q < VPL; ++q) gr[j][q] += p * du[q];
    }
  }
  T mn[VPL], mx[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) mn[q] = mx[q] = u0[q];
#pragma unroll
  for (int f = 0; f < NFM; ++f) {
    const int j = CM ? a.t.nbrC[(long)cell * NFM + f] : a.t.nbr[(long)f * N + cell];
    if (j >= 0) {
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        const T u = a.U[(long)(v0 + q) * N + j];
        mn[q] = fmin(mn[q], u);
        mx[q] = fmax(mx[q], u);
      }
    }
  }
  T psb[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j)
    psb[j] = CM ? a.t.psibarC[(long)cell * n_unknowns(DIM, R) + j] : a.t.psibar[(long)j * N + cell];
  const int ng = a.t.ngp[cell];
  const bool venkat = a.limiter == HFV_LIM_VENKAT;
  const T e2 = venkat ? a.t.veps2[cell] : (T)0;
  T th[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) th[q] = (T)1;
  for (int g0 = 0; g0 < ng; g0 += GP_BATCH) {
    T xs[GP_BATCH][DIM];
    load_points<GP_BATCH, DIM, T, CM>(a, cell, g0, 1, ng, xs);
#pragma unroll
    for (int p = 0; p < GP_BATCH; ++p) {
      if (g0 + p < ng) {
#pragma unroll
        for (int q = 0; q < VPL; ++q) {
          T d = 0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) d += gr[j][q] * (xs[p][j] - psb[j]);
          T ratio = (T)1;
          if (d != 0) {
            const T dp = (d > 0 ? mx[q] : mn[q]) - u0[q];   // room to the bound in the direction of d
            if (venkat)   // smooth limiter function of Venkatakrishnan (1995)
              ratio = ((dp * dp + e2) * d + (T)2 * d * d * dp) / (d * (dp * dp + (T)2 * d * d + dp * d + e2));
            else          // Barth-Jespersen
              ratio = fmin((T)1, dp / d);
          }
          th[q] = fmin(th[q], ratio);
        }
      }
    }
  }
  T all0[NV];
  group_state<NV, G, T>(u0, all0, L.base);
  const T rho_b = all0[0];
  const T p_b = pressure<NV, T>(all0, a.gamma);
  // limited states and their Harten check; the rare failure rewrites the
  // cell's points with the first-order state afterwards
  bool hok = true;
  for (int g0 = 0; g0 < ng; g0 += GP_BATCH) {
    T xs[GP_BATCH][DIM];
    load_points<GP_BATCH, DIM, T, CM>(a, cell, g0, 1, ng, xs);
#pragma unroll
    for (int p = 0; p < GP_BATCH; ++p) {
      if (g0 + p < ng) {
        T val[VPL];
#pragma unroll
        for (int q = 0; q < VPL; ++q) {
          T d = 0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) d += gr[j][q] * (xs[p][j] - psb[j]);
          val[q] = u0[q] + th[q] * d;
        }
        T all[NV];
        group_state<NV, G, T>(val, all, L.base);
        hok = hok && (a.frozen || harten_point<NV, T>(all, rho_b, p_b, a));
#pragma unroll
        for (int q = 0; q < VPL; ++q) store<NV, T>(a, g0 + p, cell, v0 + q, val[q]);
      }
    }
  }
  if (!hok) {
    for (int g = 0; g < ng; ++g)
#pragma unroll
      for (int q = 0; q < VPL; ++q) store<NV, T>(a, g, cell, v0 + q, u0[q]);
  }
  if (L.sub == 0 && !a.frozen) a.cls[cell] = hok ? HFV_CLASS_MUSCL : HFV_CLASS_FIRST_ORDER;
}

// K5: one cell of the first-order list: the cell average at every Gauss point.
template <int DIM, typename T, int G>
__device__ __forceinline__ void first_order_cell(const HotArgs<T> &a, int cell, const Lane<G> &L) {
  constexpr int NV = DIM + 2, VPL = NV / G;
  const int N = a.N, v0 = L.sub * VPL;
  T u0[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) u0[q] = a.U[(long)(v0 + q) * N + cell];
  const int ng = a.t.ngp[cell];
#pragma unroll 4
  for (int g = 0; g < ng; ++g)
#pragma unroll
    for (int q = 0; q < VPL; ++q) store<NV, T>(a, g, cell, v0 + q, u0[q]);
}

// K3: CWENOZ over the class-1 list (every cell when direct).  REUSE: the
// central fit is read from the linear pass's copy instead of refitted.  The
// body stays written out in the kernel: moved into a device function (even
// inlined) it was allocated more registers (2D r = 3 FP64, two lanes: 255 +
// 12 AGPRs instead of 245, one wave per SIMD instead of two).
// MERGED (lists only): the same launch then also serves the MUSCL and the
// first-order lists, as items past the CWENOZ list, so their cells fill the
// waves CWENOZ leaves idle instead of waiting for a launch of their own.
// They run in a loop of their own after the CWENOZ loop (each lane continues
// its item sequence there); a template parameter, so that the plain kernel's
// code is not changed by them.  CM: OI is read from its cell-major copy (a
// sparse list then reads each cell's entries from consecutive cache lines;
// the directional stencils' ids and fits likewise; compile-time, since runtime
// strides cost the kernel registers and occupancy).
template <int DIM, int R, typename T, int G, bool REUSE, bool MERGED, bool CM>
__global__ __launch_bounds__(256) void k_cwenoz(HotArgs<T> a, int direct) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R), VPL = NV / G, NFM = nf_max(DIM), MD = 2 * DIM;
  constexpr int NOI = K * (K + 1) / 2;
  constexpr int CPW = 64 / G;
  const int total = direct ? a.N : a.counts[1];
  Lane<G> L(a.xcd);
  if (!L.ok) return;
  const long stride = (long)gridDim.x * (blockDim.x / 64) * CPW;
  long item = L.item;
  for (; item < total; item += stride) {
    const int cell = direct ? (int)item : a.lists[item];
    const int N = a.N, v0 = L.sub * VPL;
    T u0[VPL];
#pragma unroll
    for (int q = 0; q < VPL; ++q) u0[q] = a.U[(long)(v0 + q) * N + cell];
    T co[K][VPL];
    if constexpr (REUSE) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < VPL; ++q) co[k][q] = a.coef[((long)k * NV + v0 + q) * N + cell];
    } else {
      lsq_coeffs<DIM, R, VPL, T>(a, cell, v0, u0, co);
    }
    // directional degree-1 fits (Section 2.3)
    const int nd = a.t.ndir[cell];
    T ad[NFM][DIM][VPL];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
#pragma unroll
      for (int j = 0; j < DIM; ++j)
#pragma unroll
        for (int q = 0; q < VPL; ++q) ad[s][j][q] = (T)0;
      // the guard also keeps the compiler from hoisting every stencil's loads
      // at once, which would cost occupancy (two lanes: 1 wave/SIMD); stencils
      // past the count have zero weights on the cell itself, so they add exact
      // zeros.  With a kept fit and four or five lanes the registers allow the
      // hoisting, which then hides the averages' latency that the refit's
      // gathers would otherwise have warmed up (85k-cell mesh, FP64 four lanes:
      // 67 -> 52 us; FP32: 29 -> 26 us)
      if ((REUSE && G >= 4) || s < nd) {
#pragma unroll
        for (int m = 0; m < MD; ++m) {
          const int jc = CM ? a.t.dstenC[((long)cell * NFM + s) * MD + m] : a.t.dsten[((long)s * MD + m) * N + cell];
          T du[VPL];
#pragma unroll
          for (int q = 0; q < VPL; ++q) du[q] = a.U[(long)(v0 + q) * N + jc] - u0[q];
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            const T p = CM ? a.t.PdirC[(((long)cell * NFM + s) * DIM + j) * MD + m]
                           : a.t.Pdir[(((long)s * DIM + j) * MD + m) * N + cell];
#pragma unroll
            for (int q = 0; q < VPL; ++q) ad[s][j][q] += p * du[q];
          }
        }
      }
    }
    const T lam1 = (T)1 - (T)1 / a.lam1p;
    const T lams = ((T)1 - lam1) / (T)nd;
    // p_1 = (p_opt - sum lambda_s p_s) / lambda_1, in place
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        T sdir = 0;
#pragma unroll
        for (int s = 0; s < NFM; ++s) sdir += ad[s][j][q];
        co[j][q] = co[j][q] - lams * sdir;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < VPL; ++q) co[k][q] /= lam1;
    // smoothness indicators SI = a^T OI a, accumulated in double, then the
    // nonlinear weights and the CWENOZ coefficients omega_1 p_1 + sum_s
    // omega_s p_s; one variable at a time keeps few doubles live
    const double eps = (double)a.eps_w, b = (double)a.b_w;
#pragma unroll
    for (int q = 0; q < VPL; ++q) {
      double si1 = 0, sis[NFM];
#pragma unroll
      for (int s = 0; s < NFM; ++s) sis[s] = 0;
      int pidx = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double ck = (double)co[k][q];
        double row = 0;
#pragma unroll
        for (int kq = k; kq < K; ++kq, ++pidx) {
          const double o = CM ? (double)a.t.OIc[(long)cell * NOI + pidx] : (double)a.t.OI[(long)pidx * N + cell];
          row += (kq == k ? o : 2.0 * o) * (double)co[kq][q];
          if (kq < DIM) {
#pragma unroll
            for (int s = 0; s < NFM; ++s)
              sis[s] += (kq == k ? o : 2.0 * o) * (double)ad[s][k][q] * (double)ad[s][kq][q];
          }
        }
        si1 += ck * row;
        // large K in FP64: keep each row's loads from being hoisted over the
        // others (measured: spills otherwise; FP32 is faster without)
        if constexpr (K > 20 && sizeof(T) == 8) __builtin_amdgcn_sched_barrier(0);
      }
      double tau = 0;
#pragma unroll
      for (int s = 0; s < NFM; ++s)
        if (s < nd) tau += fabs(sis[s] - si1);
      tau /= (double)nd;
      const bool zform = a.form == HFV_WENOZ_POW;
      const double taub = zform ? 0.0 : powb(tau, b, a.ib_w);
      const double w1 = (double)lam1 * (1.0 + (zform ? powb(tau / (eps + si1), b, a.ib_w) : taub / (eps + si1)));
      double tot = w1, ws[NFM];
#pragma unroll
      for (int s = 0; s < NFM; ++s) {
        ws[s] = 0;
        if (s < nd)
          ws[s] = (double)lams * (1.0 + (zform ? powb(tau / (eps + sis[s]), b, a.ib_w) : taub / (eps + sis[s])));
        tot += ws[s];
      }
      const double it = 1.0 / tot;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double v = w1 * it * (double)co[k][q];
        if (k < DIM) {
#pragma unroll
          for (int s = 0; s < NFM; ++s) v += ws[s] * it * (double)ad[s][k][q];
        }
        co[k][q] = (T)v;
      }
    }
    // face states, Harten check
    T all0[NV];
    group_state<NV, G, T>(u0, all0, L.base);
    const T rho_b = all0[0];
    const T p_b = pressure<NV, T>(all0, a.gamma);
    T psb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) psb[k] = CM ? a.t.psibarC[(long)cell * K + k] : a.t.psibar[(long)k * N + cell];
    const int ng = a.t.ngp[cell];
    bool hok = true;
    // points one at a time in FP64 with one or two lanes per cell (measured:
    // batched loads made that kernel's schedule slower, 61 -> 85 us on the
    // 85k-cell mixed mesh; faster everywhere else)
    constexpr int PB = (sizeof(T) == 8 && G <= 2) ? 1 : GP_BATCH;
    for (int g0 = 0; g0 < ng && hok; g0 += PB) {
      T xs[PB][DIM];
      load_points<PB, DIM, T, CM>(a, cell, g0, 1, ng, xs);
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        if (g0 + p < ng && hok) {
          T phi[K];
          basis_at<DIM, R, T>(xs[p], psb, phi);
          T val[VPL];
#pragma unroll
          for (int q = 0; q < VPL; ++q) {
            T s = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) s += co[k][q] * phi[k];
            val[q] = u0[q] + s;
          }
          T all[NV];
          group_state<NV, G, T>(val, all, L.base);
          hok = a.frozen || harten_point<NV, T>(all, rho_b, p_b, a);
#pragma unroll
          for (int q = 0; q < VPL; ++q) store<NV, T>(a, g0 + p, cell, v0 + q, val[q]);
        }
      }
    }
    if (!hok) {
      // first-order fallback: every point of the cell takes U_i (the points
      // after the failing one were not evaluated)
      for (int g = 0; g < ng; ++g) {
#pragma unroll
        for (int q = 0; q < VPL; ++q) store<NV, T>(a, g, cell, v0 + q, u0[q]);
      }
    }
    if (L.sub == 0 && !a.frozen) a.cls[cell] = hok ? HFV_CLASS_CWENOZ : HFV_CLASS_FIRST_ORDER;
  }
  if constexpr (MERGED) {
    const int n2 = a.counts[2], n3 = a.counts[3];
    for (long i2 = item - total; i2 < (long)n2 + n3; i2 += stride) {
      if (i2 < n2)
        muscl_cell<DIM, R, T, G, CM>(a, a.lists[(long)a.N + i2], L);
      else
        first_order_cell<DIM, T, G>(a, a.lists[2L * a.N + (i2 - n2)], L);
    }
  }
}

// K4 + K5 as a launch of their own: list 2 (every cell when direct), then
// list 3.
template <int DIM, int R, typename T, int G, bool CM>
__global__ __launch_bounds__(256) void k_muscl(HotArgs<T> a, int direct) {
  constexpr int CPW = 64 / G;
  const int total = direct ? a.N : a.counts[2];
  Lane<G> L(a.xcd);
  if (!L.ok) return;
  const long stride = (long)gridDim.x * (blockDim.x / 64) * CPW;
  for (long item = L.item; item < total; item += stride)
    muscl_cell<DIM, R, T, G, CM>(a, direct ? (int)item : a.lists[(long)a.N + item], L);
  const int total3 = direct ? 0 : a.counts[3];
  for (long item = L.item; item < total3; item += stride) first_order_cell<DIM, T, G>(a, a.lists[2L * a.N + item], L);
}

// K6: the two sides of face f at its i-th Gauss point are slot gl + i of the
// owner and slot gr + i of the neighbour (the owner again at a boundary face:
// transmissive ghost).
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_flux(int NF, int N, const T *fs, const int *gp_off, const int *fc,
                                              const int *fgb, const T *fn, const T *gpw, T gamma, int hllc,
                                              T *Ff, int xcd) {
  constexpr int NV = DIM + 2;
  const int f = (int)(block_id(xcd) * blockDim.x + threadIdx.x);
  if (f >= NF) return;
  T n[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) n[j] = fn[(long)j * NF + f];
  const int cL = fc[f], cR0 = fc[NF + f], cR = cR0 >= 0 ? cR0 : cL;
  const int code = fgb[f];
  const T *pL = fs + (long)(code & 255) * NV * N + cL;
  const T *pR = fs + (long)((code >> 8) & 255) * NV * N + cR;
  T acc[NV] = {};
  // Gauss points two at a time: both points' states are requested before the
  // first solve (an odd count repeats its last point, which is loaded but not
  // added); the sum keeps the point order
  const int g0 = gp_off[f], ng = gp_off[f + 1] - g0;
  for (int i = 0; i < ng; i += 2) {
    const int i1 = min(i + 1, ng - 1);
    T qL[2][NV], qR[2][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qL[0][v] = pL[((long)i * NV + v) * N];
      qR[0][v] = pR[((long)i * NV + v) * N];
      qL[1][v] = pL[((long)i1 * NV + v) * N];
      qR[1][v] = pR[((long)i1 * NV + v) * N];
    }
    const T w0 = gpw[g0 + i], w1 = gpw[g0 + i1];
    T F[NV];
    riemann<DIM, T>(qL[0], qR[0], n, gamma, hllc, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += w0 * F[v];
    if (i + 1 < ng) {
      riemann<DIM, T>(qL[1], qR[1], n, gamma, hllc, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += w1 * F[v];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Ff[(long)v * NF + f] = acc[v];
}

template <int NV, typename T>
__global__ __launch_bounds__(256) void k_gather(int N, int NF, const int *cf_off, const int *cf, const T *Ff,
                                                const T *ivol, T *R, int xcd) {
  const int c = (int)(block_id(xcd) * blockDim.x + threadIdx.x);
  if (c >= N) return;
  // every face of the cell (3 to nf_max, checked at create) requested at once:
  // the codes, then the fluxes; entries past the count repeat the last face
  // and are not added, and the sum keeps the face order
  constexpr int FB = nf_max(NV - 2);
  const int e0 = cf_off[c], ne = cf_off[c + 1] - e0;
  int code[FB];
#pragma unroll
  for (int b = 0; b < FB; ++b) code[b] = cf[e0 + min(b, ne - 1)];
  T fv[FB][NV];
#pragma unroll
  for (int b = 0; b < FB; ++b)
#pragma unroll
    for (int v = 0; v < NV; ++v) fv[b][v] = Ff[(long)v * NF + (code[b] & 0x7fffffff)];
  T acc[NV] = {};
#pragma unroll
  for (int b = 0; b < FB; ++b)
    if (b < ne) {
      const T sg = (code[b] < 0) ? (T)1 : (T)-1;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += sg * fv[b][v];
    }
  const T iv = ivol[c];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[(long)v * N + c] = acc[v] * iv;
}

// K6+K7 fused, owner computes: each cell integrates the Riemann flux over its
// faces' Gauss points and sums them with its orientation signs.  An interior
// face's flux is evaluated by both of its cells from the same operands in the
// same order (left state, right state, the face's own normal), so the two
// values are bitwise equal and the residual conserves exactly; the sums match
// k_flux followed by k_gather bit for bit.
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_residual(int N, int NF, const T *fs, const int *cf_off, const int *cf,
                                                  const int *fc, const int *fgb, const int *gp_off, const T *fn,
                                                  const T *gpw, const T *ivol, T gamma, int hllc, T *R,
                                                  int xcd) {
  constexpr int NV = DIM + 2;
  const int c = (int)(block_id(xcd) * blockDim.x + threadIdx.x);
  if (c >= N) return;
  T acc[NV] = {};
  for (int e = cf_off[c]; e < cf_off[c + 1]; ++e) {
    const int code = cf[e];
    const int f = code & 0x7fffffff;
    const T sg = (code < 0) ? (T)1 : (T)-1;
    const int cL = fc[f], cR0 = fc[NF + f], cR = cR0 >= 0 ? cR0 : cL;
    const int t = fgb[f];
    const T *pL = fs + (long)(t & 255) * NV * N + cL;
    const T *pR = fs + (long)((t >> 8) & 255) * NV * N + cR;
    T n[DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j) n[j] = fn[(long)j * NF + f];
    T af[NV] = {};
    for (int g = gp_off[f], i = 0; g < gp_off[f + 1]; ++g, ++i) {
      T qL[NV], qR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qL[v] = pL[((long)i * NV + v) * N];
        qR[v] = pR[((long)i * NV + v) * N];
      }
      T F[NV];
      riemann<DIM, T>(qL, qR, n, gamma, hllc, F);
      const T w = gpw[g];
#pragma unroll
      for (int v = 0; v < NV; ++v) af[v] += w * F[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += sg * af[v];
  }
  const T iv = ivol[c];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[(long)v * N + c] = acc[v] * iv;
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
static HotArgs<T> make_args(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, uint8_t *cls) {
  HotArgs<T> a;
  a.N = ctx->N;
  a.NF = ctx->NF;
  a.mode = ctx->p.mode;
  a.form = ctx->p.form;
  a.frozen = 0;
  a.cls_in = nullptr;
  a.U = (const T *)U;
  a.fs = (T *)fs;
  // the linear pass keeps every cell's central fit for CWENOZ (reuse), and
  // always with viscous fluxes, whose gradients come from the kept fits
  const bool keep = ctx->p.viscous ? (ctx->p.mode == HFV_HYBRID || ctx->p.mode == HFV_ALL_LINEAR)
                                   : (ctx->cw_reuse && ctx->p.mode == HFV_HYBRID);
  a.coef = keep ? (T *)ctx->coef : nullptr;
  a.xcd = ctx->xcd_remap;
  a.limiter = ctx->p.limiter;
  a.own = ctx->own;
  a.cls = cls;
  a.lists = ctx->lists;
  a.counts = ctx->counts;
  a.t = t;
  a.gamma = (T)ctx->p.gamma;
  a.alpha_m = (T)ctx->p.alpha_m;
  a.beta_m = (T)ctx->p.beta_m;
  a.alpha_w = (T)ctx->p.alpha_w;
  a.beta_w = (T)ctx->p.beta_w;
  a.lam1p = (T)ctx->p.lam1p;
  a.eps_w = (T)ctx->p.eps_w;
  a.b_w = (T)ctx->p.b_w;
  a.theta = (T)ctx->p.theta;
  a.tvd_eps = (T)ctx->p.tvd_eps;
  const double bw = ctx->p.b_w;
  a.ib_w = (bw >= 1.0 && bw <= 8.0 && bw == (double)(int)bw) ? (int)bw : 0;
  a.margin = nullptr;
  a.NGPC = ctx->NGPC;
  return a;
}

static __global__ void k_zero_counts(int *c) {
  if (threadIdx.x < 8) c[threadIdx.x] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *x, int n, T v) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) x[i] = v;
}

// The linear + NAD kernel in the configured mapping: variables (split 0),
// stencil members (1) or unknowns (2) per lane, lin_lanes lanes per cell.
template <int DIM, typename T>
static void launch_classify(const hfv_ctx *ctx, const HotArgs<T> &a, hipStream_t s) {
  k_classify<T, nf_max(DIM)><<<nblk(ctx->N, CLASSIFY_BLOCK), CLASSIFY_BLOCK, 0, s>>>(a);
}

template <int DIM, int R, typename T, bool MG>
static void launch_linear_mg(const hfv_ctx *ctx, const HotArgs<T> &a, hipStream_t s) {
  const int B = ctx->block, GL = ctx->lin_lanes;
  const long waves = ((long)ctx->N + 64 / GL - 1) / (64 / GL);
  const unsigned grid = nblk(waves * 64, B);
  switch (ctx->lin_split * 16 + GL) {
    case 1: k_linear<DIM, R, T, 1, MG><<<grid, B, 0, s>>>(a); break;
    case 2:
      if constexpr (DIM == 2) k_linear<DIM, R, T, 2, MG><<<grid, B, 0, s>>>(a);
      break;
    case DIM + 2: k_linear<DIM, R, T, DIM + 2, MG><<<grid, B, 0, s>>>(a); break;
    case 16 + 2: k_linear_ms<DIM, R, T, 2, MG><<<grid, B, 0, s>>>(a); break;
    case 16 + 4: k_linear_ms<DIM, R, T, 4, MG><<<grid, B, 0, s>>>(a); break;
    case 16 + 8: k_linear_ms<DIM, R, T, 8, MG><<<grid, B, 0, s>>>(a); break;
    case 32 + 2: k_linear_ks<DIM, R, T, 2, MG><<<grid, B, 0, s>>>(a); break;
    case 32 + 4: k_linear_ks<DIM, R, T, 4, MG><<<grid, B, 0, s>>>(a); break;
    case 32 + 8: k_linear_ks<DIM, R, T, 8, MG><<<grid, B, 0, s>>>(a); break;
  }
}
template <int DIM, int R, typename T>
static void launch_linear(const hfv_ctx *ctx, const HotArgs<T> &a, hipStream_t s) {
  if (a.margin)
    launch_linear_mg<DIM, R, T, true>(ctx, a, s);
  else
    launch_linear_mg<DIM, R, T, false>(ctx, a, s);
}

// The MUSCL / first-order pass with its own lane count (muscl_lanes, or the
// class-list kernels' lanes_per_cell when 0) and the grid that count needs.
template <int DIM, int R, typename T, int G>
static void launch_muscl_g(hfv_ctx *ctx, const HotArgs<T> &a, int direct, hipStream_t s) {
  const int B = ctx->block;
  const long waves = ((long)ctx->N + 64 / G - 1) / (64 / G);
  const unsigned grid_cells = nblk(waves * 64, B);
  const unsigned grid =
      ctx->list_blocks > 0 ? std::min<unsigned>(grid_cells, (unsigned)ctx->list_blocks) : grid_cells;
  if (ctx->lists_cm)
    k_muscl<DIM, R, T, G, true><<<grid, B, 0, s>>>(a, direct);
  else
    k_muscl<DIM, R, T, G, false><<<grid, B, 0, s>>>(a, direct);
}
template <int DIM, int R, typename T>
static void launch_muscl(hfv_ctx *ctx, const HotArgs<T> &a, int direct, hipStream_t s) {
  const int l = ctx->muscl_lanes ? ctx->muscl_lanes : ctx->lanes;
  if (l == 1)
    launch_muscl_g<DIM, R, T, 1>(ctx, a, direct, s);
  else if (l == DIM + 2)
    launch_muscl_g<DIM, R, T, DIM + 2>(ctx, a, direct, s);
  else if constexpr (DIM == 2)
    launch_muscl_g<DIM, R, T, 2>(ctx, a, direct, s);
}

// The CWENOZ launch in its compile-time variants: fit kept or refitted, MUSCL
// and first-order lists merged in, OI read cell-major (not with one lane per
// cell, which keeps the [entry][cell] reads).
template <int DIM, int R, typename T, int G, bool CM>
static void launch_cwenoz_cm(const hfv_ctx *ctx, const HotArgs<T> &a, unsigned grid, int direct, bool reuse,
                             bool merged, hipStream_t s) {
  const int B = ctx->block;
  if (reuse) {
    if (merged) k_cwenoz<DIM, R, T, G, true, true, CM><<<grid, B, 0, s>>>(a, direct);
    else k_cwenoz<DIM, R, T, G, true, false, CM><<<grid, B, 0, s>>>(a, direct);
  } else {
    if (merged) k_cwenoz<DIM, R, T, G, false, true, CM><<<grid, B, 0, s>>>(a, direct);
    else k_cwenoz<DIM, R, T, G, false, false, CM><<<grid, B, 0, s>>>(a, direct);
  }
}
template <int DIM, int R, typename T, int G>
static void launch_cwenoz(const hfv_ctx *ctx, const HotArgs<T> &a, unsigned grid, int direct, bool reuse,
                          bool merged, hipStream_t s) {
  if constexpr (G != 1) {
    if (ctx->lists_cm) {
      launch_cwenoz_cm<DIM, R, T, G, true>(ctx, a, grid, direct, reuse, merged, s);
      return;
    }
  }
  launch_cwenoz_cm<DIM, R, T, G, false>(ctx, a, grid, direct, reuse, merged, s);
}

template <int DIM, int R, typename T, int G>
static hfv_status recon_impl(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, uint8_t *cls, void *margin,
                             hipStream_t s) {
  HotArgs<T> a = make_args<T>(ctx, t, U, fs, cls);
  a.margin = (T *)margin;
  const int B = ctx->block;
  const long items = (long)ctx->N;
  const long waves = (items + 64 / G - 1) / (64 / G);
  const unsigned grid_cells = nblk(waves * 64, B);
  const unsigned grid_list =
      ctx->list_blocks > 0 ? std::min<unsigned>(grid_cells, (unsigned)ctx->list_blocks) : grid_cells;
  const int mode = ctx->p.mode;
  if (margin && (mode == HFV_ALL_CWENOZ || mode == HFV_ALL_MUSCL))   // no linear pass: no decision to report
    k_fill<T><<<nblk(ctx->N, 256), 256, 0, s>>>((T *)margin, ctx->N, (T)INFINITY);
  const bool chr = ctx->p.cvars == HFV_CHARACTERISTIC;
  if (ctx->p.viscous && (mode == HFV_ALL_CWENOZ || mode == HFV_ALL_MUSCL)) {
    // no linear pass to keep the central fits the viscous gradients use
    hfv_status e = run_keep_fits(ctx, U, s);
    if (e != HFV_OK) return e;
  }
  if (mode == HFV_ALL_CWENOZ) {
    k_zero_counts<<<1, 64, 0, s>>>(ctx->counts);
    ProfScope ps(ctx, HFV_SLOT_CWENOZ, s);
    if (chr) {
      a.coef = nullptr;
      hfv_status e = launch_cwenoz_char<T>(ctx, a, 1, s);
      if (e != HFV_OK) return e;
    } else {
      launch_cwenoz<DIM, R, T, G>(ctx, a, grid_list, 1, false, false, s);
    }
  } else if (mode == HFV_ALL_MUSCL) {
    k_zero_counts<<<1, 64, 0, s>>>(ctx->counts);
    { ProfScope ps(ctx, HFV_SLOT_MUSCL, s); launch_muscl<DIM, R, T>(ctx, a, 1, s); }
  } else {
    { ProfScope ps(ctx, HFV_SLOT_LINEAR, s); launch_linear<DIM, R, T>(ctx, a, s); }
    { ProfScope ps(ctx, HFV_SLOT_CLASSIFY, s); launch_classify<DIM, T>(ctx, a, s); }
    // the MUSCL and first-order lists ride in the CWENOZ launch when merged
    const int merged = mode == HFV_HYBRID && !chr && ctx->merged_lists;
    if (mode == HFV_HYBRID) {
      ProfScope ps(ctx, HFV_SLOT_CWENOZ, s);
      if (chr) {
        hfv_status e = launch_cwenoz_char<T>(ctx, a, 0, s);
        if (e != HFV_OK) return e;
      } else {
        launch_cwenoz<DIM, R, T, G>(ctx, a, grid_list, 0, a.coef != nullptr, merged, s);
      }
    }
    // MUSCL list (empty unless hybrid) and the first-order list
    if (!merged) {
      ProfScope ps(ctx, HFV_SLOT_MUSCL, s);
      launch_muscl<DIM, R, T>(ctx, a, 0, s);
    }
  }
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

// Face states for given (frozen) classes: the linear candidate everywhere,
// then CWENOZ / MUSCL / first-order states on the given class lists, with no
// NAD and no Harten re-check.
template <int DIM, int R, typename T, int G>
static hfv_status frozen_impl(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, const uint8_t *cls,
                              hipStream_t s) {
  HotArgs<T> a = make_args<T>(ctx, t, U, fs, nullptr);
  a.frozen = 1;
  a.cls_in = cls;
  a.mode = HFV_ALL_LINEAR;
  a.coef = nullptr;
  const int B = ctx->block;
  const long waves = ((long)ctx->N + 64 / G - 1) / (64 / G);
  const unsigned grid_cells = nblk(waves * 64, B);
  const unsigned grid_list =
      ctx->list_blocks > 0 ? std::min<unsigned>(grid_cells, (unsigned)ctx->list_blocks) : grid_cells;
  launch_linear<DIM, R, T>(ctx, a, s);
  launch_classify<DIM, T>(ctx, a, s);
  if (ctx->p.cvars == HFV_CHARACTERISTIC) {
    hfv_status e = launch_cwenoz_char<T>(ctx, a, 0, s);
    if (e != HFV_OK) return e;
    launch_muscl<DIM, R, T>(ctx, a, 0, s);
  } else if (ctx->merged_lists) {
    launch_cwenoz<DIM, R, T, G>(ctx, a, grid_list, 0, false, true, s);
  } else {
    launch_cwenoz<DIM, R, T, G>(ctx, a, grid_list, 0, false, false, s);
    launch_muscl<DIM, R, T>(ctx, a, 0, s);
  }
  HFV_HIP(hipGetLastError());
  if (ctx->p.viscous) return run_keep_fits(ctx, U, s);   // the viscous gradients' fits
  return HFV_OK;
}

// Per (dim, order) entry points of the forward kernels.  The translation unit
// is compiled once per group of orders (HFV_HOT_PART 1..8, each instantiating
// its orders' kernels) and once for the dispatch below (HFV_HOT_PART 0), so
// the build runs in parallel; without HFV_HOT_PART it holds everything.
template <int DIM, int R, typename T>
hfv_status frozen_dr(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, const uint8_t *cls, hipStream_t s) {
  return frozen_impl<DIM, R, T, DIM + 2>(ctx, t, U, fs, cls, s);
}

template <int DIM, int R, typename T>
hfv_status recon_dr(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, uint8_t *cls, void *mg, hipStream_t s) {
  switch (ctx->lanes) {
    case 1: return recon_impl<DIM, R, T, 1>(ctx, t, U, fs, cls, mg, s);
    case DIM + 2: return recon_impl<DIM, R, T, DIM + 2>(ctx, t, U, fs, cls, mg, s);
    default:
      if constexpr (DIM == 2) {
        if (ctx->lanes == 2) return recon_impl<DIM, R, T, 2>(ctx, t, U, fs, cls, mg, s);
      }
      ctx->err = "unsupported lanes per cell";
      return HFV_ERR_PARAM;
  }
}

#ifndef HFV_HOT_PART
#define HFV_HOT_PART -1
#endif
// X: "extern" to declare the instantiations made in another part, or empty
#define HFV_ORDER(X, D, R)                                                                                          \
  X template hfv_status recon_dr<D, R, double>(hfv_ctx *, Tables<double> &, const void *, void *, uint8_t *,     \
                                               void *, hipStream_t);                                                \
  X template hfv_status recon_dr<D, R, float>(hfv_ctx *, Tables<float> &, const void *, void *, uint8_t *, void *, \
                                              hipStream_t);                                                         \
  X template hfv_status frozen_dr<D, R, double>(hfv_ctx *, Tables<double> &, const void *, void *,                 \
                                                const uint8_t *, hipStream_t);                                      \
  X template hfv_status frozen_dr<D, R, float>(hfv_ctx *, Tables<float> &, const void *, void *, const uint8_t *,  \
                                               hipStream_t);
#define HFV_NOTHING
#if HFV_HOT_PART == 0
#define HFV_PART_ORDER(P, D, R) HFV_ORDER(extern, D, R)
#else
#define HFV_PART_ORDER(P, D, R) HFV_PART_ORDER_##P(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 1
#define HFV_PART_ORDER_1(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_1(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 2
#define HFV_PART_ORDER_2(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_2(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 3
#define HFV_PART_ORDER_3(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_3(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 4
#define HFV_PART_ORDER_4(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_4(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 5
#define HFV_PART_ORDER_5(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_5(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 6
#define HFV_PART_ORDER_6(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_6(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 7
#define HFV_PART_ORDER_7(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_7(D, R)
#endif
#if HFV_HOT_PART == -1 || HFV_HOT_PART == 8
#define HFV_PART_ORDER_8(D, R) HFV_ORDER(HFV_NOTHING, D, R)
#else
#define HFV_PART_ORDER_8(D, R)
#endif
HFV_PART_ORDER(1, 2, 1)
HFV_PART_ORDER(1, 2, 2)
HFV_PART_ORDER(2, 2, 3)
HFV_PART_ORDER(3, 2, 4)
HFV_PART_ORDER(4, 2, 5)
HFV_PART_ORDER(5, 2, 6)
HFV_PART_ORDER(6, 3, 1)
HFV_PART_ORDER(6, 3, 2)
HFV_PART_ORDER(7, 3, 3)
HFV_PART_ORDER(8, 3, 4)

#if HFV_HOT_PART <= 0
template <typename T>
static hfv_status frozen_t(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, const uint8_t *cls, hipStream_t s) {
  switch (ctx->dim * 10 + ctx->r) {
    case 21: return frozen_dr<2, 1, T>(ctx, t, U, fs, cls, s);
    case 22: return frozen_dr<2, 2, T>(ctx, t, U, fs, cls, s);
    case 23: return frozen_dr<2, 3, T>(ctx, t, U, fs, cls, s);
    case 24: return frozen_dr<2, 4, T>(ctx, t, U, fs, cls, s);
    case 25: return frozen_dr<2, 5, T>(ctx, t, U, fs, cls, s);
    case 26: return frozen_dr<2, 6, T>(ctx, t, U, fs, cls, s);
    case 31: return frozen_dr<3, 1, T>(ctx, t, U, fs, cls, s);
    case 32: return frozen_dr<3, 2, T>(ctx, t, U, fs, cls, s);
    case 33: return frozen_dr<3, 3, T>(ctx, t, U, fs, cls, s);
    case 34: return frozen_dr<3, 4, T>(ctx, t, U, fs, cls, s);
  }
  ctx->err = "unsupported (dim, order_r)";
  return HFV_ERR_PARAM;
}

// Class lists of given classes alone (no face states): the lengths are
// cleared by a fill kernel, then the compaction runs in frozen mode.

template <typename T>
static hfv_status lists_t(hfv_ctx *ctx, Tables<T> &t, const uint8_t *cls, hipStream_t s) {
  HotArgs<T> a = make_args<T>(ctx, t, nullptr, nullptr, nullptr);
  a.frozen = 1;
  a.cls_in = cls;
  k_zero_counts<<<1, 64, 0, s>>>(ctx->counts);
  if (ctx->dim == 2)
    launch_classify<2, T>(ctx, a, s);
  else
    launch_classify<3, T>(ctx, a, s);
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

hfv_status run_class_lists(hfv_ctx *ctx, const uint8_t *cls, hipStream_t s) {
  return ctx->prec == 64 ? lists_t<double>(ctx, ctx->t64, cls, s) : lists_t<float>(ctx, ctx->t32, cls, s);
}

hfv_status run_reconstruct_frozen(hfv_ctx *ctx, const void *U, void *fs, const uint8_t *cls, hipStream_t s) {
  return ctx->prec == 64 ? frozen_t<double>(ctx, ctx->t64, U, fs, cls, s)
                         : frozen_t<float>(ctx, ctx->t32, U, fs, cls, s);
}

template <typename T>
static hfv_status recon_t(hfv_ctx *ctx, Tables<T> &t, const void *U, void *fs, uint8_t *cls, void *mg,
                          hipStream_t s) {
  switch (ctx->dim * 10 + ctx->r) {
    case 21: return recon_dr<2, 1, T>(ctx, t, U, fs, cls, mg, s);
    case 22: return recon_dr<2, 2, T>(ctx, t, U, fs, cls, mg, s);
    case 23: return recon_dr<2, 3, T>(ctx, t, U, fs, cls, mg, s);
    case 24: return recon_dr<2, 4, T>(ctx, t, U, fs, cls, mg, s);
    case 25: return recon_dr<2, 5, T>(ctx, t, U, fs, cls, mg, s);
    case 26: return recon_dr<2, 6, T>(ctx, t, U, fs, cls, mg, s);
    case 31: return recon_dr<3, 1, T>(ctx, t, U, fs, cls, mg, s);
    case 32: return recon_dr<3, 2, T>(ctx, t, U, fs, cls, mg, s);
    case 33: return recon_dr<3, 3, T>(ctx, t, U, fs, cls, mg, s);
    case 34: return recon_dr<3, 4, T>(ctx, t, U, fs, cls, mg, s);
  }
  ctx->err = "unsupported (dim, order_r)";
  return HFV_ERR_PARAM;
}

hfv_status run_reconstruct(hfv_ctx *ctx, const void *U, void *fs, uint8_t *cls, hipStream_t s, void *margin) {
  return ctx->prec == 64 ? recon_t<double>(ctx, ctx->t64, U, fs, cls, margin, s)
                         : recon_t<float>(ctx, ctx->t32, U, fs, cls, margin, s);
}

template <typename T>
static hfv_status tail_t(hfv_ctx *ctx, Tables<T> &t, const void *fs, void *R, hipStream_t s) {
  const int hllc = ctx->p.riemann == HFV_HLLC;
  T *Ff = (T *)ctx->fflux;
  const unsigned gf = nblk(ctx->NF, 256), gc = nblk(ctx->N, 256);
  if (ctx->fused_residual && !ctx->p.viscous) {
    ProfScope ps(ctx, HFV_SLOT_FLUX, s);
    if (ctx->dim == 2)
      k_residual<2, T><<<gc, 256, 0, s>>>(ctx->N, ctx->NF, (const T *)fs, t.cf_off, t.cf, t.face_cells, t.fgb,
                                          t.gp_off, t.fnormal, t.gpw, t.ivol, (T)ctx->p.gamma, hllc, (T *)R, ctx->xcd_remap);
    else
      k_residual<3, T><<<gc, 256, 0, s>>>(ctx->N, ctx->NF, (const T *)fs, t.cf_off, t.cf, t.face_cells, t.fgb,
                                          t.gp_off, t.fnormal, t.gpw, t.ivol, (T)ctx->p.gamma, hllc, (T *)R, ctx->xcd_remap);
    HFV_HIP(hipGetLastError());
    return HFV_OK;
  }
  if (ctx->dim == 2) {
    { ProfScope ps(ctx, HFV_SLOT_FLUX, s);
      k_flux<2, T><<<gf, 256, 0, s>>>(ctx->NF, ctx->N, (const T *)fs, t.gp_off, t.face_cells, t.fgb, t.fnormal,
                                       t.gpw, (T)ctx->p.gamma, hllc, Ff, ctx->xcd_remap);
      if (ctx->p.viscous) {
        hfv_status e = run_viscous_flux(ctx, fs, Ff, s);
        if (e != HFV_OK) return e;
      } }
    { ProfScope ps(ctx, HFV_SLOT_GATHER, s);
      k_gather<4, T><<<gc, 256, 0, s>>>(ctx->N, ctx->NF, t.cf_off, t.cf, Ff, t.ivol, (T *)R, ctx->xcd_remap); }
  } else {
    { ProfScope ps(ctx, HFV_SLOT_FLUX, s);
      k_flux<3, T><<<gf, 256, 0, s>>>(ctx->NF, ctx->N, (const T *)fs, t.gp_off, t.face_cells, t.fgb, t.fnormal,
                                       t.gpw, (T)ctx->p.gamma, hllc, Ff, ctx->xcd_remap);
      if (ctx->p.viscous) {
        hfv_status e = run_viscous_flux(ctx, fs, Ff, s);
        if (e != HFV_OK) return e;
      } }
    { ProfScope ps(ctx, HFV_SLOT_GATHER, s);
      k_gather<5, T><<<gc, 256, 0, s>>>(ctx->N, ctx->NF, t.cf_off, t.cf, Ff, t.ivol, (T *)R, ctx->xcd_remap); }
  }
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

hfv_status run_residual_tail(hfv_ctx *ctx, const void *fs, void *R, hipStream_t s) {
  return ctx->prec == 64 ? tail_t<double>(ctx, ctx->t64, fs, R, s) : tail_t<float>(ctx, ctx->t32, fs, R, s);
}
#endif  // dispatch

}  // namespace hfv
