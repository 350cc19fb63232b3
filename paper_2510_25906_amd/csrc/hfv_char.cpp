// CWENOZ in characteristic variables (Section 2.3: the reconstruction may act
// on characteristic, primitive or conserved variables).
//
// Each face f of a CWENOZ cell i has its own projection: the eigenvectors of
// the Euler flux Jacobian d(F . n)/dU in the face's unit normal n (outward
// from i), at the Roe average of the averages of i and of the cell across f
// (i itself at a boundary face).  With velocity u, sound speed c, total
// enthalpy H, u_n = u . n, q2 = |u|^2, b1 = (gamma - 1) / c^2, b2 = b1 q2 / 2
// and unit tangents t_k completing n to an orthonormal basis, the fields are,
// in order, acoustic u_n - c, entropy, shear along t_1 (and t_2), acoustic
// u_n + c, with
//   left rows   ((b2 + u_n/c)/2, -(b1 u + n/c)/2, b1/2), (1 - b2, b1 u, -b1),
//               (-u . t_k, t_k, 0), ((b2 - u_n/c)/2, -(b1 u - n/c)/2, b1/2)
//   right cols  (1, u - c n, H - c u_n), (1, u, q2/2), (0, t_k, u . t_k),
//               (1, u + c n, H + c u_n).
// Tangents: t_1 = (-n_y, n_x) in 2D; in 3D t_1 = e x n / |e x n| with e the
// axis of the smallest |n_k| (the first on a tie), t_2 = n x t_1.
//
// Every candidate fit is linear in the data, so the characteristic fits of a
// face are L times the conserved fits, which are computed once per cell; the
// smoothness indicators, the nonlinear weights (FP64, as in the conserved
// kernel) and the combined polynomial are then taken per characteristic
// field, the polynomial is evaluated at the face's Gauss points and mapped
// back, U(x) = U_i + R dW(x).  One lane per cell: the projections mix every
// variable of the cell.
#include "hfv_device.hpp"

namespace hfv {

template <int DIM, typename T>
struct CharBasis {
  T n[DIM], t[DIM - 1][DIM], u[DIM], un, q2, c, H, b1, b2, ut[DIM - 1];

  __device__ CharBasis(const T (&uL)[DIM + 2], const T (&uR)[DIM + 2], const T (&nn)[DIM], T gamma) {
    constexpr int NV = DIM + 2;
    for (int j = 0; j < DIM; ++j) n[j] = nn[j];
    if constexpr (DIM == 2) {
      t[0][0] = -n[1];
      t[0][1] = n[0];
    } else {
      int k = 0;
      if (fabs(n[1]) < fabs(n[k])) k = 1;
      if (fabs(n[2]) < fabs(n[k])) k = 2;
      T e[3] = {(T)0, (T)0, (T)0};
      e[k] = (T)1;
      T a[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
      const T ia = (T)1 / sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      for (int j = 0; j < 3; ++j) t[0][j] = a[j] * ia;
      t[1][0] = n[1] * t[0][2] - n[2] * t[0][1];
      t[1][1] = n[2] * t[0][0] - n[0] * t[0][2];
      t[1][2] = n[0] * t[0][1] - n[1] * t[0][0];
    }
    // Roe average
    const T sL = sqrt(uL[0]), sR = sqrt(uR[0]), wL = sL / (sL + sR), wR = sR / (sL + sR);
    T kL = 0, kR = 0;
    for (int j = 0; j < DIM; ++j) {
      const T vL = uL[1 + j] / uL[0], vR = uR[1 + j] / uR[0];
      u[j] = wL * vL + wR * vR;
      kL += vL * vL;
      kR += vR * vR;
    }
    const T pL = (gamma - (T)1) * (uL[NV - 1] - (T)0.5 * uL[0] * kL);
    const T pR = (gamma - (T)1) * (uR[NV - 1] - (T)0.5 * uR[0] * kR);
    H = wL * (uL[NV - 1] + pL) / uL[0] + wR * (uR[NV - 1] + pR) / uR[0];
    un = 0;
    q2 = 0;
    for (int j = 0; j < DIM; ++j) {
      un += u[j] * n[j];
      q2 += u[j] * u[j];
    }
    for (int k = 0; k < DIM - 1; ++k) {
      ut[k] = 0;
      for (int j = 0; j < DIM; ++j) ut[k] += u[j] * t[k][j];
    }
    c = sqrt((gamma - (T)1) * (H - (T)0.5 * q2));
    b1 = (gamma - (T)1) / (c * c);
    b2 = (T)0.5 * b1 * q2;
  }

  // row v of L applied to x
  __device__ T left(int v, const T (&x)[DIM + 2]) const {
    constexpr int NV = DIM + 2;
    T s;
    if (v == 0 || v == NV - 1) {
      const T sg = v == 0 ? (T)1 : (T)-1;
      s = (T)0.5 * (b2 + sg * un / c) * x[0] + (T)0.5 * b1 * x[NV - 1];
      for (int j = 0; j < DIM; ++j) s -= (T)0.5 * (b1 * u[j] + sg * n[j] / c) * x[1 + j];
    } else if (v == 1) {
      s = ((T)1 - b2) * x[0] - b1 * x[NV - 1];
      for (int j = 0; j < DIM; ++j) s += b1 * u[j] * x[1 + j];
    } else {
      const int k = v - 2;
      s = -ut[k] * x[0];
      for (int j = 0; j < DIM; ++j) s += t[k][j] * x[1 + j];
    }
    return s;
  }

  // R w
  __device__ void right(const T (&w)[DIM + 2], T (&x)[DIM + 2]) const {
    constexpr int NV = DIM + 2;
    const T a = w[0], e = w[1], b = w[NV - 1];
    x[0] = a + e + b;
    for (int j = 0; j < DIM; ++j) {
      T s = a * (u[j] - c * n[j]) + e * u[j] + b * (u[j] + c * n[j]);
      for (int k = 0; k < DIM - 1; ++k) s += w[2 + k] * t[k][j];
      x[1 + j] = s;
    }
    T s = a * (H - c * un) + e * (T)0.5 * q2 + b * (H + c * un);
    for (int k = 0; k < DIM - 1; ++k) s += w[2 + k] * ut[k];
    x[NV - 1] = s;
  }
};

// largest number of Gauss points on one face
template <int DIM, int R>
constexpr int max_gp_face() {
  return DIM == 2 ? (R + 2) / 2 : (((R + 2) / 2) * ((R + 2) / 2) > 6 ? ((R + 2) / 2) * ((R + 2) / 2) : 6);
}

template <int DIM, int R, typename T, bool REUSE>
__global__ __launch_bounds__(256) void k_cwenoz_char(HotArgs<T> a, int direct) {
  constexpr int NV = DIM + 2, K = n_unknowns(DIM, R), NFM = nf_max(DIM), MD = 2 * DIM;
  constexpr int GF = max_gp_face<DIM, R>();
  const int total = direct ? a.N : a.counts[1];
  const long stride = (long)gridDim.x * blockDim.x;
  for (long item = block_id(a.xcd) * blockDim.x + threadIdx.x; item < total; item += stride) {
    const int cell = direct ? (int)item : a.lists[item];
    const int N = a.N;
    T u0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u0[v] = a.U[(long)v * N + cell];
    // conserved central fit and directional fits (Section 2.3)
    T co[K][NV];
    if constexpr (REUSE) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) co[k][v] = a.coef[((long)k * NV + v) * N + cell];
    } else {
      lsq_coeffs<DIM, R, NV, T>(a, cell, 0, u0, co);
    }
    const int nd = a.t.ndir[cell];
    T ad[NFM][DIM][NV];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
#pragma unroll
      for (int j = 0; j < DIM; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) ad[s][j][v] = (T)0;
      if (s < nd) {
#pragma unroll
        for (int m = 0; m < MD; ++m) {
          const int jc = a.t.dsten[((long)s * MD + m) * N + cell];
          T du[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) du[v] = a.U[(long)v * N + jc] - u0[v];
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            const T p = a.t.Pdir[(((long)s * DIM + j) * MD + m) * N + cell];
#pragma unroll
            for (int v = 0; v < NV; ++v) ad[s][j][v] += p * du[v];
          }
        }
      }
    }
    // p_1 = (p_opt - sum_s lambda_s p_s) / lambda_1, in conserved variables
    const T lam1 = (T)1 - (T)1 / a.lam1p;
    const T lams = ((T)1 - lam1) / (T)nd;
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T sdir = 0;
#pragma unroll
        for (int s = 0; s < NFM; ++s) sdir += ad[s][j][v];
        co[j][v] -= lams * sdir;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) co[k][v] /= lam1;
    T psb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) psb[k] = a.t.psibar[(long)k * N + cell];
    const T rho_b = u0[0];
    const T p_b = pressure<NV, T>(u0, a.gamma);
    const double eps = (double)a.eps_w, b = (double)a.b_w;
    const bool zform = a.form == HFV_WENOZ_POW;
    bool hok = true;
    const int e0 = a.t.cf_off[cell], e1 = a.t.cf_off[cell + 1];
    int slot = 0;
    for (int e = e0; e < e1 && hok; ++e) {
      const int code = a.t.cf[e];
      const int f = code & 0x7fffffff;
      const bool right_side = code < 0;
      const int ngf = a.t.gp_off[f + 1] - a.t.gp_off[f];
      int jn = a.t.nbr[(long)(e - e0) * N + cell];
      if (jn < 0) jn = cell;
      T un_[NV], nrm[DIM];
#pragma unroll
      for (int v = 0; v < NV; ++v) un_[v] = a.U[(long)v * N + jn];
#pragma unroll
      for (int j = 0; j < DIM; ++j) nrm[j] = right_side ? -a.t.fnormal[(long)j * a.NF + f] : a.t.fnormal[(long)j * a.NF + f];
      const CharBasis<DIM, T> cb(u0, un_, nrm, a.gamma);
      T dW[GF][NV];
#pragma unroll
      for (int g = 0; g < GF; ++g)
#pragma unroll
        for (int v = 0; v < NV; ++v) dW[g][v] = (T)0;
      // one characteristic field at a time
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T cw[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          T x[NV];
#pragma unroll
          for (int w = 0; w < NV; ++w) x[w] = co[k][w];
          cw[k] = cb.left(v, x);
        }
        T dw[NFM][DIM];
#pragma unroll
        for (int s = 0; s < NFM; ++s)
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            T x[NV];
#pragma unroll
            for (int w = 0; w < NV; ++w) x[w] = ad[s][j][w];
            dw[s][j] = cb.left(v, x);
          }
        double si1 = 0, sis[NFM];
#pragma unroll
        for (int s = 0; s < NFM; ++s) sis[s] = 0;
        int pidx = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double row = 0;
#pragma unroll
          for (int kq = k; kq < K; ++kq, ++pidx) {
            const double o = (double)a.t.OI[(long)pidx * N + cell];
            row += (kq == k ? o : 2.0 * o) * (double)cw[kq];
            if (kq < DIM) {
#pragma unroll
              for (int s = 0; s < NFM; ++s)
                sis[s] += (kq == k ? o : 2.0 * o) * (double)dw[s][k] * (double)dw[s][kq];
            }
          }
          si1 += (double)cw[k] * row;
        }
        double tau = 0;
#pragma unroll
        for (int s = 0; s < NFM; ++s)
          if (s < nd) tau += fabs(sis[s] - si1);
        tau /= (double)nd;
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
          double c = w1 * it * (double)cw[k];
          if (k < DIM) {
#pragma unroll
            for (int s = 0; s < NFM; ++s) c += ws[s] * it * (double)dw[s][k];
          }
          cw[k] = (T)c;
        }
        // this field at the face's Gauss points
#pragma unroll
        for (int g = 0; g < GF; ++g) {
          if (g < ngf) {
            T xi[DIM];
#pragma unroll
            for (int j = 0; j < DIM; ++j) xi[j] = a.t.gpxi[((long)(slot + g) * DIM + j) * N + cell];
            T phi[K];
            basis_at<DIM, R, T>(xi, psb, phi);
            T sum = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) sum += cw[k] * phi[k];
            dW[g][v] = sum;
          }
        }
      }
      // back to conserved variables, Harten check, store
#pragma unroll
      for (int g = 0; g < GF; ++g) {
        if (g < ngf) {
          T d[NV], val[NV];
          cb.right(dW[g], d);
#pragma unroll
          for (int v = 0; v < NV; ++v) val[v] = u0[v] + d[v];
          hok = a.frozen || (hok && harten_point<NV, T>(val, rho_b, p_b, a));
#pragma unroll
          for (int v = 0; v < NV; ++v) store<NV, T>(a, slot + g, cell, v, val[v]);
        }
      }
      slot += ngf;
    }
    if (!hok) {  // first-order fallback: every point of the cell takes U_i
      const int ng = a.t.ngp[cell];
      for (int g = 0; g < ng; ++g)
#pragma unroll
        for (int v = 0; v < NV; ++v) store<NV, T>(a, g, cell, v, u0[v]);
    }
    if (!a.frozen) a.cls[cell] = hok ? HFV_CLASS_CWENOZ : HFV_CLASS_FIRST_ORDER;
  }
}

template <int DIM, int R, typename T>
static void launch_dr(const hfv_ctx *ctx, const HotArgs<T> &a, int direct, hipStream_t s) {
  const int B = ctx->block;
  const unsigned grid_cells = (unsigned)((ctx->N + B - 1) / B);
  const unsigned grid =
      ctx->list_blocks > 0 ? std::min<unsigned>(grid_cells, (unsigned)ctx->list_blocks) : grid_cells;
  if (a.coef)
    k_cwenoz_char<DIM, R, T, true><<<grid, B, 0, s>>>(a, direct);
  else
    k_cwenoz_char<DIM, R, T, false><<<grid, B, 0, s>>>(a, direct);
}

template <typename T>
hfv_status launch_cwenoz_char(hfv_ctx *ctx, const HotArgs<T> &a, int direct, hipStream_t s) {
  switch (ctx->dim * 10 + ctx->r) {
    case 21: launch_dr<2, 1, T>(ctx, a, direct, s); break;
    case 22: launch_dr<2, 2, T>(ctx, a, direct, s); break;
    case 23: launch_dr<2, 3, T>(ctx, a, direct, s); break;
    case 24: launch_dr<2, 4, T>(ctx, a, direct, s); break;
    case 25: launch_dr<2, 5, T>(ctx, a, direct, s); break;
    case 26: launch_dr<2, 6, T>(ctx, a, direct, s); break;
    case 31: launch_dr<3, 1, T>(ctx, a, direct, s); break;
    case 32: launch_dr<3, 2, T>(ctx, a, direct, s); break;
    case 33: launch_dr<3, 3, T>(ctx, a, direct, s); break;
    case 34: launch_dr<3, 4, T>(ctx, a, direct, s); break;
    default: ctx->err = "unsupported (dim, order_r)"; return HFV_ERR_PARAM;
  }
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

template hfv_status launch_cwenoz_char<double>(hfv_ctx *, const HotArgs<double> &, int, hipStream_t);
template hfv_status launch_cwenoz_char<float>(hfv_ctx *, const HotArgs<float> &, int, hipStream_t);

}  // namespace hfv
