// One-time precomputation of the reconstruction tables, in FP64 on the GPU.
//
// The paper computes the least-squares pseudo-inverses once at the start of
// a simulation, by Householder QR (Section 2.1, after Eq. dofMatrix), and
// precomputes the oscillation-indicator matrices (Section 2.3, definition of
// OI).  This file does the same on the device:
//   k_cell_geom   volumes, centroids, h_c from a simplex tiling of each element
//                 (non-simplex elements are tiled for reconstruction, Section 2.1)
//   k_face_geom   face normals, Gauss points and weights (Section 2, Gauss-
//                 Legendre on edges / quads, symmetric rules on triangles)
//   k_moments     monomial moments of every cell in its own frame
//                 xi = (x - x_c)/h_c, basis means psi_bar
//   k_oi          OI_kq = sum_{1<=|beta|<=r} int D^beta phi_k D^beta phi_q
//   k_lsq_rows    A_mk = int_{V_m'} phi_k  (Eq. dofMatrix), |V_m'|
//   k_qr_pinv     Householder QR of A, pseudo-inverse, |V_m'| folded in
//   k_small_pinv  degree-1 directional (Section 2.3) and MUSCL fits (Section 2.2)
//   k_cell_gp     Gauss points of each cell in its own frame
// Quadrature inside cells uses collapsed Gauss-Legendre rules on the
// simplices of the tiling, exact for the polynomial degrees involved.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hfv_internal.hpp"

namespace hfv {

// ---------------------------------------------------------------------------
// Quadrature rules, generated on the host.
struct Rules {
  double glx[8][8];  // Gauss-Legendre on [0,1], n = 1..7 (row n)
  double glw[8][8];
  double tri_bc[6][3];  // symmetric triangle rule (barycentric), per face point
  double tri_w[6];
  int tri_n;
  int n_line;
};

// Gauss-Legendre nodes and weights on [0,1] by Newton iteration on the
// three-term Legendre recurrence; ascending nodes.
static void gauss_legendre01(int n, double *x, double *w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = n == 1 ? z : p1;
      double pm = n == 1 ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
    dp = n * (z * pn - pm) / (z * z - 1.0);
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) halved for [0,1]
  }
}

// Symmetric triangle rule of degree >= r: one orbit (a,a,1-2a), a = 1/6, for
// r <= 2; for r <= 4 two orbits whose positions and weights solve the
// moment equations of the symmetric invariants 1, e2, e3, e2^2 of the
// barycentric coordinates (Newton iteration).
static bool triangle_rule(int r, Rules &R) {
  double orb[2][2];
  int no;
  if (r <= 2) {
    orb[0][0] = 1.0 / 6.0;
    orb[0][1] = 1.0 / 3.0;
    no = 1;
  } else if (r <= 4) {
    // unknowns a1, a2, W1, W2 with W = 3 w (orbit weights)
    double z[4] = {0.44, 0.09, 0.66, 0.34};
    const double rhs[4] = {1.0, 0.25, 1.0 / 60.0, 1.0 / 15.0};
    auto F = [&](const double *q, double *f) {
      double e2a = 2 * q[0] - 3 * q[0] * q[0], e2b = 2 * q[1] - 3 * q[1] * q[1];
      double e3a = q[0] * q[0] * (1 - 2 * q[0]), e3b = q[1] * q[1] * (1 - 2 * q[1]);
      f[0] = q[2] + q[3] - rhs[0];
      f[1] = q[2] * e2a + q[3] * e2b - rhs[1];
      f[2] = q[2] * e3a + q[3] * e3b - rhs[2];
      f[3] = q[2] * e2a * e2a + q[3] * e2b * e2b - rhs[3];
    };
    for (int it = 0; it < 100; ++it) {
      double f[4], J[4][4];
      F(z, f);
      double nrm = 0;
      for (double v : f) nrm += v * v;
      if (nrm < 1e-34) break;
      for (int c = 0; c < 4; ++c) {
        double zz[4];
        std::memcpy(zz, z, sizeof zz);
        double hh = 1e-7 * std::max(1.0, std::fabs(z[c]));
        zz[c] += hh;
        double fp[4];
        F(zz, fp);
        zz[c] -= 2 * hh;
        double fm[4];
        F(zz, fm);
        for (int rr = 0; rr < 4; ++rr) J[rr][c] = (fp[rr] - fm[rr]) / (2 * hh);
      }
      // solve J dz = -f by Gaussian elimination with partial pivoting
      double Aug[4][5];
      for (int rr = 0; rr < 4; ++rr) {
        for (int c = 0; c < 4; ++c) Aug[rr][c] = J[rr][c];
        Aug[rr][4] = -f[rr];
      }
      for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int rr = c + 1; rr < 4; ++rr)
          if (std::fabs(Aug[rr][c]) > std::fabs(Aug[piv][c])) piv = rr;
        for (int k = 0; k < 5; ++k) std::swap(Aug[c][k], Aug[piv][k]);
        for (int rr = c + 1; rr < 4; ++rr) {
          double m = Aug[rr][c] / Aug[c][c];
          for (int k = c; k < 5; ++k) Aug[rr][k] -= m * Aug[c][k];
        }
      }
      double dz[4];
      for (int c = 3; c >= 0; --c) {
        double s = Aug[c][4];
        for (int k = c + 1; k < 4; ++k) s -= Aug[c][k] * dz[k];
        dz[c] = s / Aug[c][c];
      }
      for (int c = 0; c < 4; ++c) z[c] += dz[c];
    }
    if (!(z[1] > 0 && z[1] < z[0] && z[0] < 0.5 && z[2] > 0 && z[3] > 0)) return false;
    orb[0][0] = z[0];
    orb[0][1] = z[2] / 3.0;
    orb[1][0] = z[1];
    orb[1][1] = z[3] / 3.0;
    no = 2;
  } else {
    return false;
  }
  int q = 0;
  for (int o = 0; o < no; ++o) {
    double a = orb[o][0];
    double pts[3][3] = {{1 - 2 * a, a, a}, {a, 1 - 2 * a, a}, {a, a, 1 - 2 * a}};
    for (int k = 0; k < 3; ++k, ++q) {
      for (int l = 0; l < 3; ++l) R.tri_bc[q][l] = pts[k][l];
      R.tri_w[q] = orb[o][1];
    }
  }
  R.tri_n = q;
  return true;
}

// Simplex tilings of the element types (local vertex indices).
__constant__ int c_ntile[6] = {1, 2, 1, 2, 3, 6};
__constant__ int c_tile[6][6][4] = {
    {{0, 1, 2, 0}},
    {{0, 1, 2, 0}, {0, 2, 3, 0}},
    {{0, 1, 2, 3}},
    {{0, 1, 2, 4}, {0, 2, 3, 4}},
    {{0, 1, 2, 3}, {1, 2, 3, 4}, {2, 3, 4, 5}},
    {{0, 1, 2, 6}, {0, 3, 2, 6}, {0, 3, 7, 6}, {0, 4, 7, 6}, {0, 4, 5, 6}, {0, 1, 5, 6}}};

template <int DIM>
__device__ inline double simplex_det(const double (&X)[DIM + 1][DIM]) {
  if constexpr (DIM == 2) {
    return (X[1][0] - X[0][0]) * (X[2][1] - X[0][1]) - (X[1][1] - X[0][1]) * (X[2][0] - X[0][0]);
  } else {
    double a[3], b[3], c[3];
    for (int j = 0; j < 3; ++j) {
      a[j] = X[1][j] - X[0][j];
      b[j] = X[2][j] - X[0][j];
      c[j] = X[3][j] - X[0][j];
    }
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
  }
}

template <int DIM>
__device__ inline void load_simplex(const double *vtx, const int *cv, int off, int t, int s, const double *shift,
                                    double (&X)[DIM + 1][DIM]) {
  for (int l = 0; l <= DIM; ++l) {
    int v = cv[off + c_tile[t][s][l]];
    for (int j = 0; j < DIM; ++j) X[l][j] = vtx[v * DIM + j] + shift[j];
  }
}

// geom = [DIM][N] centroid, [N] volume, [N] h_c
template <int DIM>
__global__ void k_cell_geom(int N, const double *vtx, const int8_t *type, const int *cvo, const int *cv,
                            double *geom) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  int t = type[c], off = cvo[c];
  double vol = 0.0, cen[DIM] = {};
  const double zero[3] = {0, 0, 0};
  for (int s = 0; s < c_ntile[t]; ++s) {
    double X[DIM + 1][DIM];
    load_simplex<DIM>(vtx, cv, off, t, s, zero, X);
    double v = fabs(simplex_det<DIM>(X)) / (DIM == 2 ? 2.0 : 6.0);
    vol += v;
    for (int j = 0; j < DIM; ++j) {
      double m = 0;
      for (int l = 0; l <= DIM; ++l) m += X[l][j];
      cen[j] += v * m / (DIM + 1);
    }
  }
  for (int j = 0; j < DIM; ++j) geom[j * N + c] = cen[j] / vol;
  geom[DIM * N + c] = vol;
  geom[(DIM + 1) * N + c] = pow(vol, 1.0 / DIM);
}

// Integrate the monomials of E over the simplex tiling of cell `cell` (image
// shifted by `shift`), in the frame (x - xc)/h; acc[k] += int xi^E_k dxi.
template <int DIM, int NQ, int LO, int HI>
__device__ inline void integrate_cell(const double *vtx, const int8_t *type, const int *cvo, const int *cv,
                                      int cell, const double *shift, const double *xc, double h,
                                      const Rules &RU, double *acc, double &vsum) {
  constexpr Exps<DIM, LO, HI> E{};
  constexpr int NE = Exps<DIM, LO, HI>::count();
  int t = type[cell], off = cvo[cell];
  const double ih = 1.0 / h;
  const double ihd = DIM == 2 ? ih * ih : ih * ih * ih;
  for (int s = 0; s < c_ntile[t]; ++s) {
    double X[DIM + 1][DIM];
    load_simplex<DIM>(vtx, cv, off, t, s, shift, X);
    double dj = fabs(simplex_det<DIM>(X)) * ihd;
    vsum += dj / (DIM == 2 ? 2.0 : 6.0);
    // collapsed Gauss rule on the unit simplex
    for (int a = 0; a < NQ; ++a)
      for (int b = 0; b < NQ; ++b)
        for (int c3 = 0; c3 < (DIM == 3 ? NQ : 1); ++c3) {
          double sa = RU.glx[NQ][a], tb = RU.glx[NQ][b];
          double w = RU.glw[NQ][a] * RU.glw[NQ][b];
          double bc[DIM + 1];
          if constexpr (DIM == 2) {
            w *= (1 - sa);
            bc[1] = sa;
            bc[2] = tb * (1 - sa);
            bc[0] = 1 - bc[1] - bc[2];
          } else {
            double uc = RU.glx[NQ][c3];
            w *= RU.glw[NQ][c3] * (1 - sa) * (1 - sa) * (1 - tb);
            bc[1] = sa;
            bc[2] = tb * (1 - sa);
            bc[3] = uc * (1 - sa) * (1 - tb);
            bc[0] = 1 - bc[1] - bc[2] - bc[3];
          }
          double xi[DIM];
          for (int j = 0; j < DIM; ++j) {
            double x = 0;
            for (int l = 0; l <= DIM; ++l) x += bc[l] * X[l][j];
            xi[j] = (x - xc[j]) * ih;
          }
          double pw[DIM][HI + 1];
          for (int j = 0; j < DIM; ++j) {
            pw[j][0] = 1.0;
#pragma unroll
            for (int p = 1; p <= HI; ++p) pw[j][p] = pw[j][p - 1] * xi[j];
          }
          const double wq = w * dj;
#pragma unroll
          for (int k = 0; k < NE; ++k) {
            double m = wq;
#pragma unroll
            for (int j = 0; j < DIM; ++j) m *= pw[j][E.e[k][j]];
            acc[k] += m;
          }
        }
  }
}

template <int DIM, int R>
struct MomCfg {
  static constexpr int DEG = (R > 2 * R - 2) ? R : 2 * R - 2;
  static constexpr int NM = binom(DEG + DIM, DIM);
  static constexpr int NQ = (DEG + DIM + 1) / 2;
};

template <int DIM, int R>
__global__ void k_moments(int N, const double *vtx, const int8_t *type, const int *cvo, const int *cv,
                          const double *geom, Rules RU, double *mom, double *psibar) {
  using C = MomCfg<DIM, R>;
  constexpr int K = n_unknowns(DIM, R);
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double xc[DIM];
  for (int j = 0; j < DIM; ++j) xc[j] = geom[j * N + c];
  double h = geom[(DIM + 1) * N + c];
  double acc[C::NM] = {};
  double vs = 0;
  const double zero[3] = {0, 0, 0};
  integrate_cell<DIM, C::NQ, 0, C::DEG>(vtx, type, cvo, cv, c, zero, xc, h, RU, acc, vs);
  for (int k = 0; k < C::NM; ++k) mom[k * N + c] = acc[k];
  // basis means: the monomials of degree 1..R follow the constant in the same order
  for (int k = 0; k < K; ++k) psibar[k * N + c] = acc[1 + k] / acc[0];
}

// OI from moments through a host-built term list: for packed pair p,
// OI_p = sum_{t in [start[p], start[p+1])} coef[t] * mom[idx[t]].
__global__ void k_oi(int N, int npair, const int *start, const double *coef, const int *idx, const double *mom,
                     double *OI) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  for (int p = 0; p < npair; ++p) {
    double s = 0;
    for (int t = start[p]; t < start[p + 1]; ++t) s += coef[t] * mom[idx[t] * N + c];
    OI[p * N + c] = s;
  }
}

// One thread per (member m, cell c): A[k][m][c] = int_{V_m'} phi_k, wv[m][c] = |V_m'|.
template <int DIM, int R>
__global__ void k_lsq_rows(int N, int M, const double *vtx, const int8_t *type, const int *cvo, const int *cv,
                           const int *central, const int8_t *cshift, const double *period, const double *geom,
                           const double *psibar, Rules RU, double *A, double *wv) {
  constexpr int K = n_unknowns(DIM, R);
  constexpr int NQ = (R + DIM + 1) / 2;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * M) return;
  int m = (int)(idx / N), c = (int)(idx % N);
  int j = central[(long)c * M + m];
  double sh[3] = {0, 0, 0};
  if (cshift)
    for (int q = 0; q < DIM; ++q) sh[q] = cshift[((long)c * M + m) * DIM + q] * period[q];
  double xc[DIM];
  for (int q = 0; q < DIM; ++q) xc[q] = geom[q * N + c];
  double h = geom[(DIM + 1) * N + c];
  double acc[K] = {};
  double vs = 0;
  integrate_cell<DIM, NQ, 1, R>(vtx, type, cvo, cv, j, sh, xc, h, RU, acc, vs);
  for (int k = 0; k < K; ++k) A[((long)k * M + m) * N + c] = acc[k] - vs * psibar[k * N + c];
  wv[(long)m * N + c] = vs;
}

// Householder QR of the M x K column-major system of each cell (stored
// [K][M][N]) and its pseudo-inverse R^{-1} Q^T, with |V_m'| folded in:
// P[k][m] = (A^+)_{km} |V_m'|.  Flags cells whose R diagonal spans more than
// 12 orders of magnitude.
__global__ void k_qr_pinv(int N, int K, int M, double *A, const double *wv, double *rdiag, double *vn2,
                          double *y, double *P, int *bad) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  auto a = [&](int row, int col) -> double & { return A[((long)col * M + row) * N + c]; };
  double dmax = 0, dmin = 1e300;
  for (int j = 0; j < K; ++j) {
    double nrm = 0;
    for (int i = j; i < M; ++i) nrm += a(i, j) * a(i, j);
    nrm = sqrt(nrm);
    double alpha = a(j, j) > 0 ? -nrm : nrm;
    a(j, j) -= alpha;
    double v2 = 0;
    for (int i = j; i < M; ++i) v2 += a(i, j) * a(i, j);
    vn2[(long)j * N + c] = v2;
    rdiag[(long)j * N + c] = alpha;
    dmax = fmax(dmax, fabs(alpha));
    dmin = fmin(dmin, fabs(alpha));
    if (v2 > 0) {
      for (int col = j + 1; col < K; ++col) {
        double s = 0;
        for (int i = j; i < M; ++i) s += a(i, j) * a(i, col);
        double f = 2.0 * s / v2;
        for (int i = j; i < M; ++i) a(i, col) -= f * a(i, j);
      }
    }
  }
  bad[c] = (dmin < 1e-12 * dmax || !(dmax > 0)) ? 1 : 0;
  for (int col = 0; col < M; ++col) {
    for (int i = 0; i < M; ++i) y[(long)i * N + c] = (i == col) ? 1.0 : 0.0;
    for (int j = 0; j < K; ++j) {
      double v2 = vn2[(long)j * N + c];
      if (!(v2 > 0)) continue;
      double s = 0;
      for (int i = j; i < M; ++i) s += a(i, j) * y[(long)i * N + c];
      double f = 2.0 * s / v2;
      for (int i = j; i < M; ++i) y[(long)i * N + c] -= f * a(i, j);
    }
    // back substitution R x = y[0:K]; x overwrites y[0:K]
    for (int k = K - 1; k >= 0; --k) {
      double s = y[(long)k * N + c];
      for (int q = k + 1; q < K; ++q) s -= a(k, q) * y[(long)q * N + c];
      y[(long)k * N + c] = s / rdiag[(long)k * N + c];
    }
    double w = wv[(long)col * N + c];
    for (int k = 0; k < K; ++k) P[((long)k * M + col) * N + c] = y[(long)k * N + c] * w;
  }
}

// Degree-1 least squares of one directional stencil (s < NFM) or of the
// MUSCL neighbours (s == NFM) of a cell.  Rows are exact integrals of the
// linear basis: int_{V_q'} phi_j = |V_q'| (xi_centroid(q)_j - psi_bar_j).
template <int DIM>
__global__ void k_small_pinv(int N, int NFM, int Md, const int *dir, const int8_t *dshift, const int *ndir,
                             const int *mus, const int8_t *mshift, const int *nmus, const double *period,
                             const double *geom, const double *psibar, double *Pdir, double *Pmus, int *bad) {
  constexpr int MAXR = 6;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * (NFM + 1)) return;
  int s = (int)(idx / N), c = (int)(idx % N);
  int cnt;
  const int *ids;
  const int8_t *shs;
  if (s < NFM) {
    cnt = s < ndir[c] ? Md : 0;
    ids = dir + ((long)c * NFM + s) * Md;
    shs = dshift ? dshift + ((long)c * NFM + s) * Md * DIM : nullptr;
  } else {
    cnt = nmus[c];
    ids = mus + (long)c * NFM;
    shs = mshift ? mshift + (long)c * NFM * DIM : nullptr;
  }
  const double h = geom[(DIM + 1) * N + c];
  const double ihd = DIM == 2 ? 1.0 / (h * h) : 1.0 / (h * h * h);
  double A[MAXR][DIM], w[MAXR];
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    w[q] = 0;
    for (int j = 0; j < DIM; ++j) A[q][j] = 0;
    if (q < cnt) {
      int m = ids[q];
      w[q] = geom[DIM * N + m] * ihd;
      for (int j = 0; j < DIM; ++j) {
        double sh = shs ? shs[q * DIM + j] * period[j] : 0.0;
        double xi = (geom[j * N + m] + sh - geom[j * N + c]) / h;
        A[q][j] = w[q] * (xi - psibar[j * N + c]);
      }
    }
  }
  // Householder QR in registers
  double vv[DIM][MAXR], v2[DIM], rd[DIM], Rm[DIM][DIM];
  double dmax = 0, dmin = 1e300;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double nrm = 0;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) nrm += (i >= j) ? A[i][j] * A[i][j] : 0.0;
    nrm = sqrt(nrm);
    double alpha = A[j][j] > 0 ? -nrm : nrm;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) vv[j][i] = (i >= j) ? A[i][j] : 0.0;
    vv[j][j] -= alpha;
    double n2 = 0;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) n2 += vv[j][i] * vv[j][i];
    v2[j] = n2;
    rd[j] = alpha;
    dmax = fmax(dmax, fabs(alpha));
    dmin = fmin(dmin, fabs(alpha));
#pragma unroll
    for (int col = j + 1; col < DIM; ++col) {
      double sdot = 0;
#pragma unroll
      for (int i = 0; i < MAXR; ++i) sdot += vv[j][i] * A[i][col];
      double f = n2 > 0 ? 2.0 * sdot / n2 : 0.0;
#pragma unroll
      for (int i = 0; i < MAXR; ++i) A[i][col] -= f * vv[j][i];
    }
#pragma unroll
    for (int col = 0; col < DIM; ++col) Rm[j][col] = A[j][col];
    Rm[j][j] = alpha;
  }
  bool rank_bad = cnt > 0 && (dmin < 1e-12 * dmax || !(dmax > 0));
  if (rank_bad) atomicOr(bad + c, 2);
#pragma unroll
  for (int col = 0; col < MAXR; ++col) {
    double yv[MAXR];
#pragma unroll
    for (int i = 0; i < MAXR; ++i) yv[i] = (i == col) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      double sdot = 0;
#pragma unroll
      for (int i = 0; i < MAXR; ++i) sdot += vv[j][i] * yv[i];
      double f = v2[j] > 0 ? 2.0 * sdot / v2[j] : 0.0;
#pragma unroll
      for (int i = 0; i < MAXR; ++i) yv[i] -= f * vv[j][i];
    }
    double x[DIM];
#pragma unroll
    for (int k = DIM - 1; k >= 0; --k) {
      double sdot = yv[k];
#pragma unroll
      for (int q = k + 1; q < DIM; ++q) sdot -= Rm[k][q] * x[q];
      x[k] = (cnt > 0 && rd[k] != 0.0) ? sdot / rd[k] : 0.0;
    }
    bool live = col < cnt && !rank_bad;
    if (s < NFM) {
      if (col < Md)
        for (int j = 0; j < DIM; ++j)
          Pdir[(((long)s * DIM + j) * Md + col) * N + c] = live ? x[j] * w[col] : 0.0;
    } else if (col < NFM) {
      for (int j = 0; j < DIM; ++j) Pmus[((long)j * NFM + col) * N + c] = live ? x[j] * w[col] : 0.0;
    }
  }
}

// Face normals (outward from the left cell), Gauss points and weights.
template <int DIM>
__global__ void k_face_geom(int NF, const double *vtx, const int *fvo, const int *fv, const int *gp_off, Rules RU,
                            double *gpx, double *gpw, double *fn, int NGPT) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= NF) return;
  int o = fvo[f], nv = fvo[f + 1] - o;
  double V[4][3] = {};
  for (int k = 0; k < nv && k < 4; ++k)
    for (int j = 0; j < DIM; ++j) V[k][j] = vtx[fv[o + k] * DIM + j];
  int g0 = gp_off[f];
  if constexpr (DIM == 2) {
    double tx = V[1][0] - V[0][0], ty = V[1][1] - V[0][1];
    double L = sqrt(tx * tx + ty * ty);
    fn[f] = ty / L;
    fn[NF + f] = -tx / L;
    int n = RU.n_line;
    for (int i = 0; i < n; ++i) {
      gpx[g0 + i] = V[0][0] + RU.glx[n][i] * tx;
      gpx[NGPT + g0 + i] = V[0][1] + RU.glx[n][i] * ty;
      gpw[g0 + i] = RU.glw[n][i] * L;
    }
  } else {
    auto cross = [](const double *a, const double *b, double *o3) {
      o3[0] = a[1] * b[2] - a[2] * b[1];
      o3[1] = a[2] * b[0] - a[0] * b[2];
      o3[2] = a[0] * b[1] - a[1] * b[0];
    };
    double av[3] = {0, 0, 0};
    if (nv == 3) {
      double e1[3], e2[3];
      for (int j = 0; j < 3; ++j) {
        e1[j] = V[1][j] - V[0][j];
        e2[j] = V[2][j] - V[0][j];
      }
      cross(e1, e2, av);
      for (int j = 0; j < 3; ++j) av[j] *= 0.5;
    } else {
      for (int k = 0; k < 4; ++k) {
        double cr[3];
        cross(V[k], V[(k + 1) % 4], cr);
        for (int j = 0; j < 3; ++j) av[j] += 0.5 * cr[j];
      }
    }
    double A = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
    for (int j = 0; j < 3; ++j) fn[j * NF + f] = av[j] / A;
    if (nv == 3) {
      for (int q = 0; q < RU.tri_n; ++q) {
        for (int j = 0; j < 3; ++j)
          gpx[j * NGPT + g0 + q] =
              RU.tri_bc[q][0] * V[0][j] + RU.tri_bc[q][1] * V[1][j] + RU.tri_bc[q][2] * V[2][j];
        gpw[g0 + q] = RU.tri_w[q] * A;
      }
    } else {
      int n = RU.n_line;
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          double s = RU.glx[n][a], t = RU.glx[n][b];
          double Nsh[4] = {(1 - s) * (1 - t), s * (1 - t), s * t, (1 - s) * t};
          double dNs[4] = {-(1 - t), (1 - t), t, -t};
          double dNt[4] = {-(1 - s), -s, s, (1 - s)};
          double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0};
          int g = g0 + a * n + b;
          for (int j = 0; j < 3; ++j) {
            double x = 0;
            for (int k = 0; k < 4; ++k) {
              x += Nsh[k] * V[k][j];
              xs[j] += dNs[k] * V[k][j];
              xt[j] += dNt[k] * V[k][j];
            }
            gpx[j * NGPT + g] = x;
          }
          double cr[3];
          cross(xs, xt, cr);
          gpw[g] = RU.glw[n][a] * RU.glw[n][b] * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        }
    }
  }
}

// Gauss points of every cell in its own frame, listed face by face in the
// cell's face order (increasing face id), quadrature index fastest.
template <int DIM>
__global__ void k_cell_gp(int N, int NGPT, int NGPC, const int *cf_off, const int *cf, const int *gp_off,
                          const double *gpx, const int8_t *fshift, const double *period, const double *geom,
                          double *gpxi, uint8_t *ngp) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double xc[DIM];
  for (int j = 0; j < DIM; ++j) xc[j] = geom[j * N + c];
  double h = geom[(DIM + 1) * N + c];
  int slot = 0;
  for (int e = cf_off[c]; e < cf_off[c + 1]; ++e) {
    int code = cf[e];
    int f = code & 0x7fffffff;
    int side = (code >> 31) & 1;
    for (int g = gp_off[f]; g < gp_off[f + 1]; ++g, ++slot) {
      for (int j = 0; j < DIM; ++j) {
        double x = gpx[j * NGPT + g];
        if (side && fshift) x -= fshift[(long)f * DIM + j] * period[j];
        gpxi[((long)slot * DIM + j) * N + c] = (x - xc[j]) / h;
      }
    }
  }
  ngp[c] = (uint8_t)slot;
  for (; slot < NGPC; ++slot) {
    for (int j = 0; j < DIM; ++j) gpxi[((long)slot * DIM + j) * N + c] = 0.0;
  }
}

template <typename T>
__global__ void k_convert(long n, const double *src, T *dst) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

// [rows][n] -> [n][rows] (cell-major copy of a per-cell table)
template <typename T>
__global__ void k_cell_major(long n, int rows, const double *src, T *dst) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * rows) dst[i] = (T)src[(i % rows) * n + i / rows];
}

// 1 / h_c per cell, and per face 1 / L_int, the distance between the two
// cell centres with the right cell's periodic image next to the left cell
// (0 at boundary faces): the penalty of Eq. viscous_jump.
template <typename T>
__global__ void k_visc_geom(int N, int NF, int DIM, const double *geom, const int *fcells, const int8_t *fshift,
                            const double *period, T *hinv, T *linv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) hinv[i] = (T)(1.0 / geom[(DIM + 1) * N + i]);
  if (i < NF) {
    const int l = fcells[i], r = fcells[NF + i];
    double v = 0.0;
    if (r >= 0) {
      double d2 = 0.0;
      for (int j = 0; j < DIM; ++j) {
        const double dx = geom[j * N + r] + (fshift ? fshift[(long)i * DIM + j] * period[j] : 0.0) - geom[j * N + l];
        d2 += dx * dx;
      }
      v = 1.0 / sqrt(d2);
    }
    linv[i] = (T)v;
  }
}

template <typename T>
__global__ void k_thresholds(int N, int DIM, const double *geom, double kappa, double nexp, T *thr, T *ivol,
                             T *veps2) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double kh = kappa * geom[(DIM + 1) * N + c];
  thr[c] = (T)pow(kh, nexp);
  veps2[c] = (T)(kh * kh * kh);
  ivol[c] = (T)(1.0 / geom[DIM * N + c]);
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

hfv_status dev_alloc(hfv_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    ctx->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
    return HFV_ERR_OOM;
  }
  ctx->allocs.push_back(*p);
  return HFV_OK;
}

template <typename U>
static hfv_status upload(hfv_ctx *ctx, U **dst, const U *src, size_t n, hipStream_t s) {
  hfv_status st = dev_alloc(ctx, (void **)dst, n * sizeof(U));
  if (st != HFV_OK) return st;
  if (n) HFV_HIP(hipMemcpyAsync(*dst, src, n * sizeof(U), hipMemcpyHostToDevice, s));
  return HFV_OK;
}

struct Temp {
  std::vector<void *> p;
  ~Temp() {
    for (void *q : p) (void)hipFree(q);
  }
  template <typename U>
  hipError_t alloc(U **q, size_t n) {
    hipError_t e = hipMalloc((void **)q, std::max<size_t>(n * sizeof(U), 16));
    if (e == hipSuccess) p.push_back(*q);
    return e;
  }
};

#define TMP_ALLOC(ptr, n)                                                            \
  do {                                                                               \
    if (tmp.alloc(&(ptr), (n)) != hipSuccess) {                                      \
      ctx->err = "temporary device allocation failed";                               \
      return HFV_ERR_OOM;                                                            \
    }                                                                                \
  } while (0)

template <int DIM, int R>
static hfv_status setup_dr(hfv_ctx *ctx, const hfv_mesh *mesh, const hfv_stencils *st, hipStream_t s,
                           const Rules &RU, std::vector<int> &h_cf_off, std::vector<int> &h_cf,
                           std::vector<int> &h_gp_off) {
  constexpr int K = n_unknowns(DIM, R);
  const int N = ctx->N, NF = ctx->NF, M = ctx->M, NFM = ctx->NFM, Md = ctx->Md, NGPT = ctx->NGPT,
            NGPC = ctx->NGPC, nvar = ctx->nvar;
  const int B = 128;
  Temp tmp;
  // mesh upload (temporary)
  double *vtx, *period;
  int8_t *type, *fshift = nullptr, *cshift = nullptr, *dshift = nullptr, *mshift = nullptr;
  int *cvo, *cv, *fvo, *fv, *central, *dir, *ndir, *mus, *nmus, *gp_off, *cf_off, *cf, *fcells;
  TMP_ALLOC(vtx, (size_t)mesh->n_vertices * DIM);
  TMP_ALLOC(period, 3);
  TMP_ALLOC(type, N);
  TMP_ALLOC(cvo, N + 1);
  TMP_ALLOC(cv, mesh->cell_vtx_off[N]);
  TMP_ALLOC(fvo, NF + 1);
  TMP_ALLOC(fv, mesh->face_vtx_off[NF]);
  TMP_ALLOC(central, (size_t)N * M);
  TMP_ALLOC(dir, (size_t)N * NFM * Md);
  TMP_ALLOC(ndir, N);
  TMP_ALLOC(mus, (size_t)N * NFM);
  TMP_ALLOC(nmus, N);
  double hper[3] = {0, 0, 0};
  if (mesh->period)
    for (int j = 0; j < DIM; ++j) hper[j] = mesh->period[j];
  HFV_HIP(hipMemcpyAsync(vtx, mesh->vertices, sizeof(double) * mesh->n_vertices * DIM, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(period, hper, sizeof hper, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(type, mesh->cell_type, N, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(cvo, mesh->cell_vtx_off, sizeof(int) * (N + 1), hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(cv, mesh->cell_vtx, sizeof(int) * mesh->cell_vtx_off[N], hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(fvo, mesh->face_vtx_off, sizeof(int) * (NF + 1), hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(fv, mesh->face_vtx, sizeof(int) * mesh->face_vtx_off[NF], hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(central, st->central, sizeof(int) * N * M, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(dir, st->dir, sizeof(int) * N * NFM * Md, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(ndir, st->n_dir, sizeof(int) * N, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(mus, st->muscl, sizeof(int) * N * NFM, hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(nmus, st->n_muscl, sizeof(int) * N, hipMemcpyHostToDevice, s));
  if (mesh->face_shift) {
    TMP_ALLOC(fshift, (size_t)NF * DIM);
    HFV_HIP(hipMemcpyAsync(fshift, mesh->face_shift, NF * DIM, hipMemcpyHostToDevice, s));
  }
  if (st->central_shift) {
    TMP_ALLOC(cshift, (size_t)N * M * DIM);
    HFV_HIP(hipMemcpyAsync(cshift, st->central_shift, (size_t)N * M * DIM, hipMemcpyHostToDevice, s));
  }
  if (st->dir_shift) {
    TMP_ALLOC(dshift, (size_t)N * NFM * Md * DIM);
    HFV_HIP(hipMemcpyAsync(dshift, st->dir_shift, (size_t)N * NFM * Md * DIM, hipMemcpyHostToDevice, s));
  }
  if (st->muscl_shift) {
    TMP_ALLOC(mshift, (size_t)N * NFM * DIM);
    HFV_HIP(hipMemcpyAsync(mshift, st->muscl_shift, (size_t)N * NFM * DIM, hipMemcpyHostToDevice, s));
  }
  TMP_ALLOC(gp_off, NF + 1);
  TMP_ALLOC(cf_off, N + 1);
  TMP_ALLOC(cf, h_cf.size());
  TMP_ALLOC(fcells, (size_t)2 * NF);
  std::vector<int> h_fc(2 * (size_t)NF);
  for (int f = 0; f < NF; ++f) {
    h_fc[f] = mesh->face_cells[2 * f];
    h_fc[NF + f] = mesh->face_cells[2 * f + 1];
  }
  HFV_HIP(hipMemcpyAsync(gp_off, h_gp_off.data(), sizeof(int) * (NF + 1), hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(cf_off, h_cf_off.data(), sizeof(int) * (N + 1), hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(cf, h_cf.data(), sizeof(int) * h_cf.size(), hipMemcpyHostToDevice, s));
  HFV_HIP(hipMemcpyAsync(fcells, h_fc.data(), sizeof(int) * 2 * NF, hipMemcpyHostToDevice, s));

  // FP64 tables
  double *geom;
  HFV_HIP(hipMalloc((void **)&geom, sizeof(double) * (DIM + 2) * N));
  ctx->allocs.push_back(geom);
  ctx->geom = geom;
  using MC = MomCfg<DIM, R>;
  double *mom, *psibar, *OI, *A, *wv, *rdiag, *vn2, *y, *P, *Pdir, *Pmus, *gpx, *gpw, *fn, *gpxi;
  int *bad;
  uint8_t *ngp;
  TMP_ALLOC(mom, (size_t)MC::NM * N);
  TMP_ALLOC(psibar, (size_t)K * N);
  TMP_ALLOC(OI, (size_t)K * (K + 1) / 2 * N);
  TMP_ALLOC(A, (size_t)K * M * N);
  TMP_ALLOC(wv, (size_t)M * N);
  TMP_ALLOC(rdiag, (size_t)K * N);
  TMP_ALLOC(vn2, (size_t)K * N);
  TMP_ALLOC(y, (size_t)M * N);
  TMP_ALLOC(P, (size_t)K * M * N);
  TMP_ALLOC(Pdir, (size_t)NFM * DIM * Md * N);
  TMP_ALLOC(Pmus, (size_t)DIM * NFM * N);
  TMP_ALLOC(gpx, (size_t)DIM * NGPT);
  TMP_ALLOC(gpw, (size_t)NGPT);
  TMP_ALLOC(fn, (size_t)DIM * NF);
  TMP_ALLOC(gpxi, (size_t)NGPC * DIM * N);
  TMP_ALLOC(bad, (size_t)N);
  TMP_ALLOC(ngp, (size_t)N);
  HFV_HIP(hipMemsetAsync(bad, 0, sizeof(int) * N, s));

  k_cell_geom<DIM><<<nblk(N, B), B, 0, s>>>(N, vtx, type, cvo, cv, geom);
  k_face_geom<DIM><<<nblk(NF, B), B, 0, s>>>(NF, vtx, fvo, fv, gp_off, RU, gpx, gpw, fn, NGPT);
  k_moments<DIM, R><<<nblk(N, 64), 64, 0, s>>>(N, vtx, type, cvo, cv, geom, RU, mom, psibar);
  // OI term list
  {
    constexpr Exps<DIM, 1, R> E{};
    constexpr Exps<DIM, 0, MC::DEG> EM{};
    auto mom_index = [&](const int *g) {
      for (int q = 0; q < MC::NM; ++q) {
        bool eq = true;
        for (int j = 0; j < DIM; ++j) eq = eq && EM.e[q][j] == g[j];
        if (eq) return q;
      }
      return -1;
    };
    std::vector<int> start(1, 0), idx;
    std::vector<double> coef;
    for (int k = 0; k < K; ++k)
      for (int q = k; q < K; ++q) {
        for (int b = 0; b < K; ++b) {  // multi-indices beta with 1 <= |beta| <= R
          double cf_ = 1.0;
          int g[3] = {0, 0, 0};
          for (int j = 0; j < DIM; ++j) {
            int bk = E.e[b][j], ak = E.e[k][j], aq = E.e[q][j];
            if (bk > ak || bk > aq) {
              cf_ = 0;
              break;
            }
            for (int t = 0; t < bk; ++t) cf_ *= double(ak - t) * double(aq - t);
            g[j] = ak + aq - 2 * bk;
          }
          if (cf_ == 0) continue;
          int mi = mom_index(g);
          if (mi < 0) {
            ctx->err = "internal: missing moment";
            return HFV_ERR_STATE;
          }
          coef.push_back(cf_);
          idx.push_back(mi);
        }
        start.push_back((int)coef.size());
      }
    int *d_start, *d_idx;
    double *d_coef;
    TMP_ALLOC(d_start, start.size());
    TMP_ALLOC(d_idx, idx.size());
    TMP_ALLOC(d_coef, coef.size());
    HFV_HIP(hipMemcpyAsync(d_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice, s));
    HFV_HIP(hipMemcpyAsync(d_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, s));
    HFV_HIP(hipMemcpyAsync(d_coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, s));
    k_oi<<<nblk(N, B), B, 0, s>>>(N, K * (K + 1) / 2, d_start, d_coef, d_idx, mom, OI);
    HFV_HIP(hipGetLastError());
    HFV_HIP(hipStreamSynchronize(s));  // term lists are freed at scope exit
  }
  k_lsq_rows<DIM, R><<<nblk((long)N * M, 64), 64, 0, s>>>(N, M, vtx, type, cvo, cv, central, cshift, period,
                                                          geom, psibar, RU, A, wv);
  k_qr_pinv<<<nblk(N, 64), 64, 0, s>>>(N, K, M, A, wv, rdiag, vn2, y, P, bad);
  k_small_pinv<DIM><<<nblk((long)N * (NFM + 1), B), B, 0, s>>>(N, NFM, Md, dir, dshift, ndir, mus, mshift, nmus,
                                                               period, geom, psibar, Pdir, Pmus, bad);
  k_cell_gp<DIM><<<nblk(N, B), B, 0, s>>>(N, NGPT, NGPC, cf_off, cf, gp_off, gpx, fshift, period, geom, gpxi,
                                          ngp);
  HFV_HIP(hipGetLastError());
  std::vector<int> h_bad(N);
  HFV_HIP(hipMemcpyAsync(h_bad.data(), bad, sizeof(int) * N, hipMemcpyDeviceToHost, s));
  HFV_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < N; ++c)
    if (h_bad[c]) {
      ctx->err = std::string("rank-deficient ") + ((h_bad[c] & 1) ? "central" : "directional/MUSCL") +
                 " least-squares system at cell " + std::to_string(c);
      return HFV_ERR_RANK;
    }

  // persistent tables in the context's precision
  auto keep = [&](auto &tabs) -> hfv_status {
    using T = typename std::remove_pointer<decltype(tabs.P)>::type;
    auto conv = [&](T **dst, const double *src, size_t n) -> hfv_status {
      hfv_status e = dev_alloc(ctx, (void **)dst, n * sizeof(T));
      if (e != HFV_OK) return e;
      k_convert<T><<<nblk((long)n, 256), 256, 0, s>>>((long)n, src, *dst);
      ctx->table_bytes += n * sizeof(T);
      return HFV_OK;
    };
    hfv_status e;
    if ((e = conv(&tabs.P, P, (size_t)K * M * N))) return e;
    if ((e = conv(&tabs.psibar, psibar, (size_t)K * N))) return e;
    if ((e = conv(&tabs.gpxi, gpxi, (size_t)NGPC * DIM * N))) return e;
    if ((e = conv(&tabs.OI, OI, (size_t)K * (K + 1) / 2 * N))) return e;
    {  // cell-major copies of the class-list kernels' tables: a sparse list
       // reads each cell's rows contiguously
      auto cm = [&](T **dst, const double *src, int rows) -> hfv_status {
        hfv_status e3 = dev_alloc(ctx, (void **)dst, (size_t)rows * N * sizeof(T));
        if (e3 != HFV_OK) return e3;
        k_cell_major<T><<<nblk((long)rows * N, 256), 256, 0, s>>>((long)N, rows, src, *dst);
        ctx->table_bytes += (size_t)rows * N * sizeof(T);
        return HFV_OK;
      };
      if ((e = cm(&tabs.OIc, OI, K * (K + 1) / 2))) return e;
      if ((e = cm(&tabs.PdirC, Pdir, NFM * DIM * Md))) return e;
      if ((e = cm(&tabs.psibarC, psibar, K))) return e;
      if ((e = cm(&tabs.gpxiC, gpxi, NGPC * DIM))) return e;
      if ((e = cm(&tabs.PmusC, Pmus, DIM * NFM))) return e;
    }
    if ((e = conv(&tabs.Pdir, Pdir, (size_t)NFM * DIM * Md * N))) return e;
    if ((e = conv(&tabs.Pmus, Pmus, (size_t)DIM * NFM * N))) return e;
    if ((e = conv(&tabs.fnormal, fn, (size_t)DIM * NF))) return e;
    if ((e = conv(&tabs.gpw, gpw, (size_t)NGPT))) return e;
    if ((e = dev_alloc(ctx, (void **)&tabs.thr, sizeof(T) * N))) return e;
    if ((e = dev_alloc(ctx, (void **)&tabs.ivol, sizeof(T) * N))) return e;
    if ((e = dev_alloc(ctx, (void **)&tabs.veps2, sizeof(T) * N))) return e;
    k_thresholds<T><<<nblk(N, 256), 256, 0, s>>>(N, DIM, geom, ctx->p.kappa, ctx->p.n_exp, tabs.thr, tabs.ivol,
                                                 tabs.veps2);
    if ((e = dev_alloc(ctx, (void **)&tabs.hinv, sizeof(T) * N))) return e;
    if ((e = dev_alloc(ctx, (void **)&tabs.linv, sizeof(T) * NF))) return e;
    k_visc_geom<T><<<nblk(std::max(N, NF), 256), 256, 0, s>>>(N, NF, DIM, geom, fcells, fshift, period, tabs.hinv,
                                                             tabs.linv);
    // integer tables (shared layout for both precisions)
    if ((e = dev_alloc(ctx, (void **)&tabs.ngp, N))) return e;
    HFV_HIP(hipMemcpyAsync(tabs.ngp, ngp, N, hipMemcpyDeviceToDevice, s));
    HFV_HIP(hipGetLastError());
    return HFV_OK;
  };
  hfv_status e = ctx->prec == 64 ? keep(ctx->t64) : keep(ctx->t32);
  if (e != HFV_OK) return e;
  HFV_HIP(hipStreamSynchronize(s));
  return HFV_OK;
}

static hfv_status build_vjp_tables(hfv_ctx *ctx, const hfv_mesh *mesh, const hfv_stencils *st,
                                   const std::vector<int> &cf_off, const std::vector<int> &cf, hipStream_t s);

hfv_status setup_tables(hfv_ctx *ctx, const hfv_mesh *mesh, const hfv_stencils *st, hipStream_t s) {
  const int N = ctx->N, NF = ctx->NF, DIM = ctx->dim, NFM = ctx->NFM, r = ctx->r;
  Rules RU{};
  for (int n = 1; n <= 7; ++n) gauss_legendre01(n, RU.glx[n], RU.glw[n]);
  RU.n_line = (r + 2) / 2;
  if (DIM == 3 && !triangle_rule(r, RU)) {
    ctx->err = "triangle face rule unavailable for this order";
    return HFV_ERR_PARAM;
  }
  // cell -> face incidence in face order, face Gauss point offsets
  std::vector<int> cnt(N + 1, 0);
  for (int f = 0; f < NF; ++f) {
    cnt[mesh->face_cells[2 * f] + 1]++;
    if (mesh->face_cells[2 * f + 1] >= 0) cnt[mesh->face_cells[2 * f + 1] + 1]++;
  }
  std::vector<int> cf_off(N + 1, 0);
  for (int c = 0; c < N; ++c) cf_off[c + 1] = cf_off[c] + cnt[c + 1];
  std::vector<int> cf(cf_off[N]), fill(cf_off.begin(), cf_off.end() - 1);
  for (int f = 0; f < NF; ++f) {
    cf[fill[mesh->face_cells[2 * f]]++] = f;
    int rr = mesh->face_cells[2 * f + 1];
    if (rr >= 0) cf[fill[rr]++] = f | (int)0x80000000u;
  }
  std::vector<int> gp_off(NF + 1, 0);
  for (int f = 0; f < NF; ++f) {
    int nv = mesh->face_vtx_off[f + 1] - mesh->face_vtx_off[f];
    int n = DIM == 2 ? RU.n_line : (nv == 3 ? RU.tri_n : RU.n_line * RU.n_line);
    gp_off[f + 1] = gp_off[f] + n;
  }
  ctx->NGPT = gp_off[NF];
  int ngpc = 0;
  std::vector<int> nbr((size_t)NFM * N, -1);
  std::vector<uint8_t> nfc(N);
  std::vector<int> fgb(NF, 0);  // local Gauss-point slot of each face in its two cells
  for (int c = 0; c < N; ++c) {
    int g = 0, k = 0;
    for (int e = cf_off[c]; e < cf_off[c + 1]; ++e, ++k) {
      int f = cf[e] & 0x7fffffff;
      int side = (cf[e] >> 31) & 1;
      if (side)
        fgb[f] |= g << 8;
      else
        fgb[f] |= g | (mesh->face_cells[2 * f + 1] < 0 ? g << 8 : 0);
      g += gp_off[f + 1] - gp_off[f];
      nbr[(size_t)k * N + c] = side ? mesh->face_cells[2 * f] : mesh->face_cells[2 * f + 1];
    }
    if (g > 255) {  // slots are stored in bytes
      ctx->err = "more than 255 face Gauss points in cell " + std::to_string(c);
      return HFV_ERR_MESH;
    }
    nfc[c] = (uint8_t)k;
    ngpc = std::max(ngpc, g);
  }
  ctx->NGPC = ngpc;
  hfv_status e;
  switch (DIM * 10 + r) {
    case 21: e = setup_dr<2, 1>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 22: e = setup_dr<2, 2>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 23: e = setup_dr<2, 3>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 24: e = setup_dr<2, 4>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 25: e = setup_dr<2, 5>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 26: e = setup_dr<2, 6>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 31: e = setup_dr<3, 1>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 32: e = setup_dr<3, 2>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 33: e = setup_dr<3, 3>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    case 34: e = setup_dr<3, 4>(ctx, mesh, st, s, RU, cf_off, cf, gp_off); break;
    default: ctx->err = "unsupported (dim, order_r)"; return HFV_ERR_PARAM;
  }
  if (e != HFV_OK) return e;
  // integer tables in hot-path layouts
  const int M = ctx->M, Md = ctx->Md;
  std::vector<int> sten((size_t)M * N), dsten((size_t)NFM * Md * N), dstenC((size_t)NFM * Md * N),
      msten((size_t)NFM * N), mstenC((size_t)NFM * N), nbrC((size_t)NFM * N);
  std::vector<uint8_t> ndir(N), nmus(N);
  for (int c = 0; c < N; ++c) {
    for (int m = 0; m < M; ++m) sten[(size_t)m * N + c] = st->central[(size_t)c * M + m];
    for (int sidx = 0; sidx < NFM; ++sidx)
      for (int q = 0; q < Md; ++q) {
        int v = st->dir[((size_t)c * NFM + sidx) * Md + q];
        dsten[((size_t)sidx * Md + q) * N + c] = v >= 0 ? v : c;
        dstenC[((size_t)c * NFM + sidx) * Md + q] = v >= 0 ? v : c;
      }
    for (int q = 0; q < NFM; ++q) {
      int v = st->muscl[(size_t)c * NFM + q];
      msten[(size_t)q * N + c] = v >= 0 ? v : c;
      mstenC[(size_t)c * NFM + q] = v >= 0 ? v : c;
      nbrC[(size_t)c * NFM + q] = nbr[(size_t)q * N + c];
    }
    ndir[c] = (uint8_t)st->n_dir[c];
    nmus[c] = (uint8_t)st->n_muscl[c];
  }
  std::vector<int> fcells(2 * (size_t)NF);
  for (int f = 0; f < NF; ++f) {
    fcells[f] = mesh->face_cells[2 * f];
    fcells[NF + f] = mesh->face_cells[2 * f + 1];
  }
  auto put = [&](auto &tabs) -> hfv_status {
    hfv_status e2;
    if ((e2 = upload(ctx, &tabs.sten, sten.data(), sten.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.nbr, nbr.data(), nbr.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.nfc, nfc.data(), nfc.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.dsten, dsten.data(), dsten.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.dstenC, dstenC.data(), dstenC.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.ndir, ndir.data(), ndir.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.msten, msten.data(), msten.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.mstenC, mstenC.data(), mstenC.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.nbrC, nbrC.data(), nbrC.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.nmus, nmus.data(), nmus.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.gp_off, gp_off.data(), gp_off.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.face_cells, fcells.data(), fcells.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.fgb, fgb.data(), fgb.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.cf_off, cf_off.data(), cf_off.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.cf, cf.data(), cf.size(), s))) return e2;
    ctx->table_bytes += sizeof(int) * (sten.size() + 2 * nbr.size() + 2 * dsten.size() + 2 * msten.size());
    return HFV_OK;
  };
  e = ctx->prec == 64 ? put(ctx->t64) : put(ctx->t32);
  if (e != HFV_OK) return e;
  HFV_HIP(hipStreamSynchronize(s));
  return build_vjp_tables(ctx, mesh, st, cf_off, cf, s);
}

// Adjoint tables: where the directional, MUSCL and face-neighbour members sit
// inside each central stencil, and the transpose of the central stencil.
static hfv_status build_vjp_tables(hfv_ctx *ctx, const hfv_mesh *mesh, const hfv_stencils *st,
                                   const std::vector<int> &cf_off, const std::vector<int> &cf, hipStream_t s) {
  const int N = ctx->N, M = ctx->M, NFM = ctx->NFM, Md = ctx->Md, D = ctx->dim;
  std::vector<uint8_t> dpos((size_t)NFM * Md * N, 0), mpos((size_t)NFM * N, 0), nbpos((size_t)NFM * N, 255);
  ctx->vjp_ok = true;
  auto find = [&](int c, int id, const int8_t *sh) -> int {
    for (int m = 0; m < M; ++m) {
      if (st->central[(size_t)c * M + m] != id) continue;
      bool eq = true;
      for (int j = 0; j < D; ++j) {
        int a = st->central_shift ? st->central_shift[((size_t)c * M + m) * D + j] : 0;
        int b = sh ? sh[j] : 0;
        eq = eq && a == b;
      }
      if (eq) return m;
    }
    return -1;
  };
  auto fail = [&](const std::string &why) {
    if (ctx->vjp_ok) ctx->vjp_why = why;
    ctx->vjp_ok = false;
  };
  for (int c = 0; c < N && ctx->vjp_ok; ++c) {
    for (int sd = 0; sd < st->n_dir[c]; ++sd)
      for (int q = 0; q < Md; ++q) {
        size_t e = ((size_t)c * NFM + sd) * Md + q;
        int m = find(c, st->dir[e], st->dir_shift ? st->dir_shift + e * D : nullptr);
        if (m < 0) fail("directional member outside the central stencil at cell " + std::to_string(c));
        dpos[((size_t)sd * Md + q) * N + c] = (uint8_t)std::max(m, 0);
      }
    for (int q = 0; q < st->n_muscl[c]; ++q) {
      size_t e = (size_t)c * NFM + q;
      int m = find(c, st->muscl[e], st->muscl_shift ? st->muscl_shift + e * D : nullptr);
      if (m < 0) fail("MUSCL member outside the central stencil at cell " + std::to_string(c));
      mpos[(size_t)q * N + c] = (uint8_t)std::max(m, 0);
    }
    int k = 0;
    for (int e = cf_off[c]; e < cf_off[c + 1]; ++e, ++k) {
      int f = cf[e] & 0x7fffffff;
      int side = (cf[e] >> 31) & 1;
      int nb = side ? mesh->face_cells[2 * f] : mesh->face_cells[2 * f + 1];
      if (nb < 0) continue;
      int8_t sh[3] = {0, 0, 0};
      if (mesh->face_shift)
        for (int j = 0; j < D; ++j) sh[j] = (int8_t)(side ? -mesh->face_shift[(size_t)f * D + j] : mesh->face_shift[(size_t)f * D + j]);
      int m = find(c, nb, sh);
      if (m < 0) fail("face neighbour outside the central stencil at cell " + std::to_string(c));
      nbpos[(size_t)k * N + c] = (uint8_t)std::max(m, 0);
    }
  }
  std::vector<int> inv_off(N + 1, 0), inv_idx((size_t)N * M);
  for (size_t e = 0; e < (size_t)N * M; ++e) inv_off[st->central[e] + 1]++;
  for (int j = 0; j < N; ++j) inv_off[j + 1] += inv_off[j];
  std::vector<int> fill(inv_off.begin(), inv_off.end() - 1);
  for (int i = 0; i < N; ++i)
    for (int m = 0; m < M; ++m) inv_idx[fill[st->central[(size_t)i * M + m]]++] = m * N + i;
  auto put = [&](auto &tabs) -> hfv_status {
    hfv_status e2;
    if ((e2 = upload(ctx, &tabs.dpos, dpos.data(), dpos.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.mpos, mpos.data(), mpos.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.nbpos, nbpos.data(), nbpos.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.inv_off, inv_off.data(), inv_off.size(), s))) return e2;
    if ((e2 = upload(ctx, &tabs.inv_idx, inv_idx.data(), inv_idx.size(), s))) return e2;
    return HFV_OK;
  };
  hfv_status e = ctx->prec == 64 ? put(ctx->t64) : put(ctx->t32);
  if (e != HFV_OK) return e;
  const size_t ts = ctx->prec == 64 ? 8 : 4;
  if ((e = dev_alloc(ctx, &ctx->vjp_C, ts * (size_t)M * ctx->nvar * N))) return e;
  if ((e = dev_alloc(ctx, &ctx->vjp_S, ts * (size_t)ctx->nvar * N))) return e;
  if ((e = dev_alloc(ctx, &ctx->vjp_gfs, ts * (size_t)ctx->NGPC * ctx->nvar * ctx->N))) return e;
  HFV_HIP(hipStreamSynchronize(s));
  return HFV_OK;
}

// Re-derive the deactivation thresholds after a parameter change.
hfv_status refresh_thresholds(hfv_ctx *ctx, hipStream_t s) {
  const int N = ctx->N;
  if (ctx->prec == 64)
    k_thresholds<double><<<nblk(N, 256), 256, 0, s>>>(N, ctx->dim, ctx->geom, ctx->p.kappa, ctx->p.n_exp,
                                                      ctx->t64.thr, ctx->t64.ivol, ctx->t64.veps2);
  else
    k_thresholds<float><<<nblk(N, 256), 256, 0, s>>>(N, ctx->dim, ctx->geom, ctx->p.kappa, ctx->p.n_exp,
                                                     ctx->t32.thr, ctx->t32.ivol, ctx->t32.veps2);
  HFV_HIP(hipGetLastError());
  return HFV_OK;
}

}  // namespace hfv
