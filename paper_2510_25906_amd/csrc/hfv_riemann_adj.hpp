// Reverse mode of the Riemann fluxes (Section 2.4: HLLC and HLL with Davis
// wave-speed estimates), written out by hand.
//
// Given the cotangent gF of one face flux F(qL, qR), riemann_vjp returns
// gL = (dF/dqL)^T gF and gR = (dF/dqR)^T gF.  The primal runs once; the
// cotangent then flows back through the branch the primal took (supersonic,
// HLL average, left or right HLLC star region), with the wave-speed choices
// of min/max held where the primal put them (the left side on ties).  Every
// expression differentiated here is the one the forward flux evaluates, so
// the result is the exact Jacobian-transpose product up to rounding order.
#pragma once

namespace hfv {

// One side of the face: conserved state, primitive intermediates and their
// cotangents.
template <int DIM, typename T>
struct RSide {
  static constexpr int NV = DIM + 2;
  T q[NV], v[DIM], un, p, c;
  T gq[NV], gv[DIM], gun, gp, gc;

  __device__ inline void init(const T (&qi)[NV], const T (&n)[DIM], T gamma) {
    T k = 0;
    un = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      q[i] = qi[i];
      gq[i] = 0;
    }
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      v[j] = q[1 + j] / q[0];
      un += v[j] * n[j];
      k += v[j] * v[j];
      gv[j] = 0;
    }
    p = (gamma - (T)1) * (q[NV - 1] - (T)0.5 * q[0] * k);
    c = sqrt(gamma * p / q[0]);
    gun = gp = gc = 0;
  }

  // Physical flux F = (r un, m un + p n, un (E + p)).
  __device__ inline void flux(const T (&n)[DIM], T (&F)[NV]) const {
    F[0] = q[0] * un;
#pragma unroll
    for (int j = 0; j < DIM; ++j) F[1 + j] = q[1 + j] * un + p * n[j];
    F[NV - 1] = un * (q[NV - 1] + p);
  }

  // Adds w^T dF/d(q, un, p) of the physical flux to the cotangents.
  __device__ inline void flux_adj(const T (&n)[DIM], const T (&w)[NV]) {
    gq[0] += w[0] * un;
    gun += w[0] * q[0];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      gq[1 + j] += w[1 + j] * un;
      gun += w[1 + j] * q[1 + j];
      gp += w[1 + j] * n[j];
    }
    gun += w[NV - 1] * (q[NV - 1] + p);
    gq[NV - 1] += w[NV - 1] * un;
    gp += w[NV - 1] * un;
  }

  // Moves the cotangents of c, p, un and v onto the conserved state:
  // c = sqrt(gamma p / r), p = (gamma - 1)(E - r |v|^2 / 2), un = v . n, v = m / r.
  __device__ inline void finish(const T (&n)[DIM], T gamma) {
    const T r = q[0], gm1 = gamma - (T)1;
    gp += gc * gamma / (2 * c * r);
    T gr = -gc * c / (2 * r);
    gq[NV - 1] += gm1 * gp;
    T k = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      k += v[j] * v[j];
      gv[j] += n[j] * gun - gm1 * r * v[j] * gp;
    }
    gr -= (T)0.5 * gm1 * k * gp;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      gq[1 + j] += gv[j] / r;
      gr -= gv[j] * v[j] / r;
    }
    gq[0] += gr;
  }
};

// Star-region flux of side s, F = F_s + S (U*_s - q_s), with the HLLC star
// state U*_s = r (S - un) / (S - Ss) (1, v + (Ss - un) n, E / r + (Ss - un)(Ss + p / (r (S - un)))).
// Adds gF^T dF to the cotangents of s, S and Ss.
template <int DIM, typename T>
__device__ inline void hllc_star_adj(RSide<DIM, T> &s, const T (&n)[DIM], T S, T Ss, const T (&gF)[DIM + 2],
                                     T &gS, T &gSs) {
  constexpr int NV = DIM + 2;
  const T r = s.q[0], A = S - s.un, B = S - Ss, fac = r * A / B, d = Ss - s.un, G = Ss + s.p / (r * A);
  T W[NV];
  W[0] = 1;
#pragma unroll
  for (int j = 0; j < DIM; ++j) W[1 + j] = s.v[j] + d * n[j];
  W[NV - 1] = s.q[NV - 1] / r + d * G;
  s.flux_adj(n, gF);
  T gfac = 0, gd = 0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    s.gq[i] -= S * gF[i];
    gS += gF[i] * (fac * W[i] - s.q[i]);
    gfac += S * gF[i] * W[i];
  }
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const T wb = S * gF[1 + j] * fac;
    s.gv[j] += wb;
    gd += wb * n[j];
  }
  const T wE = S * gF[NV - 1] * fac;
  s.gq[NV - 1] += wE / r;
  T gr = -wE * s.q[NV - 1] / (r * r);
  gd += wE * G;
  const T gG = wE * d;
  gSs += gG;
  s.gp += gG / (r * A);
  gr -= gG * s.p / (r * r * A);
  T gA = -gG * s.p / (r * A * A);
  gSs += gd;
  s.gun -= gd;
  gr += gfac * A / B;
  gA += gfac * r / B;
  const T gB = -gfac * fac / B;
  gS += gB;
  gSs -= gB;
  gS += gA;
  s.gun -= gA;
  s.gq[0] += gr;
}

template <int DIM, typename T>
__device__ inline void riemann_vjp(const T (&qL)[DIM + 2], const T (&qR)[DIM + 2], const T (&n)[DIM], T gamma,
                                   int hllc, const T (&gF)[DIM + 2], T (&gL)[DIM + 2], T (&gR)[DIM + 2]) {
  constexpr int NV = DIM + 2;
  RSide<DIM, T> L, R;
  L.init(qL, n, gamma);
  R.init(qR, n, gamma);
  const bool sl_left = L.un - L.c <= R.un - R.c, sr_left = L.un + L.c >= R.un + R.c;
  const T SL = sl_left ? L.un - L.c : R.un - R.c;
  const T SR = sr_left ? L.un + L.c : R.un + R.c;
  T gSL = 0, gSR = 0;
  if (SL >= (T)0) {
    L.flux_adj(n, gF);
  } else if (!hllc) {
    if (SR <= (T)0) {
      R.flux_adj(n, gF);
    } else {
      // F = (SR FL - SL FR + SL SR (qR - qL)) / (SR - SL)
      T FL[NV], FR[NV], wL[NV], wR[NV];
      L.flux(n, FL);
      R.flux(n, FR);
      const T D = SR - SL;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const T dq = R.q[i] - L.q[i];
        const T F = (SR * FL[i] - SL * FR[i] + SL * SR * dq) / D;
        gSR += gF[i] * (FL[i] + SL * dq - F) / D;
        gSL += gF[i] * (F - FR[i] + SR * dq) / D;
        wL[i] = gF[i] * SR / D;
        wR[i] = -gF[i] * SL / D;
        R.gq[i] += gF[i] * SL * SR / D;
        L.gq[i] -= gF[i] * SL * SR / D;
      }
      L.flux_adj(n, wL);
      R.flux_adj(n, wR);
    }
  } else {
    const T AL = SL - L.un, AR = SR - R.un;
    const T num = R.p - L.p + L.q[0] * L.un * AL - R.q[0] * R.un * AR;
    const T den = L.q[0] * AL - R.q[0] * AR;
    const T Ss = num / den;
    T gSs = 0;
    if (Ss >= (T)0) {
      hllc_star_adj<DIM, T>(L, n, SL, Ss, gF, gSL, gSs);
    } else if (SR > (T)0) {
      hllc_star_adj<DIM, T>(R, n, SR, Ss, gF, gSR, gSs);
    } else {
      R.flux_adj(n, gF);
    }
    // Ss = num / den
    const T gnum = gSs / den, gden = -gSs * Ss / den;
    R.gp += gnum;
    L.gp -= gnum;
    L.gq[0] += (gnum * L.un + gden) * AL;
    L.gun += gnum * L.q[0] * AL;
    const T gAL = (gnum * L.un + gden) * L.q[0];
    R.gq[0] -= (gnum * R.un + gden) * AR;
    R.gun -= gnum * R.q[0] * AR;
    const T gAR = -(gnum * R.un + gden) * R.q[0];
    gSL += gAL;
    L.gun -= gAL;
    gSR += gAR;
    R.gun -= gAR;
  }
  // SL = min(unL - cL, unR - cR), SR = max(unL + cL, unR + cR)
  if (sl_left) {
    L.gun += gSL;
    L.gc -= gSL;
  } else {
    R.gun += gSL;
    R.gc -= gSL;
  }
  if (sr_left) {
    L.gun += gSR;
    L.gc += gSR;
  } else {
    R.gun += gSR;
    R.gc += gSR;
  }
  L.finish(n, gamma);
  R.finish(n, gamma);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    gL[i] = L.gq[i];
    gR[i] = R.gq[i];
  }
}

}  // namespace hfv
