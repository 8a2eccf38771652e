// Device-side equation of state, two-point volume fluxes and Riemann solvers.
//
// Conservative state u = (rho, rho v1, rho v2, rho v3, rho e[, rho Y1]) of the
// inviscid part of eq. ns_equation.  Pressure from eq. eos with the mixture
// ratio of eq. mix_R_kappa / eq. mix_cp_cv for two species.  All fluxes are
// returned already contracted with an (unnormalised) direction vector.
#pragma once

#include "dgfv_internal.h"

namespace dgfv {

struct Prim {
  double rho, v1, v2, v3, p, E, kap, Y;
};

template <int NV>
__device__ __forceinline__ Prim cons2prim(const double* u, const GasDev& g) {
  Prim q;
  q.rho = u[0];
  const double ir = 1.0 / q.rho;
  q.v1 = u[1] * ir;
  q.v2 = u[2] * ir;
  q.v3 = u[3] * ir;
  q.E = u[4];
  if constexpr (NV == 6) {
    q.Y = u[5] * ir;
    const double Y2 = 1.0 - q.Y;
    q.kap = (q.Y * g.cp0 + Y2 * g.cp1) / (q.Y * g.cv0 + Y2 * g.cv1);
  } else {
    q.Y = 0.0;
    q.kap = g.gamma;
  }
  q.p = (q.kap - 1.0) * (q.E - 0.5 * q.rho * (q.v1 * q.v1 + q.v2 * q.v2 + q.v3 * q.v3));
  return q;
}

// Physical flux F(u) . a
template <int NV>
__device__ __forceinline__ void euler_flux(const Prim& q, double a1, double a2, double a3,
                                           double* f) {
  const double vn = q.v1 * a1 + q.v2 * a2 + q.v3 * a3;
  const double m = q.rho * vn;
  f[0] = m;
  f[1] = m * q.v1 + q.p * a1;
  f[2] = m * q.v2 + q.p * a2;
  f[3] = m * q.v3 + q.p * a3;
  f[4] = (q.E + q.p) * vn;
  if constexpr (NV == 6) f[5] = m * q.Y;
}

// Logarithmic mean (a - b) / (ln a - ln b) from precomputed logarithms, with the
// Ismail-Roe series F = 1 + u/3 + u^2/5 + u^3/7, u = ((a-b)/(a+b))^2, below u = 1e-4.
__device__ __forceinline__ double log_mean(double a, double b, double la, double lb) {
  const double s = a + b;
  const double f = (a - b) / s;
  const double u = f * f;
  if (u < 1e-4) {
    const double F = 1.0 + u * (1.0 / 3.0 + u * (0.2 + u * (1.0 / 7.0)));
    return s / (2.0 * F);
  }
  return (a - b) / (la - lb);
}

// ---------------------------------------------------------------------------
// Per-node auxiliary records of the volume two-point fluxes.  Each kind stores
// NA doubles per node in LDS (structure of arrays) and evaluates
// f#(u_i, u_m) . a from two records.
// ---------------------------------------------------------------------------

// Ranocha's entropy-conserving, kinetic-energy-preserving flux (single species).
struct FluxRanocha {
  static constexpr int NA = 8;  // rho, v1, v2, v3, p, ln rho, beta = rho/p, ln beta
  template <int NV>
  __device__ __forceinline__ static void make(const Prim& q, double* r) {
    r[0] = q.rho; r[1] = q.v1; r[2] = q.v2; r[3] = q.v3; r[4] = q.p;
    r[5] = log(q.rho);
    const double beta = q.rho / q.p;
    r[6] = beta;
    r[7] = log(beta);
  }
  template <int NV>
  __device__ __forceinline__ static void flux(const double* a_, const double* b_, double a1,
                                              double a2, double a3, const GasDev& g, double* f) {
    const double rho_ln = log_mean(a_[0], b_[0], a_[5], b_[5]);
    const double beta_ln = log_mean(a_[6], b_[6], a_[7], b_[7]);
    const double v1 = 0.5 * (a_[1] + b_[1]), v2 = 0.5 * (a_[2] + b_[2]), v3 = 0.5 * (a_[3] + b_[3]);
    const double pbar = 0.5 * (a_[4] + b_[4]);
    const double vn = v1 * a1 + v2 * a2 + v3 * a3;
    const double fr = rho_ln * vn;
    f[0] = fr;
    f[1] = fr * v1 + pbar * a1;
    f[2] = fr * v2 + pbar * a2;
    f[3] = fr * v3 + pbar * a3;
    const double vv = 0.5 * (a_[1] * b_[1] + a_[2] * b_[2] + a_[3] * b_[3]);
    const double vna = a_[1] * a1 + a_[2] * a2 + a_[3] * a3;
    const double vnb = b_[1] * a1 + b_[2] * a2 + b_[3] * a3;
    f[4] = fr * (1.0 / ((g.gamma - 1.0) * beta_ln) + vv) + 0.5 * (a_[4] * vnb + b_[4] * vna);
  }
};

// Pirozzoli's kinetic-energy-preserving flux (Section 3.5); f_rhoY = f_rho {Y}.
struct FluxPirozzoli {
  static constexpr int NA = 7;  // rho, v1, v2, v3, p, H, Y
  template <int NV>
  __device__ __forceinline__ static void make(const Prim& q, double* r) {
    r[0] = q.rho; r[1] = q.v1; r[2] = q.v2; r[3] = q.v3; r[4] = q.p;
    r[5] = (q.E + q.p) / q.rho;
    r[6] = q.Y;
  }
  template <int NV>
  __device__ __forceinline__ static void flux(const double* a_, const double* b_, double a1,
                                              double a2, double a3, const GasDev&, double* f) {
    const double rho = 0.5 * (a_[0] + b_[0]);
    const double v1 = 0.5 * (a_[1] + b_[1]), v2 = 0.5 * (a_[2] + b_[2]), v3 = 0.5 * (a_[3] + b_[3]);
    const double pbar = 0.5 * (a_[4] + b_[4]);
    const double fr = rho * (v1 * a1 + v2 * a2 + v3 * a3);
    f[0] = fr;
    f[1] = fr * v1 + pbar * a1;
    f[2] = fr * v2 + pbar * a2;
    f[3] = fr * v3 + pbar * a3;
    f[4] = fr * (0.5 * (a_[5] + b_[5]));
    if constexpr (NV == 6) f[5] = fr * (0.5 * (a_[6] + b_[6]));
  }
};

// Arithmetic mean of the physical fluxes.
struct FluxCentral {
  static constexpr int NA = 7;  // rho, v1, v2, v3, p, E, Y
  template <int NV>
  __device__ __forceinline__ static void make(const Prim& q, double* r) {
    r[0] = q.rho; r[1] = q.v1; r[2] = q.v2; r[3] = q.v3; r[4] = q.p; r[5] = q.E; r[6] = q.Y;
  }
  template <int NV>
  __device__ __forceinline__ static void flux(const double* a_, const double* b_, double a1,
                                              double a2, double a3, const GasDev&, double* f) {
    const double vna = a_[1] * a1 + a_[2] * a2 + a_[3] * a3;
    const double vnb = b_[1] * a1 + b_[2] * a2 + b_[3] * a3;
    const double ma = a_[0] * vna, mb = b_[0] * vnb;
    f[0] = 0.5 * (ma + mb);
    f[1] = 0.5 * (ma * a_[1] + a_[4] * a1 + mb * b_[1] + b_[4] * a1);
    f[2] = 0.5 * (ma * a_[2] + a_[4] * a2 + mb * b_[2] + b_[4] * a2);
    f[3] = 0.5 * (ma * a_[3] + a_[4] * a3 + mb * b_[3] + b_[4] * a3);
    f[4] = 0.5 * ((a_[5] + a_[4]) * vna + (b_[5] + b_[4]) * vnb);
    if constexpr (NV == 6) f[5] = 0.5 * (ma * a_[6] + mb * b_[6]);
  }
};

// Two-point flux of the chosen volume kind evaluated from conservative states
// (used at faces with the EC selector).
template <int NV>
__device__ __forceinline__ void two_point_cons(int kind, const double* uL, const double* uR,
                                               double n1, double n2, double n3, const GasDev& g,
                                               double* F) {
  const Prim qL = cons2prim<NV>(uL, g), qR = cons2prim<NV>(uR, g);
  double ra[8], rb[8];
  if (kind == 0) {
    FluxRanocha::make<NV>(qL, ra);
    FluxRanocha::make<NV>(qR, rb);
    FluxRanocha::flux<NV>(ra, rb, n1, n2, n3, g, F);
  } else if (kind == 1) {
    FluxPirozzoli::make<NV>(qL, ra);
    FluxPirozzoli::make<NV>(qR, rb);
    FluxPirozzoli::flux<NV>(ra, rb, n1, n2, n3, g, F);
  } else {
    FluxCentral::make<NV>(qL, ra);
    FluxCentral::make<NV>(qR, rb);
    FluxCentral::flux<NV>(ra, rb, n1, n2, n3, g, F);
  }
}

// Local Lax-Friedrichs flux times the area element |nvec|.
template <int NV>
__device__ __forceinline__ void riemann_llf(const double* uL, const double* uR, double n1,
                                            double n2, double n3, const GasDev& g, double* F) {
  const double s = sqrt(n1 * n1 + n2 * n2 + n3 * n3);
  const double is = 1.0 / s;
  const double e1 = n1 * is, e2 = n2 * is, e3 = n3 * is;
  const Prim qL = cons2prim<NV>(uL, g), qR = cons2prim<NV>(uR, g);
  const double cL = sqrt(qL.kap * qL.p / qL.rho), cR = sqrt(qR.kap * qR.p / qR.rho);
  const double lam = fmax(fabs(qL.v1 * e1 + qL.v2 * e2 + qL.v3 * e3) + cL,
                          fabs(qR.v1 * e1 + qR.v2 * e2 + qR.v3 * e3) + cR);
  double fL[NV], fR[NV];
  euler_flux<NV>(qL, e1, e2, e3, fL);
  euler_flux<NV>(qR, e1, e2, e3, fR);
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = (0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v])) * s;
}

// Roe flux with the Harten-Hyman entropy fix on the acoustic waves, times |nvec| (1 species).
__device__ __forceinline__ double hh_fix(double lam, double lamL, double lamR) {
  const double delta = fmax(0.0, fmax(lam - lamL, lamR - lam));
  const double al = fabs(lam);
  return (al < delta) ? 0.5 * (lam * lam / delta + delta) : al;
}

__device__ __forceinline__ void riemann_roe(const double* uL, const double* uR, double n1, double n2,
                                            double n3, const GasDev& g, double* F) {
  const double s = sqrt(n1 * n1 + n2 * n2 + n3 * n3);
  const double is = 1.0 / s;
  const double e1 = n1 * is, e2 = n2 * is, e3 = n3 * is;
  const Prim qL = cons2prim<5>(uL, g), qR = cons2prim<5>(uR, g);
  const double gm1 = g.gamma - 1.0;
  const double sL = sqrt(qL.rho), sR = sqrt(qR.rho);
  const double iw = 1.0 / (sL + sR);
  const double v1 = (sL * qL.v1 + sR * qR.v1) * iw;
  const double v2 = (sL * qL.v2 + sR * qR.v2) * iw;
  const double v3 = (sL * qL.v3 + sR * qR.v3) * iw;
  const double HL = (qL.E + qL.p) / qL.rho, HR = (qR.E + qR.p) / qR.rho;
  const double H = (sL * HL + sR * HR) * iw;
  const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
  const double c2 = gm1 * (H - 0.5 * vsq);
  const double c = sqrt(c2);
  const double rt = sL * sR;
  const double vn = v1 * e1 + v2 * e2 + v3 * e3;

  const double drho = qR.rho - qL.rho, dp = qR.p - qL.p;
  const double d1 = qR.v1 - qL.v1, d2 = qR.v2 - qL.v2, d3 = qR.v3 - qL.v3;
  const double dvn = d1 * e1 + d2 * e2 + d3 * e3;
  const double a1 = (dp - rt * c * dvn) / (2.0 * c2);
  const double a5 = (dp + rt * c * dvn) / (2.0 * c2);
  const double a2 = drho - dp / c2;
  const double t1 = d1 - dvn * e1, t2 = d2 - dvn * e2, t3 = d3 - dvn * e3;

  const double cL = sqrt(qL.kap * qL.p / qL.rho), cR = sqrt(qR.kap * qR.p / qR.rho);
  const double vnL = qL.v1 * e1 + qL.v2 * e2 + qL.v3 * e3;
  const double vnR = qR.v1 * e1 + qR.v2 * e2 + qR.v3 * e3;
  const double l1 = hh_fix(vn - c, vnL - cL, vnR - cR);
  const double l5 = hh_fix(vn + c, vnL + cL, vnR + cR);
  const double l2 = fabs(vn);

  const double w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2, wt = l2 * rt;
  double D[5];
  D[0] = w1 + w5 + w2;
  D[1] = w1 * (v1 - c * e1) + w5 * (v1 + c * e1) + w2 * v1 + wt * t1;
  D[2] = w1 * (v2 - c * e2) + w5 * (v2 + c * e2) + w2 * v2 + wt * t2;
  D[3] = w1 * (v3 - c * e3) + w5 * (v3 + c * e3) + w2 * v3 + wt * t3;
  D[4] = w1 * (H - c * vn) + w5 * (H + c * vn) + w2 * (0.5 * vsq) + wt * (v1 * t1 + v2 * t2 + v3 * t3);

  double fL[5], fR[5];
  euler_flux<5>(qL, e1, e2, e3, fL);
  euler_flux<5>(qR, e1, e2, e3, fR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = (0.5 * (fL[v] + fR[v]) - 0.5 * D[v]) * s;
}

template <int NV>
__device__ __forceinline__ void riemann(int kind, int vol_kind, const double* uL, const double* uR,
                                        double n1, double n2, double n3, const GasDev& g,
                                        double* F) {
  if (kind == 1) {
    riemann_llf<NV>(uL, uR, n1, n2, n3, g, F);
  } else if (kind == 0) {
    if constexpr (NV == 5) {
      riemann_roe(uL, uR, n1, n2, n3, g, F);
    } else {
      riemann_llf<NV>(uL, uR, n1, n2, n3, g, F);  // rejected on the host
    }
  } else {
    two_point_cons<NV>(vol_kind, uL, uR, n1, n2, n3, g, F);
  }
}

// Face-grid index map of an orientation code on an n x n grid.
__device__ __forceinline__ void orient_map(int o, int p, int q, int n, int& pp, int& qq) {
  int a = (o & 4) ? q : p;
  int b = (o & 4) ? p : q;
  pp = (o & 1) ? n - 1 - a : a;
  qq = (o & 2) ? n - 1 - b : b;
}

// Volume node index of face-grid point (p, q) on side s of an element with n nodes per direction.
__device__ __forceinline__ int side_node(int s, int p, int q, int n) {
  const int last = (s & 1) ? n - 1 : 0;
  switch (s >> 1) {
    case 0: return (q * n + p) * n + last;        // i = last, j = p, k = q
    case 1: return (q * n + last) * n + p;        // j = last, i = p, k = q
    default: return (last * n + q) * n + p;       // k = last, i = p, j = q
  }
}

}  // namespace dgfv
