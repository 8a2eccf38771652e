// Device-side equation of state, two-point volume fluxes and Riemann solvers.
//
// Conservative state u = (rho, rho v1, rho v2, rho v3, rho e[, rho Y1]) of the
// inviscid part of eq. ns_equation.  Pressure from eq. eos with the mixture
// ratio of eq. mix_R_kappa / eq. mix_cp_cv for two species.  All fluxes are
// returned already contracted with an (unnormalised) direction vector.
//
// The state-dependent functions are templated on the scalar type S (double,
// or a forward-mode Dual<K> for local Jacobians in the adjoint kernels).
#pragma once

#include "dgfv_dual.h"
#include "dgfv_internal.h"

namespace dgfv {

__host__ __device__ inline double sqrt(double x) { return ::sqrt(x); }
__host__ __device__ inline double log(double x) { return ::log(x); }
__host__ __device__ inline double fabs(double x) { return ::fabs(x); }
__host__ __device__ inline double fmax(double a, double b) { return ::fmax(a, b); }

template <class S>
struct PrimT {
  S rho, v1, v2, v3, p, E, kap, Y;
};
using Prim = PrimT<double>;

__device__ __forceinline__ double kappa_mix(double Y, const GasDev& g) {
  const double Y2 = 1.0 - Y;
  return (Y * g.cp0 + Y2 * g.cp1) / (Y * g.cv0 + Y2 * g.cv1);
}

template <int NV, class S>
__device__ __forceinline__ PrimT<S> cons2prim(const S* u, const GasDev& g) {
  PrimT<S> q;
  q.rho = u[0];
  const S ir = 1.0 / q.rho;
  q.v1 = u[1] * ir;
  q.v2 = u[2] * ir;
  q.v3 = u[3] * ir;
  q.E = u[4];
  if constexpr (NV == 6) {
    q.Y = u[5] * ir;
    const S Y2 = 1.0 - q.Y;
    q.kap = (q.Y * g.cp0 + Y2 * g.cp1) / (q.Y * g.cv0 + Y2 * g.cv1);
  } else {
    q.Y = S(0.0);
    q.kap = S(g.gamma);
  }
  q.p = (q.kap - 1.0) * (q.E - 0.5 * q.rho * (q.v1 * q.v1 + q.v2 * q.v2 + q.v3 * q.v3));
  return q;
}

// Primitive vector w = (rho, v1, v2, v3, p[, Y1]) of a conservative state, and back.
template <int NV>
__device__ __forceinline__ void cons_to_w(const double* u, const GasDev& g, double* w) {
  const PrimT<double> q = cons2prim<NV>(u, g);
  w[0] = q.rho;
  w[1] = q.v1;
  w[2] = q.v2;
  w[3] = q.v3;
  w[4] = q.p;
  if constexpr (NV == 6) w[5] = q.Y;
}

template <int NV>
__device__ __forceinline__ void w_to_cons(const double* w, const GasDev& g, double* u) {
  double kap = g.gamma;
  if constexpr (NV == 6) kap = kappa_mix(w[5], g);
  u[0] = w[0];
  u[1] = w[0] * w[1];
  u[2] = w[0] * w[2];
  u[3] = w[0] * w[3];
  u[4] = w[4] / (kap - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  if constexpr (NV == 6) u[5] = w[0] * w[5];
}

// minmod(a, b): the argument of smaller magnitude where both have one sign, else 0.
__device__ __forceinline__ double minmod(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return a > 0.0 ? (a < b ? a : b) : (a > b ? a : b);
}

// Physical flux F(u) . a
template <int NV, class S>
__device__ __forceinline__ void euler_flux(const PrimT<S>& q, double a1, double a2, double a3, S* f) {
  const S vn = q.v1 * a1 + q.v2 * a2 + q.v3 * a3;
  const S m = q.rho * vn;
  f[0] = m;
  f[1] = m * q.v1 + q.p * a1;
  f[2] = m * q.v2 + q.p * a2;
  f[3] = m * q.v3 + q.p * a3;
  f[4] = (q.E + q.p) * vn;
  if constexpr (NV == 6) f[5] = m * q.Y;
}

// Logarithmic mean (a - b) / (ln a - ln b) from precomputed logarithms, with the
// Ismail-Roe series F = 1 + u/3 + u^2/5 + u^3/7, u = ((a-b)/(a+b))^2, below u = 1e-4.
template <class S>
__device__ __forceinline__ S log_mean(const S& a, const S& b, const S& la, const S& lb) {
  const S s = a + b;
  const S f = (a - b) / s;
  const S u = f * f;
  if (u < 1e-4) {
    const S F = 1.0 + u * (1.0 / 3.0 + u * (0.2 + u * (1.0 / 7.0)));
    return s / (2.0 * F);
  }
  return (a - b) / (la - lb);
}

// Partial derivatives of log_mean with respect to its first value and first logarithm.
// 1/x from the hardware estimate (v_rcp_f64) refined by two Newton-Raphson
// steps, e = 1 - x r, r <- r + r e: within about one ulp, not correctly rounded.
// x must be finite and nonzero.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double log_mean_d(double a, double b, double la, double lb, double& d_a,
                                             double& d_la) {
  const double s = a + b;
  const double is = rcp_nr(s);
  const double f = (a - b) * is;
  const double u = f * f;
  if (u < 1e-4) {
    const double F = 1.0 + u * (1.0 / 3.0 + u * (0.2 + u * (1.0 / 7.0)));
    const double dF = 1.0 / 3.0 + u * (0.4 + u * (3.0 / 7.0));
    const double iF = rcp_nr(F);
    const double dfa = 2.0 * b * is * is;
    const double lm = 0.5 * s * iF;
    d_a = 0.5 * iF - lm * iF * dF * (2.0 * f * dfa);
    d_la = 0.0;
    return lm;
  }
  const double il = rcp_nr(la - lb);
  const double lm = (a - b) * il;
  d_a = il;
  d_la = -lm * il;
  return lm;
}

// ---------------------------------------------------------------------------
// Per-node auxiliary records of the volume two-point fluxes.  Each kind stores
// NA doubles per node in LDS (structure of arrays) and evaluates
// f#(u_i, u_m) . a from two records.  For the adjoint each kind also provides
//   flux_adj_a : abar += (d f# / d a_record)^T c     (first argument)
//   make_adj   : ubar  = (d record / d u)^T abar
// ---------------------------------------------------------------------------

// Ranocha's entropy-conserving, kinetic-energy-preserving flux (single species).
struct FluxRanocha {
  static constexpr int NA = 8;  // rho, v1, v2, v3, p, ln rho, beta = rho/p, ln beta
  template <int NV, class S>
  __device__ __forceinline__ static void make(const PrimT<S>& q, S* r) {
    r[0] = q.rho; r[1] = q.v1; r[2] = q.v2; r[3] = q.v3; r[4] = q.p;
    r[5] = log(q.rho);
    const S beta = q.rho / q.p;
    r[6] = beta;
    r[7] = log(beta);
  }
  // Double-precision evaluation with one reciprocal (rcp_nr) per logarithmic mean.
  // rho_ln: near-equal arguments use (a+b)/2 times the reciprocal of the
  // Ismail-Roe series, 1/F(u) = 1 - u/3 - 4u^2/45 - 44u^3/945 + O(u^4), with
  // u = ((a-b)/(a+b))^2; otherwise (a-b)/(ln a - ln b).  The energy flux needs
  // 1/beta_ln, formed directly as 2F(u)/(a+b) or (ln a - ln b)/(a-b).  Both
  // arguments are positive, so u < 1e-4 is tested as |a-b| < 0.01 (a+b).
  // flux_fast returns TWICE the flux: the arithmetic means then cost one add
  // each, and the caller's weights carry the factor 1/2 (FAST_WEIGHT).
  static constexpr double FAST_WEIGHT = 0.5;
  template <int NV>
  __device__ __forceinline__ static void flux_fast(const double* a_, const double* b_, double a1,
                                                   double a2, double a3, const GasDev& g, double* f) {
    double rho_ln, ibeta_ln;
    {
      const double s = a_[0] + b_[0], d = a_[0] - b_[0], dl = a_[5] - b_[5];
      const bool small = fabs(d) < 1e-2 * s;
      const double r = rcp_nr(small ? s : dl);
      const double u = (d * r) * (d * r);
      const double iF = 1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0)));
      rho_ln = small ? 0.5 * s * iF : d * r;
    }
    {
      const double s = a_[6] + b_[6], d = a_[6] - b_[6], dl = a_[7] - b_[7];
      const bool small = fabs(d) < 1e-2 * s;
      const double r = rcp_nr(small ? s : d);
      const double u = (d * r) * (d * r);
      const double F = 1.0 + u * (1.0 / 3.0 + u * (0.2 + u * (1.0 / 7.0)));
      ibeta_ln = small ? 2.0 * F * r : dl * r;
    }
    // normal velocities of both states; 2 vn = vna + vnb
    const double vna = a_[1] * a1 + a_[2] * a2 + a_[3] * a3;
    const double vnb = b_[1] * a1 + b_[2] * a2 + b_[3] * a3;
    const double f0 = rho_ln * (vna + vnb);      // 2 rho_ln vn
    const double fr = 0.5 * f0;                   // rho_ln vn
    const double sp = a_[4] + b_[4];              // 2 pbar
    f[0] = f0;
    f[1] = fr * (a_[1] + b_[1]) + sp * a1;        // 2 (rho_ln vn v1 + pbar a1)
    f[2] = fr * (a_[2] + b_[2]) + sp * a2;
    f[3] = fr * (a_[3] + b_[3]) + sp * a3;
    const double vab = a_[1] * b_[1] + a_[2] * b_[2] + a_[3] * b_[3];
    const double igm1 = 1.0 / (g.gamma - 1.0);
    // 2 [rho_ln vn (1/((gamma-1) beta_ln) + vab/2) + (p_a vnb + p_b vna)/2]
    f[4] = f0 * (ibeta_ln * igm1) + fr * vab + (a_[4] * vnb + b_[4] * vna);
  }
  template <int NV, class S>
  __device__ __forceinline__ static void flux(const S* a_, const S* b_, double a1, double a2,
                                              double a3, const GasDev& g, S* f) {
    const S rho_ln = log_mean(a_[0], b_[0], a_[5], b_[5]);
    const S beta_ln = log_mean(a_[6], b_[6], a_[7], b_[7]);
    const S v1 = 0.5 * (a_[1] + b_[1]), v2 = 0.5 * (a_[2] + b_[2]), v3 = 0.5 * (a_[3] + b_[3]);
    const S pbar = 0.5 * (a_[4] + b_[4]);
    const S vn = v1 * a1 + v2 * a2 + v3 * a3;
    const S fr = rho_ln * vn;
    f[0] = fr;
    f[1] = fr * v1 + pbar * a1;
    f[2] = fr * v2 + pbar * a2;
    f[3] = fr * v3 + pbar * a3;
    const S vv = 0.5 * (a_[1] * b_[1] + a_[2] * b_[2] + a_[3] * b_[3]);
    const S vna = a_[1] * a1 + a_[2] * a2 + a_[3] * a3;
    const S vnb = b_[1] * a1 + b_[2] * a2 + b_[3] * a3;
    f[4] = fr * (1.0 / ((g.gamma - 1.0) * beta_ln) + vv) + 0.5 * (a_[4] * vnb + b_[4] * vna);
  }
  template <int NV>
  __device__ __forceinline__ static void flux_adj_a(const double* a_, const double* b_, double n1,
                                                    double n2, double n3, const GasDev& g,
                                                    const double* c, double* ab) {
    double drho_a, drho_la, dbeta_a, dbeta_la;
    const double rho_ln = log_mean_d(a_[0], b_[0], a_[5], b_[5], drho_a, drho_la);
    const double beta_ln = log_mean_d(a_[6], b_[6], a_[7], b_[7], dbeta_a, dbeta_la);
    const double v1 = 0.5 * (a_[1] + b_[1]), v2 = 0.5 * (a_[2] + b_[2]), v3 = 0.5 * (a_[3] + b_[3]);
    const double vn = v1 * n1 + v2 * n2 + v3 * n3;
    const double fr = rho_ln * vn;
    const double gm1 = g.gamma - 1.0;
    const double ib = rcp_nr(gm1 * beta_ln);
    const double vv = 0.5 * (a_[1] * b_[1] + a_[2] * b_[2] + a_[3] * b_[3]);
    const double vnb = b_[1] * n1 + b_[2] * n2 + b_[3] * n3;
    const double frb = c[0] + c[1] * v1 + c[2] * v2 + c[3] * v3 + c[4] * (ib + vv);
    const double pbarb = c[1] * n1 + c[2] * n2 + c[3] * n3;
    const double betab = -c[4] * fr * gm1 * ib * ib;
    const double vvb = c[4] * fr;
    const double vnab = 0.5 * c[4] * b_[4];
    const double rholnb = frb * vn;
    const double vnbar = frb * rho_ln;
    ab[0] += rholnb * drho_a;
    ab[5] += rholnb * drho_la;
    ab[6] += betab * dbeta_a;
    ab[7] += betab * dbeta_la;
    ab[1] += 0.5 * (c[1] * fr + vnbar * n1) + 0.5 * vvb * b_[1] + vnab * n1;
    ab[2] += 0.5 * (c[2] * fr + vnbar * n2) + 0.5 * vvb * b_[2] + vnab * n2;
    ab[3] += 0.5 * (c[3] * fr + vnbar * n3) + 0.5 * vvb * b_[3] + vnab * n3;
    ab[4] += 0.5 * pbarb + 0.5 * c[4] * vnb;
  }
  template <int NV>
  __device__ __forceinline__ static void make_adj(const double* u, const GasDev& g, const double* ab,
                                                  double* ub) {
    const double rho = u[0], ir = 1.0 / rho;
    const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
    const double gm1 = g.gamma - 1.0;
    const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
    const double p = gm1 * (u[4] - 0.5 * rho * vsq);
    const double beta = rho / p;
    const double betab = ab[6] + ab[7] / beta;
    double rhob = ab[0] + ab[5] * ir + betab / p;
    const double pb = ab[4] - betab * beta / p;
    // p = (gamma-1) (E - |m|^2 / (2 rho))
    ub[4] = gm1 * pb;
    double m1b = -gm1 * pb * v1, m2b = -gm1 * pb * v2, m3b = -gm1 * pb * v3;
    rhob += gm1 * pb * 0.5 * vsq;
    // v = m / rho
    m1b += ab[1] * ir;
    m2b += ab[2] * ir;
    m3b += ab[3] * ir;
    rhob -= (ab[1] * v1 + ab[2] * v2 + ab[3] * v3) * ir;
    ub[0] = rhob;
    ub[1] = m1b;
    ub[2] = m2b;
    ub[3] = m3b;
  }
};

// Chain rule of (rho, v, p, E, Y) with respect to u, shared by the Pirozzoli
// and central records: given bars of rho, v, p, E, Y accumulate ub.
template <int NV>
__device__ __forceinline__ void prim_adj(const double* u, const GasDev& g, double rhob, double v1b,
                                         double v2b, double v3b, double pb, double Eb, double Yb,
                                         double* ub) {
  const double rho = u[0], ir = 1.0 / rho;
  const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
  const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
  const double qe = u[4] - 0.5 * rho * vsq;                // p = (kappa - 1) qe
  double kap = g.gamma;
  double Y = 0.0;
  if constexpr (NV == 6) {
    Y = u[5] * ir;
    const double num = Y * g.cp0 + (1.0 - Y) * g.cp1, den = Y * g.cv0 + (1.0 - Y) * g.cv1;
    kap = num / den;
    const double dkdY = ((g.cp0 - g.cp1) * den - num * (g.cv0 - g.cv1)) / (den * den);
    Yb += pb * qe * dkdY;
  }
  const double qb = (kap - 1.0) * pb;
  Eb += qb;
  double m1b = -qb * v1, m2b = -qb * v2, m3b = -qb * v3;
  rhob += qb * 0.5 * vsq;
  m1b += v1b * ir;
  m2b += v2b * ir;
  m3b += v3b * ir;
  rhob -= (v1b * v1 + v2b * v2 + v3b * v3) * ir;
  if constexpr (NV == 6) {
    ub[5] = Yb * ir;
    rhob -= Yb * Y * ir;
  }
  ub[0] = rhob;
  ub[1] = m1b;
  ub[2] = m2b;
  ub[3] = m3b;
  ub[4] = Eb;
}

// Pirozzoli's kinetic-energy-preserving flux (Section 3.5); f_rhoY = f_rho {Y}.
struct FluxPirozzoli {
  static constexpr int NA = 7;  // rho, v1, v2, v3, p, H, Y
  static constexpr double FAST_WEIGHT = 1.0;   // flux_fast is the flux itself
  template <int NV>
  __device__ __forceinline__ static void flux_fast(const double* a_, const double* b_, double a1,
                                                   double a2, double a3, const GasDev& g, double* f) {
    flux<NV>(a_, b_, a1, a2, a3, g, f);
  }
  template <int NV, class S>
  __device__ __forceinline__ static void make(const PrimT<S>& q, S* r) {
    r[0] = q.rho; r[1] = q.v1; r[2] = q.v2; r[3] = q.v3; r[4] = q.p;
    r[5] = (q.E + q.p) / q.rho;
    r[6] = q.Y;
  }
  template <int NV, class S>
  __device__ __forceinline__ static void flux(const S* a_, const S* b_, double a1, double a2,
                                              double a3, const GasDev&, S* f) {
    const S rho = 0.5 * (a_[0] + b_[0]);
    const S v1 = 0.5 * (a_[1] + b_[1]), v2 = 0.5 * (a_[2] + b_[2]), v3 = 0.5 * (a_[3] + b_[3]);
    const S pbar = 0.5 * (a_[4] + b_[4]);
    const S fr = rho * (v1 * a1 + v2 * a2 + v3 * a3);
    f[0] = fr;
    f[1] = fr * v1 + pbar * a1;
    f[2] = fr * v2 + pbar * a2;
    f[3] = fr * v3 + pbar * a3;
    f[4] = fr * (0.5 * (a_[5] + b_[5]));
    if constexpr (NV == 6) f[5] = fr * (0.5 * (a_[6] + b_[6]));
  }
  template <int NV>
  __device__ __forceinline__ static void flux_adj_a(const double* a_, const double* b_, double n1,
                                                    double n2, double n3, const GasDev&,
                                                    const double* c, double* ab) {
    const double rho = 0.5 * (a_[0] + b_[0]);
    const double v1 = 0.5 * (a_[1] + b_[1]), v2 = 0.5 * (a_[2] + b_[2]), v3 = 0.5 * (a_[3] + b_[3]);
    const double vn = v1 * n1 + v2 * n2 + v3 * n3;
    const double fr = rho * vn;
    const double Hbar = 0.5 * (a_[5] + b_[5]);
    double frb = c[0] + c[1] * v1 + c[2] * v2 + c[3] * v3 + c[4] * Hbar;
    double Yb = 0.0;
    if constexpr (NV == 6) {
      frb += c[5] * 0.5 * (a_[6] + b_[6]);
      Yb = c[5] * fr;
    }
    const double vnb = frb * rho;
    ab[0] += 0.5 * frb * vn;
    ab[1] += 0.5 * (c[1] * fr + vnb * n1);
    ab[2] += 0.5 * (c[2] * fr + vnb * n2);
    ab[3] += 0.5 * (c[3] * fr + vnb * n3);
    ab[4] += 0.5 * (c[1] * n1 + c[2] * n2 + c[3] * n3);
    ab[5] += 0.5 * c[4] * fr;
    ab[6] += 0.5 * Yb;
  }
  template <int NV>
  __device__ __forceinline__ static void make_adj(const double* u, const GasDev& g, const double* ab,
                                                  double* ub) {
    // H = (E + p) / rho
    const double ir = 1.0 / u[0];
    const PrimT<double> q = cons2prim<NV>(u, g);
    const double H = (q.E + q.p) * ir;
    const double Hb = ab[5];
    prim_adj<NV>(u, g, ab[0] - Hb * H * ir, ab[1], ab[2], ab[3], ab[4] + Hb * ir, Hb * ir, ab[6], ub);
  }
};

// Arithmetic mean of the physical fluxes.
struct FluxCentral {
  static constexpr int NA = 7;  // rho, v1, v2, v3, p, E, Y
  static constexpr double FAST_WEIGHT = 1.0;   // flux_fast is the flux itself
  template <int NV>
  __device__ __forceinline__ static void flux_fast(const double* a_, const double* b_, double a1,
                                                   double a2, double a3, const GasDev& g, double* f) {
    flux<NV>(a_, b_, a1, a2, a3, g, f);
  }
  template <int NV, class S>
  __device__ __forceinline__ static void make(const PrimT<S>& q, S* r) {
    r[0] = q.rho; r[1] = q.v1; r[2] = q.v2; r[3] = q.v3; r[4] = q.p; r[5] = q.E; r[6] = q.Y;
  }
  template <int NV, class S>
  __device__ __forceinline__ static void flux(const S* a_, const S* b_, double a1, double a2,
                                              double a3, const GasDev&, S* f) {
    const S vna = a_[1] * a1 + a_[2] * a2 + a_[3] * a3;
    const S vnb = b_[1] * a1 + b_[2] * a2 + b_[3] * a3;
    const S ma = a_[0] * vna, mb = b_[0] * vnb;
    f[0] = 0.5 * (ma + mb);
    f[1] = 0.5 * (ma * a_[1] + a_[4] * a1 + mb * b_[1] + b_[4] * a1);
    f[2] = 0.5 * (ma * a_[2] + a_[4] * a2 + mb * b_[2] + b_[4] * a2);
    f[3] = 0.5 * (ma * a_[3] + a_[4] * a3 + mb * b_[3] + b_[4] * a3);
    f[4] = 0.5 * ((a_[5] + a_[4]) * vna + (b_[5] + b_[4]) * vnb);
    if constexpr (NV == 6) f[5] = 0.5 * (ma * a_[6] + mb * b_[6]);
  }
  template <int NV>
  __device__ __forceinline__ static void flux_adj_a(const double* a_, const double*, double n1,
                                                    double n2, double n3, const GasDev&,
                                                    const double* c, double* ab) {
    const double vna = a_[1] * n1 + a_[2] * n2 + a_[3] * n3;
    const double ma = a_[0] * vna;
    double mab = 0.5 * (c[0] + c[1] * a_[1] + c[2] * a_[2] + c[3] * a_[3]);
    if constexpr (NV == 6) {
      mab += 0.5 * c[5] * a_[6];
      ab[6] += 0.5 * c[5] * ma;
    }
    const double vnab = mab * a_[0] + 0.5 * c[4] * (a_[5] + a_[4]);
    ab[0] += mab * vna;
    ab[1] += 0.5 * c[1] * ma + vnab * n1;
    ab[2] += 0.5 * c[2] * ma + vnab * n2;
    ab[3] += 0.5 * c[3] * ma + vnab * n3;
    ab[4] += 0.5 * (c[1] * n1 + c[2] * n2 + c[3] * n3) + 0.5 * c[4] * vna;
    ab[5] += 0.5 * c[4] * vna;
  }
  template <int NV>
  __device__ __forceinline__ static void make_adj(const double* u, const GasDev& g, const double* ab,
                                                  double* ub) {
    prim_adj<NV>(u, g, ab[0], ab[1], ab[2], ab[3], ab[4], ab[5], ab[6], ub);
  }
};

// Two-point flux of the chosen volume kind evaluated from conservative states
// (used at faces with the EC selector).
template <int NV, class S>
__device__ __forceinline__ void two_point_cons(int kind, const S* uL, const S* uR, double n1,
                                               double n2, double n3, const GasDev& g, S* F) {
  const PrimT<S> qL = cons2prim<NV>(uL, g), qR = cons2prim<NV>(uR, g);
  S ra[8], rb[8];
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
template <int NV, class S>
__device__ __forceinline__ void riemann_llf(const S* uL, const S* uR, double n1, double n2, double n3,
                                            const GasDev& g, S* F) {
  const double s = ::sqrt(n1 * n1 + n2 * n2 + n3 * n3);
  const double is = 1.0 / s;
  const double e1 = n1 * is, e2 = n2 * is, e3 = n3 * is;
  const PrimT<S> qL = cons2prim<NV>(uL, g), qR = cons2prim<NV>(uR, g);
  const S cL = sqrt(qL.kap * qL.p / qL.rho), cR = sqrt(qR.kap * qR.p / qR.rho);
  const S lam = fmax(fabs(qL.v1 * e1 + qL.v2 * e2 + qL.v3 * e3) + cL,
                     fabs(qR.v1 * e1 + qR.v2 * e2 + qR.v3 * e3) + cR);
  S fL[NV], fR[NV];
  euler_flux<NV>(qL, e1, e2, e3, fL);
  euler_flux<NV>(qR, e1, e2, e3, fR);
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = (0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v])) * s;
}

// Harten-Hyman entropy fix on an acoustic wave speed.
template <class S>
__device__ __forceinline__ S hh_fix(const S& lam, const S& lamL, const S& lamR) {
  const S delta = fmax(0.0, fmax(lam - lamL, lamR - lam));
  const S al = fabs(lam);
  return (al < delta) ? 0.5 * (lam * lam / delta + delta) : al;
}

// Roe flux with the Harten-Hyman entropy fix on the acoustic waves, times |nvec| (1 species).
template <class S>
__device__ __forceinline__ void riemann_roe(const S* uL, const S* uR, double n1, double n2, double n3,
                                            const GasDev& g, S* F) {
  const double s = ::sqrt(n1 * n1 + n2 * n2 + n3 * n3);
  const double is = 1.0 / s;
  const double e1 = n1 * is, e2 = n2 * is, e3 = n3 * is;
  const PrimT<S> qL = cons2prim<5>(uL, g), qR = cons2prim<5>(uR, g);
  const double gm1 = g.gamma - 1.0;
  const S sL = sqrt(qL.rho), sR = sqrt(qR.rho);
  const S iw = 1.0 / (sL + sR);
  const S v1 = (sL * qL.v1 + sR * qR.v1) * iw;
  const S v2 = (sL * qL.v2 + sR * qR.v2) * iw;
  const S v3 = (sL * qL.v3 + sR * qR.v3) * iw;
  const S HL = (qL.E + qL.p) / qL.rho, HR = (qR.E + qR.p) / qR.rho;
  const S H = (sL * HL + sR * HR) * iw;
  const S vsq = v1 * v1 + v2 * v2 + v3 * v3;
  const S c2 = gm1 * (H - 0.5 * vsq);
  const S c = sqrt(c2);
  const S rt = sL * sR;
  const S vn = v1 * e1 + v2 * e2 + v3 * e3;

  const S drho = qR.rho - qL.rho, dp = qR.p - qL.p;
  const S d1 = qR.v1 - qL.v1, d2 = qR.v2 - qL.v2, d3 = qR.v3 - qL.v3;
  const S dvn = d1 * e1 + d2 * e2 + d3 * e3;
  const S a1 = (dp - rt * c * dvn) / (2.0 * c2);
  const S a5 = (dp + rt * c * dvn) / (2.0 * c2);
  const S a2 = drho - dp / c2;
  const S t1 = d1 - dvn * e1, t2 = d2 - dvn * e2, t3 = d3 - dvn * e3;

  const S cL = sqrt(qL.kap * qL.p / qL.rho), cR = sqrt(qR.kap * qR.p / qR.rho);
  const S vnL = qL.v1 * e1 + qL.v2 * e2 + qL.v3 * e3;
  const S vnR = qR.v1 * e1 + qR.v2 * e2 + qR.v3 * e3;
  const S l1 = hh_fix(vn - c, vnL - cL, vnR - cR);
  const S l5 = hh_fix(vn + c, vnL + cL, vnR + cR);
  const S l2 = fabs(vn);

  const S w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2, wt = l2 * rt;
  S D[5];
  D[0] = w1 + w5 + w2;
  D[1] = w1 * (v1 - c * e1) + w5 * (v1 + c * e1) + w2 * v1 + wt * t1;
  D[2] = w1 * (v2 - c * e2) + w5 * (v2 + c * e2) + w2 * v2 + wt * t2;
  D[3] = w1 * (v3 - c * e3) + w5 * (v3 + c * e3) + w2 * v3 + wt * t3;
  D[4] = w1 * (H - c * vn) + w5 * (H + c * vn) + w2 * (0.5 * vsq) + wt * (v1 * t1 + v2 * t2 + v3 * t3);

  S fL[5], fR[5];
  euler_flux<5>(qL, e1, e2, e3, fL);
  euler_flux<5>(qR, e1, e2, e3, fR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = (0.5 * (fL[v] + fR[v]) - 0.5 * D[v]) * s;
}

template <int NV, class S>
__device__ __forceinline__ void riemann(int kind, int vol_kind, const S* uL, const S* uR, double n1,
                                        double n2, double n3, const GasDev& g, S* F) {
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

// (dF*/duL)^T Fb and (dF*/duR)^T Fb of the Riemann flux, by forward-mode duals.
template <int NV>
__device__ __forceinline__ void riemann_vjp(int kind, int vol_kind, const double* uL, const double* uR,
                                            double n1, double n2, double n3, const GasDev& g,
                                            const double* Fb, double* uLb, double* uRb) {
  using D = Dual<NV>;
  D a[NV], b[NV], F[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    a[v] = D::seed(uL[v], v);
    b[v] = D(uR[v]);
  }
  riemann<NV>(kind, vol_kind, a, b, n1, n2, n3, g, F);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s += F[v].d[k] * Fb[v];
    uLb[k] = s;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    a[v] = D(uL[v]);
    b[v] = D::seed(uR[v], v);
  }
  riemann<NV>(kind, vol_kind, a, b, n1, n2, n3, g, F);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s += F[v].d[k] * Fb[v];
    uRb[k] = s;
  }
}

// One side of riemann_vjp: (dF*/du_side)^T Fb with side 0 = left, 1 = right.
template <int NV>
__device__ __forceinline__ void riemann_vjp_side(int side, int kind, int vol_kind, const double* uL,
                                                 const double* uR, double n1, double n2, double n3,
                                                 const GasDev& g, const double* Fb, double* ub) {
  using D = Dual<NV>;
  D a[NV], b[NV], F[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    a[v] = side == 0 ? D::seed(uL[v], v) : D(uL[v]);
    b[v] = side == 1 ? D::seed(uR[v], v) : D(uR[v]);
  }
  riemann<NV>(kind, vol_kind, a, b, n1, n2, n3, g, F);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s += F[v].d[k] * Fb[v];
    ub[k] = s;
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

// Viscous fluxes F^v_x (x = 0, 1, 2) at one point from the state u and its
// gradient gr[x][v] = d u_v / d x_x (Section 2): with the flux on the
// left-hand side, F^v_x = -(0, tau_x., (tau v)_x - q_h,x - q_d,x, -J_1,x),
// tau = mu (grad v + grad v^T - 2/3 div v I), q_h = -lambda grad T, and for
// two species J_1 = -rho grad Y1 (D_1 Y2 + D_2 Y1) = -J_2 (Fick's law with
// the mass-conserving correction) and q_d = (c_p,1 - c_p,2) T J_1.  Velocity,
// temperature and mass-fraction gradients follow from grad u by the chain
// rule.  One species: T = (gamma - 1) e_int with unit gas constant, which
// cancels in lambda grad T = mu c_p grad T / Pr.
template <int NV>
__device__ __forceinline__ void viscous_flux(const double (&u)[NV], const double (&gr)[3][NV], const GasDev& gas,
                                             const ViscDev& tr, double (&f)[3][NV]) {
  const double ir = 1.0 / u[0];
  const double w[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  const double es = u[4] * ir;
  const double eint = es - 0.5 * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double gw[3][3];                         // gw[x][i] = d v_i / d x_x
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int i = 0; i < 3; ++i) gw[x][i] = (gr[x][1 + i] - w[i] * gr[x][0]) * ir;
  double cv, cp, mu, Pr, Y = 0.0, dcv = 0.0, dcp = 0.0, Dm = 0.0;
  if constexpr (NV == 6) {
    Y = u[5] * ir;
    const double Y2 = 1.0 - Y;
    cv = Y * gas.cv0 + Y2 * gas.cv1;
    cp = Y * gas.cp0 + Y2 * gas.cp1;
    mu = Y * tr.mu0 + Y2 * tr.mu1;
    Pr = Y * tr.Pr0 + Y2 * tr.Pr1;
    dcv = gas.cv0 - gas.cv1;
    dcp = gas.cp0 - gas.cp1;
    Dm = tr.D0 * Y2 + tr.D1 * Y;
  } else {
    cv = 1.0 / (gas.gamma - 1.0);
    cp = gas.gamma * cv;
    mu = tr.mu0;
    Pr = tr.Pr0;
  }
  const double T = eint / cv;
  const double lam = mu * cp / Pr;
  const double div3 = (2.0 / 3.0) * (gw[0][0] + gw[1][1] + gw[2][2]);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    double tau[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) tau[i] = mu * (gw[x][i] + gw[i][x] - (i == x ? div3 : 0.0));
    const double geint = (gr[x][4] - es * gr[x][0]) * ir - (w[0] * gw[x][0] + w[1] * gw[x][1] + w[2] * gw[x][2]);
    double gT, qd = 0.0;
    if constexpr (NV == 6) {
      const double gY = (gr[x][5] - Y * gr[x][0]) * ir;
      gT = (geint - T * dcv * gY) / cv;
      const double J1 = -u[0] * gY * Dm;
      qd = dcp * T * J1;
      f[x][5] = J1;
    } else {
      gT = geint / cv;
    }
    f[x][0] = 0.0;
    f[x][1] = -tau[0];
    f[x][2] = -tau[1];
    f[x][3] = -tau[2];
    f[x][4] = -(tau[0] * w[0] + tau[1] * w[1] + tau[2] * w[2]) - lam * gT + qd;
  }
}

}  // namespace dgfv
