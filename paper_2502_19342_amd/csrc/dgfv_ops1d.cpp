// One-dimensional operators of the collocated DGSEM and of the FV sub-cell maps,
// computed in long double and rounded once to double.
//
//  * LGL nodes: +-1 and the roots of P_N' (Newton on the Legendre recurrence);
//    weights 2 / (N (N+1) P_N(x_i)^2)  (Section 3.1.1, LGL collocation);
//  * D_ij = l_j'(x_i) by the barycentric formula, diagonal from the row sums
//    (eq. dgsem_abbrev);
//  * V_Leg: orthonormal Legendre polynomials at the nodes (Section 3.4);
//  * V^{N->M}: Lagrange interpolation; V^{M->N} = V^N_Leg [I 0] (V^M_Leg)^{-1}
//    (Section 3.2, degree change);
//  * V^{DG->FV}: sub-cell means of l_j, integrated exactly through the
//    Legendre expansion of l_j and the antiderivative (P_{k+1} - P_{k-1})/(2k+1);
//    V^{FV->DG} = (V^T V)^{-1} V^T (Section 3.2, DG/FV switch);
//  * face_interp: l_j at the N_FV + 1 sub-cell interfaces.
#include "dgfv_ops1d.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace dgfv {

using LD = long double;

static void legendre(int n, LD x, LD& p, LD& dp) {
  if (n == 0) {
    p = 1.0L;
    dp = 0.0L;
    return;
  }
  LD p0 = 1.0L, p1 = x;
  for (int k = 2; k <= n; ++k) {
    LD p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  if (std::fabs(x) == 1.0L) {
    // P_n'(1) = n(n+1)/2 and P_n'(-1) = (-1)^(n+1) n(n+1)/2
    dp = 0.5L * n * (n + 1) * ((x < 0 && (n % 2 == 0)) ? -1.0L : 1.0L);
  } else {
    dp = n * (x * p1 - p0) / (x * x - 1.0L);
  }
}

static LD legendre_p(int n, LD x) {
  LD p, dp;
  legendre(n, x, p, dp);
  return p;
}

std::vector<LD> lgl_nodes(int N) {
  std::vector<LD> x(N + 1);
  x[0] = -1.0L;
  x[N] = 1.0L;
  const LD pi = 3.141592653589793238462643383279502884L;
  for (int j = 1; j < N; ++j) {
    LD z = -std::cos(pi * j / N);
    for (int it = 0; it < 100; ++it) {
      LD p, dp;
      legendre(N, z, p, dp);
      const LD ddp = (2.0L * z * dp - N * (N + 1) * p) / (1.0L - z * z);
      const LD dz = dp / ddp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    x[j] = z;
  }
  // exact symmetry
  for (int j = 0; j <= N / 2; ++j) {
    const LD s = 0.5L * (x[N - j] - x[j]);
    x[j] = -s;
    x[N - j] = s;
  }
  if (N % 2 == 0) x[N / 2] = 0.0L;
  return x;
}

std::vector<LD> lgl_weights(int N) {
  const auto x = lgl_nodes(N);
  std::vector<LD> w(N + 1);
  for (int i = 0; i <= N; ++i) {
    const LD p = legendre_p(N, x[i]);
    w[i] = 2.0L / (N * (N + 1) * p * p);
  }
  return w;
}

static LD lagrange(const std::vector<LD>& x, int j, LD t) {
  LD v = 1.0L;
  for (size_t k = 0; k < x.size(); ++k)
    if ((int)k != j) v *= (t - x[k]) / (x[j] - x[k]);
  return v;
}

static std::vector<LD> inverse(std::vector<LD> A, int n) {
  std::vector<LD> I(n * n, 0.0L);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0L;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0L) throw std::runtime_error("singular matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(I[c * n + k], I[piv * n + k]);
    }
    const LD d = 1.0L / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= d;
      I[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const LD f = A[r * n + c];
      if (f == 0.0L) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        I[r * n + k] -= f * I[c * n + k];
      }
    }
  }
  return I;
}

static std::vector<double> to_double(const std::vector<LD>& a) {
  std::vector<double> r(a.size());
  for (size_t i = 0; i < a.size(); ++i) r[i] = (double)a[i];
  return r;
}

static std::vector<LD> dmat_ld(int N) {
  const auto x = lgl_nodes(N);
  const int n = N + 1;
  std::vector<LD> bw(n);
  for (int j = 0; j < n; ++j) {
    LD p = 1.0L;
    for (int k = 0; k < n; ++k)
      if (k != j) p *= (x[j] - x[k]);
    bw[j] = 1.0L / p;
  }
  std::vector<LD> D(n * n, 0.0L);
  for (int i = 0; i < n; ++i) {
    LD s = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      D[i * n + j] = (bw[j] / bw[i]) / (x[i] - x[j]);
      s += D[i * n + j];
    }
    D[i * n + i] = -s;
  }
  return D;
}

static std::vector<LD> vleg_ld(int N) {
  const auto x = lgl_nodes(N);
  const int n = N + 1;
  std::vector<LD> V(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = std::sqrt((2.0L * j + 1.0L) / 2.0L) * legendre_p(j, x[i]);
  return V;
}

std::vector<double> op_weights(int N) { return to_double(lgl_weights(N)); }
std::vector<double> op_nodes(int N) { return to_double(lgl_nodes(N)); }
std::vector<double> op_D(int N) { return to_double(dmat_ld(N)); }
std::vector<double> op_vleg_inv(int N) { return to_double(inverse(vleg_ld(N), N + 1)); }

std::vector<LD> ld_D(int N) { return dmat_ld(N); }

std::vector<LD> ld_interp(int N, int M) {
  const auto xN = lgl_nodes(N), xM = lgl_nodes(M);
  std::vector<LD> V((M + 1) * (N + 1));
  for (int i = 0; i <= M; ++i)
    for (int j = 0; j <= N; ++j) V[i * (N + 1) + j] = lagrange(xN, j, xM[i]);
  return V;
}

std::vector<double> op_interp(int N, int M) { return to_double(ld_interp(N, M)); }

std::vector<double> op_project(int M, int N) {
  const auto VN = vleg_ld(N);
  const auto VMi = inverse(vleg_ld(M), M + 1);
  std::vector<LD> P((N + 1) * (M + 1), 0.0L);
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= M; ++j) {
      LD s = 0.0L;
      for (int k = 0; k <= N; ++k) s += VN[i * (N + 1) + k] * VMi[k * (M + 1) + j];
      P[i * (M + 1) + j] = s;
    }
  return to_double(P);
}

static std::vector<LD> dg2fv_ld(int N, int NFV) {
  const int n = N + 1;
  const auto Vi = inverse(vleg_ld(N), n);     // column j: Legendre coefficients of l_j
  const LD h = 2.0L / NFV;
  std::vector<LD> V(NFV * n);
  for (int s = 0; s < NFV; ++s) {
    const LD a = -1.0L + s * h, b = -1.0L + (s + 1) * h;
    std::vector<LD> intP(n);                  // integral of orthonormal L_k over [a, b]
    for (int k = 0; k < n; ++k) {
      LD ip;
      if (k == 0) ip = b - a;
      else ip = (legendre_p(k + 1, b) - legendre_p(k - 1, b) - legendre_p(k + 1, a) + legendre_p(k - 1, a)) /
                (2.0L * k + 1.0L);
      intP[k] = std::sqrt((2.0L * k + 1.0L) / 2.0L) * ip;
    }
    for (int j = 0; j < n; ++j) {
      LD v = 0.0L;
      for (int k = 0; k < n; ++k) v += Vi[k * n + j] * intP[k];
      V[s * n + j] = v / h;
    }
  }
  return V;
}

std::vector<double> op_dg2fv(int N, int NFV) { return to_double(dg2fv_ld(N, NFV)); }

std::vector<double> op_fv2dg(int N, int NFV) {
  const int n = N + 1;
  const auto V = dg2fv_ld(N, NFV);
  std::vector<LD> VtV(n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      LD s = 0.0L;
      for (int r = 0; r < NFV; ++r) s += V[r * n + i] * V[r * n + j];
      VtV[i * n + j] = s;
    }
  const auto inv = inverse(VtV, n);
  std::vector<LD> P(n * NFV);
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < NFV; ++r) {
      LD s = 0.0L;
      for (int k = 0; k < n; ++k) s += inv[i * n + k] * V[r * n + k];
      P[i * NFV + r] = s;
    }
  return to_double(P);
}

std::vector<double> op_face_interp(int N, int NFV) {
  const auto x = lgl_nodes(N);
  const LD h = 2.0L / NFV;
  std::vector<LD> I((NFV + 1) * (N + 1));
  for (int q = 0; q <= NFV; ++q)
    for (int j = 0; j <= N; ++j) I[q * (N + 1) + j] = (q == 0) ? (j == 0 ? 1.0L : 0.0L)
                                                     : (q == NFV ? (j == N ? 1.0L : 0.0L)
                                                                 : lagrange(x, j, -1.0L + q * h));
  return to_double(I);
}

// ---- mortars -------------------------------------------------------------
// Gauss-Legendre rule of m points (Newton on P_m from the cosine guesses).
static void gauss_legendre(int m, std::vector<LD>& x, std::vector<LD>& w) {
  const LD pi = 3.141592653589793238462643383279502884L;
  x.resize(m);
  w.resize(m);
  for (int i = 0; i < m; ++i) {
    LD z = std::cos(pi * (i + 0.75L) / (m + 0.5L));
    LD p = 0, dp = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(m, z, p, dp);
      const LD dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    legendre(m, z, p, dp);
    x[i] = z;
    w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}

// The big side's nodal polynomial at the nodes of half k, in the half's own
// coordinate s: xi = (s + 2k - 1) / 2.
std::vector<double> op_mortar_interp(int N, int k) {
  const auto x = lgl_nodes(N);
  const int n = N + 1;
  std::vector<LD> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = lagrange(x, j, (x[i] + 2 * k - 1) * 0.5L);
  return to_double(A);
}

// The big side's share of a flux F_k given (per unit of the half's own length)
// at the degree-N nodes of half k: the L2 projection over [-1, 1] of the
// function 2 F_k on half k, 0 elsewhere, as the solution of the mass-matrix
// system  Mass F_0 = B F_k  with  Mass_ij = int l_i l_j dxi  and
// B_il = int_half 2 l_i(xi) l_l(s(xi)) dxi = int_{-1}^{1} l_i((s + 2k - 1)/2) l_l(s) ds,
// both by an (N+2)-point Gauss rule (exact for the degree-2N integrands).
std::vector<double> op_mortar_project(int N, int k) {
  const auto x = lgl_nodes(N);
  const int n = N + 1;
  std::vector<LD> g, gw;
  gauss_legendre(n + 1, g, gw);
  std::vector<LD> mass((size_t)n * n, 0.0L), B((size_t)n * n, 0.0L);
  for (size_t q = 0; q < g.size(); ++q) {
    const LD t = (g[q] + 2 * k - 1) * 0.5L;
    for (int i = 0; i < n; ++i) {
      const LD li = lagrange(x, i, g[q]), lit = lagrange(x, i, t);
      for (int j = 0; j < n; ++j) {
        const LD lj = lagrange(x, j, g[q]);
        mass[(size_t)i * n + j] += gw[q] * li * lj;
        B[(size_t)i * n + j] += gw[q] * lit * lj;
      }
    }
  }
  const auto Mi = inverse(mass, n);
  std::vector<LD> P((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      LD acc = 0.0L;
      for (int l = 0; l < n; ++l) acc += Mi[(size_t)i * n + l] * B[(size_t)l * n + j];
      P[(size_t)i * n + j] = acc;
    }
  return to_double(P);
}

// Sub-face j of half k spans [(j + k NFV)/2, (j + 1 + k NFV)/2) in units of the big side's
// sub-faces; A[j][i] is the share of that span lying in big sub-face i (twice the overlap).
static std::vector<LD> fv_half_overlap(int NFV, int k) {
  std::vector<LD> A((size_t)NFV * NFV, 0.0L);
  for (int j = 0; j < NFV; ++j) {
    const LD lo = 0.5L * (j + k * NFV), hi = lo + 0.5L;
    for (int i = 0; i < NFV; ++i) {
      const LD ov = std::min(hi, (LD)(i + 1)) - std::max(lo, (LD)i);
      A[(size_t)j * NFV + i] = ov > 0 ? 2.0L * ov : 0.0L;
    }
  }
  return A;
}

std::vector<double> op_mortar_fv_interp(int NFV, int k) { return to_double(fv_half_overlap(NFV, k)); }

std::vector<double> op_mortar_fv_project(int NFV, int k) {
  const auto A = fv_half_overlap(NFV, k);
  std::vector<LD> P((size_t)NFV * NFV);
  for (int i = 0; i < NFV; ++i)
    for (int j = 0; j < NFV; ++j) P[(size_t)i * NFV + j] = A[(size_t)j * NFV + i];
  return to_double(P);
}

}  // namespace dgfv

