// Per-degree kernels of the viscous terms (Section 3.1.1, eq. lift_weak,
// eq. semidiscrete_lift and the viscous part of eq. semidiscrete; Section
// 3.2.2).  This translation unit is compiled once per element degree with
// -DDGFV_N=<N>.
//
//  lift_kernel    BR1 lifting of the conservative state: for each node and
//                 physical direction x,
//                   g_x = (1/J) sum_d [ sum_m D_im (Ja^d_x u)_m
//                                       +- Ja^d_x (u* - u) / w_0 on the sides ],
//                 the strong form on LGL nodes with the element's own
//                 contravariant vectors at its boundary nodes.  On a side
//                 shared with an element of the same degree the node forms
//                 u* = (u + u_nbr) / 2 itself from the neighbour's matching
//                 node (the neighbour's xi_1 ends from the traces of the
//                 previous RK stage where it wrote them); at a degree jump u*
//                 comes from m.vside.  Its boundary
//                 nodes then leave the viscous flux of (u, g) dotted with the
//                 element's own outward contravariant vector in m.vside for
//                 each same-degree side: half of that face's viscous flux.
//  visc_kernel    viscous rate: F^v_x from (u, g) at each node, the
//                 contravariant fluxes Ft^d = sum_x Ja^d_x F^v_x, and
//                   R^v = -(1/J) sum_d [ sum_m D_im Ft^d_m
//                                        + (F^v*_out - (+-Ft^d)) / w_0 on the sides ],
//                 with the outward F^v* = (own half - the neighbour's half) / 2
//                 at a same-degree side (both outward, left in m.vside by
//                 the lift kernel; the two sides' contravariant vectors at a
//                 face agree up to rounding) and the outward flux of m.vside
//                 at a degree jump.
//
// Both run one element per NP^3 lanes, several elements per workgroup at low
// degree; the partners of a node along each line are read from LDS.
#include "dgfv_internal.h"
#include "dgfv_physics.h"

#ifndef DGFV_N
#error "compile with -DDGFV_N=<degree>"
#endif

namespace dgfv {
namespace {

constexpr int kN = DGFV_N;

template <int N>
struct VGeo {
  static constexpr int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  // elements per workgroup: about 256 lanes
  static constexpr int EPB = NP3 >= 256 ? 1 : 256 / NP3;
};

// Left-grid point (p, q) of a face whose right side holds (pp, qq): the
// inverse of orient_map.
__device__ __forceinline__ void orient_inverse(int o, int pp, int qq, int n, int& p, int& q) {
  const int a = (o & 1) ? n - 1 - pp : pp;
  const int b = (o & 2) ? n - 1 - qq : qq;
  p = (o & 4) ? b : a;
  q = (o & 4) ? a : b;
}

// The point (a, b) of an element's side seen from the face: the neighbour's
// node, the neighbour's side and its face-grid index there.
struct FacePoint {
  int64_t nbr_node;
  int nbr_side, nbr_fidx;
};
template <int N>
__device__ __forceinline__ FacePoint face_point(const SideRec& sr, int a, int b) {
  constexpr int NP = N + 1;
  const int sL = sr.code & 7, sR = (sr.code >> 3) & 7, o = (sr.code >> 6) & 7;
  FacePoint fp;
  if ((sr.code >> 9) & 1) {              // this element is the face's left side
    int pp, qq;
    orient_map(o, a, b, NP, pp, qq);
    fp.nbr_node = sr.baseR + side_node(sR, pp, qq, NP);
    fp.nbr_side = sR;
    fp.nbr_fidx = qq * NP + pp;
  } else {
    int p, q;
    orient_inverse(o, a, b, NP, p, q);
    fp.nbr_node = sr.baseL + side_node(sL, p, q, NP);
    fp.nbr_side = sL;
    fp.nbr_fidx = q * NP + p;
  }
  return fp;
}

// Calls f(side, face-grid index) for each side this node lies on.
template <int N, class F>
__device__ __forceinline__ void for_sides(int i, int j, int k, F&& f) {
  if (i == 0) f(0, k * (N + 1) + j);
  if (i == N) f(1, k * (N + 1) + j);
  if (j == 0) f(2, k * (N + 1) + i);
  if (j == N) f(3, k * (N + 1) + i);
  if (k == 0) f(4, j * (N + 1) + i);
  if (k == N) f(5, j * (N + 1) + i);
}

template <int N, int NV>
__global__ void __launch_bounds__(VGeo<N>::EPB * VGeo<N>::NP3)
lift_kernel(MeshView m, const int32_t* __restrict__ elist, int count, const double* __restrict__ u,
            const double* __restrict__ trace) {
  using G = VGeo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3, EPB = G::EPB;
  __shared__ double sD[NP * NP];
  __shared__ double sU[EPB][NV][NP3];
  __shared__ double sJa[EPB][9][NP3];
  __shared__ double sSt[EPB][6][NV][NP2];    // per side point: the neighbour's u (same degree) or u*
  const int tid = threadIdx.x;
  const int slot = tid / NP3, node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool active = idx < count;
  for (int t = tid; t < NP * NP; t += blockDim.x) sD[t] = m.ops[m.tab.D[N] + t];
  // side points first, so that their dependent loads (side record, then the
  // neighbour's node) overlap the element's own loads and the volume sums
  for (int r = tid; r < EPB * 6 * NP2; r += blockDim.x) {
    const int sl = r / (6 * NP2), rr = r - sl * 6 * NP2, sd = rr / NP2, fidx = rr - sd * NP2;
    const int ix = blockIdx.x * EPB + sl;
    if (ix >= count) continue;
    const int e2 = elist[ix];
    const SideRec sr = m.side_rec[6 * (int64_t)e2 + sd];
    double x[NV];
    if ((sr.code >> 10) & 1) {
      const FacePoint fp = face_point<N>(sr, fidx % NP, fidx / NP);
      if (trace && fp.nbr_side < 2) {      // the neighbour's xi_1 ends, contiguous in the traces
        const double* t = trace + m.side_off[sr.nbr] / 3 + fp.nbr_side * NV * NP2 + fp.nbr_fidx;
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = t[v * NP2];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = u[v * m.n_node + fp.nbr_node];
      }
    } else {
      const double* vs2 = m.vside + m.side_off[e2] + sd * NV * NP2 + fidx;
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v] = vs2[v * NP2];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sSt[sl][sd][v][fidx] = x[v];
  }
  int e = 0;
  int64_t base = 0;
  double ui[NV], ja[9];
  if (active) {
    e = elist[idx];
    base = m.elem_offset[e] + node;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ui[v] = u[v * m.n_node + base];
      sU[slot][v][node] = ui[v];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      ja[c] = m.metric[c * m.n_node + base];
      sJa[slot][c][node] = ja[c];
    }
  }
  __syncthreads();
  if (!active) return;
  const int i = node % NP, j = (node / NP) % NP, k = node / NP2;
  double acc[3][NV];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[x][v] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int id = d == 0 ? i : (d == 1 ? j : k);
    const int stride = d == 0 ? 1 : (d == 1 ? NP : NP2);
    const int first = node - id * stride;
#pragma unroll 2
    for (int mm = 0; mm < NP; ++mm) {
      const int pn = first + mm * stride;
      const double Dim = sD[id * NP + mm];
      double um[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) um[v] = sU[slot][v][pn];
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        const double c = Dim * sJa[slot][3 * d + x][pn];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[x][v] += c * um[v];
      }
    }
  }
  // sides: +- Ja^d_x (u* - u) / w_0, outward sign by side parity
  const double inv_w0 = 1.0 / m.ops[m.tab.w[N]];
  double* vs = m.vside + m.side_off[e];
  const SideRec* srs = m.side_rec + 6 * (int64_t)e;
  for_sides<N>(i, j, k, [&](int s, int fidx) {
    const int d = s >> 1;
    const double sg = (s & 1) ? inv_w0 : -inv_w0;
    const SideRec sr = srs[s];
    double jump[NV];
    if ((sr.code >> 10) & 1) {             // same degree: u* = (u + u_nbr) / 2
#pragma unroll
      for (int v = 0; v < NV; ++v) jump[v] = 0.5 * (sSt[slot][s][v][fidx] - ui[v]);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) jump[v] = sSt[slot][s][v][fidx] - ui[v];
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const double c = sg * ja[3 * d + x];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[x][v] += c * jump[v];
    }
  });
  const double invJ = 1.0 / m.metric[9 * m.n_node + base];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      acc[x][v] *= invJ;
      m.grad[(x * NV + v) * m.n_node + base] = acc[x][v];
    }
  // half fluxes of the same-degree sides: F^v(u, g) . n with the element's own
  // outward contravariant vector, which the face shares (up to rounding) with
  // the neighbour's, reversed
  if (i == 0 || i == N || j == 0 || j == N || k == 0 || k == N) {
    double f[3][NV];
    viscous_flux<NV>(ui, acc, m.gas, m.visc, f);
    for_sides<N>(i, j, k, [&](int s, int fidx) {
      if (!((srs[s].code >> 10) & 1)) return;
      const int d = s >> 1;
      const double sg = (s & 1) ? 1.0 : -1.0;
      const double n0 = sg * ja[3 * d], n1 = sg * ja[3 * d + 1], n2 = sg * ja[3 * d + 2];
#pragma unroll
      for (int v = 0; v < NV; ++v) vs[(s * NV + v) * NP2 + fidx] = f[0][v] * n0 + f[1][v] * n1 + f[2][v] * n2;
    });
  }
}

template <int N, int NV>
__global__ void __launch_bounds__(VGeo<N>::EPB * VGeo<N>::NP3)
visc_kernel(MeshView m, const int32_t* __restrict__ elist, int count, const double* __restrict__ u,
            double* __restrict__ rv) {
  using G = VGeo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3, EPB = G::EPB;
  __shared__ double sD[NP * NP];
  __shared__ double sF[EPB][3][NV][NP3];
  __shared__ double sFo[EPB][6][NV][NP2];    // per side point: the outward viscous face flux
  const int tid = threadIdx.x;
  const int slot = tid / NP3, node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool active = idx < count;
  for (int t = tid; t < NP * NP; t += blockDim.x) sD[t] = m.ops[m.tab.D[N] + t];
  // side points first: a same-degree side takes half the difference of its own
  // outward half flux and the neighbour's (both from the lift kernel); a
  // degree jump takes the face kernel's flux
  for (int r = tid; r < EPB * 6 * NP2; r += blockDim.x) {
    const int sl = r / (6 * NP2), rr = r - sl * 6 * NP2, sd = rr / NP2, fidx = rr - sd * NP2;
    const int ix = blockIdx.x * EPB + sl;
    if (ix >= count) continue;
    const int e2 = elist[ix];
    const SideRec sr = m.side_rec[6 * (int64_t)e2 + sd];
    const double* own = m.vside + m.side_off[e2] + sd * NV * NP2 + fidx;
    double x[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = own[v * NP2];
    if ((sr.code >> 10) & 1) {
      const FacePoint fp = face_point<N>(sr, fidx % NP, fidx / NP);
      const double* hn = m.vside + m.side_off[sr.nbr] + fp.nbr_side * NV * NP2 + fp.nbr_fidx;
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v] = 0.5 * (x[v] - hn[v * NP2]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sFo[sl][sd][v][fidx] = x[v];
  }
  int e = 0;
  int64_t base = 0;
  double Ft[3][NV];
  if (active) {
    e = elist[idx];
    base = m.elem_offset[e] + node;
    double ui[NV], gr[3][NV], f[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ui[v] = u[v * m.n_node + base];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int v = 0; v < NV; ++v) gr[x][v] = m.grad[(x * NV + v) * m.n_node + base];
    viscous_flux<NV>(ui, gr, m.gas, m.visc, f);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a0 = m.metric[(3 * d) * m.n_node + base];
      const double a1 = m.metric[(3 * d + 1) * m.n_node + base];
      const double a2 = m.metric[(3 * d + 2) * m.n_node + base];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Ft[d][v] = a0 * f[0][v] + a1 * f[1][v] + a2 * f[2][v];
        sF[slot][d][v][node] = Ft[d][v];
      }
    }
  }
  __syncthreads();
  if (!active) return;
  const int i = node % NP, j = (node / NP) % NP, k = node / NP2;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int id = d == 0 ? i : (d == 1 ? j : k);
    const int stride = d == 0 ? 1 : (d == 1 ? NP : NP2);
    const int first = node - id * stride;
#pragma unroll 2
    for (int mm = 0; mm < NP; ++mm) {
      const double Dim = sD[id * NP + mm];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += Dim * sF[slot][d][v][first + mm * stride];
    }
  }
  const double inv_w0 = 1.0 / m.ops[m.tab.w[N]];
  for_sides<N>(i, j, k, [&](int s, int fidx) {
    const int d = s >> 1;
    const double sg = (s & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += (sFo[slot][s][v][fidx] - sg * Ft[d][v]) * inv_w0;
  });
  const double invJ = 1.0 / m.metric[9 * m.n_node + base];
#pragma unroll
  for (int v = 0; v < NV; ++v) rv[v * m.n_node + base] = -acc[v] * invJ;
}

// Time step of Section 3.3, per element: the convective signal speed
// lambda^c = max_nodes sum_d (|v . Ja^d| + c |Ja^d|) / J and, with viscous
// terms, the parabolic rate lambda^v = max_nodes delta^v sum_d |Ja^d|^2 / J^2
// with delta^v = max(4/3 mu / rho, kappa mu / (Pr rho), D_1, D_2); then
// dt^c_e = 2 / ((2N + 1) lambda^c), dt^v_e = 4 / ((2N + 1) lambda^v), a blended
// element also bounded by the sub-cell spacing h_FV = 2 / N_FV (h_FV /
// lambda^c, h_FV^2 / lambda^v).  The maxima over an element's nodes use
// unsigned 64-bit atomics in LDS on the bit patterns (order-preserving for
// non-negative doubles; a NaN outranks every number and comes through).
template <int N, int NV>
__global__ void __launch_bounds__(VGeo<N>::EPB * VGeo<N>::NP3)
timestep_kernel(MeshView m, const int32_t* __restrict__ elist, int count, const double* __restrict__ u,
                const double* __restrict__ alpha, int viscous, double* __restrict__ dt_e) {
  using G = VGeo<N>;
  constexpr int NP3 = G::NP3, EPB = G::EPB;
  __shared__ unsigned long long sMax[EPB][2];
  const int tid = threadIdx.x;
  const int slot = tid / NP3, node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool active = idx < count;
  if (node < 2) sMax[slot][node] = 0ull;
  __syncthreads();
  int e = 0;
  if (active) {
    e = elist[idx];
    const int64_t base = m.elem_offset[e] + node;
    double uo[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uo[v] = u[v * m.n_node + base];
    const Prim q = cons2prim<NV>(uo, m.gas);
    const double c = sqrt(q.kap * q.p / q.rho);
    const double iJ = 1.0 / m.metric[9 * m.n_node + base];
    double lc = 0.0, a2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a0 = m.metric[(3 * d) * m.n_node + base];
      const double a1 = m.metric[(3 * d + 1) * m.n_node + base];
      const double a2d = m.metric[(3 * d + 2) * m.n_node + base];
      const double nn = a0 * a0 + a1 * a1 + a2d * a2d;
      lc += fabs(q.v1 * a0 + q.v2 * a1 + q.v3 * a2d) + c * sqrt(nn);
      a2 += nn;
    }
    lc *= iJ;
    atomicMax(&sMax[slot][0], (unsigned long long)__double_as_longlong(lc));
    if (viscous) {
      double mu, Pr, dmax = 0.0;
      if constexpr (NV == 6) {
        mu = q.Y * m.visc.mu0 + (1.0 - q.Y) * m.visc.mu1;
        Pr = q.Y * m.visc.Pr0 + (1.0 - q.Y) * m.visc.Pr1;
        dmax = fmax(m.visc.D0, m.visc.D1);
      } else {
        mu = m.visc.mu0;
        Pr = m.visc.Pr0;
      }
      const double delta = fmax(fmax((4.0 / 3.0) * mu / q.rho, q.kap * mu / (Pr * q.rho)), dmax);
      const double lv = delta * a2 * iJ * iJ;
      atomicMax(&sMax[slot][1], (unsigned long long)__double_as_longlong(lv));
    }
  }
  __syncthreads();
  if (!active || node != 0) return;
  const double lc = __longlong_as_double((long long)sMax[slot][0]);
  const double lv = __longlong_as_double((long long)sMax[slot][1]);
  const bool blended = alpha && alpha[e] > 0.0;
  const double hfv = 2.0 / m.n_fv;
  double dc = 2.0 / ((2 * N + 1) * lc);
  if (blended) dc = fmin(dc, hfv / lc);
  double dv = 0.0;
  if (viscous) {
    dv = 4.0 / ((2 * N + 1) * lv);
    if (blended) dv = fmin(dv, hfv * hfv / lv);
  }
  dt_e[e] = dc;
  dt_e[m.K + e] = dv;
}

namespace per_degree {
hipError_t lift(const MeshView& m, const int32_t* elist, int count, const double* u, bool trace_in,
                hipStream_t s) {
  using G = VGeo<kN>;
  if (count <= 0) return hipSuccess;
  const int blocks = (count + G::EPB - 1) / G::EPB;
  const double* tr = trace_in && kN >= TRACE_MIN_N ? m.trace : nullptr;
  if (m.nvar == 5)
    hipLaunchKernelGGL((lift_kernel<kN, 5>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u, tr);
  else
    hipLaunchKernelGGL((lift_kernel<kN, 6>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u, tr);
  return hipGetLastError();
}

hipError_t volume(const MeshView& m, const int32_t* elist, int count, const double* u, double* rv,
                  hipStream_t s) {
  using G = VGeo<kN>;
  if (count <= 0) return hipSuccess;
  const int blocks = (count + G::EPB - 1) / G::EPB;
  if (m.nvar == 5)
    hipLaunchKernelGGL((visc_kernel<kN, 5>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u, rv);
  else
    hipLaunchKernelGGL((visc_kernel<kN, 6>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u, rv);
  return hipGetLastError();
}
hipError_t timestep(const MeshView& m, const int32_t* elist, int count, const double* u, const double* alpha,
                    int viscous, double* dt_e, hipStream_t s) {
  using G = VGeo<kN>;
  if (count <= 0) return hipSuccess;
  const int blocks = (count + G::EPB - 1) / G::EPB;
  if (m.nvar == 5)
    hipLaunchKernelGGL((timestep_kernel<kN, 5>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u,
                       alpha, viscous, dt_e);
  else
    hipLaunchKernelGGL((timestep_kernel<kN, 6>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u,
                       alpha, viscous, dt_e);
  return hipGetLastError();
}
}  // namespace per_degree
}  // namespace

#define DGFV_CAT2(a, b) a##b
#define DGFV_CAT(a, b) DGFV_CAT2(a, b)
ViscousOps DGFV_CAT(viscous_ops_, DGFV_N)() {
  return ViscousOps{&per_degree::lift, &per_degree::volume, &per_degree::timestep};
}

}  // namespace dgfv
