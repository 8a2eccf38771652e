// Per-degree kernels of the viscous terms (Section 3.1.1, eq. lift_weak,
// eq. semidiscrete_lift and the viscous part of eq. semidiscrete; Section
// 3.2.2).  This translation unit is compiled once per element degree with
// -DDGFV_N=<N>.
//
//  lift_kernel    BR1 lifting of the conservative state: for each node and
//                 physical direction x,
//                   g_x = (1/J) sum_d [ sum_m D_im (Ja^d_x u)_m
//                                       +- Ja^d_x (u* - u) / w_0 on the sides ],
//                 the strong form on LGL nodes, with u* the face value the lift
//                 face kernel left in m.vside and the element's own
//                 contravariant vectors at its boundary nodes.
//  visc_kernel    viscous rate: F^v_x from (u, g) at each node, the
//                 contravariant fluxes Ft^d = sum_x Ja^d_x F^v_x, and
//                   R^v = -(1/J) sum_d [ sum_m D_im Ft^d_m
//                                        + (F^v*_out - (+-Ft^d)) / w_0 on the sides ],
//                 with the outward face fluxes F^v*_out of m.vside.
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

// Adds side s's term at this node (if the node lies on it) to acc.
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
lift_kernel(MeshView m, const int32_t* __restrict__ elist, int count, const double* __restrict__ u) {
  using G = VGeo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3, EPB = G::EPB;
  __shared__ double sD[NP * NP];
  __shared__ double sU[EPB][NV][NP3];
  __shared__ double sJa[EPB][9][NP3];
  const int tid = threadIdx.x;
  const int slot = tid / NP3, node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool active = idx < count;
  for (int t = tid; t < NP * NP; t += blockDim.x) sD[t] = m.ops[m.tab.D[N] + t];
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
  const double* us = m.vside + m.side_off[e];
  for_sides<N>(i, j, k, [&](int s, int fidx) {
    const int d = s >> 1;
    const double sg = (s & 1) ? inv_w0 : -inv_w0;
    double jump[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) jump[v] = us[(s * NV + v) * NP2 + fidx] - ui[v];
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
    for (int v = 0; v < NV; ++v) m.grad[(x * NV + v) * m.n_node + base] = acc[x][v] * invJ;
}

template <int N, int NV>
__global__ void __launch_bounds__(VGeo<N>::EPB * VGeo<N>::NP3)
visc_kernel(MeshView m, const int32_t* __restrict__ elist, int count, const double* __restrict__ u,
            double* __restrict__ rv) {
  using G = VGeo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3, EPB = G::EPB;
  __shared__ double sD[NP * NP];
  __shared__ double sF[EPB][3][NV][NP3];
  const int tid = threadIdx.x;
  const int slot = tid / NP3, node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool active = idx < count;
  for (int t = tid; t < NP * NP; t += blockDim.x) sD[t] = m.ops[m.tab.D[N] + t];
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
  const double* fs = m.vside + m.side_off[e];
  for_sides<N>(i, j, k, [&](int s, int fidx) {
    const int d = s >> 1;
    const double sg = (s & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += (fs[(s * NV + v) * NP2 + fidx] - sg * Ft[d][v]) * inv_w0;
  });
  const double invJ = 1.0 / m.metric[9 * m.n_node + base];
#pragma unroll
  for (int v = 0; v < NV; ++v) rv[v * m.n_node + base] = -acc[v] * invJ;
}

namespace per_degree {
hipError_t lift(const MeshView& m, const int32_t* elist, int count, const double* u, hipStream_t s) {
  using G = VGeo<kN>;
  if (count <= 0) return hipSuccess;
  const int blocks = (count + G::EPB - 1) / G::EPB;
  if (m.nvar == 5)
    hipLaunchKernelGGL((lift_kernel<kN, 5>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u);
  else
    hipLaunchKernelGGL((lift_kernel<kN, 6>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, u);
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
}  // namespace per_degree
}  // namespace

#define DGFV_CAT2(a, b) a##b
#define DGFV_CAT(a, b) DGFV_CAT2(a, b)
ViscousOps DGFV_CAT(viscous_ops_, DGFV_N)() { return ViscousOps{&per_degree::lift, &per_degree::volume}; }

}  // namespace dgfv
