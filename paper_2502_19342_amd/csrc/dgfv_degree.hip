// Per-degree kernels of the hybrid DG/FV right-hand side.  This translation
// unit is compiled once per element degree with -DDGFV_N=<N>.
//
//  element_kernel  split-form DGSEM volume term (flux differencing, Section 3.5),
//                  surface lift (eq. semidiscrete), blend with the FV residual,
//                  and optionally the fused 2N Runge-Kutta stage (Section 3.3)
//  fv_means        J-weighted sub-cell means of blended elements (V^{DG->FV}, Section 3.2)
//  fv_residual     first-order FV sub-cell operator (eq. semidiscrete_fv) mapped
//                  back with V^{FV->DG}
//  indicator       modal decay indicator and blending ramp (Section 3.4)
#include <type_traits>

#include "dgfv_internal.h"
#include "dgfv_physics.h"
#include "dgfv_lds.h"

#ifndef DGFV_N
#error "compile with -DDGFV_N=<degree>"
#endif

namespace dgfv {
namespace {

constexpr int kN = DGFV_N;

template <int N>
struct Geo {
  static constexpr int NP = N + 1, NP2 = NP * NP, NP3 = NP2 * NP;
  // elements per workgroup of the element kernel: fill about 512 lanes
  static constexpr int EPB = NP3 >= 256 ? 1 : (512 / NP3 > 64 ? 64 : 512 / NP3);
};

// Tile shapes of the element kernel, chosen per degree by the autotuner:
// variant 0 fills about 512 lanes per workgroup, variant 1 about 256 (only
// where a workgroup holds more than one element).
template <int N, int V>
constexpr int elem_epb() { return V == 0 || Geo<N>::EPB == 1 ? Geo<N>::EPB : Geo<N>::EPB / 2; }
constexpr int elem_variants(int N) { return (N + 1) * (N + 1) * (N + 1) >= 256 ? 1 : 2; }

// ---------------------------------------------------------------------------
// element kernel
// ---------------------------------------------------------------------------
template <int N, int NV, class FLUX, int EPB, bool FUSE>
__global__ void __launch_bounds__(EPB * Geo<N>::NP3)
element_kernel(MeshView m, ParamsDev prm, const int32_t* __restrict__ elist, int count, const double* u,
               double* uout, const double* __restrict__ alpha, double* __restrict__ ut, double* k, int stage,
               double dt, double A, double B, int flags) {
  using G = Geo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3;
  constexpr int NA = FLUX::NA;
  // Each pair (i, m) of a line is evaluated once: offsets o = 1..NOFF send the
  // partner's share D_mi f# through sInc; for even NP the pairs at offset
  // NP/2 are evaluated from both ends (no exchange).
  constexpr int NOFF = (NP - 1) / 2;
  constexpr bool HALF = (NP % 2) == 0;
  __shared__ double sD[NP * NP];
  __shared__ double sAux[EPB][NA][NP3];
  __shared__ double sJa[EPB][3][NP3];          // Ja^d of the current direction
  __shared__ double sInc[NOFF > 0 ? EPB : 1][NV][NOFF > 0 ? NP3 : 1];
  // One element per workgroup: the element's side fluxes (one contiguous block
  // of 6 NV (N+1)^2 values) are loaded beside the state and parked in LDS before
  // the first barrier, so the lift reads LDS instead of waiting on global loads
  // at the end of the kernel.
  constexpr bool STAGE_SIDES = EPB == 1;
  constexpr int NSIDE = 6 * NV * NP2;
  constexpr int SIDE_PER = STAGE_SIDES ? (NSIDE + NP3 - 1) / NP3 : 1;
  __shared__ double sSide[STAGE_SIDES ? NSIDE : 1];

  const int tid = threadIdx.x;
  const int slot = tid / NP3;
  const int node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool in_range = idx < count;        // lanes past the list mirror element 0 and write nothing

  // The two-point fluxes are linear in the metric direction: they are evaluated
  // with the sum Ja_i + Ja_m instead of the mean, so the weights are D_im
  // instead of 2 D_im (times FAST_WEIGHT, where flux_fast returns a multiple
  // of the flux).
  for (int t = tid; t < NP * NP; t += blockDim.x) sD[t] = FLUX::FAST_WEIGHT * m.ops[m.tab.D[N] + t];

  // with one element per workgroup the element index is wave-uniform: kept in
  // a scalar register, its per-element records (offsets, alpha, side block)
  // are scalar loads held in scalar registers for the whole kernel
  int e = elist[in_range ? idx : 0];
  if constexpr (EPB == 1) e = __builtin_amdgcn_readfirstlane(e);
  const int64_t base = m.elem_offset[e] + node;
  const double inv_w0 = 1.0 / m.ops[m.tab.w[N]];    // lift weight, loaded early
  double uo[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) uo[v] = u[v * m.n_node + base];
  const double al = alpha ? alpha[e] : 0.0;
  // An FV-stored element (ELEM_SKIP_FV, alpha >= 1) is left alone: its lanes
  // compute on its unused nodal slot and write nothing (one element per
  // workgroup: the whole workgroup leaves before the first barrier).
  const bool skip_fv = (flags & ELEM_SKIP_FV) && al >= 1.0;
  if constexpr (EPB == 1) {
    if (skip_fv) return;
  }
  const bool active = in_range && !skip_fv;
  const double* fs = m.fside + m.side_off[e];
  const bool write_trace = flags & ELEM_WRITE_TRACE;
  // Fused faces (one element per workgroup): lane t < 6 (N+1)^2 takes point
  // t mod (N+1)^2 of side t / (N+1)^2 on the face's left grid.  A face shared
  // with a pure DG element of the same degree gets its Riemann flux here, with
  // exactly the operands and operations of the conforming face kernel (the
  // right element stores the negated flux, re-indexed through the orientation);
  // the other sides (degree jumps, FV faces) take the point's value from the
  // side buffer, written by the face kernels.  The neighbour's state is read
  // from u, which no workgroup of this launch writes (stage 0, or uout != u).
  // (a separate instantiation: the unfused kernel carries none of this code)
  constexpr bool CAN_FUSE = STAGE_SIDES && FUSE;
  constexpr bool fuse = CAN_FUSE;
  double sv[SIDE_PER];
  double fv[NV];
  int fdst = -1;                           // this lane's point in sSide (fused), or none
  if constexpr (STAGE_SIDES) {
    if (al < 1.0 && !fuse) {        // a pure FV element needs no side fluxes
#pragma unroll
      for (int r = 0; r < SIDE_PER; ++r) {
        const int q = tid + r * NP3;
        sv[r] = q < NSIDE ? fs[q] : 0.0;
      }
    }
    // (the side record and the operands are loaded whatever this element's
    // alpha, so that they do not wait for it)
    if (CAN_FUSE && fuse && tid < 6 * NP2) {
      const int s = tid / NP2, r = tid - s * NP2;
      const SideRec sr = m.side_rec[6 * (int64_t)e + s];
      const int sL = sr.code & 7, sR = (sr.code >> 3) & 7, o = (sr.code >> 6) & 7;
      const bool own_left = (sr.code >> 9) & 1, same_degree = (sr.code >> 10) & 1;
      const int p = r % NP, q = r / NP;
      int pp, qq;
      orient_map(o, p, q, NP, pp, qq);
      const double an = alpha ? alpha[sr.nbr] : 0.0;
      double uL[NV], uR[NV], n0 = 0.0, n1 = 0.0, n2 = 0.0;
      if (same_degree) {                   // both elements have (N+1)^3 nodes: in range
        const double* srcL = u + sr.baseL + side_node(sL, p, q, NP);
        const double* srcR = u + sr.baseR + side_node(sR, pp, qq, NP);
        const double* nrm = m.face_norm + sr.nrm;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          uL[v] = srcL[v * m.n_node];
          uR[v] = srcR[v * m.n_node];
        }
        n0 = nrm[r];
        n1 = nrm[NP2 + r];
        n2 = nrm[2 * NP2 + r];
      }
      if (!(al < 1.0)) {
        // a pure FV element takes no side fluxes
      } else if (same_degree && !(al > 0.0) && !(an > 0.0)) {
        double F[NV];
        riemann<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, n0, n1, n2, m.gas, F);
#pragma unroll
        for (int v = 0; v < NV; ++v) fv[v] = own_left ? F[v] : -F[v];
        fdst = s * NV * NP2 + (own_left ? q * NP + p : qq * NP + pp);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) fv[v] = fs[(s * NV + v) * NP2 + r];
        fdst = s * NV * NP2 + r;
      }
    }
  }

  const int i = node % NP, j = (node / NP) % NP, kk = node / NP2;
  // stage 0: ut = R; stage s: k <- A k + dt R (k not read at stage 1), u <- u + B k,
  // and with write_trace the new state of the xi_1 ends (sides 0 and 1) also in
  // m.trace, contiguous per side for the next stage's face fluxes.  Only at
  // N >= TRACE_MIN_N, where the N+1 stride of those sides in u costs the face
  // kernels most; below it the extra stores cost more than they save.
  constexpr bool TRACE = N >= TRACE_MIN_N;
  auto store = [&](const double* R, const double* k_old) {
    if (stage == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) ut[v * m.n_node + base] = R[v];
    } else {
      double* uw = uout;
      double* tr = nullptr;
      if (TRACE && write_trace && (i == 0 || i == N))
        tr = m.trace + m.side_off[e] / 3 + ((i == 0 ? 0 : 1) * NV) * NP2 + kk * NP + j;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t g = v * m.n_node + base;
        const double kv = (stage == 1) ? dt * R[v] : A * k_old[v] + dt * R[v];
        const double un = uo[v] + B * kv;
        k[g] = kv;
        uw[g] = un;
        if (tr) tr[v * NP2] = un;
      }
    }
  };
  if constexpr (EPB == 1) {
    // alpha = 1: a pure FV element.  The DG part has weight 0, so R = R^FV
    // exactly and none of it is evaluated (one element per workgroup: the
    // branch is uniform and comes before every barrier).
    if (al >= 1.0) {
      if (!active) return;
      const Prim q = cons2prim<NV>(uo, m.gas);
      if (!(q.rho > 0.0) || !(q.p > 0.0)) m.state_flag[0] = 1;   // rho <= 0, p <= 0 or NaN
      double R[NV], k_old[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R[v] = m.rfv[v * m.n_node + base];
        if (m.rvisc) R[v] += m.rvisc[v * m.n_node + base];
        k_old[v] = stage > 1 ? k[v * m.n_node + base] : 0.0;
      }
      store(R, k_old);
      return;
    }
  }
  {
    const Prim q = cons2prim<NV>(uo, m.gas);
    if (active && (!(q.rho > 0.0) || !(q.p > 0.0))) m.state_flag[0] = 1;   // rho <= 0, p <= 0 or NaN
    double r[NA];
    FLUX::template make<NV>(q, r);
#pragma unroll
    for (int a = 0; a < NA; ++a) sAux[slot][a][node] = r[a];
  }
  if constexpr (STAGE_SIDES) {
    if (fuse) {
      if (fdst >= 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sSide[fdst + v * NP2] = fv[v];
      }
    } else {
#pragma unroll
      for (int r = 0; r < SIDE_PER; ++r) {
        const int q = tid + r * NP3;
        if (q < NSIDE) sSide[q] = sv[r];
      }
    }
  }
  const double invJ = 1.0 / m.metric[9 * m.n_node + base];

  const int lane = tid & 63;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  __syncthreads();                            // sAux complete
  double me[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) me[a] = sAux[slot][a][node];

  // One direction of the flux differencing.  Where every line of direction d
  // lies inside one 64-lane wave (N+1 dividing 64 for d = 0, 1; (N+1)^3
  // dividing 64 for d = 2), the partner's metric and the partner's share move
  // by cross-lane shuffles and need no workgroup barrier; otherwise through LDS.
  auto direction = [&](auto dtag, bool lds_was_used, const double* ja) {
    constexpr int d = decltype(dtag)::value;
    constexpr bool in_wave = d < 2 ? (64 % NP == 0) : (64 % NP3 == 0);
    constexpr int stride = d == 0 ? 1 : (d == 1 ? NP : NP2);
    const int id = d == 0 ? i : (d == 1 ? j : kk);
    const double ja1 = ja[0], ja2 = ja[1], ja3 = ja[2];
    if constexpr (!in_wave) {
      if (lds_was_used) __syncthreads();      // previous direction done with sJa and sInc
      sJa[slot][0][node] = ja1;
      sJa[slot][1][node] = ja2;
      sJa[slot][2][node] = ja3;
      __syncthreads();
    }
    auto partner_metric = [&](int pn, double& b1, double& b2, double& b3) {
      if constexpr (in_wave) {
        const int sl = (lane + pn - node) & 63;
        b1 = __shfl(ja1, sl);
        b2 = __shfl(ja2, sl);
        b3 = __shfl(ja3, sl);
      } else {
        b1 = sJa[slot][0][pn];
        b2 = sJa[slot][1][pn];
        b3 = sJa[slot][2][pn];
      }
    };
#pragma unroll 1
    for (int o = 1; o <= NOFF; ++o) {
      int mm = id + o;
      if (mm >= NP) mm -= NP;
      const int pn = node + (mm - id) * stride;
      double other[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) other[a] = sAux[slot][a][pn];
      double b1, b2, b3;
      partner_metric(pn, b1, b2, b3);
      double f[NV];
      FLUX::template flux_fast<NV>(me, other, ja1 + b1, ja2 + b2, ja3 + b3, m.gas, f);
      const double c1 = sD[id * NP + mm];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += c1 * f[v];
      if constexpr (in_wave) {
        // the share for this node comes from the node at offset -o on the line:
        // its flux, weighted here by D[id][mr]
        int mr = id - o;
        if (mr < 0) mr += NP;
        const int sl = (lane + (mr - id) * stride) & 63;
        const double cr = sD[id * NP + mr];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += cr * __shfl(f[v], sl);
      } else {
        const double c2 = sD[mm * NP + id];
        if (o > 1) __syncthreads();           // partner has read the previous round's share
#pragma unroll
        for (int v = 0; v < NV; ++v) sInc[slot][v][pn] = c2 * f[v];
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += sInc[slot][v][node];
      }
    }
    if constexpr (HALF) {
      int mm = id + NP / 2;
      if (mm >= NP) mm -= NP;
      const int pn = node + (mm - id) * stride;
      double other[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) other[a] = sAux[slot][a][pn];
      double b1, b2, b3;
      partner_metric(pn, b1, b2, b3);
      double f[NV];
      FLUX::template flux_fast<NV>(me, other, ja1 + b1, ja2 + b2, ja3 + b3, m.gas, f);
      const double c1 = sD[id * NP + mm];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += c1 * f[v];
    }
    return lds_was_used || !in_wave;
  };
  // Ja^d of the next direction is loaded while the current one is computed
  auto load_ja = [&](int d, double* ja) {
#pragma unroll
    for (int c = 0; c < 3; ++c) ja[c] = m.metric[(3 * d + c) * m.n_node + base];
  };
  double jaA[3], jaB[3];
  load_ja(0, jaA);
  load_ja(1, jaB);
  bool lds_used = direction(std::integral_constant<int, 0>{}, false, jaA);
  // At N = 7 with one element per workgroup (an 8 x 8 plane per wave) the
  // xi_3 lines cross waves.  There the xi_3 pairs are computed under a
  // transposed ownership instead, wave w taking the plane j = w and lane l the
  // node (i, k) = (l mod 8, l div 8), so that every xi_3 line lies in one wave
  // and moves by shuffles; one LDS pass hands the sums back to the owners.
  constexpr bool XI3_TRANSPOSED = NP == 8 && EPB == 1;
  if constexpr (XI3_TRANSPOSED) {
    const int nt = (lane % NP) + NP * (tid >> 6) + NP2 * (lane / NP);
    const int64_t bt = m.elem_offset[e] + nt;
#pragma unroll
    for (int c = 0; c < 3; ++c) jaA[c] = m.metric[(6 + c) * m.n_node + bt];
  } else {
    load_ja(2, jaA);
  }
  lds_used = direction(std::integral_constant<int, 1>{}, lds_used, jaB);
  double k_old[NV];                            // the RK register, loaded while xi_3 is computed
  if constexpr (!XI3_TRANSPOSED) {
#pragma unroll
    for (int v = 0; v < NV; ++v) k_old[v] = stage > 1 ? k[v * m.n_node + base] : 0.0;
  }
  if constexpr (XI3_TRANSPOSED) {
    // the owners park their xi_1, xi_2 sums in LDS, which frees their registers
#pragma unroll
    for (int v = 0; v < NV; ++v) sInc[0][v][node] = acc[v];
    const int it = lane % NP, kt = lane / NP;
    const int nt = it + NP * (tid >> 6) + NP2 * kt;
    double mt[NA], at[NV];
#pragma unroll
    for (int a = 0; a < NA; ++a) mt[a] = sAux[0][a][nt];
#pragma unroll
    for (int v = 0; v < NV; ++v) at[v] = 0.0;
    const double ja1 = jaA[0], ja2 = jaA[1], ja3 = jaA[2];
    auto pair = [&](int mm, bool exchange, int o) {
      const int pn = nt + (mm - kt) * NP2;
      const int sl = (lane + (mm - kt) * NP) & 63;
      double other[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) other[a] = sAux[0][a][pn];
      const double b1 = __shfl(ja1, sl), b2 = __shfl(ja2, sl), b3 = __shfl(ja3, sl);
      double f[NV];
      FLUX::template flux_fast<NV>(mt, other, ja1 + b1, ja2 + b2, ja3 + b3, m.gas, f);
      const double c1 = sD[kt * NP + mm];
#pragma unroll
      for (int v = 0; v < NV; ++v) at[v] += c1 * f[v];
      if (exchange) {
        int mr = kt - o;
        if (mr < 0) mr += NP;
        const int sr = (lane + (mr - kt) * NP) & 63;
        const double cr = sD[kt * NP + mr];
#pragma unroll
        for (int v = 0; v < NV; ++v) at[v] += cr * __shfl(f[v], sr);
      }
    };
#pragma unroll 1
    for (int o = 1; o <= NOFF; ++o) {
      int mm = kt + o;
      if (mm >= NP) mm -= NP;
      pair(mm, true, o);
    }
    {
      int mm = kt + NP / 2;
      if (mm >= NP) mm -= NP;
      pair(mm, false, 0);
    }
    __syncthreads();                           // every owner has parked its sums
#pragma unroll
    for (int v = 0; v < NV; ++v) sInc[0][v][nt] += at[v];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = sInc[0][v][node];
#pragma unroll
    for (int v = 0; v < NV; ++v) k_old[v] = stage > 1 ? k[v * m.n_node + base] : 0.0;
  } else {
    direction(std::integral_constant<int, 2>{}, lds_used, jaA);
  }
  if (!active) return;

  // surface lift: outward numerical flux over the end weight on boundary nodes
  const double* side = STAGE_SIDES ? static_cast<const double*>(sSide) : fs;
  auto add_side = [&](int s, int fidx) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += side[(s * NV + v) * NP2 + fidx] * inv_w0;
  };
  if (i == 0) add_side(0, kk * NP + j);
  if (i == N) add_side(1, kk * NP + j);
  if (j == 0) add_side(2, kk * NP + i);
  if (j == N) add_side(3, kk * NP + i);
  if (kk == 0) add_side(4, j * NP + i);
  if (kk == N) add_side(5, j * NP + i);

  double R[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[v] = -acc[v] * invJ;

  if (al > 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] = (1.0 - al) * R[v] + al * m.rfv[v * m.n_node + base];
  }
  if (m.rvisc) {                           // viscous rate of every element, outside the blend
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] += m.rvisc[v * m.n_node + base];
  }
  store(R, k_old);
}

// ---------------------------------------------------------------------------
// FV sub-cell operator of blended elements.
//   means:    ubar = V3(J u) / V3(J)                         (V^{DG->FV}, Section 3.2)
//   residual: dC/dt = -(sum of outward sub-face fluxes),
//             R^FV = V3^+(dC/dt) / (h^3 J)                    (eq. semidiscrete_fv, V^{FV->DG})
// Sub-face normals n*s = h^2 x mean of Ja^d over the sub-face (face_interp along
// d, dg2fv along the tangential directions) depend on geometry only; they are
// formed once per mesh (fv_normals_kernel) for the NFV-1 internal planes of
// each direction: fvnorm[e][d][c][q][a][b], q = 0..NFV-2 the plane between
// sub-cells q and q+1, (a, b) the tangential sub-cell indices (slower, faster).
// ---------------------------------------------------------------------------
constexpr int FV_THREADS = 256;

template <int N>
__global__ void __launch_bounds__(FV_THREADS)
fv_normals_kernel(MeshView m, const int32_t* __restrict__ elist, int count) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP;
  constexpr int NRM = 3 * (MAXFV + 1) * MAXFV * MAXFV;
  __shared__ double sJa[9 * NP3];
  __shared__ double sA[NRM];
  __shared__ double sB[NRM];
  __shared__ double sV[MAXFV * (MAXN + 1)];
  __shared__ double sI[(MAXFV + 1) * (MAXN + 1)];
  const int idx = blockIdx.x;
  if (idx >= count) return;
  const int e = elist[idx];
  const int NFV = m.n_fv;
  const int S2 = NFV * NFV, NIF = (NFV - 1) * S2;
  const double h = 2.0 / NFV;
  const int64_t base = m.elem_offset[e];
  for (int t = threadIdx.x; t < 9 * NP3; t += blockDim.x)
    sJa[t] = m.metric[(t / NP3) * m.n_node + base + (t % NP3)];
  for (int t = threadIdx.x; t < NFV * NP; t += blockDim.x) sV[t] = m.ops[m.tab.dg2fv[N] + t];
  for (int t = threadIdx.x; t < (NFV + 1) * NP; t += blockDim.x) sI[t] = m.ops[m.tab.face_interp[N] + t];
  __syncthreads();
  double* out = m.fvnorm + (size_t)e * 9 * NIF;
  for (int d = 0; d < 3; ++d) {
    contract_axis(sJa + 3 * d * NP3, sA, sI, NFV + 1, NP, 3, NP, NP, NP, d);
    __syncthreads();
    int a2 = (d == 2) ? NFV + 1 : NP, a1 = (d == 1) ? NFV + 1 : NP, a0 = (d == 0) ? NFV + 1 : NP;
    const int ta = (d == 0) ? 1 : 0;
    const int tb = (d == 2) ? 1 : 2;
    contract_axis(sA, sB, sV, NFV, NP, 3, a2, a1, a0, ta);
    __syncthreads();
    if (ta == 0) a0 = NFV; else a1 = NFV;
    contract_axis(sB, sA, sV, NFV, NP, 3, a2, a1, a0, tb);
    __syncthreads();
    if (tb == 1) a1 = NFV; else a2 = NFV;
    const int nn = a2 * a1 * a0;
    for (int t = threadIdx.x; t < 3 * nn; t += blockDim.x) {
      const int c = t / nn, r = t % nn;
      const int x0 = r % a0, x1 = (r / a0) % a1, x2 = r / (a0 * a1);
      int q, a, b;
      if (d == 0) { q = x0; a = x2; b = x1; }
      else if (d == 1) { q = x1; a = x2; b = x0; }
      else { q = x2; a = x1; b = x0; }
      if (q == 0 || q == NFV) continue;
      out[(d * 3 + c) * NIF + ((q - 1) * NFV + a) * NFV + b] = sA[t] * (h * h);
    }
    __syncthreads();
  }
}

constexpr int FV2_THREADS = 512;

template <int N, int NFV, int NV>
__global__ void __launch_bounds__(FV2_THREADS)
fv_means_kernel(MeshView m, const double* __restrict__ u) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP, S3 = NFV * NFV * NFV;
  constexpr int NF = NV + 1;                  // J*u (NV fields) and J
  __shared__ double bufA[NF * S3];
  __shared__ double bufB[NF * S3];
  __shared__ double sV[NFV * NP];
  const int t = threadIdx.x;
  if (t < NFV * NP) sV[t] = m.ops[m.tab.dg2fv[N] + t];
  const int end = m.blend_start[N + 1];
  for (int w = m.blend_start[N] + blockIdx.x; w < end; w += gridDim.x) {
  const int e = m.blend_list[w];
  const int64_t base = m.elem_offset[e];
  for (int r = t; r < NP3; r += FV2_THREADS) {
    const double J = m.metric[9 * m.n_node + base + r];
    for (int v = 0; v < NV; ++v) bufA[v * NP3 + r] = J * u[v * m.n_node + base + r];
    bufA[NV * NP3 + r] = J;
  }
  __syncthreads();
  // Three one-dimensional contractions with V (NFV x NP).  Each thread keeps one
  // input line in registers and forms all NFV outputs along the contracted
  // axis, so every LDS word is read once per pass; V is read at uniform
  // addresses.
  // axis 0: [f][k][j][c] -> [f][k][j][s0]
  for (int r = t; r < NF * NP * NP; r += FV2_THREADS) {
    const double* src = bufA + r * NP;
    double x[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = src[c];
#pragma unroll
    for (int s0 = 0; s0 < NFV; ++s0) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) acc += sV[s0 * NP + c] * x[c];
      bufB[r * NFV + s0] = acc;
    }
  }
  __syncthreads();
  // axis 1: [f][k][c][s0] -> [f][k][s1][s0]
  for (int r = t; r < NF * NP * NFV; r += FV2_THREADS) {
    const int s0 = r % NFV, kf = r / NFV;                                   // kf = f*NP + k
    const double* src = bufB + kf * NP * NFV + s0;
    double x[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = src[c * NFV];
#pragma unroll
    for (int s1 = 0; s1 < NFV; ++s1) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) acc += sV[s1 * NP + c] * x[c];
      bufA[(kf * NFV + s1) * NFV + s0] = acc;
    }
  }
  __syncthreads();
  // axis 2: [f][c][s1][s0] -> [f][s2][s1][s0]
  for (int r = t; r < NF * NFV * NFV; r += FV2_THREADS) {
    const int s01 = r % (NFV * NFV), f = r / (NFV * NFV);
    const double* src = bufA + f * NP * NFV * NFV + s01;
    double x[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = src[c * NFV * NFV];
#pragma unroll
    for (int s2 = 0; s2 < NFV; ++s2) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) acc += sV[s2 * NP + c] * x[c];
      bufB[f * S3 + s2 * NFV * NFV + s01] = acc;
    }
  }
  __syncthreads();
  double* ub = m.ubar + (size_t)e * NV * S3;
  for (int r = t; r < S3; r += FV2_THREADS) {
    const double ivol = 1.0 / bufB[NV * S3 + r];
    for (int v = 0; v < NV; ++v) ub[v * S3 + r] = bufB[v * S3 + r] * ivol;
  }
  __syncthreads();                            // bufB is reused by the next element
  }
}

template <int N, int NFV, int NV>
__global__ void __launch_bounds__(FV2_THREADS)
fv_residual_kernel(MeshView m, ParamsDev prm) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP;
  constexpr int S2 = NFV * NFV, S3 = S2 * NFV, NIF = (NFV - 1) * S2;
  static_assert(S3 <= FV2_THREADS, "one thread per sub-cell");
  __shared__ double sU[NV * S3];
  __shared__ double sG[NV * S3];
  __shared__ double sF[6 * NV * S2];           // the six sides' FV fluxes
  __shared__ double sJ[NP3];
  __shared__ double sVp[NP * NFV];
  const int t = threadIdx.x;
  const double h = 2.0 / NFV;
  // the grid spans the whole degree bucket: workgroups past the blended range
  // leave before touching memory other than the range bounds
  const int w = m.blend_start[N] + blockIdx.x;
  if (w >= m.blend_start[N + 1]) return;
  if (t < NP * NFV) sVp[t] = m.ops[m.tab.fv2dg[N] + t];
  const int e = m.blend_list[w];
  const int64_t base = m.elem_offset[e];
  // every global read of the element is issued here, ahead of the first barrier
  // and before any of them is used: the sub-cell means, side fluxes and J go to
  // LDS, this thread's sub-face normals stay in registers.  The copy loops have
  // compile-time trip counts and unroll, so the loads do not wait on each other.
  constexpr int NUB = NV * S3, NFS = 6 * NV * S2;
  constexpr int PU = (NUB + FV2_THREADS - 1) / FV2_THREADS;
  constexpr int PF = (NFS + FV2_THREADS - 1) / FV2_THREADS;
  constexpr int PJ = (NP3 + FV2_THREADS - 1) / FV2_THREADS;
  const double* ub = m.ubar + (size_t)e * NUB;
  const double* fvs = m.fvside + (size_t)e * NFS;
  double xu[PU], xf[PF], xj[PJ];
#pragma unroll
  for (int i = 0; i < PU; ++i) {
    const int r = t + i * FV2_THREADS;
    xu[i] = ub[r < NUB ? r : NUB - 1];
  }
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    const int r = t + i * FV2_THREADS;
    xf[i] = fvs[r < NFS ? r : NFS - 1];
  }
#pragma unroll
  for (int i = 0; i < PJ; ++i) {
    const int r = t + i * FV2_THREADS;
    xj[i] = m.metric[9 * m.n_node + base + (r < NP3 ? r : NP3 - 1)];
  }
  const double* nrm = m.fvnorm + (size_t)e * 9 * NIF;
  const bool active = t < S3;
  const int s0 = t % NFV, s1 = (t / NFV) % NFV, s2 = t / S2;
  double nd[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int sd = d == 0 ? s0 : (d == 1 ? s1 : s2);
    const int ta = d == 2 ? s1 : s2, tb = d == 0 ? s1 : s0;
    const bool has = active && sd < NFV - 1;
    const int k = has ? (sd * NFV + ta) * NFV + tb : 0;     // an in-range index either way
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double x = nrm[(d * 3 + c) * NIF + k];
      nd[d][c] = has ? x : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < PU; ++i) {
    const int r = t + i * FV2_THREADS;
    if (r < NUB) sU[r] = xu[i];
  }
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    const int r = t + i * FV2_THREADS;
    if (r < NFS) sF[r] = xf[i];
  }
#pragma unroll
  for (int i = 0; i < PJ; ++i) {
    const int r = t + i * FV2_THREADS;
    if (r < NP3) sJ[r] = xj[i];
  }
  double dC[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) dC[v] = 0.0;
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int sd = d == 0 ? s0 : (d == 1 ? s1 : s2);
    const int stride = d == 0 ? 1 : (d == 1 ? NFV : S2);
    const int ta = d == 2 ? s1 : s2, tb = d == 0 ? s1 : s0;     // tangential (slower, faster)
    const int fidx = ta * NFV + tb;                            // face-grid index on the sides
    if (active && sd < NFV - 1) {
      double uL[NV], uR[NV], F[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        uL[v] = sU[v * S3 + t];
        uR[v] = sU[v * S3 + t + stride];
      }
      riemann<NV>(prm.face_flux_fv, prm.volume_flux, uL, uR, nd[d][0], nd[d][1], nd[d][2], m.gas, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) sG[v * S3 + t] = F[v];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double hi = sd < NFV - 1 ? sG[v * S3 + t] : sF[((2 * d + 1) * NV + v) * S2 + fidx];
        const double lo = sd > 0 ? sG[v * S3 + t - stride] : -sF[((2 * d) * NV + v) * S2 + fidx];
        dC[v] -= hi - lo;
      }
    }
    __syncthreads();
  }
  // nodal form: V3^+(dC) / (h^3 J), three one-dimensional contractions; each
  // thread keeps one input line in registers and forms all NP outputs along
  // the contracted axis
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sG[v * S3 + t] = dC[v];
  }
  __syncthreads();
  for (int q = t; q < NV * S2; q += FV2_THREADS) {              // [v][s2][s1][c] -> [v][s2][s1][i]
    double x[NFV];
#pragma unroll
    for (int c = 0; c < NFV; ++c) x[c] = sG[q * NFV + c];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NFV; ++c) acc += sVp[i * NFV + c] * x[c];
      sU[q * NP + i] = acc;
    }
  }
  __syncthreads();
  for (int r = t; r < NV * NFV * NP; r += FV2_THREADS) {       // [v][s2][c][i] -> [v][s2][j][i]
    const int i = r % NP, q = r / NP;                          // q = v*NFV + s2
    double x[NFV];
#pragma unroll
    for (int c = 0; c < NFV; ++c) x[c] = sU[(q * NFV + c) * NP + i];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NFV; ++c) acc += sVp[j * NFV + c] * x[c];
      sG[(q * NP + j) * NP + i] = acc;
    }
  }
  __syncthreads();
  const double ih3 = 1.0 / (h * h * h);
  for (int r = t; r < NV * NP * NP; r += FV2_THREADS) {       // [v][c][j][i] -> [v][k][j][i]
    const int ij = r % (NP * NP), v = r / (NP * NP);
    double x[NFV];
#pragma unroll
    for (int c = 0; c < NFV; ++c) x[c] = sG[(v * NFV + c) * NP * NP + ij];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NFV; ++c) acc += sVp[k * NFV + c] * x[c];
      const int node = k * NP * NP + ij;
      m.rfv[v * m.n_node + base + node] = acc * ih3 / sJ[node];
    }
  }
}

// ---------------------------------------------------------------------------
// modal decay indicator and blending factor (one element per 64-lane workgroup)
// ---------------------------------------------------------------------------
// Lanes per element of the indicator: one wave up to N = 4, two waves above.
template <int N>
constexpr int ind_threads() { return (N + 1) * (N + 1) * (N + 1) >= 216 ? 128 : 64; }

// An empty asm statement with a memory clobber: LDS values read after it are
// read there, so the operator rows of the modal transforms are not hoisted
// out of their line loops and held in registers (64 doubles at N = 7).
__device__ __forceinline__ void lds_reload() { asm volatile("" ::: "memory"); }

template <int N, int NV>
__global__ void __launch_bounds__(ind_threads<N>())
indicator_kernel(MeshView m, ParamsDev prm, const int32_t* __restrict__ elist, int count,
                 const double* __restrict__ u, double* __restrict__ alpha, double* __restrict__ ind) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP;
  constexpr int NFMAX = NV == 6 ? 3 : 2;       // p, rho (and Y)
  __shared__ double sq[NFMAX * NP3];
  __shared__ double sw[NFMAX * NP3];
  __shared__ double sVi[NP * NP];
  __shared__ double sE[NFMAX * 3 * NP];
  __shared__ double sI[NFMAX * 3];
  const int idx = blockIdx.x;
  if (idx >= count) return;
  const int e = elist[idx];
  const int64_t base = m.elem_offset[e];
  for (int t = threadIdx.x; t < NP * NP; t += blockDim.x) sVi[t] = m.ops[m.tab.vleg_inv[N] + t];
  // the state is read once; every selected variable (in the order p, rho, Y)
  // goes to its own field and the three transforms act on all fields at once
  const bool use_p = prm.ind_vars & 1, use_r = prm.ind_vars & 2, use_y = NV == 6 && (prm.ind_vars & 4);
  const int nf = (use_p ? 1 : 0) + (use_r ? 1 : 0) + (use_y ? 1 : 0);
  for (int t = threadIdx.x; t < NP3; t += blockDim.x) {
    double uu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uu[v] = u[v * m.n_node + base + t];
    const Prim q = cons2prim<NV>(uu, m.gas);
    int f = 0;
    if (use_p) sq[(f++) * NP3 + t] = q.p;
    if (use_r) sq[(f++) * NP3 + t] = q.rho;
    if (use_y) sq[f * NP3 + t] = q.Y;
  }
  __syncthreads();
  // modal coefficients: V_Leg^{-1} along each axis, one input line per thread
  // forming all NP outputs along it
  for (int r = threadIdx.x; r < nf * NP * NP; r += blockDim.x) {        // [f][k][j][c] -> [f][k][j][m0]
    lds_reload();
    double x[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = sq[r * NP + c];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) acc += sVi[o * NP + c] * x[c];
      sw[r * NP + o] = acc;
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nf * NP * NP; r += blockDim.x) {        // [f][k][c][m0] -> [f][k][m1][m0]
    const int m0 = r % NP, kf = r / NP;
    lds_reload();
    double x[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = sw[(kf * NP + c) * NP + m0];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) acc += sVi[o * NP + c] * x[c];
      sq[(kf * NP + o) * NP + m0] = acc;
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nf * NP * NP; r += blockDim.x) {        // [f][c][m1][m0] -> [f][m2][m1][m0]
    const int m01 = r % (NP * NP), f = r / (NP * NP);
    lds_reload();
    double x[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) x[c] = sq[f * NP3 + c * NP * NP + m01];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) acc += sVi[o * NP + c] * x[c];
      sw[f * NP3 + o * NP * NP + m01] = acc;
    }
  }
  __syncthreads();
  // energies per field, direction and mode (one lane each; the index is base +
  // a sa + b sb with the strides of the two directions summed over)
  for (int t = threadIdx.x; t < nf * 3 * NP; t += blockDim.x) {
    const int mm = t % NP, d = (t / NP) % 3, f = t / (3 * NP);
    const int base = d == 0 ? mm : (d == 1 ? mm * NP : mm * NP * NP);
    const int sa = d == 0 ? NP : 1, sb = d == 2 ? NP : NP * NP;
    const double* w = sw + f * NP3 + base;
    double s = 0.0;
    for (int a = 0; a < NP; ++a)
      for (int b = 0; b < NP; ++b) {
        const double x = w[a * sa + b * sb];
        s += x * x;
      }
    sE[t] = s;
  }
  __syncthreads();
  // ln of the energy shares, one lane per entry
  for (int t = threadIdx.x; t < nf * 3 * NP; t += blockDim.x) {
    const double* E = sE + (t / NP) * NP;
    double tot = 0.0;
    for (int mm = 0; mm < NP; ++mm) tot += E[mm];
    sq[t] = tot < 1e-300 ? INFINITY : log(fmax(sE[t] / tot, 1e-30));
  }
  __syncthreads();
  // decay slope per field and direction: least-squares line through (m, y_m)
  for (int t = threadIdx.x; t < nf * 3; t += blockDim.x) {
    const double* y = sq + t * NP;
    double res;
    if (y[0] == INFINITY) {                    // no energy at all
      res = INFINITY;
    } else {
      const double mbar = 0.5 * N;
      double ybar = 0.0;
      for (int mm = 0; mm < NP; ++mm) ybar += y[mm];
      ybar /= NP;
      double sxy = 0.0, sxx = 0.0;
      for (int mm = 0; mm < NP; ++mm) {
        sxy += (mm - mbar) * (y[mm] - ybar);
        sxx += (mm - mbar) * (mm - mbar);
      }
      res = fabs(-sxy / sxx);
    }
    sI[t] = res;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double Imin = INFINITY;
    for (int t = 0; t < nf * 3; ++t) Imin = fmin(Imin, sI[t]);
    const double x = (Imin - prm.ind_T) / prm.ind_dT;
    double a;
    if (x <= -1.0) a = 1.0;
    else if (x >= 1.0) a = 0.0;
    else a = 0.5 * (1.0 - sin(0.5 * M_PI * x));
    alpha[e] = a;
    if (ind) ind[e] = Imin;
  }
}

// ---------------------------------------------------------------------------
// adjoint (vector-Jacobian product) with alpha frozen.
// Forward: R = (1 - alpha) R^DG + alpha R^FV with
//   R^DG_i = -(1/J_i) [ sum_d sum_{m != i} 2 D_im F#d(u_i, u_m) + lift_i(F_side) ].
// With a_i = -(1 - alpha) w_i / J_i and the symmetry of F#,
//   g_j = sum_d sum_{m != j} (d F#d(u_j, u_m) / d u_j)^T (2 D_jm a_j + 2 D_mj a_m),
// evaluated per node through the flux record: the record adjoint is summed
// over the pairs and mapped to u once (make_adj).  As in the forward kernel the
// pair terms use the metric sum Ja_i + Ja_m with weights D instead of the mean
// with weights 2 D.  The lift gives the side cotangents a_i / w_0 at the
// boundary nodes.
// ---------------------------------------------------------------------------
template <int N, int NV, class FLUX>
__global__ void __launch_bounds__(Geo<N>::EPB * Geo<N>::NP3, 4)   // 4 waves per SIMD: two workgroups per CU
vjp_volume_kernel(MeshView m, const int32_t* __restrict__ elist, int count,
                  const double* __restrict__ u, const double* __restrict__ alpha,
                  const double* __restrict__ w, double* __restrict__ g) {
  using G = Geo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3, EPB = G::EPB;
  constexpr int NA = FLUX::NA;
  // The partners' metric moves by wave shuffles where the lines lie inside one
  // wave (xi_1, xi_2 when N+1 divides 64; xi_3 when (N+1)^3 does); only the
  // other components are kept in LDS.
  constexpr bool SH01 = 64 % NP == 0, SH2 = 64 % NP3 == 0;
  constexpr int JL = SH01 ? (SH2 ? 1 : 3) : 9;
  __shared__ double sD[NP * NP];
  __shared__ double sAux[EPB][NA][NP3];
  __shared__ double sJa[EPB][JL][NP3];
  __shared__ double sA[EPB][NV][NP3];

  const int tid = threadIdx.x;
  const int slot = tid / NP3;
  const int node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  const bool active = idx < count;
  // metric sums with weights D_im, as in the forward kernel
  for (int t = tid; t < NP * NP; t += blockDim.x) sD[t] = m.ops[m.tab.D[N] + t];

  int e = 0;
  int64_t base = 0;
  double uo[NV], ame[NV];
  if (active) {
    e = elist[idx];
    base = m.elem_offset[e] + node;
#pragma unroll
    for (int v = 0; v < NV; ++v) uo[v] = u[v * m.n_node + base];
    const Prim q = cons2prim<NV>(uo, m.gas);
    double r[NA];
    FLUX::template make<NV>(q, r);
#pragma unroll
    for (int a = 0; a < NA; ++a) sAux[slot][a][node] = r[a];
    if constexpr (JL == 9) {
#pragma unroll
      for (int c = 0; c < 9; ++c) sJa[slot][c][node] = m.metric[c * m.n_node + base];
    } else if constexpr (JL == 3) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sJa[slot][c][node] = m.metric[(6 + c) * m.n_node + base];
    }
    const double al = alpha ? alpha[e] : 0.0;
    const double sc = -(1.0 - al) / m.metric[9 * m.n_node + base];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ame[v] = sc * w[v * m.n_node + base];
      sA[slot][v][node] = ame[v];
    }
  }
  __syncthreads();
  if (!active) return;

  const int i = node % NP, j = (node / NP) % NP, kk = node / NP2;
  double me[NA], ab[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    me[a] = sAux[slot][a][node];
    ab[a] = 0.0;
  }
  const int lane = tid & 63;
  auto direction = [&](auto dtag) {
    constexpr int d = decltype(dtag)::value;
    constexpr bool sh = d < 2 ? SH01 : SH2;
    constexpr int stride = d == 0 ? 1 : (d == 1 ? NP : NP2);
    const int id = d == 0 ? i : (d == 1 ? j : kk);
    const double ja1 = m.metric[(3 * d + 0) * m.n_node + base];
    const double ja2 = m.metric[(3 * d + 1) * m.n_node + base];
    const double ja3 = m.metric[(3 * d + 2) * m.n_node + base];
#pragma unroll 1
    for (int o = 1; o < NP; ++o) {
      int mm = id + o;
      if (mm >= NP) mm -= NP;
      const int pn = node + (mm - id) * stride;
      double other[NA], c[NV];
#pragma unroll
      for (int a = 0; a < NA; ++a) other[a] = sAux[slot][a][pn];
      const double cme = sD[id * NP + mm], cot = sD[mm * NP + id];
#pragma unroll
      for (int v = 0; v < NV; ++v) c[v] = cme * ame[v] + cot * sA[slot][v][pn];
      double b1, b2, b3;
      if constexpr (sh) {
        const int sl = (lane + pn - node) & 63;
        b1 = __shfl(ja1, sl);
        b2 = __shfl(ja2, sl);
        b3 = __shfl(ja3, sl);
      } else if constexpr (JL == 9) {
        b1 = sJa[slot][3 * d + 0][pn];
        b2 = sJa[slot][3 * d + 1][pn];
        b3 = sJa[slot][3 * d + 2][pn];
      } else {                                 // JL == 3: only xi_3 is kept in LDS
        b1 = sJa[slot][0][pn];
        b2 = sJa[slot][1][pn];
        b3 = sJa[slot][2][pn];
      }
      FLUX::template flux_adj_a<NV>(me, other, ja1 + b1, ja2 + b2, ja3 + b3, m.gas, c, ab);
    }
  };
  direction(std::integral_constant<int, 0>{});
  direction(std::integral_constant<int, 1>{});
  direction(std::integral_constant<int, 2>{});
  double ub[NV];
  FLUX::template make_adj<NV>(uo, m.gas, ab, ub);
#pragma unroll
  for (int v = 0; v < NV; ++v) g[v * m.n_node + base] = ub[v];

  // cotangents of the side fluxes through the lift
  const double inv_w0 = 1.0 / m.ops[m.tab.w[N]];
  double* fs = m.fside + m.side_off[e];
  auto put_side = [&](int s, int fidx) {
#pragma unroll
    for (int v = 0; v < NV; ++v) fs[(s * NV + v) * NP2 + fidx] = ame[v] * inv_w0;
  };
  if (i == 0) put_side(0, kk * NP + j);
  if (i == N) put_side(1, kk * NP + j);
  if (j == 0) put_side(2, kk * NP + i);
  if (j == N) put_side(3, kk * NP + i);
  if (kk == 0) put_side(4, j * NP + i);
  if (kk == N) put_side(5, j * NP + i);
}

// Adjoint of the FV residual of a blended element: from w to the cotangents of
// its sub-cell means (internal sub-faces) and of its boundary sub-face fluxes.
//   R^FV = V3^+(dC) / (h^3 J)           ->  dCb = V3^+^T (alpha w / (h^3 J))
//   dC[s] -= G[s+1] - G[s] along each d  ->  Gb[q] = dCb[q] - dCb[q-1]
//   internal G = Riemann(ubar_l, ubar_r) ->  ubar_bar via the Riemann VJP
//   G[0] = -F_fv(side 2d), G[NFV] = F_fv(side 2d+1)
template <int N, int NV>
__global__ void __launch_bounds__(FV_THREADS)
vjp_fv_kernel(MeshView m, ParamsDev prm, const int32_t* __restrict__ elist, int count,
              const double* __restrict__ alpha, const double* __restrict__ w) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP;
  constexpr int S3MAX = MAXFV * MAXFV * MAXFV;
  constexpr int NRM = 3 * (MAXFV + 1) * MAXFV * MAXFV;
  __shared__ double sU[NV * S3MAX];
  __shared__ double sC[NV * S3MAX];
  __shared__ double sUb[NV * S3MAX];
  __shared__ double sJa[9 * NP3];
  __shared__ double sNrm[NRM];
  __shared__ double sScr[NRM];
  __shared__ double sV[MAXFV * (MAXN + 1)];
  __shared__ double sVpT[MAXFV * (MAXN + 1)];
  __shared__ double sI[(MAXFV + 1) * (MAXN + 1)];

  const int idx = blockIdx.x;
  if (idx >= count) return;
  const int e = elist[idx];
  const double al = alpha[e];
  if (!(al > 0.0)) return;
  const int NFV = m.n_fv;
  const int S2 = NFV * NFV, S3 = S2 * NFV;
  const double h = 2.0 / NFV;
  const int64_t base = m.elem_offset[e];
  const double* ub = m.ubar + (size_t)e * NV * S3;
  for (int t = threadIdx.x; t < NV * S3; t += blockDim.x) sU[t] = ub[t];
  for (int t = threadIdx.x; t < 9 * NP3; t += blockDim.x)
    sJa[t] = m.metric[(t / NP3) * m.n_node + base + (t % NP3)];
  for (int t = threadIdx.x; t < NFV * NP; t += blockDim.x) {
    sV[t] = m.ops[m.tab.dg2fv[N] + t];
    sVpT[t] = m.ops[m.tab.fv2dgT[N] + t];
  }
  for (int t = threadIdx.x; t < (NFV + 1) * NP; t += blockDim.x) sI[t] = m.ops[m.tab.face_interp[N] + t];
  const double ih3 = 1.0 / (h * h * h);
  for (int t = threadIdx.x; t < NP3; t += blockDim.x) {
    const double sc = al * ih3 / m.metric[9 * m.n_node + base + t];
    for (int v = 0; v < NV; ++v) sUb[v * NP3 + t] = sc * w[v * m.n_node + base + t];
  }
  __syncthreads();
  // dCb = (V^+)^T (x) (V^+)^T (x) (V^+)^T q
  contract_axis(sUb, sC, sVpT, NFV, NP, NV, NP, NP, NP, 0);
  __syncthreads();
  contract_axis(sC, sUb, sVpT, NFV, NP, NV, NP, NP, NFV, 1);
  __syncthreads();
  contract_axis(sUb, sC, sVpT, NFV, NP, NV, NP, NFV, NFV, 2);
  __syncthreads();
  for (int t = threadIdx.x; t < NV * S3; t += blockDim.x) sUb[t] = 0.0;

  double* fvs = m.fvside + (size_t)e * 6 * NV * S2;
  for (int d = 0; d < 3; ++d) {
    __syncthreads();
    // sub-face normals, exactly as in the forward residual
    const double* src = sJa + 3 * d * NP3;
    contract_axis(src, sScr, sI, NFV + 1, NP, 3, NP, NP, NP, d);
    __syncthreads();
    int a2 = (d == 2) ? NFV + 1 : NP, a1 = (d == 1) ? NFV + 1 : NP, a0 = (d == 0) ? NFV + 1 : NP;
    const int ta = (d == 0) ? 1 : 0;
    const int tb = (d == 2) ? 1 : 2;
    contract_axis(sScr, sNrm, sV, NFV, NP, 3, a2, a1, a0, ta);
    __syncthreads();
    if (ta == 0) a0 = NFV; else a1 = NFV;
    contract_axis(sNrm, sScr, sV, NFV, NP, 3, a2, a1, a0, tb);
    __syncthreads();
    if (tb == 1) a1 = NFV; else a2 = NFV;
    const int nn = a2 * a1 * a0;
    for (int t = threadIdx.x; t < 3 * nn; t += blockDim.x) sNrm[t] = sScr[t] * (h * h);
    __syncthreads();
    const int stride = d == 0 ? 1 : (d == 1 ? NFV : S2);
    for (int t = threadIdx.x; t < S3; t += blockDim.x) {
      const int s0 = t % NFV, s1 = (t / NFV) % NFV, s2 = t / S2;
      const int sd = d == 0 ? s0 : (d == 1 ? s1 : s2);
      int lo;
      if (d == 0) lo = (s2 * NFV + s1) * (NFV + 1) + s0;
      else if (d == 1) lo = (s2 * (NFV + 1) + s1) * NFV + s0;
      else lo = (s2 * NFV + s1) * NFV + s0;
      const int istr = d == 0 ? 1 : (d == 1 ? NFV : S2);   // interface stride along d
      const int hi = lo + istr;
      double acc[NV];
      for (int v = 0; v < NV; ++v) acc[v] = 0.0;
      double uc[NV];
      for (int v = 0; v < NV; ++v) uc[v] = sU[v * S3 + t];
      if (sd + 1 <= NFV - 1) {   // internal interface on the +d side: this cell is its left state
        double un[NV], Gb[NV], r[NV];
        for (int v = 0; v < NV; ++v) {
          un[v] = sU[v * S3 + t + stride];
          Gb[v] = sC[v * S3 + t + stride] - sC[v * S3 + t];
        }
        riemann_vjp_side<NV>(0, prm.face_flux_fv, prm.volume_flux, uc, un, sNrm[hi], sNrm[nn + hi],
                             sNrm[2 * nn + hi], m.gas, Gb, r);
        for (int v = 0; v < NV; ++v) acc[v] += r[v];
      }
      if (sd >= 1) {             // internal interface on the -d side: this cell is its right state
        double un[NV], Gb[NV], r[NV];
        for (int v = 0; v < NV; ++v) {
          un[v] = sU[v * S3 + t - stride];
          Gb[v] = sC[v * S3 + t] - sC[v * S3 + t - stride];
        }
        riemann_vjp_side<NV>(1, prm.face_flux_fv, prm.volume_flux, un, uc, sNrm[lo], sNrm[nn + lo],
                             sNrm[2 * nn + lo], m.gas, Gb, r);
        for (int v = 0; v < NV; ++v) acc[v] += r[v];
      }
      for (int v = 0; v < NV; ++v) sUb[v * S3 + t] += acc[v];
      // boundary sub-face flux cotangents
      int fp, fq;
      if (d == 0) { fp = s1; fq = s2; }
      else if (d == 1) { fp = s0; fq = s2; }
      else { fp = s0; fq = s1; }
      if (sd == 0)
        for (int v = 0; v < NV; ++v) fvs[((2 * d) * NV + v) * S2 + fq * NFV + fp] = -sC[v * S3 + t];
      if (sd == NFV - 1)
        for (int v = 0; v < NV; ++v) fvs[((2 * d + 1) * NV + v) * S2 + fq * NFV + fp] = -sC[v * S3 + t];
    }
  }
  __syncthreads();
  double* out = m.ubar_bar + (size_t)e * NV * S3;
  for (int t = threadIdx.x; t < NV * S3; t += blockDim.x) out[t] = sUb[t];
}

// Gather of the trace cotangents (left in fside by the face adjoint) into g,
// one thread per node.
template <int N, int NV>
__global__ void __launch_bounds__(Geo<N>::EPB * Geo<N>::NP3)
vjp_trace_kernel(MeshView m, const int32_t* __restrict__ elist, int count, double* __restrict__ g) {
  using G = Geo<N>;
  constexpr int NP = G::NP, NP2 = G::NP2, NP3 = G::NP3, EPB = G::EPB;
  const int tid = threadIdx.x;
  const int slot = tid / NP3;
  const int node = tid - slot * NP3;
  const int idx = blockIdx.x * EPB + slot;
  if (idx >= count) return;
  const int e = elist[idx];
  const int i = node % NP, j = (node / NP) % NP, kk = node / NP2;
  if (!(i == 0 || i == N || j == 0 || j == N || kk == 0 || kk == N)) return;
  const int64_t base = m.elem_offset[e] + node;
  const double* fs = m.fside + m.side_off[e];
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  auto add_side = [&](int s, int fidx) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += fs[(s * NV + v) * NP2 + fidx];
  };
  if (i == 0) add_side(0, kk * NP + j);
  if (i == N) add_side(1, kk * NP + j);
  if (j == 0) add_side(2, kk * NP + i);
  if (j == N) add_side(3, kk * NP + i);
  if (kk == 0) add_side(4, j * NP + i);
  if (kk == N) add_side(5, j * NP + i);
#pragma unroll
  for (int v = 0; v < NV; ++v) g[v * m.n_node + base] += acc[v];
}

// Adjoint of the sub-cell means of a blended element:
//   ubar = V3(J u) / V3(J)  ->  g += J (V^T (x) V^T (x) V^T)(ubar_bar / V3(J)),
// where ubar_bar collects the internal part (vjp_fv) and the boundary-layer
// trace cotangents of the six sides (left in fvside by the face adjoint).
template <int N, int NV>
__global__ void __launch_bounds__(FV_THREADS)
vjp_fv_gather_kernel(MeshView m, const int32_t* __restrict__ elist, int count,
                     const double* __restrict__ alpha, double* __restrict__ g) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP;
  constexpr int CAP = (NV + 1) * MAXFV * MAXFV * MAXFV;
  __shared__ double bufA[CAP];
  __shared__ double bufB[CAP];
  __shared__ double sV[MAXFV * (MAXN + 1)];
  __shared__ double sVT[MAXFV * (MAXN + 1)];
  const int idx = blockIdx.x;
  if (idx >= count) return;
  const int e = elist[idx];
  if (!(alpha[e] > 0.0)) return;
  const int NFV = m.n_fv;
  const int S2 = NFV * NFV, S3 = S2 * NFV;
  const int64_t base = m.elem_offset[e];
  for (int t = threadIdx.x; t < NFV * NP; t += blockDim.x) {
    sV[t] = m.ops[m.tab.dg2fv[N] + t];
    sVT[t] = m.ops[m.tab.dg2fvT[N] + t];
  }
  for (int t = threadIdx.x; t < NP3; t += blockDim.x) bufA[t] = m.metric[9 * m.n_node + base + t];
  __syncthreads();
  // V3(J)
  contract_axis(bufA, bufB, sV, NFV, NP, 1, NP, NP, NP, 0);
  __syncthreads();
  contract_axis(bufB, bufA, sV, NFV, NP, 1, NP, NP, NFV, 1);
  __syncthreads();
  contract_axis(bufA, bufB, sV, NFV, NP, 1, NP, NFV, NFV, 2);   // bufB[0..S3) = V3(J)
  __syncthreads();
  const double* ubb = m.ubar_bar + (size_t)e * NV * S3;
  const double* fvs = m.fvside + (size_t)e * 6 * NV * S2;
  for (int t = threadIdx.x; t < S3; t += blockDim.x) {
    const int s0 = t % NFV, s1 = (t / NFV) % NFV, s2 = t / S2;
    const double ivol = 1.0 / bufB[t];
    for (int v = 0; v < NV; ++v) {
      double x = ubb[v * S3 + t];
      if (s0 == 0) x += fvs[(0 * NV + v) * S2 + s2 * NFV + s1];
      if (s0 == NFV - 1) x += fvs[(1 * NV + v) * S2 + s2 * NFV + s1];
      if (s1 == 0) x += fvs[(2 * NV + v) * S2 + s2 * NFV + s0];
      if (s1 == NFV - 1) x += fvs[(3 * NV + v) * S2 + s2 * NFV + s0];
      if (s2 == 0) x += fvs[(4 * NV + v) * S2 + s1 * NFV + s0];
      if (s2 == NFV - 1) x += fvs[(5 * NV + v) * S2 + s1 * NFV + s0];
      bufA[v * S3 + t] = x * ivol;
    }
  }
  __syncthreads();
  contract_axis(bufA, bufB, sVT, NP, NFV, NV, NFV, NFV, NFV, 0);
  __syncthreads();
  contract_axis(bufB, bufA, sVT, NP, NFV, NV, NFV, NFV, NP, 1);
  __syncthreads();
  contract_axis(bufA, bufB, sVT, NP, NFV, NV, NFV, NP, NP, 2);
  __syncthreads();
  for (int t = threadIdx.x; t < NP3; t += blockDim.x) {
    const double J = m.metric[9 * m.n_node + base + t];
    for (int v = 0; v < NV; ++v) g[v * m.n_node + base + t] += J * bufB[v * NP3 + t];
  }
}

// ---------------------------------------------------------------------------
// positivity-preserving limiter of Zhang and Shu (Section 3.5), one element per
// workgroup, single species.  With the element mean ubar = sum w J u / sum w J,
// each point value becomes ubar + theta (u_P - ubar): first the density alone
// with theta_rho = min(1, min_P (rhobar - eps) / (rhobar - rho_P)) over points
// with rho_P < eps, then every variable with theta_p = min_P t_P, t_P the root
// in (0, 1) of p(ubar + t (u~_P - ubar)) = eps (rho p / (gamma - 1) is a
// quadratic in t) over points whose pressure is below eps after step 1.
// eps = 1e-10 rhobar for density and 1e-10 p(ubar) for pressure (a fixed 1e-13 lies
// below the rounding of E - |m|^2 / (2 rho) when E is of order one).
// Points: the LGL nodes, and on blended elements the J-weighted sub-cell means
// in m.ubar (written for the current state before this kernel).  theta_out[e]
// receives min(theta_rho, theta_p), or -1 when the mean itself has rho <= 0 or
// p <= 0 (left unchanged).  An element within the bounds is not written.
// Reductions: wave shuffles, then LDS across the workgroup's waves.
// ---------------------------------------------------------------------------
template <int N>
constexpr int lim_threads() { return (N + 1) * (N + 1) * (N + 1) > 64 ? 256 : 64; }
constexpr double LIM_EPS_REL = 1e-10;

template <int T_>
__device__ __forceinline__ double block_reduce(double v, bool is_min, double* sRed) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl(v, lane ^ off);
    v = is_min ? (o < v ? o : v) : v + o;
  }
  if constexpr (T_ > 64) {
    __syncthreads();                           // sRed free from the previous reduction
    if (lane == 0) sRed[wave] = v;
    __syncthreads();
    v = sRed[0];
#pragma unroll
    for (int w = 1; w < T_ / 64; ++w) v = is_min ? (sRed[w] < v ? sRed[w] : v) : v + sRed[w];
  }
  return v;
}

__device__ __forceinline__ double lim_pressure(const double* w, double gamma) {
  return (gamma - 1.0) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0]);
}

// root in (0, 1) of p(ub + t d) = eps for a point below eps (the mean above it)
__device__ __forceinline__ double lim_root(const double* ub, const double* d, double eps, double gamma) {
  const double g1 = 1.0 / (gamma - 1.0);
  const double a = d[0] * d[4] - 0.5 * (d[1] * d[1] + d[2] * d[2] + d[3] * d[3]);
  const double b = ub[0] * d[4] + ub[4] * d[0] - (ub[1] * d[1] + ub[2] * d[2] + ub[3] * d[3]) - eps * g1 * d[0];
  const double c = ub[0] * ub[4] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2] + ub[3] * ub[3]) - eps * g1 * ub[0];
  if (a == 0.0) {
    const double t = -c / b;
    return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  }
  double disc = b * b - 4.0 * a * c;
  if (disc < 0.0) disc = 0.0;
  const double q = -0.5 * (b + (b >= 0.0 ? 1.0 : -1.0) * sqrt(disc));
  const double r1 = q / a;
  const double r2 = q != 0.0 ? c / q : 2.0;
  if (r2 >= 0.0 && r2 <= 1.0) return r2;
  if (r1 >= 0.0 && r1 <= 1.0) return r1;
  return 0.0;
}

template <int N>
__global__ void __launch_bounds__(lim_threads<N>())
limiter_kernel(MeshView m, const int32_t* __restrict__ elist, int count, double* __restrict__ u,
               const double* __restrict__ alpha, double* __restrict__ theta_out) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP, TH = lim_threads<N>();
  __shared__ double sw[NP];
  __shared__ double sRed[TH / 64];
  const int idx = blockIdx.x;
  if (idx >= count) return;
  const int e = elist[idx];
  const int64_t base = m.elem_offset[e];
  const int t0 = threadIdx.x;
  if (t0 < NP) sw[t0] = m.ops[m.tab.w[N] + t0];
  __syncthreads();
  const double gamma = m.gas.gamma;
  // element mean of the conserved variables
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = t0; t < NP3; t += TH) {
    const int i = t % NP, j = (t / NP) % NP, k = t / (NP * NP);
    const double wJ = sw[i] * sw[j] * sw[k] * m.metric[9 * m.n_node + base + t];
#pragma unroll
    for (int v = 0; v < 5; ++v) s[v] += wJ * u[v * m.n_node + base + t];
    s[5] += wJ;
  }
  double ub[5];
  const double vol = block_reduce<TH>(s[5], false, sRed);
#pragma unroll
  for (int v = 0; v < 5; ++v) ub[v] = block_reduce<TH>(s[v], false, sRed) / vol;
  const double pb = lim_pressure(ub, gamma);
  if (!(ub[0] > 0.0) || !(pb > 0.0)) {
    if (theta_out && t0 == 0) theta_out[e] = -1.0;
    return;
  }
  const double eps_r = LIM_EPS_REL * ub[0];
  const double eps_p = LIM_EPS_REL * pb;
  const bool sub = alpha && alpha[e] > 0.0;
  const int S3 = m.n_fv * m.n_fv * m.n_fv;
  const int npts = NP3 + (sub ? S3 : 0);
  const double* ubar_e = m.ubar + (size_t)e * 5 * S3;
  auto point = [&](int t, double* w) {
    if (t < NP3) {
#pragma unroll
      for (int v = 0; v < 5; ++v) w[v] = u[v * m.n_node + base + t];
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) w[v] = ubar_e[v * S3 + (t - NP3)];
    }
  };
  // step 1: density
  double th = 1.0;
  for (int t = t0; t < npts; t += TH) {
    double w[5];
    point(t, w);
    if (w[0] < eps_r) {
      const double r = (ub[0] - eps_r) / (ub[0] - w[0]);
      th = r < th ? r : th;
    }
  }
  const double th_r = block_reduce<TH>(th, true, sRed);
  // step 2: pressure of the density-limited points
  th = 1.0;
  for (int t = t0; t < npts; t += TH) {
    double w[5];
    point(t, w);
    w[0] = ub[0] + th_r * (w[0] - ub[0]);
    if (lim_pressure(w, gamma) < eps_p) {
      double d[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) d[v] = w[v] - ub[v];
      const double r = lim_root(ub, d, eps_p, gamma);
      th = r < th ? r : th;
    }
  }
  const double th_p = block_reduce<TH>(th, true, sRed);
  if (theta_out && t0 == 0) theta_out[e] = th_r < th_p ? th_r : th_p;
  if (!(th_r < 1.0) && !(th_p < 1.0)) return;
  for (int t = t0; t < NP3; t += TH) {
    double w[5];
    point(t, w);
    w[0] = ub[0] + th_r * (w[0] - ub[0]);
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v * m.n_node + base + t] = ub[v] + th_p * (w[v] - ub[v]);
  }
}

// ---------------------------------------------------------------------------
// FV-stored elements (Sections 3.1.2 and 3.2): the sub-cell means of J, set up
// once, and the switch of an element between its nodal DG state and its
// sub-cell means.
// ---------------------------------------------------------------------------
constexpr int FVS_THREADS = 512;

// Tensor map A (x) A (x) A (A: NOUT x NIN, row-major) of F fields on LDS:
// in: a[F][NIN^3] (c fastest) -> out: b[F][NOUT^3]; a is overwritten.  One
// one-dimensional contraction per pass, each thread holding one input line
// in registers and forming every output along the contracted axis.
template <int NIN, int NOUT, int F, int TH>
__device__ void map3(const double* __restrict__ A, double* a, double* b) {
  const int t = threadIdx.x;
  for (int r = t; r < F * NIN * NIN; r += TH) {                // axis 0: [f][k][j][c] -> [f][k][j][s0]
    double x[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) x[c] = a[r * NIN + c];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NIN; ++c) acc += A[o * NIN + c] * x[c];
      b[r * NOUT + o] = acc;
    }
  }
  __syncthreads();
  for (int r = t; r < F * NIN * NOUT; r += TH) {               // axis 1: [f][k][c][s0] -> [f][k][s1][s0]
    const int s0 = r % NOUT, kf = r / NOUT;
    double x[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) x[c] = b[(kf * NIN + c) * NOUT + s0];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NIN; ++c) acc += A[o * NIN + c] * x[c];
      a[(kf * NOUT + o) * NOUT + s0] = acc;
    }
  }
  __syncthreads();
  for (int r = t; r < F * NOUT * NOUT; r += TH) {              // axis 2: [f][c][s1][s0] -> [f][s2][s1][s0]
    const int s01 = r % (NOUT * NOUT), f = r / (NOUT * NOUT);
    double x[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) x[c] = a[(f * NIN + c) * NOUT * NOUT + s01];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NIN; ++c) acc += A[o * NIN + c] * x[c];
      b[(f * NOUT + o) * NOUT * NOUT + s01] = acc;
    }
  }
  __syncthreads();
}

// m.fvjbar[e] = V3(J) for the elements of one bucket, one element per workgroup.
template <int N, int NFV>
__global__ void __launch_bounds__(FVS_THREADS)
fv_jbar_kernel(MeshView m, const int32_t* __restrict__ elist, int count) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP, S3 = NFV * NFV * NFV;
  constexpr int BIG = NP3 > S3 ? NP3 : S3;
  __shared__ double a[BIG], b[BIG];
  __shared__ double sV[NFV * NP];
  if ((int)blockIdx.x >= count) return;
  const int t = threadIdx.x;
  const int e = elist[blockIdx.x];
  const int64_t base = m.elem_offset[e];
  if (t < NFV * NP) sV[t] = m.ops[m.tab.dg2fv[N] + t];
  for (int r = t; r < NP3; r += FVS_THREADS) a[r] = m.metric[9 * m.n_node + base + r];
  __syncthreads();
  map3<NP, NFV, 1, FVS_THREADS>(sV, a, b);
  for (int r = t; r < S3; r += FVS_THREADS) m.fvjbar[(size_t)e * S3 + r] = b[r];
}

// Switch of the bucket's elements whose flag changes (fv > 0: FV-stored).
//   DG -> FV: ufv = V3(J u) / V3(J)         (J-weighted sub-cell means)
//   FV -> DG: u = V3^+(ufv V3(J)) / J       (least-squares nodal state with those contents)
template <int N, int NFV, int NV>
__global__ void __launch_bounds__(FVS_THREADS)
fv_switch_kernel(MeshView m, const int32_t* __restrict__ elist, int count, double* __restrict__ u,
                 double* __restrict__ ufv, const double* __restrict__ fv_old, const double* __restrict__ fv_new) {
  constexpr int NP = N + 1, NP3 = NP * NP * NP, S3 = NFV * NFV * NFV;
  constexpr int BIG = (NV + 1) * (NP3 > S3 ? NP3 : S3);
  __shared__ double a[BIG], b[BIG];
  __shared__ double sA[NFV * NP];
  if ((int)blockIdx.x >= count) return;
  const int t = threadIdx.x;
  const int e = elist[blockIdx.x];
  const bool was_fv = fv_old[e] > 0.0, is_fv = fv_new[e] > 0.0;
  if (was_fv == is_fv) return;                    // uniform over the workgroup
  const int64_t base = m.elem_offset[e];
  double* ue = ufv + (size_t)e * NV * S3;
  if (is_fv) {
    if (t < NFV * NP) sA[t] = m.ops[m.tab.dg2fv[N] + t];
    for (int r = t; r < NP3; r += FVS_THREADS) {
      const double J = m.metric[9 * m.n_node + base + r];
#pragma unroll
      for (int v = 0; v < NV; ++v) a[v * NP3 + r] = J * u[v * m.n_node + base + r];
      a[NV * NP3 + r] = J;
    }
    __syncthreads();
    map3<NP, NFV, NV + 1, FVS_THREADS>(sA, a, b);
    for (int r = t; r < S3; r += FVS_THREADS) {
      const double ivol = 1.0 / b[NV * S3 + r];
#pragma unroll
      for (int v = 0; v < NV; ++v) ue[v * S3 + r] = b[v * S3 + r] * ivol;
    }
  } else {
    if (t < NFV * NP) sA[t] = m.ops[m.tab.fv2dg[N] + t];
    for (int r = t; r < S3; r += FVS_THREADS) {
      const double jb = m.fvjbar[(size_t)e * S3 + r];
#pragma unroll
      for (int v = 0; v < NV; ++v) a[v * S3 + r] = ue[v * S3 + r] * jb;
    }
    __syncthreads();
    map3<NFV, NP, NV, FVS_THREADS>(sA, a, b);
    for (int r = t; r < NP3; r += FVS_THREADS) {
      const double iJ = 1.0 / m.metric[9 * m.n_node + base + r];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v * m.n_node + base + r] = b[v * NP3 + r] * iJ;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers for this degree
// ---------------------------------------------------------------------------
template <int NV, class FLUX, int V>
static hipError_t launch_elem_v(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                                const double* u, double* uout, const double* alpha, double* ut, double* k,
                                int stage, double dt, double A, double B, int flags, hipStream_t s) {
  constexpr int EPB = elem_epb<kN, V>();
  const int blocks = (count + EPB - 1) / EPB;
  if constexpr (EPB == 1) {
    if (flags & ELEM_FUSE_FACES) {
      hipLaunchKernelGGL((element_kernel<kN, NV, FLUX, EPB, true>), dim3(blocks), dim3(EPB * Geo<kN>::NP3), 0, s, m,
                         p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, flags);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((element_kernel<kN, NV, FLUX, EPB, false>), dim3(blocks), dim3(EPB * Geo<kN>::NP3), 0, s, m,
                     p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, flags);
  return hipGetLastError();
}

template <int NV, class FLUX>
static hipError_t launch_elem_t(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                                const double* u, double* uout, const double* alpha, double* ut, double* k,
                                int stage, double dt, double A, double B, int variant, int flags, hipStream_t s) {
  if (variant == 1 && elem_variants(kN) > 1)
    return launch_elem_v<NV, FLUX, 1>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, flags, s);
  return launch_elem_v<NV, FLUX, 0>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, flags, s);
}

namespace per_degree {
hipError_t element(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                   const double* u, double* uout, const double* alpha, double* ut, double* k, int stage,
                   double dt, double A, double B, int variant, int flags, hipStream_t s) {
  if (count == 0) return hipSuccess;
  // fused faces read the neighbours' state from u: nothing of this launch may write it
  if ((flags & ELEM_FUSE_FACES) && (kN < FUSE_MIN_N || (stage > 0 && uout == u) || !m.side_rec))
    return hipErrorInvalidValue;
  const int v = variant;
  if (m.nvar == 5) {
    if (p.volume_flux == 0) return launch_elem_t<5, FluxRanocha>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, v, flags, s);
    if (p.volume_flux == 1) return launch_elem_t<5, FluxPirozzoli>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, v, flags, s);
    return launch_elem_t<5, FluxCentral>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, v, flags, s);
  }
  if (p.volume_flux == 1) return launch_elem_t<6, FluxPirozzoli>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, v, flags, s);
  return launch_elem_t<6, FluxCentral>(m, p, elist, count, u, uout, alpha, ut, k, stage, dt, A, B, v, flags, s);
}

// fv_means is persistent: as many workgroups as fit on the device at once (at
// most `count`, the bucket size) walk this degree's range of the blended-element
// list built for the call.  fv_residual runs one workgroup per list entry over
// a grid of the bucket size, the workgroups past the range leaving at once:
// its register footprint grows by half in the persistent loop form.
template <auto KERNEL>
int persistent_grid(int block, const MeshView& m, int count, int share) {
  static const int per_cu = resident_per_cu(reinterpret_cast<const void*>(KERNEL), block);
  const int g = (per_cu * m.n_cu + share - 1) / share;   // the device is shared by `share` branches
  return count < g ? count : g;
}

template <int NFV>
hipError_t fv_means_t(const MeshView& m, int count, int share, const double* u, hipStream_t s) {
  if constexpr (NFV >= kN + 1) {
    if (m.nvar == 5)
      hipLaunchKernelGGL((fv_means_kernel<kN, NFV, 5>),
                         dim3(persistent_grid<fv_means_kernel<kN, NFV, 5>>(FV2_THREADS, m, count, share)),
                         dim3(FV2_THREADS), 0, s, m, u);
    else
      hipLaunchKernelGGL((fv_means_kernel<kN, NFV, 6>),
                         dim3(persistent_grid<fv_means_kernel<kN, NFV, 6>>(FV2_THREADS, m, count, share)),
                         dim3(FV2_THREADS), 0, s, m, u);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t fv_means(const MeshView& m, int count, int share, const double* u, hipStream_t s) {
  if (count == 0) return hipSuccess;
  switch (m.n_fv) {
    case 2: return fv_means_t<2>(m, count, share, u, s);
    case 3: return fv_means_t<3>(m, count, share, u, s);
    case 4: return fv_means_t<4>(m, count, share, u, s);
    case 5: return fv_means_t<5>(m, count, share, u, s);
    case 6: return fv_means_t<6>(m, count, share, u, s);
    case 7: return fv_means_t<7>(m, count, share, u, s);
    case 8: return fv_means_t<8>(m, count, share, u, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NFV>
hipError_t fv_residual_t(const MeshView& m, const ParamsDev& p, int count, hipStream_t s) {
  if constexpr (NFV >= kN + 1) {
    if (m.nvar == 5)
      hipLaunchKernelGGL((fv_residual_kernel<kN, NFV, 5>),
                         dim3(count),
                         dim3(FV2_THREADS), 0, s, m, p);
    else
      hipLaunchKernelGGL((fv_residual_kernel<kN, NFV, 6>),
                         dim3(count),
                         dim3(FV2_THREADS), 0, s, m, p);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t fv_residual(const MeshView& m, const ParamsDev& p, int count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  switch (m.n_fv) {
    case 2: return fv_residual_t<2>(m, p, count, s);
    case 3: return fv_residual_t<3>(m, p, count, s);
    case 4: return fv_residual_t<4>(m, p, count, s);
    case 5: return fv_residual_t<5>(m, p, count, s);
    case 6: return fv_residual_t<6>(m, p, count, s);
    case 7: return fv_residual_t<7>(m, p, count, s);
    case 8: return fv_residual_t<8>(m, p, count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t fv_normals(const MeshView& m, const int32_t* elist, int count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL((fv_normals_kernel<kN>), dim3(count), dim3(FV_THREADS), 0, s, m, elist, count);
  return hipGetLastError();
}

hipError_t indicator(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                     const double* u, double* alpha, double* ind, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((indicator_kernel<kN, 5>), dim3(count), dim3(ind_threads<kN>()), 0, s, m, p, elist, count,
                       u, alpha, ind);
  else
    hipLaunchKernelGGL((indicator_kernel<kN, 6>), dim3(count), dim3(ind_threads<kN>()), 0, s, m, p, elist, count,
                       u, alpha, ind);
  return hipGetLastError();
}

template <int NFV>
hipError_t fv_jbar_t(const MeshView& m, const int32_t* elist, int count, hipStream_t s) {
  if constexpr (NFV >= kN + 1) {
    hipLaunchKernelGGL((fv_jbar_kernel<kN, NFV>), dim3(count), dim3(FVS_THREADS), 0, s, m, elist, count);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t fv_jbar(const MeshView& m, const int32_t* elist, int count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  switch (m.n_fv) {
    case 2: return fv_jbar_t<2>(m, elist, count, s);
    case 3: return fv_jbar_t<3>(m, elist, count, s);
    case 4: return fv_jbar_t<4>(m, elist, count, s);
    case 5: return fv_jbar_t<5>(m, elist, count, s);
    case 6: return fv_jbar_t<6>(m, elist, count, s);
    case 7: return fv_jbar_t<7>(m, elist, count, s);
    case 8: return fv_jbar_t<8>(m, elist, count, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NFV>
hipError_t fv_switch_t(const MeshView& m, const int32_t* elist, int count, double* u, double* ufv,
                       const double* fv_old, const double* fv_new, hipStream_t s) {
  if constexpr (NFV >= kN + 1) {
    if (m.nvar == 5)
      hipLaunchKernelGGL((fv_switch_kernel<kN, NFV, 5>), dim3(count), dim3(FVS_THREADS), 0, s, m, elist, count, u,
                         ufv, fv_old, fv_new);
    else
      hipLaunchKernelGGL((fv_switch_kernel<kN, NFV, 6>), dim3(count), dim3(FVS_THREADS), 0, s, m, elist, count, u,
                         ufv, fv_old, fv_new);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t fv_switch(const MeshView& m, const int32_t* elist, int count, double* u, double* ufv,
                     const double* fv_old, const double* fv_new, hipStream_t s) {
  if (count == 0) return hipSuccess;
  switch (m.n_fv) {
    case 2: return fv_switch_t<2>(m, elist, count, u, ufv, fv_old, fv_new, s);
    case 3: return fv_switch_t<3>(m, elist, count, u, ufv, fv_old, fv_new, s);
    case 4: return fv_switch_t<4>(m, elist, count, u, ufv, fv_old, fv_new, s);
    case 5: return fv_switch_t<5>(m, elist, count, u, ufv, fv_old, fv_new, s);
    case 6: return fv_switch_t<6>(m, elist, count, u, ufv, fv_old, fv_new, s);
    case 7: return fv_switch_t<7>(m, elist, count, u, ufv, fv_old, fv_new, s);
    case 8: return fv_switch_t<8>(m, elist, count, u, ufv, fv_old, fv_new, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t limiter(const MeshView& m, const int32_t* elist, int count, double* u, const double* alpha,
                   double* theta, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (m.nvar != 5) return hipErrorInvalidValue;
  hipLaunchKernelGGL((limiter_kernel<kN>), dim3(count), dim3(lim_threads<kN>()), 0, s, m, elist, count, u, alpha,
                     theta);
  return hipGetLastError();
}

template <int NV, class FLUX>
hipError_t launch_vjp_volume_t(const MeshView& m, const int32_t* elist, int count, const double* u,
                               const double* alpha, const double* w, double* g, hipStream_t s) {
  using G = Geo<kN>;
  const int blocks = (count + G::EPB - 1) / G::EPB;
  hipLaunchKernelGGL((vjp_volume_kernel<kN, NV, FLUX>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m,
                     elist, count, u, alpha, w, g);
  return hipGetLastError();
}

hipError_t vjp_volume(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                      const double* u, const double* alpha, const double* w, double* g, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (m.nvar == 5) {
    if (p.volume_flux == 0) return launch_vjp_volume_t<5, FluxRanocha>(m, elist, count, u, alpha, w, g, s);
    if (p.volume_flux == 1) return launch_vjp_volume_t<5, FluxPirozzoli>(m, elist, count, u, alpha, w, g, s);
    return launch_vjp_volume_t<5, FluxCentral>(m, elist, count, u, alpha, w, g, s);
  }
  if (p.volume_flux == 1) return launch_vjp_volume_t<6, FluxPirozzoli>(m, elist, count, u, alpha, w, g, s);
  return launch_vjp_volume_t<6, FluxCentral>(m, elist, count, u, alpha, w, g, s);
}

hipError_t vjp_fv(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                  const double* alpha, const double* w, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((vjp_fv_kernel<kN, 5>), dim3(count), dim3(FV_THREADS), 0, s, m, p, elist, count, alpha, w);
  else
    hipLaunchKernelGGL((vjp_fv_kernel<kN, 6>), dim3(count), dim3(FV_THREADS), 0, s, m, p, elist, count, alpha, w);
  return hipGetLastError();
}

hipError_t vjp_gather(const MeshView& m, const int32_t* elist, int count, const double* alpha,
                      double* g, hipStream_t s) {
  if (count == 0) return hipSuccess;
  using G = Geo<kN>;
  const int blocks = (count + G::EPB - 1) / G::EPB;
  if (m.nvar == 5)
    hipLaunchKernelGGL((vjp_trace_kernel<kN, 5>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, g);
  else
    hipLaunchKernelGGL((vjp_trace_kernel<kN, 6>), dim3(blocks), dim3(G::EPB * G::NP3), 0, s, m, elist, count, g);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !alpha) return err;
  if (m.nvar == 5)
    hipLaunchKernelGGL((vjp_fv_gather_kernel<kN, 5>), dim3(count), dim3(FV_THREADS), 0, s, m, elist, count, alpha, g);
  else
    hipLaunchKernelGGL((vjp_fv_gather_kernel<kN, 6>), dim3(count), dim3(FV_THREADS), 0, s, m, elist, count, alpha, g);
  return hipGetLastError();
}
}  // namespace per_degree
}  // namespace

// The dispatcher's handle on this degree's launchers.
#define DGFV_CAT2(a, b) a##b
#define DGFV_CAT(a, b) DGFV_CAT2(a, b)
DegreeOps DGFV_CAT(degree_ops_, DGFV_N)() {
  return DegreeOps{&per_degree::element,    &per_degree::fv_means, &per_degree::fv_residual,
                   &per_degree::indicator,  &per_degree::vjp_volume, &per_degree::vjp_fv,
                   &per_degree::vjp_gather, &per_degree::fv_normals, &per_degree::limiter,
                   &per_degree::fv_jbar,    &per_degree::fv_switch,  elem_variants(kN)};
}

}  // namespace dgfv
