// Rates of FV-stored elements (Section 3.1.2, eq. semidiscrete_fv).
//
// An FV-stored element carries the means of N_FV^3 equidistant reference
// sub-cells.  Every sub-cell face sees a second-order reconstruction: per
// reference direction, the slope of a sub-cell is the minmod of its backward
// and forward differences of the primitive variables (rho, v, p[, Y1]), the
// state across an element side taken from m.fvghost; each internal sub-cell
// face gets one Riemann flux with the sub-face normal of m.fvnorm, the
// element's sides the fluxes the FV face kernel wrote to m.fvside.  The rate
// of a mean is minus the sum of its outward fluxes over h^3 Jbar (Jbar = V3(J),
// m.fvjbar), and the 2N Runge-Kutta update of (ufv, kfv) is fused in.
#include "dgfv_internal.h"
#include "dgfv_physics.h"

namespace dgfv {
namespace {

constexpr int FVS_THREADS = 512;

// One workgroup per entry of the call's FV-element list (a grid of K, the
// workgroups past the list leaving at once), one thread per sub-cell.  The
// thread of sub-cell c evaluates the internal face c + 1/2 along each
// direction: its left state from c's slope, its right state from the slope of
// c + 1, which the thread forms itself from the primitives in LDS (the same
// arithmetic as c + 1's own), so that the states need no LDS round trip.
// 4 waves per SIMD: two workgroups per CU at N_FV = 8.
template <int NFV, int NV>
__global__ void __launch_bounds__(FVS_THREADS, 4)
fv_stored_kernel(MeshView m, ParamsDev prm, double* __restrict__ ufv, double* __restrict__ kfv,
                 double* __restrict__ utfv, int stage, double dt, double A, double B) {
  constexpr int S2 = NFV * NFV, S3 = S2 * NFV, NIF = (NFV - 1) * S2, NSD = 6 * NV * S2;
  static_assert(S3 <= FVS_THREADS, "one thread per sub-cell");
  __shared__ double sW[NV * S3];      // primitives of the means
  __shared__ double sL[NV * S3];      // flux through each sub-cell's + face
  __shared__ double sG[NSD];          // primitives across the six sides
  __shared__ double sF[NSD];          // the six sides' outward fluxes
  if ((int)blockIdx.x >= m.blend_start[MAXN + 1]) return;
  const int e = m.blend_list[blockIdx.x];
  const int t = threadIdx.x;
  const bool active = t < S3;
  const int c = active ? t : 0;
  const int s0 = c % NFV, s1 = (c / NFV) % NFV, s2 = c / S2;
  const double h = 2.0 / NFV;
  double* ue = ufv + (size_t)e * NV * S3;
  const double* gh = m.fvghost + (size_t)e * NSD;
  const double* fs = m.fvside + (size_t)e * NSD;
  const double* nrm = m.fvnorm + (size_t)e * 9 * NIF;
  // loads: this thread's mean, J mean and sub-face normals; the sides' data
  double um[NV], nd[3][3];
#pragma unroll
  for (int v = 0; v < NV; ++v) um[v] = ue[v * S3 + c];
  const double jb = m.fvjbar[(size_t)e * S3 + c];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int sd = d == 0 ? s0 : (d == 1 ? s1 : s2);
    const int ta = d == 2 ? s1 : s2, tb = d == 0 ? s1 : s0;
    const bool has = active && sd < NFV - 1;
    const int k = has ? (sd * NFV + ta) * NFV + tb : 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double x = nrm[(d * 3 + q) * NIF + k];
      nd[d][q] = has ? x : 0.0;
    }
  }
  for (int r = t; r < NSD; r += FVS_THREADS) sF[r] = fs[r];
  for (int r = t; r < 6 * S2; r += FVS_THREADS) {       // ghost points: conservative -> primitive
    const int side = r / S2, i = r % S2;
    double g[NV], w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = gh[(side * NV + v) * S2 + i];
    cons_to_w<NV>(g, m.gas, w);
#pragma unroll
    for (int v = 0; v < NV; ++v) sG[(side * NV + v) * S2 + i] = w[v];
  }
  {
    double wc[NV];
    cons_to_w<NV>(um, m.gas, wc);
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sW[v * S3 + c] = wc[v];
    }
  }
  __syncthreads();
  double dC[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) dC[v] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int sd = d == 0 ? s0 : (d == 1 ? s1 : s2);
    const int stride = d == 0 ? 1 : (d == 1 ? NFV : S2);
    const int ta = d == 2 ? s1 : s2, tb = d == 0 ? s1 : s0;
    const int fidx = ta * NFV + tb;                       // face-grid index on the two sides
    const int glo = ((2 * d) * NV) * S2 + fidx, ghi = ((2 * d + 1) * NV) * S2 + fidx;
    if (active && sd < NFV - 1) {                         // the internal face at this sub-cell's + side
      double ul[NV], ur[NV];
      {
        double wl[NV], wr[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double w0 = sW[v * S3 + c];
          const double wm = sd > 0 ? sW[v * S3 + c - stride] : sG[glo + v * S2];
          const double w1 = sW[v * S3 + c + stride];
          const double w2 = sd + 2 < NFV ? sW[v * S3 + c + 2 * stride] : sG[ghi + v * S2];
          wl[v] = w0 + 0.5 * minmod(w0 - wm, w1 - w0);
          wr[v] = w1 - 0.5 * minmod(w1 - w0, w2 - w1);
        }
        w_to_cons<NV>(wl, m.gas, ul);
        w_to_cons<NV>(wr, m.gas, ur);
      }
      double Fl[NV];
      riemann<NV>(prm.face_flux_fv, prm.volume_flux, ul, ur, nd[d][0], nd[d][1], nd[d][2], m.gas, Fl);
#pragma unroll
      for (int v = 0; v < NV; ++v) sL[v * S3 + c] = Fl[v];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double hi = sd < NFV - 1 ? sL[v * S3 + c] : sF[((2 * d + 1) * NV + v) * S2 + fidx];
        const double lo = sd > 0 ? sL[v * S3 + c - stride] : -sF[((2 * d) * NV + v) * S2 + fidx];
        dC[v] -= hi - lo;
      }
    }
    __syncthreads();                                      // sL is rewritten by the next direction
  }
  if (!active) return;
  const double scale = 1.0 / (h * h * h * jb);
  if (stage == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) utfv[(size_t)e * NV * S3 + v * S3 + c] = dC[v] * scale;
    return;
  }
  double* ke = kfv + (size_t)e * NV * S3;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double R = dC[v] * scale;
    const double kv = stage == 1 ? dt * R : A * ke[v * S3 + c] + dt * R;
    ke[v * S3 + c] = kv;
    ue[v * S3 + c] = um[v] + B * kv;
  }
}

template <int NFV>
hipError_t launch_t(const MeshView& m, const ParamsDev& p, double* ufv, double* kfv, double* utfv, int stage,
                    double dt, double A, double B, hipStream_t s) {
  if (m.nvar == 5)
    hipLaunchKernelGGL((fv_stored_kernel<NFV, 5>), dim3(m.K), dim3(FVS_THREADS), 0, s, m, p, ufv, kfv, utfv, stage,
                       dt, A, B);
  else
    hipLaunchKernelGGL((fv_stored_kernel<NFV, 6>), dim3(m.K), dim3(FVS_THREADS), 0, s, m, p, ufv, kfv, utfv, stage,
                       dt, A, B);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fv_stored(const MeshView& m, const ParamsDev& p, double* ufv, double* kfv, double* utfv,
                            int stage, double dt, double A, double B, hipStream_t s) {
  switch (m.n_fv) {
    case 2: return launch_t<2>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    case 3: return launch_t<3>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    case 4: return launch_t<4>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    case 5: return launch_t<5>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    case 6: return launch_t<6>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    case 7: return launch_t<7>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    case 8: return launch_t<8>(m, p, ufv, kfv, utfv, stage, dt, A, B, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgfv
