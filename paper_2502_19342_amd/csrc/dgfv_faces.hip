// Interface fluxes of the hybrid DG/FV operator (Section 3.2.1).
//
// Three kernels per call, by face class (the class is fixed by the degrees and
// blending factors of the two elements):
//  * DG / DG, same degree: the Riemann flux at each face node with the left
//    side's outward normal n*s = +-Ja^d (eq. conv_flux);
//  * DG / DG, degrees NL != NR: both traces at M = max(NL, NR) through
//    V^{N->M}, flux at the M nodes, and the lower side receives the modal L2
//    projection V^{M->N} of it;
//  * FV face (either alpha > 0): sub-face traces on the N_FV^2 grid (sub-cell
//    means of a blended side, V^{DG->FV} of a DG side's nodal trace), one
//    Riemann flux per sub-face with n*s = h^2 V^{DG->FV}(Ja); the FV part of
//    a blended side receives it directly and every DG part V^{FV->DG} of it / h^2.
// The first class runs one lane per face node over static per-degree face
// lists; the second runs one face per 64-lane workgroup over a static list;
// FV faces come from the blended-element list of the call.
// Results go to per-element side buffers: the right side gets the negated flux
// re-indexed through the face orientation.
#include "dgfv_internal.h"
#include "dgfv_lds.h"
#include "dgfv_physics.h"

namespace dgfv {
namespace {

constexpr int FACE_THREADS = 64;
constexpr int GRID = 64;  // max points of a face grid: (MAXN+1)^2 = MAXFV^2 = 64
static_assert(FACE_THREADS == 64, "the face workgroups are one wavefront");

// Synchronisation of the one-wavefront face workgroups through LDS.  The LDS
// operations of a wavefront are performed in program order, so a fence at
// wavefront scope (no wait instruction; it only keeps the compiler from
// moving memory accesses across it) is enough.  A workgroup barrier would in
// addition wait for every global store still in flight.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Gather a side's nodal trace into `dst[NV][n*n]` on the left side's face grid.
template <int NV>
__device__ void gather_trace(const MeshView& m, const double* u, int e, int side, int o, bool right,
                             int n, double* dst) {
  const int64_t base = m.elem_offset[e];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int p = t % n, q = t / n;
    if (right) orient_map(o, p, q, n, p, q);
    const int64_t g = base + side_node(side, p, q, n);
    for (int v = 0; v < NV; ++v) dst[v * GRID + t] = u[v * m.n_node + g];
  }
}

// Boundary-layer sub-cell means of side `side` on the left side's sub-face grid.
template <int NV>
__device__ void gather_subcells(const MeshView& m, int e, int side, int o, bool right, double* dst) {
  const int n = m.n_fv;
  const int S3 = n * n * n;
  const double* ub = m.ubar + (size_t)e * NV * S3;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int p = t % n, q = t / n;
    if (right) orient_map(o, p, q, n, p, q);
    const int s = side_node(side, p, q, n);
    for (int v = 0; v < NV; ++v) dst[v * GRID + t] = ub[v * S3 + s];
  }
}

// 2D tensor map A (x) A on face data [nf][GRID] with grids nin x nin -> nout x nout.
__device__ void map2d(const double* src, double* tmp, double* dst, const double* A, int nout,
                      int nin, int nf) {
  // compact src into tmp as [nf][nin][nin] for the generic contraction
  for (int t = threadIdx.x; t < nf * nin * nin; t += blockDim.x) {
    const int f = t / (nin * nin), r = t % (nin * nin);
    tmp[t] = src[f * GRID + r];
  }
  __syncthreads();
  double* mid = tmp + nf * GRID;     // disjoint from both the compacted input and the output
  contract_axis(tmp, mid, A, nout, nin, nf, 1, nin, nin, 0);   // [nf][nin][nout]
  __syncthreads();
  double* out = tmp;                 // the compacted input is dead now
  contract_axis(mid, out, A, nout, nin, nf, 1, nin, nout, 1);  // [nf][nout][nout]
  __syncthreads();
  for (int t = threadIdx.x; t < nf * nout * nout; t += blockDim.x) {
    const int f = t / (nout * nout), r = t % (nout * nout);
    dst[f * GRID + r] = out[t];
  }
  __syncthreads();
}

// Write face data [NV][n*n] (left grid) into a side buffer, with sign and orientation.
template <int NV>
__device__ void write_side(double* dst_block, const double* src, int side, int o, bool right, int n,
                           double scale) {
  const int n2 = n * n;
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    int p = t % n, q = t / n;
    if (right) orient_map(o, p, q, n, p, q);
    for (int v = 0; v < NV; ++v) dst_block[(side * NV + v) * n2 + q * n + p] = scale * src[v * GRID + t];
  }
}

// The maps below take their sizes at run time but unroll over MAXN + 1 terms
// without a branch per term: a coefficient past nin is zero, and the operand
// index is clamped to nin - 1, so the extra terms add exact zeros to the sums
// (a branch per term would make each one wait for its own LDS read).
__device__ __forceinline__ int clamp_last(int k, int n) { return k < n ? k : n - 1; }

// Row r of A ([nout][nin] row-major, nin <= MAXN + 1) in registers, zero-padded.
__device__ __forceinline__ void load_row(const double* A, int nin, int r, double (&a)[MAXN + 1]) {
#pragma unroll
  for (int k = 0; k <= MAXN; ++k) {
    const double x = A[r * nin + clamp_last(k, nin)];
    a[k] = k < nin ? x : 0.0;
  }
}

// sum_k a[k] src[k * stride] over k < nin, in order of k
__device__ __forceinline__ double dot_row(const double (&a)[MAXN + 1], const double* src, int stride, int nin) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k <= MAXN; ++k) acc += a[k] * src[clamp_last(k, nin) * stride];
  return acc;
}

// 2D tensor maps A (x) A of face data [NF][GRID] on [nin][nin] grids (p
// fastest) to [nout][nout] grids, in two passes, for the one-wavefront face
// workgroups: pass 1 contracts p into T[f][q][pp] (nin rows of nout), pass 2
// contracts q, so each output is the sum over q of A[qq][q] times the sum over
// p of A[pp][p] src[q][p], at nin + nout products per output point and field.  T must alias neither src nor dst; one wave_sync
// inside, the caller synchronises around the call.
template <int NF>
__device__ void map2d_pass1(const double* src, double* T, const double* A, int nout, int nin) {
  for (int t = threadIdx.x; t < nin * nout; t += blockDim.x) {
    const int pp = t % nout, q = t / nout;
    double a[MAXN + 1];
    load_row(A, nin, pp, a);
#pragma unroll
    for (int f = 0; f < NF; ++f) T[f * GRID + t] = dot_row(a, src + f * GRID + q * nin, 1, nin);
  }
}

template <int NF>
__device__ void map2d_sep_to(const double* src, double* T, double* dst, const double* A, int nout, int nin) {
  map2d_pass1<NF>(src, T, A, nout, nin);
  wave_sync();
  for (int t = threadIdx.x; t < nout * nout; t += blockDim.x) {
    const int pp = t % nout, qq = t / nout;
    double a[MAXN + 1];
    load_row(A, nin, qq, a);
#pragma unroll
    for (int f = 0; f < NF; ++f) dst[f * GRID + t] = dot_row(a, T + f * GRID + pp, nout, nin);
  }
}

// pass 2 of the map from T written straight into a side buffer (orientation
// and scale as in write_side)
template <int NV>
__device__ void map2d_pass2_side(double* dst_block, const double* T, const double* A, int nout, int nin,
                                 int side, int o, bool right, double scale) {
  const int n2 = nout * nout;
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    const int pp = t % nout, qq = t / nout;
    int p = pp, q = qq;
    if (right) orient_map(o, pp, qq, nout, p, q);
    double a[MAXN + 1];
    load_row(A, nin, qq, a);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      dst_block[(side * NV + v) * n2 + q * nout + p] = scale * dot_row(a, T + v * GRID + pp, nout, nin);
  }
}

template <int NV>
__device__ void map2d_sep_side(double* dst_block, const double* src, double* T, const double* A, int nout,
                               int nin, int side, int o, bool right, double scale) {
  map2d_pass1<NV>(src, T, A, nout, nin);
  wave_sync();
  map2d_pass2_side<NV>(dst_block, T, A, nout, nin, side, o, right, scale);
}

// One face, any class, by the whole (64-lane) workgroup, with a few
// wave_syncs; B0..B3 are [NV][GRID] and sN, sNF [3][GRID] LDS arrays
// of the caller.  Degree-jump and FV faces need them; conforming DG faces
// take the pointwise branch.  The caller synchronises before reusing them.
template <int NV>
__device__ void face_body(const MeshView& m, const ParamsDev& prm, const double* __restrict__ u,
                          const double* __restrict__ alpha, int f, double* B0, double* B1, double* B2,
                          double* B3, double* sN, double* sNF) {
  const int32_t* fc = m.faces + 5 * f;
  const int eL = fc[0], sideL = fc[1], eR = fc[2], sideR = fc[3], o = fc[4];
  const int NL = m.degree[eL], NR = m.degree[eR];
  const int M = NL > NR ? NL : NR;
  const int nL = NL + 1, nR = NR + 1, nM = M + 1;
  const double aL = alpha ? alpha[eL] : 0.0;
  const double aR = alpha ? alpha[eR] : 0.0;
  const double* nrm = m.face_norm + m.face_norm_off[f];   // [3][nM*nM]
  double* bL = m.fside + m.side_off[eL];
  double* bR = m.fside + m.side_off[eR];

  if (!(aL > 0.0) && !(aR > 0.0)) {
    if (NL == NR) {
      // conforming DG face: pointwise
      const int n = nL, n2 = n * n;
      const int64_t baseL = m.elem_offset[eL], baseR = m.elem_offset[eR];
      for (int t = threadIdx.x; t < n2; t += blockDim.x) {
        const int p = t % n, q = t / n;
        int pp, qq;
        orient_map(o, p, q, n, pp, qq);
        const int64_t gL = baseL + side_node(sideL, p, q, n);
        const int64_t gR = baseR + side_node(sideR, pp, qq, n);
        double uL[NV], uR[NV], F[NV];
        for (int v = 0; v < NV; ++v) {
          uL[v] = u[v * m.n_node + gL];
          uR[v] = u[v * m.n_node + gR];
        }
        riemann<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, nrm[t], nrm[n2 + t], nrm[2 * n2 + t],
                    m.gas, F);
        for (int v = 0; v < NV; ++v) {
          bL[(sideL * NV + v) * n2 + q * n + p] = F[v];
          bR[(sideR * NV + v) * n2 + qq * n + pp] = -F[v];
        }
      }
      return;
    }
    // degree jump: both traces at the common degree M, flux there, the lower
    // side receives the L2 projection (two-pass maps; exactly one side is lower,
    // and the buffers the other side leaves free serve as their scratch)
    // both traces and this lane's normal at the common degree are loaded
    // before the first store (separate copy loops would wait for each other's
    // loads); the flux loop below visits at most one point per lane, that of
    // threadIdx.x, as a face grid has at most GRID = FACE_THREADS points
    static_assert(GRID == FACE_THREADS, "one point per lane");
    const int n2 = nM * nM;
    {
      const int t = threadIdx.x;
      const int tl = t < nL * nL ? t : 0, tr = t < nR * nR ? t : 0;
      int pr = tr % nR, qr = tr / nR;
      orient_map(o, pr, qr, nR, pr, qr);
      const double* srcL = u + m.elem_offset[eL] + side_node(sideL, tl % nL, tl / nL, nL);
      const double* srcR = u + m.elem_offset[eR] + side_node(sideR, pr, qr, nR);
      double xl[NV], xr[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        xl[v] = srcL[v * m.n_node];
        xr[v] = srcR[v * m.n_node];
      }
      if (t < nL * nL)
        for (int v = 0; v < NV; ++v) B0[v * GRID + t] = xl[v];
      if (t < nR * nR)
        for (int v = 0; v < NV; ++v) B1[v * GRID + t] = xr[v];
    }
    const int tn = (int)threadIdx.x < n2 ? (int)threadIdx.x : 0;
    const double xn0 = nrm[tn], xn1 = nrm[n2 + tn], xn2 = nrm[2 * n2 + tn];
    wave_sync();
    const double* LM = B0;
    const double* RM = B1;
    if (NL < M) { map2d_sep_to<NV>(B0, B3, B2, m.ops + m.tab.interp[NL][M], nM, nL); LM = B2; }
    if (NR < M) { map2d_sep_to<NV>(B1, B2, B3, m.ops + m.tab.interp[NR][M], nM, nR); RM = B3; }
    wave_sync();
    double* F = NL < M ? B0 : B2;
    for (int t = threadIdx.x; t < n2; t += blockDim.x) {
      double uL[NV], uR[NV], Fl[NV];
      for (int v = 0; v < NV; ++v) {
        uL[v] = LM[v * GRID + t];
        uR[v] = RM[v * GRID + t];
      }
      riemann<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, xn0, xn1, xn2, m.gas, Fl);
      for (int v = 0; v < NV; ++v) F[v * GRID + t] = Fl[v];
      const int p = t % nM, q = t / nM;
      if (NL == M)
        for (int v = 0; v < NV; ++v) bL[(sideL * NV + v) * n2 + q * nM + p] = Fl[v];
      if (NR == M) {
        int pp, qq;
        orient_map(o, p, q, nM, pp, qq);
        for (int v = 0; v < NV; ++v) bR[(sideR * NV + v) * n2 + qq * nM + pp] = -Fl[v];
      }
    }
    wave_sync();
    if (NL < M) map2d_sep_side<NV>(bL, F, B3, m.ops + m.tab.project[M][NL], nL, nM, sideL, o, false, 1.0);
    if (NR < M) map2d_sep_side<NV>(bR, F, B1, m.ops + m.tab.project[M][NR], nR, nM, sideR, o, true, -1.0);
    return;
  }

  // FV face: sub-face traces, one flux per sub-face
  const int nF = m.n_fv, n2F = nF * nF;
  const double h = 2.0 / nF;
  {
    // both sides' data (sub-cell means of a blended side, the nodal trace of a
    // DG side, the right side re-indexed onto the left grid) and the normals:
    // one point of each grid per lane, every load issued before the first store
    // (separate copy loops would wait for each other's loads)
    static_assert(GRID == FACE_THREADS, "one point per lane");
    const int t = threadIdx.x;
    const int nl = aL > 0.0 ? nF : nL, nr = aR > 0.0 ? nF : nR, nn = nM * nM;
    const int S3 = nF * nF * nF;
    auto source = [&](int e, int side, double a, int n, bool right, const double*& src, int64_t& vs) {
      const int tc = t < n * n ? t : 0;          // in-range index for idle lanes
      int p = tc % n, q = tc / n;
      if (right) orient_map(o, p, q, n, p, q);
      if (a > 0.0) {
        src = m.ubar + (size_t)e * NV * S3 + side_node(side, p, q, n);
        vs = S3;
      } else {
        src = u + m.elem_offset[e] + side_node(side, p, q, n);
        vs = m.n_node;
      }
    };
    const double *srcL, *srcR;
    int64_t vL, vR;
    source(eL, sideL, aL, nl, false, srcL, vL);
    source(eR, sideR, aR, nr, true, srcR, vR);
    const int tn = t < nn ? t : 0;
    double xl[NV], xr[NV], xn[3];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xl[v] = srcL[v * vL];
      xr[v] = srcR[v * vR];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) xn[c] = nrm[c * nn + tn];
    if (t < nl * nl)
      for (int v = 0; v < NV; ++v) B0[v * GRID + t] = xl[v];
    if (t < nr * nr)
      for (int v = 0; v < NV; ++v) B1[v * GRID + t] = xr[v];
    if (t < nn)
      for (int c = 0; c < 3; ++c) sN[c * GRID + t] = xn[c];
  }
  wave_sync();
  // the normals go to the sub-face grid first (B2 as scratch); at most one
  // side is pure DG, and its trace follows by the two-pass map, with the
  // buffer the blended side leaves free as scratch
  const double* LF = B0;
  const double* RF = B1;
  map2d_sep_to<3>(sN, B2, sNF, m.ops + m.tab.dg2fv[M], nF, nM);
  wave_sync();
  if (!(aL > 0.0)) { map2d_sep_to<NV>(B0, B3, B2, m.ops + m.tab.dg2fv[NL], nF, nL); LF = B2; }
  if (!(aR > 0.0)) { map2d_sep_to<NV>(B1, B2, B3, m.ops + m.tab.dg2fv[NR], nF, nR); RF = B3; }
  wave_sync();
  double* F = LF == B2 ? B0 : B2;
  double* fvL = m.fvside + (size_t)eL * 6 * NV * n2F;
  double* fvR = m.fvside + (size_t)eR * 6 * NV * n2F;
  const double a = h * h;
  for (int t = threadIdx.x; t < n2F; t += blockDim.x) {
    double uL[NV], uR[NV], Fl[NV];
    for (int v = 0; v < NV; ++v) {
      uL[v] = LF[v * GRID + t];
      uR[v] = RF[v * GRID + t];
    }
    riemann<NV>(prm.face_flux_fv, prm.volume_flux, uL, uR, a * sNF[t], a * sNF[GRID + t],
                a * sNF[2 * GRID + t], m.gas, Fl);
    for (int v = 0; v < NV; ++v) F[v * GRID + t] = Fl[v];
    const int p = t % nF, q = t / nF;
    if (aL > 0.0)
      for (int v = 0; v < NV; ++v) fvL[(sideL * NV + v) * n2F + q * nF + p] = Fl[v];
    if (aR > 0.0) {
      int pp, qq;
      orient_map(o, p, q, nF, pp, qq);
      for (int v = 0; v < NV; ++v) fvR[(sideR * NV + v) * n2F + qq * nF + pp] = -Fl[v];
    }
  }
  wave_sync();
  // both DG parts receive V^{FV->DG} F: first passes into two of the buffers
  // other than F (all dead now), one wave_sync, second passes into the sides
  const double ih2 = 1.0 / (h * h);
  double* TL = F == B0 ? B1 : B0;
  double* TR = F == B2 ? B3 : B2;
  map2d_pass1<NV>(F, TL, m.ops + m.tab.fv2dg[NL], nL, nF);
  map2d_pass1<NV>(F, TR, m.ops + m.tab.fv2dg[NR], nR, nF);
  wave_sync();
  map2d_pass2_side<NV>(bL, TL, m.ops + m.tab.fv2dg[NL], nL, nF, sideL, o, false, ih2);
  map2d_pass2_side<NV>(bR, TR, m.ops + m.tab.fv2dg[NR], nR, nF, sideR, o, true, -ih2);
}

// Conforming same-degree faces whose two elements are both pure DG: one thread
// per face node, several faces per workgroup, no LDS.  FV faces are skipped
// here (face_fv_kernel handles them).
constexpr int CONF_THREADS = 256;

template <int N, int NV>
__global__ void __launch_bounds__(CONF_THREADS)
face_conforming_kernel(MeshView m, ParamsDev prm, const ConfRec* __restrict__ rec, int fcount,
                       const double* __restrict__ u, const double* __restrict__ alpha,
                       const double* __restrict__ trace) {
  constexpr int NP = N + 1, NP2 = NP * NP, FPB = CONF_THREADS / NP2;
  const int t = threadIdx.x;
  // At N = 7 a face has 64 nodes.  Each wave takes half the nodes of two
  // consecutive faces of the list (lanes 0-31 the even slot, 32-63 the odd
  // one), and the odd slot loads its right side first: on a structured mesh
  // the even face's right element is the odd face's left element, so one load
  // instruction reads both opposite sides of that element, which share their
  // cache lines along xi_1.
  constexpr bool PAIRED = NP2 == 64;
  int slot, r;
  if constexpr (PAIRED) {
    const int w = t >> 6, l = t & 63;
    slot = (w & ~1) + (l >> 5);
    r = (l & 31) + ((w & 1) << 5);
  } else {
    slot = t / NP2;
    r = t - slot * NP2;
  }
  if (slot >= FPB) return;
  const int fi = blockIdx.x * FPB + slot;
  if (fi >= fcount) return;
  const ConfRec rc = rec[fi];
  const int sideL = rc.code & 7, sideR = (rc.code >> 3) & 7, o = rc.code >> 6;
  if (alpha && (alpha[rc.eL] > 0.0 || alpha[rc.eR] > 0.0)) return;
  const int p = r % NP, q = r / NP;
  int pp, qq;
  orient_map(o, p, q, NP, pp, qq);
  // where each side's state comes from: u, or for sides 0 and 1 (strided by
  // N+1 in u) the trace the previous stage wrote, contiguous per side
  auto source = [&](int64_t base, int64_t sblk, int side, int sp, int sq, const double*& src,
                    int64_t& vstride) {
    if (trace && side < 2) {
      src = trace + sblk / 3 + side * NV * NP2 + sq * NP + sp;
      vstride = NP2;
    } else {
      src = u + base + side_node(side, sp, sq, NP);
      vstride = m.n_node;
    }
  };
  const double *sL, *sR;
  int64_t vL, vR;
  source(rc.baseL, rc.sideL, sideL, p, q, sL, vL);
  source(rc.baseR, rc.sideR, sideR, pp, qq, sR, vR);
  const double* nrm = m.face_norm + rc.nrm;
  const bool flip = PAIRED && (slot & 1);
  const double* sA = flip ? sR : sL;
  const double* sB = flip ? sL : sR;
  const int64_t vA = flip ? vR : vL, vB = flip ? vL : vR;
  double a[NV], b[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) a[v] = sA[v * vA];
#pragma unroll
  for (int v = 0; v < NV; ++v) b[v] = sB[v * vB];
  double uL[NV], uR[NV], F[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    uL[v] = flip ? b[v] : a[v];
    uR[v] = flip ? a[v] : b[v];
  }
  riemann<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, nrm[r], nrm[NP2 + r], nrm[2 * NP2 + r], m.gas, F);
  double* bL = m.fside + rc.sideL;
  double* bR = m.fside + rc.sideR;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bL[(sideL * NV + v) * NP2 + q * NP + p] = F[v];
    bR[(sideR * NV + v) * NP2 + qq * NP + pp] = -F[v];
  }
}

// Degree-jump faces between two pure DG elements (static list); FV faces are
// skipped here.  Grid-stride loop, one face per workgroup at a time.
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
face_mixed_kernel(MeshView m, ParamsDev prm, const int32_t* __restrict__ flist, int fcount,
                  const double* __restrict__ u, const double* __restrict__ alpha) {
  __shared__ double B0[NV * GRID], B1[NV * GRID], B2[NV * GRID], B3[NV * GRID], sN[3 * GRID], sNF[3 * GRID];
  for (int fi = blockIdx.x; fi < fcount; fi += gridDim.x) {
    const int f = flist[fi];
    const int32_t* fc = m.faces + 5 * f;
    if (alpha && (alpha[fc[0]] > 0.0 || alpha[fc[2]] > 0.0)) continue;
    face_body<NV>(m, prm, u, alpha, f, B0, B1, B2, B3, sN, sNF);
    wave_sync();
  }
}

// FV faces: one workgroup per entry of the blended-element list of the call
// (a grid of K, the workgroups past the list leaving at once); each blended
// element processes the faces it owns (the left element owns a face when it is
// blended, otherwise the right one), so that the element's sub-cell means are
// read through one L2.  (Persistent workgroups over (element, side) pairs ran
// twice as long.)

template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
face_fv_kernel(MeshView m, ParamsDev prm, const double* __restrict__ u, const double* __restrict__ alpha) {
  __shared__ double B0[NV * GRID], B1[NV * GRID], B2[NV * GRID], B3[NV * GRID], sN[3 * GRID], sNF[3 * GRID];
  if ((int)blockIdx.x >= m.blend_start[MAXN + 1]) return;
  const int e = m.blend_list[blockIdx.x];
  for (int side = 0; side < 6; ++side) {
    const int f = m.elem_face[6 * e + side];
    if (f < 0) continue;                            // a mortar side: the mortar kernel's
    const int32_t* fc = m.faces + 5 * f;
    const bool left = fc[0] == e && fc[1] == side;
    if (!left && alpha[fc[0]] > 0.0) continue;      // the blended left element owns it
    face_body<NV>(m, prm, u, alpha, f, B0, B1, B2, B3, sN, sNF);
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Faces with an FV-stored side (Sections 3.1.2 and 3.2, fig. h_coupling).
// Each side's value on the sub-face grid: an FV side's boundary sub-cell mean
// reconstructed to the face, w_b + minmod(w_b - w_i, w_g - w_b) / 2 on the
// primitives (w_i the next sub-cell inwards, w_g the state across the face);
// a DG side's nodal trace mapped with V^{DG->FV} in both face directions.
// The state across the face (the other side's boundary sub-cell mean, or the
// mapped DG trace) goes to m.fvghost for the FV element's own slopes.  One
// Riemann flux per sub-face goes to m.fvside of FV sides and, through
// V^{FV->DG} / h^2, to m.fside of a DG side.
// ---------------------------------------------------------------------------
template <int NV>
__device__ void face_body_fvs(const MeshView& m, const ParamsDev& prm, const double* __restrict__ u,
                              const double* __restrict__ ufv, const double* __restrict__ fv, int f, double* B0,
                              double* B1, double* B2, double* B3, double* sN, double* sNF) {
  static_assert(GRID == FACE_THREADS, "one point per lane");
  const int32_t* fc = m.faces + 5 * f;
  const int eL = fc[0], sideL = fc[1], eR = fc[2], sideR = fc[3], o = fc[4];
  const int NL = m.degree[eL], NR = m.degree[eR];
  const int M = NL > NR ? NL : NR;
  const int nL = NL + 1, nR = NR + 1, nM = M + 1, nn = nM * nM;
  const bool fL = fv[eL] > 0.0, fR = fv[eR] > 0.0;
  const double* nrm = m.face_norm + m.face_norm_off[f];
  const int nF = m.n_fv, n2F = nF * nF, S3 = n2F * nF;
  const double h = 2.0 / nF;
  const int t = threadIdx.x;
  // the next sub-cell inwards of an FV side stays in this lane's registers: the
  // lane of sub-face t reconstructs sub-face t only
  double yl[NV], yr[NV];
  {
    // one point of each grid per lane, every load issued before the first store
    auto source = [&](int e, int side, bool is_fv, int n, bool right, const double*& s0, const double*& s1,
                      int64_t& vs) {
      const int tc = t < n * n ? t : 0;            // in-range index for idle lanes
      int p = tc % n, q = tc / n;
      if (right) orient_map(o, p, q, n, p, q);
      if (is_fv) {
        const double* ub = ufv + (size_t)e * NV * S3;
        const int b0 = side_node(side, p, q, n);
        const int step = (side >> 1) == 0 ? 1 : ((side >> 1) == 1 ? n : n * n);
        s0 = ub + b0;
        s1 = ub + ((side & 1) ? b0 - step : b0 + step);      // the next sub-cell inwards
        vs = S3;
      } else {
        s0 = u + m.elem_offset[e] + side_node(side, p, q, n);
        s1 = s0;
        vs = m.n_node;
      }
    };
    const int nl = fL ? nF : nL, nr = fR ? nF : nR;
    const double *aL0, *aL1, *aR0, *aR1;
    int64_t vL, vR;
    source(eL, sideL, fL, nl, false, aL0, aL1, vL);
    source(eR, sideR, fR, nr, true, aR0, aR1, vR);
    const int tn = t < nn ? t : 0;
    double xl[NV], xr[NV], xn[3];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xl[v] = aL0[v * vL];
      xr[v] = aR0[v * vR];
      yl[v] = aL1[v * vL];
      yr[v] = aR1[v * vR];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) xn[c] = nrm[c * nn + tn];
    if (t < nl * nl)
      for (int v = 0; v < NV; ++v) B0[v * GRID + t] = xl[v];
    if (t < nr * nr)
      for (int v = 0; v < NV; ++v) B1[v * GRID + t] = xr[v];
    if (t < nn)
      for (int c = 0; c < 3; ++c) sN[c * GRID + t] = xn[c];
  }
  wave_sync();
  // normals to the sub-face grid (B2 as scratch); at most one side is DG, and
  // its trace follows, with the buffers the FV side leaves free as scratch
  const double* LF = B0;
  const double* RF = B1;
  map2d_sep_to<3>(sN, B2, sNF, m.ops + m.tab.dg2fv[M], nF, nM);
  wave_sync();
  if (!fL) { map2d_sep_to<NV>(B0, B3, B2, m.ops + m.tab.dg2fv[NL], nF, nL); LF = B2; }
  if (!fR) { map2d_sep_to<NV>(B1, B2, B3, m.ops + m.tab.dg2fv[NR], nF, nR); RF = B3; }
  wave_sync();
  double* F = LF == B2 ? B0 : B2;
  double* fvL = m.fvside + (size_t)eL * 6 * NV * n2F;
  double* fvR = m.fvside + (size_t)eR * 6 * NV * n2F;
  double* ghL = m.fvghost + (size_t)eL * 6 * NV * n2F;
  double* ghR = m.fvghost + (size_t)eR * 6 * NV * n2F;
  const double a = h * h;
  if (t < n2F) {
    const int tt = t;
    double cL[NV], cR[NV], vL[NV], vR[NV], Fl[NV];
    for (int v = 0; v < NV; ++v) {
      cL[v] = LF[v * GRID + tt];
      cR[v] = RF[v * GRID + tt];
      vL[v] = cL[v];
      vR[v] = cR[v];
    }
    auto reconstruct = [&](const double* cb, const double* ci, const double* cg, double* out) {
      double wb[NV], wi[NV], wg[NV], wf[NV];
      cons_to_w<NV>(cb, m.gas, wb);
      cons_to_w<NV>(ci, m.gas, wi);
      cons_to_w<NV>(cg, m.gas, wg);
      for (int v = 0; v < NV; ++v) wf[v] = wb[v] + 0.5 * minmod(wb[v] - wi[v], wg[v] - wb[v]);
      w_to_cons<NV>(wf, m.gas, out);
    };
    if (fL) reconstruct(cL, yl, cR, vL);
    if (fR) reconstruct(cR, yr, cL, vR);
    riemann<NV>(prm.face_flux_fv, prm.volume_flux, vL, vR, a * sNF[tt], a * sNF[GRID + tt],
                a * sNF[2 * GRID + tt], m.gas, Fl);
    for (int v = 0; v < NV; ++v) F[v * GRID + tt] = Fl[v];
    const int p = tt % nF, q = tt / nF;
    if (fL)
      for (int v = 0; v < NV; ++v) {
        fvL[(sideL * NV + v) * n2F + q * nF + p] = Fl[v];
        ghL[(sideL * NV + v) * n2F + q * nF + p] = cR[v];
      }
    if (fR) {
      int pp, qq;
      orient_map(o, p, q, nF, pp, qq);
      for (int v = 0; v < NV; ++v) {
        fvR[(sideR * NV + v) * n2F + qq * nF + pp] = -Fl[v];
        ghR[(sideR * NV + v) * n2F + qq * nF + pp] = cL[v];
      }
    }
  }
  wave_sync();
  // a DG side receives V^{FV->DG} F / h^2 (two passes through a buffer other than F)
  const double ih2 = 1.0 / (h * h);
  double* Tt = F == B0 ? B1 : B0;
  if (!fL) {
    map2d_pass1<NV>(F, Tt, m.ops + m.tab.fv2dg[NL], nL, nF);
    wave_sync();
    map2d_pass2_side<NV>(m.fside + m.side_off[eL], Tt, m.ops + m.tab.fv2dg[NL], nL, nF, sideL, o, false, ih2);
  }
  if (!fR) {
    map2d_pass1<NV>(F, Tt, m.ops + m.tab.fv2dg[NR], nR, nF);
    wave_sync();
    map2d_pass2_side<NV>(m.fside + m.side_off[eR], Tt, m.ops + m.tab.fv2dg[NR], nR, nF, sideR, o, true, -ih2);
  }
}

// One workgroup per FV-stored element of the call's list (a grid of K, the
// workgroups past the list leaving at once), over the faces it owns (the left
// element owns a face when it is FV-stored, otherwise the right one).
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
face_fvs_kernel(MeshView m, ParamsDev prm, const double* __restrict__ u, const double* __restrict__ ufv,
                const double* __restrict__ fv) {
  __shared__ double B0[NV * GRID], B1[NV * GRID], B2[NV * GRID], B3[NV * GRID], sN[3 * GRID], sNF[3 * GRID];
  if ((int)blockIdx.x >= m.blend_start[MAXN + 1]) return;
  const int e = m.blend_list[blockIdx.x];
  for (int side = 0; side < 6; ++side) {
    const int f = m.elem_face[6 * e + side];
    if (f < 0) continue;                             // no mortars with FV-stored elements
    const int32_t* fc = m.faces + 5 * f;
    const bool left = fc[0] == e && fc[1] == side;
    if (!left && fv[fc[0]] > 0.0) continue;          // the FV-stored left element owns it
    face_body_fvs<NV>(m, prm, u, ufv, fv, f, B0, B1, B2, B3, sN, sNF);
    wave_sync();
  }
}

// Gather side data [NV][n*n] from a side block (`right` re-indexes onto the left grid).
template <int NV>
__device__ void gather_side(const double* blk, int side, int o, bool right, int n, double* dst) {
  const int n2 = n * n;
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    int p = t % n, q = t / n;
    if (right) orient_map(o, p, q, n, p, q);
    for (int v = 0; v < NV; ++v) dst[v * GRID + t] = blk[(side * NV + v) * n2 + q * n + p];
  }
}

// Adjoint of the face fluxes (face_body: degree-jump and FV faces; conforming
// DG faces go to face_vjp_conforming_kernel).  On entry fside holds, per element side, the
// cotangent of the side flux it received; fvside holds the cotangents of the
// FV side fluxes of blended elements.  On exit fside holds the cotangents of
// each side's nodal trace, and fvside (blended sides of FV faces) those of the
// boundary sub-cell means.  Each element side belongs to one face, so the
// in-place update has no cross-workgroup hazard.
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
face_vjp_kernel(MeshView m, ParamsDev prm, const double* __restrict__ u, const double* __restrict__ alpha,
                bool skip_conforming) {
  __shared__ double sL[NV * GRID];
  __shared__ double sR[NV * GRID];
  __shared__ double sF[NV * GRID];
  __shared__ double sN[3 * GRID];
  __shared__ double sTmp[3 * NV * GRID];

  const int f = blockIdx.x;
  if (f >= m.n_face) return;
  const int32_t* fc = m.faces + 5 * f;
  const int eL = fc[0], sideL = fc[1], eR = fc[2], sideR = fc[3], o = fc[4];
  const int NL = m.degree[eL], NR = m.degree[eR];
  const int M = NL > NR ? NL : NR;
  const int nL = NL + 1, nR = NR + 1, nM = M + 1;
  const double aL = alpha ? alpha[eL] : 0.0;
  const double aR = alpha ? alpha[eR] : 0.0;
  const double* nrm = m.face_norm + m.face_norm_off[f];
  double* bL = m.fside + m.side_off[eL];
  double* bR = m.fside + m.side_off[eR];

  if (!(aL > 0.0) && !(aR > 0.0)) {
    if (NL == NR) {
      if (skip_conforming) return;              // done by face_vjp_conforming_kernel
      const int n = nL, n2 = n * n;
      const int64_t baseL = m.elem_offset[eL], baseR = m.elem_offset[eR];
      for (int t = threadIdx.x; t < n2; t += blockDim.x) {
        const int p = t % n, q = t / n;
        int pp, qq;
        orient_map(o, p, q, n, pp, qq);
        const int64_t gL = baseL + side_node(sideL, p, q, n);
        const int64_t gR = baseR + side_node(sideR, pp, qq, n);
        double uL[NV], uR[NV], Fb[NV], uLb[NV], uRb[NV];
        for (int v = 0; v < NV; ++v) {
          uL[v] = u[v * m.n_node + gL];
          uR[v] = u[v * m.n_node + gR];
          Fb[v] = bL[(sideL * NV + v) * n2 + q * n + p] - bR[(sideR * NV + v) * n2 + qq * n + pp];
        }
        riemann_vjp<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, nrm[t], nrm[n2 + t], nrm[2 * n2 + t],
                        m.gas, Fb, uLb, uRb);
        for (int v = 0; v < NV; ++v) {
          bL[(sideL * NV + v) * n2 + q * n + p] = uLb[v];
          bR[(sideR * NV + v) * n2 + qq * n + pp] = uRb[v];
        }
      }
      return;
    }
    // degree jump: Fb at M = P_L^T FbL - P_R^T FbR, then the interpolations' transposes
    gather_side<NV>(bL, sideL, o, false, nL, sL);
    gather_side<NV>(bR, sideR, o, true, nR, sR);
    __syncthreads();
    if (NL < M) map2d(sL, sTmp, sL, m.ops + m.tab.projectT[M][NL], nM, nL, NV);
    if (NR < M) map2d(sR, sTmp, sR, m.ops + m.tab.projectT[M][NR], nM, nR, NV);
    const int n2 = nM * nM;
    for (int t = threadIdx.x; t < n2; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sF[v * GRID + t] = sL[v * GRID + t] - sR[v * GRID + t];
    __syncthreads();
    gather_trace<NV>(m, u, eL, sideL, o, false, nL, sL);
    gather_trace<NV>(m, u, eR, sideR, o, true, nR, sR);
    __syncthreads();
    if (NL < M) map2d(sL, sTmp, sL, m.ops + m.tab.interp[NL][M], nM, nL, NV);
    if (NR < M) map2d(sR, sTmp, sR, m.ops + m.tab.interp[NR][M], nM, nR, NV);
    for (int t = threadIdx.x; t < n2; t += blockDim.x) {
      double uL[NV], uR[NV], Fb[NV], uLb[NV], uRb[NV];
      for (int v = 0; v < NV; ++v) {
        uL[v] = sL[v * GRID + t];
        uR[v] = sR[v * GRID + t];
        Fb[v] = sF[v * GRID + t];
      }
      riemann_vjp<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, nrm[t], nrm[n2 + t], nrm[2 * n2 + t],
                      m.gas, Fb, uLb, uRb);
      for (int v = 0; v < NV; ++v) {
        sL[v * GRID + t] = uLb[v];
        sR[v * GRID + t] = uRb[v];
      }
    }
    __syncthreads();
    if (NL < M) map2d(sL, sTmp, sL, m.ops + m.tab.interpT[NL][M], nL, nM, NV);
    write_side<NV>(bL, sL, sideL, o, false, nL, 1.0);
    if (NR < M) map2d(sR, sTmp, sR, m.ops + m.tab.interpT[NR][M], nR, nM, NV);
    write_side<NV>(bR, sR, sideR, o, true, nR, 1.0);
    return;
  }

  // FV face
  const int nF = m.n_fv, n2F = nF * nF;
  const double h = 2.0 / nF;
  const double ih2 = 1.0 / (h * h);
  double* fvL = m.fvside + (size_t)eL * 6 * NV * n2F;
  double* fvR = m.fvside + (size_t)eR * 6 * NV * n2F;
  gather_side<NV>(bL, sideL, o, false, nL, sL);
  gather_side<NV>(bR, sideR, o, true, nR, sR);
  __syncthreads();
  map2d(sL, sTmp, sL, m.ops + m.tab.fv2dgT[NL], nF, nL, NV);
  map2d(sR, sTmp, sR, m.ops + m.tab.fv2dgT[NR], nF, nR, NV);
  for (int t = threadIdx.x; t < n2F; t += blockDim.x) {
    int pp, qq;
    orient_map(o, t % nF, t / nF, nF, pp, qq);
    for (int v = 0; v < NV; ++v) {
      double x = (sL[v * GRID + t] - sR[v * GRID + t]) * ih2;
      if (aL > 0.0) x += fvL[(sideL * NV + v) * n2F + t];
      if (aR > 0.0) x -= fvR[(sideR * NV + v) * n2F + qq * nF + pp];
      sF[v * GRID + t] = x;
    }
  }
  __syncthreads();
  // linearisation point: the forward traces and sub-face normals
  if (aL > 0.0) gather_subcells<NV>(m, eL, sideL, o, false, sL);
  else gather_trace<NV>(m, u, eL, sideL, o, false, nL, sL);
  if (aR > 0.0) gather_subcells<NV>(m, eR, sideR, o, true, sR);
  else gather_trace<NV>(m, u, eR, sideR, o, true, nR, sR);
  for (int t = threadIdx.x; t < 3 * nM * nM; t += blockDim.x)
    sN[(t / (nM * nM)) * GRID + t % (nM * nM)] = nrm[t];
  __syncthreads();
  if (!(aL > 0.0)) map2d(sL, sTmp, sL, m.ops + m.tab.dg2fv[NL], nF, nL, NV);
  if (!(aR > 0.0)) map2d(sR, sTmp, sR, m.ops + m.tab.dg2fv[NR], nF, nR, NV);
  map2d(sN, sTmp, sN, m.ops + m.tab.dg2fv[M], nF, nM, 3);
  for (int t = threadIdx.x; t < n2F; t += blockDim.x) {
    double uL[NV], uR[NV], Fb[NV], uLb[NV], uRb[NV];
    for (int v = 0; v < NV; ++v) {
      uL[v] = sL[v * GRID + t];
      uR[v] = sR[v * GRID + t];
      Fb[v] = sF[v * GRID + t];
    }
    const double a = h * h;
    riemann_vjp<NV>(prm.face_flux_fv, prm.volume_flux, uL, uR, a * sN[t], a * sN[GRID + t],
                    a * sN[2 * GRID + t], m.gas, Fb, uLb, uRb);
    for (int v = 0; v < NV; ++v) {
      sL[v * GRID + t] = uLb[v];
      sR[v * GRID + t] = uRb[v];
    }
  }
  __syncthreads();
  if (aL > 0.0) {
    write_side<NV>(fvL, sL, sideL, o, false, nF, 1.0);
    for (int t = threadIdx.x; t < nL * nL; t += blockDim.x)
      for (int v = 0; v < NV; ++v) bL[(sideL * NV + v) * nL * nL + t] = 0.0;
  } else {
    map2d(sL, sTmp, sL, m.ops + m.tab.dg2fvT[NL], nL, nF, NV);
    write_side<NV>(bL, sL, sideL, o, false, nL, 1.0);
  }
  if (aR > 0.0) {
    write_side<NV>(fvR, sR, sideR, o, true, nF, 1.0);
    for (int t = threadIdx.x; t < nR * nR; t += blockDim.x)
      for (int v = 0; v < NV; ++v) bR[(sideR * NV + v) * nR * nR + t] = 0.0;
  } else {
    map2d(sR, sTmp, sR, m.ops + m.tab.dg2fvT[NR], nR, nF, NV);
    write_side<NV>(bR, sR, sideR, o, true, nR, 1.0);
  }
}

// Adjoint of face_conforming_kernel: same-degree faces between pure DG
// elements, one lane per face node, several faces per workgroup.  In place:
// the side-flux cotangents become the trace cotangents of both sides.
template <int N, int NV>
__global__ void __launch_bounds__(CONF_THREADS)
face_vjp_conforming_kernel(MeshView m, ParamsDev prm, const int32_t* __restrict__ flist, int fcount,
                           const double* __restrict__ u, const double* __restrict__ alpha) {
  constexpr int NP = N + 1, NP2 = NP * NP, FPB = CONF_THREADS / NP2;
  const int t = threadIdx.x;
  const int slot = t / NP2, r = t - slot * NP2;
  if (slot >= FPB) return;
  const int fi = blockIdx.x * FPB + slot;
  if (fi >= fcount) return;
  const int f = flist[fi];
  const int32_t* fc = m.faces + 5 * f;
  const int eL = fc[0], sideL = fc[1], eR = fc[2], sideR = fc[3], o = fc[4];
  if (alpha && (alpha[eL] > 0.0 || alpha[eR] > 0.0)) return;
  const int p = r % NP, q = r / NP;
  int pp, qq;
  orient_map(o, p, q, NP, pp, qq);
  const int64_t gL = m.elem_offset[eL] + side_node(sideL, p, q, NP);
  const int64_t gR = m.elem_offset[eR] + side_node(sideR, pp, qq, NP);
  const double* nrm = m.face_norm + m.face_norm_off[f];
  double* bL = m.fside + m.side_off[eL];
  double* bR = m.fside + m.side_off[eR];
  double uL[NV], uR[NV], Fb[NV], uLb[NV], uRb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    uL[v] = u[v * m.n_node + gL];
    uR[v] = u[v * m.n_node + gR];
    Fb[v] = bL[(sideL * NV + v) * NP2 + q * NP + p] - bR[(sideR * NV + v) * NP2 + qq * NP + pp];
  }
  riemann_vjp<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, nrm[r], nrm[NP2 + r], nrm[2 * NP2 + r], m.gas,
                  Fb, uLb, uRb);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bL[(sideL * NV + v) * NP2 + q * NP + p] = uLb[v];
    bR[(sideR * NV + v) * NP2 + qq * NP + pp] = uRb[v];
  }
}

// ---------------------------------------------------------------------------
// Viscous face terms at degree jumps (Section 3.1.1, eq. lift_flux and
// eq. visc_flux; Section 3.2.2), one face per one-wavefront workgroup; both
// write m.vside, the side layout of fside.  Same-degree faces are formed by
// the per-degree lift and viscous kernels themselves.
//  lift:    u* = (u^- + u^+) / 2: the higher side's trace projected to the
//           lower degree, u* formed there, the higher side receiving its
//           interpolation.
//  viscous: F^v* = (F^v(u^-, g^-) + F^v(u^+, g^+)) / 2 . n s with both
//           sides' traces of u and g on the higher degree and the face normal
//           (left outward) there; the left side receives +F^v*, the right
//           side -F^v*, the lower side its projection.
// ---------------------------------------------------------------------------
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
lift_face_mixed_kernel(MeshView m, const double* __restrict__ u) {
  __shared__ double B0[NV * GRID];
  __shared__ double B1[NV * GRID];
  __shared__ double B2[NV * GRID];
  __shared__ double B3[NV * GRID];
  const int fi = blockIdx.x;
  if (fi >= m.face_mixed_count) return;
  const int32_t* fc = m.faces + 5 * m.face_mixed[fi];
  const int eL = fc[0], sideL = fc[1], eR = fc[2], sideR = fc[3], o = fc[4];
  const int NL = m.degree[eL], NR = m.degree[eR];
  const bool left_low = NL < NR;
  const int lo = left_low ? NL : NR, hi = left_low ? NR : NL;
  const int nlo = lo + 1, nhi = hi + 1;
  gather_trace<NV>(m, u, eL, sideL, o, false, NL + 1, B0);
  gather_trace<NV>(m, u, eR, sideR, o, true, NR + 1, B1);
  wave_sync();
  const double* H = left_low ? B1 : B0;
  const double* L = left_low ? B0 : B1;
  map2d_sep_to<NV>(H, B3, B2, m.ops + m.tab.project[hi][lo], nlo, nhi);   // higher trace on the lower degree
  wave_sync();
  for (int t = threadIdx.x; t < nlo * nlo; t += blockDim.x)
    for (int v = 0; v < NV; ++v) B2[v * GRID + t] = 0.5 * (B2[v * GRID + t] + L[v * GRID + t]);
  wave_sync();
  double* bL = m.vside + m.side_off[eL];
  double* bR = m.vside + m.side_off[eR];
  if (left_low) {
    write_side<NV>(bL, B2, sideL, o, false, nlo, 1.0);
    map2d_sep_side<NV>(bR, B2, B3, m.ops + m.tab.interp[lo][hi], nhi, nlo, sideR, o, true, 1.0);
  } else {
    write_side<NV>(bR, B2, sideR, o, true, nlo, 1.0);
    map2d_sep_side<NV>(bL, B2, B3, m.ops + m.tab.interp[lo][hi], nhi, nlo, sideL, o, false, 1.0);
  }
}

template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
visc_face_mixed_kernel(MeshView m, const double* __restrict__ u) {
  constexpr int NW = 4 * NV;          // fields per face point: u, then g_x for x = 0, 1, 2
  __shared__ double SL[NW * GRID];
  __shared__ double SR[NW * GRID];
  __shared__ double ST[NW * GRID];
  __shared__ double SM[NW * GRID];
  const int fi = blockIdx.x;
  if (fi >= m.face_mixed_count) return;
  const int f = m.face_mixed[fi];
  const int32_t* fc = m.faces + 5 * f;
  const int eL = fc[0], sideL = fc[1], eR = fc[2], sideR = fc[3], o = fc[4];
  const int NL = m.degree[eL], NR = m.degree[eR];
  const bool left_low = NL < NR;
  const int lo = left_low ? NL : NR, M = left_low ? NR : NL;
  const int nlo = lo + 1, nM = M + 1, n2 = nM * nM;
  gather_trace<NV>(m, u, eL, sideL, o, false, NL + 1, SL);
  gather_trace<NV>(m, u, eR, sideR, o, true, NR + 1, SR);
  for (int x = 0; x < 3; ++x) {
    gather_trace<NV>(m, m.grad + (size_t)x * NV * m.n_node, eL, sideL, o, false, NL + 1, SL + (1 + x) * NV * GRID);
    gather_trace<NV>(m, m.grad + (size_t)x * NV * m.n_node, eR, sideR, o, true, NR + 1, SR + (1 + x) * NV * GRID);
  }
  wave_sync();
  map2d_sep_to<NW>(left_low ? SL : SR, ST, SM, m.ops + m.tab.interp[lo][M], nM, nlo);   // lower side on degree M
  wave_sync();
  const double* A = left_low ? SM : SL;
  const double* B = left_low ? SR : SM;
  const double* nrm = m.face_norm + m.face_norm_off[f];
  double* bL = m.vside + m.side_off[eL];
  double* bR = m.vside + m.side_off[eR];
  double* Fb = ST;                    // the flux on the degree-M grid, for the projection
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    double ua[NV], ub[NV], ga[3][NV], gb[3][NV], fa[3][NV], fb[3][NV], F[NV];
    for (int v = 0; v < NV; ++v) {
      ua[v] = A[v * GRID + t];
      ub[v] = B[v * GRID + t];
      for (int x = 0; x < 3; ++x) {
        ga[x][v] = A[((1 + x) * NV + v) * GRID + t];
        gb[x][v] = B[((1 + x) * NV + v) * GRID + t];
      }
    }
    viscous_flux<NV>(ua, ga, m.gas, m.visc, fa);
    viscous_flux<NV>(ub, gb, m.gas, m.visc, fb);
    const double n0 = nrm[t], n1 = nrm[n2 + t], n2v = nrm[2 * n2 + t];
    for (int v = 0; v < NV; ++v) {
      F[v] = 0.5 * ((fa[0][v] * n0 + fa[1][v] * n1 + fa[2][v] * n2v) + (fb[0][v] * n0 + fb[1][v] * n1 + fb[2][v] * n2v));
      Fb[v * GRID + t] = F[v];
    }
    const int p = t % nM, q = t / nM;
    if (left_low) {
      int pp, qq;
      orient_map(o, p, q, nM, pp, qq);
      for (int v = 0; v < NV; ++v) bR[(sideR * NV + v) * n2 + qq * nM + pp] = -F[v];
    } else {
      for (int v = 0; v < NV; ++v) bL[(sideL * NV + v) * n2 + q * nM + p] = F[v];
    }
  }
  wave_sync();
  if (left_low)
    map2d_sep_side<NV>(bL, Fb, SL, m.ops + m.tab.project[M][lo], nlo, nM, sideL, o, false, 1.0);
  else
    map2d_sep_side<NV>(bR, Fb, SR, m.ops + m.tab.project[M][lo], nlo, nM, sideR, o, true, -1.0);
}

// dst[f][qq][pp] = sum_q Aq[qq][q] sum_p Ap[pp][p] src[f][q][p] on an n x n face
// grid, a null matrix standing for the identity; T aliases neither src nor
// dst; one wave_sync inside, the caller synchronises around the call.
template <int NF>
__device__ void map2d_pq(const double* src, double* T, double* dst, const double* Ap, const double* Aq, int n) {
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int pp = t % n, q = t / n;
    if (Ap) {
      double a[MAXN + 1];
      load_row(Ap, n, pp, a);
#pragma unroll
      for (int f = 0; f < NF; ++f) T[f * GRID + t] = dot_row(a, src + f * GRID + q * n, 1, n);
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) T[f * GRID + t] = src[f * GRID + t];
    }
  }
  wave_sync();
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int pp = t % n, qq = t / n;
    if (Aq) {
      double a[MAXN + 1];
      load_row(Aq, n, qq, a);
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f * GRID + t] = dot_row(a, T + f * GRID + pp, n, n);
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f * GRID + t] = T[f * GRID + t];
    }
  }
}

// One small side's DG mortar flux (steps 2-5 of Section 3.2.3, both sides DG):
// sV holds the big side's data on the half (degree N0, step 1), sS and sN the
// small side's trace and reversed normal on the half's grid (degree Nk).  The
// small side's share goes to m.fside (bk, side sk, orientation ok); the big
// side's, mapped with M_k0, is added to sA.  sVM, sSM, sNM, sF, sT and sT2 are
// scratch; sV is overwritten.
template <int NV>
__device__ void mortar_dg_half(const MeshView& m, const ParamsDev& prm, int N0, int Nk, double* bk, int sk, int ok,
                               int kp, int kq, double* sV, double* sS, double* sN, double* sVM, double* sSM,
                               double* sNM, double* sF, double* sT, double* sT2, double* sA) {
  const int n0 = N0 + 1, nk = Nk + 1;
  const int M = N0 > Nk ? N0 : Nk, nM = M + 1;
  const double* VV = sV;
  const double* SS = sS;
  const double* NN = sN;
  if (N0 < M) {
    map2d_sep_to<NV>(sV, sT, sVM, m.ops + m.tab.interp[N0][M], nM, n0);
    VV = sVM;
    wave_sync();
  }
  if (Nk < M) {
    map2d_sep_to<NV>(sS, sT, sSM, m.ops + m.tab.interp[Nk][M], nM, nk);
    wave_sync();
    map2d_sep_to<3>(sN, sT, sNM, m.ops + m.tab.interp[Nk][M], nM, nk);
    SS = sSM;
    NN = sNM;
    wave_sync();
  }
  for (int t = threadIdx.x; t < nM * nM; t += blockDim.x) {
    double uL[NV], uR[NV], F[NV];
    for (int v = 0; v < NV; ++v) {
      uL[v] = VV[v * GRID + t];
      uR[v] = SS[v * GRID + t];
    }
    riemann<NV>(prm.face_flux_dg, prm.volume_flux, uL, uR, NN[t], NN[GRID + t], NN[2 * GRID + t], m.gas, F);
    for (int v = 0; v < NV; ++v) sF[v * GRID + t] = F[v];
  }
  wave_sync();
  if (Nk < M)
    map2d_sep_side<NV>(bk, sF, sT, m.ops + m.tab.project[M][Nk], nk, nM, sk, ok, true, -1.0);
  else
    write_side<NV>(bk, sF, sk, ok, true, nk, -1.0);
  wave_sync();
  const double* FB = sF;
  if (N0 < M) {
    map2d_sep_to<NV>(sF, sT, sT2, m.ops + m.tab.project[M][N0], n0, nM);
    FB = sT2;
    wave_sync();
  }
  map2d_pq<NV>(FB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_proj[N0][kp] : nullptr,
               kq >= 0 ? m.ops + m.tab.mortar_proj[N0][kq] : nullptr, n0);
  wave_sync();
  for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
    for (int v = 0; v < NV; ++v) sA[v * GRID + t] += sV[v * GRID + t];
  wave_sync();
}

// Non-conforming faces (Section 3.2.3), one mortar per one-wavefront
// workgroup.  For each small side k, when both sides are pure DG (the five
// steps): (1) the big side's trace interpolated to half (quarter) k with M_0k
// along the split directions; (2) it, the small side's trace on the half's
// grid (orientation o_k) and the small side's outward normal reversed, on the
// common degree max(N0, N_k); (3) the DG Riemann flux there; (4) the small
// side receives its projection to N_k, reversed, and the big side's share is
// projected to N0; (5) that share is mapped with M_k0 along the split
// directions and summed into the big side's flux.
// When either side is blended (the FV variants) the flux is taken on the small
// side's N_FV^2 sub-face grid: the big side's boundary sub-cell means mapped
// with M^FV_0k (a DG big side: its half's data of step 1 through V^{DG->FV}),
// the small side's boundary sub-cell means (a DG small side: V^{DG->FV} of its
// trace), and h^2 V^{DG->FV} of the reversed normal.  The small side takes the
// flux reversed (its FV part directly, its DG part through V^{FV->DG} / h^2);
// the big side's DG part takes V^{FV->DG} of it at N0 / h^2 mapped with M_k0,
// a blended big side's FV part the sub-face fluxes summed with M^FV_k0.
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
face_mortar_kernel(MeshView m, ParamsDev prm, const double* __restrict__ u, const double* __restrict__ alpha) {
  __shared__ double sB[NV * GRID];    // big side's trace (its boundary sub-cell means if blended)
  __shared__ double sA[NV * GRID];    // big side's flux, summed over its small sides
  __shared__ double sV[NV * GRID];    // the half's data from the big side
  __shared__ double sS[NV * GRID];    // small side's trace (or boundary sub-cell means) on the half's grid
  __shared__ double sN[3 * GRID];     // small side's normal, reversed
  __shared__ double sVM[NV * GRID];   // the three on the common degree or the sub-face grid; a blended
  __shared__ double sSM[NV * GRID];   // big side's FV flux sum lives in sVM (its half's data then
  __shared__ double sNM[3 * GRID];    // come straight from the sub-cell means, in sV)
  __shared__ double sF[NV * GRID];    // flux on the common degree or the sub-face grid
  __shared__ double sT[NV * GRID];    // scratch of the two-pass maps
  __shared__ double sT2[NV * GRID];
  const int qm = blockIdx.x;
  if (qm >= m.n_mortar) return;
  const int32_t* mr = m.mortars + 15 * qm;
  const int e0 = mr[0], s0 = mr[1], mt = mr[2];
  const int N0 = m.degree[e0], n0 = N0 + 1;
  const int nsub = mt == 3 ? 4 : 2;
  const bool a0 = alpha && alpha[e0] > 0.0;
  const int nF = m.n_fv, n2F = nF * nF;
  const double h2 = (2.0 / nF) * (2.0 / nF);
  double* sAF = sVM;
  if (a0) {
    gather_subcells<NV>(m, e0, s0, 0, false, sB);
    for (int t = threadIdx.x; t < n2F; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sAF[v * GRID + t] = 0.0;
  } else {
    gather_trace<NV>(m, u, e0, s0, 0, false, n0, sB);
  }
  for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
    for (int v = 0; v < NV; ++v) sA[v * GRID + t] = 0.0;
  wave_sync();
  for (int k = 0; k < nsub; ++k) {
    const int ek = mr[3 + k], sk = mr[7 + k], ok = mr[11 + k];
    const int kp = mt == 1 ? k : (mt == 2 ? -1 : (k & 1));
    const int kq = mt == 1 ? -1 : (mt == 2 ? k : (k >> 1));
    const bool ak = alpha && alpha[ek] > 0.0;
    if (a0)
      map2d_pq<NV>(sB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_fv_interp[kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_fv_interp[kq] : nullptr, nF);
    else
      map2d_pq<NV>(sB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_interp[N0][kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_interp[N0][kq] : nullptr, n0);
    const int Nk = m.degree[ek], nk = Nk + 1;
    if (ak)
      gather_subcells<NV>(m, ek, sk, ok, true, sS);
    else
      gather_trace<NV>(m, u, ek, sk, ok, true, nk, sS);
    gather_trace<3>(m, m.metric + (size_t)3 * (sk >> 1) * m.n_node, ek, sk, ok, true, nk, sN);
    wave_sync();
    const double rev = (sk & 1) ? -1.0 : 1.0;       // minus the outward sign of side sk
    for (int t = threadIdx.x; t < nk * nk; t += blockDim.x)
      for (int c = 0; c < 3; ++c) sN[c * GRID + t] *= rev;
    wave_sync();
    double* bk = m.fside + m.side_off[ek];
    if (a0 || ak) {
      const double* VV = sV;
      const double* SS = sS;
      if (!a0) {
        map2d_sep_to<NV>(sV, sT, sVM, m.ops + m.tab.dg2fv[N0], nF, n0);
        VV = sVM;
        wave_sync();
      }
      if (!ak) {
        map2d_sep_to<NV>(sS, sT, sSM, m.ops + m.tab.dg2fv[Nk], nF, nk);
        SS = sSM;
        wave_sync();
      }
      map2d_sep_to<3>(sN, sT, sNM, m.ops + m.tab.dg2fv[Nk], nF, nk);
      wave_sync();
      for (int t = threadIdx.x; t < n2F; t += blockDim.x) {
        double uL[NV], uR[NV], F[NV];
        for (int v = 0; v < NV; ++v) {
          uL[v] = VV[v * GRID + t];
          uR[v] = SS[v * GRID + t];
        }
        riemann<NV>(prm.face_flux_fv, prm.volume_flux, uL, uR, h2 * sNM[t], h2 * sNM[GRID + t],
                    h2 * sNM[2 * GRID + t], m.gas, F);
        for (int v = 0; v < NV; ++v) sF[v * GRID + t] = F[v];
      }
      wave_sync();
      map2d_sep_side<NV>(bk, sF, sT, m.ops + m.tab.fv2dg[Nk], nk, nF, sk, ok, true, -1.0 / h2);
      if (ak) write_side<NV>(m.fvside + (size_t)ek * 6 * NV * n2F, sF, sk, ok, true, nF, -1.0);
      wave_sync();
      map2d_sep_to<NV>(sF, sT, sT2, m.ops + m.tab.fv2dg[N0], n0, nF);
      wave_sync();
      map2d_pq<NV>(sT2, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_proj[N0][kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_proj[N0][kq] : nullptr, n0);
      wave_sync();
      const double ih2 = 1.0 / h2;
      for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
        for (int v = 0; v < NV; ++v) sA[v * GRID + t] += ih2 * sV[v * GRID + t];
      if (a0) {
        map2d_pq<NV>(sF, sT2, sS, kp >= 0 ? m.ops + m.tab.mortar_fv_proj[kp] : nullptr,
                     kq >= 0 ? m.ops + m.tab.mortar_fv_proj[kq] : nullptr, nF);
        wave_sync();
        for (int t = threadIdx.x; t < n2F; t += blockDim.x)
          for (int v = 0; v < NV; ++v) sAF[v * GRID + t] += sS[v * GRID + t];
      }
      wave_sync();
      continue;
    }
    mortar_dg_half<NV>(m, prm, N0, Nk, bk, sk, ok, kp, kq, sV, sS, sN, sVM, sSM, sNM, sF, sT, sT2, sA);
  }
  write_side<NV>(m.fside + m.side_off[e0], sA, s0, 0, false, n0, 1.0);
  if (a0) write_side<NV>(m.fvside + (size_t)e0 * 6 * NV * n2F, sAF, s0, 0, false, nF, 1.0);
}

// Viscous terms at the mortars (Sections 3.1.1, 3.2.2 and 3.2.3), one mortar
// per one-wavefront workgroup, into m.vside of the big side and of each small
// side, where the lift and viscous kernels read them as at a degree jump.
// Lift: on half (quarter) k the big side's trace mapped with M_0k and the
// small side's trace meet on the lower of the two degrees (the higher one
// projected down); their mean, interpolated up, goes to the small side, and
// the big side takes (1/2)^s sum_k M_k0 of it (s split directions).
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
mortar_lift_kernel(MeshView m, const double* __restrict__ u) {
  __shared__ double sB[NV * GRID];    // big side's trace
  __shared__ double sA[NV * GRID];    // big side's face value, summed over its small sides
  __shared__ double sV[NV * GRID];    // the half's data from the big side
  __shared__ double sS[NV * GRID];    // small side's trace on the half's grid
  __shared__ double sW[NV * GRID];    // a trace projected to the lower degree
  __shared__ double sP[NV * GRID];    // the big side's share of half k
  __shared__ double sT[NV * GRID];    // scratch of the two-pass maps
  const int qm = blockIdx.x;
  if (qm >= m.n_mortar) return;
  const int32_t* mr = m.mortars + 15 * qm;
  const int e0 = mr[0], s0 = mr[1], mt = mr[2];
  const int N0 = m.degree[e0], n0 = N0 + 1;
  const int nsub = mt == 3 ? 4 : 2;
  const double share = mt == 3 ? 0.25 : 0.5;
  gather_trace<NV>(m, u, e0, s0, 0, false, n0, sB);
  for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
    for (int v = 0; v < NV; ++v) sA[v * GRID + t] = 0.0;
  wave_sync();
  for (int k = 0; k < nsub; ++k) {
    const int ek = mr[3 + k], sk = mr[7 + k], ok = mr[11 + k];
    const int kp = mt == 1 ? k : (mt == 2 ? -1 : (k & 1));
    const int kq = mt == 1 ? -1 : (mt == 2 ? k : (k >> 1));
    map2d_pq<NV>(sB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_interp[N0][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_interp[N0][kq] : nullptr, n0);
    const int Nk = m.degree[ek], nk = Nk + 1;
    gather_trace<NV>(m, u, ek, sk, ok, true, nk, sS);
    wave_sync();
    const int lo = N0 < Nk ? N0 : Nk, nlo = lo + 1;
    double* X = sV;                   // the mean on the lower degree (in place where possible)
    const double* Y = sS;
    if (N0 > lo) {
      map2d_sep_to<NV>(sV, sT, sW, m.ops + m.tab.project[N0][lo], nlo, n0);
      X = sW;
      wave_sync();
    } else if (Nk > lo) {
      map2d_sep_to<NV>(sS, sT, sW, m.ops + m.tab.project[Nk][lo], nlo, nk);
      Y = sW;
      wave_sync();
    }
    for (int t = threadIdx.x; t < nlo * nlo; t += blockDim.x)
      for (int v = 0; v < NV; ++v) X[v * GRID + t] = 0.5 * (X[v * GRID + t] + Y[v * GRID + t]);
    wave_sync();
    double* bk = m.vside + m.side_off[ek];
    if (Nk > lo)
      map2d_sep_side<NV>(bk, X, sT, m.ops + m.tab.interp[lo][Nk], nk, nlo, sk, ok, true, 1.0);
    else
      write_side<NV>(bk, X, sk, ok, true, nk, 1.0);
    wave_sync();
    const double* Z = X;
    if (N0 > lo) {
      map2d_sep_to<NV>(X, sT, sS, m.ops + m.tab.interp[lo][N0], n0, nlo);
      Z = sS;
      wave_sync();
    }
    map2d_pq<NV>(Z, sT, sP, kp >= 0 ? m.ops + m.tab.mortar_proj[N0][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_proj[N0][kq] : nullptr, n0);
    wave_sync();
    for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sA[v * GRID + t] += share * sP[v * GRID + t];
    wave_sync();
  }
  write_side<NV>(m.vside + m.side_off[e0], sA, s0, 0, false, n0, 1.0);
}

// Viscous flux: on half (quarter) k the big side's traces of u and g mapped
// with M_0k, the small side's traces and its outward normal reversed, all on
// the common degree max(N0, N_k); the mean of the two sides' fluxes there;
// the small side takes its projection to N_k, reversed, the big side sum_k
// M_k0 of its projection to N0.
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
mortar_visc_kernel(MeshView m, const double* __restrict__ u) {
  constexpr int NW = 4 * NV;          // fields per face point: u, then g_x for x = 0, 1, 2
  __shared__ double sB[NW * GRID];    // big side's traces
  __shared__ double sV[NW * GRID];    // the half's data from the big side
  __shared__ double sS[NW * GRID];    // small side's traces on the half's grid
  __shared__ double sM[NW * GRID];    // the side of lower degree on the common degree
  __shared__ double sT[NW * GRID];    // scratch of the two-pass maps, then the flux
  __shared__ double sN[3 * GRID];     // small side's normal, reversed
  __shared__ double sNM[3 * GRID];
  __shared__ double sA[NV * GRID];    // big side's flux, summed over its small sides
  const int qm = blockIdx.x;
  if (qm >= m.n_mortar) return;
  const int32_t* mr = m.mortars + 15 * qm;
  const int e0 = mr[0], s0 = mr[1], mt = mr[2];
  const int N0 = m.degree[e0], n0 = N0 + 1;
  const int nsub = mt == 3 ? 4 : 2;
  auto gather_ug = [&](int e, int side, int o, bool right, int n, double* dst) {
    gather_trace<NV>(m, u, e, side, o, right, n, dst);
    for (int x = 0; x < 3; ++x)
      gather_trace<NV>(m, m.grad + (size_t)x * NV * m.n_node, e, side, o, right, n, dst + (1 + x) * NV * GRID);
  };
  gather_ug(e0, s0, 0, false, n0, sB);
  for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
    for (int v = 0; v < NV; ++v) sA[v * GRID + t] = 0.0;
  wave_sync();
  for (int k = 0; k < nsub; ++k) {
    const int ek = mr[3 + k], sk = mr[7 + k], ok = mr[11 + k];
    const int kp = mt == 1 ? k : (mt == 2 ? -1 : (k & 1));
    const int kq = mt == 1 ? -1 : (mt == 2 ? k : (k >> 1));
    map2d_pq<NW>(sB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_interp[N0][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_interp[N0][kq] : nullptr, n0);
    const int Nk = m.degree[ek], nk = Nk + 1;
    gather_ug(ek, sk, ok, true, nk, sS);
    gather_trace<3>(m, m.metric + (size_t)3 * (sk >> 1) * m.n_node, ek, sk, ok, true, nk, sN);
    wave_sync();
    const double rev = (sk & 1) ? -1.0 : 1.0;       // minus the outward sign of side sk
    for (int t = threadIdx.x; t < nk * nk; t += blockDim.x)
      for (int c = 0; c < 3; ++c) sN[c * GRID + t] *= rev;
    wave_sync();
    const int M = N0 > Nk ? N0 : Nk, nM = M + 1;
    const double* A = sV;
    const double* B = sS;
    const double* NN = sN;
    if (N0 < M) {
      map2d_sep_to<NW>(sV, sT, sM, m.ops + m.tab.interp[N0][M], nM, n0);
      A = sM;
      wave_sync();
    } else if (Nk < M) {
      map2d_sep_to<NW>(sS, sT, sM, m.ops + m.tab.interp[Nk][M], nM, nk);
      wave_sync();
      map2d_sep_to<3>(sN, sT, sNM, m.ops + m.tab.interp[Nk][M], nM, nk);
      B = sM;
      NN = sNM;
      wave_sync();
    }
    double* Fb = sT;                  // the flux on the common degree
    for (int t = threadIdx.x; t < nM * nM; t += blockDim.x) {
      double ua[NV], ub[NV], ga[3][NV], gb[3][NV], fa[3][NV], fb[3][NV];
      for (int v = 0; v < NV; ++v) {
        ua[v] = A[v * GRID + t];
        ub[v] = B[v * GRID + t];
        for (int x = 0; x < 3; ++x) {
          ga[x][v] = A[((1 + x) * NV + v) * GRID + t];
          gb[x][v] = B[((1 + x) * NV + v) * GRID + t];
        }
      }
      viscous_flux<NV>(ua, ga, m.gas, m.visc, fa);
      viscous_flux<NV>(ub, gb, m.gas, m.visc, fb);
      const double c0 = NN[t], c1 = NN[GRID + t], c2 = NN[2 * GRID + t];
      for (int v = 0; v < NV; ++v)
        Fb[v * GRID + t] = 0.5 * ((fa[0][v] * c0 + fa[1][v] * c1 + fa[2][v] * c2) +
                                  (fb[0][v] * c0 + fb[1][v] * c1 + fb[2][v] * c2));
    }
    wave_sync();
    double* bk = m.vside + m.side_off[ek];
    if (Nk < M)
      map2d_sep_side<NV>(bk, Fb, sS, m.ops + m.tab.project[M][Nk], nk, nM, sk, ok, true, -1.0);
    else
      write_side<NV>(bk, Fb, sk, ok, true, nk, -1.0);
    wave_sync();
    const double* FB = Fb;
    if (N0 < M) {
      map2d_sep_to<NV>(Fb, sS, sV, m.ops + m.tab.project[M][N0], n0, nM);
      FB = sV;
      wave_sync();
    }
    map2d_pq<NV>(FB, sS, sM, kp >= 0 ? m.ops + m.tab.mortar_proj[N0][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_proj[N0][kq] : nullptr, n0);
    wave_sync();
    for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sA[v * GRID + t] += sM[v * GRID + t];
    wave_sync();
  }
  write_side<NV>(m.vside + m.side_off[e0], sA, s0, 0, false, n0, 1.0);
}

// Adjoint of the mortar fluxes, pure DG, one degree on both sides of each
// mortar, one mortar per one-wavefront workgroup.  Forward, per small side k:
// F = F*(M_0k t_0, t_k, n_k) gave the small side -F and the big side M_k0 F.
// Reverse, with the side-flux cotangents b_k (small side) and A (big side):
// F_bar = M_k0^T A - b_k, (t_v_bar, t_k_bar) = (dF*/d(t_v, t_k))^T F_bar; the
// small side's trace cotangent is t_k_bar, the big side's sum_k M_0k^T t_v_bar.
// In place in m.fside, like the face adjoint kernels (each side belongs to one
// face or mortar).
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
mortar_vjp_kernel(MeshView m, ParamsDev prm, const double* __restrict__ u) {
  __shared__ double sB[NV * GRID];    // big side's trace
  __shared__ double sAb[NV * GRID];   // big side's flux cotangent
  __shared__ double sUb[NV * GRID];   // big side's trace cotangent, summed over its small sides
  __shared__ double sV[NV * GRID];    // the half's data from the big side, then its cotangent
  __shared__ double sS[NV * GRID];    // small side's trace on the half's grid
  __shared__ double sC[NV * GRID];    // small side's flux cotangent, then its trace cotangent
  __shared__ double sG[NV * GRID];    // M_k0^T A
  __shared__ double sN[3 * GRID];     // small side's normal, reversed
  __shared__ double sT[NV * GRID];    // scratch of the two-pass maps
  __shared__ double sT2[NV * GRID];
  const int qm = blockIdx.x;
  if (qm >= m.n_mortar) return;
  const int32_t* mr = m.mortars + 15 * qm;
  const int e0 = mr[0], s0 = mr[1], mt = mr[2];
  const int N = m.degree[e0], n = N + 1;
  const int nsub = mt == 3 ? 4 : 2;
  gather_trace<NV>(m, u, e0, s0, 0, false, n, sB);
  gather_side<NV>(m.fside + m.side_off[e0], s0, 0, false, n, sAb);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x)
    for (int v = 0; v < NV; ++v) sUb[v * GRID + t] = 0.0;
  wave_sync();
  for (int k = 0; k < nsub; ++k) {
    const int ek = mr[3 + k], sk = mr[7 + k], ok = mr[11 + k];
    const int kp = mt == 1 ? k : (mt == 2 ? -1 : (k & 1));
    const int kq = mt == 1 ? -1 : (mt == 2 ? k : (k >> 1));
    map2d_pq<NV>(sB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_interp[N][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_interp[N][kq] : nullptr, n);
    map2d_pq<NV>(sAb, sT2, sG, kp >= 0 ? m.ops + m.tab.mortar_projT[N][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_projT[N][kq] : nullptr, n);
    double* bk = m.fside + m.side_off[ek];
    gather_trace<NV>(m, u, ek, sk, ok, true, n, sS);
    gather_side<NV>(bk, sk, ok, true, n, sC);
    gather_trace<3>(m, m.metric + (size_t)3 * (sk >> 1) * m.n_node, ek, sk, ok, true, n, sN);
    wave_sync();
    const double rev = (sk & 1) ? -1.0 : 1.0;       // minus the outward sign of side sk
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
      double uv[NV], us[NV], Fb[NV], uvb[NV], usb[NV];
      for (int v = 0; v < NV; ++v) {
        uv[v] = sV[v * GRID + t];
        us[v] = sS[v * GRID + t];
        Fb[v] = sG[v * GRID + t] - sC[v * GRID + t];
      }
      riemann_vjp<NV>(prm.face_flux_dg, prm.volume_flux, uv, us, rev * sN[t], rev * sN[GRID + t],
                      rev * sN[2 * GRID + t], m.gas, Fb, uvb, usb);
      for (int v = 0; v < NV; ++v) {
        sV[v * GRID + t] = uvb[v];
        sC[v * GRID + t] = usb[v];
      }
    }
    wave_sync();
    write_side<NV>(bk, sC, sk, ok, true, n, 1.0);
    map2d_pq<NV>(sV, sT, sT2, kp >= 0 ? m.ops + m.tab.mortar_interpT[N][kp] : nullptr,
                 kq >= 0 ? m.ops + m.tab.mortar_interpT[N][kq] : nullptr, n);
    wave_sync();
    for (int t = threadIdx.x; t < n * n; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sUb[v * GRID + t] += sT2[v * GRID + t];
    wave_sync();
  }
  write_side<NV>(m.fside + m.side_off[e0], sUb, s0, 0, false, n, 1.0);
}

// Sub-cell layer `depth` (0 at the side) of side `side` of element e's means
// (ub: [K][NV][n^3]) on the left side's sub-face grid.
template <int NV>
__device__ void gather_layer(const double* ub, int e, int side, int depth, int o, bool right, int n, double* dst) {
  const int S3 = n * n * n;
  const double* b = ub + (size_t)e * NV * S3;
  const int step = (side >> 1) == 0 ? 1 : ((side >> 1) == 1 ? n : n * n);
  const int inward = (side & 1) ? -depth * step : depth * step;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int p = t % n, q = t / n;
    if (right) orient_map(o, p, q, n, p, q);
    const int c = side_node(side, p, q, n) + inward;
    for (int v = 0; v < NV; ++v) dst[v * GRID + t] = b[v * S3 + c];
  }
}

// dst = the minmod-reconstructed face value of boundary means cb with the next
// means ci and the ghost cg (primitives; cb + minmod(cb - ci, cg - cb) / 2).
template <int NV>
__device__ void reconstruct_face(const double* cb, const double* ci, const double* cg, const GasDev& gas, int n2,
                                 double* dst) {
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    double xb[NV], xi[NV], xg[NV], wb[NV], wi[NV], wg[NV], wf[NV], out[NV];
    for (int v = 0; v < NV; ++v) {
      xb[v] = cb[v * GRID + t];
      xi[v] = ci[v * GRID + t];
      xg[v] = cg[v * GRID + t];
    }
    cons_to_w<NV>(xb, gas, wb);
    cons_to_w<NV>(xi, gas, wi);
    cons_to_w<NV>(xg, gas, wg);
    for (int v = 0; v < NV; ++v) wf[v] = wb[v] + 0.5 * minmod(wb[v] - wi[v], wg[v] - wb[v]);
    w_to_cons<NV>(wf, gas, out);
    for (int v = 0; v < NV; ++v) dst[v * GRID + t] = out[v];
  }
}

// Mortars with FV-stored elements (fv[e] > 0; Sections 3.1.2, 3.2.3), one
// mortar per one-wavefront workgroup.  A small side whose half has no
// FV-stored side takes the DG mortar flux.  Otherwise the flux is taken on the
// small side's N_FV^2 sub-face grid with the FV Riemann flux, as for blended
// elements, between minmod-reconstructed values: an FV-stored small side
// reconstructs from its boundary and next layers with the big side's data on
// its half as ghost (the big side's boundary means through M^FV_0k, or a DG
// big side's half trace through V^{DG->FV}); an FV-stored big side's ghost
// on each of its sub-faces is the mean of the small sides' boundary data
// over it, (1/2)^s sum_k M^FV_k0 c_k, and its reconstructed face values reach
// the halves through M^FV_0k.  The small side takes the flux reversed
// (m.fvside, or m.fside through V^{FV->DG} / h^2); the big side sum_k M^FV_k0
// of it (m.fvside) or sum_k M_k0 of its V^{FV->DG} / h^2 (m.fside).  The
// ghosts of FV-stored sides go to m.fvghost.
template <int NV>
__global__ void __launch_bounds__(FACE_THREADS)
mortar_fvs_kernel(MeshView m, ParamsDev prm, const double* __restrict__ u, const double* __restrict__ ufv,
                  const double* __restrict__ fv) {
  __shared__ double sB[NV * GRID];    // big side's trace (DG) or boundary means (FV)
  __shared__ double sI[NV * GRID];    // FV big side: its next layer, then its reconstructed face values
  __shared__ double sG0[NV * GRID];   // FV big side: its ghost
  __shared__ double sA[NV * GRID];    // big side's flux, summed over its small sides
  __shared__ double sV[NV * GRID];    // the big side's data on the half
  __shared__ double sS[NV * GRID];    // small side's trace or boundary means on the half's grid
  __shared__ double sSI[NV * GRID];   // FV small side: its next layer
  __shared__ double sCG[NV * GRID];   // FV small side: its ghost, then its reconstructed values
  __shared__ double sN[3 * GRID];     // small side's normal, reversed
  __shared__ double sNM[3 * GRID];    // on the common degree or the sub-face grid
  __shared__ double sVM[NV * GRID];   // DG data on the common degree or the sub-face grid
  __shared__ double sSM[NV * GRID];
  __shared__ double sF[NV * GRID];    // flux
  __shared__ double sT[NV * GRID];    // scratch of the two-pass maps
  __shared__ double sT2[NV * GRID];
  const int qm = blockIdx.x;
  if (qm >= m.n_mortar) return;
  const int32_t* mr = m.mortars + 15 * qm;
  const int e0 = mr[0], s0 = mr[1], mt = mr[2];
  const int N0 = m.degree[e0], n0 = N0 + 1;
  const int nsub = mt == 3 ? 4 : 2;
  const bool a0 = fv[e0] > 0.0;
  const int nF = m.n_fv, n2F = nF * nF;
  const double h2 = (2.0 / nF) * (2.0 / nF);
  const size_t fblk = (size_t)6 * NV * n2F;
  auto split = [&](int k, int& kp, int& kq) {
    kp = mt == 1 ? k : (mt == 2 ? -1 : (k & 1));
    kq = mt == 1 ? -1 : (mt == 2 ? k : (k >> 1));
  };
  if (a0) {
    // the big side's ghost from every small side's boundary data, then its face values
    gather_layer<NV>(ufv, e0, s0, 0, 0, false, nF, sB);
    gather_layer<NV>(ufv, e0, s0, 1, 0, false, nF, sI);
    for (int t = threadIdx.x; t < n2F; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sG0[v * GRID + t] = 0.0;
    wave_sync();
    const double share = mt == 3 ? 0.25 : 0.5;
    for (int k = 0; k < nsub; ++k) {
      const int ek = mr[3 + k], sk = mr[7 + k], ok = mr[11 + k];
      int kp, kq;
      split(k, kp, kq);
      const double* C = sS;
      if (fv[ek] > 0.0) {
        gather_layer<NV>(ufv, ek, sk, 0, ok, true, nF, sS);
      } else {
        const int nk = m.degree[ek] + 1;
        gather_trace<NV>(m, u, ek, sk, ok, true, nk, sSM);
        wave_sync();
        map2d_sep_to<NV>(sSM, sT, sS, m.ops + m.tab.dg2fv[nk - 1], nF, nk);
      }
      wave_sync();
      map2d_pq<NV>(C, sT, sT2, kp >= 0 ? m.ops + m.tab.mortar_fv_proj[kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_fv_proj[kq] : nullptr, nF);
      wave_sync();
      for (int t = threadIdx.x; t < n2F; t += blockDim.x)
        for (int v = 0; v < NV; ++v) sG0[v * GRID + t] += share * sT2[v * GRID + t];
      wave_sync();
    }
    write_side<NV>(m.fvghost + (size_t)e0 * fblk, sG0, s0, 0, false, nF, 1.0);
    reconstruct_face<NV>(sB, sI, sG0, m.gas, n2F, sI);     // in place: each lane its own point
    for (int t = threadIdx.x; t < n2F; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sA[v * GRID + t] = 0.0;
  } else {
    gather_trace<NV>(m, u, e0, s0, 0, false, n0, sB);
    for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
      for (int v = 0; v < NV; ++v) sA[v * GRID + t] = 0.0;
  }
  wave_sync();
  for (int k = 0; k < nsub; ++k) {
    const int ek = mr[3 + k], sk = mr[7 + k], ok = mr[11 + k];
    int kp, kq;
    split(k, kp, kq);
    const bool ak = fv[ek] > 0.0;
    const int Nk = m.degree[ek], nk = Nk + 1;
    double* bk = m.fside + m.side_off[ek];
    gather_trace<3>(m, m.metric + (size_t)3 * (sk >> 1) * m.n_node, ek, sk, ok, true, nk, sN);
    if (!a0)
      map2d_pq<NV>(sB, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_interp[N0][kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_interp[N0][kq] : nullptr, n0);
    if (ak) {
      gather_layer<NV>(ufv, ek, sk, 0, ok, true, nF, sS);
      gather_layer<NV>(ufv, ek, sk, 1, ok, true, nF, sSI);
    } else {
      gather_trace<NV>(m, u, ek, sk, ok, true, nk, sS);
    }
    wave_sync();
    const double rev = (sk & 1) ? -1.0 : 1.0;       // minus the outward sign of side sk
    for (int t = threadIdx.x; t < nk * nk; t += blockDim.x)
      for (int c = 0; c < 3; ++c) sN[c * GRID + t] *= rev;
    wave_sync();
    if (!a0 && !ak) {                     // the DG mortar flux on the common degree
      mortar_dg_half<NV>(m, prm, N0, Nk, bk, sk, ok, kp, kq, sV, sS, sN, sVM, sSM, sNM, sF, sT, sT2, sA);
      continue;
    }
    // the FV variant on the small side's sub-face grid: the big side's value on the half (sVM)
    if (a0) {
      map2d_pq<NV>(sI, sT, sVM, kp >= 0 ? m.ops + m.tab.mortar_fv_interp[kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_fv_interp[kq] : nullptr, nF);
    } else {
      map2d_sep_to<NV>(sV, sT, sVM, m.ops + m.tab.dg2fv[N0], nF, n0);
    }
    wave_sync();
    // the small side's value (sSM): reconstructed with its ghost, or its mapped trace
    if (ak) {
      if (a0)
        map2d_pq<NV>(sB, sT, sCG, kp >= 0 ? m.ops + m.tab.mortar_fv_interp[kp] : nullptr,
                     kq >= 0 ? m.ops + m.tab.mortar_fv_interp[kq] : nullptr, nF);
      else
        for (int t = threadIdx.x; t < n2F; t += blockDim.x)
          for (int v = 0; v < NV; ++v) sCG[v * GRID + t] = sVM[v * GRID + t];
      wave_sync();
      write_side<NV>(m.fvghost + (size_t)ek * fblk, sCG, sk, ok, true, nF, 1.0);
      reconstruct_face<NV>(sS, sSI, sCG, m.gas, n2F, sSM);
    } else {
      map2d_sep_to<NV>(sS, sT, sSM, m.ops + m.tab.dg2fv[Nk], nF, nk);
    }
    map2d_sep_to<3>(sN, sT2, sNM, m.ops + m.tab.dg2fv[Nk], nF, nk);
    wave_sync();
    for (int t = threadIdx.x; t < n2F; t += blockDim.x) {
      double uL[NV], uR[NV], F[NV];
      for (int v = 0; v < NV; ++v) {
        uL[v] = sVM[v * GRID + t];
        uR[v] = sSM[v * GRID + t];
      }
      riemann<NV>(prm.face_flux_fv, prm.volume_flux, uL, uR, h2 * sNM[t], h2 * sNM[GRID + t],
                  h2 * sNM[2 * GRID + t], m.gas, F);
      for (int v = 0; v < NV; ++v) sF[v * GRID + t] = F[v];
    }
    wave_sync();
    if (ak)
      write_side<NV>(m.fvside + (size_t)ek * fblk, sF, sk, ok, true, nF, -1.0);
    else
      map2d_sep_side<NV>(bk, sF, sT, m.ops + m.tab.fv2dg[Nk], nk, nF, sk, ok, true, -1.0 / h2);
    wave_sync();
    if (a0) {
      map2d_pq<NV>(sF, sT, sT2, kp >= 0 ? m.ops + m.tab.mortar_fv_proj[kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_fv_proj[kq] : nullptr, nF);
      wave_sync();
      for (int t = threadIdx.x; t < n2F; t += blockDim.x)
        for (int v = 0; v < NV; ++v) sA[v * GRID + t] += sT2[v * GRID + t];
    } else {
      map2d_sep_to<NV>(sF, sT, sT2, m.ops + m.tab.fv2dg[N0], n0, nF);
      wave_sync();
      map2d_pq<NV>(sT2, sT, sV, kp >= 0 ? m.ops + m.tab.mortar_proj[N0][kp] : nullptr,
                   kq >= 0 ? m.ops + m.tab.mortar_proj[N0][kq] : nullptr, n0);
      wave_sync();
      for (int t = threadIdx.x; t < n0 * n0; t += blockDim.x)
        for (int v = 0; v < NV; ++v) sA[v * GRID + t] += sV[v * GRID + t] / h2;
    }
    wave_sync();
  }
  if (a0)
    write_side<NV>(m.fvside + (size_t)e0 * fblk, sA, s0, 0, false, nF, 1.0);
  else
    write_side<NV>(m.fside + m.side_off[e0], sA, s0, 0, false, n0, 1.0);
}

}  // namespace

template <int NV>
static hipError_t launch_faces_vjp_t(const MeshView& m, const ParamsDev& p, const double* u,
                                     const double* alpha, hipStream_t s) {
  for (int N = 1; N <= MAXN; ++N) {
    const int cnt = m.face_conf_count[N];
    if (cnt == 0) continue;
    const int np2 = (N + 1) * (N + 1), fpb = CONF_THREADS / np2;
    const dim3 grid((cnt + fpb - 1) / fpb), block(CONF_THREADS);
    const int32_t* fl = m.face_conf[N];
    switch (N) {
      case 1: hipLaunchKernelGGL((face_vjp_conforming_kernel<1, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
      case 2: hipLaunchKernelGGL((face_vjp_conforming_kernel<2, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
      case 3: hipLaunchKernelGGL((face_vjp_conforming_kernel<3, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
      case 4: hipLaunchKernelGGL((face_vjp_conforming_kernel<4, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
      case 5: hipLaunchKernelGGL((face_vjp_conforming_kernel<5, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
      case 6: hipLaunchKernelGGL((face_vjp_conforming_kernel<6, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
      default: hipLaunchKernelGGL((face_vjp_conforming_kernel<7, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha); break;
    }
    if (hipError_t e = hipGetLastError()) return e;
  }
  // degree jumps and FV faces, one face per workgroup
  if (m.face_mixed_count > 0 || alpha) {
    hipLaunchKernelGGL((face_vjp_kernel<NV>), dim3(m.n_face), dim3(FACE_THREADS), 0, s, m, p, u, alpha, true);
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipSuccess;
}

hipError_t launch_faces_vjp(const MeshView& m, const ParamsDev& p, const double* u, const double* alpha,
                            hipStream_t s) {
  if (m.n_face == 0) return hipSuccess;
  return m.nvar == 5 ? launch_faces_vjp_t<5>(m, p, u, alpha, s) : launch_faces_vjp_t<6>(m, p, u, alpha, s);
}

template <int NV>
static hipError_t launch_face_class_t(const MeshView& m, const ParamsDev& p, const double* u,
                                      const double* alpha, int cls, bool read_trace, hipStream_t s) {
  const double* tr = read_trace && cls >= TRACE_MIN_N && cls <= MAXN ? m.trace : nullptr;
  if (cls >= 1 && cls <= MAXN) {
    const int N = cls, cnt = m.face_conf_count[N];
    if (cnt == 0) return hipSuccess;
    const int np2 = (N + 1) * (N + 1), fpb = CONF_THREADS / np2;
    const dim3 grid((cnt + fpb - 1) / fpb), block(CONF_THREADS);
    const ConfRec* fl = m.face_conf_rec[N];
    switch (N) {
      case 1: hipLaunchKernelGGL((face_conforming_kernel<1, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
      case 2: hipLaunchKernelGGL((face_conforming_kernel<2, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
      case 3: hipLaunchKernelGGL((face_conforming_kernel<3, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
      case 4: hipLaunchKernelGGL((face_conforming_kernel<4, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
      case 5: hipLaunchKernelGGL((face_conforming_kernel<5, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
      case 6: hipLaunchKernelGGL((face_conforming_kernel<6, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
      default: hipLaunchKernelGGL((face_conforming_kernel<7, NV>), grid, block, 0, s, m, p, fl, cnt, u, alpha, tr); break;
    }
    return hipGetLastError();
  }
  if (cls == FACE_CLASS_MIXED) {
    if (m.face_mixed_count == 0) return hipSuccess;
    const int grid = m.face_mixed_count < 65536 ? m.face_mixed_count : 65536;
    hipLaunchKernelGGL((face_mixed_kernel<NV>), dim3(grid), dim3(FACE_THREADS), 0, s, m, p, m.face_mixed,
                       m.face_mixed_count, u, alpha);
    return hipGetLastError();
  }
  if (cls == FACE_CLASS_FV) {
    if (!alpha) return hipSuccess;
    hipLaunchKernelGGL((face_fv_kernel<NV>), dim3(m.K), dim3(FACE_THREADS), 0, s, m, p, u, alpha);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_face_fv_stored(const MeshView& m, const ParamsDev& p, const double* u, const double* ufv,
                                 const double* fv, hipStream_t s) {
  if (m.n_face == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((face_fvs_kernel<5>), dim3(m.K), dim3(FACE_THREADS), 0, s, m, p, u, ufv, fv);
  else
    hipLaunchKernelGGL((face_fvs_kernel<6>), dim3(m.K), dim3(FACE_THREADS), 0, s, m, p, u, ufv, fv);
  return hipGetLastError();
}

bool face_class_present(const MeshView& m, const double* alpha, int cls) {
  if (cls >= 1 && cls <= MAXN) return m.face_conf_count[cls] > 0;
  if (cls == FACE_CLASS_MIXED) return m.face_mixed_count > 0;
  if (cls == FACE_CLASS_FV) return alpha != nullptr && m.n_face > 0;
  return false;
}

hipError_t launch_face_class(const MeshView& m, const ParamsDev& p, const double* u, const double* alpha,
                             int cls, bool read_trace, hipStream_t s) {
  if (m.n_face == 0) return hipSuccess;
  return m.nvar == 5 ? launch_face_class_t<5>(m, p, u, alpha, cls, read_trace, s)
                     : launch_face_class_t<6>(m, p, u, alpha, cls, read_trace, s);
}

template <int NV, bool LIFT>
static hipError_t launch_visc_faces_t(const MeshView& m, const double* u, hipStream_t s) {
  if (m.face_mixed_count == 0) return hipSuccess;
  if constexpr (LIFT)
    hipLaunchKernelGGL((lift_face_mixed_kernel<NV>), dim3(m.face_mixed_count), dim3(FACE_THREADS), 0, s, m, u);
  else
    hipLaunchKernelGGL((visc_face_mixed_kernel<NV>), dim3(m.face_mixed_count), dim3(FACE_THREADS), 0, s, m, u);
  return hipGetLastError();
}

hipError_t launch_lift_faces(const MeshView& m, const double* u, hipStream_t s) {
  return m.nvar == 5 ? launch_visc_faces_t<5, true>(m, u, s) : launch_visc_faces_t<6, true>(m, u, s);
}

hipError_t launch_visc_faces(const MeshView& m, const double* u, hipStream_t s) {
  return m.nvar == 5 ? launch_visc_faces_t<5, false>(m, u, s) : launch_visc_faces_t<6, false>(m, u, s);
}

hipError_t launch_mortars_fv_stored(const MeshView& m, const ParamsDev& p, const double* u, const double* ufv,
                                   const double* fv, hipStream_t s) {
  if (m.n_mortar == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((mortar_fvs_kernel<5>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, p, u, ufv, fv);
  else
    hipLaunchKernelGGL((mortar_fvs_kernel<6>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, p, u, ufv, fv);
  return hipGetLastError();
}

hipError_t launch_mortars_vjp(const MeshView& m, const ParamsDev& p, const double* u, hipStream_t s) {
  if (m.n_mortar == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((mortar_vjp_kernel<5>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, p, u);
  else
    hipLaunchKernelGGL((mortar_vjp_kernel<6>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, p, u);
  return hipGetLastError();
}

hipError_t launch_mortar_lift(const MeshView& m, const double* u, hipStream_t s) {
  if (m.n_mortar == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((mortar_lift_kernel<5>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, u);
  else
    hipLaunchKernelGGL((mortar_lift_kernel<6>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, u);
  return hipGetLastError();
}

hipError_t launch_mortar_visc(const MeshView& m, const double* u, hipStream_t s) {
  if (m.n_mortar == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((mortar_visc_kernel<5>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, u);
  else
    hipLaunchKernelGGL((mortar_visc_kernel<6>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, u);
  return hipGetLastError();
}

hipError_t launch_face_mortars(const MeshView& m, const ParamsDev& p, const double* u, const double* alpha,
                               hipStream_t s) {
  if (m.n_mortar == 0) return hipSuccess;
  if (m.nvar == 5)
    hipLaunchKernelGGL((face_mortar_kernel<5>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, p, u, alpha);
  else
    hipLaunchKernelGGL((face_mortar_kernel<6>), dim3(m.n_mortar), dim3(FACE_THREADS), 0, s, m, p, u, alpha);
  return hipGetLastError();
}

}  // namespace dgfv

