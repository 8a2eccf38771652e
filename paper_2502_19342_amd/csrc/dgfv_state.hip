// Pointwise state kernels: primitive -> conservative variables, and the two
// pointwise halves of the reverse of a 2N Runge-Kutta stage.
//
// prim_to_cons: rho, v, p (and Y1) -> rho, rho v, rho e = p/(kappa - 1) + rho |v|^2 / 2
//   (and rho Y1), with the mixture ratio of the linear mixing rules for two
//   species (Section 2, eq. eos, eq. mix_R_kappa, eq. mix_cp_cv).
// Reverse of stage s (Section 3.3): the forward stage is
//   k_s = A_s k_{s-1} + dt R(u_{s-1}),  u_s = u_{s-1} + B_s k_s,
// so with the cotangents ubar of u_s and kbar of k_s from the later stages
//   kt = kbar + B_s ubar;   ubar <- ubar + dt (dR/du)^T kt;   kbar <- A_s kt.
// rk_adjoint_pre forms kt in place of kbar; rk_adjoint_post takes g = (dR/du)^T kt.
#include <cmath>
#include <mutex>

#include "dgfv_internal.h"

// Fixed device buffer of dg_rk_stage_vjp_noalloc, for callers that cannot
// allocate: each GPU the library runs on holds one copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in, not a device address): it passes the address that
// hipGetSymbolAddress returns for the current device (static_scratch_ptr).
static __device__ __align__(256) double scratch[dgfv::STATIC_SCRATCH_DOUBLES];

namespace dgfv {
namespace {

std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};

constexpr int STATE_THREADS = 256;

template <int NV>
__global__ void __launch_bounds__(STATE_THREADS)
prim_to_cons_kernel(int64_t n, GasDev gas, const double* __restrict__ w, double* __restrict__ u) {
  for (int64_t i = blockIdx.x * (int64_t)STATE_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * STATE_THREADS) {
    const double rho = w[i], v1 = w[n + i], v2 = w[2 * n + i], v3 = w[3 * n + i], p = w[4 * n + i];
    double kappa = gas.gamma;
    if constexpr (NV == 6) {
      const double Y = w[5 * n + i];
      kappa = (Y * gas.cp0 + (1.0 - Y) * gas.cp1) / (Y * gas.cv0 + (1.0 - Y) * gas.cv1);
      u[5 * n + i] = rho * Y;
    }
    u[i] = rho;
    u[n + i] = rho * v1;
    u[2 * n + i] = rho * v2;
    u[3 * n + i] = rho * v3;
    u[4 * n + i] = p / (kappa - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3);
  }
}

__global__ void __launch_bounds__(STATE_THREADS)
rk_adjoint_pre_kernel(int64_t n, double B, const double* __restrict__ ubar, double* __restrict__ kbar) {
  for (int64_t i = blockIdx.x * (int64_t)STATE_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * STATE_THREADS)
    kbar[i] = kbar[i] + B * ubar[i];
}

__global__ void __launch_bounds__(STATE_THREADS)
rk_adjoint_post_kernel(int64_t n, double dt, double A, const double* __restrict__ g, double* __restrict__ ubar,
                       double* __restrict__ kbar) {
  for (int64_t i = blockIdx.x * (int64_t)STATE_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * STATE_THREADS) {
    ubar[i] = ubar[i] + dt * g[i];
    kbar[i] = A == 0.0 ? 0.0 : A * kbar[i];     // stage 1: exact zero, whatever kbar held
  }
}

// p-adaptation (Section 3.2): an element's state from degree Nf to degree Nt by
// the 1D map table[Nf][Nt] ((Nt+1) x (Nf+1), interpolation up, modal
// truncation down, identity otherwise) along each reference direction; one
// element per 512-lane workgroup, the three one-dimensional passes through LDS.
constexpr int TRANSFER_THREADS = 512;
constexpr int TMAX = MAXN + 1;

template <int NV>
__global__ void __launch_bounds__(TRANSFER_THREADS)
transfer_kernel(int K, const double* __restrict__ u_from, const int64_t* __restrict__ off_from,
                const int8_t* __restrict__ deg_from, int64_t n_from, double* __restrict__ u_to,
                const int64_t* __restrict__ off_to, const int8_t* __restrict__ deg_to, int64_t n_to,
                const double* __restrict__ table) {
  __shared__ double a[NV * TMAX * TMAX * TMAX], b[NV * TMAX * TMAX * TMAX];
  __shared__ double A[TMAX * TMAX];
  const int e = blockIdx.x;
  if (e >= K) return;
  const int t = threadIdx.x;
  const int Nf = deg_from[e], Nt = deg_to[e];
  const int ni = Nf + 1, no = Nt + 1;
  const int ni3 = ni * ni * ni;
  if (t < no * ni) A[t] = table[(Nf * TMAX + Nt) * TMAX * TMAX + t];
  const int64_t bf = off_from[e], bt = off_to[e];
  for (int r = t; r < ni3; r += TRANSFER_THREADS)
    for (int v = 0; v < NV; ++v) a[v * ni3 + r] = u_from[v * n_from + bf + r];
  __syncthreads();
  // axis 0: [f][k][j][c] -> [f][k][j][o]
  for (int r = t; r < NV * ni * ni; r += TRANSFER_THREADS)
    for (int o = 0; o < no; ++o) {
      double acc = 0.0;
      for (int c = 0; c < ni; ++c) acc += A[o * ni + c] * a[r * ni + c];
      b[r * no + o] = acc;
    }
  __syncthreads();
  // axis 1: [f][k][c][o0] -> [f][k][o1][o0]
  for (int r = t; r < NV * ni * no; r += TRANSFER_THREADS) {
    const int o0 = r % no, kf = r / no;
    for (int o = 0; o < no; ++o) {
      double acc = 0.0;
      for (int c = 0; c < ni; ++c) acc += A[o * ni + c] * b[(kf * ni + c) * no + o0];
      a[(kf * no + o) * no + o0] = acc;
    }
  }
  __syncthreads();
  // axis 2: [f][c][o1][o0] -> [f][o2][o1][o0], written to the new layout
  const int no2 = no * no;
  for (int r = t; r < NV * no2; r += TRANSFER_THREADS) {
    const int o01 = r % no2, f = r / no2;
    for (int o = 0; o < no; ++o) {
      double acc = 0.0;
      for (int c = 0; c < ni; ++c) acc += A[o * ni + c] * a[(f * ni + c) * no2 + o01];
      u_to[f * n_to + bt + o * no2 + o01] = acc;
    }
  }
}

int grid_for(int64_t n, const MeshView& m) {
  const int64_t want = (n + STATE_THREADS - 1) / STATE_THREADS;
  const int64_t cap = (int64_t)m.n_cu * 32;       // grid-stride beyond this
  return (int)(want < cap ? (want > 0 ? want : 1) : cap);
}

}  // namespace

hipError_t static_scratch_ptr(double** out) {
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return e;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

// Minimum of each half of dt_e (the per-element convective and parabolic time
// steps), one workgroup: a strided pass per lane, then the lanes' minima
// combined with unsigned 64-bit atomics in LDS on the bit patterns (order-
// preserving for non-negative doubles; a NaN outranks every number, and
// comes through as the maximum, never as the minimum: the lanes keep it
// apart so that the host sees it).
constexpr int MIN_THREADS = 1024;
__global__ void __launch_bounds__(MIN_THREADS) min_pairs_kernel(const double* __restrict__ dt_e, int K,
                                                                double* __restrict__ out) {
  __shared__ unsigned long long sMin[2];
  __shared__ int sNan;
  if (threadIdx.x < 2) sMin[threadIdx.x] = ~0ull;
  if (threadIdx.x == 0) sNan = 0;
  __syncthreads();
  for (int h = 0; h < 2; ++h) {
    double best = INFINITY;
    bool nan = false;
    for (int e = threadIdx.x; e < K; e += blockDim.x) {
      const double x = dt_e[(size_t)h * K + e];
      if (x != x) nan = true;
      else best = fmin(best, x);
    }
    if (nan) sNan = 1;
    atomicMin(&sMin[h], (unsigned long long)__double_as_longlong(best));
  }
  __syncthreads();
  if (threadIdx.x < 2)
    out[threadIdx.x] = sNan ? NAN : __longlong_as_double((long long)sMin[threadIdx.x]);
}

hipError_t launch_min_pairs(const double* dt_e, int K, double* out, hipStream_t s) {
  hipLaunchKernelGGL(min_pairs_kernel, dim3(1), dim3(MIN_THREADS), 0, s, dt_e, K, out);
  return hipGetLastError();
}

hipError_t launch_prim_to_cons(const MeshView& m, const double* w, double* u, hipStream_t s) {
  const int64_t n = m.n_node;
  if (m.nvar == 5)
    hipLaunchKernelGGL((prim_to_cons_kernel<5>), dim3(grid_for(n, m)), dim3(STATE_THREADS), 0, s, n, m.gas, w, u);
  else
    hipLaunchKernelGGL((prim_to_cons_kernel<6>), dim3(grid_for(n, m)), dim3(STATE_THREADS), 0, s, n, m.gas, w, u);
  return hipGetLastError();
}

hipError_t launch_transfer(const MeshView& from, const MeshView& to, const double* u_from, double* u_to,
                           const double* table, hipStream_t s) {
  if (from.K == 0) return hipSuccess;
  if (from.nvar == 5)
    hipLaunchKernelGGL(transfer_kernel<5>, dim3(from.K), dim3(TRANSFER_THREADS), 0, s, from.K, u_from,
                       from.elem_offset, from.degree, from.n_node, u_to, to.elem_offset, to.degree, to.n_node, table);
  else
    hipLaunchKernelGGL(transfer_kernel<6>, dim3(from.K), dim3(TRANSFER_THREADS), 0, s, from.K, u_from,
                       from.elem_offset, from.degree, from.n_node, u_to, to.elem_offset, to.degree, to.n_node, table);
  return hipGetLastError();
}

hipError_t launch_rk_adjoint_pre(const MeshView& m, double B, const double* ubar, double* kbar, hipStream_t s) {
  const int64_t n = (int64_t)m.nvar * m.n_node;
  hipLaunchKernelGGL(rk_adjoint_pre_kernel, dim3(grid_for(n, m)), dim3(STATE_THREADS), 0, s, n, B, ubar, kbar);
  return hipGetLastError();
}

hipError_t launch_rk_adjoint_post(const MeshView& m, double dt, double A, const double* g, double* ubar,
                                  double* kbar, hipStream_t s) {
  const int64_t n = (int64_t)m.nvar * m.n_node;
  hipLaunchKernelGGL(rk_adjoint_post_kernel, dim3(grid_for(n, m)), dim3(STATE_THREADS), 0, s, n, dt, A, g, ubar,
                     kbar);
  return hipGetLastError();
}

}  // namespace dgfv
