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

hipError_t launch_prim_to_cons(const MeshView& m, const double* w, double* u, hipStream_t s) {
  const int64_t n = m.n_node;
  if (m.nvar == 5)
    hipLaunchKernelGGL((prim_to_cons_kernel<5>), dim3(grid_for(n, m)), dim3(STATE_THREADS), 0, s, n, m.gas, w, u);
  else
    hipLaunchKernelGGL((prim_to_cons_kernel<6>), dim3(grid_for(n, m)), dim3(STATE_THREADS), 0, s, n, m.gas, w, u);
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
