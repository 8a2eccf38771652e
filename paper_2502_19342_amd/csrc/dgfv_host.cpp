// Host runtime of the hybrid DG/FV right-hand side: mesh setup (operators,
// curl-form metrics, face tables, degree buckets, device buffers) and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dgfv.h"
#include "dgfv_internal.h"
#include "dgfv_ops1d.h"

using namespace dgfv;

namespace {

thread_local std::string g_last_error;

dgfv_status fail(dgfv_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

bool msg_oom(const HipError& e) { return std::string(e.what()).find("out of memory") != std::string::npos; }

template <class T>
T* dev_upload(const std::vector<T>& h) {
  T* d = nullptr;
  if (h.empty()) return nullptr;
  hip_check(hipMalloc(&d, h.size() * sizeof(T)), "hipMalloc");
  hip_check(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return d;
}

template <class T>
T* dev_alloc(size_t n) {
  T* d = nullptr;
  if (n == 0) n = 1;
  hip_check(hipMalloc(&d, n * sizeof(T)), "hipMalloc");
  return d;
}

// Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients.
const double RK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double RK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

template <class F>
void parallel_for(int64_t n, F&& body) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 256) nt = 1;
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &body] {
      for (int64_t i = a; i < b; ++i) body(i);
    });
  }
  for (auto& x : th) x.join();
}

DegreeOps ops_for(int N) {
  switch (N) {
    case 1: return degree_ops_1();
    case 2: return degree_ops_2();
    case 3: return degree_ops_3();
    case 4: return degree_ops_4();
    case 5: return degree_ops_5();
    case 6: return degree_ops_6();
    default: return degree_ops_7();
  }
}

ViscousOps viscous_ops_for(int N) {
  switch (N) {
    case 1: return viscous_ops_1();
    case 2: return viscous_ops_2();
    case 3: return viscous_ops_3();
    case 4: return viscous_ops_4();
    case 5: return viscous_ops_5();
    case 6: return viscous_ops_6();
    default: return viscous_ops_7();
  }
}

}  // namespace

struct dgfv_mesh {
  int K = 0, nvar = 0, n_fv = 0, NJ = 0, F = 0;
  int64_t n_node = 0;
  std::vector<int8_t> degree;
  std::vector<int64_t> offset;
  std::vector<double> coords;            // [3][n_node]
  std::array<std::vector<int32_t>, MAXN + 1> bucket;
  std::array<int32_t*, MAXN + 1> d_bucket{};
  std::vector<void*> allocations;
  MeshView view{};

  // concurrent branches: per-degree launches of one phase fork from the
  // caller's stream onto side streams and join back (graph branches when captured)
  std::array<hipStream_t, FACE_CLASS_COUNT> side{};
  hipEvent_t fork_ev = nullptr;
  std::array<hipEvent_t, FACE_CLASS_COUNT> join_ev{};

  // hipGraph cache of dg_rk_step / dg_rk_stage, keyed on the full argument set
  struct GraphKey {
    int kind, stage, fuse;
    const void *u, *k, *alpha;
    double dt;
    dgfv_params prm;
    bool operator==(const GraphKey& o) const {
      return kind == o.kind && stage == o.stage && fuse == o.fuse && u == o.u && k == o.k && alpha == o.alpha &&
             std::memcmp(&dt, &o.dt, sizeof dt) == 0 && std::memcmp(&prm, &o.prm, sizeof prm) == 0;
    }
  };
  static constexpr size_t GRAPH_CACHE = 16;
  int launch_mode = DGFV_LAUNCH_BRANCHES;
  bool limiter_on = false;                      // positivity limiter after every RK stage
  std::array<int, MAXN + 1> elem_variant{};    // element-kernel tile shape per degree (autotuned)
  hipStream_t cap_stream = nullptr;
  mutable std::vector<std::pair<GraphKey, hipGraphExec_t>> graph_cache;

  // non-physical state: the element kernels set view.state_flag; each RHS or RK
  // call copies it to pinned host memory behind an event, and a later call
  // reports it once that copy has landed (mutable: bookkeeping only)
  int32_t* flag_host = nullptr;
  hipEvent_t flag_ev = nullptr;
  mutable bool flag_pending = false;

  // state-sized buffer of dg_rk_stage_vjp, allocated by its first call
  mutable double* stage_g = nullptr;

  // fused face fluxes (element kernels of degree >= FUSE_MIN_N evaluate the
  // conforming DG faces themselves), off unless asked for; the RK stages of one
  // dg_rk_step then alternate between u and u_alt (state-sized, allocated by
  // the first such call), so that no launch writes the state it reads
  bool fuse_faces = false;
  mutable double* u_alt = nullptr;

  // FV-stored elements: ghost layers [K][6][nvar][N_FV^2] and V3(J) [K][N_FV^3],
  // made by the first call that has FV-stored elements
  mutable double* fvghost = nullptr;
  mutable double* fvjbar = nullptr;

  // p-adaptation: the maps between degrees (made by the first transfer into this
  // mesh) and the indicator values of the degree decision
  mutable double* pmap = nullptr;
  mutable double* pind = nullptr;

  // viscous terms: on once transport coefficients are set; the lifted gradient,
  // the face values / viscous face fluxes per side and the viscous rate live
  // in view.grad, view.vside and rvisc
  bool viscous = false;
  double* rvisc = nullptr;
  int n_mortar = 0;                             // non-conforming faces
  bool mortar_jump = false;                     // a mortar whose sides differ in degree
  size_t side_total = 0;                        // doubles of one side buffer (fside, vside)

  // dg_timestep: per-element steps [2][K] and the two minima (made by its first call)
  mutable double* dt_buf = nullptr;

  // kernel timing (mutable: recording does not change the mesh)
  mutable bool profile = false;
  mutable std::array<std::vector<std::pair<hipEvent_t, hipEvent_t>>, DGFV_KERNEL_COUNT> ev;
  mutable std::array<size_t, DGFV_KERNEL_COUNT> ev_used{};

  void drop_graphs() const {
    for (auto& pr : graph_cache) (void)hipGraphExecDestroy(pr.second);
    graph_cache.clear();
  }
  ~dgfv_mesh() {
    drop_graphs();
    for (hipStream_t st : side)
      if (st) (void)hipStreamDestroy(st);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (flag_ev) (void)hipEventDestroy(flag_ev);
    if (flag_host) (void)hipHostFree(flag_host);
    for (hipEvent_t e : join_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& list : ev)
      for (auto& pr : list) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
    for (void* p : allocations) (void)hipFree(p);
    if (stage_g) (void)hipFree(stage_g);
    if (u_alt) (void)hipFree(u_alt);
    if (fvghost) (void)hipFree(fvghost);
    if (fvjbar) (void)hipFree(fvjbar);
    if (pmap) (void)hipFree(pmap);
    if (pind) (void)hipFree(pind);
    if (view.grad) (void)hipFree(view.grad);
    if (view.vside) (void)hipFree(view.vside);
    if (rvisc) (void)hipFree(rvisc);
    if (dt_buf) (void)hipFree(dt_buf);
  }
  template <class T>
  T* keep(T* p) {
    allocations.push_back((void*)p);
    return p;
  }
};

namespace {

// Trilinear map and its Jacobian at reference point (x1, x2, x3).
void trilinear(const double* c, double x1, double x2, double x3, double X[3], double G[3][3]) {
  const double ph[2][3] = {{0.5 * (1 - x1), 0.5 * (1 - x2), 0.5 * (1 - x3)},
                           {0.5 * (1 + x1), 0.5 * (1 + x2), 0.5 * (1 + x3)}};
  const double dph[2] = {-0.5, 0.5};
  for (int n = 0; n < 3; ++n) {
    X[n] = 0;
    for (int a = 0; a < 3; ++a) G[n][a] = 0;
  }
  for (int k = 0; k < 8; ++k) {
    const int b0 = k & 1, b1 = (k >> 1) & 1, b2 = (k >> 2) & 1;
    const double w = ph[b0][0] * ph[b1][1] * ph[b2][2];
    const double g0 = dph[b0] * ph[b1][1] * ph[b2][2];
    const double g1 = ph[b0][0] * dph[b1] * ph[b2][2];
    const double g2 = ph[b0][0] * ph[b1][1] * dph[b2];
    for (int n = 0; n < 3; ++n) {
      const double cn = c[3 * k + n];
      X[n] += cn * w;
      G[n][0] += cn * g0;
      G[n][1] += cn * g1;
      G[n][2] += cn * g2;
    }
  }
}

// Derivative along reference axis `a` of a nodal field f[(k*n + j)*n + i] on n^3 nodes.
void dxi(const std::vector<double>& D, int n, const double* f, double* out, int a) {
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int m = 0; m < n; ++m) {
          int idx;
          if (a == 0) idx = (k * n + j) * n + m;
          else if (a == 1) idx = (k * n + m) * n + i;
          else idx = (m * n + j) * n + i;
          s += D[(a == 0 ? i : (a == 1 ? j : k)) * n + m] * f[idx];
        }
        out[(k * n + j) * n + i] = s;
      }
}

// Conservative curl-form metrics Ja^d_n of one element at the degree-NJ LGL nodes:
// Ja^d_n = -(curl_xi (X_l grad_xi X_m))_d with (n, m, l) cyclic.  Output [9][nJ^3].
void curl_metrics(const double* corners, int NJ, const std::vector<double>& xJ,
                  const std::vector<double>& DJ, std::vector<double>& out) {
  const int n = NJ + 1, n3 = n * n * n;
  std::vector<double> X(3 * n3);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double x[3], G[3][3];
        trilinear(corners, xJ[i], xJ[j], xJ[k], x, G);
        for (int c = 0; c < 3; ++c) X[c * n3 + (k * n + j) * n + i] = x[c];
      }
  std::vector<double> dX(3 * n3), W(3 * n3), dW(n3), tmp(n3);
  out.assign(9 * n3, 0.0);
  for (int nn = 0; nn < 3; ++nn) {
    const int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
    for (int a = 0; a < 3; ++a) {
      dxi(DJ, n, &X[mm * n3], tmp.data(), a);
      for (int t = 0; t < n3; ++t) W[a * n3 + t] = X[ll * n3 + t] * tmp[t];
    }
    // curl components
    for (int d = 0; d < 3; ++d) {
      const int b = (d + 1) % 3, c = (d + 2) % 3;   // (curl W)_d = d_b W_c - d_c W_b
      dxi(DJ, n, &W[c * n3], dW.data(), b);
      dxi(DJ, n, &W[b * n3], tmp.data(), c);
      for (int t = 0; t < n3; ++t) out[(3 * d + nn) * n3 + t] = -(dW[t] - tmp[t]);
    }
  }
}

int side_node_h(int s, int p, int q, int n);

// Per-element metrics whose face normals match the neighbours' (metric_degree 0).
// The curl form Ja^d_n = -(curl_xi W)_d, W = X_l grad_xi X_m, is taken at the
// element degree N.  A face shared with a neighbour of lower degree Nf gets, in
// place of W's two tangential components at its nodes, their degree-Nf
// interpolant (through W's exact values at the Nf face points), so the face
// normal (the tangential curl of W on the face) is the neighbour's polynomial.
// On trilinear elements W's component along an edge is linear along it, so
// two faces never disagree on a shared edge.  Long double throughout, rounded
// once, so that the two sides of a face hold the same normal to rounding.
void trilinear_ld(const double* c, long double x1, long double x2, long double x3, long double X[3],
                  long double G[3][3]) {
  using LD = long double;
  const LD ph[2][3] = {{0.5L * (1 - x1), 0.5L * (1 - x2), 0.5L * (1 - x3)},
                       {0.5L * (1 + x1), 0.5L * (1 + x2), 0.5L * (1 + x3)}};
  const LD dph[2] = {-0.5L, 0.5L};
  for (int n = 0; n < 3; ++n) {
    X[n] = 0;
    for (int a = 0; a < 3; ++a) G[n][a] = 0;
  }
  for (int k = 0; k < 8; ++k) {
    const int b0 = k & 1, b1 = (k >> 1) & 1, b2 = (k >> 2) & 1;
    const LD w = ph[b0][0] * ph[b1][1] * ph[b2][2];
    const LD g0 = dph[b0] * ph[b1][1] * ph[b2][2];
    const LD g1 = ph[b0][0] * dph[b1] * ph[b2][2];
    const LD g2 = ph[b0][0] * ph[b1][1] * dph[b2];
    for (int n = 0; n < 3; ++n) {
      const LD cn = c[3 * k + n];
      X[n] += cn * w;
      G[n][0] += cn * g0;
      G[n][1] += cn * g1;
      G[n][2] += cn * g2;
    }
  }
}

void dxi_ld(const std::vector<long double>& D, int n, const long double* f, long double* out, int a) {
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        long double s = 0.0L;
        const int r = a == 0 ? i : (a == 1 ? j : k);
        for (int m = 0; m < n; ++m) {
          const int idx = a == 0 ? (k * n + j) * n + m : (a == 1 ? (k * n + m) * n + i : (m * n + j) * n + i);
          s += D[r * n + m] * f[idx];
        }
        out[(k * n + j) * n + i] = s;
      }
}

// out: [9][(N+1)^3], component 3d + n; nbr[s]: degree across side s.
void matched_metrics(const double* corners, int N, const int nbr[6], double* out) {
  using LD = long double;
  const int n = N + 1, n3 = n * n * n;
  const std::vector<LD> x = lgl_nodes(N), D = ld_D(N);
  std::vector<LD> X(3 * n3), G(9 * n3);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        LD Xp[3], Gp[3][3];
        trilinear_ld(corners, x[i], x[j], x[k], Xp, Gp);
        for (int c = 0; c < 3; ++c) X[c * n3 + (k * n + j) * n + i] = Xp[c];
      }
  std::vector<LD> W(3 * n3), tmp(n3), dA(n3), dB(n3);
  for (int nn = 0; nn < 3; ++nn) {
    const int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
    for (int a = 0; a < 3; ++a) {
      dxi_ld(D, n, &X[mm * n3], tmp.data(), a);
      for (int t = 0; t < n3; ++t) W[a * n3 + t] = X[ll * n3 + t] * tmp[t];
    }
    for (int s = 0; s < 6; ++s) {
      const int Nf = nbr[s];
      if (Nf >= N) continue;
      const int d = s / 2, nf = Nf + 1;
      const LD endv = (s & 1) ? 1.0L : -1.0L;
      const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;   // face grid: p along ta, q along tb
      const std::vector<LD> xf = lgl_nodes(Nf), V = ld_interp(Nf, N);
      for (int a = 0; a < 3; ++a) {
        if (a == d) continue;
        std::vector<LD> Wf(nf * nf), mid(nf * n);
        for (int qf = 0; qf < nf; ++qf)
          for (int pf = 0; pf < nf; ++pf) {
            LD r[3];
            r[d] = endv;
            r[ta] = xf[pf];
            r[tb] = xf[qf];
            LD Xp[3], Gp[3][3];
            trilinear_ld(corners, r[0], r[1], r[2], Xp, Gp);
            Wf[qf * nf + pf] = Xp[ll] * Gp[mm][a];
          }
        for (int qf = 0; qf < nf; ++qf)          // interpolate along p
          for (int p = 0; p < n; ++p) {
            LD acc = 0.0L;
            for (int pf = 0; pf < nf; ++pf) acc += V[p * nf + pf] * Wf[qf * nf + pf];
            mid[qf * n + p] = acc;
          }
        for (int q = 0; q < n; ++q)              // then along q, into W's face nodes
          for (int p = 0; p < n; ++p) {
            LD acc = 0.0L;
            for (int qf = 0; qf < nf; ++qf) acc += V[q * nf + qf] * mid[qf * n + p];
            W[a * n3 + side_node_h(s, p, q, n)] = acc;
          }
      }
    }
    for (int d = 0; d < 3; ++d) {
      const int b = (d + 1) % 3, c = (d + 2) % 3;  // (curl W)_d = d_b W_c - d_c W_b
      dxi_ld(D, n, &W[c * n3], dA.data(), b);
      dxi_ld(D, n, &W[b * n3], dB.data(), c);
      for (int t = 0; t < n3; ++t) out[(3 * d + nn) * n3 + t] = (double)(-(dA[t] - dB[t]));
    }
  }
}

// Tensor interpolation of nodal fields [nf][nin^3] to [nf][nout^3] with the 1D matrix V (nout x nin).
void interp3(const std::vector<double>& V, int nin, int nout, const double* src, double* dst, int nf) {
  std::vector<double> a(nin * nin * nout), b(nin * nout * nout);
  for (int f = 0; f < nf; ++f) {
    const double* s = src + (size_t)f * nin * nin * nin;
    double* o = dst + (size_t)f * nout * nout * nout;
    for (int k = 0; k < nin; ++k)
      for (int j = 0; j < nin; ++j)
        for (int i = 0; i < nout; ++i) {
          double acc = 0;
          for (int c = 0; c < nin; ++c) acc += V[i * nin + c] * s[(k * nin + j) * nin + c];
          a[(k * nin + j) * nout + i] = acc;
        }
    for (int k = 0; k < nin; ++k)
      for (int j = 0; j < nout; ++j)
        for (int i = 0; i < nout; ++i) {
          double acc = 0;
          for (int c = 0; c < nin; ++c) acc += V[j * nin + c] * a[(k * nin + c) * nout + i];
          b[(k * nout + j) * nout + i] = acc;
        }
    for (int k = 0; k < nout; ++k)
      for (int j = 0; j < nout; ++j)
        for (int i = 0; i < nout; ++i) {
          double acc = 0;
          for (int c = 0; c < nin; ++c) acc += V[k * nin + c] * b[(c * nout + j) * nout + i];
          o[(k * nout + j) * nout + i] = acc;
        }
  }
}

// r x c row-major -> c x r row-major
std::vector<double> transpose(const std::vector<double>& a, int r, int c) {
  std::vector<double> t((size_t)r * c);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < c; ++j) t[(size_t)j * r + i] = a[(size_t)i * c + j];
  return t;
}

int side_node_h(int s, int p, int q, int n) {
  const int last = (s & 1) ? n - 1 : 0;
  switch (s >> 1) {
    case 0: return (q * n + p) * n + last;
    case 1: return (q * n + last) * n + p;
    default: return (last * n + q) * n + p;
  }
}

dgfv_status check_params(const dgfv_mesh* m, const dgfv_params* p) {
  if (!p) return fail(DGFV_ERR_ARG, "params is NULL");
  if (p->volume_flux < 0 || p->volume_flux > 2) return fail(DGFV_ERR_ARG, "volume_flux out of range");
  if (p->face_flux_dg < 0 || p->face_flux_dg > 2 || p->face_flux_fv < 0 || p->face_flux_fv > 2)
    return fail(DGFV_ERR_ARG, "face flux selector out of range");
  if (m->nvar == 6 && p->volume_flux == DGFV_VOL_RANOCHA)
    return fail(DGFV_ERR_UNSUPPORTED, "the entropy-conserving volume flux is single-species only");
  if (m->nvar == 6 && (p->face_flux_dg == DGFV_RIEMANN_ROE_HH || p->face_flux_fv == DGFV_RIEMANN_ROE_HH))
    return fail(DGFV_ERR_UNSUPPORTED, "the Roe solver is single-species only");
  return DGFV_OK;
}

// Records an event pair around one launch when profiling is on.
struct Timed {
  const dgfv_mesh* m;
  int kind;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  Timed(const dgfv_mesh* mesh, int k, hipStream_t st) : m(mesh), kind(k), s(st) {
    if (!m->profile || k < 0) return;             // k < 0: not timed
    auto& list = m->ev[kind];
    size_t& used = m->ev_used[kind];
    if (used == list.size()) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "hipEventCreate");
      hip_check(hipEventCreate(&b), "hipEventCreate");
      list.emplace_back(a, b);
    }
    hip_check(hipEventRecord(list[used].first, s), "hipEventRecord");
    stop = list[used].second;
    ++used;
  }
  ~Timed() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

ParamsDev to_dev(const dgfv_params* p) {
  ParamsDev d;
  d.volume_flux = p->volume_flux;
  d.face_flux_dg = p->face_flux_dg;
  d.face_flux_fv = p->face_flux_fv;
  d.ind_vars = p->ind_vars;
  d.ind_T = p->ind_T;
  d.ind_dT = p->ind_dT;
  return d;
}

// Runs launch(item, stream) for every item in `items`; with more than one, as
// parallel branches on the mesh's side streams that fork from and join back
// into s (parallel graph branches when s is being captured).
template <class F>
void fork_join(const dgfv_mesh* m, hipStream_t s, const std::vector<int>& items, F&& launch) {
  if (items.size() <= 1 || m->launch_mode == DGFV_LAUNCH_SERIAL) {
    for (int it : items) launch(it, s);
    return;
  }
  hip_check(hipEventRecord(m->fork_ev, s), "hipEventRecord");
  for (size_t b = 0; b < items.size(); ++b) {
    hipStream_t ss = m->side[b];
    hip_check(hipStreamWaitEvent(ss, m->fork_ev, 0), "hipStreamWaitEvent");
    launch(items[b], ss);
    hip_check(hipEventRecord(m->join_ev[b], ss), "hipEventRecord");
  }
  for (size_t b = 0; b < items.size(); ++b)
    hip_check(hipStreamWaitEvent(s, m->join_ev[b], 0), "hipStreamWaitEvent");
}

std::vector<int> degrees_present(const dgfv_mesh* m) {
  std::vector<int> d;
  for (int N = 1; N <= MAXN; ++N)
    if (!m->bucket[N].empty()) d.push_back(N);
  return d;
}

// Positivity limiter on u (one species): with alpha, the sub-cell means of the
// blended elements of the current u first (the blended list must be current).
void enqueue_limiter(const dgfv_mesh* m, double* u, const double* alpha, double* theta, hipStream_t s,
                     bool build_list) {
  const MeshView& v = m->view;
  if (alpha) {
    if (build_list) hip_check(launch_blend_list(v, alpha, s), "blended list launch");
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).fv_means(v, (int)m->bucket[N].size(), 1, u, s), "fv_means launch");
  }
  for (int N = 1; N <= MAXN; ++N)
    if (!m->bucket[N].empty())
      hip_check(ops_for(N).limiter(v, m->d_bucket[N], (int)m->bucket[N].size(), u, alpha, theta, s),
                "limiter launch");
}

// Enqueue one evaluation: stage 0 -> ut = R(u); stage 1..5 -> RK stage on (u, k).
// Phases: blended list + sub-cell means, face fluxes, FV residuals, element
// kernels (volume, lift, blend, RK update); the per-degree (per face class)
// launches of a phase are independent branches.
// trace_in: the conforming faces read sides 0 and 1 from m->view.trace, which
// the previous stage of the same step wrote (trace_out) from the state it left
// in u; only dg_rk_step sets them, as within one call nothing else writes u.
// uout: where a stage puts the new state (u itself for an in-place stage).
// fuse: the element kernels of degree >= FUSE_MIN_N evaluate their conforming
// DG faces themselves (stage 0, or uout != u), and those face classes are not
// launched.
// Viscous rate of u into m->rvisc (Section 3.1.1, Section 3.2.2): the BR1 face
// values, the lifted gradient, the viscous face fluxes, the volume terms.
void enqueue_viscous(const dgfv_mesh* m, const double* u, hipStream_t s, bool trace_in) {
  const MeshView& v = m->view;
  const std::vector<int> degs = degrees_present(m);
  Timed t(m, DGFV_KERNEL_VISCOUS, s);
  hip_check(launch_lift_faces(v, u, s), "lift face launch");
  hip_check(launch_mortar_lift(v, u, s), "mortar lift launch");
  fork_join(m, s, degs, [&](int N, hipStream_t ss) {
    hip_check(viscous_ops_for(N).lift(v, m->d_bucket[N], (int)m->bucket[N].size(), u, trace_in, ss),
              "lift launch");
  });
  hip_check(launch_visc_faces(v, u, s), "viscous face launch");
  hip_check(launch_mortar_visc(v, u, s), "mortar viscous launch");
  fork_join(m, s, degs, [&](int N, hipStream_t ss) {
    hip_check(viscous_ops_for(N).volume(v, m->d_bucket[N], (int)m->bucket[N].size(), u, m->rvisc, ss),
              "viscous volume launch");
  });
}

void enqueue_rhs_impl(const dgfv_mesh* m, const ParamsDev& p, const double* u, double* uout,
                      const double* alpha, double* ut, double* k, int stage, double dt, hipStream_t s,
                      bool trace_in = false, bool trace_out = false, bool fuse = false) {
  const MeshView& v = m->view;
  const double A = stage > 0 ? RK_A[stage - 1] : 0.0;
  const double B = stage > 0 ? RK_B[stage - 1] : 0.0;
  const std::vector<int> degs = degrees_present(m);
  if (m->viscous) enqueue_viscous(m, u, s, trace_in);
  // The face phase as concurrent branches, one per DG face class (conforming
  // per degree, degree jumps), which read neither the sub-cell means nor the
  // blended-element list (they test alpha per face) and write only sides of
  // DG/DG faces.  The FV work is either one more branch, in order: the list,
  // the means, the FV faces, the FV residual (which needs only the FV faces'
  // sub-face fluxes); or the list and the means come first, the FV faces (and
  // the mortars, whose blended sides read the means) are branches of the face
  // phase, and the FV residual follows the join, each per-degree step as
  // concurrent branches.  The second form serves meshes with mortars, and
  // graph replays of meshes with several degrees, where the per-degree means
  // and residuals would otherwise run one after another (measured on the
  // mixed-degree workload: 4.20e9 against 4.38e9 DOF-updates/s).
  std::vector<int> classes;
  for (int c = 1; c < FACE_CLASS_COUNT; ++c)
    if (c != FACE_CLASS_FV && face_class_present(v, alpha, c) && !(fuse && c >= FUSE_MIN_N && c <= MAXN))
      classes.push_back(c);
  constexpr int FV_BRANCH = FACE_CLASS_FV, MORTARS = FACE_CLASS_COUNT;
  static_assert(FACE_CLASS_COUNT >= MAXN + 3, "a side stream for every DG face class, the FV work and the mortars");
  const bool mortars = m->n_mortar > 0;
  const bool chain = alpha && !mortars && (m->launch_mode != DGFV_LAUNCH_GRAPH || degs.size() == 1);
  auto fv_faces = [&](hipStream_t ss) {
    if (!face_class_present(v, alpha, FACE_CLASS_FV)) return;
    Timed tf(m, DGFV_KERNEL_FV_FACE, ss);
    hip_check(launch_face_class(v, p, u, alpha, FACE_CLASS_FV, trace_in, ss), "face launch");
  };
  if (alpha && !chain) {
    Timed tm(m, DGFV_KERNEL_FV_MEANS, s);
    hip_check(launch_blend_list(v, alpha, s), "blended list launch");
    const int share = m->launch_mode == DGFV_LAUNCH_SERIAL ? 1 : (int)degs.size();
    fork_join(m, s, degs, [&](int N, hipStream_t ss) {
      hip_check(ops_for(N).fv_means(v, (int)m->bucket[N].size(), share, u, ss), "fv_means launch");
    });
  }
  {
    Timed t(m, DGFV_KERNEL_FACE, s);
    if (alpha) classes.push_back(FV_BRANCH);
    if (mortars) classes.push_back(MORTARS);
    fork_join(m, s, classes, [&](int c, hipStream_t ss) {
      if (c == MORTARS) {
        hip_check(launch_face_mortars(v, p, u, alpha, ss), "mortar launch");
      } else if (c != FV_BRANCH) {
        hip_check(launch_face_class(v, p, u, alpha, c, trace_in, ss), "face launch");
      } else if (!chain) {
        fv_faces(ss);
      } else {
        {
          Timed tm(m, DGFV_KERNEL_FV_MEANS, ss);
          hip_check(launch_blend_list(v, alpha, ss), "blended list launch");
          for (int N : degs)
            hip_check(ops_for(N).fv_means(v, (int)m->bucket[N].size(), 1, u, ss), "fv_means launch");
        }
        fv_faces(ss);
        Timed tr(m, DGFV_KERNEL_FV_RESIDUAL, ss);
        for (int N : degs)
          hip_check(ops_for(N).fv_residual(v, p, (int)m->bucket[N].size(), ss), "fv_residual launch");
      }
    });
  }
  if (alpha && !chain) {
    Timed t(m, DGFV_KERNEL_FV_RESIDUAL, s);
    fork_join(m, s, degs, [&](int N, hipStream_t ss) {
      hip_check(ops_for(N).fv_residual(v, p, (int)m->bucket[N].size(), ss), "fv_residual launch");
    });
  }
  {
    Timed t(m, DGFV_KERNEL_ELEMENT, s);
    MeshView ve = v;
    if (m->viscous) ve.rvisc = m->rvisc;
    fork_join(m, s, degs, [&](int N, hipStream_t ss) {
      const int flags = (trace_out ? ELEM_WRITE_TRACE : 0) | (fuse && N >= FUSE_MIN_N ? ELEM_FUSE_FACES : 0);
      hip_check(ops_for(N).element(ve, p, m->d_bucket[N], (int)m->bucket[N].size(), u, uout, alpha, ut, k,
                                   stage, dt, A, B, m->elem_variant[N], flags, ss),
                "element launch");
    });
  }
  if (stage > 0 && m->limiter_on) enqueue_limiter(m, uout, alpha, nullptr, s, false);
}

// The mesh view with the FV-stored elements' buffers.
MeshView fvs_view(const dgfv_mesh* m) {
  MeshView v = m->view;
  v.fvghost = m->fvghost;
  v.fvjbar = m->fvjbar;
  return v;
}

// The FV-stored elements' buffers and V3(J), once (enqueued on s).
void ensure_fv_stored(const dgfv_mesh* m, hipStream_t s) {
  if (m->fvghost) return;
  const size_t nf = (size_t)m->n_fv;
  double* g = dev_alloc<double>((size_t)m->K * 6 * m->nvar * nf * nf);
  double* j = nullptr;
  try {
    j = dev_alloc<double>((size_t)m->K * nf * nf * nf);
  } catch (...) {
    (void)hipFree(g);
    throw;
  }
  m->fvghost = g;
  m->fvjbar = j;
  const MeshView v = fvs_view(m);
  for (int N = 1; N <= MAXN; ++N)
    if (!m->bucket[N].empty())
      hip_check(ops_for(N).fv_jbar(v, m->d_bucket[N], (int)m->bucket[N].size(), s), "fv_jbar launch");
}

// One evaluation with FV-stored elements (fv[e] > 0): stage 0 -> ut = R(u) on
// DG elements and utfv = R(ufv) on FV elements; stage 1..5 -> the RK stage on
// (u, k) and (ufv, kfv).  Phases: the FV-element list; the DG faces (both
// sides DG) beside the faces with an FV side and the mortars; the FV
// elements' rates; the DG element kernels, which leave the FV elements alone.
// trace_in / trace_out as in enqueue_rhs_impl (dg_rk_step_fv between its stages).
void enqueue_rhs_fvs(const dgfv_mesh* m, const ParamsDev& p, double* u, double* ufv, const double* fv, double* ut,
                     double* utfv, double* k, double* kfv, int stage, double dt, hipStream_t s,
                     bool trace_in = false, bool trace_out = false) {
  ensure_fv_stored(m, s);
  const MeshView v = fvs_view(m);
  const double A = stage > 0 ? RK_A[stage - 1] : 0.0;
  const double B = stage > 0 ? RK_B[stage - 1] : 0.0;
  const std::vector<int> degs = degrees_present(m);
  hip_check(launch_blend_list(v, fv, s), "FV element list launch");
  {
    Timed t(m, DGFV_KERNEL_FACE, s);
    std::vector<int> classes;
    for (int c = 1; c < FACE_CLASS_COUNT; ++c)
      if (c != FACE_CLASS_FV && face_class_present(v, fv, c)) classes.push_back(c);
    classes.push_back(FACE_CLASS_FV);
    // the FV-stored faces and the mortars are one branch beside the DG face
    // classes; the FV elements' rates follow the join (as one more step of that
    // branch they measured no faster: 1.050e10 against 1.051e10 DOF-updates/s)
    fork_join(m, s, classes, [&](int c, hipStream_t ss) {
      if (c != FACE_CLASS_FV) {
        hip_check(launch_face_class(v, p, u, fv, c, trace_in, ss), "face launch");
        return;
      }
      Timed tf(m, DGFV_KERNEL_FV_FACE, ss);
      hip_check(launch_face_fv_stored(v, p, u, ufv, fv, ss), "FV-stored face launch");
      hip_check(launch_mortars_fv_stored(v, p, u, ufv, fv, ss), "FV-stored mortar launch");
    });
  }
  {
    Timed t(m, DGFV_KERNEL_FV_RESIDUAL, s);
    hip_check(launch_fv_stored(v, p, ufv, kfv, utfv, stage, dt, A, B, s), "FV-stored element launch");
  }
  {
    Timed t(m, DGFV_KERNEL_ELEMENT, s);
    fork_join(m, s, degs, [&](int N, hipStream_t ss) {
      const int flags = ELEM_SKIP_FV | (trace_out ? ELEM_WRITE_TRACE : 0);
      hip_check(ops_for(N).element(v, p, m->d_bucket[N], (int)m->bucket[N].size(), u, u, fv, ut, k, stage, dt,
                                   A, B, m->elem_variant[N], flags, ss),
                "element launch");
    });
  }
}

bool has_fused_degree(const dgfv_mesh* m) {
  for (int N = FUSE_MIN_N; N <= MAXN; ++N)
    if (!m->bucket[N].empty()) return true;
  return false;
}

// Stages first..last, each reading one state buffer and writing another where
// faces are fused: the stages alternate between u and m->u_alt, and the last
// one, whose result must be in u, runs in place without fusion when its input
// is u.  Traces go from a stage to a following in-place stage.
void enqueue_stages(const dgfv_mesh* m, const ParamsDev& p, int first, int last, double dt, double* u, double* k,
                    const double* alpha, hipStream_t s, bool fuse) {
  const bool tr = !m->limiter_on;              // the limiter changes u after the traces are written
  double* cur = u;
  for (int st = first; st <= last; ++st) {
    double* out = u;
    bool fused = false;
    if (fuse) {
      if (st < last) {
        out = cur == u ? m->u_alt : u;
        fused = true;
      } else if (cur != u) {
        fused = true;                          // from u_alt back into u
      }
    }
    const bool next_in_place = st < last && !(fuse && (st + 1 < last || out != u));
    const bool prev_wrote = st > first && !fused && (!fuse || cur == u);
    enqueue_rhs_impl(m, p, cur, out, alpha, nullptr, k, st, dt, s, tr && prev_wrote, tr && next_in_place, fused);
    cur = out;
  }
}

// Whether stages first..last of a call on stream s alternate state buffers;
// allocates the second buffer when needed (never while s is captured).
bool use_fused_stages(const dgfv_mesh* m, int first, int last, hipStream_t s);

dgfv_status enqueue_rhs(const dgfv_mesh* m, const dgfv_params* prm, const double* u,
                        const double* alpha, double* ut, double* k, int stage, double dt,
                        hipStream_t s) {
  try {
    const bool fuse = stage == 0 && m->fuse_faces && !m->viscous && has_fused_degree(m);
    enqueue_rhs_impl(m, to_dev(prm), u, const_cast<double*>(u), alpha, ut, k, stage, dt, s, false, false, fuse);
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

// Stages first..last of an RK step, replayed from a cached hipGraph when the
// mesh has graphs on (and profiling off), else enqueued directly.
dgfv_status run_stages(const dgfv_mesh* m, const dgfv_params* prm, int kind, int first, int last, double dt,
                       double* u, double* k, const double* alpha, hipStream_t s) {
  try {
    const bool fuse = use_fused_stages(m, first, last, s);
    if (m->launch_mode != DGFV_LAUNCH_GRAPH || m->profile) {
      enqueue_stages(m, to_dev(prm), first, last, dt, u, k, alpha, s, fuse);
      return DGFV_OK;
    }
    dgfv_mesh::GraphKey key;
    std::memset(&key, 0, sizeof key);             // padding too: the key is compared bytewise in part
    key.kind = kind;
    key.stage = first;
    key.fuse = fuse;
    key.u = u;
    key.k = k;
    key.alpha = alpha;
    key.dt = dt;
    key.prm.volume_flux = prm->volume_flux;
    key.prm.face_flux_dg = prm->face_flux_dg;
    key.prm.face_flux_fv = prm->face_flux_fv;
    key.prm.ind_vars = prm->ind_vars;
    key.prm.ind_T = prm->ind_T;
    key.prm.ind_dT = prm->ind_dT;
    hipGraphExec_t exec = nullptr;
    for (auto& pr : m->graph_cache)
      if (pr.first == key) exec = pr.second;
    if (!exec) {
      const ParamsDev p = to_dev(prm);
      hipGraph_t graph = nullptr;
      hip_check(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      try {
        enqueue_stages(m, p, first, last, dt, u, k, alpha, m->cap_stream, fuse);
      } catch (...) {
        (void)hipStreamEndCapture(m->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      hip_check(hipStreamEndCapture(m->cap_stream, &graph), "hipStreamEndCapture");
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      hip_check(ie, "hipGraphInstantiate");
      if (m->graph_cache.size() >= dgfv_mesh::GRAPH_CACHE) {
        (void)hipGraphExecDestroy(m->graph_cache.front().second);
        m->graph_cache.erase(m->graph_cache.begin());
      }
      m->graph_cache.emplace_back(key, exec);
    }
    hip_check(hipGraphLaunch(exec, s), "hipGraphLaunch");
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

bool use_fused_stages(const dgfv_mesh* m, int first, int last, hipStream_t s) {
  if (!m->fuse_faces || m->viscous || last <= first || !has_fused_degree(m)) return false;
  if (!m->u_alt) {
    if (capturing(s)) return false;
    double* p = nullptr;
    if (hipMalloc((void**)&p, sizeof(double) * (size_t)m->nvar * (size_t)m->n_node) != hipSuccess) {
      (void)hipGetLastError();                // out of memory: the stages run in place
      return false;
    }
    m->u_alt = p;
  }
  return true;
}

// A non-physical state seen by an earlier call whose flag copy has landed:
// DGFV_ERR_STATE, reported once (the flag is cleared).  Never blocks; a copy
// still in flight is looked at by a later call.
dgfv_status state_seen(const dgfv_mesh* m, hipStream_t s) {
  if (!m->flag_pending || capturing(s)) return DGFV_OK;
  if (hipEventQuery(m->flag_ev) != hipSuccess) return DGFV_OK;
  m->flag_pending = false;
  if (*m->flag_host == 0) return DGFV_OK;
  *m->flag_host = 0;
  if (hipMemsetAsync(m->view.state_flag, 0, sizeof(int32_t), s) != hipSuccess)
    return fail(DGFV_ERR_HIP, "hipMemsetAsync of the state flag");
  return fail(DGFV_ERR_STATE, "an earlier call read a state with rho <= 0, p <= 0 or NaN");
}

// After a call: copy the flag to pinned host memory behind an event (not
// while the caller captures the stream; dgfv_check_state covers that case).
dgfv_status state_post(const dgfv_mesh* m, hipStream_t s) {
  if (capturing(s)) return DGFV_OK;
  if (hipMemcpyAsync(m->flag_host, m->view.state_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipEventRecord(m->flag_ev, s) != hipSuccess)
    return fail(DGFV_ERR_HIP, "copy of the state flag");
  m->flag_pending = true;
  return DGFV_OK;
}

// state check, the call, then the flag copy
template <class F>
dgfv_status guarded(const dgfv_mesh* m, hipStream_t s, F&& call) {
  if (dgfv_status st = state_seen(m, s)) return st;
  if (dgfv_status st = call()) return st;
  return state_post(m, s);
}

// Which adjoint paths run (see dg_rhs_vjp).
dgfv_status vjp_paths_enabled(const dgfv_mesh* m, const double* alpha) {
  if (m->viscous) return fail(DGFV_ERR_UNSUPPORTED, "dg_rhs_vjp: the adjoint of the viscous terms is not built");
  if (m->n_mortar > 0 && (alpha || m->mortar_jump))
    return fail(DGFV_ERR_UNSUPPORTED,
                "dg_rhs_vjp: on meshes with mortars only pure DG (alpha = NULL) without degree jumps across a mortar");
#ifndef DGFV_CPU_ADJOINT_ALL_PATHS
  // The adjoint of FV-blended elements and of degree-jump faces faulted the GPU
  // once with no cause found: the same kernels run clean and exact in the CPU
  // build of the library (every thread a fiber with wavefront semantics,
  // guarded allocations, AddressSanitizer), which alone defines the macro
  // above.  On the GPU those paths stay off until a cause is shown.
  if (alpha) return fail(DGFV_ERR_UNSUPPORTED, "dg_rhs_vjp: only alpha = NULL (pure DG) is enabled");
  int degrees = 0;
  for (int N = 1; N <= MAXN; ++N) degrees += !m->bucket[N].empty();
  if (degrees > 1) return fail(DGFV_ERR_UNSUPPORTED, "dg_rhs_vjp: meshes with degree jumps are not enabled");
#else
  (void)m;
  (void)alpha;
#endif
  return DGFV_OK;
}

// g_b = (dR/du)^T w_b for b < batch, enqueued on s (throws HipError).
void enqueue_vjp(const dgfv_mesh* m, const ParamsDev& p, const double* u, const double* alpha, const double* w,
                 double* g, int batch, hipStream_t s, bool timed = true) {
  const MeshView& v = m->view;
  const size_t plane = (size_t)m->nvar * m->n_node;
  Timed t(m, timed ? DGFV_KERNEL_VJP : -1, s);
  if (alpha) {
    hip_check(launch_blend_list(v, alpha, s), "blended list launch");
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).fv_means(v, (int)m->bucket[N].size(), 1, u, s), "fv_means launch");
  }
  for (int b = 0; b < batch; ++b) {
    const double* wb = w + b * plane;
    double* gb = g + b * plane;
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).vjp_volume(v, p, m->d_bucket[N], (int)m->bucket[N].size(), u, alpha, wb, gb, s),
                  "vjp_volume launch");
    if (alpha)
      for (int N = 1; N <= MAXN; ++N)
        if (!m->bucket[N].empty())
          hip_check(ops_for(N).vjp_fv(v, p, m->d_bucket[N], (int)m->bucket[N].size(), alpha, wb, s),
                    "vjp_fv launch");
    hip_check(launch_faces_vjp(v, p, u, alpha, s), "face vjp launch");
    if (m->n_mortar > 0) hip_check(launch_mortars_vjp(v, p, u, s), "mortar vjp launch");
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).vjp_gather(v, m->d_bucket[N], (int)m->bucket[N].size(), alpha, gb, s),
                  "vjp_gather launch");
  }
}

}  // namespace

extern "C" {

const char* dgfv_last_error(void) { return g_last_error.c_str(); }

dgfv_status dgfv_check_state(dgfv_mesh* m, void* stream) {
  if (!m) return fail(DGFV_ERR_ARG, "NULL argument");
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return fail(DGFV_ERR_HIP, "hipStreamSynchronize");
  int32_t h = 0;
  if (hipMemcpy(&h, m->view.state_flag, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(DGFV_ERR_HIP, "hipMemcpy of the state flag");
  m->flag_pending = false;
  *m->flag_host = 0;
  if (h == 0) return DGFV_OK;
  if (hipMemset(m->view.state_flag, 0, sizeof(int32_t)) != hipSuccess) return fail(DGFV_ERR_HIP, "hipMemset");
  return fail(DGFV_ERR_STATE, "a state with rho <= 0, p <= 0 or NaN was read since the last check");
}

dgfv_status dgfv_mesh_create(const dgfv_mesh_desc* d, dgfv_mesh** out) {
  if (!d || !out) return fail(DGFV_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (d->n_elem <= 0) return fail(DGFV_ERR_ARG, "n_elem must be positive");
  if (d->n_var != 5 && d->n_var != 6) return fail(DGFV_ERR_ARG, "n_var must be 5 or 6");
  if (!d->degree || !d->corners || !d->faces) return fail(DGFV_ERR_ARG, "NULL mesh array");
  int nmin = 99, nmax = 0;
  for (int e = 0; e < d->n_elem; ++e) {
    const int N = d->degree[e];
    if (N < 1 || N > MAXN) return fail(DGFV_ERR_UNSUPPORTED, "element degree must be in 1..7");
    nmin = std::min(nmin, N);
    nmax = std::max(nmax, N);
  }
  if (d->metric_degree < 0 || d->metric_degree > nmin)
    return fail(DGFV_ERR_ARG, "metric_degree must be 0 (per element) or in 1..min(degree)");
  if (d->n_fv < nmax + 1 || d->n_fv > MAXFV)
    return fail(DGFV_ERR_UNSUPPORTED, "n_fv must be in max(degree)+1 .. 8");
  if (d->n_face < 0 || d->n_mortar < 0 || (d->n_mortar > 0 && !d->mortars))
    return fail(DGFV_ERR_ARG, "face or mortar count out of range");
  if (d->n_mortar > 0 && d->metric_degree == 0)
    return fail(DGFV_ERR_UNSUPPORTED, "meshes with mortars take a mesh-wide metric degree (metric_degree >= 1)");
  {
    std::vector<uint8_t> seen((size_t)d->n_elem * 6, 0);
    auto mark = [&](int e, int s) {
      if (e < 0 || e >= d->n_elem || s < 0 || s > 5) return 1;
      return seen[(size_t)e * 6 + s]++ ? 2 : 0;
    };
    for (int f = 0; f < d->n_face; ++f) {
      const int32_t* fc = d->faces + 5 * f;
      for (int side = 0; side < 2; ++side) {
        const int r = mark(fc[2 * side], fc[2 * side + 1]);
        if (r == 1) return fail(DGFV_ERR_ARG, "face entry out of range");
        if (r == 2) return fail(DGFV_ERR_ARG, "element side used twice");
      }
      if (fc[4] < 0 || fc[4] > 7) return fail(DGFV_ERR_ARG, "orientation code out of range");
    }
    for (int q = 0; q < d->n_mortar; ++q) {
      const int32_t* mr = d->mortars + 15 * q;
      if (mr[2] < 1 || mr[2] > 3) return fail(DGFV_ERR_ARG, "mortar type must be 1, 2 or 3");
      const int nsub = mr[2] == 3 ? 4 : 2;
      int r = mark(mr[0], mr[1]);
      for (int k = 0; k < 4 && r == 0; ++k) {
        if (k < nsub) {
          r = mark(mr[3 + k], mr[7 + k]);
          if (r == 0 && (mr[11 + k] < 0 || mr[11 + k] > 7)) r = 1;
        } else if (mr[3 + k] != -1 || mr[7 + k] != -1 || mr[11 + k] != -1) {
          r = 1;
        }
      }
      if (r == 1) return fail(DGFV_ERR_ARG, "mortar entry out of range");
      if (r == 2) return fail(DGFV_ERR_ARG, "element side used twice");
    }
    for (uint8_t c : seen)
      if (c != 1) return fail(DGFV_ERR_ARG, "every element side must belong to exactly one face or mortar");
  }
  if (d->n_var == 5 && !(d->gamma > 1.0)) return fail(DGFV_ERR_ARG, "gamma must exceed 1");
  if (d->n_var == 6 && !(d->kappa[0] > 1.0 && d->kappa[1] > 1.0 && d->R[0] > 0 && d->R[1] > 0))
    return fail(DGFV_ERR_ARG, "invalid species constants");

  std::unique_ptr<dgfv_mesh> m(new dgfv_mesh);
  try {
    m->K = d->n_elem;
    m->nvar = d->n_var;
    m->n_fv = d->n_fv;
    m->NJ = d->metric_degree;
    m->F = d->n_face;
    m->n_mortar = d->n_mortar;
    m->degree.assign(d->degree, d->degree + d->n_elem);
    for (int q = 0; q < d->n_mortar; ++q) {
      const int32_t* mr = d->mortars + 15 * q;
      for (int k = 0; k < 4; ++k)
        if (mr[3 + k] >= 0 && d->degree[mr[3 + k]] != d->degree[mr[0]]) m->mortar_jump = true;
    }
    m->offset.resize(m->K + 1);
    m->offset[0] = 0;
    for (int e = 0; e < m->K; ++e) {
      const int n = m->degree[e] + 1;
      m->offset[e + 1] = m->offset[e] + n * n * n;
    }
    m->n_node = m->offset[m->K];
    const int NFV = m->n_fv, NJ = m->NJ;
    bool present[MAXN + 1] = {false};
    for (int e = 0; e < m->K; ++e) present[m->degree[e]] = true;

    // ---- operator tables --------------------------------------------------
    std::vector<double> ops;
    OpTables tab;
    std::memset(&tab, 0xff, sizeof(tab));   // -1 everywhere
    auto push = [&](const std::vector<double>& a) {
      const int off = (int)ops.size();
      ops.insert(ops.end(), a.begin(), a.end());
      return off;
    };
    for (int N = 1; N <= MAXN; ++N) {
      if (!present[N]) continue;
      tab.D[N] = push(op_D(N));
      tab.w[N] = push(op_weights(N));
      tab.vleg_inv[N] = push(op_vleg_inv(N));
      tab.dg2fv[N] = push(op_dg2fv(N, NFV));
      tab.fv2dg[N] = push(op_fv2dg(N, NFV));
      tab.dg2fvT[N] = push(transpose(op_dg2fv(N, NFV), NFV, N + 1));
      tab.fv2dgT[N] = push(transpose(op_fv2dg(N, NFV), N + 1, NFV));
      tab.face_interp[N] = push(op_face_interp(N, NFV));
      if (d->n_mortar > 0)
        for (int k = 0; k < 2; ++k) {
          tab.mortar_interp[N][k] = push(op_mortar_interp(N, k));
          tab.mortar_proj[N][k] = push(op_mortar_project(N, k));
          tab.mortar_interpT[N][k] = push(transpose(op_mortar_interp(N, k), N + 1, N + 1));
          tab.mortar_projT[N][k] = push(transpose(op_mortar_project(N, k), N + 1, N + 1));
        }
      if (d->n_mortar > 0 && tab.mortar_fv_interp[0] < 0)
        for (int k = 0; k < 2; ++k) {
          tab.mortar_fv_interp[k] = push(op_mortar_fv_interp(NFV, k));
          tab.mortar_fv_proj[k] = push(op_mortar_fv_project(NFV, k));
        }
      for (int M = N + 1; M <= MAXN; ++M) {
        if (!present[M]) continue;
        tab.interp[N][M] = push(op_interp(N, M));
        tab.project[M][N] = push(op_project(M, N));
        tab.interpT[N][M] = push(transpose(op_interp(N, M), M + 1, N + 1));
        tab.projectT[M][N] = push(transpose(op_project(M, N), N + 1, M + 1));
      }
    }

    // ---- metrics and coordinates -------------------------------------------
    // NJ >= 1: curl form at one mesh-wide degree NJ, interpolated to each degree;
    // NJ == 0: per element at its own degree, faces matched to lower-degree neighbours
    const int NJc = NJ > 0 ? NJ : 1;
    const auto xJ = op_nodes(NJc);
    const auto DJ = op_D(NJc);
    std::array<std::vector<double>, MAXN + 1> xN, VJN;
    for (int N = 1; N <= MAXN; ++N) {
      if (present[N] || N == NJc) {
        xN[N] = op_nodes(N);
        VJN[N] = op_interp(NJc, N);
      }
    }
    std::vector<int32_t> nbr((size_t)m->K * 6, 0);
    for (int f = 0; f < d->n_face; ++f) {
      const int32_t* fc = d->faces + 5 * f;
      nbr[(size_t)fc[0] * 6 + fc[1]] = m->degree[fc[2]];
      nbr[(size_t)fc[2] * 6 + fc[3]] = m->degree[fc[0]];
    }
    std::vector<double> metric((size_t)10 * m->n_node);
    m->coords.assign((size_t)3 * m->n_node, 0.0);
    std::vector<uint8_t> bad(m->K, 0);
    const int nJ = NJc + 1, nJ3 = nJ * nJ * nJ;
    std::vector<double> JaJ_all(NJ > 0 ? (size_t)m->K * 9 * nJ3 : 0);
    parallel_for(m->K, [&](int64_t e) {
      const double* c = d->corners + 24 * e;
      const int N = m->degree[e], n = N + 1, n3 = n * n * n;
      std::vector<double> JaN(9 * n3);
      if (NJ > 0) {
        std::vector<double> JaJ;
        curl_metrics(c, NJ, xJ, DJ, JaJ);
        std::copy(JaJ.begin(), JaJ.end(), JaJ_all.begin() + e * 9 * nJ3);
        interp3(VJN[N], nJ, n, JaJ.data(), JaN.data(), 9);
      } else {
        matched_metrics(c, N, &nbr[(size_t)e * 6], JaN.data());
      }
      const int64_t base = m->offset[e];
      for (int t = 0; t < n3; ++t) {
        for (int comp = 0; comp < 9; ++comp) metric[(size_t)comp * m->n_node + base + t] = JaN[comp * n3 + t];
        const int i = t % n, j = (t / n) % n, k = t / (n * n);
        double X[3], G[3][3];
        trilinear(c, xN[N][i], xN[N][j], xN[N][k], X, G);
        const double J = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                         G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                         G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
        if (!(J > 0)) bad[e] = 1;
        metric[(size_t)9 * m->n_node + base + t] = J;
        for (int a = 0; a < 3; ++a) m->coords[(size_t)a * m->n_node + base + t] = X[a];
      }
    });
    for (int e = 0; e < m->K; ++e)
      if (bad[e]) return fail(DGFV_ERR_ARG, "element " + std::to_string(e) + " has a non-positive Jacobian");

    // ---- faces: left outward normal at the common degree M -----------------
    std::vector<int64_t> fnorm_off(m->F);
    int64_t tot = 0;
    for (int f = 0; f < m->F; ++f) {
      const int M = std::max(m->degree[d->faces[5 * f]], m->degree[d->faces[5 * f + 2]]);
      fnorm_off[f] = tot;
      tot += 3 * (M + 1) * (M + 1);
    }
    std::vector<double> fnorm(tot);
    std::array<std::array<std::vector<double>, MAXN + 1>, MAXN + 1> VLM;   // [NL][M], per-element mode
    if (NJ == 0)
      for (int a = 1; a <= MAXN; ++a)
        for (int b = a; b <= MAXN; ++b)
          if (present[a] && present[b]) VLM[a][b] = op_interp(a, b);
    parallel_for(m->F, [&](int64_t f) {
      const int32_t* fc = d->faces + 5 * f;
      const int eL = fc[0], sL = fc[1];
      const int M = std::max(m->degree[eL], m->degree[fc[2]]);
      const int nM = M + 1, dd = sL / 2;
      const double sign = (sL & 1) ? 1.0 : -1.0;
      // face slice of the left element's Ja^dd (at NJ, or at its own degree NL
      // per element), then 2D interpolation to M
      const int nS = NJ > 0 ? nJ : m->degree[eL] + 1;
      const auto& V = NJ > 0 ? VJN[M] : VLM[nS - 1][M];
      for (int comp = 0; comp < 3; ++comp) {
        std::vector<double> sl(nS * nS);
        for (int q = 0; q < nS; ++q)
          for (int p = 0; p < nS; ++p) {
            const int node = side_node_h(sL, p, q, nS);
            sl[q * nS + p] = NJ > 0 ? JaJ_all[(size_t)eL * 9 * nJ3 + (3 * dd + comp) * nJ3 + node]
                                    : metric[(size_t)(3 * dd + comp) * m->n_node + m->offset[eL] + node];
          }
        for (int q = 0; q < nM; ++q)
          for (int p = 0; p < nM; ++p) {
            double acc = 0.0;
            for (int b = 0; b < nS; ++b)
              for (int a = 0; a < nS; ++a) acc += V[q * nS + b] * V[p * nS + a] * sl[b * nS + a];
            fnorm[fnorm_off[f] + comp * nM * nM + q * nM + p] = sign * acc;
          }
      }
    });

    // ---- per-element side blocks -------------------------------------------
    std::vector<int64_t> side_off(m->K);
    int64_t stot = 0;
    for (int e = 0; e < m->K; ++e) {
      const int n = m->degree[e] + 1;
      side_off[e] = stot;
      stot += (int64_t)6 * m->nvar * n * n;
    }

    // ---- buckets -----------------------------------------------------------
    for (int e = 0; e < m->K; ++e) m->bucket[m->degree[e]].push_back(e);

    // ---- device ------------------------------------------------------------
    MeshView& v = m->view;
    v.K = m->K;
    v.nvar = m->nvar;
    v.n_fv = NFV;
    v.n_face = m->F;
    v.n_node = m->n_node;
    v.elem_offset = m->keep(dev_upload(m->offset));
    v.degree = m->keep(dev_upload(m->degree));
    v.metric = m->keep(dev_upload(metric));
    std::vector<int32_t> faces(d->faces, d->faces + 5 * (size_t)m->F);
    v.faces = m->keep(dev_upload(faces));
    v.face_norm_off = m->keep(dev_upload(fnorm_off));
    v.face_norm = m->keep(dev_upload(fnorm));
    v.side_off = m->keep(dev_upload(side_off));
    v.fside = m->keep(dev_alloc<double>(stot));
    m->side_total = (size_t)stot;
    v.trace = m->keep(dev_alloc<double>(stot / 3));    // sides 0 and 1 of every element
    v.fvside = m->keep(dev_alloc<double>((size_t)m->K * 6 * m->nvar * NFV * NFV));
    v.ubar = m->keep(dev_alloc<double>((size_t)m->K * m->nvar * NFV * NFV * NFV));
    v.rfv = m->keep(dev_alloc<double>((size_t)m->nvar * m->n_node));
    v.ubar_bar = m->keep(dev_alloc<double>((size_t)m->K * m->nvar * NFV * NFV * NFV));
    v.fvnorm = m->keep(dev_alloc<double>((size_t)m->K * 9 * (NFV - 1) * NFV * NFV));
    v.ops = m->keep(dev_upload(ops));
    v.tab = tab;
    v.gas.gamma = d->gamma;
    if (m->nvar == 6) {
      v.gas.cv0 = d->R[0] / (d->kappa[0] - 1.0);
      v.gas.cp0 = d->kappa[0] * v.gas.cv0;
      v.gas.cv1 = d->R[1] / (d->kappa[1] - 1.0);
      v.gas.cp1 = d->kappa[1] * v.gas.cv1;
    } else {
      v.gas.cv0 = v.gas.cp0 = v.gas.cv1 = v.gas.cp1 = 0.0;
    }
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty()) m->d_bucket[N] = m->keep(dev_upload(m->bucket[N]));
    // face classes: conforming lists per degree, degree-jump list, element -> face map
    {
      std::array<std::vector<int32_t>, MAXN + 1> conf;
      std::vector<int32_t> mixed, elem_face((size_t)m->K * 6, -1);
      for (int f = 0; f < m->F; ++f) {
        const int32_t* fc = d->faces + 5 * f;
        const int NL = m->degree[fc[0]], NR = m->degree[fc[2]];
        if (NL == NR) conf[NL].push_back(f);
        else mixed.push_back(f);
        elem_face[(size_t)fc[0] * 6 + fc[1]] = f;
        elem_face[(size_t)fc[2] * 6 + fc[3]] = f;
      }
      for (int N = 0; N <= MAXN; ++N) {
        v.face_conf[N] = conf[N].empty() ? nullptr : m->keep(dev_upload(conf[N]));
        v.face_conf_count[N] = (int)conf[N].size();
        std::vector<ConfRec> rec(conf[N].size());
        for (size_t i = 0; i < conf[N].size(); ++i) {
          const int32_t* fc = d->faces + 5 * (size_t)conf[N][i];
          ConfRec& r = rec[i];
          r.baseL = m->offset[fc[0]];
          r.baseR = m->offset[fc[2]];
          r.sideL = side_off[fc[0]];
          r.sideR = side_off[fc[2]];
          r.nrm = fnorm_off[conf[N][i]];
          r.eL = fc[0];
          r.eR = fc[2];
          r.code = fc[1] | (fc[3] << 3) | (fc[4] << 6);
          r.pad = 0;
        }
        v.face_conf_rec[N] = rec.empty() ? nullptr : m->keep(dev_upload(rec));
      }
      v.face_mixed = mixed.empty() ? nullptr : m->keep(dev_upload(mixed));
      v.face_mixed_count = (int)mixed.size();
      v.elem_face = m->keep(dev_upload(elem_face));
      std::vector<SideRec> srec((size_t)m->K * 6);
      for (int e = 0; e < m->K; ++e)
        for (int sd = 0; sd < 6; ++sd) {
          const int f = elem_face[(size_t)e * 6 + sd];
          SideRec& r = srec[(size_t)e * 6 + sd];
          if (f < 0) {                      // a mortar side: no neighbour of its own
            r.baseL = r.baseR = m->offset[e];
            r.nrm = 0;
            r.nbr = e;
            r.code = sd | (sd << 3) | (1 << 9) | (1 << 11);
            continue;
          }
          const int32_t* fc = d->faces + 5 * (size_t)f;
          const bool left = fc[0] == e && fc[1] == sd;
          r.baseL = m->offset[fc[0]];
          r.baseR = m->offset[fc[2]];
          r.nrm = fnorm_off[f];
          r.nbr = left ? fc[2] : fc[0];
          r.code = fc[1] | (fc[3] << 3) | (fc[4] << 6) | ((left ? 1 : 0) << 9) |
                   ((m->degree[fc[0]] == m->degree[fc[2]] ? 1 : 0) << 10);
        }
      v.side_rec = m->keep(dev_upload(srec));
      if (d->n_mortar > 0) {
        std::vector<int32_t> mort(d->mortars, d->mortars + 15 * (size_t)d->n_mortar);
        v.mortars = m->keep(dev_upload(mort));
      }
      v.n_mortar = d->n_mortar;
    }
    // blended-element work list: buckets concatenated in ascending degree
    {
      std::vector<int32_t> order;
      order.reserve(m->K);
      for (int N = 0; N <= MAXN + 1; ++N) v.bucket_pos[N] = 0;
      for (int N = 1; N <= MAXN; ++N) {
        v.bucket_pos[N] = (int)order.size();
        order.insert(order.end(), m->bucket[N].begin(), m->bucket[N].end());
      }
      v.bucket_pos[MAXN + 1] = (int)order.size();
      v.order = m->keep(dev_upload(order));
      v.n_chunk = (m->K + LIST_CHUNK - 1) / LIST_CHUNK;
      v.chunk_cnt = m->keep(dev_alloc<int32_t>(v.n_chunk));
      v.chunk_off = m->keep(dev_alloc<int32_t>(v.n_chunk));
      v.blend_list = m->keep(dev_alloc<int32_t>(m->K));
      v.blend_start = m->keep(dev_alloc<int32_t>(MAXN + 2));
      v.state_flag = m->keep(dev_alloc<int32_t>(1));
      hip_check(hipMemset(v.state_flag, 0, sizeof(int32_t)), "hipMemset");
      hip_check(hipHostMalloc((void**)&m->flag_host, sizeof(int32_t), hipHostMallocDefault), "hipHostMalloc");
      *m->flag_host = 0;
      hip_check(hipEventCreateWithFlags(&m->flag_ev, hipEventDisableTiming), "hipEventCreate");
      int dev = 0, cus = 0;
      hip_check(hipGetDevice(&dev), "hipGetDevice");
      hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
      v.n_cu = cus > 0 ? cus : 1;
    }
    {
      double* sp = nullptr;                  // the no-allocation entry point's buffer on this device
      hip_check(static_scratch_ptr(&sp), "hipGetSymbolAddress of the fixed device buffer");
    }
    for (auto& st : m->side) hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreateWithFlags(&m->fork_ev, hipEventDisableTiming), "hipEventCreate");
    for (auto& e : m->join_ev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).fv_normals(v, m->d_bucket[N], (int)m->bucket[N].size(), nullptr),
                  "fv_normals launch");
    hip_check(hipDeviceSynchronize(), "mesh upload");
  } catch (const HipError& e) {
    const std::string msg = e.what();
    return fail(msg.find("out of memory") != std::string::npos ? DGFV_ERR_OOM : DGFV_ERR_HIP, msg);
  } catch (const std::exception& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  *out = m.release();
  return DGFV_OK;
}

void dgfv_mesh_destroy(dgfv_mesh* m) { delete m; }

dgfv_status dgfv_mesh_info(const dgfv_mesh* m, int64_t* n_node, int64_t* elem_offset) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  if (n_node) *n_node = m->n_node;
  if (elem_offset) std::copy(m->offset.begin(), m->offset.end(), elem_offset);
  return DGFV_OK;
}

dgfv_status dgfv_mesh_node_coords(const dgfv_mesh* m, double* xyz) {
  if (!m || !xyz) return fail(DGFV_ERR_ARG, "NULL argument");
  std::copy(m->coords.begin(), m->coords.end(), xyz);
  return DGFV_OK;
}

dgfv_status dg_indicator(const dgfv_mesh* m, const dgfv_params* prm, const double* u,
                         double* alpha, double* ind, void* stream) {
  if (!m || !u || !alpha) return fail(DGFV_ERR_ARG, "NULL argument");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (!(prm->ind_dT > 0.0)) return fail(DGFV_ERR_ARG, "ind_dT must be positive");
  if ((prm->ind_vars & 7) == 0) return fail(DGFV_ERR_ARG, "ind_vars selects no variable");
  const ParamsDev p = to_dev(prm);
  try {
    Timed t(m, DGFV_KERNEL_INDICATOR, (hipStream_t)stream);
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).indicator(m->view, p, m->d_bucket[N], (int)m->bucket[N].size(), u, alpha,
                                       ind, (hipStream_t)stream),
                  "indicator launch");
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dg_p_degrees(const dgfv_mesh* m, const dgfv_params* prm, const double* u, double t_refine,
                         double t_coarsen, int n_min, int n_max, int8_t* degree_out, void* stream) {
  if (!m || !u || !degree_out) return fail(DGFV_ERR_ARG, "NULL argument");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (n_min < 1 || n_max > MAXN || n_min > n_max) return fail(DGFV_ERR_ARG, "need 1 <= n_min <= n_max <= 7");
  if (!(t_refine < t_coarsen)) return fail(DGFV_ERR_ARG, "need t_refine < t_coarsen");
  hipStream_t s = (hipStream_t)stream;
  if (capturing(s)) return fail(DGFV_ERR_ARG, "dg_p_degrees waits for its result: not under capture");
  try {
    if (!m->pind) m->pind = dev_alloc<double>(2 * (size_t)m->K);      // alpha scratch, then I
    ParamsDev p = to_dev(prm);
    p.ind_vars = 2;                                                   // I_p-adapt = I(rho)
    p.ind_T = 0.0;
    p.ind_dT = 1.0;
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).indicator(m->view, p, m->d_bucket[N], (int)m->bucket[N].size(), u, m->pind,
                                       m->pind + m->K, s),
                  "indicator launch");
    std::vector<double> I(m->K);
    hip_check(hipMemcpyAsync(I.data(), m->pind + m->K, sizeof(double) * m->K, hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int e = 0; e < m->K; ++e) {
      int N = m->degree[e];
      if (I[e] < t_refine) N = std::min(N + 1, n_max);
      else if (I[e] > t_coarsen) N = std::max(N - 1, n_min);
      degree_out[e] = (int8_t)N;
    }
  } catch (const HipError& e) {
    return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dg_transfer_degree(const dgfv_mesh* from, const dgfv_mesh* to, const double* u_from, double* u_to,
                               void* stream) {
  if (!from || !to || !u_from || !u_to) return fail(DGFV_ERR_ARG, "NULL argument");
  if (from->K != to->K || from->nvar != to->nvar) return fail(DGFV_ERR_ARG, "the meshes differ in n_elem or n_var");
  if (u_from == u_to) return fail(DGFV_ERR_ARG, "u_from and u_to must not overlap");
  hipStream_t s = (hipStream_t)stream;
  try {
    if (!to->pmap) {
      if (capturing(s)) return fail(DGFV_ERR_ARG, "the first transfer into a mesh allocates: not under capture");
      constexpr int TM = MAXN + 1;
      std::vector<double> tab((size_t)TM * TM * TM * TM, 0.0);
      for (int Nf = 1; Nf <= MAXN; ++Nf)
        for (int Nt = 1; Nt <= MAXN; ++Nt) {
          std::vector<double> A;
          if (Nt > Nf) A = op_interp(Nf, Nt);
          else if (Nt < Nf) A = op_project(Nf, Nt);
          else {
            A.assign((size_t)(Nf + 1) * (Nf + 1), 0.0);
            for (int i = 0; i <= Nf; ++i) A[(size_t)i * (Nf + 1) + i] = 1.0;
          }
          std::copy(A.begin(), A.end(), tab.begin() + ((size_t)Nf * TM + Nt) * TM * TM);
        }
      double* d = dev_upload(tab);
      to->pmap = d;
    }
    hip_check(launch_transfer(from->view, to->view, u_from, u_to, to->pmap, s), "transfer launch");
  } catch (const HipError& e) {
    return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dg_rhs(const dgfv_mesh* m, const dgfv_params* prm, const double* u, const double* alpha,
                   double* ut, void* stream) {
  if (!m || !u || !ut) return fail(DGFV_ERR_ARG, "NULL argument");
  if (u == ut) return fail(DGFV_ERR_ARG, "u and ut must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  hipStream_t s = (hipStream_t)stream;
  return guarded(m, s, [&] { return enqueue_rhs(m, prm, u, alpha, ut, nullptr, 0, 0.0, s); });
}

dgfv_status dg_rk_stage(const dgfv_mesh* m, const dgfv_params* prm, int stage, double dt, double* u,
                        double* k, const double* alpha, void* stream) {
  if (!m || !u || !k) return fail(DGFV_ERR_ARG, "NULL argument");
  if (stage < 1 || stage > 5) return fail(DGFV_ERR_ARG, "stage must be 1..5");
  if (!std::isfinite(dt)) return fail(DGFV_ERR_ARG, "dt must be finite");
  if (u == k) return fail(DGFV_ERR_ARG, "u and k must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  hipStream_t s = (hipStream_t)stream;
  return guarded(m, s, [&] { return run_stages(m, prm, 0, stage, stage, dt, u, k, alpha, s); });
}

dgfv_status dg_rk_step(const dgfv_mesh* m, const dgfv_params* prm, double dt, double* u, double* k,
                       const double* alpha, void* stream) {
  if (!m || !u || !k) return fail(DGFV_ERR_ARG, "NULL argument");
  if (!std::isfinite(dt)) return fail(DGFV_ERR_ARG, "dt must be finite");
  if (u == k) return fail(DGFV_ERR_ARG, "u and k must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  hipStream_t s = (hipStream_t)stream;
  return guarded(m, s, [&] { return run_stages(m, prm, 1, 1, 5, dt, u, k, alpha, s); });
}

dgfv_status dgfv_autotune(dgfv_mesh* m, const dgfv_params* prm, const double* u, const double* alpha,
                          double* ms_out, void* stream) {
  if (!m || !u) return fail(DGFV_ERR_ARG, "NULL argument");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (ms_out) std::fill(ms_out, ms_out + 2 * (MAXN + 1), 0.0);
  hipStream_t s = (hipStream_t)stream;
  double* scratch = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool prof = m->profile;
  m->profile = false;
  try {
    scratch = dev_alloc<double>((size_t)m->nvar * m->n_node);
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    const ParamsDev p = to_dev(prm);
    // one full evaluation (faces not fused) fills the side-flux and FV buffers that the element kernel reads
    enqueue_rhs_impl(m, p, u, const_cast<double*>(u), alpha, scratch, nullptr, 0, 0.0, s);
    const MeshView& v = m->view;
    constexpr int REPS = 5;
    for (int N = 1; N <= MAXN; ++N) {
      const DegreeOps ops = ops_for(N);
      if (m->bucket[N].empty() || ops.element_variants < 2) continue;
      const int cnt = (int)m->bucket[N].size();
      double best = 0.0;
      int choice = 0;
      for (int var = 0; var < ops.element_variants; ++var) {
        hip_check(ops.element(v, p, m->d_bucket[N], cnt, u, const_cast<double*>(u), alpha, scratch, nullptr, 0, 0.0,
                              0.0, 0.0, var, 0, s),
                  "element launch");
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < REPS; ++r)
          hip_check(ops.element(v, p, m->d_bucket[N], cnt, u, const_cast<double*>(u), alpha, scratch, nullptr, 0, 0.0,
                              0.0, 0.0, var, 0, s),
                    "element launch");
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        const double avg = ms / REPS;
        if (ms_out) ms_out[2 * N + var] = avg;
        if (var == 0 || avg < best) {
          best = avg;
          choice = var;
        }
      }
      m->elem_variant[N] = choice;
    }
    m->drop_graphs();
  } catch (const HipError& e) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (scratch) (void)hipFree(scratch);
    m->profile = prof;
    return fail(DGFV_ERR_HIP, e.what());
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(scratch);
  m->profile = prof;
  return DGFV_OK;
}

dgfv_status dgfv_set_element_shape(dgfv_mesh* m, int degree, int shape) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  if (degree < 1 || degree > MAXN) return fail(DGFV_ERR_ARG, "degree must be in 1..7");
  if (shape < 0 || shape >= ops_for(degree).element_variants)
    return fail(DGFV_ERR_ARG, "no such element-kernel shape at this degree");
  m->elem_variant[degree] = shape;
  m->drop_graphs();
  return DGFV_OK;
}

dgfv_status dg_positivity_limiter(const dgfv_mesh* m, const dgfv_params* prm, double* u, const double* alpha,
                                  double* theta, void* stream) {
  if (!m || !u) return fail(DGFV_ERR_ARG, "NULL argument");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (m->nvar != 5) return fail(DGFV_ERR_UNSUPPORTED, "the positivity limiter is single-species only");
  try {
    enqueue_limiter(m, u, alpha, theta, (hipStream_t)stream, true);
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dg_rhs_fv(const dgfv_mesh* m, const dgfv_params* prm, const double* u, const double* ufv,
                      const double* fv, double* ut, double* utfv, void* stream) {
  if (!m || !u || !ufv || !fv || !ut || !utfv) return fail(DGFV_ERR_ARG, "NULL argument");
  if (u == ut || ufv == utfv) return fail(DGFV_ERR_ARG, "inputs and outputs must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (m->viscous) return fail(DGFV_ERR_UNSUPPORTED, "FV-stored elements with viscous terms are not built");
  hipStream_t s = (hipStream_t)stream;
  if (!m->fvghost && capturing(s)) return fail(DGFV_ERR_ARG, "the first call with FV-stored elements allocates: not under capture");
  return guarded(m, s, [&] {
    try {
      enqueue_rhs_fvs(m, to_dev(prm), const_cast<double*>(u), const_cast<double*>(ufv), fv, ut, utfv, nullptr,
                      nullptr, 0, 0.0, s);
    } catch (const HipError& e) {
      return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
    }
    return DGFV_OK;
  });
}

dgfv_status dg_rk_stage_fv(const dgfv_mesh* m, const dgfv_params* prm, int stage, double dt, double* u, double* k,
                           double* ufv, double* kfv, const double* fv, void* stream) {
  if (!m || !u || !k || !ufv || !kfv || !fv) return fail(DGFV_ERR_ARG, "NULL argument");
  if (stage < 1 || stage > 5) return fail(DGFV_ERR_ARG, "stage must be 1..5");
  if (!std::isfinite(dt)) return fail(DGFV_ERR_ARG, "dt must be finite");
  if (u == k || ufv == kfv) return fail(DGFV_ERR_ARG, "states and registers must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (m->viscous) return fail(DGFV_ERR_UNSUPPORTED, "FV-stored elements with viscous terms are not built");
  hipStream_t s = (hipStream_t)stream;
  if (!m->fvghost && capturing(s)) return fail(DGFV_ERR_ARG, "the first call with FV-stored elements allocates: not under capture");
  return guarded(m, s, [&] {
    try {
      enqueue_rhs_fvs(m, to_dev(prm), u, ufv, fv, nullptr, nullptr, k, kfv, stage, dt, s);
    } catch (const HipError& e) {
      return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
    }
    return DGFV_OK;
  });
}

dgfv_status dg_rk_step_fv(const dgfv_mesh* m, const dgfv_params* prm, double dt, double* u, double* k, double* ufv,
                          double* kfv, const double* fv, void* stream) {
  if (!m || !u || !k || !ufv || !kfv || !fv) return fail(DGFV_ERR_ARG, "NULL argument");
  if (!std::isfinite(dt)) return fail(DGFV_ERR_ARG, "dt must be finite");
  if (u == k || ufv == kfv) return fail(DGFV_ERR_ARG, "states and registers must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (m->viscous) return fail(DGFV_ERR_UNSUPPORTED, "FV-stored elements with viscous terms are not built");
  hipStream_t s = (hipStream_t)stream;
  if (!m->fvghost && capturing(s)) return fail(DGFV_ERR_ARG, "the first call with FV-stored elements allocates: not under capture");
  return guarded(m, s, [&] {
    try {
      const ParamsDev p = to_dev(prm);
      // between its own stages nothing else writes u: the DG faces read sides 0 and 1
      // from the traces the previous stage wrote
      for (int st = 1; st <= 5; ++st)
        enqueue_rhs_fvs(m, p, u, ufv, fv, nullptr, nullptr, k, kfv, st, dt, s, st > 1, st < 5);
    } catch (const HipError& e) {
      return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
    }
    return DGFV_OK;
  });
}

dgfv_status dg_switch_fv(const dgfv_mesh* m, double* u, double* ufv, const double* fv_old, const double* fv_new,
                         void* stream) {
  if (!m || !u || !ufv || !fv_old || !fv_new) return fail(DGFV_ERR_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (!m->fvghost && capturing(s)) return fail(DGFV_ERR_ARG, "the first call with FV-stored elements allocates: not under capture");
  try {
    ensure_fv_stored(m, s);
    const MeshView v = fvs_view(m);
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(ops_for(N).fv_switch(v, m->d_bucket[N], (int)m->bucket[N].size(), u, ufv, fv_old, fv_new, s),
                  "fv_switch launch");
  } catch (const HipError& e) {
    return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dgfv_set_positivity_limiter(dgfv_mesh* m, int enable) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  if (enable && m->nvar != 5) return fail(DGFV_ERR_UNSUPPORTED, "the positivity limiter is single-species only");
  m->limiter_on = enable != 0;
  m->drop_graphs();
  return DGFV_OK;
}

dgfv_status dgfv_set_transport(dgfv_mesh* m, const dgfv_transport* tr) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  if (!tr) {
    m->viscous = false;
    m->drop_graphs();
    return DGFV_OK;
  }
  for (int j = 0; j < 2; ++j) {
    if (!(tr->mu[j] >= 0.0) || !(tr->D[j] >= 0.0) || !(tr->Pr[j] > 0.0) || !std::isfinite(tr->mu[j]) ||
        !std::isfinite(tr->D[j]) || !std::isfinite(tr->Pr[j]))
      return fail(DGFV_ERR_ARG, "dgfv_set_transport: mu, D >= 0 and Pr > 0, finite");
  }
  if (!m->view.grad) {
    double* g = nullptr;
    double* vs = nullptr;
    double* rv = nullptr;
    const size_t plane = (size_t)m->nvar * (size_t)m->n_node;
    if (hipMalloc((void**)&g, sizeof(double) * 3 * plane) != hipSuccess ||
        hipMalloc((void**)&vs, sizeof(double) * m->side_total) != hipSuccess ||
        hipMalloc((void**)&rv, sizeof(double) * plane) != hipSuccess) {
      (void)hipGetLastError();
      if (g) (void)hipFree(g);
      if (vs) (void)hipFree(vs);
      return fail(DGFV_ERR_OOM, "dgfv_set_transport: device memory for the viscous terms");
    }
    m->view.grad = g;
    m->view.vside = vs;
    m->rvisc = rv;
  }
  m->view.visc = ViscDev{tr->mu[0], tr->mu[1], tr->Pr[0], tr->Pr[1], tr->D[0], tr->D[1]};
  m->viscous = true;
  m->drop_graphs();
  return DGFV_OK;
}

dgfv_status dg_timestep(const dgfv_mesh* m, const double* u, const double* alpha, double cfl, double cfl_v,
                        double* dt, void* stream) {
  if (!m || !u || !dt) return fail(DGFV_ERR_ARG, "NULL argument");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DGFV_ERR_ARG, "dg_timestep: cfl must be positive and finite");
  if (m->viscous && (!(cfl_v > 0.0) || !std::isfinite(cfl_v)))
    return fail(DGFV_ERR_ARG, "dg_timestep: cfl_v must be positive and finite");
  const hipStream_t s = (hipStream_t)stream;
  if (capturing(s)) return fail(DGFV_ERR_ARG, "dg_timestep waits for its result: not under capture");
  try {
    if (!m->dt_buf) m->dt_buf = dev_alloc<double>(2 * (size_t)m->K + 2);
    const MeshView& v = m->view;
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(viscous_ops_for(N).timestep(v, m->d_bucket[N], (int)m->bucket[N].size(), u, alpha,
                                              m->viscous ? 1 : 0, m->dt_buf, s),
                  "timestep launch");
    hip_check(launch_min_pairs(m->dt_buf, m->K, m->dt_buf + 2 * (size_t)m->K, s), "minimum launch");
    double h[2] = {0.0, 0.0};
    hip_check(hipMemcpyAsync(h, m->dt_buf + 2 * (size_t)m->K, sizeof h, hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    const double out = m->viscous ? 1.0 / (1.0 / (cfl * h[0]) + 1.0 / (cfl_v * h[1])) : cfl * h[0];
    if (!(out > 0.0) || !std::isfinite(out))
      return fail(DGFV_ERR_STATE, "dg_timestep: no positive finite time step (non-physical state)");
    *dt = out;
  } catch (const HipError& e) {
    return fail(msg_oom(e) ? DGFV_ERR_OOM : DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dg_lift(const dgfv_mesh* m, const double* u, double* g, void* stream) {
  if (!m || !u || !g) return fail(DGFV_ERR_ARG, "NULL argument");
  if (!m->viscous) return fail(DGFV_ERR_ARG, "dg_lift: no transport coefficients set (dgfv_set_transport)");
  const hipStream_t s = (hipStream_t)stream;
  try {
    MeshView v = m->view;
    v.grad = g;                                // the lift kernels write the caller's buffer
    hip_check(launch_lift_faces(v, u, s), "lift face launch");
  hip_check(launch_mortar_lift(v, u, s), "mortar lift launch");
    for (int N = 1; N <= MAXN; ++N)
      if (!m->bucket[N].empty())
        hip_check(viscous_ops_for(N).lift(v, m->d_bucket[N], (int)m->bucket[N].size(), u, false, s),
                  "lift launch");
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dgfv_set_face_fusion(dgfv_mesh* m, int enable) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  if (enable && m->n_mortar > 0) return fail(DGFV_ERR_UNSUPPORTED, "face fusion on meshes with mortars is not built");
  m->fuse_faces = enable != 0;
  m->drop_graphs();
  return DGFV_OK;
}

dgfv_status dgfv_set_launch_mode(dgfv_mesh* m, int mode) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  if (mode != DGFV_LAUNCH_SERIAL && mode != DGFV_LAUNCH_BRANCHES && mode != DGFV_LAUNCH_GRAPH)
    return fail(DGFV_ERR_ARG, "unknown launch mode");
  m->launch_mode = mode;
  if (mode != DGFV_LAUNCH_GRAPH) m->drop_graphs();
  return DGFV_OK;
}

dgfv_status dgfv_profile_enable(dgfv_mesh* m, int enable) {
  if (!m) return fail(DGFV_ERR_ARG, "mesh is NULL");
  m->profile = enable != 0;
  for (auto& u : m->ev_used) u = 0;
  return DGFV_OK;
}

dgfv_status dgfv_profile_read(dgfv_mesh* m, int kernel, double* total_ms, int64_t* launches) {
  if (!m || !total_ms || !launches) return fail(DGFV_ERR_ARG, "NULL argument");
  if (kernel < 0 || kernel >= DGFV_KERNEL_COUNT) return fail(DGFV_ERR_ARG, "kernel id out of range");
  double tot = 0.0;
  try {
    for (size_t i = 0; i < m->ev_used[kernel]; ++i) {
      auto& pr = m->ev[kernel][i];
      hip_check(hipEventSynchronize(pr.second), "hipEventSynchronize");
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
      tot += ms;
    }
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  *total_ms = tot;
  *launches = (int64_t)m->ev_used[kernel];
  return DGFV_OK;
}

dgfv_status dg_rhs_vjp(const dgfv_mesh* m, const dgfv_params* prm, const double* u,
                       const double* alpha, const double* w, double* g, int batch, void* stream) {
  if (!m || !u || !w || !g) return fail(DGFV_ERR_ARG, "NULL argument");
  if (batch < 1) return fail(DGFV_ERR_ARG, "batch must be positive");
  if (g == w || g == u) return fail(DGFV_ERR_ARG, "g must not overlap u or w");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (dgfv_status st = vjp_paths_enabled(m, alpha)) return st;
  try {
    enqueue_vjp(m, to_dev(prm), u, alpha, w, g, batch, (hipStream_t)stream);
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dg_rk_stage_vjp(const dgfv_mesh* m, const dgfv_params* prm, int stage, double dt,
                            const double* u_stage, double* ubar, double* kbar, const double* alpha,
                            void* stream) {
  if (!m || !u_stage || !ubar || !kbar) return fail(DGFV_ERR_ARG, "NULL argument");
  if (stage < 1 || stage > 5) return fail(DGFV_ERR_ARG, "stage must be 1..5");
  if (!std::isfinite(dt)) return fail(DGFV_ERR_ARG, "dt must be finite");
  if (ubar == kbar || ubar == u_stage || kbar == u_stage)
    return fail(DGFV_ERR_ARG, "u_stage, ubar and kbar must not overlap");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (dgfv_status st = vjp_paths_enabled(m, alpha)) return st;
  hipStream_t s = (hipStream_t)stream;
  try {
    if (!m->stage_g) m->stage_g = dev_alloc<double>((size_t)m->nvar * m->n_node);
    const MeshView& v = m->view;
    hip_check(launch_rk_adjoint_pre(v, RK_B[stage - 1], ubar, kbar, s), "rk adjoint launch");
    enqueue_vjp(m, to_dev(prm), u_stage, alpha, kbar, m->stage_g, 1, s);
    hip_check(launch_rk_adjoint_post(v, dt, RK_A[stage - 1], m->stage_g, ubar, kbar, s), "rk adjoint launch");
  } catch (const HipError& e) {
    const std::string msg = e.what();
    return fail(msg.find("out of memory") != std::string::npos ? DGFV_ERR_OOM : DGFV_ERR_HIP, msg);
  }
  return DGFV_OK;
}

dgfv_status dg_rk_stage_vjp_noalloc(const dgfv_mesh* m, const dgfv_params* prm, int stage, double dt,
                                    const double* u_stage, double* ubar, double* kbar, const double* alpha,
                                    void* stream) {
  if (!m || !u_stage || !ubar || !kbar) return fail(DGFV_ERR_ARG, "NULL argument");
  if (stage < 1 || stage > 5) return fail(DGFV_ERR_ARG, "stage must be 1..5");
  if (!std::isfinite(dt)) return fail(DGFV_ERR_ARG, "dt must be finite");
  if (ubar == kbar || ubar == u_stage || kbar == u_stage)
    return fail(DGFV_ERR_ARG, "u_stage, ubar and kbar must not overlap");
  if ((size_t)m->nvar * (size_t)m->n_node > STATIC_SCRATCH_DOUBLES)
    return fail(DGFV_ERR_ARG, "dg_rk_stage_vjp_noalloc: n_var * n_node = " +
                                  std::to_string((size_t)m->nvar * (size_t)m->n_node) +
                                  " exceeds the fixed buffer of " + std::to_string(STATIC_SCRATCH_DOUBLES) +
                                  " doubles");
  if (dgfv_status st = check_params(m, prm)) return st;
  if (dgfv_status st = vjp_paths_enabled(m, alpha)) return st;
  hipStream_t s = (hipStream_t)stream;
  try {
    double* g = nullptr;                     // this device's copy of the fixed buffer
    hip_check(static_scratch_ptr(&g), "hipGetSymbolAddress of the fixed device buffer");
    const MeshView& v = m->view;
    hip_check(launch_rk_adjoint_pre(v, RK_B[stage - 1], ubar, kbar, s), "rk adjoint launch");
    enqueue_vjp(m, to_dev(prm), u_stage, alpha, kbar, g, 1, s, false);
    hip_check(launch_rk_adjoint_post(v, dt, RK_A[stage - 1], g, ubar, kbar, s), "rk adjoint launch");
  } catch (const HipError& e) {
    return fail(DGFV_ERR_HIP, e.what());
  }
  return DGFV_OK;
}

dgfv_status dgfv_prim_to_cons(const dgfv_mesh* m, const double* w, double* u, void* stream) {
  if (!m || !w || !u) return fail(DGFV_ERR_ARG, "NULL argument");
  if (w == u) return fail(DGFV_ERR_ARG, "w and u must not overlap");
  if (hipError_t e = launch_prim_to_cons(m->view, w, u, (hipStream_t)stream))
    return fail(DGFV_ERR_HIP, std::string("prim_to_cons launch: ") + hipGetErrorString(e));
  return DGFV_OK;
}

}  // extern "C"
