// Internal declarations shared by the host runtime and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgfv {

constexpr int MAXN = 7;   // highest element degree
constexpr int MAXFV = 8;  // most FV sub-cells per direction

// Offsets (in doubles) of the small 1D operator tables inside one device buffer.
// A value of -1 marks a table that the mesh does not need.
struct OpTables {
  int D[MAXN + 1];                    // (N+1)^2, D[i*(N+1)+j] = l_j'(xi_i)
  int w[MAXN + 1];                    // (N+1) LGL weights
  int vleg_inv[MAXN + 1];             // (N+1)^2 nodal -> orthonormal Legendre modal
  int interp[MAXN + 1][MAXN + 1];     // [N][M]: (M+1) x (N+1), N < M
  int project[MAXN + 1][MAXN + 1];    // [M][N]: (N+1) x (M+1), M > N, modal L2 truncation
  int dg2fv[MAXN + 1];                // NFV x (N+1), sub-cell means of l_j
  int fv2dg[MAXN + 1];                // (N+1) x NFV, pseudo-inverse of dg2fv
  int face_interp[MAXN + 1];          // (NFV+1) x (N+1), l_j at the sub-cell interfaces
  // transposes, for the adjoint
  int interpT[MAXN + 1][MAXN + 1];    // [N][M]: (N+1) x (M+1)
  int projectT[MAXN + 1][MAXN + 1];   // [M][N]: (M+1) x (N+1)
  int dg2fvT[MAXN + 1];               // (N+1) x NFV
  int fv2dgT[MAXN + 1];               // NFV x (N+1)
  // mortars: [N][k] for half k of a degree-N big side, (N+1) x (N+1) each
  int mortar_interp[MAXN + 1][2];     // big side -> the nodes of half k
  int mortar_proj[MAXN + 1][2];       // half k's flux -> the big side
  int mortar_interpT[MAXN + 1][2];    // their transposes, for the adjoint
  int mortar_projT[MAXN + 1][2];
  int mortar_fv_interp[2];            // NFV x NFV: the big side's sub-faces -> those of half k
  int mortar_fv_proj[2];              // NFV x NFV: half k's sub-face fluxes -> the big side's
};

struct GasDev {
  double gamma;            // single species
  double cp0, cv0, cp1, cv1;  // two species (Y1 weights species 0)
};

// Constant species transport coefficients of the viscous terms (species 1,
// weighted by Y1, first; one species uses mu0, Pr0).
struct ViscDev {
  double mu0, mu1, Pr0, Pr1, D0, D1;
};

struct ParamsDev {
  int volume_flux, face_flux_dg, face_flux_fv;
  int ind_vars;
  double ind_T, ind_dT;
};

// One entry of a per-degree conforming face list with everything the face
// kernel addresses, gathered at set-up: one load replaces the dependent chain
// list -> face -> element offsets.
struct alignas(16) ConfRec {
  int64_t baseL, baseR;   // elem_offset of the left and right elements
  int64_t sideL, sideR;   // side_off of the left and right elements
  int64_t nrm;            // face_norm_off of the face
  int32_t eL, eR;         // the elements
  int32_t code;           // left side | right side << 3 | orientation << 6
  int32_t pad;
};

// One element side as the element kernel sees it when it evaluates the face
// flux itself: the face's two elements (left one first, as in the face
// table), the normals of the face, and
// code = left side | right side << 3 | orientation << 6 | (this element is the
// face's left one) << 9 | (both elements have the same degree) << 10 | (the
// side belongs to a mortar: no face record, nbr = the element itself) << 11.
struct alignas(16) SideRec {
  int64_t baseL, baseR;   // elem_offset of the left and right elements
  int64_t nrm;            // face_norm_off of the face
  int32_t nbr;            // the other element of the face
  int32_t code;
};

// Everything a kernel needs to address the mesh (device pointers).
struct MeshView {
  int K, nvar, n_fv, n_face;
  int64_t n_node;
  const int64_t* elem_offset;   // [K+1]
  const int8_t* degree;         // [K]
  const double* metric;         // [10][n_node]: Ja^d_n at component 3d+n, J at 9
  const int32_t* faces;         // [F][5]
  const int64_t* face_norm_off; // [F] offset into face_norm
  const double* face_norm;      // per face [3][(M+1)^2] left outward n*s at degree M = max(NL,NR)
  const int64_t* side_off;      // [K] offset of element e's side-flux block: 6*nvar*(N+1)^2 doubles
  double* fside;                // DG surface fluxes per element side, [6][nvar][(N+1)^2]
  double* trace;                // state on element sides 0 and 1 (the xi_1 ends), [2][nvar][(N+1)^2]
                                // at offset side_off[e] / 3, written by one RK stage for the next
                                // (elements of degree >= TRACE_MIN_N)
  double* fvside;               // FV sub-face fluxes, [K][6][nvar][NFV^2]
  double* ubar;                 // sub-cell means, [K][nvar][NFV^3]
  double* rfv;                  // FV residual in nodal form, [nvar][n_node]
  double* ubar_bar;             // adjoint of the sub-cell means, [K][nvar][NFV^3]
  double* fvnorm;               // sub-face normals of internal planes, [K][3][3][(NFV-1) NFV^2]
  // FV-stored elements (allocated by the first call that has them):
  double* fvghost;              // per FV element side the state across it on the sub-face grid,
                                // [K][6][nvar][NFV^2], written by the FV face kernel
  double* fvjbar;               // sub-cell means of J, V3(J), [K][NFV^3]
  const int32_t* elem_face;     // [K][6] face of each element side
  const SideRec* side_rec;      // [K][6] the same sides as records (element kernels of degree >= FUSE_MIN_N)
  const int32_t* face_conf[MAXN + 1];   // faces with NL = NR = N
  const ConfRec* face_conf_rec[MAXN + 1];   // the same lists as records
  int face_conf_count[MAXN + 1];
  const int32_t* face_mixed;    // faces with NL != NR
  int face_mixed_count;
  // blended-element work list, rebuilt from alpha by every call that has alpha
  const int32_t* order;         // [K] all elements, degree buckets in ascending degree
  int bucket_pos[MAXN + 2];     // start of degree N's bucket in `order`; [MAXN + 1] = K
  int n_chunk;                  // ceil(K / LIST_CHUNK)
  int32_t* chunk_cnt;           // [n_chunk] blended elements per chunk of `order`
  int32_t* chunk_off;           // [n_chunk] exclusive prefix sum of chunk_cnt
  int32_t* blend_list;          // [K] blended elements, in `order` order
  int32_t* blend_start;         // [MAXN + 2] blend_list range of degree N: [start[N], start[N + 1])
  int n_cu;                     // compute units of the device (persistent grid sizes)
  int32_t* state_flag;          // [1] set to 1 by an element kernel that reads rho <= 0, p <= 0 or NaN
  const double* ops;            // operator tables
  OpTables tab;
  GasDev gas;
  // non-conforming faces: [n_mortar][15] rows (big element, big side, type,
  // small elements[4], small sides[4], orientations[4])
  const int32_t* mortars;
  int n_mortar;
  // viscous terms (allocated when transport coefficients are set)
  ViscDev visc;
  double* grad;                 // BR1-lifted gradient of u, [3][nvar][n_node]
  double* vside;                // per element side, the layout of fside: at a degree jump the
                                // BR1 face value u*, then the outward viscous face flux; at a
                                // same-degree face the side's own viscous flux . its outward
                                // contravariant vector, which the neighbour's viscous kernel reads
  const double* rvisc;          // viscous rate [nvar][n_node] that the element kernel adds, or null
};

// ---- launchers (defined in the .hip translation units) ----------------------
// Per-degree launchers; each acts on one degree bucket: `count` elements listed
// in `elist` (device).  stage 0 writes ut = R(u); stage 1..5 performs the RK
// stage with coefficients (A, B) on k and writes the new state to uout (u
// itself when uout is u).
// Element-kernel flags:
//  ELEM_WRITE_TRACE  also store the new state of sides 0 and 1 in m.trace;
//  ELEM_FUSE_FACES   (degrees >= FUSE_MIN_N) evaluate the Riemann flux of every
//                    conforming face between two pure DG elements in the element
//                    kernel, from u, which the launch must not write: stage 0,
//                    or uout != u.  The face kernels then skip that degree's
//                    conforming class.
//  ELEM_SKIP_FV      elements with alpha >= 1 are FV-stored: the kernel leaves
//                    them alone (no reads of their side blocks, no writes).
constexpr int ELEM_WRITE_TRACE = 1, ELEM_FUSE_FACES = 2, ELEM_SKIP_FV = 4;
constexpr int FUSE_MIN_N = 6;    // one element per workgroup from here on
struct DegreeOps {
  // element kernel in tile shape `variant` (0 .. element_variants - 1)
  hipError_t (*element)(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                        const double* u, double* uout, const double* alpha, double* ut, double* k, int stage,
                        double dt, double A, double B, int variant, int flags, hipStream_t s);
  // FV kernels walk this degree's range of the blended-element list (m.blend_list,
  // m.blend_start); `count` bounds the range size.  fv_means runs persistent
  // workgroups, a 1/share part of the device (share = concurrent degree branches)
  hipError_t (*fv_means)(const MeshView& m, int count, int share, const double* u, hipStream_t s);
  hipError_t (*fv_residual)(const MeshView& m, const ParamsDev& p, int count, hipStream_t s);
  hipError_t (*indicator)(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                          const double* u, double* alpha, double* ind, hipStream_t s);
  // adjoint: g = (dR/du)^T w, alpha frozen (see dg_rhs_vjp)
  hipError_t (*vjp_volume)(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                           const double* u, const double* alpha, const double* w, double* g,
                           hipStream_t s);
  hipError_t (*vjp_fv)(const MeshView& m, const ParamsDev& p, const int32_t* elist, int count,
                       const double* alpha, const double* w, hipStream_t s);
  hipError_t (*vjp_gather)(const MeshView& m, const int32_t* elist, int count, const double* alpha,
                           double* g, hipStream_t s);
  // setup: sub-face normals of the FV sub-cell grid (geometry only)
  hipError_t (*fv_normals)(const MeshView& m, const int32_t* elist, int count, hipStream_t s);
  // positivity limiter (one species); sub-cell points of blended elements from m.ubar
  hipError_t (*limiter)(const MeshView& m, const int32_t* elist, int count, double* u, const double* alpha,
                        double* theta, hipStream_t s);
  // FV-stored elements: m.fvjbar = V3(J) of this bucket (setup), and the switch
  // of the elements whose flag changes: DG -> FV ufv = V3(J u) / V3(J),
  // FV -> DG u = V3^+(ufv V3(J)) / J
  hipError_t (*fv_jbar)(const MeshView& m, const int32_t* elist, int count, hipStream_t s);
  hipError_t (*fv_switch)(const MeshView& m, const int32_t* elist, int count, double* u, double* ufv,
                          const double* fv_old, const double* fv_new, hipStream_t s);
  int element_variants;   // tile shapes of the element kernel at this degree
};
// Per-degree launchers of the viscous terms (dgfv_viscous.hip), over the
// degree bucket `elist[0 .. count)`:
//  lift    m.grad = BR1-lifted gradient of u, from the face values in m.vside
//  volume  rv = -(1/J) [viscous volume term + viscous face fluxes of m.vside]
struct ViscousOps {
  // trace_in: the neighbours' sides 0 and 1 come from m.trace (written by the
  // previous RK stage's element kernels, degrees >= TRACE_MIN_N)
  hipError_t (*lift)(const MeshView& m, const int32_t* elist, int count, const double* u, bool trace_in,
                     hipStream_t s);
  hipError_t (*volume)(const MeshView& m, const int32_t* elist, int count, const double* u, double* rv,
                       hipStream_t s);
  // time step per element: dt_e[e] convective, dt_e[K + e] parabolic (0 unless viscous)
  hipError_t (*timestep)(const MeshView& m, const int32_t* elist, int count, const double* u,
                         const double* alpha, int viscous, double* dt_e, hipStream_t s);
};
ViscousOps viscous_ops_1();
ViscousOps viscous_ops_2();
ViscousOps viscous_ops_3();
ViscousOps viscous_ops_4();
ViscousOps viscous_ops_5();
ViscousOps viscous_ops_6();
ViscousOps viscous_ops_7();

DegreeOps degree_ops_1();
DegreeOps degree_ops_2();
DegreeOps degree_ops_3();
DegreeOps degree_ops_4();
DegreeOps degree_ops_5();
DegreeOps degree_ops_6();
DegreeOps degree_ops_7();

// Workgroups of `kernel` (block size `block`) resident on one compute unit at
// once; a persistent launch uses this times the compute units, so that every
// workgroup starts at once and the static round-robin split stays balanced.
inline int resident_per_cu(const void* kernel, int block) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0) != hipSuccess || n < 1) n = 1;
  return n;
}

// Blended-element work list of one call: m.blend_list and m.blend_start from alpha.
constexpr int LIST_CHUNK = 1024;
hipError_t launch_blend_list(const MeshView& m, const double* alpha, hipStream_t s);

// Interface fluxes into the per-side buffers, one launch per face class:
// 1..MAXN conforming DG faces of that degree, FACE_CLASS_MIXED degree jumps
// between DG elements, FACE_CLASS_FV faces with a blended side (needs the
// blended-element list of the call).  The classes write disjoint sides and
// may run concurrently.  With read_trace the conforming classes take the
// state on sides 0 and 1 from m.trace (written by the previous RK stage of
// the same step) instead of u.
constexpr int FACE_CLASS_MIXED = MAXN + 1, FACE_CLASS_FV = MAXN + 2, FACE_CLASS_COUNT = MAXN + 3;
constexpr int TRACE_MIN_N = 6;   // lowest degree whose sides 0 and 1 go through m.trace
bool face_class_present(const MeshView& m, const double* alpha, int cls);
hipError_t launch_face_class(const MeshView& m, const ParamsDev& p, const double* u, const double* alpha,
                             int cls, bool read_trace, hipStream_t s);

// Viscous face terms of the degree-jump faces (dgfv_faces.hip): the BR1 face
// value u* of both sides into m.vside, formed on the lower degree; then the
// arithmetic-mean viscous flux from u and m.grad on the higher degree, each
// side receiving its outward part at its own degree.  The per-degree lift and
// viscous kernels form the same-degree faces themselves.
hipError_t launch_lift_faces(const MeshView& m, const double* u, hipStream_t s);
hipError_t launch_visc_faces(const MeshView& m, const double* u, hipStream_t s);
// Fluxes of the non-conforming faces into m.fside, and into m.fvside for the
// FV parts of blended sides (dgfv_faces.hip), one mortar per workgroup, after
// the other face kernels.
hipError_t launch_face_mortars(const MeshView& m, const ParamsDev& p, const double* u, const double* alpha,
                               hipStream_t s);
// Adjoint of the mortar fluxes of pure DG meshes of one degree (dgfv_faces.hip):
// in place in m.fside, the cotangents of the side fluxes of each mortar's sides
// become those of their nodal traces (as launch_faces_vjp does for the faces).
hipError_t launch_mortars_vjp(const MeshView& m, const ParamsDev& p, const double* u, hipStream_t s);
// Viscous face terms of the mortars into m.vside (dgfv_faces.hip): the BR1
// values (before the lift kernels) and the viscous fluxes (after them).
hipError_t launch_mortar_lift(const MeshView& m, const double* u, hipStream_t s);
hipError_t launch_mortar_visc(const MeshView& m, const double* u, hipStream_t s);
hipError_t launch_faces_vjp(const MeshView& m, const ParamsDev& p, const double* u, const double* alpha,
                            hipStream_t s);

// FV-stored elements (flag fv[e] > 0; the blended-element list of the call holds
// them).  Faces with an FV side: minmod-reconstructed sub-face states, one
// Riemann flux per sub-face into m.fvside (FV sides) and, through
// V^{FV->DG} / h^2, m.fside (DG sides); the ghost layers into m.fvghost.
hipError_t launch_face_fv_stored(const MeshView& m, const ParamsDev& p, const double* u, const double* ufv,
                                 const double* fv, hipStream_t s);
// The mortars of a mesh with FV-stored elements: the DG mortar flux where a
// half has no FV-stored side, else the FV variant with the reconstruction
// (m.fvside, m.fside, m.fvghost).
hipError_t launch_mortars_fv_stored(const MeshView& m, const ParamsDev& p, const double* u, const double* ufv,
                                    const double* fv, hipStream_t s);
// Rates of the FV elements' means: stage 0 writes utfv = R; stage s updates
// kfv <- A kfv + dt R, ufv <- ufv + B kfv.
hipError_t launch_fv_stored(const MeshView& m, const ParamsDev& p, double* ufv, double* kfv, double* utfv,
                            int stage, double dt, double A, double B, hipStream_t s);

// Fixed device buffer (a file-scope device array in dgfv_state.hip) of the
// entry point that allocates nothing: its address on the current device,
// looked up once per device (hipGetSymbolAddress) and kept.
constexpr size_t STATIC_SCRATCH_DOUBLES = size_t(1) << 24;   // 128 MiB
constexpr int MAX_DEVICES = 64;
hipError_t static_scratch_ptr(double** out);

// p-adaptation: every element's state from its degree in `from` to its degree in
// `to` (same elements), with table[(Nf * 8 + Nt) * 64 ...] the (Nt+1) x (Nf+1) map.
hipError_t launch_transfer(const MeshView& from, const MeshView& to, const double* u_from, double* u_to,
                           const double* table, hipStream_t s);

// Pointwise state kernels (dgfv_state.hip).
// out[0] = min of dt_e[0 .. K), out[1] = min of dt_e[K .. 2K) (one workgroup).
hipError_t launch_min_pairs(const double* dt_e, int K, double* out, hipStream_t s);
hipError_t launch_prim_to_cons(const MeshView& m, const double* w, double* u, hipStream_t s);
hipError_t launch_rk_adjoint_pre(const MeshView& m, double B, const double* ubar, double* kbar, hipStream_t s);
hipError_t launch_rk_adjoint_post(const MeshView& m, double dt, double A, const double* g, double* ubar,
                                  double* kbar, hipStream_t s);

}  // namespace dgfv
