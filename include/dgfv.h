/*
 * dgfv.h - C ABI of the MI355X (gfx950) hybrid DG/FV right-hand side.
 *
 * The library evaluates, in FP64 on one GPU, the semi-discrete operator of the
 * hp-adaptive hybrid discontinuous-Galerkin / finite-volume scheme of
 * arXiv 2502.19342 (Section 3): per element e with degree N_e and blending
 * factor alpha_e in [0, 1]
 *
 *     d u_e / dt = R_e(u) = (1 - alpha_e) R^DG_e(u) + alpha_e R^FV_e(u)
 *
 * where R^DG is the split-form DGSEM of eq. semidiscrete (flux differencing
 * with a two-point flux on LGL nodes, Section 3.5) with Riemann fluxes and the
 * surface lift at element faces, and R^FV the sub-cell finite-volume operator
 * of eq. semidiscrete_fv reached through the V^{DG->FV} / V^{FV->DG} maps
 * (Section 3.2).  Faces between elements of different degree use the
 * interpolation V^{N->M} / modal projection V^{M->N} of Section 3.2.1.
 * Only the inviscid (Euler) part of eq. ns_equation is implemented, for one
 * species (n_var = 5) or two ideal-gas species (n_var = 6, eq. mix_R_kappa).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Device pointers (suffix _d) are HIP device pointers to contiguous FP64
 *   memory owned by the caller.  The library never frees them and keeps no
 *   reference to them after the call returns.
 * - State layout (structure of arrays):
 *       u[v * n_node + elem_offset[e] + (k * (N_e+1) + j) * (N_e+1) + i]
 *   v = 0..n_var-1 over (rho, rho v1, rho v2, rho v3, rho e[, rho Y1]),
 *   (i, j, k) the LGL node indices along xi1, xi2, xi3, elem_offset[e] the
 *   prefix sum of (N_e+1)^3 in element order (dgfv_mesh_info).
 * - `stream` is a hipStream_t (NULL = the default stream).  Compute calls
 *   only enqueue work; they return before it finishes.  Faults inside kernels
 *   surface at the caller's next synchronisation, as HIP defines.
 * - Every call returns a status; no C++ exception crosses the ABI.  Argument
 *   errors are detected synchronously and leave all buffers untouched.
 *   dgfv_last_error() gives a text for the last non-OK status of the thread.
 * - A mesh object owns scratch buffers: calls on one mesh must not overlap
 *   (use one stream per mesh, or synchronise).
 */
#ifndef DGFV_H
#define DGFV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgfv_mesh dgfv_mesh; /* opaque; owns device geometry and scratch */

typedef enum {
  DGFV_OK = 0,
  DGFV_ERR_ARG = 1,         /* invalid argument (null pointer, range, shape)   */
  DGFV_ERR_UNSUPPORTED = 2, /* valid but not implemented (degree, flux combo)  */
  DGFV_ERR_HIP = 3,         /* a HIP runtime call failed                       */
  DGFV_ERR_OOM = 4,         /* device allocation failed                        */
  DGFV_ERR_STATE = 5        /* non-physical state (rho <= 0, p <= 0 or NaN)   */
} dgfv_status;

/* Two-point volume fluxes (Section 3.5). */
enum { DGFV_VOL_RANOCHA = 0,   /* entropy-conserving + kinetic-energy-preserving, 1 species */
       DGFV_VOL_PIROZZOLI = 1, /* kinetic-energy-preserving flux of Pirozzoli                */
       DGFV_VOL_CENTRAL = 2 }; /* arithmetic mean of the physical fluxes                     */
/* Numerical (Riemann) fluxes at faces (eq. conv_flux). */
enum { DGFV_RIEMANN_ROE_HH = 0, /* Roe with the Harten-Hyman entropy fix, 1 species */
       DGFV_RIEMANN_LLF = 1,    /* local Lax-Friedrichs                              */
       DGFV_RIEMANN_EC = 2 };   /* the volume two-point flux used at the face        */

/*
 * Mesh description (host arrays, copied by dgfv_mesh_create).
 * Geometry: trilinear hexahedra.  corners[e][c][3] with corner c at local
 * reference coordinates xi_d = -1 + 2 * bit_d(c) (bit 0 -> xi1, 1 -> xi2, 2 -> xi3).
 * Faces: faces[f] = {eL, sideL, eR, sideR, orient}; side s is xi_{s/2} = -1 (s even)
 * or +1 (s odd).  A face grid index (p, q) runs p along the lower tangential
 * reference direction, q along the higher one.  `orient` maps the left
 * side's (p, q) on an n x n grid to the right side's (p', q'): (a, b) = (q, p)
 * if bit 2 is set, else (p, q); then p' = n-1-a if bit 0, else a; q' = n-1-b
 * if bit 1, else b.  Every element side must appear in exactly one face or
 * mortar (periodic meshes).
 * Mortars (non-conforming faces, Section 3.2.3, fig. mortarTypes): row
 * {e0, s0, type, e_0..e_3, s_0..s_3, o_0..o_3} gives a big side (element e0,
 * side s0) and its small sides.  Type 1 splits the big side's face grid along
 * p into halves k = 0 (p in [-1, 0]) and 1; type 2 along q; type 3 both, into
 * quarters k = kp + 2 kq.  o_k maps the half's (or quarter's) face grid, p and
 * q along the big side's, to the small side's grid as `orient` does for a
 * face with the big side on the left; unused entries are -1.  The big side's
 * flux follows the paper's five steps for DG sides, and their FV variants
 * where either side is blended (see dgfv_mesh_create).  Meshes with
 * mortars need metric_degree >= 1 (>= 2 on curved elements, where the face
 * normals of a small side must be the restriction of the big side's); they
 * take no face fusion (DGFV_ERR_UNSUPPORTED); the adjoint takes them pure
 * DG with one degree across each mortar.  FV-stored elements at mortars (see
 * dg_rhs_fv) take the FV variants with the reconstruction.
 * Viscous terms at mortars (see dgfv_set_transport) go through the same
 * virtual small sides.
 * Metrics Ja^d are formed in the conservative curl form (Section 3.1.1):
 *  - metric_degree >= 1 (at most min N_e): on the degree-metric_degree nodes,
 *    interpolated to each element's degree;
 *  - metric_degree == 0: at each element's own degree.  On a face shared with
 *    a neighbour of lower degree Nf, the two tangential components of
 *    X_l grad X_m on the face are replaced by their degree-Nf interpolant
 *    before the curl, so both sides hold the same face normal polynomial
 *    (free-stream preservation across degree jumps); formed in long double
 *    and rounded once.  Exact for trilinear elements where the element and
 *    the neighbour across each face have degree >= 2.
 */
typedef struct {
  int32_t n_elem;
  int32_t n_var;           /* 5 (Euler) or 6 (two species, rho*Y1 last) */
  const int8_t* degree;    /* [n_elem], 1..7                            */
  const double* corners;   /* [n_elem][8][3]                            */
  int32_t n_face;
  const int32_t* faces;    /* [n_face][5]                               */
  int32_t n_fv;            /* FV sub-cells per direction, max(N_e)+1 .. 8 */
  int32_t metric_degree;   /* N_J, 1 <= N_J <= min(N_e), or 0: per element */
  double gamma;            /* ratio of specific heats, n_var = 5        */
  double kappa[2];         /* species heat-capacity ratios, n_var = 6   */
  double R[2];             /* species gas constants, n_var = 6          */
  int32_t n_mortar;        /* non-conforming faces (0: a conforming mesh) */
  const int32_t* mortars;  /* [n_mortar][15], see below, or NULL        */
} dgfv_mesh_desc;

typedef struct {
  int32_t volume_flux;     /* DGFV_VOL_*                                           */
  int32_t face_flux_dg;    /* DGFV_RIEMANN_* at faces between two DG (alpha=0) sides */
  int32_t face_flux_fv;    /* DGFV_RIEMANN_* at FV faces and inside sub-cell grids   */
  int32_t ind_vars;        /* indicator variables: bit 0 p, bit 1 rho, bit 2 Y1    */
  double ind_T;            /* blending ramp centre on the indicator I              */
  double ind_dT;           /* blending ramp half-width (> 0)                       */
} dgfv_params;

/* Build the device geometry of a mesh (synchronous; allocates device memory).
 * Mortar faces: for each small side k of a big side of degree N0, the big
 * trace is interpolated to the half (quarter) k, M_0k(xi) = l_j((xi + 2k - 1)/2)
 * along the split directions; it and the small side's trace (degree N_k) go to
 * the common degree max(N0, N_k); the Riemann flux of the DG faces is taken
 * there with the small side's outward normal reversed; the small side
 * receives its projection to N_k, reversed; the big side receives the
 * projection to N0 mapped with M_k0, the L2 projection of twice the half's
 * flux per split direction (the half's surface element is half the big
 * side's), summed over k.  Where either side is blended (alpha > 0, the FV
 * variants) the flux is taken on the small side's N_FV^2 sub-face grid
 * instead, with the FV Riemann flux: the big side's boundary sub-cell means
 * averaged over each sub-face of the half by overlap (a DG big side: its
 * half's trace through V^{DG->FV}), the small side's boundary sub-cell means
 * (or V^{DG->FV} of its trace), and h^2 V^{DG->FV} of the reversed normal.
 * The small side receives it reversed (its DG part through V^{FV->DG} / h^2);
 * the big side's DG part receives V^{FV->DG} of it / h^2 mapped with M_k0,
 * a blended big side's FV part the sub-face fluxes summed by overlap. */
dgfv_status dgfv_mesh_create(const dgfv_mesh_desc* desc, dgfv_mesh** out);
void dgfv_mesh_destroy(dgfv_mesh* mesh);

/* Node count and (optionally, host array of n_elem+1) element node offsets. */
dgfv_status dgfv_mesh_info(const dgfv_mesh* mesh, int64_t* n_node, int64_t* elem_offset);

/* Physical node coordinates, host array [3][n_node] (synchronous). */
dgfv_status dgfv_mesh_node_coords(const dgfv_mesh* mesh, double* xyz);

/*
 * Modal decay indicator (Section 3.4, eq. modal_contribution .. eq. modal_indicator)
 * and blending factor.  Per element: the variables selected by params->ind_vars
 * are transformed to the orthonormal Legendre basis; the share w_m of mode m
 * per direction is fitted by a least-squares line through (m, ln max(w_m, 1e-30)),
 * I = min over directions (and variables) of |slope|; energies below 1e-300 give
 * I = +inf.  alpha = 1 for I <= T - dT, 0 for I >= T + dT, and
 * (1 - sin(pi (I - T) / (2 dT))) / 2 between.
 * alpha_d: [n_elem] output.  ind_d: [n_elem] output, may be NULL.
 */
dgfv_status dg_indicator(const dgfv_mesh* mesh, const dgfv_params* params, const double* u_d,
                         double* alpha_d, double* ind_d, void* stream);

/*
 * ut = R(u) with blending factors alpha (eq. semidiscrete, eq. semidiscrete_fv,
 * Section 3.2).  alpha_d: [n_elem] in [0, 1]; NULL means all zero (pure DG).
 * u_d, ut_d: [n_var][n_node]; they must not overlap.
 */
dgfv_status dg_rhs(const dgfv_mesh* mesh, const dgfv_params* params, const double* u_d,
                   const double* alpha_d, double* ut_d, void* stream);

/*
 * One stage of the five-stage fourth-order 2N-storage Runge-Kutta scheme
 * (Section 3.3; Carpenter-Kennedy coefficients A_s, B_s):
 *     k <- A_s k + dt R(u),  u <- u + B_s k,   stage = 1..5.
 * Stage 1 writes k = dt R(u) without reading k.  u_d and k_d are updated in
 * place; alpha_d as for dg_rhs (frozen over the stages of a step).
 */
dgfv_status dg_rk_stage(const dgfv_mesh* mesh, const dgfv_params* params, int stage, double dt,
                        double* u_d, double* k_d, const double* alpha_d, void* stream);

/*
 * One whole Runge-Kutta step: stages 1..5 of dg_rk_stage in order, with the
 * same arguments and in-place updates (k need not be initialised).
 */
dgfv_status dg_rk_step(const dgfv_mesh* mesh, const dgfv_params* params, double dt, double* u_d,
                       double* k_d, const double* alpha_d, void* stream);

/*
 * Positivity-preserving limiter of Zhang and Shu (Section 3.5), one species.
 * Per element, with the mean ubar = sum w J u / sum w J (which it keeps), every
 * point value becomes ubar + theta (u_P - ubar): first the density alone, with
 * the largest theta_rho <= 1 that keeps rho_P >= eps at every point, then all
 * variables with the largest theta_p <= 1 that keeps p_P >= eps (the exact
 * root of a quadratic per point).  eps = 1e-10 rhobar for the density and
 * 1e-10 p(ubar) for the pressure.  The points are the LGL nodes and, on
 * elements with alpha > 0 (alpha_d may be NULL), the J-weighted sub-cell means
 * that the FV operator evaluates.  u_d is updated in place; an element within
 * the bounds is not written.  theta_d (nullable, [n_elem]) receives
 * min(theta_rho, theta_p), or -1 where the mean itself has rho <= 0 or p <= 0
 * (left as it is).  DGFV_ERR_UNSUPPORTED for two species.
 */
dgfv_status dg_positivity_limiter(const dgfv_mesh* mesh, const dgfv_params* params, double* u_d,
                                  const double* alpha_d, double* theta_d, void* stream);

/*
 * With enable != 0, dg_rk_stage and dg_rk_step apply dg_positivity_limiter to
 * u after every stage (with the stage's alpha; cached graphs are dropped).
 */
dgfv_status dgfv_set_positivity_limiter(dgfv_mesh* mesh, int enable);

/*
 * Non-physical states (failure detection, not part of the method).  The
 * element kernels of dg_rhs, dg_rk_stage and dg_rk_step set a flag of the mesh
 * when a node of the state they read has rho <= 0, p <= 0 or a NaN in either
 * (the RK stages read the previous stage's output, so a bad step shows in the
 * next call).  Each of these calls then copies the flag to pinned host memory
 * behind an event on its stream, without waiting.  A later call on the mesh
 * whose predecessor's copy has completed returns DGFV_ERR_STATE, clears the
 * flag, and enqueues nothing; the caller decides (e.g. a smaller dt from a
 * stored state).  Nothing is copied while the caller captures the stream.
 * dgfv_check_state synchronises `stream`, returns DGFV_ERR_STATE if the flag
 * is set (and clears it), else DGFV_OK.
 */
dgfv_status dgfv_check_state(dgfv_mesh* mesh, void* stream);

/*
 * Launch batching (not part of the method).  Within each phase of an
 * evaluation (sub-cell means, face fluxes, FV residuals, element kernels) the
 * launches of the different degree buckets and face classes are independent.
 *   DGFV_LAUNCH_SERIAL:   all launches in order on the caller's stream;
 *   DGFV_LAUNCH_BRANCHES: (default) the launches of a phase fork from the
 *                         caller's stream onto streams owned by the mesh and
 *                         join back, so that small buckets run side by side;
 *   DGFV_LAUNCH_GRAPH:    as BRANCHES, but dg_rk_step and dg_rk_stage capture
 *                         their launches into a hipGraph once per argument set
 *                         (params, stage, dt and the u, k, alpha pointers) and
 *                         replay it on later calls.  Up to 16 graphs are cached
 *                         per mesh (the oldest is dropped); leaving this mode
 *                         frees them.  Graphs are not used while profiling is on.
 * Capture and instantiation errors are reported as DGFV_ERR_HIP.
 */
enum { DGFV_LAUNCH_SERIAL = 0, DGFV_LAUNCH_BRANCHES = 1, DGFV_LAUNCH_GRAPH = 2 };
dgfv_status dgfv_set_launch_mode(dgfv_mesh* mesh, int mode);

/*
 * FV-stored elements (Section 3.1.2, eq. semidiscrete_fv; Section 3.2).
 * An element with fv_d[e] > 0 carries, instead of its nodal DG state, the
 * means of N_FV^3 equidistant reference sub-cells (N_FV = the mesh's n_fv, up
 * to 8: any N_FV >= N + 1 of the paper's range up to 2 N_max + 1 that fits,
 * e.g. 2N+1 for N <= 3):
 *   ufv_d: [n_elem][n_var][N_FV^3] device doubles, sub-cell (s1, s2, s3) at
 *          (s3 N_FV + s2) N_FV + s1; read and written only on FV elements;
 *   fv_d:  [n_elem] device doubles, > 0 on FV elements, 0 on DG elements.
 * The means are J-weighted, ufv = V3(J u) / V3(J).  Their rate is minus the sum
 * of the six sub-face fluxes over h^3 V3(J) (h = 2 / N_FV), each flux taken
 * between states reconstructed to the sub-face: per reference direction the
 * slope of a sub-cell's primitive variables (rho, v, p[, Y1]) is the minmod of
 * its backward and forward differences, and across an element side the
 * neighbour is the adjacent sub-cell mean of an FV element or the DG
 * element's nodal trace mapped with V^{DG->FV} in both face directions
 * (fig. h_coupling); a DG side's own value on such a face is that mapped
 * trace, and it receives the flux through V^{FV->DG} / h^2.  Faces between two
 * DG elements, and the DG elements, are as in dg_rhs with alpha = 0; the
 * nodal slots of FV elements are neither read nor written.  At a mortar
 * (Section 3.2.3) a half with an FV side takes the flux on the small side's
 * sub-face grid: an FV small side's ghost is the big side's data on its half
 * (boundary means through the overlap map, or the mapped half trace of a DG
 * big side), an FV big side's ghost on each of its sub-faces the mean of the
 * small sides' boundary data over it, and its reconstructed values reach the
 * halves by overlap; the small side takes the flux reversed, the big side the
 * sub-face fluxes summed by overlap (FV) or M_k0 of their V^{FV->DG} / h^2 (DG).
 *   dg_rhs_fv:      ut_d = R(u) on DG elements, utfv_d = R(ufv) on FV elements;
 *   dg_rk_stage_fv: stage s of dg_rk_stage on (u, k) and on (ufv, kfv);
 *   dg_rk_step_fv:  the five stages in turn (between them the DG faces read the
 *                   xi_1 sides from traces the previous stage wrote, as in
 *                   dg_rk_step);
 *   dg_switch_fv:   converts the elements whose flag goes from fv_old_d to
 *                   fv_new_d: DG -> FV ufv = V3(J u) / V3(J); FV -> DG
 *                   u = V3^+(ufv V3(J)) / J (the least-squares nodal state
 *                   with those sub-cell contents; exact inverse for
 *                   N_FV = N + 1).  Other elements are untouched.
 * The first call allocates the mesh's ghost-layer buffer (n_elem 6 n_var N_FV^2
 * doubles) and V3(J) (n_elem N_FV^3): DGFV_ERR_ARG while the stream is
 * captured, DGFV_ERR_OOM when the memory is short.  No positivity limiter and
 * no graphs on this path.
 */
dgfv_status dg_rhs_fv(const dgfv_mesh* mesh, const dgfv_params* params, const double* u_d, const double* ufv_d,
                      const double* fv_d, double* ut_d, double* utfv_d, void* stream);
dgfv_status dg_rk_stage_fv(const dgfv_mesh* mesh, const dgfv_params* params, int stage, double dt, double* u_d,
                           double* k_d, double* ufv_d, double* kfv_d, const double* fv_d, void* stream);
dgfv_status dg_rk_step_fv(const dgfv_mesh* mesh, const dgfv_params* params, double dt, double* u_d, double* k_d,
                          double* ufv_d, double* kfv_d, const double* fv_d, void* stream);
dgfv_status dg_switch_fv(const dgfv_mesh* mesh, double* u_d, double* ufv_d, const double* fv_old_d,
                         const double* fv_new_d, void* stream);

/*
 * Dynamic p-adaptation (Section 3.4: I_p-adapt = I(rho); Section 3.2: the maps
 * between ansatz degrees).
 * dg_p_degrees: the modal decay indicator of the density (as dg_indicator with
 *   the density selected, whatever params->ind_vars) decides each element's next
 *   degree: I < t_refine raises N by one, I > t_coarsen lowers it by one,
 *   clamped to [n_min, n_max] (t_refine < t_coarsen; I = +inf coarsens).
 *   degree_out: host int8 [n_elem].  Synchronous: the call waits for the
 *   indicator on `stream` (DGFV_ERR_ARG while the stream is captured).
 * The caller then builds the mesh of the new degrees with dgfv_mesh_create (the
 *   same corners, faces and constants; a mesh-wide metric degree above the new
 *   lowest degree must come down): the new mesh has its own degree buckets, work
 *   lists and graph cache.
 * dg_transfer_degree: u_to_d (layout of mesh `to`) from u_from_d (layout of mesh
 *   `from`), element by element along each reference direction: interpolation
 *   V^{N->M} to a higher degree (exact), the modal L2 truncation V^{M->N} to a
 *   lower one (keeps the Legendre modes up to the lower degree), the identity
 *   where the degree stays; on the conservative state.  Constants are kept
 *   exactly, and on affine elements every element's content.  The meshes must
 *   have the same n_elem and n_var.  The first transfer into a mesh uploads the
 *   maps (32 KB; DGFV_ERR_ARG while the stream is captured).
 */
dgfv_status dg_p_degrees(const dgfv_mesh* mesh, const dgfv_params* params, const double* u_d, double t_refine,
                         double t_coarsen, int n_min, int n_max, int8_t* degree_out, void* stream);
dgfv_status dg_transfer_degree(const dgfv_mesh* from, const dgfv_mesh* to, const double* u_from_d, double* u_to_d,
                               void* stream);

/*
 * Fused face fluxes (not part of the method; off by default).  Elements of
 * degree 6 and 7 evaluate the Riemann flux (eq. conv_flux) of each face they
 * share with a pure DG element of the same degree themselves, with the same
 * operands and operations as the face kernel, instead of reading it from the
 * side buffer the face kernel fills: one launch and one round trip of the
 * side fluxes less.  The element then reads its neighbour's state while the
 * launch runs, so no launch may write the state it reads: dg_rhs fuses
 * always; dg_rk_step alternates its stages between u and a second state
 * buffer owned by the mesh (n_var x n_node doubles, allocated by the first
 * such call, never while the stream is captured; without it the stages run in
 * place, unfused), and runs the fifth stage in place and unfused; dg_rk_stage
 * never fuses.  Results are those of the unfused path to rounding (the
 * compiler may contract the flux's products and sums differently in the two
 * kernels).  Changing the setting drops the mesh's cached graphs.  On the
 * 64^3 N=7 shear-layer workload the fused stages take as long as the separate
 * kernels: the element kernel gains the face flux on its critical path, and
 * the FV faces lose the conforming face kernel they overlapped with.
 */
dgfv_status dgfv_set_face_fusion(dgfv_mesh* mesh, int enable);

/*
 * Viscous multi-species Navier-Stokes terms (Section 2, eq. visc_stress,
 * eq. fourier_law, eq. enthalpy_flux, eq. fickian_law, eq. mix_lambda_mu;
 * Section 3.1.1, eq. lift_weak, eq. semidiscrete_lift, eq. lift_flux,
 * eq. visc_flux; Section 3.2.2 for degree jumps).
 *
 * dgfv_set_transport sets constant species transport coefficients and turns
 * the viscous terms on for every later dg_rhs, dg_rk_stage and dg_rk_step on
 * the mesh (tr = NULL turns them off).  Index 0 is the species weighted by Y1
 * (the only one for n_var = 5), index 1 the other: mixture mu and Pr mix
 * linearly in Y, lambda = mu c_p / Pr; D are the Fickian diffusivities, with
 * the mass-conserving correction (the species fluxes sum to zero).  One
 * species takes its temperature from p / rho with a unit gas constant, which
 * cancels in the heat flux.  The first call allocates 3 n_var n_node doubles
 * (the lifted gradient), n_var n_node (the viscous rate) and one side buffer
 * (synchronous; DGFV_ERR_OOM when they do not fit); changing the setting
 * drops the mesh's cached graphs.  mu, D >= 0 and Pr > 0, finite, else
 * DGFV_ERR_ARG.
 *
 * The rate becomes R = (1 - alpha) R^c_DG + alpha R^c_FV + R^v: the BR1
 * operator R^v acts on every element, the sub-cell blending on the
 * convective part.  R^v: the conservative state is lifted to its gradient g
 * (the face value u* = (u^- + u^+)/2 formed on the lower degree of a degree
 * jump and interpolated to the higher side); the viscous fluxes of (u, g)
 * meet at each face in their arithmetic mean on the higher degree, the lower
 * side receiving the projection.  At a mortar both terms use its virtual
 * small sides (Section 3.2.3): on half (quarter) k the big side's traces
 * mapped with M_0k meet the small side's as at a conforming face (u* on the
 * lower degree; the fluxes with the small side's normal reversed, on the
 * higher), and the big side takes (1/2)^s sum_k M_k0 u*_k for its face value
 * (s split directions) and sum_k M_k0 of the flux.  Face fusion is off while the viscous terms
 * are on; the FV-stored calls (dg_rhs_fv and its stages) and the adjoint
 * return DGFV_ERR_UNSUPPORTED.
 *
 * dg_lift writes the lifted gradient of u_d alone, g_d [3][n_var][n_node]
 * (d u_v / d x_x at component x * n_var + v), for inspection; DGFV_ERR_ARG
 * when no transport coefficients are set.  Enqueued on `stream`.
 */
typedef struct {
  double mu[2];            /* dynamic viscosities      */
  double Pr[2];            /* Prandtl numbers          */
  double D[2];             /* diffusion coefficients   */
} dgfv_transport;
dgfv_status dgfv_set_transport(dgfv_mesh* mesh, const dgfv_transport* tr);
dgfv_status dg_lift(const dgfv_mesh* mesh, const double* u_d, double* g_d, void* stream);

/*
 * Time step of Section 3.3 for u_d (and the blending factors alpha_d, or
 * NULL), with alpha_RK = beta_RK = 1: the convective step
 *   dt^c = min_e 2 / ((2 N_e + 1) lambda^c_e),
 *   lambda^c_e = max over e's nodes of sum_d (|v . Ja^d| + c |Ja^d|) / J,
 * a blended element (alpha > 0) also bounded by h_FV / lambda^c_e with the
 * sub-cell spacing h_FV = 2 / N_FV; with viscous terms (dgfv_set_transport)
 * the parabolic step
 *   dt^v = min_e 4 / ((2 N_e + 1) lambda^v_e),
 *   lambda^v_e = max over e's nodes of delta sum_d |Ja^d|^2 / J^2,
 *   delta = max(4/3 mu / rho, kappa mu / (Pr rho), D_1, D_2),
 * a blended element also bounded by h_FV^2 / lambda^v_e, and the two join as
 *   *dt = 1 / (1 / (cfl dt^c) + 1 / (cfl_v dt^v));
 * without viscous terms *dt = cfl dt^c (cfl_v unused).  The reference length
 * 2 (squared) stands for the element size, (2N + 1) enters to the first power
 * as printed.  Synchronous: waits for `stream` and copies two doubles; the
 * first call allocates 2 n_elem + 2 doubles; not while the stream is
 * captured (DGFV_ERR_ARG).  cfl (and cfl_v when viscous) positive and finite,
 * else DGFV_ERR_ARG; DGFV_ERR_STATE if the state gives no positive finite step
 * (rho <= 0, p <= 0 or NaN somewhere).
 */
dgfv_status dg_timestep(const dgfv_mesh* mesh, const double* u_d, const double* alpha_d, double cfl,
                        double cfl_v, double* dt, void* stream);

/*
 * Autotuning (not part of the method).  The element kernel has two tile
 * shapes at degrees N <= 5: about 512 or about 256 lanes per workgroup (the
 * number of elements per workgroup).  dgfv_autotune evaluates the RHS once on
 * (u_d, alpha_d), then times each shape of every degree bucket over 5 launches
 * after one warm-up (HIP events on `stream`) and keeps the faster shape per
 * degree for all later calls on the mesh; cached graphs are dropped.
 * Synchronous; allocates and frees one state-sized scratch buffer.
 * ms_out (nullable): host array [8][2], the average launch time (ms) per
 * degree and shape, 0 where not timed.
 */
dgfv_status dgfv_autotune(dgfv_mesh* mesh, const dgfv_params* params, const double* u_d,
                          const double* alpha_d, double* ms_out, void* stream);

/* Sets the element-kernel shape of one degree by hand (0, or 1 where
 * available); DGFV_ERR_ARG for a shape the degree does not have. */
dgfv_status dgfv_set_element_shape(dgfv_mesh* mesh, int degree, int shape);

/*
 * Vector-Jacobian product of the right-hand side with alpha frozen:
 *     g_b = (dR/du (u))^T w_b,  b = 0..batch-1,
 * w_d, g_d: [batch][n_var][n_node]; alpha_d as for dg_rhs.  Derivatives at
 * the switches of the Riemann solvers (entropy fix, max) are those of the
 * branch taken.  Built for alpha_d = NULL (pure DG) on meshes of one degree,
 * mortars included (their fluxes reversed per small side: F_bar = M_k0^T A -
 * b_k, the Riemann flux's VJP at the half's nodes, M_0k^T back to the big
 * side); other cases, and meshes with the viscous terms, return
 * DGFV_ERR_UNSUPPORTED.
 */
dgfv_status dg_rhs_vjp(const dgfv_mesh* mesh, const dgfv_params* params, const double* u_d,
                       const double* alpha_d, const double* w_d, double* g_d, int batch,
                       void* stream);

/*
 * Reverse of one Runge-Kutta stage (Section 3.3) with alpha frozen.  The
 * forward stage s maps (u_{s-1}, k_{s-1}) to k_s = A_s k_{s-1} + dt R(u_{s-1}),
 * u_s = u_{s-1} + B_s k_s.  Given the cotangents ubar of u_s and kbar of k_s,
 * this call replaces them, in place, by those of u_{s-1} and k_{s-1}:
 *     kt = kbar + B_s ubar;  ubar <- ubar + dt (dR/du (u_{s-1}))^T kt;  kbar <- A_s kt
 * (kbar <- 0 at stage 1), with the coefficients of dg_rk_stage.  u_stage_d is
 * u_{s-1}, the state the forward stage read.  All three are [n_var][n_node]
 * and must not overlap; alpha_d as for dg_rhs_vjp.  The first call on a mesh
 * allocates one state-sized buffer, kept by the mesh (synchronous).
 * A multi-step adjoint stores the state at each step start, recomputes the
 * stage inputs with dg_rk_stage and calls this for stages 5..1.
 */
dgfv_status dg_rk_stage_vjp(const dgfv_mesh* mesh, const dgfv_params* params, int stage, double dt,
                            const double* u_stage_d, double* ubar_d, double* kbar_d, const double* alpha_d,
                            void* stream);

/*
 * dg_rk_stage_vjp for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments and results as dg_rk_stage_vjp, but its state-sized
 * cotangent buffer is a fixed device array of the library (128 MiB, one per
 * GPU, held until the process ends), looked up once per device at mesh
 * creation; the call allocates nothing.  DGFV_ERR_ARG when
 * n_var * n_node > 16777216 (2^24 doubles).  Every call on one GPU shares
 * that array: calls that overlap on one GPU (on any mesh or stream) race.
 */
dgfv_status dg_rk_stage_vjp_noalloc(const dgfv_mesh* mesh, const dgfv_params* params, int stage, double dt,
                                    const double* u_stage_d, double* ubar_d, double* kbar_d,
                                    const double* alpha_d, void* stream);

/*
 * Primitive to conservative variables (Section 2, eq. eos; mixing rules of
 * eq. mix_R_kappa and eq. mix_cp_cv for two species) with the mesh's gas:
 * w_d = (rho, v1, v2, v3, p[, Y1]) -> u_d = (rho, rho v, rho e[, rho Y1]),
 * rho e = p / (kappa - 1) + rho |v|^2 / 2.  Both [n_var][n_node], distinct.
 */
dgfv_status dgfv_prim_to_cons(const dgfv_mesh* mesh, const double* w_d, double* u_d, void* stream);

/*
 * Kernel timing with HIP events (measurement support, not part of the method).
 * dgfv_profile_enable(mesh, 1) clears the counters and makes every later call
 * on the mesh record an event pair around each phase below, on the stream the
 * phase runs on; 0 stops recording.  dgfv_profile_read synchronises the
 * recorded events and returns the summed duration (ms) and the count of one
 * class.  FV_FACE lies inside the FACE interval (in the concurrent launch
 * modes it runs beside the DG face fluxes).
 */
enum { DGFV_KERNEL_ELEMENT = 0,     /* volume + lift + blend (+ RK update), all degree buckets   */
       DGFV_KERNEL_FACE = 1,        /* face phase: every interface flux; with alpha on a mesh     */
                                    /* without mortars it holds the FV chain (means, FV faces,    */
                                    /* FV residuals) as a branch beside the DG face classes,      */
                                    /* except in graph replays of meshes with several degrees     */
       DGFV_KERNEL_FV_MEANS = 2,    /* blended list + sub-cell means                             */
       DGFV_KERNEL_FV_RESIDUAL = 3, /* FV sub-cell residuals                                     */
       DGFV_KERNEL_INDICATOR = 4,
       DGFV_KERNEL_VJP = 5,
       DGFV_KERNEL_FV_FACE = 6,     /* fluxes of the faces with a blended side                   */
       DGFV_KERNEL_VISCOUS = 7,     /* viscous terms: lifting, viscous face fluxes and rates     */
       DGFV_KERNEL_COUNT = 8 };
dgfv_status dgfv_profile_enable(dgfv_mesh* mesh, int enable);
dgfv_status dgfv_profile_read(dgfv_mesh* mesh, int kernel, double* total_ms, int64_t* launches);

/* Text of the last non-OK status returned to this thread. */
const char* dgfv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGFV_H */
