"""Python binding of the C ABI in ``include/dgfv.h`` (argument marshalling only).

Every computation runs in the HIP library ``libdgfv.so``; this module only
converts mesh descriptions to the C structs, checks tensor shapes, dtypes and
devices, and passes device pointers and the current HIP stream.  Importing it
without the built library raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgfv.so")

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_OOM, ERR_STATE = range(6)


class DgfvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dgfv status {status}: {msg}")
        self.status = status


class _MeshDesc(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("n_var", ctypes.c_int32),
                ("degree", ctypes.POINTER(ctypes.c_int8)), ("corners", ctypes.POINTER(ctypes.c_double)),
                ("n_face", ctypes.c_int32), ("faces", ctypes.POINTER(ctypes.c_int32)),
                ("n_fv", ctypes.c_int32), ("metric_degree", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("kappa", ctypes.c_double * 2), ("R", ctypes.c_double * 2),
                ("n_mortar", ctypes.c_int32), ("mortars", ctypes.POINTER(ctypes.c_int32))]


class _Params(ctypes.Structure):
    _fields_ = [("volume_flux", ctypes.c_int32), ("face_flux_dg", ctypes.c_int32),
                ("face_flux_fv", ctypes.c_int32), ("ind_vars", ctypes.c_int32),
                ("ind_T", ctypes.c_double), ("ind_dT", ctypes.c_double)]


class _Transport(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double * 2), ("Pr", ctypes.c_double * 2), ("D", ctypes.c_double * 2)]


EXPORTED = ("dgfv_mesh_create", "dgfv_mesh_destroy", "dgfv_mesh_info", "dgfv_mesh_node_coords",
            "dg_indicator", "dg_rhs", "dg_rk_stage", "dg_rk_step", "dg_rhs_vjp", "dg_rk_stage_vjp",
            "dg_rk_stage_vjp_noalloc", "dgfv_prim_to_cons", "dg_positivity_limiter",
            "dgfv_set_positivity_limiter", "dgfv_set_launch_mode", "dgfv_set_face_fusion", "dgfv_autotune",
            "dgfv_set_element_shape", "dgfv_check_state", "dg_rhs_fv", "dg_rk_stage_fv", "dg_rk_step_fv",
            "dg_switch_fv", "dg_p_degrees", "dg_transfer_degree", "dgfv_set_transport", "dg_lift", "dg_timestep",
            "dgfv_profile_enable", "dgfv_profile_read", "dgfv_last_error")
(KERNEL_ELEMENT, KERNEL_FACE, KERNEL_FV_MEANS, KERNEL_FV_RESIDUAL, KERNEL_INDICATOR, KERNEL_VJP, KERNEL_FV_FACE,
 KERNEL_VISCOUS) = range(8)
LAUNCH_SERIAL, LAUNCH_BRANCHES, LAUNCH_GRAPH = range(3)


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2502_19342_amd.build`")
    lib = ctypes.CDLL(path)
    P, c_int, c_double = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.dgfv_mesh_create.argtypes = [ctypes.POINTER(_MeshDesc), ctypes.POINTER(P)]
    lib.dgfv_mesh_destroy.argtypes = [P]
    lib.dgfv_mesh_destroy.restype = None
    lib.dgfv_mesh_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.dgfv_mesh_node_coords.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.dg_indicator.argtypes = [P, ctypes.POINTER(_Params), P, P, P, P]
    lib.dg_rhs.argtypes = [P, ctypes.POINTER(_Params), P, P, P, P]
    lib.dg_rk_stage.argtypes = [P, ctypes.POINTER(_Params), c_int, c_double, P, P, P, P]
    lib.dg_rk_step.argtypes = [P, ctypes.POINTER(_Params), c_double, P, P, P, P]
    lib.dg_rhs_vjp.argtypes = [P, ctypes.POINTER(_Params), P, P, P, P, c_int, P]
    lib.dg_rk_stage_vjp.argtypes = [P, ctypes.POINTER(_Params), c_int, c_double, P, P, P, P, P]
    lib.dg_rk_stage_vjp_noalloc.argtypes = [P, ctypes.POINTER(_Params), c_int, c_double, P, P, P, P, P]
    lib.dgfv_prim_to_cons.argtypes = [P, P, P, P]
    lib.dg_positivity_limiter.argtypes = [P, ctypes.POINTER(_Params), P, P, P, P]
    lib.dgfv_set_positivity_limiter.argtypes = [P, c_int]
    lib.dgfv_set_launch_mode.argtypes = [P, c_int]
    lib.dgfv_set_face_fusion.argtypes = [P, c_int]
    lib.dg_rhs_fv.argtypes = [P, ctypes.POINTER(_Params), P, P, P, P, P, P]
    lib.dg_rk_stage_fv.argtypes = [P, ctypes.POINTER(_Params), c_int, c_double, P, P, P, P, P, P]
    lib.dg_rk_step_fv.argtypes = [P, ctypes.POINTER(_Params), c_double, P, P, P, P, P, P]
    lib.dg_switch_fv.argtypes = [P, P, P, P, P, P]
    lib.dg_p_degrees.argtypes = [P, ctypes.POINTER(_Params), P, c_double, c_double, c_int, c_int,
                                 ctypes.POINTER(ctypes.c_int8), P]
    lib.dg_transfer_degree.argtypes = [P, P, P, P, P]
    lib.dgfv_set_element_shape.argtypes = [P, c_int, c_int]
    lib.dgfv_set_transport.argtypes = [P, ctypes.POINTER(_Transport)]
    lib.dg_lift.argtypes = [P, P, P, P]
    lib.dg_timestep.argtypes = [P, P, P, c_double, c_double, ctypes.POINTER(ctypes.c_double), P]
    lib.dgfv_autotune.argtypes = [P, ctypes.POINTER(_Params), P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.dgfv_profile_enable.argtypes = [P, c_int]
    lib.dgfv_profile_read.argtypes = [P, c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.dgfv_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("dgfv_mesh_destroy", "dgfv_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = load_library()


def _check(status: int):
    if status != OK:
        raise DgfvError(status, _lib.dgfv_last_error().decode())


@dataclass
class Params:
    volume_flux: int = 0
    face_flux_dg: int = 0
    face_flux_fv: int = 1
    ind_vars: int = 1
    ind_T: float = 2.0
    ind_dT: float = 1.0

    def c(self) -> _Params:
        return _Params(self.volume_flux, self.face_flux_dg, self.face_flux_fv, self.ind_vars,
                       float(self.ind_T), float(self.ind_dT))


def params_of(wl) -> Params:
    return Params(wl.volume_flux, wl.face_flux_dg, wl.face_flux_fv, wl.ind_vars, wl.ind_T, wl.ind_dT)


class Mesh:
    """Device geometry of a hexahedral mesh (owns the library handle); ``mortars`` lists its
    non-conforming faces ([M, 15] rows, ``workloads.mortar_mesh``), if any."""

    def __init__(self, degree, corners, faces, n_var=5, n_fv=None, metric_degree=1, gamma=1.4,
                 kappa=(1.4, 1.4), R=(287.0, 287.0), mortars=None):
        self.degree = np.ascontiguousarray(degree, dtype=np.int8)
        self.corners = np.ascontiguousarray(corners, dtype=np.float64)
        self.faces = np.ascontiguousarray(faces, dtype=np.int32)
        self.mortars = np.ascontiguousarray(np.zeros((0, 15)) if mortars is None else mortars,
                                            dtype=np.int32).reshape(-1, 15)
        K = self.degree.shape[0]
        if self.corners.shape != (K, 8, 3) or self.faces.ndim != 2 or self.faces.shape[1] != 5:
            raise ValueError("corners must be [K,8,3] and faces [F,5]")
        self.n_elem = K
        self.n_var = int(n_var)
        self.n_fv = int(n_fv if n_fv is not None else int(self.degree.max()) + 1)
        self._args = dict(n_var=self.n_var, n_fv=self.n_fv, metric_degree=int(metric_degree), gamma=float(gamma),
                          kappa=tuple(kappa), R=tuple(R), mortars=self.mortars)
        desc = _MeshDesc(K, self.n_var, self.degree.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                         self.corners.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self.faces.shape[0], self.faces.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         self.n_fv, int(metric_degree), float(gamma),
                         (ctypes.c_double * 2)(*kappa), (ctypes.c_double * 2)(*R), self.mortars.shape[0],
                         self.mortars.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if len(self.mortars) else None)
        h = ctypes.c_void_p()
        _check(_lib.dgfv_mesh_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        off = np.zeros(K + 1, dtype=np.int64)
        _check(_lib.dgfv_mesh_info(h, ctypes.byref(n), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        self.n_node = int(n.value)
        self.elem_offset = off

    @classmethod
    def from_config(cls, cfg: str, **kw) -> "Mesh":
        """Mesh of a named seeded workload (C1..C5; keyword arguments as for
        ``workloads.make_workload``)."""
        from . import workloads as W
        return cls.from_workload(W.make_workload(cfg, **kw))

    @classmethod
    def from_workload(cls, wl) -> "Mesh":
        m = wl.mesh
        mesh = cls(m.degree, m.corners, m.faces, wl.n_var, wl.n_fv, wl.metric_degree, wl.gamma,
                   tuple(wl.kappa), tuple(wl.R), getattr(m, "mortars", None))
        if getattr(wl, "viscous", False):
            mesh.transport(wl.mu, wl.Pr, wl.D)
        return mesh

    def transport(self, mu=None, Pr=(0.72, 0.72), D=(0.0, 0.0)) -> None:
        """Viscous terms with these species coefficients, or off with ``mu=None`` (``dgfv_set_transport``)."""
        if mu is None:
            _check(_lib.dgfv_set_transport(self._h, None))
            self._transport = None
            return
        tr = _Transport((ctypes.c_double * 2)(*mu), (ctypes.c_double * 2)(*Pr), (ctypes.c_double * 2)(*D))
        _check(_lib.dgfv_set_transport(self._h, ctypes.byref(tr)))
        self._transport = (tuple(mu), tuple(Pr), tuple(D))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.dgfv_mesh_destroy(h)
            self._h = None

    def redegree(self, degree) -> "Mesh":
        """The mesh of the same elements at new degrees (a mesh-wide metric degree
        above the new lowest degree comes down to it)."""
        kw = dict(self._args)
        if kw["metric_degree"] > 0:
            kw["metric_degree"] = min(kw["metric_degree"], int(np.min(degree)))
        out = Mesh(degree, self.corners, self.faces, **kw)
        if getattr(self, "_transport", None) is not None:
            out.transport(*self._transport)
        return out

    def launch_mode(self, mode: int) -> None:
        """LAUNCH_SERIAL, LAUNCH_BRANCHES (default) or LAUNCH_GRAPH (``dgfv_set_launch_mode``)."""
        _check(_lib.dgfv_set_launch_mode(self._h, int(mode)))

    def autotune(self, params: "Params", u: torch.Tensor, alpha: torch.Tensor | None = None,
                 stream=None) -> dict:
        """Pick the element kernel's tile shape per degree (``dgfv_autotune``).

        Returns ``{N: (ms_shape0, ms_shape1)}`` for the degrees that were timed.
        """
        ms = (ctypes.c_double * 16)()
        _check(_lib.dgfv_autotune(self._h, ctypes.byref(params.c()), self._state(u, "u"), self._alpha(alpha),
                                  ms, _stream(stream)))
        return {N: (ms[2 * N], ms[2 * N + 1]) for N in range(1, 8) if ms[2 * N] > 0}

    def set_element_shape(self, degree: int, shape: int) -> None:
        """Element-kernel tile shape of one degree by hand (``dgfv_set_element_shape``)."""
        _check(_lib.dgfv_set_element_shape(self._h, int(degree), int(shape)))

    def positivity_limiter(self, enable: bool = True) -> None:
        """Apply the positivity limiter after every RK stage (``dgfv_set_positivity_limiter``)."""
        _check(_lib.dgfv_set_positivity_limiter(self._h, int(enable)))

    def face_fusion(self, enable: bool = True) -> None:
        """Element kernels of degree 6, 7 evaluate their conforming DG faces (``dgfv_set_face_fusion``)."""
        _check(_lib.dgfv_set_face_fusion(self._h, int(enable)))

    def graphs(self, enable: bool = True) -> None:
        """Capture and replay RK steps and stages as hipGraphs, or go back to branch launches."""
        self.launch_mode(LAUNCH_GRAPH if enable else LAUNCH_BRANCHES)

    def profile(self, enable: bool = True) -> None:
        """Start (clearing the counters) or stop event timing of every kernel launch."""
        _check(_lib.dgfv_profile_enable(self._h, int(enable)))

    def kernel_time(self, kernel: int):
        """``(total_ms, launches)`` of one kernel class since profiling was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(_lib.dgfv_profile_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def node_coords(self) -> np.ndarray:
        xyz = np.zeros((3, self.n_node), dtype=np.float64)
        _check(_lib.dgfv_mesh_node_coords(self._h, xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return xyz

    # ------------------------------------------------------------------
    def _state(self, t: torch.Tensor, name: str, batch: int | None = None) -> int:
        shape = (self.n_var, self.n_node) if batch is None else (batch, self.n_var, self.n_node)
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}")
        return t.data_ptr()

    def _fv_state(self, t: torch.Tensor, name: str) -> int:
        shape = (self.n_elem, self.n_var, self.n_fv ** 3)
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}")
        return t.data_ptr()

    def _alpha(self, a) -> int | None:
        if a is None:
            return None
        if a.dtype != torch.float64 or not a.is_cuda or tuple(a.shape) != (self.n_elem,) or not a.is_contiguous():
            raise ValueError("alpha must be a contiguous float64 device tensor of shape [n_elem]")
        return a.data_ptr()


def _stream(stream) -> int | None:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def rhs(mesh: Mesh, params: Params, u: torch.Tensor, alpha: torch.Tensor | None = None,
        out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """``R(u)`` (``dg_rhs``)."""
    if out is None:
        out = torch.empty_like(u)
    _check(_lib.dg_rhs(mesh._h, ctypes.byref(params.c()), mesh._state(u, "u"), mesh._alpha(alpha),
                       mesh._state(out, "out"), _stream(stream)))
    return out


def lift(mesh: Mesh, u: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """BR1-lifted gradient ``[3, n_var, n_node]`` of ``u`` (``dg_lift``; viscous meshes)."""
    if out is None:
        out = torch.empty((3,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    if (tuple(out.shape) != (3,) + tuple(u.shape) or not out.is_contiguous() or out.dtype != torch.float64
            or not out.is_cuda):
        raise ValueError("out must be a contiguous float64 [3, n_var, n_node] tensor")
    _check(_lib.dg_lift(mesh._h, mesh._state(u, "u"), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def timestep(mesh: Mesh, u: torch.Tensor, alpha: torch.Tensor | None = None, cfl: float = 0.5,
             cfl_v: float = 0.5, stream=None) -> float:
    """Time step of the state: convective, joined with the parabolic one on viscous meshes (``dg_timestep``)."""
    out = ctypes.c_double()
    _check(_lib.dg_timestep(mesh._h, mesh._state(u, "u"), mesh._alpha(alpha), float(cfl), float(cfl_v),
                            ctypes.byref(out), _stream(stream)))
    return out.value


def rk_stage(mesh: Mesh, params: Params, stage: int, dt: float, u: torch.Tensor, k: torch.Tensor,
             alpha: torch.Tensor | None = None, stream=None) -> None:
    """In-place 2N Runge-Kutta stage ``stage`` in 1..5 (``dg_rk_stage``)."""
    _check(_lib.dg_rk_stage(mesh._h, ctypes.byref(params.c()), int(stage), float(dt),
                            mesh._state(u, "u"), mesh._state(k, "k"), mesh._alpha(alpha), _stream(stream)))


def rk_step(mesh: Mesh, params: Params, dt: float, u: torch.Tensor, k: torch.Tensor,
            alpha: torch.Tensor | None = None, stream=None) -> None:
    """In-place five-stage 2N Runge-Kutta step (``dg_rk_step``)."""
    _check(_lib.dg_rk_step(mesh._h, ctypes.byref(params.c()), float(dt), mesh._state(u, "u"),
                           mesh._state(k, "k"), mesh._alpha(alpha), _stream(stream)))


def rhs_fv(mesh: Mesh, params: Params, u: torch.Tensor, ufv: torch.Tensor, fv: torch.Tensor, out=None,
           out_fv=None, stream=None):
    """Rates with FV-stored elements (``dg_rhs_fv``): ``(R on DG elements, R of the FV elements' means)``."""
    out = torch.empty_like(u) if out is None else out
    out_fv = torch.empty_like(ufv) if out_fv is None else out_fv
    _check(_lib.dg_rhs_fv(mesh._h, ctypes.byref(params.c()), mesh._state(u, "u"), mesh._fv_state(ufv, "ufv"),
                          mesh._alpha(fv), mesh._state(out, "out"), mesh._fv_state(out_fv, "out_fv"),
                          _stream(stream)))
    return out, out_fv


def rk_stage_fv(mesh: Mesh, params: Params, stage: int, dt: float, u, k, ufv, kfv, fv, stream=None) -> None:
    """In-place RK stage of (u, k) and (ufv, kfv) with FV-stored elements (``dg_rk_stage_fv``)."""
    _check(_lib.dg_rk_stage_fv(mesh._h, ctypes.byref(params.c()), int(stage), float(dt), mesh._state(u, "u"),
                               mesh._state(k, "k"), mesh._fv_state(ufv, "ufv"), mesh._fv_state(kfv, "kfv"),
                               mesh._alpha(fv), _stream(stream)))


def rk_step_fv(mesh: Mesh, params: Params, dt: float, u, k, ufv, kfv, fv, stream=None) -> None:
    """In-place five-stage RK step of (u, k) and (ufv, kfv) (``dg_rk_step_fv``)."""
    _check(_lib.dg_rk_step_fv(mesh._h, ctypes.byref(params.c()), float(dt), mesh._state(u, "u"), mesh._state(k, "k"),
                              mesh._fv_state(ufv, "ufv"), mesh._fv_state(kfv, "kfv"), mesh._alpha(fv),
                              _stream(stream)))


def switch_fv(mesh: Mesh, u, ufv, fv_old, fv_new, stream=None) -> None:
    """Convert the elements whose FV flag changes (``dg_switch_fv``), in place."""
    _check(_lib.dg_switch_fv(mesh._h, mesh._state(u, "u"), mesh._fv_state(ufv, "ufv"), mesh._alpha(fv_old),
                             mesh._alpha(fv_new), _stream(stream)))


def p_degrees(mesh: Mesh, params: Params, u: torch.Tensor, t_refine: float, t_coarsen: float, n_min: int,
              n_max: int, stream=None) -> np.ndarray:
    """Next degree of every element from I(rho) (``dg_p_degrees``; waits for the result)."""
    out = np.zeros(mesh.n_elem, dtype=np.int8)
    _check(_lib.dg_p_degrees(mesh._h, ctypes.byref(params.c()), mesh._state(u, "u"), float(t_refine),
                             float(t_coarsen), int(n_min), int(n_max),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _stream(stream)))
    return out


def transfer_degree(mesh_from: Mesh, mesh_to: Mesh, u: torch.Tensor, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """The state on ``mesh_to`` from the state on ``mesh_from`` (``dg_transfer_degree``)."""
    if out is None:
        out = torch.empty(mesh_to.n_var, mesh_to.n_node, dtype=torch.float64, device=u.device)
    _check(_lib.dg_transfer_degree(mesh_from._h, mesh_to._h, mesh_from._state(u, "u"), mesh_to._state(out, "out"),
                                   _stream(stream)))
    return out


def positivity_limiter(mesh: Mesh, params: Params, u: torch.Tensor, alpha: torch.Tensor | None = None,
                       theta: torch.Tensor | None = None, stream=None) -> torch.Tensor | None:
    """In-place Zhang-Shu limiter of ``u`` (``dg_positivity_limiter``); returns ``theta`` if given."""
    _check(_lib.dg_positivity_limiter(mesh._h, ctypes.byref(params.c()), mesh._state(u, "u"), mesh._alpha(alpha),
                                      mesh._alpha(theta), _stream(stream)))
    return theta


def check_state(mesh: Mesh, stream=None) -> None:
    """Raise DgfvError(ERR_STATE) if a state with rho <= 0, p <= 0 or NaN was read
    since the last report (``dgfv_check_state``; synchronises the stream)."""
    _check(_lib.dgfv_check_state(mesh._h, _stream(stream)))


def indicator(mesh: Mesh, params: Params, u: torch.Tensor, stream=None,
              alpha: torch.Tensor | None = None, ind: torch.Tensor | None = None):
    """Per-element ``(alpha, I)`` (``dg_indicator``), into ``alpha`` and ``ind`` when given."""
    if alpha is None:
        alpha = torch.empty(mesh.n_elem, dtype=torch.float64, device=u.device)
    if ind is None:
        ind = torch.empty_like(alpha)
    mesh._alpha(alpha)
    mesh._alpha(ind)
    _check(_lib.dg_indicator(mesh._h, ctypes.byref(params.c()), mesh._state(u, "u"), alpha.data_ptr(),
                             ind.data_ptr(), _stream(stream)))
    return alpha, ind


def rhs_vjp(mesh: Mesh, params: Params, u: torch.Tensor, alpha: torch.Tensor | None, w: torch.Tensor,
            out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """``(dR/du)^T w`` for a batch ``w[B, n_var, n_node]`` (``dg_rhs_vjp``)."""
    squeeze = w.dim() == 2
    given = out
    if squeeze:
        w = w.unsqueeze(0)
        if out is not None:
            out = out.unsqueeze(0)
    B = w.shape[0]
    if out is None:
        out = torch.empty_like(w)
    _check(_lib.dg_rhs_vjp(mesh._h, ctypes.byref(params.c()), mesh._state(u, "u"), mesh._alpha(alpha),
                           mesh._state(w, "w", B), mesh._state(out, "out", B), B, _stream(stream)))
    if given is not None:
        return given
    return out[0] if squeeze else out


def prim_to_cons(mesh: Mesh, w: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Primitive ``(rho, v1, v2, v3, p[, Y1])`` -> conservative state on the device (``dgfv_prim_to_cons``)."""
    if out is None:
        out = torch.empty_like(w)
    _check(_lib.dgfv_prim_to_cons(mesh._h, mesh._state(w, "w"), mesh._state(out, "out"), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# differentiation: torch.autograd bindings of dg_rhs / dg_rhs_vjp
# ---------------------------------------------------------------------------

class RHSFunction(torch.autograd.Function):
    """``R(u)`` with the blending factors frozen; backward calls ``dg_rhs_vjp``."""

    @staticmethod
    def forward(ctx, u, mesh, params, alpha=None):
        ctx.mesh, ctx.params, ctx.alpha = mesh, params, alpha
        ctx.save_for_backward(u)
        return rhs(mesh, params, u.contiguous(), alpha)

    @staticmethod
    def backward(ctx, grad):
        (u,) = ctx.saved_tensors
        g = rhs_vjp(ctx.mesh, ctx.params, u, ctx.alpha, grad.contiguous())
        return g, None, None, None


def rk_stage_vjp(mesh: Mesh, params: Params, stage: int, dt: float, u_stage: torch.Tensor, ubar: torch.Tensor,
                 kbar: torch.Tensor, alpha: torch.Tensor | None = None, stream=None) -> None:
    """In-place reverse of Runge-Kutta stage ``stage`` (``dg_rk_stage_vjp``)."""
    _check(_lib.dg_rk_stage_vjp(mesh._h, ctypes.byref(params.c()), int(stage), float(dt),
                                mesh._state(u_stage, "u_stage"), mesh._state(ubar, "ubar"),
                                mesh._state(kbar, "kbar"), mesh._alpha(alpha), _stream(stream)))


def rk_stage_vjp_noalloc(mesh: Mesh, params: Params, stage: int, dt: float, u_stage: torch.Tensor,
                         ubar: torch.Tensor, kbar: torch.Tensor, alpha: torch.Tensor | None = None,
                         stream=None) -> None:
    """``rk_stage_vjp`` through the library's fixed device buffer (``dg_rk_stage_vjp_noalloc``)."""
    _check(_lib.dg_rk_stage_vjp_noalloc(mesh._h, ctypes.byref(params.c()), int(stage), float(dt),
                                        mesh._state(u_stage, "u_stage"), mesh._state(ubar, "ubar"),
                                        mesh._state(kbar, "kbar"), mesh._alpha(alpha), _stream(stream)))


def rk_step_vjp(mesh: Mesh, params: Params, dt: float, u0: torch.Tensor, ubar: torch.Tensor,
                alpha: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Cotangent of the state at the start of one RK step, given that of its end.

    The stage inputs are recomputed from ``u0`` with ``dg_rk_stage``, then
    ``dg_rk_stage_vjp`` runs stages 5..1 (the cotangent of k starts at zero:
    nothing after the step reads its k).
    """
    stages = [u0]
    u = u0.clone()
    k = torch.empty_like(u)
    for s in range(1, 5):
        rk_stage(mesh, params, s, dt, u, k, alpha, stream)
        stages.append(u.clone())
    ub = ubar.clone()
    kb = torch.zeros_like(ub)
    for s in range(5, 0, -1):
        rk_stage_vjp(mesh, params, s, dt, stages[s - 1], ub, kb, alpha, stream)
    return ub


class CheckpointedRollout(torch.autograd.Function):
    """``n`` RK steps from ``u0``; stores the state at every step start (RK-stage checkpointing).

    Backward replays each step's stages from its checkpoint and runs the stage
    adjoints in reverse (``rk_step_vjp``).
    """

    @staticmethod
    def forward(ctx, u0, mesh, params, n_steps, dt, alpha=None):
        u = u0.detach().clone().contiguous()
        k = torch.empty_like(u)
        checkpoints = []
        for _ in range(int(n_steps)):
            checkpoints.append(u.clone())
            rk_step(mesh, params, dt, u, k, alpha)
        ctx.mesh, ctx.params, ctx.dt, ctx.alpha = mesh, params, dt, alpha
        ctx.checkpoints = checkpoints
        return u

    @staticmethod
    def backward(ctx, grad):
        ub = grad.contiguous()
        for u0 in reversed(ctx.checkpoints):
            ub = rk_step_vjp(ctx.mesh, ctx.params, ctx.dt, u0, ub, ctx.alpha)
        ctx.checkpoints = None
        return ub, None, None, None, None, None


def checkpointed_rollout(u0, mesh, params, n_steps, dt, alpha=None):
    return CheckpointedRollout.apply(u0, mesh, params, n_steps, dt, alpha)
