"""Run C-ABI calls of the CPU build of the library (child process; test infrastructure).

Usage: ``python drive.py in.npz out.npz`` with libasan preloaded.  ``in.npz``
holds the mesh description, the parameters, the state and the list of calls;
the results go to ``out.npz``.  Only numpy is imported here: the parent test
computes the oracle's side.
"""
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("n_var", ctypes.c_int32),
                ("degree", ctypes.c_void_p), ("corners", ctypes.c_void_p),
                ("n_face", ctypes.c_int32), ("faces", ctypes.c_void_p),
                ("n_fv", ctypes.c_int32), ("metric_degree", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("kappa", ctypes.c_double * 2), ("R", ctypes.c_double * 2),
                ("n_mortar", ctypes.c_int32), ("mortars", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("volume_flux", ctypes.c_int32), ("face_flux_dg", ctypes.c_int32),
                ("face_flux_fv", ctypes.c_int32), ("ind_vars", ctypes.c_int32),
                ("ind_T", ctypes.c_double), ("ind_dT", ctypes.c_double)]


def ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def main(src, dst):
    z = dict(np.load(src, allow_pickle=False))
    lib = ctypes.CDLL(os.path.join(HERE, "_build", "libdgfv_cpu.so"))
    lib.dgfv_last_error.restype = ctypes.c_char_p
    P = ctypes.c_void_p

    def check(st, what):
        if st != 0:
            raise RuntimeError(f"{what}: status {st}: {lib.dgfv_last_error().decode()}")

    degree = np.ascontiguousarray(z["degree"], dtype=np.int8)
    corners = np.ascontiguousarray(z["corners"], dtype=np.float64)
    faces = np.ascontiguousarray(z["faces"], dtype=np.int32)
    K = degree.shape[0]
    mortars = np.ascontiguousarray(z["mortars"], dtype=np.int32).reshape(-1, 15) if "mortars" in z else None
    desc = MeshDesc(K, int(z["n_var"]), ptr(degree), ptr(corners), faces.shape[0], ptr(faces),
                    int(z["n_fv"]), int(z["metric_degree"]), float(z["gamma"]),
                    (ctypes.c_double * 2)(*z["kappa"]), (ctypes.c_double * 2)(*z["R"]),
                    0 if mortars is None else mortars.shape[0], ptr(mortars) if mortars is not None and len(mortars) else None)
    h = P()
    check(lib.dgfv_mesh_create(ctypes.byref(desc), ctypes.byref(h)), "dgfv_mesh_create")
    n_node = ctypes.c_int64()
    check(lib.dgfv_mesh_info(h, ctypes.byref(n_node), None), "dgfv_mesh_info")
    pr = z["params"]
    prm = Params(int(pr[0]), int(pr[1]), int(pr[2]), int(pr[3]), float(pr[4]), float(pr[5]))
    if "launch_mode" in z:
        check(lib.dgfv_set_launch_mode(h, int(z["launch_mode"])), "launch mode")
    if "transport" in z:                       # mu[2], Pr[2], D[2]
        tr = (ctypes.c_double * 6)(*[float(x) for x in z["transport"]])
        check(lib.dgfv_set_transport(h, tr), "dgfv_set_transport")
    u = np.ascontiguousarray(z["u"], dtype=np.float64)
    alpha = np.ascontiguousarray(z["alpha"], dtype=np.float64) if "alpha" in z else None
    out = {}
    for call in [str(c) for c in z["calls"]]:
        print(f"[cpu_hip] {call}", flush=True)
        if call in ("fusion_off", "fusion_on"):
            check(lib.dgfv_set_face_fusion(h, int(call == "fusion_on")), call)
        elif call == "rhs_unfused":
            r = np.empty_like(u)
            check(lib.dgfv_set_face_fusion(h, 0), "fusion off")
            check(lib.dg_rhs(h, ctypes.byref(prm), ptr(u), ptr(alpha), ptr(r), None), "dg_rhs")
            out["rhs_unfused"] = r
        elif call == "rk_step_unfused":
            uu = u.copy()
            k = np.empty_like(u)
            check(lib.dgfv_set_face_fusion(h, 0), "fusion off")
            check(lib.dg_rk_step(h, ctypes.byref(prm), ctypes.c_double(float(z["dt"])), ptr(uu), ptr(k),
                                 ptr(alpha), None), "dg_rk_step")
            out["rk_step_unfused"] = uu
        elif call == "rhs_fv":
            ufv = np.ascontiguousarray(z["ufv"], dtype=np.float64)
            fvf = np.ascontiguousarray(z["fv"], dtype=np.float64)
            r, rf = np.empty_like(u), np.empty_like(ufv)
            check(lib.dg_rhs_fv(h, ctypes.byref(prm), ptr(u), ptr(ufv), ptr(fvf), ptr(r), ptr(rf), None), "dg_rhs_fv")
            out["rhs_fv_dg"], out["rhs_fv_fv"] = r, rf
        elif call == "rk_step_fv":
            uu = u.copy()
            uf = np.ascontiguousarray(z["ufv"], dtype=np.float64).copy()
            fvf = np.ascontiguousarray(z["fv"], dtype=np.float64)
            k, kf = np.empty_like(uu), np.empty_like(uf)
            for st in range(1, 6):
                check(lib.dg_rk_stage_fv(h, ctypes.byref(prm), ctypes.c_int(st), ctypes.c_double(float(z["dt"])),
                                         ptr(uu), ptr(k), ptr(uf), ptr(kf), ptr(fvf), None), "dg_rk_stage_fv")
            out["step_fv_dg"], out["step_fv_fv"] = uu, uf
        elif call == "rk_step_fv_one_call":
            uu = u.copy()
            uf = np.ascontiguousarray(z["ufv"], dtype=np.float64).copy()
            fvf = np.ascontiguousarray(z["fv"], dtype=np.float64)
            k, kf = np.empty_like(uu), np.empty_like(uf)
            check(lib.dg_rk_step_fv(h, ctypes.byref(prm), ctypes.c_double(float(z["dt"])), ptr(uu), ptr(k), ptr(uf),
                                    ptr(kf), ptr(fvf), None), "dg_rk_step_fv")
            out["step1_fv_dg"], out["step1_fv_fv"] = uu, uf
        elif call == "p_degrees":
            nd = np.zeros(K, dtype=np.int8)
            th = z["p_thresholds"]
            check(lib.dg_p_degrees(h, ctypes.byref(prm), ptr(u), ctypes.c_double(float(th[0])),
                                   ctypes.c_double(float(th[1])), ctypes.c_int(int(th[2])), ctypes.c_int(int(th[3])),
                                   ptr(nd), None), "dg_p_degrees")
            out["p_degrees"] = nd
        elif call == "transfer":
            deg2 = np.ascontiguousarray(z["degree_to"], dtype=np.int8)
            desc2 = MeshDesc(K, int(z["n_var"]), ptr(deg2), ptr(corners), faces.shape[0], ptr(faces),
                             int(z["n_fv"]), int(z["metric_degree_to"]), float(z["gamma"]),
                             (ctypes.c_double * 2)(*z["kappa"]), (ctypes.c_double * 2)(*z["R"]))
            h2 = P()
            check(lib.dgfv_mesh_create(ctypes.byref(desc2), ctypes.byref(h2)), "dgfv_mesh_create (new degrees)")
            n2 = ctypes.c_int64()
            check(lib.dgfv_mesh_info(h2, ctypes.byref(n2), None), "dgfv_mesh_info")
            u2 = np.empty((u.shape[0], n2.value))
            check(lib.dg_transfer_degree(h, h2, ptr(u), ptr(u2), None), "dg_transfer_degree")
            lib.dgfv_mesh_destroy(h2)
            out["transfer"] = u2
        elif call == "switch_fv":
            uu = u.copy()
            uf = np.ascontiguousarray(z["ufv"], dtype=np.float64).copy()
            check(lib.dg_switch_fv(h, ptr(uu), ptr(uf), ptr(np.ascontiguousarray(z["fv"], dtype=np.float64)),
                                   ptr(np.ascontiguousarray(z["fv_new"], dtype=np.float64)), None), "dg_switch_fv")
            out["switch_dg"], out["switch_fv"] = uu, uf
        elif call == "timestep":
            cf = z["cfl"]
            dt = ctypes.c_double()
            check(lib.dg_timestep(h, ptr(u), ptr(alpha), ctypes.c_double(float(cf[0])), ctypes.c_double(float(cf[1])),
                                  ctypes.byref(dt), None), "dg_timestep")
            out["timestep"] = np.array([dt.value])
        elif call == "lift":
            g = np.empty((3,) + u.shape)
            check(lib.dg_lift(h, ptr(u), ptr(g), None), "dg_lift")
            out["lift"] = g
        elif call == "rhs":
            r = np.empty_like(u)
            check(lib.dg_rhs(h, ctypes.byref(prm), ptr(u), ptr(alpha), ptr(r), None), "dg_rhs")
            out["rhs"] = r
        elif call == "vjp":
            w = np.ascontiguousarray(z["w"], dtype=np.float64)
            g = np.empty_like(w)
            check(lib.dg_rhs_vjp(h, ctypes.byref(prm), ptr(u), ptr(alpha), ptr(w), ptr(g),
                                 ctypes.c_int(w.shape[0]), None), "dg_rhs_vjp")
            out["vjp"] = g
        elif call == "rk_step":
            uu = u.copy()
            k = np.empty_like(u)
            check(lib.dg_rk_step(h, ctypes.byref(prm), ctypes.c_double(float(z["dt"])), ptr(uu), ptr(k),
                                 ptr(alpha), None), "dg_rk_step")
            out["rk_step"] = uu
        elif call == "rk_stages":               # five dg_rk_stage calls: no traces between them
            uu = u.copy()
            k = np.empty_like(u)
            for st in range(1, 6):
                check(lib.dg_rk_stage(h, ctypes.byref(prm), ctypes.c_int(st), ctypes.c_double(float(z["dt"])),
                                      ptr(uu), ptr(k), ptr(alpha), None), "dg_rk_stage")
            out["rk_stages"] = uu
        elif call == "indicator":
            a = np.empty(K)
            ind = np.empty(K)
            check(lib.dg_indicator(h, ctypes.byref(prm), ptr(u), ptr(a), ptr(ind), None), "dg_indicator")
            out["alpha"], out["ind"] = a, ind
        elif call == "stage_vjp":
            ub = np.ascontiguousarray(z["ubar"], dtype=np.float64).copy()
            kb = np.ascontiguousarray(z["kbar"], dtype=np.float64).copy()
            check(lib.dg_rk_stage_vjp(h, ctypes.byref(prm), ctypes.c_int(int(z["stage"])),
                                      ctypes.c_double(float(z["dt"])), ptr(u), ptr(ub), ptr(kb), ptr(alpha),
                                      None), "dg_rk_stage_vjp")
            out["ubar"], out["kbar"] = ub, kb
        elif call == "limiter":
            ul = u.copy()
            th = np.empty(K)
            check(lib.dg_positivity_limiter(h, ctypes.byref(prm), ptr(ul), ptr(alpha), ptr(th), None),
                  "dg_positivity_limiter")
            out["limited"], out["theta"] = ul, th
        elif call == "prim_to_cons":
            cu = np.empty_like(u)
            check(lib.dgfv_prim_to_cons(h, ptr(u), ptr(cu), None), "dgfv_prim_to_cons")
            out["cons"] = cu
        elif call == "coords":
            xyz = np.empty((3, n_node.value))
            check(lib.dgfv_mesh_node_coords(h, ptr(xyz)), "coords")
            out["coords"] = xyz
        else:
            raise ValueError(call)
    lib.dgfv_mesh_destroy(h)
    np.savez(dst, **out)
    print("[cpu_hip] done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
