"""The C-ABI library loads, exports every declared entry point and rejects bad input on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgfv.h")
LIB = os.path.join(ROOT, "paper_2502_19342_amd", "libdgfv.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dg\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdgfv.so is not built: run `python -m paper_2502_19342_amd.build`")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dg_rhs", "dg_rk_stage", "dg_rhs_vjp", "dg_indicator", "dgfv_mesh_create",
                     "dgfv_mesh_destroy", "dgfv_mesh_info", "dgfv_mesh_node_coords", "dgfv_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2502_19342_amd import dgfv
    assert sorted(dgfv.EXPORTED) == declared_functions()


def test_mesh_create_rejects_bad_descriptions_without_touching_the_gpu():
    from paper_2502_19342_amd import dgfv
    from paper_2502_19342_amd import workloads as W
    spec = W.structured_mesh(2, (0, 0, 0), (1, 1, 1), 3)
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.Mesh(np.full(spec.n_elem, 9), spec.corners, spec.faces)           # degree 9
    assert e.value.status == dgfv.ERR_UNSUPPORTED
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.Mesh(spec.degree, spec.corners, spec.faces[:-1])                  # missing face
    assert e.value.status == dgfv.ERR_ARG
    bad = spec.faces.copy()
    bad[0, 4] = 9
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.Mesh(spec.degree, spec.corners, bad)                              # orientation code
    assert e.value.status == dgfv.ERR_ARG
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.Mesh(spec.degree, spec.corners, spec.faces, n_fv=3)               # n_fv < N+1
    assert e.value.status == dgfv.ERR_UNSUPPORTED
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.Mesh(spec.degree, spec.corners, spec.faces, metric_degree=4)      # N_J > N
    assert e.value.status == dgfv.ERR_ARG
    dup = spec.faces.copy()
    dup[1] = dup[0]
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.Mesh(spec.degree, spec.corners, dup)                              # side used twice
    assert e.value.status == dgfv.ERR_ARG
