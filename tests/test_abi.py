"""CPU checks of the boundary: libp3t.so loads without a GPU and exports
every entry point include/p3t.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "p3t.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(p3t_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2007_15432_amd as p3t

    if not os.path.exists(p3t.LIB_PATH):
        from paper_2007_15432_amd import build

        build.build()
    return p3t.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("p3t_build_tree", "p3t_compute_soft_force", "p3t_neighbour_list", "p3t_hermite_cluster_step",
                     "p3t_compute_cutoffs", "p3t_kick"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header(lib):
    from paper_2007_15432_amd import _lib

    assert sorted(_lib.SIGNATURES) == _declared()


def test_default_params_match_paper(lib):
    import json

    from paper_2007_15432_amd import Params

    p = Params.defaults()
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    for k in ("eta", "r_search0", "r_search1", "r_search2", "r_search3", "r_cut1", "G", "m_star"):
        assert getattr(p, k) == g[k]["value"], k
    assert abs(p.eta0 - 0.1 * p.eta) < 1e-18
    assert p.theta in g["theta_values"]["value"]


def test_create_rejects_bad_params_without_gpu(lib):
    from paper_2007_15432_amd import _lib

    cp = _lib.CParams()
    lib.p3t_default_params(ctypes.byref(cp))
    cp.gamma = 1.5
    h = ctypes.c_void_p()
    assert lib.p3t_create(ctypes.byref(cp), None, ctypes.byref(h)) == _lib.P3T_ERR_ARG
    assert not h.value


def test_isolated_solver_parameter(lib):
    """Clusters of one member: Hermite (0) by default, the Kepler drift (1) on
    request; anything else is rejected before any device call."""
    from paper_2007_15432_amd import _lib

    cp = _lib.CParams()
    lib.p3t_default_params(ctypes.byref(cp))
    assert cp.isolated == 0 and cp.cluster_cap == 1024  # the field after it still lines up
    cp.isolated = 2
    h = ctypes.c_void_p()
    assert lib.p3t_create(ctypes.byref(cp), None, ctypes.byref(h)) == _lib.P3T_ERR_ARG
    assert not h.value


def test_kepler_drift_without_context_is_an_argument_error(lib):
    from paper_2007_15432_amd import _lib

    n = ctypes.c_int64(0)
    assert lib.p3t_kepler_drift(None, 0, 0.1, None, None, None, 0, None, ctypes.byref(n)) == _lib.P3T_ERR_ARG
