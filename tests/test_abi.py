"""CPU-side checks of the C ABI: the library loads, exports every symbol
declared in include/jsweep.h, and rejects invalid arguments before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1803_09876_amd as J
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "jsweep.h")).read()
    return sorted(set(re.findall(r"\b(jsweep_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = J.load_library()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(J.EXPORTED) == names


def test_error_strings():
    for code in range(0, -10, -1):
        assert J.jsweep_error_string(code)
    assert J.jsweep_error_string(-99) == "unknown error"


def _build(mesh, om, w, flags=0):
    return J.jsweep_build_graph(mesh.dim, mesh.cell_type, mesh.coords, mesh.cells, om, w, flags)


def test_rejects_bad_quadrature():
    m = W.kuhn_tets(2, 0.1, 1)
    om, w = W.quadrature(4, 3)
    with pytest.raises(J.JsweepError) as e:
        _build(m, om, w * 1.01)
    assert e.value.code == J.JSWEEP_E_QUADRATURE
    bad = om.copy()
    bad[0] *= 1.1
    with pytest.raises(J.JsweepError) as e:
        _build(m, bad, w)
    assert e.value.code == J.JSWEEP_E_QUADRATURE


def test_rejects_bad_mesh_arguments():
    m = W.kuhn_tets(2, 0.1, 1)
    om, w = W.quadrature(4, 3)
    with pytest.raises(J.JsweepError) as e:
        J.jsweep_build_graph(2, J.JSWEEP_TET, m.coords, m.cells, om, w)
    assert e.value.code == J.JSWEEP_E_INVALID_ARG
    coords = m.coords.copy()
    coords[3, 1] = np.nan
    with pytest.raises(J.JsweepError) as e:
        J.jsweep_build_graph(3, J.JSWEEP_TET, coords, m.cells, om, w)
    assert e.value.code == J.JSWEEP_E_MESH
    with pytest.raises(J.JsweepError) as e:
        J.jsweep_build_graph(3, J.JSWEEP_TET, m.coords, m.cells, om, w, flags=0x80)
    assert e.value.code == J.JSWEEP_E_INVALID_ARG


def test_null_handles_rejected():
    lib = J.load_library()
    assert lib.jsweep_graph_info(None, None, None, None, None) == J.JSWEEP_E_INVALID_ARG
    assert lib.jsweep_program_info(None, None, None, None) == J.JSWEEP_E_INVALID_ARG
    assert lib.jsweep_sweep(None, None, None, None, None, 0.0, None) == J.JSWEEP_E_INVALID_ARG
    assert lib.jsweep_profile(None, 1) == J.JSWEEP_E_INVALID_ARG
    lib.jsweep_graph_destroy(None)
    assert "graph is NULL" in J.jsweep_last_error() or J.jsweep_last_error()


def test_set_params_and_patch_info_reject_null():
    """The two parameter calls refuse a NULL graph (no device work)."""
    lib = J.load_library()
    assert lib.jsweep_set_params(None, None) == J.JSWEEP_E_INVALID_ARG
    out = np.zeros(6, dtype=np.int64)
    assert lib.jsweep_patch_info(None, None, out.ctypes.data) == J.JSWEEP_E_INVALID_ARG


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with a message before any
    device work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
