"""The allocation-free Compton table builder (rrt_compton_tables_noalloc)
against the allocating one (rrt_compton_tables), through the C ABI."""
import ctypes

import numpy as np
import pytest

from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

pytestmark = pytest.mark.gpu

_dp = ctypes.POINTER(ctypes.c_double)


def _noalloc(edges, mec2, lmax, kT):
    L = B.lib()
    f = L.rrt_compton_tables_noalloc
    f.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                  ctypes.c_void_p]
    f.restype = ctypes.c_int
    e = np.ascontiguousarray(edges, dtype=np.float64)
    t = np.ascontiguousarray(np.atleast_1d(kT), dtype=np.float64)
    G, nt = len(e) - 1, len(t)
    s = np.zeros((nt, G))
    p = np.zeros((nt, lmax + 1, G, G))
    st = f(G, e.ctypes.data_as(_dp), 1, float(mec2), int(lmax), nt, t.ctypes.data_as(_dp), s.ctypes.data_as(_dp),
           p.ctypes.data_as(_dp), None)
    if st != 0:
        raise B.RRTError(st, L.rrt_last_error().decode())
    return s, p


def test_noalloc_tables_equal_the_allocating_builder():
    """Two calls in a row, the second smaller: the 32-group, L = 15 tables of
    the 64^3 Compton jet at its nine 10-100 keV nodes, then 8 groups, L = 3 at
    rest and at 50 keV; identical to the allocating builder (same kernels)."""
    cases = [(np.exp(np.linspace(np.log(1e-3), np.log(1e3), 33)), 15, 10.0 ** (1 + np.arange(9) / 8)),
             (np.exp(np.linspace(np.log(1.0), np.log(200.0), 9)), 3, np.array([0.0, 50.0]))]
    for edges, lmax, kT in cases:
        print(f"noalloc tables G={len(edges) - 1} L={lmax} nt={len(kT)}", flush=True)
        s_ref, p_ref = B.compton_tables(edges, W.MEC2_KEV, lmax, kT)
        s, p = _noalloc(edges, W.MEC2_KEV, lmax, kT)
        assert np.abs(s - s_ref).max() <= 1e-13 * np.abs(s_ref).max()
        assert np.abs(p - p_ref).max() <= 1e-13 * np.abs(p_ref).max()


def test_noalloc_refuses_sizes_beyond_its_scratch():
    edges = np.exp(np.linspace(np.log(1e-3), np.log(1e3), 129))
    with pytest.raises(B.RRTError, match="scratch"):
        _noalloc(edges, W.MEC2_KEV, 15, 10.0 ** (1 + np.arange(9) / 8))
