"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/rrt.h, and rejects bad sizes without
touching a device."""
import ctypes
import os
import re

import pytest

from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rrt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rrt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("librrt.so has not been built")
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_footprint_and_size_validation(lib):
    spec = W.thomson_jet()
    fp = B.footprint_bytes(spec, B.FP32)
    dob = 32 ** 3 * 16 * 512 * 4
    # four ordinate-size arrays, the remap plan of the moving medium (two 32-byte entries
    # per point and ordinate: one more ordinate-size array at 16 groups) and the lab
    # extinction, bounded by its per-group size (one more)
    assert 6 * dob < fp < 7 * dob
    assert B.footprint_bytes(spec, B.FP64) > 1.9 * fp
    bad = dict(spec, nmu=15)                    # odd polar count: a horizontal ray
    assert B.footprint_bytes(bad) == 0
    bad = dict(spec, lmax=16)                   # mesh does not resolve lmax
    assert B.footprint_bytes(bad) == 0
    assert b"lmax" in lib.rrt_last_error()


def test_null_problem_is_an_error(lib):
    assert lib.rrt_sweep(None, 0.0, None) == B.RRT_E_INVALID
    assert lib.rrt_synchronize(None) == B.RRT_E_INVALID
    lib.rrt_destroy(None)


def test_batch_calls_validate_arguments(lib):
    assert lib.rrt_batch_create(1 << 20, None) == B.RRT_E_INVALID
    assert lib.rrt_batch_step(None, 1, None) == B.RRT_E_INVALID
    assert lib.rrt_batch_admit(None, None, 1e-6, 10, 1) == B.RRT_E_INVALID
    assert lib.rrt_batch_remove(None, None) == B.RRT_E_INVALID
    lib.rrt_batch_destroy(None)
    assert lib.rrt_device_bytes(None) == 0
