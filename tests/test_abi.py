"""The C-ABI library loads and exports every entry point its header declares (no GPU calls)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfhk.h")
LIB = os.path.join(ROOT, "paper_2601_17164_amd", "libsfhk.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(sfhk_\w+)\s*\(", src, re.M)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("sfhk_propagate", "sfhk_dipole", "sfhk_spectrum", "sfhk_job_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libsfhk.so is not built: run `python -m paper_2601_17164_amd.build`")
    lib = ct.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2601_17164_amd import sfhk
    assert sorted(sfhk.exported_symbols()) == declared_functions()


def test_status_strings_without_a_device():
    lib = ct.CDLL(LIB)
    lib.sfhk_status_string.restype = ct.c_char_p
    assert lib.sfhk_status_string(0) == b"ok"
    assert lib.sfhk_status_string(-5) == b"HBM budget exceeded"


def test_job_footprint_of_the_benchmark_workload():
    """A job's device memory (state, tiles, field table and the per-step exact accumulators of the
    dipole) is known before it is created; the 2^20-trajectory, 35303-step workload fits in 1 GB:
    43 doubles of state per trajectory (361 MB) plus small per-trajectory and per-step terms."""
    from paper_2601_17164_amd import sfhk
    n, ns = 1 << 20, 35303
    f = sfhk.job_footprint(n, ns)
    assert 43 * 8 * n < f <= 1_000_000_000
    fv = sfhk.job_footprint(n, ns, velocity=True)
    assert fv - f == (ns + 1) * 2 * 68 * 8
