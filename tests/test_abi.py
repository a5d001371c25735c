"""The C-ABI library on the host (no GPU needed): it loads, exports every
entry point that include/ef.h declares, validates CSR input with the
documented status codes, and reports missing devices instead of failing."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2306_00606_amd import efgpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ef.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ef_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = efgpu.lib()
    names = declared_functions()
    assert names, "no declarations parsed"
    for name in names:
        assert hasattr(L, name), f"{name} declared in ef.h but not exported"
    assert sorted(efgpu.EXPORTS) == names


def test_version_and_error_text():
    assert efgpu.lib().ef_version() >= 10000
    assert isinstance(efgpu.last_error(), str)


def _valid():
    # path 0-1-2 plus isolated node 3
    return np.array([0, 1, 3, 4, 4], np.int32), np.array([1, 0, 2, 1], np.int32)


CASES = [
    ("self_loop", [0, 2, 3, 4], [0, 1, 0, 1], "EF_ERR_SELF_LOOP"),
    ("duplicate", [0, 2, 4], [1, 1, 0, 0], "EF_ERR_DUPLICATE"),
    ("unsorted", [0, 2, 3, 4], [2, 1, 0, 0], "EF_ERR_UNSORTED"),
    ("row_ptr_decreasing", [0, 2, 1, 2], [1, 2], "EF_ERR_UNSORTED"),
    ("out_of_range", [0, 1, 2], [1, 5], "EF_ERR_RANGE"),
    ("negative_id", [0, 1, 2], [1, -1], "EF_ERR_RANGE"),
    ("row_ptr_start", [1, 2, 3], [1, 0], "EF_ERR_RANGE"),
    ("not_symmetric", [0, 1, 1, 1], [1], "EF_ERR_NOT_SYMMETRIC"),
]


def test_valid_csr_passes():
    efgpu.validate_csr(*_valid())
    efgpu.validate_csr(np.zeros(1, np.int32), np.zeros(0, np.int32))  # empty graph


@pytest.mark.parametrize("name,rp,ci,code", CASES, ids=[c[0] for c in CASES])
def test_malformed_csr_reports_specific_status(name, rp, ci, code):
    with pytest.raises(efgpu.EFError) as ei:
        efgpu.validate_csr(np.array(rp, np.int32), np.array(ci, np.int32))
    assert ei.value.name == code
    assert efgpu.last_error()


def test_overflow_and_null_arguments():
    L = efgpu.lib()
    rp = np.zeros(2, np.int32)
    assert L.ef_validate_csr(1, 2 ** 31, rp.ctypes.data, rp.ctypes.data) == 7  # EF_ERR_OVERFLOW
    assert L.ef_validate_csr(1, 0, None, None) == 1  # EF_ERR_ARG
    assert L.ef_validate_csr(-1, 0, rp.ctypes.data, None) == 1
    assert L.ef_graph_free(None) == 1
    assert L.ef_stats(None, None) == 1
    assert L.ef_compute(None, 0, 0, None, 0, None, None, None, 0, None) == 1
    assert L.ef_device_count(None) == 1


def test_graph_info_struct_layout_matches_header():
    # the ctypes mirrors of the two structs must match the C declarations
    text = open(HEADER).read()
    for struct, fields in (("ef_graph_info", efgpu.GraphInfo._fields_),
                           ("ef_run_stats", efgpu.RunStats._fields_)):
        body = re.search(r"typedef struct \{([^}]*)\}\s*" + struct + ";", text).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"\b([a-z0-9_]+)\s*;", body)
        assert names == [f for f, _ in fields], struct


def _has_gpu():
    try:
        return efgpu.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_no_device_is_reported_not_fatal():
    assert efgpu.device_count() == 0
    with pytest.raises(efgpu.EFError) as ei:
        efgpu.Graph(*_valid())
    assert ei.value.name == "EF_ERR_DEVICE"


def test_union_and_batch_validation_on_host():
    rp, ci = (np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32))
    node_off, rpu, ciu = efgpu.union_csr([(rp, ci), (rp, ci)])
    assert node_off.tolist() == [0, 2, 4]
    assert rpu.tolist() == [0, 1, 2, 3, 4] and ciu.tolist() == [1, 0, 3, 2]
    # a symmetric edge list whose arcs 0-2 and 1-3 cross between the graphs
    h = ctypes.c_void_p()
    bad = np.array([2, 3, 0, 1], np.int32)
    st = efgpu.lib().ef_batch_create(2, node_off.ctypes.data, 4, rpu.ctypes.data, bad.ctypes.data,
                                     efgpu.EF_VALIDATE, None, ctypes.byref(h))
    assert st == 6  # EF_ERR_RANGE
    assert "leaves graph" in efgpu.last_error()


def test_package_build_compiles_the_whole_oracle():
    """The package build (run by the entry point's build()) compiles every C
    source of the oracle, so the library it leaves exports the Expected Force
    and the SIR functions that the tests load."""
    from paper_2306_00606_amd import build as b

    path = b.build_oracle()
    lib = ctypes.CDLL(path)
    for name in ("oracle_ef", "oracle_ef3", "oracle_histogram", "oracle_histogram3",
                 "oracle_splitmix64", "oracle_sir"):
        assert hasattr(lib, name), name


def _load_status(rp, ci, flags=0):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    st = efgpu.lib().ef_graph_load_csr(rp.size - 1, ci.size, rp.ctypes.data,
                                       ci.ctypes.data if ci.size else None, flags, None,
                                       ctypes.byref(h))
    if st == 0:
        efgpu.lib().ef_graph_free(h)
    return st


@pytest.mark.parametrize("name,rp,ci,code", [
    ("row_ptr_decreasing", [0, 2, 1, 2], [1, 2], 5),     # EF_ERR_UNSORTED
    ("offset_past_end", [0, 9, 1, 2], [1, 2], 5),
    ("out_of_range", [0, 1, 2], [1, 5], 6),              # EF_ERR_RANGE
    ("negative_id", [0, 1, 2], [1, -1], 6),
    ("row_ptr_end", [0, 1, 1], [1, 0], 6),
])
def test_load_without_validation_still_checks_bounds(name, rp, ci, code):
    """Without EF_VALIDATE the loader still rejects offsets and ids that a
    kernel could not index safely, on the host, before any device work."""
    assert _load_status(rp, ci, flags=0) == code
    assert "ef_graph_load_csr" in efgpu.last_error()


def test_device_byte_cap_reports_nomem(monkeypatch):
    """EF_MAX_DEVICE_BYTES caps the library's device memory; a graph whose
    fixed arrays exceed it is refused with EF_ERR_NOMEM before the device is
    used (so this holds with or without a GPU)."""
    rp, ci = _valid()
    monkeypatch.setenv("EF_MAX_DEVICE_BYTES", "100")
    assert _load_status(rp, ci) == 8  # EF_ERR_NOMEM
    assert "EF_MAX_DEVICE_BYTES" in efgpu.last_error()
    monkeypatch.setenv("EF_MAX_DEVICE_BYTES", str(1 << 40))
    assert _load_status(rp, ci) in (0, 9)  # loads, or EF_ERR_DEVICE without a GPU
