"""The C-ABI library on the host: it loads, exports every symbol that
include/pbp.h declares, and its host-only calls behave (construction equals
the oracle's; bad arguments are rejected before any device work)."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from helpers import frozen_mask

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbp.h")


@pytest.fixture(scope="module")
def pbp():
    import paper_1505_04979_amd as p
    p.lib()
    return p


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pbp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("pbp_construct", "pbp_code_create", "pbp_encode", "pbp_decode",
              "pbp_status_string"):
        assert s in syms


def test_library_exports_every_declared_symbol(pbp):
    from paper_1505_04979_amd.binding import LIB_PATH
    out = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (pbp_\w+)", out))
    for s in declared_symbols():
        assert s in exported, s
        assert hasattr(pbp.lib(), s)
    # the binding wraps exactly the declared calls
    assert sorted(pbp.exported_symbols()) == declared_symbols()


def test_status_strings(pbp):
    assert pbp.status_string(0) == "ok"
    assert pbp.status_string(-1) == "invalid argument"
    assert pbp.status_string(12345) == "unknown status"


@pytest.mark.parametrize("N,K", [(2, 1), (8, 4), (64, 32), (128, 64), (256, 85),
                                 (256, 128), (256, 213), (1024, 341),
                                 (1024, 512), (1024, 853), (4096, 1365),
                                 (4096, 2048), (4096, 3413), (16384, 8192),
                                 (16, 0), (16, 16)])
def test_construct_equals_oracle(pbp, N, K):
    assert np.array_equal(pbp.pbp_construct(N, K, 0.0), frozen_mask(N, K))


def test_construct_other_design_points(pbp):
    for N, K, d in ((1024, 512, 2.0), (512, 256, -1.0), (64, 20, 4.5)):
        want = np.array(oracle.construct(N, K, d)[0], np.uint8)
        assert np.array_equal(pbp.pbp_construct(N, K, d), want)


def test_construct_rejects_bad_arguments(pbp):
    L = pbp.lib()
    buf = (ctypes.c_uint8 * 64)()
    for N, K in ((0, 0), (1, 0), (3, 1), (96, 10), (32768, 100), (64, -1),
                 (64, 65)):
        assert L.pbp_construct(N, K, 0.0, buf) == -1
    assert L.pbp_construct(64, 32, 0.0, None) == -1
    assert L.pbp_construct(64, 32, float("nan"), buf) == -1


def test_code_create_rejects_bad_arguments_before_device_work(pbp):
    L = pbp.lib()
    h = ctypes.c_void_p()
    fz = np.zeros(64, np.uint8)
    fz[:32] = 1
    p = fz.ctypes.data_as(ctypes.c_void_p)
    assert L.pbp_code_create(64, 31, p, ctypes.byref(h)) == -1   # count != N-K
    assert L.pbp_code_create(63, 31, p, ctypes.byref(h)) == -1
    assert L.pbp_code_create(64, 32, None, ctypes.byref(h)) == -1
    assert L.pbp_code_create(64, 32, p, None) == -1
    assert h.value is None


def test_device_calls_reject_null_handles(pbp):
    L = pbp.lib()
    o = pbp.make_opts()
    assert L.pbp_decode(None, None, 0, ctypes.byref(o), None, None, None, None,
                        None) == -1
    assert L.pbp_encode(None, None, 0, None, None) == -1
    assert L.pbp_code_dims(None, None, None) == -1
    L.pbp_code_destroy(None)
