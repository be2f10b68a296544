"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/cip.h declares, and validates arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cip.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cip_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2006_08303_amd import cip
    if not os.path.exists(cip.LIB_PATH):
        pytest.skip("libcip.so not built")
    return cip.lib()


def test_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert "cip_solve" in names and "cip_plan_create" in names
    for n in names:
        assert hasattr(L, n), n


def test_workspace_bytes_and_validation(L):
    from paper_2006_08303_amd import cip
    n = cip.workspace_bytes(3, 3, 1024, 1024, "dct2d")
    # at least the FP32 tables: Lambda (K S F), A (S^2 F), M (S K F), x_hat0 (S F)
    F = 1024 * 513
    assert n >= (9 * 8 + 9 * 4 + 9 * 8 + 3 * 8) * F
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(3, 3, 1000, 1024, "dct2d")
    assert e.value.code == -2
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(0, 3, 64, 64, "dct2d")
    assert e.value.code == -1
    with pytest.raises(cip.CipError):
        cip.workspace_bytes(3, 3, 64, 64, "dct2d", beta=0.0)


def test_create_rejects_bad_workspace(L):
    from paper_2006_08303_amd import cip
    desc = cip._PriorDesc(cip.CIP_PRIOR_DCT2D, 1.0)
    h = ctypes.c_void_p()
    # too small a workspace is refused before any device work
    rc = L.cip_plan_create(2, 2, 64, 64, ctypes.c_void_p(256), ctypes.byref(desc), 0.1, 0.01,
                           ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert rc == -3
    assert b"workspace" in L.cip_last_error()
    rc = L.cip_plan_create(2, 2, 64, 64, None, ctypes.byref(desc), 0.1, 0.01,
                           ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h))
    assert rc == -1
