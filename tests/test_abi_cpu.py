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


def test_workspace_grows_with_adaptive_flag_and_dct3d(L):
    """The adaptive flag keeps the FP64 spectra (K S F 16 bytes, which
    otherwise share memory with the solve state) and adds the iterate
    buffers; the 3D DCT adds its S x S band matrix."""
    from paper_2006_08303_amd import cip
    K, S, N = 3, 3, 256
    F = N * (N // 2 + 1)
    base = cip.workspace_bytes(K, S, N, N, "dct2d")
    ad = cip.workspace_bytes(K, S, N, N, "dct2d", flags=cip.CIP_PLAN_ADAPTIVE)
    assert ad >= K * S * F * 16 + 2 * S * N * N * 4 and ad > base
    assert cip.workspace_bytes(K, S, N, N, "dct3d") >= base
    for n in (384, 768, 1536):
        assert cip.workspace_bytes(2, 2, n, n, "tv3d") > 0
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(2, 2, 640, 640, "dct2d")   # 5 * 2^7 is not served
    assert e.value.code == -2


def test_new_entry_points_validate_before_device_work(L):
    """Argument errors are reported without touching the device."""
    from paper_2006_08303_amd import cip
    info = cip._SolveInfo()
    prm = cip._AdaptiveParams(10, 1, 2.0, 10.0, 1e-4)
    assert L.cip_solve_adaptive(None, None, ctypes.byref(prm), None, None, ctypes.byref(info)) == -1
    assert L.cip_plan_set_tuning(None, 4, 16) == -1
    assert L.cip_plan_autotune(None, 10, None, None) == -1
    h = ctypes.c_void_p()
    cfg = cip._ServerConfig(1 << 30, 0, 0)          # no slots
    assert L.cip_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    cfg = cip._ServerConfig(1 << 30, 17, 0)         # too many slots
    assert L.cip_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    cfg = cip._ServerConfig(1024, 2, 0)             # budget below 1 MiB
    assert L.cip_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert L.cip_batch_create(0, None, None, None, None, 4, 1, ctypes.byref(h)) == -1
    desc = cip._desc("conv2d", 1.0)
    desc.n_filters, desc.filt_l, desc.mu = 4, 3, -1.0   # negative Tikhonov weight
    n = ctypes.c_size_t()
    assert L.cip_plan_workspace_bytes(2, 2, 64, 64, ctypes.byref(desc), ctypes.byref(n)) == -1


def test_conv3d_and_dictionary_learning_validation(L):
    """3D conv prior: workspace holds the band tables; dictionary learning
    (patch and conv priors only) is refused for other priors and with a
    negative sigma, and grows the solve state (conv: d, e and the g - e
    spectra are full size; patch: the FP32 codes, the split products and the
    two 256 x 256 systems)."""
    from paper_2006_08303_amd import cip
    K, S, N, M, Lf = 3, 3, 64, 4, 5
    base = cip.workspace_bytes(K, S, N, N, "conv3d", n_filters=M, filt_l=Lf)
    learn = cip.workspace_bytes(K, S, N, N, "conv3d", n_filters=M, filt_l=Lf,
                                flags=cip.CIP_PLAN_DICT_UPDATE)
    F = N * (N // 2 + 1)
    assert learn >= base + 2 * M * S * F * 8 + 2 * M * S * N * N * 4
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(K, S, N, N, "dct2d", flags=cip.CIP_PLAN_DICT_UPDATE)
    assert e.value.code == -2
    b2 = cip.workspace_bytes(K, S, N, N, "conv2d", n_filters=M, filt_l=Lf)
    l2 = cip.workspace_bytes(K, S, N, N, "conv2d", n_filters=M, filt_l=Lf,
                             flags=cip.CIP_PLAN_DICT_UPDATE)
    assert l2 >= b2 + 2 * M * F * 8 + 2 * M * N * N * 4
    A, J = 256, (N // 4) ** 2
    pb = cip.workspace_bytes(K, S, N, N, "patch", n_atoms=A)
    pl = cip.workspace_bytes(K, S, N, N, "patch", n_atoms=A, flags=cip.CIP_PLAN_DICT_UPDATE)
    KS = min(16, J // 32)
    assert pl >= pb + A * J * 4 + KS * (64 * S + A) * A * 4 + 2 * 256 * 256 * 4
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(K, S, N, N, "patch", n_atoms=A, flags=cip.CIP_PLAN_DICT_UPDATE,
                            sigma=-1.0)
    assert e.value.code == -1
    desc = cip._desc("conv3d", 1.0, flags=cip.CIP_PLAN_DICT_UPDATE, sigma=-1.0)
    desc.n_filters, desc.filt_l = M, Lf
    n = ctypes.c_size_t()
    assert L.cip_plan_workspace_bytes(K, S, N, N, ctypes.byref(desc), ctypes.byref(n)) == -1
    desc = cip._desc("conv3d", 1.0, mu=0.01)
    desc.n_filters, desc.filt_l = M, Lf
    assert L.cip_plan_workspace_bytes(K, S, N, N, ctypes.byref(desc), ctypes.byref(n)) == -2
    assert L.cip_plan_dictionary(None, None, None) == -1


def test_wavelet_prior_validation(L):
    """Wavelet (x) DCT prior: grids must be multiples of 2^wt_levels, levels
    in [0, 10] (0: 3); the state is v plus coefficient, staging and image
    buffers."""
    from paper_2006_08303_amd import cip
    K, S = 3, 3
    n3 = cip.workspace_bytes(K, S, 64, 64, "wdct3d")
    assert n3 >= 4 * S * 64 * 64 * 4
    assert cip.workspace_bytes(K, S, 384, 384, "wdct3d", wt_levels=7) > 0
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(K, S, 384, 384, "wdct3d", wt_levels=8)
    assert e.value.code == -2
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(K, S, 64, 64, "wdct3d", wt_levels=11)
    assert e.value.code == -1
    with pytest.raises(cip.CipError) as e:
        cip.workspace_bytes(K, S, 64, 64, "wdct3d", wt_levels=-1)
    assert e.value.code == -1


def test_solve_static_refuses_problems_beyond_its_buffer(L):
    """cip_solve_static checks the workspace a problem needs against its
    static buffer before touching the GPU (1024^2 x 3 needs about 178 MiB)."""
    from paper_2006_08303_amd import cip
    desc = cip._PriorDesc(cip.CIP_PRIOR_DCT2D, 1.0)
    dummy = ctypes.c_void_p(256)     # never dereferenced: the call fails first
    rc = L.cip_solve_static(3, 3, 1024, 1024, dummy, ctypes.byref(desc), 0.1, 0.01, dummy, 10,
                            dummy, None)
    assert rc == -3
    assert b"static buffer" in L.cip_last_error()
    assert cip.workspace_bytes(3, 3, 512, 512, "dct2d") <= cip.STATIC_WORKSPACE_BYTES
    rc = L.cip_solve_static(3, 3, 64, 64, dummy, ctypes.byref(desc), 0.1, 0.01, dummy, 0,
                            dummy, None)
    assert rc == -1


def test_batch_solve_and_descriptor_fields_are_checked_on_the_host(L):
    """cip_batch_solve refuses empty batches and a plan listed twice before
    any device work (the plan handles are not dereferenced); the descriptor
    fields patch_t (patch depth) and per_band (conv filter sets) accept
    the served values and refuse the others."""
    from paper_2006_08303_amd import cip
    vp = ctypes.c_void_p
    plans = (vp * 2)(256, 256)
    ptrs = (vp * 2)(256, 512)
    its = (ctypes.c_int * 2)(3, 3)
    assert L.cip_batch_solve(0, plans, ptrs, its, ptrs, None) == -1
    assert L.cip_batch_solve(2, plans, ptrs, its, ptrs, None) == -1
    assert b"once" in L.cip_last_error()
    n = ctypes.c_size_t()
    for pt, rc in ((0, 0), (3, 0), (1, -2), (2, -2)):
        d = cip._PriorDesc(cip.CIP_PRIOR_PATCH, 500.0)
        d.n_atoms, d.patch_q, d.patch_stride, d.patch_t = 256, 8, 4, pt
        assert L.cip_plan_workspace_bytes(3, 3, 256, 256, ctypes.byref(d), ctypes.byref(n)) == rc
    for pb, rc in ((0, 0), (1, -2), (2, -1)):
        d = cip._PriorDesc(cip.CIP_PRIOR_CONV2D, 8.0)
        d.n_filters, d.filt_l, d.per_band = 32, 11, pb
        assert L.cip_plan_workspace_bytes(3, 3, 256, 256, ctypes.byref(d), ctypes.byref(n)) == rc


def test_band_coupled_isotropic_tv_validation(L):
    """The band-coupled isotropic TV keeps a third dual component in both
    dual buffers (8 floats per voxel against 6 for the per-plane form) and
    checks its inner iteration count like the per-plane form."""
    from paper_2006_08303_amd import cip
    K, S, N = 3, 3, 256
    d2 = cip.workspace_bytes(K, S, N, N, "itv2d")
    d3 = cip.workspace_bytes(K, S, N, N, "itv3d")
    assert d3 - d2 == 2 * S * N * N * 4
    assert cip.workspace_bytes(8, 8, 16, 16, "itv3d", tv_inner=10000) > 0
    for bad in (-1, 10001):
        with pytest.raises(cip.CipError) as e:
            cip.workspace_bytes(K, S, N, N, "itv3d", tv_inner=bad)
        assert e.value.code == -1
