"""CPU tests of the C ABI: the library loads, exports every declared symbol,
validates its arguments and builds host tables that agree with the oracle.
No compute call needs a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import kernels as okernels

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

api = pytest.importorskip("paper_1511_05578_amd.api", reason="libcurvelet.so not built")


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "curvelet.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cvl_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    syms = _declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(api.lib, s), s
        assert s in api.SIGNATURES, s


def test_scale_geometry():
    assert api.num_scales(32) == 5
    assert api.num_scales(256) == 8
    assert api.num_scales(1024) == 10
    assert [api.scale_shape(256, j)[0] for j in range(2, 9)] == [8, 16, 32, 64, 128, 256, 256]
    assert api.scale_shape(256, 5) == (64, 64)
    assert api.scaling_bandlimit(256) == 4
    assert api.scaling_bandlimit(32, 2.0, 1) == 2
    # non-dyadic dilation: L_j = min(ceil(lambda^(j+1)), L)
    assert api.num_scales(50, 1.5) == okernels.num_scales(50, 1.5)
    for j in range(2, api.num_scales(50, 1.5) + 1):
        assert api.scale_shape(50, j, 1.5, 2)[0] == okernels.scale_bandlimit(j, 50, 1.5)


def test_workspace_grows_with_L():
    a = api.workspace_bytes(32)
    b = api.workspace_bytes(64)
    c = api.workspace_bytes(256)
    assert 0 < a < b < c
    # finest-scale alpha/gamma intermediate (L x (2L-1) x L complex) dominates
    assert c >= 256 * 511 * 256 * 16


@pytest.mark.parametrize("kw,code", [
    (dict(L=1), api.CVL_EINVAL),
    (dict(L=4096), api.CVL_EINVAL),
    (dict(L=32, N=16), api.CVL_EINVAL),
    (dict(L=32, lam=1.0), api.CVL_EINVAL),
    (dict(L=32, lam=float("nan")), api.CVL_EINVAL),
    (dict(L=32, J0=0), api.CVL_EINVAL),
    (dict(L=32, J0=6), api.CVL_EINVAL),
    (dict(L=32, spin=2), api.CVL_EINVAL),             # a spin signal is complex
    (dict(L=32, flags=0, spin=2, precision=api.CVL_FP32), api.CVL_EUNSUPPORTED),  # rotated spin: FP64
    (dict(L=32, flags=0, spin=32), api.CVL_EINVAL),
    (dict(L=32, flags=0, spin=-32), api.CVL_EINVAL),
    (dict(L=32, flags=api.CVL_REAL_GRIDS), api.CVL_EINVAL),  # complex map, real grids
    (dict(L=32, flags=api.CVL_REAL | 8), api.CVL_EINVAL),
])
def test_parameter_validation(kw, code):
    L = kw.pop("L")
    p = api.params(L, **kw)
    J = ctypes.c_int(-7)
    rc = api.lib.cvl_num_scales(ctypes.byref(p), ctypes.byref(J))
    assert rc == code
    assert J.value == -7                       # nothing written on failure
    assert len(api.lib.cvl_last_error()) > 0


@pytest.mark.parametrize("kw", [dict(flags=0), dict(flags=api.CVL_UNROTATED, spin=2),
                                dict(flags=0, spin=2), dict(flags=0, spin=-5),
                                dict(flags=api.CVL_UNROTATED, spin=-31),
                                dict(flags=0, precision=api.CVL_FP32)])
def test_complex_and_spin_params_accepted(kw):
    p = api.params(32, **kw)
    J = ctypes.c_int(-7)
    assert api.lib.cvl_num_scales(ctypes.byref(p), ctypes.byref(J)) == api.CVL_OK
    assert J.value == 5


def test_complex_workspace_larger():
    # a complex map carries a second W2 plane, coefficient sets and SHT scratch
    for unrot in (False, True):
        r = api.workspace_bytes(64, unrotated=unrot)
        c = api.workspace_bytes(64, unrotated=unrot, complex_map=True)
        assert c > r
        assert api.scale_workspace_bytes(64, unrotated=unrot, complex_map=True) <= c


def test_real_grids_flag_accepted():
    p = api.params(32, real_grids=True)
    assert p.flags == api.CVL_REAL | api.CVL_REAL_GRIDS
    J = ctypes.c_int(-7)
    assert api.lib.cvl_num_scales(ctypes.byref(p), ctypes.byref(J)) == api.CVL_OK
    assert J.value == 5


def test_unrotated_flag_accepted_and_sizes_workspace():
    p = api.params(32, unrotated=True)
    assert p.flags == api.CVL_REAL | api.CVL_UNROTATED
    J = ctypes.c_int(-7)
    assert api.lib.cvl_num_scales(ctypes.byref(p), ctypes.byref(J)) == api.CVL_OK
    assert J.value == 5
    # the unrotated cube holds every n (2 L_j rows per plane): a larger workspace
    for L in (32, 256):
        assert api.workspace_bytes(L, unrotated=True) > api.workspace_bytes(L)


def test_scale_workspace_excludes_side_stream_buffers():
    # the per-scale calls run on one stream: no side-stream cube buffers
    for L, prec, unrot in [(32, "fp64", False), (256, "fp64", False), (256, "fp32", True),
                           (1024, "fp32", False)]:
        full = api.workspace_bytes(L, precision=prec, unrotated=unrot)
        scale = api.scale_workspace_bytes(L, precision=prec, unrotated=unrot)
        assert 0 < scale < full
    p = api.params(32)
    assert api.lib.cvl_scale_workspace_bytes(ctypes.byref(p), None) == api.CVL_EINVAL
    bad = api.params(32, lam=1.0)
    v = ctypes.c_size_t(7)
    assert api.lib.cvl_scale_workspace_bytes(ctypes.byref(bad), ctypes.byref(v)) == api.CVL_EINVAL
    assert v.value == 7


def test_null_arguments_rejected():
    assert api.lib.cvl_num_scales(None, None) == api.CVL_EINVAL
    p = api.params(32)
    assert api.lib.cvl_workspace_bytes(ctypes.byref(p), 0, ctypes.byref(ctypes.c_size_t())) == api.CVL_EINVAL
    assert api.lib.cvl_sht_forward(None, 32, 0, None, None, None, 0, None) == api.CVL_EINVAL
    assert api.lib.cvl_curvelet_analysis(None, ctypes.byref(p), 1, None, None, None, None, 0, None) \
        == api.CVL_EINVAL
    assert api.lib.cvl_wigner_workspace_bytes(8, 9, ctypes.byref(ctypes.c_size_t())) == api.CVL_EINVAL


@pytest.mark.parametrize("L,lam,J0", [(64, 2.0, 2), (40, 2.0, 1), (50, 1.5, 3)])
def test_host_kernel_tables_match_oracle(L, lam, J0):
    # host C++ Gauss-Legendre quadrature vs the oracle's tanh-sinh quadrature
    kap, phi = api.kernel_tables(L, lam, J0)
    J = okernels.num_scales(L, lam)
    ok = okernels.kappa_table(J0, J, L, lam)
    assert np.abs(kap - ok).max() < 1e-13
    assert np.abs(phi - okernels.phi_table(L, lam, J0)).max() < 1e-13


def test_host_tables_admissible():
    L, lam, J0 = 128, 2.0, 2
    kap, phi = api.kernel_tables(L, lam, J0)
    tot = 4 * np.pi / (2 * np.arange(L) + 1) * phi ** 2 + np.sum(kap ** 2, axis=0)
    assert np.abs(tot - 1).max() < 1e-14


def test_context_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    h = ctypes.c_void_p()
    rc = api.lib.cvl_context_create(ctypes.byref(h), 32, 0)
    assert rc == api.CVL_EDEVICE
    assert h.value is None
