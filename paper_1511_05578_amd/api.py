"""Thin ctypes binding of libcurvelet.so (include/curvelet.h).

Argument marshalling only: every step of every transform runs in the HIP
kernels of the library.  PyTorch provides device memory and the current
stream.  Importing this module loads the library and raises if it has not
been built (``python -m paper_1511_05578_amd.build``); there is no fallback.
"""
import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcurvelet.so")

CVL_OK, CVL_EINVAL, CVL_ENOMEM, CVL_EDEVICE, CVL_EUNSUPPORTED = 0, -1, -2, -3, -4
CVL_REAL, CVL_REAL_GRIDS, CVL_UNROTATED = 1, 2, 4
CVL_FP64, CVL_FP32, CVL_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": CVL_FP64, "fp32": CVL_FP32, "bf16x3": CVL_BF16X3}

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_size_p = ctypes.POINTER(ctypes.c_size_t)
_c_double_p = ctypes.POINTER(ctypes.c_double)


class CvlParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("N", ctypes.c_int), ("lambda_", ctypes.c_double),
                ("J0", ctypes.c_int), ("spin", ctypes.c_int), ("precision", ctypes.c_int),
                ("flags", ctypes.c_uint)]


# name -> (restype, argtypes)
SIGNATURES = {
    "cvl_context_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int]),
    "cvl_context_destroy": (None, [ctypes.c_void_p]),
    "cvl_num_scales": (ctypes.c_int, [ctypes.POINTER(CvlParams), _c_int_p]),
    "cvl_scale_shape": (ctypes.c_int, [ctypes.POINTER(CvlParams), ctypes.c_int, _c_int_p, _c_int_p]),
    "cvl_scaling_bandlimit": (ctypes.c_int, [ctypes.POINTER(CvlParams), _c_int_p]),
    "cvl_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(CvlParams), ctypes.c_int, _c_size_p]),
    "cvl_scale_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(CvlParams), _c_size_p]),
    "cvl_sht_workspace_bytes": (ctypes.c_int, [ctypes.c_int, _c_size_p]),
    "cvl_wigner_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_size_p]),
    "cvl_prepare": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams)]),
    "cvl_sht_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_sht_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_sht_forward_complex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_void_p]),
    "cvl_sht_inverse_complex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_void_p]),
    "cvl_wigner_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_wigner_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_curvelet_analysis": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams), ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_curvelet_analysis_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams),
                                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                     ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "cvl_curvelet_synthesis": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams), ctypes.c_int,
                                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                              ctypes.c_void_p]),
    "cvl_curvelet_analysis_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams), ctypes.c_int,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_curvelet_synthesis_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams), ctypes.c_int,
                                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_curvelet_scaling_analysis": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams),
                                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                     ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_curvelet_scaling_synthesis": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CvlParams),
                                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_size_t, ctypes.c_void_p]),
    "cvl_kernel_tables": (ctypes.c_int, [ctypes.POINTER(CvlParams), _c_double_p, _c_double_p]),
    "cvl_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "cvl_profile_filter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "cvl_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_int_p,
                                        ctypes.POINTER(ctypes.c_char_p), _c_int_p, _c_double_p]),
    "cvl_profile_read_detail": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_int_p, _c_int_p,
                                                _c_int_p, _c_int_p, _c_double_p]),
    "cvl_delta_block": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_double_p]),
    "cvl_last_error": (ctypes.c_char_p, []),
}

# torch ships its own HIP runtime under the same soname as the system one; load
# it first so that the library and torch share one runtime in the process
# (two runtimes in one process do not see the same devices).
import torch  # noqa: E402,F401

if not os.path.exists(_LIB_PATH):
    raise ImportError("libcurvelet.so is not built: run `python -m paper_1511_05578_amd.build`")
lib = ctypes.CDLL(_LIB_PATH)
for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class CvlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("cvl error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != CVL_OK:
        raise CvlError(rc, lib.cvl_last_error().decode())


def _prec(precision):
    if isinstance(precision, str):
        return PRECISIONS[precision.lower()]
    return int(precision)


def params(L, lam=2.0, J0=2, N=0, spin=0, flags=None, precision=CVL_FP64, real_grids=False,
           unrotated=False, complex_map=False):
    """cvl_params; a complex map (complex_map) clears CVL_REAL."""
    if flags is None:
        flags = 0 if complex_map else CVL_REAL
    if real_grids:
        flags |= CVL_REAL_GRIDS
    if unrotated:
        flags |= CVL_UNROTATED
    return CvlParams(L, N, float(lam), J0, spin, _prec(precision), flags)


def num_scales(L, lam=2.0, J0=2):
    J = ctypes.c_int()
    _check(lib.cvl_num_scales(ctypes.byref(params(L, lam, J0)), ctypes.byref(J)))
    return J.value


def scale_shape(L, j, lam=2.0, J0=2):
    Lj, Nj = ctypes.c_int(), ctypes.c_int()
    _check(lib.cvl_scale_shape(ctypes.byref(params(L, lam, J0)), j, ctypes.byref(Lj), ctypes.byref(Nj)))
    return Lj.value, Nj.value


def scaling_bandlimit(L, lam=2.0, J0=2):
    v = ctypes.c_int()
    _check(lib.cvl_scaling_bandlimit(ctypes.byref(params(L, lam, J0)), ctypes.byref(v)))
    return v.value


def workspace_bytes(L, lam=2.0, J0=2, batch=1, precision=CVL_FP64, unrotated=False,
                    complex_map=False, spin=0):
    v = ctypes.c_size_t()
    p = params(L, lam, J0, spin=spin, precision=precision, unrotated=unrotated,
               complex_map=complex_map)
    _check(lib.cvl_workspace_bytes(ctypes.byref(p), batch, ctypes.byref(v)))
    return v.value


def scale_workspace_bytes(L, lam=2.0, J0=2, precision=CVL_FP64, unrotated=False,
                          complex_map=False, spin=0):
    """Workspace of the per-scale (streaming) calls."""
    v = ctypes.c_size_t()
    p = params(L, lam, J0, spin=spin, precision=precision, unrotated=unrotated,
               complex_map=complex_map)
    _check(lib.cvl_scale_workspace_bytes(ctypes.byref(p), ctypes.byref(v)))
    return v.value


def kernel_tables(L, lam=2.0, J0=2):
    """Host tables (no GPU): kappa[j - J0, l] and phi[l]."""
    J = num_scales(L, lam, J0)
    kap = np.zeros((J - J0 + 1, L))
    phi = np.zeros(L)
    _check(lib.cvl_kernel_tables(ctypes.byref(params(L, lam, J0)),
                                 kap.ctypes.data_as(_c_double_p), phi.ctypes.data_as(_c_double_p)))
    return kap, phi


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Resident Delta table (and kernel / DFT tables built on first use).

    The binding keeps one scratch workspace per HIP stream (the stream current
    when a method is called), because calls that share a workspace must be
    ordered on one stream.  A workspace grows (and is replaced) when a call
    needs more: a HIP graph captured from these methods keeps pointing at the
    workspace it was captured with, so prepare the largest call first (or
    pass the raw C entry points a workspace of your own) before capturing."""

    def __init__(self, L_max, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.L_max = L_max
        h = ctypes.c_void_p()
        _check(lib.cvl_context_create(ctypes.byref(h), L_max, device))
        self.h = h
        self._ws = {}

    def close(self):
        if getattr(self, "h", None):
            lib.cvl_context_destroy(self.h)
            self.h = None
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes):
        """The current stream's workspace, at least nbytes."""
        t = self.torch
        key = t.cuda.current_stream(self.device).cuda_stream
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = t.empty(max(nbytes, 256), dtype=t.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def prepare(self, L, lam=2.0, J0=2, spin=0, complex_map=False, unrotated=False):
        p = params(L, lam, J0, spin=spin, unrotated=unrotated, complex_map=complex_map or spin != 0)
        _check(lib.cvl_prepare(self.h, ctypes.byref(p)))

    # ---- SHT ----
    def _sht_ws(self, L):
        nb = ctypes.c_size_t()
        _check(lib.cvl_sht_workspace_bytes(L, ctypes.byref(nb)))
        return self.workspace(nb.value)

    def sht_forward(self, fmap, out=None, spin=0):
        """f_lm (L^2 complex128) of a real map (float64, spin 0) or of a
        complex map (complex128) of spin `spin`."""
        t = self.torch
        L = fmap.shape[-2]
        assert fmap.is_contiguous() and fmap.shape[-1] == 2 * L - 1
        if out is None:
            out = t.empty(L * L, dtype=t.complex128, device=self.device)
        ws = self._sht_ws(L)
        if fmap.dtype == t.complex128:
            _check(lib.cvl_sht_forward_complex(self.h, L, spin, fmap.data_ptr(), out.data_ptr(),
                                               ws.data_ptr(), ws.numel(), _stream(t)))
            return out
        assert fmap.dtype == t.float64 and spin == 0
        _check(lib.cvl_sht_forward(self.h, L, 0, fmap.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream(t)))
        return out

    def sht_inverse(self, flm, L, out=None, spin=0, complex_map=False):
        """Map of f_lm: real (float64; m >= 0 read) by default, complex
        (complex128; every m read) with complex_map or spin != 0."""
        t = self.torch
        assert flm.dtype == t.complex128 and flm.is_contiguous() and flm.numel() == L * L
        cplx = complex_map or spin != 0
        if out is None:
            out = t.empty((L, 2 * L - 1), dtype=t.complex128 if cplx else t.float64,
                          device=self.device)
        ws = self._sht_ws(L)
        if cplx:
            _check(lib.cvl_sht_inverse_complex(self.h, L, spin, flm.data_ptr(), out.data_ptr(),
                                               ws.data_ptr(), ws.numel(), _stream(t)))
            return out
        _check(lib.cvl_sht_inverse(self.h, L, 0, flm.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream(t)))
        return out

    # ---- Wigner ----
    def wigner_inverse(self, F, L, N, out=None):
        t = self.torch
        assert F.dtype == t.complex128 and F.is_contiguous() and F.shape == (L, 2 * L - 1, 2 * N - 1)
        if out is None:
            out = t.empty((2 * L - 1, L, 2 * N - 1), dtype=t.complex128, device=self.device)
        nb = ctypes.c_size_t()
        _check(lib.cvl_wigner_workspace_bytes(L, N, ctypes.byref(nb)))
        ws = self.workspace(nb.value)
        _check(lib.cvl_wigner_inverse(self.h, L, N, F.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _stream(t)))
        return out

    def wigner_forward(self, grid, L, N, out=None):
        t = self.torch
        assert grid.dtype == t.complex128 and grid.is_contiguous() and grid.shape == (2 * L - 1, L, 2 * N - 1)
        if out is None:
            out = t.empty((L, 2 * L - 1, 2 * N - 1), dtype=t.complex128, device=self.device)
        nb = ctypes.c_size_t()
        _check(lib.cvl_wigner_workspace_bytes(L, N, ctypes.byref(nb)))
        ws = self.workspace(nb.value)
        _check(lib.cvl_wigner_forward(self.h, L, N, grid.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _stream(t)))
        return out

    # ---- curvelets ----
    def grid_shapes(self, L, lam=2.0, J0=2):
        J = num_scales(L, lam, J0)
        out = []
        for j in range(J0, J + 1):
            Lj, Nj = scale_shape(L, j, lam, J0)
            out.append((2 * Lj - 1, Lj, 2 * Nj - 1))
        return out

    def grid_dtype(self, precision=CVL_FP64, real_grids=False):
        """Element type of the curvelet grids: complex128 (precision "fp64") or
        complex64 ("fp32", "bf16x3") (zero imaginary parts for a real map), or
        with real_grids float64 / float32 holding the same (real) coefficients."""
        t = self.torch
        if real_grids:
            return t.float64 if _prec(precision) == CVL_FP64 else t.float32
        return t.complex128 if _prec(precision) == CVL_FP64 else t.complex64

    def alloc_outputs(self, L, lam=2.0, J0=2, batch=1, precision=CVL_FP64, real_grids=False,
                      complex_map=False):
        t = self.torch
        Lp = scaling_bandlimit(L, lam, J0)
        scal = t.empty((batch, Lp, 2 * Lp - 1), dtype=t.complex128 if complex_map else t.float64,
                       device=self.device)
        dt = self.grid_dtype(precision, real_grids)
        grids = [[t.empty(s, dtype=dt, device=self.device)
                  for s in self.grid_shapes(L, lam, J0)] for _ in range(batch)]
        return scal, grids

    def curvelet_analysis(self, maps, lam=2.0, J0=2, out=None, precision=CVL_FP64,
                          real_grids=False, unrotated=False, spin=0):
        """maps: (batch, L, 2L-1) or (L, 2L-1), float64 (real maps) or
        complex128 (complex maps of spin `spin`).  Returns (scal, grids);
        grids of grid_dtype(precision, real_grids).  unrotated: coefficients
        of the unrotated curvelets (CVL_UNROTATED)."""
        t = self.torch
        single = maps.dim() == 2
        if single:
            maps = maps.unsqueeze(0)
        cplx = maps.dtype == t.complex128
        assert (cplx or maps.dtype == t.float64) and maps.is_contiguous()
        batch, L = maps.shape[0], maps.shape[1]
        if out is None:
            out = self.alloc_outputs(L, lam, J0, batch, precision, real_grids, cplx)
        scal, grids = out
        flat = [g for per in grids for g in per]
        dt = self.grid_dtype(precision, real_grids)
        for g in flat:
            assert g.dtype == dt and g.is_contiguous()
        arr = (ctypes.c_void_p * len(flat))(*[g.data_ptr() for g in flat])
        ws = self.workspace(workspace_bytes(L, lam, J0, batch, precision, unrotated, cplx, spin))
        p = params(L, lam, J0, spin=spin, precision=precision, real_grids=real_grids,
                   unrotated=unrotated, complex_map=cplx)
        _check(lib.cvl_curvelet_analysis(self.h, ctypes.byref(p), batch,
                                         maps.data_ptr(), scal.data_ptr(), arr, ws.data_ptr(),
                                         ws.numel(), _stream(t)))
        if single:
            return scal[0], grids[0]
        return scal, grids

    def curvelet_synthesis(self, scal, grids, L, lam=2.0, J0=2, out=None, precision=CVL_FP64,
                           real_grids=False, unrotated=False, spin=0):
        """Maps from scaling maps and grids; complex maps when the scaling maps
        are complex128 (the analysis of complex maps of spin `spin`)."""
        t = self.torch
        single = scal.dim() == 2
        if single:
            scal = scal.unsqueeze(0)
            grids = [grids]
        cplx = scal.dtype == t.complex128
        batch = scal.shape[0]
        if out is None:
            out = t.empty((batch, L, 2 * L - 1), dtype=t.complex128 if cplx else t.float64,
                          device=self.device)
        flat = [g for per in grids for g in per]
        dt = self.grid_dtype(precision, real_grids)
        for g in flat:
            assert g.dtype == dt and g.is_contiguous()
        arr = (ctypes.c_void_p * len(flat))(*[g.data_ptr() for g in flat])
        ws = self.workspace(workspace_bytes(L, lam, J0, batch, precision, unrotated, cplx, spin))
        p = params(L, lam, J0, spin=spin, precision=precision, real_grids=real_grids,
                   unrotated=unrotated, complex_map=cplx)
        _check(lib.cvl_curvelet_synthesis(self.h, ctypes.byref(p), batch,
                                          scal.data_ptr(), arr, out.data_ptr(), ws.data_ptr(),
                                          ws.numel(), _stream(t)))
        return out[0] if single else out

    # ---- streaming (one scale at a time) ----
    # complex_map: flm holds every m of a complex signal (spin `spin`) and the
    # scaling maps are complex128; otherwise a real map's coefficients.
    def analysis_scale(self, flm, L, j, lam=2.0, J0=2, out=None, precision=CVL_FP64,
                       real_grids=False, unrotated=False, complex_map=False, spin=0):
        """Grid of scale j from harmonic coefficients flm (L^2 complex128)."""
        t = self.torch
        assert flm.dtype == t.complex128 and flm.is_contiguous() and flm.numel() == L * L
        dt = self.grid_dtype(precision, real_grids)
        if out is None:
            Lj, _ = scale_shape(L, j, lam, J0)
            out = t.empty((2 * Lj - 1, Lj, 2 * Lj - 1), dtype=dt, device=self.device)
        assert out.dtype == dt and out.is_contiguous()
        ws = self.workspace(scale_workspace_bytes(L, lam, J0, precision, unrotated, complex_map, spin))
        p = params(L, lam, J0, spin=spin, precision=precision, real_grids=real_grids,
                   unrotated=unrotated, complex_map=complex_map)
        _check(lib.cvl_curvelet_analysis_scale(self.h, ctypes.byref(p), j, flm.data_ptr(),
                                               out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(t)))
        return out

    def synthesis_scale(self, grid, L, j, flm_acc, lam=2.0, J0=2, precision=CVL_FP64,
                        real_grids=False, unrotated=False, complex_map=False, spin=0):
        """flm_acc += f^(j)_lm from scale j's grid."""
        t = self.torch
        assert grid.dtype == self.grid_dtype(precision, real_grids) and grid.is_contiguous()
        assert flm_acc.dtype == t.complex128 and flm_acc.numel() == L * L
        ws = self.workspace(scale_workspace_bytes(L, lam, J0, precision, unrotated, complex_map, spin))
        p = params(L, lam, J0, spin=spin, precision=precision, real_grids=real_grids,
                   unrotated=unrotated, complex_map=complex_map)
        _check(lib.cvl_curvelet_synthesis_scale(self.h, ctypes.byref(p), j, grid.data_ptr(),
                                                flm_acc.data_ptr(), ws.data_ptr(), ws.numel(),
                                                _stream(t)))
        return flm_acc

    # The scaling part is FP64 at every precision; `precision` only names the
    # streaming workspace (cvl_scale_workspace_bytes of the same parameters) to use.
    def scaling_analysis(self, flm, L, lam=2.0, J0=2, out=None, precision=CVL_FP64,
                         unrotated=False, complex_map=False, spin=0):
        t = self.torch
        Lp = scaling_bandlimit(L, lam, J0)
        if out is None:
            out = t.empty((Lp, 2 * Lp - 1), dtype=t.complex128 if complex_map else t.float64,
                          device=self.device)
        ws = self.workspace(scale_workspace_bytes(L, lam, J0, precision, unrotated, complex_map, spin))
        p = params(L, lam, J0, spin=spin, precision=precision, unrotated=unrotated,
                   complex_map=complex_map)
        _check(lib.cvl_curvelet_scaling_analysis(self.h, ctypes.byref(p), flm.data_ptr(),
                                                 out.data_ptr(), ws.data_ptr(), ws.numel(),
                                                 _stream(t)))
        return out

    def scaling_synthesis(self, scal, L, flm_acc, lam=2.0, J0=2, precision=CVL_FP64,
                          unrotated=False, complex_map=False, spin=0):
        ws = self.workspace(scale_workspace_bytes(L, lam, J0, precision, unrotated, complex_map, spin))
        p = params(L, lam, J0, spin=spin, precision=precision, unrotated=unrotated,
                   complex_map=complex_map)
        _check(lib.cvl_curvelet_scaling_synthesis(self.h, ctypes.byref(p), scal.data_ptr(),
                                                  flm_acc.data_ptr(), ws.data_ptr(), ws.numel(),
                                                  _stream(self.torch)))
        return flm_acc

    def round_trip_streamed(self, fmap, lam=2.0, J0=2, precision=CVL_FP64, on_grid=None,
                            real_grids=False, unrotated=False, spin=0):
        """Analysis + synthesis of one map (real float64, or complex128 of spin
        `spin`), one scale at a time (a single grid buffer of the largest
        scale is reused).  on_grid(j, grid), if given, sees each scale's grid
        between its analysis and synthesis."""
        t = self.torch
        L = fmap.shape[-2]
        cplx = fmap.dtype == t.complex128
        kw = dict(precision=precision, unrotated=unrotated, complex_map=cplx, spin=spin)
        flm = self.sht_forward(fmap, spin=spin)
        acc = t.zeros(L * L, dtype=t.complex128, device=self.device)
        scal = self.scaling_analysis(flm, L, lam, J0, **kw)
        J = num_scales(L, lam, J0)
        Lt, _ = scale_shape(L, J, lam, J0)
        buf = t.empty((2 * Lt - 1) * Lt * (2 * Lt - 1),
                      dtype=self.grid_dtype(precision, real_grids), device=self.device)
        for j in range(J0, J + 1):
            Lj, _ = scale_shape(L, j, lam, J0)
            g = buf[:(2 * Lj - 1) * Lj * (2 * Lj - 1)].view(2 * Lj - 1, Lj, 2 * Lj - 1)
            self.analysis_scale(flm, L, j, lam, J0, out=g, real_grids=real_grids, **kw)
            if on_grid is not None:
                on_grid(j, g)
            self.synthesis_scale(g, L, j, acc, lam, J0, real_grids=real_grids, **kw)
        self.scaling_synthesis(scal, L, acc, lam, J0, **kw)
        return self.sht_inverse(acc, L, spin=spin, complex_map=cplx), scal

    def delta_block(self, l):
        out = np.zeros((l + 1, l + 1))
        _check(lib.cvl_delta_block(self.h, l, out.ctypes.data_as(_c_double_p)))
        return out

    # ---- profiling ----
    def profile_enable(self, on=True):
        _check(lib.cvl_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        n = ctypes.c_int()
        mx = 32
        names = (ctypes.c_char_p * mx)()
        launches = (ctypes.c_int * mx)()
        ms = (ctypes.c_double * mx)()
        _check(lib.cvl_profile_read(self.h, mx, ctypes.byref(n), names, launches, ms))
        return {names[i].decode(): (launches[i], ms[i]) for i in range(min(n.value, mx))}

    def profile_filter(self, stage=None, bandlimit=0):
        """Time only the launches of `stage` (a name from profile_read) at
        `bandlimit`; None times every launch again."""
        idx = -1 if stage is None else list(self.profile_read().keys()).index(stage)
        _check(lib.cvl_profile_filter(self.h, idx, int(bandlimit)))

    def profile_read_detail(self):
        """{(stage name, band-limit): (launches, ms)} of the timed launches."""
        stage_names = list(self.profile_read().keys())
        n = ctypes.c_int()
        mx = 512
        st = (ctypes.c_int * mx)()
        bl = (ctypes.c_int * mx)()
        launches = (ctypes.c_int * mx)()
        ms = (ctypes.c_double * mx)()
        _check(lib.cvl_profile_read_detail(self.h, mx, ctypes.byref(n), st, bl, launches, ms))
        return {(stage_names[st[i]], bl[i]): (launches[i], ms[i]) for i in range(min(n.value, mx))}
