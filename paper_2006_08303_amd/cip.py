"""ctypes binding of the C ABI in include/cip.h.

Argument marshalling only: every step of the reconstruction runs in the HIP
library. Device memory and streams come from PyTorch (ROCm build); the
library is loaded from this package directory and a missing library is an
error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CIP_LIBRARY_PATH") or os.path.join(_HERE, "libcip.so")

SUPPORTED_N = (16, 32, 64, 128, 256, 384, 512, 768, 1024, 1536, 2048)   # grid sizes served

CIP_PRIOR_TV2D = 0
CIP_PRIOR_TV3D = 1
CIP_PRIOR_DCT2D = 2
CIP_PRIOR_PATCH = 3
CIP_PRIOR_CONV2D = 4
CIP_PRIOR_DCT3D = 5
CIP_PRIOR_ITV2D = 6
CIP_PRIOR_CONV3D = 7
CIP_PRIOR_WDCT3D = 8
CIP_PRIOR_ITV3D = 9
PRIORS = {"tv2d": CIP_PRIOR_TV2D, "tv3d": CIP_PRIOR_TV3D, "dct2d": CIP_PRIOR_DCT2D,
          "patch": CIP_PRIOR_PATCH, "conv2d": CIP_PRIOR_CONV2D, "dct3d": CIP_PRIOR_DCT3D,
          "itv2d": CIP_PRIOR_ITV2D, "conv3d": CIP_PRIOR_CONV3D, "wdct3d": CIP_PRIOR_WDCT3D,
          "itv3d": CIP_PRIOR_ITV3D}


class CipError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cip error {code}: {msg}")
        self.code = code


class _PriorDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("beta", ctypes.c_double),
                ("dict", ctypes.c_void_p), ("n_atoms", ctypes.c_int),
                ("patch_q", ctypes.c_int), ("patch_stride", ctypes.c_int),
                ("filters", ctypes.c_void_p), ("n_filters", ctypes.c_int),
                ("filt_l", ctypes.c_int), ("mu", ctypes.c_double), ("tv_inner", ctypes.c_int),
                ("flags", ctypes.c_int), ("sigma", ctypes.c_double),
                ("wt_levels", ctypes.c_int), ("patch_t", ctypes.c_int), ("per_band", ctypes.c_int)]


class _AdaptiveParams(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int), ("every", ctypes.c_int), ("tau", ctypes.c_double),
                ("mu", ctypes.c_double), ("tol", ctypes.c_double), ("adapt_sigma", ctypes.c_int)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rho_changes", ctypes.c_int), ("rho", ctypes.c_double),
                ("rel_change", ctypes.c_double), ("r_norm", ctypes.c_double),
                ("s_norm", ctypes.c_double), ("sigma", ctypes.c_double),
                ("sigma_changes", ctypes.c_int)]


CIP_PLAN_ADAPTIVE = 1
CIP_PLAN_DICT_UPDATE = 2


class _Tuning(ctypes.Structure):
    _fields_ = [("row_np", ctypes.c_int), ("row_ppt", ctypes.c_int), ("candidates", ctypes.c_int),
                ("row_us", ctypes.c_double), ("default_us", ctypes.c_double)]


def _desc(prior, beta, dictionary=None, filters=None, mu=0.0, flags=0, tv_inner=0, sigma=0.0,
          wt_levels=0):
    d = _PriorDesc(PRIORS[prior], float(beta), None, 0, 8, 4, None, 0, 0, float(mu),
                   int(tv_inner), int(flags), float(sigma), int(wt_levels))
    if dictionary is not None:
        d.dict = ctypes.c_void_p(dictionary.data_ptr())
        d.n_atoms = int(dictionary.shape[1])
    if filters is not None:
        d.filters = ctypes.c_void_p(filters.data_ptr())
        d.n_filters = int(filters.shape[0])
        d.filt_l = int(filters.shape[-1])
    return d


class _ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("n_slots", ctypes.c_int),
                ("autotune", ctypes.c_int)]


class _Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("y", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("iters", ctypes.c_int)]


_lib = None


def lib():
    """Load libcip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.cip_plan_workspace_bytes.argtypes = [i, i, i, i, ctypes.POINTER(_PriorDesc),
                                               ctypes.POINTER(sz)]
        L.cip_plan_create.argtypes = [i, i, i, i, vp, ctypes.POINTER(_PriorDesc), d, d, vp, sz,
                                      vp, ctypes.POINTER(vp)]
        L.cip_forward.argtypes = [vp, vp, vp, vp]
        L.cip_adjoint.argtypes = [vp, vp, vp, vp]
        L.cip_solve.argtypes = [vp, vp, i, vp, vp]
        L.cip_plan_dictionary.argtypes = [vp, vp, vp]
        L.cip_plan_destroy.argtypes = [vp]
        L.cip_last_error.restype = ctypes.c_char_p
        L.cip_time_kernel.argtypes = [vp, i, i, vp, ctypes.POINTER(d)]
        L.cip_batch_create.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(i), ctypes.POINTER(vp), i, i,
                                       ctypes.POINTER(vp)]
        L.cip_batch_launch.argtypes = [vp, vp]
        L.cip_batch_solve.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i),
                                      ctypes.POINTER(vp), vp]
        L.cip_batch_destroy.argtypes = [vp]
        L.cip_plan_state_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.cip_plan_attach.argtypes = [vp, vp, sz, ctypes.POINTER(vp)]
        L.cip_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
        L.cip_server_add_operator.argtypes = [vp, i, i, i, i, vp, ctypes.POINTER(_PriorDesc), d, d,
                                              ctypes.POINTER(i)]
        L.cip_server_submit.argtypes = [vp, ctypes.POINTER(_Request),
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.cip_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i), ctypes.POINTER(d)]
        L.cip_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(d), ctypes.POINTER(d)]
        L.cip_server_destroy.argtypes = [vp]
        L.cip_solve_adaptive.argtypes = [vp, vp, ctypes.POINTER(_AdaptiveParams), vp, vp,
                                         ctypes.POINTER(_SolveInfo)]
        L.cip_plan_autotune.argtypes = [vp, i, vp, ctypes.POINTER(_Tuning)]
        L.cip_plan_set_tuning.argtypes = [vp, i, i]
        L.cip_solve_static.argtypes = [i, i, i, i, vp, ctypes.POINTER(_PriorDesc), d, d, vp, i, vp,
                                       vp]
        for name in ("cip_plan_workspace_bytes", "cip_plan_create", "cip_forward", "cip_adjoint",
                     "cip_solve", "cip_plan_destroy", "cip_time_kernel", "cip_batch_create",
                     "cip_batch_launch", "cip_batch_destroy", "cip_plan_state_bytes",
                     "cip_plan_attach", "cip_server_create", "cip_server_add_operator",
                     "cip_server_submit", "cip_server_poll", "cip_server_wait",
                     "cip_server_destroy", "cip_solve_adaptive", "cip_plan_autotune",
                     "cip_plan_set_tuning", "cip_solve_static", "cip_batch_solve"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise CipError(rc, lib().cip_last_error().decode())


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, shape, name):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def workspace_bytes(K, S, N1, N2, prior="dct2d", beta=1.0, n_atoms=0, n_filters=0, filt_l=0,
                    flags=0, sigma=0.0, wt_levels=0, tv_inner=0):
    desc = _desc(prior, beta, flags=flags, tv_inner=tv_inner, sigma=sigma, wt_levels=wt_levels)
    desc.n_atoms = int(n_atoms)
    desc.n_filters = int(n_filters)
    desc.filt_l = int(filt_l)
    n = ctypes.c_size_t()
    _check(lib().cip_plan_workspace_bytes(K, S, N1, N2, ctypes.byref(desc), ctypes.byref(n)))
    return n.value


class Plan:
    """One problem shape and operator: y_k = sum_s h_{k,s} * x_s.

    psf: float32 CUDA tensor [K, S, N1, N2] (unshifted kernels, origin at [0, 0]).
    dictionary: for prior="patch", float32 CUDA tensor [64 S, A] (atoms as
    columns, row s*64 + a*8 + b = pixel (a, b) of plane s).
    filters: for prior="conv2d", float32 CUDA tensor [M, L, L] (tap (a, b) at
    offset (a - L//2, b - L//2)); for prior="conv3d", [M, S, L, L] (band tap
    s' at band offset s'); mu: gradient (Tikhonov) weight on the codes
    (conv2d only). dict_update (patch and conv priors): learn the dictionary
    online in every solve with penalty sigma (0: 1 for the patch prior, 10 for
    the conv priors); dictionary() returns the learned dictionary or filters.
    wt_levels: wavelet levels of prior="wdct3d" (0: 3)."""

    def __init__(self, psf, prior="dct2d", rho=0.1, lam=0.01, beta=1.0, dictionary=None,
                 filters=None, stream=None, mu=0.0, adaptive=False, tv_inner=0,
                 dict_update=False, sigma=0.0, wt_levels=0):
        K, S, N1, N2 = psf.shape
        self.K, self.S, self.N1, self.N2 = int(K), int(S), int(N1), int(N2)
        self.prior, self.rho, self.lam, self.beta = prior, float(rho), float(lam), float(beta)
        if prior == "patch":
            if dictionary is None:
                raise ValueError("the patch prior needs a dictionary")
            _dev_f32(dictionary, (64 * self.S, dictionary.shape[1]), "dictionary")
        if prior in ("conv2d", "conv3d"):
            if filters is None:
                raise ValueError(f"the {prior} prior needs filters")
            if prior == "conv3d" and (filters.dim() != 4 or int(filters.shape[1]) != self.S):
                raise ValueError("conv3d filters must have shape [M, S, L, L]")
            _dev_f32(filters, tuple(filters.shape), "filters")
        flags = (CIP_PLAN_ADAPTIVE if adaptive else 0) | (CIP_PLAN_DICT_UPDATE if dict_update else 0)
        desc = _desc(prior, beta, dictionary, filters, mu, flags, tv_inner, sigma, wt_levels)
        self.filters_shape = (tuple(filters.shape) if filters is not None else
                              tuple(dictionary.shape) if dictionary is not None else None)
        nbytes = workspace_bytes(self.K, self.S, self.N1, self.N2, prior, beta,
                                 desc.n_atoms, desc.n_filters, desc.filt_l, desc.flags,
                                 desc.sigma, desc.wt_levels)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=psf.device)
        h = ctypes.c_void_p()
        _check(lib().cip_plan_create(self.K, self.S, self.N1, self.N2,
                                     _dev_f32(psf, (K, S, N1, N2), "psf"), ctypes.byref(desc),
                                     self.rho, self.lam, ctypes.c_void_p(self.workspace.data_ptr()),
                                     nbytes, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def forward(self, x, out=None, stream=None):
        y = out if out is not None else torch.empty((self.K, self.N1, self.N2),
                                                    dtype=torch.float32, device=x.device)
        _check(lib().cip_forward(self._h, _dev_f32(x, (self.S, self.N1, self.N2), "x"),
                                 _dev_f32(y, (self.K, self.N1, self.N2), "y"), _stream_ptr(stream)))
        return y

    def adjoint(self, y, out=None, stream=None):
        x = out if out is not None else torch.empty((self.S, self.N1, self.N2),
                                                    dtype=torch.float32, device=y.device)
        _check(lib().cip_adjoint(self._h, _dev_f32(y, (self.K, self.N1, self.N2), "y"),
                                 _dev_f32(x, (self.S, self.N1, self.N2), "x"), _stream_ptr(stream)))
        return x

    def solve(self, y, iters, out=None, stream=None):
        x = out if out is not None else torch.empty((self.S, self.N1, self.N2),
                                                    dtype=torch.float32, device=y.device)
        _check(lib().cip_solve(self._h, _dev_f32(y, (self.K, self.N1, self.N2), "y"), int(iters),
                               _dev_f32(x, (self.S, self.N1, self.N2), "x"), _stream_ptr(stream)))
        return x

    def solve_adaptive(self, y, max_iters, every=1, tau=2.0, mu=10.0, tol=1e-4, out=None,
                       stream=None, adapt_sigma=False):
        """cip_solve_adaptive; returns (x, info dict)."""
        x = out if out is not None else torch.empty((self.S, self.N1, self.N2),
                                                    dtype=torch.float32, device=y.device)
        prm = _AdaptiveParams(int(max_iters), int(every), float(tau), float(mu), float(tol),
                              1 if adapt_sigma else 0)
        info = _SolveInfo()
        _check(lib().cip_solve_adaptive(self._h, _dev_f32(y, (self.K, self.N1, self.N2), "y"),
                                        ctypes.byref(prm),
                                        _dev_f32(x, (self.S, self.N1, self.N2), "x"),
                                        _stream_ptr(stream), ctypes.byref(info)))
        return x, {f: getattr(info, f) for f, _ in _SolveInfo._fields_}

    def autotune(self, reps=20, stream=None):
        """cip_plan_autotune: returns the chosen row-pass shape and timings."""
        tu = _Tuning()
        _check(lib().cip_plan_autotune(self._h, int(reps), _stream_ptr(stream), ctypes.byref(tu)))
        return {f: getattr(tu, f) for f, _ in _Tuning._fields_}

    def set_tuning(self, row_np, row_ppt):
        _check(lib().cip_plan_set_tuning(self._h, int(row_np), int(row_ppt)))

    def attach(self):
        """A plan sharing this plan's tables with a solve state of its own
        (cip_plan_attach); the state buffer is allocated here."""
        return AttachedPlan(self)

    def dictionary(self, stream=None):
        """The dictionary learned in the last solve (dict_update plans): the
        filters' shape, or [64 S, A] for the patch prior."""
        out = torch.empty(self.filters_shape, dtype=torch.float32, device=self.workspace.device)
        _check(lib().cip_plan_dictionary(self._h, ctypes.c_void_p(out.data_ptr()),
                                         _stream_ptr(stream)))
        return out

    def time_kernel(self, which, reps, stream=None):
        us = ctypes.c_double()
        _check(lib().cip_time_kernel(self._h, int(which), int(reps), _stream_ptr(stream),
                                     ctypes.byref(us)))
        return us.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cip_plan_destroy(h)
            self._h = None


STATIC_WORKSPACE_BYTES = 64 << 20   # CIP_STATIC_WORKSPACE_BYTES


def solve_static(psf, y, iters, prior="dct2d", rho=0.1, lam=0.01, beta=1.0, dictionary=None,
                 filters=None, mu=0.0, tv_inner=0, wt_levels=0, out=None, stream=None):
    """cip_solve_static: a whole reconstruction (plan tables and solve state)
    in the library's static device buffer; no device memory is allocated by
    the library (out is allocated here unless given). Synchronous."""
    K, S, N1, N2 = (int(v) for v in psf.shape)
    desc = _desc(prior, beta, dictionary, filters, mu, 0, tv_inner, 0.0, wt_levels)
    x = out if out is not None else torch.empty((S, N1, N2), dtype=torch.float32, device=y.device)
    _check(lib().cip_solve_static(K, S, N1, N2, _dev_f32(psf, (K, S, N1, N2), "psf"),
                                  ctypes.byref(desc), float(rho), float(lam),
                                  _dev_f32(y, (K, N1, N2), "y"), int(iters),
                                  _dev_f32(x, (S, N1, N2), "x"), _stream_ptr(stream)))
    return x


def batch_solve(problems, stream=None):
    """cip_batch_solve: problems is a list of (plan, y, iters, x) with
    distinct plans; the solves run over the library's internal streams,
    asynchronously on `stream`."""
    n = len(problems)
    if n == 0:
        raise ValueError("empty batch")
    vp = ctypes.c_void_p
    plans, ys, xs, its = (vp * n)(), (vp * n)(), (vp * n)(), (ctypes.c_int * n)()
    for j, (plan, y, iters, x) in enumerate(problems):
        plans[j] = plan._h.value
        ys[j] = _dev_f32(y, (plan.K, plan.N1, plan.N2), "y").value
        xs[j] = _dev_f32(x, (plan.S, plan.N1, plan.N2), "x").value
        its[j] = int(iters)
    _check(lib().cip_batch_solve(n, plans, ys, its, xs, _stream_ptr(stream)))


class Batch:
    """Independent solves run together (cip_batch_create / cip_batch_launch).

    problems: list of (plan, y, iters, x) with distinct plans; y [K, N1, N2] and
    x [S, N1, N2] float32 CUDA tensors that must outlive the batch. With
    graph=True the whole batch is captured once into a hipGraph and every
    launch() replays it."""

    def __init__(self, problems, n_streams=4, graph=True):
        n = len(problems)
        if n == 0:
            raise ValueError("empty batch")
        vp = ctypes.c_void_p
        plans = (vp * n)()
        ys = (vp * n)()
        xs = (vp * n)()
        its = (ctypes.c_int * n)()
        for j, (plan, y, iters, x) in enumerate(problems):
            plans[j] = plan._h.value
            ys[j] = _dev_f32(y, (plan.K, plan.N1, plan.N2), "y").value
            xs[j] = _dev_f32(x, (plan.S, plan.N1, plan.N2), "x").value
            its[j] = int(iters)
        self._keep = list(problems)
        h = vp()
        _check(lib().cip_batch_create(n, plans, ys, its, xs, int(n_streams), int(bool(graph)),
                                      ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().cip_batch_launch(self._h, _stream_ptr(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cip_batch_destroy(h)
            self._h = None


class AttachedPlan(Plan):
    """Plan that shares `base`'s tables (cip_plan_attach) and owns a solve
    state buffer."""

    def __init__(self, base):
        self.K, self.S, self.N1, self.N2 = base.K, base.S, base.N1, base.N2
        self.prior, self.rho, self.lam, self.beta = base.prior, base.rho, base.lam, base.beta
        self._base = base
        n = ctypes.c_size_t()
        _check(lib().cip_plan_state_bytes(base._h, ctypes.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=base.workspace.device)
        h = ctypes.c_void_p()
        _check(lib().cip_plan_attach(base._h, ctypes.c_void_p(self.workspace.data_ptr()), n.value,
                                     ctypes.byref(h)))
        self._h = h


class Server:
    """Request server (cip_server_*): operators registered once, requests
    with host numpy buffers, continuous batching over n_slots streams."""

    def __init__(self, hbm_budget_bytes, n_slots=4, autotune=False):
        cfg = _ServerConfig(int(hbm_budget_bytes), int(n_slots), int(bool(autotune)))
        h = ctypes.c_void_p()
        _check(lib().cip_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self.ops = []

    def add_operator(self, psf, prior="tv3d", rho=1e-2, lam=1e-3, beta=1.0, dictionary=None,
                     filters=None):
        K, S, N1, N2 = (int(v) for v in psf.shape)
        desc = _desc(prior, beta, dictionary, filters)
        # the library reads the kernels on its own stream: finish writing them
        torch.cuda.current_stream(psf.device).synchronize()
        op = ctypes.c_int()
        _check(lib().cip_server_add_operator(self._h, K, S, N1, N2,
                                             _dev_f32(psf, (K, S, N1, N2), "psf"),
                                             ctypes.byref(desc), float(rho), float(lam),
                                             ctypes.byref(op)))
        self.ops.append((K, S, N1, N2))
        return op.value

    def submit(self, op, y, x, iters):
        """y: float32 C-contiguous numpy [K, N1, N2]; x: float32 numpy
        [S, N1, N2] written on completion. Returns the ticket."""
        import numpy as np
        K, S, N1, N2 = self.ops[op]
        for a, shp, nm in ((y, (K, N1, N2), "y"), (x, (S, N1, N2), "x")):
            if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags.c_contiguous
                    and a.shape == shp):
                raise ValueError(f"{nm} must be a C-contiguous float32 array of shape {shp}")
        req = _Request(int(op), ctypes.c_void_p(y.ctypes.data), ctypes.c_void_p(x.ctypes.data),
                       int(iters))
        t = ctypes.c_uint64()
        _check(lib().cip_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (y, x)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int()
        lat = ctypes.c_double()
        _check(lib().cip_server_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(lat)))
        return bool(done.value), lat.value

    def wait(self, ticket):
        """Block until done; returns (latency_s, queue_s)."""
        lat, qs = ctypes.c_double(), ctypes.c_double()
        rc = lib().cip_server_wait(self._h, int(ticket), ctypes.byref(lat), ctypes.byref(qs))
        self._keep.pop(int(ticket), None)
        _check(rc)
        return lat.value, qs.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cip_server_destroy(h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        self.close()
