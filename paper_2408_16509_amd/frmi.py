"""Thin ctypes binding of libfrmi.so (the C ABI declared in include/frmi.h).

Argument marshalling only: every step of the right-hand side, the RK update, the
filter and the MLP run in the library's HIP kernels.  Device buffers are PyTorch
CUDA tensors (device memory and the stream come from PyTorch).  Importing this
module raises if the built library is missing.
"""
from __future__ import annotations

import ctypes
import functools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrmi.so")

FR_EULER, FR_NAVIER_STOKES = 0, 1
FR_RUSANOV, FR_HLLC = 0, 1
FR_FP64, FR_FP32, FR_FP32_BF16X3 = 0, 1, 2
FR_HEX, FR_TET, FR_PYR = 0, 1, 2
FR_METRIC_CONSERVATIVE, FR_METRIC_CROSS = 0, 1
(FR_OK, FR_ERR_ARG, FR_ERR_MESH, FR_ERR_ALLOC, FR_ERR_DEVICE, FR_ERR_NONFINITE, FR_ERR_STATE,
 FR_ERR_UNSUPPORTED) = range(8)
FR_MLP_STATIC_MAX_BATCH = 4096       # batch limit of fr_mlp_grad_static
STATUS = {0: "FR_OK", 1: "FR_ERR_ARG", 2: "FR_ERR_MESH", 3: "FR_ERR_ALLOC", 4: "FR_ERR_DEVICE",
          5: "FR_ERR_NONFINITE", 6: "FR_ERR_STATE", 7: "FR_ERR_UNSUPPORTED"}


class FrParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("system", ctypes.c_int32), ("order", ctypes.c_int32),
        ("riemann", ctypes.c_int32), ("precision", ctypes.c_int32), ("elem_order", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("ldg_beta", ctypes.c_double), ("ldg_tau", ctypes.c_double), ("u_ref", ctypes.c_double * 5),
        ("filt_eps_rho", ctypes.c_double), ("filt_eps_p", ctypes.c_double), ("filt_eps_s", ctypes.c_double),
        ("filt_zeta_max_coef", ctypes.c_double), ("filt_bits", ctypes.c_int32), ("hex_metric", ctypes.c_int32),
    ]


class FrLayout(ctypes.Structure):
    _fields_ = [
        ("n_types", ctypes.c_int32), ("etype", ctypes.c_int32 * 2), ("n_elem", ctypes.c_int64 * 2),
        ("e_pad", ctypes.c_int64 * 2), ("n_sp", ctypes.c_int32 * 2), ("n_fp", ctypes.c_int32 * 2),
        ("canon_offset", ctypes.c_int64 * 2), ("native_offset", ctypes.c_int64 * 2),
        ("canon_len", ctypes.c_int64), ("native_len", ctypes.c_int64),
        ("native_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class FrFilterStats(ctypes.Structure):
    _fields_ = [("n_troubled", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("n_evals", ctypes.c_int64), ("seconds", ctypes.c_double), ("n_candidates", ctypes.c_int64)]


class FrAdaptiveParams(ctypes.Structure):
    _fields_ = [("atol", ctypes.c_double), ("rtol", ctypes.c_double), ("safety", ctypes.c_double),
                ("fac_min", ctypes.c_double), ("fac_max", ctypes.c_double), ("max_attempts", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class FrAdaptiveStats(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64), ("n_rhs", ctypes.c_int64),
                ("t", ctypes.c_double), ("dt_next", ctypes.c_double), ("last_norm", ctypes.c_double)]


class FrKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


EXPORTS = [
    "fr_default_params", "fr_setup_mesh", "fr_setup_mesh_curved", "fr_setup_mesh_curved_tet", "fr_layout", "fr_sol_points", "fr_pack", "fr_unpack",
    "fr_pack64", "fr_unpack64", "fr_unpack_rhs",
    "fr_rhs", "fr_rk_step", "fr_default_adaptive_params", "fr_rk_adaptive", "fr_filter", "fr_mlp_set_weights", "fr_mlp_get_weights",
    "fr_mlp_features", "fr_mlp_collect", "fr_mlp_forward", "fr_mlp_grad", "fr_mlp_grad_static", "fr_mlp_train", "fr_check", "fr_sync",
    "fr_profile", "fr_profile_read",
    "fr_destroy", "fr_last_error",
]


def load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2408_16509_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "fr_default_params": (None, [P(FrParams)]),
        "fr_setup_mesh": (i32, [P(FrParams), i64, vp, vp, i64, vp, vp, vp, P(vp)]),
        "fr_setup_mesh_curved": (i32, [P(FrParams), i32, i64, vp, vp, i64, vp, vp, P(vp)]),
        "fr_setup_mesh_curved_tet": (i32, [P(FrParams), i32, i64, vp, vp, i64, vp, vp, P(vp)]),
        "fr_layout": (i32, [vp, P(FrLayout)]),
        "fr_sol_points": (i32, [vp, vp]),
        "fr_pack": (i32, [vp, vp, vp]),
        "fr_unpack": (i32, [vp, vp, vp]),
        "fr_pack64": (i32, [vp, vp, vp]),
        "fr_unpack64": (i32, [vp, vp, vp]),
        "fr_unpack_rhs": (i32, [vp, vp, vp]),
        "fr_rhs": (i32, [vp, vp, vp]),
        "fr_rk_step": (i32, [vp, vp, dbl, i32, i32]),
        "fr_default_adaptive_params": (None, [P(FrAdaptiveParams)]),
        "fr_rk_adaptive": (i32, [vp, vp, dbl, dbl, P(FrAdaptiveParams), P(FrAdaptiveStats)]),
        "fr_filter": (i32, [vp, vp, vp, i32, vp, P(FrFilterStats)]),
        "fr_mlp_set_weights": (i32, [vp, vp, vp, vp]),
        "fr_mlp_get_weights": (i32, [vp, vp]),
        "fr_mlp_features": (i32, [vp, vp, vp, vp, vp, vp, i64, P(i64)]),
        "fr_mlp_collect": (i32, [vp, vp, dbl, i32, vp, vp, i64, P(i64)]),
        "fr_mlp_forward": (i32, [vp, vp, i64, vp]),
        "fr_mlp_grad": (i32, [vp, vp, vp, i64, vp, vp]),
        "fr_mlp_grad_static": (i32, [vp, vp, vp, i64, vp, vp]),
        "fr_mlp_train": (i32, [vp, vp, vp, i64, vp, i32, i32, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, vp]),
        "fr_check": (i32, [vp, vp]),
        "fr_sync": (i32, [vp]),
        "fr_profile": (i32, [vp, i32]),
        "fr_profile_read": (i32, [vp, vp, i32, P(i32)]),
        "fr_destroy": (None, [vp]),
        "fr_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class FrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def default_params(**kw) -> FrParams:
    p = FrParams()
    lib().fr_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "u_ref":
            for i in range(5):
                p.u_ref[i] = float(v[i])
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _on_ctx_stream(fn):
    """Run a method's torch work (allocations, host-to-device copies) on the context's stream,
    so buffers the binding creates are ordered with the library calls that consume them."""
    @functools.wraps(fn)
    def wrapped(self, *a, **kw):
        with self._torch.cuda.stream(self._tstream):
            return fn(self, *a, **kw)
    return wrapped


class Context:
    """An FR context on one mesh.  `stream` defaults to torch's current stream.  Buffers the
    binding creates (packed states, outputs) are made on the context's stream; tensors the
    caller passes in must be ready on that stream, and results read on another stream need
    that stream to wait for this one, as for any stream-ordered library.

    A mesh with `ho_enodes` set (curved elements of geometry order `mesh.geo_order`) is
    set up through fr_setup_mesh_curved (hexahedra, tensor-order nodes) or
    fr_setup_mesh_curved_tet (tetrahedra), with the metric chosen by the `hex_metric`
    parameter (FR_METRIC_CONSERVATIVE or FR_METRIC_CROSS); any other mesh through
    fr_setup_mesh.  Keyword parameters are fr_params fields."""

    def __init__(self, mesh, stream=None, **params):
        import torch
        self._torch = torch
        self.params = default_params(**params)
        xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        per = np.ascontiguousarray(mesh.period, dtype=np.float64)
        et = np.ascontiguousarray(mesh.etype, dtype=np.int32)
        en = np.ascontiguousarray(mesh.enodes, dtype=np.int64)
        cur = torch.cuda.current_stream()
        if stream is None or stream == cur.cuda_stream:
            stream, self._tstream = cur.cuda_stream, cur
        else:
            self._tstream = torch.cuda.ExternalStream(stream)
        self.stream = stream
        h = ctypes.c_void_p()
        ho = getattr(mesh, "ho_enodes", None)
        if ho is not None:
            # curved elements of one type, nodes of geometry order mesh.geo_order
            ho = np.ascontiguousarray(ho, dtype=np.int64)
            setup = lib().fr_setup_mesh_curved_tet if np.all(et == 1) else lib().fr_setup_mesh_curved
            st = setup(ctypes.byref(self.params), int(mesh.geo_order), xyz.shape[0],
                       xyz.ctypes.data, per.ctypes.data, ho.shape[0], ho.ctypes.data,
                       ctypes.c_void_p(stream), ctypes.byref(h))
        else:
            st = lib().fr_setup_mesh(ctypes.byref(self.params), xyz.shape[0], xyz.ctypes.data, per.ctypes.data,
                                     et.shape[0], et.ctypes.data, en.ctypes.data, ctypes.c_void_p(stream),
                                     ctypes.byref(h))
        if st != 0:
            raise FrError(st, lib().fr_last_error(None).decode())
        self.h = h
        lay = FrLayout()
        self._check(lib().fr_layout(self.h, ctypes.byref(lay)))
        self.layout = lay

    def _check(self, st):
        if st != 0:
            raise FrError(st, lib().fr_last_error(self.h).decode())

    # --------------------------------------------------------------- buffers
    @property
    def native_dtype(self):
        return self._torch.float64 if self.layout.native_dtype == FR_FP64 else self._torch.float32

    @_on_ctx_stream
    def new_native(self, dtype=None):
        return self._torch.zeros(self.layout.native_len, dtype=dtype or self.native_dtype, device="cuda")

    @_on_ctx_stream
    def new_native64(self):
        return self._torch.zeros(self.layout.native_len, dtype=self._torch.float64, device="cuda")

    def sol_points(self):
        n = self.layout.canon_len // 5
        out = np.empty((n, 3), dtype=np.float64)
        self._check(lib().fr_sol_points(self.h, out.ctypes.data))
        return out

    @_on_ctx_stream
    def pack(self, canon, out=None):
        torch = self._torch
        c = torch.as_tensor(canon, dtype=torch.float64, device="cuda").contiguous()
        if out is None:
            out = self.new_native()
        self._check(lib().fr_pack(self.h, _ptr(c), _ptr(out)))
        return out

    @_on_ctx_stream
    def unpack(self, native, out=None):
        torch = self._torch
        if out is None:
            out = torch.empty(self.layout.canon_len, dtype=torch.float64, device="cuda")
        self._check(lib().fr_unpack(self.h, _ptr(native), _ptr(out)))
        return out

    @_on_ctx_stream
    def pack64(self, canon, out=None):
        """Canonical FP64 -> FP64 native state (what rk_step / filter / check use)."""
        torch = self._torch
        c = torch.as_tensor(canon, dtype=torch.float64, device="cuda").contiguous()
        if out is None:
            out = self.new_native64()
        self._check(lib().fr_pack64(self.h, _ptr(c), _ptr(out)))
        return out

    @_on_ctx_stream
    def unpack64(self, native, out=None):
        torch = self._torch
        if out is None:
            out = torch.empty(self.layout.canon_len, dtype=torch.float64, device="cuda")
        self._check(lib().fr_unpack64(self.h, _ptr(native), _ptr(out)))
        return out

    @_on_ctx_stream
    def unpack_rhs(self, r, out=None):
        """Native right-hand side -> canonical FP64 (no reference state added)."""
        torch = self._torch
        if out is None:
            out = torch.empty(self.layout.canon_len, dtype=torch.float64, device="cuda")
        self._check(lib().fr_unpack_rhs(self.h, _ptr(r), _ptr(out)))
        return out

    # --------------------------------------------------------------- compute
    def rhs(self, u, r):
        self._check(lib().fr_rhs(self.h, _ptr(u), _ptr(r)))

    def rk_step(self, u, dt, n_steps=1, filter_mode=-1):
        self._check(lib().fr_rk_step(self.h, _ptr(u), float(dt), int(n_steps), int(filter_mode)))

    @_on_ctx_stream
    def rk_adaptive(self, u, t_end, dt0, **params):
        """Adaptive steps of the embedded pair from t = 0 to t_end (FP64 native state u, in
        place); params override fr_default_adaptive_params (atol, rtol, safety, fac_min,
        fac_max, max_attempts).  Returns the FrAdaptiveStats."""
        p = FrAdaptiveParams()
        lib().fr_default_adaptive_params(ctypes.byref(p))
        for k, v in params.items():
            setattr(p, k, v)
        st = FrAdaptiveStats()
        self._check(lib().fr_rk_adaptive(self.h, _ptr(u), float(t_end), float(dt0), ctypes.byref(p),
                                          ctypes.byref(st)))
        return st

    @_on_ctx_stream
    def filter(self, u, u_prev=None, mode=0, k=None, stats=False):
        s = FrFilterStats() if stats else None
        self._check(lib().fr_filter(self.h, _ptr(u), _ptr(u if u_prev is None else u_prev), int(mode),
                                    _ptr(k), ctypes.byref(s) if stats else None))
        return s

    # --------------------------------------------------------------- learned warm start
    def mlp_set_weights(self, w, x_mean, x_std):
        w = np.ascontiguousarray(w, dtype=np.float32)
        xm = np.ascontiguousarray(x_mean, dtype=np.float32)
        xs = np.ascontiguousarray(x_std, dtype=np.float32)
        self._check(lib().fr_mlp_set_weights(self.h, w.ctypes.data, xm.ctypes.data, xs.ctypes.data))

    def mlp_get_weights(self):
        w = np.empty(5313, dtype=np.float32)
        self._check(lib().fr_mlp_get_weights(self.h, w.ctypes.data))
        return w

    @_on_ctx_stream
    def mlp_features(self, u, u_prev, cap):
        torch = self._torch
        x = torch.zeros((max(cap, 1), 16), dtype=torch.float32, device="cuda")
        el = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
        k = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
        n = ctypes.c_int64()
        self._check(lib().fr_mlp_features(self.h, _ptr(u), _ptr(u_prev), _ptr(x), _ptr(el), _ptr(k), int(cap),
                                          ctypes.byref(n)))
        m = min(n.value, cap)
        return x[:m], el[:m], k[:m], n.value

    @_on_ctx_stream
    def mlp_collect(self, u, dt, n_steps, cap):
        torch = self._torch
        x = torch.zeros((max(cap, 1), 16), dtype=torch.float32, device="cuda")
        k = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
        n = ctypes.c_int64()
        self._check(lib().fr_mlp_collect(self.h, _ptr(u), float(dt), int(n_steps), _ptr(x), _ptr(k), int(cap),
                                         ctypes.byref(n)))
        return x[:n.value], k[:n.value]

    @_on_ctx_stream
    def mlp_forward(self, x):
        torch = self._torch
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        self._check(lib().fr_mlp_forward(self.h, _ptr(x), int(x.shape[0]), _ptr(y)))
        return y

    @_on_ctx_stream
    def mlp_grad(self, x, y):
        torch = self._torch
        g = torch.empty(5313, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        self._check(lib().fr_mlp_grad(self.h, _ptr(x), _ptr(y), int(x.shape[0]), _ptr(g), _ptr(loss)))
        return g, loss

    def mlp_grad_static(self, x, y, grad, loss):
        """fr_mlp_grad_static: the caller brings the outputs (grad [5313], loss [1], FP32 device)."""
        self._check(lib().fr_mlp_grad_static(self.h, _ptr(x), _ptr(y), int(x.shape[0]), _ptr(grad), _ptr(loss)))
        return grad, loss

    @_on_ctx_stream
    def mlp_train(self, x, y, perm, n_steps, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        torch = self._torch
        hist = torch.empty(max(n_steps, 1), dtype=torch.float32, device="cuda")
        self._check(lib().fr_mlp_train(self.h, _ptr(x), _ptr(y), int(x.shape[0]), _ptr(perm), int(n_steps),
                                       int(batch), lr, beta1, beta2, eps, _ptr(hist)))
        return hist[:n_steps]

    def check(self, u):
        st = lib().fr_check(self.h, _ptr(u))
        if st == 5:
            return False
        self._check(st)
        return True

    def sync(self):
        self._check(lib().fr_sync(self.h))

    def profile(self, enable=True):
        self._check(lib().fr_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """{kernel family: (launches, total device ms)} from the event timing."""
        buf = (FrKernelTime * 64)()
        n = ctypes.c_int32()
        self._check(lib().fr_profile_read(self.h, buf, 64, ctypes.byref(n)))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n.value)}

    def close(self):
        if getattr(self, "h", None):
            lib().fr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # canonical helpers (host numpy <-> device)
    def split_canon(self, flat):
        """Canonical flat array -> list of per-block [n][5][nsp] arrays."""
        out = []
        for i in range(self.layout.n_types):
            o, n, s = self.layout.canon_offset[i], self.layout.n_elem[i], self.layout.n_sp[i]
            out.append(flat[o:o + n * 5 * s].reshape(n, 5, s))
        return out

    def join_canon(self, blocks):
        return np.concatenate([np.asarray(b, dtype=np.float64).ravel() for b in blocks])
