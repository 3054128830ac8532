"""ctypes binding of the gfx950 2SHOC-RK4 library (C ABI in include/nlse.h).

Argument marshalling only: every numerical step runs in the HIP kernels of
``libnlse_hip.so``.  There is no CPU path; if the library is missing the import
fails.  PyTorch, when used, only provides device memory and the stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlse_hip.so")

OK, E_INVAL, E_DT_UNSTABLE, E_NONFINITE, E_NOMEM, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PREC = {"f64": 0, "f32": 1, "mixed": 2}
BC = {"dirichlet": 0, "msd": 1}
_STATUS = {E_INVAL: "NLSE_E_INVAL", E_DT_UNSTABLE: "NLSE_E_DT_UNSTABLE", E_NONFINITE: "NLSE_E_NONFINITE",
           E_NOMEM: "NLSE_E_NOMEM", E_HIP: "NLSE_E_HIP", E_UNSUPPORTED: "NLSE_E_UNSUPPORTED"}


class NLSEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("a", ctypes.c_double), ("s", ctypes.c_double), ("V", ctypes.POINTER(ctypes.c_double)),
                ("bc", ctypes.c_int32), ("prec", ctypes.c_int32), ("allow_unstable", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


EXPORTS = ["nlse_create", "nlse_set_field", "nlse_step", "nlse_get_field", "nlse_mass", "nlse_energy",
           "nlse_max_dt", "nlse_sync", "nlse_destroy", "nlse_last_error", "nlse_launches_per_step",
           "nlse_variant_count", "nlse_set_variant", "nlse_get_variant", "nlse_autotune",
           "nlse_set_stencil", "nlse_get_stencil",
           "nlse_batch_create", "nlse_batch_count", "nlse_batch_set_field", "nlse_batch_get_field",
           "nlse_batch_set_dt", "nlse_batch_max_dt", "nlse_batch_mass", "nlse_batch_step", "nlse_batch_sync",
           "nlse_batch_variant_count", "nlse_batch_set_variant", "nlse_batch_get_variant",
           "nlse_batch_autotune", "nlse_batch_destroy",
           "nlse_corr_param_count", "nlse_corr_create", "nlse_corr_set_params", "nlse_corr_get_params",
           "nlse_corr_infer", "nlse_corr_grads", "nlse_corr_train_step", "nlse_corr_apply",
           "nlse_step_corrected", "nlse_corr_destroy", "nlse_inject", "nlse_corr_set_target_filter",
           "nlse_corr_set_augment", "nlse_mass_noalloc", "nlse_corr_tensor", "nlse_corr_stage"]

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1109_1027_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    L.nlse_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params)]
    L.nlse_set_field.argtypes = [vp, vp, ctypes.c_int]
    L.nlse_step.argtypes = [vp, i64, dbl]
    L.nlse_get_field.argtypes = [vp, vp, ctypes.c_int]
    for f in ("nlse_mass", "nlse_energy", "nlse_max_dt"):
        getattr(L, f).argtypes = [vp, ctypes.POINTER(dbl)]
    L.nlse_sync.argtypes = [vp]
    L.nlse_destroy.argtypes = [vp]
    L.nlse_destroy.restype = None
    L.nlse_last_error.restype = ctypes.c_char_p
    L.nlse_launches_per_step.argtypes = [vp]
    L.nlse_variant_count.argtypes = [vp]
    L.nlse_set_variant.argtypes = [vp, ctypes.c_int]
    L.nlse_get_variant.argtypes = [vp]
    L.nlse_set_stencil.argtypes = [vp, ctypes.c_int32]
    L.nlse_get_stencil.argtypes = [vp]
    L.nlse_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    i32 = ctypes.c_int32
    L.nlse_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), i32]
    L.nlse_batch_count.argtypes = [vp]
    L.nlse_batch_set_field.argtypes = [vp, i32, vp, ctypes.c_int]
    L.nlse_batch_get_field.argtypes = [vp, i32, vp, ctypes.c_int]
    L.nlse_batch_set_dt.argtypes = [vp, i32, dbl]
    L.nlse_batch_max_dt.argtypes = [vp, i32, ctypes.POINTER(dbl)]
    L.nlse_batch_mass.argtypes = [vp, i32, ctypes.POINTER(dbl)]
    L.nlse_batch_step.argtypes = [vp, i64]
    L.nlse_batch_sync.argtypes = [vp]
    L.nlse_batch_variant_count.argtypes = [vp]
    L.nlse_batch_set_variant.argtypes = [vp, ctypes.c_int]
    L.nlse_batch_get_variant.argtypes = [vp]
    L.nlse_batch_autotune.argtypes = [vp, i64, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.nlse_batch_destroy.argtypes = [vp]
    L.nlse_batch_destroy.restype = None
    fp = ctypes.POINTER(ctypes.c_float)
    L.nlse_corr_param_count.argtypes = []
    L.nlse_corr_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, ctypes.POINTER(dbl), vp]
    L.nlse_corr_set_params.argtypes = [vp, fp, dbl]
    L.nlse_corr_get_params.argtypes = [vp, fp]
    L.nlse_corr_infer.argtypes = [vp, vp, i32, vp]
    L.nlse_corr_grads.argtypes = [vp, vp, vp, i32, fp, ctypes.POINTER(dbl)]
    L.nlse_corr_train_step.argtypes = [vp, vp, vp, i32, dbl, ctypes.POINTER(dbl)]
    L.nlse_corr_apply.argtypes = [vp, vp]
    L.nlse_step_corrected.argtypes = [vp, vp, i64, dbl, i32]
    L.nlse_corr_destroy.argtypes = [vp]
    L.nlse_corr_destroy.restype = None
    L.nlse_inject.argtypes = [vp, i32, i64, vp, i64, i32, vp]
    L.nlse_corr_set_target_filter.argtypes = [vp, i32]
    L.nlse_corr_set_augment.argtypes = [vp, dbl, ctypes.c_uint64]
    L.nlse_mass_noalloc.argtypes = [i32, ctypes.POINTER(i64), dbl, i32, vp, vp, vp]
    L.nlse_corr_tensor.argtypes = [vp, i32, i32, vp, i64]
    L.nlse_corr_stage.argtypes = [vp, i32, i32]
    for f in EXPORTS:
        if f not in ("nlse_destroy", "nlse_last_error", "nlse_batch_destroy", "nlse_corr_destroy"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        raise NLSEError(rc, load().nlse_last_error().decode())


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return None


class Solver:
    """One NLSE problem on the GPU: i Psi_t + a Lap Psi - V Psi + s|Psi|^2 Psi = 0.

    n: intervals per axis (int or sequence), h: grid step, V: potential on all nodes
    (numpy, field order [z][y][x]) or None, bc: "dirichlet" | "msd" (1D),
    prec: "f64" | "f32" | "mixed".  Fields are complex128 ("f64", "mixed") or
    complex64 ("f32"), all (n+1)^d nodes including the boundary."""

    def __init__(self, ndim, n, h, a, s, V=None, bc="dirichlet", prec="f64", allow_unstable=False,
                 stream="current"):
        L = load()
        nn = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n,) * ndim))
        self.ndim, self.n, self.h, self.a, self.s = int(ndim), nn, float(h), float(a), float(s)
        self.prec, self.bc = prec, bc
        self.shape = tuple(v + 1 for v in reversed(nn[:ndim]))
        self.dtype = np.complex64 if prec == "f32" else np.complex128
        p = Params()
        p.ndim = self.ndim
        for i in range(3):
            p.n[i] = nn[i] if i < ndim else 0
        p.h, p.a, p.s = self.h, self.a, self.s
        self._V = None
        if V is not None:
            self._V = np.ascontiguousarray(V, dtype=np.float64)
            if self._V.size != int(np.prod(self.shape)):
                raise ValueError("V must hold one value per node")
            p.V = self._V.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.bc = BC[bc]
        p.prec = PREC[prec]
        p.allow_unstable = int(bool(allow_unstable))
        self.stream = _current_stream() if stream == "current" else stream
        p.stream = self.stream
        h_ = ctypes.c_void_p()
        _check(L.nlse_create(ctypes.byref(h_), ctypes.byref(p)))
        self._h = h_

    @classmethod
    def from_spec(cls, spec, prec="f64", **kw):
        g = spec.grid
        return cls(g.dim, g.n, g.h, spec.a, spec.s, spec.V, spec.bc, prec, **kw)

    def close(self):
        if getattr(self, "_h", None):
            load().nlse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- fields
    def set_field(self, psi):
        """psi: numpy array (host) or torch tensor on the GPU, all nodes, field dtype."""
        if _is_torch(psi):
            self._check_tensor(psi)
            _check(load().nlse_set_field(self._h, ctypes.c_void_p(psi.data_ptr()), 1))
        else:
            arr = np.ascontiguousarray(psi, dtype=self.dtype).reshape(self.shape)
            _check(load().nlse_set_field(self._h, arr.ctypes.data_as(ctypes.c_void_p), 0))

    def get_field(self, out=None):
        """Return the field as numpy, or copy it into the given GPU torch tensor."""
        if out is not None and _is_torch(out):
            self._check_tensor(out)
            _check(load().nlse_get_field(self._h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        arr = np.empty(self.shape, dtype=self.dtype)
        _check(load().nlse_get_field(self._h, arr.ctypes.data_as(ctypes.c_void_p), 0))
        return arr

    def _check_tensor(self, t):
        import torch
        want = torch.complex64 if self.dtype == np.complex64 else torch.complex128
        if t.dtype != want or not t.is_cuda or not t.is_contiguous() or t.numel() != int(np.prod(self.shape)):
            raise ValueError(f"tensor must be a contiguous {want} GPU tensor with {int(np.prod(self.shape))} elements")

    # ---- time stepping and diagnostics
    def step(self, nsteps, dt):
        _check(load().nlse_step(self._h, int(nsteps), float(dt)))

    def step_corrected(self, corrector, nsteps, dt, every=10):
        """nsteps RK4 steps with a learned correction after every `every` steps."""
        _check(load().nlse_step_corrected(self._h, corrector._h, int(nsteps), float(dt), int(every)))

    def sync(self):
        _check(load().nlse_sync(self._h))

    def _scalar(self, fn):
        v = ctypes.c_double()
        _check(fn(self._h, ctypes.byref(v)))
        return v.value

    def mass(self):
        return self._scalar(load().nlse_mass)

    def energy(self):
        return self._scalar(load().nlse_energy)

    def max_dt(self):
        return self._scalar(load().nlse_max_dt)

    def launches_per_step(self):
        return load().nlse_launches_per_step(self._h)

    # ---- tile variants and the autotuner
    def variant_count(self):
        return load().nlse_variant_count(self._h)

    @property
    def variant(self):
        return load().nlse_get_variant(self._h)

    @variant.setter
    def variant(self, v):
        _check(load().nlse_set_variant(self._h, int(v)))

    # ---- Laplacian (Dirichlet; 2D and 3D in the stage kernels): "2shoc" (default), "noncompact", "cd"
    STENCILS = {"2shoc": 0, "noncompact": 1, "cd": 2}

    @property
    def stencil(self):
        v = load().nlse_get_stencil(self._h)
        names = {c: k for k, c in self.STENCILS.items()}
        return names.get(v, v)

    @stencil.setter
    def stencil(self, name):
        _check(load().nlse_set_stencil(self._h, self.STENCILS[name]))

    def autotune(self, reps=5, force=False):
        """Time RK4 steps of every kernel variant on this problem, keep the fastest; returns its index."""
        ch = ctypes.c_int()
        _check(load().nlse_autotune(self._h, int(reps), int(bool(force)), ctypes.byref(ch)))
        return ch.value


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _params_from_spec(spec, prec, allow_unstable, stream):
    """Params for one spec (nlse_inputs.ProblemSpec); returns (Params, V array kept alive)."""
    g = spec.grid
    p = Params()
    p.ndim = g.dim
    for i in range(3):
        p.n[i] = g.n if i < g.dim else 0
    p.h, p.a, p.s = g.h, float(spec.a), float(spec.s)
    V = None
    if spec.V is not None:
        V = np.ascontiguousarray(spec.V, dtype=np.float64)
        p.V = V.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.bc = BC[spec.bc]
    p.prec = PREC[prec]
    p.allow_unstable = int(bool(allow_unstable))
    p.stream = stream
    return p, V


class Batch:
    """Many independent 1D / 2D problems advanced by one persistent, graph-captured launch.

    specs: sequence of nlse_inputs.ProblemSpec (1D or 2D).  set_fields() loads every
    spec's psi0; set_dts(frac) gives each instance dt = frac * its own stability bound."""

    def __init__(self, specs, prec="f32", allow_unstable=False, stream="current"):
        L = load()
        self.prec = prec
        self.stream = _current_stream() if stream == "current" else stream
        self.shapes = [tuple(v + 1 for v in (sp.grid.n,) * sp.grid.dim) for sp in specs]
        self.dtype = np.complex64 if prec == "f32" else np.complex128
        arr = (Params * len(specs))()
        keep = []
        for i, sp in enumerate(specs):
            p, V = _params_from_spec(sp, prec, allow_unstable, self.stream)
            arr[i] = p
            keep.append(V)
        h_ = ctypes.c_void_p()
        _check(L.nlse_batch_create(ctypes.byref(h_), arr, len(specs)))
        self._h = h_
        self.count = len(specs)

    def close(self):
        if getattr(self, "_h", None):
            load().nlse_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_field(self, i, psi):
        arr = np.ascontiguousarray(psi, dtype=self.dtype).reshape(self.shapes[i])
        _check(load().nlse_batch_set_field(self._h, int(i), arr.ctypes.data_as(ctypes.c_void_p), 0))

    def get_field(self, i):
        arr = np.empty(self.shapes[i], dtype=self.dtype)
        _check(load().nlse_batch_get_field(self._h, int(i), arr.ctypes.data_as(ctypes.c_void_p), 0))
        return arr

    def set_dt(self, i, dt):
        _check(load().nlse_batch_set_dt(self._h, int(i), float(dt)))

    def max_dt(self, i):
        v = ctypes.c_double()
        _check(load().nlse_batch_max_dt(self._h, int(i), ctypes.byref(v)))
        return v.value

    def mass(self, i):
        v = ctypes.c_double()
        _check(load().nlse_batch_mass(self._h, int(i), ctypes.byref(v)))
        return v.value

    def set_fields(self, specs):
        for i, sp in enumerate(specs):
            self.set_field(i, sp.psi0)

    def set_dts(self, frac=0.5):
        dts = []
        for i in range(self.count):
            dt = frac * self.max_dt(i)
            self.set_dt(i, dt)
            dts.append(dt)
        return dts

    def step(self, nsteps):
        _check(load().nlse_batch_step(self._h, int(nsteps)))

    def sync(self):
        _check(load().nlse_batch_sync(self._h))

    @property
    def variant(self):
        return load().nlse_batch_get_variant(self._h)

    @variant.setter
    def variant(self, v):
        _check(load().nlse_batch_set_variant(self._h, int(v)))

    def variant_count(self):
        return load().nlse_batch_variant_count(self._h)

    def autotune(self, nsteps=20, force=False):
        ch = ctypes.c_int()
        _check(load().nlse_batch_autotune(self._h, int(nsteps), int(bool(force)), ctypes.byref(ch)))
        return ch.value


class Corrector:
    """The learned coarse-grid corrector (3-layer 3x3 conv, BF16 MFMA, FP32 accumulate).

    H, W: nodes of the fields it corrects; V: potential on those nodes (numpy [H, W]) or None.
    Field arguments are torch complex64 GPU tensors of shape [batch, H, W] (or [H, W])."""

    def __init__(self, H, W, max_batch=4, V=None, stream="current"):
        L = load()
        self.H, self.W, self.max_batch = int(H), int(W), int(max_batch)
        self.stream = _current_stream() if stream == "current" else stream
        self._V = None if V is None else np.ascontiguousarray(V, dtype=np.float64).reshape(H, W)
        vptr = None if self._V is None else self._V.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h_ = ctypes.c_void_p()
        _check(L.nlse_corr_create(ctypes.byref(h_), self.H, self.W, self.max_batch, vptr, self.stream))
        self._h = h_
        self.nparam = L.nlse_corr_param_count()

    def close(self):
        if getattr(self, "_h", None):
            load().nlse_corr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, scale):
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        _check(load().nlse_corr_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), float(scale)))
        self.scale = float(scale)

    def set_augment(self, sigma, seed=0):
        _check(load().nlse_corr_set_augment(self._h, float(sigma), int(seed)))

    def set_target_filter(self, smooth):
        _check(load().nlse_corr_set_target_filter(self._h, int(smooth)))

    def get_params(self):
        p = np.empty(self.nparam, dtype=np.float32)
        _check(load().nlse_corr_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def _fields(self, t):
        import torch
        if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("fields must be contiguous complex64 GPU tensors")
        b = 1 if t.dim() == 2 else t.shape[0]
        if t.shape[-2:] != (self.H, self.W) or b > self.max_batch:
            raise ValueError("field shape does not match the corrector")
        return b

    def infer(self, psi):
        import torch
        b = self._fields(psi)
        y = torch.empty((b, self.H, self.W, 2), dtype=torch.float32, device=psi.device)
        _check(load().nlse_corr_infer(self._h, ctypes.c_void_p(psi.data_ptr()), b, ctypes.c_void_p(y.data_ptr())))
        return y

    def grads(self, pred, ref):
        b = self._fields(pred)
        g = np.empty(self.nparam, dtype=np.float32)
        loss = ctypes.c_double()
        _check(load().nlse_corr_grads(self._h, ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(ref.data_ptr()), b,
                                      g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, pred, ref, lr):
        b = self._fields(pred)
        loss = ctypes.c_double()
        _check(load().nlse_corr_train_step(self._h, ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
                                           b, float(lr), ctypes.byref(loss)))
        return loss.value

    def apply(self, solver):
        _check(load().nlse_corr_apply(self._h, solver._h))

    # ---- validation access to the training passes (nlse_corr_tensor / nlse_corr_stage)
    TENSORS = {"X0": 0, "A1": 1, "A2": 2, "Z1": 3, "Z2": 4, "Y": 5, "dY": 6, "dZ2": 7, "dZ1": 8, "grads": 9}
    STAGES = {"fwd1": 1, "fwd2": 2, "fwd3": 3, "wgrad3": 4, "bwd3": 5, "wgrad2": 6, "bwd2": 7, "wgrad1": 8}

    def put_tensor(self, name, arr):
        """Copy a host array (uint16 bf16 patterns or float32, layout of nlse.h) into a tensor."""
        a = np.ascontiguousarray(arr)
        _check(load().nlse_corr_tensor(self._h, self.TENSORS[name], 1, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))

    def get_tensor(self, name, shape, dtype):
        a = np.empty(shape, dtype=dtype)
        _check(load().nlse_corr_tensor(self._h, self.TENSORS[name], 0, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))
        return a

    def stage(self, name, batch):
        _check(load().nlse_corr_stage(self._h, self.STAGES[name], int(batch)))


def inject(src, src_n, dst, factor, stream="current"):
    """dst[y, x] = src[factor y, factor x] for dense square complex GPU tensors (dst complex64)."""
    import torch
    prec = PREC["f32"] if src.dtype == torch.complex64 else PREC["f64"]
    st = _current_stream() if stream == "current" else stream
    _check(load().nlse_inject(ctypes.c_void_p(src.data_ptr()), prec, int(src_n), ctypes.c_void_p(dst.data_ptr()),
                              int(src_n) // int(factor), int(factor), st))


def mass_noalloc(psi, h, prec, out, stream="current"):
    """nlse_mass_noalloc: the mass h^ndim sum |Psi|^2 of a dense device field (a torch tensor
    of (n+1)^ndim complex nodes, complex128 for "f64"/"mixed", complex64 for "f32") into
    `out`, a one-element float64 device tensor, without any allocation in the library."""
    ndim = psi.dim()
    n = (ctypes.c_int64 * 3)(*[int(d) - 1 for d in reversed(psi.shape)], *([0] * (3 - ndim)))
    st = _current_stream() if stream == "current" else stream
    _check(load().nlse_mass_noalloc(ndim, n, float(h), PREC[prec], ctypes.c_void_p(psi.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), st))
