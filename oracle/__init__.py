"""Plain FP64 CPU oracle for 2SHOC-RK4 on the NLSE -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it; the two meet only through the seeded inputs of
``nlse_inputs``.

The arithmetic lives in ``nlse_oracle.c`` (plain C, FP64, no FMA contraction),
which follows the paper step by step:

* 2SHOC step 1 / step 2 (Sec. 2, Eqs. 2shoc1d-2, 2d2shocs1-2, 3d2shocs-2) and
  the per-axis, non-compact and second-order CD alternatives;
* Dirichlet and MSD boundary closures (Sec. 3.2, Eqs. dbc_lap, dbc_ut,
  msdbc_lap, msdbc_ut);
* classic RK4 as the ten array operations of Sec. 3.1 (Eq. RK4);
* the linearised step-size bound (Sec. 3.3, Eq. kdfull, Tables t:bc2,
  t:sumresults);
* mass and the discrete Hamiltonian (not in the paper; plain definitions).

This module adds the paper's error metric (Sec. 4: per-part RMS over all nodes
at 100 equally spaced instants, averaged; order = ln(E1/E2)/ln(h1/h2)).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
(closed forms, exact solutions, the paper's printed tables, brute force on tiny
grids); the learned-corrector reference in ``conv.py`` is pinned by finite
differences, its trained weights are parity unpinned.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlse_oracle.c")
_LIB = os.path.join(_HERE, "libnlse_oracle.so")

LAP_2SHOC, LAP_2SHOC_AXIS, LAP_NONCOMPACT, LAP_CD = 0, 1, 2, 3
_LAPS = {"2shoc": LAP_2SHOC, "axis": LAP_2SHOC_AXIS, "noncompact": LAP_NONCOMPACT, "cd": LAP_CD}
_BCS = {"dirichlet": 0, "msd": 1}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_long * 3), ("h", ctypes.c_double),
                ("a", ctypes.c_double), ("s", ctypes.c_double),
                ("V", ctypes.POINTER(ctypes.c_double)), ("bc", ctypes.c_int), ("lap", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        for name in ("orc_laplacian", "orc_step1", "orc_rhs"):
            getattr(L, name).argtypes = [P, dp, dp]
            getattr(L, name).restype = ctypes.c_int
        L.orc_rk4.argtypes = [P, dp, ctypes.c_long, ctypes.c_double]
        L.orc_rk4.restype = ctypes.c_int
        L.orc_mass.argtypes = [P, dp]
        L.orc_mass.restype = ctypes.c_double
        L.orc_energy.argtypes = [P, dp]
        L.orc_energy.restype = ctypes.c_double
        L.orc_max_dt.argtypes = [P, dp, dp]
        L.orc_max_dt.restype = ctypes.c_double
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def threads() -> int:
    return lib().orc_threads()


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def _dptr(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Problem:
    """An NLSE problem for the oracle: uniform grid of n intervals per axis, step h."""

    def __init__(self, dim, n, h, a, s, V=None, bc="dirichlet", lap="2shoc"):
        self.dim, self.h, self.a, self.s = int(dim), float(h), float(a), float(s)
        self.n = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n,) * self.dim))
        self.shape = tuple(v + 1 for v in reversed(self.n))   # [z][y][x]
        self.V = None if V is None else np.ascontiguousarray(V, dtype=np.float64).reshape(self.shape)
        self.bc, self.lap = bc, lap
        self._c = _Problem()
        self._c.dim = self.dim
        for i in range(3):
            self._c.n[i] = self.n[i] if i < self.dim else 0
        self._c.h, self._c.a, self._c.s = self.h, self.a, self.s
        self._c.V = _dptr(self.V) if self.V is not None else ctypes.POINTER(ctypes.c_double)()
        self._c.bc = _BCS[bc]
        self._c.lap = _LAPS[lap]

    @classmethod
    def from_spec(cls, spec, lap="2shoc"):
        g = spec.grid
        return cls(g.dim, g.n, g.h, spec.a, spec.s, spec.V, spec.bc, lap)

    def with_lap(self, lap):
        return Problem(self.dim, self.n, self.h, self.a, self.s, self.V, self.bc, lap)

    def _field(self, psi):
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        if psi.shape != self.shape:
            psi = psi.reshape(self.shape)
        return psi

    def _check(self, rc):
        if rc != 0:
            raise ValueError(f"oracle rejected the problem (code {rc})")

    def laplacian(self, psi):
        psi = self._field(psi)
        out = np.zeros_like(psi)
        self._check(lib().orc_laplacian(ctypes.byref(self._c), _dptr(psi.view(np.float64)),
                                        _dptr(out.view(np.float64))))
        return out

    def step1(self, psi):
        psi = self._field(psi)
        out = np.zeros_like(psi)
        self._check(lib().orc_step1(ctypes.byref(self._c), _dptr(psi.view(np.float64)),
                                    _dptr(out.view(np.float64))))
        return out

    def rhs(self, psi):
        psi = self._field(psi)
        out = np.zeros_like(psi)
        self._check(lib().orc_rhs(ctypes.byref(self._c), _dptr(psi.view(np.float64)),
                                  _dptr(out.view(np.float64))))
        return out

    def rk4(self, psi, nsteps, k):
        """Return Psi after nsteps RK4 steps of size k (input is not modified)."""
        out = self._field(psi).copy()
        self._check(lib().orc_rk4(ctypes.byref(self._c), _dptr(out.view(np.float64)),
                                  int(nsteps), float(k)))
        return out

    def mass(self, psi):
        psi = self._field(psi)
        return lib().orc_mass(ctypes.byref(self._c), _dptr(psi.view(np.float64)))

    def energy(self, psi):
        psi = self._field(psi)
        return lib().orc_energy(ctypes.byref(self._c), _dptr(psi.view(np.float64)))

    def max_dt(self, psi, return_aux=False):
        psi = self._field(psi)
        aux = np.zeros(3)
        k = lib().orc_max_dt(ctypes.byref(self._c), _dptr(psi.view(np.float64)), _dptr(aux))
        return (k, aux) if return_aux else k


# ---------------------------------------------------------------------------
# Step-size choice and the paper's error metric (Sec. 4)
# ---------------------------------------------------------------------------

def steps_for(t_end: float, k_max: float, frac: float = 0.5):
    """Number of steps and dt = t_end / ceil(t_end / (frac k_max)) (dt <= frac k_max)."""
    nsteps = int(math.ceil(t_end / (frac * k_max)))
    return nsteps, t_end / nsteps


def rms_parts(psi, ref):
    """Per-part RMS error over all nodes: (||Re d||_2 / sqrt(N), ||Im d||_2 / sqrt(N))."""
    d = np.asarray(psi) - np.asarray(ref)
    N = d.size
    return (math.sqrt(float(np.sum(d.real ** 2)) / N), math.sqrt(float(np.sum(d.imag ** 2)) / N))


def rel_l2(psi, ref):
    d = np.asarray(psi, dtype=np.complex128) - np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(d.ravel()) / np.linalg.norm(np.asarray(ref).ravel()))


def paper_error(problem: Problem, psi0, exact, t_end, nsteps, samples=100):
    """Run RK4 to t_end in `samples` equal chunks and return the paper's averaged errors.

    exact(t) gives the analytic field at time t.  The error at each sample instant is
    the per-part RMS over all nodes; the result is the mean over the samples j = 1..K."""
    if nsteps % samples:
        raise ValueError("nsteps must be a multiple of the number of samples")
    k = t_end / nsteps
    chunk = nsteps // samples
    psi = np.array(psi0, dtype=np.complex128)
    er, ei = [], []
    for j in range(1, samples + 1):
        psi = problem.rk4(psi, chunk, k)
        r, i = rms_parts(psi, exact(j * chunk * k))
        er.append(r)
        ei.append(i)
    return float(np.mean(er)), float(np.mean(ei)), psi


def order(e1, e2, h1, h2):
    """Order of accuracy between two runs: ln(E1/E2) / ln(h1/h2)."""
    return math.log(e1 / e2) / math.log(h1 / h2)
