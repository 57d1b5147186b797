"""FP64 CPU oracle for the cell-centred multigrid (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1306_6883_amd``) and never imports it.

Two parts:

* the multigrid algorithm itself, step by step, in plain C
  (``mg_oracle.c``; pyro paper Sec. 3.3), wrapped here with ctypes;
* exact discrete solutions (``oracle.exact``): dense direct solves and
  fast-transform solves of the same 5-point operator.

Fields are numpy float64 arrays of shape (n+2, n+2): row index j+1, column
index i+1 for valid cell (i, j), x contiguous, one ghost layer.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB = os.path.join(_HERE, "libmg_oracle.so")

DIRICHLET, NEUMANN, PERIODIC = 0, 1, 2
_BC_CODES = {"D": DIRICHLET, "N": NEUMANN, "P": PERIODIC,
             DIRICHLET: DIRICHLET, NEUMANN: NEUMANN, PERIODIC: PERIODIC}
OK, NOT_CONVERGED, EINVAL = 0, 1, -1
HISTORY = 256


def build() -> str:
    """Compile the C oracle with gcc (FP contraction off, OpenMP on)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("h", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("bc", ctypes.c_int * 4), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("nu_bottom", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("rtol", ctypes.c_double), ("n_bottom", ctypes.c_int)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int),
                ("rel_resid0", ctypes.c_double), ("rel_resid", ctypes.c_double),
                ("history", ctypes.c_double * HISTORY)]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib_handle = _load(_LIB)
    return _lib_handle


def _load(path: str):
    """Load a compiled oracle library and declare its entry points."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.og_fill.argtypes = [ctypes.c_int, ip, dp]
    lib.og_smooth.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ip, dp, dp, ctypes.c_int]
    lib.og_residual.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ip, dp, dp, dp]
    lib.og_restrict.argtypes = [ctypes.c_int, dp, dp]
    lib.og_prolong_add.argtypes = [ctypes.c_int, ip, dp, dp]
    lib.og_norm.argtypes = [ctypes.c_int, ctypes.c_double, dp]
    lib.og_norm.restype = ctypes.c_double
    lib.og_mean.argtypes = [ctypes.c_int, dp]
    lib.og_mean.restype = ctypes.c_double
    lib.og_vcycle.argtypes = [ctypes.POINTER(_Params), dp, dp]
    lib.og_fmg.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.og_solve.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.c_int,
                             ctypes.POINTER(_Result)]
    lib.og_smooth_solve.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.c_int,
                                    ctypes.POINTER(_Result)]
    lib.og_cn_rhs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ip, dp, dp]
    lib.og_cn_step.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.POINTER(_Result)]
    bp = ctypes.POINTER(dp)
    lib.og_fill_bc.argtypes = [ctypes.c_int, ctypes.c_double, ip, bp, dp]
    lib.og_bc_rhs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ip, bp, dp, dp]
    lib.og_solve_bc.argtypes = [ctypes.POINTER(_Params), dp, dp, bp, ctypes.c_int, ctypes.POINTER(_Result)]
    lib.og_divergence.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
    lib.og_subtract_gradient.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
    lib.og_project.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, ctypes.POINTER(_Result)]
    return lib


def bc_codes(bc) -> tuple:
    """Normalise a BC spec: a 4-tuple (xlo, xhi, ylo, yhi) of 'D'/'N'/'P' or ints,
    or a single letter for all sides."""
    if isinstance(bc, str) and len(bc) == 1:
        bc = (bc,) * 4
    out = tuple(_BC_CODES[b] for b in bc)
    if len(out) != 4:
        raise ValueError("bc needs four sides")
    if (out[0] == PERIODIC) != (out[1] == PERIODIC) or (out[2] == PERIODIC) != (out[3] == PERIODIC):
        raise ValueError("periodic must pair opposite sides")
    return out


@dataclass
class Problem:
    """(alpha - beta Lap) phi = f on an n x n grid of square cells of width h."""
    n: int
    h: float
    alpha: float = 0.0
    beta: float = -1.0
    bc: tuple = ("D", "D", "D", "D")
    nu1: int = 2
    nu2: int = 2
    nu_bottom: int = 50
    max_cycles: int = 100
    rtol: float = 1e-10
    n_bottom: int = 2      # 4, 8, ...: exact solve on that level, nothing below

    def _c(self) -> _Params:
        p = _Params()
        p.n, p.h, p.alpha, p.beta = self.n, self.h, self.alpha, self.beta
        p.bc[:] = list(bc_codes(self.bc))
        p.nu1, p.nu2, p.nu_bottom = self.nu1, self.nu2, self.nu_bottom
        p.max_cycles, p.rtol = self.max_cycles, self.rtol
        p.n_bottom = self.n_bottom
        return p

    @property
    def singular(self) -> bool:
        return self.alpha == 0.0 and DIRICHLET not in bc_codes(self.bc)


@dataclass
class Result:
    status: int
    cycles: int
    rel_resid0: float
    rel_resid: float
    history: list = field(default_factory=list)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _bcp(bc):
    arr = (ctypes.c_int * 4)(*bc_codes(bc))
    return arr


def field_zeros(n: int) -> np.ndarray:
    return np.zeros((n + 2, n + 2), dtype=np.float64)


def embed(valid: np.ndarray) -> np.ndarray:
    """Place an (n, n) array of valid cells (index [j, i]) into a ghosted field."""
    n = valid.shape[0]
    a = field_zeros(n)
    a[1:n + 1, 1:n + 1] = valid
    return a


def interior(a: np.ndarray) -> np.ndarray:
    n = a.shape[0] - 2
    return a[1:n + 1, 1:n + 1]


def fill(a: np.ndarray, bc) -> np.ndarray:
    _lib().og_fill(a.shape[0] - 2, _bcp(bc), _ptr(a))
    return a


def smooth(p: Problem, phi: np.ndarray, f: np.ndarray, iters: int, level: int = 0) -> np.ndarray:
    n, h = p.n >> level, p.h * (1 << level)
    assert phi.shape == (n + 2, n + 2) and f.shape == phi.shape
    _lib().og_smooth(n, h, p.alpha, p.beta, _bcp(p.bc), _ptr(phi), _ptr(f), iters)
    return phi


def residual(p: Problem, phi: np.ndarray, f: np.ndarray, level: int = 0) -> np.ndarray:
    n, h = p.n >> level, p.h * (1 << level)
    r = field_zeros(n)
    _lib().og_residual(n, h, p.alpha, p.beta, _bcp(p.bc), _ptr(phi), _ptr(f), _ptr(r))
    return r


def restrict(fine: np.ndarray) -> np.ndarray:
    n = fine.shape[0] - 2
    c = field_zeros(n // 2)
    _lib().og_restrict(n, _ptr(fine), _ptr(c))
    return c


def prolong_add(coarse: np.ndarray, fine: np.ndarray, bc) -> np.ndarray:
    _lib().og_prolong_add(coarse.shape[0] - 2, _bcp(bc), _ptr(coarse), _ptr(fine))
    return fine


def norm(a: np.ndarray, h: float) -> float:
    return _lib().og_norm(a.shape[0] - 2, h, _ptr(a))


def mean(a: np.ndarray) -> float:
    return _lib().og_mean(a.shape[0] - 2, _ptr(a))


def vcycle(p: Problem, phi: np.ndarray, f: np.ndarray) -> np.ndarray:
    st = _lib().og_vcycle(ctypes.byref(p._c()), _ptr(phi), _ptr(f))
    if st != OK:
        raise ValueError("oracle vcycle: bad problem")
    return phi


def fmg(p: Problem, f: np.ndarray, top_n: int = 2, ncyc_top: int = 1, ncyc: int = 1) -> np.ndarray:
    """Full multigrid start (mg_oracle.c og_fmg): f restricted down to the
    level of top_n cells per side, ncyc_top V-cycles there from zero, then per
    finer level the prolongated coarse phi and ncyc V-cycles.  Returns the
    finest phi (ghosts filled)."""
    phi = field_zeros(p.n)
    st = _lib().og_fmg(ctypes.byref(p._c()), _ptr(phi), _ptr(f), top_n, ncyc_top, ncyc)
    if st != OK:
        raise ValueError("oracle fmg: bad arguments")
    return phi


def _result(r: _Result) -> Result:
    hist = [r.history[i] for i in range(min(r.cycles + 1, HISTORY))]
    return Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist)


def solve(p: Problem, f: np.ndarray, phi: np.ndarray | None = None):
    """V-cycles until ||r||/||f|| <= rtol.  Returns (phi, Result)."""
    use_guess = phi is not None
    phi = field_zeros(p.n) if phi is None else phi
    res = _Result()
    st = _lib().og_solve(ctypes.byref(p._c()), _ptr(phi), _ptr(f), int(use_guess), ctypes.byref(res))
    if st == EINVAL:
        raise ValueError("oracle solve: bad problem")
    return phi, _result(res)


def smooth_solve(p: Problem, f: np.ndarray, max_iters: int, phi: np.ndarray | None = None):
    """Relaxation only (no coarse grids) until the same stopping rule holds."""
    phi = field_zeros(p.n) if phi is None else phi
    res = _Result()
    _lib().og_smooth_solve(ctypes.byref(p._c()), _ptr(phi), _ptr(f), max_iters, ctypes.byref(res))
    return phi, _result(res)


def cn_rhs(n: int, h: float, beta: float, bc, phi: np.ndarray) -> np.ndarray:
    """Right-hand side of a Crank-Nicolson diffusion step (Sec. 3.4):
    f = phi + beta Lap phi with beta = k dt / 2 (phi's ghosts are filled)."""
    f = field_zeros(n)
    _lib().og_cn_rhs(n, h, beta, _bcp(bc), _ptr(phi), _ptr(f))
    return f


def cn_step(p: Problem, phi: np.ndarray):
    """One Crank-Nicolson step of phi_t = k Lap phi in place: p.alpha = 1 and
    p.beta = k dt / 2; the old phi is the solve's initial guess.  Returns
    (phi, Result)."""
    work = field_zeros(p.n)
    res = _Result()
    st = _lib().og_cn_step(ctypes.byref(p._c()), _ptr(phi), _ptr(work), ctypes.byref(res))
    if st == EINVAL:
        raise ValueError("oracle cn_step: bad problem (alpha must be 1)")
    return phi, _result(res)


def _sides(b):
    """Four side-data arrays (or None) -> a C array of four pointers; the
    arrays are kept alive by the returned tuple."""
    keep = [None if v is None else np.ascontiguousarray(v, dtype=np.float64) for v in (b or [None] * 4)]
    if len(keep) != 4:
        raise ValueError("side data needs four entries")
    dp = ctypes.POINTER(ctypes.c_double)
    arr = (dp * 4)(*[ctypes.cast(None, dp) if v is None else v.ctypes.data_as(dp) for v in keep])
    return arr, keep


def fill_bc(a: np.ndarray, h: float, bc, b) -> np.ndarray:
    """Ghost cells with side data b (four arrays of n values or None): a
    Dirichlet value v gives ghost 2v - phi, a Neumann derivative d gives
    phi - h d (lo sides) or phi + h d (hi sides)."""
    n = a.shape[0] - 2
    arr, _keep = _sides(b)
    _lib().og_fill_bc(n, h, _bcp(bc), arr, _ptr(a))
    return a


def bc_rhs(n: int, h: float, beta: float, bc, b, f: np.ndarray) -> np.ndarray:
    """The right-hand side of the equivalent homogeneous problem."""
    arr, _keep = _sides(b)
    out = field_zeros(n)
    _lib().og_bc_rhs(n, h, beta, _bcp(bc), arr, _ptr(f), _ptr(out))
    return out


def solve_bc(p: Problem, f: np.ndarray, b, phi: np.ndarray | None = None):
    """V-cycles with side data b until ||r||/||f'|| <= rtol (f' the shifted
    right-hand side); the returned field's ghosts carry the data."""
    use_guess = phi is not None
    phi = field_zeros(p.n) if phi is None else phi
    arr, _keep = _sides(b)
    res = _Result()
    st = _lib().og_solve_bc(ctypes.byref(p._c()), _ptr(phi), _ptr(f), arr, int(use_guess), ctypes.byref(res))
    if st == EINVAL:
        raise ValueError("oracle solve_bc: bad problem")
    return phi, _result(res)


def divergence(n: int, h: float, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Centred-difference divergence of a cell-centred periodic field (Sec. 3.5)."""
    f = field_zeros(n)
    _lib().og_divergence(n, h, _ptr(u), _ptr(v), _ptr(f))
    return f


def project(n: int, u: np.ndarray, v: np.ndarray, rtol: float = 1e-10):
    """Approximate cell-centred projection of (u, v) on the periodic unit
    square, in place: Lap phi = D U, U -= G phi.  Returns (u, v, phi, Result)."""
    p = Problem(n=n, h=1.0 / n, alpha=0.0, beta=-1.0, bc="PPPP", rtol=rtol)
    phi = field_zeros(n)
    res = _Result()
    st = _lib().og_project(ctypes.byref(p._c()), _ptr(u), _ptr(v), _ptr(phi), ctypes.byref(res))
    if st == EINVAL:
        raise ValueError("oracle project: bad problem")
    return u, v, phi, _result(res)
