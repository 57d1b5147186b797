"""Python binding of the ccmg HIP library (include/ccmg.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch supplies device memory (fields and workspaces are torch
tensors on a ROCm device) and the stream (torch's current HIP stream).  The
library must be built (``python -m paper_1306_6883_amd.build``); importing
this module does not fall back to anything when it is missing.

Fields are torch tensors of shape (n+2, pitch) with pitch >= n+2 (row stride
in elements), one ghost layer, x contiguous: valid cell (i, j) is
``t[j+1, i+1]``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccmg.so")

BC_DIRICHLET, BC_NEUMANN, BC_PERIODIC = 0, 1, 2
FP64, MIXED = 0, 1
OK, NOT_CONVERGED, EINVAL, ESIZE, EBC, EINCOMPAT, ENONFINITE, EHIP, EWORKSPACE = 0, 1, -1, -2, -3, -4, -5, -6, -7
HISTORY = 128
OPT_FUSED, OPT_FUSED_KEEP, OPT_MIXED_INNER, OPT_FMG, OPT_VISIT = 1, 2, 3, 4, 5
BATCH_OPT_EAGER = 1
_BC = {"D": BC_DIRICHLET, "N": BC_NEUMANN, "P": BC_PERIODIC,
       BC_DIRICHLET: BC_DIRICHLET, BC_NEUMANN: BC_NEUMANN, BC_PERIODIC: BC_PERIODIC}


class CcmgError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {ccmg_status_str(status)} ({status})" if what else ccmg_status_str(status))


class ccmg_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("ng", ctypes.c_int),
                ("xmin", ctypes.c_double), ("xmax", ctypes.c_double),
                ("ymin", ctypes.c_double), ("ymax", ctypes.c_double),
                ("bc", ctypes.c_int * 4), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("nu_bottom", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("rtol", ctypes.c_double), ("prec", ctypes.c_int)]


class ccmg_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int),
                ("rel_resid0", ctypes.c_double), ("rel_resid", ctypes.c_double),
                ("history", ctypes.c_double * HISTORY), ("ms", ctypes.c_float),
                ("inner_cycles", ctypes.c_int)]


class ccmg_batch_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("converged", ctypes.c_int), ("ms", ctypes.c_float)]


class ccmg_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library.  Raises if it has not been built: there is no other path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1306_6883_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, sz, pd, i = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_ssize_t, ctypes.c_int
        P = ctypes.POINTER(ccmg_problem)
        L.ccmg_status_str.restype = ctypes.c_char_p
        L.ccmg_status_str.argtypes = [i]
        L.ccmg_problem_init.argtypes = [P, i]
        L.ccmg_problem_check.argtypes = [P]
        L.ccmg_workspace_bytes.restype = sz
        L.ccmg_workspace_bytes.argtypes = [P]
        L.ccmg_plan_create.argtypes = [P, vp, sz, vp, ctypes.POINTER(vp)]
        L.ccmg_plan_destroy.argtypes = [vp]
        L.ccmg_solve.argtypes = [vp, dp, dp, pd, i, ctypes.POINTER(ccmg_result)]
        L.ccmg_vcycle.argtypes = [vp, dp, dp, pd]
        L.ccmg_fmg.argtypes = [vp, dp, dp, pd, i, i]
        L.ccmg_fill_ghosts.argtypes = [vp, i, dp, pd]
        L.ccmg_smooth.argtypes = [vp, i, i, dp, dp, dp, pd]
        L.ccmg_residual.argtypes = [vp, i, dp, dp, dp, pd]
        L.ccmg_restrict_residual.argtypes = [vp, i, dp, dp, pd, dp, pd]
        L.ccmg_restrict.argtypes = [vp, i, dp, pd, dp, pd]
        L.ccmg_prolong_add.argtypes = [vp, i, dp, pd, dp, dp, pd]
        L.ccmg_plan_profile.argtypes = [vp, i]
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.ccmg_batch_workspace_bytes.restype = sz
        L.ccmg_batch_workspace_bytes.argtypes = [i, P]
        L.ccmg_batch_create.argtypes = [i, P, vp, sz, vp, ctypes.POINTER(vp)]
        L.ccmg_batch_destroy.argtypes = [vp]
        L.ccmg_batch_solve.argtypes = [vp, PP, PP, ctypes.POINTER(pd), i, ctypes.POINTER(ccmg_result),
                                       ctypes.POINTER(ccmg_batch_info)]
        L.ccmg_batch_autotune.argtypes = [vp, PP, PP, ctypes.POINTER(pd)]
        L.ccmg_batch_shapes.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), i, ctypes.POINTER(i),
                                        ctypes.POINTER(i)]
        L.ccmg_plan_autotune.argtypes = [vp, dp, dp, pd]
        ip = ctypes.POINTER(ctypes.c_int)
        L.ccmg_plan_shapes.argtypes = [vp, ip, ip, ip, ip, i]
        b4 = ctypes.c_void_p * 4
        L.ccmg_bc_rhs.argtypes = [vp, dp, dp, pd, b4]
        L.ccmg_fill_ghosts_bc.argtypes = [vp, dp, pd, b4]
        L.ccmg_solve_bc.argtypes = [vp, dp, dp, pd, i, b4, dp, ctypes.POINTER(ccmg_result)]
        L.ccmg_project.argtypes = [vp, dp, dp, pd, dp, dp, ctypes.POINTER(ccmg_result)]
        L.ccmg_cn_rhs.argtypes = [vp, dp, dp, pd]
        L.ccmg_cn_step.argtypes = [vp, dp, dp, pd, ctypes.POINTER(ccmg_result)]
        L.ccmg_plan_fused_shape.argtypes = [vp, i, ip, ip]
        L.ccmg_plan_set_shape.argtypes = [vp, i, i, i, i]
        L.ccmg_plan_shape.argtypes = [vp, i, i, ip, ip]
        L.ccmg_plan_set_bottom.argtypes = [vp, i]
        L.ccmg_plan_kernel_stats.argtypes = [vp, ctypes.POINTER(ccmg_kernel_stat), i, ctypes.POINTER(i)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.ccmg_net_param_count.argtypes = []
        L.ccmg_net_workspace_bytes.restype = sz
        L.ccmg_net_workspace_bytes.argtypes = [i, i]
        L.ccmg_net_create.argtypes = [i, i, vp, sz, vp, ctypes.POINTER(vp)]
        L.ccmg_net_destroy.argtypes = [vp]
        L.ccmg_net_set_params.argtypes = [vp, vp]
        L.ccmg_net_state_count.argtypes = []
        L.ccmg_net_get_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int)]
        L.ccmg_net_set_state.argtypes = [vp, vp, i]
        L.ccmg_net_get_params.argtypes = [vp, vp]
        L.ccmg_net_forward.argtypes = [vp, vp, vp, i]
        L.ccmg_net_loss_grad.argtypes = [vp, vp, vp, i, vp, fp]
        L.ccmg_net_train_step.argtypes = [vp, vp, vp, i, ctypes.c_float, fp]
        L.ccmg_net_encode.argtypes = [vp, dp, pd, i, dp, pd, vp]
        L.ccmg_net_guess.argtypes = [vp, dp, pd, i, ctypes.c_double, i, dp, pd]
        L.ccmg_solve_learned.argtypes = [vp, vp, dp, dp, pd, i, ctypes.POINTER(ccmg_result), ip]
        L.ccmg_probe_stream.argtypes = [dp, dp, dp, sz, i, vp, fp, ctypes.POINTER(ctypes.c_int)]
        L.ccmg_plan_set_option.argtypes = [vp, i, ctypes.c_double]
        L.ccmg_plan_get_option.argtypes = [vp, i, ctypes.POINTER(ctypes.c_double)]
        L.ccmg_batch_set_option.argtypes = [vp, i, ctypes.c_double]
        L.ccmg_vcycle_noalloc.argtypes = [P, dp, dp, pd, vp]
        L.ccmg_noalloc_scratch_bytes.restype = sz
        L.ccmg_noalloc_scratch_bytes.argtypes = []
        _lib = L
    return _lib


def ccmg_status_str(status: int) -> str:
    return lib().ccmg_status_str(status).decode()


def _check(status: int, what: str, allow=(OK,)):
    if status not in allow:
        raise CcmgError(status, what)
    return status


@dataclass
class Problem:
    """Mirror of ccmg_problem.  bc: 4 sides (xlo, xhi, ylo, yhi) as 'D'/'N'/'P' or
    codes, or one letter for all sides."""
    n: int
    bc: object = "D"
    alpha: float = 0.0
    beta: float = -1.0
    xmin: float = 0.0
    xmax: float = 1.0
    ymin: float = 0.0
    ymax: float = 1.0
    nu1: int = 2
    nu2: int = 2
    nu_bottom: int = 50
    max_cycles: int = 100
    rtol: float = 1e-10
    prec: int = FP64

    def bc_codes(self):
        b = self.bc
        if isinstance(b, str) and len(b) == 1:
            b = (b,) * 4
        return tuple(x if isinstance(x, int) else _BC[x] for x in b)

    def to_c(self) -> ccmg_problem:
        p = ccmg_problem()
        p.n, p.ng = self.n, 1
        p.xmin, p.xmax, p.ymin, p.ymax = self.xmin, self.xmax, self.ymin, self.ymax
        p.bc[:] = list(self.bc_codes())
        p.alpha, p.beta = self.alpha, self.beta
        p.nu1, p.nu2, p.nu_bottom = self.nu1, self.nu2, self.nu_bottom
        p.max_cycles, p.rtol, p.prec = self.max_cycles, self.rtol, self.prec
        return p

    @property
    def h(self) -> float:
        return (self.xmax - self.xmin) / self.n


@dataclass
class Result:
    status: int
    cycles: int
    rel_resid0: float
    rel_resid: float
    history: list = field(default_factory=list)
    ms: float = 0.0
    inner_cycles: int = 0


def ccmg_problem_check(prob: Problem) -> int:
    return lib().ccmg_problem_check(ctypes.byref(prob.to_c()))


def ccmg_workspace_bytes(prob: Problem) -> int:
    return lib().ccmg_workspace_bytes(ctypes.byref(prob.to_c()))


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _field_args(t: torch.Tensor, n: int, dtype=torch.float64):
    if not t.is_cuda or t.dtype != dtype or t.dim() != 2 or t.shape[0] != n + 2 or t.shape[1] < n + 2:
        raise ValueError(f"expected a {dtype} device tensor of shape ({n + 2}, >= {n + 2})")
    if t.stride(1) != 1 or t.stride(0) < n + 2:
        raise ValueError("field must be x-contiguous with row stride >= n+2")
    return t.data_ptr(), t.stride(0)


class Plan:
    """A ccmg plan with its own workspace tensor (caller-owned device memory)."""

    def __init__(self, prob: Problem, device=None, stream=None):
        self.prob = prob
        self._c = prob.to_c()
        st = lib().ccmg_problem_check(ctypes.byref(self._c))
        _check(st, "problem")
        nbytes = lib().ccmg_workspace_bytes(ctypes.byref(self._c))
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        _check(lib().ccmg_plan_create(ctypes.byref(self._c), ctypes.c_void_p(aligned), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "plan_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ccmg_plan_destroy(h)
            self.handle = None

    @property
    def n(self):
        return self.prob.n

    def level_n(self, level: int) -> int:
        return self.prob.n >> level


def ccmg_vcycle_noalloc(prob: Problem, f: torch.Tensor, phi: torch.Tensor, stream=None) -> None:
    """One V-cycle of `prob` in place on phi without a plan: the library's
    static device scratch holds the coarse levels (nothing is allocated)."""
    fp, pitch = _field_args(f, prob.n)
    pp, p2 = _field_args(phi, prob.n)
    if pitch != p2:
        raise ValueError("f and phi must share one pitch")
    c = prob.to_c()
    _check(lib().ccmg_vcycle_noalloc(ctypes.byref(c), fp, pp, pitch, _stream_handle(stream)), "ccmg_vcycle_noalloc")


def ccmg_noalloc_scratch_bytes() -> int:
    return lib().ccmg_noalloc_scratch_bytes()


def ccmg_plan_set_option(plan: Plan, option: int, value: float) -> None:
    _check(lib().ccmg_plan_set_option(plan.handle, option, float(value)), "ccmg_plan_set_option")


def ccmg_plan_get_option(plan: Plan, option: int) -> float:
    v = ctypes.c_double()
    _check(lib().ccmg_plan_get_option(plan.handle, option, ctypes.byref(v)), "ccmg_plan_get_option")
    return v.value


def ccmg_solve(plan: Plan, f: torch.Tensor, phi: torch.Tensor, use_guess: bool = False) -> Result:
    n = plan.n
    fp, pitch = _field_args(f, n)
    pp, pitch2 = _field_args(phi, n)
    if pitch != pitch2:
        raise ValueError("f and phi must share one pitch")
    r = ccmg_result()
    st = lib().ccmg_solve(plan.handle, fp, pp, pitch, int(use_guess), ctypes.byref(r))
    _check(st, "ccmg_solve", allow=(OK, NOT_CONVERGED))
    hist = [r.history[k] for k in range(min(r.cycles + 1, HISTORY))]
    return Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist, r.ms, r.inner_cycles)


def ccmg_fmg(plan: Plan, f: torch.Tensor, phi: torch.Tensor, ncyc_top: int = 1, ncyc: int = 1) -> None:
    """Full multigrid pass into phi (enqueued on the plan's stream)."""
    fp, pitch = _field_args(f, plan.n)
    pp, pitch2 = _field_args(phi, plan.n)
    if pitch != pitch2:
        raise ValueError("f and phi must share one pitch")
    _check(lib().ccmg_fmg(plan.handle, fp, pp, pitch, ncyc_top, ncyc), "ccmg_fmg")


def _side_data(plan: Plan, b) -> "ctypes.Array":
    """Four 1-d FP64 device tensors of n values (or None) -> the host array
    of device pointers the library takes."""
    arr = (ctypes.c_void_p * 4)()
    for s_, v in enumerate(b or [None] * 4):
        if v is None:
            arr[s_] = None
            continue
        if v.dtype != torch.float64 or not v.is_cuda or v.numel() != plan.n or not v.is_contiguous():
            raise ValueError("side data: contiguous float64 device tensors of n values")
        arr[s_] = v.data_ptr()
    return arr


def ccmg_bc_rhs(plan: Plan, f: torch.Tensor, f_out: torch.Tensor, b) -> None:
    fp, pitch = _field_args(f, plan.n)
    op, pitch2 = _field_args(f_out, plan.n)
    if pitch != pitch2:
        raise ValueError("f and f_out must share one pitch")
    _check(lib().ccmg_bc_rhs(plan.handle, fp, op, pitch, _side_data(plan, b)), "ccmg_bc_rhs")


def ccmg_fill_ghosts_bc(plan: Plan, phi: torch.Tensor, b) -> None:
    pp, pitch = _field_args(phi, plan.n)
    _check(lib().ccmg_fill_ghosts_bc(plan.handle, pp, pitch, _side_data(plan, b)), "ccmg_fill_ghosts_bc")


def ccmg_solve_bc(plan: Plan, f: torch.Tensor, phi: torch.Tensor, b, work: torch.Tensor,
                  use_guess: bool = False) -> Result:
    """Solve with side data b: four 1-d device tensors of n values (Dirichlet
    face values / Neumann derivatives) or None per side (x-lo, x-hi, y-lo,
    y-hi); `work` is scratch of f's layout."""
    fp, pitch = _field_args(f, plan.n)
    pp, pitch2 = _field_args(phi, plan.n)
    wp, pitch3 = _field_args(work, plan.n)
    if not (pitch == pitch2 == pitch3):
        raise ValueError("f, phi and work must share one pitch")
    r = ccmg_result()
    st = lib().ccmg_solve_bc(plan.handle, fp, pp, pitch, int(use_guess), _side_data(plan, b), wp, ctypes.byref(r))
    _check(st, "ccmg_solve_bc", allow=(OK, NOT_CONVERGED))
    hist = [r.history[k] for k in range(min(r.cycles + 1, HISTORY))]
    return Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist, r.ms, r.inner_cycles)


def ccmg_project(plan: Plan, u: torch.Tensor, v: torch.Tensor, phi: torch.Tensor, work: torch.Tensor) -> Result:
    """Approximate cell-centred projection of (u, v) in place (periodic
    Poisson plan); phi receives the potential, work is scratch."""
    ptrs = [_field_args(t, plan.n) for t in (u, v, phi, work)]
    if len({p_[1] for p_ in ptrs}) != 1:
        raise ValueError("u, v, phi and work must share one pitch")
    r = ccmg_result()
    st = lib().ccmg_project(plan.handle, ptrs[0][0], ptrs[1][0], ptrs[0][1], ptrs[2][0], ptrs[3][0], ctypes.byref(r))
    _check(st, "ccmg_project", allow=(OK, NOT_CONVERGED))
    hist = [r.history[k] for k in range(min(r.cycles + 1, HISTORY))]
    return Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist, r.ms, r.inner_cycles)


def ccmg_cn_rhs(plan: Plan, phi: torch.Tensor, f: torch.Tensor) -> None:
    """f = phi + beta Lap phi (the Crank-Nicolson right-hand side) with the
    plan's beta = k dt / 2 and side rules; asynchronous."""
    pp, pitch = _field_args(phi, plan.n)
    fp, pitch2 = _field_args(f, plan.n)
    if pitch != pitch2:
        raise ValueError("phi and f must share one pitch")
    _check(lib().ccmg_cn_rhs(plan.handle, pp, fp, pitch), "ccmg_cn_rhs")


def ccmg_cn_step(plan: Plan, phi: torch.Tensor, work: torch.Tensor) -> Result:
    """One Crank-Nicolson step of phi_t = k Lap phi in place (plan made with
    alpha = 1, beta = k dt / 2); `work` is scratch of phi's layout."""
    pp, pitch = _field_args(phi, plan.n)
    wp, pitch2 = _field_args(work, plan.n)
    if pitch != pitch2:
        raise ValueError("phi and work must share one pitch")
    r = ccmg_result()
    st = lib().ccmg_cn_step(plan.handle, pp, wp, pitch, ctypes.byref(r))
    _check(st, "ccmg_cn_step", allow=(OK, NOT_CONVERGED))
    hist = [r.history[k] for k in range(min(r.cycles + 1, HISTORY))]
    return Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist, r.ms, r.inner_cycles)


def ccmg_vcycle(plan: Plan, f: torch.Tensor, phi: torch.Tensor) -> None:
    fp, pitch = _field_args(f, plan.n)
    pp, pitch2 = _field_args(phi, plan.n)
    if pitch != pitch2:
        raise ValueError("f and phi must share one pitch")
    _check(lib().ccmg_vcycle(plan.handle, fp, pp, pitch), "ccmg_vcycle")


def ccmg_fill_ghosts(plan: Plan, level: int, a: torch.Tensor) -> None:
    ap, pitch = _field_args(a, plan.level_n(level))
    _check(lib().ccmg_fill_ghosts(plan.handle, level, ap, pitch), "ccmg_fill_ghosts")


def ccmg_smooth(plan: Plan, level: int, iters: int, f, phi_in, phi_out) -> None:
    n = plan.level_n(level)
    fp, pitch = _field_args(f, n)
    ip, p2 = _field_args(phi_in, n)
    op, p3 = _field_args(phi_out, n)
    if not (pitch == p2 == p3):
        raise ValueError("f, phi_in and phi_out must share one pitch")
    _check(lib().ccmg_smooth(plan.handle, level, iters, fp, ip, op, pitch), "ccmg_smooth")


def ccmg_residual(plan: Plan, level: int, f, phi, r) -> None:
    n = plan.level_n(level)
    fp, pitch = _field_args(f, n)
    pp, p2 = _field_args(phi, n)
    rp, p3 = _field_args(r, n)
    if not (pitch == p2 == p3):
        raise ValueError("f, phi and r must share one pitch")
    _check(lib().ccmg_residual(plan.handle, level, fp, pp, rp, pitch), "ccmg_residual")


def ccmg_restrict_residual(plan: Plan, level: int, f, phi, fc) -> None:
    n = plan.level_n(level)
    fp, pitch = _field_args(f, n)
    pp, p2 = _field_args(phi, n)
    cp, pc = _field_args(fc, n // 2)
    if pitch != p2:
        raise ValueError("f and phi must share one pitch")
    _check(lib().ccmg_restrict_residual(plan.handle, level, fp, pp, pitch, cp, pc), "ccmg_restrict_residual")


def ccmg_restrict(plan: Plan, level: int, fine, coarse) -> None:
    n = plan.level_n(level)
    fp, pitch = _field_args(fine, n)
    cp, pc = _field_args(coarse, n // 2)
    _check(lib().ccmg_restrict(plan.handle, level, fp, pitch, cp, pc), "ccmg_restrict")


def ccmg_prolong_add(plan: Plan, level: int, ec, phi_in, phi_out) -> None:
    n = plan.level_n(level)
    ep, pc = _field_args(ec, n // 2)
    ip, pitch = _field_args(phi_in, n)
    op, p2 = _field_args(phi_out, n)
    if pitch != p2:
        raise ValueError("phi_in and phi_out must share one pitch")
    _check(lib().ccmg_prolong_add(plan.handle, level, ep, pc, ip, op, pitch), "ccmg_prolong_add")


def ccmg_plan_autotune(plan: Plan, f: torch.Tensor, phi: torch.Tensor) -> None:
    fp, pitch = _field_args(f, plan.n)
    pp, pitch2 = _field_args(phi, plan.n)
    if pitch != pitch2:
        raise ValueError("f and phi must share one pitch")
    _check(lib().ccmg_plan_autotune(plan.handle, fp, pp, pitch), "ccmg_plan_autotune")


def ccmg_plan_set_shape(plan: Plan, level: int, kind: int, ty: int, wpb: int) -> None:
    _check(lib().ccmg_plan_set_shape(plan.handle, level, kind, ty, wpb), "ccmg_plan_set_shape")


def ccmg_plan_set_bottom(plan: Plan, n_bottom: int) -> None:
    """Bottom of the V-cycle: 2 = relaxations on 2 x 2 (default), 4 or 8 =
    exact solve on that level."""
    _check(lib().ccmg_plan_set_bottom(plan.handle, n_bottom), "ccmg_plan_set_bottom")


def ccmg_plan_fused_shape(plan: Plan, kind: int = 2) -> tuple:
    """(ty, wpb) of the fused finest launch: kind 2 FP64, 3 FP32."""
    ty, wpb = ctypes.c_int(), ctypes.c_int()
    _check(lib().ccmg_plan_fused_shape(plan.handle, kind, ctypes.byref(ty), ctypes.byref(wpb)),
           "ccmg_plan_fused_shape")
    return ty.value, wpb.value


def ccmg_plan_shape(plan: Plan, level: int, kind: int) -> tuple:
    """(ty, wpb) of one launch, kinds as for ccmg_plan_set_shape (kind 5:
    ty = 0 for a level that does not run as a visit)."""
    ty, wpb = ctypes.c_int(), ctypes.c_int()
    _check(lib().ccmg_plan_shape(plan.handle, level, kind, ctypes.byref(ty), ctypes.byref(wpb)), "ccmg_plan_shape")
    return ty.value, wpb.value


def ccmg_plan_shapes(plan: Plan) -> list:
    """[(ty_pre, wpb_pre, ty_post, wpb_post)] per level."""
    L = 16
    a, b, c, d = [(ctypes.c_int * L)() for _ in range(4)]
    _check(lib().ccmg_plan_shapes(plan.handle, a, b, c, d, L), "ccmg_plan_shapes")
    levels = plan.n.bit_length() - 1
    return [(a[k], b[k], c[k], d[k]) for k in range(min(levels, L))]


def ccmg_plan_profile(plan: Plan, enable: bool) -> None:
    _check(lib().ccmg_plan_profile(plan.handle, int(enable)), "ccmg_plan_profile")


def ccmg_plan_kernel_stats(plan: Plan) -> list:
    """[{name, launches, ms, bytes}] summed since profiling was enabled."""
    cnt = ctypes.c_int()
    _check(lib().ccmg_plan_kernel_stats(plan.handle, None, 0, ctypes.byref(cnt)), "ccmg_plan_kernel_stats")
    arr = (ccmg_kernel_stat * max(1, cnt.value))()
    _check(lib().ccmg_plan_kernel_stats(plan.handle, arr, cnt.value, ctypes.byref(cnt)), "ccmg_plan_kernel_stats")
    return [dict(name=arr[k].name.decode(), launches=arr[k].launches, ms=arr[k].ms, bytes=arr[k].bytes)
            for k in range(cnt.value)]


def ccmg_probe_stream(a, b, c, reps: int = 20):
    """c = a + b over the elements of three float64 CUDA tensors of equal size
    (the library's streaming probe, fastest of its launch shapes); returns
    (mean ms per launch, shape: workgroups per compute unit, + 1000 if
    nontemporal)."""
    for t in (a, b, c):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("ccmg_probe_stream: contiguous float64 CUDA tensors")
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("ccmg_probe_stream: tensors of one size")
    ms, cfg = ctypes.c_float(), ctypes.c_int()
    _check(lib().ccmg_probe_stream(a.data_ptr(), b.data_ptr(), c.data_ptr(), a.numel(), reps, _stream_handle(),
                                   ctypes.byref(ms), ctypes.byref(cfg)), "ccmg_probe_stream")
    return ms.value, cfg.value


class Batch:
    """A ccmg batch of independent problems with its own workspace tensor."""

    def __init__(self, probs, device=None, stream=None):
        self.probs = list(probs)
        self.m = len(self.probs)
        arr = (ccmg_problem * self.m)(*[p.to_c() for p in self.probs])
        self._c = arr
        nbytes = lib().ccmg_batch_workspace_bytes(self.m, arr)
        if nbytes == 0:
            raise CcmgError(EINVAL, "batch problems (each needs a valid problem with nu1 = nu2 = 2)")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        _check(lib().ccmg_batch_create(self.m, arr, ctypes.c_void_p(aligned), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "batch_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ccmg_batch_destroy(h)
            self.handle = None


def _batch_arrays(batch: Batch, fs, phis):
    if len(fs) != batch.m or len(phis) != batch.m:
        raise ValueError("one f and one phi per problem")
    fp = (ctypes.c_void_p * batch.m)()
    pp = (ctypes.c_void_p * batch.m)()
    pit = (ctypes.c_ssize_t * batch.m)()
    for i, (f, phi, pr) in enumerate(zip(fs, phis, batch.probs)):
        a, p1 = _field_args(f, pr.n)
        b, p2 = _field_args(phi, pr.n)
        if p1 != p2:
            raise ValueError("f and phi of one problem must share a pitch")
        fp[i], pp[i], pit[i] = a, b, p1
    return fp, pp, pit


def ccmg_batch_solve(batch: Batch, fs, phis, use_guess: bool = False):
    """Returns (list of Result, {steps, converged, ms})."""
    fp, pp, pit = _batch_arrays(batch, fs, phis)
    res = (ccmg_result * batch.m)()
    info = ccmg_batch_info()
    st = lib().ccmg_batch_solve(batch.handle, fp, pp, pit, int(use_guess), res, ctypes.byref(info))
    if st in (EINVAL, EHIP, EWORKSPACE):
        raise CcmgError(st, "ccmg_batch_solve")
    out = []
    for r in res:
        hist = [r.history[k] for k in range(min(r.cycles + 1, HISTORY))]
        out.append(Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist, r.ms, r.inner_cycles))
    return out, dict(status=st, steps=info.steps, converged=info.converged, ms=info.ms)


def ccmg_batch_set_option(batch: Batch, option: int, value: float) -> None:
    _check(lib().ccmg_batch_set_option(batch.handle, option, float(value)), "ccmg_batch_set_option")


def ccmg_batch_autotune(batch: Batch, fs, phis) -> None:
    fp, pp, pit = _batch_arrays(batch, fs, phis)
    _check(lib().ccmg_batch_autotune(batch.handle, fp, pp, pit), "ccmg_batch_autotune")


def ccmg_batch_shapes(batch: Batch) -> dict:
    sizes, ty = (ctypes.c_int * 16)(), (ctypes.c_int * 16)()
    cnt, waves = ctypes.c_int(), ctypes.c_int()
    _check(lib().ccmg_batch_shapes(batch.handle, sizes, ty, 16, ctypes.byref(cnt), ctypes.byref(waves)),
           "ccmg_batch_shapes")
    return dict(sizes=[sizes[k] for k in range(cnt.value)], ty=[ty[k] for k in range(cnt.value)],
                waves=waves.value)


NET_G = 128  # side of the network's grid


def ccmg_net_param_count() -> int:
    return lib().ccmg_net_param_count()


def ccmg_net_workspace_bytes(batch: int, n_max: int) -> int:
    return lib().ccmg_net_workspace_bytes(batch, n_max)


class Net:
    """A ccmg net (learned initial guess) with its own workspace tensor.
    `batch`: largest training batch; `n_max`: largest problem side it guesses for."""

    def __init__(self, batch: int = 32, n_max: int = 1024, device=None, stream=None):
        nbytes = lib().ccmg_net_workspace_bytes(batch, n_max)
        if nbytes == 0:
            raise CcmgError(EINVAL, "net sizes (batch 1..1024, n_max a power of two in 128..16384)")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.batch, self.n_max, self.device = batch, n_max, dev
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        _check(lib().ccmg_net_create(batch, n_max, ctypes.c_void_p(aligned), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "net_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ccmg_net_destroy(h)
            self.handle = None


def _net_images(net: Net, t: torch.Tensor, what: str) -> int:
    if (not t.is_cuda or t.dtype != torch.float32 or t.dim() != 3 or tuple(t.shape[1:]) != (NET_G, NET_G)
            or not t.is_contiguous()):
        raise ValueError(f"{what}: expected a contiguous float32 device tensor of shape (nb, {NET_G}, {NET_G})")
    if not 1 <= t.shape[0] <= net.batch:
        raise ValueError(f"{what}: batch of {t.shape[0]} outside 1..{net.batch}")
    return t.shape[0]


def _param_vec(t: torch.Tensor) -> None:
    if (not t.is_cuda or t.dtype != torch.float32 or t.numel() != ccmg_net_param_count()
            or not t.is_contiguous()):
        raise ValueError("parameters: expected a contiguous float32 device vector of ccmg_net_param_count()")


def ccmg_net_set_params(net: Net, params: torch.Tensor) -> None:
    _param_vec(params)
    _check(lib().ccmg_net_set_params(net.handle, params.data_ptr()), "ccmg_net_set_params")


def ccmg_net_get_params(net: Net) -> torch.Tensor:
    out = torch.empty(ccmg_net_param_count(), dtype=torch.float32, device=net.device)
    _check(lib().ccmg_net_get_params(net.handle, out.data_ptr()), "ccmg_net_get_params")
    return out


def ccmg_net_state_count() -> int:
    return lib().ccmg_net_state_count()


def ccmg_net_get_state(net: Net):
    """(state, step): parameters and Adam moments as one FP32 device tensor,
    and Adam's step counter."""
    out = torch.empty(ccmg_net_state_count(), dtype=torch.float32, device=net.device)
    step = ctypes.c_int()
    _check(lib().ccmg_net_get_state(net.handle, out.data_ptr(), ctypes.byref(step)), "ccmg_net_get_state")
    return out, step.value


def ccmg_net_set_state(net: Net, state: torch.Tensor, step: int) -> None:
    if state.dtype != torch.float32 or not state.is_cuda or not state.is_contiguous() or \
            state.numel() != ccmg_net_state_count():
        raise ValueError("ccmg_net_set_state: a contiguous float32 CUDA tensor of ccmg_net_state_count() values")
    _check(lib().ccmg_net_set_state(net.handle, state.data_ptr(), int(step)), "ccmg_net_set_state")


def ccmg_net_forward(net: Net, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    nb = _net_images(net, x, "x")
    if y is None:
        y = torch.empty_like(x)
    _net_images(net, y, "y")
    _check(lib().ccmg_net_forward(net.handle, x.data_ptr(), y.data_ptr(), nb), "ccmg_net_forward")
    return y


def ccmg_net_loss_grad(net: Net, x: torch.Tensor, t: torch.Tensor):
    """(loss, gradient vector) of the mean squared error of net(x) against t."""
    nb = _net_images(net, x, "x")
    if _net_images(net, t, "t") != nb:
        raise ValueError("x and t differ in batch")
    g = torch.empty(ccmg_net_param_count(), dtype=torch.float32, device=net.device)
    loss = ctypes.c_float()
    _check(lib().ccmg_net_loss_grad(net.handle, x.data_ptr(), t.data_ptr(), nb, g.data_ptr(), ctypes.byref(loss)),
           "ccmg_net_loss_grad")
    return loss.value, g


def ccmg_net_train_step(net: Net, x: torch.Tensor, t: torch.Tensor, lr: float, want_loss: bool = True):
    """One Adam step; returns the loss before the step (None unless want_loss:
    reading it back synchronises the stream)."""
    nb = _net_images(net, x, "x")
    if _net_images(net, t, "t") != nb:
        raise ValueError("x and t differ in batch")
    loss = ctypes.c_float()
    _check(lib().ccmg_net_train_step(net.handle, x.data_ptr(), t.data_ptr(), nb, float(lr),
                                     ctypes.byref(loss) if want_loss else None), "ccmg_net_train_step")
    return loss.value if want_loss else None


def ccmg_net_encode(net: Net, a: torch.Tensor, scale_src: torch.Tensor, out: torch.Tensor | None = None):
    """Block means of the field `a` on the network grid, divided by the RMS of
    the field `scale_src`; out: (NET_G, NET_G) float32 (a view into a batch is fine)."""
    n = a.shape[0] - 2
    ap, pa = _field_args(a, n)
    sp, ps = _field_args(scale_src, n)
    if out is None:
        out = torch.empty((NET_G, NET_G), dtype=torch.float32, device=a.device)
    if out.dtype != torch.float32 or tuple(out.shape) != (NET_G, NET_G) or not out.is_contiguous():
        raise ValueError(f"out: expected a contiguous float32 ({NET_G}, {NET_G}) tensor")
    _check(lib().ccmg_net_encode(net.handle, ap, pa, n, sp, ps, out.data_ptr()), "ccmg_net_encode")
    return out


COARSE_ITERS = 32  # default relaxation iterations on the network's grid


def ccmg_net_guess(net: Net, f: torch.Tensor, phi: torch.Tensor, length: float = 1.0,
                   coarse_iters: int = COARSE_ITERS) -> None:
    n = f.shape[0] - 2
    fp, pf = _field_args(f, n)
    pp, pph = _field_args(phi, n)
    _check(lib().ccmg_net_guess(net.handle, fp, pf, n, float(length), int(coarse_iters), pp, pph), "ccmg_net_guess")


def ccmg_solve_learned(plan: Plan, net: Net, f: torch.Tensor, phi: torch.Tensor, coarse_iters: int = COARSE_ITERS):
    """Guess with the net, then plain multigrid to tolerance; returns (Result, guess_used)."""
    n = plan.n
    fp, pitch = _field_args(f, n)
    pp, pitch2 = _field_args(phi, n)
    if pitch != pitch2:
        raise ValueError("f and phi must share one pitch")
    r = ccmg_result()
    used = ctypes.c_int()
    st = lib().ccmg_solve_learned(plan.handle, net.handle, fp, pp, pitch, int(coarse_iters), ctypes.byref(r),
                                  ctypes.byref(used))
    _check(st, "ccmg_solve_learned", allow=(OK, NOT_CONVERGED))
    hist = [r.history[k] for k in range(min(r.cycles + 1, HISTORY))]
    return Result(r.status, r.cycles, r.rel_resid0, r.rel_resid, hist, r.ms, r.inner_cycles), bool(used.value)


def field(n: int, dtype=torch.float64, device="cuda", pitch: int | None = None) -> torch.Tensor:
    """A zeroed (n+2, pitch) field on the device (a view when pitch > n+2)."""
    p = pitch or (n + 2)
    return torch.zeros((n + 2, p), dtype=dtype, device=device)


def to_field(valid, device="cuda", pitch: int | None = None) -> torch.Tensor:
    """Upload an (n, n) host array of valid cells into a zero-ghost device field."""
    v = torch.as_tensor(valid, dtype=torch.float64)
    n = v.shape[0]
    t = field(n, device=device, pitch=pitch)
    t[1:n + 1, 1:n + 1] = v.to(device)
    return t


def solve(prob: Problem, f_valid, guess=None):
    """Convenience: solve on the current device from host arrays; returns (phi field, Result)."""
    plan = Plan(prob)
    f = to_field(f_valid)
    phi = to_field(guess) if guess is not None else field(prob.n)
    res = ccmg_solve(plan, f, phi, use_guess=guess is not None)
    return phi, res
