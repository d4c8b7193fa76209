"""ctypes binding of libfot.so (include/fot.h) with the same entry-point names.

Only argument marshalling lives here: every step of the solve runs in the HIP kernels of
libfot.so.  Device arrays are passed as raw pointers of CUDA (HIP) float64 tensors and work
is issued on torch's current stream.  If the library is missing the import-time loader
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfot.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fot.h")

FOT_OK, FOT_E_INVALID, FOT_E_NOMEM, FOT_E_HIP, FOT_E_NONFINITE, FOT_E_STATE, FOT_E_UNSUPPORTED, FOT_E_RANGE = range(8)
FOT_F64, FOT_F32, FOT_BF16, FOT_F16, FOT_BF16X3 = range(5)
FOT_FLAG_PROFILE = 1
FOT_FLAG_NO_GRAPH = 2
FOT_FLAG_NO_HISTORY = 4
FOT_FLAG_CFOT = 8
FOT_FLAG_SMALL_TILES = 16
FOT_FLAG_F64_REVERSE = 32
FOT_FLAG_STAGED_LAMBDA = 64
PRECISIONS = {"f64": FOT_F64, "f32": FOT_F32, "bf16": FOT_BF16, "f16": FOT_F16, "bf16x3": FOT_BF16X3}
STATUS_NAMES = {0: "FOT_OK", 1: "FOT_E_INVALID", 2: "FOT_E_NOMEM", 3: "FOT_E_HIP", 4: "FOT_E_NONFINITE",
                5: "FOT_E_STATE", 6: "FOT_E_UNSUPPORTED", 7: "FOT_E_RANGE"}


class fot_plan_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("batch", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_iters", ctypes.c_int), ("checkpoint_every", ctypes.c_int), ("flags", ctypes.c_int),
                ("tail_precision", ctypes.c_int), ("tail_iters", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)


class fot_report(ctypes.Structure):
    _fields_ = [("err_a", _dp), ("err_b", _dp), ("dual", _dp), ("transport_cost", _dp),
                ("err_a_history", _dp), ("err_b_history", _dp), ("iters_done", ctypes.c_int),
                ("nonfinite", ctypes.c_int), ("ms_total", ctypes.c_double), ("ms_iterations", ctypes.c_double),
                ("ms_contract", ctypes.c_double), ("n_contract", ctypes.c_int), ("graph", ctypes.c_int),
                ("err_products", _dp), ("range_iter", ctypes.POINTER(ctypes.c_int)), ("range_loss", _dp),
                ("ms_launches", _dp)]


class FOTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def header_functions(path: str = HEADER) -> list:
    """Names of the functions declared in include/fot.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fot_[a-z_]+)\s*\(", text)))


def _hip_runtimes_mapped() -> list:
    """Paths of the HIP runtime libraries mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return sorted(paths)


def load(path: str = LIB_PATH):
    """Load libfot.so (once) and declare the signatures of fot.h.

    torch ships its own HIP runtime with the same SONAME as the system one.  torch is
    imported first so that libfot.so binds to that runtime: torch's device memory and
    streams are then valid handles for the library (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfot.so not found at {path}; build it with `python -m paper_2512_19072_amd.build`")
    try:
        import torch  # noqa: F401  (binds the process to torch's HIP runtime before libfot loads)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    rts = _hip_runtimes_mapped()
    if len(rts) > 1:
        raise RuntimeError("two HIP runtimes are loaded in this process: " + ", ".join(rts))
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.fot_plan.argtypes = [ctypes.POINTER(fot_plan_desc), vp, ctypes.POINTER(vp)]
    lib.fot_plan.restype = ip
    lib.fot_solve.argtypes = [vp, vp, vp, ctypes.POINTER(dp), ip, ip, ip, vp, ctypes.POINTER(fot_report)]
    lib.fot_solve.restype = ip
    lib.fot_solve_noalloc.argtypes = [ctypes.POINTER(fot_plan_desc), vp, vp, vp, ctypes.POINTER(dp), ip, ip, vp, vp,
                                      vp, ctypes.POINTER(fot_report)]
    lib.fot_solve_noalloc.restype = ip
    lib.fot_potentials.argtypes = [vp, vp, vp, vp, vp]
    lib.fot_potentials.restype = ip
    lib.fot_backward.argtypes = [vp, ctypes.POINTER(dp), vp, vp]
    lib.fot_backward.restype = ip
    lib.fot_output_beam.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(dp)]
    lib.fot_output_beam.restype = ip
    lib.fot_polish_gs.argtypes = [vp, vp, vp, vp, ip]
    lib.fot_polish_gs.restype = ip
    lib.fot_destroy.argtypes = [vp]
    lib.fot_destroy.restype = ip
    lib.fot_last_error.argtypes = []
    lib.fot_last_error.restype = ctypes.c_char_p
    lib.fot_version.argtypes = []
    lib.fot_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != FOT_OK:
        msg = load().fot_last_error().decode(errors="replace")
        raise FOTError(status, f"{what}: {msg}")


def _ptr(t) -> Optional[int]:
    """Device pointer of a contiguous CUDA float64 tensor (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device arrays must be CUDA (HIP) tensors")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("device arrays must be contiguous float64")
    return t.data_ptr()


def _stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# ----------------------------------------------------------------------------- raw API
def fot_version() -> str:
    return load().fot_version().decode()


def fot_last_error() -> str:
    return load().fot_last_error().decode(errors="replace")


def fot_plan(n: int, batch: int = 1, precision="f32", max_iters: int = 1000, checkpoint_every: int = 0,
             flags: int = 0, stream=None, tail_precision=None, tail_iters: int = 0) -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if tail_precision is None:
        tprec = 0
    else:
        tprec = PRECISIONS[tail_precision] if isinstance(tail_precision, str) else int(tail_precision)
    d = fot_plan_desc(n, batch, prec, max_iters, checkpoint_every, flags, tprec, int(tail_iters))
    h = ctypes.c_void_p()
    _check(load().fot_plan(ctypes.byref(d), ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)), "fot_plan")
    return h.value


def fot_solve(plan: int, g, G, eps, iters: int, warm_start: bool = False, phase_out=None,
              report: Optional[fot_report] = None, check: bool = True) -> int:
    e = np.ascontiguousarray(np.atleast_1d(np.asarray(eps, dtype=np.float64)))
    st = load().fot_solve(ctypes.c_void_p(plan), ctypes.c_void_p(_ptr(g)), ctypes.c_void_p(_ptr(G)),
                          e.ctypes.data_as(_dp), int(e.size), int(iters), int(bool(warm_start)),
                          ctypes.c_void_p(_ptr(phase_out)), ctypes.byref(report) if report is not None else None)
    if check:
        _check(st, "fot_solve")
    return st


def fot_solve_noalloc(n: int, batch: int, precision, g, G, eps, iters: int, f_out=None, psi_out=None,
                      phase_out=None, report: Optional[fot_report] = None, flags: int = 0, max_iters=None,
                      tail_precision=None, tail_iters: int = 0, stream=None, check: bool = True) -> int:
    """fot_solve_noalloc: one cold-start solve on the library's static scratch array."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tprec = 0 if tail_precision is None else (PRECISIONS[tail_precision] if isinstance(tail_precision, str)
                                              else int(tail_precision))
    d = fot_plan_desc(n, batch, prec, int(max_iters or iters), 0, flags, tprec, int(tail_iters))
    e = np.ascontiguousarray(np.atleast_1d(np.asarray(eps, dtype=np.float64)))
    st = load().fot_solve_noalloc(ctypes.byref(d), ctypes.c_void_p(_stream_handle(stream)), ctypes.c_void_p(_ptr(g)),
                                  ctypes.c_void_p(_ptr(G)), e.ctypes.data_as(_dp), int(e.size), int(iters),
                                  ctypes.c_void_p(_ptr(f_out)), ctypes.c_void_p(_ptr(psi_out)),
                                  ctypes.c_void_p(_ptr(phase_out)),
                                  ctypes.byref(report) if report is not None else None)
    if check:
        _check(st, "fot_solve_noalloc")
    return st


def fot_potentials(plan: int, f_out=None, psi_out=None, f_in=None, psi_in=None):
    _check(load().fot_potentials(ctypes.c_void_p(plan), ctypes.c_void_p(_ptr(f_out)),
                                 ctypes.c_void_p(_ptr(psi_out)), ctypes.c_void_p(_ptr(f_in)),
                                 ctypes.c_void_p(_ptr(psi_in))), "fot_potentials")


def fot_backward(plan: int, dL_dDual: Optional[Sequence[float]], dL_dphase, dL_dG):
    if dL_dDual is None:
        dd = None
    else:
        arr = np.ascontiguousarray(np.asarray(dL_dDual, dtype=np.float64))
        dd = arr.ctypes.data_as(_dp)
    _check(load().fot_backward(ctypes.c_void_p(plan), dd, ctypes.c_void_p(_ptr(dL_dphase)),
                               ctypes.c_void_p(_ptr(dL_dG))), "fot_backward")


def fot_output_beam(plan: int, g, phase, G=None, intensity=None, l1: Optional[np.ndarray] = None):
    """fot_output_beam; ``l1`` is a host float64 array of length batch (or None)."""
    lp = None if l1 is None else l1.ctypes.data_as(_dp)
    _check(load().fot_output_beam(ctypes.c_void_p(plan), ctypes.c_void_p(_ptr(g)), ctypes.c_void_p(_ptr(phase)),
                                  ctypes.c_void_p(_ptr(G)), ctypes.c_void_p(_ptr(intensity)), lp),
           "fot_output_beam")


def fot_polish_gs(plan: int, g, G, phase, iters: int):
    _check(load().fot_polish_gs(ctypes.c_void_p(plan), ctypes.c_void_p(_ptr(g)), ctypes.c_void_p(_ptr(G)),
                                ctypes.c_void_p(_ptr(phase)), int(iters)), "fot_polish_gs")


def fot_destroy(plan: int):
    _check(load().fot_destroy(ctypes.c_void_p(plan)), "fot_destroy")


# ----------------------------------------------------------------------------- convenience
class Report:
    """Host-side buffers for fot_report."""

    def __init__(self, batch: int, iters: int):
        self.err_a = np.zeros(batch)
        self.err_b = np.zeros(batch)
        self.dual = np.zeros(batch)
        self.transport_cost = np.zeros(batch)
        self.err_a_history = np.zeros((iters, batch))
        self.err_b_history = np.zeros((iters, batch))
        self.err_products = np.zeros(batch)
        self.range_iter = np.zeros(batch, dtype=np.int32)
        self.range_loss = np.zeros(batch)
        self.ms_launches = np.zeros(4 * iters)
        self.raw = fot_report()
        r = self.raw
        r.err_a = self.err_a.ctypes.data_as(_dp)
        r.err_b = self.err_b.ctypes.data_as(_dp)
        r.dual = self.dual.ctypes.data_as(_dp)
        r.transport_cost = self.transport_cost.ctypes.data_as(_dp)
        r.err_a_history = self.err_a_history.ctypes.data_as(_dp)
        r.err_b_history = self.err_b_history.ctypes.data_as(_dp)
        r.err_products = self.err_products.ctypes.data_as(_dp)
        r.range_iter = self.range_iter.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        r.range_loss = self.range_loss.ctypes.data_as(_dp)
        r.ms_launches = self.ms_launches.ctypes.data_as(_dp)

    def __getattr__(self, name):
        return getattr(self.__dict__["raw"], name)


class Plan:
    """Owning wrapper of a fot_plan_t bound to torch's current stream."""

    def __init__(self, n: int, batch: int = 1, precision="f32", max_iters: int = 1000,
                 checkpoint_every: int = 0, profile: bool = False, graph: bool = True, history: bool = True,
                 cfot: bool = False, small_tiles: bool = False, tail_precision=None, tail_iters: int = 0,
                 f64_reverse: bool = False, staged_lambda: bool = False):
        """``tail_precision``/``tail_iters``: the precision schedule of fot_plan_desc (the last
        ``tail_iters`` iterations of every solve with ``tail_precision`` operands)."""
        self.n, self.batch, self.precision = n, batch, precision
        self.max_iters = max_iters
        self.checkpoint_every = checkpoint_every
        flags = ((FOT_FLAG_PROFILE if profile else 0) | (0 if graph else FOT_FLAG_NO_GRAPH)
                 | (0 if history else FOT_FLAG_NO_HISTORY) | (FOT_FLAG_CFOT if cfot else 0)
                 | (FOT_FLAG_SMALL_TILES if small_tiles else 0) | (FOT_FLAG_F64_REVERSE if f64_reverse else 0)
                 | (FOT_FLAG_STAGED_LAMBDA if staged_lambda else 0))
        self.handle = fot_plan(n, batch, precision, max_iters, checkpoint_every, flags,
                               tail_precision=tail_precision, tail_iters=tail_iters)
        # bumped by every call that replaces the state fot_backward would differentiate
        self.state_version = 0

    def solve(self, g, G, eps, iters: int, warm_start: bool = False, phase: bool = True, check: bool = True,
              out=None):
        """Run fot_solve; returns (phase tensor or None, Report, status).  ``out`` is an optional
        preallocated [batch][n][n] float64 device tensor for the phase."""
        import torch
        if out is not None:
            phase_out = out
        else:
            phase_out = torch.empty((self.batch, self.n, self.n), dtype=torch.float64, device=g.device) if phase else None
        rep = Report(self.batch, iters)
        self.state_version += 1
        st = fot_solve(self.handle, g, G, eps, iters, warm_start, phase_out, rep.raw, check=check)
        return phase_out, rep, st

    def potentials(self):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        f = torch.empty((self.batch, self.n, self.n), dtype=torch.float64, device=dev)
        psi = torch.empty_like(f)
        fot_potentials(self.handle, f, psi, None, None)
        return f, psi

    def set_potentials(self, f=None, psi=None):
        self.state_version += 1
        fot_potentials(self.handle, None, None, f, psi)

    def backward(self, dL_dDual, dL_dphase):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        out = torch.empty((self.batch, self.n, self.n), dtype=torch.float64, device=dev)
        fot_backward(self.handle, dL_dDual, dL_dphase, out)
        return out

    def output_beam(self, g, phase, G=None, intensity: bool = True):
        """(unit-power output intensity [batch][n][n] or None, L1 loss per target or None)."""
        import torch
        I = torch.empty((self.batch, self.n, self.n), dtype=torch.float64, device=g.device) if intensity else None
        l1 = np.zeros(self.batch) if G is not None else None
        fot_output_beam(self.handle, g, phase, G, I, l1)
        return I, l1

    def polish_gs(self, g, G, phase, iters: int):
        """Gerchberg-Saxton rounds on ``phase`` (in place); returns it."""
        fot_polish_gs(self.handle, g, G, phase, iters)
        return phase

    def close(self):
        if getattr(self, "handle", None):
            fot_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- autograd
def _autograd_function():
    import torch

    class FOTFunction(torch.autograd.Function):
        """(dual [B], phase [B][n][n]) = FOT(G) for a fixed input amplitude g.

        The forward pass runs fot_solve on ``plan`` (which must have checkpoint_every > 0);
        the backward pass runs fot_backward, replaying the iterations from the checkpoints.
        fot_backward differentiates the plan's last solve, so a backward after another solve
        (or a potentials write) on the same plan raises instead of returning that solve's
        gradient."""

        @staticmethod
        def forward(ctx, G, g, plan, eps, iters):
            phase, rep, _ = plan.solve(g, G.detach().contiguous(), eps, iters)
            ctx.plan = plan
            ctx.state_version = plan.state_version
            dual = torch.tensor(rep.dual, dtype=torch.float64, device=G.device)
            return dual, phase

        @staticmethod
        def backward(ctx, grad_dual, grad_phase):
            if ctx.plan.state_version != ctx.state_version:
                raise RuntimeError("fot_apply: the plan ran another solve (or its potentials were set) after this "
                                   "forward pass; its tape no longer belongs to this node (use one plan per "
                                   "differentiated solve)")
            dd = None if grad_dual is None else grad_dual.detach().double().cpu().numpy()
            gp = None if grad_phase is None else grad_phase.detach().double().contiguous()
            dG = ctx.plan.backward(dd, gp)
            return dG, None, None, None, None

    return FOTFunction


_FOT_FUNCTION = None


def fot_apply(G, g, plan: "Plan", eps, iters: int):
    """Differentiable solve: returns (dual [B], phase [B][n][n]) as torch tensors."""
    global _FOT_FUNCTION
    if _FOT_FUNCTION is None:
        _FOT_FUNCTION = _autograd_function()
    return _FOT_FUNCTION.apply(G, g, plan, eps, iters)
