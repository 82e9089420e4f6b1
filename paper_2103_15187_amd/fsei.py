"""Python binding of libfsei (ctypes; argument marshalling only).

Every step of the projection runs in the HIP kernels of ``libfsei.so``; this
module only passes device pointers, sizes and the current HIP stream.  PyTorch
provides device memory (fields and workspace) and streams.  If the native
library has not been built, every entry point raises ``RuntimeError``: there
is no fallback implementation.

Functions follow the C ABI in ``include/fsei.h``:
``fsei_poisson_plan_create`` / ``fsei_poisson_solve`` / ``fsei_project`` /
``fsei_project_backward`` (+ FP32 variants), and ``fsei_viscous_solve`` (the
implicit viscous step).  ``ProjectFn`` wraps the forward
projection and its hand-written adjoint as a ``torch.autograd.Function``.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PERIODIC = 0
WALL = 1
PREC_FP64 = 0
PREC_FP32_REFINE = 1
PREC_FP32 = 2
NUM_KERNEL_SLOTS = 22   # FSEI_NUM_KERNEL_SLOTS

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsei.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "fsei.h")

_lib = None


class FseiError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = lib().fsei_status_string(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("rhs_vmean_removed", ctypes.c_double), ("floor_reached", ctypes.c_int)]


def lib():
    """Load libfsei.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(there is no non-native fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    S = ctypes.c_size_t
    sig = {
        "fsei_poisson_plan_create": (I, [I, I, I, ctypes.POINTER(I), D, D, ctypes.POINTER(D), ctypes.POINTER(P)]),
        "fsei_poisson_plan_destroy": (None, [P]),
        "fsei_plan_set_precision": (I, [P, I, D, I]),
        "fsei_plan_workspace_size": (I, [P, ctypes.POINTER(S)]),
        "fsei_plan_set_workspace": (I, [P, P, S]),
        "fsei_plan_set_stream": (I, [P, P]),
        "fsei_poisson_solve": (I, [P, P, P, ctypes.POINTER(Info)]),
        "fsei_project": (I, [P, P, P, P, P, D, ctypes.POINTER(Info)]),
        "fsei_project_noalloc": (I, [P, P, P, P, P, D, ctypes.POINTER(Info)]),
        "fsei_project_noalloc_max_bytes": (S, []),
        "fsei_project_backward": (I, [P, P, P, P, P, D]),
        "fsei_project_f32": (I, [P, P, P, P, P, ctypes.c_float]),
        "fsei_project_backward_f32": (I, [P, P, P, P, P, ctypes.c_float]),
        "fsei_viscous_solve": (I, [P, I, P, D]),
        "fsei_viscous_solve_add": (I, [P, I, P, P, D]),
        "fsei_momentum_rhs": (I, [P, P, P, P, P, P, P, P, P, P, D, D, D, D]),
        "fsei_ib_interpolate": (I, [P, I, P, P, ctypes.c_long, P]),
        "fsei_ib_spread": (I, [P, I, P, P, P, P, ctypes.c_long]),
        "fsei_plan_set_timing": (I, [P, I]),
        "fsei_plan_reset_timing": (I, [P]),
        "fsei_plan_kernel_time": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_long),
                                      ctypes.POINTER(ctypes.c_char_p)]),
        "fsei_status_string": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/fsei.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fsei_[a-z0-9_]+)\s*\(", txt)))


def _check(status, what):
    if status != 0:
        raise FseiError(status, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A solver plan for one grid: nx x ny x nz cells, bc = (bc_x, bc_y),
    uniform dx, dy, z-face coordinates zc (nz+1, strictly increasing).
    The workspace is a torch uint8 tensor on `device`."""

    def __init__(self, nx, ny, nz, bc, dx, dy, zc, precision=PREC_FP64, rtol=1e-10, max_iter=4,
                 device="cuda", accept_floor=False, workspace=True):
        import torch
        L = lib()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.bc = (int(bc[0]), int(bc[1]))
        self.dx, self.dy = float(dx), float(dy)
        self.zc = np.ascontiguousarray(zc, dtype=np.float64)
        if self.zc.shape != (self.nz + 1,):
            raise ValueError("zc must hold nz+1 face coordinates")
        h = ctypes.c_void_p()
        bca = (ctypes.c_int * 2)(*self.bc)
        _check(L.fsei_poisson_plan_create(self.nx, self.ny, self.nz, bca, self.dx, self.dy,
                                          self.zc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.byref(h)), "fsei_poisson_plan_create")
        self._h = h
        self.precision = precision
        # FP32_REFINE: when the refinement stops at the FP64 rounding floor of
        # the right-hand side above rtol, return the iterate (with a warning)
        # instead of raising FseiError(FSEI_ERR_NOT_CONVERGED)
        self.accept_floor = bool(accept_floor)
        _check(L.fsei_plan_set_precision(h, precision, float(rtol), int(max_iter)), "fsei_plan_set_precision")
        nbytes = ctypes.c_size_t()
        _check(L.fsei_plan_workspace_size(h, ctypes.byref(nbytes)), "fsei_plan_workspace_size")
        self.workspace_bytes = nbytes.value
        self.device = torch.device(device)
        self._ws = None
        if workspace:
            # workspace=False: a plan for project_noalloc only (no device memory)
            self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
            with torch.cuda.device(self.device):   # the plan's side stream is made on its device
                _check(L.fsei_plan_set_workspace(h, _ptr(self._ws), self.workspace_bytes), "fsei_plan_set_workspace")

    @classmethod
    def from_spec(cls, spec, **kw):
        return cls(spec.nx, spec.ny, spec.nz, (spec.bcx, spec.bcy), spec.dx, spec.dy, spec.zc(), **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fsei_poisson_plan_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    # -- helpers --------------------------------------------------------------
    def _stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().fsei_plan_set_stream(self._h, ctypes.c_void_p(s)), "fsei_plan_set_stream")

    def _field(self, t, dtype, name):
        import torch
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device.type != "cuda" \
                or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {self.shape}")
        return t

    def _floor_ok(self):
        return self.accept_floor and self.precision == PREC_FP32_REFINE

    def _status(self, status, what, inf):
        if status == -6 and self._floor_ok() and inf.floor_reached:
            import warnings
            warnings.warn(f"{what}: refinement stopped at the FP64 rounding floor, relative residual "
                          f"{inf.rel_residual:.3e} (above rtol)", RuntimeWarning, stacklevel=3)
            return
        _check(status, what)

    # -- entry points ---------------------------------------------------------
    def poisson_solve(self, f, p=None, info=False):
        """p = L^+ f (double; p may be f for an in-place solve)."""
        import torch
        f = self._field(f, torch.float64, "f")
        if p is None:
            p = torch.empty_like(f)
        p = self._field(p, torch.float64, "p")
        self._stream()
        inf = Info()
        want = info or self._floor_ok()
        self._status(lib().fsei_poisson_solve(self._h, _ptr(f), _ptr(p), ctypes.byref(inf) if want else None),
                     "fsei_poisson_solve", inf)
        return (p, _info_dict(inf)) if info else p

    def project(self, u, v, w, p=None, dt=1.0, info=False, want_p=True):
        """In place: u, v, w <- projected velocity; returns p (and info)."""
        import torch
        if self.precision == PREC_FP32:
            u, v, w = (self._field(a, torch.float32, n) for a, n in ((u, "u"), (v, "v"), (w, "w")))
            if p is None and want_p:
                p = torch.empty_like(u)
            self._stream()
            _check(lib().fsei_project_f32(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(p), float(dt)),
                   "fsei_project_f32")
            return (p, None) if info else p
        u, v, w = (self._field(a, torch.float64, n) for a, n in ((u, "u"), (v, "v"), (w, "w")))
        if p is None and want_p:
            p = torch.empty_like(u)
        p = self._field(p, torch.float64, "p")
        self._stream()
        inf = Info()
        want = info or self._floor_ok()
        self._status(lib().fsei_project(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(p), float(dt),
                                        ctypes.byref(inf) if want else None), "fsei_project", inf)
        return (p, _info_dict(inf)) if info else p

    def project_noalloc(self, u, v, w, p=None, dt=1.0, info=False):
        """As project (double I/O plans), on the library's static device
        scratch instead of the plan's workspace; allocates nothing itself
        (p must then be given, or no pressure is returned)."""
        import torch
        u, v, w = (self._field(a, torch.float64, n) for a, n in ((u, "u"), (v, "v"), (w, "w")))
        p = self._field(p, torch.float64, "p")
        self._stream()
        inf = Info()
        want = info or self._floor_ok()
        with torch.cuda.device(self.device):   # the scratch copy of the plan's GPU
            st = lib().fsei_project_noalloc(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(p), float(dt),
                                            ctypes.byref(inf) if want else None)
        self._status(st, "fsei_project_noalloc", inf)
        return (p, _info_dict(inf)) if info else p

    def project_backward(self, gu, gv, gw, gp=None, dt=1.0):
        """In place: gu, gv, gw <- dLoss/du* given dLoss/du (and dLoss/dp)."""
        import torch
        dtype = torch.float32 if self.precision == PREC_FP32 else torch.float64
        gu, gv, gw = (self._field(a, dtype, n) for a, n in ((gu, "gu"), (gv, "gv"), (gw, "gw")))
        gp = self._field(gp, dtype, "gp")
        self._stream()
        if dtype == torch.float32:
            _check(lib().fsei_project_backward_f32(self._h, _ptr(gu), _ptr(gv), _ptr(gw), _ptr(gp), float(dt)),
                   "fsei_project_backward_f32")
        else:
            _check(lib().fsei_project_backward(self._h, _ptr(gu), _ptr(gv), _ptr(gw), _ptr(gp), float(dt)),
                   "fsei_project_backward")

    def viscous_solve(self, q, component, beta):
        """In place: q <- dq with (I - beta Lx)(I - beta Ly)(I - beta Lz) dq = q
        for velocity component 0 (u), 1 (v) or 2 (w) (implicit viscous step)."""
        import torch
        q = self._field(q, torch.float64, "q")
        self._stream()
        _check(lib().fsei_viscous_solve(self._h, int(component), _ptr(q), float(beta)), "fsei_viscous_solve")
        return q

    def momentum_rhs(self, u, v, w, n, r, dt, re, gamma=1.5, rho=-0.5):
        """r <- dt [-(gamma N^n + rho N^{n-1}) + Lap u^n / Re] per component and
        n <- N^n (n holds N^{n-1} on entry; r, n: 3-tuples of fields)."""
        import torch
        u, v, w = (self._field(a, torch.float64, nm) for a, nm in ((u, "u"), (v, "v"), (w, "w")))
        n = [self._field(a, torch.float64, "n") for a in n]
        r = [self._field(a, torch.float64, "r") for a in r]
        self._stream()
        _check(lib().fsei_momentum_rhs(self._h, _ptr(u), _ptr(v), _ptr(w), *(_ptr(a) for a in n),
                                       *(_ptr(a) for a in r), float(dt), float(re), float(gamma), float(rho)),
               "fsei_momentum_rhs")
        return r

    def _markers(self, t, cols, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda" \
                or not t.is_contiguous() or (t.dim() != (2 if cols else 1)) or (cols and t.shape[1] != cols):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (nb{', 3' if cols else ''})")
        return t

    def ib_interpolate(self, field, comp, xb, ub=None):
        """ub[b] = MLS interpolation of field (component comp) at marker xb[b]."""
        import torch
        field = self._field(field, torch.float64, "field")
        xb = self._markers(xb, 3, "xb")
        if ub is None:
            ub = torch.empty(xb.shape[0], dtype=torch.float64, device=xb.device)
        ub = self._markers(ub, 0, "ub")
        self._stream()
        _check(lib().fsei_ib_interpolate(self._h, int(comp), _ptr(field), _ptr(xb), xb.shape[0], _ptr(ub)),
               "fsei_ib_interpolate")
        return ub

    def ib_spread(self, field, comp, xb, fb, dvb):
        """field += MLS spreading of the marker values fb (volumes dvb)."""
        import torch
        field = self._field(field, torch.float64, "field")
        xb = self._markers(xb, 3, "xb")
        fb = self._markers(fb, 0, "fb")
        dvb = self._markers(dvb, 0, "dvb")
        self._stream()
        _check(lib().fsei_ib_spread(self._h, int(comp), _ptr(field), _ptr(xb), _ptr(fb), _ptr(dvb), xb.shape[0]),
               "fsei_ib_spread")
        return field

    def viscous_solve_add(self, rhs, u, component, beta):
        """In place: u <- u + dq with (I - beta Lx)(I - beta Ly)(I - beta Lz) dq = rhs
        (rhs is used as scratch)."""
        import torch
        rhs = self._field(rhs, torch.float64, "rhs")
        u = self._field(u, torch.float64, "u")
        self._stream()
        _check(lib().fsei_viscous_solve_add(self._h, int(component), _ptr(rhs), _ptr(u), float(beta)),
               "fsei_viscous_solve_add")
        return u

    def viscous_step(self, u, v, w, beta):
        """viscous_solve of the three components, each in place."""
        for c, q in enumerate((u, v, w)):
            self.viscous_solve(q, c, beta)
        return u, v, w

    # -- measurement ----------------------------------------------------------
    def set_timing(self, enable=True):
        _check(lib().fsei_plan_set_timing(self._h, 1 if enable else 0), "fsei_plan_set_timing")

    def reset_timing(self):
        _check(lib().fsei_plan_reset_timing(self._h), "fsei_plan_reset_timing")

    def kernel_times(self):
        """{kernel name: (total ms, launches)} for kernels launched while timing was on."""
        out = {}
        for slot in range(NUM_KERNEL_SLOTS):
            ms = ctypes.c_double()
            n = ctypes.c_long()
            name = ctypes.c_char_p()
            _check(lib().fsei_plan_kernel_time(self._h, slot, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(name)),
                   "fsei_plan_kernel_time")
            if n.value > 0:
                out[name.value.decode()] = (ms.value, n.value)
        return out


def _info_dict(inf):
    return {"iterations": inf.iterations, "rel_residual": inf.rel_residual,
            "rhs_vmean_removed": inf.rhs_vmean_removed, "floor_reached": bool(inf.floor_reached)}


def _autograd_fn():
    import torch

    class ProjectFn(torch.autograd.Function):
        """(u*, v*, w*) -> (u, v, w, p) with the hand-written adjoint."""

        @staticmethod
        def forward(ctx, plan, dt, u, v, w):
            uo, vo, wo = u.detach().clone(), v.detach().clone(), w.detach().clone()
            p = plan.project(uo, vo, wo, dt=dt)
            ctx.plan = plan
            ctx.dt = dt
            return uo, vo, wo, p

        @staticmethod
        def backward(ctx, gu, gv, gw, gp):
            plan = ctx.plan
            like = gu if gu is not None else (gv if gv is not None else gw)

            def g(t):
                return torch.zeros(plan.shape, dtype=like.dtype, device=like.device) if t is None \
                    else t.detach().contiguous().clone()
            a, b, c = g(gu), g(gv), g(gw)
            gpc = None if gp is None else gp.detach().contiguous()
            plan.project_backward(a, b, c, gpc, dt=ctx.dt)
            return None, None, a, b, c

    return ProjectFn


_ProjectFn = None


def ProjectFn():
    global _ProjectFn
    if _ProjectFn is None:
        _ProjectFn = _autograd_fn()
    return _ProjectFn


def project(u, v, w, plan, dt=1.0):
    """Differentiable projection: returns (u, v, w, p)."""
    return ProjectFn().apply(plan, dt, u, v, w)
