"""Thin Python front end of the C ABI: device memory and streams come from
PyTorch, every computation runs in libfsd.so.

    prob = Problem(dim=3, n=(127,)*3, delta=(0.3, 0.5, 0.7), kplus=(1,)*3,
                   kminus=(1,)*3, M=32, T=1.0, tol=1e-10)
    u = torch.zeros(prob.shape, dtype=torch.float64, device="cuda")
    u, stats = prob.cn_step(u, F)
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _native as nat
from ._native import check, lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def make_params(dim: int, n: Sequence[int], delta: Sequence[float], kplus: Sequence[float],
                kminus: Sequence[float], M: int = 1, T: float = 1.0, solver: str = "auto",
                restart: int = 20, tol: float = 1e-9, maxit: int = 0, precision: str = "fp64",
                inner_tol: float = 1e-5, max_outer: int = 8, x0: str = "prev", domain=None,
                allow_delta_zero: bool = False, dst_mfma: bool = False,
                reorth_eta2: Optional[float] = None, precond: str = "tau") -> nat.Params:
    """fsd_params from keyword arguments (defaults from fsd_default_params)."""
    p = nat.Params()
    check(lib.fsd_default_params(C.byref(p)), "fsd_default_params")
    p.dim = dim
    for i in range(dim):
        p.n[i] = int(n[i])
        p.delta[i] = float(delta[i])
        p.kplus[i] = float(kplus[i])
        p.kminus[i] = float(kminus[i])
        if domain is not None:
            p.a[i], p.b[i] = float(domain[i][0]), float(domain[i][1])
    p.M = int(M)
    p.T = float(T)
    p.solver = {"auto": nat.SOLVER_AUTO, "pcg": nat.SOLVER_PCG, "gmres": nat.SOLVER_PGMRES,
                "pgmres": nat.SOLVER_PGMRES, "gmres2": nat.SOLVER_PGMRES2}[solver]
    p.restart = int(restart)
    p.tol = float(tol)
    p.maxit = int(maxit)
    p.precision = {"fp64": nat.PREC_FP64, "mixed": nat.PREC_MIXED}[precision]
    p.inner_tol = float(inner_tol)
    p.max_outer = int(max_outer)
    p.x0_mode = {"prev": nat.X0_PREV, "zero": nat.X0_ZERO, "external": nat.X0_EXTERNAL,
                 "extrap": nat.X0_EXTRAP, "guarded": nat.X0_GUARDED}[x0]
    p.allow_delta_zero = int(allow_delta_zero)
    p.dst_mfma = int(dst_mfma)
    p.reorth_eta2 = -1.0 if reorth_eta2 is None else float(reorth_eta2)
    p.precond = {"tau": nat.PC_TAU, "none": nat.PC_NONE, "tchan": nat.PC_TCHAN,
                 "strang": nat.PC_STRANG}[precond]
    return p


class Problem:
    """One CN-FV problem bound to a caller-owned device workspace."""

    def __init__(self, dim: int, n: Sequence[int], delta: Sequence[float],
                 kplus: Sequence[float], kminus: Sequence[float], M: int = 1, T: float = 1.0,
                 solver: str = "auto", restart: int = 20, tol: float = 1e-9, maxit: int = 0,
                 precision: str = "fp64", inner_tol: float = 1e-5, max_outer: int = 8,
                 x0: str = "prev", domain=None, allow_delta_zero: bool = False,
                 dst_mfma: bool = False, reorth_eta2: Optional[float] = None,
                 device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None, precond: str = "tau"):
        p = make_params(dim, n, delta, kplus, kminus, M, T, solver, restart, tol, maxit, precision,
                        inner_tol, max_outer, x0, domain, allow_delta_zero, dst_mfma, reorth_eta2,
                        precond)
        self.params = p
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        h = C.c_void_p()
        check(lib.fsd_init_problem(C.byref(p), C.byref(h)), "fsd_init_problem")
        self._h = h
        self.device = torch.device(device or "cuda")
        nbytes = int(lib.fsd_workspace_bytes(h))
        # 256-byte alignment: over-allocate and offset
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        self.stream = stream or torch.cuda.current_stream(self.device)
        check(lib.fsd_bind(h, C.c_void_p(base + off), nbytes, C.c_void_p(self.stream.cuda_stream)),
              "fsd_bind")
        self.workspace_bytes = nbytes

    @property
    def shape(self):
        return tuple(reversed(self.n))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.fsd_destroy(h)
            self._h = None

    def _out(self, out):
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        return out

    def apply_A(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self._out(out)
        check(lib.fsd_apply_A(self._h, _ptr(x), _ptr(out)), "fsd_apply_A")
        return out

    def apply_rhs(self, u: torch.Tensor, F: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self._out(out)
        check(lib.fsd_apply_rhs(self._h, _ptr(u), _ptr(F), _ptr(out)), "fsd_apply_rhs")
        return out

    def apply_Pinv(self, r: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self._out(out)
        check(lib.fsd_apply_Pinv(self._h, _ptr(r), _ptr(out)), "fsd_apply_Pinv")
        return out

    def apply_A32(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The float32 matvec of the mixed-precision inner solve."""
        out = self._out(out)
        check(lib.fsd_apply_A32(self._h, _ptr(x), _ptr(out)), "fsd_apply_A32")
        return out

    def apply_Pinv32(self, r: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The float32 preconditioner of the mixed-precision inner solve."""
        out = self._out(out)
        check(lib.fsd_apply_Pinv32(self._h, _ptr(r), _ptr(out)), "fsd_apply_Pinv32")
        return out

    def solve(self, b: torch.Tensor, x: torch.Tensor, raise_on_error: bool = True):
        st = nat.Stats()
        s = lib.fsd_solve(self._h, _ptr(b), _ptr(x), C.byref(st))
        if raise_on_error:
            check(s, "fsd_solve")
        return x, st.as_dict()

    def cn_step(self, u_prev: torch.Tensor, F: Optional[torch.Tensor] = None,
                guess: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                stats: bool = True, raise_on_error: bool = True):
        out = self._out(out)
        st = nat.Stats()
        s = lib.fsd_cn_step(self._h, _ptr(u_prev), _ptr(F), _ptr(guess), _ptr(out),
                            C.byref(st) if stats else None)
        if raise_on_error:
            check(s, "fsd_cn_step")
        return out, (st.as_dict() if stats else None)

    def set_engine(self, pass_name: str, engine: str, precision: str = "fp64"):
        """Engine of one line pass (fsd_set_engine): pass_name in
        nat.PASSES, engine in nat.ENGINES, precision "fp64" (float64
        passes) or "mixed" (float32 passes)."""
        prec = nat.PREC_MIXED if precision == "mixed" else nat.PREC_FP64
        check(lib.fsd_set_engine(self._h, prec, nat.PASSES[pass_name], nat.ENGINES[engine]),
              "fsd_set_engine")

    def autotune(self) -> str:
        """Time every engine of every pass and keep the fastest (the
        built-in one unless another is more than 5% faster)
        (fsd_autotune); returns the chosen engines."""
        check(lib.fsd_autotune(self._h), "fsd_autotune")
        return self.engines()

    def engines(self) -> str:
        n = lib.fsd_engines(self._h, None, 0)
        buf = C.create_string_buffer(n + 1)
        lib.fsd_engines(self._h, buf, n + 1)
        return buf.value.decode()

    def set_graphs(self, on: bool = True):
        """Replay captured launch graphs of the Krylov iteration chunks
        (fsd_set_graphs)."""
        check(lib.fsd_set_graphs(self._h, int(on)), "fsd_set_graphs")

    def reset_history(self):
        """Forget the time history used by x0="extrap"."""
        check(lib.fsd_reset_history(self._h), "fsd_reset_history")

    def profile(self, on: bool = True):
        """Record hipEvents around every heavy kernel launch (see
        fsd_profile_enable)."""
        check(lib.fsd_profile_enable(self._h, int(on)), "fsd_profile_enable")

    def profile_read(self):
        """Per-kernel-kind totals since the last read: name -> dict(launches,
        total_ms, bytes, avg_ms, gbps)."""
        buf = (nat.ProfileEntry * 64)()
        k = lib.fsd_profile_read(self._h, buf, 64)
        if k < 0:
            raise nat.FsdError(nat.EHIP, "fsd_profile_read")
        out = {}
        for e in buf[:k]:
            avg = e.total_ms / max(e.launches, 1)
            out[e.name.decode()] = dict(launches=e.launches, total_ms=e.total_ms, bytes=e.bytes,
                                        avg_ms=avg,
                                        gbps=(e.bytes / max(e.launches, 1)) / (avg * 1e-3) / 1e9
                                        if avg > 0 else 0.0)
        return out

    def coefficients(self, axis: int):
        n = self.n[axis]
        q = (C.c_double * (n + 1))()
        lam = (C.c_double * n)()
        eta = C.c_double()
        check(lib.fsd_get_coefficients(self._h, axis, q, lam, C.byref(eta)), "fsd_get_coefficients")
        return list(q), list(lam), eta.value


def hbm_copy(src: torch.Tensor, dst: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    """fsd_hbm_copy: streaming copy of src into dst (contiguous CUDA tensors
    of the same byte size, a multiple of 16) on `stream` (default: the
    current stream)."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("expected contiguous CUDA tensors")
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("source and destination sizes differ")
    st = stream or torch.cuda.current_stream(src.device)
    check(lib.fsd_hbm_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                           C.c_void_p(st.cuda_stream)), "fsd_hbm_copy")
    return dst
