"""Thin Python front end of include/fsd_batch.h: many independent CN
problems advanced together by the library's native executor.

    b = Batch([dict(dim=2, n=(255, 127), delta=..., kplus=..., kminus=..., M=8, T=1.0,
                    solver="pcg", precision="mixed", tol=1e-8), ...], streams=8)
    outs, stats = b.cn_step(us, Fs)
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import torch

from . import _native as nat
from ._native import check, lib
from .solver import make_params


def _ptrs(ts: Optional[Sequence[Optional[torch.Tensor]]], count: int):
    if ts is None:
        return None
    if len(ts) != count:
        raise ValueError(f"expected {count} tensors")
    arr = (C.c_void_p * count)()
    for i, t in enumerate(ts):
        if t is None:
            arr[i] = None
            continue
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("expected contiguous float64 CUDA tensors")
        arr[i] = t.data_ptr()
    return arr


class Batch:
    def __init__(self, problems: Sequence[dict], streams: int = 8, device=None):
        self.count = len(problems)
        params = (nat.Params * self.count)()
        for i, kw in enumerate(problems):
            params[i] = make_params(**kw)
        self.shapes = [tuple(reversed([int(v) for v in kw["n"][:kw["dim"]]])) for kw in problems]
        h = C.c_void_p()
        check(lib.fsd_batch_create(params, self.count, C.byref(h)), "fsd_batch_create")
        self._h = h
        self.device = torch.device(device or "cuda")
        nbytes = int(lib.fsd_batch_workspace_bytes(h))
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        # default-priority streams, one per executor lane
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        sarr = (C.c_void_p * streams)(*[s.cuda_stream for s in self.streams])
        torch.cuda.synchronize(self.device)
        check(lib.fsd_batch_bind(h, C.c_void_p(base + off), nbytes, sarr, streams), "fsd_batch_bind")
        self.workspace_bytes = nbytes

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.fsd_batch_destroy(h)
            self._h = None

    @property
    def lanes(self) -> int:
        return int(lib.fsd_batch_lanes(self._h))

    def set_lanes(self, lanes: int):
        check(lib.fsd_batch_set_lanes(self._h, int(lanes)), "fsd_batch_set_lanes")

    @property
    def graphs(self) -> bool:
        return bool(lib.fsd_batch_graphs(self._h))

    def set_graphs(self, on: bool):
        """Launch graphs of the Krylov iteration chunks for every problem."""
        check(lib.fsd_batch_set_graphs(self._h, int(on)), "fsd_batch_set_graphs")

    def engines(self, i: int) -> str:
        """Problem i's pass engines (fsd_engines)."""
        h = lib.fsd_batch_problem(self._h, int(i))
        n = lib.fsd_engines(h, None, 0)
        buf = C.create_string_buffer(n + 1)
        lib.fsd_engines(h, buf, n + 1)
        return buf.value.decode()

    def empty(self) -> List[torch.Tensor]:
        return [torch.empty(s, dtype=torch.float64, device=self.device) for s in self.shapes]

    def cn_step(self, u_prev, F=None, guess=None, out=None, raise_on_error=True):
        """One step of every problem.  The caller's pending work on the
        current stream is finished first (inputs are ready); outputs are
        complete on return."""
        out = out if out is not None else self.empty()
        st = (nat.Stats * self.count)()
        torch.cuda.current_stream(self.device).synchronize()
        s = lib.fsd_batch_cn_step(self._h, _ptrs(u_prev, self.count), _ptrs(F, self.count),
                                  _ptrs(guess, self.count), _ptrs(out, self.count), st)
        if raise_on_error:
            check(s, "fsd_batch_cn_step")
        return out, [x.as_dict() for x in st]

    def autotune(self, u_prev, F=None):
        """Time one step per lane count 1, 2, 4, ... with direct launches
        and with launch graphs, and keep the fastest; returns (lanes,
        {(lanes, graphs): ms}); the chosen launch mode is `graphs`."""
        out = self.empty()
        ms = (C.c_double * 32)()
        torch.cuda.current_stream(self.device).synchronize()
        r = lib.fsd_batch_autotune(self._h, _ptrs(u_prev, self.count), _ptrs(F, self.count),
                                   _ptrs(out, self.count), ms)
        if r < 0:
            raise nat.FsdError(-r, "fsd_batch_autotune")
        cands = {}
        k = 0
        for g in (False, True):
            l = 1
            while l <= min(len(self.streams), self.count):
                cands[(l, g)] = ms[k]
                l *= 2
                k += 1
        return r, cands
