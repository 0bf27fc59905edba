"""Batch plans: many uneven 2D grids swept in one persistent launch."""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import check, load


class BatchPlan:
    """Owns a lope_batch_plan and keeps the grids it borrows alive.

    ``entries`` is a sequence of (src Grid, dst Grid, stencil, bc).  After
    ``apply`` each grid has advanced ``n_steps`` sweeps; its state is in src
    when n_steps is even, else in dst.
    """

    def __init__(self, entries, n_steps: int, stream=None):
        from . import _Stencil, _bc, _stream
        self.entries = list(entries)
        self.n_steps = int(n_steps)
        self._stencils = [_Stencil(e[2]) for e in self.entries]
        arr = (_lib.lope_batch_item * max(1, len(self.entries)))()
        for i, (src, dst, _, bc) in enumerate(self.entries):
            arr[i].src = src.descriptor()
            arr[i].dst = dst.descriptor()
            arr[i].stencil = self._stencils[i].c
            arr[i].bc = _bc(bc, 2)
        self._items = arr
        self._stream = _stream
        out = ctypes.c_void_p()
        check(load().lope_batch_plan_create(arr, len(self.entries), self.n_steps, _stream(stream), ctypes.byref(out)))
        self.handle = out

    def apply(self, stream=None) -> None:
        check(load().lope_batch_apply(self.handle, self._stream(stream)))

    def apply_per_grid(self, stream=None) -> None:
        check(load().lope_batch_apply_per_grid(self.handle, self._stream(stream)))

    def error(self, stream=None) -> int:
        v = ctypes.c_int(-1)
        check(load().lope_batch_plan_error(self.handle, self._stream(stream), ctypes.byref(v)))
        return v.value

    def result(self, i: int):
        src, dst = self.entries[i][0], self.entries[i][1]
        return src if self.n_steps % 2 == 0 else dst

    def close(self) -> None:
        if self.handle is not None and self.handle.value:
            load().lope_batch_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lope_batch_plan_create(entries, n_steps: int, stream=None) -> BatchPlan:
    return BatchPlan(entries, n_steps, stream)


def lope_batch_apply(plan: BatchPlan, stream=None) -> None:
    plan.apply(stream)


def lope_batch_apply_per_grid(plan: BatchPlan, stream=None) -> None:
    plan.apply_per_grid(stream)


def lope_batch_plan_destroy(plan: BatchPlan) -> None:
    plan.close()
