"""Batch plans: many uneven 2D grids swept together, every pass in one
persistent launch (or one launch per fused pass)."""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import check, load


class BatchPlan:
    """Owns a lope_batch_plan and keeps the grids it borrows alive.

    ``entries`` is a sequence of (src Grid, dst Grid, stencil, bc).  Each
    ``apply`` advances every grid ``n_steps`` sweeps starting from its src in
    one persistent kernel launch; ``result(i)`` is the grid holding the
    outcome.  ``apply_passes`` does the same with one launch per fused pass
    (replayed from a recorded graph), and ``apply_per_grid`` with one launch
    per grid per sweep, leaving the outcome in src when n_steps is even, else
    in dst.
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

    def apply_passes(self, stream=None) -> None:
        """The sweeps of ``apply`` as one launch per fused pass (same result)."""
        check(load().lope_batch_apply_passes(self.handle, self._stream(stream)))

    def check_persistent(self) -> None:
        """Synchronise; raise if a wait of an earlier ``apply`` ran out."""
        check(load().lope_batch_persistent_check(self.handle))

    def set_depth(self, tdepth: int) -> None:
        """Sweeps fused per launch (1..8)."""
        check(load().lope_batch_plan_set_depth(self.handle, int(tdepth)))

    def set_tiles(self, tdepth: int, rows: int = 0) -> None:
        """Sweeps fused per launch (1..8) and rows per strip (0 keeps them)."""
        check(load().lope_batch_plan_set_tiles(self.handle, int(tdepth), int(rows)))

    def tiles(self):
        """(sweeps per launch, rows per strip) the plan runs with."""
        d, r = ctypes.c_int32(-1), ctypes.c_int32(-1)
        check(load().lope_batch_plan_get_tiles(self.handle, ctypes.byref(d), ctypes.byref(r)))
        return d.value, r.value

    def result_index(self) -> int:
        v = ctypes.c_int32(-1)
        check(load().lope_batch_result_index(self.handle, ctypes.byref(v)))
        return v.value

    def result(self, i: int):
        """The grid that holds entry i's state after apply() or apply_passes()."""
        return self.entries[i][1] if self.result_index() else self.entries[i][0]

    def per_grid_result(self, i: int):
        """The grid that holds entry i's state after apply_per_grid()."""
        return self.entries[i][1] if self.n_steps % 2 else self.entries[i][0]

    def close(self) -> None:
        if self.handle is not None and self.handle.value:
            load().lope_batch_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _item_array(entries):
    from . import _Stencil, _bc
    stencils = [_Stencil(e[2]) for e in entries]
    arr = (_lib.lope_batch_item * max(1, len(entries)))()
    for i, (src, dst, _, bc) in enumerate(entries):
        arr[i].src = src.descriptor()
        arr[i].dst = dst.descriptor()
        arr[i].stencil = stencils[i].c
        arr[i].bc = _bc(bc, 2)
    return arr, stencils


def lope_batch_apply_noalloc(entries, n_steps: int, tdepth: int = 0, rows: int = 0, stream=None) -> int:
    """Advance every (src, dst, stencil, bc) entry n_steps sweeps without a
    plan (no device allocation: the tables go to the library's static
    scratch); returns 0 if the states end in the src grids, 1 if in dst."""
    from . import _stream
    entries = list(entries)
    arr, stencils = _item_array(entries)
    idx = ctypes.c_int32(-1)
    check(load().lope_batch_apply_noalloc(arr, len(entries), int(n_steps), int(tdepth), int(rows), _stream(stream),
                                          ctypes.byref(idx)))
    return idx.value


def lope_batch_plan_create(entries, n_steps: int, stream=None) -> BatchPlan:
    return BatchPlan(entries, n_steps, stream)


def lope_batch_apply(plan: BatchPlan, stream=None) -> None:
    plan.apply(stream)


def lope_batch_apply_per_grid(plan: BatchPlan, stream=None) -> None:
    plan.apply_per_grid(stream)


def lope_batch_apply_passes(plan: BatchPlan, stream=None) -> None:
    plan.apply_passes(stream)


def lope_batch_persistent_check(plan: BatchPlan) -> None:
    plan.check_persistent()


def lope_batch_plan_destroy(plan: BatchPlan) -> None:
    plan.close()


def lope_batch_tune_set(dtype, points: int, tdepth: int, rows: int) -> None:
    """Register the tiling of batches of this dtype (torch dtype) and size
    bucket (tdepth 0 removes it)."""
    import torch
    code = _lib.LOPE_F64 if dtype == torch.float64 else _lib.LOPE_F32
    check(load().lope_batch_tune_set(code, int(points), int(tdepth), int(rows)))
