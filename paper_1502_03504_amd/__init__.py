"""MI355X-native LOPe stencil sweeps: Python binding of liblope.so.

The functions below keep the names of the C ABI (include/lope.h) and only
marshal arguments: every step of the computation runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  Importing
this package fails loudly if the library has not been built.

Arrays use numpy/torch axis order: a 3D interior has shape (nz, ny, nx), so
the paper's first index x (left/right, contiguous in memory) is the last
tensor axis.  Boundary kinds are given per paper axis, x first.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import _lib
from ._lib import LopeError, check, load

__all__ = [
    "Grid", "LopeError", "lope_get_device", "lope_halo_fill", "lope_apply", "lope_iterate",
    "lope_iterate_tuned", "lope_iterate_until", "lope_apply_stages", "lope_iterate_stages", "lope_apply_adjoint",
    "gbar_buffer", "LOPE_GBAR_DOUBLES", "lope_apply_var", "lope_apply_var_adjoint",
    "lope_accumulate", "lope_variant_count", "lope_variant_info", "lope_select_variant",
    "lope_tune_set", "variants", "BatchPlan", "lope_batch_plan_create", "lope_batch_apply",
    "lope_batch_apply_per_grid", "lope_batch_apply_passes", "lope_batch_persistent_check",
    "lope_batch_plan_destroy", "lope_batch_tune_set", "lope_batch_apply_noalloc", "lope_copy_stream", "DIRICHLET", "PERIODIC",
]

DIRICHLET = "dirichlet"
PERIODIC = "periodic"

_ALIGN_BYTES = 128


def _register_default_tuning():
    if os.environ.get("LOPE_NO_TUNE_CACHE") == "1":
        return
    from .tune import register_cache
    register_cache()


_lib._ON_LOAD.append(_register_default_tuning)


def library_path() -> str:
    """Load the HIP library (raises ImportError if it is not built) and return its path."""
    load()
    return _lib.LIB_PATH


def _dtype_code(dtype) -> int:
    if dtype == torch.float32:
        return _lib.LOPE_F32
    if dtype == torch.float64:
        return _lib.LOPE_F64
    raise TypeError("grids hold float32 or float64, not %s" % dtype)


def _align(v: int, a: int) -> int:
    return (v + a - 1) // a * a


def _halo_pairs(h, ndim: int):
    """Per paper axis (x first) the (left, right) halo widths: h is one width
    for both sides of every axis, or a sequence of (lo, hi) pairs (the M:*:N
    halo of section 2.2, per dimension)."""
    if np.ndim(h) == 0:
        return [(int(h), int(h))] * ndim
    w = [(int(lo), int(hi)) for lo, hi in h]
    if len(w) != ndim or min(min(p) for p in w) < 0:
        raise ValueError("one (lo, hi) pair of non-negative halo widths per axis")
    return w


class Grid:
    """A padded grid in device memory: interior plus halo cells on each side.

    ``h`` is one halo width for both sides of every axis, or a sequence of
    (lo, hi) widths per paper axis, x first (left/right, below/above, ...).
    Storage layout (the padded allocation of section 3.2, x contiguous): each
    row starts ``lead`` elements before interior x = 0 (lead >= the left x
    halo, rounded so the interior row start is 128-byte aligned), rows are
    ``sy`` elements apart (a multiple of 128 bytes) and planes ``sz`` apart.
    """

    def __init__(self, storage: torch.Tensor, shape, h, lead: int, sy: int, sz: int):
        self.storage = storage
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        d = self.ndim
        self.halo = _halo_pairs(h, d)                       # per paper axis, x first
        self.symmetric = np.ndim(h) == 0
        self.h = int(h) if self.symmetric else max(max(p) for p in self.halo)
        self.lead = int(lead)
        self.sy = int(sy)
        self.sz = int(sz)
        lo = [p[0] for p in self.halo] + [0] * (3 - d)
        hi = [p[1] for p in self.halo] + [0] * (3 - d)
        self.offset = self.lead + (lo[1] * self.sy if d >= 2 else 0) + (lo[2] * self.sz if d >= 3 else 0)
        if storage.dim() != 1:
            raise ValueError("storage must be a flat tensor")
        nx = self.shape[-1]
        if self.lead < lo[0] or (d >= 2 and self.sy < self.lead + nx + hi[0]) or \
                (d >= 3 and self.sz < self.sy * (self.shape[-2] + lo[1] + hi[1])):
            raise ValueError("strides do not hold the padded rows/planes")
        last = self.offset + nx - 1 + hi[0]
        if d >= 2:
            last += (self.shape[-2] - 1 + hi[1]) * self.sy
        if d >= 3:
            last += (self.shape[-3] - 1 + hi[2]) * self.sz
        first = self.offset - lo[0] - (lo[1] * self.sy if d >= 2 else 0) - (lo[2] * self.sz if d >= 3 else 0)
        if min(self.shape) > 0 and (first < 0 or last >= storage.numel()):
            raise ValueError("storage of %d elements does not hold the padded box" % storage.numel())

    # ---- construction ----
    @classmethod
    def allocate(cls, shape, h, dtype=torch.float32, device="cuda", halo_src=None, fill=0.0):
        """New padded grid (h: one width, or (lo, hi) per paper axis); with
        ``halo_src`` (a tensor or Grid) its interior is copied in, like
        allocating with HALO_SRC in section 3.2."""
        shape = tuple(int(s) for s in shape)
        if not 1 <= len(shape) <= 3:
            raise ValueError("1..3 dimensions")
        d = len(shape)
        w = _halo_pairs(h, d) + [(0, 0)] * (3 - d)
        esize = torch.empty((), dtype=dtype).element_size()
        a = _ALIGN_BYTES // esize
        nx = shape[-1]
        lead = _align(w[0][0], a) if w[0][0] > 0 else 0
        sy = _align(lead + nx + w[0][1], a)
        ny = shape[-2] if d >= 2 else 1
        nz = shape[-3] if d >= 3 else 1
        rows = (ny + w[1][0] + w[1][1]) if d >= 2 else 1
        sz = sy * rows
        planes = (nz + w[2][0] + w[2][1]) if d >= 3 else 1
        storage = torch.full((sz * planes,), float(fill), dtype=dtype, device=device)
        g = cls(storage, shape, h, lead, sy, sz)
        if halo_src is not None:
            src = halo_src.interior() if isinstance(halo_src, Grid) else halo_src
            g.interior().copy_(torch.as_tensor(src).to(device=device, dtype=dtype))
        return g

    @classmethod
    def from_array(cls, arr, h, device="cuda", dtype=None):
        arr = np.asarray(arr)
        tdt = dtype or (torch.float64 if arr.dtype == np.float64 else torch.float32)
        return cls.allocate(arr.shape, h, tdt, device, halo_src=torch.from_numpy(np.ascontiguousarray(arr)))

    def empty_like(self, h=None):
        if h is None:
            h = self.h if self.symmetric else self.halo
        return Grid.allocate(self.shape, h, self.dtype, self.storage.device)

    # ---- views ----
    @property
    def dtype(self):
        return self.storage.dtype

    def _strides(self):
        return {1: (1,), 2: (self.sy, 1), 3: (self.sz, self.sy, 1)}[self.ndim]

    def interior(self) -> torch.Tensor:
        # as_strided offsets count from the start of the underlying storage
        return self.storage.as_strided(self.shape, self._strides(), self.storage.storage_offset() + self.offset)

    def padded(self) -> torch.Tensor:
        d = self.ndim
        # numpy axis npax is paper axis d-1-npax
        shp = tuple(self.shape[npax] + sum(self.halo[d - 1 - npax]) for npax in range(d))
        lo = [p[0] for p in self.halo] + [0] * (3 - d)
        off = self.offset - lo[0] - (lo[1] * self.sy if d >= 2 else 0) - (lo[2] * self.sz if d >= 3 else 0)
        return self.storage.as_strided(shp, self._strides(), self.storage.storage_offset() + off)

    def numpy(self) -> np.ndarray:
        return self.interior().detach().cpu().numpy().copy()

    def descriptor(self) -> _lib.lope_grid:
        g = _lib.lope_grid()
        g.ndim = self.ndim
        g.h = self.h
        g.dtype = _dtype_code(self.dtype)
        if not self.symmetric:
            g.halo_mode = 1
            for a in range(self.ndim):
                g.hlo[a], g.hhi[a] = self.halo[a]
        n = list(reversed(self.shape)) + [1] * (3 - self.ndim)
        for a in range(3):
            g.n[a] = n[a]
        g.stride[0] = 1
        g.stride[1] = self.sy if self.ndim >= 2 else 0
        g.stride[2] = self.sz if self.ndim >= 3 else 0
        g.origin = self.storage.data_ptr() + self.offset * self.storage.element_size()
        return g


# ---- argument marshalling ----
def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _bc(bc, ndim: int) -> _lib.lope_bc:
    """bc: an object with .kinds/.value, a (kinds, value) pair or a kinds tuple."""
    if hasattr(bc, "kinds"):
        kinds, value = bc.kinds, bc.value
    elif isinstance(bc, (tuple, list)) and len(bc) == 2 and not isinstance(bc[0], str):
        kinds, value = bc
    else:
        kinds, value = bc, 0.0
    out = _lib.lope_bc()
    for a in range(3):
        k = kinds[a] if a < len(kinds) else PERIODIC
        if isinstance(k, str):
            k = {DIRICHLET: _lib.LOPE_BC_DIRICHLET, PERIODIC: _lib.LOPE_BC_PERIODIC}[k]
        out.kind[a] = int(k)
    out.value = float(value)
    return out


class _Stencil:
    """Keeps the host coefficient table alive for the duration of a call."""

    def __init__(self, st):
        coeffs = st.coeffs if hasattr(st, "coeffs") else st
        self.arr = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        r = (self.arr.shape[0] - 1) // 2 if self.arr.ndim else 0
        self.c = _lib.lope_stencil()
        self.c.ndim = int(getattr(st, "ndim", self.arr.ndim))
        self.c.radius = int(getattr(st, "radius", r))
        self.c.coeffs = self.arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ref(x):
    return ctypes.byref(x)


# ---- the C ABI, by name ----
def lope_get_device(ordinal: int = 0) -> int:
    out = ctypes.c_int(-2)
    check(load().lope_get_device(int(ordinal), _ref(out)))
    return out.value


def lope_halo_fill(grid: Grid, bc, stream=None) -> None:
    g = grid.descriptor()
    check(load().lope_halo_fill(_ref(g), _ref(_bc(bc, grid.ndim)), _stream(stream)))


def lope_apply(src: Grid, dst: Grid, stencil, bc, stream=None) -> None:
    s = _Stencil(stencil)
    a, b = src.descriptor(), dst.descriptor()
    check(load().lope_apply(_ref(a), _ref(b), _ref(s.c), _ref(_bc(bc, src.ndim)), _stream(stream)))


def lope_iterate(a: Grid, b: Grid, stencil, bc, n_steps: int, tdepth: int = 0, stream=None) -> int:
    """Returns 0 if the final state is in ``a``, 1 if in ``b``."""
    s = _Stencil(stencil)
    ga, gb = a.descriptor(), b.descriptor()
    idx = ctypes.c_int32(-1)
    check(load().lope_iterate(_ref(ga), _ref(gb), _ref(s.c), _ref(_bc(bc, a.ndim)), int(n_steps), int(tdepth),
                              _stream(stream), _ref(idx)))
    return idx.value


def lope_iterate_tuned(a: Grid, b: Grid, stencil, bc, n_steps: int, variant: int = 0, tdepth: int = 0,
                       chunk: int = 0, stream=None) -> int:
    s = _Stencil(stencil)
    ga, gb = a.descriptor(), b.descriptor()
    t = _lib.lope_tuning(int(variant), int(tdepth), int(chunk), 0)
    idx = ctypes.c_int32(-1)
    check(load().lope_iterate_tuned(_ref(ga), _ref(gb), _ref(s.c), _ref(_bc(bc, a.ndim)), int(n_steps), _ref(t),
                                    _stream(stream), _ref(idx)))
    return idx.value


def lope_iterate_until(a: Grid, b: Grid, stencil, bc, max_steps: int, check_every: int, tol: float,
                       tdepth: int = 0, scratch: torch.Tensor = None, stream=None):
    """Sweeps until the max-norm change of a checked sweep is <= tol (checked
    every ``check_every`` sweeps) or ``max_steps`` sweeps ran.  Waits on the
    stream after each check.  Returns (result_index, steps_done, residual);
    ``scratch`` is an optional float64 device tensor of >= 1 element."""
    st = _Stencil(stencil)
    ga, gb = a.descriptor(), b.descriptor()
    if scratch is None:
        scratch = torch.empty(1, dtype=torch.float64, device=a.storage.device)
    if scratch.dtype != torch.float64 or scratch.numel() < 1 or not scratch.is_cuda:
        raise TypeError("scratch must be a float64 device tensor")
    steps = ctypes.c_int64(-1)
    res = ctypes.c_double(0.0)
    idx = ctypes.c_int32(-1)
    check(load().lope_iterate_until(_ref(ga), _ref(gb), _ref(st.c), _ref(_bc(bc, a.ndim)), int(max_steps),
                                    int(check_every), float(tol), int(tdepth), ctypes.c_void_p(scratch.data_ptr()),
                                    _stream(stream), _ref(steps), _ref(res), _ref(idx)))
    return idx.value, steps.value, res.value


def _stages(first, second, alpha):
    s1, s2 = _Stencil(first), _Stencil(second)
    sg = _lib.lope_stages(ctypes.pointer(s1.c), ctypes.pointer(s2.c), float(alpha))
    return sg, (s1, s2)


def lope_apply_stages(src: Grid, dst: Grid, first, second, alpha: float, bc, stream=None) -> None:
    """One two-stage step: dst = alpha*src + S2(B(S1(B(src))))."""
    sg, keep = _stages(first, second, alpha)
    check(load().lope_apply_stages(_ref(src.descriptor()), _ref(dst.descriptor()), _ref(sg),
                                   _ref(_bc(bc, src.ndim)), _stream(stream)))


def lope_iterate_stages(a: Grid, b: Grid, first, second, alpha: float, bc, n_steps: int, stream=None) -> int:
    """n_steps two-stage steps alternating between a and b; returns 0 if the
    final state is in a, 1 if in b."""
    sg, keep = _stages(first, second, alpha)
    idx = ctypes.c_int32(-1)
    check(load().lope_iterate_stages(_ref(a.descriptor()), _ref(b.descriptor()), _ref(sg), _ref(_bc(bc, a.ndim)),
                                     int(n_steps), _stream(stream), _ref(idx)))
    return idx.value


LOPE_GBAR_DOUBLES = 1024   # doubles of the array lope_apply_adjoint's gbar points to


def lope_copy_stream(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst <- src (contiguous device tensors of equal byte size, a multiple of
    16 bytes) with the library's streaming copy kernel."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_contiguous() and dst.is_contiguous()) or dst.numel() * dst.element_size() != nbytes:
        raise ValueError("contiguous tensors of equal byte size")
    check(load().lope_copy_stream(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                  _stream(stream)))


def gbar_buffer(device="cuda", fill=0.0) -> torch.Tensor:
    """A float64 device array for lope_apply_adjoint's gbar (element 0 gets
    dL/dg; the rest is the call's workspace)."""
    return torch.full((LOPE_GBAR_DOUBLES,), float(fill), dtype=torch.float64, device=device)


def lope_apply_adjoint(ybar: Grid, xbar: Grid, stencil, bc, gbar: torch.Tensor = None, stream=None) -> None:
    """xbar = S^T ybar; if ``gbar`` (a float64 device tensor of at least
    LOPE_GBAR_DOUBLES elements, see gbar_buffer) is given, gbar[0] receives
    dL/dg and the other elements are overwritten."""
    s = _Stencil(stencil)
    a, b = ybar.descriptor(), xbar.descriptor()
    gp = None
    if gbar is not None:
        if gbar.dtype != torch.float64 or gbar.numel() < LOPE_GBAR_DOUBLES or not gbar.is_cuda \
                or not gbar.is_contiguous():
            raise TypeError("gbar must be a contiguous float64 device tensor of %d elements" % LOPE_GBAR_DOUBLES)
        gp = ctypes.c_void_p(gbar.data_ptr())
    check(load().lope_apply_adjoint(_ref(a), _ref(b), _ref(s.c), _ref(_bc(bc, ybar.ndim)), gp, _stream(stream)))


def _varcoef(kappa: Grid, dt: float):
    kd = kappa.descriptor()
    vc = _lib.lope_varcoef(ctypes.pointer(kd), float(dt))
    return kd, vc


def lope_apply_var(src: Grid, dst: Grid, kappa: Grid, dt: float, bc, stream=None) -> None:
    kd, vc = _varcoef(kappa, dt)
    a, b = src.descriptor(), dst.descriptor()
    check(load().lope_apply_var(_ref(a), _ref(b), _ref(vc), _ref(_bc(bc, src.ndim)), _stream(stream)))


def lope_apply_var_adjoint(lam_next: Grid, lam: Grid, u_t: Grid, kappa: Grid, dt: float, bc, gkappa: Grid,
                           stream=None) -> None:
    kd, vc = _varcoef(kappa, dt)
    a, b, u, g = lam_next.descriptor(), lam.descriptor(), u_t.descriptor(), gkappa.descriptor()
    check(load().lope_apply_var_adjoint(_ref(a), _ref(b), _ref(u), _ref(vc), _ref(_bc(bc, 3)), _ref(g),
                                        _stream(stream)))


def lope_apply_var_adjoint2(lam_next: Grid, lam: Grid, u_t: Grid, u_tm1: Grid, kappa: Grid, dt: float, bc,
                            gkappa: Grid, stream=None) -> None:
    """Two reverse steps in one pass: lam = dL/du_{t-1} from lam_next = dL/du_{t+1}."""
    kd, vc = _varcoef(kappa, dt)
    a, b, u, v, g = (lam_next.descriptor(), lam.descriptor(), u_t.descriptor(), u_tm1.descriptor(),
                     gkappa.descriptor())
    check(load().lope_apply_var_adjoint2(_ref(a), _ref(b), _ref(u), _ref(v), _ref(vc), _ref(_bc(bc, 3)), _ref(g),
                                         _stream(stream)))


def lope_accumulate(partial: Grid, total: Grid, stream=None) -> None:
    a, b = partial.descriptor(), total.descriptor()
    check(load().lope_accumulate(_ref(a), _ref(b), _stream(stream)))


def lope_variant_count() -> int:
    return load().lope_variant_count()


def lope_variant_info(vid: int) -> str:
    buf = ctypes.create_string_buffer(256)
    check(load().lope_variant_info(int(vid), buf, 256))
    return buf.value.decode()


def variants():
    return [lope_variant_info(i) for i in range(1, lope_variant_count() + 1)]


def lope_select_variant(grid: Grid, stencil, tdepth: int = 0, bc=None) -> int:
    """The variant lope_iterate would use (bc None: periodic on every axis)."""
    s = _Stencil(stencil)
    g = grid.descriptor()
    b = _bc(bc, grid.ndim) if bc is not None else None
    return check(load().lope_select_variant(_ref(g), _ref(s.c), _ref(b) if b is not None else None, int(tdepth)))


def rule_class(bc, ndim: int) -> int:
    """The tuning table's boundary-rule class: 1 if some axis is Dirichlet."""
    b = _bc(bc, ndim)
    return int(any(b.kind[a] == _lib.LOPE_BC_DIRICHLET for a in range(ndim)))


def lope_tune_set(grid: Grid, stencil, variant: int, tdepth: int = 0, chunk: int = 0, bc=None) -> None:
    """Register a choice for grids, stencils and rules like these (bc None:
    periodic on every axis); variant 0 removes it."""
    s = _Stencil(stencil)
    g = grid.descriptor()
    rules = rule_class(bc, grid.ndim) if bc is not None else 0
    t = _lib.lope_tuning(int(variant), int(tdepth), int(chunk), rules)
    check(load().lope_tune_set(_ref(g), _ref(s.c), _ref(t)))


from .batch import (  # noqa: E402,F401
    BatchPlan, lope_batch_plan_create, lope_batch_apply, lope_batch_apply_per_grid, lope_batch_apply_passes,
    lope_batch_persistent_check, lope_batch_plan_destroy, lope_batch_tune_set, lope_batch_apply_noalloc,
)
