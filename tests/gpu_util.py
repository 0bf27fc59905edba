"""Helpers shared by the GPU tests (tolerances and grid construction)."""
import numpy as np
import torch

import paper_1502_03504_amd as L

# Normwise relative tolerance: max|gpu - oracle| / max|oracle| over the interior.
TOL = {np.float64: 1e-12, np.float32: 1e-5}


def tol(dtype):
    return TOL[np.dtype(dtype).type]


def rel_err(got: np.ndarray, want: np.ndarray) -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if want.size == 0:
        return 0.0
    scale = np.max(np.abs(want))
    diff = np.max(np.abs(got - want))
    return float(diff / scale) if scale > 0 else float(diff)


def grid_from(arr: np.ndarray, h: int, fill=0.0) -> L.Grid:
    tdt = torch.float64 if arr.dtype == np.float64 else torch.float32
    g = L.Grid.allocate(arr.shape, h, tdt, "cuda", fill=fill)
    g.interior().copy_(torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    return g


def packed_grid_from(arr: np.ndarray, h: int) -> L.Grid:
    """A grid with tightly packed padded rows (lead = h, row pitch nx + 2h):
    origins and strides are generally not 16-byte multiples, which forces the
    scalar kernels."""
    tdt = torch.float64 if arr.dtype == np.float64 else torch.float32
    shape = arr.shape
    d = len(shape)
    nx = shape[-1]
    sy = nx + 2 * h
    rows = shape[-2] + 2 * h if d >= 2 else 1
    sz = sy * rows
    planes = shape[-3] + 2 * h if d >= 3 else 1
    storage = torch.zeros(sz * planes + 1, dtype=tdt, device="cuda")[1:]     # shift by one element
    g = L.Grid(storage, shape, h, h, sy, sz)
    g.interior().copy_(torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    return g


def empty_grid(shape, h: int, dtype, fill=0.0) -> L.Grid:
    tdt = torch.float64 if np.dtype(dtype) == np.float64 else torch.float32
    return L.Grid.allocate(shape, h, tdt, "cuda", fill=fill)


def halo_mask(g: L.Grid) -> np.ndarray:
    """Boolean mask over the padded box, True on halo cells."""
    shp = tuple(s + 2 * g.h for s in g.shape)
    m = np.ones(shp, dtype=bool)
    m[tuple(slice(g.h, g.h + s) for s in g.shape)] = False
    return m


def variants_for(ndim, radius, dtype, shape=None, tdepth=None):
    """Ids and descriptions of compiled variants matching the filters."""
    out = []
    dt = "f64" if np.dtype(dtype) == np.float64 else "f32"
    for vid, info in enumerate(L.variants(), start=1):
        f = dict(kv.split("=") for kv in info.split()[1:])
        if int(f["ndim"]) != ndim or int(f["radius"]) != radius or f["dtype"] != dt:
            continue
        if shape is not None and f["shape"] != shape:
            continue
        if tdepth is not None and int(f["tdepth"]) != tdepth:
            continue
        out.append((vid, info))
    return out
