"""The C ABI without a GPU: the library loads, exports every declared symbol,
and structural validation returns the documented codes before any HIP call."""
import ctypes
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_1502_03504_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lope.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lope_\w+)\s*\(", text, flags=re.M)))


def test_header_functions_parsed():
    names = declared_functions()
    assert "lope_apply" in names and "lope_batch_apply" in names and len(names) >= 20


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_exported_symbols_with_nm():
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lope_\w+)", out))
    assert set(declared_functions()) <= exported


L = _lib.load()


def grid(n=(8, 8, 8), h=1, ndim=3, dtype=_lib.LOPE_F32, origin=0x100000, sy=None, sz=None):
    g = _lib.lope_grid()
    g.ndim = ndim
    g.h = h
    g.dtype = dtype
    nn = list(n)[:ndim] + [1] * (3 - ndim)
    for a in range(3):
        g.n[a] = nn[a]
    g.stride[0] = 1
    g.stride[1] = sy if sy is not None else nn[0] + 2 * h
    g.stride[2] = sz if sz is not None else g.stride[1] * (nn[1] + 2 * h)
    g.origin = origin
    return g


def bc(kind=_lib.LOPE_BC_PERIODIC, value=0.0):
    b = _lib.lope_bc()
    for a in range(3):
        b.kind[a] = kind
    b.value = value
    return b


def stencil(ndim=3, r=1, fill=0.1):
    arr = np.full((2 * r + 1) ** ndim, fill)
    s = _lib.lope_stencil()
    s.ndim = ndim
    s.radius = r
    s.coeffs = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return s, arr


def far():
    return 0x40000000


def apply(a, b, st, bcv):
    return L.lope_apply(ctypes.byref(a), ctypes.byref(b), ctypes.byref(st), ctypes.byref(bcv), None)


def test_get_device_falls_back_to_host():
    out = ctypes.c_int(7)
    assert L.lope_get_device(0, ctypes.byref(out)) == _lib.LOPE_OK
    assert out.value == _lib.LOPE_HOST
    assert L.lope_get_device(0, None) == _lib.LOPE_ERR_INVALID_ARG


def test_valid_call_without_device_reports_no_device():
    s, _keep = stencil()
    assert apply(grid(), grid(origin=far()), s, bc()) == _lib.LOPE_ERR_NO_DEVICE
    assert b"device" in L.lope_last_error()


def test_force_no_device_env():
    code = ("import ctypes,sys; sys.path.insert(0, %r); from paper_1502_03504_amd import _lib; L=_lib.load(); "
            "o=ctypes.c_int(5); L.lope_get_device(0, ctypes.byref(o)); print(o.value)" % ROOT)
    env = dict(os.environ, LOPE_FORCE_NO_DEVICE="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env)
    assert out.stdout.strip() == "-1"


def test_invalid_arguments():
    s, _keep = stencil()
    E = _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_apply(None, ctypes.byref(grid()), ctypes.byref(s), ctypes.byref(bc()), None) == E
    g = grid(ndim=3)
    g.ndim = 4
    assert apply(g, grid(origin=far()), s, bc()) == E
    g = grid()
    g.dtype = 7
    assert apply(g, grid(origin=far()), s, bc()) == E
    g = grid()
    g.stride[0] = 2
    assert apply(g, grid(origin=far()), s, bc()) == E
    assert apply(grid(sy=5), grid(origin=far()), s, bc()) == E            # rows overlap
    assert apply(grid(sz=10), grid(origin=far()), s, bc()) == E           # planes overlap
    assert apply(grid(origin=0), grid(origin=far()), s, bc()) == E        # null origin
    assert apply(grid(n=(8, 8, 9)), grid(origin=far()), s, bc()) == E     # extents differ
    assert apply(grid(dtype=_lib.LOPE_F64), grid(origin=far()), s, bc()) == E
    b = bc()
    b.kind[1] = 5
    assert apply(grid(), grid(origin=far()), s, b) == E
    s2, _k2 = stencil(ndim=2)
    assert apply(grid(), grid(origin=far()), s2, bc()) == E              # stencil ndim
    g = grid(ndim=2)
    g.n[2] = 4                                                             # unused axis must be 1
    assert apply(g, grid(ndim=2, origin=far()), s2, bc()) == E
    s5, _k5 = stencil(r=5)
    assert apply(grid(h=5), grid(h=5, origin=far()), s5, bc()) == E       # radius > 4
    huge = grid(n=(8, 8, 1 << 10), sz=1 << 45)                             # z span beyond 2^50 elements
    assert apply(huge, grid(n=(8, 8, 1 << 10), origin=far()), s, bc()) == E
    assert "2^50" in L.lope_last_error().decode()
    idx = ctypes.c_int32()
    assert L.lope_iterate(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), ctypes.byref(s),
                          ctypes.byref(bc()), -1, 0, None, ctypes.byref(idx)) == E
    assert L.lope_iterate(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), ctypes.byref(s),
                          ctypes.byref(bc()), 1, 9, None, ctypes.byref(idx)) == E
    assert L.lope_iterate(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), ctypes.byref(s),
                          ctypes.byref(bc()), 1, 0, None, None) == E


def test_iterate_until_validation():
    s, _keep = stencil()
    E = _lib.LOPE_ERR_INVALID_ARG
    steps, res, idx = ctypes.c_int64(9), ctypes.c_double(0), ctypes.c_int32(9)
    outs = (ctypes.byref(steps), ctypes.byref(res), ctypes.byref(idx))

    def call(max_steps=10, every=2, scratch=0x200000, tdepth=0, a=None, o=outs):
        return L.lope_iterate_until(ctypes.byref(a or grid()), ctypes.byref(grid(origin=far())), ctypes.byref(s),
                                    ctypes.byref(bc()), max_steps, every, 1e-6, tdepth, scratch, None, *o)

    assert call(every=0) == E
    assert steps.value == 0 and idx.value == 0 and math.isnan(res.value)
    assert call(max_steps=-1) == E
    assert call(scratch=None) == E
    assert call(scratch=0x200004) == E                     # not 8-byte aligned
    assert call(o=(None, ctypes.byref(res), ctypes.byref(idx))) == E
    assert call(tdepth=7) == E
    assert call(a=grid(sy=5)) == E
    assert call() == _lib.LOPE_ERR_NO_DEVICE                  # valid, but no GPU here


def test_halo_too_small():
    s, _keep = stencil(r=2)
    assert apply(grid(h=1), grid(h=2, origin=far()), s, bc()) == _lib.LOPE_ERR_HALO_TOO_SMALL
    s1, _k = stencil(r=1)
    assert apply(grid(h=0), grid(h=0, origin=far()), s1, bc()) == _lib.LOPE_ERR_HALO_TOO_SMALL


def test_alias_rejected():
    s, _keep = stencil()
    a = grid()
    assert apply(a, grid(), s, bc()) == _lib.LOPE_ERR_ALIAS
    # interiors overlapping by one plane
    b = grid(origin=0x100000 + 4 * 7 * 10 * 10)
    assert apply(a, b, s, bc()) == _lib.LOPE_ERR_ALIAS


def test_too_many_taps_unsupported():
    s, _keep = stencil(ndim=3, r=3, fill=1.0)     # 343 non-zero taps
    assert apply(grid(h=3), grid(h=3, origin=far()), s, bc()) == _lib.LOPE_ERR_UNSUPPORTED


def test_variable_coefficient_restrictions():
    kap = grid(origin=0x80000000)
    vc = _lib.lope_varcoef(ctypes.pointer(kap), 0.1)
    assert L.lope_apply_var(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), ctypes.byref(vc),
                            ctypes.byref(bc(_lib.LOPE_BC_DIRICHLET)), None) == _lib.LOPE_ERR_UNSUPPORTED
    k2 = grid(ndim=2, origin=0x80000000)
    vc2 = _lib.lope_varcoef(ctypes.pointer(k2), 0.1)
    assert L.lope_apply_var(ctypes.byref(grid(ndim=2)), ctypes.byref(grid(ndim=2, origin=far())), ctypes.byref(vc2),
                            ctypes.byref(bc()), None) == _lib.LOPE_ERR_UNSUPPORTED
    assert L.lope_apply_var(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), ctypes.byref(vc),
                            ctypes.byref(bc()), None) == _lib.LOPE_ERR_NO_DEVICE


def test_batch_validation():
    s2, _k = stencil(ndim=2, r=1)
    it = (_lib.lope_batch_item * 1)()
    it[0].src = grid(ndim=2)
    it[0].dst = grid(ndim=2, origin=far())
    it[0].stencil = s2
    it[0].bc = bc()
    out = ctypes.c_void_p()
    assert L.lope_batch_plan_create(it, 1, 10, None, ctypes.byref(out)) == _lib.LOPE_ERR_NO_DEVICE
    s3, _k3 = stencil(ndim=2, r=2)
    it[0].stencil = s3
    it[0].src = grid(ndim=2, h=2)
    it[0].dst = grid(ndim=2, h=2, origin=far())
    assert L.lope_batch_plan_create(it, 1, 10, None, ctypes.byref(out)) == _lib.LOPE_ERR_UNSUPPORTED
    assert L.lope_batch_plan_create(it, 1, 10, None, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_plan_destroy(None) == _lib.LOPE_OK
    assert L.lope_batch_apply(None, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_apply_passes(None, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_persistent_check(None) == _lib.LOPE_ERR_INVALID_ARG
    assert _lib.status_string(_lib.LOPE_ERR_TIMEOUT) == "device wait timed out"


def test_batch_buffers_shared_across_items_rejected():
    """Every pass writes one buffer of every item while reading the other, so
    a buffer overlapping another item's buffer is an alias (checked on the
    host before the device is touched), for plans and the no-alloc call."""
    s2, _k = stencil(ndim=2, r=1)
    it = (_lib.lope_batch_item * 3)()
    base = [0x100000, 0x200000, 0x300000, 0x400000, 0x500000, 0x600000]
    for i in range(3):
        it[i].src = grid(ndim=2, origin=base[2 * i])
        it[i].dst = grid(ndim=2, origin=base[2 * i + 1])
        it[i].stencil = s2
        it[i].bc = bc()
    out = ctypes.c_void_p()
    idx = ctypes.c_int32()
    assert L.lope_batch_plan_create(it, 3, 10, None, ctypes.byref(out)) == _lib.LOPE_ERR_NO_DEVICE
    assert L.lope_batch_apply_noalloc(it, 3, 10, 0, 0, None, ctypes.byref(idx)) == _lib.LOPE_ERR_NO_DEVICE
    it[2].dst = grid(ndim=2, origin=base[0] + 4 * 20)      # inside item 0's src interior
    assert L.lope_batch_plan_create(it, 3, 10, None, ctypes.byref(out)) == _lib.LOPE_ERR_ALIAS
    assert b"items[0].src" in L.lope_last_error() and b"items[2].dst" in L.lope_last_error()
    assert L.lope_batch_apply_noalloc(it, 3, 10, 0, 0, None, ctypes.byref(idx)) == _lib.LOPE_ERR_ALIAS
    it[2].dst = grid(ndim=2, origin=base[5])
    it[1].src = grid(ndim=2, origin=base[4])               # the same buffer as item 2's src
    assert L.lope_batch_plan_create(it, 3, 10, None, ctypes.byref(out)) == _lib.LOPE_ERR_ALIAS


def test_batch_noalloc_validation():
    s2, _k = stencil(ndim=2, r=1)
    it = (_lib.lope_batch_item * 1)()
    it[0].src = grid(ndim=2)
    it[0].dst = grid(ndim=2, origin=far())
    it[0].stencil = s2
    it[0].bc = bc()
    idx = ctypes.c_int32(5)
    assert L.lope_batch_apply_noalloc(it, 1, 4, 0, 0, None, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_apply_noalloc(it, 1, 4, 9, 0, None, ctypes.byref(idx)) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_apply_noalloc(it, 1, 4, 0, -1, None, ctypes.byref(idx)) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_apply_noalloc(it, 1, 4, 0, 1 << 17, None, ctypes.byref(idx)) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_apply_noalloc(it, -1, 4, 0, 0, None, ctypes.byref(idx)) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_apply_noalloc(it, 1, 4, 0, 0, None, ctypes.byref(idx)) == _lib.LOPE_ERR_NO_DEVICE
    assert idx.value == 0
    many = 1 + (4 << 20) // 192                            # more descriptors than the scratch holds
    assert L.lope_batch_apply_noalloc(None, many, 4, 0, 0, None, ctypes.byref(idx)) == _lib.LOPE_ERR_UNSUPPORTED


def test_copy_stream_validation():
    assert L.lope_copy_stream(None, ctypes.c_void_p(0x1000), 16, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_copy_stream(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 17, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_copy_stream(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 16, None) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_copy_stream(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1010), 64, None) == _lib.LOPE_ERR_ALIAS
    assert L.lope_copy_stream(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 64, None) == _lib.LOPE_ERR_NO_DEVICE


def test_status_strings_and_variants():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.lope_status_string(code)
    n = L.lope_variant_count()
    assert n > 10
    buf = ctypes.create_string_buffer(256)
    assert L.lope_variant_info(1, buf, 256) == 0 and b"ndim=" in buf.value
    assert L.lope_variant_info(0, buf, 256) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_variant_info(n + 1, buf, 256) == _lib.LOPE_ERR_INVALID_ARG


def test_variant_selection_and_tuning_table():
    s, _keep = stencil(ndim=3, r=1, fill=0.0)
    arr = _keep
    arr[13] = 1.0
    arr[12] = arr[14] = arr[10] = arr[16] = arr[4] = arr[22] = 0.1     # 7-point star
    g = grid(n=(64, 64, 64))
    v1 = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 1)
    assert v1 > 0
    buf = ctypes.create_string_buffer(256)
    L.lope_variant_info(v1, buf, 256)
    assert b"star3d" in buf.value and b"tdepth=1" in buf.value
    v2 = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 2)
    L.lope_variant_info(v2, buf, 256)
    assert b"tdepth=2" in buf.value
    v0 = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 0)
    t = _lib.lope_tuning(v2, 0, 32, 0)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(t)) == 0
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 0) == v2
    # variant 0 removes the choice: the request falls back to the default
    for req in (0, 3):
        clear = _lib.lope_tuning(0, req, 0, 0)
        assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(clear)) == 0
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 0) == v0
    bad = _lib.lope_tuning(0, 5, 0, 0)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(bad)) == _lib.LOPE_ERR_INVALID_ARG
    # choices are kept per boundary-rule class: a Dirichlet-class choice does
    # not answer all-periodic requests, and the other way round
    dirichlet = bc(kind=_lib.LOPE_BC_DIRICHLET)
    vd0 = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), ctypes.byref(dirichlet), 0)
    td = _lib.lope_tuning(v2, 0, 32, 1)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(td)) == 0
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), ctypes.byref(dirichlet), 0) == v2
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 0) == v0
    mixed = bc()
    mixed.kind[2] = _lib.LOPE_BC_DIRICHLET                                   # one Dirichlet axis: same class
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), ctypes.byref(mixed), 0) == v2
    clear = _lib.lope_tuning(0, 0, 0, 1)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(clear)) == 0
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), ctypes.byref(dirichlet), 0) == vd0
    bad = _lib.lope_tuning(v2, 0, 0, 2)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(bad)) == _lib.LOPE_ERR_INVALID_ARG
    box, _kb = stencil(ndim=3, r=1, fill=0.1)                            # 3D box: generic kernel
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(box), None, 1) == 0


def test_grid_views_match_descriptor():
    """Grid views and the descriptor handed to the library address the same
    elements, also for storage that starts at a non-zero offset."""
    import torch
    import paper_1502_03504_amd as P
    st = torch.zeros(12 * 11 * 10 + 1)[1:]
    g = P.Grid(st, (8, 9, 10), 1, 1, 12, 132)
    d = g.descriptor()
    assert g.interior().data_ptr() == d.origin
    assert g.padded().data_ptr() == d.origin - 4 * (1 + 12 + 132)
    assert (d.n[0], d.n[1], d.n[2], d.stride[1], d.stride[2]) == (10, 9, 8, 12, 132)
    a = P.Grid.allocate((5, 6, 7), 2, torch.float64, "cpu")
    assert a.interior().data_ptr() == a.descriptor().origin
    # the interior row start sits 128 bytes past a 128-byte multiple of the storage start
    assert (a.descriptor().origin - a.storage.data_ptr()) % 128 == 0
    with pytest.raises(ValueError):
        P.Grid(torch.zeros(100), (8, 9, 10), 1, 1, 12, 132)


def test_asymmetric_halo_views_and_descriptor():
    """Per-axis (left, right) halos: the padded view, the interior view and
    the descriptor agree, and the padded box holds exactly the widths."""
    import torch
    import paper_1502_03504_amd as P
    halo = [(2, 0), (0, 1), (1, 3)]            # x, y, z
    g = P.Grid.allocate((4, 5, 6), halo, torch.float32, "cpu")
    d = g.descriptor()
    assert d.halo_mode == 1 and list(d.hlo) == [2, 0, 1] and list(d.hhi) == [0, 1, 3]
    assert g.padded().shape == (4 + 4, 5 + 1, 6 + 2)
    assert g.interior().data_ptr() == d.origin
    assert (d.origin - g.storage.data_ptr()) % 128 == 0
    pad = g.padded()
    pad.copy_(torch.arange(pad.numel(), dtype=torch.float32).reshape(pad.shape))
    assert torch.equal(g.interior(), pad[1:5, 0:5, 2:8])
    e = g.empty_like()
    assert e.halo == g.halo and not e.symmetric
    with pytest.raises(ValueError):
        P.Grid.allocate((4, 5), [(1, -1), (0, 0)], torch.float32, "cpu")


def test_asymmetric_halo_validation():
    """The halo must cover the stencil's reach on each side; a one-sided
    stencil needs a halo on that side only; the adjoint reaches the other way."""
    E, H = _lib.LOPE_ERR_INVALID_ARG, _lib.LOPE_ERR_HALO_TOO_SMALL
    NODEV = _lib.LOPE_ERR_NO_DEVICE

    def agrid(lo, hi, origin=0x100000, n=(8, 8, 1), ndim=2):
        g = grid(n=n, h=0, ndim=ndim, origin=origin, sy=n[0] + lo[0] + hi[0] + 4)
        g.halo_mode = 1
        for a in range(3):
            g.hlo[a], g.hhi[a] = lo[a], hi[a]
        return g

    arr = np.zeros(9)
    arr[3] = 1.0                                  # tap at ox = -1, oy = 0 (upwind)
    s = _lib.lope_stencil()
    s.ndim, s.radius = 2, 1
    s.coeffs = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    left = agrid((1, 0, 0), (0, 0, 0))
    right = agrid((0, 0, 0), (1, 0, 0))
    assert apply(left, agrid((1, 0, 0), (0, 0, 0), origin=far()), s, bc()) == NODEV
    assert apply(right, agrid((1, 0, 0), (0, 0, 0), origin=far()), s, bc()) == H
    assert b"reaches" in L.lope_last_error()
    adj = lambda y: L.lope_apply_adjoint(ctypes.byref(y), ctypes.byref(agrid((0, 0, 0), (0, 0, 0), origin=far())),
                                         ctypes.byref(s), ctypes.byref(bc()), None, None)
    assert adj(left) == H                         # the reflected tap reads to the right
    assert adj(right) == NODEV
    # coefficients count once rounded: 1e-50 vanishes in float32, not in float64
    arr2 = np.zeros(9)
    arr2[4], arr2[5] = 1.0, 1e-50
    s2 = _lib.lope_stencil()
    s2.ndim, s2.radius = 2, 1
    s2.coeffs = arr2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    none = agrid((0, 0, 0), (0, 0, 0))
    assert apply(none, agrid((0, 0, 0), (0, 0, 0), origin=far()), s2, bc()) == NODEV
    none64 = agrid((0, 0, 0), (0, 0, 0))
    none64.dtype = _lib.LOPE_F64
    other64 = agrid((0, 0, 0), (0, 0, 0), origin=far())
    other64.dtype = _lib.LOPE_F64
    assert apply(none64, other64, s2, bc()) == H
    # malformed widths
    bad = agrid((1, 0, 0), (0, 0, 0))
    bad.halo_mode = 2
    assert apply(bad, agrid((1, 0, 0), (0, 0, 0), origin=far()), s, bc()) == E
    assert apply(agrid((-1, 0, 0), (0, 0, 0)), agrid((1, 0, 0), (0, 0, 0), origin=far()), s, bc()) == E
    assert apply(agrid((1, 0, 1), (0, 0, 0)), agrid((1, 0, 0), (0, 0, 0), origin=far()), s, bc()) == E  # unused z
    tight = agrid((1, 0, 0), (2, 0, 0))
    tight.stride[1] = 8 + 2                       # < n[0] + 1 + 2
    assert apply(tight, agrid((1, 0, 0), (0, 0, 0), origin=far()), s, bc()) == E


def test_stages_validation():
    E, H, U, NODEV = (_lib.LOPE_ERR_INVALID_ARG, _lib.LOPE_ERR_HALO_TOO_SMALL, _lib.LOPE_ERR_UNSUPPORTED,
                      _lib.LOPE_ERR_NO_DEVICE)
    s1, _k1 = stencil(r=1)
    star3 = np.zeros((7, 7, 7))                    # radius-3 star: 19 non-zero taps
    star3[3, 3, :] = star3[3, :, 3] = star3[:, 3, 3] = 0.05
    s3 = _lib.lope_stencil()
    s3.ndim, s3.radius = 3, 3
    s3.coeffs = star3.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    big, _kb = stencil(r=2)                        # 125 non-zero taps
    idx = ctypes.c_int32(5)

    def run(a, b, first, second, n=2, out=True):
        sg = _lib.lope_stages(ctypes.pointer(first) if first is not None else None,
                              ctypes.pointer(second) if second is not None else None, 0.5)
        return L.lope_iterate_stages(ctypes.byref(a), ctypes.byref(b), ctypes.byref(sg), ctypes.byref(bc()), n,
                                     None, ctypes.byref(idx) if out else None)

    assert run(grid(), grid(origin=far()), s1, s3) == NODEV      # only the first stencil's reach counts
    assert run(grid(), grid(origin=far()), s3, s1) == H
    assert run(grid(), grid(origin=far()), s1, None) == E
    assert run(grid(), grid(origin=far()), s1, s1, n=-1) == E
    assert run(grid(), grid(origin=far()), s1, s1, out=False) == E
    assert run(grid(h=2), grid(h=2, origin=far()), big, s1) == U
    assert run(grid(), grid(), s1, s1) == _lib.LOPE_ERR_ALIAS
    sg = _lib.lope_stages(ctypes.pointer(s1), ctypes.pointer(s1), 0.5)
    assert L.lope_apply_stages(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), None, ctypes.byref(bc()),
                               None) == E
    assert L.lope_apply_stages(ctypes.byref(grid()), ctypes.byref(grid(origin=far())), ctypes.byref(sg),
                               ctypes.byref(bc()), None) == NODEV


def test_committed_tuning_table_registers_completely():
    import json
    from paper_1502_03504_amd import tune
    with open(tune.DEFAULT_CACHE) as f:
        n = len(json.load(f))
    assert n > 0 and tune.register_cache(tune.DEFAULT_CACHE) == n


def test_tune_cache_registration(tmp_path):
    """Cached choices are keyed by variant name and requested depth and reach
    the library's table without a device."""
    import json
    import paper_1502_03504_amd as P
    from paper_1502_03504_amd import tune
    names = {f["name"]: vid for vid, f in tune._variant_table().items()}
    t1 = [n for n in names if n.startswith("star3d_float_r1_t1_")][0]
    t2 = [n for n in names if n.startswith("star3df_float_r1_t2_")][0]
    cache = {"gfx950|3|1|f32|star|18|0": {"variant": t2, "tdepth": 2, "chunk": 16, "gpts": 1.0},
             "gfx950|3|1|f32|star|18|1": {"variant": t1, "tdepth": 1, "chunk": 8, "gpts": 1.0},
             "gfx950|3|1|f32|star|18|3": {"variant": "no_such_variant", "tdepth": 3, "chunk": 8, "gpts": 1.0}}
    path = tmp_path / "cache.json"
    path.write_text(json.dumps(cache))
    assert tune.register_cache(str(path)) == 2
    s, _keep = stencil(ndim=3, r=1, fill=0.0)
    _keep[13] = 0.4
    for i in (4, 10, 12, 14, 16, 22):
        _keep[i] = 0.1
    g = grid(n=(64, 64, 64))          # 2^18 points: bucket 18
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 0) == names[t2]
    assert L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 1) == names[t1]
    bad = _lib.lope_tuning(names[t2], 1, 0, 0)       # depth 1 request answered by a depth-2 variant
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(bad)) == _lib.LOPE_ERR_INVALID_ARG


def _star7(centre=0.4, side=0.1):
    s, keep = stencil(ndim=3, r=1, fill=0.0)
    keep[13] = centre
    for i in (4, 10, 12, 14, 16, 22):
        keep[i] = side
    return s, keep


def _padded_grid(n, h=1):
    """A descriptor laid out like Grid.allocate (128-byte rows)."""
    sy = ((n[0] + 2 * h + 31) // 32) * 32 + 32
    return grid(n=n, h=h, sy=sy, sz=sy * (n[1] + 2 * h))


def test_untuned_size_takes_nearest_tuned_bucket():
    """A size whose own bucket is not in the committed table takes the choice
    of the nearest tuned bucket of its class (the committed 512^3 float32
    periodic heat entries), so automatic requests keep a fused kernel."""
    s, _keep = _star7()
    buf = ctypes.create_string_buffer(256)
    for n in ((256, 256, 256), (1024, 512, 512), (96, 80, 72)):
        g = _padded_grid(n)
        v = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 0)
        assert v > 0
        L.lope_variant_info(v, buf, 256)
        depth = int(dict(kv.split("=") for kv in buf.value.decode().split()[1:])["tdepth"])
        assert depth >= 2, (n, buf.value)
    # an explicit depth is answered by the nearest bucket's choice of that depth
    g = _padded_grid((256, 256, 256))
    for req in (1, 2, 3, 4):
        v = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, req)
        L.lope_variant_info(v, buf, 256)
        assert b"tdepth=%d " % req in buf.value, (req, buf.value)


def test_tune_set_rejects_negative_chunk():
    s, _keep = _star7()
    g = _padded_grid((64, 64, 64))
    v = L.lope_select_variant(ctypes.byref(g), ctypes.byref(s), None, 1)
    bad = _lib.lope_tuning(v, 1, -3, 0)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(bad)) == _lib.LOPE_ERR_INVALID_ARG
    big = _lib.lope_tuning(v, 1, 2 ** 31 - 1, 0)     # clamped to the marched extent at launch
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(big)) == 0
    clear = _lib.lope_tuning(0, 1, 0, 0)
    assert L.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(clear)) == 0


def test_gbar_size_matches_header():
    import paper_1502_03504_amd as P
    text = open(HEADER).read()
    m = re.search(r"#define LOPE_GBAR_DOUBLES (\d+)", text)
    assert m and int(m.group(1)) == P.LOPE_GBAR_DOUBLES


def test_batch_tune_set_validation_and_cache(tmp_path):
    import json
    from paper_1502_03504_amd import tune
    F32 = _lib.LOPE_F32
    assert L.lope_batch_tune_set(7, 1 << 20, 4, 128) == _lib.LOPE_ERR_INVALID_ARG      # dtype
    assert L.lope_batch_tune_set(F32, 0, 4, 128) == _lib.LOPE_ERR_INVALID_ARG          # points
    assert L.lope_batch_tune_set(F32, 1 << 20, 9, 128) == _lib.LOPE_ERR_INVALID_ARG    # depth
    assert L.lope_batch_tune_set(F32, 1 << 20, 4, 0) == _lib.LOPE_ERR_INVALID_ARG      # rows
    assert L.lope_batch_tune_set(F32, 1 << 20, 4, 1 << 17) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_tune_set(F32, 1 << 20, 4, 64) == 0
    assert L.lope_batch_tune_set(F32, 1 << 20, 0, 0) == 0                              # removes it
    d, r = ctypes.c_int32(), ctypes.c_int32()
    assert L.lope_batch_plan_get_tiles(None, ctypes.byref(d), ctypes.byref(r)) == _lib.LOPE_ERR_INVALID_ARG
    assert L.lope_batch_plan_set_tiles(None, 2, 64) == _lib.LOPE_ERR_INVALID_ARG
    cache = {tune.batch_key(F32, 1 << 21): {"tdepth": 5, "rows": 64, "gpts": 1.0},
             "other_arch|batch|f32|21": {"tdepth": 5, "rows": 64, "gpts": 1.0}}
    path = tmp_path / "cache.json"
    path.write_text(json.dumps(cache))
    assert tune.register_cache(str(path)) == 1
    assert L.lope_batch_tune_set(F32, 1 << 21, 0, 0) == 0


def test_committed_tuning_table_names_built_variants():
    """Every kernel entry of the committed gfx950 table names a variant the
    library builds (a removed build must leave no stale entry), and every
    batch entry holds a depth and strip height the batch plan accepts."""
    import json

    import paper_1502_03504_amd as pkg
    with open(os.path.join(ROOT, "paper_1502_03504_amd", "tuned_gfx950.json")) as f:
        table = json.load(f)
    built = {info.split()[0] for info in pkg.variants()}
    assert table
    for key, entry in table.items():
        if "|batch|" in key:
            assert 1 <= entry["tdepth"] <= 8 and 1 <= entry["rows"] <= 65536, key
        else:
            assert entry["variant"] in built, (key, entry["variant"])
