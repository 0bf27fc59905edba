"""Plant plausible mistakes in the oracle (on the CPU) and check a pin fails.

Each mutant replaces one internal step of the oracle with a wrong variant —
a flipped offset, a transposed axis, a dropped tap, an unrounded
coefficient, a wrong face average, a reversed scatter — and runs the pins that
should catch it.  A mutant that no pin catches fails this test.
"""
import numpy as np
import pytest

import oracle
import oracle.diffusion as odiff
import oracle.stencil as ost
from tests import test_oracle_diffusion as tdiff
from tests import test_oracle_pins as tp


def _caught(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _brute_all():
    return any(_caught(tp.test_sweep_iterate_adjoint_brute_force, *case)
               for case in tp.BRUTE_CASES)


def test_flipped_offsets(monkeypatch):
    orig = ost._taps
    monkeypatch.setattr(ost, "_taps", lambda c, dt: [(tuple(-o for o in off), v)
                                                     for off, v in orig(c, dt)])
    assert _caught(tp.test_single_tap_is_a_shift, 2)


def test_transposed_boundary_axes(monkeypatch):
    orig = ost._gather
    monkeypatch.setattr(ost, "_gather", lambda u, rg, kinds, g: orig(u, rg, tuple(kinds)[::-1], g))
    assert _brute_all()


def test_dropped_tap(monkeypatch):
    orig = ost._taps
    monkeypatch.setattr(ost, "_taps", lambda c, dt: orig(c, dt)[:-1])
    assert _caught(tp.test_polynomial_exact_7pt_heat)


def test_unrounded_coefficients(monkeypatch):
    orig = ost._taps
    monkeypatch.setattr(ost, "_taps", lambda c, dt: orig(c, np.float64))
    assert any(_caught(tp.test_float32_state_rounding, *case) for case in tp.BRUTE_CASES[:8])


def test_periodic_treated_as_clamp(monkeypatch):
    orig = ost._axis_map

    def clamp(n, lo, hi, kind):
        zi, out = orig(n, lo, hi, "dirichlet")
        return zi, np.zeros_like(out)
    monkeypatch.setattr(ost, "_axis_map", clamp)
    assert _caught(tp.test_heat_mode_decay_closed_form, ("periodic",) * 3)


def test_adjoint_without_transpose(monkeypatch):
    def gather_instead(ybar, coeffs, kinds):
        return ost.sweep(ybar, coeffs, kinds, 0.0), 0.0
    monkeypatch.setattr(ost, "adjoint", gather_instead)
    monkeypatch.setattr(oracle, "adjoint", gather_instead)
    assert _caught(tp.test_adjoint_dot_product)


def test_diffusion_face_not_averaged(monkeypatch):
    orig = odiff._shift
    monkeypatch.setattr(odiff, "diffusion_step",
                        lambda u, k, dt: (u.astype(np.float64) + dt * sum(
                            k * (orig(u.astype(np.float64), s, ax) - u)
                            for ax in range(u.ndim) for s in (-1, 1))).astype(u.dtype))
    monkeypatch.setattr(oracle, "diffusion_step", odiff.diffusion_step)
    assert _caught(tdiff.test_step_matches_brute_force_and_is_symmetric)


def test_diffusion_transpose_wrong_direction(monkeypatch):
    def wrong(lam, kappa, dt):
        lf = lam.astype(np.float64)
        out = lf.copy()
        for ax in range(lam.ndim):
            for s in (-1, 1):
                face = 0.5 * (kappa + odiff._shift(kappa, s, ax))
                w = dt * face * lf
                out -= w
                out += np.roll(w, -s, axis=ax)
        return out
    monkeypatch.setattr(odiff, "diffusion_step_transpose", wrong)
    monkeypatch.setattr(oracle, "diffusion_step_transpose", wrong)
    assert _caught(tdiff.test_step_matches_brute_force_and_is_symmetric)
