"""The spectral helper of the full-size GPU tests against the oracle on small
periodic grids (odd and even extents, non-symmetric stencils, 1D-3D), and
against a one-tap shift, whose n sweeps are an exact roll."""
import numpy as np

import oracle
import synth
from synth import PERIODIC as P
from tests.spectral import spectral


def test_matches_oracle_float64():
    rng = np.random.default_rng([synth.CFG_TEST, 1700])
    for shape, r, kind in [((37,), 2, "box"), ((12, 17), 1, "box"), ((9, 10, 11), 1, "star"),
                           ((8, 6, 13), 2, "star")]:
        st = synth.contractive(synth.random_stencil(rng, len(shape), r, kind))
        u = rng.uniform(-1, 1, shape)
        want = oracle.iterate(u, st.coeffs, (P,) * len(shape), 0.0, 9)
        got = spectral(u, st.coeffs, 9)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), shape


def test_one_tap_is_a_roll():
    u = np.random.default_rng(3).uniform(0, 1, (6, 7, 10))
    c = np.zeros((3, 3, 3))
    c[1, 1, 2] = 1.0                       # y[x] = u[x + 1] along the last numpy axis
    got = spectral(u, c, 4)
    np.testing.assert_allclose(got, np.roll(u, -4, axis=2), rtol=0, atol=1e-14)
