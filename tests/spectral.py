"""Spectral solution of a constant stencil iterated on a periodic grid.

Every Fourier mode exp(2 pi i k.x / N) is an eigenvector of a constant
stencil under periodic wrap, with eigenvalue
    lambda(k) = sum_o c_o exp(2 pi i sum_a k_a o_a / N_a),
so n sweeps give u_n = IFFT(lambda^n FFT(u_0)) (a library routine, float64).
Used by the full-size GPU tests for whole runs the oracle cannot finish; pinned
against the oracle on small grids by tests/test_spectral.py.
"""
import os

import numpy as np


def spectral(u, coeffs, steps):
    """u after `steps` sweeps of the stencil `coeffs` (numpy axis order, odd
    side 2r+1 on every axis) on a periodic grid, in float64."""
    import scipy.fft as sf
    shape = u.shape
    d = len(shape)
    r = (coeffs.shape[0] - 1) // 2
    # one 1D phase vector per axis, broadcast along the others (rfft on the last)
    ks = [np.fft.fftfreq(n) * n for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    lam = 0.0
    for idx in zip(*np.nonzero(coeffs)):
        term = complex(coeffs[idx])
        for ax in range(d):
            ph = np.exp(2j * np.pi * ks[ax] * (idx[ax] - r) / shape[ax])
            term = term * ph.reshape([-1 if a == ax else 1 for a in range(d)])
        lam = lam + term
    workers = min(16, os.cpu_count() or 1)
    spec = sf.rfftn(np.asarray(u, dtype=np.float64), workers=workers)
    spec *= lam ** steps
    del lam
    return sf.irfftn(spec, s=shape, workers=workers)
