"""CPU oracle for the LOPe stencil sweep — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, calls or links it, and this package imports
nothing from the product: the two share only the seeded input generators in
``synth``.

Everything here is the plain definition of what the method computes, written
for a reader to check against the paper by eye, in float64 arithmetic with the
state rounded to the grid dtype after every sweep:

* ``stencil``   — halo widths (symmetric or per-axis left/right), halo rule,
  stencil reach, sweep, iteration, two-stage steps (fixed count or until a
  convergence test holds), windowed sampling, adjoint;
* ``diffusion`` — the variable-coefficient diffusion step and its gradient.

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, invariants, library spectral routines or brute force; none is
"parity unpinned".
"""
from .stencil import (  # noqa: F401
    rule_extend, halo_widths, halo_fill, stencil_reach, sweep, iterate, iterate_until, sweep_at, adjoint,
    result_index, stages_step, stages_iterate,
)
from .diffusion import (  # noqa: F401
    diffusion_step, diffusion_forward, diffusion_loss, diffusion_gradient,
    diffusion_step_transpose, diffusion_kappa_vjp,
)
