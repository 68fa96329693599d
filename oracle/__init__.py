"""CPU FP64 oracle for the shallow-water + Lagrangian-mean hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or runs anything in this package; only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.
It shares no code with the GPU path: the two meet only through the seeded
inputs built by the ``synth`` package.

Contents
--------
``lagmean``   the discretisation, step by step, in float64 NumPy: the rotating
              shallow-water equations (section 4.2, eq. (4.6), dimensional form)
              advanced pseudospectrally with classical RK4, and in the same RK4
              stages the Lagrangian-mean PDEs of both strategies:
              strategy 1, eqs. (3.5)/(4.1) for the partial mean in the g-tilde
              form and eq. (3.9) for the inverse lift map (integrated as
              P = (t - tau)(x - Xi^{-1}), see ``lagmean``), and strategy 2,
              eqs. (4.5a,b) for the displacement xi and g-bar; plus the
              Eulerian mean; optionally (Params.momentum) the strategy-2 mean
              of the momentum 1-form u . dx (appendix C, eq. (C.4)).
``tracker``   the definition oracle: brute-force particle tracking
              (eq. (2.1)) and time averaging along trajectories (eqs. (2.3),
              (2.4), (3.1)), and the pulled-back 1-form average of eq. (C.1)
              with label derivatives from the variational equation, used only
              to check that ``lagmean`` converges to the true means on small
              grids.
``closed``    closed forms used as pins (exact kinematic plane-wave means,
              small-amplitude Stokes corrections, dispersion relation).
``euler2d``   two-dimensional incompressible inviscid flow (section 4.1) with
              strategy 1 pseudospectral (eqs. (4.1), (3.9)) and
              semi-Lagrangian (appendix B, eqs. (B.2), (B.4), (B.5)).
``remap``     strategy 1 remapped to Lagrangian-mean positions (eq. (3.8)):
              the end position of the particle with mean position y as the
              fixed point x = y + eta(x), then f-bar^L(y) = f~^L(x).

Parity pins: every function of ``lagmean``, ``remap`` and ``euler2d`` is pinned by the
not-gpu tests (closed forms, invariants, brute-force tracking, a lift map
inverted by Newton's method); none is "parity unpinned".
"""

from . import lagmean, closed, tracker  # noqa: F401
