"""Reference oracle for the shrinking-domain particle-mesh step (Llinares 2017).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library or its
Python binding; it is a plain, slow FP64 CPU implementation written from the
paper's equations (Sec. 2.1 Eqs. 1-4, Sec. 2.2 Eqs. 7-9, Sec. 2.3 Table 2,
Sec. 2.4 Eq. 10 and the active-cell / active-particle rules) so that the GPU
path can be checked against it element by element.

Modules
-------
cosmology : background scalars E(a), conformal time, lightcone radius,
            linear growth D(a), f(a)  (Sec. 2.1, Sec. 2.4 Eq. 10, App. A).
pm        : CIC deposit, source assembly, exact mesh solves (FFT / DST-I),
            finite-difference force, CIC interpolation, synchronised
            leapfrog, lightcone removal, active-box rule, one full step.
direct    : O(N^2) direct summation for isolated systems.
conv      : FP64 3D convolution forward/backward (learned warm start).

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force or library routines (see each
function's docstring).  Functions with no such check say "parity unpinned".
"""
