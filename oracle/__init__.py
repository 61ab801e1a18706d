"""Plain FP64 CPU oracle for the surface hopping Gaussian beam (SHGB) ensemble.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constant generators); the
only thing both sides see is the seeded input data the tests hand them.

The oracle follows Cai & Lu, "A surface hopping Gaussian beam method for
high-dimensional transport systems" (arXiv:1703.06116):

* ``philox``      Philox4x64-10 counter-based generator (Salmon et al., SC'11),
                  the source of every random number the method draws.
* ``models``      coefficient functions alpha_i, beta_i, gamma_ij of the
                  transport system (Sec. 1, eq:equations): the two-level QCLE of
                  Sec. 3.3 written as a four-component instance, plus two
                  test families with closed-form solutions.
* ``sampling``    initial beam parameters (Sec. 2.5, step 2 of Sec. 2.4).
* ``shgb``        the beam ODEs (Sec. 2.3, eq:shgb_odes), classical RK4, the
                  hop-time / hop / weight algorithm (Sec. 2.4 steps 3-5).
* ``observables`` the estimator U_i = E[exp(omega) G delta_{i,l_t}]
                  (Sec. 2.3, eq:shgb): populations and the superposition
                  at evaluation points.

Every floating point quantity is float64 (complex128 for complex values).

Parity pins (what fixes each part independently of this code) live in
``tests/test_oracle_*.py``.  Parity unpinned: the true populations of the
nonlinear QCLE workloads have no closed form; the oracle is validated on the
same code paths by exact propagation (linear/quadratic coefficients), by the
matrix exponential for x-independent coefficients, by QCLE invariants and by
library routines, and the GPU is pinned to the oracle.
"""

from . import philox, models, sampling, shgb, observables  # noqa: F401
