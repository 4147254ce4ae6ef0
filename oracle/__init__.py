"""Plain FP64 CPU oracle for the large-time-step MOT-JVIE hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and imports nothing from it.

What it computes (Kumar, Gerini, van Beurden, "Large-Time-Step Operation in a
Volume Integral Equation for Dielectric Scattering"):

* ``basis``     -- time step, lag count (Eq. 4) and the causal quadratic-spline
                   temporal basis (Sec. II, discretization paragraph).
* ``masks``     -- causal region of each interaction matrix Z_k (Fig. 1 and its
                   discussion in Sec. III-A) and the Z0 nonzero count (Table III).
* ``green``     -- the Green dyad G_k(d) of the voxel discretization of Eq. 1,
                   evaluated from its definition by face and edge integrals.
* ``operators`` -- Z0 = D - X G (Eq. 10) as a dense matrix, as a direct
                   Toeplitz sum and in the FFT form of Eq. 11 / Eq. 12.
* ``krylov``    -- Freund's TFQMR (Sec. II, solver paragraph), real arithmetic.
* ``march``     -- plane-wave excitation (Eq. 7, Eq. 8) and the MOT recursion
                   of Eq. 3.
* ``adjoint``   -- the transposed operators Z_k^T (contrast on the input), the
                   far-field signature of the current history and its energy,
                   the time-reversed adjoint march and the gradient of the
                   energy with respect to eps_r.

Transforms use ``scipy.fft`` (one thread by default; a caller may lend it
more with ``scipy.fft.set_workers``, which changes nothing but the speed).

Parity status of each function is stated in its docstring; every function is
pinned by ``tests/test_oracle_*.py`` against values the paper prints, closed
forms or invariants, unless it says "parity unpinned".
"""

from . import basis, masks, green, operators, krylov, march, adjoint  # noqa: F401
