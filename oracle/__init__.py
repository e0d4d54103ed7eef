"""CPU ORACLE -- test infrastructure, not part of the solver.

Plain, slow, FP64 reference implementations used to check the GPU library:

* ``core``   -- C sequential sweep (Thomas) per right-hand side, a general
  tridiagonal solve, and the adjoint (gradient) of X = A^{-1} F.
* ``method`` -- the paper's own steps in NumPy, in its order and notation:
  rows G_k of A^{-1} (Lemma 2), vectors Z^R_k, Z^L_k (eq. z_vector), the
  weights beta (eq. beta_symn), the interface values by the double sum of
  Theorem 2 (eq. theor_2), Lemma 1's independent block solves, and the
  dichotomy level sets (eq. omega_i) with Theorem 3's evaluation order.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path.
"""
from .core import build, thomas, tridiag_general, grad, num_threads, OracleError  # noqa: F401
from . import method  # noqa: F401
