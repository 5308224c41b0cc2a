"""Plain FP64 CPU oracle for the SMW-split SAI method (Jia & Zhang, arXiv:1211.6866).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(no kernels, headers, helpers or tables) and never imports it.

Every function is a slow, direct transcription of what the paper defines,
one column or one right-hand side at a time, in float64:

* ``split``      - Procedure * step 1 and Section 4 (irregular columns, sparsification)
* ``pattern``    - static patterns P(A~) and P(|A~|^2) (Section 2.2, BPSAI envelope)
* ``lsq``        - the column least-squares problems (Section 2, (subprob), (lsprob))
* ``spai``       - SPAI augmentation (Section 2.1, (candi), (ls1d), (muj), (rhoj))
* ``psai``       - PSAI(tol): power patterns P(|A~|^l e_k) with the (tolk) drop (Section 2.2)
* ``drop``       - dropping of small entries of m_k (Section 2.2, (tolk)) and assembly of M
* ``krylov``     - right-preconditioned BiCGStab and GMRES(m) with the stopping
                   rules of the Section 4 theorem ((stopb), (stopU2), c = 1)
* ``smw``        - SMW recovery x = y - W (I + V^T W)^{-1} V^T y (Procedure *, (update1)),
                   (composi) and the relative residual (rrnorm)
* ``adjoint``    - gradient of a loss through x = A^{-1} b via the SMW split of A^T
                   (Theorem 3.1 applied to A^T = A~^T + V U^T)
* ``pipeline``   - Procedure * end to end

Parity status: every function above is pinned by ``tests/test_oracle_*.py``
against closed forms, library routines, invariants, brute force or values the
paper prints; none is "parity unpinned".
"""
from . import split, pattern, lsq, spai, psai, drop, krylov, smw, adjoint, pipeline  # noqa: F401
