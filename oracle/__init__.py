"""FP64 CPU oracle of compressive spectral clustering (static and dynamic).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct restatement
of what the paper computes, in float64 with NumPy/SciPy.  It shares no code with the HIP
library and neither side imports the other; only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path never
routes through it.

Modules
  operator   normalized adjacency / Laplacian of Sec. 2.1 and its spectrum
  chebyshev  step-function coefficients, Jackson damping, the three-term filter and the
             dense filter U h(Lambda) U^T (Sec. 2.2 and Sec. 3.2)
  eigcount   Hutchinson eigencount, Chebyshev moments (direct and doubled) and the
             dichotomy on lambda_k (Sec. 3.2 and Sec. 4.1)
  kmeans     assignment, Lloyd update, k-means++ and the cost of eq. (SC_cost) (Sec. 2.1)
  dynamic    Algorithm 1 (dynamic CSC) and static CSC (Sec. 4.1)
  adjoint    reverse-mode derivative of the Chebyshev filter
  philox     Philox4x32-10 counter-based generator and the Gaussian draw built on it
"""

from . import adjoint, chebyshev, dynamic, eigcount, kmeans, operator, philox  # noqa: F401
