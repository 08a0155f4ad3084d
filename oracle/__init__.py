"""Plain, slow FP64 CPU oracle of the Volterra-integral TDSE marching scheme.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constants with the HIP library; the only inputs both sides see come
from ``workloads`` (seeded problem descriptions, no solver arithmetic).

Each function follows the paper step by step (Kaye, Barnett, Greengard,
"A high-order integral equation-based solver for the time-dependent
Schrodinger equation", arXiv:2001.06113) and cites the passage it implements.

Modules
  adams      implicit Adams coefficients (Section 2.2, Table 1) and the
             iterated Richardson weights (Section 2.2)
  periodic   the periodic scheme (Sections 2.1-2.2): trapezoid sub-step,
             Richardson start-up, implicit Adams marching; the moving
             periodic Gaussian well of Section 6, Example 1
  quadrature Gauss-Legendre and Alpert end-corrected trapezoid rules on the
             contour Gamma (Section 3.4)
  chebyshev  C-type transforms through the Chebyshev interpolant (Section 4.1)
  potential  potentials given as samples at the step times, interpolated in time
  freespace  the complex-frequency scheme by dense transforms (Sections 3.3-3.4),
             and its representation evaluated at arbitrary points (Remark on
             evaluation outside [-1,1])
  adjoint    the discrete reverse sweep of the periodic scheme (gradients with
             respect to stepwise field samples and u0)
"""
