"""FP64 CPU oracle for the two-asset exponential-Levy PIDE scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything from this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP path (``paper_2511_02700_amd``) and does not import it.

It is a plain, slow, step-by-step NumPy/SciPy implementation of the method of
Moda, in 't Hout, Vanmaele and Benth, "Numerical valuation of European options
under two-asset infinite-activity exponential Levy models" (arXiv 2511.02700),
transformed to log-moneyness coordinates y_i = ln(S_i / K) on a uniform grid:

* ``levy``      -- the 2D Normal Tempered Stable Levy density and its closed-form
                   moments / characteristic exponent (Sec. 4, Appendix A).
* ``integral``  -- the integral discretization: regions R_I/R_II/R_III, the
                   quadrature weights omega, the artificial diffusion matrix and
                   the modified drift / kill rate (Sec. 3.1, Sec. 4 settings).
* ``scheme``    -- the spatial operators D, B (direct sum or FFT), the
                   semi-Lagrangian interpolation, cell-averaged initial data and
                   the time march of Algorithm 1 (Sec. 3.2, 3.3).
* ``output``    -- prices and deltas at spot pairs by cubic Lagrange
                   interpolation (Sec. 4).
* ``adjoint``   -- the exact discrete adjoint of the theta-scheme march with
                   dense matrices (small grids): gradients with respect to the
                   diffusion coefficients, kill rate, drift and weights.

Every function states the passage of the paper it follows.  Where the paper is
silent or ambiguous on the log-grid, the reading taken is stated in the
function's docstring.
"""

from . import levy, integral, scheme, output, adjoint  # noqa: F401
