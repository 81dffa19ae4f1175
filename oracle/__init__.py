"""Plain FP64 CPU oracle for the fast spectral sum-of-Gaussians (SOG) method for
quasi-2D electrostatics (periodic in x and y, free in z).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` may import it.  The HIP library never calls it, and it imports
nothing from the HIP library or its Python binding.

Modules (each function cites the passage of the paper it follows):

* ``sog``      -- the u-series SOG decomposition (Sec. 2.2, Table 1).
* ``ewald2d``  -- the classical O(N^2) Ewald2D lattice sum (the paper's accuracy
                  reference, Sec. 5), written from the standard Parry form, plus
                  a brute-force truncated image sum for tiny inputs.
* ``direct``   -- SOG-direct: the exact value of every term of the SOG
                  decomposition (eqs. SOGdecomp, phiNDR, trun2) with no
                  discretisation, for any set of target particles.
* ``fast``     -- the plain fast method: mid-range Fourier spectral solver
                  (Alg. al::mid), long-range Fourier-Chebyshev solver in its
                  direct form (App. B, Alg. al::long_nonfft) and FFT form
                  (Alg. al::long), near field over a neighbour list, totals.
* ``planner``  -- the oracle's own choice of discretisation parameters
                  (Sec. 4.3), used when a test asks the oracle for a
                  tolerance rather than explicit parameters.

Everything is float64 NumPy/SciPy.  Speed is not a goal; every step is the
formula of the paper written out.
"""
