"""Oracle: a plain, slow, independent CPU implementation of what the library computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links it, and this package never imports the product path.  The only code the
two sides share is the seeded input generator ``paper_2306_11324_amd.inputs``,
which constructs NURBS control nets and random vectors and holds none of the
method's arithmetic.

Contents (all floating point in fp64 / complex128):

* ``bspline``   -- B-spline bases by the Cox-de Boor recursion (Sec. 3.1).
* ``geometry``  -- NURBS patch maps F_j, tangents, normals, surface measure
                   (Sec. 3.2, Sec. 4.2).
* ``spaces``    -- the spline spaces S^2_{p,m} and S^0_{p,m} (Sec. 3.3).
* ``quadrature``-- Gauss-Legendre and Duffy-type singular rules for element
                   pairs (the paper defers quadrature to its references; see
                   the module docstring for the reading taken).
* ``galerkin``  -- O1: the dense Galerkin matrices of the CFIE (Sec. 4.1-4.3),
                   right-hand sides, LU solve and far-field pattern.
* ``h2``        -- O2: the reference-domain interpolation H^2 matrix built and
                   applied step by step (Sec. 4.4).
* ``mie``       -- closed-form sphere solutions used as pins.

Parity status per function is stated in the module docstrings.
"""
