"""CPU FP64 oracle for the lattice Green's function (LGF) Poisson path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only the tests, the smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with
the HIP implementation in ``paper_2010_13213_amd``.

What it computes (paper: Yu, Dorschner & Colonius, "Multi-resolution
lattice Green's function method for incompressible flows", Sec. 2.2,
eqs. discrete_laplace / lgf_convolution; Sec. 3.4, eqs. AMR-LGF-2 ...
FLGF-AMR):

* ``lgf_table``   -- the LGF G of the unscaled 7-point Laplacian, exact
                      near field from the Bessel-integral representation,
                      asymptotic far field (Sec. 5, "exact values for near
                      points, asymptotic expansions for far points").
* ``direct``      -- the plain O(N_src * N_tgt) lattice convolution
                      u(n) = dx^2 * sum_m G(n - m) f(m)  (C, OpenMP).
* ``composite``   -- the multi-level FLGF-AMR recursion of Sec. 3.4 with
                      each L_k^{-1} a direct sum.
"""
