"""CPU FP64 oracle for the Fourier-basis Helmholtz FMM (Cecka & Darve, arXiv 0911.4114).

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the C-ABI library, its Python binding)
may import, call, link or execute anything in this package. Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark use it.

The oracle shares no code with the HIP path. It is written from the paper:

* ``direct``     -- the definition: the dense Helmholtz matrix-vector product
                    (Section 2, eqn. HelmholtzMatrixVector), plain C + OpenMP, FP64.
* ``special``    -- spherical Bessel/Hankel functions, Legendre polynomials (Table 1 notation).
* ``fourier``    -- Fourier coefficients, |sin| spectrum, 1D Fourier inter/anterpolation
                    (Section 3.1.2, 3.1.3).
* ``quadrature`` -- choice of the Gegenbauer truncation ell (Section 2.1), of N_theta
                    (Alg. Ntheta) and of N_phi(theta_n) (Alg. Nphi) (Section 3.3).
* ``transfer``   -- the band-limited modified transfer function (Alg. BMTF, Section 3.2).
* ``tree``       -- octree, Morton order, neighbour and interaction lists (Section 2).
* ``resample``   -- the five-step FFT inter/anterpolation between level quadratures (Section 3.4).
* ``ffmm``       -- the full multilevel FMM matvec, stage by stage (Section 2 and Section 3).

Every function cites the passage it follows.
"""
