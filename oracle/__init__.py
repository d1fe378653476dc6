"""FP64 CPU oracle for the interior-point multigrid method (Kocvara & Mohammed,
"Primal-dual interior-point multigrid method for topology optimization").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: it exists so that tests, the smoke check and the CPU-baseline leg
of the benchmark can compare the GPU library against a plain, slow, obviously
correct implementation written from the paper.  It shares no code with the HIP
path (no kernels, headers, tables or constant generators).

Modules
-------
fem    grid / DOF indexing, Q1 element matrices, assembly of K(x)   (Sec. 1, Sec. 7)
mg     prolongation, Galerkin hierarchy, damped Jacobi, V-cycle      (Sec. 5.1, Sec. 7)
pcg    Algorithm PCG with one V-cycle as preconditioner              (Sec. 5.2, Sec. 6.1)
ip     KKT residuals, Newton systems, augmented system Z, IP loop    (Sec. 2, Sec. 3)
sens   element sensitivities and adjoint gradient                    (Sec. 2, eq. (KKT3))

Every floating-point computation is IEEE double precision.
"""
