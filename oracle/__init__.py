"""Reference oracle for the implicit AMR radiation-diffusion hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU
restatement of what the method computes, written from the paper (Philip et
al., "Dynamic Implicit 3D Adaptive Mesh Refinement for Non-Equilibrium
Radiation Diffusion", arXiv:1302.6303).  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path (the
HIP library and its Python binding) never does, and shares no code with it.

Modules
-------
hierarchy   patch hierarchy, covered cells, restriction, ghost fill (Sec. 3.2)
operators   flux-limited residual, analytic Jacobian action and its transpose
            (Sec. 3.1-3.3, 4.1)
precond     physics-based preconditioner: 2x2 coupling solve, diffusion-block
            FAC V(1,0) with a multigrid base solve (Sec. 4.2-4.3, Alg. 1)
solvers     FGMRES, inexact Newton with Eisenstat-Walker forcing, BDF1/BDF2
            steps with the leapfrog predictor, discrete adjoint (Sec. 3.3, 4.1)
direct      assembled sparse Jacobian and the exact discrete BDF solution
            (definition layer used to pin the iterative layers)

Parity status of each function is stated in its docstring; readings of the
paper where it is silent or ambiguous are listed in the design notes.
"""
