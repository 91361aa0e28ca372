"""Plain CPU FP64 oracle for the field-split additive-Schwarz GMG-GMRES solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the GPU library; both read the
same seeded inputs from ``paper_1909_13201_amd.inputs`` (passed in as data).

Every function is a slow, direct transcription of what the paper (Calandrini,
Aulisa, Ke, "A field-split preconditioning technique for fluid-structure
interaction problems with applications in biomedicine") defines, in FP64,
using NumPy / SciPy primitives (sparse matrices, dense LU) and no blocking,
fusion or reordering beyond the definitions.

Modules
-------
mesh       nested structured hierarchy, node types, J2 DOF layout, Dirichlet
fem        Q2/Q1 assembly of the linearized monolithic system (Section 2.2)
transfer   prolongation and equation-routed restriction (Section 3.3)
schwarz    Vanka / overlapping blocks, the additive update and the colour-ordered
           multiplicative sweep (Section 3.2)
multigrid  the V-, W- and F-cycles and their transposes (Section 3)
krylov     restarted FGMRES with classical Gram-Schmidt twice
adjoint    adjoint solve and parameter gradients
"""
