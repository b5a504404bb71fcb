"""Plain FP64 CPU oracle for the immersed Newmark IMEX method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
and its C++ host setup: basis, quadrature, space-tree integration, assembly,
partitioning and the time loop are written here again, from the paper, in
the most direct form (global sparse matrices, SciPy's sparse LU for the
implicit block, as the paper itself uses).

Modules
  basis    GLL/GL points, Lagrange basis (Section "Spatial Discretization")
  fcm      finite-cell geometry, space-tree quadrature, element matrices,
           global assembly and the d/c partition (Sections "Spatial
           Discretization", "Partitioning of the Degrees of Freedom")
  newmark  CDM, trapezoidal Newmark and Newmark IMEX loops (Section "Time
           Integration", Newmark IMEX flowchart figure), discrete energy
  springs  the ten spring-coupled masses (Section "Spring-coupled masses")
  mlp      FP64 reference of the learned per-cut-element preconditioner
           network (not part of the paper; parity unpinned beyond finite
           differences)
"""
