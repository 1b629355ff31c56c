"""Plain FP64 CPU oracle of the element-local ADER-DG update (test infrastructure).

This package is test infrastructure only. It is called by the tests, by the
smoke check and by the CPU-baseline leg of the benchmark, never by the library.
It shares no code with the GPU path: it builds its own basis, quadrature,
adjacency and Riemann solver, and it works at physical quadrature points
instead of precomputed reference matrices.

Modules
    basis       orthonormal Dubiner basis on the reference tetrahedron (Sec. 4.1)
    quadrature  collapsed Gauss-Jacobi rules on the tetrahedron and triangle
    physics     Jacobians of the velocity-stress system (Sec. 3, Sec. 4.1)
    riemann     pointwise Godunov state at faces (Sec. 4.2) and boundaries (Sec. 4.3)
    mesh        geometry and face adjacency
    solver      ADER predictor / corrector, gravity faces and clustered LTS (Sec. 4)
    analytic    closed-form solutions used as pins
"""
