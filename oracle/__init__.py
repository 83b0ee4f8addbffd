"""Plain FP64 CPU oracle for the stabilised nodal spectral element method
(Engsig-Karup, Eskilsson & Bigoni, arXiv:1512.02548).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; the two meet only in the seeded input
generators, which hold none of the method's arithmetic.

Everything here is deliberately slow and explicit: element matrices are formed
one by one, assembled into scipy sparse matrices and solved directly (the
paper's own solver class, Sec. 3.1.2), so that a reader can check each step
against the paper by eye.

Modules
  refelem   1D/2D reference element: GLL nodes, orthonormal bases,
            Vandermonde matrices, Dr, Ds, M, interpolation, modal filter
  mesh      structured quad->triangle mesh in the sigma-domain
  laplace   coefficient tensor K, quadrature-free stiffness, Dirichlet lift,
            direct solve, reference PCG with element-block Jacobi
  surface   1D gradient recovery, vertical-velocity projection,
            over-integrated free-surface right-hand side, filter
  stepper   one RK4 step of the semi-discrete free-surface system
  exact     closed-form linear-wave solutions used by the pins
"""
