"""Oracle: a plain, slow, FP64 CPU implementation of the coupled 3D-1D method.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  The GPU library never
calls into it and shares no code with it; the two meet only through the seeded
inputs of the `synth` module.

Modules
  fem     finite-element assembly of the block system A u = F (Section 2.1)
  krylov  restarted GMRES / flexible GMRES, Jacobi and block preconditioners
          (Sections 2.2 and 4)
  cnn     the U-net preconditioner: forward, adjoint (backward), loss, Adam
          (Sections 4.2 and 5.1)

Every function states the passage of the paper it follows.  Where the paper
is silent or ambiguous the reading taken is the one listed in the design notes
of the repository.

Parity status: every function here is pinned by a `-m "not gpu"` test in
`tests/test_oracle_*.py` against something other than itself (dense LU, closed
forms, invariants, brute force on tiny inputs, finite differences or a library
routine).
"""
