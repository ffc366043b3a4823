"""CPU FP64 oracle for finite-element-projection FFT homogenization.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the package
entry point and the CPU-baseline leg of the benchmark may import, call, link or
run anything in this directory.  The GPU library never routes through it, and
it shares no code with the GPU library.

Modules
  fe          canonical periodic linear finite elements (the plain definition):
              assembly of the stiffness K and load f, direct / plain-CG solve,
              strain and stress fields, average stress, effective stiffness
  projection  discrete derivative symbols and the small-strain projection
              operator of the paper's small-strain appendix; dense brute force
  pcg         the paper's projected conjugate gradients in strain space
  cg          ctypes wrapper of the plain C CSR conjugate-gradient solver
  adjoint     sensitivities of the effective stiffness to the per-voxel
              Lame constants (energy form, no second solve)
  finite      finite strain: Saint Venant-Kirchhoff law, gradient projection,
              Newton + projected CG, and the canonical nonlinear FE solve
"""
