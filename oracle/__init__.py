"""Plain FP64 CPU reference of the DLRA proton-transport step (test infrastructure).

This package is the checker for the HIP library: a slow, literal implementation
of what the paper's method computes, written from the paper's equations.  It is
used only by the tests, by the smoke check and by the benchmark's CPU-baseline
leg; no product code imports it, and it shares no code with the HIP path.

Modules
  pn          real spherical harmonics, streaming matrices A_d and their
              eigen-split, beam moment vector (Sec. 3.3.1, Sec. 3.3.2)
  transport   second-order upwind differences, the semi-discrete streaming
              operator and its K-, L- and S-step forms (Sec. 3.3.2, eq. KLS)
  coeffs      energy grid and per-step coefficients (Sec. 3.3, eq. discAngle)
  linalg      truncation, augmentation and completion rules (Sec. 2.2)
  fullrank    the full-rank step (eq. streamscattsplit with the Lie splitting)
  dlra        the dynamical low-rank step (Sec. 2.2 and Sec. 3.3.3)
  raytrace    the uncollided ray tracer (Sec. 3.2)
  solver      drivers that run whole problems
  adjoint     plan objective over beam weights and its closed-form gradient
"""
