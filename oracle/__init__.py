"""Plain FP64 CPU oracle for the anisotropic Cahn-Hilliard MRT lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything from this package; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

Modules
-------
lbm       the method itself (Sections 2-3 of the paper), literal dense
          matrices, ``np.roll`` periodic shifts, float64 throughout.
linear    hand-derived linearisation of one LB step about a uniform state and
          the continuum dispersion relation of the recovered PDE (eq 38 with
          eq 13 at alpha = 0).
spectral  pseudo-spectral (FFT) evaluation of the chemical potential of
          eqs 11/13/15 and an RK4 solver of the Cahn-Hilliard equation eq 10.
unet      float64 NumPy reference of the convolutional surrogate.

Every function cites the passage of the paper it follows.  Readings of
silent / garbled passages are parameters (see ``lbm.Params``).
"""
