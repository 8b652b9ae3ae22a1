"""FP64 CPU oracle for the LPP projected-tensor power-spectrum estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path: the
GPU side factorises the line-of-sight kernels into spin-weighted harmonics of
the object direction, while this oracle follows the paper's own Cartesian
decomposition (Sec. III.A, eqs. def_of_Xiij, def_of_Xiijkl, delta_ell) and, on
tiny inputs, the defining double sum directly.

Modules
  special   Legendre / associated Legendre polynomials in exact rationals,
            multipole prefactors, the P_- -> Legendre map, Wigner 3j window
            coefficients (Sec. II.D eqs. def_of_asso, ortho_asso_legendre;
            Sec. III.B eq. def_of_Q_llp).
  geometry  line-of-sight basis (App. E eq. def_standard_rotation) and the
            helicity tensor e_ij (Sec. II.B eq. def_of_eij_+2).
  mesh      mass assignment (NGP/CIC/TSC, interlacing, compensation) and the
            k-shell binning definition.
  estimator the LPP estimators: ``brute`` (definition, tiny inputs), ``mesh64``
            (FFT route with Cartesian tensors), ``gpp`` (global line of sight).
  window    window multipoles and the Hankel/FFTLog window-convolved template
            (Sec. III.B eqs. windowQ_ell, window_convolution_X_hankel).
"""
