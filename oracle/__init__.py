"""CPU oracle for the PEXSI hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy/scipy code written from the paper
(arXiv:1405.0194, Sec. II.A-II.D).  Only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(the compiled library and its binding) never does, and this package imports
nothing from the product package.  The two sides share no code: they only
consume the same seeded inputs.

Modules
  fermi     Fermi-Dirac occupation and the other occupation-like functions
            whose pole expansions the method uses (eq. fermidirac, eq. gammaF,
            the N'(mu) expansion of Sec. II.C).
  poles     the pole table {z_l, omega_l} (eq. polerho), by contour
            quadrature of the Cauchy integral after a conformal map (the
            construction the paper refers to; see the module docstring).
  dense     dense routes to Gamma, Gamma^E, the selected inverse, traces and
            inertia counts (eqs. gammaeq, gammapole, gammaF, Nmu; Sec. II.C).
  symbolic  brute-force boolean elimination: the pattern of L and the
            elimination tree by its definition (eq. parent).
  chempot   the chemical-potential search of Sec. II.C (N_beta from inertia
            samples, band-edge bracketing, the exact root of N_P(mu) = N_e).
  dos       DOS bin averages and the LDOS (2/pi) Im [H - (eps + i eta) S]^{-1}
            (Sec. II.D).
  hermitian complex Hermitian pencils: Gamma as (M - M^H)/2i (conclusion).
  sparse    single columns of A^{-1} by a Krylov solve, for systems too large
            for the dense routes.

Every function here is pinned by tests/test_oracle_*.py against closed forms,
special cases, brute force or invariants -- see those files.
"""
