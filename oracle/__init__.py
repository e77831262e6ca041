"""FP64 CPU oracle for the COLA particle-mesh method.

Tassev, Zaldarriaga & Eisenstein, "Solving Large Scale Structure in Ten Easy Steps
with COLA" (arXiv:1301.0322).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code,
table or constant generator with the HIP library under ``paper_1301_0322_amd/``
and never imports it.

It is a plain, slow, obviously-correct statement of what the method computes:

* ``cosmology`` -- background Q(a), growth factors D1, D2 and their T, T^2
  derivatives, the BBKS spectrum and its sigma8 normalisation, and the COLA
  kick/drift coefficients of eq. (KDKALC) on the time grid of eq. (ALCtimestep),
  and of the variants eq. (KDKALCstd) and eq. (KDKStd), steps uniform in a or log a.
* ``lpt``       -- second-order LPT displacement fields s1, s2 from a Gaussian field.
* ``pm``        -- cloud-in-cell deposit, k-space Poisson solve with spectral
  gradient, cloud-in-cell gather: the force -(3/2) Om a d d^-2 delta of eq. (eom).
* ``cola``      -- the COLA time evolution L+ (prod K D K) L- of eqs. (ALCtimestep),
  (Lops) and (KDKALC), or the plain PM leapfrog of eq. (KDKStd).
* ``power``     -- the shell-averaged power spectrum used to compare final densities.
* ``philox``    -- Philox4x32-10 counter-based generator and Box-Muller normals.

Every floating-point computation is FP64.  Fields are torch CPU float64 tensors
so that autograd through the oracle yields a reference gradient.

Every function here has a pin in ``tests/test_oracle_*.py`` (closed forms,
conservation laws, special cases and brute force) except where its docstring says
"parity unpinned".
"""
