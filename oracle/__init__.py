"""FP64 CPU oracle for the S-fraction multiscale finite-volume method (arXiv 1406.6923).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, NumPy/SciPy
implementation of what the GPU path computes, written from the paper.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
imports it; inputs come from the separate ``workloads`` module.

Modules, in the order of the method:

* ``grid``        fine reference grid operator and FDTD (the semi-discrete wave
                  equation of the Introduction, eq. "wave", and the
                  acoustic model of the Numerical experiments section);
* ``subdomains``  domain decomposition, per-subdomain operators and the boundary
                  basis F (Stage 1 section: F^{alpha beta}, F^alpha; non-overlap
                  condition after eq. "mass");
* ``lanczos``     projection subspaces and block Lanczos tridiagonalisation
                  (Stage 1: K_n(sigma), eq. "krylov0"; Stage 2: T, R);
* ``sfraction``   S-fraction transform (eqs. "GammaU", "GammaTrans") and the
                  transfer functions (eqs. "NtD", "NtDROM", "NtDtri");
* ``rom``         Algorithm 1 Stage 1 per subdomain (steps 1.1-1.4, eq. "Uj");
* ``coupled``     Algorithm 1 Stage 2 (eqs. "mass", "bdrytstep", "intrtstep")
                  with leapfrog, energy and the CFL bound;
* ``adjoint``     discrete adjoint of the Stage 2 leapfrog and the misfit gradients
                  with respect to the S-fraction blocks (the FWI use of the Introduction);
* ``cnn``         the learned ROM surrogate network, forward and backward;
* ``surrogate``   the sound-speed gradient through that network (chain rule).

Every function cites the passage it follows.  Pins against closed forms and
invariants live in ``tests/test_oracle_*.py``.
"""
