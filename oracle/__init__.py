"""Plain FP64 CPU oracle for the ensemble lattice-Boltzmann + rare-event path.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2005_09323_amd``) never imports, calls or links anything here, and
nothing here imports the product path: the two share no code, no constants
module and no helpers.  The only inputs both sides see come from the seeded
generators in ``workloads.py``, which hold none of the method's arithmetic.

Everything is written to be checked against the paper by eye:

* ``philox``  -- counter-based Philox4x64-10 generator (Salmon et al., SC'11),
  written from its published definition; used for every random draw the
  method itself makes (initial density noise, GKTL uniforms, AMS parents,
  branching perturbation weights).
* ``lbm``     -- D2Q9 lattice BGK with Guo body forcing, halfway bounce-back
  and momentum-exchange drag (paper Appendix A; Section 2 for the boundary
  treatment).  Full populations f_i in FP64, never deviations.
* ``perturb`` -- branching perturbation by a random combination of snapshots
  with mass rescaling (paper Appendix D).
* ``gktl``    -- GKTL cloning weights, multinomial selection, SCGF and the
  return-time estimator (paper Section 4.2 and Appendix C).
* ``ams``     -- trajectory-AMS kill/branch selection and the unbiased
  estimator (paper Section 4.1 and Appendix B).
* ``ou``      -- the Ornstein-Uhlenbeck test process of Appendix B.2 and its
  closed forms.
* ``cnn``     -- the small convolutional score network (forward, hand-written
  backward, Adam) in FP64.
* ``features``-- the near-wake (u_x, u_y, rho-1) feature patch fed to the
  score network.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
something other than itself (closed forms, invariants, a library routine,
brute force); the few functions with no such pin say "parity unpinned" in
their docstring.
"""
