"""Plain FP64 CPU oracle for the self-tuning-EOS multiphase lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check in
``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of ``bench.py`` may
import anything from this package.  The GPU library never calls it, and it
never calls the GPU library: the two share no code.

The oracle follows Huang, Wu & Adams, "Lattice Boltzmann model with
self-tuning equation of state for multiphase flows" (arXiv:1809.02390):

* ``hostmap``  -- Carnahan-Starling EOS (main Eq. 20), Maxwell construction
  (main Eq. 19), flat-interface surface tension and thickness from the
  pressure tensor (main Eqs. 17-18), the sigma/W -> K_EOS/K_INT map
  (main Eqs. 21-23), the coefficient constraints (main Eq. 7) and the
  relaxation-rate constraint (main Eq. 16).
* ``lbm``      -- one time step written as the defining collision equation
  (supplement Eq. 1, i.e. main Eq. 13) with dense per-node matrices, the
  force stencil (main Eq. 12), streaming (supplement Eq. 2); plus the
  six-step implementation sequence of supplement Sec. IV, kept as an
  independent second form.
* ``measure``  -- macroscopic read-outs: mass, momentum, interface thickness,
  droplet radius, Laplace pressure jump, domain length.
* ``adjoint``  -- exact derivatives of the oracle step by the complex-step
  method (transposed Jacobian products and loss gradients).

Every function computes in float64 (or complex128 for complex-step
derivatives).  Nothing here is tuned for speed.
"""
