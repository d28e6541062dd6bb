"""FP64 CPU oracle for the DiffWind simulation step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (``paper_2603_09668_amd``) never imports it and
must fail loudly instead of falling back to it.

Every function here is a plain, slow, obviously-correct restatement of the
paper's equations (DiffWind, ICLR 2026) in float64:

* ``oracle.mpm``   -- MLS-MPM with APIC transfers (Sec. 3.2 "Interaction
  Modeling", Appendix "Material Point Method": Eq. P2G, Eq. G2P,
  Eq. deformation_update; constitutive model Eq. constitutive_model and
  Eq. young_poisson), the grid update of the continuum momentum equation
  (Eq. continuum_mechanics) with the wind force field applied on the MPM
  grid (Sec. 3, problem specification), and the cell sort that the GPU path
  uses to group particles.
* ``oracle.wind``  -- the wind force field on a grid mapped to MPM nodes, and
  the aerodynamic drag relation of Sec. 3.4 ("Physics-Informed Loss").
* ``oracle.lbm``   -- the lattice Boltzmann equation with BGK collision
  (Eq. lbe, Eq. lbm_sum_v2), D3Q19, and the particle-to-voxel solid rule
  (Eq. point2voxel).
* ``oracle.home``  -- the moment-encoded HOME-LBM step (appendix "More
  details on HOME-LBM Algorithm"): third-order Hermite reconstruction of the
  populations from rho, u, S and the moment-space collision.
* ``oracle.gauss`` -- the covariance of each Gaussian kernel after
  deformation, Sigma(t) = F Sigma F^T (Sec. 3.2, "Interaction Modeling").
* ``oracle.recon`` -- the physics-informed loss of Sec. 3.4, the LBM
  direction guide at the wind-grid nodes, and the CosSim / NMSE metrics of
  reconstructed force fields.
* ``oracle.conv``  -- the 3-D convolutional wind surrogate, written with
  ``torch.nn.functional.conv3d`` in float64.

The reverse mode of every function comes from ``torch.autograd`` over these
forward definitions; it is independent of the hand-written adjoints of the
HIP path.

Parity status of each function is stated in its module header; the pins are
the ``-m "not gpu"`` tests under ``tests/test_oracle_*.py``.
"""
