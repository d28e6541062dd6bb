"""Pins of the oracle's elastic force against the mathematics (CPU).

The momentum pins of P2G cannot see the stress part of the MLS affine matrix
(sum_i w d = 0 removes it from the linear momentum, the symmetry of tau from
the angular momentum, and F = I makes it zero), and P = d psi / d F holds for
any scaling of psi.  These tests pin what they leave open:

* energy consistency (MLS-MPM, appendix "Material Point Method"): the stress
  part of P2G's grid momentum equals minus the gradient of the total elastic
  energy sum_p V0_p psi(F_p') with respect to the grid velocities, where F_p'
  is the deformation gradient that G2P's update F' = (I + dt C) F gives for
  those grid velocities, taken at zero grid velocity.  This ties the sign,
  the 4/dx^2, V0 and dt factors of A_p = m C - dt V0 (4/dx^2) tau and the
  form tau = P F^T to the energy of Eq. constitutive_model; it is checked by
  central differences of that energy.
* the small-strain limit of both models: P(I + e) = 2 mu sym(e) + lam tr(e) I
  + O(|e|^2), which fixes which coefficient multiplies which term and the
  scale of psi;
* the meaning of E and nu (Eq. young_poisson): under a strain with axial part
  e and lateral parts -nu e (small e), the stress is uniaxial with magnitude
  E e.

`test_pins_catch_planted_mistakes` feeds each pin a deliberately wrong
oracle variant and requires the pin to reject it."""
import numpy as np
import pytest
import torch

from oracle import mpm
from oracle.mpm import FIXED_COROTATED, NEO_HOOKEAN, Grid
from paper_2603_09668_amd import scenes

DT = torch.float64


@pytest.fixture(autouse=True)
def _float64_default():
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def _tiny_scene(seed=21, n=5, res=8):
    """A few particles with distinct masses, volumes, materials and strains."""
    grid = Grid(res, res, res, 1.0 / res)
    rng = np.random.default_rng(seed)
    x = torch.tensor(scenes.random_particles_in_box(seed, n, [0.35] * 3, [0.65] * 3))
    F = torch.eye(3) + 0.08 * torch.tensor(rng.standard_normal((n, 3, 3)))
    mass = torch.tensor(rng.uniform(0.5, 2.0, n))
    vol0 = torch.tensor(rng.uniform(0.3, 3.0, n)) * 1e-3
    mu = torch.tensor(rng.uniform(20.0, 60.0, n))
    lam = torch.tensor(rng.uniform(80.0, 150.0, n))
    return grid, x, F, mass, vol0, mu, lam


def _stress_momentum(grid, x, F, mass, vol0, mu, lam, dt, material):
    """Grid momentum of P2G with v = C = 0: only the stress part of A_p."""
    n = x.shape[0]
    _, gmv = mpm.p2g(grid, x, torch.zeros(n, 3), torch.zeros(n, 3, 3), F, mass, vol0, mu, lam, dt, material)
    return gmv


def _energy_gradient_fd(grid, x, F, vol0, mu, lam, dt, material, nodes, energy=mpm.energy_density, h=1e-7):
    """- d/d v_i of sum_p V0_p psi((I + dt C_p(v)) F_p) at v = 0, by central
    differences, for the grid velocity components `nodes` = [(node, axis)].
    C_p(v) and the update of F are G2P's (Eq. G2P, Eq. deformation_update)."""
    def total(gv):
        _, _, _, Fn = mpm.g2p(grid, gv, x, F, dt)
        return (vol0 * energy(Fn, mu, lam, material)).sum()

    out = []
    for node, a in nodes:
        gp = torch.zeros(grid.n_nodes, 3)
        gm_ = torch.zeros(grid.n_nodes, 3)
        gp[node, a] = h
        gm_[node, a] = -h
        out.append(-(total(gp) - total(gm_)).item() / (2 * h))
    return torch.tensor(out)


def _touched(grid, x):
    base, _, _ = mpm.stencil(x, grid)
    nodes = set()
    for o in mpm._offsets():
        nodes.update(mpm._node_index(grid, base, o).tolist())
    return sorted(nodes)


def _energy_consistency_error(grid, x, F, mass, vol0, mu, lam, dt, material, p2g_vol0=None, p2g_dt=None,
                              p2g_stress=None, energy=mpm.energy_density):
    """Relative max-norm mismatch between P2G's stress momentum and minus the
    energy gradient over every touched node and axis.  The p2g_* arguments
    substitute what P2G is given (to plant a mistake)."""
    vol_p = vol0 if p2g_vol0 is None else p2g_vol0
    dt_p = dt if p2g_dt is None else p2g_dt
    if p2g_stress is None:
        gmv = _stress_momentum(grid, x, F, mass, vol_p, mu, lam, dt_p, material)
    else:
        saved = mpm.kirchhoff_stress
        mpm.kirchhoff_stress = p2g_stress
        try:
            gmv = _stress_momentum(grid, x, F, mass, vol_p, mu, lam, dt_p, material)
        finally:
            mpm.kirchhoff_stress = saved
    comps = [(i, a) for i in _touched(grid, x) for a in range(3)]
    fd = _energy_gradient_fd(grid, x, F, vol0, mu, lam, dt, material, comps, energy=energy)
    got = torch.stack([gmv[i, a] for i, a in comps])
    return ((got - fd).abs().max() / fd.abs().max()).item()


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_mls_stress_is_energy_gradient(material):
    grid, x, F, mass, vol0, mu, lam = _tiny_scene()
    err = _energy_consistency_error(grid, x, F, mass, vol0, mu, lam, 0.37, material)
    assert err < 1e-6, err


def _small_strain_error(material, stress=mpm.pk1_stress, seed=22):
    rng = np.random.default_rng(seed)
    n = 16
    e = 1e-6 * torch.tensor(rng.standard_normal((n, 3, 3)))
    mu = torch.tensor(rng.uniform(1.0, 5.0, n))
    lam = torch.tensor(rng.uniform(6.0, 12.0, n))
    P = stress(torch.eye(3) + e, mu, lam, material)
    sym = 0.5 * (e + e.transpose(1, 2))
    tr = torch.diagonal(e, dim1=1, dim2=2).sum(-1)
    lin = 2.0 * mu[:, None, None] * sym + lam[:, None, None] * tr[:, None, None] * torch.eye(3)
    return ((P - lin).abs().max() / lin.abs().max()).item()


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_small_strain_limit_is_linear_elasticity(material):
    assert _small_strain_error(material) < 1e-4


def _uniaxial_error(material, lame=mpm.lame, E=2.5e4, nu=0.3):
    mu, lam = lame(E, nu)
    e = 1e-7
    F = torch.diag(torch.tensor([1.0 + e, 1.0 - nu * e, 1.0 - nu * e]))[None]
    P = mpm.pk1_stress(F, mu.reshape(1), lam.reshape(1), material)[0]
    target = torch.zeros(3, 3)
    target[0, 0] = E * e
    return ((P - target).abs().max() / (E * e)).item()


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_young_modulus_and_poisson_ratio(material):
    assert _uniaxial_error(material) < 1e-5


def test_pins_catch_planted_mistakes():
    grid, x, F, mass, vol0, mu, lam = _tiny_scene()
    dt = 0.37
    args = (grid, x, F, mass, vol0, mu, lam, dt)
    for material in (FIXED_COROTATED, NEO_HOOKEAN):
        assert _energy_consistency_error(*args, material) < 1e-6
        # flipped sign of the stress term
        flip = lambda Fm, m, l, mat, _k=mpm.kirchhoff_stress: -_k(Fm, m, l, mat)
        assert _energy_consistency_error(*args, material, p2g_stress=flip) > 0.5
        # tau = F^T P instead of P F^T
        wrong_side = lambda Fm, m, l, mat: Fm.transpose(-1, -2) @ mpm.pk1_stress(Fm, m, l, mat)
        assert _energy_consistency_error(*args, material, p2g_stress=wrong_side) > 1e-2
        # V0 dropped, dt dropped, 4/dx^2 dropped (each equals giving P2G a
        # changed volume or step, since the stress term is their product)
        assert _energy_consistency_error(*args, material, p2g_vol0=torch.ones_like(vol0)) > 0.5
        assert _energy_consistency_error(*args, material, p2g_dt=1.0) > 0.5
        assert _energy_consistency_error(*args, material, p2g_dt=dt * grid.dx ** 2 / 4.0) > 0.5
        # mu and lambda exchanged in the stress, or psi and P scaled together
        swapped = lambda Fm, m, l, mat, _s=mpm.pk1_stress: _s(Fm, l, m, mat)
        scaled = lambda Fm, m, l, mat, _s=mpm.pk1_stress: 2.0 * _s(Fm, m, l, mat)
        assert _small_strain_error(material, stress=swapped) > 0.1
        assert _small_strain_error(material, stress=scaled) > 0.5
        # the Lame map with mu and lambda exchanged
        bad_lame = lambda E, nu, _l=mpm.lame: tuple(reversed(_l(E, nu)))
        assert _uniaxial_error(material, lame=bad_lame) > 0.1
