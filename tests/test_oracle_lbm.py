"""Pins of the float64 D3Q19 BGK oracle against closed forms and invariants."""
import math

import numpy as np
import pytest
import torch

from oracle import lbm
from oracle.lbm import BOUNCEBACK, INLET, OUTLET, PERIODIC, Lattice, LBMParams
from paper_2603_09668_amd import scenes

DT = torch.float64


@pytest.fixture(autouse=True)
def _float64_default():
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def _near_eq(lat, seed, amp=0.01):
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * torch.tensor(rng.standard_normal((lat.nz, lat.ny, lat.nx)))
    u = 0.05 * torch.tensor(rng.standard_normal((3, lat.nz, lat.ny, lat.nx)))
    f = lbm.equilibrium(rho, u) + amp * 0.01 * torch.tensor(rng.standard_normal((19, lat.nz, lat.ny, lat.nx)))
    return f


def test_lattice_tables():
    c = lbm.C
    assert torch.all(c[lbm.OPP] == -c)
    assert abs(lbm.W.sum().item() - 1.0) < 1e-15
    # isotropy: sum w c_a c_b = delta / 3, fourth moment sum w c_a^2 c_b^2 = 1/9 (a != b)
    cd = c.to(DT)
    M2 = torch.einsum("q,qa,qb->ab", lbm.W, cd, cd)
    assert (M2 - torch.eye(3) / 3).abs().max() < 1e-15
    assert abs(torch.einsum("q,q,q->", lbm.W, cd[:, 0] ** 2, cd[:, 1] ** 2).item() - 1 / 9) < 1e-15


def test_equilibrium_moments():
    rng = np.random.default_rng(1)
    rho = 1.0 + 0.1 * torch.tensor(rng.standard_normal((5,)))
    u = 0.1 * torch.tensor(rng.standard_normal((3, 5)))
    feq = lbm.equilibrium(rho, u)
    c = lbm.C.to(DT)
    assert (feq.sum(0) - rho).abs().max() < 1e-14
    assert (torch.einsum("qa,qn->an", c, feq) - rho * u).abs().max() < 1e-15
    Pi = torch.einsum("qa,qb,qn->abn", c, c, feq)
    ref = rho[None, None] * (torch.eye(3)[:, :, None] / 3 + u[:, None] * u[None, :])
    assert (Pi - ref).abs().max() < 1e-15


def test_periodic_box_conserves_mass_and_momentum():
    lat = Lattice(6, 5, 4)
    p = LBMParams(tau=0.7)
    f = _near_eq(lat, 2)
    m0 = f.sum()
    c = lbm.C.to(DT)
    j0 = torch.einsum("qa,qzyx->a", c, f)
    for t in range(20):
        f, rho, u = lbm.lbm_step(lat, p, f, t=t)
    assert abs(f.sum() - m0) / m0 < 1e-13
    assert (torch.einsum("qa,qzyx->a", c, f) - j0).abs().max() < 1e-13


def test_uniform_equilibrium_stays_uniform_with_inlet_outlet():
    lat = Lattice(8, 6, 5)
    uin = (0.05, 0.0, 0.0)
    p = LBMParams(tau=0.6, u_in=uin, bc=(INLET, OUTLET, PERIODIC, PERIODIC, PERIODIC, PERIODIC))
    u = torch.tensor(uin, dtype=DT).view(3, 1, 1, 1).expand(3, 5, 6, 8)
    f = lbm.equilibrium(torch.ones(5, 6, 8, dtype=DT), u)
    f0 = f.clone()
    for t in range(5):
        f, rho, uo = lbm.lbm_step(lat, p, f, t=t)
    assert (f - f0).abs().max() < 1e-15


def test_fluid_at_rest_with_obstacle_stays_at_rest():
    lat = Lattice(8, 8, 8)
    p = LBMParams(tau=0.8, bc=(BOUNCEBACK,) * 6)
    solid = torch.zeros(8, 8, 8, dtype=torch.bool)
    solid[3:5, 2:6, 4:7] = True
    f = lbm.W.view(19, 1, 1, 1).expand(19, 8, 8, 8).clone()
    for t in range(4):
        f, rho, u = lbm.lbm_step(lat, p, f, solid, t)
    assert (f - lbm.W.view(19, 1, 1, 1)).abs().max() < 1e-16


def _poiseuille(tau, H, steps):
    lat = Lattice(1, H, 1)
    g = 1e-5
    p = LBMParams(tau=tau, force=(g, 0.0, 0.0), bc=(PERIODIC, PERIODIC, BOUNCEBACK, BOUNCEBACK, PERIODIC, PERIODIC))
    f = lbm.W.view(19, 1, 1, 1).expand(19, 1, H, 1).clone()
    for t in range(steps):
        f, rho, u = lbm.lbm_step(lat, p, f, t=t)
    nu = (tau - 0.5) / 3.0
    y = torch.arange(H, dtype=DT) + 0.5  # halfway walls at -1/2 and H - 1/2
    exact = g / (2.0 * nu) * y * (H - y)
    return u[0, 0, :, 0], exact


def test_poiseuille_exact_at_magic_tau():
    # BGK with halfway bounce-back puts the wall exactly halfway when
    # (tau - 1/2)^2 = 3/16, so the parabolic profile is reproduced to round-off.
    u, exact = _poiseuille(0.5 + math.sqrt(3.0 / 16.0), 8, 1500)
    assert ((u - exact).abs().max() / exact.max()).item() < 1e-10


def test_poiseuille_second_order_at_tau_06():
    u, exact = _poiseuille(0.6, 12, 2500)
    assert ((u - exact).abs().max() / exact.max()).item() < 1e-2


def test_shear_wave_decay():
    n = 32
    lat = Lattice(4, n, 4)
    tau = 0.8
    p = LBMParams(tau=tau)
    U = 1e-3
    k = 2 * math.pi / n
    y = torch.arange(n, dtype=DT)
    u = torch.zeros(3, 4, n, 4, dtype=DT)
    u[0] = U * torch.sin(k * y)[None, :, None]
    f = lbm.equilibrium(torch.ones(4, n, 4, dtype=DT), u)
    steps = 200
    for t in range(steps):
        f, rho, uo = lbm.lbm_step(lat, p, f, t=t)
    nu = (tau - 0.5) / 3.0
    amp = (uo[0, 0, :, 0] * torch.sin(k * y)).sum() * 2 / n
    expect = U * math.exp(-nu * k * k * steps)
    assert abs(amp.item() - expect) / expect < 1e-2


def test_voxelize_matches_brute_force():
    lat = Lattice(6, 5, 7, dx=0.1, origin=(0.05, -0.1, 0.0))
    x = torch.tensor(scenes.random_particles_in_box(3, 60, [0.0, -0.2, -0.1], [0.7, 0.5, 0.8]))
    assert torch.equal(lbm.voxelize(lat, x), lbm.voxelize_brute(lat, x))


def test_inlet_gust_profile():
    lat = Lattice(4, 8, 6)
    p = LBMParams(u_in=(0.08, 0.0, 0.0), gust_amp=0.05, gust_period=200.0, gust_ky=1.0, gust_phase=0.3)
    u = lbm.inlet_velocity(lat, p, 17)
    j = 3
    expect = 0.08 * (1 + 0.05 * math.sin(2 * math.pi * (17 / 200 + j / 8) + 0.3))
    assert abs(u[0, 2, j].item() - expect) < 1e-16
    assert u[1].abs().max() == 0


def test_two_part_voxel_decision():
    """The voxel index from a reference plus a displacement reduces to the
    one-part rule for a zero displacement and equals the exact cell away
    from cell faces."""
    lat = lbm.Lattice(16, 12, 10, 1.0 / 16, (0.0, 0.1, 0.2))
    rng = np.random.default_rng(42)
    xr = torch.tensor(rng.uniform(0.1, 0.7, (3000, 3))).float()
    d = torch.tensor(1e-2 * rng.standard_normal((3000, 3))).float()
    assert torch.equal(lbm.voxelize(lat, torch.zeros_like(xr), x_ref=xr), lbm.voxelize(lat, xr))
    q = (xr.double() + d.double() - torch.tensor(lat.origin, dtype=torch.float64)) / lat.dx
    far = ((q - torch.round(q)).abs() > 1e-5).all(dim=1)
    assert torch.equal(lbm.voxelize(lat, d[far], x_ref=xr[far]), lbm.voxelize(lat, (xr.double() + d.double())[far]))
