"""Pins of the float64 HOME-LBM oracle (moment-encoded D3Q19 step) against
the Hermite expansion written in general tensor form, invariants, the
collision's relaxation rates, and closed-form flows."""
import math

import numpy as np
import pytest
import torch

from oracle import home, lbm
from oracle.lbm import BOUNCEBACK, INLET, OUTLET, PERIODIC, Lattice, LBMParams

DT = torch.float64


def _random_moments(shape, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * torch.tensor(rng.standard_normal(shape))
    u = amp * torch.tensor(rng.standard_normal((3,) + shape))
    S = torch.stack([u[a] * u[b] for a, b in home.S_PAIRS]) + 1e-3 * torch.tensor(rng.standard_normal((6,) + shape))
    return rho, u, S


def test_expansion_matches_general_tensor_form():
    """f_i = w_i rho sum_n H^(n)(c_i) : a^(n) / (n! c_s^(2n)) over all index
    tuples, with a^(1) = u, a^(2) = S and the full recursive third-order
    tensor a_abc = S_ab u_c + S_bc u_a + S_ac u_b - 2 u_a u_b u_c; on D3Q19
    H_xxx and H_xyz vanish, which leaves the six classes of the oracle."""
    rho, u, S = _random_moments((7,), 1)
    c = lbm.C.to(DT)
    cs2 = 1.0 / 3.0
    I = torch.eye(3, dtype=DT)
    H1 = c
    H2 = c[:, :, None] * c[:, None, :] - cs2 * I
    H3 = (c[:, :, None, None] * c[:, None, :, None] * c[:, None, None, :]
          - cs2 * (c[:, :, None, None] * I[None, None] + c[:, None, :, None] * I[None, :, None, :]
                   + c[:, None, None, :] * I[None, :, :, None]))
    Sm = torch.zeros(3, 3, 7, dtype=DT)
    for s, (a, b) in enumerate(home.S_PAIRS):
        Sm[a, b] = S[s]
        Sm[b, a] = S[s]
    a3 = (torch.einsum("abn,cn->abcn", Sm, u) + torch.einsum("bcn,an->abcn", Sm, u)
          + torch.einsum("acn,bn->abcn", Sm, u) - 2.0 * torch.einsum("an,bn,cn->abcn", u, u, u))
    series = (1.0 + torch.einsum("qa,an->qn", H1, u) / cs2 + torch.einsum("qab,abn->qn", H2, Sm) / (2 * cs2 ** 2)
              + torch.einsum("qabc,abcn->qn", H3, a3) / (6 * cs2 ** 3))
    ref = lbm.W[:, None] * rho[None] * series
    assert (home.populations(rho, u, S) - ref).abs().max() < 1e-15


def test_expansion_reproduces_lower_moments():
    rho, u, S = _random_moments((4, 3, 5), 2)
    f = home.populations(rho, u, S)
    r2, u2, S2 = home.moments(f, (0.0, 0.0, 0.0))
    assert (r2 - rho).abs().max() < 1e-14
    assert (u2 - u).abs().max() < 1e-14
    assert (S2 - S).abs().max() < 1e-14


def test_equilibrium_expansion_is_the_bgk_equilibrium_to_second_order():
    """With S = u u the expansion differs from the quadratic BGK equilibrium
    only by the third-order terms, which are O(u^3)."""
    rng = np.random.default_rng(3)
    rho = 1.0 + 0.01 * torch.tensor(rng.standard_normal(6))
    udir = torch.tensor(rng.standard_normal((3, 6)))
    d = []
    for scale in (1e-2, 1e-3):
        u = scale * udir
        d.append((home.populations(*home.equilibrium_moments(rho, u)) - lbm.equilibrium(rho, u)).abs().max().item())
    assert 0.9e3 < d[0] / d[1] < 1.1e3


def test_collision_relaxation_rates():
    """Without force: the deviatoric non-equilibrium part of S decays by
    (1 - 1/tau), a trace excess is removed at once, equilibrium is a fixed
    point; rho and u pass unchanged."""
    rng = np.random.default_rng(4)
    n = 5
    rho = 1.0 + 0.01 * torch.tensor(rng.standard_normal(n))
    u = 0.05 * torch.tensor(rng.standard_normal((3, n)))
    Seq = home.equilibrium_moments(rho, u)[2]
    D = torch.tensor(rng.standard_normal((6, n))) * 1e-3
    D[:3] -= D[:3].mean(dim=0, keepdim=True)   # traceless
    tau = 0.7
    zero = (0.0, 0.0, 0.0)
    up, Sp = home.collide(rho, u, Seq + D, tau, zero)
    assert (up - u).abs().max() < 1e-17
    assert (Sp - (Seq + (1 - 1 / tau) * D)).abs().max() < 1e-16
    trace = torch.zeros(6, n, dtype=DT)
    trace[:3] = 2e-3
    _, Sp = home.collide(rho, u, Seq + trace, tau, zero)
    assert (Sp - Seq).abs().max() < 1e-16


def test_collision_force_terms_are_guo_source():
    """With a force, the post-collision second moment gains
    (1 - 1/(2 tau)) (F u + u F) / rho in its deviatoric part and
    F . u / rho in its trace (the trace relaxes at rate 1, where Guo's
    factor is 1/2); the velocity gains F / (2 rho)."""
    rng = np.random.default_rng(5)
    n = 4
    rho = 1.0 + 0.01 * torch.tensor(rng.standard_normal(n))
    u = 0.05 * torch.tensor(rng.standard_normal((3, n)))
    Seq = home.equilibrium_moments(rho, u)[2]
    F = (2e-4, -1e-4, 5e-5)
    tau = 0.9
    up, Sp = home.collide(rho, u, Seq, tau, F)
    _, S0 = home.collide(rho, u, Seq, tau, (0.0, 0.0, 0.0))
    Fv = torch.tensor(F, dtype=DT)[:, None]
    assert (up - (u + 0.5 * Fv / rho)).abs().max() < 1e-17
    G = torch.einsum("an,bn->abn", Fv.expand(3, n), u) + torch.einsum("an,bn->abn", u, Fv.expand(3, n))
    G = G / rho
    tr = G[0, 0] + G[1, 1] + G[2, 2]
    dS = Sp - S0
    for s, (a, b) in enumerate(home.S_PAIRS):
        dev = G[a, b] - (tr / 3.0 if a == b else 0.0)
        expect = (1.0 - 0.5 / tau) * dev + (0.5 * tr / 3.0 if a == b else 0.0)
        assert (dS[s] - expect).abs().max() < 1e-17, (a, b)


def test_periodic_box_conserves_mass_and_momentum():
    lat = Lattice(6, 5, 4)
    p = LBMParams(tau=0.7)
    rho, u, S = _random_moments((4, 5, 6), 6)
    m0 = rho.sum()
    j0 = (rho[None] * u).sum(dim=(1, 2, 3))
    for t in range(15):
        rho, u, S, _, _ = home.home_step(lat, p, rho, u, S, t=t)
    assert abs(rho.sum() - m0) / m0 < 1e-13
    assert ((rho[None] * u).sum(dim=(1, 2, 3)) - j0).abs().max() < 1e-13


def test_uniform_force_adds_momentum():
    lat = Lattice(4, 3, 5)
    F = (1e-4, 0.0, -2e-5)
    p = LBMParams(tau=0.8, force=F)
    rho, u, S = home.equilibrium_moments(torch.ones(5, 3, 4, dtype=DT), torch.zeros(3, 5, 3, 4, dtype=DT))
    for t in range(10):
        rho, u, S, _, _ = home.home_step(lat, p, rho, u, S, t=t)
    j = (rho[None] * u).sum(dim=(1, 2, 3)) / lat.n_nodes
    assert (j - 10 * torch.tensor(F, dtype=DT)).abs().max() < 1e-16


def test_uniform_equilibrium_stays_uniform_with_inlet_outlet():
    lat = Lattice(8, 6, 5)
    uin = (0.05, 0.01, 0.0)
    p = LBMParams(tau=0.6, u_in=uin, bc=(INLET, OUTLET, PERIODIC, PERIODIC, PERIODIC, PERIODIC))
    u0 = torch.tensor(uin, dtype=DT).view(3, 1, 1, 1).expand(3, 5, 6, 8).clone()
    rho, u, S = home.equilibrium_moments(torch.ones(5, 6, 8, dtype=DT), u0)
    S0 = S.clone()
    for t in range(5):
        rho, u, S, rr, ur = home.home_step(lat, p, rho, u, S, t=t)
    assert (u - u0).abs().max() < 1e-16
    assert (S - S0).abs().max() < 1e-16
    assert (rho - 1.0).abs().max() < 1e-15


def test_fluid_at_rest_with_obstacle_stays_at_rest():
    lat = Lattice(8, 8, 8)
    p = LBMParams(tau=0.8, bc=(BOUNCEBACK,) * 6)
    solid = torch.zeros(8, 8, 8, dtype=torch.bool)
    solid[3:5, 2:6, 4:7] = True
    rho, u, S = home.equilibrium_moments(torch.ones(8, 8, 8, dtype=DT), torch.zeros(3, 8, 8, 8, dtype=DT))
    for t in range(4):
        rho, u, S, _, _ = home.home_step(lat, p, rho, u, S, solid, t)
    assert (rho - 1).abs().max() < 1e-15 and u.abs().max() < 1e-16 and S.abs().max() < 1e-16


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
    rho, u, S = home.equilibrium_moments(torch.ones(4, n, 4, dtype=DT), u)
    steps = 200
    for t in range(steps):
        rho, u, S, _, ur = home.home_step(lat, p, rho, u, S, t=t)
    nu = (tau - 0.5) / 3.0
    amp = (ur[0, 0, :, 0] * torch.sin(k * y)).sum() * 2 / n
    expect = U * math.exp(-nu * k * k * steps)
    assert abs(amp.item() - expect) / expect < 1e-2


@pytest.mark.parametrize("tau", [0.6, 0.9])
def test_poiseuille(tau):
    H = 12
    lat = Lattice(1, H, 1)
    g = 1e-5
    p = LBMParams(tau=tau, force=(g, 0.0, 0.0), bc=(PERIODIC, PERIODIC, BOUNCEBACK, BOUNCEBACK, PERIODIC, PERIODIC))
    rho, u, S = home.equilibrium_moments(torch.ones(1, H, 1, dtype=DT), torch.zeros(3, 1, H, 1, dtype=DT))
    for t in range(3000):
        rho, u, S, _, ur = home.home_step(lat, p, rho, u, S, t=t)
    nu = (tau - 0.5) / 3.0
    y = torch.arange(H, dtype=DT) + 0.5  # halfway walls at -1/2 and H - 1/2
    exact = g / (2.0 * nu) * y * (H - y)
    err = ((ur[0, 0, :, 0] - exact).abs().max() / exact.max()).item()
    assert err < 2e-2
