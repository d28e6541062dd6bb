"""Pins of the float64 physics-informed loss, direction metrics and LBM
guide of the wind-force reconstruction."""
import numpy as np
import torch

from oracle import recon

DT = torch.float64


def _rand(n, seed):
    return torch.tensor(np.random.default_rng(seed).standard_normal((3, n)))


def test_phys_loss_closed_forms():
    g = _rand(50, 1)
    assert recon.phys_loss(3.0 * g, g).abs() < 1e-13
    assert recon.phys_loss(-0.5 * g, g).abs() < 1e-13
    # perpendicular: one per node
    e = torch.tensor([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]], dtype=DT)
    p = torch.tensor([[0.0, 0.0], [2.0, 0.0], [0.0, -1.0]], dtype=DT)
    assert abs(recon.phys_loss(p, e).item() - 2.0) < 1e-15
    # 45 degrees: sin^2 = 1/2
    a = torch.tensor([[1.0], [1.0], [0.0]], dtype=DT)
    b = torch.tensor([[1.0], [0.0], [0.0]], dtype=DT)
    assert abs(recon.phys_loss(a, b).item() - 0.5) < 1e-15
    # lengths do not matter, zero vectors are skipped
    W = _rand(40, 2)
    s = torch.tensor(np.random.default_rng(3).uniform(0.1, 10, 40))
    assert abs(recon.phys_loss(W * s, g[:, :40]) - recon.phys_loss(W, g[:, :40])) < 1e-12
    W[:, 5] = 0.0
    ref = recon.phys_loss(torch.cat([W[:, :5], W[:, 6:]], 1), torch.cat([g[:, :5], g[:, 6:40]], 1))
    assert abs(recon.phys_loss(W, g[:, :40]) - ref) < 1e-12
    # and such a node has a zero (finite) gradient
    Wv = W.clone().requires_grad_(True)
    recon.phys_loss(Wv, g[:, :40]).backward()
    assert torch.isfinite(Wv.grad).all() and Wv.grad[:, 5].abs().max() == 0


def test_phys_loss_gradient_matches_central_differences():
    W = _rand(12, 4).requires_grad_(True)
    g = _rand(12, 5)
    recon.phys_loss(W, g).backward()
    h = 1e-6
    Wd = W.detach()
    for i in range(3):
        for j in (0, 5, 11):
            Wp, Wm = Wd.clone(), Wd.clone()
            Wp[i, j] += h
            Wm[i, j] -= h
            fd = (recon.phys_loss(Wp, g) - recon.phys_loss(Wm, g)) / (2 * h)
            assert abs(fd.item() - W.grad[i, j].item()) < 1e-7


def test_direction_metrics():
    a = _rand(30, 6)
    c, m, n = recon.direction_metrics(a, 2.0 * a)
    assert abs(c - 1) < 1e-15 and m < 1e-30 and n == 30
    c, m, _ = recon.direction_metrics(a, -a)
    assert abs(c + 1) < 1e-15 and abs(m - 4) < 1e-14
    b = _rand(30, 7)
    c, m, _ = recon.direction_metrics(a, b)
    assert abs(m - (2 - 2 * c)) < 1e-14
    b[:, 3] = 0
    _, _, n = recon.direction_metrics(a, b)
    assert n == 29


def test_guide_reproduces_linear_field():
    lat_dims = (10, 8, 6)
    nx, ny, nz = lat_dims
    dx = 0.1
    origin = (0.05, -0.1, 0.0)
    z, y, x = torch.meshgrid(torch.arange(nz, dtype=DT), torch.arange(ny, dtype=DT), torch.arange(nx, dtype=DT),
                             indexing="ij")
    px, py, pz = origin[0] + dx * x, origin[1] + dx * y, origin[2] + dx * z
    u = torch.stack([0.1 + 0.2 * px - 0.3 * pz, py, 0.5 * px + py]).reshape(3, -1)
    nw, lo, hi = (5, 4, 3), (0.1, 0.0, 0.1), (0.9, 0.5, 0.45)
    g = recon.guide_from_lattice(nw, lo, hi, lat_dims, dx, origin, u)
    pos = recon.wind_grid_positions(nw, lo, hi)
    ref = torch.stack([0.1 + 0.2 * pos[:, 0] - 0.3 * pos[:, 2], pos[:, 1], 0.5 * pos[:, 0] + pos[:, 1]])
    assert (g - ref).abs().max() < 1e-14
    # a node outside the lattice box gets no guide
    g2 = recon.guide_from_lattice((2, 2, 2), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5), lat_dims, dx, origin, u)
    assert g2[:, 0].abs().max() == 0
