"""Pins of the wind-to-grid and surrogate-convolution oracles."""
import math

import numpy as np
import pytest
import torch

from oracle import conv, wind
from oracle import mpm as ompm
from oracle.mpm import Grid, node_positions

DT = torch.float64


def test_trilinear_reproduces_linear_field():
    grid = Grid(10, 9, 8, 0.1)
    nw = (5, 4, 6)
    lo, hi = (0.0, 0.0, 0.0), (0.9, 0.8, 0.7)
    g = [torch.linspace(lo[a], hi[a], nw[a], dtype=DT) for a in range(3)]
    Z, Y, X = torch.meshgrid(g[2], g[1], g[0], indexing="ij")
    a = torch.tensor([0.3, -1.0, 2.0], dtype=DT)
    B = torch.tensor([[1.0, 2.0, -0.5], [0.0, 1.5, 0.25], [-2.0, 0.1, 0.3]], dtype=DT)
    P = torch.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], 1)
    Wf = (a + P @ B.T).T.contiguous()
    acc = wind.force_grid_to_nodes(grid, Wf, nw, lo, hi)
    pos = node_positions(grid)
    assert (acc - (a + pos @ B.T)).abs().max() < 1e-13


def test_trilinear_partition_of_unity_and_clamp():
    grid = Grid(12, 12, 12, 0.1)
    nw = (4, 4, 4)
    Wf = torch.ones(3, 64, dtype=DT) * 2.5
    acc = wind.force_grid_to_nodes(grid, Wf, nw, (0.2, 0.2, 0.2), (0.8, 0.8, 0.8))
    assert (acc - 2.5).abs().max() < 1e-15
    # a node below the box reads the box corner value
    Wr = torch.arange(3 * 64, dtype=DT).view(3, 64)
    acc = wind.force_grid_to_nodes(grid, Wr, nw, (0.2, 0.2, 0.2), (0.8, 0.8, 0.8))
    assert torch.equal(acc[0], Wr[:, 0])


def test_trilinear_single_point_by_hand():
    grid = Grid(4, 4, 4, 0.25)
    nw = (3, 3, 3)
    rng = np.random.default_rng(0)
    Wf = torch.tensor(rng.standard_normal((3, 27)))
    acc = wind.force_grid_to_nodes(grid, Wf, nw, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    # node (1, 2, 3) sits at (0.25, 0.5, 0.75) -> wind coords (0.5, 1.0, 1.5)
    node = 1 + 4 * (2 + 4 * 3)
    q = (0.5, 1.0, 1.5)
    ref = torch.zeros(3, dtype=DT)
    for k in range(3):
        for j in range(3):
            for i in range(3):
                wx = max(0.0, 1 - abs(q[0] - i))
                wy = max(0.0, 1 - abs(q[1] - j))
                wz = max(0.0, 1 - abs(q[2] - k))
                ref += wx * wy * wz * Wf[:, i + 3 * (j + 3 * k)]
    assert (acc[node] - ref).abs().max() < 1e-15


def test_drag_uniform_flow_and_outside():
    grid = Grid(8, 8, 8, 1.0 / 8)
    dims = (4, 4, 4)
    u = torch.zeros(3, 64, dtype=DT)
    u[0] = 0.05
    u[2] = -0.02
    a = wind.lbm_drag_to_nodes(grid, dims, 0.125, (0.25, 0.25, 0.25), u, 20.0, 9.8)
    pos = node_positions(grid)
    inside = ((pos >= 0.25 - 1e-12) & (pos <= 0.25 + 3 * 0.125 + 1e-12)).all(1)
    up = torch.tensor([1.0, 0.0, -0.4], dtype=DT)
    ref = 9.8 * up.norm() * up
    assert (a[inside] - ref).abs().max() < 1e-13
    assert a[~inside].abs().max() == 0
    # still air gives no force and a finite gradient
    u0 = torch.zeros(3, 64, dtype=DT, requires_grad=True)
    a0 = wind.lbm_drag_to_nodes(grid, dims, 0.125, (0.25, 0.25, 0.25), u0, 20.0, 9.8)
    (g,) = torch.autograd.grad(a0.sum(), u0)
    assert torch.isfinite(g).all() and a0.abs().max() == 0


def test_relative_drag():
    """Relative drag: equals the absolute drag for a node at rest, vanishes
    for a node moving with the wind, opposes the slip, and enters the grid
    update as an acceleration evaluated at v* = mv / m."""
    grid = Grid(8, 8, 8, 1.0 / 8)
    dims = (4, 4, 4)
    rng = np.random.default_rng(3)
    u = torch.tensor(0.05 * rng.standard_normal((3, 64)))
    args = (grid, dims, 0.125, (0.25, 0.25, 0.25), u, 20.0)
    U, inside = wind.lbm_velocity_to_nodes(*args)
    a_abs = wind.lbm_drag_to_nodes(*args, 9.8)
    zero = torch.zeros_like(U)
    assert (wind.relative_drag(U, zero, inside, 9.8) - a_abs).abs().max() < 1e-13
    assert wind.relative_drag(U, U, inside, 9.8).abs().max() == 0
    v = torch.tensor(rng.standard_normal(U.shape))
    a = wind.relative_drag(U, v, inside, 9.8)
    assert ((a * (U - v)).sum(1) >= 0).all()
    assert a[~inside].abs().max() == 0
    # one node by hand: |r| r with r = U - v
    i = int(torch.nonzero(inside)[5])
    r = U[i] - v[i]
    assert (a[i] - 9.8 * r.norm() * r).abs().max() < 1e-14
    # in the grid update
    N = grid.n_nodes
    m = torch.tensor(rng.uniform(0.5, 2.0, N))
    mv = m[:, None] * v
    dt = 1e-3
    vo = ompm.grid_update(grid, m, mv, dt, (0.0, -9.8, 0.0), bound=0, drag_rel=(U, inside, 9.8))
    ref = v + dt * (torch.tensor([0.0, -9.8, 0.0], dtype=DT) + a)
    assert (vo - ref).abs().max() < 1e-14
    # its derivative with respect to the momentum, against central differences
    mvv = mv.clone().requires_grad_(True)
    w = torch.tensor(rng.standard_normal((N, 3)))
    (gmv,) = torch.autograd.grad((ompm.grid_update(grid, m, mvv, dt, bound=0, drag_rel=(U, inside, 9.8)) * w).sum(),
                                 mvv)
    h = 1e-6
    for node in (i, int(torch.nonzero(inside)[20])):
        for c in range(3):
            p, q = mv.clone(), mv.clone()
            p[node, c] += h
            q[node, c] -= h
            fp = (ompm.grid_update(grid, m, p, dt, bound=0, drag_rel=(U, inside, 9.8)) * w).sum()
            fm = (ompm.grid_update(grid, m, q, dt, bound=0, drag_rel=(U, inside, 9.8)) * w).sum()
            assert abs((fp - fm).item() / (2 * h) - gmv[node, c].item()) < 1e-6


def test_conv_direct_matches_library():
    rng = np.random.default_rng(1)
    x = torch.tensor(rng.standard_normal((2, 3, 5, 4, 6)))
    w = torch.tensor(rng.standard_normal((4, 3, 3, 3, 3)))
    b = torch.tensor(rng.standard_normal(4))
    ref = torch.nn.functional.conv3d(x, w, b, padding=1)
    assert (conv.conv3d_direct(x, w, b) - ref).abs().max() < 1e-12


def test_surrogate_gradients_match_fd():
    rng = np.random.default_rng(2)
    Ws = [torch.tensor(0.3 * rng.standard_normal((4, 3, 3, 3, 3)), requires_grad=True),
          torch.tensor(0.3 * rng.standard_normal((4, 4, 3, 3, 3)), requires_grad=True),
          torch.tensor(0.3 * rng.standard_normal((3, 4, 3, 3, 3)), requires_grad=True)]
    bs = [torch.tensor(0.1 * rng.standard_normal(4), requires_grad=True),
          torch.tensor(0.1 * rng.standard_normal(4), requires_grad=True),
          torch.tensor(0.1 * rng.standard_normal(3), requires_grad=True)]
    u = torch.tensor(0.05 * rng.standard_normal((2, 3, 4, 5, 3)))
    tgt = torch.tensor(0.05 * rng.standard_normal((2, 3, 4, 5, 3)))
    s = torch.tensor([0.05, 0.08], dtype=DT)

    def loss(Ws, bs):
        return ((conv.surrogate_forward(u, Ws, bs, s) - tgt) ** 2).sum()

    L = loss(Ws, bs)
    grads = torch.autograd.grad(L, Ws + bs)
    h = 1e-6
    for li, W in enumerate(Ws):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, d)) for d in W.shape)
            Wp = [w.detach().clone() for w in Ws]
            Wm = [w.detach().clone() for w in Ws]
            Wp[li][idx] += h
            Wm[li][idx] -= h
            fd = (loss(Wp, bs) - loss(Wm, bs)) / (2 * h)
            assert abs(fd.item() - grads[li][idx].item()) < 1e-8 * max(1.0, abs(fd.item()))


def test_divergence_of_analytic_fields():
    n = 10
    z, y, x = torch.meshgrid(*(torch.arange(n, dtype=DT),) * 3, indexing="ij")
    # solenoidal: u = (sin y, sin z, sin x) has zero divergence, also discretely
    u = torch.stack([torch.sin(0.3 * y), torch.sin(0.4 * z), torch.sin(0.5 * x)])
    assert conv.divergence_rms(u).item() < 1e-15
    # linear: u = (2x, -y, 3z) has divergence 4 everywhere
    u = torch.stack([2 * x, -y, 3 * z])
    assert abs(conv.divergence_rms(u).item() - 4.0) < 1e-13
    assert abs(conv.kinetic_energy(torch.ones(3, 2, 2, 2, dtype=DT)).item() - 12.0) < 1e-15


def test_adam_matches_torch_optimizer():
    """The oracle's Adam step against torch.optim.Adam over several steps."""
    rng = np.random.default_rng(3)
    p0 = torch.tensor(rng.standard_normal(50))
    grads = [torch.tensor(rng.standard_normal(50)) for _ in range(5)]
    q = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([q], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.clone(), torch.zeros(50, dtype=DT), torch.zeros(50, dtype=DT)
    for k, g in enumerate(grads):
        q.grad = g.clone()
        opt.step()
        p, m, v = conv.adam_step(p, g, m, v, 1e-2, 0.9, 0.999, 1e-8, k + 1)
    assert (p - q.detach()).abs().max() < 1e-14


def test_increment_mse_closed_form():
    u = torch.zeros(2, 3, 4, dtype=DT)
    t = torch.ones(2, 3, 4, dtype=DT)
    s = torch.tensor([1.0, 2.0], dtype=DT)
    # field 0 contributes 1 per element, field 1 contributes 1/4
    assert abs(conv.increment_mse(u, t, s).item() - 0.625) < 1e-15
