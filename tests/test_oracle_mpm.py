"""Pins of the float64 MPM oracle against facts fixed by the mathematics.

Each test would fail on a plausible slip in oracle/mpm.py (a dropped stress
term, a sign or index error, a transposed operand, a wrong weight)."""
import math

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


def _rand_rot(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)
    return torch.tensor(R)


def _grid(res=16):
    return Grid(res, res, res, 1.0 / res)


def _particles(seed, n, grid, lo=0.3, hi=0.7):
    x = torch.tensor(scenes.random_particles_in_box(seed, n, [lo] * 3, [hi] * 3))
    v, C, F = scenes.random_state(seed + 100, n)
    return x, torch.tensor(v), torch.tensor(C), torch.tensor(F)


def test_weights_moments():
    grid = _grid(16)
    x, *_ = _particles(1, 500, grid)
    base, fx, w = mpm.stencil(x, grid)
    assert torch.all((fx >= 0.5) & (fx < 1.5))
    wsum = torch.zeros(500)
    first = torch.zeros(500, 3)
    second = torch.zeros(500, 3, 3)
    for o in mpm._offsets():
        ww = w[:, o[0], 0] * w[:, o[1], 1] * w[:, o[2], 2]
        d = (torch.tensor(o, dtype=DT) - fx) * grid.dx
        wsum += ww
        first += ww[:, None] * d
        second += ww[:, None, None] * d[:, :, None] * d[:, None, :]
    assert torch.allclose(wsum, torch.ones(500), atol=1e-14, rtol=0)
    assert first.abs().max() < 1e-15
    target = torch.eye(3) * grid.dx ** 2 / 4.0
    assert (second - target).abs().max() < 1e-15


def test_weights_brute_force():
    grid = Grid(8, 8, 8, 1.0 / 8)
    x, *_ = _particles(2, 5, grid, 0.3, 0.7)
    pos = mpm.node_positions(grid)
    base, fx, w = mpm.stencil(x, grid)
    for p in range(5):
        dense = torch.zeros(grid.n_nodes)
        for o in mpm._offsets():
            idx = mpm._node_index(grid, base[p:p + 1], o)
            dense[idx] += w[p, o[0], 0] * w[p, o[1], 1] * w[p, o[2], 2]
        brute = torch.tensor([
            mpm.bspline_1d((x[p, 0] - q[0]).item() / grid.dx)
            * mpm.bspline_1d((x[p, 1] - q[1]).item() / grid.dx)
            * mpm.bspline_1d((x[p, 2] - q[2]).item() / grid.dx) for q in pos])
        assert (dense - brute).abs().max() < 1e-14


def test_lame():
    mu, lam = mpm.lame(1e4, 0.3)
    # shear and bulk moduli of linear elasticity: K = lam + 2 mu / 3 = E / (3 (1 - 2 nu))
    assert abs(mu.item() - 1e4 / 2.6) < 1e-9
    assert abs((lam + 2 * mu / 3).item() - 1e4 / (3 * 0.4)) < 1e-9


def test_polar_matches_svd():
    rng = np.random.default_rng(3)
    F = torch.eye(3) + 0.3 * torch.tensor(rng.standard_normal((64, 3, 3)))
    F = F[torch.linalg.det(F) > 0]
    R = mpm.polar_rotation(F)
    U, S, Vh = torch.linalg.svd(F)
    R_svd = U @ Vh
    assert (R - R_svd).abs().max() < 1e-12
    assert mpm.polar_rotation(torch.eye(3)[None]).sub(torch.eye(3)).abs().max() == 0


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_stress_zero_on_rotations_and_symmetric(material):
    rng = np.random.default_rng(4)
    R = _rand_rot(rng, 32)
    P = mpm.pk1_stress(R, torch.full((32,), 3.0), torch.full((32,), 5.0), material)
    assert P.abs().max() < 1e-12
    F = torch.eye(3) + 0.2 * torch.tensor(rng.standard_normal((32, 3, 3)))
    tau = mpm.kirchhoff_stress(F, torch.full((32,), 3.0), torch.full((32,), 5.0), material)
    assert (tau - tau.transpose(1, 2)).abs().max() < 1e-12


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_stress_is_energy_derivative(material):
    rng = np.random.default_rng(5)
    F = torch.eye(3) + 0.2 * torch.tensor(rng.standard_normal((8, 3, 3)))
    mu, lam = torch.full((8,), 2.0), torch.full((8,), 3.0)
    P = mpm.pk1_stress(F, mu, lam, material)
    h = 1e-6
    P_fd = torch.zeros_like(F)
    for a in range(3):
        for b in range(3):
            Fp = F.clone()
            Fm = F.clone()
            Fp[:, a, b] += h
            Fm[:, a, b] -= h
            P_fd[:, a, b] = (mpm.energy_density(Fp, mu, lam, material)
                             - mpm.energy_density(Fm, mu, lam, material)) / (2 * h)
    assert ((P - P_fd).abs().max() / P.abs().max()) < 1e-8


def _scene_state(seed=7, n=400, res=16):
    grid = _grid(res)
    x, v, C, F = _particles(seed, n, grid)
    mass = torch.tensor(np.random.default_rng(seed).uniform(0.5, 2.0, n))
    vol0 = torch.tensor(np.random.default_rng(seed + 1).uniform(0.5, 2.0, n)) * 1e-4
    mu = torch.full((n,), 50.0)
    lam = torch.full((n,), 70.0)
    return grid, x, v, C, F, mass, vol0, mu, lam


def _eps_C(C):
    # vector with components eps_abc C_cb
    return torch.stack([C[:, 2, 1] - C[:, 1, 2], C[:, 0, 2] - C[:, 2, 0], C[:, 1, 0] - C[:, 0, 1]], 1)


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_p2g_conserves_mass_and_momenta(material):
    grid, x, v, C, F, mass, vol0, mu, lam = _scene_state()
    gm, gmv = mpm.p2g(grid, x, v, C, F, mass, vol0, mu, lam, 1e-3, material)
    assert abs(gm.sum() - mass.sum()) / mass.sum() < 1e-13
    P = (mass[:, None] * v).sum(0)
    assert (gmv.sum(0) - P).abs().max() / P.abs().max() < 1e-12
    xi = mpm.node_positions(grid)
    L_grid = torch.cross(xi, gmv, dim=1).sum(0)
    L_part = (mass[:, None] * (torch.cross(x, v, dim=1)
                               + grid.dx ** 2 / 4.0 * _eps_C(C))).sum(0)
    assert (L_grid - L_part).abs().max() / L_part.abs().max() < 1e-11


def test_g2p_momenta_and_affine_reproduction():
    grid, x, v, C, F, mass, vol0, mu, lam = _scene_state(8)
    rng = np.random.default_rng(9)
    gv = torch.tensor(rng.standard_normal((grid.n_nodes, 3)))
    gm, _ = mpm.p2g(grid, x, v, C, F, mass, vol0, mu, lam, 0.0, FIXED_COROTATED)
    x1, vp, Cp, F1 = mpm.g2p(grid, gv, x, F, 1e-3)
    P_grid = (gm[:, None] * gv).sum(0)
    P_part = (mass[:, None] * vp).sum(0)
    assert (P_grid - P_part).abs().max() / P_grid.abs().max() < 1e-12
    xi = mpm.node_positions(grid)
    L_grid = torch.cross(xi, gm[:, None] * gv, dim=1).sum(0)
    L_part = (mass[:, None] * (torch.cross(x, vp, dim=1) + grid.dx ** 2 / 4.0 * _eps_C(Cp))).sum(0)
    assert (L_grid - L_part).abs().max() / L_grid.abs().max() < 1e-11
    # affine field v(x) = a + B x is reproduced exactly: v_p = a + B x_p, C_p = B
    a = torch.tensor([0.3, -0.2, 0.1])
    B = torch.tensor(rng.standard_normal((3, 3)))
    gv_aff = a + xi @ B.T
    x2, vp2, Cp2, F2 = mpm.g2p(grid, gv_aff, x, F, 1e-3)
    assert (vp2 - (a + x @ B.T)).abs().max() < 1e-13
    assert (Cp2 - B).abs().max() < 1e-12
    assert (x2 - (x + 1e-3 * vp2)).abs().max() < 1e-15
    assert (F2 - (torch.eye(3) + 1e-3 * B) @ F).abs().max() < 1e-13


@pytest.mark.parametrize("material", [FIXED_COROTATED, NEO_HOOKEAN])
def test_rest_state_is_bit_exact(material):
    sc = scenes.sheet_scene(seed=0, n=2000)
    grid = Grid(**{k: sc.grid[k] for k in ("nx", "ny", "nz", "dx", "origin")})
    x = torch.tensor(sc.x)
    n = x.shape[0]
    st = {"x": x, "v": torch.zeros(n, 3), "C": torch.zeros(n, 3, 3), "F": torch.eye(3).repeat(n, 1, 1)}
    mu, lam = mpm.particle_mu_lam(torch.tensor(sc.E), torch.tensor(sc.nu), torch.tensor(sc.region).long())
    out, _ = mpm.substep(grid, st, torch.tensor(sc.mass), torch.tensor(sc.vol0), mu, lam, sc.dt,
                         material, gravity=(0.0, 0.0, 0.0), pin=torch.tensor(sc.pin))
    for k in ("x", "v", "C", "F"):
        assert torch.equal(out[k], st[k]), k


def test_free_flight_and_translation():
    grid, x, v, C, F, mass, vol0, mu, lam = _scene_state(11)
    n = x.shape[0]
    eye = torch.eye(3).repeat(n, 1, 1)
    g = (0.0, -9.8, 0.0)
    st = {"x": x, "v": torch.zeros(n, 3), "C": torch.zeros(n, 3, 3), "F": eye}
    dt = 1e-3
    out, _ = mpm.substep(grid, st, mass, vol0, mu, lam, dt, FIXED_COROTATED, gravity=g, bound=0)
    assert (out["v"] - torch.tensor(g) * dt).abs().max() < 1e-15
    assert out["C"].abs().max() < 1e-12
    v0 = torch.tensor([0.2, -0.1, 0.05])
    st = {"x": x, "v": v0.repeat(n, 1), "C": torch.zeros(n, 3, 3), "F": eye}
    out, _ = mpm.substep(grid, st, mass, vol0, mu, lam, dt, NEO_HOOKEAN, bound=0)
    assert (out["v"] - v0).abs().max() < 1e-14
    assert out["C"].abs().max() < 1e-11
    assert (out["x"] - (x + dt * v0)).abs().max() < 1e-15


def test_walls_and_pins():
    grid = Grid(8, 8, 8, 1.0 / 8)
    gm = torch.ones(grid.n_nodes)
    gmv = torch.tensor([[-1.0, 1.0, 2.0]]).repeat(grid.n_nodes, 1)
    pin = torch.zeros(grid.n_nodes, dtype=torch.uint8)
    pin[5 + 8 * (5 + 8 * 5)] = 1
    v = mpm.grid_update(grid, gm, gmv, 0.0, pin=pin, bound=2)
    n = torch.arange(grid.n_nodes)
    i, j, k = n % 8, (n // 8) % 8, n // 64
    free = pin == 0
    assert torch.all(v[i < 2, 0] == 0) and torch.all(v[(i >= 2) & free, 0] == -1.0)
    assert torch.all(v[j >= 6, 1] == 0) and torch.all(v[(j < 6) & free, 1] == 1.0)
    assert torch.all(v[k >= 6, 2] == 0)
    assert torch.all(v[pin.bool()] == 0)
    gm[0] = 0.0
    v = mpm.grid_update(grid, gm, gmv, 1.0, gravity=(0, -9.8, 0))
    assert torch.all(v[0] == 0)


def test_sort_keys_brute_force():
    grid = Grid(16, 12, 20, 1.0 / 16)
    x = torch.tensor(scenes.random_particles_in_box(12, 300, [0.2, 0.2, 0.2], [0.5, 0.5, 1.0]))
    keys = mpm.cell_tile_keys(x, grid)
    TX, TY = 4, 3
    for p in range(300):
        b = [math.floor(x[p, a].item() / grid.dx - 0.5) // 4 for a in range(3)]
        assert keys[p].item() == b[0] + TX * (b[1] + TY * b[2])
    tiles = set(mpm.active_node_tiles(x, grid))
    base, _, _ = mpm.stencil(x, grid)
    brute = set()
    for p in range(300):
        for o in mpm._offsets():
            node = [base[p, a].item() + o[a] for a in range(3)]
            brute.add(node[0] // 4 + TX * (node[1] // 4 + TY * (node[2] // 4)))
    assert tiles == brute


def test_autograd_matches_finite_differences():
    """Reverse mode of a 6-substep rollout w.r.t. the wind force grid and E."""
    from oracle import wind
    grid = Grid(8, 8, 8, 1.0 / 8)
    n = 40
    x0 = torch.tensor(scenes.random_particles_in_box(13, n, [0.35] * 3, [0.65] * 3))
    mass = torch.full((n,), 1.0 / n)
    vol0 = torch.full((n,), 1.0 / n)
    region = torch.tensor([p % 2 for p in range(n)])
    nu = torch.tensor([0.3, 0.3])
    W = torch.tensor(scenes.smooth_force_field(14, K=2, nw=4, amp=2.0)).requires_grad_(True)
    E = torch.tensor([3.0, 6.0], requires_grad=True)

    def loss_fn(W, E):
        mu, lam = mpm.particle_mu_lam(E, nu, region)
        st = {"x": x0, "v": torch.zeros(n, 3), "C": torch.zeros(n, 3, 3), "F": torch.eye(3).repeat(n, 1, 1)}
        for s in range(6):
            acc = wind.force_grid_to_nodes(grid, W[s // 3], (4, 4, 4), (0, 0, 0), (1, 1, 1))
            st, _ = mpm.substep(grid, st, mass, vol0, mu, lam, 2e-3, FIXED_COROTATED,
                                gravity=(0, -2.0, 0), acc=acc, bound=0)
        return ((st["x"] - x0) ** 2).sum() * 1e4 + ((st["F"] - torch.eye(3)) ** 2).sum()

    L = loss_fn(W, E)
    gW, gE = torch.autograd.grad(L, (W, E))
    h = 1e-6
    rng = np.random.default_rng(15)
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in W.shape)
        Wp = W.detach().clone()
        Wm = W.detach().clone()
        Wp[idx] += h
        Wm[idx] -= h
        fd = (loss_fn(Wp, E) - loss_fn(Wm, E)) / (2 * h)
        assert abs(fd - gW[idx]) <= 1e-6 * max(1.0, abs(gW[idx].item())) + 1e-9
    for r in range(2):
        hE = 1e-3 * E[r].item()  # the E-gradient is small; a larger step keeps FD above round-off
        Ep = E.detach().clone()
        Em = E.detach().clone()
        Ep[r] += hE
        Em[r] -= hE
        fd = (loss_fn(W, Ep) - loss_fn(W, Em)) / (2 * hE)
        assert abs(fd - gE[r]) <= 1e-6 * max(abs(gE[r].item()), 1e-6)


def test_two_part_stencil_decision():
    """With a position reference the float32 base decision is taken from the
    two parts; it reduces to the one-part decision for a zero displacement
    and equals the exact floor away from cell boundaries."""
    grid = Grid(32, 32, 32, 1.0 / 32)
    rng = np.random.default_rng(41)
    xr = torch.tensor(rng.uniform(0.2, 0.8, (4000, 3))).float()
    d = torch.tensor(1e-2 * rng.standard_normal((4000, 3))).float()
    assert torch.equal(mpm.stencil_base_f32(torch.zeros_like(xr), grid, xref32=xr), mpm.stencil_base_f32(xr, grid))
    got = mpm.stencil_base_f32(d, grid, xref32=xr)
    X = (xr.double() + d.double()) / grid.dx - 0.5
    exact = torch.floor(X).long()
    far = ((X - torch.round(X)).abs() > 1e-5).all(dim=1)
    assert far.sum() > 3900
    assert torch.equal(got[far], exact[far])
