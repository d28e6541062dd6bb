"""FP64 oracle: MLS-MPM substep with APIC transfers (test infrastructure only).

Follows the paper's appendix "Material Point Method" and Sec. 3.2/3.3:

* particle state is the tuple (x_p, m_p, u_p, C_p, F_p) (Appendix, MPM);
* P2G (Eq. P2G): m_i = sum_p w_ip m_p and
  m_i u_i = sum_p w_ip m_p (u_p + C_p (x_i - x_p)), plus the MLS-MPM elastic
  force term that the paper defers to MLS-MPM (Hu et al. 2018): the affine
  matrix becomes A_p = m_p C_p - dt V0_p (4/dx^2) tau_p with tau = P F^T the
  Kirchhoff stress;
* the grid update integrates the momentum equation (Eq. continuum_mechanics)
  with gravity and the wind force field F_w applied on the MPM grid nodes
  (Sec. 3, problem specification; Sec. 3.2) -- F_w is an acceleration;
* G2P (Eq. G2P): u_p = sum_i w_ip u_i, x_p += dt u_p, the APIC affine
  matrix C_p = (4/dx^2) sum_i w_ip u_i (x_i - x_p)^T;
* deformation update (Eq. deformation_update): F <- (I + dt C) F, applied
  with the C that G2P has just produced;
* constitutive models: Neo-Hookean (Eq. constitutive_model; the printed
  first Piola-Kirchhoff stress has F - F^T where the derivative of the printed
  energy gives F - F^{-T}, which is what is used) and fixed-corotated; Lame
  parameters from E and nu (Eq. young_poisson).

Quadratic B-spline weights, brute-force kernel N(r) (MLS-MPM):
N(r) = 3/4 - r^2 for |r| < 1/2, (3/2 - |r|)^2 / 2 for 1/2 <= |r| < 3/2, else 0.

Grid layout: dense, node (i, j, k) at origin + dx * (i, j, k), linear index
i + nx * (j + ny * k).  Grid vectors are (N, 3).

Parity pins (tests/test_oracle_mpm.py): partition of unity and the first and
second moments of the weights, brute force over every node for a few random
particles, P(R) = 0 for rotations, P against a central finite difference of
psi, tau symmetric, exact mass / linear / angular momentum conservation in
P2G and G2P, affine-field reproduction in G2P, rest-state invariance
(bit-exact), free flight and uniform translation, and autograd against
central finite differences.  The elastic force is pinned separately
(tests/test_oracle_stress_pins.py): the stress part of P2G's momentum equals
minus the gradient, by central differences, of the total energy
sum_p V0_p psi after a G2P deformation update driven by the grid velocities
(sign, 4/dx^2, V0, dt and tau = P F^T); the small-strain limit
P(I + e) = 2 mu sym(e) + lam tr(e) I of both models; and uniaxial stress
E e under the strain (e, -nu e, -nu e), which is what E and nu mean.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

FIXED_COROTATED = 0
NEO_HOOKEAN = 1

_DT = torch.float64


@dataclass
class Grid:
    """MPM background grid: nodes at origin + dx * (i, j, k)."""

    nx: int
    ny: int
    nz: int
    dx: float
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)


# ---------------------------------------------------------------- material

def lame(E, nu):
    """Eq. young_poisson: mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu))."""
    E = torch.as_tensor(E, dtype=_DT)
    nu = torch.as_tensor(nu, dtype=_DT)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def polar_rotation(F, max_iter: int = 60, tol: float = 1e-15):
    """Rotation factor R of the polar decomposition F = R S (det F > 0).

    Scaled Newton iteration (Higham 1986):
    X <- (zeta X + X^{-T} / zeta) / 2 with zeta = sqrt(|X^{-1}|_F / |X|_F),
    iterated until the update stalls.  F = I gives R = I exactly.
    """
    X = F
    for _ in range(max_iter):
        Xinv = torch.linalg.inv(X)
        zeta = torch.sqrt(torch.linalg.matrix_norm(Xinv) / torch.linalg.matrix_norm(X))
        zeta = zeta[..., None, None]
        Xn = 0.5 * (zeta * X + Xinv.transpose(-1, -2) / zeta)
        delta = torch.linalg.matrix_norm(Xn - X).max().item() if X.numel() else 0.0
        X = Xn
        if delta <= tol:
            break
    return X


def energy_density(F, mu, lam, material: int):
    """Hyperelastic energy psi(F).

    Neo-Hookean (Eq. constitutive_model):
      psi = mu/2 sum_i ((F^T F)_ii - 1) - mu log J + lam/2 log^2 J.
    Fixed-corotated: psi = mu |F - R|_F^2 + lam/2 (J - 1)^2.
    """
    J = torch.linalg.det(F)
    mu = torch.as_tensor(mu, dtype=_DT)
    lam = torch.as_tensor(lam, dtype=_DT)
    if material == NEO_HOOKEAN:
        trFtF = (F * F).sum(dim=(-1, -2))
        return 0.5 * mu * (trFtF - 3.0) - mu * torch.log(J) + 0.5 * lam * torch.log(J) ** 2
    R = polar_rotation(F)
    return mu * ((F - R) ** 2).sum(dim=(-1, -2)) + 0.5 * lam * (J - 1.0) ** 2


def pk1_stress(F, mu, lam, material: int):
    """First Piola-Kirchhoff stress P = d psi / d F.

    Neo-Hookean: P = mu (F - F^{-T}) + lam log J F^{-T}.
    Fixed-corotated: P = 2 mu (F - R) + lam (J - 1) J F^{-T}.
    """
    J = torch.linalg.det(F)[..., None, None]
    FinvT = torch.linalg.inv(F).transpose(-1, -2)
    mu = torch.as_tensor(mu, dtype=_DT)[..., None, None]
    lam = torch.as_tensor(lam, dtype=_DT)[..., None, None]
    if material == NEO_HOOKEAN:
        return mu * (F - FinvT) + lam * torch.log(J) * FinvT
    R = polar_rotation(F)
    return 2.0 * mu * (F - R) + lam * (J - 1.0) * J * FinvT


def kirchhoff_stress(F, mu, lam, material: int):
    """Kirchhoff stress tau = P F^T (= J sigma, Eq. continuum_mechanics)."""
    return pk1_stress(F, mu, lam, material) @ F.transpose(-1, -2)


# ----------------------------------------------------------------- weights

def bspline_1d(r):
    """Quadratic B-spline N(r) by its piecewise definition (brute force)."""
    a = abs(r)
    if a < 0.5:
        return 0.75 - a * a
    if a < 1.5:
        return 0.5 * (1.5 - a) ** 2
    return 0.0


def stencil(x, grid: Grid):
    """Stencil base node, fractional position and per-axis weights.

    X = (x - origin) / dx, base = floor(X - 1/2), fx = X - base in [1/2, 3/2);
    weights of the three nodes base + 0, 1, 2 on each axis:
    w0 = (3/2 - fx)^2 / 2, w1 = 3/4 - (fx - 1)^2, w2 = (fx - 1/2)^2 / 2.
    Returns base (n, 3) int64, fx (n, 3), w (n, 3 offsets, 3 axes).
    """
    origin = torch.tensor(grid.origin, dtype=_DT)
    X = (x - origin) / grid.dx
    base = torch.floor(X.detach() - 0.5).to(torch.int64)
    fx = X - base.to(_DT)
    w = torch.stack([0.5 * (1.5 - fx) ** 2, 0.75 - (fx - 1.0) ** 2, 0.5 * (fx - 0.5) ** 2], dim=1)
    return base, fx, w


def _offsets():
    for k in range(3):
        for j in range(3):
            for i in range(3):
                yield i, j, k


def _node_index(grid: Grid, base, o):
    i = base[:, 0] + o[0]
    j = base[:, 1] + o[1]
    k = base[:, 2] + o[2]
    if (i.min() < 0 or j.min() < 0 or k.min() < 0 or i.max() >= grid.nx
            or j.max() >= grid.ny or k.max() >= grid.nz):
        raise ValueError("particle stencil leaves the grid")
    return i + grid.nx * (j + grid.ny * k)


def node_positions(grid: Grid):
    """(N, 3) positions of all grid nodes, linear order i + nx (j + ny k)."""
    k, j, i = torch.meshgrid(torch.arange(grid.nz, dtype=_DT), torch.arange(grid.ny, dtype=_DT),
                             torch.arange(grid.nx, dtype=_DT), indexing="ij")
    pos = torch.stack([i.reshape(-1), j.reshape(-1), k.reshape(-1)], dim=1) * grid.dx
    return pos + torch.tensor(grid.origin, dtype=_DT)


# --------------------------------------------------------------- transfers

def particle_mu_lam(E, nu, region):
    mu_r, lam_r = lame(E, nu)
    return mu_r[region], lam_r[region]


def p2g(grid: Grid, x, v, C, F, mass, vol0, mu_p, lam_p, dt: float, material: int):
    """Eq. P2G with the MLS-MPM stress term.

    A_p = m_p C_p - dt V0_p (4/dx^2) tau_p;
    m_i  = sum_p w_ip m_p;
    mv_i = sum_p w_ip (m_p v_p + A_p (x_i - x_p)).
    Returns (m (N,), mv (N, 3)).
    """
    n_nodes = grid.n_nodes
    base, fx, w = stencil(x, grid)
    tau = kirchhoff_stress(F, mu_p, lam_p, material)
    A = mass[:, None, None] * C - (dt * 4.0 / grid.dx ** 2) * vol0[:, None, None] * tau
    mom = mass[:, None] * v
    gm = torch.zeros(n_nodes, dtype=_DT)
    gmv = torch.zeros(n_nodes, 3, dtype=_DT)
    for o in _offsets():
        weight = w[:, o[0], 0] * w[:, o[1], 1] * w[:, o[2], 2]
        d = (torch.tensor(o, dtype=_DT) - fx) * grid.dx
        idx = _node_index(grid, base, o)
        gm = gm.index_add(0, idx, weight * mass)
        contrib = weight[:, None] * (mom + (A @ d[:, :, None])[:, :, 0])
        gmv = gmv.index_add(0, idx, contrib)
    return gm, gmv


def grid_update(grid: Grid, gm, gmv, dt: float, gravity=(0.0, 0.0, 0.0), acc=None, pin=None,
                bound: int = 3, drag_rel=None):
    """Grid momentum update (Eq. continuum_mechanics, explicit in time).

    For m_i > 0: v_i = mv_i / m_i + dt (g + a_i), where a_i is the wind force
    field (an acceleration) at node i; otherwise v_i = 0.  Separating-slip walls
    ``bound`` nodes deep: on axis a, if i_a < bound and v_a < 0, or
    i_a >= n_a - bound and v_a > 0, then v_a = 0.  Pinned nodes get v = 0.
    ``drag_rel`` = (U (N, 3), inside (N,), k_drag) replaces ``acc`` by the
    relative drag k_D |U - v*| (U - v*) with v* = mv / m (oracle.wind).
    """
    from .wind import relative_drag
    g = torch.tensor(gravity, dtype=_DT)
    has_mass = gm > 0
    m_safe = torch.where(has_mass, gm, torch.ones_like(gm))
    vstar = gmv / m_safe[:, None]
    v = vstar + dt * g
    if acc is not None:
        v = v + dt * acc
    if drag_rel is not None:
        U, inside, k_drag = drag_rel
        v = v + dt * relative_drag(U, vstar, inside, k_drag)
    v = torch.where(has_mass[:, None], v, torch.zeros_like(v))
    n = torch.arange(grid.n_nodes)
    ijk = torch.stack([n % grid.nx, (n // grid.nx) % grid.ny, n // (grid.nx * grid.ny)], dim=1)
    dims = torch.tensor(grid.dims)
    lo = (ijk < bound) & (v < 0)
    hi = (ijk >= dims - bound) & (v > 0)
    v = torch.where(lo | hi, torch.zeros_like(v), v)
    if pin is not None:
        v = torch.where(pin.bool()[:, None], torch.zeros_like(v), v)
    return v


def g2p(grid: Grid, gv, x, F, dt: float):
    """Eq. G2P, APIC C and Eq. deformation_update (F advanced with the new C).

    v_p = sum_i w_ip v_i; C_p = (4/dx^2) sum_i w_ip v_i (x_i - x_p)^T;
    x_p <- x_p + dt v_p; F_p <- (I + dt C_p) F_p.
    """
    base, fx, w = stencil(x, grid)
    vp = torch.zeros_like(x)
    Bp = torch.zeros(x.shape[0], 3, 3, dtype=_DT)
    for o in _offsets():
        weight = w[:, o[0], 0] * w[:, o[1], 1] * w[:, o[2], 2]
        d = (torch.tensor(o, dtype=_DT) - fx) * grid.dx
        idx = _node_index(grid, base, o)
        vi = gv[idx]
        vp = vp + weight[:, None] * vi
        Bp = Bp + weight[:, None, None] * vi[:, :, None] * d[:, None, :]
    Cp = (4.0 / grid.dx ** 2) * Bp
    x_new = x + dt * vp
    eye = torch.eye(3, dtype=_DT)
    F_new = (eye + dt * Cp) @ F
    return x_new, vp, Cp, F_new


def substep(grid: Grid, state: dict, mass, vol0, mu_p, lam_p, dt: float, material: int,
            gravity=(0.0, 0.0, 0.0), acc=None, pin=None, bound: int = 3):
    """One MPM substep S (Eq. simulation_mpm): P2G, grid update, G2P.

    ``state`` holds x (n,3), v (n,3), C (n,3,3), F (n,3,3); returns the new
    state dict plus the intermediate grid fields.
    """
    gm, gmv = p2g(grid, state["x"], state["v"], state["C"], state["F"], mass, vol0, mu_p, lam_p,
                  dt, material)
    gv = grid_update(grid, gm, gmv, dt, gravity, acc, pin, bound)
    x, v, C, F = g2p(grid, gv, state["x"], state["F"], dt)
    return {"x": x, "v": v, "C": C, "F": F}, {"m": gm, "mv": gmv, "v": gv}


# ------------------------------------------------------------ cell sorting

TILE = 4


def stencil_base_f32(x32, grid: Grid, xref32=None):
    """Stencil base cell decided in float32 the way a float32 implementation
    decides it: X = (x - origin) * fl32(1/dx), base = floor(X - 1/2), each
    operation rounded to float32.  With a position reference (the position
    is xref + x, x the displacement) the coordinate is taken in two parts,
    X = fl32((xref - origin) * inv) + fl32(x * inv), rounded once more.  Used
    where the integer decision has to be taken in the kernel's precision."""
    x32 = x32.to(torch.float32)
    o = torch.tensor(grid.origin, dtype=torch.float32)
    inv = torch.tensor(1.0 / grid.dx, dtype=torch.float32)
    if xref32 is None:
        X = (x32 - o) * inv
    else:
        X = (xref32.to(torch.float32) - o) * inv + x32 * inv
    return torch.floor(X - torch.tensor(0.5, dtype=torch.float32)).to(torch.int64)


def cell_tile_keys(x, grid: Grid, base=None):
    """Sort key of each particle: linear index of the 4x4x4 tile of its stencil
    base cell, tile (bx, by, bz) = base // 4, key = bx + TX (by + TY bz) with
    TX = ceil(nx / 4), TY = ceil(ny / 4)."""
    if base is None:
        base, _, _ = stencil(x, grid)
    t = base // TILE
    TX = -(-grid.nx // TILE)
    TY = -(-grid.ny // TILE)
    return t[:, 0] + TX * (t[:, 1] + TY * t[:, 2])


def active_node_tiles(x, grid: Grid, base=None):
    """Sorted list of 4x4x4 node tiles that hold at least one node of some
    particle's 27-node stencil (the nodes a P2G writes and a grid update reads)."""
    if base is None:
        base, _, _ = stencil(x, grid)
    TX = -(-grid.nx // TILE)
    TY = -(-grid.ny // TILE)
    keys = set()
    lo = (base // TILE).tolist()
    hi = ((base + 2) // TILE).tolist()
    for a, b in zip(lo, hi):
        for tz in {a[2], b[2]}:
            for ty in {a[1], b[1]}:
                for tx in {a[0], b[0]}:
                    keys.add(tx + TX * (ty + TY * tz))
    return sorted(keys)
