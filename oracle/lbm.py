"""FP64 oracle: D3Q19 lattice Boltzmann step with BGK collision (test infrastructure only).

Eq. lbe: f_i(x + c_i, t + 1) - f_i(x, t) = Omega_i + F_i with the BGK
collision Omega_i = -(f_i - f_i^eq) / tau, written as a pull: the population
arriving at x in direction i comes from x - c_i.  Moments (Eq. lbm_sum_v2):
rho = sum_i f_i and rho u = sum_i c_i f_i + F / 2 (the half-force shift; F
is the body-force density vector at the node).  The force enters the
collision through Guo's source term
(1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F, and
f^eq_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u^2), c_s^2 = 1/3,
kinematic viscosity nu = (tau - 1/2) / 3.

D3Q19 velocity order: c_0 = 0; 1..6 = +x, -x, +y, -y, +z, -z; 7..18 the
twelve edge vectors (+1,+1,0), (-1,-1,0), (+1,0,+1), (-1,0,-1), (0,+1,+1),
(0,-1,-1), (+1,-1,0), (-1,+1,0), (+1,0,-1), (-1,0,+1), (0,+1,-1), (0,-1,+1);
directions 2k-1 and 2k are opposite.  Weights 1/3, 1/18, 1/36.

Streaming rule for fluid node x and direction i, source s = x - c_i:
1. periodic faces wrap s;
2. if s is outside the lattice through a bounce-back face: halfway
   bounce-back, f_i(x) = f*_{opp(i)}(x) (the post-collision population of x
   from the previous step);
3. else if s is outside through the inlet face (x = -1): f_i(x) =
   f^eq_i(rho = 1, u_in(t, s_y, s_z));
4. else if s is outside through the outlet face (x = nx): s_x = nx - 1
   (zero gradient);
5. if s is a solid node: bounce-back as in 2;
6. otherwise f_i(x) = f*_i(s).
Solid nodes (Eq. point2voxel) are not updated: they hold the rest
equilibrium f_i = w_i and report u = 0, rho = 1.

Inlet velocity (Sec. 3.4, wind source inference gives an inlet boundary
condition): u_in(t, y, z) = u0 (1 + A sin(2 pi (t / P + a y / ny + b z / nz) + phi));
A = 0 gives a uniform inflow.

Pins (tests/test_oracle_lbm.py): moment identities of f^eq, total mass and
momentum conservation in a periodic box, a uniform equilibrium stays uniform,
Poiseuille flow between bounce-back walls against the closed form, shear-wave
decay against exp(-nu k^2 t), and the brute-force voxel rule.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

_DT = torch.float64

C = torch.tensor([[0, 0, 0],
                  [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, -1], [0, 1, 1], [0, -1, -1],
                  [1, -1, 0], [-1, 1, 0], [1, 0, -1], [-1, 0, 1], [0, 1, -1], [0, -1, 1]],
                 dtype=torch.int64)
W = torch.tensor([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=_DT)
OPP = torch.tensor([0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17])
Q = 19

PERIODIC, BOUNCEBACK, INLET, OUTLET = 0, 1, 2, 3


@dataclass
class Lattice:
    """LBM lattice: nodes at origin + dx * (i, j, k); arrays are (.., nz, ny, nx)."""

    nx: int
    ny: int
    nz: int
    dx: float = 1.0
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz


@dataclass
class LBMParams:
    tau: float = 0.6
    u_in: tuple = (0.0, 0.0, 0.0)
    force: tuple = (0.0, 0.0, 0.0)
    # boundary type per face: x-, x+, y-, y+, z-, z+
    bc: tuple = (PERIODIC,) * 6
    gust_amp: float = 0.0
    gust_period: float = 1.0
    gust_ky: float = 0.0
    gust_kz: float = 0.0
    gust_phase: float = 0.0


def equilibrium(rho, u):
    """f^eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u); rho (...), u (3, ...)."""
    c = C.to(_DT)
    cu = torch.einsum("qa,a...->q...", c, u)
    uu = (u * u).sum(dim=0)
    shape = (Q,) + (1,) * rho.dim()
    return W.view(shape) * rho[None] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu[None])


def moments(f, force):
    """rho = sum f, u = (sum c f + F / 2) / rho (Eq. lbm_sum_v2)."""
    c = C.to(_DT)
    rho = f.sum(dim=0)
    j = torch.einsum("qa,q...->a...", c, f)
    Fv = torch.tensor(force, dtype=_DT).view((3,) + (1,) * rho.dim())
    u = (j + 0.5 * Fv) / rho[None]
    return rho, u


def inlet_velocity(lat: Lattice, p: LBMParams, t: int):
    """u_in on the inlet plane, (3, nz, ny)."""
    kz, ky = torch.meshgrid(torch.arange(lat.nz, dtype=_DT), torch.arange(lat.ny, dtype=_DT),
                            indexing="ij")
    phase = 2.0 * math.pi * (t / p.gust_period + p.gust_ky * ky / lat.ny + p.gust_kz * kz / lat.nz)
    s = 1.0 + p.gust_amp * torch.sin(phase + p.gust_phase)
    u0 = torch.tensor(p.u_in, dtype=_DT)
    return u0[:, None, None] * s[None]


def stream(lat: Lattice, p: LBMParams, f_in, solid, t: int, f_inlet=None):
    """Pull streaming with the boundary rules of the module docstring.

    f_in (19, nz, ny, nx); solid (nz, ny, nx) bool.  Returns the pulled
    populations f* (19, nz, ny, nx) for every node (solid ones are overwritten
    later).  f_inlet (19, nz, ny): the populations of the inlet ghost nodes,
    by default the equilibrium at rho = 1, u_in(t)."""
    nx, ny, nz = lat.dims
    kz, jy, ix = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx), indexing="ij")
    coords = [ix, jy, kz]
    dims = [nx, ny, nz]
    out = torch.empty_like(f_in)
    if f_inlet is None:
        u_inlet = inlet_velocity(lat, p, t)  # (3, nz, ny)
        f_inlet = equilibrium(torch.ones(nz, ny, dtype=_DT), u_inlet)  # (19, nz, ny)
    for i in range(Q):
        src = [coords[a] - int(C[i, a]) for a in range(3)]
        bounce = torch.zeros(nz, ny, nx, dtype=torch.bool)
        inlet = torch.zeros_like(bounce)
        for a in range(3):
            lo_face, hi_face = p.bc[2 * a], p.bc[2 * a + 1]
            below = src[a] < 0
            above = src[a] >= dims[a]
            if lo_face == PERIODIC:
                src[a] = torch.where(below, src[a] + dims[a], src[a])
                below = torch.zeros_like(below)
            if hi_face == PERIODIC:
                src[a] = torch.where(above, src[a] - dims[a], src[a])
                above = torch.zeros_like(above)
            if lo_face == BOUNCEBACK:
                bounce |= below
            if hi_face == BOUNCEBACK:
                bounce |= above
            if lo_face == INLET:
                inlet |= below
            if hi_face == OUTLET:
                src[a] = torch.where(above, torch.full_like(src[a], dims[a] - 1), src[a])
            if lo_face == OUTLET or hi_face == INLET:
                raise ValueError("inlet is only supported on a low face, outlet on a high face")
        inlet &= ~bounce
        valid = ~(bounce | inlet)
        sx = torch.clamp(src[0], 0, nx - 1)
        sy = torch.clamp(src[1], 0, ny - 1)
        sz = torch.clamp(src[2], 0, nz - 1)
        src_solid = solid[sz, sy, sx] & valid
        bounce |= src_solid
        pulled = f_in[i][sz, sy, sx]
        bb = f_in[int(OPP[i])]
        # inlet value for the ghost node at (s_y, s_z)
        inl = f_inlet[i][sz, sy]
        val = torch.where(bounce, bb, torch.where(inlet, inl, pulled))
        out[i] = val
    return out


def collide(f_star, tau: float, force):
    """BGK collision with Guo forcing; returns (f_out, rho, u)."""
    rho, u = moments(f_star, force)
    feq = equilibrium(rho, u)
    c = C.to(_DT)
    Fv = torch.tensor(force, dtype=_DT)
    cu = torch.einsum("qa,a...->q...", c, u)
    cF = torch.einsum("qa,a->q", c, Fv).view((Q,) + (1,) * rho.dim())
    uF = torch.einsum("a...,a->...", u, Fv)
    shape = (Q,) + (1,) * rho.dim()
    src = W.view(shape) * (3.0 * (cF - uF[None]) + 9.0 * cu * cF)
    f_out = f_star - (f_star - feq) / tau + (1.0 - 0.5 / tau) * src
    return f_out, rho, u


def lbm_step(lat: Lattice, p: LBMParams, f_in, solid=None, t: int = 0):
    """One stream-collide step.  Returns (f_out, rho, u) with u = 0, rho = 1 and
    f = w on solid nodes."""
    nx, ny, nz = lat.dims
    if solid is None:
        solid = torch.zeros(nz, ny, nx, dtype=torch.bool)
    f_star = stream(lat, p, f_in, solid, t)
    f_out, rho, u = collide(f_star, p.tau, p.force)
    rest = W.view(Q, 1, 1, 1).expand(Q, nz, ny, nx)
    f_out = torch.where(solid[None], rest, f_out)
    u = torch.where(solid[None], torch.zeros_like(u), u)
    rho = torch.where(solid, torch.ones_like(rho), rho)
    return f_out, rho, u


def voxelize(lat: Lattice, x, x_ref=None):
    """Eq. point2voxel: node x_w is solid iff some particle satisfies
    0 <= x_p,d - x_w,d < dx on every axis, i.e. sits in the cell
    [x_w, x_w + dx); index floor((x_p - origin) / dx), ignored off-lattice.
    The index is computed in the precision of ``x`` (float32 input gives the
    float32 decision).  With ``x_ref`` the position is x_ref + x (x the
    displacement) and the cell coordinate is taken in two parts,
    (x_ref - origin) / dx + x / dx, each rounded in that precision."""
    nx, ny, nz = lat.dims
    solid = torch.zeros(nz, ny, nx, dtype=torch.bool)
    o = torch.tensor(lat.origin, dtype=x.dtype)
    h = torch.tensor(lat.dx, dtype=x.dtype)
    if x_ref is None:
        q = (x - o) / h
    else:
        q = (x_ref.to(x.dtype) - o) / h + x / h
    idx = torch.floor(q).to(torch.int64)
    ok = ((idx >= 0) & (idx < torch.tensor([nx, ny, nz]))).all(dim=1)
    idx = idx[ok]
    solid[idx[:, 2], idx[:, 1], idx[:, 0]] = True
    return solid


def voxelize_brute(lat: Lattice, x):
    """Eq. point2voxel evaluated literally: every node against every particle."""
    nx, ny, nz = lat.dims
    solid = torch.zeros(nz, ny, nx, dtype=torch.bool)
    o = torch.tensor(lat.origin, dtype=_DT)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                xw = o + lat.dx * torch.tensor([i, j, k], dtype=_DT)
                d = x - xw
                hit = ((d >= 0) & (d < lat.dx)).all(dim=1).any()
                solid[k, j, i] = bool(hit)
    return solid
