"""FP64 oracle: moment-encoded D3Q19 lattice Boltzmann step, the HOME-LBM
scheme of the appendix "More details on HOME-LBM Algorithm" (test
infrastructure only).

State per node: density rho, velocity u (3) and the second-order moment S
(6: xx, yy, zz, xy, xz, yz), with rho S_ab = sum_i H2_ab(c_i) f_i and
H2_ab(c) = c_a c_b - c_s^2 delta_ab, c_s^2 = 1/3 (Eq. lbm_sum_v2 read as
in the module docstring of the BGK oracle: the printed (c_i^2 - delta/3) is
the second Hermite polynomial).  At equilibrium S = u u.  Stored moments are
post-collision: rho u is the momentum after the collision, S its second
moment.

One step, in the appendix's order:
1. post-collision populations of every node, from its moments, by the
   Hermite expansion to third order (first equation of the appendix):
     f_i = w_i rho [1 + c.u / c_s^2 + H2(c):S / (2 c_s^4)
                    + sum_{(a,a,b)} H3_aab(c) a3_aab / (2 c_s^6)]
   over the six third-order classes the D3Q19 set carries, (x,x,y), (x,x,z),
   (y,y,x), (y,y,z), (z,z,x), (z,z,y), with H3_aab(c) = (c_a^2 - c_s^2) c_b
   and a3_aab = S_aa u_b + 2 S_ab u_a - 2 u_a^2 u_b (reading: the printed
   coefficients carry index typos; H_xyz vanishes on D3Q19);
2. pull streaming with the boundary rules of the BGK oracle (stream()); an
   inlet ghost node holds the equilibrium moments rho = 1, u = u_in,
   S = u_in u_in and is expanded the same way;
3. moments of the pulled populations: rho* = sum f, u* = (sum c f + F/2) /
   rho*, S*_ab = sum H2_ab f / rho*;
4. collision in moment space (second equation of the appendix):
     rho = rho*,  u = u* + F / (2 rho*),
     S_ab (a != b) = (1 - 1/tau) S*_ab + u*_a u*_b / tau
                     + (2 tau - 1) / (2 tau rho*) (F_a u*_b + F_b u*_a),
     S_aa = (tau - 1) / (3 tau) (2 S*_aa - S*_bb - S*_cc)
            + (u*_a^2 - |u*|^2 / 3) / tau + |u*|^2 / 3
            + F_a u*_a / rho* + (tau - 1) / (3 tau rho*) (2 F_a u*_a - F_b u*_b - F_c u*_c)
   i.e. the deviatoric part of S relaxes with 1/tau towards that of u* u*,
   its trace is set to the equilibrium |u*|^2, and the force enters as
   Guo's source.  Reading: the printed diagonal update lacks the term
   (u*_a^2 - |u*|^2/3) / tau, without which a uniform flow would not be a
   fixed point of the collision.
Solid nodes hold the rest state rho = 1, u = 0, S = 0 (f = w) and report
u = 0, rho = 1.  The reported velocity of a fluid node is the macroscopic
u* of step 3, as for the BGK step.

Pins (tests/test_oracle_home.py): the expansion reproduces rho, rho u, rho S
and the six third-order moments it encodes; a uniform equilibrium stays
uniform with inlet and outlet; mass and momentum are conserved in a periodic
box; a shear wave decays as exp(-nu k^2 t) with nu = (tau - 1/2) / 3;
forced Poiseuille flow between bounce-back walls against its closed form;
a uniform force accelerates a periodic box by F / rho per step.
"""
from __future__ import annotations

import torch

from . import lbm
from .lbm import Q, W

_DT = torch.float64
CS2 = 1.0 / 3.0
# S components in storage order and the index pairs they stand for
S_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
# third-order classes (a, a, b) carried by D3Q19
H3_CLASSES = ((0, 0, 1), (0, 0, 2), (1, 1, 0), (1, 1, 2), (2, 2, 0), (2, 2, 1))


def _S_matrix(S):
    """(6, ...) -> (3, 3, ...) symmetric."""
    M = torch.empty((3, 3) + S.shape[1:], dtype=S.dtype)
    for s, (a, b) in enumerate(S_PAIRS):
        M[a, b] = S[s]
        M[b, a] = S[s]
    return M


def hermite2(c):
    """H2_ab(c) for the 19 velocities: (19, 3, 3)."""
    c = c.to(_DT)
    return c[:, :, None] * c[:, None, :] - CS2 * torch.eye(3, dtype=_DT)[None]


def hermite3(c, cls):
    """H3_aab(c) = (c_a^2 - c_s^2) c_b for class (a, a, b): (19,)."""
    a, _, b = cls
    c = c.to(_DT)
    return (c[:, a] ** 2 - CS2) * c[:, b]


def third_moments(u, S):
    """a3_aab = S_aa u_b + 2 S_ab u_a - 2 u_a^2 u_b for the six classes: (6, ...)."""
    M = _S_matrix(S)
    return torch.stack([M[a, a] * u[b] + 2.0 * M[a, b] * u[a] - 2.0 * u[a] ** 2 * u[b] for a, _, b in H3_CLASSES])


def populations(rho, u, S):
    """Post-collision populations (19, ...) from the moments (first equation
    of the appendix)."""
    c = lbm.C.to(_DT)
    shape = (Q,) + (1,) * rho.dim()
    cu = torch.einsum("qa,a...->q...", c, u)
    H2S = torch.einsum("qab,ab...->q...", hermite2(lbm.C), _S_matrix(S))
    a3 = third_moments(u, S)
    H3a = sum(hermite3(lbm.C, cls).view(shape) * a3[k][None] for k, cls in enumerate(H3_CLASSES))
    series = 1.0 + cu / CS2 + H2S / (2.0 * CS2 ** 2) + H3a / (2.0 * CS2 ** 3)
    return W.view(shape) * rho[None] * series


def moments(f, force):
    """rho* = sum f, u* = (sum c f + F / 2) / rho*, S*_ab = sum H2_ab f / rho*."""
    c = lbm.C.to(_DT)
    rho = f.sum(dim=0)
    j = torch.einsum("qa,q...->a...", c, f)
    Fv = torch.tensor(force, dtype=_DT).view((3,) + (1,) * rho.dim())
    u = (j + 0.5 * Fv) / rho[None]
    Pi = torch.einsum("qab,q...->ab...", hermite2(lbm.C), f)
    S = torch.stack([Pi[a, b] for a, b in S_PAIRS]) / rho[None]
    return rho, u, S


def collide(rho, u, S, tau: float, force):
    """Moment-space collision (second equation of the appendix, with the
    equilibrium term of the diagonal restored).  Returns (u_post, S_post)."""
    Fv = torch.tensor(force, dtype=_DT).view((3,) + (1,) * rho.dim())
    u_post = u + 0.5 * Fv / rho[None]
    M = _S_matrix(S)
    uu = (u * u).sum(dim=0)
    Fu = (Fv * u).sum(dim=0)
    tr = M[0, 0] + M[1, 1] + M[2, 2]
    out = []
    for a, b in S_PAIRS:
        if a != b:
            s = ((1.0 - 1.0 / tau) * M[a, b] + u[a] * u[b] / tau
                 + (2.0 * tau - 1.0) / (2.0 * tau * rho) * (Fv[a] * u[b] + Fv[b] * u[a]))
        else:
            s = ((tau - 1.0) / (3.0 * tau) * (3.0 * M[a, a] - tr)
                 + (u[a] ** 2 - uu / 3.0) / tau + uu / 3.0
                 + Fv[a] * u[a] / rho + (tau - 1.0) / (3.0 * tau * rho) * (3.0 * Fv[a] * u[a] - Fu))
        out.append(s)
    return u_post, torch.stack(out)


def equilibrium_moments(rho, u):
    """(rho, u, S = u u)."""
    return rho, u, torch.stack([u[a] * u[b] for a, b in S_PAIRS])


def home_step(lat: lbm.Lattice, p: lbm.LBMParams, rho, u, S, solid=None, t: int = 0):
    """One step.  rho (nz, ny, nx), u (3, ...), S (6, ...) post-collision
    moments.  Returns (rho, u, S) after the step and the reported (rho*, u*)."""
    nx, ny, nz = lat.dims
    if solid is None:
        solid = torch.zeros(nz, ny, nx, dtype=torch.bool)
    f = populations(rho, u, S)
    u_in = lbm.inlet_velocity(lat, p, t)
    f_inlet = populations(*equilibrium_moments(torch.ones(nz, ny, dtype=_DT), u_in))
    f_star = lbm.stream(lat, p, f, solid, t, f_inlet=f_inlet)
    rho_s, u_s, S_s = moments(f_star, p.force)
    u_post, S_post = collide(rho_s, u_s, S_s, p.tau, p.force)
    fluid = ~solid
    one = torch.ones_like(rho_s)
    rho_n = torch.where(fluid, rho_s, one)
    u_n = torch.where(fluid[None], u_post, torch.zeros_like(u_post))
    S_n = torch.where(fluid[None], S_post, torch.zeros_like(S_post))
    rho_r = torch.where(fluid, rho_s, one)
    u_r = torch.where(fluid[None], u_s, torch.zeros_like(u_s))
    return rho_n, u_n, S_n, rho_r, u_r

