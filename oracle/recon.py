"""FP64 oracle: the physics-informed loss and the evaluation metrics of the
wind-force reconstruction (test infrastructure only).

Sec. 3.4 ("Physics-Informed Loss"): with D_recon the direction of the
reconstructed force field and D_guide the direction of the LBM wind velocity
at the same place, L_phys = || D_recon - (D_recon . D_guide) D_guide ||^2,
summed over the wind-grid nodes: the squared length of the part of the
reconstructed direction perpendicular to the guide.  Directions are the
vectors scaled to unit length; a node where either vector is zero
contributes nothing (its direction is undefined).

Metrics (the appendix's evaluation of reconstructed wind force fields): the
force vectors are normalised per grid location and
CosSim = mean_i Fhat_gt_i . Fhat_rec_i,
NMSE   = mean_i || Fhat_gt_i - Fhat_rec_i ||^2,
over the locations where both vectors are non-zero.

The guide is the lattice velocity sampled trilinearly at the wind-grid node
positions (vertex-centred grid of nw^3 nodes spanning [lo, hi]); nodes
outside the lattice box get no guide.

Pins (tests/test_oracle_recon.py): L_phys is 0 for aligned or opposite
directions and 1 per node for perpendicular ones, does not depend on the
vectors' lengths; CosSim and NMSE of identical, opposite and perpendicular
fields; NMSE = 2 - 2 CosSim; the gradient of L_phys against central
differences; the guide of a linear velocity field reproduced exactly.
"""
from __future__ import annotations

import torch

from .wind import trilinear

_DT = torch.float64


def _unit(v):
    """(3, n) -> unit vectors and a mask of the non-zero ones (zero vectors
    map to zero with a zero derivative: their direction is undefined)."""
    sq = (v * v).sum(dim=0)
    ok = sq > 0
    nrm = torch.sqrt(torch.where(ok, sq, torch.ones_like(sq)))
    return torch.where(ok[None], v / nrm[None], torch.zeros_like(v)), ok


def phys_loss(W, guide):
    """L_phys summed over nodes; W and guide (3, n)."""
    d, ok_d = _unit(W)
    g, ok_g = _unit(guide)
    dg = (d * g).sum(dim=0)
    perp = d - dg[None] * g
    per_node = (perp * perp).sum(dim=0)
    return torch.where(ok_d & ok_g, per_node, torch.zeros_like(per_node)).sum()


def direction_metrics(F_gt, F_rec):
    """(CosSim, NMSE, count) over the locations where both are non-zero."""
    a, ok_a = _unit(F_gt)
    b, ok_b = _unit(F_rec)
    ok = ok_a & ok_b
    cnt = int(ok.sum())
    cos = (a * b).sum(dim=0)[ok]
    diff = ((a - b) ** 2).sum(dim=0)[ok]
    return cos.sum().item() / max(cnt, 1), diff.sum().item() / max(cnt, 1), cnt


def wind_grid_positions(nw, lo, hi):
    """Positions (n, 3) of the vertex-centred wind-grid nodes, x fastest."""
    axes = [torch.linspace(lo[a], hi[a], nw[a], dtype=_DT) for a in range(3)]
    z, y, x = torch.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return torch.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], dim=1)


def guide_from_lattice(nw, lo, hi, lat_dims, lat_dx, lat_origin, u_lat):
    """The lattice velocity u_lat (3, L) at the wind-grid nodes, (3, n); zero
    outside the lattice box."""
    pos = wind_grid_positions(nw, lo, hi)
    q = (pos - torch.tensor(lat_origin, dtype=_DT)) / lat_dx
    n_t = torch.tensor(lat_dims, dtype=_DT) - 1.0
    inside = ((q >= 0) & (q <= n_t)).all(dim=1)
    qc = torch.minimum(torch.maximum(q, torch.zeros(3, dtype=_DT)), n_t)
    u = trilinear(u_lat, lat_dims, qc)
    return torch.where(inside[None], u, torch.zeros_like(u))
