"""FP64 oracle: wind force field on the MPM grid (test infrastructure only).

Sec. 3 (problem specification) and Sec. 3.2 model the wind as a grid field
whose *force* property is applied to the MPM background grid.  Two sources of
that per-node acceleration a_i are provided:

* force-grid mode (the reconstruction unknown F_w of Eq. simulation_mpm): a
  vertex-centred grid of nw_x x nw_y x nw_z nodes spanning the box
  [lo, hi], one 3-vector per node and per time slot; a_i is the trilinear
  interpolation of slot ``slot`` at the MPM node position, with the
  position clamped into the box;
* LBM-drag mode (Sec. 3.4, drag relation F_w = 1/2 rho_w C_D |v|^2 v/|v|):
  the lattice velocity u (zero on solid nodes) is interpolated trilinearly at
  the MPM node position, scaled to physical units by ``vel_scale``, and
  a_i = k_D |u| u; k_D folds 1/2 rho_w C_D and the area-to-mass ratio into
  one constant, and |u| = 0 gives a = 0.  MPM nodes outside the lattice box
  receive no wind.

* relative LBM drag (a variant the paper leaves open: its drag relation
  uses the wind velocity itself): the same interpolated wind velocity U_i,
  taken relative to the node's own velocity v_i = mv_i / m_i from P2G,
  a_i = k_D |U_i - v_i| (U_i - v_i), zero outside the lattice box and where
  U_i = v_i.  It is evaluated inside the grid update (it needs mv, m).

Trilinear interpolation along one axis at coordinate q in [0, n-1]:
i0 = min(floor(q), n - 2), t = q - i0, value = (1 - t) f[i0] + t f[i0 + 1].

Pins (tests/test_oracle_wind.py): a linear field is reproduced exactly, the
transpose weights of every node sum to one, and the adjoint identity
<A w, y> = <w, A^T y> holds with A^T from autograd.
"""
from __future__ import annotations

import torch

from .mpm import Grid, node_positions

_DT = torch.float64


def _axis_weights(q, n):
    i0 = torch.clamp(torch.floor(q), 0, n - 2).to(torch.int64)
    t = q - i0.to(_DT)
    return i0, t


def trilinear(field, dims, q):
    """Interpolate ``field`` (c, nz*ny*nx flattened as x fastest) at fractional
    node coordinates q (m, 3); q must already lie in [0, n-1] per axis."""
    nx, ny, nz = dims
    ix, tx = _axis_weights(q[:, 0], nx)
    iy, ty = _axis_weights(q[:, 1], ny)
    iz, tz = _axis_weights(q[:, 2], nz)
    out = torch.zeros(field.shape[0], q.shape[0], dtype=_DT)
    for dz in (0, 1):
        wz = tz if dz else 1.0 - tz
        for dy in (0, 1):
            wy = ty if dy else 1.0 - ty
            for dxo in (0, 1):
                wx = tx if dxo else 1.0 - tx
                idx = (ix + dxo) + nx * ((iy + dy) + ny * (iz + dz))
                out = out + (wx * wy * wz)[None, :] * field[:, idx]
    return out


def force_grid_to_nodes(grid: Grid, W_slot, nw, lo, hi):
    """Force-grid mode: a_i = trilinear(W_slot)(clamp(x_i)); W_slot is (3, nw_z*nw_y*nw_x).

    Returns (N, 3)."""
    pos = node_positions(grid)
    lo_t = torch.tensor(lo, dtype=_DT)
    hi_t = torch.tensor(hi, dtype=_DT)
    nw_t = torch.tensor(nw, dtype=_DT)
    q = (pos - lo_t) / (hi_t - lo_t) * (nw_t - 1.0)
    q = torch.minimum(torch.maximum(q, torch.zeros(3, dtype=_DT)), nw_t - 1.0)
    return trilinear(W_slot, nw, q).T.contiguous()


def lbm_drag_to_nodes(grid: Grid, lat_dims, lat_dx, lat_origin, u_lat, vel_scale, k_drag):
    """LBM-drag mode: u at the MPM node by trilinear interpolation of the lattice
    velocity u_lat (3, L), a = k_D |u| u with u in physical units.  Nodes outside
    the lattice box [origin, origin + (n-1) dx] get a = 0.  Returns (N, 3)."""
    pos = node_positions(grid)
    q = (pos - torch.tensor(lat_origin, dtype=_DT)) / lat_dx
    n_t = torch.tensor(lat_dims, dtype=_DT) - 1.0
    inside = ((q >= 0) & (q <= n_t)).all(dim=1)
    qc = torch.minimum(torch.maximum(q, torch.zeros(3, dtype=_DT)), n_t)
    u = vel_scale * trilinear(u_lat, lat_dims, qc).T
    u2 = (u * u).sum(dim=1)
    moving = u2 > 0
    speed = torch.where(moving, torch.sqrt(torch.where(moving, u2, torch.ones_like(u2))),
                        torch.zeros_like(u2))
    a = k_drag * speed[:, None] * u
    return torch.where(inside[:, None], a, torch.zeros_like(a))


def lbm_velocity_to_nodes(grid: Grid, lat_dims, lat_dx, lat_origin, u_lat, vel_scale):
    """The wind velocity U_i = vel_scale * trilinear(u_lat) at the MPM nodes and
    the mask of nodes inside the lattice box (U = 0 outside).  Returns
    (U (N, 3), inside (N,))."""
    pos = node_positions(grid)
    q = (pos - torch.tensor(lat_origin, dtype=_DT)) / lat_dx
    n_t = torch.tensor(lat_dims, dtype=_DT) - 1.0
    inside = ((q >= 0) & (q <= n_t)).all(dim=1)
    qc = torch.minimum(torch.maximum(q, torch.zeros(3, dtype=_DT)), n_t)
    U = vel_scale * trilinear(u_lat, lat_dims, qc).T
    return torch.where(inside[:, None], U, torch.zeros_like(U)), inside


def relative_drag(U, v, inside, k_drag):
    """a = k_D |U - v| (U - v) on nodes inside the lattice box, 0 elsewhere;
    U, v (N, 3)."""
    r = U - v
    r2 = (r * r).sum(dim=1)
    moving = r2 > 0
    s = torch.sqrt(torch.where(moving, r2, torch.ones_like(r2)))
    a = k_drag * torch.where(moving, s, torch.zeros_like(s))[:, None] * r
    return torch.where(inside[:, None], a, torch.zeros_like(a))
