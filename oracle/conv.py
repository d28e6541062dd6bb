"""FP64 oracle: 3-D convolutional wind surrogate and its field checks (test infrastructure only).

The paper has no learned wind model; the surrogate advances the LBM wind
velocity field by k lattice steps in one call and its error is measured
against the LBM of Eq. lbe.  Network (fixed by the workload definition): four 3x3x3
convolutions with zero "same" padding, channels 3 -> 32 -> 32 -> 32 -> 3,
SiLU after the first three, residual output scaled by the per-sample inflow
speed s and a fixed output gain g:

    u_{t+k} = u_t + g s * net(u_t / s).

Layout here is torch's NCDHW (batch, channel, z, y, x).  The convolution is
``torch.nn.functional.conv3d`` (a library routine) in float64; its gradients
come from autograd.

Field checks used to accept or reject a surrogate prediction:
* divergence by central differences on interior nodes,
  div u = (u_x[i+1] - u_x[i-1] + u_y[j+1] - u_y[j-1] + u_z[k+1] - u_z[k-1]) / 2,
  reduced to its RMS over interior fluid nodes;
* kinetic energy 1/2 sum |u|^2 over fluid nodes.

Training uses Adam (Kingma & Ba 2015) on the mean squared error of the
scaled increments, mean over (b, c, voxel) of ((u_out - u_tgt) / s_b)^2.

Pins (tests/test_oracle_wind_conv.py): central finite differences of the
loss against autograd, a direct 27-tap loop against the library convolution
on a tiny input, the divergence of analytic fields (zero for a solenoidal
field, the closed form for a linear one), and Adam against torch.optim.Adam.
"""
from __future__ import annotations

import torch
import torch.nn.functional as tF

_DT = torch.float64


def silu(x):
    return x * torch.sigmoid(x)


def net(h, weights, biases):
    """weights[l]: (Cout, Cin, 3, 3, 3); biases[l]: (Cout,)."""
    n = len(weights)
    for l in range(n):
        h = tF.conv3d(h, weights[l], biases[l], padding=1)
        if l < n - 1:
            h = silu(h)
    return h


def surrogate_forward(u, weights, biases, scale, gain=1.0):
    """u (B, 3, D, H, W); scale (B,) per-sample inflow speed; the increment
    is multiplied by the fixed output gain g (u + g s net(u / s))."""
    s = scale.view(-1, 1, 1, 1, 1)
    return u + net(u / s, weights, biases) * (s * gain)


def conv3d_direct(x, w, b):
    """Same-padded 3x3x3 convolution written as its 27-tap sum (tiny inputs only)."""
    B, Cin, D, H, Wd = x.shape
    xp = tF.pad(x, (1, 1, 1, 1, 1, 1))
    out = b.view(1, -1, 1, 1, 1).expand(B, -1, D, H, Wd).clone()
    for dz in range(3):
        for dy in range(3):
            for dxx in range(3):
                patch = xp[:, :, dz:dz + D, dy:dy + H, dxx:dxx + Wd]
                out = out + torch.einsum("oc,bczyx->bozyx", w[:, :, dz, dy, dxx], patch)
    return out


def divergence_rms(u, fluid=None):
    """RMS of the central-difference divergence over interior (fluid) nodes; u (3, D, H, W)."""
    ux, uy, uz = u[0], u[1], u[2]
    div = (ux[1:-1, 1:-1, 2:] - ux[1:-1, 1:-1, :-2]
           + uy[1:-1, 2:, 1:-1] - uy[1:-1, :-2, 1:-1]
           + uz[2:, 1:-1, 1:-1] - uz[:-2, 1:-1, 1:-1]) * 0.5
    if fluid is not None:
        m = fluid[1:-1, 1:-1, 1:-1]
        div = div[m]
    return torch.sqrt((div * div).mean())


def kinetic_energy(u, fluid=None):
    e = 0.5 * (u * u).sum(dim=0)
    if fluid is not None:
        e = e[fluid]
    return e.sum()


def increment_mse(u_out, u_tgt, scale):
    """Mean over (b, c, voxel) of ((u_out - u_tgt) / s_b)^2."""
    s = scale.view(-1, *([1] * (u_out.dim() - 1)))
    return (((u_out - u_tgt) / s) ** 2).mean()


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) with bias correction;
    returns new (p, m, v); step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (torch.sqrt(vh) + eps), m, v
