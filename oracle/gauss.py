"""FP64 oracle: covariance of each Gaussian kernel after deformation (test
infrastructure only).

Sec. 3.2 ("Interaction Modeling") binds every Gaussian kernel to an MPM
particle and updates its covariance with the particle's deformation
gradient: Sigma_p(t) = F_p(t) Sigma_p F_p(t)^T, with Sigma_p the covariance
at rest.  Symmetric matrices are stored as six entries (xx, yy, zz, xy, xz,
yz); F is handed over as F (n, 3, 3).  The reverse mode is torch.autograd
over this definition, taken with respect to the stored entries.

Pins (tests/test_oracle_gauss.py): F = I leaves Sigma unchanged, a rotation
keeps the eigenvalues, F = s I scales by s^2, det Sigma(t) = det(F)^2
det Sigma, and an explicit triple loop.
"""
from __future__ import annotations

import torch

_DT = torch.float64
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def unpack(s6):
    """(n, 6) -> (n, 3, 3) symmetric."""
    n = s6.shape[0]
    M = torch.zeros(n, 3, 3, dtype=s6.dtype)
    for e, (a, b) in enumerate(PAIRS):
        M[:, a, b] = s6[:, e]
        M[:, b, a] = s6[:, e]
    return M


def pack(M):
    """(n, 3, 3) -> (n, 6)."""
    return torch.stack([M[:, a, b] for a, b in PAIRS], dim=1)


def covariance(F, sigma0):
    """Sigma(t) = F Sigma F^T for F (n, 3, 3) and Sigma (n, 6)."""
    return pack(F @ unpack(sigma0) @ F.transpose(1, 2))
