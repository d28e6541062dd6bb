"""Pins of the float64 covariance-update oracle (Sigma(t) = F Sigma F^T)."""
import numpy as np
import torch

from oracle import gauss

DT = torch.float64


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    A = torch.tensor(rng.standard_normal((n, 3, 3)))
    return gauss.pack(A @ A.transpose(1, 2) * 1e-4 + 1e-5 * torch.eye(3, dtype=DT))


def test_identity_and_scaling():
    s0 = _spd(5, 1)
    I = torch.eye(3, dtype=DT).repeat(5, 1, 1)
    assert torch.equal(gauss.covariance(I, s0), s0)
    assert (gauss.covariance(1.5 * I, s0) - 2.25 * s0).abs().max() < 1e-18


def test_rotation_keeps_eigenvalues():
    s0 = _spd(6, 2)
    rng = np.random.default_rng(3)
    Q, _ = torch.linalg.qr(torch.tensor(rng.standard_normal((6, 3, 3))))
    ev0 = torch.linalg.eigvalsh(gauss.unpack(s0))
    ev1 = torch.linalg.eigvalsh(gauss.unpack(gauss.covariance(Q, s0)))
    assert (ev0 - ev1).abs().max() < 1e-17


def test_determinant():
    s0 = _spd(7, 4)
    rng = np.random.default_rng(5)
    F = torch.eye(3, dtype=DT) + 0.2 * torch.tensor(rng.standard_normal((7, 3, 3)))
    d1 = torch.linalg.det(gauss.unpack(gauss.covariance(F, s0)))
    d0 = torch.linalg.det(gauss.unpack(s0)) * torch.linalg.det(F) ** 2
    assert ((d1 - d0).abs() / d0.abs()).max() < 1e-12


def test_triple_loop():
    s0 = _spd(3, 6)
    rng = np.random.default_rng(7)
    F = torch.tensor(rng.standard_normal((3, 3, 3)))
    out = gauss.covariance(F, s0)
    S = gauss.unpack(s0)
    for p in range(3):
        for e, (a, b) in enumerate(gauss.PAIRS):
            ref = sum(F[p, a, c] * S[p, c, d] * F[p, b, d] for c in range(3) for d in range(3))
            assert abs(out[p, e].item() - ref.item()) < 1e-17
