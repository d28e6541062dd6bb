"""Shared helpers of the GPU parity tests: seeded inputs on both sides, layout
conversion between the library's SoA device arrays and the oracle's
(n, 3) / (n, 3, 3) float64 tensors, and norm-wise relative errors."""
import sys

import numpy as np
import torch

from oracle import mpm as ompm
from paper_2603_09668_amd import api, scenes

DEV = "cuda"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """norm-wise relative error |a - b|_inf / |b|_inf (b the oracle)."""
    a = torch.as_tensor(a).double().cpu()
    b = torch.as_tensor(b).double().cpu()
    den = b.abs().max().item()
    return (a - b).abs().max().item() / (den if den > 0 else 1.0)


def vec_to_dev(v):   # (n, 3) -> (3, n) float32 device
    return torch.as_tensor(v).double().T.contiguous().float().to(DEV)


def mat_to_dev(M):   # (n, 3, 3) -> (9, n)
    M = torch.as_tensor(M).double()
    return M.reshape(M.shape[0], 9).T.contiguous().float().to(DEV)


def vec_from_dev(t):
    return t.double().cpu().T.contiguous()


def mat_from_dev(t):
    return t.double().cpu().T.contiguous().reshape(-1, 3, 3)


def f32(t):
    """round an oracle input to float32 and back (both sides see the same value)."""
    return torch.as_tensor(t).float().double()


def oracle_grid(g: dict):
    return ompm.Grid(g["nx"], g["ny"], g["nz"], g["dx"], tuple(g["origin"]))


def api_grid(g: dict):
    return api.make_grid(g["nx"], g["ny"], g["nz"], g["dx"], g["origin"])


EYE = torch.eye(3, dtype=torch.float64)


def h_to_dev(F):
    """deformation gradients (n, 3, 3) -> the library's shifted storage F - I."""
    return mat_to_dev(torch.as_tensor(F).double() - EYE)


def F_from_dev(t):
    return mat_from_dev(t) + EYE


def device_particles(x, v, C, F, mass, vol0, region, E, nu, xref=None):
    """Device particle arrays; with xref (n, 3) the x given is the
    displacement from it."""
    return api.ParticleArrays(
        x=vec_to_dev(x), v=vec_to_dev(v), C=mat_to_dev(C), F=h_to_dev(F),
        mass=torch.as_tensor(mass).float().to(DEV), vol0=torch.as_tensor(vol0).float().to(DEV),
        region=torch.as_tensor(region).to(torch.int32).to(DEV),
        E=torch.as_tensor(E).float().to(DEV), nu=torch.as_tensor(nu).float().to(DEV),
        xref=None if xref is None else vec_to_dev(xref))


def scene_state(sc, seed=None, scale_v=0.1, scale_c=1.0, scale_f=0.05, ref=False, disp=0.0):
    """float32-rounded particle state of a scene (float64 tensors) plus the
    device copy.  seed=None gives the rest state (v = C = 0, F = I).  With
    ref=True the device keeps the scene's positions as the position
    reference and a displacement (zero, or seeded normal of size `disp`);
    st["x"] is then the exact float64 sum and st["xref"], st["disp"] its
    two parts."""
    n = sc.n
    x = f32(sc.x)
    xref = d = None
    if ref:
        xref = x
        d = torch.zeros(n, 3, dtype=torch.float64)
        if disp:
            rng = np.random.default_rng(977 if seed is None else seed + 977)
            d = f32(disp * rng.standard_normal((n, 3)))
        x = xref + d  # exact in float64
    if seed is None:
        v = torch.zeros(n, 3, dtype=torch.float64)
        C = torch.zeros(n, 3, 3, dtype=torch.float64)
        F = torch.eye(3, dtype=torch.float64).repeat(n, 1, 1)
    else:
        v, C, F = scenes.random_state(seed, n, scale_v, scale_c, scale_f)
        # the library stores F - I in float32: round that, on both sides
        v, C, F = f32(v), f32(C), f32(torch.as_tensor(F) - EYE) + EYE
    st = dict(x=x, v=v, C=C, F=F, mass=f32(sc.mass), vol0=f32(sc.vol0),
              region=torch.as_tensor(sc.region).long(), E=f32(sc.E), nu=f32(sc.nu), xref=xref, disp=d)
    dev = device_particles(x if xref is None else d, v, C, F, st["mass"], st["vol0"], sc.region, st["E"], st["nu"],
                           xref=xref)
    return st, dev
