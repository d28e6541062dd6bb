"""Gradients of a checkpointed multi-substep rollout through the hand-written
adjoints, against the float64 oracle's reverse mode and central finite
differences of the oracle's forward (the reconstruction setting of Sec. 3.3:
wind force grid per time slot and per-region E)."""
import numpy as np
import pytest
import torch

from oracle import mpm as ompm
from oracle import wind as owind
from paper_2603_09668_amd import api, scenes
from paper_2603_09668_amd.autograd import RolloutPlan, rollout

from gpu_util import DEV, EYE, f32, say

pytestmark = pytest.mark.gpu


def _setup(material, n=600, res=16, K=2, nw=4, n_sub=12, ckpt=4, seed=21):
    rng = np.random.default_rng(seed)
    x0 = f32(scenes.random_particles_in_box(seed, n, [0.35] * 3, [0.65] * 3))
    region = torch.tensor(rng.integers(0, 2, n), dtype=torch.long)
    mass = f32(np.full(n, 1.0 / n))
    vol0 = f32(np.full(n, 1.0 / n))
    E = f32(np.array([30.0, 60.0]))
    nu = f32(np.array([0.3, 0.25]))
    W = f32(scenes.smooth_force_field(seed + 1, K=K, nw=nw, amp=2.0))
    target = x0 + f32(0.01 * rng.standard_normal((n, 3)))
    grid = dict(nx=res, ny=res, nz=res, dx=1.0 / res, origin=(0.0, 0.0, 0.0))
    cfg = dict(dt=2e-3, gravity=(0.0, -2.0, 0.0), material=material, bound=0, nw=(nw,) * 3, K=K, n_sub=n_sub,
               ckpt=ckpt)
    return grid, x0, region, mass, vol0, E, nu, W, target, cfg


def _oracle_loss(grid, x0, region, mass, vol0, E, nu, W, target, cfg):
    og = ompm.Grid(grid["nx"], grid["ny"], grid["nz"], grid["dx"])
    mu, lam = ompm.particle_mu_lam(E, nu, region)
    n = x0.shape[0]
    st = {"x": x0, "v": torch.zeros(n, 3, dtype=torch.float64), "C": torch.zeros(n, 3, 3, dtype=torch.float64),
          "F": EYE.repeat(n, 1, 1)}
    for s in range(cfg["n_sub"]):
        k = s * cfg["K"] // cfg["n_sub"]
        acc = owind.force_grid_to_nodes(og, W[k], cfg["nw"], (0, 0, 0), (1, 1, 1))
        st, _ = ompm.substep(og, st, mass, vol0, mu, lam, cfg["dt"], cfg["material"], gravity=cfg["gravity"],
                             acc=acc, bound=cfg["bound"])
    return ((st["x"] - target) ** 2).sum()


def _gpu_grad(grid, x0, region, mass, vol0, E, nu, W, target, cfg, ref=False, deterministic=False):
    """Loss and gradients through the library; ref=True keeps the positions
    as x0 (reference) plus a displacement."""
    n = x0.shape[0]
    xd = x0.T.contiguous().float().to(DEV)
    plan = RolloutPlan(grid, n, mass.float().to(DEV), vol0.float().to(DEV), region.to(torch.int32).to(DEV),
                       nu.float().to(DEV), None, cfg["dt"], cfg["gravity"], cfg["material"], cfg["bound"],
                       cfg["nw"], (0, 0, 0), (1, 1, 1), cfg["K"], cfg["n_sub"], cfg["ckpt"],
                       xref=xd if ref else None, deterministic=deterministic)
    Wd = W.float().to(DEV).contiguous().requires_grad_(True)
    Ed = E.float().to(DEV).requires_grad_(True)
    x = torch.zeros_like(xd) if ref else xd
    z3 = torch.zeros(3, n, device=DEV)
    z9 = torch.zeros(9, n, device=DEV)
    xT, vT, CT, HT = rollout(plan, Wd, Ed, x, z3, z9, z9.clone())
    pos = xT.double() + (xd.double() if ref else 0.0)
    L = ((pos - target.T.to(DEV)) ** 2).sum()
    gW, gE = torch.autograd.grad(L, (Wd, Ed))
    return L.item(), gW.double().cpu(), gE.double().cpu()


@pytest.mark.parametrize("ref", [False, True])
@pytest.mark.parametrize("material", [api.FIXED_COROTATED, api.NEO_HOOKEAN])
def test_rollout_gradient_matches_oracle(material, ref):
    say(f"rollout gradient material={material} ref={ref}")
    args = _setup(material)
    grid, x0, region, mass, vol0, E, nu, W, target, cfg = args
    Wo = W.clone().requires_grad_(True)
    Eo = E.clone().requires_grad_(True)
    Lo = _oracle_loss(grid, x0, region, mass, vol0, Eo, nu, Wo, target, cfg)
    gWo, gEo = torch.autograd.grad(Lo, (Wo, Eo))
    L, gW, gE = _gpu_grad(*args, ref=ref)
    say(f"  loss gpu {L:.6e} oracle {Lo.item():.6e}")
    assert abs(L - Lo.item()) / Lo.item() < 1e-4
    eW = ((gW - gWo).norm() / gWo.norm()).item()
    eE = ((gE - gEo).norm() / gEo.norm()).item()
    say(f"  rel err dL/dW {eW:.2e} dL/dE {eE:.2e}")
    assert eW < 1e-3 and eE < 1e-3
    # central finite differences of the oracle's forward at seeded coordinates
    rng = np.random.default_rng(5)
    scale = gWo.abs().max().item()
    for _ in range(4):
        idx = tuple(int(rng.integers(0, d)) for d in W.shape)
        h = 1e-4
        Wp, Wm = W.clone(), W.clone()
        Wp[idx] += h
        Wm[idx] -= h
        fd = (_oracle_loss(grid, x0, region, mass, vol0, E, nu, Wp, target, cfg)
              - _oracle_loss(grid, x0, region, mass, vol0, E, nu, Wm, target, cfg)).item() / (2 * h)
        assert abs(gW[idx].item() - fd) <= 1e-3 * scale, (idx, gW[idx].item(), fd)


def test_rollout_checkpoint_invariance():
    """The gradient does not depend on the checkpoint interval (recompute is exact)."""
    say("rollout checkpoint invariance")
    base = _setup(api.FIXED_COROTATED, ckpt=1)
    L1, gW1, gE1 = _gpu_grad(*base)
    grid, x0, region, mass, vol0, E, nu, W, target, cfg = base
    cfg = dict(cfg, ckpt=5)
    L5, gW5, gE5 = _gpu_grad(grid, x0, region, mass, vol0, E, nu, W, target, cfg)
    assert abs(L1 - L5) <= 1e-6 * abs(L1)
    assert ((gW1 - gW5).norm() / gW1.norm()).item() < 1e-5


def test_rollout_deterministic_gradient_is_bit_reproducible():
    """In the deterministic mode every reduction of the forward and reverse
    substeps has a fixed order: two runs give bit-identical gradients, which
    still match the oracle's reverse mode."""
    say("rollout gradient deterministic x2")
    args = _setup(api.FIXED_COROTATED)
    La, gWa, gEa = _gpu_grad(*args, ref=True, deterministic=True)
    Lb, gWb, gEb = _gpu_grad(*args, ref=True, deterministic=True)
    assert La == Lb and torch.equal(gWa, gWb) and torch.equal(gEa, gEb)
    grid, x0, region, mass, vol0, E, nu, W, target, cfg = args
    Wo = W.clone().requires_grad_(True)
    Eo = E.clone().requires_grad_(True)
    Lo = _oracle_loss(grid, x0, region, mass, vol0, Eo, nu, Wo, target, cfg)
    gWo, gEo = torch.autograd.grad(Lo, (Wo, Eo))
    eW = ((gWa - gWo).norm() / gWo.norm()).item()
    eE = ((gEa - gEo).norm() / gEo.norm()).item()
    say(f"  rel err dL/dW {eW:.2e} dL/dE {eE:.2e}")
    assert eW < 1e-3 and eE < 1e-3
