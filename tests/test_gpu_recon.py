"""GPU parity of the reconstruction losses and metrics against the float64
oracle, and the sequential reconstruction of Sec. 3.3 with the
physics-informed loss of Sec. 3.4 on a synthetic target."""
import numpy as np
import pytest
import torch

from oracle import recon as orecon
from paper_2603_09668_amd import api, recon, scenes

from gpu_util import DEV, f32, rel, say

pytestmark = pytest.mark.gpu


def _rand(shape, seed, scale=1.0):
    return f32(scale * torch.tensor(np.random.default_rng(seed).standard_normal(shape)))


@pytest.mark.parametrize("n", [1, 300, 70_001])
def test_phys_loss_parity(n):
    say(f"phys_loss n={n}")
    W = _rand((3, n), 1, 3.0)
    g = _rand((3, n), 2)
    if n > 10:
        W[:, 3] = 0.0        # undefined directions contribute nothing
        g[:, 7] = 0.0
        g[:, 8] = W[:, 8]    # aligned
    Wv = W.clone().requires_grad_(True)
    ref = orecon.phys_loss(Wv, g)
    ref.backward()
    loss = torch.full((1,), 0.5, device=DEV)
    Wb = torch.full((3, n), 0.25, device=DEV)
    api.phys_loss(W.float().to(DEV), g.float().to(DEV), 2.0, loss, Wb)
    torch.cuda.synchronize()
    assert abs((loss.item() - 0.5) - 2.0 * ref.item()) <= 1e-5 * max(1.0, 2.0 * ref.item())
    assert rel(Wb.cpu() - 0.25, 2.0 * Wv.grad) < 1e-5


def test_position_loss_parity():
    n = 12_345
    x = _rand((3, n), 3)
    xt = f32(x + _rand((3, n), 4, 1e-3))
    loss = torch.zeros(1, device=DEV)
    xb = torch.empty(3, n, device=DEV)
    api.position_loss(x.float().to(DEV), xt.float().to(DEV), loss, xb)
    torch.cuda.synchronize()
    ref = ((x - xt) ** 2).sum().item()
    assert abs(loss.item() - ref) <= 1e-5 * ref
    assert rel(xb.cpu(), 2 * (x - xt)) < 1e-5


def test_direction_metrics_parity():
    n = 5000
    a = _rand((3, n), 5)
    b = a + _rand((3, n), 6, 0.5)
    b[:, 10] = 0.0
    out = torch.zeros(3, device=DEV)
    api.direction_metrics(a.float().to(DEV), b.float().to(DEV), out)
    torch.cuda.synchronize()
    c, m, cnt = orecon.direction_metrics(a, b)
    assert int(out[2].item()) == cnt == n - 1
    assert abs(out[0].item() / cnt - c) < 1e-5 and abs(out[1].item() / cnt - m) < 1e-5


def test_wind_guide_parity():
    sc = scenes.flag_and_leaves_scene(seed=2, n=5_000, res=32, n_clusters=3, lbm_dims=(32, 16, 16))
    lt = sc.lattice
    lat = api.make_lattice(lt["nx"], lt["ny"], lt["nz"], lt["dx"], lt["origin"])
    L = lt["nx"] * lt["ny"] * lt["nz"]
    u = _rand((3, L), 7, 0.05)
    nw, lo, hi = (7, 5, 6), (0.05, 0.2, 0.1), (0.95, 0.8, 0.9)
    g = torch.empty(3, 7 * 5 * 6, device=DEV)
    api.wind_guide(lat, u.float().to(DEV), nw, lo, hi, g)
    torch.cuda.synchronize()
    ref = orecon.guide_from_lattice(nw, lo, hi, (lt["nx"], lt["ny"], lt["nz"]), lt["dx"], lt["origin"], u)
    assert rel(g.cpu(), ref) < 1e-5


def test_sequential_reconstruction_with_phys_loss():
    """Targets from a drag-shaped force field along the LBM wind (two
    frames).  Both runs fit the motion; the physics-informed loss turns the
    reconstructed force directions towards the guide.  L_phys cannot tell a
    direction from its opposite, so weakly constrained nodes may end up
    reversed and CosSim stays below one."""
    sc = scenes.flag_and_leaves_scene(seed=1, n=20_000, res=32, n_clusters=4, lbm_dims=(32, 16, 16))
    nw, lo, hi = (6, 6, 6), (0.2, 0.1, 0.1), (0.95, 0.9, 0.9)
    say("reconstruction: LBM guide")
    guide, _ = recon.lbm_guide(sc, nw, lo, hi, steps=200)
    F_gt = recon.drag_field(guide, 20.0)
    assert recon.metrics(F_gt, guide)[0] > 0.999999
    rc = recon.Reconstructor(sc, nw, lo, hi, substeps_per_frame=16)
    state0 = rc.initial_state()  # positions as displacements from the scene's positions
    frames = 2
    targets, st = [], state0
    for _ in range(frames):
        st = rc.advance(st, F_gt)
        targets.append(st[0].clone())
    out = {}
    for lam in (0.0, 1.0):
        say(f"reconstruction lam={lam}")
        st = state0
        per_frame = []
        for k in range(frames):
            r = rc.frame(st, targets[k], guide, lam=lam, iters=25, lr=1.0)
            assert r.loss[-1] < 0.2 * r.loss[0], (lam, k, r.loss[0], r.loss[-1])
            c, m, cnt = recon.metrics(F_gt, r.W)
            assert cnt > 0 and abs(m - (2 - 2 * c)) < 1e-4
            per_frame.append((c, m))
            st = rc.advance(st, r.W)
        err = torch.sqrt(((st[0] - targets[-1]) ** 2).sum(dim=0)).max().item()
        out[lam] = per_frame
        say(f"  CosSim/NMSE per frame {per_frame}  final max position error {err:.2e}")
        assert err < 1e-4
    assert out[1.0][0][0] > 0.6
    assert out[1.0][0][0] > out[0.0][0][0] + 0.1
    assert out[1.0][0][1] < out[0.0][0][1]
