"""Adjoint parity at the differentiable workload's size, in the launch
configuration of its rollouts.

Workload: 256,000 particles (flag sheet + leaf clusters, per-region E) on a
96^3 grid driven by a 16^3 wind force grid, particles stored in cell-tile
order with positions as reference plus float32 displacement, as the
reconstruction rollouts run them.  After warm-up substeps one substep is run
forward and its reverse is applied with seeded output adjoints, phase by
phase: mpm_g2p_adj, mpm_grid_update_adj, wind_to_grid_adj (force grid),
mpm_p2g_adj.  Each phase is checked against float64 autograd of the oracle on
the same float32 inputs (the GPU's own input adjoints are fed to the oracle,
so each kernel is isolated):

* G2P reverse: x and F adjoints of sampled particles (random, and the first
  and last particles of work items of tiles split over several items); the
  grid-velocity adjoint at sampled nodes, from every particle whose stencil
  reaches them;
* grid-update reverse: every node of every active node tile;
* wind transpose: the whole force-grid adjoint;
* P2G reverse: x, v, C, F adjoints of the sampled particles, and the E
  adjoint of the regions whose particles the oracle differentiates in full.

Bar: |g - g_oracle|_2 / |g_oracle|_2 <= 1e-3 per checked set."""
import numpy as np
import pytest
import torch

from oracle import mpm as ompm
from oracle import wind as owind
from paper_2603_09668_amd import api, scenes

from gpu_util import DEV, EYE, f32, mat_from_dev, oracle_grid, say, vec_from_dev

pytestmark = pytest.mark.gpu
TOL = 1e-3
NW = 16
WORK_CHUNK = api.WORK_CHUNK


def rel2(a, b):
    a = torch.as_tensor(a).double().cpu().reshape(-1)
    b = torch.as_tensor(b).double().cpu().reshape(-1)
    return ((a - b).norm() / b.norm()).item()


def _cpu(t):
    return t.detach().double().cpu()


@pytest.fixture(scope="module")
def run():
    say("full-size adjoint: scene 256k / 96^3")
    sc = scenes.flag_and_leaves_scene(seed=3, n=256_000, res=96, lbm_dims=(96, 48, 48))
    f = dict(dtype=torch.float32, device=DEV)
    n = sc.n
    g = api.make_grid(96, 96, 96, 1.0 / 96)
    N = 96 ** 3
    ws = api.alloc_workspace(g, n)
    prm = api.make_mpm_params(sc.dt, sc.gravity, sc.bound, sc.material)
    xref0 = torch.tensor(np.ascontiguousarray(sc.x.T), **f)
    p = api.ParticleArrays(torch.zeros(3, n, **f), torch.zeros(3, n, **f), torch.zeros(9, n, **f),
                           torch.zeros(9, n, **f), torch.tensor(sc.mass, **f), torch.tensor(sc.vol0, **f),
                           torch.tensor(sc.region, dtype=torch.int32, device=DEV), torch.tensor(sc.E, **f),
                           torch.tensor(sc.nu, **f), xref=xref0)
    api.mpm_sort(g, prm, p.x, ws, xref=p.xref)
    p = api.mpm_reorder(g, p, ws)  # cell-tile order, as the rollouts keep it
    W = torch.tensor(scenes.smooth_force_field(7, K=1, nw=NW, amp=200.0)[0], **f).contiguous()
    wind = api.wind_force_grid(W, (NW,) * 3, (0, 0, 0), (1, 1, 1))
    pin = torch.tensor(sc.pin, dtype=torch.uint8, device=DEV)
    gm, gmv, gv = torch.zeros(N, **f), torch.zeros(3, N, **f), torch.zeros(3, N, **f)
    say("full-size adjoint: 24 warm-up substeps")
    for _ in range(24):
        api.mpm_sort(g, prm, p.x, ws, xref=p.xref)
        api.mpm_p2g(g, prm, p, gm, gmv, ws)
        api.mpm_grid_update(g, prm, gm, gmv, wind, pin, gv, ws)
        api.mpm_g2p(g, prm, gv, p, p.x, p.v, p.C, p.F)
    # the substep under test: forward inputs kept
    api.mpm_sort(g, prm, p.x, ws, xref=p.xref)
    api.mpm_p2g(g, prm, p, gm, gmv, ws)
    api.mpm_grid_update(g, prm, gm, gmv, wind, pin, gv, ws)
    torch.cuda.synchronize()
    assert api.read_status(ws) == 0
    V = api.workspace_views(g, n, ws)
    r = dict(sc=sc, n=n, N=N)
    r["counts"] = V["tile_count"].cpu().long()
    r["starts"] = V["tile_start"].cpu().long()
    r["perm"] = V["perm"][:n].cpu().long()
    r["nodes_active"] = V["node_tiles"][:int(V["n_node_tiles"])].cpu().long()
    for k in ("x", "v", "C", "F", "mass", "vol0", "xref"):
        r[k] = _cpu(getattr(p, k))
    r["region"] = p.region.cpu().long()
    r["E"], r["nu"] = _cpu(p.E), _cpu(p.nu)
    r["W"], r["gm"], r["gmv"], r["gv"] = _cpu(W), _cpu(gm), _cpu(gmv), _cpu(gv)
    rng = np.random.default_rng(17)
    cot = [torch.tensor(rng.standard_normal((3, n)), **f), torch.tensor(rng.standard_normal((3, n)), **f),
           torch.tensor(rng.standard_normal((9, n)), **f), torch.tensor(rng.standard_normal((9, n)), **f)]
    r["cot"] = [_cpu(c) for c in cot]
    say("full-size adjoint: reverse phases")
    xb, Fb, gvb = torch.zeros(3, n, **f), torch.zeros(9, n, **f), torch.zeros(3, N, **f)
    api.mpm_g2p_adj(g, prm, gv, p, *cot, x_bar=xb, F_bar=Fb, grid_v_bar=gvb, ws=ws)
    r["g2p_xb"], r["g2p_Fb"], r["gvb"] = _cpu(xb), _cpu(Fb), _cpu(gvb)
    mb, mvb, ab = torch.zeros(N, **f), torch.zeros(3, N, **f), torch.zeros(3, N, **f)
    api.mpm_grid_update_adj(g, prm, gm, gmv, wind, pin, gvb, mb, mvb, ab, ws)
    Wb = torch.zeros(3, NW ** 3, **f)
    api.wind_to_grid_adj(g, wind, ab, Wb)
    bars = [torch.zeros(3, n, **f), torch.zeros(3, n, **f), torch.zeros(9, n, **f), torch.zeros(9, n, **f)]
    Eb = torch.zeros_like(p.E)
    api.mpm_p2g_adj(g, prm, p, mb, mvb, *bars, E_bar=Eb)
    torch.cuda.synchronize()
    r["mb"], r["mvb"], r["ab"], r["Wb"], r["Eb"] = _cpu(mb), _cpu(mvb), _cpu(ab), _cpu(Wb), _cpu(Eb)
    r["p2g_bars"] = [_cpu(b) for b in bars]
    r["pin"] = pin.cpu()
    # sampled particles: random, plus the ends of the work items of tiles
    # that hold more than one item
    split = torch.nonzero(r["counts"] > WORK_CHUNK).flatten()
    r["split_tiles"] = split
    ends = []
    for t in split[:64].tolist():
        s0, c = int(r["starts"][t]), int(r["counts"][t])
        for b in range(s0, s0 + c, WORK_CHUNK):
            ends += [b, b + 1, min(b + WORK_CHUNK, s0 + c) - 1]
    sel = torch.unique(torch.cat([torch.as_tensor(rng.choice(n, 3000, replace=False)),
                                  r["perm"][torch.tensor(ends, dtype=torch.long)]]))
    r["sample"] = sel
    yield r
    torch.cuda.empty_cache()


def _og(r):
    return oracle_grid(r["sc"].grid)


def _abs_x(r, idx):
    return (r["xref"] + r["x"])[:, idx].T.contiguous()


def test_tiles_span_several_work_items(run):
    say(f"full-size adjoint: {run['split_tiles'].numel()} tiles hold more than {WORK_CHUNK} particles")
    assert run["split_tiles"].numel() > 0


def test_g2p_adj_particles(run):
    say("full-size adjoint: mpm_g2p_adj particle adjoints")
    r, idx = run, run["sample"]
    og = _og(r)
    dt = r["sc"].dt
    x = _abs_x(r, idx).requires_grad_(True)
    F = (mat_from_dev(r["F"][:, idx]) + EYE).requires_grad_(True)
    x1, v1, C1, F1 = ompm.g2p(og, r["gv"].T, x, F, dt)
    xob, vob, Cob, Fob = (c[:, idx] for c in r["cot"])
    L = (x1 * xob.T).sum() + (v1 * vob.T).sum() + (C1 * mat_from_dev(Cob)).sum() + (F1 * mat_from_dev(Fob)).sum()
    gx, gF = torch.autograd.grad(L, (x, F))
    errs = dict(x=rel2(vec_from_dev(r["g2p_xb"][:, idx]), gx), F=rel2(mat_from_dev(r["g2p_Fb"][:, idx]), gF))
    say("  " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e < TOL, k


def test_g2p_adj_grid_velocity(run):
    say("full-size adjoint: mpm_g2p_adj grid-velocity adjoint")
    r = run
    og = _og(r)
    rng = np.random.default_rng(18)
    active = torch.nonzero(r["gm"] > 0).flatten()
    nodes = torch.unique(torch.cat([active[torch.as_tensor(rng.choice(active.numel(), 150, replace=False))],
                                    r["gm"].argmax().view(1)]))
    xyz = torch.stack([nodes % og.nx, (nodes // og.nx) % og.ny, nodes // (og.nx * og.ny)], dim=1)
    xa = _abs_x(r, torch.arange(r["n"]))
    base, _, _ = ompm.stencil(xa, og)
    want = torch.zeros(og.n_nodes, dtype=torch.bool)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                b = xyz - torch.tensor([dx, dy, dz])
                ok = (b >= 0).all(dim=1)
                want[b[ok, 0] + og.nx * (b[ok, 1] + og.ny * b[ok, 2])] = True
    sel = torch.nonzero(want[base[:, 0] + og.nx * (base[:, 1] + og.ny * base[:, 2])]).flatten()
    say(f"  {nodes.numel()} nodes, {sel.numel()} particles")
    gv = r["gv"].T.clone().requires_grad_(True)
    x1, v1, C1, F1 = ompm.g2p(og, gv, xa[sel], mat_from_dev(r["F"][:, sel]) + EYE, r["sc"].dt)
    xob, vob, Cob, Fob = (c[:, sel] for c in r["cot"])
    L = (x1 * xob.T).sum() + (v1 * vob.T).sum() + (C1 * mat_from_dev(Cob)).sum() + (F1 * mat_from_dev(Fob)).sum()
    (ggv,) = torch.autograd.grad(L, (gv,))
    err = rel2(r["gvb"][:, nodes].T, ggv[nodes])
    say(f"  grid velocity adjoint {err:.2e}")
    assert err < TOL


def test_grid_update_adj_active_tiles(run):
    say("full-size adjoint: mpm_grid_update_adj")
    r = run
    og = _og(r)
    sc = r["sc"]
    m = r["gm"].clone().requires_grad_(True)
    mv = r["gmv"].T.clone().requires_grad_(True)
    W = r["W"].clone().requires_grad_(True)
    acc = owind.force_grid_to_nodes(og, W, (NW,) * 3, (0, 0, 0), (1, 1, 1))
    vo = ompm.grid_update(og, m, mv, sc.dt, sc.gravity, acc=acc, pin=r["pin"], bound=sc.bound)
    T = ompm.TILE
    TX = -(-og.nx // T)
    t = r["nodes_active"]
    tx, ty, tz = t % TX, (t // TX) % TX, t // (TX * TX)
    o = torch.arange(T)
    ox, oy, oz = torch.meshgrid(o, o, o, indexing="ij")
    nodes = ((tx[:, None] * T + ox.reshape(1, -1)) + og.nx * ((ty[:, None] * T + oy.reshape(1, -1))
                                                              + og.ny * (tz[:, None] * T + oz.reshape(1, -1))))
    nodes = nodes.reshape(-1)
    vbar = torch.zeros(og.n_nodes, 3, dtype=torch.float64)
    vbar[nodes] = r["gvb"].T[nodes]
    acc_leaf = acc
    gm_, gmv_, ga_ = torch.autograd.grad((vo * vbar).sum(), (m, mv, acc_leaf), retain_graph=True)
    errs = dict(m=rel2(r["mb"][nodes], gm_[nodes]), mv=rel2(r["mvb"][:, nodes].T, gmv_[nodes]),
                acc=rel2(r["ab"][:, nodes].T, ga_[nodes]))
    say(f"  {nodes.numel()} nodes: " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e < TOL, k


def test_wind_to_grid_adj_force_grid(run):
    say("full-size adjoint: wind_to_grid_adj")
    r = run
    og = _og(r)
    W = r["W"].clone().requires_grad_(True)
    acc = owind.force_grid_to_nodes(og, W, (NW,) * 3, (0, 0, 0), (1, 1, 1))
    (gW,) = torch.autograd.grad((acc * r["ab"].T).sum(), (W,))
    err = rel2(r["Wb"], gW)
    say(f"  force-grid adjoint {err:.2e}")
    assert err < TOL


def test_p2g_adj(run):
    say("full-size adjoint: mpm_p2g_adj")
    r = run
    og = _og(r)
    sc = r["sc"]
    idx = r["sample"]
    counts = torch.bincount(r["region"], minlength=r["E"].numel())
    # regions the oracle differentiates in full (their E adjoint is complete)
    small = [int(q) for q in torch.argsort(counts) if 0 < counts[q] <= 4000][:6]
    full = torch.nonzero(torch.isin(r["region"], torch.tensor(small))).flatten()
    idx = torch.unique(torch.cat([idx, full]))
    say(f"  {idx.numel()} particles; regions {small} in full")
    x = _abs_x(r, idx).requires_grad_(True)
    v = r["v"][:, idx].T.clone().requires_grad_(True)
    C = mat_from_dev(r["C"][:, idx]).requires_grad_(True)
    F = (mat_from_dev(r["F"][:, idx]) + EYE).requires_grad_(True)
    E = r["E"].clone().requires_grad_(True)
    mu, lam = ompm.particle_mu_lam(E, r["nu"], r["region"][idx])
    m, mv = ompm.p2g(og, x, v, C, F, r["mass"][idx], r["vol0"][idx], mu, lam, sc.dt, sc.material)
    L = (m * r["mb"]).sum() + (mv * r["mvb"].T).sum()
    gx, gv, gC, gF, gE = torch.autograd.grad(L, (x, v, C, F, E))
    # the sampled particles' own adjoints (the extra full regions included)
    xb, vb, Cb, Fb = r["p2g_bars"]
    errs = dict(x=rel2(vec_from_dev(xb[:, idx]), gx), v=rel2(vec_from_dev(vb[:, idx]), gv),
                C=rel2(mat_from_dev(Cb[:, idx]), gC), F=rel2(mat_from_dev(Fb[:, idx]), gF),
                E=rel2(r["Eb"][small], gE[small]))
    say("  " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e < TOL, k
