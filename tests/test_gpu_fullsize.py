"""GPU parity at the benchmark sizes, in the launch configuration the
benchmark times.

Workloads: the flag-and-leaves scene with 500k particles on a 128^3 grid and a
128x64x64 lattice, and with 4M particles on 256^3 and 256x128x128 (the
largest single-GPU case).  The coupled simulation is set up as the benchmark
sets it up (particles stored in cell-tile order, substeps replayed from a HIP
graph); after warm-up substeps one more substep runs phase by phase and every
phase is checked against the float64 oracle on the same float32 inputs:

* voxelize: the whole mask, bit-exact;
* LBM step: every population and velocity of the lattice;
* sort: a permutation grouping the particles by tile (the order inside a
  tile is left free), tile counts, ranges and active tile lists against
  their definition, bit-exact;
* P2G: sampled nodes (the largest ones, tile corners and random active
  nodes); the oracle scatters exactly the particles whose stencil reaches
  them, which gives its full sum at those nodes;
* grid update: every node of every active node tile, with the LBM drag
  interpolated by the oracle from the library's lattice velocity;
* G2P: sampled particles gathered by the oracle from the library's grid
  velocity; the substep's displacement x_new - x is compared with the
  oracle's at 1e-5 of its own size.

Positions are kept, as the benchmark keeps them, as the scene's positions
(the reference) plus a float32 displacement; the oracle sees their exact
float64 sum and takes the integer decisions (voxel, stencil base) the way a
float32 kernel takes them from the two parts.

Errors are norm-wise (|gpu - oracle|_inf / |oracle|_inf, 1e-5 per call)."""
import numpy as np
import pytest
import torch

from oracle import lbm as olbm
from oracle import mpm as ompm
from oracle import wind as owind
from paper_2603_09668_amd import api, scenes
from paper_2603_09668_amd.sim import CoupledSim

from gpu_util import DEV, EYE, mat_from_dev, oracle_grid, rel, say, vec_from_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5
WQ = olbm.W.view(19, 1)
WORKLOADS = {
    "500k_grid128": dict(n=500_000, res=128, warm=40),
    "4M_grid256": dict(n=4_000_000, res=256, warm=10),
}


def _cpu(t):
    return t.detach().double().cpu()


@pytest.fixture(scope="module", params=list(WORKLOADS))
def run(request):
    """Warm up with graph replays, then one eager substep phase by phase with
    every phase's inputs and outputs copied to the host."""
    w = WORKLOADS[request.param]
    say(f"full-size {request.param}: scene")
    sc = scenes.flag_and_leaves_scene(seed=0, n=w["n"], res=w["res"], lbm_dims=(w["res"], w["res"] // 2,
                                                                                   w["res"] // 2))
    sim = CoupledSim(sc)
    sim.capture(2)
    say(f"full-size {request.param}: {w['warm']} warm-up substeps")
    for _ in range(w["warm"] // 2):
        sim.replay()
    torch.cuda.synchronize()
    assert sim.status() == 0
    r = dict(name=request.param, sc=sc, sim=sim)
    say(f"full-size {request.param}: phases")
    r["x_pre"] = _cpu(sim.p.x)
    r["xref"] = _cpu(sim.p.xref)
    sim.voxelize()
    r["solid"] = sim.solid.cpu().clone()
    r["f_in"] = _cpu(sim.fa)
    r["t_lbm"] = int(sim.t_a.item())
    sim.lbm()
    r["f_out"] = _cpu(sim.fa)
    r["u"] = _cpu(sim.u)
    sim.sort()
    V = api.workspace_views(sim.grid, sim.p.n, sim.ws)
    torch.cuda.synchronize()
    r["sort"] = {k: (V[k].cpu().clone() if torch.is_tensor(V[k]) else V[k]) for k in V}
    r["state"] = {k: _cpu(getattr(sim.p, k)) for k in ("x", "v", "C", "F", "mass", "vol0")}
    r["region"] = sim.p.region.cpu().long()
    sim.p2g()
    r["gm"] = _cpu(sim.gm)
    r["gmv"] = _cpu(sim.gmv)
    sim.grid_update()
    r["gv"] = _cpu(sim.gv)
    sim.g2p()
    r["post"] = {k: _cpu(getattr(sim.p, k)) for k in ("x", "v", "C", "F")}
    torch.cuda.synchronize()
    assert sim.status() == 0
    yield r
    del r["sim"]
    torch.cuda.empty_cache()


def _olat(sc):
    lat = sc.lattice
    return olbm.Lattice(lat["nx"], lat["ny"], lat["nz"], lat["dx"], lat["origin"])


def test_voxelize(run):
    say(f"full-size {run['name']}: voxelize")
    olat = _olat(run["sc"])
    ref = olbm.voxelize(olat, run["x_pre"].T.float(), x_ref=run["xref"].T.float())
    assert torch.equal(run["solid"].bool().view(olat.nz, olat.ny, olat.nx), ref)


def test_lbm_step(run):
    say(f"full-size {run['name']}: lbm_step")
    sc = run["sc"]
    olat = _olat(sc)
    lb = sc.lbm
    op = olbm.LBMParams(tau=lb["tau"], u_in=lb["u_in"], force=lb["force"], bc=lb["bc"], gust_amp=lb["gust_amp"],
                        gust_period=lb["gust_period"], gust_ky=lb["gust_ky"], gust_kz=lb["gust_kz"],
                        gust_phase=lb["gust_phase"])
    nx, ny, nz = olat.dims
    f = (run["f_in"] + WQ).view(19, nz, ny, nx)
    solid = run["solid"].bool().view(nz, ny, nx)
    fo, _, u = olbm.lbm_step(olat, op, f, solid, run["t_lbm"])
    L = nx * ny * nz
    assert rel(run["f_out"], (fo.reshape(19, L) - WQ)) < TOL
    assert (run["u"] - u.reshape(3, L)).abs().max().item() / abs(lb["u_in"][0]) < TOL


def test_sort(run):
    say(f"full-size {run['name']}: sort")
    sc = run["sc"]
    og = oracle_grid(sc.grid)
    V = run["sort"]
    x = run["state"]["x"].T
    n = x.shape[0]
    base = ompm.stencil_base_f32(x, og, xref32=run["xref"].T)
    keys = ompm.cell_tile_keys(None, og, base=base)
    perm = V["perm"][:n].long()
    assert int(V["status"]) == 0
    assert torch.equal(torch.sort(perm).values, torch.arange(n))
    sk = keys[perm]
    # grouped by tile; the order inside a tile is unspecified in the default mode
    assert torch.all(sk[1:] >= sk[:-1])
    counts = torch.bincount(keys, minlength=V["n_tiles"])
    assert torch.equal(V["tile_count"].long(), counts)
    start = torch.zeros(V["n_tiles"] + 1, dtype=torch.long)
    start[1:] = torch.cumsum(counts, 0)
    assert torch.equal(V["tile_start"].long(), start)
    ncell = int(V["n_cell_tiles"])
    assert torch.equal(V["cell_tiles"][:ncell].long(), torch.nonzero(counts).flatten())
    nnode = int(V["n_node_tiles"])
    assert V["node_tiles"][:nnode].tolist() == ompm.active_node_tiles(None, og, base=base)


def _node_xyz(og, idx):
    idx = torch.as_tensor(idx).long()
    return torch.stack([idx % og.nx, (idx // og.nx) % og.ny, idx // (og.nx * og.ny)], dim=1)


def _active_tile_nodes(og, tiles):
    """Linear indices of every node of the given 4x4x4 node tiles."""
    T = ompm.TILE
    TX, TY = -(-og.nx // T), -(-og.ny // T)
    t = torch.as_tensor(tiles).long()
    tx, ty, tz = t % TX, (t // TX) % TY, t // (TX * TY)
    o = torch.arange(T)
    ox, oy, oz = torch.meshgrid(o, o, o, indexing="ij")
    X = (tx[:, None] * T + ox.reshape(1, -1))
    Y = (ty[:, None] * T + oy.reshape(1, -1))
    Z = (tz[:, None] * T + oz.reshape(1, -1))
    ok = (X < og.nx) & (Y < og.ny) & (Z < og.nz)
    return (X + og.nx * (Y + og.ny * Z))[ok]


def test_p2g_sampled(run):
    say(f"full-size {run['name']}: p2g")
    sc = run["sc"]
    og = oracle_grid(sc.grid)
    st = run["state"]
    gm, gmv = run["gm"], run["gmv"]
    rng = np.random.default_rng(1)
    active = torch.nonzero(gm > 0).flatten()
    assert active.numel() > 0
    # tile corners and faces are where work items and wave blocks meet
    xyz = _node_xyz(og, active)
    corner = active[((xyz % ompm.TILE) == 0).all(dim=1) | ((xyz % ompm.TILE) == ompm.TILE - 1).all(dim=1)]
    pick = [active[torch.as_tensor(rng.choice(active.numel(), 400, replace=False))],
            corner[torch.as_tensor(rng.choice(corner.numel(), min(100, corner.numel()), replace=False))],
            gm.argmax().view(1), gmv.abs().amax(dim=0).argmax().view(1)]
    nodes = torch.unique(torch.cat(pick))
    nxyz = _node_xyz(og, nodes)
    # particles whose 3x3x3 stencil (oracle's float64 base) reaches a sampled node
    x = (run["xref"] + st["x"]).T
    base, _, _ = ompm.stencil(x, og)
    lin = base[:, 0] + og.nx * (base[:, 1] + og.ny * base[:, 2])
    want = torch.zeros(og.n_nodes, dtype=torch.bool)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                b = nxyz - torch.tensor([dx, dy, dz])
                ok = (b >= 0).all(dim=1)
                want[(b[ok, 0] + og.nx * (b[ok, 1] + og.ny * b[ok, 2]))] = True
    sel = want[lin]
    say(f"  {nodes.numel()} nodes, {int(sel.sum())} particles")
    E = run["sim"].p.E.cpu().double()
    nu = run["sim"].p.nu.cpu().double()
    mu, lam = ompm.particle_mu_lam(E, nu, run["region"][sel])
    om, omv = ompm.p2g(og, x[sel], st["v"].T[sel], mat_from_dev(st["C"][:, sel]),
                       mat_from_dev(st["F"][:, sel]) + EYE, st["mass"][sel], st["vol0"][sel], mu, lam, sc.dt,
                       sc.material)
    assert rel(gm[nodes], om[nodes]) < TOL
    assert rel(gmv[:, nodes].T, omv[nodes]) < TOL


def test_grid_update_active_tiles(run):
    say(f"full-size {run['name']}: grid_update")
    sc = run["sc"]
    og = oracle_grid(sc.grid)
    lat = sc.lattice
    acc = owind.lbm_drag_to_nodes(og, (lat["nx"], lat["ny"], lat["nz"]), lat["dx"], lat["origin"], run["u"],
                                  sc.wind["vel_scale"], sc.wind["k_drag"])
    pin = torch.as_tensor(sc.pin)
    ov = ompm.grid_update(og, run["gm"], run["gmv"].T, sc.dt, sc.gravity, acc=acc, pin=pin, bound=sc.bound)
    V = run["sort"]
    nodes = _active_tile_nodes(og, V["node_tiles"][:int(V["n_node_tiles"])])
    say(f"  {nodes.numel()} nodes in active tiles")
    assert rel(run["gv"][:, nodes].T, ov[nodes]) < TOL


def test_g2p_sampled(run):
    say(f"full-size {run['name']}: g2p")
    sc = run["sc"]
    og = oracle_grid(sc.grid)
    st = run["state"]
    n = st["x"].shape[1]
    rng = np.random.default_rng(2)
    V = run["sort"]
    # random particles plus the first and last of a run of work items
    first = V["tile_start"][:-1][V["tile_count"] > 0].long()
    idx = torch.unique(torch.cat([torch.as_tensor(rng.choice(n, 20_000, replace=False)),
                                  first[torch.as_tensor(rng.choice(first.numel(), min(2000, first.numel()),
                                                                   replace=False))],
                                  torch.tensor([0, n - 1])]))
    xa = (run["xref"] + st["x"]).T[idx]
    x1, v1, C1, F1 = ompm.g2p(og, run["gv"].T, xa, mat_from_dev(st["F"][:, idx]) + EYE, sc.dt)
    post = run["post"]
    assert rel(vec_from_dev(post["x"][:, idx] - st["x"][:, idx]), x1 - xa) < TOL
    assert rel(vec_from_dev(post["v"][:, idx]), v1) < TOL
    assert rel(mat_from_dev(post["C"][:, idx]), C1) < TOL
    assert rel(mat_from_dev(post["F"][:, idx]), F1 - EYE) < TOL
