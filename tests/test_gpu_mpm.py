"""GPU parity of the MPM entry points against the float64 oracle.

Inputs are seeded scenes rounded to float32 and fed identically to both
sides; outputs are compared element by element with norm-wise relative
errors |gpu - oracle|_inf / |oracle|_inf per field (1e-5 per call), and the
integer sort results bit-exactly against the oracle's definition taken in
float32."""
import numpy as np
import pytest
import torch

from oracle import mpm as ompm
from oracle import wind as owind
from paper_2603_09668_amd import api, scenes

from gpu_util import (DEV, EYE, api_grid, device_particles, f32, mat_from_dev, oracle_grid, rel, say, scene_state,
                      vec_from_dev, vec_to_dev)

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def sheet():
    return scenes.sheet_scene(seed=0, n=20_000)


@pytest.fixture(scope="module")
def leaves():
    # a small paper-style scene: sheet + leaf clusters on a 64^3 grid, ragged tiles
    return scenes.flag_and_leaves_scene(seed=3, n=30_000, res=64, n_clusters=6, lbm_dims=(64, 32, 32))


def _mu_lam(st):
    return ompm.particle_mu_lam(st["E"], st["nu"], st["region"])


@pytest.mark.parametrize("ref", [False, True])
def test_sort_matches_definition(sheet, leaves, ref):
    for sc in (sheet, leaves):
        say(f"mpm_sort {sc.name} ref={ref}")
        # with a position reference: a displacement of about a cell, so that
        # particles change cells and tiles relative to the reference
        st, dev = scene_state(sc, ref=ref, disp=0.5 * sc.grid["dx"] if ref else 0.0)
        g = api_grid(sc.grid)
        og = oracle_grid(sc.grid)
        ws = api.alloc_workspace(g, sc.n)
        api.mpm_sort(g, api.make_mpm_params(sc.dt), dev.x, ws, xref=dev.xref)
        torch.cuda.synchronize()
        V = api.workspace_views(g, sc.n, ws)
        if ref:
            base = ompm.stencil_base_f32(st["disp"], og, xref32=st["xref"])
        else:
            base = ompm.stencil_base_f32(st["x"], og)
        keys = ompm.cell_tile_keys(None, og, base=base)
        perm = V["perm"].cpu().long()
        assert int(V["status"]) == 0
        assert torch.equal(torch.sort(perm).values, torch.arange(sc.n))
        assert torch.all(keys[perm][1:] >= keys[perm][:-1])
        counts = torch.bincount(keys, minlength=V["n_tiles"])
        assert torch.equal(V["tile_count"].cpu().long(), counts)
        start = torch.zeros(V["n_tiles"] + 1, dtype=torch.long)
        start[1:] = torch.cumsum(counts, 0)
        assert torch.equal(V["tile_start"].cpu().long(), start)
        ncell = int(V["n_cell_tiles"])
        assert torch.equal(V["cell_tiles"][:ncell].cpu().long(), torch.nonzero(counts).flatten())
        nnode = int(V["n_node_tiles"])
        assert V["node_tiles"][:nnode].cpu().tolist() == ompm.active_node_tiles(None, og, base=base)


def test_reorder_is_the_sort_permutation(leaves):
    """mpm_reorder writes every per-particle array in the sort's order,
    bit for bit, and the result is grouped by cell tile; a substep of the
    reordered set equals the original substep, permuted."""
    sc = leaves
    say(f"mpm_reorder {sc.name}")
    st, dev = scene_state(sc)
    g = api_grid(sc.grid)
    og = oracle_grid(sc.grid)
    ws = api.alloc_workspace(g, sc.n)
    prm = api.make_mpm_params(sc.dt, sc.gravity, sc.bound, sc.material)
    rng = np.random.default_rng(3)
    dev = dev.with_state(dev.x, torch.tensor(rng.standard_normal((3, sc.n)), dtype=torch.float32, device=DEV),
                         torch.tensor(0.1 * rng.standard_normal((9, sc.n)), dtype=torch.float32, device=DEV),
                         torch.tensor(0.01 * rng.standard_normal((9, sc.n)), dtype=torch.float32, device=DEV))
    api.mpm_sort(g, prm, dev.x, ws)
    perm = torch.empty(sc.n, dtype=torch.int32, device=DEV)
    out = api.mpm_reorder(g, dev, ws, perm_out=perm)
    V = api.workspace_views(g, sc.n, ws)
    assert torch.equal(perm, V["perm"][:sc.n])
    pl = perm.long()
    for name in ("x", "v", "C", "F"):
        assert torch.equal(getattr(out, name), getattr(dev, name)[:, pl]), name
    for name in ("mass", "vol0", "region"):
        assert torch.equal(getattr(out, name), getattr(dev, name)[pl]), name
    base = ompm.stencil_base_f32(torch.as_tensor(out.x.T.double().cpu()), og)
    keys = ompm.cell_tile_keys(None, og, base=base)
    assert torch.all(keys[1:] >= keys[:-1])
    # one substep on each order
    N = sc.grid["nx"] * sc.grid["ny"] * sc.grid["nz"]
    res = []
    for p in (dev, out):
        gm, gmv, gv = torch.zeros(N, device=DEV), torch.zeros(3, N, device=DEV), torch.zeros(3, N, device=DEV)
        api.mpm_sort(g, prm, p.x, ws)
        api.mpm_p2g(g, prm, p, gm, gmv, ws)
        api.mpm_grid_update(g, prm, gm, gmv, api.wind_none(), None, gv, ws)
        o = [torch.empty_like(t) for t in (p.x, p.v, p.C, p.F)]
        api.mpm_g2p(g, prm, gv, p, *o)
        res.append(o)
    for a, b in zip(res[0], res[1]):
        assert rel(b, a[:, pl]) < 1e-5
    # in and out sharing arrays is refused before any launch
    same = dev.struct()
    rc = api.lib().mpm_reorder(api.ctypes.byref(g), api.ctypes.byref(same), api.ctypes.byref(same), None,
                               api._ptr(ws, torch.uint8, "ws"), ws.numel(), api._stream())
    assert rc != 0 and "share" in api.dw_last_error()


@pytest.mark.parametrize("strain", [0.05, 0.005])
@pytest.mark.parametrize("material", [api.FIXED_COROTATED, api.NEO_HOOKEAN])
@pytest.mark.parametrize("scene_name", ["sheet", "leaves"])
def test_p2g_parity(material, scene_name, strain, request):
    """strain 0.05 takes the fixed-corotated stress through the polar
    decomposition, 0.005 (|F F^T - I| below 0.05) through the stretch series."""
    sc = request.getfixturevalue(scene_name)
    say(f"mpm_p2g {sc.name} material={material} strain={strain}")
    st, dev = scene_state(sc, seed=5, scale_f=strain)
    g = api_grid(sc.grid)
    og = oracle_grid(sc.grid)
    N = og.n_nodes
    ws = api.alloc_workspace(g, sc.n)
    gm = torch.zeros(N, device=DEV)
    gmv = torch.zeros(3, N, device=DEV)
    prm = api.make_mpm_params(sc.dt, material=material)
    api.mpm_sort(g, prm, dev.x, ws)
    api.mpm_p2g(g, prm, dev, gm, gmv, ws)
    torch.cuda.synchronize()
    mu, lam = _mu_lam(st)
    om, omv = ompm.p2g(og, st["x"], st["v"], st["C"], st["F"], st["mass"], st["vol0"], mu, lam, sc.dt, material)
    assert rel(gm.cpu(), om) < TOL
    assert rel(gmv.cpu().T, omv) < TOL
    assert api.read_status(ws) == 0


def test_p2g_overwrites_active_tiles(sheet):
    """A second call on a dirty grid gives the same sums (active tiles are cleared)."""
    st, dev = scene_state(sheet, seed=6)
    g = api_grid(sheet.grid)
    N = sheet.grid["nx"] ** 3
    ws = api.alloc_workspace(g, sheet.n)
    gm = torch.zeros(N, device=DEV)
    gmv = torch.zeros(3, N, device=DEV)
    prm = api.make_mpm_params(sheet.dt)
    api.mpm_sort(g, prm, dev.x, ws)
    api.mpm_p2g(g, prm, dev, gm, gmv, ws)
    m1, mv1 = gm.clone(), gmv.clone()
    api.mpm_p2g(g, prm, dev, gm, gmv, ws)
    torch.cuda.synchronize()
    # atomics may sum in another order; a stale grid would double the sums
    assert rel(gm, m1) < 1e-5 and rel(gmv, mv1) < 1e-5


def _wind_cases(sc, og):
    """(name, api wind, oracle acceleration (N, 3)) for the three wind sources."""
    rng = np.random.default_rng(8)
    N = og.n_nodes
    cases = [("none", None, torch.zeros(N, 3, dtype=torch.float64))]
    W = f32(scenes.smooth_force_field(9, K=1, nw=6, amp=4.0))[0]
    lo, hi = (0.1, 0.0, 0.05), (0.9, 1.0, 0.95)
    cases.append(("force_grid", api.wind_force_grid(W.float().to(DEV).contiguous(), (6, 6, 6), lo, hi),
                  owind.force_grid_to_nodes(og, W, (6, 6, 6), lo, hi)))
    lat = sc.lattice
    L = lat["nx"] * lat["ny"] * lat["nz"]
    u = f32(0.05 * rng.standard_normal((3, L)))
    alat = api.make_lattice(lat["nx"], lat["ny"], lat["nz"], lat["dx"], lat["origin"])
    cases.append(("lbm_drag", api.wind_lbm_drag(alat, u.float().to(DEV).contiguous(), 20.0, 9.8),
                  owind.lbm_drag_to_nodes(og, (lat["nx"], lat["ny"], lat["nz"]), lat["dx"], lat["origin"], u,
                                          20.0, 9.8)))
    return cases


@pytest.mark.parametrize("scene_name", ["sheet", "leaves"])
def test_grid_update_parity(scene_name, request):
    sc = request.getfixturevalue(scene_name)
    st, dev = scene_state(sc, seed=7)
    g = api_grid(sc.grid)
    og = oracle_grid(sc.grid)
    N = og.n_nodes
    mu, lam = _mu_lam(st)
    om, omv = ompm.p2g(og, st["x"], st["v"], st["C"], st["F"], st["mass"], st["vol0"], mu, lam, sc.dt,
                       api.FIXED_COROTATED)
    om, omv = f32(om), f32(omv)
    ws = api.alloc_workspace(g, sc.n)
    prm = api.make_mpm_params(sc.dt, gravity=sc.gravity, bound=3)
    api.mpm_sort(g, prm, dev.x, ws)
    pin = torch.as_tensor(sc.pin)
    for name, wind, acc in _wind_cases(sc, og):
        say(f"mpm_grid_update {sc.name} wind={name}")
        gv = torch.zeros(3, N, device=DEV)
        api.mpm_grid_update(g, prm, om.float().to(DEV), omv.T.contiguous().float().to(DEV), wind,
                            pin.to(DEV), gv, ws)
        torch.cuda.synchronize()
        ov = ompm.grid_update(og, om, omv, sc.dt, sc.gravity, acc=acc, pin=pin, bound=3)
        assert rel(gv.cpu().T, ov) < TOL, name


@pytest.mark.parametrize("ref", [False, True])
@pytest.mark.parametrize("scene_name", ["sheet", "leaves"])
def test_g2p_parity(scene_name, ref, request):
    sc = request.getfixturevalue(scene_name)
    say(f"mpm_g2p {sc.name} ref={ref}")
    # a stored displacement of ~1e-4: the new displacement is rounded to
    # float32 at its own size, 2^-24 |x| ~ 6e-12, against a step dt v of
    # 4e-6 (leaves) to 2e-5 (sheet)
    st, dev = scene_state(sc, seed=11, ref=ref, disp=1e-4 if ref else 0.0)
    _g2p_check(sc, st, dev)


def test_g2p_parity_unsorted_particles(leaves):
    """Particles in random order: the blocks' stencil boxes are too large to
    stage and G2P gathers from global memory."""
    sc = leaves
    say(f"mpm_g2p {sc.name} shuffled")
    st, _ = scene_state(sc, seed=11)
    perm = torch.as_tensor(np.random.default_rng(5).permutation(sc.n))
    st = {k: (v[perm] if torch.is_tensor(v) and v.shape[:1] == (sc.n,) else v) for k, v in st.items()}
    dev = device_particles(st["x"], st["v"], st["C"], st["F"], st["mass"], st["vol0"], st["region"], st["E"],
                           st["nu"])
    _g2p_check(sc, st, dev)


def _g2p_check(sc, st, dev):
    og = oracle_grid(sc.grid)
    g = api_grid(sc.grid)
    rng = np.random.default_rng(12)
    gv = f32(0.2 * rng.standard_normal((og.n_nodes, 3)))
    xo = torch.empty_like(dev.x)
    vo = torch.empty_like(dev.v)
    Co = torch.empty_like(dev.C)
    Fo = torch.empty_like(dev.F)
    api.mpm_g2p(g, api.make_mpm_params(sc.dt), gv.T.contiguous().float().to(DEV), dev, xo, vo, Co, Fo)
    torch.cuda.synchronize()
    x1, v1, C1, F1 = ompm.g2p(og, gv, st["x"], st["F"], sc.dt)
    if dev.xref is None:
        assert rel(vec_from_dev(xo), x1) < TOL
    else:
        # displacements: the step dt v_p itself is resolved
        assert rel(vec_from_dev(xo) - st["disp"], x1 - st["x"]) < TOL
    assert rel(vec_from_dev(vo), v1) < TOL
    assert rel(mat_from_dev(Co), C1) < TOL
    # F is stored as F - I: compare the strain part itself
    assert rel(mat_from_dev(Fo), F1 - EYE) < TOL


def test_wind_to_grid_parity(sheet):
    og = oracle_grid(sheet.grid)
    g = api_grid(sheet.grid)
    for name, wind, acc in _wind_cases(sheet, og)[1:]:
        say(f"wind_to_grid {name}")
        out = torch.empty(3, og.n_nodes, device=DEV)
        api.wind_to_grid(g, wind, out)
        torch.cuda.synchronize()
        assert rel(out.cpu().T, acc) < TOL, name


def _gpu_rollout(sc, dev, steps, W=None, nw=None, material=api.FIXED_COROTATED):
    g = api_grid(sc.grid)
    N = sc.grid["nx"] * sc.grid["ny"] * sc.grid["nz"]
    ws = api.alloc_workspace(g, sc.n)
    gm = torch.zeros(N, device=DEV)
    gmv = torch.zeros(3, N, device=DEV)
    gv = torch.zeros(3, N, device=DEV)
    pin = torch.as_tensor(sc.pin).to(DEV)
    prm = api.make_mpm_params(sc.dt, gravity=sc.gravity, bound=3, material=material)
    p = dev
    for s in range(steps):
        wind = None if W is None else api.wind_force_grid(W[s * W.shape[0] // steps], nw, (0, 0, 0), (1, 1, 1))
        api.mpm_sort(g, prm, p.x, ws, xref=p.xref)
        api.mpm_p2g(g, prm, p, gm, gmv, ws)
        api.mpm_grid_update(g, prm, gm, gmv, wind, pin, gv, ws)
        xo, vo, Co, Fo = (torch.empty_like(p.x), torch.empty_like(p.v), torch.empty_like(p.C), torch.empty_like(p.F))
        api.mpm_g2p(g, prm, gv, p, xo, vo, Co, Fo)
        p = p.with_state(xo, vo, Co, Fo)
    torch.cuda.synchronize()
    return p, api.read_status(ws)


def _oracle_rollout(sc, st, steps, W=None, nw=None, material=api.FIXED_COROTATED):
    og = oracle_grid(sc.grid)
    mu, lam = _mu_lam(st)
    state = {k: st[k] for k in ("x", "v", "C", "F")}
    pin = torch.as_tensor(sc.pin)
    for s in range(steps):
        acc = None
        if W is not None:
            acc = owind.force_grid_to_nodes(og, W[s * W.shape[0] // steps].double(), nw, (0, 0, 0), (1, 1, 1))
        state, _ = ompm.substep(og, state, st["mass"], st["vol0"], mu, lam, sc.dt, material, gravity=sc.gravity,
                                acc=acc, pin=pin, bound=3)
    return state


@pytest.mark.parametrize("ref", [False, True])
def test_one_substep_parity(sheet, ref):
    """One substep; with a position reference the displacement of the
    substep, x_new - x, is held to 1e-5 of its own size."""
    say(f"substep sheet32 x1 ref={ref}")
    st, dev = scene_state(sheet, seed=13, scale_f=0.02, ref=ref, disp=1e-4 if ref else 0.0)
    p, status = _gpu_rollout(sheet, dev, 1)
    o = _oracle_rollout(sheet, st, 1)
    assert status == 0
    if ref:
        err = rel(vec_from_dev(p.x) - st["disp"], o["x"] - st["x"])
        say(f"  substep displacement {err:.2e}")
        assert err < TOL
    else:
        assert rel(vec_from_dev(p.x), o["x"]) < TOL
    assert rel(vec_from_dev(p.v), o["v"]) < TOL
    assert rel(mat_from_dev(p.C), o["C"]) < TOL
    assert rel(mat_from_dev(p.F), o["F"] - EYE) < TOL


def test_rest_state_is_exact(sheet):
    say("substep rest state")
    st, dev = scene_state(sheet)
    sc = sheet
    g = api_grid(sc.grid)
    N = sc.grid["nx"] ** 3
    ws = api.alloc_workspace(g, sc.n)
    gm, gmv, gv = torch.zeros(N, device=DEV), torch.zeros(3, N, device=DEV), torch.zeros(3, N, device=DEV)
    prm = api.make_mpm_params(sc.dt, bound=3)
    api.mpm_sort(g, prm, dev.x, ws)
    api.mpm_p2g(g, prm, dev, gm, gmv, ws)
    api.mpm_grid_update(g, prm, gm, gmv, None, None, gv, ws)
    xo, vo, Co, Fo = (torch.empty_like(dev.x), torch.empty_like(dev.v), torch.empty_like(dev.C),
                      torch.empty_like(dev.F))
    api.mpm_g2p(g, prm, gv, dev, xo, vo, Co, Fo)
    torch.cuda.synchronize()
    assert torch.equal(xo, dev.x) and torch.equal(Fo, dev.F)
    assert vo.abs().max().item() == 0 and Co.abs().max().item() == 0


def test_rollout_100_substeps(sheet):
    """Plain method: 100 substeps of the pinned sheet under gravity and a
    force-grid wind, against the float64 oracle at 1e-3 relative per field.
    F is compared through its stored strain part F - I.  Positions are kept
    as the scene's positions plus a float32 displacement, and the
    displacement x(T) - x(0) is held to 1e-3 of |x(T) - x(0)|_oracle,inf."""
    say("rollout sheet32 x100")
    steps = 100
    W = f32(scenes.smooth_force_field(21, K=4, nw=8, amp=20.0))
    st, dev = scene_state(sheet, ref=True)
    p, status = _gpu_rollout(sheet, dev, steps, W.float().to(DEV).contiguous(), (8, 8, 8))
    o = _oracle_rollout(sheet, st, steps, W, (8, 8, 8))
    assert status == 0
    errs = {
        "disp": rel(vec_from_dev(p.x), o["x"] - st["x"]),
        "v": rel(vec_from_dev(p.v), o["v"]),
        "C": rel(mat_from_dev(p.C), o["C"]),
        "F-I": rel(mat_from_dev(p.F), o["F"] - EYE),
    }
    say("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e < 1e-3, (k, e)


def test_out_of_grid_particle_is_flagged(sheet):
    say("mpm_p2g out-of-grid status")
    st, dev = scene_state(sheet, seed=14)
    x = dev.x.clone()
    x[0, 0] = 0.01  # base cell -1 on x
    dev2 = dev.with_state(x, dev.v, dev.C, dev.F)
    g = api_grid(sheet.grid)
    N = sheet.grid["nx"] ** 3
    ws = api.alloc_workspace(g, sheet.n)
    gm, gmv = torch.zeros(N, device=DEV), torch.zeros(3, N, device=DEV)
    prm = api.make_mpm_params(sheet.dt)
    api.mpm_sort(g, prm, dev2.x, ws)
    api.mpm_p2g(g, prm, dev2, gm, gmv, ws)
    torch.cuda.synchronize()
    assert api.read_status(ws) & api.STATUS_OUT_OF_GRID
    # the other particles are all deposited
    assert abs(gm.sum().item() - (st["mass"].sum().item() - st["mass"][0].item())) < 1e-5 * st["mass"].sum().item()


def test_empty_particle_set(sheet):
    say("mpm_p2g n=0")
    g = api_grid(sheet.grid)
    N = sheet.grid["nx"] ** 3
    ws = api.alloc_workspace(g, 0)
    e = torch.empty(3, 0, device=DEV)
    e9 = torch.empty(9, 0, device=DEV)
    z = torch.empty(0, device=DEV)
    p = api.ParticleArrays(e, e.clone(), e9, e9.clone(), z, z.clone(), torch.empty(0, dtype=torch.int32, device=DEV),
                           torch.ones(1, device=DEV), torch.full((1,), 0.3, device=DEV))
    gm, gmv = torch.zeros(N, device=DEV), torch.zeros(3, N, device=DEV)
    api.mpm_sort(g, api.make_mpm_params(1e-4), p.x, ws)
    api.mpm_p2g(g, api.make_mpm_params(1e-4), p, gm, gmv, ws)
    torch.cuda.synchronize()
    assert gm.abs().max().item() == 0
    V = api.workspace_views(g, 0, ws)
    assert int(V["n_cell_tiles"]) == 0 and int(V["n_node_tiles"]) == 0


def _det_rollout(sc, steps, deterministic):
    st, dev = scene_state(sc, seed=31, scale_f=0.01)
    g = api_grid(sc.grid)
    N = sc.grid["nx"] * sc.grid["ny"] * sc.grid["nz"]
    ws = api.alloc_workspace(g, sc.n, deterministic=deterministic)
    gm, gmv, gv = torch.zeros(N, device=DEV), torch.zeros(3, N, device=DEV), torch.zeros(3, N, device=DEV)
    prm = api.make_mpm_params(sc.dt, gravity=sc.gravity, bound=3, deterministic=deterministic)
    pin = torch.as_tensor(sc.pin).to(DEV)
    p = dev
    for s in range(steps):
        api.mpm_sort(g, prm, p.x, ws)
        api.mpm_p2g(g, prm, p, gm, gmv, ws)
        api.mpm_grid_update(g, prm, gm, gmv, None, pin, gv, ws)
        api.mpm_g2p(g, prm, gv, p, p.x, p.v, p.C, p.F)
    torch.cuda.synchronize()
    return p, gm, gmv, api.read_status(ws)


def test_deterministic_mode_is_bit_reproducible(leaves):
    say("deterministic rollout x2")
    a, gma, gmva, sa = _det_rollout(leaves, 20, True)
    b, gmb, gmvb, sb = _det_rollout(leaves, 20, True)
    assert sa == 0 and sb == 0
    for name in ("x", "v", "C", "F"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert torch.equal(gma, gmb) and torch.equal(gmva, gmvb)
    c, gmc, gmvc, _ = _det_rollout(leaves, 20, False)
    assert rel(vec_from_dev(a.v), vec_from_dev(c.v)) < 1e-5


def test_deterministic_p2g_matches_oracle(leaves):
    say("mpm_p2g deterministic vs oracle")
    sc = leaves
    st, dev = scene_state(sc, seed=32)
    g = api_grid(sc.grid)
    og = oracle_grid(sc.grid)
    ws = api.alloc_workspace(g, sc.n, deterministic=True)
    gm = torch.full((og.n_nodes,), 7.0, device=DEV)  # dirty: active tiles are overwritten
    gmv = torch.zeros(3, og.n_nodes, device=DEV)
    prm = api.make_mpm_params(sc.dt, deterministic=True)
    api.mpm_sort(g, prm, dev.x, ws)
    api.mpm_p2g(g, prm, dev, gm, gmv, ws)
    torch.cuda.synchronize()
    mu, lam = _mu_lam(st)
    om, omv = ompm.p2g(og, st["x"], st["v"], st["C"], st["F"], st["mass"], st["vol0"], mu, lam, sc.dt,
                       api.FIXED_COROTATED)
    V = api.workspace_views(g, sc.n, ws)
    tiles = V["node_tiles"][:int(V["n_node_tiles"])].cpu().long()
    # compare on the active node tiles (the rest keeps the dirty value)
    nx = sc.grid["nx"]
    T = nx // 4
    loc = torch.stack(torch.meshgrid(torch.arange(4), torch.arange(4), torch.arange(4), indexing="ij"), -1).reshape(-1, 3)
    tz, ty, tx = tiles // (T * T), (tiles // T) % T, tiles % T
    k = (tz[:, None] * 4 + loc[None, :, 0]).reshape(-1)
    j = (ty[:, None] * 4 + loc[None, :, 1]).reshape(-1)
    i = (tx[:, None] * 4 + loc[None, :, 2]).reshape(-1)
    nodes = i + nx * (j + nx * k)
    assert rel(gm.cpu()[nodes], om[nodes]) < TOL
    assert rel(gmv.cpu().T[nodes], omv[nodes]) < TOL
    assert rel(gm.cpu()[nodes].sum(), om.sum()) < 1e-6
