"""GPU parity of the hand-written adjoints against the oracle's float64 reverse
mode (torch.autograd over the forward definitions).

Each entry point's adjoint is fed seeded cotangents; the oracle differentiates
<cotangent, forward(inputs)> with autograd.  Gradients are compared with the
relative 2-norm error |g - g_oracle|_2 / |g_oracle|_2 <= 1e-3."""
import numpy as np
import pytest
import torch

from oracle import lbm as olbm
from oracle import mpm as ompm
from oracle import wind as owind
from paper_2603_09668_amd import api, scenes

from gpu_util import (DEV, EYE, api_grid, f32, mat_from_dev, mat_to_dev, oracle_grid, say, scene_state,
                      vec_from_dev, vec_to_dev)

pytestmark = pytest.mark.gpu
TOL = 1e-3


def rel2(a, b):
    a = torch.as_tensor(a).double().cpu().reshape(-1)
    b = torch.as_tensor(b).double().cpu().reshape(-1)
    return ((a - b).norm() / b.norm()).item()


@pytest.fixture(scope="module")
def scene():
    return scenes.flag_and_leaves_scene(seed=7, n=12_000, res=32, n_clusters=5, lbm_dims=(32, 16, 16),
                                        n_regions=3, E_range=(1e3, 1e4))


@pytest.mark.parametrize("det", [False, True])
@pytest.mark.parametrize("material", [api.FIXED_COROTATED, api.NEO_HOOKEAN])
def test_p2g_adj(scene, material, det):
    """det: the E adjoint summed in a fixed order (bit-identical on a second call)."""
    say(f"mpm_p2g_adj material={material} deterministic={det}")
    sc = scene
    st, dev = scene_state(sc, seed=3, scale_f=0.05)
    og = oracle_grid(sc.grid)
    g = api_grid(sc.grid)
    N = og.n_nodes
    rng = np.random.default_rng(4)
    mbar = f32(rng.standard_normal(N))
    mvbar = f32(rng.standard_normal((N, 3)))
    dt = 2e-4
    x = st["x"].clone().requires_grad_(True)
    v = st["v"].clone().requires_grad_(True)
    C = st["C"].clone().requires_grad_(True)
    F = st["F"].clone().requires_grad_(True)
    E = st["E"].clone().requires_grad_(True)
    mu, lam = ompm.particle_mu_lam(E, st["nu"], st["region"])
    m, mv = ompm.p2g(og, x, v, C, F, st["mass"], st["vol0"], mu, lam, dt, material)
    L = (m * mbar).sum() + (mv * mvbar).sum()
    gx, gv, gC, gF, gE = torch.autograd.grad(L, (x, v, C, F, E))
    xb = torch.zeros_like(dev.x)
    vb = torch.zeros_like(dev.v)
    Cb = torch.zeros_like(dev.C)
    Fb = torch.zeros_like(dev.F)
    Eb = torch.zeros_like(dev.E)
    prm = api.make_mpm_params(dt, material=material, deterministic=det)
    ws = api.alloc_workspace(g, sc.n, deterministic=True) if det else None
    args = (mbar.float().to(DEV), mvbar.T.contiguous().float().to(DEV))
    api.mpm_p2g_adj(g, prm, dev, *args, xb, vb, Cb, Fb, Eb, ws=ws)
    if det:
        Eb2 = torch.zeros_like(dev.E)
        api.mpm_p2g_adj(g, prm, dev, *args, E_bar=Eb2, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(Eb, Eb2)
    torch.cuda.synchronize()
    errs = dict(x=rel2(vec_from_dev(xb), gx), v=rel2(vec_from_dev(vb), gv), C=rel2(mat_from_dev(Cb), gC),
                F=rel2(mat_from_dev(Fb), gF), E=rel2(Eb.cpu(), gE))
    say("  " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e < TOL, k


def test_grid_update_adj(scene):
    sc = scene
    st, dev = scene_state(sc, seed=5)
    og = oracle_grid(sc.grid)
    g = api_grid(sc.grid)
    N = og.n_nodes
    mu, lam = ompm.particle_mu_lam(st["E"], st["nu"], st["region"])
    m0, mv0 = ompm.p2g(og, st["x"], st["v"], st["C"], st["F"], st["mass"], st["vol0"], mu, lam, sc.dt,
                       api.FIXED_COROTATED)
    m0, mv0 = f32(m0), f32(mv0)
    rng = np.random.default_rng(6)
    acc0 = f32(3.0 * rng.standard_normal((N, 3)))
    vbar = f32(rng.standard_normal((N, 3)))
    pin = torch.as_tensor(sc.pin)
    say("mpm_grid_update_adj")
    m = m0.clone().requires_grad_(True)
    mv = mv0.clone().requires_grad_(True)
    acc = acc0.clone().requires_grad_(True)
    vo = ompm.grid_update(og, m, mv, sc.dt, sc.gravity, acc=acc, pin=pin, bound=3)
    gm, gmv, ga = torch.autograd.grad((vo * vbar).sum(), (m, mv, acc))
    ws = api.alloc_workspace(g, sc.n)
    prm = api.make_mpm_params(sc.dt, gravity=sc.gravity, bound=3)
    api.mpm_sort(g, prm, dev.x, ws)
    mb = torch.zeros(N, device=DEV)
    mvb = torch.zeros(3, N, device=DEV)
    ab = torch.zeros(3, N, device=DEV)
    acc_d = acc0.T.contiguous().float().to(DEV)
    api.mpm_grid_update_adj(g, prm, m0.float().to(DEV), mv0.T.contiguous().float().to(DEV), api.wind_acc(acc_d),
                            pin.to(DEV), vbar.T.contiguous().float().to(DEV), mb, mvb, ab, ws)
    torch.cuda.synchronize()
    assert rel2(mb.cpu(), gm) < TOL
    assert rel2(mvb.cpu().T, gmv) < TOL
    assert rel2(ab.cpu().T, ga) < TOL


@pytest.mark.parametrize("det", [False, True])
def test_g2p_adj(scene, det):
    """det: deterministic sort and a fixed-order grid-velocity scatter
    (bit-identical on a second call)."""
    sc = scene
    st, dev = scene_state(sc, seed=7)
    og = oracle_grid(sc.grid)
    g = api_grid(sc.grid)
    N = og.n_nodes
    rng = np.random.default_rng(8)
    gv0 = f32(0.3 * rng.standard_normal((N, 3)))
    n = sc.n
    xob, vob = f32(rng.standard_normal((n, 3))), f32(rng.standard_normal((n, 3)))
    Cob, Fob = f32(rng.standard_normal((n, 3, 3))), f32(rng.standard_normal((n, 3, 3)))
    dt = 1e-3
    say(f"mpm_g2p_adj deterministic={det}")
    gvt = gv0.clone().requires_grad_(True)
    x = st["x"].clone().requires_grad_(True)
    F = st["F"].clone().requires_grad_(True)
    x1, v1, C1, F1 = ompm.g2p(og, gvt, x, F, dt)
    L = (x1 * xob).sum() + (v1 * vob).sum() + (C1 * Cob).sum() + (F1 * Fob).sum()
    ggv, gx, gF = torch.autograd.grad(L, (gvt, x, F))
    ws = api.alloc_workspace(g, n, deterministic=det)
    prm = api.make_mpm_params(dt, deterministic=det)
    api.mpm_sort(g, prm, dev.x, ws)
    xb = torch.zeros_like(dev.x)
    Fb = torch.zeros_like(dev.F)
    gvb = torch.zeros(3, N, device=DEV)
    cot = (vec_to_dev(xob), vec_to_dev(vob), mat_to_dev(Cob), mat_to_dev(Fob))
    api.mpm_g2p_adj(g, prm, gv0.T.contiguous().float().to(DEV), dev, *cot, xb, Fb, gvb, ws)
    if det:
        gvb2 = torch.zeros(3, N, device=DEV)
        api.mpm_g2p_adj(g, prm, gv0.T.contiguous().float().to(DEV), dev, *cot, None, None, gvb2, ws)
        torch.cuda.synchronize()
        assert torch.equal(gvb2, gvb)
    torch.cuda.synchronize()
    errs = dict(gv=rel2(gvb.cpu().T, ggv), x=rel2(vec_from_dev(xb), gx), F=rel2(mat_from_dev(Fb), gF))
    say("  " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e < TOL, k


@pytest.mark.parametrize("det", [False, True])
def test_wind_to_grid_adj(scene, det):
    """det: the transposes as fixed-order gathers (bit-identical on a second call)."""
    sc = scene
    og = oracle_grid(sc.grid)
    g = api_grid(sc.grid)
    N = og.n_nodes
    rng = np.random.default_rng(9)
    abar = f32(rng.standard_normal((N, 3)))
    abar[rng.random(N) < 0.5] = 0.0  # inactive nodes carry no adjoint
    say("wind_to_grid_adj force grid")
    nw = (16, 16, 16)
    W0 = f32(scenes.smooth_force_field(10, K=1, nw=16, amp=3.0))[0]
    W = W0.clone().requires_grad_(True)
    a = owind.force_grid_to_nodes(og, W, nw, (0, 0, 0), (1, 1, 1))
    (gW,) = torch.autograd.grad((a * abar).sum(), (W,))
    Wb = torch.zeros(3, 16 ** 3, device=DEV)
    wf = api.wind_force_grid(W0.float().to(DEV).contiguous(), nw, (0, 0, 0), (1, 1, 1), deterministic=det)
    api.wind_to_grid_adj(g, wf, abar.T.contiguous().float().to(DEV), Wb)
    if det:
        Wb2 = torch.zeros(3, 16 ** 3, device=DEV)
        api.wind_to_grid_adj(g, wf, abar.T.contiguous().float().to(DEV), Wb2)
        torch.cuda.synchronize()
        assert torch.equal(Wb, Wb2)
    torch.cuda.synchronize()
    assert rel2(Wb.cpu(), gW) < TOL
    say("wind_to_grid_adj drag")
    lat = sc.lattice
    dims = (lat["nx"], lat["ny"], lat["nz"])
    Lq = dims[0] * dims[1] * dims[2]
    u0 = f32(torch.tensor([0.08, 0.0, 0.0]).view(3, 1) + 0.02 * torch.tensor(rng.standard_normal((3, Lq))))
    u = u0.clone().requires_grad_(True)
    a = owind.lbm_drag_to_nodes(og, dims, lat["dx"], lat["origin"], u, 12.5, 9.8)
    (gu,) = torch.autograd.grad((a * abar).sum(), (u,))
    ub = torch.zeros(3, Lq, device=DEV)
    alat = api.make_lattice(*dims, lat["dx"], lat["origin"])
    wd = api.wind_lbm_drag(alat, u0.float().to(DEV).contiguous(), 12.5, 9.8, deterministic=det)
    api.wind_to_grid_adj(g, wd, abar.T.contiguous().float().to(DEV), ub)
    if det:
        ub2 = torch.zeros(3, Lq, device=DEV)
        api.wind_to_grid_adj(g, wd, abar.T.contiguous().float().to(DEV), ub2)
        torch.cuda.synchronize()
        assert torch.equal(ub, ub2)
    torch.cuda.synchronize()
    assert rel2(ub.cpu(), gu) < TOL


LBM_ADJ_CASES = {
    # inlet / outlet in x, bounce-back y, periodic z, gusty inflow
    "tunnel": dict(dims=(18, 12, 10), bc=(olbm.INLET, olbm.OUTLET, olbm.BOUNCEBACK, olbm.BOUNCEBACK,
                                          olbm.PERIODIC, olbm.PERIODIC), solid=(slice(3, 6), slice(4, 8), slice(7, 10))),
    # solids on the faces of a periodic box: wrapped pulls from solid nodes
    "periodic_face_solids": dict(dims=(14, 9, 8), bc=(olbm.PERIODIC,) * 6,
                                 solid=(slice(0, 2), slice(7, 9), slice(12, 14))),
    # solids against the outlet: clamped outlet pulls that land on solid nodes
    "outlet_solids": dict(dims=(20, 7, 6), bc=(olbm.INLET, olbm.OUTLET) + (olbm.BOUNCEBACK,) * 4,
                          solid=(slice(1, 4), slice(2, 5), slice(17, 20))),
    # bounce-back on all six faces
    "closed_box": dict(dims=(9, 8, 7), bc=(olbm.BOUNCEBACK,) * 6, solid=(slice(2, 4), slice(3, 5), slice(3, 6))),
    # rows wider than a workgroup, outlet clamps onto periodic y rows
    "wide_row": dict(dims=(200, 5, 4), bc=(olbm.INLET, olbm.OUTLET, olbm.PERIODIC, olbm.PERIODIC, olbm.BOUNCEBACK,
                                           olbm.BOUNCEBACK), solid=(slice(1, 3), slice(1, 3), slice(140, 180))),
}


@pytest.mark.parametrize("forced", [False, True])
@pytest.mark.parametrize("case", list(LBM_ADJ_CASES))
def test_lbm_step_adj(case, forced):
    """The reverse BGK step against float64 autograd of the oracle step:
    d/d f_in of <f_out_bar, f_out> + <u_bar, u_out>; bit-identical between
    calls (no atomics)."""
    c = LBM_ADJ_CASES[case]
    nx, ny, nz = c["dims"]
    say(f"lbm_step_adj {case} forced={forced}")
    rng = np.random.default_rng(11)
    rho = 1.0 + 0.01 * torch.tensor(rng.standard_normal((nz, ny, nx)))
    u = torch.tensor([0.05, 0.0, 0.0]).view(3, 1, 1, 1) + 0.02 * torch.tensor(rng.standard_normal((3, nz, ny, nx)))
    WQ = olbm.W.view(19, 1, 1, 1)
    fs = f32(olbm.equilibrium(rho.double(), u.double()) - WQ)
    solid = torch.zeros(nz, ny, nx, dtype=torch.bool)
    solid[c["solid"]] = True
    force = (2e-5, 1e-5, 0.0) if forced else (0.0, 0.0, 0.0)
    bc = c["bc"]
    op = olbm.LBMParams(tau=0.62, u_in=(0.05, 0, 0), force=force, bc=bc, gust_amp=0.05, gust_period=80.0,
                        gust_ky=1.0)
    ap = api.make_lbm_params(0.62, (0.05, 0, 0), force, bc, 0.05, 80.0, 1.0, 0.0, 0.0, t=5)
    lat = olbm.Lattice(nx, ny, nz)
    L = nx * ny * nz
    gbar = f32(rng.standard_normal((19, nz, ny, nx)))
    ubar = f32(rng.standard_normal((3, nz, ny, nx)))
    f = (fs + WQ).clone().requires_grad_(True)
    fo, rho_o, uo = olbm.lbm_step(lat, op, f, solid, 5)
    (gf,) = torch.autograd.grad((fo * gbar).sum() + (uo * ubar).sum(), (f,))
    alat = api.make_lattice(nx, ny, nz)
    args = (fs.reshape(19, L).float().to(DEV).contiguous(), solid.reshape(-1).to(torch.uint8).to(DEV),
            gbar.reshape(19, L).float().to(DEV).contiguous(), ubar.reshape(3, L).float().to(DEV).contiguous())
    fb = torch.full((19, L), 0.25, device=DEV)        # accumulates onto what is there
    work = torch.full((19, L), float("nan"), device=DEV)   # scratch: every entry is written before it is read
    api.lbm_step_adj(alat, ap, *args, fb, work=work)
    fb2 = torch.full((19, L), 0.25, device=DEV)
    api.lbm_step_adj(alat, ap, *args, fb2)
    torch.cuda.synchronize()
    assert torch.equal(fb, fb2)
    err = rel2(fb.cpu() - 0.25, gf.reshape(19, L))
    say(f"  rel error {err:.2e}")
    assert err < 1e-5      # measured about 9e-8 on every lattice


def _rel_drag_inputs(sc, og, seed):
    """Grid mass/momentum from P2G of a seeded state and a lattice velocity,
    rounded to float32 for both sides."""
    st, dev = scene_state(sc, seed=seed)
    mu, lam = ompm.particle_mu_lam(st["E"], st["nu"], st["region"])
    m0, mv0 = ompm.p2g(og, st["x"], st["v"], st["C"], st["F"], st["mass"], st["vol0"], mu, lam, sc.dt,
                       api.FIXED_COROTATED)
    lat = sc.lattice
    dims = (lat["nx"], lat["ny"], lat["nz"])
    Lq = dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(seed + 100)
    u0 = f32(torch.tensor([0.08, 0.0, 0.0]).view(3, 1) + 0.03 * torch.tensor(rng.standard_normal((3, Lq))))
    return st, dev, f32(m0), f32(mv0), lat, dims, u0


def test_grid_update_relative_drag(scene):
    """Forward and reverse of the grid update with the drag of the wind
    relative to the node velocity v* = mv / m."""
    sc = scene
    og = oracle_grid(sc.grid)
    g = api_grid(sc.grid)
    N = og.n_nodes
    st, dev, m0, mv0, lat, dims, u0 = _rel_drag_inputs(sc, og, 12)
    vs, kd = 12.5, 9.8
    alat = api.make_lattice(*dims, lat["dx"], lat["origin"])
    wind = api.wind_lbm_drag(alat, u0.float().to(DEV).contiguous(), vs, kd, relative=True)
    pin = torch.as_tensor(sc.pin)
    ws = api.alloc_workspace(g, sc.n)
    prm = api.make_mpm_params(sc.dt, gravity=sc.gravity, bound=3)
    api.mpm_sort(g, prm, dev.x, ws)
    say("mpm_grid_update relative drag")
    gv = torch.zeros(3, N, device=DEV)
    api.mpm_grid_update(g, prm, m0.float().to(DEV), mv0.T.contiguous().float().to(DEV), wind, pin.to(DEV), gv, ws)
    torch.cuda.synchronize()
    U, inside = owind.lbm_velocity_to_nodes(og, dims, lat["dx"], lat["origin"], u0, vs)
    ov = ompm.grid_update(og, m0, mv0, sc.dt, sc.gravity, pin=pin, bound=3, drag_rel=(U, inside, kd))
    assert (gv.cpu().T.double() - ov).abs().max().item() / ov.abs().max().item() < 1e-5
    # the drag really is relative: it differs from the absolute one
    gva = torch.zeros(3, N, device=DEV)
    api.mpm_grid_update(g, prm, m0.float().to(DEV), mv0.T.contiguous().float().to(DEV),
                        api.wind_lbm_drag(alat, u0.float().to(DEV).contiguous(), vs, kd), pin.to(DEV), gva, ws)
    torch.cuda.synchronize()
    assert (gva - gv).abs().max().item() > 1e-3 * gv.abs().max().item()
    say("mpm_grid_update_adj relative drag")
    rng = np.random.default_rng(13)
    vbar = f32(rng.standard_normal((N, 3)))
    m = m0.clone().requires_grad_(True)
    mv = mv0.clone().requires_grad_(True)
    Uv = U.clone().requires_grad_(True)
    vo = ompm.grid_update(og, m, mv, sc.dt, sc.gravity, pin=pin, bound=3, drag_rel=(Uv, inside, kd))
    gm, gmv, gU = torch.autograd.grad((vo * vbar).sum(), (m, mv, Uv))
    mb = torch.zeros(N, device=DEV)
    mvb = torch.zeros(3, N, device=DEV)
    Ub = torch.zeros(3, N, device=DEV)
    api.mpm_grid_update_adj(g, prm, m0.float().to(DEV), mv0.T.contiguous().float().to(DEV), wind, pin.to(DEV),
                            vbar.T.contiguous().float().to(DEV), mb, mvb, Ub, ws)
    torch.cuda.synchronize()
    assert rel2(mb.cpu(), gm) < TOL
    assert rel2(mvb.cpu().T, gmv) < TOL
    assert rel2(Ub.cpu().T, gU) < TOL
    say("wind_to_grid_adj relative drag (velocity transpose)")
    uv = u0.clone().requires_grad_(True)
    U2, _ = owind.lbm_velocity_to_nodes(og, dims, lat["dx"], lat["origin"], uv, vs)
    Ubar = f32(rng.standard_normal((N, 3)))
    (gu,) = torch.autograd.grad((U2 * Ubar).sum(), (uv,))
    ub = torch.zeros(3, dims[0] * dims[1] * dims[2], device=DEV)
    api.wind_to_grid_adj(g, wind, Ubar.T.contiguous().float().to(DEV), ub)
    torch.cuda.synchronize()
    assert rel2(ub.cpu(), gu) < TOL
    # wind_to_grid has no node velocity and refuses the relative drag
    with pytest.raises(api.DiffWindError):
        api.wind_to_grid(g, wind, torch.empty(3, N, device=DEV))


def test_lbm_reverse_work_checks():
    """The reverse LBM steps reject aliased outputs and work buffers of the
    wrong shape before launching anything; valid calls on the same buffers
    run."""
    nx, ny, nz = 8, 6, 5
    L = nx * ny * nz
    lat = api.make_lattice(nx, ny, nz)
    ap = api.make_lbm_params(0.7, (0.05, 0.0, 0.0), (0.0, 0.0, 0.0), (olbm.PERIODIC,) * 6, 0.0, 1.0, 0.0, 0.0, 0.0)
    f = torch.zeros(19, L, device=DEV)
    gb = torch.zeros_like(f)
    fb = torch.zeros_like(f)
    with pytest.raises(api.DiffWindError):
        api.lbm_step_adj(lat, ap, f, None, gb, None, fb, work=fb)
    with pytest.raises(ValueError):
        api.lbm_step_adj(lat, ap, f, None, gb, None, fb, work=torch.zeros(10, L, device=DEV))
    m = torch.zeros(10, L, device=DEV)
    mbar = torch.zeros_like(m)
    mib = torch.zeros_like(m)
    work = torch.zeros(19, L, device=DEV)
    with pytest.raises(api.DiffWindError):
        api.lbm_home_step_adj(lat, ap, m, None, mbar, None, m, work=work)   # m_in_bar aliases m_in
    with pytest.raises(ValueError):
        api.lbm_home_step_adj(lat, ap, m, None, mbar, None, mib, work=torch.zeros(10, L, device=DEV))
    # a valid call on the same buffers runs (zero adjoints stay zero)
    api.lbm_home_step_adj(lat, ap, m, None, mbar, None, mib, work=work)
    api.lbm_step_adj(lat, ap, f, None, gb, None, fb, work=work)
    torch.cuda.synchronize()
    assert mib.abs().max().item() == 0.0 and fb.abs().max().item() == 0.0
