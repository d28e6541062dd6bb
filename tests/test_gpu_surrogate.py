"""Parity of the BF16 MFMA surrogate kernels with the float64 oracle
convolution, on identical BF16-rounded inputs and weights, and tests of the
surrogate's training, checks and plain-LBM fallback.

Tolerances follow from the arithmetic: products of BF16 numbers are exact in
FP32, so an FP32 result differs from the float64 one by the accumulation
error, bounded here by 1e-4 of the sum of absolute terms (at most ~900 terms
per output, ~30 sequential additions per wgrad partial); a BF16 output adds
half an ulp, 2^-8 relative."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as tF

from oracle import conv as oconv
from paper_2603_09668_amd import api
from paper_2603_09668_amd import surrogate as sg

from gpu_util import DEV, say

pytestmark = pytest.mark.gpu

U_BF = 2.0 ** -8
ACC = 1e-4


def _bf(t):
    """round to BF16 (nearest even) and return float64."""
    return t.to(torch.bfloat16).double()


def _to_dev_act(x, cp):
    """(B, C, nz, ny, nx) float64 -> device BF16 [B][L][cp] (channels zero padded)."""
    B, C = x.shape[:2]
    a = torch.zeros(B, *x.shape[2:], cp, dtype=torch.float64)
    a[..., :C] = x.permute(0, 2, 3, 4, 1)
    return a.to(torch.bfloat16).reshape(-1).to(DEV)


def _from_dev_act(a, dims, C, cp):
    B, nx, ny, nz = dims
    return a.view(B, nz, ny, nx, cp)[..., :C].permute(0, 4, 1, 2, 3).double().cpu()


def _rand_act(rng, dims, C, scale=1.0):
    B, nx, ny, nz = dims
    return _bf(torch.tensor(scale * rng.standard_normal((B, C, nz, ny, nx))))


def _rand_w(rng, cin, cout):
    w = torch.tensor(rng.standard_normal((cout, cin, 27)) / math.sqrt(27 * cin), dtype=torch.float32)
    return w, _bf(w).view(cout, cin, 3, 3, 3)


def _cp(c):
    return 8 if c == 3 else 32


def _pack(w, cin, cout, flip):
    n = api.conv_packed_weight_elems(cout if flip else cin, cin if flip else cout)
    wk = torch.empty(n, dtype=torch.bfloat16, device=DEV)
    api.conv_pack_weights(w.to(DEV), cin, cout, flip, wk)
    return wk


def _check(name, got, ref, bound):
    err = (got - ref).abs()
    worst = (err - bound).max().item()
    say(f"  {name}: max err {err.max().item():.3e}  max|ref| {ref.abs().max().item():.3e}  slack {worst:.3e}")
    assert worst <= 0, f"{name}: error exceeds bound by {worst}"


DIMS = [(2, 40, 9, 6), (1, 32, 8, 8)]  # ragged edge tiles; exact tiles


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("cin", [3, 32])
def test_hidden_layer_forward(dims, cin):
    say(f"hidden forward dims={dims} cin={cin}")
    rng = np.random.default_rng(10 + cin)
    x = _rand_act(rng, dims, cin)
    w, w64 = _rand_w(rng, cin, 32)
    b = torch.tensor(0.1 * rng.standard_normal(32), dtype=torch.float32)
    B, nx, ny, nz = dims
    y = torch.empty(B * nx * ny * nz * 32, dtype=torch.bfloat16, device=DEV)
    zp = torch.empty_like(y)
    api.conv3d_bf16(dims, cin, 32, api.CONV_HIDDEN, _to_dev_act(x, _cp(cin)), _pack(w, cin, 32, 0),
                    bias=b.to(DEV), y=y, zpre=zp)
    z_ref = tF.conv3d(x, w64, b.double(), padding=1)
    a_ref = tF.conv3d(x.abs(), w64.abs(), b.double().abs(), padding=1)
    _check("zpre", _from_dev_act(zp, dims, 32, 32), z_ref, U_BF * z_ref.abs() + 2 * ACC * a_ref)
    s_ref = oconv.silu(z_ref)
    _check("silu", _from_dev_act(y, dims, 32, 32), s_ref, U_BF * s_ref.abs() + 3 * ACC * a_ref + 1e-6)


@pytest.mark.parametrize("dims", DIMS)
def test_output_layer_forward(dims):
    say(f"output forward dims={dims}")
    rng = np.random.default_rng(7)
    B, nx, ny, nz = dims
    x = _rand_act(rng, dims, 32)
    w, w64 = _rand_w(rng, 32, 3)
    b = torch.tensor(0.1 * rng.standard_normal(3), dtype=torch.float32)
    u = torch.tensor(0.05 * rng.standard_normal((B, 3, nz * ny * nx)), dtype=torch.float32)
    s = torch.tensor(rng.uniform(0.02, 0.1, B), dtype=torch.float32)
    uo = torch.empty(B, 3, nz * ny * nx, device=DEV)
    api.conv3d_bf16(dims, 32, 3, api.CONV_OUTPUT, _to_dev_act(x, 32), _pack(w, 32, 3, 0), bias=b.to(DEV),
                    u=u.to(DEV), scale=s.to(DEV), u_out=uo)
    z = tF.conv3d(x, w64, b.double(), padding=1).reshape(B, 3, -1)
    a = tF.conv3d(x.abs(), w64.abs(), b.double().abs(), padding=1).reshape(B, 3, -1)
    sv = s.double().view(-1, 1, 1)
    ref = u.double() + sv * z
    _check("u_out", uo.double().cpu(), ref, 2 * ACC * sv * a + 1e-6 * (u.double().abs() + sv * z.abs()))


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("cout", [32, 3])
def test_data_gradient(dims, cout):
    """conv^T of the output gradient times silu'(zgate), for the layer 32 -> cout."""
    say(f"dgrad dims={dims} cout={cout}")
    rng = np.random.default_rng(20 + cout)
    B, nx, ny, nz = dims
    g = _rand_act(rng, dims, cout, 1e-3)
    zg = _rand_act(rng, dims, 32, 2.0)
    w, w64 = _rand_w(rng, 32, cout)
    y = torch.empty(B * nx * ny * nz * 32, dtype=torch.bfloat16, device=DEV)
    api.conv3d_bf16(dims, 32, cout, api.CONV_DGRAD, _to_dev_act(g, _cp(cout)), _pack(w, 32, cout, 1), y=y,
                    zgate=_to_dev_act(zg, 32))
    shape = (B, 32, nz, ny, nx)
    dx = torch.nn.grad.conv3d_input(shape, w64, g, padding=1)
    da = torch.nn.grad.conv3d_input(shape, w64.abs(), g.abs(), padding=1)
    sig = torch.sigmoid(zg)
    gate = sig * (1 + zg * (1 - sig))
    ref = dx * gate
    _check("dgrad", _from_dev_act(y, dims, 32, 32), ref, U_BF * ref.abs() + 2 * ACC * da * gate.abs())


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("cin,cout", [(3, 32), (32, 32), (32, 3)])
def test_weight_and_bias_gradient(dims, cin, cout):
    say(f"wgrad dims={dims} {cin}->{cout}")
    rng = np.random.default_rng(30 + cin + cout)
    B, nx, ny, nz = dims
    x = _rand_act(rng, dims, cin)
    dz = _rand_act(rng, dims, cout, 1e-2)
    dw = torch.empty(cout, cin, 27, device=DEV)
    db = torch.empty(cout, device=DEV)
    scratch = torch.empty(api.conv_wgrad_scratch_floats(), device=DEV)
    xd, dzd = _to_dev_act(x, _cp(cin)), _to_dev_act(dz, _cp(cout))
    api.conv3d_bf16_wgrad(dims, cin, cout, xd, dzd, dw, db, scratch)
    wshape = (cout, cin, 3, 3, 3)
    ref = torch.nn.grad.conv3d_weight(x, wshape, dz, padding=1).reshape(cout, cin, 27)
    a = torch.nn.grad.conv3d_weight(x.abs(), wshape, dz.abs(), padding=1).reshape(cout, cin, 27)
    _check("dW", dw.double().cpu(), ref, ACC * a + 1e-30)
    bref = dz.sum(dim=(0, 2, 3, 4))
    _check("db", db.double().cpu(), bref, ACC * dz.abs().sum(dim=(0, 2, 3, 4)) + 1e-30)
    # accumulate = 1 adds a second gradient on top
    dw1, db1 = dw.clone(), db.clone()
    api.conv3d_bf16_wgrad(dims, cin, cout, xd, dzd, dw, db, scratch, accumulate=True)
    assert torch.equal(dw, dw1 + dw1) or (dw - 2 * dw1).abs().max().item() <= 1e-6 * dw1.abs().max().item()
    assert (db - 2 * db1).abs().max().item() <= 1e-6 * db1.abs().max().item()
    # fixed-order reduction: a repeat gives identical bits
    dw2 = torch.empty_like(dw)
    api.conv3d_bf16_wgrad(dims, cin, cout, xd, dzd, dw2, None, scratch)
    assert torch.equal(dw2, dw1)


def test_prep_input_and_mse_grad():
    say("prep input / mse grad")
    rng = np.random.default_rng(3)
    dims = (3, 20, 5, 7)
    B, nx, ny, nz = dims
    L = nx * ny * nz
    u = torch.tensor(0.05 * rng.standard_normal((B, 3, L)), dtype=torch.float32)
    t = torch.tensor(0.05 * rng.standard_normal((B, 3, L)), dtype=torch.float32)
    s = torch.tensor([0.03, 0.05, 0.09], dtype=torch.float32)
    x0 = torch.empty(B * L * 8, dtype=torch.bfloat16, device=DEV)
    api.conv_prep_input(dims, u.to(DEV), s.to(DEV), x0)
    xr = x0.view(B, L, 8).double().cpu()
    ref = (u.double() / s.double().view(-1, 1, 1)).transpose(1, 2)
    _check("x0", xr[..., :3], ref, U_BF * ref.abs() + 1e-7 * ref.abs())
    assert (xr[..., 3:] == 0).all()
    dy = torch.empty(B * L * 8, dtype=torch.bfloat16, device=DEV)
    lp = torch.empty((B * L + 255) // 256, device=DEV)
    api.conv_mse_grad(dims, u.to(DEV), t.to(DEV), s.to(DEV), dy, lp)
    ud = u.double().requires_grad_(True)
    loss = oconv.increment_mse(ud, t.double(), s.double())
    (gu,) = torch.autograd.grad(loss, ud)
    g_y = (gu * s.double().view(-1, 1, 1)).transpose(1, 2)  # d loss / d net output, u_out = u + s y
    assert abs(lp.double().sum().item() - loss.item()) <= 1e-5 * loss.item()
    dyr = dy.view(B, L, 8).double().cpu()
    _check("dy", dyr[..., :3], g_y, U_BF * g_y.abs() + 1e-6 * g_y.abs())
    assert (dyr[..., 3:] == 0).all()


def test_adam_step():
    say("adam")
    rng = np.random.default_rng(4)
    n = 1000
    p = torch.tensor(rng.standard_normal(n), dtype=torch.float32)
    m = torch.zeros(n, dtype=torch.float32)
    v = torch.zeros(n, dtype=torch.float32)
    pd, md, vd = p.to(DEV), m.to(DEV), v.to(DEV)
    p64, m64, v64 = p.double(), m.double(), v.double()
    for k in range(1, 6):
        g = torch.tensor(rng.standard_normal(n), dtype=torch.float32)
        api.adam_step(pd, g.to(DEV), md, vd, 1e-3, 0.9, 0.999, 1e-8, k)
        p64, m64, v64 = oconv.adam_step(p64, g.double(), m64, v64, 1e-3, 0.9, 0.999, 1e-8, k)
    assert (pd.double().cpu() - p64).abs().max().item() < 1e-6
    assert (md.double().cpu() - m64).abs().max().item() < 1e-6


@pytest.mark.parametrize("dims", [(2, 12, 10, 9), (1, 300, 5, 4), (3, 64, 9, 7), (1, 100, 7, 6), (1, 256, 80, 40)])
def test_field_stats(dims):
    """Sums of the divergence and energy checks against the oracle, over row
    shapes that give one row per workgroup (nx >= 256), several rows per
    workgroup with idle lanes (nx = 100), and a grid capped at 2048
    workgroups; a repeated call gives the same bits."""
    say(f"field stats {dims}")
    rng = np.random.default_rng(5)
    B, nx, ny, nz = dims
    L = nx * ny * nz
    u = torch.tensor(rng.standard_normal((B, 3, L)), dtype=torch.float32)
    solid = torch.tensor(rng.random((B, L)) < 0.2, dtype=torch.uint8)
    out = torch.full((B, 3), float("nan"), device=DEV)
    ud, sd = u.to(DEV), solid.to(DEV)
    api.field_stats(dims, ud, sd, out)
    again = torch.empty_like(out)
    api.field_stats(dims, ud, sd, again, api.field_stats_workspace(dims))
    assert torch.equal(out, again)
    for b in range(B):
        uf = u[b].double().view(3, nz, ny, nx)
        fl = (solid[b] == 0).view(nz, ny, nx)
        rms = oconv.divergence_rms(uf, fl).item()
        ke = oconv.kinetic_energy(uf, fl).item()
        n_int = int(fl[1:-1, 1:-1, 1:-1].sum())
        o = out[b].double().cpu()
        assert int(o[1].item()) == n_int
        assert abs(math.sqrt(o[0].item() / o[1].item()) - rms) <= 1e-5 * rms
        assert abs(o[2].item() - ke) <= 1e-5 * ke


def test_bad_arguments_raise():
    with pytest.raises(api.DiffWindError):
        api.conv_pack_weights(torch.zeros(16 * 5 * 27, device=DEV), 5, 16, 0,
                              torch.empty(10, dtype=torch.bfloat16, device=DEV))
    with pytest.raises(api.DiffWindError):
        api.conv3d_bf16((1, 16, 4, 4), 32, 3, api.CONV_HIDDEN, torch.empty(16 * 16 * 32, dtype=torch.bfloat16,
                        device=DEV), torch.empty(27 * 16 * 32, dtype=torch.bfloat16, device=DEV),
                        bias=torch.zeros(3, device=DEV), y=torch.empty(16 * 16 * 8, dtype=torch.bfloat16,
                                                                        device=DEV))


# ----------------------------------------------------------- full-size sampled

def _gather_patch(xh, b, z, y, x):
    """(n, 27, C) neighbourhoods (zero outside) of voxels; xh (B, nz, ny, nx, C) float64."""
    B, nz, ny, nx, C = xh.shape
    out = torch.zeros(len(b), 27, C, dtype=torch.float64)
    for tap in range(27):
        dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
        zz, yy, xx = z + dz, y + dy, x + dx
        ok = (zz >= 0) & (zz < nz) & (yy >= 0) & (yy < ny) & (xx >= 0) & (xx < nx)
        idx = ok.nonzero().flatten()
        out[idx, tap] = xh[b[idx], zz[idx], yy[idx], xx[idx]].double()
    return out


def test_full_size_layers_sampled():
    """B = 16 fields of 64^3 (the batched inference workload): sampled outputs
    of a hidden layer forward and sampled weight-gradient entries."""
    say("full-size sampled 16 x 64^3")
    rng = np.random.default_rng(6)
    dims = (16, 64, 64, 64)
    B, nx, ny, nz = dims
    L = nx * ny * nz
    g = torch.Generator(device=DEV).manual_seed(6)
    xd = torch.randn(B * L * 32, device=DEV, generator=g).to(torch.bfloat16)
    w, w64 = _rand_w(rng, 32, 32)
    bias = torch.tensor(0.1 * rng.standard_normal(32), dtype=torch.float32)
    y = torch.empty_like(xd)
    zp = torch.empty_like(xd)
    api.conv3d_bf16(dims, 32, 32, api.CONV_HIDDEN, xd, _pack(w, 32, 32, 0), bias=bias.to(DEV), y=y, zpre=zp)
    xh = xd.view(B, nz, ny, nx, 32).cpu().float()  # BF16 values are exact in FP32
    n = 2048
    bb = torch.tensor(rng.integers(0, B, n))
    zz = torch.tensor(np.r_[rng.integers(0, nz, n - 64), np.zeros(32, int), np.full(32, nz - 1)])
    yy = torch.tensor(rng.integers(0, ny, n))
    xx = torch.tensor(np.r_[rng.integers(0, nx, n - 32), np.full(32, nx - 1)])
    P = _gather_patch(xh, bb, zz, yy, xx)                      # (n, 27, ci)
    W = w64.reshape(32, 32, 27)                                 # (co, ci, tap)
    ref = torch.einsum("ntc,oct->no", P, W) + bias.double()
    a = torch.einsum("ntc,oct->no", P.abs(), W.abs()) + bias.double().abs()
    got = zp.view(B, nz, ny, nx, 32)[bb.to(DEV), zz.to(DEV), yy.to(DEV), xx.to(DEV)].double().cpu()
    _check("zpre sampled", got, ref, U_BF * ref.abs() + 2 * ACC * a)
    # weight gradient: sampled (co, ci, tap) entries summed over all 4M voxels
    dzd = (1e-2 * torch.randn(B * L * 32, device=DEV, generator=g)).to(torch.bfloat16)
    dw = torch.empty(32, 32, 27, device=DEV)
    scratch = torch.empty(api.conv_wgrad_scratch_floats(), device=DEV)
    api.conv3d_bf16_wgrad(dims, 32, 32, xd, dzd, dw, None, scratch)
    dzh = dzd.view(B, nz, ny, nx, 32).cpu().float()
    xp = tF.pad(xh.permute(0, 4, 1, 2, 3), (1, 1, 1, 1, 1, 1))  # (B, ci, nz+2, ny+2, nx+2)
    for _ in range(12):
        co, ci, tap = (int(v) for v in (rng.integers(0, 32), rng.integers(0, 32), rng.integers(0, 27)))
        dz_, dy_, dx_ = tap // 9, (tap // 3) % 3, tap % 3
        xs = xp[:, ci, dz_:dz_ + nz, dy_:dy_ + ny, dx_:dx_ + nx].double()
        d = dzh[..., co].double()
        r = (d * xs).sum().item()
        ab = (d.abs() * xs.abs()).sum().item()
        e = abs(dw[co, ci, tap].item() - r)
        say(f"  dW[{co},{ci},{tap}] err {e:.3e} (sum|terms| {ab:.3e})")
        assert e <= ACC * ab


def _walk_samples(rng, dims, n=1536):
    """Sampled voxels of dims, with extra samples on the z planes where one
    8-plane tile ends and the next begins, on the last x and z planes, and on
    the y tile seams."""
    B, nx, ny, nz = dims
    zs = [z for z in range(7, nz, 8)] + [z for z in range(8, nz, 8)] + [nz - 1]
    k = 16 * len(zs)
    bb = torch.tensor(rng.integers(0, B, n + k))
    zz = torch.tensor(np.r_[rng.integers(0, nz, n), np.repeat(zs, 16)])
    yy = torch.tensor(np.r_[rng.integers(0, ny, n), rng.choice([3, 4, ny - 1], k)])
    xx = torch.tensor(np.r_[rng.integers(0, nx, n - 64), np.full(64, nx - 1), rng.integers(0, nx, k)])
    return bb, zz, yy, xx


def test_column_walk_layers_sampled():
    """Fields on which every workgroup walks a column of five z tiles, so the
    patch planes the tiles share go round the whole plane ring (ragged x and
    z edges): sampled outputs of the hidden, output and data-gradient layers
    against float64 sums over the gathered neighbourhoods."""
    dims = (16, 20, 64, 36)
    B, nx, ny, nz = dims
    L = nx * ny * nz
    say(f"column walk sampled {dims}")
    rng = np.random.default_rng(8)
    bb, zz, yy, xx = _walk_samples(rng, dims)
    idx = (bb.to(DEV), zz.to(DEV), yy.to(DEV), xx.to(DEV))
    # hidden layer 32 -> 32
    x = _rand_act(rng, dims, 32)
    w, w64 = _rand_w(rng, 32, 32)
    bias = torch.tensor(0.1 * rng.standard_normal(32), dtype=torch.float32)
    y = torch.empty(B * L * 32, dtype=torch.bfloat16, device=DEV)
    zp = torch.empty_like(y)
    xd = _to_dev_act(x, 32)
    api.conv3d_bf16(dims, 32, 32, api.CONV_HIDDEN, xd, _pack(w, 32, 32, 0), bias=bias.to(DEV), y=y, zpre=zp)
    xh = xd.view(B, nz, ny, nx, 32).cpu().double()
    P = _gather_patch(xh, bb, zz, yy, xx)                                   # (n, 27, ci)
    W = w64.reshape(32, 32, 27)
    ref = torch.einsum("ntc,oct->no", P, W) + bias.double()
    a = torch.einsum("ntc,oct->no", P.abs(), W.abs()) + bias.double().abs()
    _check("zpre", zp.view(B, nz, ny, nx, 32)[idx].double().cpu(), ref, U_BF * ref.abs() + 2 * ACC * a)
    s_ref = oconv.silu(ref)
    _check("silu", y.view(B, nz, ny, nx, 32)[idx].double().cpu(), s_ref, U_BF * s_ref.abs() + 3 * ACC * a + 1e-6)
    # output layer 32 -> 3 on the same input
    w3, w364 = _rand_w(rng, 32, 3)
    b3 = torch.tensor(0.1 * rng.standard_normal(3), dtype=torch.float32)
    u = torch.tensor(0.05 * rng.standard_normal((B, 3, L)), dtype=torch.float32)
    sc = torch.tensor(rng.uniform(0.02, 0.1, B), dtype=torch.float32)
    uo = torch.empty(B, 3, L, device=DEV)
    api.conv3d_bf16(dims, 32, 3, api.CONV_OUTPUT, xd, _pack(w3, 32, 3, 0), bias=b3.to(DEV), u=u.to(DEV),
                    scale=sc.to(DEV), u_out=uo)
    z3 = torch.einsum("ntc,oct->no", P, w364.reshape(3, 32, 27)) + b3.double()
    a3 = torch.einsum("ntc,oct->no", P.abs(), w364.reshape(3, 32, 27).abs()) + b3.double().abs()
    vox = xx + nx * (yy + ny * zz)
    sv = sc.double()[bb][:, None]
    ref3 = u.double()[bb, :, vox] + sv * z3
    got3 = uo.view(B, 3, L).cpu().double()[bb, :, vox]
    _check("u_out", got3, ref3, 2 * ACC * sv * a3 + 1e-6 * ref3.abs())
    # data gradient of a 32 -> 32 layer: conv^T of g, times silu'(zgate)
    gr = _rand_act(rng, dims, 32, 1e-3)
    zg = _rand_act(rng, dims, 32, 2.0)
    gd, zgd = _to_dev_act(gr, 32), _to_dev_act(zg, 32)
    yd = torch.empty_like(y)
    api.conv3d_bf16(dims, 32, 32, api.CONV_DGRAD, gd, _pack(w, 32, 32, 1), y=yd, zgate=zgd)
    Pg = _gather_patch(gd.view(B, nz, ny, nx, 32).cpu().double(), bb, zz, yy, xx)   # (n, 27, co)
    Wf = W.flip(2)                                   # conv^T: the tap at -d is tap 26 - t
    dx = torch.einsum("ntc,cot->no", Pg, Wf)
    da = torch.einsum("ntc,cot->no", Pg.abs(), Wf.abs())
    zgs = zgd.view(B, nz, ny, nx, 32)[idx].double().cpu()
    sig = torch.sigmoid(zgs)
    gate = sig * (1 + zgs * (1 - sig))
    refd = dx * gate
    _check("dgrad", yd.view(B, nz, ny, nx, 32)[idx].double().cpu(), refd, U_BF * refd.abs() + 2 * ACC * da * gate.abs())


# --------------------------------------------------------------- whole network

def _oracle_net(net):
    Ws = [_bf(w.cpu()).view(co, ci, 3, 3, 3) for (ci, co), w in zip(sg.LAYERS, net.w)]
    bs = [b.double().cpu() for b in net.b]
    return Ws, bs


def test_network_forward_and_gradients_vs_oracle():
    """Whole net: forward and all weight / bias gradients through the library's
    kernels against float64 autograd of the oracle net with the same BF16
    weights.  The library rounds each activation and gradient to BF16 between
    layers (the oracle does not), so the comparison is norm-wise at 3e-2."""
    say("network fwd/bwd vs oracle")
    rng = np.random.default_rng(8)
    dims = (2, 16, 8, 12)
    B, nx, ny, nz = dims
    L = nx * ny * nz
    net = sg.Surrogate(seed=3)
    for w in net.w:  # a non-trivial last layer
        w.copy_(torch.tensor(rng.standard_normal(tuple(w.shape)) / math.sqrt(w.shape[1] * 27), dtype=torch.float32))
    net.repack()
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([np.sin(0.3 * xx + 0.2 * yy), np.cos(0.25 * zz), np.sin(0.4 * yy - 0.1 * zz)])
    u = torch.tensor(0.05 * (base[None] + 0.3 * rng.standard_normal((B, 3, nz, ny, nx))), dtype=torch.float32)
    t = u + torch.tensor(0.0005 * rng.standard_normal(u.shape), dtype=torch.float32)
    s = torch.tensor([0.05, 0.08], dtype=torch.float32)
    ud, td, sd = u.reshape(B, 3, L).to(DEV), t.reshape(B, 3, L).to(DEV), s.to(DEV)
    uo = torch.empty(B, 3, L, device=DEV)
    so = net.forward(ud, sd, uo, dims, keep_preact=True)
    lp = net.backward(uo, td, so, dims)
    Ws, bs = _oracle_net(net)
    Ws = [w.clone().requires_grad_(True) for w in Ws]
    bs = [b.clone().requires_grad_(True) for b in bs]
    out = oconv.surrogate_forward(u.double(), Ws, bs, s.double(), gain=net.gain)
    loss = oconv.increment_mse(out, t.double(), s.double() * net.gain)
    grads = torch.autograd.grad(loss, Ws + bs)
    dinc = (uo.double().cpu() - ud.double().cpu()).norm() / (out.reshape(B, 3, L) - u.double().reshape(B, 3, L)).norm()
    e_out = ((uo.double().cpu() - out.reshape(B, 3, L)).norm()
             / (out.reshape(B, 3, L) - u.double().reshape(B, 3, L)).norm()).item()
    say(f"  increment rel err {e_out:.3e} (norm ratio {dinc.item():.4f}); loss {lp.sum().item():.6e} "
        f"oracle {loss.item():.6e}")
    assert e_out < 3e-2
    assert abs(lp.sum().item() - loss.item()) <= 3e-2 * loss.item()
    for l in range(4):
        ew = ((net.gw[l].double().cpu() - grads[l].reshape(net.gw[l].shape)).norm() / grads[l].norm()).item()
        eb = ((net.gb[l].double().cpu() - grads[4 + l]).norm() / grads[4 + l].norm()).item()
        say(f"  layer {l}: dW rel err {ew:.3e}  db rel err {eb:.3e}")
        assert ew < 3e-2 and eb < 3e-2


def test_training_reduces_loss_and_fallback():
    """A short training run on LBM pairs lowers the loss; corrupted predictions
    (NaN, energy x 1.5) are rejected and replaced by the plain-LBM block."""
    say("training on LBM pairs 48x32x32")
    dims3 = (48, 32, 32)
    U0, U1, S, M = sg.lbm_pairs(6, 4, dims=dims3, warmup=100, t_max=300, seed=1)
    net = sg.Surrogate(seed=1)
    nx, ny, nz = dims3
    ev = (U0.shape[0], nx, ny, nz)
    out = torch.empty_like(U0)
    l0 = net.loss(U0, U1, S, ev, out)
    sg.train(net, U0, U1, S, (8, nx, ny, nz), steps=150, batch=8, lr=1e-3)
    l1 = net.loss(U0, U1, S, ev, out)
    say(f"  loss on all pairs {l0:.4e} -> {l1:.4e}")
    assert l1 < 0.9 * l0
    # fallback
    lat = api.make_lattice(nx, ny, nz)
    spd = float(S[0])
    from paper_2603_09668_amd import scenes
    _, solid_np, bc = scenes.wind_tunnel_obstacles(1 * 100_003 + 0, dims3)
    solid = torch.tensor(solid_np.reshape(-1), dtype=torch.uint8, device=DEV)
    wind = sg.SurrogateWind(net, lat, dict(tau=0.6, u_in=(spd, 0.0, 0.0), bc=bc), solid, k=8, batch=1)
    u = U0[:1].contiguous()
    uo = torch.empty_like(u)
    ok = wind.advance(u, S[:1], uo, t0=0)
    say(f"  clean prediction accepted: {bool(ok[0])}")
    assert bool(ok[0])
    ref = torch.empty(3, nx * ny * nz, device=DEV)
    wind.lbm_block(u[0], 0, ref)
    for name, fn in (("nan", lambda t: t.view(-1)[123].fill_(float("nan"))), ("energy", lambda t: t.mul_(1.5 ** 0.5))):
        ok = wind.advance(u, S[:1], uo, t0=0, override=fn)
        say(f"  {name}: accepted {bool(ok[0])}")
        assert not bool(ok[0])
        assert torch.equal(uo[0], ref)
    assert wind.fallbacks == 2
    # the device-side path captured in a HIP graph: replays give the eager
    # results, for an accepted and for a rejected prediction
    for name, fn in (("clean", None), ("energy", lambda t: t.mul_(1.5 ** 0.5))):
        eager = torch.empty_like(u)
        wind.advance_device(u, S[:1], eager, t0=0, override=fn)
        torch.cuda.synchronize()
        gph = torch.cuda.CUDAGraph()
        gout = torch.empty_like(u)
        with torch.cuda.graph(gph):
            wind.advance_device(u, S[:1], gout, t0=0, override=fn)
        for _ in range(3):
            gout.fill_(-1.0)
            gph.replay()
            torch.cuda.synchronize()
            assert torch.equal(gout, eager), name
        if name == "energy":
            assert torch.equal(gout[0], ref)


def _graph_time_ms(fn, reps):
    """Average time of fn() captured in one HIP graph (events on the stream)."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        g.replay()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps


def _time_ms(fn, reps):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    fn()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        fn()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps


def test_surrogate_gain_over_lbm():
    """What the trained net gains over plain LBM on 64^3 wind tunnels with
    obstacles: <= 2 % relative wind error on held-out fields, measured against
    the library's LBM and, on one field, against the float64 oracle LBM, and
    below persistence (u_{t+8} = u_t); and the whole surrogate step (net,
    divergence and energy checks, device-side decision, the switched-off LBM
    fallback branch, output selection; one HIP graph) is faster than the 8 LBM
    steps it replaces on one 256 x 128 x 128 tunnel (the largest workload's
    node count; one HIP graph)."""
    from oracle import lbm as olbm
    from paper_2603_09668_amd import scenes

    say("surrogate gain 64^3")
    dims3 = (64, 64, 64)
    nx, ny, nz = dims3
    L = nx * ny * nz
    U0, U1, S, M = sg.lbm_pairs(24, 8, dims=dims3, seed=0)
    H0, H1, HS, HM = sg.lbm_pairs(4, 4, dims=dims3, seed=99)
    net = sg.Surrogate(seed=0)
    sg.train(net, U0, U1, S, (16, *dims3), steps=300, batch=16, lr=1e-3, seed=0)
    sg.train(net, U0, U1, S, (16, *dims3), steps=200, batch=16, lr=2e-4, seed=1)
    out = torch.empty_like(H0)
    net.forward(H0, HS, out, (H0.shape[0], *dims3))
    e_s = sg.rel_error(out, H1, HM)
    e_id = sg.rel_error(H0, H1, HM)
    say(f"  held-out error: surrogate mean {e_s.mean():.4e} max {e_s.max():.4e}; "
        f"persistence mean {e_id.mean():.4e} max {e_id.max():.4e}")
    assert e_s.max().item() <= 0.02
    assert e_s.mean().item() <= e_id.mean().item()
    assert bool(sg.check_fields(H0, out, (H0.shape[0], *dims3), HM).all())

    # one held-out field against the float64 oracle LBM
    spd, solid_np, bc = scenes.wind_tunnel_obstacles(7777, dims3)
    lat = api.make_lattice(nx, ny, nz)
    solid = torch.tensor(solid_np.reshape(-1), dtype=torch.uint8, device=DEV)
    kw = dict(tau=0.6, u_in=(spd, 0.0, 0.0), bc=bc)
    fa = torch.empty(19, L, device=DEV)
    fb = torch.empty_like(fa)
    u = torch.empty(3, L, device=DEV)
    api.lbm_equilibrium(lat, api.make_lbm_params(**kw), fa)
    t0 = 240
    for t in range(1, t0 + 1):
        api.lbm_step(lat, api.make_lbm_params(**kw, t=t), fa, fb, solid, None, u)
        fa, fb = fb, fa
    f_t, u_t = fa.clone(), u.clone()
    for t in range(t0 + 1, t0 + 9):
        api.lbm_step(lat, api.make_lbm_params(**kw, t=t), fa, fb, solid, None, u)
        fa, fb = fb, fa
    u_gpu = u.clone()
    olat = olbm.Lattice(nx, ny, nz)
    op = olbm.LBMParams(tau=0.6, u_in=(spd, 0.0, 0.0), bc=bc)
    f = f_t.double().cpu().view(19, nz, ny, nx) + olbm.W.view(19, 1, 1, 1)
    sol = torch.tensor(solid_np)
    for t in range(t0 + 1, t0 + 9):
        f, _, u_o = olbm.lbm_step(olat, op, f, sol, t)
    u_ref = u_o.reshape(1, 3, L)
    fluid = torch.tensor(~solid_np.reshape(1, -1))
    e_lbm = sg.rel_error(u_gpu.double().cpu().view(1, 3, L), u_ref, ~fluid)
    u_s = torch.empty(1, 3, L, device=DEV)
    net.forward(u_t.view(1, 3, L), torch.tensor([spd], device=DEV), u_s, (1, *dims3))
    e_o = sg.rel_error(u_s.double().cpu(), u_ref, ~fluid)
    say(f"  vs float64 oracle LBM: library LBM {e_lbm.item():.2e}, surrogate {e_o.item():.4e}")
    assert e_lbm.item() < 1e-5 and e_o.item() <= 0.02

    # speed: the whole surrogate step against 8 LBM steps on one 256 x 128 x 128 tunnel
    big = (256, 128, 128)
    Lb = big[0] * big[1] * big[2]
    spd_b, solid_b_np, bc_b = scenes.wind_tunnel_obstacles(5, big)
    lat_b = api.make_lattice(*big)
    solid_b = torch.tensor(solid_b_np.reshape(-1), dtype=torch.uint8, device=DEV)
    kw_b = dict(tau=0.6, u_in=(spd_b, 0.0, 0.0), bc=bc_b)
    ga = torch.empty(19, Lb, device=DEV)
    gb = torch.empty_like(ga)
    ub = torch.empty(1, 3, Lb, device=DEV)
    api.lbm_equilibrium(lat_b, api.make_lbm_params(**kw_b), ga)
    # a developed flow: the 256-long tunnel takes about four times the 64^3
    # tunnels' warm-up of 200 steps
    for t in range(1, 801):
        api.lbm_step(lat_b, api.make_lbm_params(**kw_b, t=t), ga, gb, solid_b, None, ub[0])
        ga, gb = gb, ga
    prms = [api.make_lbm_params(**kw_b, t=800 + j + 1) for j in range(8)]
    u8 = torch.empty(3, Lb, device=DEV)

    def lbm8():
        a, b = ga, gb
        for j in range(8):
            api.lbm_step(lat_b, prms[j], a, b, solid_b, None, u8 if j == 7 else None)
            a, b = b, a

    sw = sg.SurrogateWind(net, lat_b, kw_b, solid_b, k=8, batch=1)
    sc_b = torch.tensor([spd_b], device=DEV)
    ob = torch.empty_like(ub)
    t_lbm = _graph_time_ms(lbm8, 5)
    t_sur = _graph_time_ms(lambda: sw.advance_device(ub, sc_b, ob, t0=800), 5)
    acc = int(sw.accept.item())
    e_b = sg.rel_error(ob, u8.view(1, 3, Lb), solid_b.view(1, -1)).item()
    say(f"  256x128x128: surrogate step {t_sur:.3f} ms (accepted {acc}, error vs LBM {e_b:.2e}), "
        f"8 LBM steps {t_lbm:.3f} ms, speedup {t_lbm / t_sur:.2f}x")
    assert acc == 1 and e_b <= 0.02
    assert t_sur < t_lbm


def test_coupled_surrogate_and_frozen_wind():
    """The coupled driver's wind models on the 20k-particle sheet: with the
    untrained net (the identity u_{t+8} = u_t, accepted by the checks) the
    surrogate run keeps the warmed wind up to the solid-node masking, the
    frozen run keeps it exactly, and both differ from the LBM-driven run."""
    from paper_2603_09668_amd import scenes
    from paper_2603_09668_amd.sim import CoupledSim
    sc = scenes.sheet_scene(seed=0, n=20_000)
    say("coupled wind models on the sheet scene")
    net = sg.Surrogate(seed=3)
    out = {}
    for model in ("lbm", "surrogate", "frozen"):
        sim = CoupledSim(sc, wind=model, surrogate=net if model == "surrogate" else None, reorder=False)
        sim.warm_wind(50)
        u0 = sim.u.clone()
        for _ in range(24):
            sim.step()
        torch.cuda.synchronize()
        assert sim.status() == 0
        out[model] = (u0, sim.u.clone(), sim.p.x.clone(), sim)
    u0, uf, _, _ = out["frozen"]
    assert torch.equal(u0, uf)
    u0s, us, _, sims = out["surrogate"]
    fluid = sims.solid == 0
    assert torch.equal(us[:, fluid], u0s[:, fluid])
    assert int(sims.sw.accept.item()) == 1
    assert not torch.equal(out["lbm"][1], out["lbm"][0])
    assert not torch.equal(out["lbm"][2], out["frozen"][2])
