"""Learned wind surrogate: a BF16-MFMA 3-D convolution net that advances the LBM
velocity field k lattice steps per call, trained on rollouts of the library's
own lbm_step, with a divergence / kinetic-energy check and plain-LBM fallback.

The paper's wind is the lattice Boltzmann solution of Eq. lbe; this net is a
faster stand-in, measured against the LBM, which replaces it whenever a check fails:

    u_{t+k} = u_t + g s * net(u_t / s),  s = the field's inflow speed,
    net = conv(32->3) . silu . conv(32->32) . silu . conv(32->32) . silu . conv(3->32).

g a fixed output gain (0.01: increments over k = 8 steps are about 1 % of the
inflow speed), so that the net's outputs, and Adam's steps on its weights,
are of order one.  Every convolution, gradient, loss and optimiser step runs
in the library's kernels (conv3d_bf16, conv3d_bf16_wgrad, conv_mse_grad,
adam_step); torch holds the buffers.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api, scenes

LAYERS = ((3, 32), (32, 32), (32, 32), (32, 3))
D = "cuda"


class Surrogate:
    def __init__(self, seed: int = 0, gain: float = 0.01, device: str = D):
        self.device = device
        self.gain = float(gain)
        gen = torch.Generator().manual_seed(seed)
        self.w, self.b = [], []
        for l, (ci, co) in enumerate(LAYERS):
            std = math.sqrt(2.0 / (ci * 27))
            w = torch.randn(co, ci, 27, generator=gen) * std
            if l == len(LAYERS) - 1:
                w.zero_()  # the untrained net is the identity map u_{t+k} = u_t
            self.w.append(w.float().to(device).contiguous())
            self.b.append(torch.zeros(co, dtype=torch.float32, device=device))
        self.gw = [torch.zeros_like(w) for w in self.w]
        self.gb = [torch.zeros_like(b) for b in self.b]
        self.mw = [torch.zeros_like(w) for w in self.w]
        self.vw = [torch.zeros_like(w) for w in self.w]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step_count = 0
        self.scratch = torch.empty(api.conv_wgrad_scratch_floats(), dtype=torch.float32, device=device)
        self._buf_dims = None
        self.repack()

    # ------------------------------------------------------------ weights
    def repack(self):
        bf = dict(dtype=torch.bfloat16, device=self.device)
        self.wk, self.wkt = [], []
        for (ci, co), w in zip(LAYERS, self.w):
            wk = torch.empty(api.conv_packed_weight_elems(ci, co), **bf)
            api.conv_pack_weights(w, ci, co, 0, wk)
            self.wk.append(wk)
            if ci == 32:  # data-gradient packing (layer 1 needs none)
                wkt = torch.empty(api.conv_packed_weight_elems(co, ci), **bf)
                api.conv_pack_weights(w, ci, co, 1, wkt)
                self.wkt.append(wkt)
            else:
                self.wkt.append(None)

    def state_dict(self):
        return {"w": [w.cpu() for w in self.w], "b": [b.cpu() for b in self.b]}

    def load_state_dict(self, sd):
        for l in range(len(LAYERS)):
            self.w[l].copy_(sd["w"][l].to(self.device))
            self.b[l].copy_(sd["b"][l].to(self.device))
        self.repack()

    # ------------------------------------------------------------ buffers
    def _buffers(self, dims):
        if self._buf_dims == dims:
            return
        B, nx, ny, nz = dims
        L = nx * ny * nz
        bf = dict(dtype=torch.bfloat16, device=self.device)
        self.x0 = torch.empty(B * L * 8, **bf)
        self.a = [torch.empty(B * L * 32, **bf) for _ in range(3)]
        self.z = [torch.empty(B * L * 32, **bf) for _ in range(3)]
        self.dy = torch.empty(B * L * 8, **bf)
        self.da = [torch.empty(B * L * 32, **bf) for _ in range(2)]
        self.loss_part = torch.empty((B * L + 255) // 256, dtype=torch.float32, device=self.device)
        self._buf_dims = dims

    # ------------------------------------------------------------ forward
    def out_scale(self, scale):
        """Per-field scale of the output increment, g s (B floats)."""
        return scale * self.gain

    def forward(self, u, scale, u_out, dims, keep_preact: bool = False, out_scale=None):
        """u, u_out: (B, 3, L) float32; scale: (B,) float32 inflow speeds."""
        self._buffers(dims)
        so = self.out_scale(scale) if out_scale is None else out_scale
        api.conv_prep_input(dims, u, scale, self.x0)
        x = self.x0
        for l in range(3):
            ci, co = LAYERS[l]
            api.conv3d_bf16(dims, ci, co, api.CONV_HIDDEN, x, self.wk[l], bias=self.b[l], y=self.a[l],
                            zpre=self.z[l] if keep_preact else None)
            x = self.a[l]
        api.conv3d_bf16(dims, 32, 3, api.CONV_OUTPUT, x, self.wk[3], bias=self.b[3], u=u, scale=so, u_out=u_out)
        return so

    def backward(self, u_out, u_tgt, out_scale, dims):
        """Gradients of the loss mean(((u_out - u_tgt) / (g s))^2) into self.gw /
        self.gb; returns the per-block loss partials (their sum is the loss)."""
        api.conv_mse_grad(dims, u_out, u_tgt, out_scale, self.dy, self.loss_part)
        g = self.dy  # gradient w.r.t. the output layer's pre-activation
        inputs = [self.x0, self.a[0], self.a[1], self.a[2]]
        for l in (3, 2, 1, 0):
            ci, co = LAYERS[l]
            api.conv3d_bf16_wgrad(dims, ci, co, inputs[l], g, self.gw[l], self.gb[l], self.scratch)
            if l > 0:
                dst = self.da[l % 2]
                api.conv3d_bf16(dims, ci, co, api.CONV_DGRAD, g, self.wkt[l], y=dst, zgate=self.z[l - 1])
                g = dst
        return self.loss_part

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for l in range(len(LAYERS)):
            api.adam_step(self.w[l], self.gw[l], self.mw[l], self.vw[l], lr, b1, b2, eps, self.step_count)
            api.adam_step(self.b[l], self.gb[l], self.mb[l], self.vb[l], lr, b1, b2, eps, self.step_count)
        self.repack()

    def train_step(self, u, u_tgt, scale, dims, u_out, lr=1e-3):
        so = self.forward(u, scale, u_out, dims, keep_preact=True)
        lp = self.backward(u_out, u_tgt, so, dims)
        self.adam(lr)
        return lp

    def loss(self, u, u_tgt, scale, dims, u_out):
        """Loss of the current weights on one batch (no update)."""
        so = self.forward(u, scale, u_out, dims)
        self._buffers(dims)
        api.conv_mse_grad(dims, u_out, u_tgt, so, self.dy, self.loss_part)
        return float(self.loss_part.sum())


# ------------------------------------------------------------------ data

def lbm_pairs(n_rollouts: int, pairs_per_rollout: int, dims=(64, 64, 64), k: int = 8, warmup: int = 200,
              t_max: int = 1000, seed: int = 0, tau: float = 0.6, device: str = D):
    """Training pairs (u_t, u_{t+k}, inflow speed, solid mask) from seeded wind
    tunnels with random obstacles, produced by the library's lbm_step.  Pairs
    are drawn at random t in [warmup, t_max]."""
    nx, ny, nz = dims
    L = nx * ny * nz
    lat = api.make_lattice(nx, ny, nz)
    U0, U1, S, M = [], [], [], []
    rng = np.random.default_rng(seed)
    for r in range(n_rollouts):
        spd, solid_np, bc = scenes.wind_tunnel_obstacles(seed * 100_003 + r, dims)
        solid = torch.tensor(solid_np.reshape(-1), dtype=torch.uint8, device=device)
        prm_kw = dict(tau=tau, u_in=(spd, 0.0, 0.0), bc=bc)
        fa = torch.empty(19, L, device=device)
        fb = torch.empty_like(fa)
        api.lbm_equilibrium(lat, api.make_lbm_params(**prm_kw), fa)
        u = torch.empty(3, L, device=device)
        starts = sorted(int(t) for t in rng.integers(warmup, t_max - k, pairs_per_rollout))
        want = {}
        for t0 in starts:
            want.setdefault(t0, []).append("a")
            want.setdefault(t0 + k, []).append("b")
        snaps = {}
        for t in range(1, max(want) + 1):
            api.lbm_step(lat, api.make_lbm_params(**prm_kw, t=t), fa, fb, solid, None, u)
            fa, fb = fb, fa
            if t in want:
                snaps[t] = u.clone()
        for t0 in starts:
            U0.append(snaps[t0])
            U1.append(snaps[t0 + k])
            S.append(spd)
            M.append(solid)
    return torch.stack(U0), torch.stack(U1), torch.tensor(S, dtype=torch.float32, device=device), torch.stack(M)


def rel_error(u_pred, u_ref, solid=None):
    """Relative wind-field error |u - u_ref|_2 / |u_ref|_2 over fluid nodes, per field."""
    d = (u_pred - u_ref) ** 2
    r = u_ref ** 2
    if solid is not None:
        fluid = (solid == 0).unsqueeze(1).to(d.dtype)
        d = d * fluid
        r = r * fluid
    return torch.sqrt(d.sum(dim=(1, 2)) / r.sum(dim=(1, 2)))


def check_fields(u_prev, u_new, dims, solid=None, div_factor=2.0, ke_band=(0.9, 1.1)):
    """Acceptance test of surrogate outputs (per field): finite values, RMS
    divergence at most div_factor times the input's, kinetic energy within
    ke_band of the input's.  Returns a bool tensor (B,)."""
    B = dims[0]
    st = torch.empty(2, B, 3, dtype=torch.float32, device=u_new.device)
    ws = api.field_stats_workspace(dims, u_new.device)
    api.field_stats(dims, u_prev, solid, st[0], ws)
    api.field_stats(dims, u_new, solid, st[1], ws)
    finite = torch.isfinite(u_new).flatten(1).all(dim=1)
    rms = torch.sqrt(st[:, :, 0] / st[:, :, 1].clamp(min=1.0))
    ke = st[:, :, 2]
    ok_div = rms[1] <= div_factor * rms[0] + 1e-12
    ratio = ke[1] / ke[0].clamp(min=1e-30)
    ok_ke = (ratio >= ke_band[0]) & (ratio <= ke_band[1])
    return finite & ok_div & ok_ke


def train(net: Surrogate, U0, U1, S, dims, steps: int, batch: int = 16, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0):
    """Adam on random minibatches of the pairs (U0 -> U1); returns the loss history."""
    B = batch
    _, nx, ny, nz = dims
    bd = (B, nx, ny, nz)
    u_out = torch.empty(B, 3, nx * ny * nz, device=net.device)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for it in range(steps):
        idx = torch.randint(0, U0.shape[0], (B,), generator=gen).to(U0.device)
        u, tgt, sc = U0.index_select(0, idx), U1.index_select(0, idx), S.index_select(0, idx)
        lp = net.train_step(u, tgt, sc, bd, u_out, lr=lr)
        if log_every and (it % log_every == 0 or it == steps - 1):
            hist.append((it, float(lp.sum())))
    return hist


class SurrogateWind:
    """Advances the wind of one lattice k LBM steps per call with the surrogate,
    checked by the divergence and kinetic-energy tests; a rejected field is
    re-initialised at equilibrium (rho = 1, the current u) and advanced k plain
    LBM steps instead.  The decision is taken on the device: the checks write
    an acceptance flag that switches the LBM fallback branch off (the `skip`
    flag of its launches) and selects the output, so a call needs no host
    synchronisation and can be captured in a HIP graph."""

    def __init__(self, net: Surrogate, lat, lbm_kw: dict, solid, k: int = 8, batch: int = 1,
                 div_factor: float = 2.0, ke_band=(0.9, 1.1)):
        self.net, self.lat, self.kw, self.solid, self.k = net, lat, dict(lbm_kw), solid, k
        self.div_factor, self.ke_band = float(div_factor), tuple(ke_band)
        nx, ny, nz = lat.nx, lat.ny, lat.nz
        self.dims = (batch, nx, ny, nz)
        L = nx * ny * nz
        dev = net.device
        self.fa = torch.empty(19, L, device=dev)
        self.fb = torch.empty_like(self.fa)
        self.u_tmp = torch.empty(3, L, device=dev)
        self.u_pred = torch.empty(batch, 3, L, device=dev)
        self.u_lbm = torch.empty(batch, 3, L, device=dev)
        self.stats = torch.zeros(2, batch, 3, device=dev)
        self.stats_ws = api.field_stats_workspace(self.dims, dev)
        self.accept = torch.zeros(batch, dtype=torch.int32, device=dev)
        self.reject = torch.zeros(batch, dtype=torch.int32, device=dev)
        self.solid_b = None
        self.set_solid(solid)
        self.fallbacks = 0

    def set_solid(self, solid):
        """The solid mask (L,) of the lattice (read at every call, so a mask
        updated in place is seen)."""
        self.solid = solid
        B = self.dims[0]
        if solid is None:
            self.solid_b = None
        elif B == 1:
            self.solid_b = solid.reshape(1, -1)
        else:
            self.solid_b = solid.reshape(1, -1).expand(B, -1).contiguous()

    def lbm_block(self, u, t0: int, u_out, skip=None):
        """k LBM steps from the equilibrium at (rho = 1, u); writes u_out (3, L).
        skip: optional device int32 flag that switches the whole block off."""
        api.lbm_equilibrium(self.lat, api.make_lbm_params(**self.kw, skip=skip), self.fa, None, u)
        fa, fb = self.fa, self.fb
        for j in range(self.k):
            api.lbm_step(self.lat, api.make_lbm_params(**self.kw, t=t0 + j + 1, skip=skip), fa, fb, self.solid, None,
                         u_out if j == self.k - 1 else None)
            fa, fb = fb, fa

    def advance_device(self, u, scale, u_out, t0: int = 0, override=None):
        """u, u_out: (B, 3, L); scale (B,).  Prediction, checks, decision and
        fallback all on the device; returns the device int32 acceptance
        flags (B,).  `override(u_pred)` may alter the prediction before the
        checks (fault-injection hook).  u_out may be u itself."""
        dims = self.dims
        self.net.forward(u, scale, self.u_pred, dims)
        if override is not None:
            override(self.u_pred)
        api.field_stats(dims, u, self.solid_b, self.stats[0], self.stats_ws)
        api.field_stats(dims, self.u_pred, self.solid_b, self.stats[1], self.stats_ws)
        api.field_accept(self.stats[0], self.stats[1], self.accept, self.reject, self.div_factor, self.ke_band)
        for b in range(dims[0]):
            self.lbm_block(u[b], t0, self.u_lbm[b], skip=self.accept[b:b + 1])
        api.field_select(dims, self.accept, self.u_pred, self.u_lbm, self.solid_b, u_out)
        return self.accept

    def advance(self, u, scale, u_out, t0: int = 0, override=None):
        """advance_device, then the per-field bool tensor of accepted
        predictions (this reads the flags on the host)."""
        ok = self.advance_device(u, scale, u_out, t0, override).bool()
        self.fallbacks += int((~ok).sum().item())
        return ok
