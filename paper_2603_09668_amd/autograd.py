"""Differentiable MPM rollouts through the hand-written adjoints, with substep
checkpointing.

The reconstruction of Sec. 3.3 optimises the wind force field F_w (and can
differentiate the material parameters theta) by gradient descent through the
simulation S of Eq. simulation_mpm.  `Rollout` runs n substeps of S on the
device with a force-grid wind (one field per time slot, piecewise constant
over the substeps) and exposes them to torch as one autograd Function.

Memory: the forward keeps the particle state every `ckpt` substeps only.  The
backward walks the segments in reverse; for each it re-runs the segment from
its checkpoint, keeping every substep's particle state, sort workspace and
grid (m, mv, v: about 28 B per grid node and 20 B per particle per substep),
then for every substep (last first) applies the adjoints in reverse order:
G2P adjoint (sorted scatter into the grid adjoint), grid-update adjoint, wind
transpose into W_bar, P2G adjoint (per-particle gather, also giving E_bar).
Every step runs in the library's HIP kernels; torch provides device memory,
zero-fills (one per buffer group) and the final loss.

With `deterministic` every reduction of the forward and reverse substeps
runs in a fixed order (sort, P2G, the reverse G2P's grid scatter, the E and
force-grid adjoints), so a rollout's gradients are bit-identical run to run.

With `xref` the positions are xref + x: the rollout's x input and output are
displacements from that fixed reference (see the header), which keeps their
float32 resolution on the motion.

A particle whose stencil leaves the grid is skipped by the kernels and
flagged in the workspace status word (as are non-finite positions); the
status of every forward and recomputed substep is OR-ed on the device and
checked once per forward and once per backward, and a flagged rollout
raises instead of returning a truncated gradient.
"""
from __future__ import annotations

import torch

from . import api


class RolloutPlan:
    """Device buffers and constants for rollouts of one particle set on one grid."""

    def __init__(self, grid: dict, n: int, mass, vol0, region, nu, pin, dt: float, gravity, material: int,
                 bound: int, nw, box_lo, box_hi, K: int, n_sub: int, ckpt: int = 16, device="cuda",
                 xref=None, deterministic: bool = False):
        self.grid = api.make_grid(grid["nx"], grid["ny"], grid["nz"], grid["dx"], grid["origin"])
        self.N = grid["nx"] * grid["ny"] * grid["nz"]
        self.n = n
        self.mass, self.vol0, self.region, self.nu = mass, vol0, region, nu
        self.pin = pin
        self.xref = xref
        self.deterministic = bool(deterministic)
        self.prm = api.make_mpm_params(dt, gravity, bound, material, deterministic=self.deterministic)
        self.nw, self.box_lo, self.box_hi, self.K = tuple(nw), tuple(box_lo), tuple(box_hi), K
        self.n_sub, self.ckpt = n_sub, ckpt
        f = dict(dtype=torch.float32, device=device)
        self.device = device
        self.ws = api.alloc_workspace(self.grid, n, device, deterministic=self.deterministic)
        self.gm = torch.zeros(self.N, **f)
        self.gmv = torch.zeros(3, self.N, **f)
        self.gv = torch.zeros(3, self.N, **f)
        # grid adjoints in one buffer, cleared with one fill per substep
        self._gbar = torch.zeros(10, self.N, **f)
        self.gvb, self.gmb, self.gmvb, self.accb = (self._gbar[0:3], self._gbar[3], self._gbar[4:7],
                                                    self._gbar[7:10])
        self._seg = None  # per-substep workspaces and grids of a segment, made on first backward
        self._status = torch.zeros(1, dtype=torch.int32, device=device)  # OR of the substeps' status words

    def segment_buffers(self):
        """Sort workspaces and grids (m, mv, v) for the substeps of one segment."""
        if self._seg is None:
            f = dict(dtype=torch.float32, device=self.device)
            self._seg = [(api.alloc_workspace(self.grid, self.n, self.device, deterministic=self.deterministic),
                          torch.empty(self.N, **f),
                          torch.empty(3, self.N, **f), torch.empty(3, self.N, **f)) for _ in range(self.ckpt)]
        return self._seg

    def slot(self, s: int) -> int:
        return s * self.K // self.n_sub

    def particles(self, x, v, C, H, E):
        return api.ParticleArrays(x, v, C, H, self.mass, self.vol0, self.region, E, self.nu, self.xref)

    def check_status(self, what: str):
        """Raise if a substep since the last check met a particle outside the
        grid or a non-finite position (one host synchronisation)."""
        st = int(self._status.item())
        self._status.zero_()
        bad = st & (api.STATUS_OUT_OF_GRID | api.STATUS_NONFINITE)
        if bad:
            raise api.DiffWindError(f"rollout {what}: status {st:#x} (a particle left the grid or is not finite); "
                                    "the kernels skipped it, so the result would be truncated")

    def wind(self, W, s):
        return api.wind_force_grid(W[self.slot(s)], self.nw, self.box_lo, self.box_hi,
                                   deterministic=self.deterministic)

    # --------------------------------------------------------------- forward
    def substep(self, p: api.ParticleArrays, W, s: int, out=None, bufs=None, g2p: bool = True):
        """One substep; in place unless `out` = (x, v, C, H) buffers are given.
        `bufs` = (workspace, m, mv, v) keeps this substep's sort and grid."""
        ws, gm, gmv, gv = bufs if bufs is not None else (self.ws, self.gm, self.gmv, self.gv)
        api.mpm_sort(self.grid, self.prm, p.x, ws, xref=self.xref)
        api.mpm_p2g(self.grid, self.prm, p, gm, gmv, ws)
        self._status.bitwise_or_(ws[:4].view(torch.int32))
        api.mpm_grid_update(self.grid, self.prm, gm, gmv, self.wind(W, s), self.pin, gv, ws)
        if not g2p:
            return None
        if out is None:
            api.mpm_g2p(self.grid, self.prm, gv, p, p.x, p.v, p.C, p.F)
            return p
        api.mpm_g2p(self.grid, self.prm, gv, p, *out)
        return self.particles(*out, p.E)

    # -------------------------------------------------------------- backward
    def substep_adjoint(self, p: api.ParticleArrays, W, s: int, bar_out, bar_in, W_bar, E_bar, bufs=None):
        """Adjoint of substep s at input state p: adds into bar_in = (x, v, C, H)
        adjoints of the inputs, W_bar and E_bar, given bar_out of the outputs.
        `bufs` = the substep's kept (workspace, m, mv, v); without it the
        substep's grid is recomputed first."""
        g, prm = self.grid, self.prm
        wind = self.wind(W, s)
        if bufs is None:
            self.substep(p, W, s, g2p=False)
            bufs = (self.ws, self.gm, self.gmv, self.gv)
        ws, gm, gmv, gv = bufs
        self._gbar.zero_()
        xb, vb, Cb, Hb = bar_in
        api.mpm_g2p_adj(g, prm, gv, p, *bar_out, x_bar=xb, F_bar=Hb, grid_v_bar=self.gvb, ws=ws)
        api.mpm_grid_update_adj(g, prm, gm, gmv, wind, self.pin, self.gvb, self.gmb, self.gmvb, self.accb, ws)
        api.wind_to_grid_adj(g, wind, self.accb, W_bar[self.slot(s)])
        api.mpm_p2g_adj(g, prm, p, self.gmb, self.gmvb, xb, vb, Cb, Hb, E_bar, ws=ws)


class _RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan: RolloutPlan, W, E, x0, v0, C0, H0):
        W = W.detach().contiguous()
        E = E.detach().contiguous()
        state = [t.detach().clone() for t in (x0, v0, C0, H0)]
        ckpts = []
        for s in range(plan.n_sub):
            if s % plan.ckpt == 0:
                ckpts.append([t.clone() for t in state])
            plan.substep(plan.particles(*state, E), W, s)
        plan.check_status("forward")
        ctx.plan = plan
        ctx.ckpts = ckpts
        ctx.save_for_backward(W, E)
        return tuple(state)

    @staticmethod
    def backward(ctx, xb, vb, Cb, Hb):
        plan = ctx.plan
        W, E = ctx.saved_tensors
        bar = [torch.zeros_like(t) if b is None else b.contiguous().clone()
               for b, t in zip((xb, vb, Cb, Hb), ctx.ckpts[0])]
        W_bar = torch.zeros_like(W)
        E_bar = torch.zeros_like(E)
        seg_bufs = plan.segment_buffers()
        # particle-state adjoints: two groups of (x, v, C, H) views, one fill each
        shapes = [t.shape for t in ctx.ckpts[0]]
        sizes = [t.numel() for t in ctx.ckpts[0]]
        pair = torch.empty(2, sum(sizes), dtype=torch.float32, device=W.device)
        groups = [list(t.view(sh) for t, sh in zip(torch.split(pair[k], sizes), shapes)) for k in range(2)]
        cur = 0
        for dst, b in zip(groups[cur], bar):
            dst.copy_(b)
        bar = groups[cur]
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * plan.ckpt
            s1 = min(s0 + plan.ckpt, plan.n_sub)
            # re-run the segment, keeping each substep's state, sort and grid
            states = [[t.clone() for t in ctx.ckpts[seg]]]
            for s in range(s0, s1):
                last = s == s1 - 1
                nxt = None if last else [torch.empty_like(t) for t in states[-1]]
                plan.substep(plan.particles(*states[-1], E), W, s, out=nxt, bufs=seg_bufs[s - s0], g2p=not last)
                if not last:
                    states.append(nxt)
            for s in reversed(range(s0, s1)):
                st = states[s - s0]
                nxt_group = groups[1 - cur]
                pair[1 - cur].zero_()
                plan.substep_adjoint(plan.particles(*st, E), W, s, bar, nxt_group, W_bar, E_bar,
                                     bufs=seg_bufs[s - s0])
                bar = nxt_group
                cur = 1 - cur
        plan.check_status("backward")
        return (None, W_bar, E_bar, *[b.clone() for b in bar])


def rollout(plan: RolloutPlan, W, E, x0, v0, C0, H0):
    """Differentiable n-substep rollout: returns the final (x, v, C, H), with
    gradients flowing to W (K, 3, nw^3), E (n_regions,) and the initial state.
    With plan.xref set, x0 and the returned x are displacements from it.
    Raises DiffWindError if a particle left the grid."""
    return _RolloutFn.apply(plan, W, E, x0, v0, C0, H0)
