"""Sequential reconstruction of the wind force field (Sec. 3.3) with the
physics-informed loss (Sec. 3.4), on synthetic targets.

The paper optimises, one time step after another, the force field that
drives the object from the previous optimised state to the observed next
state (initialised from zero each time), with a photometric loss plus the
physics-informed loss that aligns the force directions with the LBM wind
velocity.  Two observation models: `frame` compares particle positions with
those of a reference rollout (the position loss sum_p |x_p - x*_p|^2);
`frame_render` compares rendered images with target images (L_render of
Sec. 3.3: every particle is a Gaussian kernel whose covariance follows its
deformation gradient, Sigma(t) = F Sigma0 F^T, rendered by `gs_render`;
the gradient runs back through `render_loss`, `gs_render_adj`,
`gaussian_covariance_adj` and the rollout).  Both losses are normalised by
their value at W = 0.  Every step runs in the library's kernels; torch holds
the buffers and calls the rollout's backward.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import api
from .autograd import RolloutPlan, rollout


@dataclass
class View:
    """One camera with its target image and its device workspaces."""
    cam: api.Camera
    target: torch.Tensor          # (3, H, W)
    ws: api.RenderWorkspace
    loss_ws: torch.Tensor
    image: torch.Tensor           # (3, H, W) scratch for the rendered image


def make_view(cam: api.Camera, target, n: int, max_pairs: int, device="cuda") -> View:
    return View(cam, target, api.RenderWorkspace(n, cam, max_pairs, device=device),
                api.render_loss_workspace(3, cam.height, cam.width, device=device),
                torch.empty(3, cam.height, cam.width, device=device))


def render_image(view: View, mu, H, sigma0, color, opacity):
    """The image of kernels at mu (3, n) with covariances F sigma0 F^T (H = F - I)."""
    sig = torch.empty_like(sigma0)
    api.gaussian_covariance(H, sigma0, sig)
    img = torch.empty_like(view.image)
    api.gs_render(view.cam, mu, sig, color, opacity, img, view.ws)
    return img


def render_loss_grad(views, mu, H, sigma0, color, opacity, lam: float = 0.1):
    """L_render = sum over views of (1 - lam) L1 + lam (1 - SSIM) of the
    rendered kernels against the views' targets, and its gradients with
    respect to the centres mu (3, n) and H (9, n) (through Sigma = F sigma0 F^T)."""
    n = mu.shape[1]
    sig = torch.empty_like(sigma0)
    api.gaussian_covariance(H, sigma0, sig)
    L = torch.zeros(1, device=mu.device)
    mu_bar = torch.zeros_like(mu)
    sig_bar = torch.zeros_like(sigma0)
    for v in views:
        api.gs_render(v.cam, mu, sig, color, opacity, v.image, v.ws)
        ib = torch.zeros_like(v.image)
        api.render_loss(v.image, v.target, v.loss_ws, lam, L, ib)
        api.gs_render_adj(v.cam, mu, sig, color, opacity, v.image, ib, v.ws, mu_bar=mu_bar, sigma_bar=sig_bar)
    H_bar = torch.zeros(9, n, device=mu.device)
    api.gaussian_covariance_adj(H, sigma0, sig_bar, H_bar=H_bar)
    return L, mu_bar, H_bar


@dataclass
class FrameResult:
    W: torch.Tensor                      # (3, nw^3) reconstructed force field
    loss: list = field(default_factory=list)


class Reconstructor:
    """Frame-by-frame reconstruction of a force-grid wind for one particle set.

    Positions are displacements from the scene's positions (the rollout's
    position reference); `initial_state()` gives the scene at rest in that
    form, and the targets of `frame` are displacements too."""

    def __init__(self, scene, nw, box_lo, box_hi, substeps_per_frame: int, ckpt: int = 16, device="cuda"):
        f32 = dict(dtype=torch.float32, device=device)
        self.device = device
        n = scene.n
        self.nw = tuple(nw)
        self.n_nodes = nw[0] * nw[1] * nw[2]
        mass = torch.tensor(scene.mass, **f32)
        vol0 = torch.tensor(scene.vol0, **f32)
        region = torch.tensor(scene.region, dtype=torch.int32, device=device)
        nu = torch.tensor(scene.nu, **f32)
        pin = torch.tensor(scene.pin, dtype=torch.uint8, device=device)
        self.E = torch.tensor(scene.E, **f32)
        self.xref = torch.tensor(scene.x.T.copy(), **f32).contiguous()
        self.plan = RolloutPlan(scene.grid, n, mass, vol0, region, nu, pin, scene.dt, scene.gravity, scene.material,
                                scene.bound, nw, box_lo, box_hi, K=1, n_sub=substeps_per_frame, ckpt=ckpt,
                                device=device, xref=self.xref)

    def initial_state(self):
        """(x, v, C, H) of the scene at rest: zero displacement, v = C = 0, F = I."""
        n = self.xref.shape[1]
        z3 = torch.zeros(3, n, device=self.device)
        z9 = torch.zeros(9, n, device=self.device)
        return (z3, z3.clone(), z9, z9.clone())

    def advance(self, state, W):
        """One frame forward with force field W (3, nw^3); returns the new state."""
        with torch.no_grad():
            return rollout(self.plan, W.view(1, 3, self.n_nodes).contiguous(), self.E, *state)

    def frame(self, state, x_target, guide=None, lam: float = 0.0, iters: int = 30, lr: float = 0.5) -> FrameResult:
        """Optimise the force field of one frame from zero: Adam on
        L_pos / L_pos(W = 0) + lam * L_phys / (nodes with a guide)."""
        dev = self.device
        W = torch.zeros(1, 3, self.n_nodes, device=dev, requires_grad=True)
        m = torch.zeros_like(W)
        v = torch.zeros_like(W)
        xb = torch.empty_like(x_target)
        res = FrameResult(W=None)
        scale = None
        n_guided = None
        if guide is not None and lam > 0:
            cnt = torch.zeros(3, device=dev)
            api.direction_metrics(guide, guide, cnt)
            n_guided = max(float(cnt[2].item()), 1.0)
        for it in range(iters):
            xT = rollout(self.plan, W, self.E, *state)[0]
            lp = torch.zeros(1, device=dev)
            api.position_loss(xT.detach(), x_target, lp, xb)
            if scale is None:
                scale = max(float(lp.item()), 1e-30)
            W.grad = None
            torch.autograd.backward(xT, grad_tensors=xb / scale)
            total = float(lp.item()) / scale
            if n_guided is not None:
                lph = torch.zeros(1, device=dev)
                api.phys_loss(W.detach()[0], guide, lam / n_guided, lph, W.grad[0])
                total += float(lph.item())
            res.loss.append(total)
            api.adam_step(W.data, W.grad, m, v, lr, 0.9, 0.999, 1e-8, it + 1)
        res.W = W.detach()[0].clone()
        return res


    def frame_render(self, state, views, sigma0, color, opacity, guide=None, lam: float = 0.0, iters: int = 30,
                     lr: float = 0.5) -> FrameResult:
        """Optimise the force field of one frame from zero against target
        images: Adam on L_render / L_render(W = 0) + lam * L_phys / (nodes
        with a guide).  sigma0 (6, n), color (3, n), opacity (n,) describe
        the particles' Gaussian kernels at rest."""
        dev = self.device
        W = torch.zeros(1, 3, self.n_nodes, device=dev, requires_grad=True)
        m = torch.zeros_like(W)
        v = torch.zeros_like(W)
        res = FrameResult(W=None)
        scale = None
        n_guided = None
        if guide is not None and lam > 0:
            cnt = torch.zeros(3, device=dev)
            api.direction_metrics(guide, guide, cnt)
            n_guided = max(float(cnt[2].item()), 1.0)
        for it in range(iters):
            xT, _, _, HT = rollout(self.plan, W, self.E, *state)
            L, xb, Hb = render_loss_grad(views, self.xref + xT.detach(), HT.detach(), sigma0, color, opacity)
            if scale is None:
                scale = max(float(L.item()), 1e-30)
            W.grad = None
            torch.autograd.backward([xT, HT], grad_tensors=[xb / scale, Hb / scale])
            total = float(L.item()) / scale
            if n_guided is not None:
                lph = torch.zeros(1, device=dev)
                api.phys_loss(W.detach()[0], guide, lam / n_guided, lph, W.grad[0])
                total += float(lph.item())
            res.loss.append(total)
            api.adam_step(W.data, W.grad, m, v, lr, 0.9, 0.999, 1e-8, it + 1)
        res.W = W.detach()[0].clone()
        return res


def metrics(F_ref, F):
    """(CosSim, NMSE, locations) of two force fields (3, n)."""
    out = torch.zeros(3, device=F.device)
    api.direction_metrics(F_ref, F, out)
    c = max(float(out[2].item()), 1.0)
    return float(out[0].item()) / c, float(out[1].item()) / c, int(out[2].item())


def lbm_guide(scene, nw, box_lo, box_hi, steps: int = 300, device="cuda"):
    """The LBM wind around the object: the scene's tunnel (BGK, inlet, solid
    mask from the particles) run for `steps` steps, its velocity sampled at
    the wind-grid nodes; returns (guide (3, nw^3), u (3, L))."""
    lt, lb = scene.lattice, scene.lbm
    lat = api.make_lattice(lt["nx"], lt["ny"], lt["nz"], lt["dx"], lt["origin"])
    L = lt["nx"] * lt["ny"] * lt["nz"]
    kw = dict(tau=lb["tau"], u_in=lb["u_in"], force=lb["force"], bc=lb["bc"], gust_amp=lb["gust_amp"],
              gust_period=lb["gust_period"], gust_ky=lb["gust_ky"], gust_kz=lb["gust_kz"],
              gust_phase=lb["gust_phase"])
    fa = torch.empty(19, L, device=device)
    fb = torch.empty_like(fa)
    api.lbm_equilibrium(lat, api.make_lbm_params(**kw), fa)
    solid = torch.zeros(L, dtype=torch.uint8, device=device)
    x = torch.tensor(scene.x.T.copy(), dtype=torch.float32, device=device).contiguous()
    api.lbm_solid_from_particles(lat, x, solid)
    u = torch.empty(3, L, device=device)
    for t in range(steps):
        api.lbm_step(lat, api.make_lbm_params(**kw, t=t), fa, fb, solid, None, u)
        fa, fb = fb, fa
    guide = torch.empty(3, nw[0] * nw[1] * nw[2], device=device)
    api.wind_guide(lat, u, nw, box_lo, box_hi, guide)
    return guide, u


def drag_field(guide, amp: float):
    """A force field along the guide with the drag law's |U| U profile,
    scaled so that its largest vector has length amp."""
    sq = (guide * guide).sum(dim=0)
    s = torch.sqrt(sq)
    return guide * (amp * s / sq.max().clamp_min(1e-30))[None]
