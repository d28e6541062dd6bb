"""Pins of the rendering oracle (oracle/render.py) against closed forms,
brute force and finite differences (CPU)."""
import math

import numpy as np
import pytest
import torch

from oracle import render as orender

DT = torch.float64


def _cam(W=24, H=20, f=30.0, **kw):
    return orender.Camera(width=W, height=H, fx=f, fy=f * 1.1, cx=W / 2, cy=H / 2, **kw)


def _rot(a, b, c):
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    Rx = torch.tensor([[1, 0, 0], [0, ca, -sa], [0, sa, ca]], dtype=DT)
    Ry = torch.tensor([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]], dtype=DT)
    Rz = torch.tensor([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]], dtype=DT)
    return Rz @ Ry @ Rx


def test_isotropic_gaussian_on_the_axis_is_a_2d_gaussian():
    """A ball of scale s at depth z on the optical axis projects to a circle
    of pixel scale f s / z: the image is o c exp(-r^2 / (2 (f s / z)^2))."""
    cam = orender.Camera(width=32, height=32, fx=40.0, fy=40.0, cx=16.0, cy=16.0)
    z, s, o = 2.0, 0.08, 0.7
    c = torch.tensor([[0.2, 0.5, 0.9]], dtype=DT)
    img = orender.render(torch.tensor([[0.0, 0.0, z]], dtype=DT), (s * s) * torch.eye(3, dtype=DT)[None], c,
                         torch.tensor([o], dtype=DT), cam)
    X = orender.pixel_centres(cam)
    r2 = ((X - torch.tensor([16.0, 16.0], dtype=DT)) ** 2).sum(dim=1)
    sp = 40.0 * s / z
    ref = o * torch.exp(-r2 / (2 * sp * sp))
    for ch in range(3):
        assert (img[ch].reshape(-1) - c[0, ch] * ref).abs().max() < 1e-14


def test_projected_covariance_uses_the_projection_jacobian():
    """Sigma' equals J R Sigma R^T J^T with J taken by central differences of
    the perspective map, for an off-axis kernel under a rotated camera."""
    cam = _cam(R=tuple(map(tuple, _rot(0.3, -0.2, 0.4).tolist())), t=(0.1, -0.2, 3.0))
    rng = np.random.default_rng(1)
    mu = torch.tensor([[0.3, -0.1, 0.2]], dtype=DT)
    A = torch.tensor(rng.standard_normal((3, 3)), dtype=DT)
    Sigma = (A @ A.T + 0.1 * torch.eye(3, dtype=DT))[None] * 1e-3
    mu2, S2, z = orender.project(mu, Sigma, cam)
    R = torch.tensor(cam.R, dtype=DT)
    h = 1e-6
    Jw = torch.zeros(2, 3, dtype=DT)  # derivative of the projection with respect to the world point
    for a in range(3):
        e = torch.zeros(1, 3, dtype=DT)
        e[0, a] = h
        Jw[:, a] = (orender.project(mu + e, Sigma, cam)[0] - orender.project(mu - e, Sigma, cam)[0])[0] / (2 * h)
    ref = Jw @ Sigma[0] @ Jw.T
    assert (S2[0] - ref).abs().max() / ref.abs().max() < 1e-8
    p = R @ mu[0] + torch.tensor(cam.t, dtype=DT)
    assert abs(z[0].item() - p[2].item()) < 1e-15
    assert abs(mu2[0, 0].item() - (cam.fx * p[0] / p[2] + cam.cx).item()) < 1e-12


def test_front_to_back_blending_and_occlusion():
    """Two kernels whose centres project onto one pixel centre: the pixel is
    o1 c1 + (1 - o1) o2 c2 with kernel 1 in front, whatever the input order;
    swapping their depths swaps the roles; an opaque front kernel hides the
    back one."""
    cam = orender.Camera(width=16, height=16, fx=20.0, fy=20.0, cx=8.0, cy=8.0)
    # centres on the ray through pixel (8, 8), i.e. through (8.5, 8.5)
    def on_ray(z):
        return [(8.5 - 8.0) * z / 20.0, (8.5 - 8.0) * z / 20.0, z]
    S = 0.01 * torch.eye(3, dtype=DT)[None].repeat(2, 1, 1)
    c = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.5]], dtype=DT)
    o = torch.tensor([0.6, 0.8], dtype=DT)
    mu = torch.tensor([on_ray(1.0), on_ray(2.0)], dtype=DT)
    px = lambda img: img[:, 8, 8]
    a = px(orender.render(mu, S, c, o, cam))
    b = px(orender.render(mu.flip(0), S.flip(0), c.flip(0), o.flip(0), cam))
    want = o[0] * c[0] + (1 - o[0]) * o[1] * c[1]
    assert (a - want).abs().max() < 1e-15 and (b - want).abs().max() < 1e-15
    mu_sw = torch.tensor([on_ray(2.0), on_ray(1.0)], dtype=DT)
    d = px(orender.render(mu_sw, S, c, o, cam))
    assert (d - (o[1] * c[1] + (1 - o[1]) * o[0] * c[0])).abs().max() < 1e-15
    e = px(orender.render(mu, S, c, torch.tensor([1.0, 0.8], dtype=DT), cam))
    assert (e - c[0]).abs().max() < 1e-15


def test_background_and_near_plane():
    """Uncovered pixels show the background; a kernel behind the near plane
    is not drawn."""
    cam = _cam(bg=(0.1, 0.2, 0.3))
    mu = torch.tensor([[0.0, 0.0, -1.0]], dtype=DT)
    img = orender.render(mu, 0.01 * torch.eye(3, dtype=DT)[None], torch.ones(1, 3, dtype=DT),
                         torch.ones(1, dtype=DT), cam)
    assert torch.equal(img, torch.tensor(cam.bg, dtype=DT).view(3, 1, 1).expand_as(img))


def _ssim_brute(a, b, size=11, sigma=1.5, C1=0.01 ** 2, C2=0.03 ** 2):
    """SSIM with explicit window sums at every pixel (zero outside the image)."""
    g = orender.gaussian_window(size, sigma)
    C, H, W = a.shape
    h = size // 2
    tot = 0.0
    for ch in range(C):
        for y in range(H):
            for x in range(W):
                s = [0.0] * 5
                for dy in range(-h, h + 1):
                    for dx in range(-h, h + 1):
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W:
                            wgt = g[dy + h, dx + h].item()
                            va, vb = a[ch, yy, xx].item(), b[ch, yy, xx].item()
                            s[0] += wgt * va
                            s[1] += wgt * vb
                            s[2] += wgt * va * va
                            s[3] += wgt * vb * vb
                            s[4] += wgt * va * vb
                ma, mb = s[0], s[1]
                va_, vb_, cab = s[2] - ma * ma, s[3] - mb * mb, s[4] - ma * mb
                tot += ((2 * ma * mb + C1) * (2 * cab + C2)) / ((ma * ma + mb * mb + C1) * (va_ + vb_ + C2))
    return tot / (C * H * W)


def test_ssim_and_l1():
    rng = np.random.default_rng(3)
    a = torch.tensor(rng.random((3, 13, 15)), dtype=DT)
    b = torch.tensor(rng.random((3, 13, 15)), dtype=DT)
    assert abs(orender.ssim(a, a).item() - 1.0) < 1e-14
    assert abs(orender.ssim(a, b).item() - _ssim_brute(a, b)) < 1e-12
    assert abs(orender.l1(a, b).item() - (a - b).abs().sum().item() / a.numel()) < 1e-15
    g = orender.gaussian_window()
    assert abs(g.sum().item() - 1.0) < 1e-15 and torch.equal(g, g.T)
    L = orender.render_loss([a, b], [b, b], lam=0.1)
    want = 0.9 * orender.l1(a, b) + 0.1 * (1 - orender.ssim(a, b))
    assert abs(L.item() - want.item()) < 1e-15


def test_render_gradients_match_finite_differences():
    """Autograd of L_render through the renderer against central differences
    for centres, covariances, colours and opacities."""
    cam = _cam(R=tuple(map(tuple, _rot(0.2, 0.1, -0.3).tolist())), t=(0.0, 0.1, 2.5))
    rng = np.random.default_rng(4)
    n = 6
    mu = torch.tensor(rng.uniform(-0.3, 0.3, (n, 3)), dtype=DT)
    A = torch.tensor(rng.standard_normal((n, 3, 3)), dtype=DT) * 0.06
    Sigma = A @ A.transpose(1, 2) + 1e-3 * torch.eye(3, dtype=DT)
    col = torch.tensor(rng.random((n, 3)), dtype=DT)
    op = torch.tensor(rng.uniform(0.3, 0.9, n), dtype=DT)
    target = torch.tensor(rng.random((3, cam.height, cam.width)), dtype=DT)
    args = [mu, Sigma, col, op]
    leaves = [t.clone().requires_grad_(True) for t in args]
    L = orender.render_loss([orender.render(*leaves, cam)], [target])
    grads = torch.autograd.grad(L, leaves)
    h = 1e-6
    for k, g in enumerate(grads):
        for idx in [tuple(int(rng.integers(0, s)) for s in args[k].shape) for _ in range(4)]:
            if k == 1:  # keep the covariance symmetric: perturb the pair
                i, a_, b_ = idx
                if a_ == b_:
                    b_ = (a_ + 1) % 3
                pert = lambda t, e: t.index_put_((torch.tensor([i]), torch.tensor([a_]), torch.tensor([b_])),
                                                 torch.tensor([e], dtype=DT), accumulate=True)
                vals = []
                for e in (h, -h):
                    S = Sigma.clone()
                    pert(S, e)
                    S[i, b_, a_] += e
                    vals.append(orender.render_loss([orender.render(mu, S, col, op, cam)], [target]).item())
                fd = (vals[0] - vals[1]) / (2 * h)
                an = g[i, a_, b_].item() + g[i, b_, a_].item()
            else:
                vals = []
                for e in (h, -h):
                    t = [x.clone() for x in args]
                    t[k][idx] += e
                    vals.append(orender.render_loss([orender.render(*t, cam)], [target]).item())
                fd = (vals[0] - vals[1]) / (2 * h)
                an = g[idx].item()
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, idx, fd, an)


def test_truncations_and_pixel_subset():
    """alpha_min drops a kernel whose alpha stays below it (the image equals
    the render without that kernel); t_min stops a pixel after the kernel
    that takes its transmittance below it; a pixel subset gives the same
    colours as the full image."""
    cam = orender.Camera(width=16, height=16, fx=20.0, fy=20.0, cx=8.0, cy=8.0, bg=(0.2, 0.3, 0.4))
    def on_ray(z):
        return [(8.5 - 8.0) * z / 20.0, (8.5 - 8.0) * z / 20.0, z]
    S = 0.01 * torch.eye(3, dtype=DT)[None].repeat(3, 1, 1)
    c = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.5], [0.3, 0.3, 0.3]], dtype=DT)
    mu = torch.tensor([on_ray(1.0), on_ray(2.0), on_ray(3.0)], dtype=DT)
    o = torch.tensor([0.6, 0.8, 1e-3], dtype=DT)
    full = orender.render(mu, S, c, o, cam)
    cam_a = orender.Camera(**{**cam.__dict__, "alpha_min": 2e-3})
    bg = torch.tensor(cam.bg, dtype=DT)
    two = o[0] * c[0] + (1 - o[0]) * o[1] * c[1] + (1 - o[0]) * (1 - o[1]) * bg
    assert (orender.render(mu, S, c, o, cam_a)[:, 8, 8] - two).abs().max() < 1e-15
    assert (full[:, 8, 8] - two).abs().max() > 5e-6
    cam_t = orender.Camera(**{**cam.__dict__, "t_min": 0.5})
    px = orender.render(mu, S, c, o, cam_t)[:, 8, 8]
    want = o[0] * c[0] + (1 - o[0]) * torch.tensor(cam.bg, dtype=DT)
    assert (px - want).abs().max() < 1e-15
    pix = torch.tensor([[8.5, 8.5], [0.5, 15.5], [3.5, 7.5]], dtype=DT)
    sub = orender.render(mu, S, c, o, cam, pixels=pix)
    for k, (x, y) in enumerate(pix.tolist()):
        assert (sub[:, k] - full[:, int(y), int(x)]).abs().max() < 1e-15
