"""The rendering pins reject plausible mistakes: each mutant below plants one
slip in a copy of the oracle's projection, blending or loss, and at least
one pin must move by far more than its tolerance (CPU)."""
import math
import types

import numpy as np
import torch

from oracle import render as orender

DT = torch.float64


def _project(mu, Sigma, cam, jsign=1.0, rot_t=False):
    R = torch.tensor(cam.R, dtype=DT)
    t = torch.tensor(cam.t, dtype=DT)
    p = mu @ R.T + t
    z = p[:, 2]
    mu2 = torch.stack([cam.fx * p[:, 0] / z + cam.cx, cam.fy * p[:, 1] / z + cam.cy], dim=1)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([cam.fx / z, zero, -jsign * cam.fx * p[:, 0] / z ** 2], dim=1),
                     torch.stack([zero, cam.fy / z, -jsign * cam.fy * p[:, 1] / z ** 2], dim=1)], dim=1)
    JR = J @ (R.T if rot_t else R)
    return mu2, JR @ Sigma @ JR.transpose(1, 2), z


def _render(mu, Sigma, color, opacity, cam, pixels=None, half=0.5, expo=0.5, inclusive=False, back_to_front=False,
            no_bg=False, project=_project):
    mu2, S2, z = project(mu, Sigma, cam)
    keep = z > cam.near
    order = torch.argsort(z[keep], stable=True, descending=back_to_front)
    mu2, S2, col, op = mu2[keep][order], S2[keep][order], color[keep][order], opacity[keep][order]
    if pixels is None:
        j, i = torch.meshgrid(torch.arange(cam.height, dtype=DT), torch.arange(cam.width, dtype=DT), indexing="ij")
        X = torch.stack([i.reshape(-1) + half, j.reshape(-1) + half], dim=1)
    else:
        X = pixels
    d = X[None] - mu2[:, None]
    q = torch.einsum("npa,nab,npb->np", d, torch.linalg.inv(S2), d)
    alpha = op[:, None] * torch.exp(-expo * q)
    T = torch.cumprod(torch.cat([torch.ones(1, X.shape[0], dtype=DT), 1.0 - alpha]), dim=0)
    Tw = T[1:] if inclusive else T[:-1]
    C = (Tw[:, :, None] * alpha[:, :, None] * col[:, None, :]).sum(dim=0)
    if not no_bg:
        C = C + T[-1][:, None] * torch.tensor(cam.bg, dtype=DT)[None]
    return C.T if pixels is not None else C.T.reshape(3, cam.height, cam.width)


def _ssim(a, b, size=11, sigma=1.5, C1=0.01 ** 2, C2=0.03 ** 2, swap_c=False, raw_var=False):
    if swap_c:
        C1, C2 = C2, C1
    w = orender.gaussian_window(size, sigma)[None, None].expand(a.shape[0], 1, size, size)
    conv = lambda x: torch.nn.functional.conv2d(x[None], w, padding=size // 2, groups=a.shape[0])[0]
    ma, mb = conv(a), conv(b)
    saa = conv(a * a) - (0 if raw_var else ma * ma)
    sbb = conv(b * b) - (0 if raw_var else mb * mb)
    sab = conv(a * b) - ma * mb
    return (((2 * ma * mb + C1) * (2 * sab + C2)) / ((ma * ma + mb * mb + C1) * (saa + sbb + C2))).mean()


def _impl(**kw):
    """A namespace of (possibly mutated) render, ssim and render_loss."""
    rkw = {k: kw[k] for k in ("half", "expo", "inclusive", "back_to_front", "no_bg") if k in kw}
    pkw = {k: kw[k] for k in ("jsign", "rot_t") if k in kw}
    skw = {k: kw[k] for k in ("swap_c", "raw_var") if k in kw}
    proj = lambda mu, S, cam: _project(mu, S, cam, **pkw)
    ssim = lambda a, b: _ssim(a, b, **skw)
    lam_swap = kw.get("lam_swap", False)

    def loss(images, targets, lam=0.1):
        l = 1.0 - lam if not lam_swap else lam
        return sum(l * orender.l1(x, y) + (1.0 - l) * (1.0 - ssim(x, y)) for x, y in zip(images, targets))
    return types.SimpleNamespace(
        project=proj, render=lambda *a, **k: _render(*a, **k, **rkw, project=proj), ssim=ssim, render_loss=loss)


def _rot(a, b, c):
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    Rx = torch.tensor([[1, 0, 0], [0, ca, -sa], [0, sa, ca]], dtype=DT)
    Ry = torch.tensor([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]], dtype=DT)
    Rz = torch.tensor([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]], dtype=DT)
    return Rz @ Ry @ Rx


def _pins(R):
    """The render pins as error measures (each 0 up to rounding for a correct
    implementation)."""
    e = {}
    # on-axis isotropic kernel: closed-form 2-D Gaussian
    cam = orender.Camera(width=32, height=32, fx=40.0, fy=40.0, cx=16.0, cy=16.0)
    z, s, o = 2.0, 0.08, 0.7
    c = torch.tensor([[0.2, 0.5, 0.9]], dtype=DT)
    img = R.render(torch.tensor([[0.0, 0.0, z]], dtype=DT), (s * s) * torch.eye(3, dtype=DT)[None], c,
                   torch.tensor([o], dtype=DT), cam)
    X = orender.pixel_centres(cam)
    ref = o * torch.exp(-((X - 16.0) ** 2).sum(dim=1) / (2 * (40.0 * s / z) ** 2))
    e["axis"] = max((img[ch].reshape(-1) - c[0, ch] * ref).abs().max().item() for ch in range(3))
    # projected covariance against central differences of the perspective map
    cam = orender.Camera(width=24, height=20, fx=30.0, fy=33.0, cx=12.0, cy=10.0,
                         R=tuple(map(tuple, _rot(0.3, -0.2, 0.4).tolist())), t=(0.1, -0.2, 3.0))
    rng = np.random.default_rng(1)
    mu = torch.tensor([[0.3, -0.1, 0.2]], dtype=DT)
    A = torch.tensor(rng.standard_normal((3, 3)), dtype=DT)
    Sig = (A @ A.T + 0.1 * torch.eye(3, dtype=DT))[None] * 1e-3
    _, S2, _ = R.project(mu, Sig, cam)
    h = 1e-6
    Jw = torch.zeros(2, 3, dtype=DT)
    for a in range(3):
        ea = torch.zeros(1, 3, dtype=DT)
        ea[0, a] = h
        Jw[:, a] = (R.project(mu + ea, Sig, cam)[0] - R.project(mu - ea, Sig, cam)[0])[0] / (2 * h)
    refS = Jw @ Sig[0] @ Jw.T
    e["jacobian"] = ((S2[0] - refS).abs().max() / refS.abs().max()).item()
    # two kernels on one pixel ray: front-to-back, background behind
    cam = orender.Camera(width=16, height=16, fx=20.0, fy=20.0, cx=8.0, cy=8.0, bg=(0.2, 0.3, 0.4))
    ray = lambda zz: [0.5 * zz / 20.0, 0.5 * zz / 20.0, zz]
    S = 0.01 * torch.eye(3, dtype=DT)[None].repeat(2, 1, 1)
    cc = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.5]], dtype=DT)
    oo = torch.tensor([0.6, 0.8], dtype=DT)
    px = R.render(torch.tensor([ray(2.0), ray(1.0)], dtype=DT), S, cc.flip(0), oo.flip(0), cam)[:, 8, 8]
    bg = torch.tensor(cam.bg, dtype=DT)
    want = oo[0] * cc[0] + (1 - oo[0]) * oo[1] * cc[1] + (1 - oo[0]) * (1 - oo[1]) * bg
    e["blend"] = (px - want).abs().max().item()
    # SSIM against explicit window sums; L_render's mix
    rng = np.random.default_rng(3)
    a = torch.tensor(rng.random((3, 9, 10)), dtype=DT)
    b = torch.tensor(rng.random((3, 9, 10)), dtype=DT)
    g = orender.gaussian_window()
    tot = 0.0
    for ch in range(3):
        for y in range(9):
            for x in range(10):
                s5 = [0.0] * 5
                for dy in range(-5, 6):
                    for dx in range(-5, 6):
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < 9 and 0 <= xx < 10:
                            wgt = g[dy + 5, dx + 5].item()
                            va, vb = a[ch, yy, xx].item(), b[ch, yy, xx].item()
                            s5 = [s5[0] + wgt * va, s5[1] + wgt * vb, s5[2] + wgt * va * va, s5[3] + wgt * vb * vb,
                                  s5[4] + wgt * va * vb]
                ma, mb = s5[0], s5[1]
                va_, vb_, cab = s5[2] - ma * ma, s5[3] - mb * mb, s5[4] - ma * mb
                tot += ((2 * ma * mb + 1e-4) * (2 * cab + 9e-4)) / ((ma * ma + mb * mb + 1e-4) * (va_ + vb_ + 9e-4))
    e["ssim"] = abs(R.ssim(a, b).item() - tot / (3 * 9 * 10))
    L = R.render_loss([a], [b], lam=0.1).item()
    want = 0.9 * (a - b).abs().mean().item() + 0.1 * (1.0 - tot / (3 * 9 * 10))
    e["loss"] = abs(L - want)
    return e


MUTANTS = {
    "Jacobian z-term sign": dict(jsign=-1.0),
    "rotation transposed in J R Sigma R^T J^T": dict(rot_t=True),
    "exponent without the 1/2": dict(expo=1.0),
    "transmittance including the kernel itself": dict(inclusive=True),
    "back-to-front order": dict(back_to_front=True),
    "background term dropped": dict(no_bg=True),
    "pixel centres at integer coordinates": dict(half=0.0),
    "SSIM constants exchanged": dict(swap_c=True),
    "SSIM variances without the mean": dict(raw_var=True),
    "L1 and D-SSIM weights exchanged": dict(lam_swap=True),
}


def test_render_pins_pass_on_the_oracle_and_reject_each_mutant():
    ref = _pins(types.SimpleNamespace(project=orender.project, render=orender.render, ssim=orender.ssim,
                                      render_loss=orender.render_loss))
    assert max(ref.values()) < 1e-7, ref
    same = _pins(_impl())  # the test's own unmutated copy agrees with the oracle
    assert max(same.values()) < 1e-7, same
    for name, kw in MUTANTS.items():
        e = _pins(_impl(**kw))
        assert max(e.values()) > 1e-4, (name, e)
