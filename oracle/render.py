"""FP64 oracle: differentiable rendering of the 3D Gaussian kernels and the
photometric loss L_render (test infrastructure only).

Follows Sec. 3.3 (Eq. rendering and the loss L_render) and the appendix
"3D Gaussian Representation":

* a Gaussian kernel has a centre mu (the MPM particle position), a
  covariance Sigma (after deformation Sigma(t) = F Sigma F^T, oracle.gauss),
  a colour c and an opacity o;
* a view is a rigid transformation W = [R | t] (world to camera) and a
  pinhole camera (focal lengths fx, fy and principal point cx, cy in pixels);
  a camera point p = R mu + t projects to (fx p_x / p_z + cx, fy p_y / p_z + cy);
* the 2-D covariance is Sigma' = J R Sigma R^T J^T with J the Jacobian of the
  projection at p (the affine approximation of the projective map);
* at pixel centre x, alpha_i = o_i exp(-1/2 (x - mu'_i)^T Sigma'_i^-1 (x - mu'_i)),
  the kernels ordered front to back by camera depth p_z, and the colour is
  C(x) = sum_i T_i c_i alpha_i with T_i = prod_{j<i} (1 - alpha_j), plus
  T_N times a background colour;
* L_render = sum over views of (1 - lambda) L1 + lambda L_D-SSIM with
  lambda = 0.1, L1 the mean absolute difference over pixels and channels,
  L_D-SSIM = 1 - SSIM, SSIM the structural similarity index (Wang et al.
  2004) per channel with an 11 x 11 Gaussian window (sigma 1.5),
  C1 = 0.01^2, C2 = 0.03^2 (unit dynamic range), windows zero-padded at the
  image border, averaged over pixels and channels.

Readings: the projected centre is the perspective projection of W mu (the
printed mu' = J W mu is the affine approximation's linear part); pixel
(i, j) (column i, row j) has its centre at (i + 1/2, j + 1/2); kernels with
camera depth at or below `near` are not drawn; no low-pass dilation is
added to Sigma' (the equations have none); colours are per-kernel RGB
(view-independent).  Two optional truncations of the sum, both off by
default (the plain sum of the equation): alpha below `alpha_min` is not
blended, and a pixel stops blending once its transmittance has fallen below
`t_min` (the kernel that takes it below still counts).  Equal depths keep
the input order.

Parity pins: tests/test_oracle_render.py.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

_DT = torch.float64


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: tuple = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    t: tuple = (0.0, 0.0, 0.0)
    near: float = 0.01
    bg: tuple = (0.0, 0.0, 0.0)
    alpha_min: float = 0.0
    t_min: float = 0.0


def project(mu, Sigma, cam: Camera):
    """Projected centres (n, 2), 2-D covariances (n, 2, 2) and camera depths (n,)."""
    R = torch.tensor(cam.R, dtype=_DT)
    t = torch.tensor(cam.t, dtype=_DT)
    p = mu @ R.T + t
    z = p[:, 2]
    mu2 = torch.stack([cam.fx * p[:, 0] / z + cam.cx, cam.fy * p[:, 1] / z + cam.cy], dim=1)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([cam.fx / z, zero, -cam.fx * p[:, 0] / z ** 2], dim=1),
                     torch.stack([zero, cam.fy / z, -cam.fy * p[:, 1] / z ** 2], dim=1)], dim=1)
    JR = J @ R
    Sigma2 = JR @ Sigma @ JR.transpose(1, 2)
    return mu2, Sigma2, z


def pixel_centres(cam: Camera):
    """(H * W, 2) pixel centres, row-major (x fastest)."""
    j, i = torch.meshgrid(torch.arange(cam.height, dtype=_DT), torch.arange(cam.width, dtype=_DT), indexing="ij")
    return torch.stack([i.reshape(-1) + 0.5, j.reshape(-1) + 0.5], dim=1)


def render(mu, Sigma, color, opacity, cam: Camera, pixels=None):
    """The image (3, H, W) of Eq. rendering by alpha blending, every kernel
    against every pixel (brute force); with `pixels` ((P, 2) pixel centres)
    the colours (3, P) of those pixels only."""
    mu2, S2, z = project(mu, Sigma, cam)
    keep = z > cam.near
    order = torch.argsort(z[keep], stable=True)
    mu2, S2, col, op = mu2[keep][order], S2[keep][order], color[keep][order], opacity[keep][order]
    X = pixel_centres(cam) if pixels is None else pixels
    d = X[None, :, :] - mu2[:, None, :]                       # (n, P, 2)
    Sinv = torch.linalg.inv(S2)                              # (n, 2, 2)
    q = torch.einsum("npa,nab,npb->np", d, Sinv, d)
    alpha = op[:, None] * torch.exp(-0.5 * q)                # (n, P)
    if cam.alpha_min > 0.0:
        alpha = alpha * (alpha.detach() >= cam.alpha_min)
    ones = torch.ones(1, X.shape[0], dtype=_DT)
    if cam.t_min > 0.0:
        # transmittance in front of each kernel before truncation: a kernel is
        # blended while it is at least t_min
        T_raw = torch.cumprod(torch.cat([ones, 1.0 - alpha.detach()], dim=0), dim=0)[:-1]
        alpha = alpha * (T_raw >= cam.t_min)
    T = torch.cumprod(torch.cat([ones, 1.0 - alpha], dim=0), dim=0)  # (n + 1, P)
    C = (T[:-1, :, None] * alpha[:, :, None] * col[:, None, :]).sum(dim=0)               # (P, 3)
    C = C + T[-1][:, None] * torch.tensor(cam.bg, dtype=_DT)[None, :]
    return C.T if pixels is not None else C.T.reshape(3, cam.height, cam.width)


def gaussian_window(size: int = 11, sigma: float = 1.5):
    """Normalised 2-D Gaussian window (size, size)."""
    r = torch.arange(size, dtype=_DT) - (size - 1) / 2.0
    g = torch.exp(-r ** 2 / (2.0 * sigma ** 2))
    g = g / g.sum()
    return g[:, None] * g[None, :]


def ssim(a, b, size: int = 11, sigma: float = 1.5, C1: float = 0.01 ** 2, C2: float = 0.03 ** 2):
    """Mean SSIM of two images (3, H, W): local means, variances and covariance
    under the Gaussian window (zero-padded), the SSIM map
    ((2 ma mb + C1)(2 s_ab + C2)) / ((ma^2 + mb^2 + C1)(s_a^2 + s_b^2 + C2)),
    averaged over pixels and channels."""
    w = gaussian_window(size, sigma)[None, None].expand(a.shape[0], 1, size, size)
    conv = lambda x: torch.nn.functional.conv2d(x[None], w, padding=size // 2, groups=a.shape[0])[0]
    ma, mb = conv(a), conv(b)
    saa = conv(a * a) - ma * ma
    sbb = conv(b * b) - mb * mb
    sab = conv(a * b) - ma * mb
    m = ((2 * ma * mb + C1) * (2 * sab + C2)) / ((ma * ma + mb * mb + C1) * (saa + sbb + C2))
    return m.mean()


def l1(a, b):
    return (a - b).abs().mean()


def render_loss(images, targets, lam: float = 0.1):
    """L_render = sum over views (1 - lam) L1 + lam (1 - SSIM)."""
    return sum((1.0 - lam) * l1(a, b) + lam * (1.0 - ssim(a, b)) for a, b in zip(images, targets))
