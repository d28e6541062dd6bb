"""Seeded synthetic wind-tunnel scenes (inputs only; no simulation arithmetic).

The paper's scenes (flags, cloth, leaves and plants reconstructed as
Gaussian splats; Sec. 4, Tab. sim_time with 52k-146k object particles on a
128^3 grid) are not available, so these generators produce inputs of the
same shape: thin sheets and ellipsoidal leaf clusters sampled uniformly, per
region Young's modulus, a pin mask, and a D3Q19 wind tunnel around them.

Everything here is plain data generation with numpy's PCG64; the same arrays
feed the HIP path and the float64 oracle.  Particle storage order is sorted
by 4x4x4 cell tile and then by cell, so that nearby particles are nearby in
memory (the way a densified splat cloud would be stored after a spatial
sort); the simulation never depends on that order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# boundary codes per lattice face, same values as the C header
BC_PERIODIC, BC_BOUNCEBACK, BC_INLET, BC_OUTLET = 0, 1, 2, 3
FIXED_COROTATED, NEO_HOOKEAN = 0, 1


@dataclass
class Scene:
    name: str
    grid: dict                 # nx, ny, nz, dx, origin
    x: np.ndarray              # (n, 3) float64
    mass: np.ndarray           # (n,)
    vol0: np.ndarray           # (n,)
    region: np.ndarray         # (n,) int32
    E: np.ndarray              # (R,)
    nu: np.ndarray             # (R,)
    pin: np.ndarray            # (N,) uint8, dense node order i + nx (j + ny k)
    dt: float
    gravity: tuple
    material: int
    bound: int = 3
    lattice: dict | None = None     # nx, ny, nz, dx, origin
    lbm: dict | None = None         # tau, u_in, bc, gust_*
    wind: dict = field(default_factory=dict)
    seed: int = 0

    @property
    def n(self):
        return self.x.shape[0]


def _sort_spatially(x, dx, origin):
    cell = np.floor((x - np.asarray(origin)) / dx).astype(np.int64)
    tile = cell // 4
    key = (((tile[:, 2] * 4096 + tile[:, 1]) * 4096 + tile[:, 0]) * 64
           + (cell[:, 2] % 4) * 16 + (cell[:, 1] % 4) * 4 + (cell[:, 0] % 4))
    return np.argsort(key, kind="stable")


def _pin_boxes(grid, boxes):
    nx, ny, nz, dx = grid["nx"], grid["ny"], grid["nz"], grid["dx"]
    o = np.asarray(grid["origin"])
    # node positions per axis (i dx + origin); a box is a product of ranges
    axes = [np.arange(m) * dx + o[a] for a, m in enumerate((nx, ny, nz))]
    pin = np.zeros((nz, ny, nx), dtype=np.uint8)
    for lo, hi in boxes:
        ix, iy, iz = [np.nonzero((axes[a] >= lo[a]) & (axes[a] <= hi[a]))[0] for a in range(3)]
        pin[np.ix_(iz, iy, ix)] = 1
    return pin.reshape(-1)


def _cfl_dt(E_max, nu, rho, dx, cfl=0.4):
    mu = E_max / (2 * (1 + nu))
    lam = E_max * nu / ((1 + nu) * (1 - 2 * nu))
    cp = math.sqrt((lam + 2 * mu) / rho)
    return cfl * dx / cp


def sheet_scene(seed: int = 0, n: int = 20_000, res: int = 32):
    """Small plain-method scene: a 0.5 x 0.5 x 0.02 sheet pinned on one edge.

    32^3 grid (dx = 1/32), fixed-corotated E = 1e4, nu = 0.3, rho = 1,
    dt = 1e-4; a 32^3 D3Q19 lattice with tau = 0.6, uniform inflow 0.05
    along +x, bounce-back walls on y and z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = 1.0 / res
    lo = np.array([0.49, 0.25, 0.25])
    hi = np.array([0.51, 0.75, 0.75])
    x = lo + (hi - lo) * rng.random((n, 3))
    vol = np.prod(hi - lo)
    grid = dict(nx=res, ny=res, nz=res, dx=dx, origin=(0.0, 0.0, 0.0))
    order = _sort_spatially(x, dx, grid["origin"])
    x = x[order]
    rho = 1.0
    vol0 = np.full(n, vol / n)
    pin = _pin_boxes(grid, [((0.49 - 2 * dx, 0.75 - dx, 0.25 - 2 * dx),
                             (0.51 + 2 * dx, 0.75 + 3 * dx, 0.75 + 2 * dx))])
    lattice = dict(nx=res, ny=res, nz=res, dx=dx, origin=(0.0, 0.0, 0.0))
    lbm = dict(tau=0.6, u_in=(0.05, 0.0, 0.0), force=(0.0, 0.0, 0.0),
               bc=(BC_INLET, BC_OUTLET, BC_BOUNCEBACK, BC_BOUNCEBACK, BC_BOUNCEBACK, BC_BOUNCEBACK),
               gust_amp=0.0, gust_period=1.0, gust_ky=0.0, gust_kz=0.0, gust_phase=0.0)
    return Scene(name=f"sheet{res}_n{n}", grid=grid, x=x, mass=rho * vol0, vol0=vol0,
                 region=np.zeros(n, np.int32), E=np.array([1e4]), nu=np.array([0.3]), pin=pin,
                 dt=1e-4, gravity=(0.0, -9.8, 0.0), material=FIXED_COROTATED, lattice=lattice,
                 lbm=lbm, wind=dict(mode="lbm", vel_scale=20.0, k_drag=9.8), seed=seed)


def _ellipsoid_points(rng, centre, axes, count):
    pts = np.empty((0, 3))
    while pts.shape[0] < count:
        cand = rng.uniform(-1.0, 1.0, (2 * count + 16, 3))
        cand = cand[np.sum(cand * cand, axis=1) <= 1.0]
        pts = np.concatenate([pts, cand], axis=0)
    return centre + pts[:count] * axes


def flag_and_leaves_scene(seed: int = 0, n: int = 500_000, res: int = 128, n_clusters: int = 40,
                          lbm_dims=(128, 64, 64), n_regions: int | None = None,
                          E_range=(1e3, 1e5), sheet_fraction: float = 0.5):
    """Paper-scale forward scene: one thin flag sheet plus ellipsoidal leaf clusters.

    Cluster semi-axes uniform in [0.01, 0.05], centres in [0.5, 0.85] x
    [0.3, 0.7]^2; particle counts proportional to volume; per-region E
    log-uniform in E_range (``n_regions`` caps the number of distinct
    materials, cycling regions over them); nu = 0.3, rho = 1; dt from the
    CFL condition dt = 0.4 dx / c_p at the stiffest E; the sheet's top edge
    and the top tenth of every cluster are pinned.  LBM tunnel of
    ``lbm_dims`` nodes at spacing 1/lbm_dims[0] centred on the objects,
    inflow 0.08 along +x with a seeded 5 % sinusoidal gust."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = 1.0 / res
    grid = dict(nx=res, ny=res, nz=res, dx=dx, origin=(0.0, 0.0, 0.0))
    s_lo = np.array([0.40, 0.27, 0.27])
    s_hi = np.array([0.42, 0.73, 0.73])
    n_sheet = int(round(n * sheet_fraction))
    axes = rng.uniform(0.01, 0.05, (n_clusters, 3))
    centres = np.stack([rng.uniform(0.5, 0.85, n_clusters), rng.uniform(0.3, 0.7, n_clusters),
                        rng.uniform(0.3, 0.7, n_clusters)], axis=1)
    vols = 4.0 / 3.0 * math.pi * np.prod(axes, axis=1)
    counts = np.floor(vols / vols.sum() * (n - n_sheet)).astype(np.int64)
    counts[: (n - n_sheet) - counts.sum()] += 1
    xs = [s_lo + (s_hi - s_lo) * rng.random((n_sheet, 3))]
    vol0 = [np.full(n_sheet, np.prod(s_hi - s_lo) / n_sheet)]
    regions = [np.zeros(n_sheet, np.int32)]
    pin_boxes = [((s_lo[0] - 2 * dx, s_hi[1] - dx, s_lo[2] - 2 * dx),
                  (s_hi[0] + 2 * dx, s_hi[1] + 3 * dx, s_hi[2] + 2 * dx))]
    for c in range(n_clusters):
        pts = _ellipsoid_points(rng, centres[c], axes[c], int(counts[c]))
        xs.append(pts)
        vol0.append(np.full(counts[c], vols[c] / max(counts[c], 1)))
        regions.append(np.full(counts[c], c + 1, np.int32))
        top = centres[c][1] + 0.8 * axes[c][1]
        pin_boxes.append(((centres[c][0] - axes[c][0] - dx, top, centres[c][2] - axes[c][2] - dx),
                          (centres[c][0] + axes[c][0] + dx, top + axes[c][1] + 2 * dx,
                           centres[c][2] + axes[c][2] + dx)))
    x = np.concatenate(xs)
    vol0 = np.concatenate(vol0)
    region = np.concatenate(regions)
    R = n_clusters + 1
    E = np.exp(rng.uniform(math.log(E_range[0]), math.log(E_range[1]), R))
    if n_regions is not None:
        region = region % n_regions
        E = E[:n_regions]
        R = n_regions
    nu = np.full(R, 0.3)
    order = _sort_spatially(x, dx, grid["origin"])
    x, vol0, region = x[order], vol0[order], region[order]
    rho = 1.0
    dt = _cfl_dt(E.max(), 0.3, rho, dx)
    pin = _pin_boxes(grid, pin_boxes)
    lnx, lny, lnz = lbm_dims
    ldx = 1.0 / lnx
    lorigin = (0.0, 0.5 - 0.5 * lny * ldx, 0.5 - 0.5 * lnz * ldx)
    lattice = dict(nx=lnx, ny=lny, nz=lnz, dx=ldx, origin=lorigin)
    lbm = dict(tau=0.6, u_in=(0.08, 0.0, 0.0), force=(0.0, 0.0, 0.0),
               bc=(BC_INLET, BC_OUTLET, BC_BOUNCEBACK, BC_BOUNCEBACK, BC_BOUNCEBACK, BC_BOUNCEBACK),
               gust_amp=0.05, gust_period=float(rng.uniform(100, 400)),
               gust_ky=float(rng.integers(0, 2)), gust_kz=float(rng.integers(0, 2)),
               gust_phase=float(rng.uniform(0, 2 * math.pi)))
    return Scene(name=f"flag_leaves{res}_n{n}", grid=grid, x=x, mass=rho * vol0, vol0=vol0,
                 region=region, E=E, nu=nu, pin=pin, dt=dt, gravity=(0.0, -9.8, 0.0),
                 material=FIXED_COROTATED, lattice=lattice, lbm=lbm,
                 wind=dict(mode="lbm", vel_scale=1.0 / 0.08, k_drag=9.8), seed=seed)


def smooth_force_field(seed: int, K: int = 8, nw: int = 16, amp: float = 5.0, modes: int = 4,
                       perturb: float = 0.0, perturb_seed: int | None = None):
    """Smooth seeded wind-force field W (K, 3, nw^3), a sum of low-frequency
    cosine modes per slot and component; ``perturb`` adds a relative seeded
    perturbation of the same kind (used to make a target rollout)."""
    def field(rng):
        g = np.linspace(0.0, 1.0, nw)
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        W = np.zeros((K, 3, nw, nw, nw))
        for s in range(K):
            for c in range(3):
                for _ in range(modes):
                    kx, ky, kz = rng.integers(0, 3, 3)
                    ph = rng.uniform(0, 2 * math.pi, 3)
                    a = rng.normal() / modes
                    W[s, c] += a * (np.cos(math.pi * kx * X + ph[0]) * np.cos(math.pi * ky * Y + ph[1])
                                    * np.cos(math.pi * kz * Z + ph[2]))
        return W
    W = amp * field(np.random.Generator(np.random.PCG64(seed)))
    if perturb:
        ps = seed + 1 if perturb_seed is None else perturb_seed
        W = W + perturb * amp * field(np.random.Generator(np.random.PCG64(ps)))
    return W.reshape(K, 3, nw ** 3)


def random_particles_in_box(seed: int, n: int, lo, hi):
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, 3))


def random_state(seed: int, n: int, scale_v: float = 0.1, scale_c: float = 1.0,
                 scale_f: float = 0.05):
    """Seeded non-trivial particle state: velocities, affine matrices and
    deformation gradients near identity (det F > 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = scale_v * rng.standard_normal((n, 3))
    C = scale_c * rng.standard_normal((n, 3, 3))
    F = np.eye(3)[None] + scale_f * rng.standard_normal((n, 3, 3))
    return v, C, F


def wind_tunnel_obstacles(seed: int, dims=(64, 64, 64)):
    """Surrogate-training lattice: inflow speed uniform in [0.02, 0.1] along +x and
    1-4 random obstacle boxes with sides of 4-16 cells; returns (u_in, solid
    (nz, ny, nx) bool, bc)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    u = float(rng.uniform(0.02, 0.1))
    solid = np.zeros((nz, ny, nx), dtype=bool)
    for _ in range(int(rng.integers(1, 5))):
        s = rng.integers(4, 17, 3)
        o = np.array([rng.integers(8, nx - 8 - s[0]), rng.integers(2, ny - 2 - s[1]),
                      rng.integers(2, nz - 2 - s[2])])
        solid[o[2]:o[2] + s[2], o[1]:o[1] + s[1], o[0]:o[0] + s[0]] = True
    bc = (BC_INLET, BC_OUTLET, BC_BOUNCEBACK, BC_BOUNCEBACK, BC_BOUNCEBACK, BC_BOUNCEBACK)
    return u, solid, bc


@dataclass
class GaussianCloud:
    """Inputs of the renderer: n kernels in the [3][n] / [6][n] layouts of
    the C header (float64 here) and one view."""
    mu: np.ndarray        # (3, n)
    sigma: np.ndarray     # (6, n): xx, yy, zz, xy, xz, yz
    color: np.ndarray     # (3, n)
    opacity: np.ndarray   # (n,)
    camera: dict          # width, height, fx, fy, cx, cy, R (3x3), t (3), near


def _look_at(eye, target):
    """World-to-camera rotation whose camera z axis points from eye to target
    (camera y down, x right) and the matching translation."""
    eye, target = np.asarray(eye, float), np.asarray(target, float)
    z = target - eye
    z /= np.linalg.norm(z)
    up = np.array([0.0, 0.0, 1.0]) if abs(z[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    x = np.cross(z, -up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return R, -R @ eye


def look_at_camera(eye, target, width: int, height: int, focal: float, near: float = 0.05) -> dict:
    """A camera dict (the GaussianCloud.camera form) at `eye` looking at `target`."""
    R, t = _look_at(eye, target)
    return dict(width=width, height=height, fx=focal, fy=focal, cx=width / 2, cy=height / 2, R=R, t=t, near=near)


def particle_splats(sc: Scene, seed: int = 0):
    """Gaussian kernels for the particles of a scene: isotropic rest
    covariances of half the particle spacing (6, n), a colour per region
    with a little per-particle variation (3, n), opacity 0.8 (n,)."""
    rng = np.random.default_rng(seed + 7)
    n = sc.n
    s2 = (0.5 * float(sc.vol0.mean()) ** (1.0 / 3.0)) ** 2
    sigma0 = np.zeros((6, n))
    sigma0[:3] = s2
    base = rng.uniform(0.15, 0.95, (3, int(sc.region.max()) + 1))
    color = np.clip(base[:, sc.region] + rng.normal(0.0, 0.05, (3, n)), 0.0, 1.0)
    return sigma0, color, np.full(n, 0.8)


def random_gaussians(seed: int, n: int, width: int = 40, height: int = 36, depth=(1.5, 3.5), scale=0.05,
                     opacity=(0.2, 0.9), min_depth_gap: float = 1e-5) -> GaussianCloud:
    """n kernels spread over the view of a camera at the origin looking along
    +z (depths in `depth`, anisotropic covariances of size ~scale, random RGB
    and opacity).  Depths are stratified (one per slot of width
    (hi - lo) / n, jittered within the middle 60 % of the slot, in random
    order), so any two differ by at least 0.4 (hi - lo) / n and the
    front-to-back order does not depend on rounding."""
    rng = np.random.default_rng(seed)
    f = 1.2 * width
    lo, hi = depth
    z = lo + (hi - lo) * (np.arange(n) + 0.2 + 0.6 * rng.uniform(0, 1, n)) / max(n, 1)
    z = z[rng.permutation(n)]
    assert n < 2 or np.min(np.diff(np.sort(z))) >= min(min_depth_gap, 0.4 * (hi - lo) / n)
    u = rng.uniform(-0.1 * width, 1.1 * width, n)
    v = rng.uniform(-0.1 * height, 1.1 * height, n)
    x = (u - width / 2) * z / f
    y = (v - height / 2) * z / f
    A = rng.standard_normal((n, 3, 3)) * scale
    S = A @ A.transpose(0, 2, 1) + (0.1 * scale) ** 2 * np.eye(3)
    sigma = np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]])
    cam = dict(width=width, height=height, fx=f, fy=1.05 * f, cx=width / 2, cy=height / 2, R=np.eye(3),
               t=np.zeros(3), near=0.1)
    return GaussianCloud(np.stack([x, y, z]), sigma, rng.uniform(0, 1, (3, n)), rng.uniform(*opacity, n), cam)


def splat_scene(seed: int = 0, n_object: int = 500_000, n_background: int = 500_000, res: int = 128,
                width: int = 1024, height: int = 1024) -> GaussianCloud:
    """A splat scene shaped like the paper's captured ones (Tab. sim_time: an
    object of 52k-146k kernels inside 0.5-4.5M background kernels): the
    object kernels sit on the flag-and-leaves particles (isotropic, half the
    particle spacing), the background kernels on a thick shell around the
    simulation box (radii 1.2-2.0, larger, flattened along the shell
    normal); one camera outside the shell looking at the box centre."""
    rng = np.random.default_rng(seed + 101)
    sc = flag_and_leaves_scene(seed=seed, n=n_object, res=res, lbm_dims=(res, res // 2, res // 2))
    dx = sc.grid["dx"]
    centre = np.array(sc.grid["origin"]) + 0.5 * dx * np.array([sc.grid["nx"], sc.grid["ny"], sc.grid["nz"]])
    spacing = (sc.vol0.mean()) ** (1.0 / 3.0)
    mu_o = sc.x.T
    s_o = (0.5 * spacing) ** 2
    sig_o = np.zeros((6, n_object))
    sig_o[:3] = s_o
    d = rng.standard_normal((n_background, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(1.2, 2.0, n_background)
    mu_b = (centre + d * r[:, None]).T
    a = rng.uniform(0.01, 0.04, n_background)
    # covariance a^2 (I - 0.9 d d^T): flattened along the shell normal
    S = a[:, None, None] ** 2 * (np.eye(3)[None] - 0.9 * d[:, :, None] * d[:, None, :])
    sig_b = np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]])
    eye_dir = np.array([-0.45, -0.8, 0.25])
    eye = centre + 2.3 * eye_dir / np.linalg.norm(eye_dir)  # outside the shell
    R, t = _look_at(eye, centre)
    f = 1.1 * width
    cam = dict(width=width, height=height, fx=f, fy=f, cx=width / 2, cy=height / 2, R=R, t=t, near=0.05)
    col = np.concatenate([rng.uniform(0.2, 0.9, (3, n_object)), rng.uniform(0, 1, (3, n_background))], axis=1)
    op = np.concatenate([rng.uniform(0.5, 0.95, n_object), rng.uniform(0.1, 0.9, n_background)])
    return GaussianCloud(np.concatenate([mu_o, mu_b], axis=1), np.concatenate([sig_o, sig_b], axis=1), col, op, cam)
