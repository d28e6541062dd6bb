"""ctypes binding of libdiffwind.so: the entry points of include/diffwind.h, same names.

Argument marshalling only: every step runs in the HIP kernels of the
library.  Tensors are torch CUDA (HIP) tensors, float32 (int32 for region,
uint8 for masks), contiguous, in the structure-of-arrays layout of the
header: particle vectors (3, n), matrices (9, n) with M_ab at row 3a+b (the
deformation gradient stored as F - I), grid
vectors (3, N), LBM populations (19, L) stored as f_i - w_i.  Calls are
enqueued on torch's current stream.  A missing library raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int, c_size_t, c_void_p
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiffwind.so")

FIXED_COROTATED, NEO_HOOKEAN = 0, 1
BC_PERIODIC, BC_BOUNCEBACK, BC_INLET, BC_OUTLET = 0, 1, 2, 3
WIND_NONE, WIND_FORCE_GRID, WIND_LBM_DRAG, WIND_ACC, WIND_LBM_DRAG_REL = 0, 1, 2, 3, 4
STATUS_OUT_OF_GRID, STATUS_NONFINITE, STATUS_INVERTED, STATUS_RENDER_OVERFLOW = 1, 2, 4, 8

# exported symbols, in the order of include/diffwind.h
SYMBOLS = [
    "dw_last_error", "mpm_workspace_bytes", "mpm_sort", "mpm_p2g", "mpm_grid_update", "mpm_g2p", "mpm_reorder",
    "wind_to_grid", "mpm_p2g_adj", "mpm_grid_update_adj", "mpm_g2p_adj", "wind_to_grid_adj",
    "lbm_step", "lbm_step_adj", "lbm_step_adj_static", "lbm_equilibrium", "lbm_home_step", "lbm_home_step_adj", "lbm_home_equilibrium",
    "lbm_solid_from_particles", "gaussian_covariance", "gaussian_covariance_adj",
    "gs_render_workspace_bytes", "gs_render", "gs_render_adj", "gs_render_status", "render_loss_workspace_bytes",
    "render_loss",
    "phys_loss", "position_loss", "direction_metrics", "wind_guide",
    "conv_packed_weight_elems", "conv_pack_weights", "conv_prep_input", "conv3d_bf16", "conv_wgrad_scratch_floats",
    "conv3d_bf16_wgrad", "conv_mse_grad", "adam_step", "field_stats_workspace_bytes", "field_stats", "field_accept", "field_select",
]
CONV_HIDDEN, CONV_OUTPUT, CONV_DGRAD = 0, 1, 2


class Grid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("dx", c_float), ("origin", c_float * 3)]


class Lattice(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("dx", c_float), ("origin", c_float * 3)]


class MPMParams(ctypes.Structure):
    _fields_ = [("dt", c_float), ("gravity", c_float * 3), ("bound", c_int), ("material", c_int),
                ("deterministic", c_int)]


class Particles(ctypes.Structure):
    _fields_ = [("n", c_int), ("x", c_void_p), ("v", c_void_p), ("C", c_void_p), ("F", c_void_p),
                ("mass", c_void_p), ("vol0", c_void_p), ("region", c_void_p), ("E", c_void_p),
                ("nu", c_void_p), ("n_regions", c_int), ("xref", c_void_p)]


class ParticlesBar(ctypes.Structure):
    _fields_ = [("n", c_int), ("x", c_void_p), ("v", c_void_p), ("C", c_void_p), ("F", c_void_p)]


class Wind(ctypes.Structure):
    _fields_ = [("mode", c_int), ("nw", c_int * 3), ("lo", c_float * 3), ("hi", c_float * 3),
                ("W", c_void_p), ("lat", Lattice), ("u", c_void_p), ("vel_scale", c_float),
                ("k_drag", c_float), ("acc", c_void_p), ("deterministic", c_int)]


class LBMParams(ctypes.Structure):
    _fields_ = [("tau", c_float), ("u_in", c_float * 3), ("force", c_float * 3), ("bc", c_int * 6),
                ("gust_amp", c_float), ("gust_period", c_float), ("gust_ky", c_float),
                ("gust_kz", c_float), ("gust_phase", c_float), ("t", c_int), ("t_in", c_void_p),
                ("t_out", c_void_p), ("skip", c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("R", c_float * 9), ("t", c_float * 3), ("near_plane", c_float),
                ("bg", c_float * 3), ("alpha_min", c_float), ("t_min", c_float)]


_lib = None


def lib():
    """Load libdiffwind.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_09668_amd.build` "
                           "or __graft_entry__.build(); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "dw_last_error": ([], ctypes.c_char_p),
        "mpm_workspace_bytes": ([POINTER(Grid), c_int, c_int], c_size_t),
        "mpm_sort": ([POINTER(Grid), POINTER(MPMParams), P, P, c_int, P, c_size_t, P], c_int),
        "mpm_p2g": ([POINTER(Grid), POINTER(MPMParams), POINTER(Particles), P, P, P, c_size_t, P], c_int),
        "mpm_grid_update": ([POINTER(Grid), POINTER(MPMParams), P, P, POINTER(Wind), P, P, P, c_size_t, P],
                            c_int),
        "mpm_g2p": ([POINTER(Grid), POINTER(MPMParams), P, POINTER(Particles), POINTER(Particles), P], c_int),
        "mpm_reorder": ([POINTER(Grid), POINTER(Particles), POINTER(Particles), P, P, c_size_t, P], c_int),
        "wind_to_grid": ([POINTER(Grid), POINTER(Wind), P, P], c_int),
        "mpm_p2g_adj": ([POINTER(Grid), POINTER(MPMParams), POINTER(Particles), P, P, POINTER(ParticlesBar), P,
                         P, c_size_t, P], c_int),
        "mpm_grid_update_adj": ([POINTER(Grid), POINTER(MPMParams), P, P, POINTER(Wind), P, P, P, P, P, P,
                                 c_size_t, P], c_int),
        "mpm_g2p_adj": ([POINTER(Grid), POINTER(MPMParams), P, POINTER(Particles), POINTER(ParticlesBar),
                         POINTER(ParticlesBar), P, P, c_size_t, P], c_int),
        "wind_to_grid_adj": ([POINTER(Grid), POINTER(Wind), P, P, P], c_int),
        "lbm_step": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P, P, P], c_int),
        "lbm_step_adj": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P, P, P, P], c_int),
        "lbm_step_adj_static": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P, P, P], c_int),
        "lbm_equilibrium": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P], c_int),
        "lbm_home_step": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P, P, P], c_int),
        "lbm_home_step_adj": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P, P, P, P], c_int),
        "lbm_home_equilibrium": ([POINTER(Lattice), POINTER(LBMParams), P, P, P, P], c_int),
        "lbm_solid_from_particles": ([POINTER(Lattice), P, P, c_int, P, c_int, P], c_int),
        "gaussian_covariance": ([c_int, P, P, P, P], c_int),
        "gaussian_covariance_adj": ([c_int, P, P, P, P, P, P], c_int),
        "gs_render_workspace_bytes": ([c_int, POINTER(Camera), ctypes.c_int64], c_size_t),
        "gs_render": ([POINTER(Camera), c_int, P, P, P, P, P, ctypes.c_int64, P, c_size_t, P], c_int),
        "gs_render_adj": ([POINTER(Camera), c_int, P, P, P, P, P, P, P, P, P, P, ctypes.c_int64, P, c_size_t, P],
                          c_int),
        "gs_render_status": ([P, P, P], c_int),
        "render_loss_workspace_bytes": ([c_int, c_int, c_int], c_size_t),
        "render_loss": ([c_int, c_int, c_int, P, P, c_float, P, P, P, c_size_t, P], c_int),
        "phys_loss": ([c_int, P, P, c_float, P, P, P], c_int),
        "position_loss": ([c_int, P, P, P, P, P], c_int),
        "direction_metrics": ([c_int, P, P, P, P], c_int),
        "wind_guide": ([POINTER(Lattice), P, POINTER(c_int), POINTER(c_float), POINTER(c_float), P, P], c_int),
        "conv_packed_weight_elems": ([c_int, c_int], c_size_t),
        "conv_pack_weights": ([P, c_int, c_int, c_int, P, P], c_int),
        "conv_prep_input": ([c_int, c_int, c_int, c_int, P, P, P, P], c_int),
        "conv3d_bf16": ([c_int, c_int, c_int, c_int, c_int, c_int, c_int, P, P, P, P, P, P, P, P, P, P], c_int),
        "conv_wgrad_scratch_floats": ([], c_size_t),
        "conv3d_bf16_wgrad": ([c_int, c_int, c_int, c_int, c_int, c_int, P, P, P, P, c_int, P, P], c_int),
        "conv_mse_grad": ([c_int, c_int, c_int, c_int, P, P, P, P, P, P], c_int),
        "adam_step": ([P, P, P, P, ctypes.c_int64, c_float, c_float, c_float, c_float, c_int, P], c_int),
        "field_stats_workspace_bytes": ([c_int, c_int, c_int, c_int], c_size_t),
        "field_stats": ([c_int, c_int, c_int, c_int, P, P, P, P, c_size_t, P], c_int),
        "field_accept": ([c_int, P, P, c_float, c_float, c_float, P, P, P], c_int),
        "field_select": ([c_int, c_int, c_int, c_int, P, P, P, P, P, P], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


class DiffWindError(RuntimeError):
    pass


def _check(rc: int, name: str):
    if rc != 0:
        msg = lib().dw_last_error().decode(errors="replace")
        raise DiffWindError(f"{name} returned {rc}: {msg}")


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=torch.float32, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return c_void_p(t.data_ptr())


def _shape(t, shape, name):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


# ----------------------------------------------------------------- structs

def make_grid(nx, ny, nz, dx, origin=(0.0, 0.0, 0.0)) -> Grid:
    return Grid(int(nx), int(ny), int(nz), float(dx), (c_float * 3)(*origin))


def make_lattice(nx, ny, nz, dx=1.0, origin=(0.0, 0.0, 0.0)) -> Lattice:
    return Lattice(int(nx), int(ny), int(nz), float(dx), (c_float * 3)(*origin))


def make_mpm_params(dt, gravity=(0.0, 0.0, 0.0), bound=3, material=FIXED_COROTATED, deterministic=False):
    return MPMParams(float(dt), (c_float * 3)(*gravity), int(bound), int(material), int(bool(deterministic)))


def make_lbm_params(tau, u_in=(0.0, 0.0, 0.0), force=(0.0, 0.0, 0.0), bc=(BC_PERIODIC,) * 6, gust_amp=0.0,
                    gust_period=1.0, gust_ky=0.0, gust_kz=0.0, gust_phase=0.0, t=0, t_in=None,
                    t_out=None, skip=None) -> LBMParams:
    """t_in / t_out: optional device int32 step counters; skip: optional
    device int32 flag that switches the call off (see the header)."""
    return LBMParams(float(tau), (c_float * 3)(*u_in), (c_float * 3)(*force), (c_int * 6)(*bc),
                     float(gust_amp), float(gust_period), float(gust_ky), float(gust_kz), float(gust_phase),
                     int(t), _ptr(t_in, torch.int32, "t_in"), _ptr(t_out, torch.int32, "t_out"),
                     _ptr(skip, torch.int32, "skip"))


def wind_none() -> Wind:
    return Wind(mode=WIND_NONE)


def wind_force_grid(W_slot, nw, lo, hi, deterministic: bool = False) -> Wind:
    """W_slot: (3, nw_z*nw_y*nw_x) device float32 (one time slot);
    deterministic: fixed-order transpose in wind_to_grid_adj."""
    w = Wind(mode=WIND_FORCE_GRID, deterministic=int(bool(deterministic)))
    w.nw = (c_int * 3)(*nw)
    w.lo = (c_float * 3)(*lo)
    w.hi = (c_float * 3)(*hi)
    w.W = _ptr(W_slot, name="W")
    w._keep = W_slot
    return w


def wind_lbm_drag(lat: Lattice, u, vel_scale, k_drag, relative: bool = False, deterministic: bool = False) -> Wind:
    """LBM drag wind; relative=True takes the wind relative to the node
    velocity (evaluated by mpm_grid_update only); deterministic: fixed-order
    transpose in wind_to_grid_adj."""
    w = Wind(mode=WIND_LBM_DRAG_REL if relative else WIND_LBM_DRAG, deterministic=int(bool(deterministic)))
    w.lat = lat
    w.u = _ptr(u, name="u")
    w.vel_scale = float(vel_scale)
    w.k_drag = float(k_drag)
    w._keep = u
    return w


def wind_acc(acc) -> Wind:
    w = Wind(mode=WIND_ACC)
    w.acc = _ptr(acc, name="acc")
    w._keep = acc
    return w


@dataclass
class ParticleArrays:
    """Device particle state in the header's layout.  With `xref` set the
    positions are xref + x and `x` holds the displacement from xref."""

    x: torch.Tensor      # (3, n)
    v: torch.Tensor      # (3, n)
    C: torch.Tensor      # (9, n)
    F: torch.Tensor      # (9, n), F - I
    mass: torch.Tensor   # (n,)
    vol0: torch.Tensor   # (n,)
    region: torch.Tensor  # (n,) int32
    E: torch.Tensor      # (R,)
    nu: torch.Tensor     # (R,)
    xref: torch.Tensor | None = None  # (3, n) position reference, or None

    @property
    def n(self):
        return self.x.shape[1]

    def positions(self):
        """Absolute positions (3, n) as float64 (xref + x is exact there)."""
        if self.xref is None:
            return self.x.double()
        return self.xref.double() + self.x.double()

    def struct(self) -> Particles:
        return Particles(self.n, _ptr(self.x, name="x"), _ptr(self.v, name="v"), _ptr(self.C, name="C"),
                         _ptr(self.F, name="F"), _ptr(self.mass, name="mass"), _ptr(self.vol0, name="vol0"),
                         _ptr(self.region, torch.int32, "region"), _ptr(self.E, name="E"),
                         _ptr(self.nu, name="nu"), int(self.E.numel()), _ptr(self.xref, name="xref"))

    def with_state(self, x, v, C, F) -> "ParticleArrays":
        return ParticleArrays(x, v, C, F, self.mass, self.vol0, self.region, self.E, self.nu, self.xref)


def _bar_struct(n, x=None, v=None, C=None, F=None) -> ParticlesBar:
    return ParticlesBar(n, _ptr(x, name="x_bar"), _ptr(v, name="v_bar"), _ptr(C, name="C_bar"),
                        _ptr(F, name="F_bar"))


# ------------------------------------------------------------ entry points

def dw_last_error() -> str:
    return lib().dw_last_error().decode(errors="replace")


def mpm_workspace_bytes(grid: Grid, n_max: int, deterministic: bool = False) -> int:
    return int(lib().mpm_workspace_bytes(ctypes.byref(grid), int(n_max), int(bool(deterministic))))


def alloc_workspace(grid: Grid, n_max: int, device="cuda", deterministic: bool = False) -> torch.Tensor:
    nb = mpm_workspace_bytes(grid, n_max, deterministic)
    if nb == 0:
        raise DiffWindError(f"mpm_workspace_bytes failed: {dw_last_error()}")
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nb]


def read_status(ws: torch.Tensor) -> int:
    return int(ws[:4].view(torch.int32).item())


def mpm_sort(grid: Grid, params: MPMParams, x, ws, xref=None):
    """x (3, n): positions, or displacements from xref (3, n) when given."""
    if xref is not None:
        _shape(xref, tuple(x.shape), "xref")
    _check(lib().mpm_sort(ctypes.byref(grid), ctypes.byref(params), _ptr(x, name="x"), _ptr(xref, name="xref"),
                          int(x.shape[1]), _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream()), "mpm_sort")


def mpm_reorder(grid: Grid, p: ParticleArrays, ws, perm_out=None) -> ParticleArrays:
    """New particle arrays in the order of the last mpm_sort (see the header)."""
    out = ParticleArrays(torch.empty_like(p.x), torch.empty_like(p.v), torch.empty_like(p.C), torch.empty_like(p.F),
                         torch.empty_like(p.mass), torch.empty_like(p.vol0), torch.empty_like(p.region), p.E, p.nu,
                         None if p.xref is None else torch.empty_like(p.xref))
    pi, po = p.struct(), out.struct()
    _check(lib().mpm_reorder(ctypes.byref(grid), ctypes.byref(pi), ctypes.byref(po),
                             _ptr(perm_out, torch.int32, "perm_out"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
                             _stream()), "mpm_reorder")
    return out


def mpm_p2g(grid: Grid, params: MPMParams, p: ParticleArrays, grid_m, grid_mv, ws):
    ps = p.struct()
    _check(lib().mpm_p2g(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(ps), _ptr(grid_m, name="grid_m"),
                         _ptr(grid_mv, name="grid_mv"), _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream()),
           "mpm_p2g")


def mpm_grid_update(grid: Grid, params: MPMParams, grid_m, grid_mv, wind: Wind | None, pin, grid_v, ws):
    _check(lib().mpm_grid_update(ctypes.byref(grid), ctypes.byref(params), _ptr(grid_m, name="grid_m"),
                                 _ptr(grid_mv, name="grid_mv"), ctypes.byref(wind) if wind is not None else None,
                                 _ptr(pin, torch.uint8, "pin"), _ptr(grid_v, name="grid_v"),
                                 _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream()), "mpm_grid_update")


def mpm_g2p(grid: Grid, params: MPMParams, grid_v, p_in: ParticleArrays, x_out, v_out, C_out, F_out):
    n = p_in.n
    pin = Particles(n, _ptr(p_in.x, name="x"), None, None, _ptr(p_in.F, name="F"), None, None, None, None, None, 0,
                    _ptr(p_in.xref, name="xref"))
    pout = Particles(n, _ptr(x_out, name="x_out"), _ptr(v_out, name="v_out"), _ptr(C_out, name="C_out"),
                     _ptr(F_out, name="F_out"), None, None, None, None, None, 0)
    _check(lib().mpm_g2p(ctypes.byref(grid), ctypes.byref(params), _ptr(grid_v, name="grid_v"), ctypes.byref(pin),
                         ctypes.byref(pout), _stream()), "mpm_g2p")


def wind_to_grid(grid: Grid, wind: Wind, acc):
    _check(lib().wind_to_grid(ctypes.byref(grid), ctypes.byref(wind), _ptr(acc, name="acc"), _stream()),
           "wind_to_grid")


def mpm_p2g_adj(grid: Grid, params: MPMParams, p: ParticleArrays, grid_m_bar, grid_mv_bar, x_bar=None, v_bar=None,
                C_bar=None, F_bar=None, E_bar=None, ws=None):
    """ws: a deterministic workspace, needed for the fixed-order E_bar of
    params.deterministic."""
    ps = p.struct()
    bar = _bar_struct(p.n, x_bar, v_bar, C_bar, F_bar)
    _check(lib().mpm_p2g_adj(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(ps),
                             _ptr(grid_m_bar, name="grid_m_bar"), _ptr(grid_mv_bar, name="grid_mv_bar"),
                             ctypes.byref(bar), _ptr(E_bar, name="E_bar"), _ptr(ws, torch.uint8, "ws"),
                             0 if ws is None else ws.numel(), _stream()), "mpm_p2g_adj")


def mpm_grid_update_adj(grid: Grid, params: MPMParams, grid_m, grid_mv, wind: Wind | None, pin, grid_v_bar,
                        grid_m_bar, grid_mv_bar, acc_bar, ws):
    _check(lib().mpm_grid_update_adj(ctypes.byref(grid), ctypes.byref(params), _ptr(grid_m, name="grid_m"),
                                     _ptr(grid_mv, name="grid_mv"),
                                     ctypes.byref(wind) if wind is not None else None, _ptr(pin, torch.uint8, "pin"),
                                     _ptr(grid_v_bar, name="grid_v_bar"), _ptr(grid_m_bar, name="grid_m_bar"),
                                     _ptr(grid_mv_bar, name="grid_mv_bar"), _ptr(acc_bar, name="acc_bar"),
                                     _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream()), "mpm_grid_update_adj")


def mpm_g2p_adj(grid: Grid, params: MPMParams, grid_v, p_in: ParticleArrays, x_out_bar=None, v_out_bar=None,
                C_out_bar=None, F_out_bar=None, x_bar=None, F_bar=None, grid_v_bar=None, ws=None):
    n = p_in.n
    pin = Particles(n, _ptr(p_in.x, name="x"), None, None, _ptr(p_in.F, name="F"), None, None, None, None, None, 0,
                    _ptr(p_in.xref, name="xref"))
    ob = _bar_struct(n, x_out_bar, v_out_bar, C_out_bar, F_out_bar)
    ib = _bar_struct(n, x_bar, None, None, F_bar)
    _check(lib().mpm_g2p_adj(ctypes.byref(grid), ctypes.byref(params), _ptr(grid_v, name="grid_v"),
                             ctypes.byref(pin), ctypes.byref(ob), ctypes.byref(ib),
                             _ptr(grid_v_bar, name="grid_v_bar"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
                             _stream()), "mpm_g2p_adj")


def wind_to_grid_adj(grid: Grid, wind: Wind, acc_bar, out_bar):
    _check(lib().wind_to_grid_adj(ctypes.byref(grid), ctypes.byref(wind), _ptr(acc_bar, name="acc_bar"),
                                  _ptr(out_bar, name="out_bar"), _stream()), "wind_to_grid_adj")


def lbm_step(lat: Lattice, params: LBMParams, f_in, f_out, solid=None, rho_out=None, u_out=None):
    _check(lib().lbm_step(ctypes.byref(lat), ctypes.byref(params), _ptr(f_in, name="f_in"),
                          _ptr(f_out, name="f_out"), _ptr(solid, torch.uint8, "solid"),
                          _ptr(rho_out, name="rho_out"), _ptr(u_out, name="u_out"), _stream()), "lbm_step")


def lbm_step_adj(lat: Lattice, params: LBMParams, f_in, solid, f_out_bar, u_out_bar, f_in_bar, work=None):
    """`work`: float32 scratch of (19, L) on the device (allocated here when None)."""
    L = lat.nx * lat.ny * lat.nz
    for t, name in ((f_in, "f_in"), (f_out_bar, "f_out_bar"), (f_in_bar, "f_in_bar")):
        _shape(t, (19, L), name)
    if u_out_bar is not None:
        _shape(u_out_bar, (3, L), "u_out_bar")
    if solid is not None:
        _shape(solid, (L,), "solid")
    if work is None:
        work = torch.empty(19, L, dtype=torch.float32, device=f_in.device)
    _shape(work, (19, L), "work")
    _check(lib().lbm_step_adj(ctypes.byref(lat), ctypes.byref(params), _ptr(f_in, name="f_in"),
                              _ptr(solid, torch.uint8, "solid"), _ptr(f_out_bar, name="f_out_bar"),
                              _ptr(u_out_bar, name="u_out_bar"), _ptr(f_in_bar, name="f_in_bar"),
                              _ptr(work, name="work"), _stream()),
           "lbm_step_adj")


STATIC_ADJ_MAX_NODES = 1 << 19  # DW_STATIC_ADJ_MAX_NODES


def lbm_step_adj_static(lat: Lattice, params: LBMParams, f_in, solid, f_out_bar, u_out_bar, f_in_bar):
    """lbm_step_adj with the library's static work buffer (no allocation;
    lattices of at most STATIC_ADJ_MAX_NODES nodes; calls on one device must
    not overlap)."""
    L = lat.nx * lat.ny * lat.nz
    for t, name in ((f_in, "f_in"), (f_out_bar, "f_out_bar"), (f_in_bar, "f_in_bar")):
        _shape(t, (19, L), name)
    if u_out_bar is not None:
        _shape(u_out_bar, (3, L), "u_out_bar")
    if solid is not None:
        _shape(solid, (L,), "solid")
    _check(lib().lbm_step_adj_static(ctypes.byref(lat), ctypes.byref(params), _ptr(f_in, name="f_in"),
                                     _ptr(solid, torch.uint8, "solid"), _ptr(f_out_bar, name="f_out_bar"),
                                     _ptr(u_out_bar, name="u_out_bar"), _ptr(f_in_bar, name="f_in_bar"), _stream()),
           "lbm_step_adj_static")


def lbm_equilibrium(lat: Lattice, params: LBMParams, f, rho=None, u=None):
    _check(lib().lbm_equilibrium(ctypes.byref(lat), ctypes.byref(params), _ptr(rho, name="rho"), _ptr(u, name="u"),
                                 _ptr(f, name="f"), _stream()), "lbm_equilibrium")


def gaussian_covariance(H, sigma0, sigma):
    """sigma = F sigma0 F^T per particle; H [9][n] = F - I, sigma0 / sigma [6][n]."""
    n = H.shape[1]
    _shape(H, (9, n), "H")
    _shape(sigma0, (6, n), "sigma0")
    _shape(sigma, (6, n), "sigma")
    _check(lib().gaussian_covariance(n, _ptr(H, name="H"), _ptr(sigma0, name="sigma0"), _ptr(sigma, name="sigma"),
                                     _stream()), "gaussian_covariance")


def gaussian_covariance_adj(H, sigma0, sigma_bar, H_bar=None, sigma0_bar=None):
    n = H.shape[1]
    _shape(H, (9, n), "H")
    _shape(sigma0, (6, n), "sigma0")
    _shape(sigma_bar, (6, n), "sigma_bar")
    if H_bar is not None:
        _shape(H_bar, (9, n), "H_bar")
    if sigma0_bar is not None:
        _shape(sigma0_bar, (6, n), "sigma0_bar")
    _check(lib().gaussian_covariance_adj(n, _ptr(H, name="H"), _ptr(sigma0, name="sigma0"),
                                         _ptr(sigma_bar, name="sigma_bar"), _ptr(H_bar, name="H_bar"),
                                         _ptr(sigma0_bar, name="sigma0_bar"), _stream()), "gaussian_covariance_adj")


def make_camera(width, height, fx, fy, cx, cy, R=((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)),
                t=(0.0, 0.0, 0.0), near_plane=0.01, bg=(0.0, 0.0, 0.0), alpha_min=0.0, t_min=0.0) -> Camera:
    """A view: world-to-camera R (3x3, row-major) and t, pinhole intrinsics in pixels."""
    Rf = [float(v) for row in R for v in row]
    return Camera(int(width), int(height), float(fx), float(fy), float(cx), float(cy), (c_float * 9)(*Rf),
                  (c_float * 3)(*t), float(near_plane), (c_float * 3)(*bg), float(alpha_min), float(t_min))


class RenderWorkspace:
    """Device workspace of gs_render / gs_render_adj for n kernels, one
    camera size and at most max_pairs (kernel, tile) pairs."""

    def __init__(self, n: int, cam: Camera, max_pairs: int, device="cuda"):
        nbytes = lib().gs_render_workspace_bytes(int(n), ctypes.byref(cam), int(max_pairs))
        if nbytes == 0:
            raise DiffWindError("gs_render_workspace_bytes: invalid sizes")
        self.n, self.max_pairs, self.size = int(n), int(max_pairs), (cam.width, cam.height)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.status_buf = torch.zeros(2, dtype=torch.int32, device=device)

    def status(self):
        """(status bits, pair count) of the last gs_render on this workspace (synchronises)."""
        _check(lib().gs_render_status(_ptr(self.buf, torch.uint8, "ws"), _ptr(self.status_buf, torch.int32, "status"),
                                      _stream()), "gs_render_status")
        s = self.status_buf.tolist()
        return int(s[0]), int(s[1])


def _render_args(cam: Camera, mu, sigma, color, opacity, ws: RenderWorkspace):
    n = mu.shape[1]
    _shape(mu, (3, n), "mu")
    _shape(sigma, (6, n), "sigma")
    _shape(color, (3, n), "color")
    _shape(opacity, (n,), "opacity")
    if ws.n != n or ws.size != (cam.width, cam.height):
        raise DiffWindError("render workspace was sized for another kernel count or image size")
    return n


def gs_render(cam: Camera, mu, sigma, color, opacity, image, ws: RenderWorkspace, check: bool = True):
    """Writes image [3][H][W]; with check, raises if the pairs overflowed the workspace (synchronises)."""
    n = _render_args(cam, mu, sigma, color, opacity, ws)
    _shape(image, (3, cam.height, cam.width), "image")
    _check(lib().gs_render(ctypes.byref(cam), n, _ptr(mu, name="mu"), _ptr(sigma, name="sigma"),
                           _ptr(color, name="color"), _ptr(opacity, name="opacity"), _ptr(image, name="image"),
                           ws.max_pairs, _ptr(ws.buf, torch.uint8, "ws"), ws.buf.numel(), _stream()), "gs_render")
    if check:
        st, pairs = ws.status()
        if st & STATUS_RENDER_OVERFLOW:
            raise DiffWindError(f"gs_render: more than max_pairs={ws.max_pairs} (kernel, tile) pairs")
        return pairs
    return None


def gs_render_adj(cam: Camera, mu, sigma, color, opacity, image, image_bar, ws: RenderWorkspace, mu_bar=None,
                  sigma_bar=None, color_bar=None, opacity_bar=None):
    """Accumulates the gradients of gs_render (same arguments, same workspace) into the given outputs."""
    n = _render_args(cam, mu, sigma, color, opacity, ws)
    _shape(image, (3, cam.height, cam.width), "image")
    _shape(image_bar, (3, cam.height, cam.width), "image_bar")
    for t, shp, nm in ((mu_bar, (3, n), "mu_bar"), (sigma_bar, (6, n), "sigma_bar"), (color_bar, (3, n), "color_bar"),
                       (opacity_bar, (n,), "opacity_bar")):
        if t is not None:
            _shape(t, shp, nm)
    _check(lib().gs_render_adj(ctypes.byref(cam), n, _ptr(mu, name="mu"), _ptr(sigma, name="sigma"),
                               _ptr(color, name="color"), _ptr(opacity, name="opacity"), _ptr(image, name="image"),
                               _ptr(image_bar, name="image_bar"), _ptr(mu_bar, name="mu_bar"),
                               _ptr(sigma_bar, name="sigma_bar"), _ptr(color_bar, name="color_bar"),
                               _ptr(opacity_bar, name="opacity_bar"), ws.max_pairs, _ptr(ws.buf, torch.uint8, "ws"),
                               ws.buf.numel(), _stream()), "gs_render_adj")


def render_loss_workspace(C, H, W, device="cuda") -> torch.Tensor:
    nbytes = lib().render_loss_workspace_bytes(int(C), int(H), int(W))
    if nbytes == 0:
        raise DiffWindError("render_loss_workspace_bytes: invalid sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def render_loss(image, target, ws, lam=0.1, loss=None, image_bar=None):
    """Adds (1 - lam) L1 + lam (1 - SSIM) to loss[0] and its gradient to image_bar; image, target [C][H][W]."""
    C, H, W = image.shape
    _shape(target, (C, H, W), "target")
    if loss is not None:
        _shape(loss, (1,), "loss")
    if image_bar is not None:
        _shape(image_bar, (C, H, W), "image_bar")
    _check(lib().render_loss(C, H, W, _ptr(image, name="image"), _ptr(target, name="target"), float(lam),
                             _ptr(loss, name="loss"), _ptr(image_bar, name="image_bar"),
                             _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream()), "render_loss")


def phys_loss(W, guide, weight=1.0, loss=None, W_bar=None):
    """Adds weight * L_phys to loss[0] and its gradient to W_bar; W, guide [3][n]."""
    n = W.shape[1]
    _shape(W, (3, n), "W")
    _shape(guide, (3, n), "guide")
    if loss is not None:
        _shape(loss, (1,), "loss")
    if W_bar is not None:
        _shape(W_bar, (3, n), "W_bar")
    _check(lib().phys_loss(n, _ptr(W, name="W"), _ptr(guide, name="guide"), float(weight), _ptr(loss, name="loss"),
                           _ptr(W_bar, name="W_bar"), _stream()), "phys_loss")


def position_loss(x, x_target, loss=None, x_bar=None):
    n = x.shape[1]
    _shape(x, (3, n), "x")
    _shape(x_target, (3, n), "x_target")
    if loss is not None:
        _shape(loss, (1,), "loss")
    if x_bar is not None:
        _shape(x_bar, (3, n), "x_bar")
    _check(lib().position_loss(n, _ptr(x, name="x"), _ptr(x_target, name="x_target"), _ptr(loss, name="loss"),
                               _ptr(x_bar, name="x_bar"), _stream()), "position_loss")


def direction_metrics(F_ref, F, out):
    """Adds (sum cos, sum |a - b|^2, count) over non-zero locations to out[0..2]."""
    n = F.shape[1]
    _shape(F_ref, (3, n), "F_ref")
    _shape(F, (3, n), "F")
    _shape(out, (3,), "out")
    _check(lib().direction_metrics(n, _ptr(F_ref, name="F_ref"), _ptr(F, name="F"), _ptr(out, name="out"),
                                   _stream()), "direction_metrics")


def wind_guide(lat: Lattice, u, nw, lo, hi, guide):
    L = lat.nx * lat.ny * lat.nz
    _shape(u, (3, L), "u")
    _shape(guide, (3, nw[0] * nw[1] * nw[2]), "guide")
    _check(lib().wind_guide(ctypes.byref(lat), _ptr(u, name="u"), (c_int * 3)(*nw), (c_float * 3)(*lo),
                            (c_float * 3)(*hi), _ptr(guide, name="guide"), _stream()), "wind_guide")


HOME_MOMENTS = 10   # rho - 1, u (3), S (6: xx yy zz xy xz yz)


def lbm_home_step(lat: Lattice, params: LBMParams, m_in, m_out, solid=None, rho_out=None, u_out=None):
    """HOME-LBM step on moments m [10][L] (see the C header)."""
    _check(lib().lbm_home_step(ctypes.byref(lat), ctypes.byref(params), _ptr(m_in, name="m_in"),
                               _ptr(m_out, name="m_out"), _ptr(solid, torch.uint8, "solid"),
                               _ptr(rho_out, name="rho_out"), _ptr(u_out, name="u_out"), _stream()),
           "lbm_home_step")


def lbm_home_step_adj(lat: Lattice, params: LBMParams, m_in, solid, m_out_bar, u_out_bar, m_in_bar, work=None):
    """`work`: float32 scratch of (19, L) on the device (allocated here when None)."""
    L = lat.nx * lat.ny * lat.nz
    if work is None:
        work = torch.empty(19, L, dtype=torch.float32, device=m_in.device)
    _shape(work, (19, L), "work")
    for t, shape, name in ((m_in, (HOME_MOMENTS, L), "m_in"), (m_out_bar, (HOME_MOMENTS, L), "m_out_bar"),
                           (m_in_bar, (HOME_MOMENTS, L), "m_in_bar")):
        _shape(t, shape, name)
    if u_out_bar is not None:
        _shape(u_out_bar, (3, L), "u_out_bar")
    if solid is not None:
        _shape(solid, (L,), "solid")
    _check(lib().lbm_home_step_adj(ctypes.byref(lat), ctypes.byref(params), _ptr(m_in, name="m_in"),
                                   _ptr(solid, torch.uint8, "solid"), _ptr(m_out_bar, name="m_out_bar"),
                                   _ptr(u_out_bar, name="u_out_bar"), _ptr(m_in_bar, name="m_in_bar"),
                                   _ptr(work, name="work"), _stream()),
           "lbm_home_step_adj")


def lbm_home_equilibrium(lat: Lattice, params: LBMParams, m, rho=None, u=None):
    _check(lib().lbm_home_equilibrium(ctypes.byref(lat), ctypes.byref(params), _ptr(rho, name="rho"),
                                      _ptr(u, name="u"), _ptr(m, name="m"), _stream()), "lbm_home_equilibrium")


def lbm_solid_from_particles(lat: Lattice, x, solid, accumulate=False, xref=None):
    """x (3, n): positions, or displacements from xref (3, n) when given."""
    if xref is not None:
        _shape(xref, tuple(x.shape), "xref")
    _check(lib().lbm_solid_from_particles(ctypes.byref(lat), _ptr(x, name="x"), _ptr(xref, name="xref"),
                                          int(x.shape[1]), _ptr(solid, torch.uint8, "solid"),
                                          int(bool(accumulate)), _stream()), "lbm_solid_from_particles")


WORK_CHUNK = 512  # particles per scatter work item (the library's constant)


def workspace_views(grid: Grid, n: int, ws: torch.Tensor) -> dict:
    """Read-only views of the sort results inside an MPM workspace (same layout
    as the library's): status, tile counts, tile ranges, active tile lists,
    keys and the permutation.  For inspection and tests."""
    tile = 4
    T = (-(-grid.nx // tile)) * (-(-grid.ny // tile)) * (-(-grid.nz // tile))
    NB = -(-T // 512)
    off = 0
    views = {}

    def take(name, count):
        nonlocal off
        views[name] = ws[off:off + 4 * count].view(torch.int32)
        off += (4 * count + 255) // 256 * 256

    take("header", 64)
    take("tile_count", T)
    take("node_flag", T)
    take("tile_start", T + 1)
    take("cell_tiles", T)
    take("node_tiles", T)
    take("block_sums", 4 * NB)
    take("key", n)
    take("rank", n)
    take("perm", n)
    take("perm_tmp", n)
    max_items = T + n // WORK_CHUNK + 1
    take("item_tile", max_items)
    take("item_begin", max_items)
    take("item_first", T)
    hdr = views["header"]
    views["status"] = hdr[0]
    views["n_sorted"] = hdr[3]
    views["n_node_tiles"] = hdr[4]
    views["n_cell_tiles"] = hdr[5]
    views["n_items"] = hdr[6]
    views["n_tiles"] = T
    return views


# ---------------------------------------------------------------- surrogate
# BF16 tensors are torch.bfloat16 on the Python side (uint16 storage in C).

def _bf(t, name):
    return _ptr(t, torch.bfloat16, name)


def conv_packed_weight_elems(cin: int, cout: int) -> int:
    return int(lib().conv_packed_weight_elems(int(cin), int(cout)))


def conv_pack_weights(w, cin, cout, flip, wk):
    _check(lib().conv_pack_weights(_ptr(w, name="w"), int(cin), int(cout), int(flip), _bf(wk, "wk"), _stream()),
           "conv_pack_weights")


def conv_prep_input(dims, u, scale, x0):
    B, nx, ny, nz = dims
    _check(lib().conv_prep_input(B, nx, ny, nz, _ptr(u, name="u"), _ptr(scale, name="scale"), _bf(x0, "x0"),
                                 _stream()), "conv_prep_input")


def conv3d_bf16(dims, cin, cout, epilogue, x, wk, bias=None, y=None, zpre=None, zgate=None, u=None, scale=None,
                u_out=None):
    B, nx, ny, nz = dims
    _check(lib().conv3d_bf16(B, nx, ny, nz, int(cin), int(cout), int(epilogue), _bf(x, "x"), _bf(wk, "wk"),
                             _ptr(bias, name="bias"), _bf(y, "y"), _bf(zpre, "zpre"), _bf(zgate, "zgate"),
                             _ptr(u, name="u"), _ptr(scale, name="scale"), _ptr(u_out, name="u_out"), _stream()),
           "conv3d_bf16")


def conv_wgrad_scratch_floats() -> int:
    return int(lib().conv_wgrad_scratch_floats())


def conv3d_bf16_wgrad(dims, cin, cout, x, dz, dw, db, scratch, accumulate=False):
    B, nx, ny, nz = dims
    _check(lib().conv3d_bf16_wgrad(B, nx, ny, nz, int(cin), int(cout), _bf(x, "x"), _bf(dz, "dz"),
                                   _ptr(dw, name="dw"), _ptr(db, name="db"), int(bool(accumulate)),
                                   _ptr(scratch, name="scratch"), _stream()), "conv3d_bf16_wgrad")


def conv_mse_grad(dims, u_out, u_tgt, scale, dy, loss_part):
    B, nx, ny, nz = dims
    _check(lib().conv_mse_grad(B, nx, ny, nz, _ptr(u_out, name="u_out"), _ptr(u_tgt, name="u_tgt"),
                               _ptr(scale, name="scale"), _bf(dy, "dy"), _ptr(loss_part, name="loss_part"),
                               _stream()), "conv_mse_grad")


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    _check(lib().adam_step(_ptr(p, name="p"), _ptr(g, name="g"), _ptr(m, name="m"), _ptr(v, name="v"), p.numel(),
                           float(lr), float(b1), float(b2), float(eps), int(step), _stream()), "adam_step")


def field_stats_workspace(dims, device="cuda") -> torch.Tensor:
    """Device workspace of field_stats for fields of these dims (B, nx, ny, nz)."""
    nbytes = lib().field_stats_workspace_bytes(*map(int, dims))
    if nbytes == 0:
        raise DiffWindError("field_stats_workspace_bytes: invalid sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def field_stats(dims, u, solid, out, ws=None):
    """out (B, 3) = the divergence and energy sums of the fields u (see the
    header); ws from field_stats_workspace (allocated here when None)."""
    B, nx, ny, nz = dims
    _shape(out, (B, 3), "out")
    if ws is None:
        ws = field_stats_workspace(dims, u.device)
    _check(lib().field_stats(B, nx, ny, nz, _ptr(u, name="u"), _ptr(solid, torch.uint8, "solid"),
                             _ptr(out, name="out"), _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream()),
           "field_stats")


def field_accept(stats_prev, stats_pred, accept, reject=None, div_factor=2.0, ke_band=(0.9, 1.1)):
    """accept[b] (int32) = the prediction passes the divergence and energy
    checks; reject = 1 - accept (see the header)."""
    B = accept.shape[0]
    _shape(stats_prev, (B, 3), "stats_prev")
    _shape(stats_pred, (B, 3), "stats_pred")
    _check(lib().field_accept(B, _ptr(stats_prev, name="stats_prev"), _ptr(stats_pred, name="stats_pred"),
                              float(div_factor), float(ke_band[0]), float(ke_band[1]),
                              _ptr(accept, torch.int32, "accept"), _ptr(reject, torch.int32, "reject"), _stream()),
           "field_accept")


def field_select(dims, accept, u_pred, u_alt, solid, u_out):
    B, nx, ny, nz = dims
    _check(lib().field_select(B, nx, ny, nz, _ptr(accept, torch.int32, "accept"), _ptr(u_pred, name="u_pred"),
                              _ptr(u_alt, name="u_alt"), _ptr(solid, torch.uint8, "solid"), _ptr(u_out, name="u_out"),
                              _stream()), "field_select")
