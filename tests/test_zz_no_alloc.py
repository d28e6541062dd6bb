"""lbm_step_adj_static, the reverse BGK step for callers that cannot
allocate (its work buffer is the library's static device array), against
lbm_step_adj with a caller-provided work buffer, through the C ABI.

Both run the same kernels without atomics, so the results must agree bit for
bit; two calls in a row, the second on a smaller lattice, check that nothing
of the first call's contents in the shared array leaks into the second."""
import numpy as np
import pytest
import torch

from paper_2603_09668_amd import api

from gpu_util import DEV, say

pytestmark = pytest.mark.gpu


def _inputs(dims, seed, bc, solid_box):
    nx, ny, nz = dims
    L = nx * ny * nz
    rng = np.random.default_rng(seed)
    f_in = torch.tensor(0.01 * rng.standard_normal((19, L)), dtype=torch.float32, device=DEV)
    solid = torch.zeros(nz, ny, nx, dtype=torch.uint8)
    if solid_box is not None:
        solid[solid_box] = 1
    gbar = torch.tensor(rng.standard_normal((19, L)), dtype=torch.float32, device=DEV)
    ubar = torch.tensor(rng.standard_normal((3, L)), dtype=torch.float32, device=DEV)
    lat = api.make_lattice(nx, ny, nz)
    prm = api.make_lbm_params(0.6, (0.08, 0.0, 0.0), (1e-5, 0.0, 0.0), bc, 0.05, 120.0, 1.0, 0.0, 0.3, t=7)
    return lat, prm, f_in, solid.reshape(-1).to(DEV), gbar, ubar


CASES = [
    # the largest lattice the static buffer takes: the 128 x 64 x 64 tunnel with an obstacle
    ("tunnel_128x64x64", (128, 64, 64), (api.BC_INLET, api.BC_OUTLET) + (api.BC_BOUNCEBACK,) * 4,
     (slice(20, 40), slice(24, 40), slice(50, 70))),
    # then a smaller periodic box with solids on its faces
    ("periodic_40x24x20", (40, 24, 20), (api.BC_PERIODIC,) * 6, (slice(0, 3), slice(20, 24), slice(30, 40))),
]


def test_static_work_buffer_matches_caller_buffer():
    for name, dims, bc, box in CASES:
        say(f"lbm_step_adj_static {name}")
        lat, prm, f_in, solid, gbar, ubar = _inputs(dims, 3, bc, box)
        L = f_in.shape[1]
        ref = torch.full((19, L), 0.25, device=DEV)
        api.lbm_step_adj(lat, prm, f_in, solid, gbar, ubar, ref, work=torch.empty(19, L, device=DEV))
        out = torch.full((19, L), 0.25, device=DEV)
        api.lbm_step_adj_static(lat, prm, f_in, solid, gbar, ubar, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), name
        assert (ref - 0.25).abs().max().item() > 0  # the reverse step did add something


def test_static_rejects_oversized_lattice():
    say("lbm_step_adj_static oversized lattice")
    lat = api.make_lattice(128, 64, 65)
    prm = api.make_lbm_params(0.6)
    t = torch.zeros(19, 1, device=DEV)
    rc = api.lib().lbm_step_adj_static(api.ctypes.byref(lat), api.ctypes.byref(prm), api._ptr(t), None,
                                       api._ptr(t), None, api._ptr(t), None)
    assert rc == -2 and "static work buffer" in api.dw_last_error()
