"""The plain-method workload as specified, coupled end to end, against the
float64 oracle.

Workload: a 0.5 x 0.5 x 0.02 sheet of 20,000 particles pinned on its top
edge, 32^3 MPM grid (dx = 1/32), fixed-corotated E = 1e4, nu = 0.3, rho = 1,
dt = 1e-4, gravity, 100 substeps; the wind is the drag (Sec. 3.4) of a
D3Q19 BGK lattice-Boltzmann flow on a 32^3 lattice (tau = 0.6, uniform
inflow 0.05 along +x, outlet, bounce-back walls), into which the particles
are voxelized as solids every substep (Eq. point2voxel).  Each substep runs
voxelize -> LBM step -> sort -> P2G -> grid update with the drag -> G2P, on
the GPU through the library (the coupled driver, positions as reference plus
float32 displacement) and in the oracle in float64; the oracle takes the
voxel decision the way the float32 kernel takes it from the two position
parts.

Bar: every field within 1e-3 after 100 substeps -- the displacement
x(T) - x(0) relative to the oracle's |x(T) - x(0)|_inf, v, C, F - I
norm-wise, and the lattice velocity relative to the inflow speed."""
import pytest
import torch

from oracle import lbm as olbm
from oracle import mpm as ompm
from oracle import wind as owind
from paper_2603_09668_amd import scenes
from paper_2603_09668_amd.sim import CoupledSim

from gpu_util import EYE, f32, mat_from_dev, oracle_grid, rel, say, vec_from_dev

pytestmark = pytest.mark.gpu
STEPS = 100


def _oracle_coupled(sc, steps):
    """The coupled loop in float64: returns the final state dict and u."""
    og = oracle_grid(sc.grid)
    lt, lb = sc.lattice, sc.lbm
    olat = olbm.Lattice(lt["nx"], lt["ny"], lt["nz"], lt["dx"], lt["origin"])
    op = olbm.LBMParams(tau=lb["tau"], u_in=lb["u_in"], force=lb["force"], bc=lb["bc"], gust_amp=lb["gust_amp"],
                        gust_period=lb["gust_period"], gust_ky=lb["gust_ky"], gust_kz=lb["gust_kz"],
                        gust_phase=lb["gust_phase"])
    n = sc.n
    xref = f32(sc.x)
    st = {"x": xref.clone(), "v": torch.zeros(n, 3, dtype=torch.float64),
          "C": torch.zeros(n, 3, 3, dtype=torch.float64), "F": EYE.repeat(n, 1, 1)}
    mass, vol0 = f32(sc.mass), f32(sc.vol0)
    mu, lam = ompm.particle_mu_lam(f32(sc.E), f32(sc.nu), torch.as_tensor(sc.region).long())
    nx, ny, nz = olat.dims
    f = olbm.equilibrium(torch.ones(nz, ny, nx, dtype=torch.float64),
                         torch.tensor(lb["u_in"], dtype=torch.float64).view(3, 1, 1, 1).expand(3, nz, ny, nx))
    pin = torch.as_tensor(sc.pin)
    u = None
    for t in range(steps):
        # the voxel decision in float32 from the reference and the displacement
        solid = olbm.voxelize(olat, (st["x"] - xref).float(), x_ref=xref.float())
        f, _, u = olbm.lbm_step(olat, op, f, solid, t)
        acc = owind.lbm_drag_to_nodes(og, olat.dims, lt["dx"], lt["origin"], u.reshape(3, -1),
                                      sc.wind["vel_scale"], sc.wind["k_drag"])
        st, _ = ompm.substep(og, st, mass, vol0, mu, lam, sc.dt, sc.material, gravity=sc.gravity, acc=acc, pin=pin,
                             bound=sc.bound)
    return st, xref, u.reshape(3, -1)


def test_plain_method_coupled_100_substeps():
    sc = scenes.sheet_scene(seed=0, n=20_000)
    say(f"config-0 coupled rollout: GPU, {STEPS} substeps")
    sim = CoupledSim(sc, reorder=False)
    for _ in range(STEPS):
        sim.step()
    torch.cuda.synchronize()
    assert sim.status() == 0
    say("config-0 coupled rollout: oracle")
    o, xref, ou = _oracle_coupled(sc, STEPS)
    p = sim.p
    errs = {
        "disp": rel(vec_from_dev(p.x), o["x"] - xref),
        "v": rel(vec_from_dev(p.v), o["v"]),
        "C": rel(mat_from_dev(p.C), o["C"]),
        "F-I": rel(mat_from_dev(p.F), o["F"] - EYE),
        "u": (sim.u.double().cpu() - ou).abs().max().item() / abs(sc.lbm["u_in"][0]),
    }
    moved = (o["x"] - xref).abs().max().item()
    say(f"  largest oracle displacement {moved:.3e}; " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert moved > 1e-4  # the sheet did move under gravity and drag
    for k, e in errs.items():
        assert e < 1e-3, (k, e)
