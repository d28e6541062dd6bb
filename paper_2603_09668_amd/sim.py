"""Device-resident coupled simulation: one MPM substep driven by a D3Q19 LBM wind.

One coupled step runs, on torch's current stream:
  1. lbm_solid_from_particles  -- solid mask from the particles (Eq. point2voxel)
  2. lbm_step                  -- R fused stream-collide steps, velocity output
                                 (or lbm_home_step, the moment-encoded form)
  3. mpm_sort                  -- cell-tile grouping of the particles
  4. mpm_p2g                   -- Eq. P2G with the MLS stress term
  5. mpm_grid_update           -- gravity, LBM drag wind (Sec. 3.4), walls, pins
  6. mpm_g2p                   -- Eq. G2P, APIC C, Eq. deformation_update (in place)
Wind models (`wind`): "lbm" steps the lattice every substep; "surrogate"
replaces each block of k LBM steps by one call of the learned surrogate
(u_{t+k} from u_t, decided and, on a failed check, replaced by k plain LBM
steps on the device), the drag then using u_{t+k} for the k substeps of the
block; "frozen" keeps the wind field fixed (the method without a wind
update, the floor the surrogate must beat).

Particle positions are stored as a fixed reference (the scene's positions)
plus a float32 displacement (`p.xref`, `p.x`; see the header), unless
`position_reference=False` keeps absolute positions in `p.x`.
Steps 1-2 (the wind branch) and 3-4 (the particle branch) are independent
and can run side by side on two streams (`step(side)`, the default in a
captured graph).  All buffers are allocated once here; a step allocates
nothing, and every launch has a data-independent shape (persistent kernels read their work
counts from device memory), so a pair of substeps can be captured once in a
HIP graph and replayed: `capture()` / `replay()`.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class CoupledSim:
    def __init__(self, scene, device="cuda", lbm_steps_per_substep: int = 1, reorder: bool = True,
                 lbm_model: str = "bgk", relative_drag: bool = False, position_reference: bool = True,
                 wind: str = "lbm", surrogate=None, k: int = 8):
        self.scene = scene
        self.device = device
        self.R = int(lbm_steps_per_substep)
        g = scene.grid
        self.grid = api.make_grid(g["nx"], g["ny"], g["nz"], g["dx"], g["origin"])
        self.N = g["nx"] * g["ny"] * g["nz"]
        n = scene.n
        f32 = dict(dtype=torch.float32, device=device)
        x0 = torch.tensor(np.ascontiguousarray(scene.x.T), **f32)
        self.p = api.ParticleArrays(
            x=torch.zeros(3, n, **f32) if position_reference else x0,
            v=torch.zeros(3, n, **f32), C=torch.zeros(9, n, **f32), F=torch.zeros(9, n, **f32),
            mass=torch.tensor(scene.mass, **f32), vol0=torch.tensor(scene.vol0, **f32),
            region=torch.tensor(scene.region, dtype=torch.int32, device=device),
            E=torch.tensor(scene.E, **f32), nu=torch.tensor(scene.nu, **f32),
            xref=x0 if position_reference else None)
        self.ws = api.alloc_workspace(self.grid, n, device)
        self.gm = torch.zeros(self.N, **f32)
        self.gmv = torch.zeros(3, self.N, **f32)
        self.gv = torch.zeros(3, self.N, **f32)
        self.pin = torch.tensor(scene.pin, dtype=torch.uint8, device=device)
        self.prm = api.make_mpm_params(scene.dt, scene.gravity, scene.bound, scene.material)
        lat = scene.lattice
        self.lat = api.make_lattice(lat["nx"], lat["ny"], lat["nz"], lat["dx"], lat["origin"])
        self.L = lat["nx"] * lat["ny"] * lat["nz"]
        lb = scene.lbm
        self.lbm_kw = dict(tau=lb["tau"], u_in=lb["u_in"], force=lb["force"], bc=lb["bc"], gust_amp=lb["gust_amp"],
                           gust_period=lb["gust_period"], gust_ky=lb["gust_ky"], gust_kz=lb["gust_kz"],
                           gust_phase=lb["gust_phase"])
        self.t = 0
        # device step counters for the inlet gust, ping-ponged with the populations
        self.t_a = torch.zeros(1, dtype=torch.int32, device=device)
        self.t_b = torch.zeros(1, dtype=torch.int32, device=device)
        self.graph = None
        # lattice state, ping-ponged: 19 shifted populations (BGK) or the 10
        # moments of the HOME-LBM form
        if lbm_model not in ("bgk", "home"):
            raise ValueError(f"unknown lbm_model {lbm_model!r}")
        self.lbm_model = lbm_model
        nstate = 19 if lbm_model == "bgk" else api.HOME_MOMENTS
        self.fa = torch.empty(nstate, self.L, **f32)
        self.fb = torch.empty(nstate, self.L, **f32)
        init = api.lbm_equilibrium if lbm_model == "bgk" else api.lbm_home_equilibrium
        init(self.lat, api.make_lbm_params(**self.lbm_kw), self.fa)
        self.solid = torch.zeros(self.L, dtype=torch.uint8, device=device)
        self.u = torch.zeros(3, self.L, **f32)
        self.wind = api.wind_lbm_drag(self.lat, self.u, scene.wind["vel_scale"], scene.wind["k_drag"],
                                      relative=relative_drag)
        if wind not in ("lbm", "surrogate", "frozen"):
            raise ValueError(f"unknown wind model {wind!r}")
        self.wind_model = wind
        self.sw = None
        if wind == "surrogate":
            if surrogate is None or lbm_model != "bgk" or self.R != 1:
                raise ValueError("the surrogate wind needs a trained net, the BGK lattice and one LBM step per substep")
            from .surrogate import SurrogateWind
            self.k = int(k)
            self.sw = SurrogateWind(surrogate, self.lat, self.lbm_kw, self.solid, k=self.k, batch=1)
            self.scale = torch.tensor([float(np.linalg.norm(lb["u_in"]))], **f32)
        # order[i] = scene index of particle i
        self.order = torch.arange(n, dtype=torch.int32, device=device)
        if reorder:
            self.reorder()

    def in_scene_order(self, t):
        """A per-particle array (.., n) back in the scene's particle order."""
        out = torch.empty_like(t)
        out[..., self.order.long()] = t
        return out

    def reorder(self):
        """Store the particles in cell-tile order (memory layout only)."""
        self.sort()
        perm = torch.empty(self.p.n, dtype=torch.int32, device=self.device)
        self.p = api.mpm_reorder(self.grid, self.p, self.ws, perm_out=perm)
        self.order = self.order[perm.long()]

    # -------------------------------------------------------------- phases
    def positions(self):
        """Absolute particle positions (3, n), float64."""
        return self.p.positions()

    def voxelize(self):
        api.lbm_solid_from_particles(self.lat, self.p.x, self.solid, xref=self.p.xref)

    def lbm(self):
        if self.wind_model == "frozen":
            self.t += self.R
            return
        if self.wind_model == "surrogate":
            # one surrogate call per block of k steps, at the block's start
            if self.t % self.k == 0:
                u = self.u.view(1, 3, self.L)
                self.sw.advance_device(u, self.scale, u, t0=self.t)
            self.t += 1
            return
        for _ in range(self.R):
            prm = api.make_lbm_params(**self.lbm_kw, t_in=self.t_a, t_out=self.t_b)
            step = api.lbm_step if self.lbm_model == "bgk" else api.lbm_home_step
            step(self.lat, prm, self.fa, self.fb, self.solid, None, self.u)
            self.fa, self.fb = self.fb, self.fa
            self.t_a, self.t_b = self.t_b, self.t_a
            self.t += 1

    def sort(self):
        api.mpm_sort(self.grid, self.prm, self.p.x, self.ws, xref=self.p.xref)

    def p2g(self):
        api.mpm_p2g(self.grid, self.prm, self.p, self.gm, self.gmv, self.ws)

    def grid_update(self):
        api.mpm_grid_update(self.grid, self.prm, self.gm, self.gmv, self.wind, self.pin, self.gv, self.ws)

    def g2p(self):
        p = self.p
        api.mpm_g2p(self.grid, self.prm, self.gv, p, p.x, p.v, p.C, p.F)

    PHASES = ("voxelize", "lbm", "sort", "p2g", "grid_update", "g2p")

    def step(self, side=None):
        """One coupled substep on the current stream.  With a `side` stream the
        wind branch (voxelize, LBM) runs on it beside the particle branch
        (sort, P2G): the two touch disjoint buffers and both read only the
        positions the previous G2P wrote; the grid update waits for both."""
        if side is None:
            for ph in self.PHASES:
                getattr(self, ph)()
            return
        main = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(main)
        side.wait_event(fork)
        # the particle branch is issued first: in a graph replay the branch
        # recorded first stays on the launch queue, whose dependent kernels
        # start back to back, and the shorter wind branch takes the other
        self.sort()
        self.p2g()
        with torch.cuda.stream(side):
            self.voxelize()
            self.lbm()
        join = torch.cuda.Event()
        join.record(side)
        main.wait_event(join)
        self.grid_update()
        self.g2p()

    def warm_wind(self, steps: int):
        """`steps` LBM steps around the particles at rest (solid mask from their
        positions), e.g. to start from a developed flow; the step index of
        the gust continues from there."""
        self.voxelize()
        model = self.wind_model
        self.wind_model = "lbm"
        for _ in range(steps):
            self.lbm()
        self.wind_model = model

    def capture(self, substeps: int = 2, concurrent: bool = True):
        """Record `substeps` coupled substeps (an even number of LBM steps, so
        the ping-pong buffers return to their roles) in one HIP graph; with
        `concurrent` the wind and particle branches are parallel graph
        branches."""
        if (substeps * self.R) % 2:
            raise ValueError("capture an even number of LBM steps")
        if self.wind_model != "lbm":
            raise ValueError("graph capture takes the LBM wind model (the others branch on the host step index)")
        t_host = self.t
        side = torch.cuda.Stream() if concurrent else None
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(substeps):
                self.step(side)
        self.t = t_host
        self.graph_substeps = substeps

    def replay(self):
        self.graph.replay()
        self.t += self.graph_substeps * self.R

    def status(self) -> int:
        return api.read_status(self.ws)

    def active_nodes(self) -> int:
        V = api.workspace_views(self.grid, self.p.n, self.ws)
        return int(V["n_node_tiles"]) * 64
