"""Throughput of the DiffWind simulation step on one MI355X.

A step is one coupled substep of the paper-scale forward workload, all on the
GPU with inputs resident in HBM: voxelize the particles into the LBM lattice,
one D3Q19 stream-collide, cell sort, P2G, grid update with the LBM drag wind,
G2P.  Workload: a 128^3 MPM grid with 500,000 float32 particles (one thin
flag sheet plus 40 ellipsoidal leaf clusters, E log-uniform in [1e3, 1e5]),
and a 128x64x64 D3Q19 lattice with inflow 0.08 and a 5 % seeded gust.

Prints one JSON line: particle-substeps/s for the whole step, the LBM MLUPS
of a standalone stream-collide loop, per-phase times from HIP events on the
launch stream, the roofline of the dominant kernel (and of every phase), a
measured device-copy bandwidth beside the 8 TB/s peak, the reverse LBM step,
the same coupled substep at the largest single-GPU size (4M particles, 256^3
grid, 256x128x128 lattice) and the float64 CPU oracle timed on a bounded
sample of the same workload (all host threads, one thread, the LBM alone).  The wind-surrogate
leg trains the BF16 conv net on 2000 LBM pairs of 64^3 wind tunnels (1800
train / 200 held out), then reports its held-out wind error against the LBM
and the speedup of one batched call over the 8 LBM steps it replaces.  The
adjoint leg times a 256-substep differentiable rollout (256k particles, 96^3,
checkpoints every 16) forward and backward, with a finite-difference check.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
METRIC = "particle-substeps/s, LBM MLUPS; surrogate-vs-LBM speedup at \u22642% wind error"


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--res", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-substeps", type=int, default=12)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-home", action="store_true", help="skip the HOME-LBM (moment-encoded) leg")
    ap.add_argument("--no-recon", action="store_true", help="skip the sequential reconstruction leg")
    ap.add_argument("--recon-only", action="store_true", help="run only the reconstruction leg (profiling)")
    ap.add_argument("--surrogate-only", action="store_true", help="run only the wind-surrogate leg (profiling)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--sg-rollouts", type=int, default=250)
    ap.add_argument("--sg-steps", type=int, default=1000)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-largest", action="store_true", help="skip the 4M-particle / 256^3 leg")
    ap.add_argument("--adjoint-only", action="store_true", help="run only the adjoint leg (profiling)")
    ap.add_argument("--fd", type=int, default=20, help="finite-difference coordinates in the adjoint leg")
    ap.add_argument("--no-render", action="store_true", help="skip the 3DGS rendering leg")
    ap.add_argument("--render-only", action="store_true", help="run only the rendering leg (profiling)")
    return ap.parse_args()


TRAFFIC_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
TRAFFIC_SOURCES = ("csrc/mpm.hip", "csrc/dw_scatter.h", "csrc/dw_internal.h", "csrc/dw_kernels.h", "csrc/lbm.hip")


def _measured_traffic(phase, n, res):
    """HBM bytes per launch of `phase` on this workload (n particles, res^3
    grid) from a committed FETCH_SIZE / WRITE_SIZE summary, if the kernel
    sources are the ones it was taken with; else None."""
    import glob
    import hashlib
    import re
    pkg = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2603_09668_amd")
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    pat = re.compile(r"^traffic %s n=%d res=%d bytes=(\d+) sha256=([0-9a-f]{64})$" % (phase, n, res), re.M)
    for path in sorted(glob.glob(os.path.join(TRAFFIC_DIR, "hbm_traffic_*.md"))):
        with open(path) as fh:
            m = pat.search(fh.read())
        if m and m.group(2) == h.hexdigest():
            return int(m.group(1))
    return None


def _graph_ms(fn, reps=5):
    """Average time of fn() captured in a HIP graph, by events on the stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    gph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gph):
        fn()
    gph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gph.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _phase_times(sim, R=10, reps=5):
    """Average launch time (ms) of every phase of a coupled substep: each
    phase alone, R launches in one HIP graph, timed with HIP events on the
    stream the kernels are launched on.  G2P runs out of place so that the
    state does not drift."""
    import torch
    from paper_2603_09668_amd import api
    scratch = [torch.empty_like(t) for t in (sim.p.x, sim.p.v, sim.p.C, sim.p.F)]

    def g2p_out_of_place():
        api.mpm_g2p(sim.grid, sim.prm, sim.gv, sim.p, *scratch)

    out = {}
    for ph in sim.PHASES:
        fn = g2p_out_of_place if ph == "g2p" else getattr(sim, ph)
        out[ph] = _graph_ms(lambda: [fn() for _ in range(R)], reps=reps) / R
    return out


def _phase_bytes(sim, active_nodes):
    """Algorithmic bytes per launch of each phase: what the method must move
    per unit of work (particle-substep 108 B read by P2G + 96 B written by
    G2P, 56 B per active grid node; LBM node 152 B + 1 B solid + 12 B u).
    The sort, the voxelisation, the position reference (12 B per particle
    wherever positions are read) and G2P's re-read of x and F are overheads
    of this implementation, counted in `_overhead_bytes`, not here."""
    n, L = sim.p.n, sim.L
    return {
        "p2g": 108 * n + 16 * active_nodes,               # read x v C F m V0 region; write m, mv
        "g2p": 96 * n + 12 * active_nodes,                # write x v C F; read grid v
        "lbm": 153 * L + 12 * L,                          # 19 pops in + out, solid, u out
        "grid_update": 29 * active_nodes,                 # read m mv pin, write v
    }


def _overhead_bytes(sim):
    """Bytes per launch beyond the algorithmic ones that each phase of this
    implementation necessarily moves (not counted in the rooflines)."""
    n, L = sim.p.n, sim.L
    ref = 12 * n if sim.p.xref is not None else 0
    return {
        "p2g": ref,                       # position reference
        "g2p": ref + 12 * n + 36 * n,     # position reference, displacement and F read back
        "sort": 2 * ref + 12 * n,         # positions read, key and rank written
        "voxelize": 2 * ref + L,          # positions read, solid flags written
    }


def _substep_rooflines(sim, active_nodes, ph_ms, ms_per_step):
    """The whole substep against its algorithmic bytes: the MPM part (204 B
    per particle + 56 B per active node) over the MPM phases' time (sort,
    P2G, grid update, G2P), and the coupled substep (+ the LBM node update)
    over the measured time per substep."""
    n, L = sim.p.n, sim.L
    mpm_b = 204 * n + 56 * active_nodes
    mpm_ms = sum(ph_ms[k] for k in ("sort", "p2g", "grid_update", "g2p"))
    cpl_b = mpm_b + 165 * L
    f = lambda b, ms: {"algorithmic_bytes": b, "ms": ms, "achieved_GBps": b / (ms * 1e-3) / 1e9,
                       "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return {"mpm": f(mpm_b, mpm_ms), "coupled": f(cpl_b, ms_per_step)}


def _rooflines(ph_ms, bytes_per):
    """Achieved algorithmic GB/s of every phase against the HBM peak."""
    out = {}
    for ph, ms in ph_ms.items():
        b = bytes_per.get(ph)
        if b and ms > 0:
            ach = b / (ms * 1e-3) / 1e9
            out[ph] = {"ms": ms, "algorithmic_bytes": b, "achieved_GBps": ach, "frac": ach / HBM_PEAK_GBS}
    return out


def _copy_bandwidth(mib=1024):
    """Device-to-device copy of `mib` MiB (torch copy_), GB/s of bytes read plus written."""
    import torch
    src = torch.ones(mib << 18, device="cuda")
    dst = torch.empty_like(src)
    ms = _graph_ms(lambda: dst.copy_(src), reps=10)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": 2 * (mib << 20) / (ms * 1e-3) / 1e9, "mib": mib, "ms": ms,
            "frac_of_peak": 2 * (mib << 20) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


_SCENES = {}


def _scene(n, res):
    """The flag-and-leaves scene of n particles on a res^3 grid (built once)."""
    from paper_2603_09668_amd import scenes
    key = (n, res)
    if key not in _SCENES:
        _SCENES[key] = scenes.flag_and_leaves_scene(seed=0, n=n, res=res, lbm_dims=(res, res // 2, res // 2))
    return _SCENES[key]


def _largest_leg(steps=20):
    """The largest single-GPU workload: 4M particles on a 256^3 grid with a
    256x128x128 lattice, the same coupled substep as the main line (HIP graph
    of two substeps, on one stream and with the wind and particle branches
    in parallel; the faster is reported), its phases and their rooflines."""
    import torch
    from paper_2603_09668_amd.sim import CoupledSim
    t0 = time.perf_counter()
    scene = _scene(4_000_000, 256)
    sim = CoupledSim(scene)
    t_setup = time.perf_counter() - t0
    for _ in range(4):
        sim.step()
    steps += steps % 2
    timed = {}
    for concurrent in (False, True):
        sim.capture(2, concurrent=concurrent)
        sim.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // 2):
            sim.replay()
        torch.cuda.synchronize()
        timed[concurrent] = time.perf_counter() - t0
    two_streams = timed[True] < timed[False]
    el = timed[two_streams]
    active = sim.active_nodes()
    ph = _phase_times(sim, R=4, reps=3)
    rl = _rooflines(ph, _phase_bytes(sim, active))
    for k in rl:
        rl[k]["traffic"] = _measured_traffic(k, scene.n, 256)
    ms = el * 1e3 / steps
    out = {"config": {"workload": "coupled MPM+LBM substep: 4000000 particles (flag sheet + 40 leaf clusters), "
                                  "256^3 MPM grid, 256x128x128 D3Q19 BGK lattice, LBM drag wind",
                      "particles": scene.n, "mpm_grid": 256, "lattice": [256, 128, 128], "dt": scene.dt,
                      "active_nodes": active, "graph": "two streams" if two_streams else "one stream"},
           "ms_per_step": ms, "value": scene.n / (ms * 1e-3), "unit": "particle-substeps/s", "steps": steps,
           "lbm_mlups": sim.L / (ph["lbm"] * 1e-3) / 1e6, "phase_ms": ph, "rooflines": rl,
           "overhead_bytes": _overhead_bytes(sim), "substep_rooflines": _substep_rooflines(sim, active, ph, ms),
           "status": sim.status(), "setup_s": t_setup}
    del sim
    torch.cuda.empty_cache()
    return out


def _lbm_adj_leg(sim):
    """The reverse BGK step (lbm_step_adj) on the scene's lattice and solids:
    228 algorithmic bytes per node (f_in and the output adjoint read, the
    input adjoint read and written; the work buffer's 76 B written and read
    again is overhead)."""
    import torch
    from paper_2603_09668_amd import api
    L = sim.L
    prm = api.make_lbm_params(**sim.lbm_kw, t=3)
    gb = torch.ones(19, L, device="cuda")
    fib = torch.zeros(19, L, device="cuda")
    work = torch.empty(19, L, device="cuda")
    ms = _graph_ms(lambda: api.lbm_step_adj(sim.lat, prm, sim.fa, sim.solid, gb, None, fib, work=work))
    b = (228 + 1) * L
    ach = b / (ms * 1e-3) / 1e9
    del gb, fib, work
    return {"ms": ms, "mlups": L / (ms * 1e-3) / 1e6, "algorithmic_bytes_per_node": 229, "achieved_GBps": ach,
            "frac": ach / HBM_PEAK_GBS}


def _home_leg(scene, sim, steps):
    """The HOME-LBM (moment-encoded) form of the lattice step: the step alone
    on the scene's lattice and solid mask, and the whole coupled substep with
    it in place of the BGK step."""
    import torch
    from paper_2603_09668_amd import api
    from paper_2603_09668_amd.sim import CoupledSim

    L = sim.L
    prm = api.make_lbm_params(**sim.lbm_kw, t=1)
    ma = torch.empty(api.HOME_MOMENTS, L, device="cuda")
    mb = torch.empty_like(ma)
    api.lbm_home_equilibrium(sim.lat, prm, ma)
    u = torch.empty(3, L, device="cuda")
    state = [ma, mb]

    def step():
        api.lbm_home_step(sim.lat, prm, state[0], state[1], sim.solid, None, u)
        state.reverse()

    R = 10
    ms = _graph_ms(lambda: [step() for _ in range(R)]) / R
    bytes_node = 2 * 4 * api.HOME_MOMENTS + 1 + 12      # moments in and out, solid, u out
    ach = bytes_node * L / (ms * 1e-3) / 1e9
    # the reverse step (per-population adjoints, then the transposed gather)
    mbar = torch.ones(api.HOME_MOMENTS, L, device="cuda")
    mib = torch.zeros_like(mbar)
    work = torch.empty(19, L, device="cuda")
    adj_ms = _graph_ms(lambda: api.lbm_home_step_adj(sim.lat, prm, ma, sim.solid, mbar, None, mib, work=work))
    del ma, mb, state, mbar, mib, work
    hs = CoupledSim(scene, lbm_model="home")
    for _ in range(4):
        hs.step()
    hs.capture(2)
    hs.replay()
    torch.cuda.synchronize()
    n2 = steps + (steps % 2)
    t0 = time.perf_counter()
    for _ in range(n2 // 2):
        hs.replay()
    torch.cuda.synchronize()
    sub_ms = (time.perf_counter() - t0) * 1e3 / n2
    return {"lbm_home_ms": ms, "lbm_home_mlups": L / (ms * 1e-3) / 1e6, "lbm_home_adj_ms": adj_ms,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_node": bytes_node},
            "coupled_ms_per_step": sub_ms, "coupled_value": scene.n / (sub_ms * 1e-3),
            "status": hs.status()}


def _recon_leg(n, res, frames, sub, iters):
    """Sequential reconstruction (Sec. 3.3) of a drag-shaped force field along
    the LBM wind of the scene's tunnel, from particle positions, with and
    without the physics-informed loss: CosSim / NMSE of the force directions
    per frame and the time of one optimisation iteration (forward, checkpointed
    backward, losses, Adam)."""
    import torch
    from paper_2603_09668_amd import recon, scenes
    sc = scenes.flag_and_leaves_scene(seed=3, n=n, res=res, lbm_dims=(res, res // 2, res // 2))
    dev = "cuda"
    nw, lo, hi = (16, 16, 16), (0.3, 0.2, 0.2), (0.95, 0.8, 0.8)
    guide, _ = recon.lbm_guide(sc, nw, lo, hi, steps=300)
    amp = 200.0
    F_gt = recon.drag_field(guide, amp)
    rc = recon.Reconstructor(sc, nw, lo, hi, substeps_per_frame=sub)
    state0 = rc.initial_state()  # positions as displacements from the scene's positions
    targets, st = [], state0
    for _ in range(frames):
        st = rc.advance(st, F_gt)
        targets.append(st[0].clone())
    out = {"config": {"workload": f"{n} particles, {res}^3 grid, 16^3 force grid, {frames} frames x {sub} substeps, "
                                  f"{iters} Adam iterations per frame (lr {amp / 40:g}), drag-shaped target field "
                                  f"along the LBM wind, largest force {amp:g}",
                      "particles": n, "grid": res, "frames": frames, "substeps_per_frame": sub,
                      "iterations": iters}}
    for lam in (0.0, 1.0):
        st = state0
        per = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(frames):
            r = rc.frame(st, targets[k], guide, lam=lam, iters=iters, lr=amp / 40)
            c, m, cnt = recon.metrics(F_gt, r.W)
            per.append({"cos_sim": c, "nmse": m, "nodes": cnt, "loss_first": r.loss[0], "loss_last": r.loss[-1]})
            st = rc.advance(st, r.W)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        err = torch.sqrt(((st[0] - targets[-1]) ** 2).sum(dim=0)).max().item()
        out[f"lambda_{lam:g}"] = {"frames": per, "ms_per_iteration": el * 1e3 / (frames * iters),
                                  "final_max_position_error": err}
    out["photometric"] = _recon_render(rc, sc, state0, F_gt, guide, frames, iters, amp)
    return out


def _recon_render(rc, sc, state0, F_gt, guide, frames, iters, amp):
    """The same reconstruction from rendered images (L_render of Sec. 3.3):
    the particles as Gaussian kernels (rest covariance of half the particle
    spacing, a colour per region, opacity 0.8) seen by two 512 x 512 views;
    the target images rendered from the reference rollout's states; L_render
    plus L_phys (lambda 1) per frame."""
    import torch
    from paper_2603_09668_amd import api, recon, scenes
    dev = "cuda"
    n = sc.n
    f = lambda a: torch.tensor(a, dtype=torch.float32, device=dev).contiguous()
    s0, col, op = (f(a) for a in scenes.particle_splats(sc))
    centre = np.array([0.6, 0.5, 0.5])
    cams = [scenes.look_at_camera(centre + np.array(d), centre, 512, 512, 700.0) for d in
            ((-0.3, -1.4, 0.3), (0.2, -0.6, -1.3))]
    cams = [api.make_camera(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"], R=c["R"].tolist(),
                            t=c["t"].tolist(), near_plane=c["near"], bg=(1.0, 1.0, 1.0), alpha_min=1.0 / 255.0,
                            t_min=1e-4) for c in cams]
    views = [recon.make_view(c, torch.empty(3, 512, 512, device=dev), n, 32 * n) for c in cams]
    st, targets = state0, []
    for _ in range(frames):
        st = rc.advance(st, F_gt)
        targets.append([recon.render_image(v, rc.xref + st[0], st[3], s0, col, op) for v in views])
    st = state0
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(frames):
        for v, img in zip(views, targets[k]):
            v.target = img
        r = rc.frame_render(st, views, s0, col, op, guide, lam=1.0, iters=iters, lr=amp / 40)
        c, m, cnt = recon.metrics(F_gt, r.W)
        per.append({"cos_sim": c, "nmse": m, "nodes": cnt, "loss_first": r.loss[0], "loss_last": r.loss[-1]})
        st = rc.advance(st, r.W)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"views": 2, "image": [512, 512], "lambda": 1.0, "frames": per,
            "ms_per_iteration": el * 1e3 / (frames * iters)}


def _surrogate_leg(n_rollouts, train_steps):
    """Train the wind surrogate on LBM pairs of 64^3 wind tunnels and compare
    it with the LBM on held-out fields: error and speed of a batch of 16."""
    import torch
    from paper_2603_09668_amd import api, scenes
    from paper_2603_09668_amd import surrogate as sg
    dims3 = (64, 64, 64)
    nx, ny, nz = dims3
    L = nx * ny * nz
    t0 = time.perf_counter()
    U0, U1, S, M = sg.lbm_pairs(n_rollouts, 8, dims=dims3, seed=0)
    n_train = (n_rollouts - n_rollouts // 10) * 8
    t_data = time.perf_counter() - t0
    print(f"[bench] surrogate data: {U0.shape[0]} pairs in {t_data:.1f} s", file=sys.stderr, flush=True)
    net = sg.Surrogate(seed=0)
    t0 = time.perf_counter()
    tr = (U0[:n_train], U1[:n_train], S[:n_train])
    sg.train(net, *tr, (16, *dims3), steps=int(train_steps * 0.7), batch=16, lr=1e-3, seed=0)
    sg.train(net, *tr, (16, *dims3), steps=train_steps - int(train_steps * 0.7), batch=16, lr=2e-4, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"[bench] surrogate trained: {train_steps} steps in {t_train:.1f} s", file=sys.stderr, flush=True)
    H0, H1, HS, HM = U0[n_train:], U1[n_train:], S[n_train:], M[n_train:]
    errs, errs_id, ok = [], [], []
    for i in range(0, H0.shape[0], 16):
        u0, u1, s_, m_ = H0[i:i + 16], H1[i:i + 16], HS[i:i + 16], M[n_train + i:n_train + i + 16]
        dims = (u0.shape[0], *dims3)
        out = torch.empty_like(u0)
        net.forward(u0, s_, out, dims)
        errs.append(sg.rel_error(out, u1, m_))
        errs_id.append(sg.rel_error(u0, u1, m_))
        ok.append(sg.check_fields(u0, out, dims, m_))
    e, e_id, ok = torch.cat(errs), torch.cat(errs_id), torch.cat(ok)
    # speed: one call on 16 fields against 16 x 8 LBM steps, both as HIP graphs
    B = 16
    ub, sb = U0[:B].contiguous(), S[:B].contiguous()
    ob = torch.empty_like(ub)
    t_sur = _graph_ms(lambda: net.forward(ub, sb, ob, (B, *dims3)))
    spd, solid_np, bc = scenes.wind_tunnel_obstacles(0, dims3)
    lat = api.make_lattice(nx, ny, nz)
    solid = torch.tensor(solid_np.reshape(-1), dtype=torch.uint8, device="cuda")
    kw = dict(tau=0.6, u_in=(spd, 0.0, 0.0), bc=bc)
    fa = torch.empty(19, L, device="cuda")
    fb = torch.empty_like(fa)
    uo = torch.empty(3, L, device="cuda")
    api.lbm_equilibrium(lat, api.make_lbm_params(**kw), fa)
    prms = [api.make_lbm_params(**kw, t=j + 1) for j in range(8)]

    def lbm_block():
        for _ in range(B):
            for j in range(8):
                api.lbm_step(lat, prms[j], fa if j % 2 == 0 else fb, fb if j % 2 == 0 else fa, solid, None,
                             uo if j == 7 else None)

    t_lbm = _graph_ms(lbm_block)
    flops = 120_960 * L * B
    tfl = flops / (t_sur * 1e-3) / 1e12
    step = _surrogate_step_timing(net)
    return {"speedup": step["speedup"], "wind_error_mean": e.mean().item(), "wind_error_max": e.max().item(),
            "persistence_error_mean": e_id.mean().item(), "persistence_error_max": e_id.max().item(),
            "accepted_by_checks": ok.float().mean().item(), "step_256x128x128": step,
            "forward_only_b16": {"ms_surrogate": t_sur, "ms_lbm_8steps": t_lbm, "ratio": t_lbm / t_sur},
            "roofline": {"bound": "mfma", "achieved": tfl, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tfl / BF16_PEAK_TFLOPS, "flop_per_voxel": 120_960},
            "_net": net,
            "config": {"workload": "64^3 wind tunnels with 1-4 obstacle boxes, inflow 0.02-0.1, tau 0.6; "
                                   "pairs (u_t, u_t+8), t in [200, 1000]; inference batch 16",
                       "pairs": int(U0.shape[0]), "train_pairs": n_train, "train_steps": train_steps,
                       "train_s": t_train, "data_s": t_data}}


def _surrogate_step_timing(net, dims3=(256, 128, 128), warm=800):
    """The whole surrogate step against the 8 LBM steps it replaces, on one
    lattice of the same node count as the largest workload's: prediction,
    divergence and energy checks, the device-side decision, the LBM fallback
    branch (switched off by the decision) and the output selection, captured
    in one HIP graph; the 8 BGK steps in another.  The flow is a developed
    tunnel flow around obstacle boxes (`warm` steps: the 256-long tunnel
    takes about four times the 64^3 tunnels' warm-up of 200 steps)."""
    import torch
    from paper_2603_09668_amd import api, scenes
    from paper_2603_09668_amd import surrogate as sg
    nx, ny, nz = dims3
    L = nx * ny * nz
    spd, solid_np, bc = scenes.wind_tunnel_obstacles(5, dims3)
    lat = api.make_lattice(nx, ny, nz)
    solid = torch.tensor(solid_np.reshape(-1), dtype=torch.uint8, device="cuda")
    kw = dict(tau=0.6, u_in=(spd, 0.0, 0.0), bc=bc)
    fa = torch.empty(19, L, device="cuda")
    fb = torch.empty_like(fa)
    u = torch.empty(1, 3, L, device="cuda")
    api.lbm_equilibrium(lat, api.make_lbm_params(**kw), fa)
    for t in range(1, warm + 1):
        api.lbm_step(lat, api.make_lbm_params(**kw, t=t), fa, fb, solid, None, u[0])
        fa, fb = fb, fa
    prms = [api.make_lbm_params(**kw, t=warm + j + 1) for j in range(8)]
    u8 = torch.empty(3, L, device="cuda")

    def lbm8():
        a, b = fa, fb
        for j in range(8):
            api.lbm_step(lat, prms[j], a, b, solid, None, u8 if j == 7 else None)
            a, b = b, a

    t_lbm = _graph_ms(lbm8, reps=10)
    sw = sg.SurrogateWind(net, lat, kw, solid, k=8, batch=1)
    scale = torch.tensor([spd], device="cuda")
    uo = torch.empty_like(u)
    t_step = _graph_ms(lambda: sw.advance_device(u, scale, uo, t0=warm), reps=10)
    t_fwd = _graph_ms(lambda: net.forward(u, scale, sw.u_pred, sw.dims), reps=10)
    accepted = int(sw.accept.item())
    err = sg.rel_error(uo, u8.view(1, 3, L), solid.view(1, -1)).item()
    err_id = sg.rel_error(u, u8.view(1, 3, L), solid.view(1, -1)).item()
    flops = 120_960 * L
    del fa, fb, u, uo, u8, sw
    torch.cuda.empty_cache()
    return {"lattice": list(dims3), "ms_surrogate_step": t_step, "ms_net_forward": t_fwd, "ms_lbm_8steps": t_lbm,
            "speedup": t_lbm / t_step, "accepted": accepted, "wind_error_vs_lbm": err,
            "persistence_error_vs_lbm": err_id,
            "roofline_net": {"bound": "mfma", "achieved": flops / (t_fwd * 1e-3) / 1e12, "peak": BF16_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": flops / (t_fwd * 1e-3) / 1e12 / BF16_PEAK_TFLOPS}}


def _tune_surrogate(net, n, res, warm, pairs=100, steps=300):
    """A copy of the net fine-tuned on the tunnel of the largest workload
    built from another seed (other particles, another gust): pairs
    (u_t, u_t+8) of its LBM flow around the particles at rest, t from
    `warm` on, `steps` Adam steps at batch 1, lr 2e-4.  Returns the net and
    the time the data and the training took."""
    import torch
    from paper_2603_09668_amd import surrogate as sg
    from paper_2603_09668_amd.sim import CoupledSim
    t0 = time.perf_counter()
    sc = scenes_mod().flag_and_leaves_scene(seed=1, n=n, res=res, lbm_dims=(res, res // 2, res // 2))
    sim = CoupledSim(sc, wind="lbm")
    sim.warm_wind(warm)
    U0 = torch.empty(pairs, 3, sim.L, device="cuda")
    U1 = torch.empty_like(U0)
    for i in range(pairs):
        U0[i].copy_(sim.u)
        sim.warm_wind(8)
        U1[i].copy_(sim.u)
    s = float(np.linalg.norm(sc.lbm["u_in"]))
    S = torch.full((pairs,), s, device="cuda")
    dims = (1, res, res // 2, res // 2)
    del sim
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    tuned = sg.Surrogate(seed=0)
    tuned.load_state_dict(net.state_dict())
    t0 = time.perf_counter()
    sg.train(tuned, U0, U1, S, dims, steps=steps, batch=1, lr=2e-4, seed=2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del U0, U1
    torch.cuda.empty_cache()
    return tuned, {"pairs": pairs, "steps": steps, "data_s": t_data, "train_s": t_train,
                   "source": "tunnel of the seed-1 scene, LBM from the particles at rest"}


def scenes_mod():
    from paper_2603_09668_amd import scenes
    return scenes


def _surrogate_coupled_leg(net, n=4_000_000, res=256, substeps=500, warm=300):
    """The largest workload driven three ways for `substeps` coupled substeps
    from the same developed flow (`warm` LBM steps around the particles at
    rest): the LBM every substep (the reference), the surrogate replacing
    every block of 8 LBM steps (with its device-side checks and LBM
    fallback), and a frozen wind.  Reports each run's time per substep and,
    against the LBM-driven run, the final wind error over fluid nodes and the
    error of the particle displacements."""
    import torch
    from paper_2603_09668_amd.sim import CoupledSim
    scene = _scene(n, res)
    tuned, tune_info = _tune_surrogate(net, n, res, warm)
    nets = {"surrogate": net, "surrogate_tuned": tuned}
    res_ = {}
    for model in ("lbm", "surrogate", "surrogate_tuned", "frozen"):
        kind = "surrogate" if model.startswith("surrogate") else model
        sim = CoupledSim(scene, wind=kind, surrogate=nets.get(model))
        sim.warm_wind(warm)
        acc = torch.zeros(1, dtype=torch.int32, device="cuda")
        calls = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(substeps):
            if kind == "surrogate" and sim.t % sim.k == 0:
                calls += 1
                sim.step()
                acc += sim.sw.accept
            else:
                sim.step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res_[model] = {"ms_per_substep": el * 1e3 / substeps, "status": sim.status(),
                       "u": sim.u.clone(), "solid": sim.solid.clone(),
                       "disp": sim.in_scene_order(sim.p.x).clone()}
        if kind == "surrogate":
            res_[model]["surrogate_calls"] = calls
            res_[model]["accepted_calls"] = int(acc.item())
        del sim
        torch.cuda.empty_cache()
    # one surrogate application on this tunnel (t = warm .. warm + 8) against
    # the 8 LBM steps it replaces, for both nets, and persistence
    from paper_2603_09668_amd import surrogate as sg
    sim = CoupledSim(scene, wind="lbm")
    sim.warm_wind(warm)
    u0 = sim.u.clone().view(1, 3, -1)
    sim.warm_wind(8)
    u8 = sim.u.clone().view(1, 3, -1)
    sol = sim.solid.view(1, -1)
    lat = sim.lat
    scale = torch.tensor([float(np.linalg.norm(scene.lbm["u_in"]))], device="cuda")
    dims = (1, lat.nx, lat.ny, lat.nz)
    one_step = {"persistence": sg.rel_error(u0, u8, sol).item()}
    for name, nt in nets.items():
        out = torch.empty_like(u0)
        nt.forward(u0, scale, out, dims)
        one_step[name] = sg.rel_error(out, u8, sol).item()
    del sim
    torch.cuda.empty_cache()
    ref = res_["lbm"]
    fluid = (ref["solid"] == 0).float()[None]
    un = torch.sqrt(((ref["u"] ** 2) * fluid).sum()).item()
    dn = torch.linalg.vector_norm(ref["disp"]).item()
    out = {"config": {"workload": f"coupled substep, {n} particles, {res}^3 grid, {res}x{res // 2}x{res // 2} "
                                  f"lattice, {substeps} substeps from {warm} LBM warm-up steps",
                      "substeps": substeps, "warm_lbm_steps": warm},
           "tuning": tune_info, "one_step_wind_error": one_step}
    for model in ("lbm", "surrogate", "surrogate_tuned", "frozen"):
        r = res_[model]
        e = {"ms_per_substep": r["ms_per_substep"], "status": r["status"]}
        if model != "lbm":
            e["wind_error_vs_lbm"] = torch.sqrt((((r["u"] - ref["u"]) ** 2) * fluid).sum()).item() / un
            e["displacement_error_vs_lbm"] = torch.linalg.vector_norm(r["disp"] - ref["disp"]).item() / dn
        for k in ("surrogate_calls", "accepted_calls"):
            if k in r:
                e[k] = r[k]
        out[model] = e
    return out


def _adjoint_leg(n, res, n_sub, ckpt, n_fd):
    """Reconstruction-style gradient: a rollout of `n_sub` substeps driven by a
    16^3 x 8 wind force grid, loss = |x_T - x_target|^2 against a rollout
    under a perturbed field, gradient with respect to the force grid and the
    per-region E through the hand-written adjoints with checkpoints every
    `ckpt` substeps; timed forward and backward, and checked by central
    differences of the same GPU forward on `n_fd` seeded coordinates."""
    import numpy as np
    import torch
    from paper_2603_09668_amd import api, scenes
    from paper_2603_09668_amd.autograd import RolloutPlan, rollout
    sc = scenes.flag_and_leaves_scene(seed=3, n=n, res=res, lbm_dims=(res, res // 2, res // 2))
    dev = "cuda"
    f32 = dict(dtype=torch.float32, device=dev)
    x0 = torch.tensor(np.ascontiguousarray(sc.x.T), **f32)
    mass, vol0 = torch.tensor(sc.mass, **f32), torch.tensor(sc.vol0, **f32)
    region = torch.tensor(sc.region, dtype=torch.int32, device=dev)
    E0, nu = torch.tensor(sc.E, **f32), torch.tensor(sc.nu, **f32)
    pin = torch.tensor(sc.pin, dtype=torch.uint8, device=dev)
    K, nw = 8, 16
    plan = RolloutPlan(sc.grid, sc.n, mass, vol0, region, nu, pin, sc.dt, sc.gravity, sc.material, sc.bound,
                       (nw,) * 3, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), K, n_sub, ckpt, device=dev)
    # particles in the sort's order (memory layout only); positions as
    # displacements from the scene's positions
    api.mpm_sort(plan.grid, plan.prm, x0, plan.ws)
    pa = api.mpm_reorder(plan.grid, api.ParticleArrays(torch.zeros(3, sc.n, **f32), torch.zeros(3, sc.n, **f32),
                                                       torch.zeros(9, sc.n, **f32), torch.zeros(9, sc.n, **f32),
                                                       mass, vol0, region, E0, nu, xref=x0),
                         plan.ws)
    plan.mass, plan.vol0, plan.region, plan.xref = pa.mass, pa.vol0, pa.region, pa.xref
    x0 = pa.x
    z3, z9 = torch.zeros(3, sc.n, **f32), torch.zeros(9, sc.n, **f32)
    amp = 200.0
    Wt = torch.tensor(scenes.smooth_force_field(7, K=K, nw=nw, amp=amp, perturb=0.3), **f32)
    W0 = torch.tensor(scenes.smooth_force_field(7, K=K, nw=nw, amp=amp), **f32)
    with torch.no_grad():
        xt = rollout(plan, Wt, E0, x0, z3, z9, z9.clone())[0].clone()

    def loss_of(W, E):
        return ((rollout(plan, W, E, x0, z3, z9, z9.clone())[0] - xt) ** 2).sum()

    W = W0.clone().requires_grad_(True)
    E = E0.clone().requires_grad_(True)
    loss_of(W, E).backward()  # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    W.grad = None
    E.grad = None
    torch.cuda.synchronize()
    ev[0].record()
    L = loss_of(W, E)
    ev[1].record()
    L.backward()
    ev[2].record()
    torch.cuda.synchronize()
    t_fwd, t_bwd = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    gW = W.grad.detach().clone()
    # central differences on seeded coordinates of the force grid
    rng = np.random.default_rng(11)
    flat = gW.reshape(-1)
    top = torch.topk(flat.abs(), 200).indices.cpu().numpy()
    coords = rng.choice(top, n_fd, replace=False)
    errs = []
    with torch.no_grad():
        for c in coords:
            h = 0.05 * amp
            Wp, Wm = W0.clone().reshape(-1), W0.clone().reshape(-1)
            Wp[c] += h
            Wm[c] -= h
            fd = (loss_of(Wp.reshape(W0.shape), E0) - loss_of(Wm.reshape(W0.shape), E0)).item() / (2 * h)
            errs.append(abs(fd - flat[c].item()) / max(abs(fd), 1e-30))
    errs = np.array(errs) if errs else np.zeros(1)
    # reverse substep: the segment recompute (sort 24, P2G 120, G2P 156 B per
    # particle) plus the adjoints (G2P 252, P2G 312 B per particle)
    b_rev = 864 * sc.n
    ach = b_rev / (t_bwd * 1e-3 / n_sub) / 1e9
    return {"ms_forward": t_fwd, "ms_backward": t_bwd, "us_per_substep_forward": 1e3 * t_fwd / n_sub,
            "us_per_substep_backward": 1e3 * t_bwd / n_sub, "loss": L.item(),
            "roofline_backward": {"bound": "hbm", "algorithmic_bytes_per_particle": 864, "achieved_GBps": ach,
                                  "frac": ach / HBM_PEAK_GBS},
            "fd_check": {"coordinates": int(n_fd), "rel_err_median": float(np.median(errs)),
                         "rel_err_max": float(errs.max()), "step": "0.05 x field amplitude, float32 forward"},
            "config": {"workload": f"reconstruction gradient: {sc.n} particles, {res}^3 grid, {n_sub} substeps, "
                                   f"checkpoint every {ckpt}, 16^3 x 8 force grid and per-region E",
                       "particles": sc.n, "grid": res, "substeps": n_sub, "checkpoint_every": ckpt}}


def _render_leg(reps=5):
    """Differentiable rendering of the particles as Gaussian kernels (Sec. 3.3,
    Eq. rendering and L_render): the splat workload of the paper's timing
    table in shape (500k object kernels on the flag-and-leaves particles,
    500k background kernels around them, one 1024 x 1024 view, the usual
    truncations alpha_min = 1/255 and t_min = 1e-4).  Times the forward
    render and the loss plus reverse pass, each as a HIP graph."""
    import torch
    from paper_2603_09668_amd import api, scenes
    g = scenes.splat_scene(seed=0)
    c = g.camera
    cam = api.make_camera(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"], R=np.asarray(c["R"]).tolist(),
                          t=np.asarray(c["t"]).tolist(), near_plane=c["near"], alpha_min=1.0 / 255.0, t_min=1e-4)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda").contiguous()
    mu, sig, col, op = f(g.mu), f(g.sigma), f(g.color), f(g.opacity)
    n = mu.shape[1]
    ws = api.RenderWorkspace(n, cam, 24 * n)
    img = torch.empty(3, c["height"], c["width"], device="cuda")
    tgt = torch.empty_like(img)
    # target: the same kernels displaced by a small uniform shift
    pairs_t = api.gs_render(cam, mu + 0.002, sig, col, op, tgt, ws)
    pairs = api.gs_render(cam, mu, sig, col, op, img, ws)
    fwd_ms = _graph_ms(lambda: api.gs_render(cam, mu, sig, col, op, img, ws, check=False), reps)
    lws = api.render_loss_workspace(3, c["height"], c["width"])
    L = torch.zeros(1, device="cuda")
    ib = torch.zeros_like(img)
    bars = [torch.zeros(3, n, device="cuda"), torch.zeros(6, n, device="cuda"), torch.zeros(3, n, device="cuda"),
            torch.zeros(n, device="cuda")]

    def back():
        L.zero_()
        ib.zero_()
        api.render_loss(img, tgt, lws, 0.1, L, ib)
        api.gs_render_adj(cam, mu, sig, col, op, img, ib, ws, *bars)
    back()
    torch.cuda.synchronize()
    loss = float(L.item())
    bwd_ms = _graph_ms(back, reps)
    st, _ = ws.status()
    return {"config": {"workload": "3DGS render of 500000 object kernels (flag-and-leaves particles) and 500000 "
                                   "background kernels, one 1024x1024 view, alpha_min 1/255, t_min 1e-4",
                       "kernels": n, "width": c["width"], "height": c["height"]},
            "pairs": pairs, "pairs_target": pairs_t, "ms_forward": fwd_ms, "ms_loss_and_reverse": bwd_ms,
            "loss": loss, "status": st, "kernels_per_s_forward": n / (fwd_ms * 1e-3)}


def _cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _cpu_baseline(scene, substeps, substeps_1t=1, lbm_steps=4):
    """The float64 oracle on the host: `substeps` coupled substeps (voxelize,
    LBM step, drag wind, MPM substep) of the full scene with torch's threads,
    the same with one thread for `substeps_1t` substeps, and the LBM step
    alone on the scene's lattice (`lbm_steps` steps)."""
    import torch
    from oracle import lbm as olbm
    from oracle import mpm as ompm
    from oracle import wind as owind
    g = scene.grid
    og = ompm.Grid(g["nx"], g["ny"], g["nz"], g["dx"], tuple(g["origin"]))
    n = scene.n
    d = torch.float64
    mu, lam = ompm.particle_mu_lam(torch.tensor(scene.E), torch.tensor(scene.nu), torch.tensor(scene.region).long())
    lat = scene.lattice
    ol = olbm.Lattice(lat["nx"], lat["ny"], lat["nz"], lat["dx"], tuple(lat["origin"]))
    lb = scene.lbm
    op = olbm.LBMParams(tau=lb["tau"], u_in=lb["u_in"], bc=lb["bc"], gust_amp=lb["gust_amp"],
                        gust_period=lb["gust_period"], gust_ky=lb["gust_ky"], gust_kz=lb["gust_kz"],
                        gust_phase=lb["gust_phase"])
    u0 = torch.tensor(lb["u_in"], dtype=d).view(3, 1, 1, 1).expand(3, ol.nz, ol.ny, ol.nx)
    mass, vol0, pin = torch.tensor(scene.mass), torch.tensor(scene.vol0), torch.tensor(scene.pin)

    def run(k):
        st = {"x": torch.tensor(scene.x), "v": torch.zeros(n, 3, dtype=d), "C": torch.zeros(n, 3, 3, dtype=d),
              "F": torch.eye(3, dtype=d).repeat(n, 1, 1)}
        f = olbm.equilibrium(torch.ones(ol.nz, ol.ny, ol.nx, dtype=d), u0)
        t0 = time.perf_counter()
        for s in range(k):
            solid = olbm.voxelize(ol, st["x"])
            f, rho, u = olbm.lbm_step(ol, op, f, solid, s)
            acc = owind.lbm_drag_to_nodes(og, ol.dims, ol.dx, ol.origin, u.reshape(3, -1), scene.wind["vel_scale"],
                                          scene.wind["k_drag"])
            st, _ = ompm.substep(og, st, mass, vol0, mu, lam, scene.dt, scene.material, gravity=scene.gravity,
                                 acc=acc, pin=pin, bound=scene.bound)
        return time.perf_counter() - t0

    threads = torch.get_num_threads()
    el = run(substeps)
    torch.set_num_threads(1)
    try:
        el1 = run(substeps_1t)
    finally:
        torch.set_num_threads(threads)
    f = olbm.equilibrium(torch.ones(ol.nz, ol.ny, ol.nx, dtype=d), u0)
    solid = torch.zeros(ol.nz, ol.ny, ol.nx, dtype=torch.bool)
    t0 = time.perf_counter()
    for s in range(lbm_steps):
        f, _, _ = olbm.lbm_step(ol, op, f, solid, s)
    el_l = time.perf_counter() - t0
    return {"value": n * substeps / el, "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{substeps} coupled substeps (voxelize, LBM step, drag wind, MPM substep) of the full "
                      f"{n}-particle scene, float64, {el:.1f} s on {threads} threads",
            "one_thread": {"value": n * substeps_1t / el1, "unit": "particle-substeps/s",
                           "sample": f"{substeps_1t} coupled substeps, {el1:.1f} s"},
            "lbm_mlups": ol.n_nodes * lbm_steps / el_l / 1e6,
            "lbm_sample": f"{lbm_steps} BGK steps of the {ol.nx}x{ol.ny}x{ol.nz} lattice, {el_l:.1f} s",
            "os_cpu_count": os.cpu_count(), "cpu_model": _cpu_model(),
            "note": "CPU float64 oracle: a baseline, not the target"}


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {a.gpus} is not supported by this build "
              "(the multi-GPU decomposition is designed but not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_09668_amd import api, scenes
    from paper_2603_09668_amd.sim import CoupledSim

    if a.copy_mib > 0:
        src = torch.ones(a.copy_mib << 18, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.recon_only:
        print(json.dumps({"metric": METRIC, "reconstruction": _recon_leg(256_000, 96, 3, 128, 20)}), flush=True)
        return
    if a.adjoint_only:
        print(json.dumps({"metric": METRIC, "adjoint": _adjoint_leg(256_000, 96, 256, 16, a.fd)}), flush=True)
        return
    if a.render_only:
        print(json.dumps({"metric": METRIC, "render": _render_leg()}), flush=True)
        return
    if a.surrogate_only:
        sgo = _surrogate_leg(a.sg_rollouts, a.sg_steps)
        net = sgo.pop("_net")
        if not a.no_largest:
            sgo["coupled_largest"] = _surrogate_coupled_leg(net)
        print(json.dumps({"metric": METRIC, "surrogate": sgo}), flush=True)
        return

    scene = scenes.flag_and_leaves_scene(seed=0, n=a.n, res=a.res, lbm_dims=(a.res, a.res // 2, a.res // 2))
    sim = CoupledSim(scene)
    torch.cuda.synchronize()
    print(f"[bench] scene {scene.name}: n={scene.n} dt={scene.dt:.3e} lattice={sim.L}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        sim.step()
    torch.cuda.synchronize()
    if sim.status() != 0:
        print(f"[bench] status word {sim.status()} after warm-up", file=sys.stderr)
    # the whole step as a HIP graph of two substeps, replayed, captured both
    # on one stream and with the wind and particle branches on two streams;
    # the faster of the two is reported, both are printed
    steps = a.steps + (a.steps % 2)
    timed = {}
    for concurrent in (False, True):
        sim.capture(2, concurrent=concurrent)
        sim.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // 2):
            sim.replay()
        torch.cuda.synchronize()
        timed[concurrent] = time.perf_counter() - t0
    two_streams = timed[True] < timed[False]
    elapsed = timed[two_streams]
    a.steps = steps
    status = sim.status()
    active_nodes = sim.active_nodes()

    # per-phase launch times: each phase alone, R launches in one graph, timed
    # with HIP events on the stream the kernels are launched on
    phases = CoupledSim.PHASES
    ph_ms = _phase_times(sim)
    lbm_ms = ph_ms["lbm"]
    mlups = sim.L / (lbm_ms * 1e-3) / 1e6

    n = scene.n
    value = n * a.steps / elapsed
    # algorithmic bytes per launch
    bytes_per = _phase_bytes(sim, active_nodes)
    dominant = max(phases, key=lambda ph: ph_ms[ph])
    ach = bytes_per.get(dominant, 0) / (ph_ms[dominant] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed * 1e3 / a.steps,
        "ms_per_step_one_stream": timed[False] * 1e3 / a.steps,
        "ms_per_step_two_streams": timed[True] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"coupled MPM+LBM substep: {n} particles (flag sheet + 40 leaf clusters), "
                               f"{a.res}^3 MPM grid, {a.res}x{a.res // 2}x{a.res // 2} D3Q19 BGK lattice, "
                               "LBM drag wind, 1 LBM step per substep",
                   "particles": n, "mpm_grid": a.res, "lattice": [a.res, a.res // 2, a.res // 2],
                   "dt": scene.dt, "active_nodes": active_nodes,
                   "graph": "two streams" if two_streams else "one stream"},
        "lbm_mlups": mlups,
        "phase_ms": ph_ms,
        "phase_sum_ms": sum(ph_ms.values()),
        "status": status,
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": _measured_traffic(dominant, a.n, a.res),
                     "algorithmic_bytes": bytes_per.get(dominant)},
        "rooflines": {k: dict(v, traffic=_measured_traffic(k, a.n, a.res))
                      for k, v in _rooflines(ph_ms, bytes_per).items()},
        "overhead_bytes": _overhead_bytes(sim),
        "substep_rooflines": _substep_rooflines(sim, active_nodes, ph_ms, elapsed * 1e3 / a.steps),
    }
    out["lbm_adjoint"] = _lbm_adj_leg(sim)
    out["copy_bandwidth"] = _copy_bandwidth()
    # covariance of the Gaussian kernels bound to the particles (Sec. 3.2)
    sig0 = torch.zeros(6, sim.p.n, device="cuda")
    sig0[:3] = (0.3 * scene.grid["dx"]) ** 2
    sig = torch.empty_like(sig0)
    cov_ms = _graph_ms(lambda: [api.gaussian_covariance(sim.p.F, sig0, sig) for _ in range(10)]) / 10
    out["covariance"] = {"ms": cov_ms, "bytes_per_particle": 84,
                         "achieved_GBps": 84 * sim.p.n / (cov_ms * 1e-3) / 1e9}
    del sig0, sig
    if not a.no_home:
        out["home_lbm"] = _home_leg(scene, sim, min(a.steps, 100))
    if not a.no_largest:
        out["largest"] = _largest_leg()
    if not a.no_render:
        out["render"] = _render_leg()
    if not a.no_surrogate:
        del sim
        torch.cuda.empty_cache()
        sgo = _surrogate_leg(a.sg_rollouts, a.sg_steps)
        net = sgo.pop("_net")
        out["surrogate_speedup"] = sgo["speedup"]
        out["surrogate"] = sgo
        if not a.no_largest:
            out["surrogate"]["coupled_largest"] = _surrogate_coupled_leg(net)
        del net
    if not a.no_adjoint:
        out["adjoint"] = _adjoint_leg(256_000, 96, 256, 16, a.fd)
    if not a.no_recon:
        out["reconstruction"] = _recon_leg(256_000, 96, 3, 128, 20)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(scene, a.cpu_substeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
