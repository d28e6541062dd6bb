"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/diffwind.h declares, its struct layouts match the ctypes
mirrors, and argument errors come back as codes (no GPU needed: every call
below fails validation before touching the device)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2603_09668_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diffwind.h")

pytestmark = pytest.mark.skipif(not os.path.exists(api.LIB_PATH), reason="libdiffwind.so not built")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return [n for n in names if n not in ("if", "while")]


def test_every_declared_symbol_is_exported():
    declared = _declared_functions()
    assert len(declared) >= 15
    L = ctypes.CDLL(api.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(declared) == sorted(api.SYMBOLS)


def test_struct_layout_matches_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "diffwind.h"
#define P(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  P(dw_grid) P(dw_lattice) P(dw_mpm_params) P(dw_particles) P(dw_particles_bar) P(dw_wind) P(dw_lbm_params)
  O(dw_wind, W) O(dw_wind, lat) O(dw_wind, u) O(dw_wind, acc) O(dw_particles, n_regions) O(dw_lbm_params, t)
  O(dw_lbm_params, bc) O(dw_mpm_params, deterministic) O(dw_particles, xref) O(dw_lbm_params, skip)
  O(dw_wind, deterministic) P(dw_camera) O(dw_camera, R) O(dw_camera, near_plane) O(dw_camera, alpha_min)
  O(dw_camera, t_min)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    mirror = {"dw_grid": api.Grid, "dw_lattice": api.Lattice, "dw_mpm_params": api.MPMParams,
              "dw_particles": api.Particles, "dw_particles_bar": api.ParticlesBar, "dw_wind": api.Wind,
              "dw_lbm_params": api.LBMParams, "dw_camera": api.Camera}
    for name, cls in mirror.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
    assert int(got["dw_wind.W"]) == api.Wind.W.offset
    assert int(got["dw_wind.lat"]) == api.Wind.lat.offset
    assert int(got["dw_wind.u"]) == api.Wind.u.offset
    assert int(got["dw_wind.acc"]) == api.Wind.acc.offset
    assert int(got["dw_particles.n_regions"]) == api.Particles.n_regions.offset
    assert int(got["dw_particles.xref"]) == api.Particles.xref.offset
    assert int(got["dw_lbm_params.skip"]) == api.LBMParams.skip.offset
    assert int(got["dw_wind.deterministic"]) == api.Wind.deterministic.offset
    assert int(got["dw_lbm_params.t"]) == api.LBMParams.t.offset
    assert int(got["dw_lbm_params.bc"]) == api.LBMParams.bc.offset
    assert int(got["dw_mpm_params.deterministic"]) == api.MPMParams.deterministic.offset
    for f in ("R", "near_plane", "alpha_min", "t_min"):
        assert int(got["dw_camera." + f]) == getattr(api.Camera, f).offset, f


def test_render_argument_errors_are_codes():
    """Camera, capacity and workspace checks of the renderer and the loss
    happen on the host before any launch (fake pointers, never read)."""
    L = api.lib()
    cam = api.make_camera(64, 48, 50.0, 50.0, 32.0, 24.0)
    nb = L.gs_render_workspace_bytes(100, ctypes.byref(cam), 1000)
    assert nb > 0 and L.gs_render_workspace_bytes(100, ctypes.byref(cam), 4000) > nb
    P = ctypes.c_void_p
    args = lambda c, n, pairs, ws_bytes: (ctypes.byref(c), n, P(256), P(512), P(768), P(1024), P(1280), pairs,
                                          P(4096), ws_bytes, None)
    assert L.gs_render(*args(cam, 100, 1000, nb - 1)) == -4
    assert "workspace too small" in api.dw_last_error()
    assert L.gs_render(*args(cam, -1, 1000, nb)) == -1
    bad = api.make_camera(0, 48, 50.0, 50.0, 32.0, 24.0)
    assert L.gs_render(*args(bad, 100, 1000, nb)) == -2
    bad = api.make_camera(64, 48, 50.0, 50.0, 32.0, 24.0, alpha_min=1.0)
    assert L.gs_render(*args(bad, 100, 1000, nb)) == -1 and "alpha_min" in api.dw_last_error()
    bad = api.make_camera(64, 48, 50.0, 50.0, 32.0, 24.0, t_min=-0.1)
    assert L.gs_render(*args(bad, 100, 1000, nb)) == -1
    assert L.gs_render(*args(cam, 100, 1 << 31, nb)) == -2
    lb = L.render_loss_workspace_bytes(3, 48, 64)
    assert lb > 0 and L.render_loss_workspace_bytes(0, 48, 64) == 0
    assert L.render_loss(3, 48, 64, P(256), P(512), ctypes.c_float(0.1), None, None, P(1024), lb - 1, None) == -4
    assert L.render_loss(3, 48, 64, P(256), P(512), ctypes.c_float(1.5), None, None, P(1024), lb, None) == -1


def test_field_stats_workspace_is_checked_on_the_host():
    """One partial triple per workgroup and field (at most 2048 workgroups,
    256 / nx rows each when nx < 256); a short workspace or a bad size is an
    error code before any launch (fake pointers, never read)."""
    L = api.lib()
    assert L.field_stats_workspace_bytes(1, 256, 128, 128) == 2048 * 12
    assert L.field_stats_workspace_bytes(2, 64, 8, 8) == 2 * 16 * 12      # 4 rows of 64 per workgroup
    assert L.field_stats_workspace_bytes(1, 100, 3, 3) == 5 * 12          # 2 rows of 100 per workgroup
    assert L.field_stats_workspace_bytes(0, 8, 8, 8) == 0
    nb = L.field_stats_workspace_bytes(3, 12, 10, 9)
    P = ctypes.c_void_p
    assert L.field_stats(3, 12, 10, 9, P(256), None, P(512), P(1024), nb - 1, None) == -4
    assert "workspace too small" in api.dw_last_error()
    assert L.field_stats(3, 12, 10, 9, P(256), None, P(512), None, nb, None) == -1
    assert L.field_stats(3, 0, 10, 9, P(256), None, P(512), P(1024), nb, None) == -1


def test_workspace_size_is_host_only_and_grows_with_n():
    g = api.make_grid(32, 32, 32, 1 / 32)
    a = api.mpm_workspace_bytes(g, 0)
    b = api.mpm_workspace_bytes(g, 1000)
    assert a > 0 and b >= a + 3 * 4 * 1000
    bad = api.make_grid(2, 32, 32, 1 / 32)
    assert api.mpm_workspace_bytes(bad, 10) == 0


def test_argument_errors_are_codes():
    L = api.lib()
    g = api.make_grid(16, 16, 16, 1 / 16)
    prm = api.make_mpm_params(1e-4)
    # null workspace
    rc = L.mpm_sort(ctypes.byref(g), ctypes.byref(prm), ctypes.c_void_p(16), None, 10, None, 0, None)
    assert rc == -1 and "workspace" in api.dw_last_error()
    # workspace too small (aligned fake pointer, never dereferenced)
    rc = L.mpm_sort(ctypes.byref(g), ctypes.byref(prm), ctypes.c_void_p(256), None, 10, ctypes.c_void_p(256), 8,
                    None)
    assert rc == -4
    bad = api.make_grid(16, 0, 16, 1 / 16)
    assert L.mpm_sort(ctypes.byref(bad), ctypes.byref(prm), None, None, 0, ctypes.c_void_p(256), 1 << 20,
                      None) == -1
    lat = api.make_lattice(8, 8, 8)
    lp = api.make_lbm_params(0.5)  # tau must exceed 1/2
    assert L.lbm_step(ctypes.byref(lat), ctypes.byref(lp), ctypes.c_void_p(256), ctypes.c_void_p(512), None, None,
                      None, None) == -1
    lp = api.make_lbm_params(0.6, bc=(api.BC_PERIODIC, api.BC_BOUNCEBACK, 0, 0, 0, 0))
    assert L.lbm_step(ctypes.byref(lat), ctypes.byref(lp), ctypes.c_void_p(256), ctypes.c_void_p(512), None, None,
                      None, None) == -1
    assert "periodic" in api.dw_last_error()
    lp = api.make_lbm_params(0.6)
    assert L.lbm_step(ctypes.byref(lat), ctypes.byref(lp), ctypes.c_void_p(256), ctypes.c_void_p(256), None, None,
                      None, None) == -1
    w = api.Wind(mode=7)
    assert L.wind_to_grid(ctypes.byref(g), ctypes.byref(w), ctypes.c_void_p(256), None) == -1
    # the allocation-free reverse step refuses lattices beyond its static buffer before any HIP call
    big = api.make_lattice(128, 64, 65)
    lp = api.make_lbm_params(0.6)
    assert L.lbm_step_adj_static(ctypes.byref(big), ctypes.byref(lp), ctypes.c_void_p(256), None,
                                 ctypes.c_void_p(512), None, ctypes.c_void_p(768), None) == -2
    assert "static work buffer" in api.dw_last_error()
