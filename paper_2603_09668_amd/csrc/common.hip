// Error reporting, workspace layout and argument checks of libdiffwind.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <climits>

#include "dw_internal.h"
#include "dw_kernels.h"

namespace dw {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(DW_ELAUNCH, "%s: launch failed: %s", what, hipGetErrorString(e));
  return DW_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t workspace_layout(const dw_grid *g, int n_max, Workspace *ws, void *base, int deterministic) {
  GridDev d = make_grid(g);
  int64_t T = (int64_t)d.tx * d.ty * d.tz;
  int64_t NB = (T + SCAN_BLOCK - 1) / SCAN_BLOCK;
  size_t off = 0;
  char *b = (char *)base;
  auto take = [&](size_t bytes) {
    char *p = b ? b + off : nullptr;
    off += align256(bytes);
    return (int32_t *)p;
  };
  int32_t *hdr = take(256);
  // hdr[0] status; hdr[3..6] scan totals: sorted particles, active node tiles, active cell tiles, work
  // items; hdr[8..9] P2G work-item tickets
  ws->status = hdr;
  ws->n_node_tiles = hdr ? hdr + 4 : nullptr;
  ws->n_cell_tiles = hdr ? hdr + 5 : nullptr;
  ws->n_items = hdr ? hdr + 6 : nullptr;
  // header .. node_flag are cleared at the start of every sort
  ws->tile_count = take(sizeof(int32_t) * T);
  ws->node_flag = take(sizeof(int32_t) * T);
  ws->tile_start = take(sizeof(int32_t) * (T + 1));
  ws->cell_tiles = take(sizeof(int32_t) * T);
  ws->node_tiles = take(sizeof(int32_t) * T);
  ws->block_sums = take(sizeof(int32_t) * 4 * NB);
  ws->key = take(sizeof(int32_t) * (size_t)n_max);
  ws->rank = take(sizeof(int32_t) * (size_t)n_max);
  ws->perm = take(sizeof(int32_t) * (size_t)n_max);
  ws->perm_tmp = take(sizeof(int32_t) * (size_t)n_max);
  int64_t max_items = T + (int64_t)n_max / WORK_CHUNK + 1;
  ws->item_tile = take(sizeof(int32_t) * max_items);
  ws->item_begin = take(sizeof(int32_t) * max_items);
  ws->item_first = take(sizeof(int32_t) * T);
  // the deterministic scratch ends the layout, so the two sizes share a prefix
  ws->item_part = deterministic ? (float *)take(sizeof(float) * 4 * 216 * (size_t)max_items) : nullptr;
  ws->item_part_floats = deterministic ? 4 * 216 * max_items : 0;
  ws->n_tiles = T;
  ws->n_scan_blocks = NB;
  ws->bytes = off;
  return off;
}

int bind_workspace(const dw_grid *g, int n, const void *ws, size_t ws_bytes, Workspace *W, int deterministic) {
  DW_REQUIRE(ws, DW_EINVAL, "workspace is NULL");
  DW_REQUIRE(((uintptr_t)ws & 255) == 0, DW_EINVAL, "workspace must be 256-byte aligned");
  size_t need = workspace_layout(g, n, W, const_cast<void *>(ws), deterministic);
  DW_REQUIRE(ws_bytes >= need, DW_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return DW_OK;
}

int make_wind(const dw_wind *w, const dw_grid *g, WindDev *o) {
  *o = WindDev{};
  o->mode = DW_WIND_NONE;
  o->N = (int64_t)g->nx * g->ny * g->nz;
  if (!w) return DW_OK;
  o->mode = w->mode;
  switch (w->mode) {
    case DW_WIND_NONE:
      return DW_OK;
    case DW_WIND_ACC:
      DW_REQUIRE(w->acc, DW_EINVAL, "wind: DW_WIND_ACC needs acc");
      o->acc = w->acc;
      return DW_OK;
    case DW_WIND_FORCE_GRID:
      DW_REQUIRE(w->W, DW_EINVAL, "wind: DW_WIND_FORCE_GRID needs W");
      DW_REQUIRE(w->nw[0] >= 2 && w->nw[1] >= 2 && w->nw[2] >= 2, DW_EINVAL, "wind: nw must be >= 2 per axis");
      for (int a = 0; a < 3; ++a)
        DW_REQUIRE(w->hi[a] > w->lo[a], DW_EINVAL, "wind: force-grid box must have hi > lo");
      o->nwx = w->nw[0];
      o->nwy = w->nw[1];
      o->nwz = w->nw[2];
      o->lox = w->lo[0];
      o->loy = w->lo[1];
      o->loz = w->lo[2];
      o->sx = (float)(w->nw[0] - 1) / (w->hi[0] - w->lo[0]);
      o->sy = (float)(w->nw[1] - 1) / (w->hi[1] - w->lo[1]);
      o->sz = (float)(w->nw[2] - 1) / (w->hi[2] - w->lo[2]);
      o->W = w->W;
      o->nw3 = (int64_t)w->nw[0] * w->nw[1] * w->nw[2];
      return DW_OK;
    case DW_WIND_LBM_DRAG:
    case DW_WIND_LBM_DRAG_REL:
      DW_REQUIRE(w->u, DW_EINVAL, "wind: LBM drag needs u");
      DW_REQUIRE(w->lat.nx >= 2 && w->lat.ny >= 2 && w->lat.nz >= 2 && w->lat.dx > 0.f, DW_EINVAL,
                 "wind: lattice must be >= 2 nodes per axis with dx > 0");
      o->lnx = w->lat.nx;
      o->lny = w->lat.ny;
      o->lnz = w->lat.nz;
      o->lox_l = w->lat.origin[0];
      o->loy_l = w->lat.origin[1];
      o->loz_l = w->lat.origin[2];
      o->inv_ldx = 1.0f / w->lat.dx;
      o->u = w->u;
      o->L = (int64_t)w->lat.nx * w->lat.ny * w->lat.nz;
      o->vel_scale = w->vel_scale;
      o->k_drag = w->k_drag;
      return DW_OK;
    default:
      return set_error(DW_EINVAL, "wind: unknown mode %d", w->mode);
  }
}

int check_grid(const dw_grid *g) {
  DW_REQUIRE(g, DW_EINVAL, "grid is NULL");
  DW_REQUIRE(g->nx >= 3 && g->ny >= 3 && g->nz >= 3, DW_EINVAL, "grid dims must be >= 3");
  DW_REQUIRE(g->dx > 0.f, DW_EINVAL, "grid dx must be > 0");
  DW_REQUIRE((int64_t)g->nx * g->ny * g->nz < (int64_t)INT_MAX / 3, DW_ERANGE, "grid too large for int32 indexing");
  return DW_OK;
}

int check_particles(const dw_particles *p, bool need_state) {
  DW_REQUIRE(p, DW_EINVAL, "particles is NULL");
  DW_REQUIRE(p->n >= 0, DW_EINVAL, "particle count must be >= 0");
  DW_REQUIRE((int64_t)p->n * 9 < (int64_t)INT_MAX, DW_ERANGE, "too many particles for int32 indexing");
  if (p->n == 0) return DW_OK;
  DW_REQUIRE(p->x, DW_EINVAL, "particles: x is NULL");
  if (need_state) {
    DW_REQUIRE(p->v && p->C && p->F && p->mass && p->vol0 && p->region && p->E && p->nu, DW_EINVAL,
               "particles: v, C, F, mass, vol0, region, E, nu must be set");
    DW_REQUIRE(p->n_regions > 0, DW_EINVAL, "particles: n_regions must be > 0");
  }
  return DW_OK;
}

}  // namespace dw

extern "C" const char *dw_last_error(void) { return dw::g_err; }

extern "C" size_t mpm_workspace_bytes(const dw_grid *grid, int n_max, int deterministic) {
  if (!grid || n_max < 0 || dw::check_grid(grid) != DW_OK) return 0;
  dw::Workspace ws;
  return dw::workspace_layout(grid, n_max, &ws, nullptr, deterministic);
}
