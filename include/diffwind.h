/*
 * diffwind.h -- C ABI of libdiffwind.so, the MI355X (gfx950) implementation of
 * the simulation step of DiffWind (ICLR 2026): one MLS-MPM substep with APIC
 * transfers coupled to a D3Q19 lattice-Boltzmann wind field, with a
 * hand-written adjoint for every forward call.
 *
 * The step is the interaction operator S of Eq. simulation_mpm,
 *   (x, v, F, C)^{t+1} = S(x, v, F, C, theta, F_w, dt),
 * split into its three MPM phases (Appendix "Material Point Method": Eq. P2G,
 * Eq. G2P, Eq. deformation_update), the wind force field mapped onto the MPM
 * grid (Sec. 3 problem specification, Sec. 3.2; drag relation of Sec. 3.4),
 * the lattice Boltzmann equation (Eq. lbe, Eq. lbm_sum_v2) and the
 * particle-to-voxel solid rule (Eq. point2voxel).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All arrays are DEVICE pointers, float32 unless stated, owned by the
 *    caller.  The library never allocates or frees memory; scratch space is a
 *    caller-provided workspace sized by mpm_workspace_bytes().
 *  - Structs (dw_grid, dw_particles, ...) are passed by HOST pointer and read
 *    before the call returns.
 *  - Layout is structure-of-arrays, component index slowest:
 *      particle vectors  x[3][n], v[3][n]             (x[a*n + p])
 *      particle matrices C[9][n], F[9][n]              (M_ab at [(3a+b)*n + p])
 *      grid scalars      m[N]                          N = nx*ny*nz
 *      grid vectors      mv[3][N], v[3][N]             node (i,j,k) at i + nx*(j + ny*k)
 *      LBM populations   f[19][L]                      L = nx*ny*nz of the lattice, x fastest
 *  - The deformation gradient is stored shifted by the identity: the F array
 *    holds H = F - I (rest state all zeros), so float32 keeps its relative
 *    resolution on small strains; stresses are evaluated from H without
 *    forming differences of numbers close to one.
 *  - Positions are absolute (dw_particles.xref == NULL: x holds them) or
 *    relative to a fixed per-particle reference (xref != NULL: the position
 *    is xref + x, and x holds the displacement from xref, zero at the start
 *    of a run).  The reference keeps float32 resolution on the motion
 *    itself: an absolute float32 position near 0.5 resolves 6e-8 while a
 *    substep moves it ~1e-6, so over 100 substeps the rounding of stored
 *    absolute positions reaches ~1 % of the displacement; a displacement is
 *    rounded relative to its own size.  Kernels form the grid coordinate as
 *    (xref - origin)/dx + x/dx with each part rounded once, G2P writes the
 *    new displacement x + dt v and never writes xref.
 *  - LBM populations are stored shifted by their lattice weight, f_i - w_i
 *    (rest fluid is all zeros); this keeps float32 resolution on the small
 *    deviations from rest.  Direction order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *    7..18 = (+1,+1,0),(-1,-1,0),(+1,0,+1),(-1,0,-1),(0,+1,+1),(0,-1,-1),
 *    (+1,-1,0),(-1,+1,0),(+1,0,-1),(-1,0,+1),(0,+1,-1),(0,-1,+1).
 *  - `stream` is a hipStream_t (torch.cuda.current_stream().cuda_stream on
 *    PyTorch-ROCm), may be NULL for the null stream.  Every call is
 *    asynchronous and never synchronises the host.
 *  - Return codes: DW_OK (0); DW_EINVAL (-1) null pointer, non-positive or
 *    inconsistent size, unsupported enum value; DW_ERANGE (-2) size beyond
 *    int32 indexing or a fixed kernel limit; DW_ELAUNCH (-3) the HIP launch
 *    failed; DW_EWORKSPACE (-4) workspace too small.  dw_last_error() gives a
 *    message for the last non-zero return on the calling host thread.  No call
 *    aborts the process.
 *  - Device-side conditions are OR-ed into the status word, the first int32
 *    of the MPM workspace (DW_STATUS_* bits); the caller reads it at its sync
 *    points.  mpm_sort() clears it.
 *  - Every *_adj call ACCUMULATES (+=) into its *_bar outputs, which the
 *    caller zeroes once; this lets autograd sum contributions.
 */
#ifndef DIFFWIND_H
#define DIFFWIND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DW_OK = 0, DW_EINVAL = -1, DW_ERANGE = -2, DW_ELAUNCH = -3, DW_EWORKSPACE = -4 };

/* constitutive models (Appendix "Continuum Mechanics", Eq. constitutive_model) */
enum { DW_FIXED_COROTATED = 0, DW_NEO_HOOKEAN = 1 };

/* lattice faces: x-, x+, y-, y+, z-, z+ */
enum { DW_BC_PERIODIC = 0, DW_BC_BOUNCEBACK = 1, DW_BC_INLET = 2, DW_BC_OUTLET = 3 };

/* sources of the per-node wind acceleration */
enum { DW_WIND_NONE = 0, DW_WIND_FORCE_GRID = 1, DW_WIND_LBM_DRAG = 2, DW_WIND_ACC = 3, DW_WIND_LBM_DRAG_REL = 4 };

/* status bits */
enum {
  DW_STATUS_OUT_OF_GRID = 1, /* a particle's 27-node stencil left the grid; it was skipped */
  DW_STATUS_NONFINITE = 2,   /* a NaN/Inf particle position was met */
  DW_STATUS_INVERTED = 4,    /* det F <= 0 met in the stress evaluation */
  DW_STATUS_RENDER_OVERFLOW = 8 /* gs_render: more (kernel, tile) pairs than max_pairs; nothing drawn */
};

/* MPM background grid: nodes at origin + dx * (i, j, k); nx, ny, nz >= 3. */
typedef struct {
  int nx, ny, nz;
  float dx;
  float origin[3];
} dw_grid;

/* LBM lattice: nodes at origin + dx * (i, j, k).  Solid cells of Eq.
 * point2voxel are the cells [x_w, x_w + dx).  The LBM calls take lattices of
 * fewer than 2^29 nodes (DW_ERANGE otherwise; node offsets are 32-bit). */
typedef struct {
  int nx, ny, nz;
  float dx;
  float origin[3];
} dw_lattice;

typedef struct {
  float dt;          /* substep */
  float gravity[3];  /* body acceleration */
  int bound;         /* separating-slip wall depth in nodes (0 = none) */
  int material;      /* DW_FIXED_COROTATED | DW_NEO_HOOKEAN */
  int deterministic; /* 1: fixed-order reductions: the sort orders each tile's
                        particles by index and P2G sums in a fixed order
                        without atomics, so sort + P2G + grid update + G2P
                        are bit-reproducible run to run (needs a workspace
                        sized with deterministic != 0) */
} dw_mpm_params;

/* Particle state (x, m, u, C, F) of the appendix five-tuple plus theta:
 * per-particle rest volume and region index, per-region Young's modulus E
 * and Poisson ratio nu (Lame parameters by Eq. young_poisson). */
typedef struct {
  int n;
  float *x, *v, *C, *F;   /* [3][n], [3][n], [9][n], [9][n]; F holds F - I;
                             x holds the displacement from xref when xref is set */
  const float *mass;      /* [n] */
  const float *vol0;      /* [n] */
  const int32_t *region;  /* [n], values in [0, n_regions) */
  const float *E, *nu;    /* [n_regions] */
  int n_regions;
  const float *xref;      /* [3][n] position reference, or NULL (x absolute) */
} dw_particles;

/* Adjoint particle state: same layout as dw_particles' x, v, C, F. */
typedef struct {
  int n;
  float *x, *v, *C, *F;
} dw_particles_bar;

/* Wind acceleration source for the MPM grid nodes (Sec. 3.2: the force
 * property of the wind grid acts on the MPM background grid). */
typedef struct {
  int mode;            /* DW_WIND_* */
  /* DW_WIND_FORCE_GRID: vertex-centred grid of nw[0]*nw[1]*nw[2] nodes
   * spanning [lo, hi], W = [3][nw_z][nw_y][nw_x] (one time slot); positions
   * outside the box are clamped onto it. */
  int nw[3];
  float lo[3], hi[3];
  const float *W;
  /* DW_WIND_LBM_DRAG: a = k_drag |U| U with U = vel_scale * trilinear(u);
   * u = [3][L] lattice velocity (zero on solid nodes); MPM nodes outside the
   * lattice box get no wind.  Drag relation of Sec. 3.4 with
   * k_drag = rho_w C_D / 2 times area over mass. */
  /* DW_WIND_LBM_DRAG_REL (same fields): the drag of the wind relative to the
   * node, a = k_drag |U - v*| (U - v*) with v* = mv / m, the node's velocity
   * from P2G (zero outside the lattice box).  Only mpm_grid_update and its
   * adjoint evaluate it (wind_to_grid has no node velocity and refuses it). */
  dw_lattice lat;
  const float *u;
  float vel_scale, k_drag;
  /* DW_WIND_ACC: precomputed acceleration [3][N] (e.g. from wind_to_grid) */
  const float *acc;
  /* 1: wind_to_grid_adj sums its transpose in a fixed order (every wind-grid
   * or lattice node gathers the MPM nodes it feeds; no atomics, bit
   * reproducible, slower); 0: float atomics */
  int deterministic;
} dw_wind;

typedef struct {
  float tau;          /* BGK relaxation time, > 0.5; viscosity (tau - 1/2) / 3 */
  float u_in[3];      /* inlet velocity (lattice units) */
  float force[3];     /* uniform body-force density (Guo forcing), lattice units */
  int bc[6];          /* DW_BC_* per face x-, x+, y-, y+, z-, z+; INLET only on x-,
                         OUTLET only on x+; PERIODIC must pair on an axis */
  /* inlet gust: u_in * (1 + amp sin(2 pi (t / period + ky j / ny + kz k / nz) + phase)) */
  float gust_amp, gust_period, gust_ky, gust_kz, gust_phase;
  int t;              /* step index for the gust */
  /* Optional device step counter (lets one captured HIP graph serve every
   * step): if t_in is not NULL the step index is read from *t_in instead of
   * t, and lbm_step writes index + 1 to *t_out (if not NULL; t_out must not
   * alias t_in -- swap the two like the population buffers). */
  const int32_t *t_in;
  int32_t *t_out;
  /* Optional device flag read by lbm_step and lbm_equilibrium: if skip is not
   * NULL and *skip != 0 the call does nothing (no output, no step counter).
   * Lets a captured HIP graph hold a branch that a device-side decision
   * switches off, e.g. the LBM fallback of an accepted surrogate step.  With
   * a switch the calls launch a bounded grid that strides over the lattice,
   * so a switched-off call costs a few thousand workgroups that return at
   * once; the results of a switched-on call are the same bits as without
   * the switch. */
  const int32_t *skip;
} dw_lbm_params;

/* ---------------------------------------------------------------- errors */

/* Message for the last non-zero return on this host thread ("" if none). */
const char *dw_last_error(void);

/* ------------------------------------------------------------- MPM forward */

/* Bytes of workspace needed by the MPM calls for this grid and up to n_max
 * particles.  The workspace holds the status word, the cell-tile sort and
 * the active-tile lists; it persists between calls of one substep.
 * deterministic != 0 adds the scratch of the fixed-order P2G (a 6^3 x 4
 * float partial block per work item: about 3.5 KB x (grid tiles + n/512)).
 * A deterministic workspace also serves the default mode.  Returns 0 on a
 * bad grid or n_max < 0. */
size_t mpm_workspace_bytes(const dw_grid *grid, int n_max, int deterministic);

/* Cell sort (groups particles for the P2G scatter).  Key of particle p =
 * linear index of the 4x4x4 tile holding its stencil base cell
 * floor((x_p - origin)/dx - 1/2).  Writes into the workspace: the permutation
 * grouping particles by tile (order inside a tile unspecified unless
 * params->deterministic), per-tile ranges, the active cell tiles, and the
 * active node tiles (4x4x4 node blocks holding a node of some particle's
 * stencil).  Clears the status word.  x: [3][n]; xref: [3][n] position
 * reference (positions xref + x) or NULL (x absolute). */
int mpm_sort(const dw_grid *grid, const dw_mpm_params *params, const float *x, const float *xref, int n,
             void *ws, size_t ws_bytes, void *stream);

/* P2G, Eq. P2G with the MLS-MPM stress term:
 *   A_p  = m_p C_p - dt V0_p (4/dx^2) tau(F_p),   tau = P F^T (Kirchhoff),
 *   m_i  = sum_p w_ip m_p,
 *   mv_i = sum_p w_ip (m_p v_p + A_p (x_i - x_p)),
 * quadratic B-spline weights w_ip.  Uses the sort that mpm_sort() left in
 * `ws` for the same p->x (call it first).  OVERWRITES grid_m [N] and grid_mv
 * [3][N] on every node of every active node tile; nodes outside active tiles
 * are not written.  Particles whose stencil leaves the grid are skipped and
 * flagged in the status word. */
int mpm_p2g(const dw_grid *grid, const dw_mpm_params *params, const dw_particles *p,
            float *grid_m, float *grid_mv, void *ws, size_t ws_bytes, void *stream);

/* Grid update, explicit integration of Eq. continuum_mechanics on active
 * nodes: for m_i > 0, v_i = mv_i / m_i + dt (g + a_i) where a_i is the wind
 * acceleration from `wind` (NULL = none); else v_i = 0.  Separating-slip
 * walls `bound` nodes deep zero the outward component; pin[i] != 0 (NULL =
 * no pins) zeroes v_i.  Writes grid_v [3][N] on active node tiles only
 * (active tiles of the last mpm_sort on this workspace). */
int mpm_grid_update(const dw_grid *grid, const dw_mpm_params *params, const float *grid_m,
                    const float *grid_mv, const dw_wind *wind, const uint8_t *pin, float *grid_v,
                    const void *ws, size_t ws_bytes, void *stream);

/* G2P, Eq. G2P with APIC C and Eq. deformation_update:
 *   v_p = sum_i w_ip v_i,  C_p = (4/dx^2) sum_i w_ip v_i (x_i - x_p)^T,
 *   x_p += dt v_p,  F_p <- (I + dt C_p) F_p   (weights at the old x_p;
 *   stored as H <- H + dt C (I + H)).
 * Reads in->x, in->F (and in->xref: with a reference, in->x and out->x are
 * displacements from it; out->xref is not used); writes out->x, v, C, F.
 * `in` and `out` may alias. */
int mpm_g2p(const dw_grid *grid, const dw_mpm_params *params, const float *grid_v,
            const dw_particles *in, dw_particles *out, void *stream);

/* Memory layout, not physics: writes the particles in the order of the
 * permutation that the last mpm_sort() left in `ws` (grouped by 4x4x4 cell
 * tile), out->a[i] = in->a[perm[i]] for x, v, C, F, mass, vol0 and region
 * (in->n entries; E and nu are per region and not touched; xref too when
 * in->xref is set, into out->xref, which must then be set).  Keeping the
 * arrays in this order lets P2G and G2P read particles of a tile from
 * neighbouring memory; particles move little per substep, so a reorder now
 * and then keeps it so.  perm_out [n] (NULL to skip) receives perm, i.e. the
 * old index of each new particle.  `in` and `out` must not share arrays;
 * out's mass, vol0 and region are written although the struct declares
 * them const (they are inputs everywhere else). */
int mpm_reorder(const dw_grid *grid, const dw_particles *in, dw_particles *out, int32_t *perm_out,
                const void *ws, size_t ws_bytes, void *stream);

/* Wind acceleration on every MPM node: acc [3][N] (overwritten). */
int wind_to_grid(const dw_grid *grid, const dw_wind *wind, float *acc, void *stream);

/* ------------------------------------------------------------- MPM adjoints */

/* Reverse of mpm_p2g, a gather per particle: given m_bar [N] and mv_bar [3][N]
 * (read at stencil nodes), accumulates into bar->x, v, C, F and E_bar
 * [n_regions] (NULL to skip).  Mass and volume are constants; so is p->xref
 * (bar->x is the adjoint of the position, i.e. of the displacement x).
 * E_bar is summed over particles with float atomics, or, with
 * params->deterministic, in a fixed order through the scratch of a
 * deterministic workspace `ws` (then required; else ws may be NULL). */
int mpm_p2g_adj(const dw_grid *grid, const dw_mpm_params *params, const dw_particles *p,
                const float *grid_m_bar, const float *grid_mv_bar, dw_particles_bar *bar,
                float *E_bar, void *ws, size_t ws_bytes, void *stream);

/* Reverse of mpm_grid_update on the active node tiles of `ws` (same sort as
 * the forward).  Recomputes the wall/pin masks from the forward inputs;
 * accumulates into grid_m_bar [N], grid_mv_bar [3][N] and acc_bar [3][N]
 * (d loss / d a_i; NULL to skip).  With DW_WIND_LBM_DRAG_REL the drag's
 * dependence on v* = mv / m goes into grid_m_bar / grid_mv_bar here, and
 * acc_bar receives d loss / d U_i, the adjoint of the interpolated wind
 * velocity at the node, which wind_to_grid_adj carries back to the lattice. */
int mpm_grid_update_adj(const dw_grid *grid, const dw_mpm_params *params, const float *grid_m,
                        const float *grid_mv, const dw_wind *wind, const uint8_t *pin,
                        const float *grid_v_bar, float *grid_m_bar, float *grid_mv_bar,
                        float *acc_bar, const void *ws, size_t ws_bytes, void *stream);

/* Reverse of mpm_g2p, a sorted scatter: reads the forward inputs in->x,
 * in->xref, in->F and grid_v, the output adjoints out_bar (x, v, C, F; any may be
 * NULL = zero); accumulates into in_bar->x, in_bar->F and grid_v_bar [3][N].
 * Uses the sort in `ws`, which must come from mpm_sort on the same in->x.
 * With params->deterministic (and a deterministic workspace and sort) the
 * grid_v_bar scatter sums in a fixed order without atomics, as the
 * deterministic mpm_p2g does. */
int mpm_g2p_adj(const dw_grid *grid, const dw_mpm_params *params, const float *grid_v,
                const dw_particles *in, const dw_particles_bar *out_bar,
                dw_particles_bar *in_bar, float *grid_v_bar, const void *ws, size_t ws_bytes,
                void *stream);

/* Reverse of wind_to_grid / of the wind term of mpm_grid_update: given
 * acc_bar [3][N], accumulates W_bar [3][nw^3] (FORCE_GRID) or u_bar [3][L]
 * (LBM_DRAG and LBM_DRAG_REL; the lattice velocity adjoint) -- pass the
 * matching pointer in `out_bar`.  For LBM_DRAG_REL acc_bar is the node wind
 * velocity adjoint written by mpm_grid_update_adj. */
int wind_to_grid_adj(const dw_grid *grid, const dw_wind *wind, const float *acc_bar,
                     float *out_bar, void *stream);

/* ----------------------------------------------------- Gaussian kernels */

/* Covariance of each Gaussian kernel after deformation (Sec. 3.2,
 * "Interaction Modeling"): sigma_p = F_p sigma0_p F_p^T for every particle.
 * H [9][n]: F - I row-major (the MPM storage); sigma0, sigma [6][n]:
 * symmetric matrices as (xx, yy, zz, xy, xz, yz); sigma must not alias
 * sigma0.  n = 0 is a no-op. */
int gaussian_covariance(int n, const float *H, const float *sigma0, float *sigma, void *stream);

/* Reverse of gaussian_covariance: given sigma_bar [6][n], the gradient with
 * respect to the six stored entries, ACCUMULATES H_bar [9][n] and
 * sigma0_bar [6][n] (gradients with respect to the stored entries; either
 * may be NULL). */
int gaussian_covariance_adj(int n, const float *H, const float *sigma0, const float *sigma_bar, float *H_bar,
                            float *sigma0_bar, void *stream);

/* ------------------------------------------------------------ rendering */

/* A view (Sec. 3.3, Eq. rendering): world-to-camera rotation R (row-major)
 * and translation t, pinhole intrinsics fx, fy, cx, cy in pixels; pixel
 * (i, j) has its centre at (i + 1/2, j + 1/2).  Kernels with camera depth
 * <= near_plane are not drawn.  bg: background colour.  alpha_min: a kernel
 * whose alpha at a pixel is below it is not blended there (0 blends every
 * kernel at every pixel, the plain sum of Eq. rendering); t_min: a pixel
 * stops blending once its transmittance falls below it (0: never). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float near_plane;
  float bg[3];
  float alpha_min;
  float t_min;
} dw_camera;

/* Workspace of gs_render / gs_render_adj for n kernels, this camera's image
 * size and at most max_pairs (kernel, 16 x 16 pixel tile) pairs. */
size_t gs_render_workspace_bytes(int n, const dw_camera *cam, int64_t max_pairs);

/* Image of n 3-D Gaussian kernels (Eq. rendering; appendix "3D Gaussian
 * Representation"): kernel g has centre mu [3][n] (world), covariance
 * sigma [6][n] (xx, yy, zz, xy, xz, yz; the gaussian_covariance output),
 * colour [3][n] and opacity [n] in [0, 1).  Its projection has centre
 * (fx p_x / p_z + cx, fy p_y / p_z + cy), p = R mu + t, and 2-D covariance
 * J R Sigma R^T J^T (J the Jacobian of the projection at p); at a pixel
 * centre x, alpha = o exp(-(x - m)^T Sigma'^-1 (x - m) / 2), and the kernels
 * are blended front to back by p_z (equal depths in index order):
 * C = sum_i T_i alpha_i c_i + T bg, T_i = prod_{j<i} (1 - alpha_j).
 * Kernels with a singular 2-D covariance are not drawn.  Writes image
 * [3][height][width].  When the kernels cover more than max_pairs (kernel,
 * tile) pairs, status bit DW_STATUS_RENDER_OVERFLOW is set in the workspace
 * (gs_render_status) and the image is not written.  The workspace keeps the
 * sorted lists that gs_render_adj reads. */
int gs_render(const dw_camera *cam, int n, const float *mu, const float *sigma, const float *color,
              const float *opacity, float *image, int64_t max_pairs, void *ws, size_t ws_bytes, void *stream);

/* Reverse of gs_render with the same arguments and the workspace it left:
 * given image (its output) and image_bar [3][H][W], ACCUMULATES mu_bar
 * [3][n], sigma_bar [6][n] (gradients with respect to the stored entries),
 * color_bar [3][n] and opacity_bar [n] (any may be NULL).  Per-kernel sums
 * use float atomics (not bit-reproducible). */
int gs_render_adj(const dw_camera *cam, int n, const float *mu, const float *sigma, const float *color,
                  const float *opacity, const float *image, const float *image_bar, float *mu_bar, float *sigma_bar,
                  float *color_bar, float *opacity_bar, int64_t max_pairs, void *ws, size_t ws_bytes, void *stream);

/* Copies the render workspace's status word and its pair count (two int32)
 * to status_out (device memory), stream-ordered. */
int gs_render_status(const void *ws, int32_t *status_out, void *stream);

/* Workspace of render_loss for a C x H x W image. */
size_t render_loss_workspace_bytes(int C, int H, int W);

/* Photometric loss of Sec. 3.3 for one view: L = (1 - lambda) L1 +
 * lambda (1 - SSIM) with L1 the mean of |image - target| over channels and
 * pixels and SSIM the mean structural similarity (per channel, 11 x 11
 * Gaussian window of sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, windows zero
 * outside the image).  ADDS L to *loss (if not NULL; the block partial sums
 * are reduced in a fixed order) and dL/dimage to image_bar (if not NULL).
 * image, target [C][H][W]. */
int render_loss(int C, int H, int W, const float *image, const float *target, float lambda, float *loss,
                float *image_bar, void *ws, size_t ws_bytes, void *stream);

/* -------------------------------------------------------- reconstruction */

/* Physics-informed loss of Sec. 3.4 over the n wind-grid nodes:
 * L_phys = sum_i |d_i - (d_i . g_i) g_i|^2, d_i and g_i the unit directions
 * of W [3][n] (reconstructed force field) and guide [3][n] (LBM velocity at
 * the nodes, see wind_guide); nodes where either vector is zero contribute
 * nothing.  ADDS weight * L_phys to *loss (if not NULL) and
 * weight * dL_phys/dW to W_bar [3][n] (if not NULL).  One workgroup sums
 * the loss in a fixed node order, so both outputs are bit-reproducible. */
int phys_loss(int n, const float *W, const float *guide, float weight, float *loss, float *W_bar, void *stream);

/* Position loss sum_p |x_p - x*_p|^2 over n particles (the synthetic stand-in
 * for the photometric loss of Sec. 3.3): ADDS it to *loss (if not NULL) and
 * WRITES its gradient 2 (x - x*) to x_bar [3][n] (if not NULL). */
int position_loss(int n, const float *x, const float *x_target, float *loss, float *x_bar, void *stream);

/* Direction metrics of the appendix's evaluation of reconstructed wind force
 * fields: with unit vectors a_i = F_ref_i / |F_ref_i| and b_i = F_i / |F_i|
 * over the n locations where both are non-zero, ADDS (sum a.b, sum |a - b|^2,
 * count) to out[0..2]; CosSim = out[0] / out[2], NMSE = out[1] / out[2]. */
int direction_metrics(int n, const float *F_ref, const float *F, float *out, void *stream);

/* The LBM direction guide: the lattice velocity u [3][L] sampled trilinearly
 * at the nodes of a vertex-centred wind grid of nw[0] x nw[1] x nw[2] nodes
 * spanning [lo, hi] (x fastest), into guide [3][nw^3]; nodes outside the
 * lattice box get 0. */
int wind_guide(const dw_lattice *lat, const float *u, const int nw[3], const float lo[3], const float hi[3],
               float *guide, void *stream);

/* ------------------------------------------------------------------ LBM */

/* One fused pull stream-collide step of Eq. lbe with BGK collision (D3Q19),
 * moments of Eq. lbm_sum_v2 with the half-force shift and Guo forcing.
 * Streaming: periodic faces wrap; a source beyond a bounce-back face or on a
 * solid node gives halfway bounce-back f_i(x) = f*_opp(i)(x); a source beyond
 * the inlet face gives f^eq(rho = 1, u_in(t)); beyond the outlet face the
 * source is clamped onto the last plane (zero gradient).  Solid nodes
 * (solid[i] != 0; NULL = none) output the rest state and u = 0, rho = 1.
 * f_in, f_out: [19][L] shifted populations, must not alias.  rho_out [L] and
 * u_out [3][L] are optional (NULL). */
int lbm_step(const dw_lattice *lat, const dw_lbm_params *params, const float *f_in, float *f_out,
             const uint8_t *solid, float *rho_out, float *u_out, void *stream);

/* Reverse of lbm_step: given f_out_bar [19][L] and u_out_bar [3][L] (NULL =
 * zero), ACCUMULATES f_in_bar [19][L].  Two passes: the first recomputes
 * every node's pulled populations and writes their adjoints through the BGK
 * collision to work [19][L] (device scratch of 76 bytes per node, owned by
 * the caller, contents on return unspecified); the second adds to every
 * f_in_bar entry the adjoint of the pull that read it (the streaming
 * transposed under the same boundary rules, bounced pulls included).  Solid
 * nodes pass nothing back.  No atomics: the result does not depend on
 * scheduling.  f_in_bar must alias neither f_in nor f_out_bar; work aliases
 * no other argument. */
int lbm_step_adj(const dw_lattice *lat, const dw_lbm_params *params, const float *f_in,
                 const uint8_t *solid, const float *f_out_bar, const float *u_out_bar,
                 float *f_in_bar, float *work, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_step_adj with its
 * work buffer in a static device array of the library instead of a
 * caller-provided one.  Same arguments, result and error behaviour as
 * lbm_step_adj, without `work`; lattices of at most DW_STATIC_ADJ_MAX_NODES
 * nodes (the 128 x 64 x 64 tunnel; larger ones return DW_ERANGE with a
 * message, before any launch).  The array (19 x DW_STATIC_ADJ_MAX_NODES
 * floats, 38 MiB) exists once per device for the life of the process; its
 * device address is looked up on the first call on each device.  No call
 * allocates or frees memory.  Every call on one device uses the same array,
 * so calls that overlap on one device (two streams, two host threads) race
 * and must be serialised by the caller; the array keeps the last call's
 * contents, which no later call reads before writing. */
enum { DW_STATIC_ADJ_MAX_NODES = 1 << 19 };
int lbm_step_adj_static(const dw_lattice *lat, const dw_lbm_params *params, const float *f_in,
                        const uint8_t *solid, const float *f_out_bar, const float *u_out_bar, float *f_in_bar,
                        void *stream);

/* Shifted equilibrium populations f^eq(rho, u) - w: rho [L] (NULL = 1) and
 * u [3][L] (NULL = the uniform params->u_in).  Used to initialise a lattice
 * and to re-initialise it from macroscopic fields. */
int lbm_equilibrium(const dw_lattice *lat, const dw_lbm_params *params, const float *rho,
                    const float *u, float *f, void *stream);

/* HOME-LBM step (appendix "More details on HOME-LBM Algorithm"): the
 * moment-encoded form of the same lattice.  A node stores its post-collision
 * moments m [10][L] = rho - 1, u (3), S (6: xx yy zz xy xz yz), with
 * rho S_ab = sum_i (c_ia c_ib - delta_ab / 3) f_i.  For each direction the
 * population of the source node is rebuilt from the source's moments by the
 * third-order Hermite expansion (first equation of the appendix, over the
 * six third-order classes D3Q19 carries, a3_aab = S_aa u_b + 2 S_ab u_a -
 * 2 u_a^2 u_b), pulled with the boundary rules of lbm_step (an inlet ghost
 * holds rho = 1, u = u_in(t), S = u_in u_in), and the moments of the pulled
 * set are relaxed in moment space (second equation of the appendix): the
 * deviatoric part of S relaxes with 1/tau towards that of u u (the printed
 * diagonal update is read with its equilibrium term (u_a^2 - |u|^2/3)/tau),
 * the trace is set to |u|^2, the force enters as Guo's source, and the
 * stored u is u* + F / (2 rho).  rho_out [L] and u_out [3][L] (optional)
 * receive the macroscopic rho* and u* = (sum c f* + F / 2) / rho*.  Solid
 * nodes store the rest state and report u = 0, rho = 1.  m_in and m_out must
 * not alias. */
int lbm_home_step(const dw_lattice *lat, const dw_lbm_params *params, const float *m_in, float *m_out,
                  const uint8_t *solid, float *rho_out, float *u_out, void *stream);

/* Reverse of lbm_home_step: given m_out_bar [10][L] and u_out_bar [3][L]
 * (the reported velocity's adjoint; NULL = zero), ACCUMULATES m_in_bar
 * [10][L].  Two passes: the first recomputes every node's pulled set and
 * writes the adjoints of its 19 pulled populations to work [19][L] (device
 * scratch of 76 bytes per node, owned by the caller, contents on return
 * unspecified); the second gathers, for every node, the adjoints of the
 * populations rebuilt from its moments (the streaming transposed under the
 * same boundary rules, bounced pulls included) and takes them back through
 * the Hermite expansion.  Solid nodes pass nothing back.  No atomics: the
 * result does not depend on scheduling.  m_in_bar must alias neither m_in
 * nor m_out_bar; work aliases no other argument. */
int lbm_home_step_adj(const dw_lattice *lat, const dw_lbm_params *params, const float *m_in,
                      const uint8_t *solid, const float *m_out_bar, const float *u_out_bar, float *m_in_bar,
                      float *work, void *stream);

/* Equilibrium moments (rho, u, S = u u) into m [10][L]: rho [L] (NULL = 1)
 * and u [3][L] (NULL = the uniform params->u_in). */
int lbm_home_equilibrium(const dw_lattice *lat, const dw_lbm_params *params, const float *rho,
                         const float *u, float *m, void *stream);

/* Eq. point2voxel: solid[floor((x_p - origin)/dx)] = 1 for every particle
 * inside the lattice.  accumulate = 0 clears solid [L] (uint8) first,
 * 1 ORs into it (static obstacles).  x [3][n]; xref [3][n] or NULL as in
 * mpm_sort (with a reference the index is floor((xref - origin)/dx + x/dx),
 * each part rounded once). */
int lbm_solid_from_particles(const dw_lattice *lat, const float *x, const float *xref, int n, uint8_t *solid,
                             int accumulate, void *stream);

/* ------------------------------------------------------ wind surrogate */

/* A learned stand-in for k LBM steps (the paper has no learned wind model;
 * the lattice Boltzmann step of Eq. lbe is its fallback and its reference):
 *   u_{t+k} = u_t + g s net(u_t / s),
 *   net = conv(32->3) o silu o conv(32->32) o silu o conv(32->32) o silu o conv(3->32),
 * 3x3x3 kernels with zero padding, s the per-field inflow speed, g a fixed
 * output gain (the binding uses 0.01; conv3d_bf16's output epilogue takes
 * g s as its per-field scale).  Fields are
 * batches of B lattices of nx * ny * nz voxels (any sizes; multiples of 16 in
 * x and 4 in y, z fill every tile).  Velocities are float [B][3][L] (as lbm_step writes u); activations
 * are BF16 (uint16 storage) channels-last [B][L][C] with C = 8 for
 * 3-channel fields (zero padded) and 32 otherwise; weights are kept in FP32
 * [cout][cin][27] (tap = 9 dz + 3 dy + dx) and packed to BF16 MFMA fragments
 * for the kernels; all products accumulate in FP32. */
enum { DW_CONV_HIDDEN = 0, DW_CONV_OUTPUT = 1, DW_CONV_DGRAD = 2 };

/* Number of BF16 elements of a packed weight buffer for a layer cin -> cout
 * (as a forward layer; the data-gradient packing of that layer has the size
 * of conv_packed_weight_elems(cout, cin)). */
size_t conv_packed_weight_elems(int cin, int cout);

/* Pack FP32 weights w [cout][cin][27] into BF16 fragments.  flip = 0: the
 * forward layer; flip = 1: its transposed convolution (taps mirrored, cin and
 * cout exchanged) used for the data gradient.  cin, cout in {3, 32}. */
int conv_pack_weights(const float *w, int cin, int cout, int flip, uint16_t *wk, void *stream);

/* x0 [B][L][8] = BF16(u [B][3][L] / scale[b]), channels 3..7 zero. */
int conv_prep_input(int B, int nx, int ny, int nz, const float *u, const float *scale, uint16_t *x0,
                    void *stream);

/* One convolution layer on MFMA.
 *  DW_CONV_HIDDEN (cin 3 or 32 -> cout 32): y = BF16(silu(conv(x) + bias)),
 *     zpre (nullable) = BF16(conv(x) + bias) kept for the backward pass.
 *  DW_CONV_OUTPUT (32 -> 3): u_out[b][c] = u[b][c] + scale[b] (conv(x) + bias)[c].
 *  DW_CONV_DGRAD (for the layer cin -> cout, cin = 32): x is the gradient of the
 *     layer's output pre-activation (channels 8 if cout = 3, else 32), wk the
 *     flip = 1 packing; y = BF16(conv^T(x) * silu'(zgate)) is the gradient of
 *     the previous layer's pre-activation (zgate = that layer's zpre). */
int conv3d_bf16(int B, int nx, int ny, int nz, int cin, int cout, int epilogue, const uint16_t *x,
                const uint16_t *wk, const float *bias, uint16_t *y, uint16_t *zpre, const uint16_t *zgate,
                const float *u, const float *scale, float *u_out, void *stream);

/* Floats of scratch that conv3d_bf16_wgrad needs. */
size_t conv_wgrad_scratch_floats(void);

/* Weight and bias gradients of the layer cin -> cout on MFMA:
 *   dw[co][ci][tap] = sum over the batch and voxels of dz[v][co] x[v + off(tap)][ci],
 *   db[co] = sum over voxels of dz[v][co]   (db nullable),
 * x the layer input (channels 8 if cin = 3, else 32), dz the gradient of the
 * layer's pre-activation output (channels 8 if cout = 3, else 32).  FP32
 * results, summed in a fixed order (bit-reproducible); accumulate = 1 adds to
 * dw, db instead of overwriting. */
int conv3d_bf16_wgrad(int B, int nx, int ny, int nz, int cin, int cout, const uint16_t *x, const uint16_t *dz,
                      float *dw, float *db, int accumulate, float *scratch, void *stream);

/* Mean squared error of the scaled increments, mean over b, c, v of
 * ((u_out - u_tgt) / scale_b)^2, and its gradient with respect to the net
 * output, written as BF16 dy [B][L][8].  loss_part receives one partial sum
 * per 256 voxels (their sum is the loss). */
int conv_mse_grad(int B, int nx, int ny, int nz, const float *u_out, const float *u_tgt, const float *scale,
                  uint16_t *dy, float *loss_part, void *stream);

/* One Adam step (Kingma & Ba 2015) on n FP32 parameters; step counts from 1. */
int adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
              int step, void *stream);

/* Checks of velocity fields u [B][3][L]: out[b][0..2] = (sum of squared
 * central-difference divergence over interior fluid nodes, number of such
 * nodes, kinetic energy 1/2 sum |u|^2 over fluid nodes); solid [B][L] (one
 * mask per field, nonzero = solid) or NULL.  out [B][3] is overwritten.
 * ws (device, ws_bytes >= field_stats_workspace_bytes, else DW_EWORKSPACE)
 * receives per-workgroup partial sums, which a second kernel adds in a
 * fixed order in double: the result is the same on every call.  Rows
 * ny * nz must be below 2^31 (DW_ERANGE). */
size_t field_stats_workspace_bytes(int B, int nx, int ny, int nz);
int field_stats(int B, int nx, int ny, int nz, const float *u, const uint8_t *solid, float *out, void *ws,
                size_t ws_bytes, void *stream);

/* Device-side acceptance of surrogate predictions (no host
 * synchronisation, capturable in a HIP graph).  stats_prev and stats_pred
 * [B][3] are field_stats of the input fields and of the predictions;
 * accept[b] = 1 iff the prediction's RMS central-difference divergence is at
 * most div_factor times the input's and its kinetic energy lies in
 * [ke_lo, ke_hi] times the input's (a non-finite prediction fails both);
 * else 0.  reject [B] (nullable) receives 1 - accept: as the `skip` flag of
 * dw_lbm_params, accept switches the LBM fallback off and reject switches a
 * branch on only for rejected fields. */
int field_accept(int B, const float *stats_prev, const float *stats_pred, float div_factor, float ke_lo, float ke_hi,
                 int32_t *accept, int32_t *reject, void *stream);

/* u_out [B][3][L] = accept[b] ? u_pred with zero velocity on solid nodes
 * (solid [B][L] nullable, as lbm_step reports solids) : u_alt.  u_out may
 * alias either input. */
int field_select(int B, int nx, int ny, int nz, const int32_t *accept, const float *u_pred, const float *u_alt,
                 const uint8_t *solid, float *u_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DIFFWIND_H */
