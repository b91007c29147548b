/*
 * lbm3d.h -- C ABI of the three-dimensional (D3Q19 / D3Q27) elastic-wave
 * lattice Boltzmann step of liblbm.so on MI355X (gfx950).
 *
 * The step is the one of lbm.h carried to the regular D3Q19 and D3Q27
 * lattices, which the paper's Chapman-Enskog analysis covers (Escande, Kolluru, Cleon & Sagaut,
 * arXiv 2009.06404, Sec. 3: the isotropy conditions of D2Q9, D3Q15, D3Q19 and
 * D3Q27): BGK collision toward the elastic equilibrium (eqs. equilibrium-solid
 * and Pn with the full 3 x 3 second moment), the source of eq. S (elastic force
 * from the centred density gradient of eq. FDrho along x, y and z, plus a
 * Gaussian x Ricker body force, Sec. 5) added through eq. Si, the absorbing
 * layers of eq. MomentChainAbsorbing (Sec. 6.4), fused with pull streaming
 * (eq. LBGK) and the periodic, rigid (eq. BB) and free-surface (Sec. 6.2) face
 * rules.
 *
 * Conventions (in addition to those of lbm.h, whose error codes, dtypes and
 * face kinds LBM_PERIODIC / LBM_FREE / LBM_FREE0 / LBM_RIGID this header uses).
 *  - Cell (x, y, z): x fastest, then y, then z; z = 0 is the TOP face and z
 *    grows with depth.
 *  - Directions: the rest vector, then (+x,-x), (+y,-y), (+z,-z), (x+y),
 *    (-x-y), (x-y), (-x+y), (x+z), (-x-z), (x-z), (-x+z), (y+z), (-y-z),
 *    (y-z), (-y+z) -- D3Q19, weights 1/3, 1/18 (axes), 1/36 (edges) -- and
 *    for D3Q27 also (x+y+z), (-x-y-z), (x+y-z), (-x-y+z), (x-y+z), (-x+y-z),
 *    (-x+y+z), (x-y-z), weights 8/27, 2/27, 1/54, 1/216 (corners); the
 *    opposite of direction 2k-1 is 2k; b^2 = 1/3.
 *  - One volume per context; kappa = b^2 (mu - lambda) / mu per cell.
 *  - Free surfaces (top and bottom faces only): anti-bounce-back toward the
 *    air state whose density and tangential stress (P_xx, P_xy, P_yy; P_xy
 *    enters through D3Q27's corner links only) are the
 *    boundary cell's (LBM_FREE0) or extrapolated half a cell out (LBM_FREE),
 *    with the stress rows along the normal zero (P_air n = 0, Sec. 6.2). A link
 *    that leaves through several faces bounces back as rigid if any of them is
 *    rigid, else follows the free rule if any is free, else wraps.
 *  - Beyond a non-periodic face the centred density gradient uses the ghost
 *    2 rho_b - rho_in.
 *  - Caller-owned arrays, asynchronous calls on the context's stream and
 *    negative error returns with lbm_last_error() as in lbm.h.
 */
#ifndef LBM3D_H_
#define LBM3D_H_

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3_ctx lbm3_ctx; /* opaque, owned by the library */

enum { LBM3_D3Q19 = 19, LBM3_D3Q27 = 27 }; /* velocity sets */

enum { LBM3_FACE_TOP = 0, LBM3_FACE_BOTTOM = 1, LBM3_FACE_LEFT = 2, LBM3_FACE_RIGHT = 3,
       LBM3_FACE_FRONT = 4, LBM3_FACE_BACK = 5 };

/* Face rules and absorbing layers of a volume. face[LBM3_FACE_*]: PERIODIC in
 * opposite pairs; FREE and FREE0 on the top and bottom faces only. Absorbing
 * layers (Sec. 6.4): damping A(x, y, z) = max over faces f with d_f < thick[f]
 * of profile[f][d_f], d_f = cells from face f; host arrays of length thick[f]
 * (0 <= thick[f] <= the extent normal to f, values >= 0), copied by lbm3_init. */
typedef struct {
  int32_t face[6];
  int32_t thick[6];
  const double *profile[6];
} lbm3_bc;

/* Gaussian-in-space, Ricker-in-time body force (Sec. 5) in three dimensions:
 * F(x, t) = amp exp(-r^2 / (2 sigma^2)) R(t) dir, r with the minimum image
 * along periodic axes, F = 0 for r > 9 sigma; R as in lbm.h. */
typedef struct {
  double x, y, z, sigma, dir_x, dir_y, dir_z, amp, period, t0;
} lbm3_source;

/* Bytes of device workspace lbm3_init needs for the q-velocity set (q =
 * LBM3_D3Q19 or LBM3_D3Q27): two population buffers of q x pitch x ny x nz
 * elements (pitch = nx rounded up to 64) and one pitch x ny x nz plane of
 * kappa. Synchronous, host only. Returns LBM_OK or LBM_E_INVALID (a side < 3,
 * another q, a bad dtype, more than 2^31 cells, or one z plane of
 * populations, q x pitch x ny elements, of 2 GiB or more). */
int lbm3_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t dtype,
                         size_t *bytes);

/* Create a context for one nx x ny x nz volume on the q-velocity set
 * (LBM3_D3Q19 or LBM3_D3Q27) at time t = 0, rest state.
 *  lam, mu, rho: DEVICE arrays of dtype, [nz][ny][nx]; 0 <= nu < 1/2 and
 *    mu, rho > 0 per cell (checked on the device).
 *  tau > 1/2. bc: host struct as above.
 *  workspace: DEVICE memory of at least lbm3_workspace_bytes, 256-B aligned,
 *    owned by the caller and used only by this context.
 *  hip_stream: the hipStream_t all work goes to (NULL = default stream).
 * Synchronous. Returns LBM_OK, LBM_E_INVALID, LBM_E_NOMEM, LBM_E_DEVICE, or
 * LBM_WARN_UNSTABLE (the context is created and usable) when a bulk mode
 * grows for the medium's Poisson ratios at tau (the factor of lbm3_vn_growth
 * on 9 points per axis at the extreme and middle ratios) or a face uses
 * LBM_FREE, with the reason in lbm_last_error. */
int lbm3_init(lbm3_ctx **ctx, int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t dtype,
              const void *lam, const void *mu, const void *rho, double tau,
              const lbm3_bc *bc, void *workspace, size_t ws_bytes, void *hip_stream);

/* Replace the sources (host array, copied; at most 256). Sources lie inside
 * the volume; sigma > 0, period > 0. Synchronous on the stream. */
int lbm3_set_sources(lbm3_ctx *ctx, const lbm3_source *src, int32_t n);

/* Record v = j / rho0 at n receiver cells at every step.
 *  xyz: host int32 triples (x, y, z), copied; cells inside the volume.
 *  comp_mask: bit 0 v_x, bit 1 v_y, bit 2 v_z (ncomp = popcount).
 *  traces: DEVICE array of dtype [max_steps][n][ncomp]; row k holds step
 *    t_now + k. n = 0 removes the receivers. Synchronous on the stream. */
int lbm3_set_receivers(lbm3_ctx *ctx, const int32_t *xyz, int32_t n, int32_t comp_mask,
                       void *traces, int64_t max_steps);

/* Advance n >= 0 steps. Asynchronous. A step runs the lean kernel on the
 * context's stream and the general kernel (see lbm3_kernel_times) on a second
 * stream of the library, forked from and joined back to the context's stream
 * by events, so work queued after the call sees the whole step. */
int lbm3_step(lbm3_ctx *ctx, int64_t n);

/* Per-kernel timing of the step. A step launches the lean kernel over the
 * tiles none of whose pulled cells lies on a non-periodic face and which hold
 * no source or receiver cell, then the general kernel over the others. */
typedef struct {
  int64_t steps;         /* steps timed */
  double lean_ms;        /* mean duration of one lean-kernel launch over the tiles
                            clear of faces, sources and receivers; 0 if none */
  double general_ms;     /* mean duration of one step's other launches: the general
                            kernel, then the lean kernel with sources over the tiles
                            clear of faces and receivers near a source; 0 if none */
  int64_t lean_cells;    /* cells the lean launch (without sources) updates */
  int64_t general_cells; /* cells the other launches update */
  double step_ms;        /* mean duration of a step (both launches) */
} lbm3_kernel_times;

/* Advance n >= 1 steps like lbm3_step, but with both kernels on the context's
 * stream one after the other and HIP events around every launch; the means go
 * to *out (host). Synchronous. Results equal those of lbm3_step. */
int lbm3_step_timed(lbm3_ctx *ctx, int64_t n, lbm3_kernel_times *out);

/* Macroscopic fields at the current time: DEVICE array of dtype [10][nz][ny][nx]
 * = rho, j_x, j_y, j_z, P_xx, P_xy, P_xz, P_yy, P_yz, P_zz (j with the source
 * and the implicit sponge, as in lbm.h). Asynchronous. */
int lbm3_moments(lbm3_ctx *ctx, void *out10);

int lbm3_get_time(const lbm3_ctx *ctx, int64_t *t);

/* Copy the state (post-collision populations of step t-1, DEVICE
 * [q][nz][ny][nx] of dtype, direction order above) out of / into the
 * context; set_state makes t the context time and restarts the receiver
 * trace at row 0 when t differs from it. Asynchronous. */
int lbm3_get_state(lbm3_ctx *ctx, void *dst);
int lbm3_set_state(lbm3_ctx *ctx, const void *src, int64_t t);

/* Workgroup tile: 64 columns (128 for the lean tiles of an FP32 context by
 * default, below) by rows_y (2, 6 or 14) rows, marching planes_z planes
 * (>= 1) in z. Defaults: rows_y 6 and planes_z 16 (12 with 128-column
 * tiles; fewer when a plane has too few tiles for 2048 workgroups, 1536 with
 * 128-column tiles); planes_z = 0
 * selects the default. The tiles near faces, sources and receivers run in
 * 64-column chunks of at most 4 planes, and of 2 rows when rows_y is 14. No
 * tile shape changes the results. Returns LBM_OK or LBM_E_INVALID. Host
 * only. */
int lbm3_set_tile(lbm3_ctx *ctx, int32_t rows_y, int32_t planes_z);
int lbm3_get_tile(const lbm3_ctx *ctx, int32_t *rows_y, int32_t *planes_z);

/* Width in columns of the tiles clear of faces, sources and receivers (the
 * bulk of the streaming and collision of eq. LBGK, Sec. 2): 64, or 128 (two
 * wavefronts per row of a tile, each population row read as 512 contiguous
 * bytes). 128 needs an FP32 context and is its default (LBM_E_INVALID for
 * FP64); rows_y 14 always runs 64. The results do not depend on it. get
 * reports the width the next step uses; planes_z keeps its value (pass
 * planes_z = 0 to lbm3_set_tile for the default of the new width). Host only. */
int lbm3_set_lean_width(lbm3_ctx *ctx, int32_t columns);
int lbm3_get_lean_width(const lbm3_ctx *ctx, int32_t *columns);

/* Largest von Neumann amplification factor of one bulk step (periodic, no
 * sponge, no source; Sec. 4's analysis carried to the q-velocity set) over an
 * nk x nk x nk grid of wavenumbers in [0, pi]^3: > 1 means some plane wave
 * grows. 0 <= nu < 1/2, tau > 1/2, 2 <= nk <= 129. Synchronous, host only.
 * Returns LBM_OK or LBM_E_INVALID. */
int lbm3_vn_growth(int32_t q, double nu, double tau, int32_t nk, double *growth);

/* The factor lbm3_init computed for this context; returns LBM_OK, or
 * LBM_WARN_UNSTABLE as lbm3_init did. Host only. */
int lbm3_stability(const lbm3_ctx *ctx, double *growth);

/* Free the context's own device tables; the workspace stays the caller's.
 * Synchronous. NULL is accepted. */
int lbm3_destroy(lbm3_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H_ */
