/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 elastic-wave lattice Boltzmann
 * library (liblbm.so).
 *
 * The library advances the single-relaxation-time D2Q9 scheme for elastic
 * waves in isotropic linear solids of Escande, Kolluru, Cleon & Sagaut
 * (arXiv 2009.06404): BGK collision toward the elastic equilibrium (Sec. 2,
 * eqs. equilibrium-solid and Pn) with the source of eq. S (elastic force from
 * the centred density gradient of eq. FDrho plus a Gaussian x Ricker body
 * force, Sec. 5) added through eq. Si, the absorbing-layer term of eq.
 * MomentChainAbsorbing (Sec. 6.4), fused with pull streaming (eq. LBGK) and the
 * periodic, rigid (bounce-back, eq. BB) and free-surface (anti-bounce-back,
 * Sec. 6.2) boundary rules.
 *
 * Conventions.
 *  - Lattice units dt = dx = 1. Cell (x, y): x is the column (fast index),
 *    y the row; row 0 is the TOP edge and y grows with depth.
 *  - Populations are perturbations about the rest state f = 0.
 *  - Elastic coefficient per cell: kappa = b^2 (mu - lambda) / mu, i.e. the
 *    paper's (mu - lambda)/rho0 with mu/rho0 = b^2 = 1/3 (Sec. 4). Only the
 *    ratio lambda/mu enters; rho0 scales the recorded velocity v = j/rho0.
 *  - The state at time t is the post-collision population set of step t-1;
 *    at t = 0 it is zero. lbm_step(n) runs the steps t .. t+n-1.
 *  - All arrays passed in are CALLER-OWNED; the library keeps non-owning
 *    pointers and never frees them. Device arrays must stay valid and
 *    unmodified by the caller while the context uses them.
 *  - Every call after lbm_init is asynchronous on the HIP stream given to
 *    lbm_init, except those documented as synchronous.
 *  - Errors: a negative return value; lbm_last_error() then describes it.
 *    Arguments are validated on the host before anything is enqueued; a call
 *    that fails validation has no effect.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 1

typedef struct lbm_ctx lbm_ctx; /* opaque, owned by the library */

enum {
  LBM_WARN_UNSTABLE = 1, /* accepted, but outside the scheme's stable window
                            (lbm_init, lbm_stability); the run proceeds */
  LBM_OK = 0,
  LBM_E_INVALID = -1,   /* argument out of range or inconsistent */
  LBM_E_NOMEM = -2,     /* workspace too small or host allocation failed */
  LBM_E_DEVICE = -3,    /* a HIP call failed */
  LBM_E_NONFINITE = -4, /* the state holds NaN or Inf */
  LBM_E_STATE = -5      /* call not valid in the context's current state */
};

enum { LBM_F32 = 0, LBM_F64 = 1 };

/* Edge types (Sec. 6). PERIODIC must be paired (top with bottom, left with
 * right). FREE and FREE0 are accepted on the top and bottom edges only.
 *  LBM_FREE   free surface (anti-bounce-back, Sec. 6.2) with rho_air and the
 *             tangential stress P_xx,air linearly extrapolated half a cell out
 *             (3/2 boundary cell - 1/2 the cell inside), as printed. This rule
 *             lets short-wavelength surface modes grow for every tau (the step
 *             has spectral radius > 1, e.g. 1.046 at nu = 0.25, tau = 1), so
 *             long runs amplify rounding noise without bound.
 *  LBM_FREE0  the same rule with the boundary cell's own rho and P_xx (zero-
 *             order extrapolation): spectral radius <= 1 for 0.1 <= nu <= 0.33
 *             at tau in [0.7, 2]; the stabilised variant for long runs.
 *  LBM_RIGID  halfway bounce-back (eq. BB). */
enum { LBM_PERIODIC = 0, LBM_FREE = 1, LBM_RIGID = 2, LBM_FREE0 = 3 };
enum { LBM_EDGE_TOP = 0, LBM_EDGE_BOTTOM = 1, LBM_EDGE_LEFT = 2, LBM_EDGE_RIGHT = 3 };

typedef struct {
  int32_t nx, ny; /* >= 3 each */
} lbm_grid;

/* Boundary rules of one grid. rigid_row = -1: none; otherwise an internal
 * rigid wall (bounce-back from both sides) between rows rigid_row-1 and
 * rigid_row, 2 <= rigid_row <= ny-2. The centred density gradient is not
 * taken across non-periodic edges or the internal wall: there the neighbour
 * density is the linear extrapolation 2 rho_b - rho_in. A link that crosses a
 * rigid and a free edge at once bounces back as rigid. */
typedef struct {
  int32_t edge[4];   /* LBM_PERIODIC / LBM_FREE / LBM_FREE0 / LBM_RIGID per LBM_EDGE_* */
  int32_t rigid_row;
} lbm_bc;

/* Absorbing layers (Sec. 6.4): damping A(x, y) = max over edges e with
 * d_e < thick[e] of profile[e][d_e], d_e = cells from edge e. Host arrays of
 * length thick[e] (0 <= thick[e] <= the extent normal to the edge), copied
 * during lbm_init. */
typedef struct {
  int32_t thick[4];
  const double *profile[4];
} lbm_sponge;

/* Gaussian-in-space, Ricker-in-time body force (Sec. 5):
 * F(x, t) = amp exp(-r^2 / (2 sigma^2)) R(t) (dir_x, dir_y), r measured with
 * the minimum image along periodic axes, F = 0 for r > 9 sigma;
 * R(t) = (1 - 2 a^2) exp(-a^2), a = pi (t - t0) / period, evaluated at the
 * integer step index t of the collision. */
typedef struct {
  double x, y, sigma, dir_x, dir_y, amp, period, t0;
} lbm_source;

/* Launch configuration chosen by the autotuner or set by the caller. */
typedef struct {
  int32_t waves;      /* wavefronts per workgroup: 1, 2, 4 or 8 (64 columns each) */
  int32_t rows;       /* rows marched per workgroup */
  int32_t graph_chunk;/* steps per captured HIP graph; 0 = direct launches */
  int32_t prefetch;   /* rows of populations in flight while marching: 1 or 2 */
  int32_t split;      /* 1: tiles clear of walls, sources and receivers run in a
                         lean interior kernel (default); 0: one kernel for all */
  int32_t pair;       /* 1: the interior kernel handles two columns per lane
                         (used when every grid's nx is even and waves >= 2) */
  int32_t overlap;    /* 1: the general kernel runs on a second stream of the
                         library, concurrently with the interior kernel, joined
                         back to the context's stream at the end of the step
                         (default); 0: one kernel after the other */
  int32_t fuse_rows;  /* 0: one kernel pass per step. 4..248: steps run in
                         pairs; blocks of 64 x max(waves, 2) columns by up to
                         fuse_rows rows that hold no boundary, receiver or
                         source take two steps in one pass (the intermediate
                         state stays on chip); the other cells take the two
                         steps one at a time through a third buffer, together
                         with the two border rows or columns of the blocks
                         next to them.
                         Results are bitwise those of single steps. With
                         graph_chunk > 0 a chunk is graph_chunk / 2 pairs in
                         one captured graph (three kernels per pair, the fork
                         and join as graph edges). The default is set by
                         size: on contexts of 2048^2 cells and more the
                         three-step path (fuse_steps 3) launched directly
                         (graph_chunk 0), in 192-column blocks (tri_waves 3)
                         of 96 rows (92 in FP64) on grids of 4096 rows and
                         more and 32 rows otherwise. */
  int32_t fuse_steps; /* steps per pass of the blocks when fuse_rows > 0: 2
                         (0 means 2) or 3. With 3 the steps run in triples:
                         blocks of 64 x tri_waves columns take
                         three steps in one pass (the two intermediate states
                         stay on chip; the blocks keep six rows and columns
                         clear of walls, the y-wrap, sources and receivers);
                         the other cells take the three steps one at a time,
                         the first beside the blocks' pass with the four
                         border rows or columns next to them, the second
                         (with two border rows or columns) and the third
                         after it. Leftover steps run as a pair and a single
                         step. Results are bitwise those of single steps;
                         with graph_chunk > 0 (rounded up to a multiple of 3)
                         a chunk is graph_chunk / 3 triples in one captured
                         graph. The recorded forward of the adjoint runs in
                         pairs either way. The path uses a second
                         intermediate buffer as large as one of the
                         workspace's population buffers, which the library
                         allocates itself when the launch is set
                         (LBM_E_NOMEM if the device cannot hold it) and
                         frees when fuse_steps changes back or the context is
                         destroyed. */
  int32_t tri_waves;  /* output wavefronts of a three-step block: 2, 3 or 4
                         (blocks of 128, 192 or 256 columns; each workgroup
                         has one more wavefront for the halo columns); 0 takes
                         min(max(waves, 2), 4). Leftover pairs and single
                         steps keep the widths that waves gives. */
} lbm_launch;

/* Bytes of device workspace lbm_init needs for nbatch grids of the given
 * sizes and dtype: three population buffers of 9 x pitch x ny elements per
 * grid (the state, the next state and the intermediate state of the two-step
 * path; pitch = nx rounded up to 64) and one x pitch x ny plane of cell
 * moduli. Synchronous, host only. Returns LBM_OK or LBM_E_INVALID (a side
 * below 3, or a grid too wide for the kernels' 32-bit row addressing: 8 rows
 * of nine population runs, 8 x 9 x pitch x 4 (FP32) or x 8 (FP64) bytes, must
 * stay below 2^31 bytes; lbm_init refuses such grids as well). */
int lbm_workspace_bytes(const lbm_grid *grids, int32_t nbatch, int32_t dtype,
                        size_t *bytes);

/* Create a context for nbatch independent grids advanced together.
 *  grids[nbatch], bc[nbatch], sponge[nbatch]: host arrays.
 *  lam, mu, rho: DEVICE arrays of dtype holding the grids' row-major fields
 *    packed one after the other (grid g starts at sum_{h<g} nx_h*ny_h).
 *    0 <= nu = lam / (2 (lam + mu)) < 5/11 (Sec. 4) and mu, rho > 0 per cell.
 *  tau > 1/2 (Sec. 3).
 *  workspace: DEVICE memory of at least lbm_workspace_bytes, 256-B aligned,
 *    owned by the caller and used exclusively by this context.
 *  hip_stream: the hipStream_t all work is enqueued on (NULL = default).
 * Synchronous (validates the fields on the device and waits for it). On
 * success *ctx holds a context at time t = 0 with the rest state; the return
 * is LBM_OK, or LBM_WARN_UNSTABLE (the context is created and usable) when a
 * bulk mode grows for the media's Poisson ratios at tau (see lbm_stability)
 * or an edge uses LBM_FREE, with the reason in lbm_last_error. */
int lbm_init(lbm_ctx **ctx, const lbm_grid *grids, int32_t nbatch,
             int32_t dtype, const void *lam, const void *mu, const void *rho,
             double tau, const lbm_bc *bc, const lbm_sponge *sponge,
             void *workspace, size_t ws_bytes, void *hip_stream);

/* Replace the sources of grid g (host array, copied). Synchronous on the
 * stream. Sources must lie inside the grid; sigma > 0, period > 0. */
int lbm_set_sources(lbm_ctx *ctx, int32_t g, const lbm_source *src, int32_t n);

/* Record v = j / rho0 at n receiver cells of grid g at every step.
 *  xy: host int32 pairs (x, y), copied; cells inside the grid.
 *  comp_mask: bit 0 records v_x, bit 1 records v_y (ncomp = popcount).
 *  traces: DEVICE array of dtype, layout [max_steps][n][ncomp]; row k holds
 *    step (t_now + k), where t_now is the context time at this call. Steps
 *    beyond max_steps are not recorded. n = 0 removes the receivers. */
int lbm_set_receivers(lbm_ctx *ctx, int32_t g, const int32_t *xy, int32_t n,
                      int32_t comp_mask, void *traces, int64_t max_steps);

/* Advance all grids n >= 0 steps. Asynchronous. */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* Per-kernel timing of the step (diagnostics for roofline measurement). A
 * step launches the interior kernel over the tiles clear of walls, sources and
 * receivers (when split is on), then the general kernel over the rest. With
 * fuse_rows > 0 the steps go in pairs: the general kernel (step t), the
 * two-step kernel (steps t and t+1 of its blocks), the general kernel (step
 * t+1); an odd last step runs alone as above. With fuse_steps = 3 they go in
 * triples: the general kernel (step t), the three-step kernel, the general
 * kernel (steps t+1 and t+2); leftover steps as a pair and a single step. */
typedef struct {
  int64_t steps;          /* steps timed */
  double interior_ms;     /* mean duration of one interior-kernel launch; 0 if none */
  double general_ms;      /* mean duration of one general-kernel launch; 0 if none */
  int64_t interior_cells; /* cells one interior-kernel launch updates */
  int64_t general_cells;  /* cells one general-kernel launch updates (of the
                             two-step path's general tiles when fuse_rows > 0) */
  double fused_ms;        /* mean duration of one multi-step-kernel launch; 0 if none */
  int64_t fused_cells;    /* cells one multi-step-kernel launch advances by
                             fused_steps steps */
  int32_t fused_steps;    /* steps per multi-step-kernel launch: 2 or 3 (0 if none) */
} lbm_kernel_times;

/* Advance all grids n >= 0 steps like lbm_step, but with direct launches and
 * a HIP event pair on the context's stream around every kernel launch; the
 * mean launch durations and the cells each kernel covers go to *out (host).
 * Synchronous (waits for every step). Results equal those of lbm_step. */
int lbm_step_timed(lbm_ctx *ctx, int64_t n, lbm_kernel_times *out);

/* Macroscopic fields of grid g at the current time t: DEVICE array of dtype,
 * layout [6][ny][nx] = rho, j_x, j_y, P_xx, P_xy, P_yy (Sec. 2: P is the
 * second moment, the stress with the opposite sign; j = sum f c + S/2 with
 * the sponge solved implicitly). Asynchronous. */
int lbm_moments(lbm_ctx *ctx, int32_t g, void *out6);

int lbm_get_time(const lbm_ctx *ctx, int64_t *t);

/* Copy the state of grid g (post-collision populations of step t-1,
 * DEVICE [9][ny][nx] of dtype, direction order (0,0),(1,0),(0,1),(-1,0),
 * (0,-1),(1,1),(-1,1),(-1,-1),(1,-1)) out of / into the context. set_state
 * with g = -1 is invalid; the context time becomes t for all grids, and when
 * t differs from the current time every grid's receiver trace restarts (row
 * 0 records step t). Asynchronous. */
int lbm_get_state(lbm_ctx *ctx, int32_t g, void *dst);
int lbm_set_state(lbm_ctx *ctx, int32_t g, const void *src, int64_t t);

/* Von Neumann stability of the step (Sec. 4): the largest amplification
 * factor per step of a plane wave exp(i k.x) under the bulk scheme (periodic,
 * no sponge, no source) over an nk x nk grid of wavenumbers in [0, pi]^2, for
 * Poisson ratio nu in [0, 1/2) and tau > 1/2, into *growth (host). A factor
 * above 1 means some mode grows without bound (the paper's instability of
 * nu != 1/4 at high wavenumbers). Synchronous, host only. Returns LBM_OK or
 * LBM_E_INVALID. */
int lbm_vn_growth(double nu, double tau, int32_t nk, double *growth);

/* The same factor per step for `every` (1..1000) steps followed by one
 * lbm_filter of strength sigma in [0, 1/16]: the spectral radius of
 * F(k) M(k)^every to the power 1/every, F the filter's factor below. Host
 * only. Returns LBM_OK or LBM_E_INVALID. */
int lbm_vn_growth_filtered(double nu, double tau, double sigma, int32_t every, int32_t nk,
                           double *growth);

/* High-wavenumber filter of the state (Sec. 4: instability of nu != 1/4
 * sits at high wavenumbers, and filtering high frequencies at the end of a
 * step restores stability; the paper leaves the filter open). Every
 * population of every grid becomes f - sigma (d4x f + d4y f), d4 the fourth
 * difference g(-2) - 4 g(-1) + 6 g(0) - 4 g(1) + g(2) along x or y; its factor
 * on a plane wave is 1 - 16 sigma (sin^4(kx/2) + sin^4(ky/2)). An axis term
 * is left out where its five-point stencil would leave the grid through a
 * non-periodic edge or cross the internal rigid wall. The time is unchanged.
 * 0 < sigma <= 1/16. Asynchronous. Returns LBM_OK, LBM_E_INVALID, or
 * LBM_E_STATE while an adjoint recording is open. */
int lbm_filter(lbm_ctx *ctx, double sigma);

/* The factor lbm_init computed for this context: the largest of
 * lbm_vn_growth(nu, tau, 33) over the media's Poisson ratios (all of them
 * for homogeneous and layered media, up to 16 evenly spaced over the range
 * otherwise). Returns LBM_OK or LBM_WARN_UNSTABLE as lbm_init did. Host only. */
int lbm_stability(const lbm_ctx *ctx, double *growth);

/* Check every grid's state for NaN/Inf. Synchronous. Returns LBM_OK or
 * LBM_E_NONFINITE. */
int lbm_check_finite(lbm_ctx *ctx);

/* Periodic finite check (numerical blow-up: the paper's instability of
 * nu != 1/4 at high wavenumbers, Sec. 4, or the printed free surface). With
 * every > 0, lbm_step checks every grid's state each time the context time
 * reaches a multiple of `every` (a read of the whole state, asynchronous on
 * the stream; steps run in segments ending there, so captured graphs serve
 * chunks that fit between checks) and records the first time whose state
 * holds NaN or Inf. Once that check has run, lbm_step returns
 * LBM_E_NONFINITE without stepping, with the time in lbm_last_error; the
 * recorded failure is cleared by lbm_set_state and by calling this again.
 * every = 0 (the default) turns it off. Synchronous (waits for the stream,
 * allocates 8 bytes of pinned host memory the first time). Returns LBM_OK,
 * LBM_E_INVALID (every < 0) or LBM_E_DEVICE. */
int lbm_set_finite_check(lbm_ctx *ctx, int64_t every);

/* Wait for the context's stream and report the periodic check: LBM_OK, or
 * LBM_E_NONFINITE with *t_bad (host, may be NULL) the first checked time
 * whose state held NaN or Inf (-1 when none). Synchronous. */
int lbm_finite_status(lbm_ctx *ctx, int64_t *t_bad);

/* lbm_check_finite for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid hipMalloc): the same check and the same
 * results, with no hipMalloc, hipFree or allocating library call. Its flags
 * live in a static device array of 4096 + 2 words (16 KiB) that the library
 * holds on each GPU it runs on until the process ends: one flag per grid,
 * the count of non-finite grids and the first of them (named in
 * lbm_last_error). Each call clears what it uses first. Calls that overlap
 * on one GPU share the array and race; call it from one thread per GPU, with
 * the context's device current. Synchronous. Returns LBM_OK,
 * LBM_E_NONFINITE, LBM_E_INVALID (more than 4096 grids) or LBM_E_DEVICE. */
int lbm_check_finite_noalloc(lbm_ctx *ctx);

/* Launch configuration in use, and a way to set it (waves in {1,2,4,8},
 * rows >= 1, graph_chunk >= 0, prefetch in {1,2} (0 means 1), split, pair and
 * overlap in {0,1}, fuse_rows 0 or in [4, 248]). An odd graph_chunk is
 * rounded up to keep the ping-pong parity. The kernels reach a tile's rows
 * through one buffer descriptor with 32-bit byte offsets, so for every grid
 * (max(rows, 2) + 6) rows of nine population runs (9 x pitch x element size
 * bytes each) must stay within 2^31 - 1 bytes and, when fuse_rows > 0,
 * (fuse_rows + 8) rows within 2^32 - 1 bytes; the default launch and the
 * autotuner keep to this on their own.
 * Returns LBM_OK or LBM_E_INVALID (the configuration in use is kept). */
int lbm_get_launch(const lbm_ctx *ctx, lbm_launch *out);
int lbm_set_launch(lbm_ctx *ctx, const lbm_launch *cfg);

/* Time each candidate launch configuration on the live context (the state is
 * saved and restored, the time unchanged) and keep the fastest. On the
 * two-step path (fuse_rows > 0) the candidates are its block widths (waves
 * 2, 4, 8) and heights (fuse_rows 16 .. 64); otherwise the single-step tile
 * widths, heights, prefetch depths and column pairing. graph_chunk, split
 * and overlap stay as set. steps: timed steps per candidate (rounded up to
 * even on the two-step path); 0 takes the cached result for this context's
 * key if there is one, else tunes with 10 steps. Results are cached per GPU
 * architecture, dtype, boundary class (edge kinds, internal rigid row,
 * sources, receivers), powers of two of the total cells, tallest grid and
 * grid count, and path, for the process and, when the environment variable
 * LBM_TUNE_CACHE names a file, in that file (one line per result, appended).
 * The tuning runs record receiver rows of the times they reach, with the
 * values those steps produce. Synchronous; allocates a copy of the state
 * while it runs. Returns LBM_OK,
 * LBM_E_INVALID (steps < 0) or LBM_E_DEVICE (a HIP call failed, the copy's
 * allocation included; the previous configuration is reinstalled). */
int lbm_autotune(lbm_ctx *ctx, int32_t steps, lbm_launch *chosen);

/* ---- Discrete adjoint: gradients of a receiver misfit ------------------
 * With kappa, the sponge and the sources fixed, a step maps the pulled
 * populations f(t) linearly to f(t+1) (plus the source term) and the
 * receivers read v(t) = j(t)/rho0 linearly from f(t). For a misfit L of the
 * traces, the adjoint state fh(t) = dL/df(t) obeys
 *   fh(t) = step^T fh(t+1) + receivers^T e(t),  fh(T) = 0,  e(t) = dL/dv(t),
 * and the gradients accumulate along the way:
 *   dL/dkappa(x) = sum_t Gh(x,t) . grad(rho)(x,t),
 *   dL/damp_s    = sum_t sum_x Gh(x,t) . d_s gauss_s(x) ricker_s(t),
 * Gh = dL/dG being the adjoint of the source G = kappa grad(rho) + F (eq. S).
 * grad(rho)(t) is recomputed per segment of seg_steps steps from checkpoints
 * of the forward state taken while the forward run is recorded.
 * Usage: lbm_adjoint_begin at the run's start time t0 (checkpoint 0 is the
 * current state), lbm_step forward to t0 + nsteps (checkpoints are taken on
 * the way), set the residual and gradient buffers per grid, then
 * lbm_adjoint_step back towards t0. lbm_set_state ends the recording. */

/* Device workspace an adjoint run of nsteps steps with checkpoints every
 * seg_steps steps needs: ceil(nsteps/seg_steps) + 4 population buffers and
 * seg_steps density planes. Host only. */
int lbm_adjoint_workspace_bytes(const lbm_ctx *ctx, int32_t seg_steps, int64_t nsteps,
                                size_t *bytes);

/* Workspace of an adjoint run that also keeps in HBM the densities of its
 * last resident_steps steps, rounded down to whole trailing segments (the
 * last segment may be short): one plane of the grids' cells per step, written
 * by the recorded forward run. Those segments then need no recompute in
 * lbm_adjoint_step; the results are the same bit for bit. resident_steps = 0
 * gives lbm_adjoint_workspace_bytes. Host only. */
int lbm_adjoint_workspace_bytes_resident(const lbm_ctx *ctx, int32_t seg_steps, int64_t nsteps,
                                         int64_t resident_steps, size_t *bytes);

/* Open a recording of the forward run from the current time t0 for nsteps
 * steps. ws: caller-owned DEVICE memory, 256-B aligned, at least
 * lbm_adjoint_workspace_bytes, used exclusively by this context until the
 * next lbm_adjoint_begin or lbm_destroy; room beyond that minimum keeps the
 * densities of as many whole trailing segments as fit (see
 * lbm_adjoint_workspace_bytes_resident). The adjoint state starts at
 * t0 + nsteps with fh = 0. At most 16 sources per grid. The recording stays
 * open until the forward run reaches t0 + nsteps; meanwhile lbm_step_timed
 * and lbm_filter are refused. Asynchronous. */
int lbm_adjoint_begin(lbm_ctx *ctx, int32_t seg_steps, int64_t nsteps, void *ws, size_t ws_bytes);

/* Per-grid adjoint inputs and outputs (DEVICE pointers, caller-owned, any may
 * be NULL): residual e(t) in the layout of the grid's traces ([steps][n]
 * [ncomp] of dtype, row k = step trace_t0 + k); grad_kappa [ny][nx] FP64 and
 * grad_amp [nsrc] FP64, both accumulated into (the caller zeroes them). */
int lbm_adjoint_set_io(lbm_ctx *ctx, int32_t g, const void *residual, double *grad_kappa,
                       double *grad_amp);

/* n adjoint steps from the adjoint time t_a down to t_a - n (>= t0), for all
 * grids. The recorded forward run must have reached t0 + nsteps. Calls that
 * overlap on one stream are ordered; the gradient buffers must stay valid
 * until the work completes. With fuse_rows > 0 the steps go in pairs (t,
 * t-1) inside each checkpoint segment, like the forward's: the general
 * adjoint kernel takes step t of its tiles and of the two-step blocks'
 * border strips, the two-step adjoint kernel both steps of its blocks (no
 * receiver within three rows of their own rows) in one pass, the general
 * kernel step t-1 of its tiles; a step left alone at a segment's start runs
 * as a single step. Asynchronous. */
int lbm_adjoint_step(lbm_ctx *ctx, int64_t n);

/* lbm_adjoint_step with direct launches and a HIP event pair on the
 * context's stream around every adjoint-kernel launch: the mean launch
 * durations and cells covered go to *out (host; interior = the single-step
 * interior adjoint kernel, general = the general adjoint kernel, on the pair
 * path its tiles of one pair's step, fused = the two-step adjoint kernel,
 * whose cells advance two steps a launch). The recompute of a segment runs
 * untimed. The adjoint state and dL/dkappa equal those of lbm_adjoint_step
 * bit for bit (dL/damp up to the order of its FP64 atomic sums). Synchronous.
 * Errors as lbm_adjoint_step, and LBM_E_INVALID for a null out. */
int lbm_adjoint_step_timed(lbm_ctx *ctx, int64_t n, lbm_kernel_times *out);

int lbm_adjoint_time(const lbm_ctx *ctx, int64_t *t);

/* The adjoint state fh(t_a) = dL/df(t_a) of grid g, DEVICE [9][ny][nx] of
 * dtype in the direction order of lbm_get_state, out of / into the context.
 * Asynchronous. */
int lbm_adjoint_get_state(lbm_ctx *ctx, int32_t g, void *dst);
int lbm_adjoint_set_state(lbm_ctx *ctx, int32_t g, const void *src);

/* Residual and misfit of grid g's first nrows trace rows: residual = traces -
 * d_obs (DEVICE, traces' layout, dtype; residual may be NULL), *misfit +=
 * 1/2 sum residual^2 accumulated in FP64 (DEVICE double). Asynchronous. */
int lbm_misfit(lbm_ctx *ctx, int32_t g, const void *d_obs, void *residual, int64_t nrows,
               double *misfit);

/* dL/dlambda = -b^2 dL/dkappa / mu and dL/dmu = b^2 lambda dL/dkappa / mu^2
 * per cell (kappa = b^2 (mu - lambda)/mu, Sec. 4) for grid g, ADDED to
 * grad_lam and grad_mu (so shots sharing a medium accumulate): lam, mu DEVICE
 * [ny][nx] of dtype; grad_* DEVICE [ny][nx] FP64 (grad_lam or grad_mu may be
 * NULL). Asynchronous. */
int lbm_lame_gradient(lbm_ctx *ctx, int32_t g, const void *lam, const void *mu,
                      const double *grad_kappa, double *grad_lam, double *grad_mu);

/* Release the context's library-owned objects (device tables, graphs). Does
 * not touch caller-owned memory. Safe on NULL. */
int lbm_destroy(lbm_ctx *ctx);

/* Description of the last error on the calling thread ("" if none). */
const char *lbm_last_error(void);

int lbm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
