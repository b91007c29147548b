/*
 * lbm_oracle.c -- plain FP64 reference implementation of the single-relaxation-
 * time D2Q9 lattice Boltzmann scheme for elastic waves of Escande, Kolluru,
 * Cleon & Sagaut, "Lattice Boltzmann Method for wave propagation in elastic
 * solids with a regular lattice" (arXiv 2009.06404).
 *
 * TEST INFRASTRUCTURE. This file is the oracle against which the GPU library
 * is checked. It shares no code, header, table or helper with the GPU library.
 * Only the test-suite, the package smoke check and the CPU-baseline leg of the
 * benchmark load it; no product code path may call it.
 *
 * Form: the paper's own collide-then-push-stream form (eq. LBGK, Sec. 2), one
 * phase at a time over the whole grid, in double precision, with no blocking,
 * fusion or reordering: moments -> density gradient -> source -> flux and
 * sponge -> equilibrium and BGK collision -> receivers -> push streaming with
 * the wall rules of Sec. 6. OpenMP only splits each phase's loop over rows.
 * The discrete adjoint (oracle_adjoint, at the end of the file) transposes
 * each of these phases on its own and applies them in the reverse order.
 *
 * Conventions (readings of the paper, each listed in the design notes):
 *  - lattice: regular D2Q9, c = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),
 *    (-1,-1),(1,-1); weights 4/9, 1/9, 1/36; b^2 = 1/3 (Sec. 2, eq. isotropy);
 *  - grid: x = column (fast index), y = row, row 0 is the top edge, y grows
 *    with depth; cell (x, y) of plane i is f[i*nx*ny + y*nx + x];
 *  - populations are perturbations about the rest state f = 0;
 *  - j = sum f c + S/2 is the flux the equilibrium is built with (first moment
 *    of eq. MomentsFeq read together with the solvability conditions, Sec. 3);
 *  - elastic coefficient kappa = (mu - lambda)/rho0 with mu/rho0 = b^2, i.e.
 *    kappa = b^2 (1 - lambda/mu) (Lambda of Sec. 4 times b^2);
 *  - sponge term -A j treated as part of the source and solved implicitly:
 *    j = (m + G/2)/(1 + A/2), S = G - A j (eq. MomentChainAbsorbing, Sec. 6.4);
 *  - density gradient at a non-periodic edge or beside the internal rigid wall:
 *    linearly extrapolated ghost density 2 rho_b - rho_in in the centred
 *    difference of eq. FDrho;
 *  - free surface allowed on the top/bottom edges only; a link that crosses a
 *    rigid and a free edge at once (a corner) bounces back as rigid;
 *  - free-surface moments rho_b, rho_in, P_b, P_in are those of time t (the
 *    post-collision populations f_i(x_b, t) are the ones reflected).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* BC_FREE: the free surface of Sec. 6.2 with rho_air and P_xx,air linearly
 * extrapolated to the interface (as printed); BC_FREE0: the same rule with the
 * boundary cell's own rho and P_xx (zero-order extrapolation), a stabilised
 * variant -- the linear extrapolation makes short-wavelength surface modes
 * grow for every tau (spectral radius of the step > 1). */
enum { BC_PERIODIC = 0, BC_FREE = 1, BC_RIGID = 2, BC_FREE0 = 3 };
enum { EDGE_TOP = 0, EDGE_BOTTOM = 1, EDGE_LEFT = 2, EDGE_RIGHT = 3 };

/* D2Q9 lattice (Sec. 2): velocities, weights, opposite directions. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double B2 = 1.0 / 3.0; /* b^2, the lattice "sound speed" squared */

typedef struct {
  int32_t nx, ny;
  int32_t bc[4];        /* top, bottom, left, right: BC_* */
  int32_t rigid_row;    /* -1: none; else a rigid wall between rows r-1 and r */
  int32_t sp_thick[4];  /* sponge thickness per edge (cells) */
  double tau;           /* relaxation time (lattice units, dt = dx = 1) */
  const double *sp_prof[4]; /* sponge damping A[k], k = cells from the edge */
  int32_t nsrc;
  int32_t nrec;
  const double *src;    /* nsrc x 8: x, y, sigma, dir_x, dir_y, amp, period, t0 */
  const int32_t *rec_xy;/* nrec x 2: x, y */
  int32_t comp_mask;    /* bit 0: record v_x, bit 1: record v_y */
  int32_t pad_;
} oracle_cfg;

int oracle_abi_version(void) { return 1; }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel regions (both oracles); n < 1 is ignored. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void oracle_lattice(int32_t *cx, int32_t *cy, double *w, int32_t *opp) {
  for (int i = 0; i < 9; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    w[i] = WT[i];
    opp[i] = OPP[i];
  }
}

/* Elastic equilibrium, eq. equilibrium-solid with P^n = P - rho b^2 I (eq. Pn).
 * P = (P_xx, P_xy, P_yy). */
void oracle_equilibrium(double rho, const double j[2], const double P[3],
                        double feq[9]) {
  const double pn_xx = P[0] - rho * B2;
  const double pn_xy = P[1];
  const double pn_yy = P[2] - rho * B2;
  for (int i = 0; i < 9; ++i) {
    const double cx = CX[i], cy = CY[i];
    const double jc = j[0] * cx + j[1] * cy;
    const double pnq = pn_xx * (cx * cx - B2) + 2.0 * pn_xy * cx * cy +
                       pn_yy * (cy * cy - B2);
    feq[i] = WT[i] * (rho + jc / B2 + pnq / (2.0 * B2 * B2));
  }
}

/* One cell of the collision (Sec. 2, eqs. MomentsFeq, Si, LBGK and the sponge
 * of eq. MomentChainAbsorbing). f: pre-collision populations; G: the source
 * without the sponge, G = kappa * grad(rho) + F; A: sponge damping. Returns the
 * post-collision populations and the flux j and source S the cell used. */
void oracle_collide_cell(const double f[9], const double G[2], double A,
                         double tau, double fstar[9], double j_out[2],
                         double S_out[2]) {
  double rho = 0.0, mx = 0.0, my = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho += f[i];
    mx += f[i] * CX[i];
    my += f[i] * CY[i];
    pxx += f[i] * CX[i] * CX[i];
    pxy += f[i] * CX[i] * CY[i];
    pyy += f[i] * CY[i] * CY[i];
  }
  /* j = m + S/2 with S = G - A j, solved for j. */
  double j[2], S[2];
  j[0] = (mx + 0.5 * G[0]) / (1.0 + 0.5 * A);
  j[1] = (my + 0.5 * G[1]) / (1.0 + 0.5 * A);
  S[0] = G[0] - A * j[0];
  S[1] = G[1] - A * j[1];
  const double P[3] = {pxx, pxy, pyy};
  double feq[9];
  oracle_equilibrium(rho, j, P, feq);
  for (int i = 0; i < 9; ++i) {
    const double Si = WT[i] * (CX[i] * S[0] + CY[i] * S[1]) / B2; /* eq. Si */
    fstar[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * Si;
  }
  if (j_out) { j_out[0] = j[0]; j_out[1] = j[1]; }
  if (S_out) { S_out[0] = S[0]; S_out[1] = S[1]; }
}

/* Ricker wavelet with peak frequency 1/period, centred at t0 (Sec. 5). */
static double ricker(double t, double period, double t0) {
  const double a = M_PI * (t - t0) / period;
  return (1.0 - 2.0 * a * a) * exp(-a * a);
}

typedef struct {
  const oracle_cfg *c;
  int nx, ny;
  size_t N;
  double *kappa;   /* per cell */
  double *A;       /* sponge damping per cell */
  double *inv_rho0_rec; /* 1/rho0 at each receiver */
  /* per-phase work planes */
  double *rho, *mx, *my, *pxx, *pxy, *pyy;
  double *dxr, *dyr;
  double *Gx, *Gy, *jx, *jy;
} oracle_grid;

/* Sponge damping A(x, y): the largest of the edge profiles that reach the cell
 * (Sec. 6.4; the profile itself is an input). */
static void build_sponge(oracle_grid *g) {
  const oracle_cfg *c = g->c;
  for (int y = 0; y < g->ny; ++y)
    for (int x = 0; x < g->nx; ++x) {
      const int d[4] = {y, g->ny - 1 - y, x, g->nx - 1 - x};
      double a = 0.0;
      for (int e = 0; e < 4; ++e)
        if (c->sp_thick[e] > 0 && d[e] < c->sp_thick[e]) {
          const double v = c->sp_prof[e][d[e]];
          if (v > a) a = v;
        }
      g->A[(size_t)y * g->nx + x] = a;
    }
}

/* Step 1: moments of f (eq. MomentsFeq; P is the second moment). */
static void phase_moments(oracle_grid *g, const double *f) {
  const size_t N = g->N;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < g->ny; ++y)
    for (int x = 0; x < g->nx; ++x) {
      const size_t k = (size_t)y * g->nx + x;
      double rho = 0, mx = 0, my = 0, pxx = 0, pxy = 0, pyy = 0;
      for (int i = 0; i < 9; ++i) {
        const double fi = f[i * N + k];
        rho += fi;
        mx += fi * CX[i];
        my += fi * CY[i];
        pxx += fi * CX[i] * CX[i];
        pxy += fi * CX[i] * CY[i];
        pyy += fi * CY[i] * CY[i];
      }
      g->rho[k] = rho; g->mx[k] = mx; g->my[k] = my;
      g->pxx[k] = pxx; g->pxy[k] = pxy; g->pyy[k] = pyy;
    }
}

/* Neighbour density across x, or a linearly extrapolated ghost where the
 * neighbour lies outside a non-periodic edge. dir = -1 (left) or +1 (right). */
static double rho_x_neighbour(const oracle_grid *g, int x, int y, int dir) {
  const int nx = g->nx;
  int xn = x + dir;
  const double *r = g->rho + (size_t)y * nx;
  if (xn < 0 || xn >= nx) {
    const int edge = (xn < 0) ? EDGE_LEFT : EDGE_RIGHT;
    if (g->c->bc[edge] == BC_PERIODIC) {
      xn = (xn + nx) % nx;
    } else {
      return 2.0 * r[x] - r[x - dir]; /* ghost: 2 rho_b - rho_in */
    }
  }
  return r[xn];
}

static double rho_y_neighbour(const oracle_grid *g, int x, int y, int dir) {
  const int nx = g->nx, ny = g->ny;
  const int rr = g->c->rigid_row;
  int yn = y + dir;
  int wall = 0;
  if (yn < 0 || yn >= ny) {
    const int edge = (yn < 0) ? EDGE_TOP : EDGE_BOTTOM;
    if (g->c->bc[edge] == BC_PERIODIC)
      yn = (yn + ny) % ny;
    else
      wall = 1;
  } else if (rr > 0 && ((dir > 0 && y == rr - 1) || (dir < 0 && y == rr))) {
    wall = 1; /* no finite-difference coupling across the internal rigid wall */
  }
  if (wall)
    return 2.0 * g->rho[(size_t)y * nx + x] - g->rho[(size_t)(y - dir) * nx + x];
  return g->rho[(size_t)yn * nx + x];
}

/* Step 2: centred finite-difference density gradient, eq. FDrho. */
static void phase_density_gradient(oracle_grid *g) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < g->ny; ++y)
    for (int x = 0; x < g->nx; ++x) {
      const size_t k = (size_t)y * g->nx + x;
      g->dxr[k] = 0.5 * (rho_x_neighbour(g, x, y, +1) - rho_x_neighbour(g, x, y, -1));
      g->dyr[k] = 0.5 * (rho_y_neighbour(g, x, y, +1) - rho_y_neighbour(g, x, y, -1));
    }
}

/* Minimum-image offset along a periodic axis. */
static double min_image(double d, int n, int periodic) {
  if (!periodic) return d;
  while (d > 0.5 * n) d -= n;
  while (d < -0.5 * n) d += n;
  return d;
}

/* Step 3: source G = kappa * grad(rho) + F (eq. S), F the Gaussian-in-space,
 * Ricker-in-time body force of Sec. 5, cut to zero beyond 9 sigma. */
static void phase_source(oracle_grid *g, int64_t t) {
  const oracle_cfg *c = g->c;
  const int px = c->bc[EDGE_LEFT] == BC_PERIODIC;
  const int py = c->bc[EDGE_TOP] == BC_PERIODIC;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < g->ny; ++y)
    for (int x = 0; x < g->nx; ++x) {
      const size_t k = (size_t)y * g->nx + x;
      double Fx = 0.0, Fy = 0.0;
      for (int s = 0; s < c->nsrc; ++s) {
        const double *p = c->src + 8 * s;
        const double dx = min_image(x - p[0], g->nx, px);
        const double dy = min_image(y - p[1], g->ny, py);
        const double r2 = dx * dx + dy * dy;
        const double sig = p[2];
        if (r2 > 81.0 * sig * sig) continue;
        const double mag = p[5] * exp(-r2 / (2.0 * sig * sig)) * ricker((double)t, p[6], p[7]);
        Fx += mag * p[3];
        Fy += mag * p[4];
      }
      g->Gx[k] = g->kappa[k] * g->dxr[k] + Fx;
      g->Gy[k] = g->kappa[k] * g->dyr[k] + Fy;
    }
}

/* Steps 4-6: flux, sponge-corrected source, equilibrium and BGK collision. */
static void phase_collide(oracle_grid *g, const double *f, double *fstar) {
  const size_t N = g->N;
  const double tau = g->c->tau;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < g->ny; ++y)
    for (int x = 0; x < g->nx; ++x) {
      const size_t k = (size_t)y * g->nx + x;
      double fc[9], fs[9], j[2];
      for (int i = 0; i < 9; ++i) fc[i] = f[i * N + k];
      const double G[2] = {g->Gx[k], g->Gy[k]};
      oracle_collide_cell(fc, G, g->A[k], tau, fs, j, NULL);
      for (int i = 0; i < 9; ++i) fstar[i * N + k] = fs[i];
      g->jx[k] = j[0];
      g->jy[k] = j[1];
    }
}

/* Step 7: receivers record v = j / rho0 at their cells (Sec. 5 seismogram). */
static void phase_receivers(oracle_grid *g, double *row) {
  const oracle_cfg *c = g->c;
  int ncomp = ((c->comp_mask & 1) ? 1 : 0) + ((c->comp_mask & 2) ? 1 : 0);
  for (int r = 0; r < c->nrec; ++r) {
    const size_t k = (size_t)c->rec_xy[2 * r + 1] * g->nx + c->rec_xy[2 * r];
    int o = 0;
    if (c->comp_mask & 1) row[r * ncomp + o++] = g->jx[k] * g->inv_rho0_rec[r];
    if (c->comp_mask & 2) row[r * ncomp + o++] = g->jy[k] * g->inv_rho0_rec[r];
  }
}

/* Free-surface anti-bounce-back value for a link leaving cell (x, y) through
 * the top or bottom edge (Sec. 6.2): -f*_i + 2 w_i (rho_air + P^n_air :
 * (c_i c_i - b^2 I) / (2 b^4)), with rho_air and the tangential stress P_xx,air
 * linearly extrapolated from the boundary cell and the cell inside it, and the
 * normal rows of P_air zero (P_air n = 0). */
static double free_surface_value(const oracle_grid *g, int x, int y, int i,
                                 int normal_y, int order, double fstar_i) {
  const int nx = g->nx;
  const size_t kb = (size_t)y * nx + x;
  const size_t kin = (size_t)(y - normal_y) * nx + x;
  /* interface half a cell outside x_b: linear extrapolation from x_b and x_in
   * (order 1, as printed), or the boundary cell's value (order 0) */
  const double cb = order ? 1.5 : 1.0, cin = order ? -0.5 : 0.0;
  const double rho_air = cb * g->rho[kb] + cin * g->rho[kin];
  const double pxx_air = cb * g->pxx[kb] + cin * g->pxx[kin];
  const double pn_xx = pxx_air - B2 * rho_air;
  const double pn_xy = 0.0;
  const double pn_yy = 0.0 - B2 * rho_air;
  const double cx = CX[i], cy = CY[i];
  const double pnq = pn_xx * (cx * cx - B2) + 2.0 * pn_xy * cx * cy + pn_yy * (cy * cy - B2);
  return -fstar_i + 2.0 * WT[i] * (rho_air + pnq / (2.0 * B2 * B2));
}

/* Step 8: push streaming f_i(x + c_i, t + 1) = f*_i(x, t) (left side of eq.
 * LBGK), periodic wrap on periodic edges, halfway bounce-back on rigid walls
 * (eq. BB, full reversal of c_i) and anti-bounce-back on free surfaces. */
static void phase_stream(oracle_grid *g, const double *fstar, double *fnext) {
  const oracle_cfg *c = g->c;
  const int nx = g->nx, ny = g->ny, rr = c->rigid_row;
  const size_t N = g->N;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const size_t k = (size_t)y * nx + x;
      for (int i = 0; i < 9; ++i) {
        int xd = x + CX[i], yd = y + CY[i];
        int rigid = 0, free_ny = 0; /* free_ny: outward normal y of a free edge */
        int order = 1;
        if (yd < 0 || yd >= ny) {
          const int edge = (yd < 0) ? EDGE_TOP : EDGE_BOTTOM;
          if (c->bc[edge] == BC_PERIODIC) yd = (yd + ny) % ny;
          else if (c->bc[edge] == BC_RIGID) rigid = 1;
          else {
            free_ny = (yd < 0) ? -1 : +1;
            order = c->bc[edge] == BC_FREE ? 1 : 0;
          }
        } else if (rr > 0 && ((CY[i] > 0 && y == rr - 1) || (CY[i] < 0 && y == rr))) {
          rigid = 1;
        }
        if (xd < 0 || xd >= nx) {
          const int edge = (xd < 0) ? EDGE_LEFT : EDGE_RIGHT;
          if (c->bc[edge] == BC_PERIODIC) xd = (xd + nx) % nx;
          else rigid = 1; /* left/right edges are periodic or rigid */
        }
        const double fs = fstar[i * N + k];
        if (rigid) {
          fnext[OPP[i] * N + k] = fs;
        } else if (free_ny != 0) {
          fnext[OPP[i] * N + k] = free_surface_value(g, x, y, i, free_ny, order, fs);
        } else {
          fnext[i * N + (size_t)yd * nx + xd] = fs;
        }
      }
    }
}

static int grid_alloc(oracle_grid *g, const oracle_cfg *c, const double *lam,
                      const double *mu, const double *rho0) {
  memset(g, 0, sizeof(*g));
  g->c = c;
  g->nx = c->nx;
  g->ny = c->ny;
  g->N = (size_t)c->nx * c->ny;
  double **planes[] = {&g->kappa, &g->A,   &g->rho, &g->mx, &g->my, &g->pxx,
                       &g->pxy,   &g->pyy, &g->dxr, &g->dyr, &g->Gx, &g->Gy,
                       &g->jx,    &g->jy};
  for (size_t p = 0; p < sizeof(planes) / sizeof(planes[0]); ++p) {
    *planes[p] = (double *)calloc(g->N, sizeof(double));
    if (!*planes[p]) return -2;
  }
  g->inv_rho0_rec = (double *)calloc(c->nrec > 0 ? c->nrec : 1, sizeof(double));
  if (!g->inv_rho0_rec) return -2;
  /* kappa = (mu - lambda)/rho0 in lattice units, mu/rho0 = b^2 (Sec. 4). */
  for (size_t k = 0; k < g->N; ++k) g->kappa[k] = B2 * (mu[k] - lam[k]) / mu[k];
  for (int r = 0; r < c->nrec; ++r) {
    const size_t k = (size_t)c->rec_xy[2 * r + 1] * c->nx + c->rec_xy[2 * r];
    g->inv_rho0_rec[r] = 1.0 / rho0[k];
  }
  build_sponge(g);
  return 0;
}

static void grid_free(oracle_grid *g) {
  double *planes[] = {g->kappa, g->A,   g->rho, g->mx, g->my, g->pxx, g->pxy,
                      g->pyy,   g->dxr, g->dyr, g->Gx, g->Gy, g->jx,  g->jy};
  for (size_t p = 0; p < sizeof(planes) / sizeof(planes[0]); ++p) free(planes[p]);
  free(g->inv_rho0_rec);
}

/* Run nsteps time steps starting at time t0.
 *   init:       initial populations (9 planes), or NULL for the rest state
 *               f = 0 at t0;
 *   init_kind:  0: init holds the post-collision populations at t0-1,
 *               1: init holds the pre-collision populations at t0;
 *   fstar_out:  post-collision populations at t0+nsteps-1 (may be NULL);
 *   f_out:      pre-collision populations at t0+nsteps (may be NULL);
 *   mom_out:    rho, j_x, j_y, P_xx, P_xy, P_yy at t0+nsteps (may be NULL);
 *   trace:      receiver traces [nsteps][nrec][ncomp] (may be NULL).
 * Returns 0, or -2 when memory runs out. */
int oracle_run(const oracle_cfg *c, const double *lam, const double *mu,
               const double *rho0, const double *init, int32_t init_kind, int64_t t0,
               int64_t nsteps, double *fstar_out, double *f_out,
               double *mom_out, double *trace) {
  oracle_grid g;
  if (grid_alloc(&g, c, lam, mu, rho0) != 0) { grid_free(&g); return -2; }
  const size_t N = g.N;
  double *f = (double *)calloc(9 * N, sizeof(double));
  double *fs = (double *)calloc(9 * N, sizeof(double));
  if (!f || !fs) { free(f); free(fs); grid_free(&g); return -2; }
  const int ncomp = ((c->comp_mask & 1) ? 1 : 0) + ((c->comp_mask & 2) ? 1 : 0);

  if (init && init_kind == 0) {
    /* f(t0) = stream(f*(t0-1)); the free-surface rule needs rho, P at t0-1,
     * which are the moments of f*(t0-1) (collision invariants, Sec. 3). */
    memcpy(fs, init, 9 * N * sizeof(double));
    phase_moments(&g, fs);
    phase_stream(&g, fs, f);
  } else if (init) {
    memcpy(f, init, 9 * N * sizeof(double));
  }
  for (int64_t n = 0; n < nsteps; ++n) {
    const int64_t t = t0 + n;
    phase_moments(&g, f);
    phase_density_gradient(&g);
    phase_source(&g, t);
    phase_collide(&g, f, fs);
    if (trace && c->nrec > 0) phase_receivers(&g, trace + (size_t)n * c->nrec * ncomp);
    phase_stream(&g, fs, f); /* uses rho, P of step 1 for the free surface */
  }
  if (fstar_out) memcpy(fstar_out, fs, 9 * N * sizeof(double));
  if (f_out) memcpy(f_out, f, 9 * N * sizeof(double));
  if (mom_out) {
    /* Macroscopic fields at t0+nsteps: steps 1-4 without the collision. */
    const int64_t t = t0 + nsteps;
    phase_moments(&g, f);
    phase_density_gradient(&g);
    phase_source(&g, t);
    for (size_t k = 0; k < N; ++k) {
      const double A = g.A[k];
      mom_out[0 * N + k] = g.rho[k];
      mom_out[1 * N + k] = (g.mx[k] + 0.5 * g.Gx[k]) / (1.0 + 0.5 * A);
      mom_out[2 * N + k] = (g.my[k] + 0.5 * g.Gy[k]) / (1.0 + 0.5 * A);
      mom_out[3 * N + k] = g.pxx[k];
      mom_out[4 * N + k] = g.pxy[k];
      mom_out[5 * N + k] = g.pyy[k];
    }
  }
  free(f);
  free(fs);
  grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ *
 * Discrete adjoint of the step above.
 *
 * With kappa, the sponge and the sources fixed, one step maps the populations
 * f(t) to f(t+1) linearly (plus the source term) and the receivers read a
 * linear function of f(t). For the misfit L = 1/2 sum_t sum_r |v_r(t) -
 * d_r(t)|^2 the adjoint populations fh(t) = dL/df(t) obey
 *     fh(t) = (step)^T fh(t+1) + (receivers)^T e(t),   fh(T) = 0,
 * with e = v - d the trace residual. Each phase of the forward step is
 * transposed here on its own and applied in the reverse order:
 *   push streaming^T  -> receivers^T -> collision, flux and sponge^T ->
 *   source^T (gradients) -> density gradient^T -> moments^T.
 * The gradients follow from the same sweep: G = kappa grad(rho) + F, so
 *   dL/dkappa(x) = sum_t Gh(x, t) . grad(rho)(x, t),
 *   dL/damp_s    = sum_t sum_x Gh(x, t) . d_s gauss_s(x) ricker_s(t).
 * grad(rho)(t) comes from a forward run kept whole in memory (one rho plane
 * per step), which suits the small grids this oracle is used on.
 * ------------------------------------------------------------------------ */

typedef struct {
  double *rho, *mx, *my, *pxx, *pxy, *pyy; /* adjoints of the moments of f(t) */
  double *Gx, *Gy, *jx, *jy;               /* adjoints of G and of j */
  double *fstar;                           /* adjoint of f*(t), 9 planes */
} oracle_adj;

/* Transpose of phase_stream: fstar_h_i(x) gathers fh_i(x + c_i) through the
 * same link classification; the free-surface values add their rho_air and
 * P_xx,air sensitivities to the moment adjoints of rows b and in. */
static void adj_stream(const oracle_grid *g, const double *fh_next, oracle_adj *a) {
  const oracle_cfg *c = g->c;
  const int nx = g->nx, ny = g->ny, rr = c->rigid_row;
  const size_t N = g->N;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const size_t k = (size_t)y * nx + x;
      for (int i = 0; i < 9; ++i) {
        int xd = x + CX[i], yd = y + CY[i];
        int rigid = 0, free_ny = 0, order = 1;
        if (yd < 0 || yd >= ny) {
          const int edge = (yd < 0) ? EDGE_TOP : EDGE_BOTTOM;
          if (c->bc[edge] == BC_PERIODIC) yd = (yd + ny) % ny;
          else if (c->bc[edge] == BC_RIGID) rigid = 1;
          else {
            free_ny = (yd < 0) ? -1 : +1;
            order = c->bc[edge] == BC_FREE ? 1 : 0;
          }
        } else if (rr > 0 && ((CY[i] > 0 && y == rr - 1) || (CY[i] < 0 && y == rr))) {
          rigid = 1;
        }
        if (xd < 0 || xd >= nx) {
          const int edge = (xd < 0) ? EDGE_LEFT : EDGE_RIGHT;
          if (c->bc[edge] == BC_PERIODIC) xd = (xd + nx) % nx;
          else rigid = 1;
        }
        if (rigid) {
          a->fstar[i * N + k] += fh_next[OPP[i] * N + k];
        } else if (free_ny != 0) {
          /* value = -f*_i + 2 w_i (rho_air + P^n_air : Q_i / (2 b^4)) */
          const double gh = fh_next[OPP[i] * N + k];
          const double cx = CX[i], cy = CY[i];
          a->fstar[i * N + k] += -gh;
          const double d_rho_air =
              2.0 * WT[i] * (1.0 + (-B2 * (cx * cx - B2) - B2 * (cy * cy - B2)) / (2.0 * B2 * B2));
          const double d_pxx_air = 2.0 * WT[i] * (cx * cx - B2) / (2.0 * B2 * B2);
          const double cb = order ? 1.5 : 1.0, cin = order ? -0.5 : 0.0;
          const size_t kb = k, kin = (size_t)(y - free_ny) * nx + x;
          a->rho[kb] += cb * d_rho_air * gh;
          a->rho[kin] += cin * d_rho_air * gh;
          a->pxx[kb] += cb * d_pxx_air * gh;
          a->pxx[kin] += cin * d_pxx_air * gh;
        } else {
          a->fstar[i * N + k] += fh_next[i * N + (size_t)yd * nx + xd];
        }
      }
    }
}

/* Transpose of phase_receivers: v = j / rho0 at each receiver. */
static void adj_receivers(const oracle_grid *g, const double *row, oracle_adj *a) {
  const oracle_cfg *c = g->c;
  const int ncomp = ((c->comp_mask & 1) ? 1 : 0) + ((c->comp_mask & 2) ? 1 : 0);
  for (int r = 0; r < c->nrec; ++r) {
    const size_t k = (size_t)c->rec_xy[2 * r + 1] * g->nx + c->rec_xy[2 * r];
    int o = 0;
    if (c->comp_mask & 1) a->jx[k] += row[r * ncomp + o++] * g->inv_rho0_rec[r];
    if (c->comp_mask & 2) a->jy[k] += row[r * ncomp + o++] * g->inv_rho0_rec[r];
  }
}

/* Transpose of oracle_collide_cell for one cell: from the adjoint of f* (and
 * of j from the receivers) to the adjoints of f (direct part), rho, m, P, G. */
static void adj_collide_cell(const double fsh[9], double A, double tau, double jh_rec[2],
                             double fh[9], double *rh, double mh[2], double ph[3],
                             double Gh[2]) {
  const double cF = 1.0 - 1.0 / (2.0 * tau);
  double jh[2] = {jh_rec[0], jh_rec[1]};
  double Sh[2] = {0.0, 0.0};
  double r = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0;
  for (int i = 0; i < 9; ++i) {
    const double cx = CX[i], cy = CY[i];
    /* f*_i = f_i - (f_i - feq_i)/tau + cF Si */
    fh[i] = (1.0 - 1.0 / tau) * fsh[i];
    const double eh = fsh[i] / tau;             /* adjoint of feq_i */
    const double sih = cF * fsh[i];             /* adjoint of Si */
    /* Si = w_i c_i . S / b^2 */
    Sh[0] += sih * WT[i] * cx / B2;
    Sh[1] += sih * WT[i] * cy / B2;
    /* feq_i = w_i (rho + j.c/b^2 + P^n:Q_i/(2 b^4)), P^n = P - rho b^2 I */
    const double qxx = (cx * cx - B2) / (2.0 * B2 * B2);
    const double qxy = 2.0 * cx * cy / (2.0 * B2 * B2);
    const double qyy = (cy * cy - B2) / (2.0 * B2 * B2);
    r += eh * WT[i] * (1.0 - B2 * qxx - B2 * qyy);
    jh[0] += eh * WT[i] * cx / B2;
    jh[1] += eh * WT[i] * cy / B2;
    pxx += eh * WT[i] * qxx;
    pxy += eh * WT[i] * qxy;
    pyy += eh * WT[i] * qyy;
  }
  const double inv = 1.0 / (1.0 + 0.5 * A);
  for (int d = 0; d < 2; ++d) {
    /* S = G - A j */
    Gh[d] = Sh[d];
    jh[d] -= A * Sh[d];
    /* j = (m + G/2) / (1 + A/2) */
    mh[d] = jh[d] * inv;
    Gh[d] += 0.5 * jh[d] * inv;
  }
  *rh = r;
  ph[0] = pxx;
  ph[1] = pxy;
  ph[2] = pyy;
}

/* Transpose of rho_x_neighbour / rho_y_neighbour: spread weight w of the
 * neighbour density (or of its ghost 2 rho_b - rho_in) back onto rho. */
static void adj_rho_x_neighbour(const oracle_grid *g, int x, int y, int dir, double w,
                                double *rh) {
  const int nx = g->nx;
  int xn = x + dir;
  double *r = rh + (size_t)y * nx;
  if (xn < 0 || xn >= nx) {
    const int edge = (xn < 0) ? EDGE_LEFT : EDGE_RIGHT;
    if (g->c->bc[edge] == BC_PERIODIC) {
      xn = (xn + nx) % nx;
    } else {
      r[x] += 2.0 * w;
      r[x - dir] -= w;
      return;
    }
  }
  r[xn] += w;
}

static void adj_rho_y_neighbour(const oracle_grid *g, int x, int y, int dir, double w,
                                double *rh) {
  const int nx = g->nx, ny = g->ny;
  const int rr = g->c->rigid_row;
  int yn = y + dir;
  int wall = 0;
  if (yn < 0 || yn >= ny) {
    const int edge = (yn < 0) ? EDGE_TOP : EDGE_BOTTOM;
    if (g->c->bc[edge] == BC_PERIODIC)
      yn = (yn + ny) % ny;
    else
      wall = 1;
  } else if (rr > 0 && ((dir > 0 && y == rr - 1) || (dir < 0 && y == rr))) {
    wall = 1;
  }
  if (wall) {
    rh[(size_t)y * nx + x] += 2.0 * w;
    rh[(size_t)(y - dir) * nx + x] -= w;
    return;
  }
  rh[(size_t)yn * nx + x] += w;
}

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* Run the forward from t0 for nsteps steps (as oracle_run), then the adjoint
 * back to t0.
 *   residual:   e(t) for t = t0 .. t0+nsteps-1, layout of the traces
 *               [nsteps][nrec][ncomp], or NULL (zero);
 *   adj_init:   fh(t0+nsteps), 9 planes, or NULL (zero);
 *   adj_out:    fh(t0), 9 planes (may be NULL);
 *   grad_kappa: N values, dL/dkappa added in;
 *   grad_amp:   nsrc values, dL/damp added in;
 *   trace_out:  the forward traces (may be NULL).
 * Returns 0, or -2 when memory runs out. */
int oracle_adjoint(const oracle_cfg *c, const double *lam, const double *mu,
                   const double *rho0, const double *init, int32_t init_kind, int64_t t0,
                   int64_t nsteps, const double *residual, const double *adj_init,
                   double *adj_out, double *grad_kappa, double *grad_amp,
                   double *trace_out) {
  oracle_grid g;
  if (grid_alloc(&g, c, lam, mu, rho0) != 0) { grid_free(&g); return -2; }
  const size_t N = g.N;
  const int ncomp = ((c->comp_mask & 1) ? 1 : 0) + ((c->comp_mask & 2) ? 1 : 0);
  double *f = zalloc(9 * N), *fs = zalloc(9 * N);
  double *rho_hist = zalloc((size_t)(nsteps > 0 ? nsteps : 1) * N);
  double *fh = zalloc(9 * N), *fh_next = zalloc(9 * N);
  oracle_adj a;
  a.rho = zalloc(N); a.mx = zalloc(N); a.my = zalloc(N);
  a.pxx = zalloc(N); a.pxy = zalloc(N); a.pyy = zalloc(N);
  a.Gx = zalloc(N); a.Gy = zalloc(N); a.jx = zalloc(N); a.jy = zalloc(N);
  a.fstar = zalloc(9 * N);
  double *dxh = zalloc(N), *dyh = zalloc(N);
  int rc = 0;
  if (!f || !fs || !rho_hist || !fh || !fh_next || !a.rho || !a.mx || !a.my || !a.pxx ||
      !a.pxy || !a.pyy || !a.Gx || !a.Gy || !a.jx || !a.jy || !a.fstar || !dxh || !dyh) {
    rc = -2;
    goto done;
  }

  /* forward, keeping rho(t) of every step */
  if (init && init_kind == 0) {
    memcpy(fs, init, 9 * N * sizeof(double));
    phase_moments(&g, fs);
    phase_stream(&g, fs, f);
  } else if (init) {
    memcpy(f, init, 9 * N * sizeof(double));
  }
  for (int64_t n = 0; n < nsteps; ++n) {
    const int64_t t = t0 + n;
    phase_moments(&g, f);
    memcpy(rho_hist + (size_t)n * N, g.rho, N * sizeof(double));
    phase_density_gradient(&g);
    phase_source(&g, t);
    phase_collide(&g, f, fs);
    if (trace_out && c->nrec > 0) phase_receivers(&g, trace_out + (size_t)n * c->nrec * ncomp);
    phase_stream(&g, fs, f);
  }

  /* adjoint, t = t0+nsteps-1 down to t0 */
  if (adj_init) memcpy(fh_next, adj_init, 9 * N * sizeof(double));
  if (nsteps == 0) memcpy(fh, fh_next, 9 * N * sizeof(double));
  for (int64_t n = nsteps - 1; n >= 0; --n) {
    const int64_t t = t0 + n;
    double *planes[] = {a.rho, a.mx, a.my, a.pxx, a.pxy, a.pyy, a.Gx, a.Gy, a.jx, a.jy};
    for (size_t p = 0; p < sizeof(planes) / sizeof(planes[0]); ++p)
      memset(planes[p], 0, N * sizeof(double));
    memset(a.fstar, 0, 9 * N * sizeof(double));
    /* the forward quantities of step t that the gradients need */
    memcpy(g.rho, rho_hist + (size_t)n * N, N * sizeof(double));
    phase_density_gradient(&g);

    adj_stream(&g, fh_next, &a);
    if (residual && c->nrec > 0) adj_receivers(&g, residual + (size_t)n * c->nrec * ncomp, &a);
    for (size_t k = 0; k < N; ++k) {
      double fsh[9], fhc[9], mh[2], ph[3], Gh[2], rh;
      double jh[2] = {a.jx[k], a.jy[k]};
      for (int i = 0; i < 9; ++i) fsh[i] = a.fstar[i * N + k];
      adj_collide_cell(fsh, g.A[k], c->tau, jh, fhc, &rh, mh, ph, Gh);
      for (int i = 0; i < 9; ++i) fh[i * N + k] = fhc[i];
      a.rho[k] += rh;
      a.mx[k] += mh[0];
      a.my[k] += mh[1];
      a.pxx[k] += ph[0];
      a.pxy[k] += ph[1];
      a.pyy[k] += ph[2];
      a.Gx[k] = Gh[0];
      a.Gy[k] = Gh[1];
    }
    /* source^T: G = kappa grad(rho) + F */
    const int px = c->bc[EDGE_LEFT] == BC_PERIODIC;
    const int py = c->bc[EDGE_TOP] == BC_PERIODIC;
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const size_t k = (size_t)y * g.nx + x;
        if (grad_kappa) grad_kappa[k] += a.Gx[k] * g.dxr[k] + a.Gy[k] * g.dyr[k];
        dxh[k] = g.kappa[k] * a.Gx[k];
        dyh[k] = g.kappa[k] * a.Gy[k];
        for (int s = 0; s < c->nsrc && grad_amp; ++s) {
          const double *p = c->src + 8 * s;
          const double dx = min_image(x - p[0], g.nx, px);
          const double dy = min_image(y - p[1], g.ny, py);
          const double r2 = dx * dx + dy * dy;
          const double sig = p[2];
          if (r2 > 81.0 * sig * sig) continue;
          const double unit = exp(-r2 / (2.0 * sig * sig)) * ricker((double)t, p[6], p[7]);
          grad_amp[s] += unit * (a.Gx[k] * p[3] + a.Gy[k] * p[4]);
        }
      }
    /* density gradient^T: D_x rho = (N(+1) - N(-1)) / 2, the same for y */
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const size_t k = (size_t)y * g.nx + x;
        adj_rho_x_neighbour(&g, x, y, +1, 0.5 * dxh[k], a.rho);
        adj_rho_x_neighbour(&g, x, y, -1, -0.5 * dxh[k], a.rho);
        adj_rho_y_neighbour(&g, x, y, +1, 0.5 * dyh[k], a.rho);
        adj_rho_y_neighbour(&g, x, y, -1, -0.5 * dyh[k], a.rho);
      }
    /* moments^T */
    for (size_t k = 0; k < N; ++k)
      for (int i = 0; i < 9; ++i) {
        const double cx = CX[i], cy = CY[i];
        fh[i * N + k] += a.rho[k] + a.mx[k] * cx + a.my[k] * cy + a.pxx[k] * cx * cx +
                         a.pxy[k] * cx * cy + a.pyy[k] * cy * cy;
      }
    double *tmp = fh_next;
    fh_next = fh;
    fh = tmp;
  }
  if (adj_out) memcpy(adj_out, nsteps > 0 ? fh_next : fh, 9 * N * sizeof(double));

done:
  free(f); free(fs); free(rho_hist); free(fh); free(fh_next);
  free(a.rho); free(a.mx); free(a.my); free(a.pxx); free(a.pxy); free(a.pyy);
  free(a.Gx); free(a.Gy); free(a.jx); free(a.jy); free(a.fstar);
  free(dxh); free(dyh);
  grid_free(&g);
  return rc;
}
