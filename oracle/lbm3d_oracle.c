/*
 * lbm3d_oracle.c -- plain FP64 reference implementation of the elastic-wave
 * lattice Boltzmann step on the regular three-dimensional D3Q19 and D3Q27
 * lattices, the extension the paper's Chapman-Enskog analysis covers for
 * regular lattices (Sec. 3: the isotropy conditions hold for D2Q9, D3Q15,
 * D3Q19 and D3Q27).
 *
 * TEST INFRASTRUCTURE. This file is the oracle against which the GPU library's
 * three-dimensional path is checked. It shares no code, header, table or
 * helper with the GPU library (nor with the two-dimensional oracle beside it).
 * Only the test-suite, the package smoke check and the CPU-baseline leg of the
 * benchmark load it; no product code path may call it.
 *
 * Form: the paper's collide-then-push-stream form (eq. LBGK, Sec. 2), one
 * phase at a time over the whole volume, in double precision, with no
 * blocking, fusion or reordering: moments -> density gradient -> source ->
 * flux and sponge -> equilibrium and BGK collision -> receivers -> push
 * streaming with the wall rules of Sec. 6 applied face by face. OpenMP only
 * splits each phase's loop.
 *
 * Conventions (readings of the paper in three dimensions):
 *  - lattices: D3Q19, the rest vector, the 6 axis vectors and the 12 edge
 *    vectors (+-1 on two axes), weights 1/3, 1/18, 1/36; D3Q27, those and
 *    the 8 corner vectors (+-1 on every axis), weights 8/27, 2/27, 1/54,
 *    1/216; b^2 = 1/3 for both. The order is the rest vector, then the pairs
 *    (+x,-x), (+y,-y), (+z,-z), (x+y), (-x-y), (x-y), (-x+y), (x+z), (-x-z),
 *    (x-z), (-x+z), (y+z), (-y-z), (y-z), (-y+z), and for D3Q27 (x+y+z),
 *    (-x-y-z), (x+y-z), (-x-y+z), (x-y+z), (-x+y-z), (-x+y+z), (x-y-z), so
 *    that the opposite of vector 2k-1 is 2k;
 *  - volume: x fastest, then y, then z; z = 0 is the top face and z grows
 *    with depth; cell (x, y, z) of plane i is f[i*N + (z*ny + y)*nx + x];
 *  - populations are perturbations about the rest state f = 0;
 *  - equilibrium: eq. equilibrium-solid with the full second moment P of the
 *    populations and P^n = P - rho b^2 I (eq. Pn), summed over x, y and z;
 *  - j = sum f c + S/2, the sponge solved implicitly, S = G - A j, G = kappa
 *    grad(rho) + F (eqs. S, Si, MomentChainAbsorbing), kappa = b^2 (mu -
 *    lambda) / mu as in two dimensions;
 *  - density gradient: centred differences along x, y and z (eq. FDrho), the
 *    neighbour beyond a non-periodic face being the ghost 2 rho_b - rho_in;
 *  - faces: 0 top (z = 0), 1 bottom (z = nz-1), 2 left (x = 0), 3 right
 *    (x = nx-1), 4 front (y = 0), 5 back (y = ny-1). Periodic faces come in
 *    opposite pairs; free surfaces (Sec. 6.2) on the top and bottom faces
 *    only; rigid faces bounce back (eq. BB);
 *  - free surface on a z face: anti-bounce-back toward the air state with
 *    rho_air and the tangential stress block (P_xx, P_xy, P_yy) taken at the
 *    interface half a cell out (FREE: linear extrapolation 3/2 boundary cell
 *    - 1/2 cell inside; FREE0: the boundary cell's own values) and the rows of
 *    P_air along the normal (P_xz, P_yz, P_zz) zero -- the traction-free
 *    condition P_air n = 0 of Sec. 6.2 written for a face normal to z;
 *  - a link whose target lies beyond several faces bounces back as rigid if
 *    any of them is rigid, else follows the free rule if any is free, else
 *    wraps on every periodic axis;
 *  - the free-surface moments are those of the step's own pre-collision
 *    populations (equal to those of the post-collision populations reflected:
 *    rho and P are collision invariants of the elastic equilibrium).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { F3_PERIODIC = 0, F3_FREE = 1, F3_RIGID = 2, F3_FREE0 = 3 };
enum { F3_TOP = 0, F3_BOTTOM = 1, F3_LEFT = 2, F3_RIGHT = 3, F3_FRONT = 4, F3_BACK = 5 };

#define Q3 27 /* the largest velocity set; D3Q19 is its first 19 vectors */

/* D3Q19 and D3Q27 velocity sets (Sec. 3, regular lattices). */
static const int V3[Q3][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
static const double B2_3 = 1.0 / 3.0;

/* Weight of vector i of the q-velocity set, by its number of nonzero
 * components (its speed class). */
static double weight3(int q, int i) {
  const int n = abs(V3[i][0]) + abs(V3[i][1]) + abs(V3[i][2]);
  if (q == 19) return n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  return n == 0 ? 8.0 / 27.0 : (n == 1 ? 2.0 / 27.0 : (n == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
}

static int opposite3(int q, int i) {
  for (int k = 0; k < q; ++k)
    if (V3[k][0] == -V3[i][0] && V3[k][1] == -V3[i][1] && V3[k][2] == -V3[i][2]) return k;
  return -1;
}

typedef struct {
  int32_t nx, ny, nz;
  int32_t face[6];        /* F3_* per face, order top, bottom, left, right, front, back */
  int32_t sp_thick[6];    /* sponge thickness per face (cells) */
  int32_t nsrc;
  double tau;
  const double *sp_prof[6]; /* sponge damping A[k], k = cells from the face */
  const double *src;      /* nsrc x 10: x, y, z, sigma, dir_x, dir_y, dir_z, amp, period, t0 */
  int32_t nrec;
  int32_t comp_mask;      /* bit 0: v_x, bit 1: v_y, bit 2: v_z */
  const int32_t *rec_xyz; /* nrec x 3: x, y, z */
  int32_t q;              /* 19 or 27 */
  int32_t pad_;
} oracle3_cfg;

/* Velocities, weights and opposites of the q-velocity set (q = 19 or 27);
 * returns q, or -1 for another q. */
int oracle3_lattice(int32_t q, int32_t *c, double *w, int32_t *opp) {
  if (q != 19 && q != 27) return -1;
  for (int i = 0; i < q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = V3[i][a];
    w[i] = weight3(q, i);
    opp[i] = opposite3(q, i);
  }
  return q;
}

/* Elastic equilibrium (eqs. equilibrium-solid and Pn) on D3Q19.
 * P = (P_xx, P_xy, P_xz, P_yy, P_yz, P_zz). */
void oracle3_equilibrium(int32_t q, double rho, const double j[3], const double P[6], double *feq) {
  double pn[3][3];
  pn[0][0] = P[0] - rho * B2_3;
  pn[0][1] = pn[1][0] = P[1];
  pn[0][2] = pn[2][0] = P[2];
  pn[1][1] = P[3] - rho * B2_3;
  pn[1][2] = pn[2][1] = P[4];
  pn[2][2] = P[5] - rho * B2_3;
  for (int i = 0; i < q; ++i) {
    double jc = 0.0, pnq = 0.0;
    for (int a = 0; a < 3; ++a) {
      jc += j[a] * V3[i][a];
      for (int b = 0; b < 3; ++b)
        pnq += pn[a][b] * ((double)V3[i][a] * V3[i][b] - (a == b ? B2_3 : 0.0));
    }
    feq[i] = weight3(q, i) * (rho + jc / B2_3 + pnq / (2.0 * B2_3 * B2_3));
  }
}

/* Moments of one cell: rho, the first moment m and P. */
static void cell_moments(int q, const double *f, double *rho, double m[3], double P[6]) {
  double r = 0.0, mm[3] = {0, 0, 0}, pp[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < q; ++i) {
    r += f[i];
    for (int a = 0; a < 3; ++a) {
      mm[a] += f[i] * V3[i][a];
      for (int b = 0; b < 3; ++b) pp[a][b] += f[i] * V3[i][a] * V3[i][b];
    }
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) m[a] = mm[a];
  P[0] = pp[0][0]; P[1] = pp[0][1]; P[2] = pp[0][2];
  P[3] = pp[1][1]; P[4] = pp[1][2]; P[5] = pp[2][2];
}

/* One cell of the collision (eqs. MomentsFeq, Si, LBGK, MomentChainAbsorbing).
 * G: source without the sponge; A: sponge damping. Returns f*, and j and S. */
void oracle3_collide_cell(int32_t q, const double *f, const double G[3], double A, double tau,
                          double *fstar, double j_out[3], double S_out[3]) {
  double rho, m[3], P[6];
  cell_moments(q, f, &rho, m, P);
  double j[3], S[3];
  for (int a = 0; a < 3; ++a) {
    j[a] = (m[a] + 0.5 * G[a]) / (1.0 + 0.5 * A);
    S[a] = G[a] - A * j[a];
  }
  double feq[Q3];
  oracle3_equilibrium(q, rho, j, P, feq);
  for (int i = 0; i < q; ++i) {
    const double Si = weight3(q, i) * (V3[i][0] * S[0] + V3[i][1] * S[1] + V3[i][2] * S[2]) / B2_3;
    fstar[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * Si;
  }
  if (j_out) for (int a = 0; a < 3; ++a) j_out[a] = j[a];
  if (S_out) for (int a = 0; a < 3; ++a) S_out[a] = S[a];
}

static double ricker3(double t, double period, double t0) {
  const double a = M_PI * (t - t0) / period;
  return (1.0 - 2.0 * a * a) * exp(-a * a);
}

typedef struct {
  const oracle3_cfg *c;
  int q;              /* velocities */
  int n[3];           /* nx, ny, nz */
  size_t N;
  double *kappa, *A, *inv_rho0_rec;
  double *rho, *m[3], *P[6], *grad[3], *G[3], *j[3];
} grid3;

static size_t idx3(const grid3 *g, int x, int y, int z) {
  return ((size_t)z * g->n[1] + y) * g->n[0] + x;
}

/* The two faces normal to each axis: axis 0 (x) left/right, 1 (y) front/back,
 * 2 (z) top/bottom. */
static const int FACE_LO[3] = {F3_LEFT, F3_FRONT, F3_TOP};
static const int FACE_HI[3] = {F3_RIGHT, F3_BACK, F3_BOTTOM};

/* Sponge damping: the largest of the face profiles reaching the cell (Sec. 6.4). */
static void build_sponge3(grid3 *g) {
  const oracle3_cfg *c = g->c;
  for (int z = 0; z < g->n[2]; ++z)
    for (int y = 0; y < g->n[1]; ++y)
      for (int x = 0; x < g->n[0]; ++x) {
        const int p[3] = {x, y, z};
        double a = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
          const int d[2] = {p[ax], g->n[ax] - 1 - p[ax]};
          const int fc[2] = {FACE_LO[ax], FACE_HI[ax]};
          for (int s = 0; s < 2; ++s)
            if (c->sp_thick[fc[s]] > 0 && d[s] < c->sp_thick[fc[s]]) {
              const double v = c->sp_prof[fc[s]][d[s]];
              if (v > a) a = v;
            }
        }
        g->A[idx3(g, x, y, z)] = a;
      }
}

/* Step 1: moments of f. */
static void phase3_moments(grid3 *g, const double *f) {
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < g->N; ++k) {
    double fc[Q3], P[6];
    for (int i = 0; i < g->q; ++i) fc[i] = f[i * g->N + k];
    double m[3];
    cell_moments(g->q, fc, &g->rho[k], m, P);
    for (int a = 0; a < 3; ++a) g->m[a][k] = m[a];
    for (int q = 0; q < 6; ++q) g->P[q][k] = P[q];
  }
}

/* Density of the neighbour one cell along axis ax in direction dir, or the
 * ghost 2 rho_b - rho_in beyond a non-periodic face. */
static double rho_neighbour3(const grid3 *g, const int p[3], int ax, int dir) {
  int q[3] = {p[0], p[1], p[2]};
  q[ax] += dir;
  if (q[ax] < 0 || q[ax] >= g->n[ax]) {
    const int face = q[ax] < 0 ? FACE_LO[ax] : FACE_HI[ax];
    if (g->c->face[face] != F3_PERIODIC) {
      int r[3] = {p[0], p[1], p[2]};
      r[ax] -= dir;
      return 2.0 * g->rho[idx3(g, p[0], p[1], p[2])] - g->rho[idx3(g, r[0], r[1], r[2])];
    }
    q[ax] = (q[ax] + g->n[ax]) % g->n[ax];
  }
  return g->rho[idx3(g, q[0], q[1], q[2])];
}

/* Step 2: centred finite-difference density gradient (eq. FDrho, per axis). */
static void phase3_gradient(grid3 *g) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->n[2]; ++z)
    for (int y = 0; y < g->n[1]; ++y)
      for (int x = 0; x < g->n[0]; ++x) {
        const int p[3] = {x, y, z};
        const size_t k = idx3(g, x, y, z);
        for (int ax = 0; ax < 3; ++ax)
          g->grad[ax][k] = 0.5 * (rho_neighbour3(g, p, ax, +1) - rho_neighbour3(g, p, ax, -1));
      }
}

static double min_image3(double d, int n, int periodic) {
  if (!periodic) return d;
  while (d > 0.5 * n) d -= n;
  while (d < -0.5 * n) d += n;
  return d;
}

/* Step 3: G = kappa grad(rho) + F, F the Gaussian x Ricker body force of
 * Sec. 5 in three dimensions, zero beyond 9 sigma. */
static void phase3_source(grid3 *g, int64_t t) {
  const oracle3_cfg *c = g->c;
  int per[3];
  for (int ax = 0; ax < 3; ++ax) per[ax] = c->face[FACE_LO[ax]] == F3_PERIODIC;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->n[2]; ++z)
    for (int y = 0; y < g->n[1]; ++y)
      for (int x = 0; x < g->n[0]; ++x) {
        const size_t k = idx3(g, x, y, z);
        const int p[3] = {x, y, z};
        double F[3] = {0, 0, 0};
        for (int s = 0; s < c->nsrc; ++s) {
          const double *q = c->src + 10 * s;
          double r2 = 0.0;
          for (int ax = 0; ax < 3; ++ax) {
            const double d = min_image3(p[ax] - q[ax], g->n[ax], per[ax]);
            r2 += d * d;
          }
          const double sig = q[3];
          if (r2 > 81.0 * sig * sig) continue;
          const double mag = q[7] * exp(-r2 / (2.0 * sig * sig)) * ricker3((double)t, q[8], q[9]);
          for (int ax = 0; ax < 3; ++ax) F[ax] += mag * q[4 + ax];
        }
        for (int ax = 0; ax < 3; ++ax) g->G[ax][k] = g->kappa[k] * g->grad[ax][k] + F[ax];
      }
}

/* Steps 4-6: flux, sponge, equilibrium and collision. */
static void phase3_collide(grid3 *g, const double *f, double *fstar) {
  const double tau = g->c->tau;
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < g->N; ++k) {
    double fc[Q3], fs[Q3], j[3];
    for (int i = 0; i < g->q; ++i) fc[i] = f[i * g->N + k];
    const double G[3] = {g->G[0][k], g->G[1][k], g->G[2][k]};
    oracle3_collide_cell(g->q, fc, G, g->A[k], tau, fs, j, NULL);
    for (int i = 0; i < g->q; ++i) fstar[i * g->N + k] = fs[i];
    for (int a = 0; a < 3; ++a) g->j[a][k] = j[a];
  }
}

/* Step 7: receivers record v = j / rho0 (Sec. 5). */
static void phase3_receivers(grid3 *g, double *row) {
  const oracle3_cfg *c = g->c;
  int o = 0;
  for (int r = 0; r < c->nrec; ++r) {
    const int32_t *q = c->rec_xyz + 3 * r;
    const size_t k = idx3(g, q[0], q[1], q[2]);
    for (int a = 0; a < 3; ++a)
      if (c->comp_mask & (1 << a)) row[o++] = g->j[a][k] * g->inv_rho0_rec[r];
  }
}

/* Anti-bounce-back value for link i leaving boundary cell k through a z face
 * of outward normal nz_out (Sec. 6.2 written for a z face): -f*_i + 2 w_i
 * (rho_air + P^n_air : (c_i c_i - b^2 I) / (2 b^4)). */
static double free_value3(const grid3 *g, size_t kb, size_t kin, int i, int order, double fs) {
  const double cb = order ? 1.5 : 1.0, cin = order ? -0.5 : 0.0;
  const double rho_air = cb * g->rho[kb] + cin * g->rho[kin];
  /* P_air: tangential block extrapolated, the rows along the normal zero. */
  double pair[6];
  pair[0] = cb * g->P[0][kb] + cin * g->P[0][kin];
  pair[1] = cb * g->P[1][kb] + cin * g->P[1][kin];
  pair[2] = 0.0;
  pair[3] = cb * g->P[3][kb] + cin * g->P[3][kin];
  pair[4] = 0.0;
  pair[5] = 0.0;
  /* w_i (rho + P^n : Q / (2 b^4)) is the equilibrium at zero flux */
  const double jz[3] = {0, 0, 0};
  double feq[Q3];
  oracle3_equilibrium(g->q, rho_air, jz, pair, feq);
  return -fs + 2.0 * feq[i];
}

/* Step 8: push streaming f_i(x + c_i, t + 1) = f*_i(x, t) with the face rules. */
static void phase3_stream(grid3 *g, const double *fstar, double *fnext) {
  const oracle3_cfg *c = g->c;
  const size_t N = g->N;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->n[2]; ++z)
    for (int y = 0; y < g->n[1]; ++y)
      for (int x = 0; x < g->n[0]; ++x) {
        const int p[3] = {x, y, z};
        const size_t k = idx3(g, x, y, z);
        for (int i = 0; i < g->q; ++i) {
          int d[3], rigid = 0, free_nz = 0, order = 0;
          for (int ax = 0; ax < 3; ++ax) {
            d[ax] = p[ax] + V3[i][ax];
            if (d[ax] >= 0 && d[ax] < g->n[ax]) continue;
            const int face = d[ax] < 0 ? FACE_LO[ax] : FACE_HI[ax];
            const int kind = c->face[face];
            if (kind == F3_PERIODIC) {
              d[ax] = (d[ax] + g->n[ax]) % g->n[ax];
            } else if (kind == F3_RIGID) {
              rigid = 1;
            } else {
              free_nz = d[ax] < 0 ? -1 : +1; /* only z faces may be free */
              order = kind == F3_FREE ? 1 : 0;
            }
          }
          const double fs = fstar[i * N + k];
          const int o = opposite3(g->q, i);
          if (rigid) {
            fnext[o * N + k] = fs;
          } else if (free_nz != 0) {
            const size_t kin = idx3(g, x, y, z - free_nz);
            fnext[o * N + k] = free_value3(g, k, kin, i, order, fs);
          } else {
            fnext[i * N + idx3(g, d[0], d[1], d[2])] = fs;
          }
        }
      }
}

static void grid3_free(grid3 *g) {
  double *planes[] = {g->kappa, g->A, g->rho, g->m[0], g->m[1], g->m[2],
                      g->P[0], g->P[1], g->P[2], g->P[3], g->P[4], g->P[5],
                      g->grad[0], g->grad[1], g->grad[2], g->G[0], g->G[1], g->G[2],
                      g->j[0], g->j[1], g->j[2]};
  for (size_t p = 0; p < sizeof(planes) / sizeof(planes[0]); ++p) free(planes[p]);
  free(g->inv_rho0_rec);
}

static int grid3_alloc(grid3 *g, const oracle3_cfg *c, const double *lam, const double *mu,
                       const double *rho0) {
  memset(g, 0, sizeof(*g));
  g->c = c;
  g->q = c->q;
  g->n[0] = c->nx; g->n[1] = c->ny; g->n[2] = c->nz;
  g->N = (size_t)c->nx * c->ny * c->nz;
  double **planes[] = {&g->kappa, &g->A, &g->rho, &g->m[0], &g->m[1], &g->m[2],
                       &g->P[0], &g->P[1], &g->P[2], &g->P[3], &g->P[4], &g->P[5],
                       &g->grad[0], &g->grad[1], &g->grad[2], &g->G[0], &g->G[1], &g->G[2],
                       &g->j[0], &g->j[1], &g->j[2]};
  for (size_t p = 0; p < sizeof(planes) / sizeof(planes[0]); ++p) {
    *planes[p] = (double *)calloc(g->N, sizeof(double));
    if (!*planes[p]) return -2;
  }
  g->inv_rho0_rec = (double *)calloc(c->nrec > 0 ? c->nrec : 1, sizeof(double));
  if (!g->inv_rho0_rec) return -2;
  for (size_t k = 0; k < g->N; ++k) g->kappa[k] = B2_3 * (mu[k] - lam[k]) / mu[k];
  for (int r = 0; r < c->nrec; ++r) {
    const int32_t *q = c->rec_xyz + 3 * r;
    g->inv_rho0_rec[r] = 1.0 / rho0[idx3(g, q[0], q[1], q[2])];
  }
  build_sponge3(g);
  return 0;
}

/* Run nsteps steps from time t0 on the lattice c->q (19 or 27).
 *   init: q planes of populations or NULL (rest state); init_kind 0: the
 *     post-collision populations of step t0-1, 1: the pre-collision
 *     populations at t0;
 *   fstar_out: post-collision populations of step t0+nsteps-1 (or NULL);
 *   f_out: pre-collision populations at t0+nsteps (or NULL);
 *   mom_out: [10][N] rho, j_x, j_y, j_z, P_xx, P_xy, P_xz, P_yy, P_yz, P_zz
 *     at t0+nsteps (or NULL);
 *   trace: [nsteps][nrec][ncomp] (or NULL).
 * Returns 0, -1 for a lattice other than 19 or 27, or -2 when memory runs
 * out. */
int oracle3_run(const oracle3_cfg *c, const double *lam, const double *mu, const double *rho0,
                const double *init, int32_t init_kind, int64_t t0, int64_t nsteps,
                double *fstar_out, double *f_out, double *mom_out, double *trace) {
  if (c->q != 19 && c->q != 27) return -1;
  grid3 g;
  if (grid3_alloc(&g, c, lam, mu, rho0) != 0) { grid3_free(&g); return -2; }
  const size_t N = g.N;
  const size_t Q = (size_t)c->q;
  double *f = (double *)calloc(Q * N, sizeof(double));
  double *fs = (double *)calloc(Q * N, sizeof(double));
  if (!f || !fs) { free(f); free(fs); grid3_free(&g); return -2; }
  int ncomp = 0;
  for (int a = 0; a < 3; ++a) ncomp += (c->comp_mask >> a) & 1;
  if (init && init_kind == 0) {
    memcpy(fs, init, Q * N * sizeof(double));
    phase3_moments(&g, fs);
    phase3_stream(&g, fs, f);
  } else if (init) {
    memcpy(f, init, Q * N * sizeof(double));
  }
  for (int64_t n = 0; n < nsteps; ++n) {
    phase3_moments(&g, f);
    phase3_gradient(&g);
    phase3_source(&g, t0 + n);
    phase3_collide(&g, f, fs);
    if (trace && c->nrec > 0) phase3_receivers(&g, trace + (size_t)n * c->nrec * ncomp);
    phase3_stream(&g, fs, f);
  }
  if (fstar_out) memcpy(fstar_out, fs, Q * N * sizeof(double));
  if (f_out) memcpy(f_out, f, Q * N * sizeof(double));
  if (mom_out) {
    phase3_moments(&g, f);
    phase3_gradient(&g);
    phase3_source(&g, t0 + nsteps);
    for (size_t k = 0; k < N; ++k) {
      mom_out[k] = g.rho[k];
      for (int a = 0; a < 3; ++a)
        mom_out[(1 + a) * N + k] = (g.m[a][k] + 0.5 * g.G[a][k]) / (1.0 + 0.5 * g.A[k]);
      for (int q = 0; q < 6; ++q) mom_out[(4 + q) * N + k] = g.P[q][k];
    }
  }
  free(f);
  free(fs);
  grid3_free(&g);
  return 0;
}
