// Fused D2Q9 elastic-wave LBM step for gfx950 (MI355X).
//
// One launch advances every grid of a context by one time step. A workgroup
// owns a tile of 64*NW columns and marches down its rows. For each row it
//   1. pulls the nine populations f_i(x, t) = f*_i(x - c_i, t-1) from the
//      state of step t-1 (pull form of eq. LBGK), applying periodic wrap,
//      halfway bounce-back (eq. BB) and free-surface anti-bounce-back (Sec.
//      6.2) on the links that cross a wall;
//   2. takes the moments rho, m, P of the pulled populations (eq. MomentsFeq);
//   3. forms the centred density gradient of eq. FDrho from rho of the row
//      above and below (kept in registers while marching) and of the left and
//      right neighbours (a two-row LDS ring written by the row's lanes plus two
//      halo lanes for the tile's outer columns);
//   4. builds the source G = kappa grad(rho) + F (eq. S; F the Gaussian x
//      Ricker force of Sec. 5), the flux j = (m + G/2)/(1 + A/2) and
//      S = G - A j with the absorbing-layer damping A (eq.
//      MomentChainAbsorbing solved implicitly);
//   5. relaxes toward the elastic equilibrium (eqs. equilibrium-solid, Pn) with
//      the forcing populations of eq. Si and writes f*(t), one store per
//      population, to the other buffer of the ping-pong pair.
// Each population is read once and written once per step from HBM; the halo
// reads for step 3 and the boundary-row moments for the free surface come from
// L2. Populations are kept as structure-of-arrays planes with a pitch of a
// multiple of 64 elements so every wavefront load and store is a full line.
#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <typename real>
__device__ __forceinline__ constexpr real weight(int i) {
  return i == 0 ? real(4) / real(9) : (i < 5 ? real(1) / real(9) : real(1) / real(36));
}

// Row classification for the pull of row y (uniform across the workgroup).
struct Row {
  int y;
  int up, dn;          // source rows of links arriving with c_y = +1 / -1
  int wall_up, wall_dn;// 0, kFree or kRigid: the wall those links cross
};

__device__ __forceinline__ Row make_row(const GridDev &g, int y) {
  Row r;
  r.y = y;
  r.wall_up = 0;
  r.wall_dn = 0;
  r.up = y - 1;
  r.dn = y + 1;
  if (y == 0) {
    if (g.bc[kEdgeTop] == kPeriodic) r.up = g.ny - 1;
    else { r.wall_up = g.bc[kEdgeTop]; r.up = y; }
  } else if (y == g.rigid_row) {
    r.wall_up = kRigid;
    r.up = y;
  }
  if (y == g.ny - 1) {
    if (g.bc[kEdgeBottom] == kPeriodic) r.dn = 0;
    else { r.wall_dn = g.bc[kEdgeBottom]; r.dn = y; }
  } else if (g.rigid_row > 0 && y == g.rigid_row - 1) {
    r.wall_dn = kRigid;
    r.dn = y;
  }
  return r;
}

// Column classification for one lane (left/right edges: periodic or rigid).
struct Col {
  int x, xl, xr;   // own column, source column for c_x = +1 and c_x = -1
  bool wl, wr;     // links with c_x = +1 / -1 cross a rigid edge
};

__device__ __forceinline__ Col make_col(const GridDev &g, int x) {
  Col c;
  c.x = x;
  c.wl = false;
  c.wr = false;
  c.xl = x - 1;
  c.xr = x + 1;
  if (x == 0) {
    if (g.bc[kEdgeLeft] == kPeriodic) c.xl = g.nx - 1;
    else { c.wl = true; c.xl = x; }
  }
  if (x == g.nx - 1) {
    if (g.bc[kEdgeRight] == kPeriodic) c.xr = 0;
    else { c.wr = true; c.xr = x; }
  }
  return c;
}

// Pulled populations f_i(x, t) of cell (c.x, r.y) from the state f*(t-1).
template <typename real>
__device__ __forceinline__ void pull(const real *__restrict__ base, const GridDev &g,
                                     const Row &r, const Col &c, real out[9]) {
  const int64_t P = g.plane;
  const int64_t ro = (int64_t)r.y * g.pitch;
  const int64_t ru = (int64_t)r.up * g.pitch;
  const int64_t rd = (int64_t)r.dn * g.pitch;
  if ((r.wall_up | r.wall_dn) == 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int64_t row = CY[i] == 0 ? ro : (CY[i] == 1 ? ru : rd);
      const int col = CX[i] == 0 ? c.x : (CX[i] == 1 ? c.xl : c.xr);
      const bool xw = CX[i] == 1 ? c.wl : (CX[i] == -1 ? c.wr : false);
      const int64_t addr = xw ? (OPP[i] * P + ro + c.x) : (i * P + row + col);
      out[i] = base[addr];
    }
    return;
  }
  // A row next to a horizontal wall. For a free surface, the anti-bounce-back
  // needs rho and the tangential stress P_xx at the boundary cell and one cell
  // inside, at time t-1: moments of the stored post-collision populations
  // (rho and P are collision invariants).
  real rho_air = real(0), pxx_air = real(0);
  const bool free_wall = (r.wall_up == kFree) || (r.wall_dn == kFree);
  if (free_wall) {
    const int yin = (r.wall_up == kFree) ? r.y + 1 : r.y - 1;
    const int64_t rin = (int64_t)yin * g.pitch;
    real rb = 0, xb = 0, ri = 0, xi = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const real vb = base[i * P + ro + c.x];
      const real vi = base[i * P + rin + c.x];
      rb += vb;
      ri += vi;
      if (CX[i] != 0) { xb += vb; xi += vi; }
    }
    rho_air = real(1.5) * rb - real(0.5) * ri;
    pxx_air = real(1.5) * xb - real(0.5) * xi;
  }
  const real b2 = real(1) / real(3);
  const real pn_xx = pxx_air - b2 * rho_air;
  const real pn_yy = -b2 * rho_air;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int ywall = CY[i] == 1 ? r.wall_up : (CY[i] == -1 ? r.wall_dn : 0);
    const bool xw = CX[i] == 1 ? c.wl : (CX[i] == -1 ? c.wr : false);
    if (ywall == 0 && !xw) {
      const int64_t row = CY[i] == 0 ? ro : (CY[i] == 1 ? ru : rd);
      const int col = CX[i] == 0 ? c.x : (CX[i] == 1 ? c.xl : c.xr);
      out[i] = base[i * P + row + col];
    } else {
      const real refl = base[OPP[i] * P + ro + c.x];
      if (xw || ywall == kRigid) {
        out[i] = refl;
      } else {
        // -f*_opp + 2 w (rho_air + P^n_air : (c c - b^2 I) / (2 b^4)), c_y^2 = 1
        const real cxx = real(CX[i] * CX[i]) - b2;
        const real q = pn_xx * cxx + pn_yy * (real(1) - b2);
        out[i] = -refl + real(2) * weight<real>(i) * (rho_air + real(4.5) * q);
      }
    }
  }
}

template <typename real>
__device__ __forceinline__ real sum9(const real f[9]) {
  return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

__device__ __forceinline__ double ricker(double t, double period, double t0) {
  const double a = 3.14159265358979323846 * (t - t0) / period;
  return (1.0 - 2.0 * a * a) * exp(-a * a);
}

__device__ __forceinline__ double min_image(double d, int n, bool periodic) {
  if (periodic) {
    if (d > 0.5 * n) d -= n;
    else if (d < -0.5 * n) d += n;
  }
  return d;
}

template <typename real, int NW, int MODE>
__global__ __launch_bounds__(64 * NW) void step_kernel(StepArgs<real> a) {
  constexpr int W = 64 * NW;
  __shared__ real srho[2][W + 2];

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;                        // padding block (uniform)
  if (MODE == kModeMoments && tile.g != a.mom_grid) return;
  const GridDev &g = a.grids[tile.g];
  const real *__restrict__ fin = a.fin + g.f_off;

  const int lane = threadIdx.x;
  const int x = tile.x0 + lane;
  const bool active = x < g.nx;
  const int xa = active ? x : g.nx - 1;
  const Col col = make_col(g, xa);
  const int x_last = min(tile.x0 + W, g.nx) - 1;

  // Lanes 0 and 1 also pull the tile's outer neighbour columns (for the
  // density gradient of the first and last column).
  int hx = 0;
  bool hvalid = false;
  if (lane == 0) {
    hx = tile.x0 - 1;
    hvalid = true;
    if (hx < 0) { hvalid = g.bc[kEdgeLeft] == kPeriodic; hx = g.nx - 1; }
  } else if (lane == 1) {
    hx = x_last + 1;
    hvalid = true;
    if (hx >= g.nx) { hvalid = g.bc[kEdgeRight] == kPeriodic; hx = 0; }
  }
  const Col hcol = make_col(g, hx);
  const int hslot = lane == 0 ? 0 : W + 1;

  const int64_t t = a.t + (a.t_dev ? a.t_dev[0] : 0);
  const real omega = a.omega;
  const real cforce = a.cforce;
  const bool px = g.bc[kEdgeLeft] == kPeriodic;
  const bool py = g.bc[kEdgeTop] == kPeriodic;

  // Prologue: first row and the density of the row above it.
  Row r = make_row(g, tile.y0);
  real fc[9];
  pull(fin, g, r, col, fc);
  real rho_c = sum9(fc);
  real rho_m = real(0);
  if (r.wall_up == 0) {
    real fm[9];
    pull(fin, g, make_row(g, r.up), col, fm);
    rho_m = sum9(fm);
  }
  srho[0][lane + 1] = rho_c;
  if (lane < 2) {
    real hr = real(0);
    if (hvalid) { real fh[9]; pull(fin, g, r, hcol, fh); hr = sum9(fh); }
    srho[0][hslot] = hr;
  }
  __syncthreads();

  for (int y = tile.y0, k = 0; y < tile.y1; ++y, ++k) {
    // Next row: needed as the next output row and/or for d rho / dy.
    int yn = y + 1;
    if (yn >= g.ny) yn = (g.bc[kEdgeBottom] == kPeriodic) ? 0 : -1;
    const bool need_next = yn >= 0 && ((y + 1 < tile.y1) || r.wall_dn == 0);
    const Row rn = make_row(g, yn < 0 ? y : yn);
    real fn[9];
    real rho_n = real(0);
    if (need_next) {
      pull(fin, g, rn, col, fn);
      rho_n = sum9(fn);
    }
    const int s = k & 1;
    const real rho_l = srho[s][lane];
    const real rho_r = (xa == x_last) ? srho[s][W + 1] : srho[s][lane + 2];
    if (need_next) {
      srho[s ^ 1][lane + 1] = rho_n;
      if (lane < 2) {
        real hr = real(0);
        if (hvalid) { real fh[9]; pull(fin, g, rn, hcol, fh); hr = sum9(fh); }
        srho[s ^ 1][hslot] = hr;
      }
    }

    // Centred density gradient (eq. FDrho); one-sided next to walls.
    real dx, dy;
    if (col.wl) dx = rho_r - rho_c;
    else if (col.wr) dx = rho_c - rho_l;
    else dx = real(0.5) * (rho_r - rho_l);
    if (r.wall_up) dy = rho_n - rho_c;
    else if (r.wall_dn) dy = rho_c - rho_m;
    else dy = real(0.5) * (rho_n - rho_m);

    // Elastic coefficient.
    real kap;
    if (g.kmode == kKappaScalar) kap = (real)g.kscalar;
    else if (g.kmode == kKappaRows) kap = a.kappa_rows[g.k_off + y];
    else kap = a.kappa_cells[g.k_off + (int64_t)y * g.pitch + xa];

    // Absorbing-layer damping.
    real A = real(0);
    {
      const int dt_ = y, db = g.ny - 1 - y, dl = xa, dr = g.nx - 1 - xa;
      if (dt_ < g.sp_thick[kEdgeTop]) A = max(A, a.sponge[g.sp_off[kEdgeTop] + dt_]);
      if (db < g.sp_thick[kEdgeBottom]) A = max(A, a.sponge[g.sp_off[kEdgeBottom] + db]);
      if (dl < g.sp_thick[kEdgeLeft]) A = max(A, a.sponge[g.sp_off[kEdgeLeft] + dl]);
      if (dr < g.sp_thick[kEdgeRight]) A = max(A, a.sponge[g.sp_off[kEdgeRight] + dr]);
    }

    // Body force (Gaussian x Ricker), only on rows within 9 sigma of a source.
    real Fx = real(0), Fy = real(0);
    for (int si = 0; si < g.nsrc; ++si) {
      const SourceDev sd = a.sources[g.src_off + si];
      const double ddy = min_image((double)y - sd.y, g.ny, py);
      const double cut = 81.0 * sd.sigma * sd.sigma;
      if (ddy * ddy > cut) continue;
      const double R = ricker((double)t, sd.period, sd.t0);
      const double ddx = min_image((double)xa - sd.x, g.nx, px);
      const double r2 = ddx * ddx + ddy * ddy;
      if (r2 <= cut) {
        const double mag = sd.amp * exp(-r2 / (2.0 * sd.sigma * sd.sigma)) * R;
        Fx += (real)(mag * sd.dir_x);
        Fy += (real)(mag * sd.dir_y);
      }
    }

    const real Gx = kap * dx + Fx;
    const real Gy = kap * dy + Fy;

    // Moments of the pulled populations.
    const real rho = rho_c;
    const real mx = (fc[1] - fc[3]) + (fc[5] - fc[6]) + (fc[8] - fc[7]);
    const real my = (fc[2] - fc[4]) + (fc[5] + fc[6]) - (fc[7] + fc[8]);
    const real diag = (fc[5] + fc[6]) + (fc[7] + fc[8]);
    const real pxx = (fc[1] + fc[3]) + diag;
    const real pyy = (fc[2] + fc[4]) + diag;
    const real pxy = (fc[5] + fc[7]) - (fc[6] + fc[8]);

    const real inv = real(1) / (real(1) + real(0.5) * A);
    const real jx = (mx + real(0.5) * Gx) * inv;
    const real jy = (my + real(0.5) * Gy) * inv;
    const real Sx = Gx - A * jx;
    const real Sy = Gy - A * jy;

    if (MODE == kModeMoments) {
      if (active) {
        const int64_t n = (int64_t)g.nx * g.ny;
        const int64_t o = (int64_t)y * g.nx + x;
        a.mom[o] = rho;
        a.mom[n + o] = jx;
        a.mom[2 * n + o] = jy;
        a.mom[3 * n + o] = pxx;
        a.mom[4 * n + o] = pxy;
        a.mom[5 * n + o] = pyy;
      }
    } else {
      // Receivers on this row.
      if (g.nrec > 0) {
        const int slot = a.itab[g.rowtab_off + y];
        if (slot >= 0 && active) {
          int rid = a.itab[g.rmap_off + (int64_t)slot * g.nx + x];
          const int64_t tk = t - g.trace_t0;
          while (rid >= 0) {
            if (tk >= 0 && tk < g.trace_max) {
              const real sc = a.rtab[g.rscale_off + rid];
              real *tr = reinterpret_cast<real *>(g.trace) + (tk * g.nrec + rid) * g.ncomp;
              int o = 0;
              if (g.comp_mask & 1) tr[o++] = jx * sc;
              if (g.comp_mask & 2) tr[o] = jy * sc;
            }
            rid = a.itab[g.rnext_off + rid];
          }
        }
      }
      // Equilibrium (b^2 = 1/3: 1/b^2 = 3, 1/(2 b^4) = 9/2) and BGK collision.
      const real b2 = real(1) / real(3);
      const real pnxx = pxx - b2 * rho;
      const real pnyy = pyy - b2 * rho;
      const real pnxy = pxy;
      if (active) {
        real *__restrict__ out = a.fout + g.f_off + (int64_t)y * g.pitch + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const real cx = real(CX[i]), cy = real(CY[i]);
          const real q = pnxx * (cx * cx - b2) + real(2) * pnxy * (cx * cy) + pnyy * (cy * cy - b2);
          const real feq = weight<real>(i) * (rho + real(3) * (jx * cx + jy * cy) + real(4.5) * q);
          const real si = weight<real>(i) * real(3) * (cx * Sx + cy * Sy);
          out[i * g.plane] = fc[i] - omega * (fc[i] - feq) + cforce * si;
        }
      }
    }

    // March.
    __syncthreads();
    r = rn;
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = need_next ? fn[i] : fc[i];
    rho_m = rho_c;
    rho_c = rho_n;
  }
}

}  // namespace

template <typename real>
hipError_t launch_step(const StepArgs<real> &a, int waves, int ntiles, int mode,
                       hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves);
#define LBM_LAUNCH(NW, MODE) \
  hipLaunchKernelGGL((step_kernel<real, NW, MODE>), grid, block, 0, stream, a)
  if (mode == kModeStep) {
    if (waves == 1) LBM_LAUNCH(1, kModeStep);
    else if (waves == 2) LBM_LAUNCH(2, kModeStep);
    else if (waves == 4) LBM_LAUNCH(4, kModeStep);
    else return hipErrorInvalidValue;
  } else {
    if (waves == 1) LBM_LAUNCH(1, kModeMoments);
    else if (waves == 2) LBM_LAUNCH(2, kModeMoments);
    else if (waves == 4) LBM_LAUNCH(4, kModeMoments);
    else return hipErrorInvalidValue;
  }
#undef LBM_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_step<float>(const StepArgs<float> &, int, int, int, hipStream_t);
template hipError_t launch_step<double>(const StepArgs<double> &, int, int, int, hipStream_t);

}  // namespace lbm
