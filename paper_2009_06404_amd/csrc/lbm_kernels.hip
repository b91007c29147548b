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
//
// Memory: each population is read once and written once per step from HBM;
// the rows above/below a tile and the halo columns are re-read from L2. The
// pulled rows (and the halo columns) are prefetched two rows ahead so that a
// wavefront keeps a full row of loads in flight while it computes; stores are
// non-temporal so the write stream does not evict the lines neighbouring
// tiles still have to read. Populations are stored row by row: population i
// of row y is a contiguous run of `pitch` elements at ((y*9 + i) * pitch), the
// pitch a multiple of 64 elements, so every wavefront access is one contiguous
// 64-element span and a tile's rows are one contiguous region (a single
// buffer descriptor covers all nine populations of a tile).
//
// Arithmetic: with b^2 = 1/3 the equilibrium and forcing populations times 36
// have small integer coefficients in (rho, j, P, S); they are formed exactly
// that way and divided by 36 once, with a two-term reciprocal (div36). Writing
// them with the rounded constants 1/3, 1/9, 1/36 instead biases every step in
// the same direction (the collision invariants drift by ~1e-8 per step in
// FP32), which grows linearly with the step count.
#include "lbm_device.h"

namespace lbm {
namespace {

using namespace dev;



// Pulled populations of a row without a horizontal wall (general addressing:
// used for halo columns and for tiles that touch a rigid side edge).
template <typename real>
__device__ __forceinline__ void pull_interior(const real *__restrict__ base, const GridDev &g,
                                              const Row &r, const Col &c, real out[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int row = CY[i] == 0 ? r.y : (CY[i] == 1 ? r.up : r.dn);
    const int col = CX[i] == 0 ? c.x : (CX[i] == 1 ? c.xl : c.xr);
    const bool xw = CX[i] == 1 ? c.wl : (CX[i] == -1 ? c.wr : false);
    const int64_t addr = xw ? qidx(g, OPP[i], r.y, c.x) : qidx(g, i, row, col);
    out[i] = base[addr];
  }
}

// Pulled populations of a row next to a horizontal wall.
template <typename real>
__device__ __forceinline__ void pull_wall(const real *__restrict__ base, const GridDev &g,
                                          const Row &r, const Col &c, real out[9]) {
  // The free surface needs rho and the tangential stress P_xx of the boundary
  // cell and of the cell inside it at time t-1: moments of the stored
  // post-collision populations (rho and P are collision invariants),
  // extrapolated half a cell out linearly (kFree, as printed) or taken from
  // the boundary cell (kFree0).
  real rho_air = real(0), pxx_air = real(0);
  const bool free_up = r.wall_up == kFree || r.wall_up == kFree0;
  const bool free_dn = r.wall_dn == kFree || r.wall_dn == kFree0;
  if (free_up || free_dn) {
    const int yin = free_up ? r.y + 1 : r.y - 1;
    const bool linear = (free_up ? r.wall_up : r.wall_dn) == kFree;
    real rb = 0, xb = 0, ri = 0, xi = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const real vb = base[qidx(g, i, r.y, c.x)];
      const real vi = base[qidx(g, i, yin, c.x)];
      rb += vb;
      ri += vi;
      if (CX[i] != 0) { xb += vb; xi += vi; }
    }
    rho_air = linear ? real(1.5) * rb - real(0.5) * ri : rb;
    pxx_air = linear ? real(1.5) * xb - real(0.5) * xi : xb;
  }
  // 36 x 2 w_i (rho_air + P^n_air : (c c - b^2 I) / (2 b^4)) for a link with
  // c_y^2 = 1, P^n_air = diag(P_xx,air - rho_air/3, -rho_air/3):
  //   vertical link 4 rho_air - 12 P_xx,air, diagonal link 6 P_xx,air - 2 rho_air.
  const real abb_axis = div36(real(4) * rho_air - real(12) * pxx_air);
  const real abb_diag = div36(real(6) * pxx_air - real(2) * rho_air);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int ywall = CY[i] == 1 ? r.wall_up : (CY[i] == -1 ? r.wall_dn : 0);
    const bool xw = CX[i] == 1 ? c.wl : (CX[i] == -1 ? c.wr : false);
    if (ywall == 0 && !xw) {
      const int row = CY[i] == 0 ? r.y : (CY[i] == 1 ? r.up : r.dn);
      const int col = CX[i] == 0 ? c.x : (CX[i] == 1 ? c.xl : c.xr);
      out[i] = base[qidx(g, i, row, col)];
    } else {
      const real refl = base[qidx(g, OPP[i], r.y, c.x)];
      if (xw || ywall == kRigid) out[i] = refl;
      else out[i] = -refl + (CX[i] == 0 ? abb_axis : abb_diag);
    }
  }
}

template <typename real>
__device__ __forceinline__ void pull(const real *__restrict__ base, const GridDev &g,
                                     const Row &r, const Col &c, real out[9]) {
  if ((r.wall_up | r.wall_dn) == 0) pull_interior(base, g, r, c, out);
  else pull_wall(base, g, r, c, out);
}


// Pull of an interior row (no horizontal wall, no wrap in y, no rigid side
// edge touched by the tile). rsrc is based at row ybase <= y - 1; rowb is the
// byte size of one row of nine population runs, qb of one run.
template <typename real>
__device__ __forceinline__ void pull_fast(__amdgpu_buffer_rsrc_t rsrc, int ybase, int y,
                                          uint32_t rowb, uint32_t qb, uint32_t o0, uint32_t ol,
                                          uint32_t orr, real out[9]) {
  const uint32_t rc = (uint32_t)(y - ybase) * rowb, ru = rc - rowb, rd = rc + rowb;
  out[0] = Buf<real>::load(rsrc, o0, rc);            // ( 0, 0)
  out[1] = Buf<real>::load(rsrc, ol, rc + qb);       // ( 1, 0) from (x-1, y)
  out[2] = Buf<real>::load(rsrc, o0, ru + 2 * qb);   // ( 0, 1) from (x, y-1)
  out[3] = Buf<real>::load(rsrc, orr, rc + 3 * qb);  // (-1, 0) from (x+1, y)
  out[4] = Buf<real>::load(rsrc, o0, rd + 4 * qb);   // ( 0,-1) from (x, y+1)
  out[5] = Buf<real>::load(rsrc, ol, ru + 5 * qb);   // ( 1, 1) from (x-1, y-1)
  out[6] = Buf<real>::load(rsrc, orr, ru + 6 * qb);  // (-1, 1) from (x+1, y-1)
  out[7] = Buf<real>::load(rsrc, orr, rd + 7 * qb);  // (-1,-1) from (x+1, y+1)
  out[8] = Buf<real>::load(rsrc, ol, rd + 8 * qb);   // ( 1,-1) from (x-1, y+1)
}

// Moments of the pulled populations with the flux and the sponge-corrected
// source: j = (m + G/2)/(1 + A/2), S = G - A j (eqs. MomentsFeq, S and
// MomentChainAbsorbing, the sponge term solved implicitly).
template <typename real>
struct CellState {
  real rho, jx, jy, pxx, pxy, pyy, Sx, Sy;
};

template <typename real>
__device__ __forceinline__ CellState<real> cell_state(const real f[9], real rho, real Gx, real Gy,
                                                      real A, real inv) {
  CellState<real> c;
  const real mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const real my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const real diag = (f[5] + f[6]) + (f[7] + f[8]);
  c.rho = rho;
  c.pxx = (f[1] + f[3]) + diag;
  c.pyy = (f[2] + f[4]) + diag;
  c.pxy = (f[5] + f[7]) - (f[6] + f[8]);
  c.jx = (mx + real(0.5) * Gx) * inv;
  c.jy = (my + real(0.5) * Gy) * inv;
  c.Sx = Gx - A * c.jx;
  c.Sy = Gy - A * c.jy;
  return c;
}

// BGK collision with forcing, f*_i = (1 - w) f_i + w f^eq_i + c_f S_i
// (w = 1/tau, c_f = 1 - 1/(2 tau); eqs. LBGK, equilibrium-solid, Pn, Si),
// written as f_i - w f_i + E_i / 36 with E_i = 36 (w f^eq_i + c_f S_i):
// 36 f^eq_i and 36 S_i have integer coefficients in rho, j, P, S (b^2 = 1/3;
// weights 16, 4, 1 over 36), and the j- and S-terms share their coefficients,
// so E_i is the equilibrium combination of (w rho, w j + c_f S, w P).
template <typename real>
__device__ __forceinline__ void collide(const real f[9], const CellState<real> &c, real omega,
                                        real cforce, real out[9]) {
  const real wr = omega * c.rho, wxx = omega * c.pxx, wyy = omega * c.pyy, wxy = omega * c.pxy;
  const real ux = fma(omega, c.jx, cforce * c.Sx);
  const real uy = fma(omega, c.jy, cforce * c.Sy);
  const real spp = wxx + wyy;
  const real e0 = real(32) * wr - real(24) * spp;
  const real ax = real(2) * wr + real(12) * wxx - real(6) * wyy;
  const real ay = real(2) * wr + real(12) * wyy - real(6) * wxx;
  const real d = real(3) * spp - wr;
  const real u12x = real(12) * ux, u12y = real(12) * uy;
  const real tp = real(3) * (ux + uy), tm = real(3) * (uy - ux), q9 = real(9) * wxy;
  const real E[9] = {e0, ax + u12x, ay + u12y, ax - u12x, ay - u12y,
                     d + tp + q9, d + tm - q9, d - tp + q9, d - tm - q9};
#pragma unroll
  for (int i = 0; i < 9; ++i) out[i] = fma(-omega, f[i], f[i]) + div36(E[i]);
}


template <typename real, int NW, int MODE, int PF>
__global__ __launch_bounds__(64 * NW) void step_kernel(StepArgs<real> a) {
  constexpr int W = 64 * NW;
  __shared__ real srho[2][W + 2];

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;                        // padding block (uniform)
  if (MODE == kModeMoments && tile.g != a.mom_grid) return;
  const GridDev &g = a.grids[tile.g];
  const real *__restrict__ fin = a.fin + g.f_off;
  const int pitch = g.pitch, nx = g.nx, ny = g.ny, rr = g.rigid_row;

  const int lane = threadIdx.x;
  const int x = tile.x0 + lane;
  const bool active = x < nx;
  const int xa = active ? x : nx - 1;
  const Col col = make_col(g, xa);
  const int x_last = min(tile.x0 + W, nx) - 1;
  const uint32_t o0 = (uint32_t)xa * sizeof(real);
  const uint32_t ol = (uint32_t)col.xl * sizeof(real);
  const uint32_t orr = (uint32_t)col.xr * sizeof(real);
  // Tiles that touch a rigid side edge take the general pull on every row.
  const bool fast_x = !((g.bc[kEdgeLeft] == kRigid && tile.x0 == 0) ||
                        (g.bc[kEdgeRight] == kRigid && x_last == nx - 1));

  // Lanes 0 and 1 also pull the tile's outer neighbour columns (for the
  // density gradient of the tile's first and last column).
  int hx = 0;
  bool hvalid = false;
  if (lane == 0) {
    hx = tile.x0 - 1;
    hvalid = true;
    if (hx < 0) { hvalid = g.bc[kEdgeLeft] == kPeriodic; hx = nx - 1; }
  } else if (lane == 1) {
    hx = x_last + 1;
    hvalid = true;
    if (hx >= nx) { hvalid = g.bc[kEdgeRight] == kPeriodic; hx = 0; }
  }
  const bool hlane = lane < 2 && hvalid;
  const Col hcol = make_col(g, hx);
  const int hslot = lane == 0 ? 0 : W + 1;

  const int64_t t = a.t + (a.t_dev ? a.t_dev[0] : 0);
  const real omega = a.omega;
  const real cforce = a.cforce;
  const bool px = g.bc[kEdgeLeft] == kPeriodic;
  const bool py = g.bc[kEdgeTop] == kPeriodic;
  const int y0 = tile.y0, y1 = tile.y1;
  // One descriptor per direction for all rows the tile touches (from two
  // rows above its first row, the lowest row an interior pull reads).
  const int ybase = max(y0 - 2, 0);
  const uint32_t qb = (uint32_t)pitch * sizeof(real);
  const uint32_t rowb = 9 * qb;
  const __amdgpu_buffer_rsrc_t rin = tile_rsrc(fin + (int64_t)ybase * 9 * pitch);
  const __amdgpu_buffer_rsrc_t rout = tile_rsrc(a.fout + g.f_off + (int64_t)ybase * 9 * pitch);

  real A_x, inv_x;
  sponge_x(a.sponge, g, xa, A_x, inv_x);

  // Rows with a horizontal wall link or a wrap in y.
  auto special = [&](int y) -> bool {
    return y == 0 || y == ny - 1 || (rr > 0 && (y == rr - 1 || y == rr));
  };
  auto pull_row = [&](int y, real out[9]) {
    if (fast_x && !special(y)) pull_fast(rin, ybase, y, rowb, qb, o0, ol, orr, out);
    else pull(fin, g, make_row(g, y), col, out);
  };
  auto pull_halo = [&](int y) -> real {
    real fh[9];
    pull(fin, g, make_row(g, y), hcol, fh);
    return sum9(fh);
  };
  // Whether the row after y is pulled while marching: as the next output row,
  // or for the density gradient of row y.
  auto need_after = [&](int y) -> bool {
    if (row_after(g, y) < 0) return false;
    if (y + 1 < y1) return true;
    return !special(y) || make_row(g, y).wall_dn == 0;
  };

  // Prologue: density of the row above the tile and the first row.
  int wall_up = special(y0) ? make_row(g, y0).wall_up : 0;
  real rho_m = real(0);
  if (wall_up == 0) {
    const int ya = y0 > 0 ? y0 - 1 : ny - 1;
    real fm[9];
    pull_row(ya, fm);
    rho_m = sum9(fm);
  }
  real fa[9], fb[9], hb[9];
  pull_row(y0, fa);
  real rho_c = sum9(fa);
  srho[0][lane + 1] = rho_c;
  if (lane < 2) srho[0][hslot] = hlane ? pull_halo(y0) : real(0);
  bool nb = need_after(y0);
  int yb = nb ? row_after(g, y0) : y0;
  if (PF == 2) {
#pragma unroll
    for (int i = 0; i < 9; ++i) { fb[i] = real(0); hb[i] = real(0); }
    if (nb) {
      pull_row(yb, fb);
      if (hlane) pull(fin, g, make_row(g, yb), hcol, hb);
    }
  }
  __syncthreads();

  for (int y = y0, k = 0; y < y1; ++y, ++k) {
    const int wall_dn = special(y) ? make_row(g, y).wall_dn : 0;
    real rho_n = real(0), hr_n = real(0);
    bool nc = false;
    int yc = y;
    real fc[9], hc[9];
    if (PF == 2) {
      // Row y+1 (fb) has been in flight since the previous iteration; issue
      // row y+2 now so it is in flight while row y is computed.
      if (nb) { rho_n = sum9(fb); hr_n = sum9(hb); }
      nc = nb && (y + 1 < y1) && need_after(yb);
      yc = nc ? row_after(g, yb) : y;
#pragma unroll
      for (int i = 0; i < 9; ++i) { fc[i] = real(0); hc[i] = real(0); }
      if (nc) {
        pull_row(yc, fc);
        if (hlane) pull(fin, g, make_row(g, yc), hcol, hc);
      }
    } else {
      nb = need_after(y);
      yb = nb ? row_after(g, y) : y;
      if (nb) {
        pull_row(yb, fb);
        rho_n = sum9(fb);
        if (hlane) hr_n = pull_halo(yb);
      }
    }

    const int s = k & 1;
    const real rho_l = srho[s][lane];
    const real rho_r = (xa == x_last) ? srho[s][W + 1] : srho[s][lane + 2];
    if (nb) {
      srho[s ^ 1][lane + 1] = rho_n;
      if (lane < 2) srho[s ^ 1][hslot] = hr_n;
    }

    // Centred density gradient (eq. FDrho); one-sided next to walls.
    real dx, dy;
    if (col.wl) dx = rho_r - rho_c;
    else if (col.wr) dx = rho_c - rho_l;
    else dx = real(0.5) * (rho_r - rho_l);
    if (wall_up) dy = rho_n - rho_c;
    else if (wall_dn) dy = rho_c - rho_m;
    else dy = real(0.5) * (rho_n - rho_m);

    const real kap = cell_kappa(a.kappa_rows, a.kappa_cells, g, y, xa);
    real A = A_x, inv = inv_x;
    sponge_y(a.sponge, g, y, A, inv);

    // Body force (Gaussian x Ricker), only on rows within 9 sigma of a source.
    real Fx = real(0), Fy = real(0);
    for (int si = 0; si < g.nsrc; ++si) {
      const SourceDev sd = a.sources[g.src_off + si];
      const double ddy = min_image((double)y - sd.y, ny, py);
      const double cut = 81.0 * sd.sigma * sd.sigma;
      if (ddy * ddy > cut) continue;
      const double R = ricker((double)t, sd.period, sd.t0);
      const double ddx = min_image((double)xa - sd.x, nx, px);
      const double r2 = ddx * ddx + ddy * ddy;
      if (r2 <= cut) {
        const double mag = sd.amp * exp(-r2 / (2.0 * sd.sigma * sd.sigma)) * R;
        Fx += (real)(mag * sd.dir_x);
        Fy += (real)(mag * sd.dir_y);
      }
    }

    const real Gx = kap * dx + Fx;
    const real Gy = kap * dy + Fy;
    const CellState<real> cs = cell_state(fa, rho_c, Gx, Gy, A, inv);
    const real rho = cs.rho, jx = cs.jx, jy = cs.jy, pxx = cs.pxx, pxy = cs.pxy, pyy = cs.pyy;

    if (MODE == kModeMoments) {
      if (active) {
        const int64_t n = (int64_t)nx * ny;
        const int64_t o = (int64_t)y * nx + x;
        a.mom[o] = rho;
        a.mom[n + o] = jx;
        a.mom[2 * n + o] = jy;
        a.mom[3 * n + o] = pxx;
        a.mom[4 * n + o] = pxy;
        a.mom[5 * n + o] = pyy;
      }
    } else {
      // the density of the step: the adjoint's recompute (kModeStash), or a
      // recorded forward step that keeps it (kModeStep with rho_out set)
      if (a.rho_out && active) a.rho_out[g.c_off + (int64_t)y * pitch + x] = rho;
      // Receivers on this row.
      if (MODE == kModeStep && g.nrec > 0) {
        const int slot = a.itab[g.rowtab_off + y];
        if (slot >= 0 && active) {
          int rid = a.itab[g.rmap_off + (int64_t)slot * nx + x];
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
      if (active) {
        real fs[9];
        collide(fa, cs, omega, cforce, fs);
        const uint32_t rs = (uint32_t)(y - ybase) * rowb;
#pragma unroll
        for (int i = 0; i < 9; ++i) Buf<real>::store_nt_device(fs[i], rout, o0, rs + i * qb);
      }
    }

    // March: row y+1 becomes current (and row y+2 is in flight).
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      fa[i] = fb[i];
      if (PF == 2) { fb[i] = fc[i]; hb[i] = hc[i]; }
    }
    if (PF == 2) { yb = yc; nb = nc; }
    wall_up = (y + 1 < y1 && special(y + 1)) ? make_row(g, y + 1).wall_up : 0;
    rho_m = rho_c;
    rho_c = rho_n;
  }
}

// The step for interior tiles: every row the tile pulls (one above, its own,
// one below) is at least one row away from a horizontal wall or wrap, every
// column it touches (with its halo) has both x-neighbours inside the grid or
// wraps periodically, no source band reaches its rows and no receiver sits
// in them. The host sorts tiles into this list; the arithmetic is the same
// code as the general kernel's, so a cell's result does not depend on which
// kernel updated it.
template <typename real, int NW, bool STASH>
__global__ __launch_bounds__(64 * NW) void interior_kernel(StepArgs<real> a) {
  constexpr int W = 64 * NW;
  __shared__ real srho[2][W + 2];

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;                        // padding block (uniform)
  const GridDev &g = a.grids[tile.g];
  const real *__restrict__ fin = a.fin + g.f_off;
  const int pitch = g.pitch, nx = g.nx;

  const int lane = threadIdx.x;
  const int x = tile.x0 + lane;
  const bool active = x < nx;
  const int xa = active ? x : nx - 1;
  const int x_last = min(tile.x0 + W, nx) - 1;
  const uint32_t esz = sizeof(real);
  auto wrapx = [&](int c) { return c < 0 ? c + nx : (c >= nx ? c - nx : c); };
  const uint32_t o0 = (uint32_t)xa * esz;
  const uint32_t ol = (uint32_t)wrapx(xa - 1) * esz;
  const uint32_t orr = (uint32_t)wrapx(xa + 1) * esz;
  // Halo columns (lanes 0 and 1).
  const int hx = lane == 0 ? wrapx(tile.x0 - 1) : wrapx(x_last + 1);
  const uint32_t ho0 = (uint32_t)hx * esz;
  const uint32_t hol = (uint32_t)wrapx(hx - 1) * esz;
  const uint32_t hor = (uint32_t)wrapx(hx + 1) * esz;
  const int hslot = lane == 0 ? 0 : W + 1;

  const real omega = a.omega;
  const real cforce = a.cforce;
  const int y0 = tile.y0, y1 = tile.y1;
  const int ybase = y0 - 2;
  const uint32_t qb = (uint32_t)pitch * esz;
  const uint32_t rowb = 9 * qb;
  const __amdgpu_buffer_rsrc_t rin = tile_rsrc(fin + (int64_t)ybase * 9 * pitch);
  const __amdgpu_buffer_rsrc_t rout = tile_rsrc(a.fout + g.f_off + (int64_t)ybase * 9 * pitch);

  real A_x, inv_x;
  sponge_x(a.sponge, g, xa, A_x, inv_x);

  real fa[9], fb[9];
  pull_fast(rin, ybase, y0 - 1, rowb, qb, o0, ol, orr, fa);
  real rho_m = sum9(fa);
  pull_fast(rin, ybase, y0, rowb, qb, o0, ol, orr, fa);
  real rho_c = sum9(fa);
  srho[0][lane + 1] = rho_c;
  if (lane < 2) {
    real fh[9];
    pull_fast(rin, ybase, y0, rowb, qb, ho0, hol, hor, fh);
    srho[0][hslot] = sum9(fh);
  }
  __syncthreads();

  for (int y = y0, k = 0; y < y1; ++y, ++k) {
    pull_fast(rin, ybase, y + 1, rowb, qb, o0, ol, orr, fb);
    const real rho_n = sum9(fb);
    real hr_n = real(0);
    if (lane < 2) {
      real fh[9];
      pull_fast(rin, ybase, y + 1, rowb, qb, ho0, hol, hor, fh);
      hr_n = sum9(fh);
    }
    const int s = k & 1;
    const real rho_l = srho[s][lane];
    const real rho_r = (xa == x_last) ? srho[s][W + 1] : srho[s][lane + 2];
    srho[s ^ 1][lane + 1] = rho_n;
    if (lane < 2) srho[s ^ 1][hslot] = hr_n;

    // Centred density gradient (eq. FDrho) and the source (eq. S).
    const real dx = real(0.5) * (rho_r - rho_l);
    const real dy = real(0.5) * (rho_n - rho_m);
    const real kap = cell_kappa(a.kappa_rows, a.kappa_cells, g, y, xa);
    real A = A_x, inv = inv_x;
    sponge_y(a.sponge, g, y, A, inv);
    const CellState<real> cs = cell_state(fa, rho_c, kap * dx, kap * dy, A, inv);
    if (active) {
      if (STASH) a.rho_out[g.c_off + (int64_t)y * pitch + x] = rho_c;
      real fs[9];
      collide(fa, cs, omega, cforce, fs);
      const uint32_t rs = (uint32_t)(y - ybase) * rowb;
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf<real>::store_nt_device(fs[i], rout, o0, rs + i * qb);
    }

    __syncthreads();
#pragma unroll
    for (int i = 0; i < 9; ++i) fa[i] = fb[i];
    rho_m = rho_c;
    rho_c = rho_n;
  }
}

// Pair of one population run shifted by one column: (x-1, x) for dir = -1,
// (x+1, x+2) for dir = +1, with the periodic wrap for the pair that straddles
// the x edge (two single loads there).
template <typename real>
__device__ __forceinline__ Pair<real> load_shift(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                                 bool wrap, uint32_t last_off) {
  if (wrap) return {Buf<real>::load(r, last_off, soff), Buf<real>::load(r, 0, soff)};
  return Buf2<real>::load(r, voff, soff);
}

// Pulled populations of the column pair (x, x+1) of an interior row.
template <typename real>
__device__ __forceinline__ void pull_pair(__amdgpu_buffer_rsrc_t rsrc, int ybase, int y, uint32_t rowb,
                                          uint32_t qb, uint32_t o0, uint32_t ol, uint32_t orr,
                                          bool wl, bool wr, uint32_t last_off, real u[9], real v[9]) {
  const uint32_t rc = (uint32_t)(y - ybase) * rowb, ru = rc - rowb, rd = rc + rowb;
  Pair<real> p;
  p = Buf2<real>::load(rsrc, o0, rc);                            u[0] = p.a; v[0] = p.b;
  p = load_shift<real>(rsrc, ol, rc + qb, wl, last_off);         u[1] = p.a; v[1] = p.b;
  p = Buf2<real>::load(rsrc, o0, ru + 2 * qb);                   u[2] = p.a; v[2] = p.b;
  p = load_shift<real>(rsrc, orr, rc + 3 * qb, wr, last_off);    u[3] = p.a; v[3] = p.b;
  p = Buf2<real>::load(rsrc, o0, rd + 4 * qb);                   u[4] = p.a; v[4] = p.b;
  p = load_shift<real>(rsrc, ol, ru + 5 * qb, wl, last_off);     u[5] = p.a; v[5] = p.b;
  p = load_shift<real>(rsrc, orr, ru + 6 * qb, wr, last_off);    u[6] = p.a; v[6] = p.b;
  p = load_shift<real>(rsrc, orr, rd + 7 * qb, wr, last_off);    u[7] = p.a; v[7] = p.b;
  p = load_shift<real>(rsrc, ol, rd + 8 * qb, wl, last_off);     u[8] = p.a; v[8] = p.b;
}

// Interior tiles with two columns per lane (grids with an even nx): the same
// per-cell arithmetic as interior_kernel, half the memory instructions per
// byte. A tile is 128*NW columns wide.
template <typename real, int NW>
__global__ __launch_bounds__(64 * NW) void interior2_kernel(StepArgs<real> a) {
  constexpr int L = 64 * NW;     // lanes
  constexpr int W = 2 * L;       // columns
  __shared__ real srho[2][W + 2];

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;
  const GridDev &g = a.grids[tile.g];
  const real *__restrict__ fin = a.fin + g.f_off;
  const int pitch = g.pitch, nx = g.nx;

  const int lane = threadIdx.x;
  const int x = tile.x0 + 2 * lane;
  const bool active = x < nx;
  const int xa = active ? x : nx - 2;
  const int x_last = min(tile.x0 + W, nx) - 1;
  const uint32_t esz = sizeof(real);
  auto wrapx = [&](int c) { return c < 0 ? c + nx : (c >= nx ? c - nx : c); };
  const uint32_t o0 = (uint32_t)xa * esz;
  const bool wl = xa == 0, wr = xa + 2 == nx;
  const uint32_t ol = wl ? 0u : (uint32_t)(xa - 1) * esz;
  const uint32_t orr = wr ? 0u : (uint32_t)(xa + 1) * esz;
  const uint32_t last_off = (uint32_t)(nx - 1) * esz;
  const int hx = lane == 0 ? wrapx(tile.x0 - 1) : wrapx(x_last + 1);
  const uint32_t ho0 = (uint32_t)hx * esz;
  const uint32_t hol = (uint32_t)wrapx(hx - 1) * esz;
  const uint32_t hor = (uint32_t)wrapx(hx + 1) * esz;
  const int hslot = lane == 0 ? 0 : W + 1;

  const real omega = a.omega;
  const real cforce = a.cforce;
  const int y0 = tile.y0, y1 = tile.y1;
  const int ybase = y0 - 2;
  const uint32_t qb = (uint32_t)pitch * esz;
  const uint32_t rowb = 9 * qb;
  const __amdgpu_buffer_rsrc_t rin = tile_rsrc(fin + (int64_t)ybase * 9 * pitch);
  const __amdgpu_buffer_rsrc_t rout = tile_rsrc(a.fout + g.f_off + (int64_t)ybase * 9 * pitch);

  real A0, inv0, A1, inv1;
  sponge_x(a.sponge, g, xa, A0, inv0);
  sponge_x(a.sponge, g, xa + 1, A1, inv1);

  real ua[9], va[9], ub[9], vb[9];
  pull_pair(rin, ybase, y0 - 1, rowb, qb, o0, ol, orr, wl, wr, last_off, ua, va);
  real rm0 = sum9(ua), rm1 = sum9(va);
  pull_pair(rin, ybase, y0, rowb, qb, o0, ol, orr, wl, wr, last_off, ua, va);
  real rc0 = sum9(ua), rc1 = sum9(va);
  srho[0][2 * lane + 1] = rc0;
  srho[0][2 * lane + 2] = rc1;
  if (lane < 2) {
    real fh[9];
    pull_fast(rin, ybase, y0, rowb, qb, ho0, hol, hor, fh);
    srho[0][hslot] = sum9(fh);
  }
  __syncthreads();

  for (int y = y0, k = 0; y < y1; ++y, ++k) {
    pull_pair(rin, ybase, y + 1, rowb, qb, o0, ol, orr, wl, wr, last_off, ub, vb);
    const real rn0 = sum9(ub), rn1 = sum9(vb);
    real hr_n = real(0);
    if (lane < 2) {
      real fh[9];
      pull_fast(rin, ybase, y + 1, rowb, qb, ho0, hol, hor, fh);
      hr_n = sum9(fh);
    }
    const int s = k & 1;
    const real rl = srho[s][2 * lane];
    const real rr = (xa + 1 == x_last) ? srho[s][W + 1] : srho[s][2 * lane + 3];
    srho[s ^ 1][2 * lane + 1] = rn0;
    srho[s ^ 1][2 * lane + 2] = rn1;
    if (lane < 2) srho[s ^ 1][hslot] = hr_n;

    const real kap0 = cell_kappa(a.kappa_rows, a.kappa_cells, g, y, xa), kap1 = cell_kappa(a.kappa_rows, a.kappa_cells, g, y, xa + 1);
    real Ay0 = A0, iy0 = inv0, Ay1 = A1, iy1 = inv1;
    sponge_y(a.sponge, g, y, Ay0, iy0);
    sponge_y(a.sponge, g, y, Ay1, iy1);
    const real dx0 = real(0.5) * (rc1 - rl), dy0 = real(0.5) * (rn0 - rm0);
    const real dx1 = real(0.5) * (rr - rc0), dy1 = real(0.5) * (rn1 - rm1);
    const CellState<real> c0 = cell_state(ua, rc0, kap0 * dx0, kap0 * dy0, Ay0, iy0);
    const CellState<real> c1 = cell_state(va, rc1, kap1 * dx1, kap1 * dy1, Ay1, iy1);
    if (active) {
      real f0[9], f1[9];
      collide(ua, c0, omega, cforce, f0);
      collide(va, c1, omega, cforce, f1);
      const uint32_t rs = (uint32_t)(y - ybase) * rowb;
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf2<real>::store_nt(f0[i], f1[i], rout, o0, rs + i * qb);
    }

    __syncthreads();
#pragma unroll
    for (int i = 0; i < 9; ++i) { ua[i] = ub[i]; va[i] = vb[i]; }
    rm0 = rc0; rm1 = rc1;
    rc0 = rn0; rc1 = rn1;
  }
}


// Two time steps of an interior tile in one pass (temporal blocking). The
// workgroup marches down the tile's rows with a four-stage pipeline:
//   A (row r):   pull f(t) from f*(t-1) in HBM (row r+1 already in flight),
//                rho(t) into an LDS ring;
//   B (row r-1): density gradient and collision of step t -> f*(t);
//   C (row r-2): pull f(t+1) from f*(t) of rows r-3 .. r-1, rho(t+1) into an
//                LDS ring;
//   D (row r-3): density gradient and collision of step t+1 -> f*(t+1) to HBM.
// Of f*(t), only the six populations that stage C takes from a neighbouring
// column go through LDS, each in a ring as deep as the rows it must wait
// (c_y = -1: this row, c_y = 0: one more, c_y = +1: two more); the three
// with c_x = 0 stay in the lane's registers. Stage B runs on the tile's
// columns plus three halo columns on each side and stage C on two, so stage
// D has every neighbour it needs; the four left halo columns (and the right
// ones of a full-width tile) are handled by an extra wavefront, so the
// output wavefronts keep aligned accesses. Rows: output rows [y0, y1) need
// f*(t) on rows y0-2 .. y1+1 and f*(t-1) on rows y0-4 .. y1+3. The row loop
// is unrolled six times, the period of its register rotations, so that
// rotating the carried rows costs no moves; the first iterations before
// row y0-3 only start the loads. The per-cell arithmetic is the single-step
// kernels' (same operations in the same order), so two steps here equal two
// single steps bit for bit. Tiles are clear of walls, the y-wrap, source
// disks and receivers over that whole reach.
template <int N>
struct Phase {
  static constexpr int value = N;
};

template <typename real, int NW, bool STASH>
__global__ __launch_bounds__(64 * NW + 64, sizeof(real) == 4 ? 5 : 3)
    void fused2_kernel(
    StepArgs<real> a) {
  constexpr int W = 64 * NW;
  constexpr int LW = W + 8;                 // LDS columns: tile plus 4 each side
  constexpr int RT = kFusedMaxRows + 8;     // per-row table: rows y0-4 .. y1+3
  __shared__ real sA[2][LW];                // rho(t) of rows r-1, r
  __shared__ real sC[2][LW];                // rho(t+1) of rows r-3, r-2
  __shared__ real s78[2][LW];               // f*(t) populations 7, 8 of row r-1
  __shared__ real s13[2][2][LW];            // populations 1, 3 of rows r-2, r-1
  __shared__ real s56[3][2][LW];            // populations 5, 6 of rows r-3 .. r-1
  __shared__ real sRowA[RT], sRowI[RT], sRowK[RT];

  const FusedTileDev tile = a.ftiles[blockIdx.x];
  if (tile.g < 0) return;
  const GridDev g = uniform_lookup_fields(a.grids[tile.g]);
  const int pitch = g.pitch, nx = g.nx;
  const int w = tile.x1 - tile.x0;          // 0 < w <= W
  const int tid = threadIdx.x;
  const int hl = tid - W;
  // LDS column lc of column x0 - 4 + lc: 0..3 the left halo (lanes of the
  // extra wavefront), 4..w+3 the tile, w+4..w+7 the right halo (the next
  // output lanes, or the extra wavefront's lanes 4..7 for a full tile)
  int lc = -1;
  if (tid < W) lc = tid + 4;
  else if (hl < 4) lc = hl;
  else if (hl < 8) lc = W + hl;
  const bool live = lc >= 0 && lc < w + 8;
  const bool outlane = tid < w;
  auto wrapx = [&](int c) { return c < 0 ? c + nx : (c >= nx ? c - nx : c); };
  // the lanes outside the block's columns (the halo wavefront's last 56, the
  // lanes past a narrow block) load a live lane's column: their unconditional
  // loads then touch no line the block does not need
  const int col = wrapx(tile.x0 - 4 + min(max(lc, 0), w + 7));
  const uint32_t esz = sizeof(real);
  const uint32_t o0 = (uint32_t)col * esz;
  const uint32_t ol = (uint32_t)wrapx(col - 1) * esz;
  const uint32_t orr = (uint32_t)wrapx(col + 1) * esz;

  const real omega = a.omega, cforce = a.cforce;
  const int y0 = tile.y0, y1 = tile.y1;
  const int ybase = y0 - 4;
  const uint32_t qb = (uint32_t)pitch * esz;
  const uint32_t rowb = 9 * qb;
  const int64_t base = g.f_off + (int64_t)ybase * 9 * pitch;
  const uint64_t rest = (uint64_t)(a.f_elems - base) * esz;
  const __amdgpu_buffer_rsrc_t rin = range_rsrc(a.fin + base, rest);
  const __amdgpu_buffer_rsrc_t rout = range_rsrc(a.fout + base, rest);

  // Per-row look-ups of the tile's rows, read once: the top/bottom sponge
  // pair of the row (combined with the column's pair by the same max/min as
  // the single-step kernels, exact operations, so the order does not matter)
  // and the row's modulus for layered media. The row loop then issues no
  // global loads besides the populations (and the modulus of cell-wise media).
  const int nrows = y1 - y0 + 8;
  for (int k = tid; k < nrows; k += W + 64) {
    real Ay = real(0), Iy = real(1);
    sponge_y(a.sponge, g, ybase + k, Ay, Iy);
    sRowA[k] = Ay;
    sRowI[k] = Iy;
    sRowK[k] = g.kmode == kKappaRows ? a.kappa_rows[g.k_off + ybase + k] : real(0);
  }
  real A_x, inv_x;
  sponge_x(a.sponge, g, col, A_x, inv_x);
  const bool kcells = g.kmode == kKappaCells;
  const real kscalar = (real)g.kscalar;
  // the cell-wise moduli from row ybase on (an empty range for the other
  // kinds of medium: their loads return 0, with no branch around them, which
  // would end in a wait for every load in flight)
  const __amdgpu_buffer_rsrc_t rk = range_rsrc(
      a.kappa_cells + (kcells ? g.k_off + (int64_t)ybase * pitch : 0),
      kcells ? (uint64_t)(g.ny - ybase) * pitch * sizeof(real) : 0);
  const bool inB = lc >= 1 && lc <= w + 6, inC = lc >= 2 && lc <= w + 5;
  __syncthreads();

  // Registers carried down the rows, each set rotated with its period:
  // F the pulled f(t) of rows r-1, r and r+1 (in flight), G the pulled
  // f(t+1) of rows r-3 and r-2, RA / RC rho(t) / rho(t+1) of three rows,
  // D0 / E2 populations 0 and 2 of f*(t) waiting one and two rows for stage
  // C; for cell-wise moduli, the modulus of rows r+1 (in flight) .. r-3.
  real F[3][9], G[2][9], D0[2], E2[3], RA[3], RC[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) { F[0][i] = F[1][i] = F[2][i] = G[0][i] = G[1][i] = real(0); }
  D0[0] = D0[1] = E2[0] = E2[1] = E2[2] = real(0);
  RA[0] = RA[1] = RA[2] = RC[0] = RC[1] = RC[2] = real(0);
  real kq = real(0), k1 = real(0), k2 = real(0), k3 = real(0);

  const int rlast = y1 + 2;
  // iterations from y0-4 (which only starts the loads of row y0-3) to rlast,
  // rounded up to whole unrolled rounds by starting earlier
  const int r0 = rlast + 1 - (rlast - (y0 - 4) + 1 + 5) / 6 * 6;

  // first: the loop's first round of six rows, whose early rows (before
  // y0-3, run only to fill the pipeline) load nothing.
  auto iter = [&](const int r, auto ph, auto first) {
    constexpr int P = decltype(ph)::value;
    real(&fa)[9] = F[P % 3];
    real(&fb)[9] = F[(P + 1) % 3];
    real(&fc)[9] = F[(P + 2) % 3];
    real(&gc)[9] = G[P % 2];
    real(&gn)[9] = G[(P + 1) % 2];
    real &rA_n = RA[P % 3], &rA_c = RA[(P + 2) % 3], &rA_m = RA[(P + 1) % 3];
    real &rC_n = RC[P % 3], &rC_c = RC[(P + 2) % 3], &rC_m = RC[(P + 1) % 3];
    real kn = real(0);
    // The row index and the store offset below go through an empty asm:
    // otherwise the compiler keeps every population's offset of every
    // unrolled row as its own scalar induction variable and spills them.
    if (decltype(first)::value) {
      if (live && r + 1 >= y0 - 3) {
        int rn = r + 1;
        asm volatile("" : "+s"(rn));
        pull_fast(rin, ybase, rn, rowb, qb, o0, ol, orr, fc);
        kn = Buf<real>::load(rk, o0, (uint32_t)(rn - ybase) * qb);
      }
    } else {
      // After the first round every lane loads a row on every iteration
      // (the row past rlast clamped to rlast, loaded again and not used), so
      // that every path through the loop issues the same loads and the waits
      // of stage A leave this prefetch in flight.
      int rn = min(r + 1, rlast);
      asm volatile("" : "+s"(rn));
      pull_fast(rin, ybase, rn, rowb, qb, o0, ol, orr, fc);
      kn = Buf<real>::load(rk, o0, (uint32_t)(rn - ybase) * qb);
    }
    // Stage A: row r of step t.
    rA_n = real(0);
    if (live && r >= y0 - 3) {
      rA_n = sum9(fb);
      sA[r & 1][lc] = rA_n;
      if (STASH && outlane && r >= y0 && r < y1) a.rho_out[g.c_off + (int64_t)r * pitch + col] = rA_n;
    }
    // Stage B: row r-1 of step t (needs rho(t) of rows r-2 .. r).
    const int rb = r - 1;
    real p0 = real(0), p2 = real(0), p4 = real(0);
    if (rb >= y0 - 2 && inB) {
      const real dx = real(0.5) * (sA[rb & 1][lc + 1] - sA[rb & 1][lc - 1]);
      const real dy = real(0.5) * (rA_n - rA_m);
      const real kap = kcells ? k1 : (g.kmode == kKappaRows ? sRowK[rb - ybase] : kscalar);
      const real A = max(A_x, sRowA[rb - ybase]), inv = min(inv_x, sRowI[rb - ybase]);
      const CellState<real> cs = cell_state(fa, rA_c, kap * dx, kap * dy, A, inv);
      real s1[9];
      collide(fa, cs, omega, cforce, s1);
      s78[0][lc] = s1[7];
      s78[1][lc] = s1[8];
      s13[rb & 1][0][lc] = s1[1];
      s13[rb & 1][1][lc] = s1[3];
      s56[rb % 3][0][lc] = s1[5];
      s56[rb % 3][1][lc] = s1[6];
      p0 = s1[0];
      p2 = s1[2];
      p4 = s1[4];
    }
    __syncthreads();
    // Stage C: row r-2 of step t+1, pulled from f*(t) of rows r-3 .. r-1.
    const int rc = r - 2;
    rC_n = real(0);
    if (rc >= y0 - 1 && inC) {
      const int s13i = rc & 1, s56i = (rc + 2) % 3;   // rows rc and rc-1
      gn[0] = D0[P % 2];                            // row rc, this column
      gn[1] = s13[s13i][0][lc - 1];
      gn[2] = E2[P % 3];                            // row rc-1, this column
      gn[3] = s13[s13i][1][lc + 1];
      gn[4] = p4;                                   // row rc+1, this column
      gn[5] = s56[s56i][0][lc - 1];
      gn[6] = s56[s56i][1][lc + 1];
      gn[7] = s78[0][lc + 1];
      gn[8] = s78[1][lc - 1];
      rC_n = sum9(gn);
      sC[rc & 1][lc] = rC_n;
      if (STASH && outlane && rc >= y0 && rc < y1) a.rho_out2[g.c_off + (int64_t)rc * pitch + col] = rC_n;
    }
    // Stage D: row r-3 of step t+1 (needs rho(t+1) of rows r-4 .. r-2).
    const int rd = r - 3;
    if (rd >= y0 && outlane) {
      const real dx = real(0.5) * (sC[rd & 1][lc + 1] - sC[rd & 1][lc - 1]);
      const real dy = real(0.5) * (rC_n - rC_m);
      const real kap = kcells ? k3 : (g.kmode == kKappaRows ? sRowK[rd - ybase] : kscalar);
      const real A = max(A_x, sRowA[rd - ybase]), inv = min(inv_x, sRowI[rd - ybase]);
      const CellState<real> cs = cell_state(gc, rC_c, kap * dx, kap * dy, A, inv);
      real s2[9];
      collide(gc, cs, omega, cforce, s2);
      uint32_t rs = (uint32_t)(rd - ybase) * rowb;
      asm volatile("" : "+s"(rs));
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf<real>::store_nt_device(s2[i], rout, o0, rs + i * qb);
    }
    __syncthreads();
    D0[(P + 1) % 2] = p0;
    E2[(P + 2) % 3] = p2;
    k3 = k2; k2 = k1; k1 = kq; kq = kn;
  };

  // at least one round: rlast - r0 + 1 is a positive multiple of six
  using First = std::true_type;
  using Steady = std::false_type;
  iter(r0, Phase<0>{}, First{});
  iter(r0 + 1, Phase<1>{}, First{});
  iter(r0 + 2, Phase<2>{}, First{});
  iter(r0 + 3, Phase<3>{}, First{});
  iter(r0 + 4, Phase<4>{}, First{});
  iter(r0 + 5, Phase<5>{}, First{});
  for (int r = r0 + 6; r <= rlast; r += 6) {
    iter(r, Phase<0>{}, Steady{});
    iter(r + 1, Phase<1>{}, Steady{});
    iter(r + 2, Phase<2>{}, Steady{});
    iter(r + 3, Phase<3>{}, Steady{});
    iter(r + 4, Phase<4>{}, Steady{});
    iter(r + 5, Phase<5>{}, Steady{});
  }
}


// Three time steps of an interior tile in one pass: the two-step kernel's
// pipeline with a third pair of stages. At iteration r:
//   A (row r):   pull f(t) from f*(t-1) in HBM (row r+1 already in flight),
//                rho(t) into an LDS ring;
//   B (row r-1): gradient and collision of step t -> f*(t) (LDS rings and
//                registers, as in the two-step kernel);
//   C (row r-2): pull f(t+1) from f*(t), rho(t+1) into an LDS ring;
//   D (row r-3): gradient and collision of step t+1 -> f*(t+1), into a
//                second set of rings of the same shape;
//   E (row r-4): pull f(t+2) from f*(t+1), rho(t+2) into an LDS ring;
//   F (row r-5): gradient and collision of step t+2 -> f*(t+2) to HBM.
// Each stage runs on one column fewer on each side than the one before:
// A on the tile plus five halo columns each side, F on the tile's own
// columns (the halo columns are lanes of an extra wavefront as in the
// two-step kernel). Rows: output rows [y0, y1) need f*(t-1) on rows
// y0-6 .. y1+5. Two barriers per iteration suffice: one after B (C reads
// B's rings) and one after D (E reads D's); the next iteration's A and B
// touch nothing E and F read, and the ring depths keep every slot a stage
// reads apart from the slots written before the next barrier. The per-cell
// arithmetic is the single-step kernels', so three steps here equal three
// single steps bit for bit. Tiles are clear of walls, the y-wrap, source
// disks and receivers over that whole reach.
template <typename real, int NW>
__global__ __launch_bounds__(64 * NW + 64, sizeof(real) == 4 ? 4 : 2)
    void fused3_kernel(StepArgs<real> a) {
  constexpr int W = 64 * NW;
  constexpr int HC = 5;                     // halo columns each side
  constexpr int LW = W + 2 * HC;            // LDS columns
  constexpr int RT = kFusedMaxRows + 12;    // per-row table: rows y0-6 .. y1+5
  __shared__ real sA[2][LW];                // rho(t)
  __shared__ real sC[2][LW];                // rho(t+1)
  __shared__ real sE[2][LW];                // rho(t+2)
  __shared__ real s78[2][LW], s13[2][2][LW], s56[3][2][LW];   // f*(t) from B
  __shared__ real u78[2][LW], u13[2][2][LW], u56[3][2][LW];   // f*(t+1) from D
  __shared__ real sRowA[RT], sRowI[RT], sRowK[RT];

  const FusedTileDev tile = a.ftiles[blockIdx.x];
  if (tile.g < 0) return;
  const GridDev g = uniform_lookup_fields(a.grids[tile.g]);
  const int pitch = g.pitch, nx = g.nx;
  const int w = tile.x1 - tile.x0;          // 0 < w <= W
  const int tid = threadIdx.x;
  const int hl = tid - W;
  // LDS column lc of column x0 - 5 + lc: 0..4 the left halo (lanes of the
  // extra wavefront), 5..w+4 the tile, w+5..w+9 the right halo (the next
  // output lanes, or the extra wavefront's lanes 5..9 past a full tile)
  int lc = -1;
  if (tid < W) lc = tid + HC;
  else if (hl < HC) lc = hl;
  else if (hl < 2 * HC) lc = W + hl;
  const bool live = lc >= 0 && lc < w + 2 * HC;
  const bool outlane = tid < w;
  auto wrapx = [&](int c) { return c < 0 ? c + nx : (c >= nx ? c - nx : c); };
  // lanes outside the block's columns load a live lane's column
  const int col = wrapx(tile.x0 - HC + min(max(lc, 0), w + 2 * HC - 1));
  const uint32_t esz = sizeof(real);
  const uint32_t o0 = (uint32_t)col * esz;
  const uint32_t ol = (uint32_t)wrapx(col - 1) * esz;
  const uint32_t orr = (uint32_t)wrapx(col + 1) * esz;

  const real omega = a.omega, cforce = a.cforce;
  const int y0 = tile.y0, y1 = tile.y1;
  const int ybase = y0 - 6;
  const uint32_t qb = (uint32_t)pitch * esz;
  const uint32_t rowb = 9 * qb;
  const int64_t base = g.f_off + (int64_t)ybase * 9 * pitch;
  const uint64_t rest = (uint64_t)(a.f_elems - base) * esz;
  const __amdgpu_buffer_rsrc_t rin = range_rsrc(a.fin + base, rest);
  const __amdgpu_buffer_rsrc_t rout = range_rsrc(a.fout + base, rest);

  const int nrows = y1 - y0 + 12;
  for (int k = tid; k < nrows; k += W + 64) {
    real Ay = real(0), Iy = real(1);
    sponge_y(a.sponge, g, ybase + k, Ay, Iy);
    sRowA[k] = Ay;
    sRowI[k] = Iy;
    sRowK[k] = g.kmode == kKappaRows ? a.kappa_rows[g.k_off + ybase + k] : real(0);
  }
  real A_x, inv_x;
  sponge_x(a.sponge, g, col, A_x, inv_x);
  const bool kcells = g.kmode == kKappaCells;
  const real kscalar = (real)g.kscalar;
  const __amdgpu_buffer_rsrc_t rk = range_rsrc(
      a.kappa_cells + (kcells ? g.k_off + (int64_t)ybase * pitch : 0),
      kcells ? (uint64_t)(g.ny - ybase) * pitch * sizeof(real) : 0);
  const int lmax = w + 2 * HC - 1;
  const bool inB = lc >= 1 && lc <= lmax - 1, inC = lc >= 2 && lc <= lmax - 2;
  const bool inD = lc >= 3 && lc <= lmax - 3, inE = lc >= 4 && lc <= lmax - 4;
  __syncthreads();

  // Registers carried down the rows: F the pulled f(t) of rows r-1, r, r+1
  // (in flight); G / H the pulled f(t+1) / f(t+2) of two rows each; RA, RC,
  // RE rho(t), rho(t+1), rho(t+2) of three rows; D0 / E2 and D0b / E2b
  // populations 0 and 2 of f*(t) and f*(t+1) waiting one and two rows; the
  // cell-wise modulus of rows r+1 (in flight) .. r-5.
  real F[3][9], G[2][9], H[2][9], D0[2], E2[3], D0b[2], E2b[3], RA[3], RC[3], RE[3];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    F[0][i] = F[1][i] = F[2][i] = real(0);
    G[0][i] = G[1][i] = H[0][i] = H[1][i] = real(0);
  }
  D0[0] = D0[1] = D0b[0] = D0b[1] = real(0);
  E2[0] = E2[1] = E2[2] = E2b[0] = E2b[1] = E2b[2] = real(0);
  RA[0] = RA[1] = RA[2] = RC[0] = RC[1] = RC[2] = RE[0] = RE[1] = RE[2] = real(0);
  real kq = real(0), k1 = real(0), k2 = real(0), k3 = real(0), k4 = real(0), k5 = real(0);

  const int rlast = y1 + 4;
  // iterations from y0-6 (which only starts the loads of row y0-5) to rlast,
  // rounded up to whole unrolled rounds by starting earlier
  const int r0 = rlast + 1 - (rlast - (y0 - 6) + 1 + 5) / 6 * 6;

  auto iter = [&](const int r, auto ph, auto first) {
    constexpr int P = decltype(ph)::value;
    real(&fa)[9] = F[P % 3];
    real(&fb)[9] = F[(P + 1) % 3];
    real(&fc)[9] = F[(P + 2) % 3];
    real(&gc)[9] = G[P % 2];
    real(&gn)[9] = G[(P + 1) % 2];
    real(&hc)[9] = H[P % 2];
    real(&hn)[9] = H[(P + 1) % 2];
    real &rA_n = RA[P % 3], &rA_c = RA[(P + 2) % 3], &rA_m = RA[(P + 1) % 3];
    real &rC_n = RC[P % 3], &rC_c = RC[(P + 2) % 3], &rC_m = RC[(P + 1) % 3];
    real &rE_n = RE[P % 3], &rE_c = RE[(P + 2) % 3], &rE_m = RE[(P + 1) % 3];
    real kn = real(0);
    if (decltype(first)::value) {
      if (live && r + 1 >= y0 - 5) {
        int rn = r + 1;
        asm volatile("" : "+s"(rn));
        pull_fast(rin, ybase, rn, rowb, qb, o0, ol, orr, fc);
        kn = Buf<real>::load(rk, o0, (uint32_t)(rn - ybase) * qb);
      }
    } else {
      int rn = min(r + 1, rlast);
      asm volatile("" : "+s"(rn));
      pull_fast(rin, ybase, rn, rowb, qb, o0, ol, orr, fc);
      kn = Buf<real>::load(rk, o0, (uint32_t)(rn - ybase) * qb);
    }
    // Stage A: row r of step t.
    rA_n = real(0);
    if (live && r >= y0 - 5) {
      rA_n = sum9(fb);
      sA[r & 1][lc] = rA_n;
    }
    // Stage B: row r-1 of step t.
    const int rb = r - 1;
    real p0 = real(0), p2 = real(0), p4 = real(0);
    if (rb >= y0 - 4 && inB) {
      const real dx = real(0.5) * (sA[rb & 1][lc + 1] - sA[rb & 1][lc - 1]);
      const real dy = real(0.5) * (rA_n - rA_m);
      const real kap = kcells ? k1 : (g.kmode == kKappaRows ? sRowK[rb - ybase] : kscalar);
      const real A = max(A_x, sRowA[rb - ybase]), inv = min(inv_x, sRowI[rb - ybase]);
      const CellState<real> cs = cell_state(fa, rA_c, kap * dx, kap * dy, A, inv);
      real s1[9];
      collide(fa, cs, omega, cforce, s1);
      s78[0][lc] = s1[7];
      s78[1][lc] = s1[8];
      s13[rb & 1][0][lc] = s1[1];
      s13[rb & 1][1][lc] = s1[3];
      s56[rb % 3][0][lc] = s1[5];
      s56[rb % 3][1][lc] = s1[6];
      p0 = s1[0];
      p2 = s1[2];
      p4 = s1[4];
    }
    __syncthreads();
    // Stage C: row r-2 of step t+1, pulled from f*(t) of rows r-3 .. r-1.
    const int rc = r - 2;
    rC_n = real(0);
    if (rc >= y0 - 3 && inC) {
      const int s13i = rc & 1, s56i = (rc + 2) % 3;
      gn[0] = D0[P % 2];
      gn[1] = s13[s13i][0][lc - 1];
      gn[2] = E2[P % 3];
      gn[3] = s13[s13i][1][lc + 1];
      gn[4] = p4;
      gn[5] = s56[s56i][0][lc - 1];
      gn[6] = s56[s56i][1][lc + 1];
      gn[7] = s78[0][lc + 1];
      gn[8] = s78[1][lc - 1];
      rC_n = sum9(gn);
      sC[rc & 1][lc] = rC_n;
    }
    // Stage D: row r-3 of step t+1.
    const int rd = r - 3;
    real q0 = real(0), q2 = real(0), q4 = real(0);
    if (rd >= y0 - 2 && inD) {
      const real dx = real(0.5) * (sC[rd & 1][lc + 1] - sC[rd & 1][lc - 1]);
      const real dy = real(0.5) * (rC_n - rC_m);
      const real kap = kcells ? k3 : (g.kmode == kKappaRows ? sRowK[rd - ybase] : kscalar);
      const real A = max(A_x, sRowA[rd - ybase]), inv = min(inv_x, sRowI[rd - ybase]);
      const CellState<real> cs = cell_state(gc, rC_c, kap * dx, kap * dy, A, inv);
      real s2[9];
      collide(gc, cs, omega, cforce, s2);
      u78[0][lc] = s2[7];
      u78[1][lc] = s2[8];
      u13[rd & 1][0][lc] = s2[1];
      u13[rd & 1][1][lc] = s2[3];
      u56[rd % 3][0][lc] = s2[5];
      u56[rd % 3][1][lc] = s2[6];
      q0 = s2[0];
      q2 = s2[2];
      q4 = s2[4];
    }
    __syncthreads();
    // Stage E: row r-4 of step t+2, pulled from f*(t+1) of rows r-5 .. r-3.
    const int re = r - 4;
    rE_n = real(0);
    if (re >= y0 - 1 && inE) {
      const int u13i = re & 1, u56i = (re + 2) % 3;
      hn[0] = D0b[P % 2];
      hn[1] = u13[u13i][0][lc - 1];
      hn[2] = E2b[P % 3];
      hn[3] = u13[u13i][1][lc + 1];
      hn[4] = q4;
      hn[5] = u56[u56i][0][lc - 1];
      hn[6] = u56[u56i][1][lc + 1];
      hn[7] = u78[0][lc + 1];
      hn[8] = u78[1][lc - 1];
      rE_n = sum9(hn);
      sE[re & 1][lc] = rE_n;
    }
    // Stage F: row r-5 of step t+2 to HBM.
    const int rf = r - 5;
    if (rf >= y0 && outlane) {
      const real dx = real(0.5) * (sE[rf & 1][lc + 1] - sE[rf & 1][lc - 1]);
      const real dy = real(0.5) * (rE_n - rE_m);
      const real kap = kcells ? k5 : (g.kmode == kKappaRows ? sRowK[rf - ybase] : kscalar);
      const real A = max(A_x, sRowA[rf - ybase]), inv = min(inv_x, sRowI[rf - ybase]);
      const CellState<real> cs = cell_state(hc, rE_c, kap * dx, kap * dy, A, inv);
      real s3[9];
      collide(hc, cs, omega, cforce, s3);
      uint32_t rs = (uint32_t)(rf - ybase) * rowb;
      asm volatile("" : "+s"(rs));
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf<real>::store_nt_device(s3[i], rout, o0, rs + i * qb);
    }
    D0[(P + 1) % 2] = p0;
    E2[(P + 2) % 3] = p2;
    D0b[(P + 1) % 2] = q0;
    E2b[(P + 2) % 3] = q2;
    k5 = k4; k4 = k3; k3 = k2; k2 = k1; k1 = kq; kq = kn;
  };

  using First = std::true_type;
  using Steady = std::false_type;
  iter(r0, Phase<0>{}, First{});
  iter(r0 + 1, Phase<1>{}, First{});
  iter(r0 + 2, Phase<2>{}, First{});
  iter(r0 + 3, Phase<3>{}, First{});
  iter(r0 + 4, Phase<4>{}, First{});
  iter(r0 + 5, Phase<5>{}, First{});
  for (int r = r0 + 6; r <= rlast; r += 6) {
    iter(r, Phase<0>{}, Steady{});
    iter(r + 1, Phase<1>{}, Steady{});
    iter(r + 2, Phase<2>{}, Steady{});
    iter(r + 3, Phase<3>{}, Steady{});
    iter(r + 4, Phase<4>{}, Steady{});
    iter(r + 5, Phase<5>{}, Steady{});
  }
}

}  // namespace

template <typename real>
hipError_t launch_step(const StepArgs<real> &a, int waves, int prefetch, int ntiles, int mode,
                       hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves);
#define LBM_LAUNCH(NW, MODE, PF) \
  hipLaunchKernelGGL((step_kernel<real, NW, MODE, PF>), grid, block, 0, stream, a)
  if (mode == kModeStash) {
    if (waves == 1) LBM_LAUNCH(1, kModeStash, 1);
    else if (waves == 2) LBM_LAUNCH(2, kModeStash, 1);
    else if (waves == 4) LBM_LAUNCH(4, kModeStash, 1);
    else if (waves == 8) LBM_LAUNCH(8, kModeStash, 1);
    else return hipErrorInvalidValue;
  } else if (mode == kModeStep) {
    if (prefetch == 2) {
      if (waves == 1) LBM_LAUNCH(1, kModeStep, 2);
      else if (waves == 2) LBM_LAUNCH(2, kModeStep, 2);
      else if (waves == 4) LBM_LAUNCH(4, kModeStep, 2);
      else if (waves == 8) LBM_LAUNCH(8, kModeStep, 2);
      else return hipErrorInvalidValue;
    } else {
      if (waves == 1) LBM_LAUNCH(1, kModeStep, 1);
      else if (waves == 2) LBM_LAUNCH(2, kModeStep, 1);
      else if (waves == 4) LBM_LAUNCH(4, kModeStep, 1);
      else if (waves == 8) LBM_LAUNCH(8, kModeStep, 1);
      else return hipErrorInvalidValue;
    }
  } else {
    if (waves == 1) LBM_LAUNCH(1, kModeMoments, 1);
    else if (waves == 2) LBM_LAUNCH(2, kModeMoments, 1);
    else if (waves == 4) LBM_LAUNCH(4, kModeMoments, 1);
    else if (waves == 8) LBM_LAUNCH(8, kModeMoments, 1);
    else return hipErrorInvalidValue;
  }
#undef LBM_LAUNCH
  return hipGetLastError();
}

// waves: the tile width in units of 64 columns; pair = 1 selects the
// two-column kernel (waves/2 wavefronts per workgroup).
template <typename real>
hipError_t launch_interior(const StepArgs<real> &a, int waves, int pair, int ntiles,
                           hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles);
  if (a.rho_out) {
    dim3 block(64 * waves);
    if (waves == 1) hipLaunchKernelGGL((interior_kernel<real, 1, true>), grid, block, 0, stream, a);
    else if (waves == 2) hipLaunchKernelGGL((interior_kernel<real, 2, true>), grid, block, 0, stream, a);
    else if (waves == 4) hipLaunchKernelGGL((interior_kernel<real, 4, true>), grid, block, 0, stream, a);
    else if (waves == 8) hipLaunchKernelGGL((interior_kernel<real, 8, true>), grid, block, 0, stream, a);
    else return hipErrorInvalidValue;
  } else if (pair) {
    dim3 block(32 * waves);
    if (waves == 2) hipLaunchKernelGGL((interior2_kernel<real, 1>), grid, block, 0, stream, a);
    else if (waves == 4) hipLaunchKernelGGL((interior2_kernel<real, 2>), grid, block, 0, stream, a);
    else if (waves == 8) hipLaunchKernelGGL((interior2_kernel<real, 4>), grid, block, 0, stream, a);
    else return hipErrorInvalidValue;
  } else {
    dim3 block(64 * waves);
    if (waves == 1) hipLaunchKernelGGL((interior_kernel<real, 1, false>), grid, block, 0, stream, a);
    else if (waves == 2) hipLaunchKernelGGL((interior_kernel<real, 2, false>), grid, block, 0, stream, a);
    else if (waves == 4) hipLaunchKernelGGL((interior_kernel<real, 4, false>), grid, block, 0, stream, a);
    else if (waves == 8) hipLaunchKernelGGL((interior_kernel<real, 8, false>), grid, block, 0, stream, a);
    else return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


template <typename real>
hipError_t launch_fused2(const StepArgs<real> &a, int waves, int ntiles, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves + 64);
  if (a.rho_out) {
    if (waves == 2) hipLaunchKernelGGL((fused2_kernel<real, 2, true>), grid, block, 0, stream, a);
    else if (waves == 4) hipLaunchKernelGGL((fused2_kernel<real, 4, true>), grid, block, 0, stream, a);
    else if (waves == 8) hipLaunchKernelGGL((fused2_kernel<real, 8, true>), grid, block, 0, stream, a);
    else return hipErrorInvalidValue;
  } else if (waves == 2) hipLaunchKernelGGL((fused2_kernel<real, 2, false>), grid, block, 0, stream, a);
  else if (waves == 4) hipLaunchKernelGGL((fused2_kernel<real, 4, false>), grid, block, 0, stream, a);
  else if (waves == 8) hipLaunchKernelGGL((fused2_kernel<real, 8, false>), grid, block, 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename real>
hipError_t launch_fused3(const StepArgs<real> &a, int waves, int ntiles, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves + 64);
  if (waves == 2) hipLaunchKernelGGL((fused3_kernel<real, 2>), grid, block, 0, stream, a);
  else if (waves == 3) hipLaunchKernelGGL((fused3_kernel<real, 3>), grid, block, 0, stream, a);
  else if (waves == 4) hipLaunchKernelGGL((fused3_kernel<real, 4>), grid, block, 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_fused2<float>(const StepArgs<float> &, int, int, hipStream_t);
template hipError_t launch_fused2<double>(const StepArgs<double> &, int, int, hipStream_t);
template hipError_t launch_fused3<float>(const StepArgs<float> &, int, int, hipStream_t);
template hipError_t launch_fused3<double>(const StepArgs<double> &, int, int, hipStream_t);

template hipError_t launch_interior<float>(const StepArgs<float> &, int, int, int, hipStream_t);
template hipError_t launch_interior<double>(const StepArgs<double> &, int, int, int, hipStream_t);
template hipError_t launch_step<float>(const StepArgs<float> &, int, int, int, int, hipStream_t);
template hipError_t launch_step<double>(const StepArgs<double> &, int, int, int, int, hipStream_t);

}  // namespace lbm
