// Discrete adjoint of the fused D2Q9 elastic-wave step, for gfx950.
//
// With kappa, the sponge and the sources fixed, one forward step maps the
// pulled populations f(t) to f(t+1) linearly plus a source term, and the
// receivers read a linear function of f(t). For a misfit L of the traces the
// adjoint populations fh(t) = dL/df(t) obey
//     fh(t) = Coll^T Stream^T fh(t+1) + Rec^T e(t),    fh(T) = 0,
// e(t) = dL/dv(t) being the trace residual. One launch takes one such step
// for every grid of a context; the shape follows the forward kernel with
// every arrow reversed. A workgroup owns a tile of 64*NW columns and marches
// down its rows; for each row it
//   1. pulls ah_k(x) = fh_k(x + c_k, t+1) -- the transpose of pull streaming
//      is a pull from the opposite side -- and, on links that cross a wall,
//      fh of the reversed population of the same cell (rigid bounce-back,
//      eq. BB) or its negative (free-surface anti-bounce-back, Sec. 6.2);
//   2. adds the receiver residual to the adjoint of the flux j and transposes
//      the collision: the flux and the implicit sponge (eq.
//      MomentChainAbsorbing), the forcing populations (eq. Si) and the
//      equilibrium (eqs. equilibrium-solid, Pn) give the adjoints of rho, m,
//      P and of the source G = kappa grad(rho) + F (eq. S);
//   3. transposes the finite-difference gradient of eq. FDrho: kappa * Gh of
//      the cell's four neighbours (a two-row LDS ring of the x-component plus
//      registers for the rows above and below, as the forward keeps rho)
//      flows back onto rho, with the one-sided weights next to walls;
//   4. transposes the moments (and the free-surface extrapolation of rho and
//      P_xx, which read the boundary row and the row inside it) and writes
//      fh(t), one store per population;
//   5. accumulates the gradients in FP64: dL/dkappa(x) += Gh . grad(rho)(x, t)
//      with grad(rho)(t) from the density stash of the forward recompute, and
//      dL/damp_s += Gh . d_s gauss_s(x) ricker_s(t), reduced over each
//      wavefront and the workgroup before one atomic add per source.
#include "lbm_device.h"

namespace lbm {
namespace {

using namespace dev;

// Step 1: transposed streaming of one cell.
template <typename real>
__device__ __forceinline__ void adj_pull(const real *__restrict__ base, const GridDev &g,
                                         const Row &r, const Col &c, real out[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    // the link leaves the cell along c_i: down (row r.dn) for c_y = +1
    const int ywall = CY[i] == 1 ? r.wall_dn : (CY[i] == -1 ? r.wall_up : 0);
    const bool xw = CX[i] == 1 ? c.wr : (CX[i] == -1 ? c.wl : false);
    if (ywall == 0 && !xw) {
      const int row = CY[i] == 0 ? r.y : (CY[i] == 1 ? r.dn : r.up);
      const int col = CX[i] == 0 ? c.x : (CX[i] == 1 ? c.xr : c.xl);
      out[i] = base[qidx(g, i, row, col)];
    } else {
      const real refl = base[qidx(g, OPP[i], r.y, c.x)];
      out[i] = (xw || ywall == kRigid) ? refl : -refl;
    }
  }
}

// Step 2 for one cell: from ah (the adjoint of f*) and the receiver term
// (the adjoint of j from the traces) to the adjoints of G and of m.
// With b^2 = 1/3, sum_k w_k c_k ah_k / b^2 = (4 (ah_1 - ah_3) + ah_5 - ah_6
// - ah_7 + ah_8) / 12 along x (likewise along y) is the adjoint shared by
// the equilibrium's j-term (weight omega) and the forcing term (weight c_f).
template <typename real>
__device__ __forceinline__ void adj_local(const real as[9], real recx, real recy, real A, real inv,
                                          real omega, real cforce, real &Gx, real &Gy, real &mx,
                                          real &my) {
  const real r12 = real(1) / real(12);
  const real ux = (real(4) * (as[1] - as[3]) + ((as[5] - as[6]) - (as[7] - as[8]))) * r12;
  const real uy = (real(4) * (as[2] - as[4]) + ((as[5] + as[6]) - (as[7] + as[8]))) * r12;
  const real sx = cforce * ux, sy = cforce * uy;        // adjoint of S
  const real jx = fma(omega, ux, recx) - A * sx;        // adjoint of j, S = G - A j
  const real jy = fma(omega, uy, recy) - A * sy;
  mx = jx * inv;                                        // j = (m + G/2) / (1 + A/2)
  my = jy * inv;
  Gx = fma(real(0.5), mx, sx);
  Gy = fma(real(0.5), my, sy);
}

// Step 4 for one cell: fh_k = (1 - w) ah_k + w (E_k / 36) + r + m.c_k + p c_kx^2,
// where E_k / 36 collects the adjoints of rho and P through the equilibrium
// (36 x its weights: rho 32, 2, -1; P_xx -24, 12 / -6, 3; P_xy 9 on the
// diagonals), r the density adjoint from the gradient and the free surface,
// p the free-surface P_xx adjoint.
template <typename real>
__device__ __forceinline__ void adj_finish(const real as[9], real omega, real r, real mx, real my,
                                           real p, real out[9]) {
  const real sa = (as[1] + as[3]) + (as[2] + as[4]);
  const real sd = (as[5] + as[6]) + (as[7] + as[8]);
  const real R36 = (real(32) * as[0] + real(2) * sa) - sd;
  const real xx = real(12) * (as[1] + as[3]) - real(6) * (as[2] + as[4]);
  const real yy = real(12) * (as[2] + as[4]) - real(6) * (as[1] + as[3]);
  const real Pxx36 = (real(3) * sd - real(24) * as[0]) + xx;
  const real Pyy36 = (real(3) * sd - real(24) * as[0]) + yy;
  const real Pxy36 = real(9) * ((as[5] + as[7]) - (as[6] + as[8]));
  const real ea = R36 + Pxx36, eb = R36 + Pyy36, ed = ea + Pyy36;
  const real E[9] = {R36, ea, eb, ea, eb, ed + Pxy36, ed - Pxy36, ed + Pxy36, ed - Pxy36};
  const real rp = r + p;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    real v = fma(-omega, as[k], as[k]) + div36(omega * E[k]);
    v += (CX[k] != 0 ? rp : r);
    if (CX[k] != 0) v += CX[k] > 0 ? mx : -mx;
    if (CY[k] != 0) v += CY[k] > 0 ? my : -my;
    out[k] = v;
  }
}

// Adjoint of the free-surface values of a boundary cell: the links that
// cross the surface carry (4 rho_air - 12 P_xx,air) / 36 (vertical) and
// (6 P_xx,air - 2 rho_air) / 36 (diagonal); fa, fd1, fd2 are fh of those
// links. Returns the adjoints of rho_air and P_xx,air.
template <typename real>
__device__ __forceinline__ void adj_abb(real fa, real fd1, real fd2, real &r, real &p) {
  const real d = fd1 + fd2;
  r = div36(real(4) * fa - real(2) * d);
  p = div36(real(6) * d - real(12) * fa);
}

template <typename real, int NW>
__global__ __launch_bounds__(64 * NW) void adjoint_kernel(AdjArgs<real> a) {
  constexpr int W = 64 * NW;
  __shared__ real sq[2][W + 2];
  __shared__ double samp[kMaxAdjSources];

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;
  const GridDev &g = a.grids[tile.g];
  const AdjGridDev io = a.io[tile.g];
  const real *__restrict__ fin = a.fin + g.f_off;
  real *__restrict__ fout = a.fout + g.f_off;
  const int nx = g.nx, ny = g.ny, pitch = g.pitch;

  const int lane = threadIdx.x;
  const int x = tile.x0 + lane;
  const bool active = x < nx;
  const int xa = active ? x : nx - 1;
  const Col col = make_col(g, xa);
  const int x_last = min(tile.x0 + W, nx) - 1;
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

  const int64_t t = a.t;
  const real omega = a.omega, cforce = a.cforce;
  const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
  const int nsrc = io.grad_amp ? min(g.nsrc, kMaxAdjSources) : 0;
  if (lane < kMaxAdjSources) samp[lane] = 0.0;

  // Weights of the transposed gradient from the x-neighbours: 1/2, or 1 from
  // a neighbour on a rigid side edge (its one-sided difference).
  const bool rigid_l = g.bc[kEdgeLeft] == kRigid, rigid_r = g.bc[kEdgeRight] == kRigid;
  const real wxl = (rigid_l && col.xl == 0) ? real(1) : real(0.5);
  const real wxr = (rigid_r && col.xr == nx - 1) ? real(1) : real(0.5);

  // Steps 1-2 for the cell (xc, r.y) of column c.
  auto cell = [&](const Row &r, const Col &c, int xc, real as[9], real &Gx, real &Gy, real &mx,
                  real &my) {
    adj_pull(fin, g, r, c, as);
    real recx = real(0), recy = real(0);
    if (g.nrec > 0 && io.residual) {
      const int slot = a.itab[g.rowtab_off + r.y];
      if (slot >= 0) {
        int rid = a.itab[g.rmap_off + (int64_t)slot * nx + xc];
        const int64_t tk = t - g.trace_t0;
        while (rid >= 0) {
          if (tk >= 0 && tk < g.trace_max) {
            const real sc = a.rtab[g.rscale_off + rid];
            const real *e = reinterpret_cast<const real *>(io.residual) + (tk * g.nrec + rid) * g.ncomp;
            int o = 0;
            if (g.comp_mask & 1) recx += e[o++] * sc;
            if (g.comp_mask & 2) recy += e[o] * sc;
          }
          rid = a.itab[g.rnext_off + rid];
        }
      }
    }
    real A, inv;
    sponge_x(a.sponge, g, xc, A, inv);
    sponge_y(a.sponge, g, r.y, A, inv);
    adj_local(as, recx, recy, A, inv, omega, cforce, Gx, Gy, mx, my);
  };

  const int y0 = tile.y0, y1 = tile.y1;
  Row rc = make_row(g, y0);
  // The row above the tile, when connected: its kappa * Gh_y and whether it
  // is a top-boundary row (one-sided difference, weight 1).
  real qy_m = real(0), wy_m = real(0.5);
  if (rc.wall_up == 0) {
    const Row ru = make_row(g, rc.up);
    real as_[9], gx_, gy_, mx_, my_;
    cell(ru, col, xa, as_, gx_, gy_, mx_, my_);
    qy_m = cell_kappa(a.kappa_rows, a.kappa_cells, g, ru.y, xa) * gy_;
    wy_m = ru.wall_up != 0 ? real(1) : real(0.5);
  }
  real as_c[9], gx_c, gy_c, mx_c, my_c;
  cell(rc, col, xa, as_c, gx_c, gy_c, mx_c, my_c);
  real kap_c = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, xa);
  sq[0][lane + 1] = kap_c * gx_c;
  if (lane < 2) {
    real hq = real(0);
    if (hlane) {
      real as_[9], gx_, gy_, mx_, my_;
      cell(rc, hcol, hx, as_, gx_, gy_, mx_, my_);
      hq = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, hx) * gx_;
    }
    sq[0][hslot] = hq;
  }
  __syncthreads();

  for (int y = y0, k = 0; y < y1; ++y, ++k) {
    // The next row: the next one of the tile, or the one below the tile's
    // last row when connected (its kappa * Gh_y).
    const bool in_tile = y + 1 < y1;
    const bool need_n = in_tile || rc.wall_dn == 0;
    const int yn = in_tile ? y + 1 : rc.dn;
    Row rn = rc;
    real as_n[9], gx_n = real(0), gy_n = real(0), mx_n = real(0), my_n = real(0), kap_n = real(0);
    real hq_n = real(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) as_n[i] = real(0);
    if (need_n) {
      rn = make_row(g, yn);
      cell(rn, col, xa, as_n, gx_n, gy_n, mx_n, my_n);
      kap_n = cell_kappa(a.kappa_rows, a.kappa_cells, g, yn, xa);
      if (in_tile && hlane) {
        real as_[9], gx_, gy_, mx_, my_;
        cell(rn, hcol, hx, as_, gx_, gy_, mx_, my_);
        hq_n = cell_kappa(a.kappa_rows, a.kappa_cells, g, yn, hx) * gx_;
      }
    }

    const int s = k & 1;
    const real qx_l = sq[s][lane];
    const real qx_r = (xa == x_last) ? sq[s][W + 1] : sq[s][lane + 2];
    if (in_tile) {
      sq[s ^ 1][lane + 1] = kap_n * gx_n;
      if (lane < 2) sq[s ^ 1][hslot] = hq_n;
    }

    // Step 3: transposed density gradient.
    const real qx_c = kap_c * gx_c, qy_c = kap_c * gy_c;
    const bool lo_y = rc.wall_up != 0, hi_y = rc.wall_dn != 0;
    real rD = real(0);
    if (col.wl) rD -= qx_c;
    else rD += wxl * qx_l;
    if (col.wr) rD += qx_c;
    else rD -= wxr * qx_r;
    if (lo_y) rD -= qy_c;
    else rD += wy_m * qy_m;
    if (hi_y) rD += qy_c;
    else rD -= (rn.wall_dn != 0 ? real(1) : real(0.5)) * (kap_n * gy_n);

    // Free-surface moment adjoints: the boundary row (extrapolation weight
    // 1.5 as printed, 1 for the zero-order rule) and the row inside it (-0.5).
    real fr = real(0), fp = real(0);
    // A diagonal link that also crosses a rigid side edge bounces back as
    // rigid and carries no free-surface term.
    auto abb_top = [&](int yb, real &r, real &p) {
      adj_abb(fin[qidx(g, 2, yb, xa)], col.wl ? real(0) : fin[qidx(g, 5, yb, xa)],
              col.wr ? real(0) : fin[qidx(g, 6, yb, xa)], r, p);
    };
    auto abb_bottom = [&](int yb, real &r, real &p) {
      adj_abb(fin[qidx(g, 4, yb, xa)], col.wr ? real(0) : fin[qidx(g, 7, yb, xa)],
              col.wl ? real(0) : fin[qidx(g, 8, yb, xa)], r, p);
    };
    if (rc.wall_up == kFree || rc.wall_up == kFree0) {
      real r, p;
      abb_top(y, r, p);
      const real cb = rc.wall_up == kFree ? real(1.5) : real(1);
      fr += cb * r;
      fp += cb * p;
    }
    if (rc.wall_dn == kFree || rc.wall_dn == kFree0) {
      real r, p;
      abb_bottom(y, r, p);
      const real cb = rc.wall_dn == kFree ? real(1.5) : real(1);
      fr += cb * r;
      fp += cb * p;
    }
    if (y == 1 && g.bc[kEdgeTop] == kFree) {
      real r, p;
      abb_top(0, r, p);
      fr -= real(0.5) * r;
      fp -= real(0.5) * p;
    }
    if (y == ny - 2 && g.bc[kEdgeBottom] == kFree) {
      real r, p;
      abb_bottom(ny - 1, r, p);
      fr -= real(0.5) * r;
      fp -= real(0.5) * p;
    }

    // Step 4.
    if (active) {
      real fh[9];
      adj_finish(as_c, omega, rD + fr, mx_c, my_c, fp, fh);
#pragma unroll
      for (int i = 0; i < 9; ++i) fout[qidx(g, i, y, x)] = fh[i];
    }

    // Step 5: gradients. grad(rho)(t) as the forward step formed it.
    if (active && io.grad_kappa) {
      const real *rs = a.rho + g.c_off;
      const real rho_c = rs[(int64_t)y * pitch + x];
      real dx, dy;
      if (col.wl) dx = rs[(int64_t)y * pitch + col.xr] - rho_c;
      else if (col.wr) dx = rho_c - rs[(int64_t)y * pitch + col.xl];
      else dx = real(0.5) * (rs[(int64_t)y * pitch + col.xr] - rs[(int64_t)y * pitch + col.xl]);
      if (lo_y) dy = rs[(int64_t)(y + 1) * pitch + x] - rho_c;
      else if (hi_y) dy = rho_c - rs[(int64_t)(y - 1) * pitch + x];
      else dy = real(0.5) * (rs[(int64_t)rc.dn * pitch + x] - rs[(int64_t)rc.up * pitch + x]);
      io.grad_kappa[(int64_t)y * nx + x] += (double)gx_c * (double)dx + (double)gy_c * (double)dy;
    }
    for (int si = 0; si < nsrc; ++si) {
      const SourceDev sd = a.sources[g.src_off + si];
      const double ddy = min_image((double)y - sd.y, ny, py);
      const double cut = 81.0 * sd.sigma * sd.sigma;
      if (ddy * ddy > cut) continue;                       // uniform across the workgroup
      const double ddx = min_image((double)xa - sd.x, nx, px);
      const double r2 = ddx * ddx + ddy * ddy;
      double v = 0.0;
      if (active && r2 <= cut)
        v = exp(-r2 / (2.0 * sd.sigma * sd.sigma)) * ricker((double)t, sd.period, sd.t0) *
            ((double)gx_c * sd.dir_x + (double)gy_c * sd.dir_y);
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((lane & 63) == 0) atomicAdd(&samp[si], v);
    }

    // March: row y+1 becomes current.
    __syncthreads();
    qy_m = qy_c;
    wy_m = lo_y ? real(1) : real(0.5);
    if (need_n) {
#pragma unroll
      for (int i = 0; i < 9; ++i) as_c[i] = as_n[i];
      gx_c = gx_n;
      gy_c = gy_n;
      mx_c = mx_n;
      my_c = my_n;
      kap_c = kap_n;
    }
    rc = rn;
  }
  if (lane < nsrc && samp[lane] != 0.0) atomicAdd(io.grad_amp + lane, samp[lane]);
}

// Transposed pull of an interior row (no wall, no wrap in y): ah_k(x) =
// fh_k(x + c_k) through the tile's buffer descriptor based at row ybase.
template <typename real>
__device__ __forceinline__ void adj_pull_fast(__amdgpu_buffer_rsrc_t rsrc, int ybase, int y,
                                              uint32_t rowb, uint32_t qb, uint32_t o0, uint32_t ol,
                                              uint32_t orr, real out[9]) {
  const uint32_t rc = (uint32_t)(y - ybase) * rowb, ru = rc - rowb, rd = rc + rowb;
  out[0] = Buf<real>::load(rsrc, o0, rc);            // ( 0, 0)
  out[1] = Buf<real>::load(rsrc, orr, rc + qb);      // ( 1, 0) from (x+1, y)
  out[2] = Buf<real>::load(rsrc, o0, rd + 2 * qb);   // ( 0, 1) from (x, y+1)
  out[3] = Buf<real>::load(rsrc, ol, rc + 3 * qb);   // (-1, 0) from (x-1, y)
  out[4] = Buf<real>::load(rsrc, o0, ru + 4 * qb);   // ( 0,-1) from (x, y-1)
  out[5] = Buf<real>::load(rsrc, orr, rd + 5 * qb);  // ( 1, 1) from (x+1, y+1)
  out[6] = Buf<real>::load(rsrc, ol, rd + 6 * qb);   // (-1, 1) from (x-1, y+1)
  out[7] = Buf<real>::load(rsrc, ol, ru + 7 * qb);   // (-1,-1) from (x-1, y-1)
  out[8] = Buf<real>::load(rsrc, orr, ru + 8 * qb);  // ( 1,-1) from (x+1, y-1)
}

// The adjoint step for interior tiles: every row the tile touches (one above
// and one below its own) is clear of walls and of the y-wrap, its columns
// (with the halo) have both x-neighbours inside the grid or wrap
// periodically, and no source band and no receiver reaches those rows. The
// per-cell arithmetic is the general kernel's.
template <typename real, int NW>
__global__ __launch_bounds__(64 * NW) void adjoint_interior_kernel(AdjArgs<real> a) {
  constexpr int W = 64 * NW;
  __shared__ real sq[2][W + 2];

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;
  const GridDev &g = a.grids[tile.g];
  double *__restrict__ gk = a.io[tile.g].grad_kappa;
  const int pitch = g.pitch, nx = g.nx;

  const int lane = threadIdx.x;
  const int x = tile.x0 + lane;
  const bool active = x < nx;
  const int xa = active ? x : nx - 1;
  const int x_last = min(tile.x0 + W, nx) - 1;
  const uint32_t esz = sizeof(real);
  auto wrapx = [&](int c) { return c < 0 ? c + nx : (c >= nx ? c - nx : c); };
  const int xl = wrapx(xa - 1), xr = wrapx(xa + 1);
  const uint32_t o0 = (uint32_t)xa * esz, ol = (uint32_t)xl * esz, orr = (uint32_t)xr * esz;
  const int hx = lane == 0 ? wrapx(tile.x0 - 1) : wrapx(x_last + 1);
  const uint32_t ho0 = (uint32_t)hx * esz;
  const uint32_t hol = (uint32_t)wrapx(hx - 1) * esz;
  const uint32_t hor = (uint32_t)wrapx(hx + 1) * esz;
  const int hslot = lane == 0 ? 0 : W + 1;

  const real omega = a.omega, cforce = a.cforce;
  const int y0 = tile.y0, y1 = tile.y1;
  const int ybase = y0 - 2;
  const uint32_t qb = (uint32_t)pitch * esz;
  const uint32_t rowb = 9 * qb;
  const __amdgpu_buffer_rsrc_t rin = tile_rsrc(a.fin + g.f_off + (int64_t)ybase * 9 * pitch);
  const __amdgpu_buffer_rsrc_t rout = tile_rsrc(a.fout + g.f_off + (int64_t)ybase * 9 * pitch);
  const __amdgpu_buffer_rsrc_t rrho = tile_rsrc(a.rho + g.c_off + (int64_t)ybase * pitch);

  real A_x, inv_x, hA_x, hinv_x;
  sponge_x(a.sponge, g, xa, A_x, inv_x);
  sponge_x(a.sponge, g, hx, hA_x, hinv_x);

  // Steps 1-2 for the lane's column (or the halo column) of row y.
  auto cell = [&](int y, bool halo, real as[9], real &Gx, real &Gy, real &mx, real &my) {
    if (halo) adj_pull_fast(rin, ybase, y, rowb, qb, ho0, hol, hor, as);
    else adj_pull_fast(rin, ybase, y, rowb, qb, o0, ol, orr, as);
    real A = halo ? hA_x : A_x, inv = halo ? hinv_x : inv_x;
    sponge_y(a.sponge, g, y, A, inv);
    adj_local(as, real(0), real(0), A, inv, omega, cforce, Gx, Gy, mx, my);
  };

  real as_c[9], gx_c, gy_c, mx_c, my_c;
  real qy_m;
  {
    real t_[9], gx_, gy_, mx_, my_;
    cell(y0 - 1, false, t_, gx_, gy_, mx_, my_);
    qy_m = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0 - 1, xa) * gy_;
  }
  cell(y0, false, as_c, gx_c, gy_c, mx_c, my_c);
  real kap_c = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, xa);
  sq[0][lane + 1] = kap_c * gx_c;
  if (lane < 2) {
    real t_[9], gx_, gy_, mx_, my_;
    cell(y0, true, t_, gx_, gy_, mx_, my_);
    sq[0][hslot] = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, hx) * gx_;
  }
  __syncthreads();

  for (int y = y0, k = 0; y < y1; ++y, ++k) {
    real as_n[9], gx_n, gy_n, mx_n, my_n;
    cell(y + 1, false, as_n, gx_n, gy_n, mx_n, my_n);
    const real kap_n = cell_kappa(a.kappa_rows, a.kappa_cells, g, y + 1, xa);
    real hq_n = real(0);
    if (lane < 2) {
      real t_[9], gx_, gy_, mx_, my_;
      cell(y + 1, true, t_, gx_, gy_, mx_, my_);
      hq_n = cell_kappa(a.kappa_rows, a.kappa_cells, g, y + 1, hx) * gx_;
    }
    const int s = k & 1;
    const real qx_l = sq[s][lane];
    const real qx_r = (xa == x_last) ? sq[s][W + 1] : sq[s][lane + 2];
    sq[s ^ 1][lane + 1] = kap_n * gx_n;
    if (lane < 2) sq[s ^ 1][hslot] = hq_n;

    // Step 3 (centred differences only) and step 4.
    const real rD = real(0.5) * ((qx_l - qx_r) + (qy_m - kap_n * gy_n));
    if (active) {
      real fh[9];
      adj_finish(as_c, omega, rD, mx_c, my_c, real(0), fh);
      const uint32_t rs = (uint32_t)(y - ybase) * rowb;
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf<real>::store_nt(fh[i], rout, o0, rs + i * qb);
      // Step 5: dL/dkappa += Gh . grad(rho)(t).
      const uint32_t pr = (uint32_t)(y - ybase) * qb;
      const real dx = real(0.5) * (Buf<real>::load(rrho, orr, pr) - Buf<real>::load(rrho, ol, pr));
      const real dy = real(0.5) * (Buf<real>::load(rrho, o0, pr + qb) - Buf<real>::load(rrho, o0, pr - qb));
      if (gk) gk[(int64_t)y * nx + x] += (double)gx_c * (double)dx + (double)gy_c * (double)dy;
    }

    __syncthreads();
    qy_m = kap_c * gy_c;
#pragma unroll
    for (int i = 0; i < 9; ++i) as_c[i] = as_n[i];
    gx_c = gx_n;
    gy_c = gy_n;
    mx_c = mx_n;
    my_c = my_n;
    kap_c = kap_n;
  }
}

// Residual e = v - d of one grid's traces and the misfit L += 1/2 sum e^2,
// accumulated in FP64: wavefront shuffles, then one atomic add per wavefront.
template <typename real>
__global__ __launch_bounds__(256) void misfit_kernel(const real *__restrict__ trace,
                                                     const real *__restrict__ d_obs,
                                                     real *__restrict__ residual, int64_t n,
                                                     double *misfit) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const real e = trace[i] - d_obs[i];
    if (residual) residual[i] = e;
    acc += (double)e * (double)e;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc != 0.0) atomicAdd(misfit, 0.5 * acc);
}

// dL/dlambda and dL/dmu from dL/dkappa with kappa = b^2 (mu - lambda)/mu
// (Sec. 4): dkappa/dlambda = -b^2/mu, dkappa/dmu = b^2 lambda/mu^2, added to
// the outputs (shots that share a medium sum their contributions).
template <typename real>
__global__ __launch_bounds__(256) void lame_gradient_kernel(const real *__restrict__ lam,
                                                            const real *__restrict__ mu,
                                                            const double *__restrict__ gk,
                                                            double *__restrict__ gl,
                                                            double *__restrict__ gm, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double m = (double)mu[i], l = (double)lam[i], g = gk[i];
    if (gl) gl[i] += -(1.0 / 3.0) * g / m;
    if (gm) gm[i] += (1.0 / 3.0) * g * l / (m * m);
  }
}

inline int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (int)(b > 4096 ? 4096 : b);
}

}  // namespace

template <typename real>
hipError_t launch_adjoint(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves);
  if (waves == 1) hipLaunchKernelGGL((adjoint_kernel<real, 1>), grid, block, 0, stream, a);
  else if (waves == 2) hipLaunchKernelGGL((adjoint_kernel<real, 2>), grid, block, 0, stream, a);
  else if (waves == 4) hipLaunchKernelGGL((adjoint_kernel<real, 4>), grid, block, 0, stream, a);
  else if (waves == 8) hipLaunchKernelGGL((adjoint_kernel<real, 8>), grid, block, 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename real>
hipError_t launch_adjoint_interior(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves);
  if (waves == 1) hipLaunchKernelGGL((adjoint_interior_kernel<real, 1>), grid, block, 0, stream, a);
  else if (waves == 2) hipLaunchKernelGGL((adjoint_interior_kernel<real, 2>), grid, block, 0, stream, a);
  else if (waves == 4) hipLaunchKernelGGL((adjoint_interior_kernel<real, 4>), grid, block, 0, stream, a);
  else if (waves == 8) hipLaunchKernelGGL((adjoint_interior_kernel<real, 8>), grid, block, 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename real>
hipError_t launch_misfit(const real *trace, const real *d_obs, real *residual, int64_t n,
                         double *misfit, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(misfit_kernel<real>, dim3(blocks_for(n)), dim3(256), 0, stream, trace, d_obs,
                     residual, n, misfit);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_lame_gradient(const real *lam, const real *mu, const double *grad_kappa,
                                double *grad_lam, double *grad_mu, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lame_gradient_kernel<real>, dim3(blocks_for(n)), dim3(256), 0, stream, lam, mu,
                     grad_kappa, grad_lam, grad_mu, n);
  return hipGetLastError();
}

#define LBM_INST(real)                                                                        \
  template hipError_t launch_adjoint<real>(const AdjArgs<real> &, int, int, hipStream_t);     \
  template hipError_t launch_adjoint_interior<real>(const AdjArgs<real> &, int, int,          \
                                                    hipStream_t);                             \
  template hipError_t launch_misfit<real>(const real *, const real *, real *, int64_t, double *, \
                                          hipStream_t);                                       \
  template hipError_t launch_lame_gradient<real>(const real *, const real *, const double *,  \
                                                 double *, double *, int64_t, hipStream_t);
LBM_INST(float)
LBM_INST(double)
#undef LBM_INST

}  // namespace lbm
