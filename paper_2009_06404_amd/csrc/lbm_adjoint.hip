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
#include <type_traits>

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

// kappa times a component of Gh, rounded on its own and never fused into the
// add or subtract that uses it: every adjoint kernel then forms the same
// transposed gradient for a cell away from walls, 1/2 ((q_l - q_r) + (q_u -
// q_d)), and the launch shape (tile lists, the two-step path) does not change
// the result.
template <typename real>
__device__ __forceinline__ real kmul(real k, real gh) {
#pragma clang fp contract(off)
  return k * gh;
}

// x / 2 rounded on its own: exact unless x is denormal, and then only the
// same in every kernel if it is never fused into the add that uses it.
template <typename real>
__device__ __forceinline__ real halve(real x) {
#pragma clang fp contract(off)
  return real(0.5) * x;
}

// Step 5's dL/dkappa term Gh . grad(rho) of one cell and step, and its
// accumulation, in FP64 with every product and sum rounded on its own, so
// that all kernels (the two-step one forms a step's term before it reads
// the sum) give the same bits.
template <typename real>
__device__ __forceinline__ double gk_term(real gx, real gy, real dx, real dy) {
#pragma clang fp contract(off)
  return (double)gx * (double)dx + (double)gy * (double)dy;
}
__device__ __forceinline__ double gk_add(double acc, double term) {
#pragma clang fp contract(off)
  return acc + term;
}

template <typename real, int NW>
__global__ __launch_bounds__(64 * NW) void adjoint_kernel(AdjArgs<real> a) {
  constexpr int W = 64 * NW;
  __shared__ real sq[2][W + 2];
  __shared__ double samp[NW][kMaxAdjSources];   // each wavefront's dL/damp sums

  const TileDev tile = a.tiles[blockIdx.x];
  if (tile.g < 0) return;
  // a border strip of a two-step block advances the state only
  const bool strip = (tile.g & kStripTile) != 0;
  const int gi = tile.g & ~kStripTile;
  const GridDev &g = a.grids[gi];
  AdjGridDev io = a.io[gi];
  if (strip) {
    io.grad_kappa = nullptr;
    io.grad_amp = nullptr;
  }
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
  if ((lane & 63) < kMaxAdjSources) samp[lane >> 6][lane & 63] = 0.0;

  // Twice the weights of the transposed gradient from the x-neighbours: 1
  // (weight 1/2), or 2 from a neighbour on a rigid side edge (its one-sided
  // difference, weight 1).
  const bool rigid_l = g.bc[kEdgeLeft] == kRigid, rigid_r = g.bc[kEdgeRight] == kRigid;
  const real wxl = (rigid_l && col.xl == 0) ? real(2) : real(1);
  const real wxr = (rigid_r && col.xr == nx - 1) ? real(2) : real(1);

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
  // The row above the tile, when connected: its kappa * Gh_y and twice its
  // weight (2 for a top-boundary row with its one-sided difference, else 1).
  real qy_m = real(0), wy_m = real(1);
  if (rc.wall_up == 0) {
    const Row ru = make_row(g, rc.up);
    real as_[9], gx_, gy_, mx_, my_;
    cell(ru, col, xa, as_, gx_, gy_, mx_, my_);
    qy_m = kmul(cell_kappa(a.kappa_rows, a.kappa_cells, g, ru.y, xa), gy_);
    wy_m = ru.wall_up != 0 ? real(2) : real(1);
  }
  real as_c[9], gx_c, gy_c, mx_c, my_c;
  cell(rc, col, xa, as_c, gx_c, gy_c, mx_c, my_c);
  real kap_c = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, xa);
  sq[0][lane + 1] = kmul(kap_c, gx_c);
  if (lane < 2) {
    real hq = real(0);
    if (hlane) {
      real as_[9], gx_, gy_, mx_, my_;
      cell(rc, hcol, hx, as_, gx_, gy_, mx_, my_);
      hq = kmul(cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, hx), gx_);
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
        hq_n = kmul(cell_kappa(a.kappa_rows, a.kappa_cells, g, yn, hx), gx_);
      }
    }

    const int s = k & 1;
    const real qx_l = sq[s][lane];
    const real qx_r = (xa == x_last) ? sq[s][W + 1] : sq[s][lane + 2];
    if (in_tile) {
      sq[s ^ 1][lane + 1] = kmul(kap_n, gx_n);
      if (lane < 2) sq[s ^ 1][hslot] = hq_n;
    }

    // Step 3: transposed density gradient, 1/2 of the x and y parts with
    // twice their weights (2 q of the cell itself at a wall): away from
    // walls 1/2 ((q_l - q_r) + (q_u - q_d)), the operations of the other
    // adjoint kernels, denormal values included.
    const real qx_c = kmul(kap_c, gx_c), qy_c = kmul(kap_c, gy_c);
    const bool lo_y = rc.wall_up != 0, hi_y = rc.wall_dn != 0;
    const real wy_n = rn.wall_dn != 0 ? real(2) : real(1);
    const real qx2 = qx_c + qx_c, qy2 = qy_c + qy_c;
    const real rx = (col.wl ? -qx2 : wxl * qx_l) - (col.wr ? -qx2 : wxr * qx_r);
    const real ry = (lo_y ? -qy2 : wy_m * qy_m) - (hi_y ? -qy2 : wy_n * kmul(kap_n, gy_n));
    const real rD = halve(rx + ry);

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
      else dx = halve(rs[(int64_t)y * pitch + col.xr] - rs[(int64_t)y * pitch + col.xl]);
      if (lo_y) dy = rs[(int64_t)(y + 1) * pitch + x] - rho_c;
      else if (hi_y) dy = rho_c - rs[(int64_t)(y - 1) * pitch + x];
      else dy = halve(rs[(int64_t)rc.dn * pitch + x] - rs[(int64_t)rc.up * pitch + x]);
      double &cell = io.grad_kappa[(int64_t)y * nx + x];
      cell = gk_add(cell, gk_term(gx_c, gy_c, dx, dy));
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
      if ((lane & 63) == 0) samp[lane >> 6][si] += v;
    }

    // March: row y+1 becomes current.
    __syncthreads();
    qy_m = qy_c;
    wy_m = lo_y ? real(2) : real(1);
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
  // The workgroup's dL/damp of this step, wavefronts summed in order, to its
  // slot of the partial sums (added to dL/damp in a fixed order by
  // amp_reduce_kernel: no atomics, so the result does not depend on the
  // order in which workgroups finish).
  if (lane < nsrc) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += samp[w][lane];
    a.amp_part[(int64_t)blockIdx.x * kMaxAdjSources + lane] = sum;
  }
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
    qy_m = kmul(cell_kappa(a.kappa_rows, a.kappa_cells, g, y0 - 1, xa), gy_);
  }
  cell(y0, false, as_c, gx_c, gy_c, mx_c, my_c);
  real kap_c = cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, xa);
  sq[0][lane + 1] = kmul(kap_c, gx_c);
  if (lane < 2) {
    real t_[9], gx_, gy_, mx_, my_;
    cell(y0, true, t_, gx_, gy_, mx_, my_);
    sq[0][hslot] = kmul(cell_kappa(a.kappa_rows, a.kappa_cells, g, y0, hx), gx_);
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
      hq_n = kmul(cell_kappa(a.kappa_rows, a.kappa_cells, g, y + 1, hx), gx_);
    }
    const int s = k & 1;
    const real qx_l = sq[s][lane];
    const real qx_r = (xa == x_last) ? sq[s][W + 1] : sq[s][lane + 2];
    sq[s ^ 1][lane + 1] = kmul(kap_n, gx_n);
    if (lane < 2) sq[s ^ 1][hslot] = hq_n;

    // Step 3 (centred differences only) and step 4.
    const real rD = halve((qx_l - qx_r) + (qy_m - kmul(kap_n, gy_n)));
    if (active) {
      real fh[9];
      adj_finish(as_c, omega, rD, mx_c, my_c, real(0), fh);
      const uint32_t rs = (uint32_t)(y - ybase) * rowb;
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf<real>::store_nt(fh[i], rout, o0, rs + i * qb);
      // Step 5: dL/dkappa += Gh . grad(rho)(t).
      const uint32_t pr = (uint32_t)(y - ybase) * qb;
      const real dx = halve(Buf<real>::load(rrho, orr, pr) - Buf<real>::load(rrho, ol, pr));
      const real dy = halve(Buf<real>::load(rrho, o0, pr + qb) - Buf<real>::load(rrho, o0, pr - qb));
      if (gk) gk[(int64_t)y * nx + x] = gk_add(gk[(int64_t)y * nx + x], gk_term(gx_c, gy_c, dx, dy));
    }

    __syncthreads();
    qy_m = kmul(kap_c, gy_c);
#pragma unroll
    for (int i = 0; i < 9; ++i) as_c[i] = as_n[i];
    gx_c = gx_n;
    gy_c = gy_n;
    mx_c = mx_n;
    my_c = my_n;
    kap_c = kap_n;
  }
}

template <int N>
using AdjPhase = std::integral_constant<int, N>;

// Two adjoint steps of a block in one pass: from fh(t+1) in HBM to fh(t-1)
// in HBM, fh(t) staying on chip, over blocks clear of walls, of the y-wrap,
// of source disks and of receivers within three rows (the blocks of the
// forward's two-step path, the rows near receivers taken out). The row loop
// is the forward two-step kernel's with every arrow reversed:
//   A (row r):   transposed pull of ah(t) from fh(t+1) (row r+1 in flight),
//                the local transpose (Gh, mh); kappa Gh_x into an LDS ring;
//   B (row r-1): transposed gradient and moments -> fh(t) of row r-1, and
//                step t's dL/dkappa contribution Gh . grad(rho)(t);
//   C (row r-2): transposed pull of ah(t-1) from fh(t) of rows r-3 .. r-1
//                (on chip), the local transpose; kappa Gh_x into a ring;
//   D (row r-3): -> fh(t-1) of row r-3 to HBM; dL/dkappa += step t's then
//                step t-1's contribution (one FP64 read and write, in the
//                order of two single steps).
// The transposed pull takes population k from row y + c_ky: of fh(t), the
// populations with c_y = +1 (2, 5, 6) come from the newest row, those with
// c_y = 0 (0, 1, 3) from one row before, those with c_y = -1 (4, 7, 8) from
// two rows before; the six with c_x != 0 pass through LDS rings of those
// depths, the three with c_x = 0 stay in registers. The per-cell operations
// are the interior adjoint kernel's, in the same order. Lanes as in the
// forward kernel: the block's 64 * NW columns plus a wavefront for the four
// halo columns on each side; stage B runs on three halo columns, C on two.
// The density stashes reach the gradient terms through register rings (the
// rows above and below, each lane its own column, loaded one row ahead) and
// LDS (the row's neighbours in x); dL/dkappa is read one row ahead too, so
// that no stage waits on a load issued in it.
template <typename real, int NW>
__global__ __launch_bounds__(64 * NW + 64, sizeof(real) == 4 ? 4 : 2) void adjoint_fused2_kernel(
    AdjArgs<real> a) {
  constexpr int W = 64 * NW;
  constexpr int LW = W + 8;
  constexpr int RT = kFusedMaxRows + 8;
  __shared__ real sQA[2][LW];               // kappa Gh_x(t) of rows r-1, r
  __shared__ real sQC[2][LW];               // kappa Gh_x(t-1) of rows r-3, r-2
  __shared__ real s56[2][LW];               // fh(t) populations 5, 6 of row r-1
  __shared__ real s13[2][2][LW];            // populations 1, 3 of rows r-2, r-1
  __shared__ real s78[3][2][LW];            // populations 7, 8 of rows r-3 .. r-1
  __shared__ real sRt[LW], sRt1[LW];        // rho(t) of row r-1, rho(t-1) of row r-3
  __shared__ real sRowA[RT], sRowI[RT], sRowK[RT];

  const FusedTileDev tile = a.ftiles[blockIdx.x];
  if (tile.g < 0) return;
  const GridDev g = uniform_lookup_fields(a.grids[tile.g]);
  const double *gk = a.io[tile.g].grad_kappa;
  const int pitch = g.pitch, nx = g.nx;
  const int w = tile.x1 - tile.x0;
  const int tid = threadIdx.x;
  const int hl = tid - W;
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
  // the density stash of steps t and t-1, rows from ybase on
  const __amdgpu_buffer_rsrc_t rt = tile_rsrc(a.rho + g.c_off + (int64_t)ybase * pitch);
  const __amdgpu_buffer_rsrc_t rt1 = tile_rsrc(a.rho2 + g.c_off + (int64_t)ybase * pitch);
  // dL/dkappa from row ybase on; without it (no gradient asked) an empty
  // range, through which loads return 0 and stores are dropped
  const __amdgpu_buffer_rsrc_t rgk = range_rsrc(
      gk ? gk + (int64_t)ybase * nx : gk, gk ? (uint64_t)(g.ny - ybase) * nx * sizeof(double) : 0);
  const uint32_t og = (uint32_t)col * sizeof(double), gkrow = (uint32_t)nx * sizeof(double);

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
  // kinds of medium: their loads return 0, with no branch around them)
  const __amdgpu_buffer_rsrc_t rk = range_rsrc(
      a.kappa_cells + (kcells ? g.k_off + (int64_t)ybase * pitch : 0),
      kcells ? (uint64_t)(g.ny - ybase) * pitch * sizeof(real) : 0);
  const bool inB = lc >= 1 && lc <= w + 6, inC = lc >= 2 && lc <= w + 5;
  __syncthreads();

  // Registers carried down the rows: F the pulled ah(t) of rows r-1, r and
  // r+1 (in flight); MA the (mh_x, mh_y, Gh_x, Gh_y) of rows r-1, r; QA
  // kappa Gh_y(t) of rows r-2, r-1, r; G the pulled ah(t-1) of rows r-3,
  // r-2 and MC, QC their moments as for step t; D0 / E4 populations 0 and 4
  // of fh(t) waiting one and two rows for stage C; CT step t's dL/dkappa
  // contributions of rows r-3 .. r-1; kq, k0, k1 the cell-wise modulus of
  // rows r, r-1, r-2 (row r+1 in flight). Indexed by row modulo 6 (the
  // unrolled round): RH rho(t) of rows r-2 .. r+1 (in flight), R1 rho(t-1)
  // of rows r-4 .. r-1 (in flight), GK dL/dkappa of rows r-3, r-2 (in
  // flight), at this lane's column.
  real F[3][9], G[2][9], MA[2][4], MC[2][4], QA[3], QC[3], D0[2], E4[3], RH[6], R1[6];
  double CT[3], GK[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) { F[0][i] = F[1][i] = F[2][i] = G[0][i] = G[1][i] = real(0); }
#pragma unroll
  for (int i = 0; i < 4; ++i) { MA[0][i] = MA[1][i] = MC[0][i] = MC[1][i] = real(0); }
  QA[0] = QA[1] = QA[2] = QC[0] = QC[1] = QC[2] = real(0);
  D0[0] = D0[1] = E4[0] = E4[1] = E4[2] = real(0);
  CT[0] = CT[1] = CT[2] = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    RH[i] = R1[i] = real(0);
    GK[i] = 0.0;
  }
  real kq = real(0), k0 = real(0), k1 = real(0);

  const int rlast = y1 + 2;
  const int r0 = rlast + 1 - (rlast - (y0 - 4) + 1 + 5) / 6 * 6;

  auto kap_row = [&](int row, real kc) {
    return kcells ? kc : (g.kmode == kKappaRows ? sRowK[row - ybase] : kscalar);
  };

  auto iter = [&](const int r, auto ph, auto first) {
    constexpr int P = decltype(ph)::value;
    real(&fb)[9] = F[(P + 1) % 3];          // row r (stage A)
    real(&fc)[9] = F[(P + 2) % 3];          // row r+1 (loads)
    real(&fa)[9] = F[P % 3];                // row r-1 (stage B)
    real(&gn)[9] = G[(P + 1) % 2];          // row r-2 (stage C)
    real(&gc)[9] = G[P % 2];                // row r-3 (stage D)
    real(&ma_n)[4] = MA[P % 2];             // row r
    real(&ma_c)[4] = MA[(P + 1) % 2];       // row r-1
    real(&mc_n)[4] = MC[P % 2];             // row r-2
    real(&mc_c)[4] = MC[(P + 1) % 2];       // row r-3
    real &qA_n = QA[P % 3], &qA_m = QA[(P + 1) % 3];   // rows r, r-2
    real &qC_n = QC[P % 3], &qC_m = QC[(P + 1) % 3];   // rows r-2, r-4
    double &ct_b = CT[P % 3], &ct_d = CT[(P + 1) % 3];
    real kn = real(0);
    // row y's slot in RH, R1 and GK: (P + y - r) mod 6
    constexpr int S_P1 = (P + 1) % 6, S_M1 = (P + 5) % 6, S_M2 = (P + 4) % 6;
    constexpr int S_M3 = (P + 3) % 6, S_M4 = (P + 2) % 6, S_0 = P;
    // dL/dkappa of row r-2 (clamped to the block's first row, in range)
    {
      const uint32_t sg = sreg((int32_t)((uint32_t)(max(r - 2, y0) - ybase) * gkrow));
      GK[S_M2] = Buf<double>::load(rgk, og, sg);
    }
    // The row index and the offsets below go through an empty asm: otherwise
    // the compiler keeps every population's offset of every unrolled row as
    // its own scalar induction variable. After the first round every lane
    // loads on every iteration (past rlast: rlast again, not used), so the
    // waits of stage A leave this prefetch in flight.
    // The densities: rho(t) of row r+1, rho(t-1) of row r-1.
    if (decltype(first)::value) {
      if (live && r + 1 >= y0 - 3) {
        int rn = r + 1;
        asm volatile("" : "+s"(rn));
        adj_pull_fast(rin, ybase, rn, rowb, qb, o0, ol, orr, fc);
        const uint32_t sr = sreg((int32_t)((uint32_t)(rn - ybase) * qb));
        kn = Buf<real>::load(rk, o0, sr);
        RH[S_P1] = Buf<real>::load(rt, o0, sr);
      }
      if (live && r - 1 >= y0 - 1)
        R1[S_M1] = Buf<real>::load(rt1, o0, sreg((int32_t)((uint32_t)(r - 1 - ybase) * qb)));
    } else {
      int rn = min(r + 1, rlast);
      asm volatile("" : "+s"(rn));
      adj_pull_fast(rin, ybase, rn, rowb, qb, o0, ol, orr, fc);
      kn = Buf<real>::load(rk, o0, sreg((int32_t)((uint32_t)(rn - ybase) * qb)));
      RH[S_P1] = Buf<real>::load(rt, o0, sreg((int32_t)((uint32_t)(r + 1 - ybase) * qb)));
      R1[S_M1] = Buf<real>::load(rt1, o0, sreg((int32_t)((uint32_t)(r - 1 - ybase) * qb)));
    }
    // Stage A: row r of step t.
    qA_n = real(0);
    if (live && r >= y0 - 3) {
      const real A = max(A_x, sRowA[r - ybase]), inv = min(inv_x, sRowI[r - ybase]);
      adj_local(fb, real(0), real(0), A, inv, omega, cforce, ma_n[2], ma_n[3], ma_n[0], ma_n[1]);
      const real kap = kap_row(r, kq);
      sQA[r & 1][lc] = kmul(kap, ma_n[2]);
      qA_n = kmul(kap, ma_n[3]);
    }
    if (live) sRt[lc] = RH[S_M1];
    __syncthreads();
    // Stage B: row r-1 of step t.
    const int rb = r - 1;
    real p0 = real(0), p2 = real(0), p4 = real(0);
    if (rb >= y0 - 2 && inB) {
      const real qx_l = sQA[rb & 1][lc - 1], qx_r = sQA[rb & 1][lc + 1];
      const real rD = halve((qx_l - qx_r) + (qA_m - qA_n));
      real fh[9];
      adj_finish(fa, omega, rD, ma_c[0], ma_c[1], real(0), fh);
      s56[0][lc] = fh[5];
      s56[1][lc] = fh[6];
      s13[rb & 1][0][lc] = fh[1];
      s13[rb & 1][1][lc] = fh[3];
      s78[rb % 3][0][lc] = fh[7];
      s78[rb % 3][1][lc] = fh[8];
      p0 = fh[0];
      p2 = fh[2];
      p4 = fh[4];
      if (gk && outlane && rb >= y0 && rb < y1) {
        const real dx = halve(sRt[lc + 1] - sRt[lc - 1]);
        const real dy = halve(RH[S_0] - RH[S_M2]);
        ct_b = gk_term(ma_c[2], ma_c[3], dx, dy);
      }
    }
    __syncthreads();
    // Stage C: row r-2 of step t-1, pulled from fh(t) of rows r-3 .. r-1.
    const int rc = r - 2;
    qC_n = real(0);
    if (rc >= y0 - 1 && inC) {
      const int s13i = rc & 1, s78i = (rc + 2) % 3;   // rows rc and rc-1
      gn[0] = D0[P % 2];                             // row rc, this column
      gn[1] = s13[s13i][0][lc + 1];                  // ( 1, 0) from (x+1, rc)
      gn[2] = p2;                                    // ( 0, 1) from (x, rc+1)
      gn[3] = s13[s13i][1][lc - 1];                  // (-1, 0) from (x-1, rc)
      gn[4] = E4[P % 3];                             // ( 0,-1) from (x, rc-1)
      gn[5] = s56[0][lc + 1];                        // ( 1, 1) from (x+1, rc+1)
      gn[6] = s56[1][lc - 1];                        // (-1, 1) from (x-1, rc+1)
      gn[7] = s78[s78i][0][lc - 1];                  // (-1,-1) from (x-1, rc-1)
      gn[8] = s78[s78i][1][lc + 1];                  // ( 1,-1) from (x+1, rc-1)
      const real A = max(A_x, sRowA[rc - ybase]), inv = min(inv_x, sRowI[rc - ybase]);
      adj_local(gn, real(0), real(0), A, inv, omega, cforce, mc_n[2], mc_n[3], mc_n[0], mc_n[1]);
      const real kap = kap_row(rc, k1);
      sQC[rc & 1][lc] = kmul(kap, mc_n[2]);
      qC_n = kmul(kap, mc_n[3]);
    }
    if (live) sRt1[lc] = R1[S_M3];
    __syncthreads();
    // Stage D: row r-3 of step t-1.
    const int rd = r - 3;
    // (uniform offsets, moved to scalar registers before the branch; rows
    // before y0 give values that are not used)
    const uint32_t rs = sreg((int32_t)((uint32_t)(rd - ybase) * rowb));
    const uint32_t sg = sreg((int32_t)((uint32_t)(rd - ybase) * gkrow));
    if (rd >= y0 && outlane) {
      const real qx_l = sQC[rd & 1][lc - 1], qx_r = sQC[rd & 1][lc + 1];
      const real rD = halve((qx_l - qx_r) + (qC_m - qC_n));
      real fh[9];
      adj_finish(gc, omega, rD, mc_c[0], mc_c[1], real(0), fh);
#pragma unroll
      for (int i = 0; i < 9; ++i) Buf<real>::store_nt(fh[i], rout, o0, rs + i * qb);
      if (gk) {
        const real dx = halve(sRt1[lc + 1] - sRt1[lc - 1]);
        const real dy = halve(R1[S_M2] - R1[S_M4]);
        const double sum = gk_add(gk_add(GK[S_M3], ct_d), gk_term(mc_c[2], mc_c[3], dx, dy));
        Buf<double>::store_nt(sum, rgk, og, sg);
      }
    }
    __syncthreads();
    D0[(P + 1) % 2] = p0;
    E4[(P + 2) % 3] = p4;
    k1 = k0;
    k0 = kq;
    kq = kn;
  };

  using First = std::true_type;
  using Steady = std::false_type;
  iter(r0, AdjPhase<0>{}, First{});
  iter(r0 + 1, AdjPhase<1>{}, First{});
  iter(r0 + 2, AdjPhase<2>{}, First{});
  iter(r0 + 3, AdjPhase<3>{}, First{});
  iter(r0 + 4, AdjPhase<4>{}, First{});
  iter(r0 + 5, AdjPhase<5>{}, First{});
  for (int r = r0 + 6; r <= rlast; r += 6) {
    iter(r, AdjPhase<0>{}, Steady{});
    iter(r + 1, AdjPhase<1>{}, Steady{});
    iter(r + 2, AdjPhase<2>{}, Steady{});
    iter(r + 3, AdjPhase<3>{}, Steady{});
    iter(r + 4, AdjPhase<4>{}, Steady{});
    iter(r + 5, AdjPhase<5>{}, Steady{});
  }
}

// Sum of v over a 256-thread workgroup in a fixed order (wavefront shuffles,
// then the four wavefronts' sums in order); the result in thread 0.
__device__ __forceinline__ double block_sum_256(double v, double *s4) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((s4[0] + s4[1]) + s4[2]) + s4[3];
}

// dL/damp of one (grid, source) per workgroup: the partial sums of the
// general kernel's workgroups that cover the grid (their slots listed in
// tiles[off[k] .. off[k+1])), added in that order.
__global__ __launch_bounds__(256) void amp_reduce_kernel(const double *__restrict__ part,
                                                         const int32_t *__restrict__ tiles,
                                                         const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ pairs,
                                                         const AdjGridDev *__restrict__ io) {
  __shared__ double s4[4];
  const int k = blockIdx.x;
  const int g = pairs[2 * k], si = pairs[2 * k + 1];
  double *out = io[g].grad_amp;
  if (!out) return;
  double v = 0.0;
  for (int i = off[k] + (int)threadIdx.x; i < off[k + 1]; i += 256)
    v += part[(int64_t)tiles[i] * kMaxAdjSources + si];
  v = block_sum_256(v, s4);
  if (threadIdx.x == 0) out[si] += v;
}

// Residual e = v - d of one grid's traces and the misfit L += 1/2 sum e^2,
// accumulated in FP64 in a fixed order: each workgroup's sum to part[], then
// misfit_sum_kernel adds them in order (no atomics, so the result does not
// depend on the order in which workgroups finish).
template <typename real>
__global__ __launch_bounds__(256) void misfit_kernel(const real *__restrict__ trace,
                                                     const real *__restrict__ d_obs,
                                                     real *__restrict__ residual, int64_t n,
                                                     double *__restrict__ part) {
  __shared__ double s4[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const real e = trace[i] - d_obs[i];
    if (residual) residual[i] = e;
    acc += (double)e * (double)e;
  }
  acc = block_sum_256(acc, s4);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void misfit_sum_kernel(const double *__restrict__ part, int nb,
                                                         double *misfit) {
  __shared__ double s4[4];
  double v = 0.0;
  for (int i = (int)threadIdx.x; i < nb; i += 256) v += part[i];
  v = block_sum_256(v, s4);
  if (threadIdx.x == 0) *misfit += 0.5 * v;
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
hipError_t launch_adjoint_fused2(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(64 * waves + 64);
  if (waves == 2) hipLaunchKernelGGL((adjoint_fused2_kernel<real, 2>), grid, block, 0, stream, a);
  else if (waves == 4) hipLaunchKernelGGL((adjoint_fused2_kernel<real, 4>), grid, block, 0, stream, a);
  else if (waves == 8) hipLaunchKernelGGL((adjoint_fused2_kernel<real, 8>), grid, block, 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_amp_reduce(const double *part, const int32_t *tiles, const int32_t *off,
                             const int32_t *pairs, int npairs, const AdjGridDev *io,
                             hipStream_t stream) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(amp_reduce_kernel, dim3(npairs), dim3(256), 0, stream, part, tiles, off,
                     pairs, io);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_misfit(const real *trace, const real *d_obs, real *residual, int64_t n,
                         double *misfit, double *part, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(misfit_kernel<real>, dim3(nb), dim3(256), 0, stream, trace, d_obs, residual,
                     n, part);
  hipLaunchKernelGGL(misfit_sum_kernel, dim3(1), dim3(256), 0, stream, part, nb, misfit);
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
  template hipError_t launch_adjoint_fused2<real>(const AdjArgs<real> &, int, int, hipStream_t); \
  template hipError_t launch_misfit<real>(const real *, const real *, real *, int64_t, double *, \
                                          double *, hipStream_t);                             \
  template hipError_t launch_lame_gradient<real>(const real *, const real *, const double *,  \
                                                 double *, double *, int64_t, hipStream_t);
LBM_INST(float)
LBM_INST(double)
#undef LBM_INST

}  // namespace lbm
