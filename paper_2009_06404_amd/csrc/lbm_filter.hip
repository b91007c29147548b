// High-wavenumber filter of the stored state (Sec. 4 proposes filtering high
// frequencies at the end of a time step to recover stability for Poisson
// ratios other than 1/4; the paper gives no form). The form used here is the
// fourth difference along each axis, applied to every population:
//   f_i <- f_i - sigma (d4x f_i + d4y f_i),
//   d4x g(x) = g(x-2) - 4 g(x-1) + 6 g(x) - 4 g(x+1) + g(x+2),
// whose factor on a plane wave is 1 - 16 sigma (sin^4(kx/2) + sin^4(ky/2)):
// 1 at k = 0, 1 - O(sigma k^4) for resolved waves, 1 - 32 sigma at the
// Nyquist corner (sigma <= 1/16 keeps it in [-1, 1]). An axis term applies
// where its five-point stencil lies in the grid (or wraps over a periodic
// edge) without crossing the internal rigid wall; elsewhere that term is
// left out, so cells next to walls are filtered along the wall only.
#include "lbm_device.h"

namespace lbm {
namespace {

using namespace dev;

// A workgroup takes a tile of 256 columns down its rows: four wavefronts own
// the tile's columns and a fifth loads the two halo columns on each side
// (its lanes 0..3; the others load a column of the tile and discard it), so
// that no load sits under a lane condition. Each lane keeps the five rows
// y-2 .. y+2 of its column in registers and the two rows after them in flight,
// and every row also goes into a four-row LDS ring for the x neighbours. One
// barrier per row. The lanes past a narrow grid's last column load the
// columns after it (wrapped, or the last column where x is not periodic), so
// the ring holds the right neighbours of the last column without the halo
// wavefront. Rows are read and written through per-row buffer descriptors
// (the row index is the same for the whole workgroup).
template <typename real>
__global__ __launch_bounds__(320) void filter_kernel(const real *__restrict__ fin, real *__restrict__ fout,
                                                     const GridDev *__restrict__ grids,
                                                     const TileDev *__restrict__ tiles, real sigma) {
  constexpr int TW = 256;
  constexpr int kDummySlot = TW + 4;     // LDS column of the halo wavefront's unused lanes
  __shared__ real srow[4][9][TW + 5];
  const TileDev t = tiles[blockIdx.x];
  if (t.g < 0) return;
  const GridDev g = uniform_lookup_fields(grids[t.g]);
  const int nx = g.nx, ny = g.ny, rr = sreg(grids[t.g].rigid_row);
  const int lane = (int)threadIdx.x;
  const bool main_lane = lane < TW;
  const int x = t.x0 + lane;
  const bool active = main_lane && x < nx;
  const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
  // the column this lane loads and its LDS slot: main lanes their own column
  // (past the grid: the column after it, wrapped or clamped); halo lanes
  // 0, 1 columns x0-2, x0-1 (slots 0, 1), 2, 3 columns x0+256, x0+257
  // (slots 258, 259)
  int c = x, slot = lane + 2;
  if (!main_lane) {
    const int hl = lane - TW;
    c = hl < 2 ? t.x0 - 2 + hl : (hl < 4 ? t.x0 + TW + hl - 2 : t.x0);
    slot = hl < 2 ? hl : (hl < 4 ? TW + hl : kDummySlot);
  }
  const int cl = px ? ((c % nx) + nx) % nx : min(max(c, 0), nx - 1);
  const uint32_t esz = sizeof(real);
  const uint32_t voff = (uint32_t)cl * esz, qb = (uint32_t)g.pitch * esz;
  // rows outside a non-periodic grid are never used (their terms are left
  // out); clamp them to stay in bounds
  auto wy = [&](int r) { return py ? (r < 0 ? r + ny : (r >= ny ? r - ny : r)) : min(max(r, 0), ny - 1); };
  auto row_in = [&](int r) {
    return tile_rsrc(fin + g.f_off + (int64_t)sreg(wy(r)) * 9 * g.pitch);
  };
  const bool xs = px ? nx >= 5 : (x >= 2 && x <= nx - 3);

  real win[9][5];   // rows y-2 .. y+2 of this lane's column
  // the two rows after them, in flight: P0 and P1 alternate (row y+2 in the
  // one of y's parity relative to y0, row y+3 in the other), so no register
  // move waits on a load
  real P0[9], P1[9];
  // prologue: rows y0-2 .. y0+1 into the window, rows y0, y0+1 into the ring
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const __amdgpu_buffer_rsrc_t R = row_in(t.y0 - 2 + k);
#pragma unroll
    for (int i = 0; i < 9; ++i) win[i][k + 1] = Buf<real>::load(R, voff, (uint32_t)i * qb);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < 9; ++i) srow[(t.y0 + k) & 3][i][slot] = win[i][k + 3];
  {
    const __amdgpu_buffer_rsrc_t R2 = row_in(t.y0 + 2), R3 = row_in(t.y0 + 3);
#pragma unroll
    for (int i = 0; i < 9; ++i) P0[i] = Buf<real>::load(R2, voff, (uint32_t)i * qb);
#pragma unroll
    for (int i = 0; i < 9; ++i) P1[i] = Buf<real>::load(R3, voff, (uint32_t)i * qb);
  }

  // row y: row y+2 (in P) joins the window and the ring, row y+4 goes into P
  auto row = [&](int y, real(&P)[9]) {
    const __amdgpu_buffer_rsrc_t R = row_in(min(y + 4, t.y1 + 2));   // no row past the stencil
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
      for (int k = 0; k < 4; ++k) win[i][k] = win[i][k + 1];
      win[i][4] = P[i];
      srow[(y + 2) & 3][i][slot] = P[i];
      P[i] = Buf<real>::load(R, voff, (uint32_t)i * qb);
    }
    __syncthreads();
    const bool ys = (py ? ny >= 5 : (y >= 2 && y <= ny - 3)) && !(rr > 0 && y >= rr - 2 && y <= rr + 1);
    const int s = y & 3;
    if (active) {
      const __amdgpu_buffer_rsrc_t O = tile_rsrc(fout + g.f_off + (int64_t)y * 9 * g.pitch);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const real cc = win[i][2];
        real acc = real(0);
        if (xs)
          acc += ((srow[s][i][lane] + srow[s][i][lane + 4]) -
                  real(4) * (srow[s][i][lane + 1] + srow[s][i][lane + 3])) +
                 real(6) * cc;
        if (ys) acc += ((win[i][0] + win[i][4]) - real(4) * (win[i][1] + win[i][3])) + real(6) * cc;
        Buf<real>::store_nt(cc - sigma * acc, O, (uint32_t)x * esz, (uint32_t)i * qb);
      }
    }
  };
  int y = t.y0;
  for (; y + 1 < t.y1; y += 2) {
    row(y, P0);
    row(y + 1, P1);
  }
  if (y < t.y1) row(y, P0);
}

}  // namespace

template <typename real>
hipError_t launch_filter(const real *fin, real *fout, const GridDev *grids, const TileDev *tiles,
                         int ntiles, real sigma, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((filter_kernel<real>), dim3(ntiles), dim3(320), 0, stream, fin, fout, grids, tiles,
                     sigma);
  return hipGetLastError();
}

template hipError_t launch_filter<float>(const float *, float *, const GridDev *, const TileDev *, int, float,
                                         hipStream_t);
template hipError_t launch_filter<double>(const double *, double *, const GridDev *, const TileDev *, int,
                                          double, hipStream_t);

}  // namespace lbm
