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

// A workgroup of 256 lanes takes a tile of 256 columns down its rows. Each
// lane keeps the five rows y-2 .. y+2 of its column in registers and the
// row two ahead of them in flight; every row also goes into a four-row LDS
// ring for the x neighbours, with four lanes loading the two halo columns on
// each side (also a row ahead). One barrier per row.
template <typename real>
__global__ __launch_bounds__(256) void filter_kernel(const real *__restrict__ fin, real *__restrict__ fout,
                                                     const GridDev *__restrict__ grids,
                                                     const TileDev *__restrict__ tiles, real sigma) {
  constexpr int TW = 256;
  __shared__ real srow[4][9][TW + 4];
  const TileDev t = tiles[blockIdx.x];
  if (t.g < 0) return;
  const GridDev &g = grids[t.g];
  const int nx = g.nx, ny = g.ny, rr = g.rigid_row;
  const int lane = (int)threadIdx.x;
  const int x = t.x0 + lane;
  const bool active = x < nx;
  const int xa = active ? x : nx - 1;
  const int x_end = min(t.x0 + TW, nx);          // columns [x0, x_end) of this tile
  const real *f = fin + g.f_off;
  real *o = fout + g.f_off;
  const int64_t pitch = g.pitch;
  const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
  auto wx = [&](int c) { return c < 0 ? c + nx : (c >= nx ? c - nx : c); };
  // rows outside a non-periodic grid are never used (their terms are left
  // out); clamp them to stay in bounds
  auto wy = [&](int r) { return py ? (r < 0 ? r + ny : (r >= ny ? r - ny : r)) : min(max(r, 0), ny - 1); };
  const bool xs = px ? nx >= 5 : (xa >= 2 && xa <= nx - 3);
  // halo lanes: 0, 1 -> columns x0-2, x0-1 (slots 0, 1); 2, 3 -> x_end,
  // x_end+1 (the slots after the tile's last column)
  int hcol = -1, hslot = 0;
  if (lane < 2) { hcol = t.x0 - 2 + lane; hslot = lane; }
  else if (lane < 4) { hcol = x_end + lane - 2; hslot = (x_end - t.x0) + 2 + lane - 2; }
  const bool hl = lane < 4 && (px || (hcol >= 0 && hcol < nx));
  const int hc = hl ? wx(hcol) : 0;

  auto at = [&](int i, int r, int c) { return f[((int64_t)r * 9 + i) * pitch + c]; };
  real win[9][5];   // rows y-2 .. y+2 of this column
  real pre[9], hpre[9];   // row y+3 of this column and of the halo column (in flight)
  // prologue: rows y0-2 .. y0+1 into the window, and rows y0, y0+1 into the ring
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) win[i][k + 1] = at(i, wy(t.y0 - 2 + k), xa);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = t.y0 + k;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (active) srow[r & 3][i][lane + 2] = win[i][k + 3];
      if (hl) srow[r & 3][i][hslot] = at(i, wy(r), hc);
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pre[i] = at(i, wy(t.y0 + 2), xa);
    hpre[i] = hl ? at(i, wy(t.y0 + 2), hc) : real(0);
  }

  for (int y = t.y0; y < t.y1; ++y) {
    // row y+2 arrives: into the window and the ring; row y+3 goes in flight
    const int yn = wy(y + 3);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
      for (int k = 0; k < 4; ++k) win[i][k] = win[i][k + 1];
      win[i][4] = pre[i];
      if (active) srow[(y + 2) & 3][i][lane + 2] = pre[i];   // (idle lanes would hit the halo slots)
      if (hl) srow[(y + 2) & 3][i][hslot] = hpre[i];
      pre[i] = at(i, yn, xa);
      if (hl) hpre[i] = at(i, yn, hc);
    }
    __syncthreads();
    const bool ys = (py ? ny >= 5 : (y >= 2 && y <= ny - 3)) && !(rr > 0 && y >= rr - 2 && y <= rr + 1);
    const int s = y & 3;
    if (active) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const real c = win[i][2];
        real acc = real(0);
        if (xs)
          acc += ((srow[s][i][lane] + srow[s][i][lane + 4]) -
                  real(4) * (srow[s][i][lane + 1] + srow[s][i][lane + 3])) +
                 real(6) * c;
        if (ys) acc += ((win[i][0] + win[i][4]) - real(4) * (win[i][1] + win[i][3])) + real(6) * c;
        o[((int64_t)y * 9 + i) * pitch + x] = c - sigma * acc;
      }
    }
  }
}

}  // namespace

template <typename real>
hipError_t launch_filter(const real *fin, real *fout, const GridDev *grids, const TileDev *tiles,
                         int ntiles, real sigma, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((filter_kernel<real>), dim3(ntiles), dim3(256), 0, stream, fin, fout, grids, tiles,
                     sigma);
  return hipGetLastError();
}

template hipError_t launch_filter<float>(const float *, float *, const GridDev *, const TileDev *, int, float,
                                         hipStream_t);
template hipError_t launch_filter<double>(const double *, double *, const GridDev *, const TileDev *, int,
                                          double, hipStream_t);

}  // namespace lbm
