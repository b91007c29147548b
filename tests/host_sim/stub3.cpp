// CPU stand-in for the launchers of the three-dimensional step (the runtime
// itself is stub.cpp's). The initialisation kernels are evaluated on the host
// so the host code takes the device's branches; every step launch checks its
// tile list against the volume and the rules of the lean / general split:
//  - each tile lies inside the volume and inside the launch's buffers, 64
//    columns wide (128 for wide lean tiles, FP32 steps only);
//  - a lean tile pulls no cell on a non-periodic face (its cells widened by
//    one in x and y, and by one plane on either side of its segment), holds
//    no cell within 9 sigma of a source (minimum image on periodic axes) and
//    no receiver;
//  - the lean and general launches of one step, and the field launch, write
//    every cell of the volume exactly once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lbm3d_internal.h"

extern "C" void sim_check_range(const void *p, size_t n, const char *what);

namespace {
std::vector<int> g_cov;             // writes per cell of the pending step
int g_nx = 0, g_ny = 0, g_nz = 0;
bool g_pending = false;
const void *g_pending_out = nullptr;
long long g_steps_checked = 0, g_lean_tiles = 0, g_general_tiles = 0, g_wide_launches = 0,
          g_lean_src_tiles = 0;

void fail(const char *msg) {
  fprintf(stderr, "stub3: %s\n", msg);
  abort();
}

void finish_pending() {
  if (!g_pending) return;
  for (size_t i = 0; i < g_cov.size(); ++i)
    if (g_cov[i] != 1) {
      fprintf(stderr, "stub3: cell %zu written %d times in one step\n", i, g_cov[i]);
      abort();
    }
  g_pending = false;
  ++g_steps_checked;
}

double gap(double s, int a, int b, int n, bool periodic) {
  auto one = [&](double q) { return q < a ? a - q : (q > b - 1 ? q - (b - 1) : 0.0); };
  double g = one(s);
  if (periodic) g = std::fmin(g, std::fmin(one(s - n), one(s + n)));
  return g;
}
}  // namespace

extern "C" long long sim3_steps_checked() {
  finish_pending();
  return g_steps_checked;
}
extern "C" long long sim3_lean_tiles() { return g_lean_tiles; }
extern "C" long long sim3_general_tiles() { return g_general_tiles; }
extern "C" long long sim3_wide_launches() { return g_wide_launches; }
extern "C" long long sim3_lean_src_tiles() { return g_lean_src_tiles; }

namespace lbm3 {

int launch_step3(bool f64, bool general, bool src, int rows_y, int tw, const Tile3Dev *tiles,
                 int ntiles, const void *fin, void *fout, void *out10, const Vol3Dev &v, int64_t t,
                 int mode, hipStream_t) {
  if (ntiles <= 0) return 0;
  if (src && (general || mode != 0)) fail("lean source launch outside lean steps");
  if (rows_y != 2 && rows_y != 6 && rows_y != 14) fail("rows_y");
  if (rows_y == 14 && (general || mode == 1)) fail("general or field tiles of 14 rows");
  if (tw != 64 && tw != 128) fail("tile width");
  if (tw == 128 && (general || mode != 0 || f64 || rows_y == 14))
    fail("128-column tiles outside lean FP32 steps in 2- or 6-row tiles");
  if (tw == 128) ++g_wide_launches;
  if (v.q != kQ19 && v.q != kQ27) fail("lattice");
  const size_t es = f64 ? 8 : 4;
  const int nx = v.nx, ny = v.ny, nz = v.nz;
  sim_check_range(tiles, sizeof(Tile3Dev) * ntiles, "tile list");
  sim_check_range(fin, es * (size_t)v.zplane * nz, "fin");
  if (mode == 0) sim_check_range(fout, es * (size_t)v.zplane * nz, "fout");
  else sim_check_range(out10, es * 10 * (size_t)nx * ny * nz, "out10");
  if (v.kcells) sim_check_range(v.kappa, es * (size_t)v.pitch * ny * nz, "kappa");
  sim_check_range(v.damp, es * (size_t)(nx + ny + nz), "damping");
  if (v.nsrc) sim_check_range(v.src, sizeof(Src3Dev) * v.nsrc, "sources");
  if (v.rec_row) {
    sim_check_range(v.rec_row, sizeof(int32_t) * ((size_t)nz * ny + 1), "rec_row");
    sim_check_range(v.rec_plane, sizeof(int32_t) * nz, "rec_plane");
    sim_check_range(v.rec_x, sizeof(int32_t) * v.nrec, "rec_x");
    sim_check_range(v.rec_id, sizeof(int32_t) * v.nrec, "rec_id");
    sim_check_range(v.rec_scale, es * v.nrec, "rec_scale");
    if (mode == 0 && t >= v.trace_t0 && t - v.trace_t0 < v.trace_max)
      sim_check_range(v.trace, es * (size_t)v.nrec * __builtin_popcount(v.comp_mask) * (size_t)v.trace_max,
                      "trace");
  }
  const bool xper = v.face[kFaceLeft] == kPeriodic, yper = v.face[kFaceFront] == kPeriodic;
  const bool zper = v.face[kFaceTop] == kPeriodic;
  // a new step (or field evaluation) starts when the output buffer changes
  // or the previous one was complete
  const void *out = mode == 0 ? fout : out10;
  if (g_pending && (out != g_pending_out || g_nx != nx || g_ny != ny || g_nz != nz)) finish_pending();
  if (!g_pending) {
    g_nx = nx; g_ny = ny; g_nz = nz;
    g_cov.assign((size_t)nx * ny * nz, 0);
    g_pending = true;
    g_pending_out = out;
  }
  for (int k = 0; k < ntiles; ++k) {
    const Tile3Dev tl = tiles[k];
    if (tl.x0 < 0 || tl.x0 >= nx || tl.x0 % tw || tl.y0 < 0 || tl.y0 >= ny || tl.y0 % rows_y ||
        tl.z0 < 0 || tl.z1 > nz || tl.z0 >= tl.z1)
      fail("tile outside the volume");
    const int w = std::min(tw, nx - tl.x0), h = std::min(rows_y, ny - tl.y0);
    if (!general) {
      ++g_lean_tiles;
      if (src) ++g_lean_src_tiles;
      if (!xper && (tl.x0 - 1 <= 0 || tl.x0 + w >= nx - 1)) fail("lean tile pulls an x-face cell");
      if (!yper && (tl.y0 - 1 <= 0 || tl.y0 + h >= ny - 1)) fail("lean tile pulls a y-face cell");
      if (!zper && (tl.z0 - 1 <= 0 || tl.z1 >= nz - 1)) fail("lean tile pulls a z-face cell");
      for (int s = 0; s < v.nsrc; ++s) {
        const Src3Dev &q = v.src[s];
        const double c = 9.0 * q.sigma;
        const double gx = gap(q.x, tl.x0, tl.x0 + w, nx, xper), gy = gap(q.y, tl.y0, tl.y0 + h, ny, yper),
                     gz = gap(q.z, tl.z0, tl.z1, nz, zper);
        if (!src && gx * gx + gy * gy + gz * gz <= c * c) fail("lean tile within 9 sigma of a source");
      }
      if (v.rec_row)
        for (int z = tl.z0; z < tl.z1; ++z)
          for (int y = tl.y0; y < tl.y0 + h; ++y)
            for (int r = v.rec_row[z * ny + y]; r < v.rec_row[z * ny + y + 1]; ++r)
              if (v.rec_x[r] >= tl.x0 && v.rec_x[r] < tl.x0 + w) fail("lean tile holds a receiver");
    } else {
      ++g_general_tiles;
    }
    for (int z = tl.z0; z < tl.z1; ++z)
      for (int y = tl.y0; y < tl.y0 + h; ++y)
        for (int x = tl.x0; x < tl.x0 + w; ++x) ++g_cov[((size_t)z * ny + y) * nx + x];
  }
  return 0;
}

int launch_kappa3(bool f64, const void *lam, const void *mu, const void *rho, void *kappa, int nx,
                  int ny, int nz, int pitch, unsigned int *bad, double *minmax, int *nblocks,
                  hipStream_t) {
  const size_t N = (size_t)nx * ny * nz, es = f64 ? 8 : 4;
  sim_check_range(lam, es * N, "lam");
  sim_check_range(mu, es * N, "mu");
  sim_check_range(rho, es * N, "rho");
  sim_check_range(kappa, es * (size_t)pitch * ny * nz, "kappa");
  double lo = 1e300, hi = -1e300;
  unsigned nb = 0;
  for (size_t k = 0; k < N; ++k) {
    auto get = [&](const void *p) { return f64 ? ((const double *)p)[k] : (double)((const float *)p)[k]; };
    const double l = get(lam), m = get(mu), r = get(rho);
    const double nu = l / (2.0 * (l + m));
    if (!(m > 0.0) || !(r > 0.0) || !(nu >= 0.0) || !(nu < 0.5)) ++nb;
    const double kv = (m - l) / m / 3.0;
    const size_t x = k % nx, yz = k / nx;
    if (f64) ((double *)kappa)[yz * pitch + x] = kv;
    else ((float *)kappa)[yz * pitch + x] = (float)kv;
    const double kr = f64 ? kv : (double)(float)kv;
    lo = std::fmin(lo, kr);
    hi = std::fmax(hi, kr);
  }
  *bad += nb;
  *nblocks = 1;
  minmax[0] = lo;
  minmax[1] = hi;
  return 0;
}

int launch_gather_inv3(bool f64, const void *rho, const int32_t *xyz, int n, int nx, int ny,
                       void *out, hipStream_t) {
  const size_t es = f64 ? 8 : 4;
  sim_check_range(xyz, sizeof(int32_t) * 3 * n, "gather xyz");
  sim_check_range(out, es * n, "gather out");
  for (int k = 0; k < n; ++k) {
    const size_t c = ((size_t)xyz[3 * k + 2] * ny + xyz[3 * k + 1]) * nx + xyz[3 * k];
    sim_check_range((const char *)rho + es * c, es, "gather rho");
    if (f64) ((double *)out)[k] = 1.0 / ((const double *)rho)[c];
    else ((float *)out)[k] = 1.0f / ((const float *)rho)[c];
  }
  return 0;
}

int launch_pack3(bool f64, int q, const void *src, void *dst, int nx, int ny, int nz, int pitch,
                 bool to_pitched, hipStream_t) {
  const size_t es = f64 ? 8 : 4;
  const size_t dense = es * (size_t)q * nx * ny * nz, pitched = es * (size_t)q * pitch * ny * nz;
  sim_check_range(src, to_pitched ? dense : pitched, "pack src");
  sim_check_range(dst, to_pitched ? pitched : dense, "pack dst");
  for (int i = 0; i < q; ++i)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y) {
        const size_t d = (((size_t)i * nz + z) * ny + y) * nx;
        const size_t p = (size_t)z * ny * q * pitch + ((size_t)y * q + i) * pitch;
        if (to_pitched) memcpy((char *)dst + es * p, (const char *)src + es * d, es * nx);
        else memcpy((char *)dst + es * d, (const char *)src + es * p, es * nx);
      }
  return 0;
}

}  // namespace lbm3
