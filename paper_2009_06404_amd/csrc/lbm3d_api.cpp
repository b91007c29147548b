// C ABI of the three-dimensional (D3Q19 / D3Q27) step of liblbm.so: argument
// validation, workspace layout, device tables (sponge damping, sources,
// receivers), launches. The kernels are in lbm3d_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lbm3d.h"
#include "lbm3d_internal.h"

namespace lbm {
int report_error(int code, const char *msg);
}

using namespace lbm3;

namespace {

int fail3(int code, const std::string &msg) { return lbm::report_error(code, msg.c_str()); }

#define HIP3_TRY(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail3(LBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

int64_t up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout3 {
  int32_t q = 19;
  int32_t pitch = 0;
  int64_t zplane = 0;    // elements per z plane of populations
  int64_t f_elems = 0;   // one population buffer
  int64_t k_elems = 0;   // kappa plane
  size_t esize = 4;
  size_t f_bytes() const { return (size_t)up(f_elems * (int64_t)esize, 256); }
  size_t bytes() const { return 2 * f_bytes() + (size_t)up(k_elems * (int64_t)esize, 256) + 256; }
};

int make_layout3(int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t dtype, Layout3 *L) {
  if (dtype != LBM_F32 && dtype != LBM_F64) return fail3(LBM_E_INVALID, "dtype must be LBM_F32 or LBM_F64");
  if (q != kQ19 && q != kQ27) return fail3(LBM_E_INVALID, "lattice must be LBM3_D3Q19 or LBM3_D3Q27");
  if (nx < 3 || ny < 3 || nz < 3) return fail3(LBM_E_INVALID, "nx, ny and nz must be >= 3");
  if ((int64_t)nx * ny * nz > (int64_t)INT32_MAX)
    return fail3(LBM_E_INVALID, "volume larger than 2^31 cells");
  L->esize = dtype == LBM_F64 ? 8 : 4;
  L->pitch = (int32_t)up(nx, 64);
  L->q = q;
  L->zplane = (int64_t)ny * q * L->pitch;
  // the kernels address a plane of populations with 32-bit byte offsets
  // behind a buffer descriptor of 2^31 - 1 bytes
  if (L->zplane * (int64_t)L->esize > (int64_t)INT32_MAX)
    return fail3(LBM_E_INVALID, "one z plane of q x ny x pitch populations must stay below 2 GiB");
  L->f_elems = L->zplane * nz;
  L->k_elems = (int64_t)L->pitch * ny * nz;
  return LBM_OK;
}

template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t put(const std::vector<T> &v, hipStream_t s) {
    if (v.size() > n || !p) {
      if (p) hipFree(p);
      p = nullptr;
      n = 0;
      hipError_t e = hipMalloc((void **)&p, std::max<size_t>(v.size(), 1) * sizeof(T));
      if (e != hipSuccess) return e;
      n = std::max<size_t>(v.size(), 1);
    }
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace

struct lbm3_ctx {
  int32_t nx = 0, ny = 0, nz = 0, dtype = LBM_F32;
  Layout3 L;
  double tau = 1.0;
  lbm3_bc bc{};
  hipStream_t stream = nullptr;
  char *fbuf[2] = {nullptr, nullptr};
  char *kappa = nullptr;
  int cur = 0;
  int64_t t = 0;
  const void *rho0 = nullptr;       // caller's density field (receiver scales)
  int32_t rows_y = 6, planes_z = 0;
  int32_t lean_width = 64;          // columns of a lean tile asked for (64 or 128)
  Vol3Dev v{};
  DBuf<char> d_damp, d_rec_scale;
  DBuf<Src3Dev> d_src;
  DBuf<int32_t> d_rec_row, d_rec_plane, d_rec_x, d_rec_id, d_xyz;
  std::vector<Src3Dev> sources;
  std::vector<int32_t> rec_xyz;     // receivers (x, y, z), for the tile classification
  // tile lists: lean, lean with sources, general, and every tile (for the
  // macroscopic fields)
  DBuf<Tile3Dev> d_lean, d_lean_src, d_general, d_all;
  int n_lean = 0, n_lean_src = 0, n_general = 0, n_all = 0;
  int64_t lean_cells = 0, general_cells = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // the general kernel runs on a second stream, beside the lean one
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  double vn_growth = 0.0;           // largest von Neumann factor over the media's nu
  bool free_printed = false;        // a face uses LBM_FREE
};

namespace {

bool f64(const lbm3_ctx *c) { return c->dtype == LBM_F64; }

// Rows per tile of the general kernel (the general lists and the field
// launch): the launch's rows, except that 14-row tiles are cut into 2-row
// ones. The general kernel with 14 rows per tile needs more than the 128
// VGPRs its 1024-lane workgroup allows and spills to scratch.
int general_rows(const lbm3_ctx *c) { return c->rows_y == 14 ? 2 : c->rows_y; }

// Width of the lean tiles: 128 columns (two wavefronts per row, so each
// population row a workgroup reads is 512 contiguous bytes in FP32) where the
// setting asks for it and the kernel exists (FP32, tiles of 2 or 6 rows: the
// FP64 kernel needs more registers than a 1024-lane workgroup allows), else
// 64. The general and field tiles are always 64 columns wide.
bool wide_ok(const lbm3_ctx *c) { return c->dtype == LBM_F32; }
int lean_tx(const lbm3_ctx *c) { return c->lean_width == 128 && wide_ok(c) && c->rows_y != 14 ? 128 : 64; }

// General tiles are cut into z chunks of at most this many planes: more,
// shorter workgroups, which hide beside the lean launch better than a few
// that march a whole segment (256^3 half-space, FP32: D3Q19 0.625 against
// 0.631 ms per step, D3Q27 0.897 against 0.930, with the general launch first).
constexpr int kGeneralPlanes = 4;

int default_planes(const lbm3_ctx *c, int rows_y, int tx) {
  // segments of 16 planes (12 with 128-column tiles; each re-pulls one plane
  // before and after it, mostly from L2), shorter when the volume has too few
  // tiles per plane for 2048 workgroups (8 per CU; 1536 of the 1024-lane
  // workgroups of 128-column tiles, one per CU at a time). 256^3 half-space,
  // FP32, 128-column tiles, whole step: D3Q19 28.3 GLUPS at 12 planes, 28.1
  // at 8, 26.8 at 6; D3Q27 20.4, 20.0 and 19.4.
  const int64_t tiles = (int64_t)((c->nx + tx - 1) / tx) * ((c->ny + rows_y - 1) / rows_y);
  const int64_t target = tx == 128 ? 1536 : 2048, cap = tx == 128 ? 12 : 16;
  const int64_t nseg = std::max<int64_t>(1, (target + tiles - 1) / tiles);
  const int64_t pz = std::max<int64_t>(4, std::min<int64_t>(cap, (c->nz + nseg - 1) / nseg));
  return (int)std::min<int64_t>(pz, c->nz);
}

// Plane segments of the z march. With non-periodic top and bottom faces the
// two planes next to each face form segments of their own (their tiles pull
// face cells), the planes between them segments of planes_z.
std::vector<std::pair<int, int>> z_segments(const lbm3_ctx *c) {
  std::vector<std::pair<int, int>> segs;
  const int nz = c->nz, pz = std::max(1, c->planes_z);
  const bool zper = c->bc.face[LBM3_FACE_TOP] == LBM_PERIODIC;
  int lo = 0, hi = nz;
  if (!zper && nz > 4) {
    segs.push_back({0, 2});
    lo = 2;
    hi = nz - 2;
  }
  for (int z = lo; z < hi; z += pz) segs.push_back({z, std::min(z + pz, hi)});
  if (!zper && nz > 4) segs.push_back({nz - 2, nz});
  return segs;
}

// Smallest distance from coordinate s to the cells [a, b) along an axis of n
// cells (the minimum image where the axis is periodic).
double axis_gap(double s, int a, int b, int n, bool periodic) {
  auto gap = [&](double q) { return q < a ? a - q : (q > b - 1 ? q - (b - 1) : 0.0); };
  double g = gap(s);
  if (periodic) g = std::min(g, std::min(gap(s - n), gap(s + n)));
  return g;
}

// Split the tiles into the lean list (no pulled cell on a non-periodic face,
// no source within 9 sigma of a cell, no receiver), the lean-with-sources
// list (the same but a source within reach) and the general list.
int build_tiles(lbm3_ctx *c) {
  const int nx = c->nx, ny = c->ny, nz = c->nz, ty = c->rows_y;
  const int tw = lean_tx(c);   // tile width of the lean and general split
  const bool xper = c->bc.face[LBM3_FACE_LEFT] == LBM_PERIODIC;
  const bool yper = c->bc.face[LBM3_FACE_FRONT] == LBM_PERIODIC;
  const bool zper = c->bc.face[LBM3_FACE_TOP] == LBM_PERIODIC;
  const auto segs = z_segments(c);
  const int ntx = (nx + tw - 1) / tw, nty = (ny + ty - 1) / ty, ns = (int)segs.size();
  std::vector<char> rec(static_cast<size_t>(ntx) * nty * ns, 0);
  std::vector<int> seg_of(nz);
  for (int k = 0; k < ns; ++k)
    for (int z = segs[k].first; z < segs[k].second; ++z) seg_of[z] = k;
  for (size_t r = 0; r + 2 < c->rec_xyz.size(); r += 3) {
    const int x = c->rec_xyz[r], y = c->rec_xyz[r + 1], z = c->rec_xyz[r + 2];
    rec[((size_t)seg_of[z] * nty + y / ty) * ntx + x / tw] = 1;
  }
  std::vector<Tile3Dev> lean, lean_src, gen, all;
  int64_t lean_cells = 0, gen_cells = 0;
  for (int k = 0; k < ns; ++k) {
    const int z0 = segs[k].first, z1 = segs[k].second;
    for (int j = 0; j < nty; ++j) {
      const int y0 = j * ty, h = std::min(ty, ny - y0);
      for (int i = 0; i < ntx; ++i) {
        const int x0 = i * tw, w = std::min(tw, nx - x0);
        bool general = rec[((size_t)k * nty + j) * ntx + i] != 0, src = false;
        // pulled cells: [x0-1, x0+w] x [y0-1, y0+h] x [z0-1, z1]
        if (!xper && (x0 - 1 <= 0 || x0 + w >= nx - 1)) general = true;
        if (!yper && (y0 - 1 <= 0 || y0 + h >= ny - 1)) general = true;
        if (!zper && (z0 - 1 <= 0 || z1 >= nz - 1)) general = true;
        for (const Src3Dev &q : c->sources) {
          const double cut = 9.0 * q.sigma;
          if (axis_gap(q.x, x0, x0 + w, nx, xper) <= cut && axis_gap(q.y, y0, y0 + h, ny, yper) <= cut &&
              axis_gap(q.z, z0, z1, nz, zper) <= cut)
            src = true;
        }
        const Tile3Dev t{x0, y0, z0, z1};
        const int64_t cells = (int64_t)w * h * (z1 - z0);
        const int gr = general_rows(c);
        // the general and field kernels take 64-column tiles
        for (int xs = x0; xs < x0 + w; xs += 64)
          for (int ys = y0; ys < y0 + h; ys += gr) all.push_back(Tile3Dev{xs, ys, z0, z1});
        if (general) {
          for (int xs = x0; xs < x0 + w; xs += 64)
            for (int ys = y0; ys < y0 + h; ys += gr)
              for (int zs = z0; zs < z1; zs += kGeneralPlanes)
                gen.push_back(Tile3Dev{xs, ys, zs, std::min(zs + kGeneralPlanes, z1)});
          gen_cells += cells;
        } else {
          (src ? lean_src : lean).push_back(t);
          (src ? gen_cells : lean_cells) += cells;   // timed with the general launch
        }
      }
    }
  }
  HIP3_TRY(c->d_lean.put(lean, c->stream));
  HIP3_TRY(c->d_lean_src.put(lean_src, c->stream));
  HIP3_TRY(c->d_general.put(gen, c->stream));
  HIP3_TRY(c->d_all.put(all, c->stream));
  c->n_lean = (int)lean.size();
  c->n_lean_src = (int)lean_src.size();
  c->n_general = (int)gen.size();
  c->n_all = (int)all.size();
  c->lean_cells = lean_cells;
  c->general_cells = gen_cells;
  return LBM_OK;
}

int launch_list(lbm3_ctx *c, bool general, const Tile3Dev *tiles, int n, const void *fin,
                void *fout, void *out10, int mode, bool src = false) {
  if (n <= 0) return LBM_OK;
  c->v.omega = 1.0 / c->tau;
  const int rc = launch_step3(f64(c), general, src, general ? general_rows(c) : c->rows_y,
                              general ? 64 : lean_tx(c), tiles, n, fin, fout, out10, c->v, c->t,
                              mode, c->stream);
  if (rc != 0) return fail3(LBM_E_DEVICE, std::string("step launch: ") + hipGetErrorString((hipError_t)rc));
  return LBM_OK;
}

// One step: the general tiles and then the lean tiles near sources on the
// context's stream, the other lean tiles beside them on the library's second
// stream, forked from the context's stream before the general launch and
// joined back after it. They read the same state and write disjoint cells.
// The general launch goes first so that its few, slower workgroups start
// before the lean ones fill the chip (the fork's wait delays the lean launch
// by a few microseconds).
int launch_step(lbm3_ctx *c) {
  const void *fin = c->fbuf[c->cur];
  void *fout = c->fbuf[c->cur ^ 1];
  if (c->n_general + c->n_lean_src > 0 && c->n_lean > 0) {
    HIP3_TRY(hipEventRecord(c->fork, c->stream));
    int rc = launch_list(c, true, c->d_general.p, c->n_general, fin, fout, nullptr, 0);
    if (!rc) rc = launch_list(c, false, c->d_lean_src.p, c->n_lean_src, fin, fout, nullptr, 0, true);
    if (rc) return rc;
    HIP3_TRY(hipStreamWaitEvent(c->side, c->fork, 0));
    hipStream_t main = c->stream;
    c->stream = c->side;
    rc = launch_list(c, false, c->d_lean.p, c->n_lean, fin, fout, nullptr, 0);
    c->stream = main;
    if (rc) return rc;
    HIP3_TRY(hipEventRecord(c->join, c->side));
    HIP3_TRY(hipStreamWaitEvent(c->stream, c->join, 0));
    return LBM_OK;
  }
  int rc = launch_list(c, false, c->d_lean.p, c->n_lean, fin, fout, nullptr, 0);
  if (!rc) rc = launch_list(c, false, c->d_lean_src.p, c->n_lean_src, fin, fout, nullptr, 0, true);
  if (!rc) rc = launch_list(c, true, c->d_general.p, c->n_general, fin, fout, nullptr, 0);
  return rc;
}

int validate_bc(const lbm3_bc *bc, int32_t nx, int32_t ny, int32_t nz) {
  const int ext[6] = {nz, nz, nx, nx, ny, ny};
  for (int f = 0; f < 6; ++f) {
    const int k = bc->face[f];
    if (k != LBM_PERIODIC && k != LBM_FREE && k != LBM_RIGID && k != LBM_FREE0)
      return fail3(LBM_E_INVALID, "unknown face kind");
    if ((k == LBM_FREE || k == LBM_FREE0) && f > LBM3_FACE_BOTTOM)
      return fail3(LBM_E_INVALID, "free surface allowed on the top and bottom faces only");
    if (bc->thick[f] < 0 || bc->thick[f] > ext[f])
      return fail3(LBM_E_INVALID, "sponge thickness out of range");
    if (bc->thick[f] > 0) {
      if (!bc->profile[f]) return fail3(LBM_E_INVALID, "sponge profile missing");
      for (int k2 = 0; k2 < bc->thick[f]; ++k2)
        if (!(bc->profile[f][k2] >= 0.0) || !std::isfinite(bc->profile[f][k2]))
          return fail3(LBM_E_INVALID, "sponge profile values must be finite and >= 0");
    }
  }
  for (int a = 0; a < 3; ++a)
    if ((bc->face[2 * a] == LBM_PERIODIC) != (bc->face[2 * a + 1] == LBM_PERIODIC))
      return fail3(LBM_E_INVALID, "periodic faces must be paired");
  return LBM_OK;
}

template <typename real>
std::vector<char> damp_table(const lbm3_ctx *c) {
  // damping per x, per y and per z: the larger of the two opposite faces'
  // profiles; a cell's damping is the largest of its three values
  std::vector<real> d((size_t)c->nx + c->ny + c->nz, real(0));
  const int n[3] = {c->nx, c->ny, c->nz};
  const int lo[3] = {LBM3_FACE_LEFT, LBM3_FACE_FRONT, LBM3_FACE_TOP};
  const int hi[3] = {LBM3_FACE_RIGHT, LBM3_FACE_BACK, LBM3_FACE_BOTTOM};
  size_t off = 0;
  for (int a = 0; a < 3; ++a) {
    for (int p = 0; p < n[a]; ++p) {
      double v = 0.0;
      const int dl = p, dh = n[a] - 1 - p;
      if (dl < c->bc.thick[lo[a]]) v = std::max(v, c->bc.profile[lo[a]][dl]);
      if (dh < c->bc.thick[hi[a]]) v = std::max(v, c->bc.profile[hi[a]][dh]);
      d[off + p] = real(v);
    }
    off += n[a];
  }
  std::vector<char> b(d.size() * sizeof(real));
  memcpy(b.data(), d.data(), b.size());
  return b;
}

// Poisson ratio of a cell from its kappa = b^2 (1 - lambda/mu).
double nu_of_kappa3(double kappa) {
  const double r = 1.0 - 3.0 * kappa;   // lambda / mu
  return r / (2.0 * (1.0 + r));
}

// The init-time stability verdict: the factor at the extreme Poisson ratios
// of the medium (and the middle one) on a 9-point grid per axis, and the
// printed free surface, which lets short surface modes grow.
int stability_verdict3(lbm3_ctx *c, double kmin, double kmax) {
  double g = 0.0;
  const double nus[3] = {nu_of_kappa3(kmin), nu_of_kappa3(kmax), nu_of_kappa3(0.5 * (kmin + kmax))};
  for (int s = 0; s < (kmin == kmax ? 1 : 3); ++s) g = std::max(g, vn_growth3(c->L.q, nus[s], c->tau, 9));
  c->vn_growth = g;
  c->free_printed = c->bc.face[LBM3_FACE_TOP] == LBM_FREE || c->bc.face[LBM3_FACE_BOTTOM] == LBM_FREE;
  if (g > 1.0 + 1e-6) {
    char buf[200];
    snprintf(buf, sizeof buf, "bulk modes grow by up to %.6f per step for these Poisson ratios at tau = %g",
             g, c->tau);
    lbm::report_error(LBM_WARN_UNSTABLE, buf);
    return LBM_WARN_UNSTABLE;
  }
  if (c->free_printed) {
    lbm::report_error(LBM_WARN_UNSTABLE,
                      "LBM_FREE (linear extrapolation) lets short surface modes grow; LBM_FREE0 is the stable variant");
    return LBM_WARN_UNSTABLE;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm3_vn_growth(int32_t q, double nu, double tau, int32_t nk, double *growth) {
  if (!growth) return fail3(LBM_E_INVALID, "growth required");
  if (q != kQ19 && q != kQ27) return fail3(LBM_E_INVALID, "lattice must be LBM3_D3Q19 or LBM3_D3Q27");
  if (!(nu >= 0.0 && nu < 0.5) || !(tau > 0.5) || !std::isfinite(tau) || nk < 2 || nk > 129)
    return fail3(LBM_E_INVALID, "0 <= nu < 1/2, tau > 1/2 and 2 <= nk <= 129 required");
  *growth = vn_growth3(q, nu, tau, nk);
  return LBM_OK;
}

int lbm3_stability(const lbm3_ctx *c, double *growth) {
  if (!c || !growth) return fail3(LBM_E_INVALID, "context and growth required");
  *growth = c->vn_growth;
  if (c->vn_growth > 1.0 + 1e-6 || c->free_printed) return LBM_WARN_UNSTABLE;
  return LBM_OK;
}

int lbm3_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t dtype,
                         size_t *bytes) {
  if (!bytes) return fail3(LBM_E_INVALID, "bytes required");
  Layout3 L;
  const int rc = make_layout3(nx, ny, nz, q, dtype, &L);
  if (rc) return rc;
  *bytes = L.bytes();
  return LBM_OK;
}

int lbm3_init(lbm3_ctx **ctx, int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t dtype,
              const void *lam, const void *mu, const void *rho, double tau, const lbm3_bc *bc,
              void *workspace, size_t ws_bytes, void *hip_stream) {
  if (!ctx) return fail3(LBM_E_INVALID, "ctx required");
  *ctx = nullptr;
  Layout3 L;
  int rc = make_layout3(nx, ny, nz, q, dtype, &L);
  if (rc) return rc;
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail3(LBM_E_INVALID, "tau must be > 1/2");
  if (!bc) return fail3(LBM_E_INVALID, "bc required");
  if ((rc = validate_bc(bc, nx, ny, nz))) return rc;
  if (!lam || !mu || !rho) return fail3(LBM_E_INVALID, "lam, mu and rho required");
  if (!workspace) return fail3(LBM_E_INVALID, "workspace required");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail3(LBM_E_INVALID, "workspace must be 256-B aligned");
  if (ws_bytes < L.bytes()) return fail3(LBM_E_NOMEM, "workspace too small");

  lbm3_ctx *c = new lbm3_ctx();
  c->nx = nx; c->ny = ny; c->nz = nz; c->dtype = dtype; c->L = L; c->tau = tau;
  c->bc = *bc;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->rho0 = rho;
  char *w = static_cast<char *>(workspace);
  c->fbuf[0] = w;
  c->fbuf[1] = w + L.f_bytes();
  c->kappa = w + 2 * L.f_bytes();
  auto bail = [&](int code) { lbm3_destroy(c); return code; };
  // profiles are copied: the host arrays need not outlive the call
  std::vector<std::vector<double>> prof(6);
  for (int f = 0; f < 6; ++f) {
    prof[f].assign(bc->profile[f] ? bc->profile[f] : nullptr,
                   bc->profile[f] ? bc->profile[f] + bc->thick[f] : nullptr);
    c->bc.profile[f] = prof[f].data();
  }
  hipError_t e = hipMemsetAsync(c->fbuf[0], 0, L.f_bytes(), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->fbuf[1], 0, L.f_bytes(), c->stream);
  if (e != hipSuccess) return bail(fail3(LBM_E_DEVICE, hipGetErrorString(e)));

  // kappa plane, field checks and the kappa range (scalar when uniform)
  unsigned int *d_bad = nullptr;
  double *d_mm = nullptr;
  e = hipMalloc((void **)&d_bad, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMalloc((void **)&d_mm, 2 * kKappaBlocks * sizeof(double));
  if (e == hipSuccess) e = hipMemsetAsync(d_bad, 0, sizeof(unsigned int), c->stream);
  int nb = 0;
  if (e == hipSuccess)
    e = (hipError_t)launch_kappa3(dtype == LBM_F64, lam, mu, rho, c->kappa, nx, ny, nz, L.pitch, d_bad,
                                  d_mm, &nb, c->stream);
  unsigned int bad = 0;
  std::vector<double> mm(2 * kKappaBlocks);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(mm.data(), d_mm, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (d_bad) hipFree(d_bad);
  if (d_mm) hipFree(d_mm);
  if (e != hipSuccess) return bail(fail3(LBM_E_DEVICE, hipGetErrorString(e)));
  if (bad) {
    char buf[160];
    snprintf(buf, sizeof buf, "%u cells outside 0 <= nu < 1/2, mu > 0, rho > 0", bad);
    return bail(fail3(LBM_E_INVALID, buf));
  }
  double kmin = mm[0], kmax = mm[1];
  for (int b = 1; b < nb; ++b) {
    kmin = std::min(kmin, mm[2 * b]);
    kmax = std::max(kmax, mm[2 * b + 1]);
  }

  std::vector<char> damp = dtype == LBM_F64 ? damp_table<double>(c) : damp_table<float>(c);
  e = c->d_damp.put(damp, c->stream);
  if (e == hipSuccess) e = c->d_src.put(std::vector<Src3Dev>(), c->stream);
  for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev[k]);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(fail3(LBM_E_DEVICE, hipGetErrorString(e)));

  Vol3Dev &v = c->v;
  v.nx = nx; v.ny = ny; v.nz = nz; v.pitch = L.pitch;
  v.q = q;
  for (int f = 0; f < 6; ++f) v.face[f] = bc->face[f];
  v.kcells = kmin != kmax;
  v.kscalar = kmin;
  v.nsrc = 0;
  v.omega = 1.0 / tau;
  v.zplane = L.zplane;
  v.kappa = c->kappa;
  v.damp = c->d_damp.p;
  v.src = c->d_src.p;
  v.rec_row = nullptr;
  c->lean_width = wide_ok(c) ? 128 : 64;
  c->planes_z = default_planes(c, c->rows_y, lean_tx(c));
  // the profiles were only needed for the damping table
  for (int f = 0; f < 6; ++f) c->bc.profile[f] = nullptr;
  if ((rc = build_tiles(c))) return bail(rc);
  *ctx = c;
  return stability_verdict3(c, kmin, kmax);
}

int lbm3_set_sources(lbm3_ctx *c, const lbm3_source *src, int32_t n) {
  if (!c) return fail3(LBM_E_INVALID, "null context");
  if (n < 0 || n > kMaxSources || (n > 0 && !src)) return fail3(LBM_E_INVALID, "0 <= n <= 256 sources required");
  std::vector<Src3Dev> s(n);
  for (int k = 0; k < n; ++k) {
    const lbm3_source &q = src[k];
    if (!(q.x >= 0 && q.x <= c->nx - 1 && q.y >= 0 && q.y <= c->ny - 1 && q.z >= 0 && q.z <= c->nz - 1))
      return fail3(LBM_E_INVALID, "source outside the volume");
    if (!(q.sigma > 0) || !(q.period > 0) || !std::isfinite(q.amp) || !std::isfinite(q.t0) ||
        !std::isfinite(q.dir_x) || !std::isfinite(q.dir_y) || !std::isfinite(q.dir_z))
      return fail3(LBM_E_INVALID, "source needs sigma > 0, period > 0 and finite values");
    s[k] = Src3Dev{q.x, q.y, q.z, q.sigma, q.dir_x, q.dir_y, q.dir_z, q.amp, q.period, q.t0};
  }
  HIP3_TRY(c->d_src.put(s, c->stream));
  c->v.src = c->d_src.p;
  c->v.nsrc = n;
  c->sources = s;
  return build_tiles(c);
}

int lbm3_set_receivers(lbm3_ctx *c, const int32_t *xyz, int32_t n, int32_t comp_mask, void *traces,
                       int64_t max_steps) {
  if (!c) return fail3(LBM_E_INVALID, "null context");
  if (n < 0 || (n > 0 && (!xyz || !traces || max_steps < 0)))
    return fail3(LBM_E_INVALID, "n >= 0 receivers with xyz, traces and max_steps >= 0 required");
  if (n > 0 && (comp_mask <= 0 || comp_mask > 7)) return fail3(LBM_E_INVALID, "comp_mask must be in 1..7");
  if (n == 0) {
    c->v.rec_row = nullptr;
    c->v.nrec = 0;
    c->v.trace = nullptr;
    c->rec_xyz.clear();
    return build_tiles(c);
  }
  std::vector<int32_t> q(xyz, xyz + 3 * (size_t)n);
  for (int k = 0; k < n; ++k)
    if (q[3 * k] < 0 || q[3 * k] >= c->nx || q[3 * k + 1] < 0 || q[3 * k + 1] >= c->ny ||
        q[3 * k + 2] < 0 || q[3 * k + 2] >= c->nz)
      return fail3(LBM_E_INVALID, "receiver outside the volume");
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto key = [&](int k) {
    return ((int64_t)q[3 * k + 2] * c->ny + q[3 * k + 1]) * c->nx + q[3 * k];
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
  const int64_t rows = (int64_t)c->nz * c->ny;
  std::vector<int32_t> row(rows + 1, 0), plane(c->nz, 0), rx(n), rid(n), sxyz(3 * (size_t)n);
  for (int k = 0; k < n; ++k) {
    const int o = order[k];
    row[(int64_t)q[3 * o + 2] * c->ny + q[3 * o + 1] + 1]++;
    plane[q[3 * o + 2]] = 1;
    rx[k] = q[3 * o];
    rid[k] = o;
    for (int a = 0; a < 3; ++a) sxyz[3 * k + a] = q[3 * o + a];
  }
  for (int64_t r = 0; r < rows; ++r) row[r + 1] += row[r];
  HIP3_TRY(c->d_rec_row.put(row, c->stream));
  HIP3_TRY(c->d_rec_plane.put(plane, c->stream));
  HIP3_TRY(c->d_rec_x.put(rx, c->stream));
  HIP3_TRY(c->d_rec_id.put(rid, c->stream));
  HIP3_TRY(c->d_xyz.put(sxyz, c->stream));
  HIP3_TRY(c->d_rec_scale.put(std::vector<char>((size_t)n * c->L.esize), c->stream));
  if (launch_gather_inv3(f64(c), c->rho0, c->d_xyz.p, n, c->nx, c->ny, c->d_rec_scale.p, c->stream))
    return fail3(LBM_E_DEVICE, "receiver scale gather failed");
  HIP3_TRY(hipStreamSynchronize(c->stream));
  Vol3Dev &v = c->v;
  v.rec_row = c->d_rec_row.p;
  v.rec_plane = c->d_rec_plane.p;
  v.rec_x = c->d_rec_x.p;
  v.rec_id = c->d_rec_id.p;
  v.rec_scale = c->d_rec_scale.p;
  v.trace = traces;
  v.trace_t0 = c->t;
  v.trace_max = max_steps;
  v.nrec = n;
  v.comp_mask = comp_mask;
  c->rec_xyz = q;
  return build_tiles(c);
}

int lbm3_step(lbm3_ctx *c, int64_t n) {
  if (!c) return fail3(LBM_E_INVALID, "null context");
  if (n < 0) return fail3(LBM_E_INVALID, "n must be >= 0");
  for (int64_t k = 0; k < n; ++k) {
    const int rc = launch_step(c);
    if (rc) return rc;
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

int lbm3_step_timed(lbm3_ctx *c, int64_t n, lbm3_kernel_times *out) {
  if (!c) return fail3(LBM_E_INVALID, "null context");
  if (n < 1 || !out) return fail3(LBM_E_INVALID, "n >= 1 and out required");
  double lean = 0.0, gen = 0.0, step = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const void *fin = c->fbuf[c->cur];
    void *fout = c->fbuf[c->cur ^ 1];
    HIP3_TRY(hipEventRecord(c->ev[0], c->stream));
    int rc = launch_list(c, false, c->d_lean.p, c->n_lean, fin, fout, nullptr, 0);
    if (rc) return rc;
    HIP3_TRY(hipEventRecord(c->ev[1], c->stream));
    rc = launch_list(c, true, c->d_general.p, c->n_general, fin, fout, nullptr, 0);
    if (!rc) rc = launch_list(c, false, c->d_lean_src.p, c->n_lean_src, fin, fout, nullptr, 0, true);
    if (rc) return rc;
    HIP3_TRY(hipEventRecord(c->ev[2], c->stream));
    HIP3_TRY(hipEventSynchronize(c->ev[2]));
    float a = 0.f, b = 0.f;
    HIP3_TRY(hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
    HIP3_TRY(hipEventElapsedTime(&b, c->ev[1], c->ev[2]));
    lean += a;
    gen += b;
    step += a + b;
    c->cur ^= 1;
    c->t += 1;
  }
  out->steps = n;
  out->lean_ms = c->n_lean ? lean / (double)n : 0.0;
  out->general_ms = c->n_general + c->n_lean_src ? gen / (double)n : 0.0;
  out->lean_cells = c->lean_cells;
  out->general_cells = c->general_cells;
  out->step_ms = step / (double)n;
  return LBM_OK;
}

int lbm3_moments(lbm3_ctx *c, void *out10) {
  if (!c || !out10) return fail3(LBM_E_INVALID, "context and out10 required");
  return launch_list(c, true, c->d_all.p, c->n_all, c->fbuf[c->cur], nullptr, out10, 1);
}

int lbm3_get_time(const lbm3_ctx *c, int64_t *t) {
  if (!c || !t) return fail3(LBM_E_INVALID, "context and t required");
  *t = c->t;
  return LBM_OK;
}

int lbm3_get_state(lbm3_ctx *c, void *dst) {
  if (!c || !dst) return fail3(LBM_E_INVALID, "context and dst required");
  if (launch_pack3(f64(c), c->L.q, c->fbuf[c->cur], dst, c->nx, c->ny, c->nz, c->L.pitch, false,
                   c->stream))
    return fail3(LBM_E_DEVICE, "state copy failed");
  return LBM_OK;
}

int lbm3_set_state(lbm3_ctx *c, const void *src, int64_t t) {
  if (!c || !src) return fail3(LBM_E_INVALID, "context and src required");
  if (t < 0) return fail3(LBM_E_INVALID, "t must be >= 0");
  if (launch_pack3(f64(c), c->L.q, src, c->fbuf[c->cur], c->nx, c->ny, c->nz, c->L.pitch, true,
                   c->stream))
    return fail3(LBM_E_DEVICE, "state copy failed");
  if (t != c->t) c->v.trace_t0 = t;
  c->t = t;
  return LBM_OK;
}

int lbm3_set_tile(lbm3_ctx *c, int32_t rows_y, int32_t planes_z) {
  if (!c) return fail3(LBM_E_INVALID, "null context");
  if (rows_y != 2 && rows_y != 6 && rows_y != 14) return fail3(LBM_E_INVALID, "rows_y must be 2, 6 or 14");
  if (planes_z < 0) return fail3(LBM_E_INVALID, "planes_z must be >= 0 (0: default)");
  c->rows_y = rows_y;
  c->planes_z = planes_z == 0 ? default_planes(c, rows_y, lean_tx(c)) : std::min(planes_z, c->nz);
  return build_tiles(c);
}

int lbm3_set_lean_width(lbm3_ctx *c, int32_t columns) {
  if (!c) return fail3(LBM_E_INVALID, "null context");
  if (columns != 64 && columns != 128) return fail3(LBM_E_INVALID, "columns must be 64 or 128");
  if (columns == 128 && !wide_ok(c)) return fail3(LBM_E_INVALID, "128-column tiles need an FP32 context");
  c->lean_width = columns;
  return build_tiles(c);
}

int lbm3_get_lean_width(const lbm3_ctx *c, int32_t *columns) {
  if (!c || !columns) return fail3(LBM_E_INVALID, "context and columns required");
  *columns = lean_tx(c);
  return LBM_OK;
}

int lbm3_get_tile(const lbm3_ctx *c, int32_t *rows_y, int32_t *planes_z) {
  if (!c || !rows_y || !planes_z) return fail3(LBM_E_INVALID, "context, rows_y and planes_z required");
  *rows_y = c->rows_y;
  *planes_z = c->planes_z;
  return LBM_OK;
}

int lbm3_destroy(lbm3_ctx *c) {
  if (!c) return LBM_OK;
  hipStreamSynchronize(c->stream);
  c->d_damp.release();
  c->d_rec_scale.release();
  c->d_src.release();
  c->d_rec_row.release();
  c->d_rec_plane.release();
  c->d_rec_x.release();
  c->d_rec_id.release();
  c->d_xyz.release();
  c->d_lean.release();
  c->d_lean_src.release();
  c->d_general.release();
  c->d_all.release();
  for (auto &e : c->ev)
    if (e) hipEventDestroy(e);
  if (c->fork) hipEventDestroy(c->fork);
  if (c->join) hipEventDestroy(c->join);
  if (c->side) {
    hipStreamSynchronize(c->side);
    hipStreamDestroy(c->side);
  }
  delete c;
  return LBM_OK;
}

}  // extern "C"
