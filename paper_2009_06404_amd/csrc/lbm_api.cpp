// C ABI of liblbm.so: argument validation, workspace layout, device tables,
// tile lists, launches, HIP-graph capture of the time loop and the autotuner.
// The kernels are in lbm_kernels.hip and lbm_util.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(LBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

constexpr int kPitchAlign = 64;     // elements; rows start on 256-B (f32) boundaries
constexpr int kXcds = 8;            // MI355X: 8 accelerator complex dies, L2 per die

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout {
  std::vector<int32_t> pitch;
  std::vector<int64_t> plane, f_off, k_off;
  int64_t f_elems = 0;   // one population buffer
  int64_t k_elems = 0;   // kappa cell planes
  size_t esize = 4;
  // three population buffers (the ping-pong pair and the two-step kernel's
  // intermediate buffer) and the kappa cell planes, each 256-B aligned
  size_t bytes() const {
    return 3 * (size_t)round_up(f_elems * (int64_t)esize, 256) +
           (size_t)round_up(k_elems * (int64_t)esize, 256) + 256;
  }
};

Layout make_layout(const lbm_grid *grids, int n, int dtype) {
  Layout L;
  L.esize = dtype == LBM_F64 ? 8 : 4;
  for (int g = 0; g < n; ++g) {
    const int32_t p = (int32_t)round_up(grids[g].nx, kPitchAlign);
    const int64_t pl = (int64_t)p * grids[g].ny;
    L.pitch.push_back(p);
    L.plane.push_back(pl);
    L.f_off.push_back(L.f_elems);
    L.k_off.push_back(L.k_elems);
    L.f_elems += 9 * pl;
    L.k_elems += pl;
  }
  return L;
}

struct RecHost {
  std::vector<int32_t> xy;
  std::vector<double> scale;   // 1/rho0 at each receiver
  int32_t comp_mask = 0;
  void *trace = nullptr;
  int64_t max_steps = 0;
  int64_t t0 = 0;
};

template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t upload(const std::vector<T> &v, hipStream_t s) {
    if (v.size() > n) {
      if (p) hipFree(p);
      p = nullptr;
      n = 0;
      hipError_t e = hipMalloc((void **)&p, std::max<size_t>(v.size(), 1) * sizeof(T));
      if (e != hipSuccess) return e;
      n = v.size();
    }
    if (!p) {
      hipError_t e = hipMalloc((void **)&p, sizeof(T));
      if (e != hipSuccess) return e;
      n = 1;
    }
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  // room for at least `count` elements, contents undefined
  hipError_t reserve(size_t count) {
    if (count <= n && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc((void **)&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    n = std::max<size_t>(count, 1);
    return hipSuccess;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace

namespace lbm {
// The error text lbm_last_error returns, for the other entry points of the
// library (the three-dimensional step).
int report_error(int code, const char *msg) { return fail(code, msg); }
}  // namespace lbm

struct lbm_ctx {
  int dtype = LBM_F32;
  int nbatch = 0;
  double tau = 1.0;
  hipStream_t stream = nullptr;
  Layout L;
  std::vector<lbm_grid> grids;
  std::vector<lbm_bc> bc;
  std::vector<std::vector<double>> sponge;       // per grid, 4 edges concatenated
  std::vector<std::array<int32_t, 4>> sp_thick;
  std::vector<std::vector<lbm_source>> sources;
  std::vector<RecHost> recs;
  std::vector<int> kmode;
  std::vector<double> kscalar;
  std::vector<double> nu_seen;   // Poisson ratios of the media (samples of their range)
  double vn_growth = 0.0;        // largest von Neumann factor over nu_seen at tau
  const void *rho = nullptr;                     // caller's density field (receiver scale)
  std::vector<int64_t> cell_off;                 // per grid offset into the packed fields
  char *ws = nullptr;
  char *fbuf[2] = {nullptr, nullptr};
  char *kcells = nullptr;
  char *fmid = nullptr;                          // intermediate state of the two-step path
  int cur = 0;                                   // buffer holding f*(t-1)
  int64_t t = 0;
  // library-owned device tables
  DevBuf<GridDev> d_grids;
  DevBuf<TileDev> d_tiles;                       // tiles for the general kernel
  DevBuf<TileDev> d_tiles_int;                   // tiles for the interior kernel
  DevBuf<char> d_krows;                          // dtype elements
  DevBuf<char> d_sponge;                         // dtype elements
  DevBuf<SourceDev> d_src;
  DevBuf<int32_t> d_itab;
  DevBuf<char> d_rtab;                           // dtype elements
  DevBuf<int64_t> d_time;
  std::vector<int64_t> krow_off;                 // per grid offset into d_krows
  std::vector<int64_t> rscale_off;               // per grid offset into d_rtab
  std::vector<char> rtab_host;
  bool tables_dirty = true;
  lbm_launch launch{4, 8, 0, 1, 1, 0, 1, 0, 2};
  // two-step path: fused tiles and the general tiles advanced step by step
  DevBuf<FusedTileDev> d_ftiles;
  DevBuf<TileDev> d_gtiles2;
  DevBuf<TileDev> d_gtiles1;   // first step of a pair: d_gtiles2 plus the two-step blocks' border strips
  // the filter's tiles: 256 columns x kFilterRows rows of every grid
  DevBuf<TileDev> d_filt_tiles;
  int nfilt_tiles = 0;
  int nftiles = 0, ngtiles2 = 0, ngtiles1 = 0;
  int64_t cells_fused = 0, cells_gen2 = 0;
  // three-step path (fuse_steps 3): its blocks, and the general tiles of the
  // triple's steps (d_tgen[k] for step t+k: the general tiles plus the
  // blocks' border strips 4 - 2k deep)
  DevBuf<FusedTileDev> d_ttiles;
  DevBuf<TileDev> d_tgen[3];
  DevBuf<char> d_fmid2;   // the triple's second intermediate state, f*(t+1) (library-owned)
  bool launch_set = false;  // the launch was set by the caller (lbm_set_launch, lbm_autotune)
  int nttiles = 0, ntgen[3] = {0, 0, 0};
  int64_t cells_tri = 0, cells_tri_gen = 0;
  // second stream and fork/join events for the overlapped general kernel
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // periodic finite check (lbm_set_finite_check): every `watch_every` steps
  // of time, the state is checked; the first failing time lands in pinned
  // host memory the check kernel writes through its device mapping
  int64_t watch_every = 0;
  int64_t *watch_host = nullptr;   // hipHostMalloc'd, -1 while no failure
  int64_t *watch_dev = nullptr;    // its device address
  int ntiles = 0, ntiles_int = 0;
  int gen_waves = 1;                             // tile width (x64) of the general list
  int64_t cells_int = 0, cells_gen = 0;          // cells each kernel's tile list covers
  std::vector<TileDev> h_tiles_int, h_tiles_gen; // host copies of the two lists
  // adjoint tile lists: interior tiles with no receiver in rows y0-1 .. y1,
  // and the rest (rebuilt after every retiling)
  DevBuf<TileDev> d_adj_int, d_adj_gen;
  int n_adj_int = 0, n_adj_gen = 0;
  // adjoint pairs on the two-step path: two-step blocks with no receiver
  // within three rows, the general tiles of the pair's second step (g2) and
  // of its first (g1: g2's plus the blocks' border strips, flagged)
  DevBuf<FusedTileDev> d_adj_ftiles;
  DevBuf<TileDev> d_adj_g2, d_adj_g1;
  int n_adj_f = 0, n_adj_g2 = 0, n_adj_g1 = 0, adj_fwaves = 2;
  int64_t cells_adj_int = 0, cells_adj_gen = 0, cells_adj_f = 0, cells_adj_g2 = 0;
  // dL/damp in a fixed order: the general adjoint kernel's per-workgroup
  // partial sums, and for a single step (its list) and for a pair (g1's
  // workgroups, then g2's, whose slots follow g1's) the workgroups that cover
  // each (grid, source) pair
  DevBuf<double> d_amp_part;
  struct AmpPlan {
    DevBuf<int32_t> tiles, off, pairs;
    int npairs = 0;
  } amp_single, amp_pair;
  DevBuf<double> d_misfit_part;   // the misfit's per-workgroup sums
  bool adj_tiles_ok = false;
  // graph of graph_chunk steps for each starting buffer parity
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gchunk = 0;
  // adjoint: checkpoints of a recorded forward run and the adjoint state
  struct Adj {
    bool begun = false;
    int32_t seg = 0;
    int64_t t_begin = 0, nsteps = 0, nseg = 0, taken = 0;
    size_t fbytes = 0, cbytes = 0;
    char *ckpt = nullptr, *rbuf[2] = {nullptr, nullptr}, *abuf[2] = {nullptr, nullptr};
    char *stash = nullptr;
    int64_t t_adj = 0, stash_seg = -1;
    // densities kept from the recorded forward for the steps res_t0 ..
    // res_t0 + res_steps - 1 (whole trailing segments): no recompute there
    char *res = nullptr;
    int64_t res_t0 = 0, res_steps = 0;
    int cur = 0;
    std::vector<AdjGridDev> io;
    bool io_dirty = true;
  } adj;
  DevBuf<AdjGridDev> d_adj_io;
};

namespace {

void drop_graphs(lbm_ctx *c) {
  for (int i = 0; i < 2; ++i)
    if (c->gexec[i]) {
      hipGraphExecDestroy(c->gexec[i]);
      c->gexec[i] = nullptr;
    }
  c->gchunk = 0;
}

// The step kernels reach a tile's rows through one buffer descriptor based
// two rows above the tile, with 32-bit byte offsets: row k of nine population
// runs from the base lies k * 9 * pitch * esize bytes in. The single-step
// kernels (descriptor range 2^31 - 1 bytes) reach at most kSingleReach rows
// beyond a tile's own (two above, the row pulled below and the prefetched
// rows); the two-step kernel (range up to 2^32 - 1) reaches kFusedReach rows
// beyond its block (four above, four below). A launch whose tiles could reach
// further would read zeros and drop stores, so it is refused. The tile height
// is taken as asked (not clipped to the grid), which errs on the safe side.
constexpr int64_t kSingleReach = 6;
constexpr int64_t kFusedReach = 8;
constexpr int64_t kFused3Reach = 12;   // the three-step kernel: six above, six below
constexpr int kMinTileRows = 2;   // the general kernel's sub-tiles

int64_t row_bytes(int32_t nx, int dtype) {
  return 9 * round_up(nx, kPitchAlign) * (dtype == LBM_F64 ? 8 : 4);
}

// Empty when every grid's tiles of `rows` rows (single steps) and blocks of
// `fuse_rows` rows (multi-step path, 0 = off; fuse_steps 2 or 3) stay inside the descriptors'
// ranges; else the reason.
std::string reach_error(const std::vector<lbm_grid> &grids, int dtype, int rows, int fuse_rows,
                        int fuse_steps = 2) {
  const int64_t freach = fuse_steps == 3 ? kFused3Reach : kFusedReach;
  for (size_t g = 0; g < grids.size(); ++g) {
    const int64_t rb = row_bytes(grids[g].nx, dtype);
    char buf[256];
    if ((std::max(rows, kMinTileRows) + kSingleReach) * rb > (int64_t)INT32_MAX) {
      snprintf(buf, sizeof buf,
               "grid %zu: %d-row tiles would address %lld bytes of populations from one "
               "descriptor (limit 2^31 - 1): use fewer rows",
               g, std::max(rows, kMinTileRows),
               (long long)((std::max(rows, kMinTileRows) + kSingleReach) * rb));
      return buf;
    }
    if (fuse_rows > 0 && (fuse_rows + freach) * rb > (int64_t)UINT32_MAX) {
      snprintf(buf, sizeof buf,
               "grid %zu: %d-row %s-step blocks would address %lld bytes of populations "
               "from one descriptor (limit 2^32 - 1): use fewer fuse_rows",
               g, fuse_rows, fuse_steps == 3 ? "three" : "two",
               (long long)((fuse_rows + freach) * rb));
      return buf;
    }
  }
  return std::string();
}

int validate_grid(const lbm_grid &g, const lbm_bc &b, const lbm_sponge *sp, int idx, int dtype) {
  char buf[256];
  if (g.nx < 3 || g.ny < 3) {
    snprintf(buf, sizeof buf, "grid %d: nx and ny must be >= 3 (got %d x %d)", idx, g.nx, g.ny);
    return fail(LBM_E_INVALID, buf);
  }
  if ((int64_t)g.nx * g.ny > (int64_t)1 << 31) {
    snprintf(buf, sizeof buf, "grid %d: more than 2^31 cells", idx);
    return fail(LBM_E_INVALID, buf);
  }
  if (!reach_error({g}, dtype, kMinTileRows, 0).empty()) {
    snprintf(buf, sizeof buf,
             "grid %d: too wide: %d rows of nine population runs of %d columns must stay "
             "below 2 GiB",
             idx, (int)(kMinTileRows + kSingleReach), g.nx);
    return fail(LBM_E_INVALID, buf);
  }
  for (int e = 0; e < 4; ++e)
    if (b.edge[e] < LBM_PERIODIC || b.edge[e] > LBM_FREE0) {
      snprintf(buf, sizeof buf, "grid %d: unknown boundary type on edge %d", idx, e);
      return fail(LBM_E_INVALID, buf);
    }
  if ((b.edge[LBM_EDGE_TOP] == LBM_PERIODIC) != (b.edge[LBM_EDGE_BOTTOM] == LBM_PERIODIC) ||
      (b.edge[LBM_EDGE_LEFT] == LBM_PERIODIC) != (b.edge[LBM_EDGE_RIGHT] == LBM_PERIODIC)) {
    snprintf(buf, sizeof buf, "grid %d: periodic edges must be paired", idx);
    return fail(LBM_E_INVALID, buf);
  }
  if (b.edge[LBM_EDGE_LEFT] == LBM_FREE || b.edge[LBM_EDGE_RIGHT] == LBM_FREE ||
      b.edge[LBM_EDGE_LEFT] == LBM_FREE0 || b.edge[LBM_EDGE_RIGHT] == LBM_FREE0) {
    snprintf(buf, sizeof buf, "grid %d: a free surface is supported on the top/bottom edges only", idx);
    return fail(LBM_E_INVALID, buf);
  }
  if (b.rigid_row != -1 && (b.rigid_row < 2 || b.rigid_row > g.ny - 2)) {
    snprintf(buf, sizeof buf, "grid %d: rigid_row must be -1 or in [2, ny-2]", idx);
    return fail(LBM_E_INVALID, buf);
  }
  if (sp) {
    for (int e = 0; e < 4; ++e) {
      const int ext = (e < 2) ? g.ny : g.nx;
      if (sp->thick[e] < 0 || sp->thick[e] > ext) {
        snprintf(buf, sizeof buf, "grid %d: sponge thickness on edge %d must be in [0, extent]", idx, e);
        return fail(LBM_E_INVALID, buf);
      }
      if (sp->thick[e] > 0 && !sp->profile[e]) {
        snprintf(buf, sizeof buf, "grid %d: missing sponge profile on edge %d", idx, e);
        return fail(LBM_E_INVALID, buf);
      }
      for (int k = 0; k < sp->thick[e]; ++k)
        if (!(sp->profile[e][k] >= 0.0) || !std::isfinite(sp->profile[e][k])) {
          snprintf(buf, sizeof buf, "grid %d: sponge profile values must be finite and >= 0", idx);
          return fail(LBM_E_INVALID, buf);
        }
    }
  }
  return LBM_OK;
}

// Blocks are handed to the 8 dies round-robin by block id, so block b takes
// the (b/8)-th tile of the die-contiguous chunk (b%8) of the list:
// neighbouring tiles, which share halo lines, run on the same die and hit the
// same L2. Padding blocks carry g = -1.
std::vector<TileDev> order_for_dies(const std::vector<TileDev> &logical) {
  const int64_t T = (int64_t)logical.size();
  const int64_t per = (T + kXcds - 1) / kXcds;
  std::vector<TileDev> phys((size_t)(per * kXcds), TileDev{-1, 0, 0, 0});
  for (int64_t b = 0; b < per * kXcds; ++b) {
    const int64_t j = b % kXcds, i = b / kXcds;
    const int64_t l = j * per + i;
    if (i < per && l < T) phys[(size_t)b] = logical[(size_t)l];
  }
  return phys;
}

// Distance from p to the nearest of the integer points lo..hi of an axis of
// n points, with the minimum image on a periodic axis.
double dist_to_range(double p, int lo, int hi, int n, bool periodic) {
  double best = 1e300;
  for (int k = periodic ? -1 : 0; k <= (periodic ? 1 : 0); ++k) {
    const double q = p + (double)k * n;
    const double d = q < lo ? lo - q : (q > hi ? q - hi : 0.0);
    best = std::min(best, d);
  }
  return best;
}

// Whether a tile can run in the interior kernel: every row it pulls (one
// above, its own, one below) has no horizontal wall link and no wrap, every
// column it touches (with the halo columns) has both x-neighbours inside the
// grid or the x edges are periodic, no source reaches its rows and no receiver
// sits in them.
bool tile_is_interior(const lbm_ctx *c, int g, int x0, int y0, int y1, int W) {
  const lbm_grid &G = c->grids[g];
  const lbm_bc &b = c->bc[g];
  const int nx = G.nx, ny = G.ny, rr = b.rigid_row;
  if (y0 - 1 < 1 || y1 > ny - 2) return false;
  if (rr > 0 && rr - 1 <= y1 && rr >= y0 - 1) return false;
  const bool px = b.edge[LBM_EDGE_LEFT] == LBM_PERIODIC;
  const bool py = b.edge[LBM_EDGE_TOP] == LBM_PERIODIC;
  const int x_last = std::min(x0 + W, nx) - 1;
  if (!px && (x0 - 2 < 0 || x_last + 2 > nx - 1)) return false;
  // the body force is zero on every cell of the tile: no cell within 9 sigma
  // of a source (minimum image on periodic axes)
  for (const lbm_source &q : c->sources[g]) {
    const double cut = 81.0 * q.sigma * q.sigma;
    const double dx = dist_to_range(q.x, x0, x_last, nx, px);
    const double dy = dist_to_range(q.y, y0, y1 - 1, ny, py);
    if (dx * dx + dy * dy <= cut) return false;
  }
  const std::vector<int32_t> &xy = c->recs[g].xy;
  for (size_t r = 1; r < xy.size(); r += 2)
    if (xy[r] >= y0 && xy[r] < y1) return false;
  return true;
}

// Tiles: columns [x0, x0 + 64*waves), rows [y0, y1), sorted into the interior
// list (when split) and the general list.
// A tile that is not interior as a whole is split into sub-tiles of at most
// kSubRows rows, each classified again: tall tiles serve the open interior
// (fewer halo rows per row) while the rows near walls, sources and receivers
// go to the general kernel in thin tiles.
constexpr int kSubRows = 2;

void build_tiles(const lbm_ctx *c, int waves, int rows, bool split, std::vector<TileDev> &interior,
                 std::vector<TileDev> &general) {
  std::vector<TileDev> li, lg;
  const int W = 64 * waves;
  for (int g = 0; g < c->nbatch; ++g) {
    const int nx = c->grids[g].nx, ny = c->grids[g].ny;
    for (int y0 = 0; y0 < ny; y0 += rows)
      for (int x0 = 0; x0 < nx; x0 += W) {
        const TileDev t{g, x0, y0, std::min(y0 + rows, ny)};
        if (!split) {
          lg.push_back(t);
        } else if (tile_is_interior(c, g, x0, t.y0, t.y1, W)) {
          li.push_back(t);
        } else {
          for (int ys = t.y0; ys < t.y1; ys += kSubRows) {
            const TileDev u{g, x0, ys, std::min(ys + kSubRows, t.y1)};
            if (tile_is_interior(c, g, x0, u.y0, u.y1, W)) {
              li.push_back(u);
            } else {
              // general tiles are one wavefront wide: the few rows they cover
              // then spread over many short workgroups
              for (int xs = x0; xs < std::min(x0 + W, nx); xs += 64) lg.push_back(TileDev{g, xs, u.y0, u.y1});
            }
          }
        }
      }
  }
  interior = order_for_dies(li);
  general = order_for_dies(lg);
}

// Default launch shape (measured on MI355X): on large grids 512-column
// interior tiles of 8 rows in FP32 and 4 rows in FP64 (taller tiles re-read
// fewer halo rows, shorter ones keep the rows in flight compact); narrower
// tiles where the grid would otherwise give too few workgroups to fill 256
// compute units.
// Launch shape by size (measured on MI355X): large contexts take the
// three-step path. Blocks of 192 columns (three output wavefronts beside the
// halo wavefront: one wavefront in four carries the halo instead of one in
// three), 96 rows high on grids of 4096 rows and more, 92 in FP64 (4096^2
// FP32: 182 GLUPS against 176 with 128-column blocks of 128 rows; 16384^2
// 203 against 191; FP64 4096^2 93.4 against 81.6) and 32 rows on shorter grids (the 512
// batched grids of side 256..2048: 170 against 162). The triples are
// launched directly: as fast as captured graphs or faster everywhere
// measured, and at 4096^2 FP32 the graphs' node scheduling leaves the
// general launches waiting for compute units the block kernel holds (141
// GLUPS in captured graphs against 182 direct). Small contexts run
// single steps in smaller tiles.
lbm_launch default_launch(const lbm_ctx *c) {
  int64_t cells = 0;
  int max_ny = 0;
  for (const auto &g : c->grids) {
    cells += (int64_t)g.nx * g.ny;
    max_ny = std::max(max_ny, g.ny);
  }
  lbm_launch l{8, c->dtype == LBM_F64 ? 4 : 8, 0, 1, 1, 0, 1, 0, 2};
  l.waves = 2;
  l.fuse_steps = 3;
  l.tri_waves = 3;
  l.fuse_rows = max_ny >= 4096 ? (c->dtype == LBM_F64 ? 92 : 96) : 32;
  l.graph_chunk = 0;
  if (cells < 2048 * 2048) {
    l.waves = 4;
    l.rows = 4;
    l.fuse_rows = 0;
    l.fuse_steps = 2;
    l.graph_chunk = 0;
  }
  if (cells < 256 * 2048) {
    l.waves = 1;
    l.rows = 4;
  }
  // very wide grids: shorter tiles and blocks so that no tile reaches past
  // its descriptor (the grids passed validation, so 2-row tiles fit)
  while (l.rows > 1 && !reach_error(c->grids, c->dtype, l.rows, 0).empty()) l.rows /= 2;
  while (l.fuse_rows >= 8 && !reach_error(c->grids, c->dtype, l.rows, l.fuse_rows, l.fuse_steps).empty())
    l.fuse_rows /= 2;
  if (l.fuse_rows > 0 && !reach_error(c->grids, c->dtype, l.rows, l.fuse_rows, l.fuse_steps).empty()) {
    l.fuse_steps = 2;   // the two-step blocks reach four rows fewer
    l.graph_chunk = 20;
  }
  if (l.fuse_rows > 0 && !reach_error(c->grids, c->dtype, l.rows, l.fuse_rows, l.fuse_steps).empty())
    l.fuse_rows = 0;
  return l;
}

template <typename real>
int commit_tables(lbm_ctx *c) {
  const hipStream_t s = c->stream;
  // sponge table (dtype): pairs (A, 1/(1 + A/2)) per profile entry
  std::vector<real> sponge;
  std::vector<std::array<int32_t, 4>> sp_off(c->nbatch);
  for (int g = 0; g < c->nbatch; ++g) {
    int64_t k = 0;
    for (int e = 0; e < 4; ++e) {
      sp_off[g][e] = (int32_t)sponge.size();
      for (int i = 0; i < c->sp_thick[g][e]; ++i) {
        const double A = c->sponge[g][k + i];
        sponge.push_back((real)A);
        sponge.push_back((real)(1.0 / (1.0 + 0.5 * A)));
      }
      k += c->sp_thick[g][e];
    }
  }
  if (sponge.empty()) sponge.push_back(real(0));
  std::vector<char> sbytes(sponge.size() * sizeof(real));
  memcpy(sbytes.data(), sponge.data(), sbytes.size());
  HIP_TRY(c->d_sponge.upload(sbytes, s));
  // sources
  std::vector<SourceDev> src;
  std::vector<int32_t> src_off(c->nbatch);
  for (int g = 0; g < c->nbatch; ++g) {
    src_off[g] = (int32_t)src.size();
    for (const auto &q : c->sources[g])
      src.push_back({q.x, q.y, q.sigma, q.dir_x, q.dir_y, q.amp, q.period, q.t0});
  }
  HIP_TRY(c->d_src.upload(src, s));
  // receivers: per grid a row table, a dense row map of receiver ids and a
  // chain for several receivers in one cell
  std::vector<int32_t> itab;
  std::vector<int64_t> rowtab_off(c->nbatch), rmap_off(c->nbatch), rnext_off(c->nbatch);
  for (int g = 0; g < c->nbatch; ++g) {
    const int nx = c->grids[g].nx, ny = c->grids[g].ny;
    const RecHost &R = c->recs[g];
    const int nrec = (int)R.xy.size() / 2;
    rowtab_off[g] = (int64_t)itab.size();
    std::vector<int32_t> rowslot(ny, -1);
    int nslots = 0;
    for (int r = 0; r < nrec; ++r) {
      const int y = R.xy[2 * r + 1];
      if (rowslot[y] < 0) rowslot[y] = nslots++;
    }
    itab.insert(itab.end(), rowslot.begin(), rowslot.end());
    rmap_off[g] = (int64_t)itab.size();
    std::vector<int32_t> rmap((size_t)nslots * nx, -1), rnext(nrec, -1);
    for (int r = nrec - 1; r >= 0; --r) {
      const int x = R.xy[2 * r], y = R.xy[2 * r + 1];
      int32_t &head = rmap[(size_t)rowslot[y] * nx + x];
      rnext[r] = head;
      head = r;
    }
    itab.insert(itab.end(), rmap.begin(), rmap.end());
    rnext_off[g] = (int64_t)itab.size();
    itab.insert(itab.end(), rnext.begin(), rnext.end());
  }
  HIP_TRY(c->d_itab.upload(itab, s));
  // 1/rho0 per receiver (dtype)
  std::vector<real> rtab;
  for (int g = 0; g < c->nbatch; ++g) {
    c->rscale_off[g] = (int64_t)rtab.size();
    for (double v : c->recs[g].scale) rtab.push_back((real)v);
  }
  if (rtab.empty()) rtab.push_back(real(0));
  std::vector<char> rbytes(rtab.size() * sizeof(real));
  memcpy(rbytes.data(), rtab.data(), rbytes.size());
  HIP_TRY(c->d_rtab.upload(rbytes, s));
  // grid descriptors
  std::vector<GridDev> gd(c->nbatch);
  for (int g = 0; g < c->nbatch; ++g) {
    GridDev &d = gd[g];
    memset(&d, 0, sizeof d);
    d.nx = c->grids[g].nx;
    d.ny = c->grids[g].ny;
    d.pitch = c->L.pitch[g];
    d.kmode = c->kmode[g];
    d.f_off = c->L.f_off[g];
    d.plane = c->L.plane[g];
    for (int e = 0; e < 4; ++e) d.bc[e] = c->bc[g].edge[e];
    d.rigid_row = c->bc[g].rigid_row;
    d.nsrc = (int32_t)c->sources[g].size();
    d.src_off = src_off[g];
    d.kscalar = c->kscalar[g];
    d.k_off = d.kmode == kKappaRows ? c->krow_off[g] : c->L.k_off[g];
    for (int e = 0; e < 4; ++e) {
      d.sp_thick[e] = c->sp_thick[g][e];
      d.sp_off[e] = sp_off[g][e];
    }
    const RecHost &R = c->recs[g];
    d.nrec = (int32_t)R.xy.size() / 2;
    d.rowtab_off = rowtab_off[g];
    d.rmap_off = rmap_off[g];
    d.rnext_off = rnext_off[g];
    d.rscale_off = c->rscale_off[g];
    d.trace = R.trace;
    d.trace_t0 = R.t0;
    d.trace_max = R.max_steps;
    d.comp_mask = R.comp_mask;
    d.ncomp = (R.comp_mask & 1) + ((R.comp_mask >> 1) & 1);
    d.c_off = c->L.k_off[g];
  }
  HIP_TRY(c->d_grids.upload(gd, s));
  c->tables_dirty = false;
  return LBM_OK;
}

int rebuild_tiles(lbm_ctx *c);

int commit(lbm_ctx *c) {
  if (!c->tables_dirty) return LBM_OK;
  drop_graphs(c);
  const int rc = c->dtype == LBM_F64 ? commit_tables<double>(c) : commit_tables<float>(c);
  if (rc) return rc;
  return rebuild_tiles(c);   // which tiles are interior depends on sources and receivers
}

// Two-step path (launch.fuse_rows > 0). Each grid is cut into row segments
// and column segments:
//  * rows: a row may be an own row of a two-step block when the block's reach
//    over two steps (step t+1 needs f*(t) 2 rows out, that needs rho(t) 3
//    rows out, pulled from 4 rows out) stays inside the grid without the
//    y-wrap and pulls across no wall link or rigid-row link, and no receiver
//    lies in it. Runs of such
//    rows are split into blocks of near-equal height <= fuse_rows (at least
//    2, the depth of the border the general kernel reads back); the other
//    rows form general segments;
//  * columns: blocks of 64 * fused_waves columns starting at a multiple of 64 (the
//    general kernel's tile width), the last one narrower (a multiple of 64,
//    or reaching nx on a periodic axis); without x-wrap the block's reach
//    (4 columns and one more for the pulls) must stay off the side walls.
// A block of an allowed row segment and an allowed column segment runs in
// the two-step kernel unless a source disk reaches into its reach; every
// other cell is advanced step by step by the general kernel in
// one-wavefront tiles of two rows. The general kernel's second step reads
// the intermediate state of the two rows, columns or corner cells of a
// two-step block next to general cells, so its first step also advances
// those (the border strips of build_fused_tiles).
// Two-step blocks are 64 * fused_waves columns wide: the launch's waves
// (2, 4 or 8; 1 counts as 2).
int fused_waves(const lbm_ctx *c) { return std::max(2, (int)c->launch.waves); }
// Three-step blocks: 128, 192 or 256 columns (the launch's tri_waves; 0
// follows waves, 8 counting as 4).
int tri_waves(const lbm_ctx *c) {
  return c->launch.tri_waves ? (int)c->launch.tri_waves : std::min(4, fused_waves(c));
}

struct Seg {
  int lo, hi;    // [lo, hi)
  bool ok;       // may hold two-step blocks
};

// rec_reach: a row with a receiver within rec_reach rows is no own row of a
// block (0 for the forward; the adjoint's blocks, whose receivers add to the
// adjoint state of every row their two steps form, take 3). steps: 2 or 3,
// the steps a block takes per pass; its reach is 2 x steps rows (the first
// step pulls rows y - 2 steps + 1 .. y + 2 steps - 1), and runs of allowed
// rows shorter than the border strips (2 x (steps - 1) rows) stay general.
std::vector<Seg> fused_row_segments(const lbm_ctx *c, int g, int rows, int rec_reach, int steps = 2) {
  const int R = 2 * steps, depth = 2 * (steps - 1);
  const int ny = c->grids[g].ny, rr = c->bc[g].rigid_row;
  std::vector<char> allowed((size_t)ny, 0);
  std::vector<char> has_rec((size_t)ny, 0);
  const std::vector<int32_t> &xy = c->recs[g].xy;
  for (size_t r = 1; r < xy.size(); r += 2)
    for (int y = std::max(0, xy[r] - rec_reach); y <= std::min(ny - 1, xy[r] + rec_reach); ++y)
      has_rec[(size_t)y] = 1;
  for (int y = 0; y < ny; ++y) {
    // the first step pulls rows y-R+1 .. y+R-1 (reading y-R .. y+R): inside
    // the grid without the wrap, and off rows 0 and ny-1 where walls cut links
    bool ok = y - R >= 0 && y + R <= ny - 1;
    // rigid-row links cross between rows rr-1 and rr: no pulled row may be
    // either of them
    if (rr > 0 && y - (R - 1) <= rr && y + (R - 1) >= rr - 1) ok = false;
    if (has_rec[(size_t)y]) ok = false;
    allowed[(size_t)y] = ok;
  }
  std::vector<Seg> segs;
  for (int y = 0; y < ny;) {
    int e = y;
    while (e < ny && allowed[(size_t)e] == allowed[(size_t)y]) ++e;
    const int len = e - y;
    if (!allowed[(size_t)y] || len < depth) {
      if (!segs.empty() && !segs.back().ok) segs.back().hi = e;
      else segs.push_back(Seg{y, e, false});
    } else {
      const int nb = (len + rows - 1) / rows;
      for (int k = 0; k < nb; ++k)
        segs.push_back(Seg{y + (int)((int64_t)len * k / nb), y + (int)((int64_t)len * (k + 1) / nb), true});
    }
    y = e;
  }
  return segs;
}

// The kernels' halo columns: 4 each side for two steps, 5 for three; no halo
// column may sit on a side wall's column.
int fused_halo(int steps) { return steps == 3 ? 5 : 4; }

std::vector<Seg> fused_col_segments(const lbm_ctx *c, int g, int waves, int steps = 2) {
  const int nx = c->grids[g].nx, bw = 64 * waves, h = fused_halo(steps);
  const bool px = c->bc[g].edge[LBM_EDGE_LEFT] == LBM_PERIODIC;
  // allowed columns [a, b): with x-wrap all; without, x-h-1 >= 0 and
  // x+h <= nx-2 for every own column x
  int a = px ? 0 : 64;                  // first multiple of 64 >= h + 1
  const int b = px ? nx : nx - h - 1;
  std::vector<Seg> segs;
  if (a > 0) segs.push_back(Seg{0, std::min(a, nx), false});
  for (int x = a; x < nx;) {
    int w = std::min(bw, b - x);
    if (!(px && x + w == nx)) w = w / 64 * 64;   // keep general tiles 64-aligned
    if (w < 64) {
      segs.push_back(Seg{x, nx, false});
      break;
    }
    segs.push_back(Seg{x, x + w, true});
    x += w;
  }
  return segs;
}

// A source disk reaching any cell the block's kernel computes (its halo
// columns and the rows of its first stage: h and 2 x steps - 1 beyond the
// block).
bool source_reaches(const lbm_ctx *c, int g, const Seg &cs, const Seg &rs, int steps = 2) {
  const int h = fused_halo(steps), v = 2 * steps - 1;
  const int nx = c->grids[g].nx, ny = c->grids[g].ny;
  const bool px = c->bc[g].edge[LBM_EDGE_LEFT] == LBM_PERIODIC;
  const bool py = c->bc[g].edge[LBM_EDGE_TOP] == LBM_PERIODIC;
  for (const lbm_source &q : c->sources[g]) {
    const double cut = 81.0 * q.sigma * q.sigma;
    const double dx = dist_to_range(q.x, cs.lo - h, cs.hi + h - 1, nx, px);
    const double dy = dist_to_range(q.y, rs.lo - v, rs.hi + v - 1, ny, py);
    if (dx * dx + dy * dy <= cut) return true;
  }
  return false;
}

// The general tiles of each step of a pass of `steps` steps. gens[steps-1]
// (the last step's) holds the general tiles; gens[k] for an earlier step adds,
// for every block next to general cells, the 2 x (steps - 1 - k) rows,
// columns or corner cells on that side (border strips), so that each general
// launch leaves the state of every cell the next one reads in its output and
// the general launches need nothing from the blocks' pass. For a pair:
// gens[0] with two-deep strips (the first step's list), gens[1] the second's.
// The adjoint builds its own lists the same way (blocks of `waves` x 64
// columns, no receiver within rec_reach rows of an own row) and flags the
// strips with strip_bit in their grid index. The general kernels reach two
// rows and columns beyond a cell in both directions, the adjoint's as the
// forward's, so the same strips serve both.
void build_multi_tiles(const lbm_ctx *c, int rows, int waves, int rec_reach, int32_t strip_bit,
                       int steps, std::vector<FusedTileDev> &fused,
                       std::vector<std::vector<TileDev>> &gens, int64_t &fused_cells) {
  std::vector<FusedTileDev> lf;
  std::vector<TileDev> lg;
  std::vector<std::vector<TileDev>> lh((size_t)steps);
  fused_cells = 0;
  for (int g = 0; g < c->nbatch; ++g) {
    const std::vector<Seg> R = fused_row_segments(c, g, rows, rec_reach, steps),
                           C = fused_col_segments(c, g, waves, steps);
    const int nr = (int)R.size(), nc = (int)C.size();
    const bool px = c->bc[g].edge[LBM_EDGE_LEFT] == LBM_PERIODIC;
    const bool py = c->bc[g].edge[LBM_EDGE_TOP] == LBM_PERIODIC;
    std::vector<char> isf((size_t)nr * nc, 0);
    for (int j = 0; j < nr; ++j)
      for (int i = 0; i < nc; ++i)
        isf[(size_t)j * nc + i] = R[j].ok && C[i].ok && !source_reaches(c, g, C[i], R[j], steps);
    auto fused_at = [&](int i, int j) -> int {   // 1 block, 0 general, -1 outside the grid
      if (i < 0 || i >= nc) { if (!px) return -1; i = (i + nc) % nc; }
      if (j < 0 || j >= nr) { if (!py) return -1; j = (j + nr) % nr; }
      return isf[(size_t)j * nc + i];
    };
    for (int j = 0; j < nr; ++j)
      for (int i = 0; i < nc; ++i) {
        const Seg &rs = R[j], &cs = C[i];
        if (isf[(size_t)j * nc + i]) {
          lf.push_back(FusedTileDev{g, cs.lo, cs.hi, rs.lo, rs.hi});
          fused_cells += (int64_t)(cs.hi - cs.lo) * (rs.hi - rs.lo);
          // border strips d deep: d rows along a general neighbour above or
          // below, d columns (one 64-column tile) along one left or right,
          // the d x d corner (one 64-column tile of d rows) toward a general
          // diagonal neighbour; rows in tiles of at most kSubRows
          for (int k = 0; k + 1 < steps; ++k) {
            const int d = 2 * (steps - 1 - k);
            std::set<std::tuple<int, int, int>> strips;
            const int xl = cs.lo, xr = std::max(cs.lo, cs.hi - 64);
            for (int dj = -1; dj <= 1; ++dj)
              for (int di = -1; di <= 1; ++di) {
                if ((di | dj) == 0 || fused_at(i + di, j + dj) != 0) continue;
                const int ya = dj < 0 ? rs.lo : rs.hi - d;   // the d rows on that side
                for (int ys = dj == 0 ? rs.lo : ya; ys < (dj == 0 ? rs.hi : ya + d); ys += kSubRows) {
                  const int ye = std::min(ys + kSubRows, dj == 0 ? rs.hi : ya + d);
                  if (di == 0) {
                    for (int xs = cs.lo; xs < cs.hi; xs += 64) strips.emplace(xs, ys, ye);
                  } else {
                    strips.emplace(di < 0 ? xl : xr, ys, ye);
                  }
                }
              }
            for (const auto &st : strips)
              lh[(size_t)k].push_back(TileDev{g | strip_bit, std::get<0>(st), std::get<1>(st), std::get<2>(st)});
          }
        } else {
          for (int ys = rs.lo; ys < rs.hi; ys += kSubRows)
            for (int xs = cs.lo; xs < cs.hi; xs += 64)
              lg.push_back(TileDev{g, xs, ys, std::min(ys + kSubRows, rs.hi)});
        }
      }
  }
  // die ordering as for the single-step lists
  const int64_t T = (int64_t)lf.size(), per = (T + kXcds - 1) / kXcds;
  fused.assign((size_t)(per * kXcds), FusedTileDev{-1, 0, 0, 0, 0});
  for (int64_t b = 0; b < per * kXcds; ++b) {
    const int64_t jx = b % kXcds, ix = b / kXcds, l = jx * per + ix;
    if (ix < per && l < T) fused[(size_t)b] = lf[(size_t)l];
  }
  gens.assign((size_t)steps, std::vector<TileDev>());
  for (int k = 0; k < steps; ++k) {
    std::vector<TileDev> l = lg;
    l.insert(l.end(), lh[(size_t)k].begin(), lh[(size_t)k].end());
    gens[(size_t)k] = order_for_dies(l);
  }
}

// The two-step path's lists: general (the pair's second step) and general1
// (its first, with the two-deep border strips).
void build_fused_tiles(const lbm_ctx *c, int rows, int waves, int rec_reach, int32_t strip_bit,
                       std::vector<FusedTileDev> &fused, std::vector<TileDev> &general,
                       std::vector<TileDev> &general1, int64_t &fused_cells) {
  std::vector<std::vector<TileDev>> gens;
  build_multi_tiles(c, rows, waves, rec_reach, strip_bit, 2, fused, gens, fused_cells);
  general1 = gens[0];
  general = gens[1];
}

constexpr int kFilterRows = 32;

// Timed steps per autotuning candidate when the caller passes 0 and nothing is
// cached for the context.
constexpr int kDefaultTuneSteps = 10;

int rebuild_tiles(lbm_ctx *c) {
  std::vector<TileDev> ti, tg;
  build_tiles(c, c->launch.waves, c->launch.rows, c->launch.split != 0, ti, tg);
  c->ntiles_int = (int)ti.size();
  c->ntiles = (int)tg.size();
  c->gen_waves = c->launch.split ? 1 : c->launch.waves;
  auto cover = [&](const std::vector<TileDev> &v, int W) {
    int64_t n = 0;
    for (const auto &t : v)
      if (t.g >= 0)   // skip the padding entries of the die ordering
        n += (int64_t)std::min(W, c->grids[t.g].nx - t.x0) * (t.y1 - t.y0);
    return n;
  };
  c->cells_int = cover(ti, 64 * c->launch.waves);
  c->cells_gen = cover(tg, 64 * c->gen_waves);
  c->h_tiles_int = ti;
  c->h_tiles_gen = tg;
  c->adj_tiles_ok = false;
  c->nftiles = c->ngtiles2 = c->ngtiles1 = 0;
  c->cells_fused = c->cells_gen2 = 0;
  if (c->launch.fuse_rows > 0) {
    std::vector<FusedTileDev> tf;
    std::vector<TileDev> tg2, tg1;
    build_fused_tiles(c, c->launch.fuse_rows, fused_waves(c), 0, 0, tf, tg2, tg1, c->cells_fused);
    c->nftiles = (int)tf.size();
    c->ngtiles2 = (int)tg2.size();
    c->ngtiles1 = (int)tg1.size();
    c->cells_gen2 = cover(tg2, 64);
    HIP_TRY(c->d_ftiles.upload(tf, c->stream));
    HIP_TRY(c->d_gtiles2.upload(tg2, c->stream));
    HIP_TRY(c->d_gtiles1.upload(tg1, c->stream));
  }
  c->nttiles = c->ntgen[0] = c->ntgen[1] = c->ntgen[2] = 0;
  c->cells_tri = c->cells_tri_gen = 0;
  if (c->launch.fuse_rows > 0 && c->launch.fuse_steps == 3) {
    if (c->d_fmid2.reserve((size_t)round_up(c->L.f_elems * (int64_t)c->L.esize, 256)) != hipSuccess) {
      hipGetLastError();
      if (c->launch_set)
        return fail(LBM_E_NOMEM, "no device memory for the three-step path's second intermediate buffer");
      // the default launch falls back to pairs
      c->launch.fuse_steps = 2;
      c->launch.graph_chunk += c->launch.graph_chunk % 2;
      return rebuild_tiles(c);
    }
    std::vector<FusedTileDev> tf;
    std::vector<std::vector<TileDev>> gens;
    build_multi_tiles(c, c->launch.fuse_rows, tri_waves(c), 0, 0, 3, tf, gens, c->cells_tri);
    c->nttiles = (int)tf.size();
    c->cells_tri_gen = cover(gens[2], 64);
    HIP_TRY(c->d_ttiles.upload(tf, c->stream));
    for (int k = 0; k < 3; ++k) {
      c->ntgen[k] = (int)gens[(size_t)k].size();
      HIP_TRY(c->d_tgen[k].upload(gens[(size_t)k], c->stream));
    }
  } else {
    c->d_fmid2.release();
  }
  HIP_TRY(c->d_tiles_int.upload(ti, c->stream));
  HIP_TRY(c->d_tiles.upload(tg, c->stream));
  if (c->nfilt_tiles == 0) {   // independent of the launch shape: built once
    std::vector<TileDev> tf;
    for (int g = 0; g < c->nbatch; ++g)
      for (int y0 = 0; y0 < c->grids[g].ny; y0 += kFilterRows)
        for (int x0 = 0; x0 < c->grids[g].nx; x0 += 256)
          tf.push_back(TileDev{g, x0, y0, std::min(y0 + kFilterRows, c->grids[g].ny)});
    tf = order_for_dies(tf);
    c->nfilt_tiles = (int)tf.size();
    HIP_TRY(c->d_filt_tiles.upload(tf, c->stream));
  }
  drop_graphs(c);
  return LBM_OK;
}

// The two-column interior kernel needs an even nx in every grid and at least
// two waves of tile width.
int use_pair(const lbm_ctx *c) {
  if (!c->launch.pair || c->launch.waves < 2) return 0;
  for (const auto &g : c->grids)
    if (g.nx % 2) return 0;
  return 1;
}

// One step: the interior tiles and the general tiles (any order: both read
// the state of step t-1 and write disjoint cells of step t).
hipError_t ensure_side_stream(lbm_ctx *c) {
  if (c->side) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  return e;
}

// The interior kernel and the general kernel of one step (forward, recompute
// or adjoint) write disjoint tiles of their output and only read their input,
// so with overlap on the general one runs on the library's second stream,
// forked from and joined back to s (under graph capture the fork and join
// become graph edges); otherwise the interior kernel runs first.
template <typename Gen, typename Int>
hipError_t launch_pair(lbm_ctx *c, hipStream_t s, bool has_int, bool has_gen, Gen general,
                       Int interior) {
  hipError_t e = hipSuccess;
  if (c->launch.overlap && has_int && has_gen) {
    e = ensure_side_stream(c);
    if (e == hipSuccess) e = hipEventRecord(c->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_fork, 0);
    if (e == hipSuccess) e = general(c->side);
    if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->side);
    if (e == hipSuccess) e = interior(s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_join, 0);
    return e;
  }
  if (has_int) e = interior(s);
  if (e == hipSuccess && has_gen) e = general(s);
  return e;
}

int use_fused(const lbm_ctx *c) { return c->launch.fuse_rows > 0 && c->nftiles > 0; }

// The three launches of a pair of steps (t and t+1) on the two-step path: the
// general kernel advances its tiles and the two-step blocks' border strips
// to f*(t) in the intermediate buffer (g1), then its tiles from there to
// f*(t+1) (g2); the fused kernel takes its tiles straight to f*(t+1) (f2).
// g1 and g2 need nothing from f2, and f2 nothing from them: they write
// disjoint cells of the output (the strips' f*(t) goes to the intermediate
// buffer only, which f2 does not use).
template <typename real>
void pair_args(lbm_ctx *c, const StepArgs<real> &a, StepArgs<real> &g1, StepArgs<real> &f2,
               StepArgs<real> &g2) {
  g1 = f2 = g2 = a;
  g1.fout = reinterpret_cast<real *>(c->fmid);
  g1.tiles = c->d_gtiles1.p;
  g1.fmid = reinterpret_cast<real *>(c->fmid);
  f2.ftiles = c->d_ftiles.p;
  f2.fmid = reinterpret_cast<real *>(c->fmid);
  f2.f_elems = c->L.f_elems;
  g2.fin = reinterpret_cast<const real *>(c->fmid);
  g2.tiles = c->d_gtiles2.p;
  g2.fmid = reinterpret_cast<real *>(c->fmid);
  g2.t = a.t + 1;
}

// Two steps on the two-step path: g1 then g2 on the library's second stream,
// beside f2 on the context's stream (or one after the other without overlap).
// With stash planes, the launches also write rho(t) and rho(t+1) of every
// cell to rho_t and rho_t1 (g1 writes the strips' rho(t) as f2 does, the same
// values) and skip the receivers, unless `receivers` (a recorded forward
// step that keeps its densities).
template <typename real>
hipError_t launch_two_steps(lbm_ctx *c, StepArgs<real> a, hipStream_t s, real *rho_t = nullptr,
                            real *rho_t1 = nullptr, bool receivers = false) {
  StepArgs<real> g1, f2, g2;
  pair_args<real>(c, a, g1, f2, g2);
  const int mode = rho_t && !receivers ? kModeStash : kModeStep;
  g1.rho_out = rho_t;
  f2.rho_out = rho_t;
  f2.rho_out2 = rho_t1;
  g2.rho_out = rho_t1;
  const int pf = c->launch.prefetch;
  return launch_pair(
      c, s, c->nftiles > 0, c->ngtiles2 > 0,
      [&](hipStream_t q) {
        hipError_t e = launch_step<real>(g1, 1, pf, c->ngtiles1, mode, q);
        if (e == hipSuccess) e = launch_step<real>(g2, 1, pf, c->ngtiles2, mode, q);
        return e;
      },
      [&](hipStream_t q) { return launch_fused2<real>(f2, fused_waves(c), c->nftiles, q); });
}

int use_tri(const lbm_ctx *c) {
  return c->launch.fuse_rows > 0 && c->launch.fuse_steps == 3 && c->nttiles > 0;
}

// The launches of a triple of steps (t, t+1, t+2) on the three-step path.
// The three-step kernel (f3) takes its blocks from f*(t-1) in fin straight to
// f*(t+2) in fout. Beside it, on the second stream, the general kernel
// advances its tiles and the blocks' four-deep border strips to f*(t) in the
// intermediate buffer (g1), its tiles and the two-deep strips from there to
// f*(t+1) in the second intermediate buffer (g2), and its tiles from there
// to f*(t+2) in fout (g3). The general launches need nothing from f3 and f3
// nothing from them; f3 and g3 write disjoint cells of fout.
template <typename real>
void tri_args(lbm_ctx *c, const StepArgs<real> &a, StepArgs<real> &g1, StepArgs<real> &f3,
              StepArgs<real> &g2, StepArgs<real> &g3) {
  g1 = f3 = g2 = g3 = a;
  g1.fout = reinterpret_cast<real *>(c->fmid);
  g1.tiles = c->d_tgen[0].p;
  g1.tri_step = 1;
  f3.ftiles = c->d_ttiles.p;
  f3.f_elems = c->L.f_elems;
  g2.fin = reinterpret_cast<const real *>(c->fmid);
  g2.fout = reinterpret_cast<real *>(c->d_fmid2.p);
  g2.tiles = c->d_tgen[1].p;
  g2.t = a.t + 1;
  g2.tri_step = 2;
  g3.fin = reinterpret_cast<const real *>(c->d_fmid2.p);
  g3.tiles = c->d_tgen[2].p;
  g3.t = a.t + 2;
  g3.tri_step = 3;
}

template <typename real>
hipError_t launch_three_steps(lbm_ctx *c, StepArgs<real> a, hipStream_t s) {
  StepArgs<real> g1, f3, g2, g3;
  tri_args<real>(c, a, g1, f3, g2, g3);
  const int pf = c->launch.prefetch;
  return launch_pair(
      c, s, true, c->ntgen[0] + c->ntgen[1] + c->ntgen[2] > 0,
      [&](hipStream_t q) {
        hipError_t e = launch_step<real>(g1, 1, pf, c->ntgen[0], kModeStep, q);
        if (e == hipSuccess) e = launch_step<real>(g2, 1, pf, c->ntgen[1], kModeStep, q);
        if (e == hipSuccess) e = launch_step<real>(g3, 1, pf, c->ntgen[2], kModeStep, q);
        return e;
      },
      [&](hipStream_t q) { return launch_fused3<real>(f3, tri_waves(c), c->nttiles, q); });
}

template <typename real>
hipError_t launch_one_step(lbm_ctx *c, StepArgs<real> a, hipStream_t s) {
  StepArgs<real> ai = a;
  ai.tiles = c->d_tiles_int.p;
  a.tiles = c->d_tiles.p;
  return launch_pair(
      c, s, c->ntiles_int > 0, c->ntiles > 0,
      [&](hipStream_t q) {
        return launch_step<real>(a, c->gen_waves, c->launch.prefetch, c->ntiles, kModeStep, q);
      },
      [&](hipStream_t q) {
        return launch_interior<real>(ai, c->launch.waves, use_pair(c), c->ntiles_int, q);
      });
}

template <typename real>
StepArgs<real> make_args(lbm_ctx *c, int src_buf) {
  StepArgs<real> a;
  memset(&a, 0, sizeof a);
  a.fin = reinterpret_cast<const real *>(c->fbuf[src_buf]);
  a.fout = reinterpret_cast<real *>(c->fbuf[src_buf ^ 1]);
  a.grids = c->d_grids.p;
  a.tiles = c->d_tiles.p;
  a.kappa_rows = reinterpret_cast<const real *>(c->d_krows.p);
  a.kappa_cells = reinterpret_cast<const real *>(c->kcells);
  a.sponge = reinterpret_cast<const real *>(c->d_sponge.p);
  a.sources = c->d_src.p;
  a.itab = c->d_itab.p;
  a.rtab = reinterpret_cast<const real *>(c->d_rtab.p);
  a.t = c->t;
  a.t_dev = nullptr;
  a.omega = (real)(1.0 / c->tau);
  a.cforce = (real)(1.0 - 0.5 / c->tau);
  a.mom = nullptr;
  a.mom_grid = -1;
  return a;
}

template <typename real>
int step_direct(lbm_ctx *c, int64_t n) {
  if (use_tri(c)) {
    for (; n >= 3; n -= 3) {
      HIP_TRY(launch_three_steps<real>(c, make_args<real>(c, c->cur), c->stream));
      c->cur ^= 1;
      c->t += 3;
    }
  }
  if (use_fused(c)) {
    for (; n >= 2; n -= 2) {
      HIP_TRY(launch_two_steps<real>(c, make_args<real>(c, c->cur), c->stream));
      c->cur ^= 1;
      c->t += 2;
    }
  }
  for (int64_t k = 0; k < n; ++k) {
    HIP_TRY(launch_one_step<real>(c, make_args<real>(c, c->cur), c->stream));
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

// Direct launches with an event pair around every kernel launch; the mean
// duration of each kernel's launches goes to out.
template <typename real>
int step_timed(lbm_ctx *c, int64_t n, lbm_kernel_times *out) {
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  double sum[4] = {0.0, 0.0, 0.0, 0.0};   // interior, general, multi-step, leftover pairs
  int64_t cnt[4] = {0, 0, 0, 0};
  // One launch between an event pair on the context's stream.
  auto timed = [&](int kind, auto &&launch) {
    if (e == hipSuccess) e = hipEventRecord(ev[0], c->stream);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e == hipSuccess) { sum[kind] += ms; cnt[kind] += 1; }
  };
  int64_t k = 0;
  const int pf = c->launch.prefetch;
  const bool tri = use_tri(c) != 0;
  if (tri) {
    for (; k + 3 <= n && e == hipSuccess; k += 3) {
      const StepArgs<real> a = make_args<real>(c, c->cur);
      StepArgs<real> g1, f3, g2, g3;
      tri_args<real>(c, a, g1, f3, g2, g3);
      if (c->ntgen[0] > 0)
        timed(1, [&] { return launch_step<real>(g1, 1, pf, c->ntgen[0], kModeStep, c->stream); });
      timed(2, [&] { return launch_fused3<real>(f3, tri_waves(c), c->nttiles, c->stream); });
      if (c->ntgen[1] > 0)
        timed(1, [&] { return launch_step<real>(g2, 1, pf, c->ntgen[1], kModeStep, c->stream); });
      if (c->ntgen[2] > 0)
        timed(1, [&] { return launch_step<real>(g3, 1, pf, c->ntgen[2], kModeStep, c->stream); });
      if (e == hipSuccess) {
        c->cur ^= 1;
        c->t += 3;
      }
    }
  }
  if (use_fused(c)) {
    for (; k + 2 <= n && e == hipSuccess; k += 2) {
      const StepArgs<real> a = make_args<real>(c, c->cur);
      StepArgs<real> g1, f2, g2;
      pair_args<real>(c, a, g1, f2, g2);
      if (c->ngtiles2 > 0) {
        timed(1, [&] { return launch_step<real>(g1, 1, pf, c->ngtiles1, kModeStep, c->stream); });
        timed(1, [&] { return launch_step<real>(g2, 1, pf, c->ngtiles2, kModeStep, c->stream); });
      }
      // on the three-step path a leftover pair's two-step launch is timed
      // apart (not reported)
      timed(tri ? 3 : 2, [&] { return launch_fused2<real>(f2, fused_waves(c), c->nftiles, c->stream); });
      if (e == hipSuccess) {
        c->cur ^= 1;
        c->t += 2;
      }
    }
  }
  for (; k < n && e == hipSuccess; ++k) {
    StepArgs<real> a = make_args<real>(c, c->cur);
    if (c->ntiles_int > 0) {
      StepArgs<real> ai = a;
      ai.tiles = c->d_tiles_int.p;
      timed(0, [&] {
        return launch_interior<real>(ai, c->launch.waves, use_pair(c), c->ntiles_int, c->stream);
      });
    }
    a.tiles = c->d_tiles.p;
    if (c->ntiles > 0)
      timed(1, [&] {
        return launch_step<real>(a, c->gen_waves, pf, c->ntiles, kModeStep, c->stream);
      });
    if (e == hipSuccess) {
      c->cur ^= 1;
      c->t += 1;
    }
  }
  for (int i = 0; i < 2; ++i)
    if (ev[i]) hipEventDestroy(ev[i]);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, hipGetErrorString(e));
  out->steps = n;
  out->interior_ms = cnt[0] ? sum[0] / (double)cnt[0] : 0.0;
  out->general_ms = cnt[1] ? sum[1] / (double)cnt[1] : 0.0;
  out->fused_ms = cnt[2] ? sum[2] / (double)cnt[2] : 0.0;
  out->interior_cells = c->cells_int;
  out->general_cells = tri ? c->cells_tri_gen : use_fused(c) ? c->cells_gen2 : c->cells_gen;
  out->fused_cells = tri ? c->cells_tri : use_fused(c) ? c->cells_fused : 0;
  out->fused_steps = tri ? 3 : use_fused(c) ? 2 : 0;
  return LBM_OK;
}

// Capture graph_chunk steps reading the time from the device counter,
// followed by a node that advances the counter. On the two-step path the
// chunk is graph_chunk / 2 pairs, each the three launches of a pair with its
// fork and join as graph edges; on the three-step path graph_chunk / 3
// triples of four launches.
template <typename real>
int build_graphs(lbm_ctx *c, int chunk) {
  drop_graphs(c);
  for (int parity = 0; parity < 2; ++parity) {
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      hipStreamDestroy(cs);
      return fail(LBM_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    int buf = parity;
    const int per = use_tri(c) ? 3 : use_fused(c) ? 2 : 1;
    for (int k = 0; k < chunk; k += per) {
      StepArgs<real> a = make_args<real>(c, buf);
      a.t = k;
      a.t_dev = c->d_time.p;
      if (per == 3) launch_three_steps<real>(c, a, cs);
      else if (per == 2) launch_two_steps<real>(c, a, cs);
      else launch_one_step<real>(c, a, cs);
      buf ^= 1;
    }
    launch_add_time(c->d_time.p, chunk, cs);
    e = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) {
      hipStreamDestroy(cs);
      return fail(LBM_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&c->gexec[parity], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    hipStreamDestroy(cs);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  c->gchunk = chunk;
  return LBM_OK;
}

// Enqueue the finite check of the current state (time c->t).
template <typename real>
int watch_state(lbm_ctx *c) {
  HIP_TRY(launch_finite_watch<real>(reinterpret_cast<const real *>(c->fbuf[c->cur]), c->L.f_elems,
                                    c->t, c->watch_dev, c->stream));
  return LBM_OK;
}

template <typename real>
int step_run(lbm_ctx *c, int64_t n);

// With the finite check on, steps run in segments that end on multiples of
// watch_every, each followed by the check of the state reached.
template <typename real>
int step_impl(lbm_ctx *c, int64_t n) {
  if (c->watch_every <= 0) return step_run<real>(c, n);
  while (n > 0) {
    const int64_t to_next = c->watch_every - (c->t % c->watch_every);
    const int64_t m = std::min(n, to_next);
    int rc = step_run<real>(c, m);
    if (rc) return rc;
    n -= m;
    if (c->t % c->watch_every == 0) {
      rc = watch_state<real>(c);
      if (rc) return rc;
    }
  }
  return LBM_OK;
}

template <typename real>
int step_chunks(lbm_ctx *c, int64_t n);

// Recorded forward steps whose densities the adjoint keeps: direct launches
// that also write rho(t) of every cell to the step's plane, receivers included.
template <typename real>
int step_keep_densities(lbm_ctx *c, int64_t n) {
  auto &A = c->adj;
  auto plane = [&](int64_t t) {
    return reinterpret_cast<real *>(A.res + (size_t)(t - A.res_t0) * A.cbytes);
  };
  if (use_fused(c)) {
    for (; n >= 2; n -= 2) {
      HIP_TRY(launch_two_steps<real>(c, make_args<real>(c, c->cur), c->stream, plane(c->t),
                                     plane(c->t + 1), true));
      c->cur ^= 1;
      c->t += 2;
    }
  }
  for (; n > 0; --n) {
    StepArgs<real> a = make_args<real>(c, c->cur);
    a.rho_out = plane(c->t);
    HIP_TRY(launch_one_step<real>(c, a, c->stream));
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

template <typename real>
int step_run(lbm_ctx *c, int64_t n) {
  int rc = commit(c);
  if (rc) return rc;
  // the steps of an open recording whose densities are kept run apart
  auto &A = c->adj;
  if (A.begun && A.res_steps > 0) {
    const int64_t r0 = A.res_t0, r1 = A.res_t0 + A.res_steps;
    if (c->t < r1 && c->t + n > r0) {
      if (c->t < r0) {
        const int64_t m = r0 - c->t;
        rc = step_chunks<real>(c, m);
        if (rc) return rc;
        n -= m;
      }
      const int64_t m = std::min(n, r1 - c->t);
      rc = step_keep_densities<real>(c, m);
      if (rc) return rc;
      n -= m;
    }
  }
  return step_chunks<real>(c, n);
}

template <typename real>
int step_chunks(lbm_ctx *c, int64_t n) {
  int rc = LBM_OK;
  // graph_chunk > 0: whole chunks run as captured graphs, one per buffer
  // parity. A single step swaps the ping-pong buffers once, a pair or a
  // triple of steps on the multi-step paths once: after an even chunk of
  // single steps the state is back in its buffer, after a chunk of an odd
  // number of pairs or triples in the other one.
  // A chunk must be a whole number of the path's units (a context on the
  // three-step path whose grids hold only two-step blocks runs pairs, and a
  // chunk of an odd multiple of 3 steps is then not whole pairs): otherwise
  // the steps run launched directly.
  const int chunk = c->launch.graph_chunk;
  const int unit = use_tri(c) ? 3 : use_fused(c) ? 2 : 1;
  if (chunk > 0 && n >= chunk && chunk % unit == 0) {
    if (c->gchunk != chunk) {
      rc = build_graphs<real>(c, chunk);
      if (rc) return rc;
    }
    const int swaps = chunk / unit;
    HIP_TRY(launch_set_time(c->d_time.p, c->t, c->stream));
    while (n >= chunk) {
      HIP_TRY(hipGraphLaunch(c->gexec[c->cur], c->stream));
      c->t += chunk;
      c->cur ^= swaps & 1;
      n -= chunk;
    }
  }
  return step_direct<real>(c, n);
}

// Poisson ratio from kappa = b^2 (mu - lambda)/mu: lambda/mu = 1 - 3 kappa.
double nu_of_kappa(double kappa) {
  const double r = 1.0 - 3.0 * kappa;
  return r / (2.0 * (1.0 + r));
}

// Largest von Neumann amplification factor over the media's Poisson ratios
// (at most 16 of them: the extremes and evenly spaced ones between) at the
// context's tau, on a 33 x 33 grid of wavenumbers in [0, pi]^2.
double context_vn_growth(const lbm_ctx *c) {
  std::vector<double> v = c->nu_seen;
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end(), [](double a, double b) { return std::fabs(a - b) < 1e-9; }),
          v.end());
  if (v.size() > 16) {
    std::vector<double> w;
    for (int q = 0; q < 16; ++q) w.push_back(v[(size_t)((v.size() - 1) * q / 15)]);
    v = w;
  }
  double g = 0.0;
  for (double nu : v) g = std::max(g, vn_growth(nu, c->tau, 33));
  return g;
}

template <typename real>
int init_fields(lbm_ctx *c, const void *lam, const void *mu, const void *rho) {
  const hipStream_t s = c->stream;
  int *d_bad = nullptr, *d_rows = nullptr;
  int64_t maxny = 0;
  for (auto &g : c->grids) maxny = std::max<int64_t>(maxny, g.ny);
  HIP_TRY(hipMalloc((void **)&d_bad, sizeof(int)));
  HIP_TRY(hipMalloc((void **)&d_rows, maxny * sizeof(int)));
  std::vector<real> krows_all;
  int64_t cell_off = 0;
  int rc = LBM_OK;
  for (int g = 0; g < c->nbatch && rc == LBM_OK; ++g) {
    const int nx = c->grids[g].nx, ny = c->grids[g].ny;
    const real *l = reinterpret_cast<const real *>(lam) + cell_off;
    const real *m = reinterpret_cast<const real *>(mu) + cell_off;
    const real *r = reinterpret_cast<const real *>(rho) + cell_off;
    real *kc = reinterpret_cast<real *>(c->kcells) + c->L.k_off[g];
    hipMemsetAsync(d_bad, 0, sizeof(int), s);
    hipMemsetAsync(d_rows, 0, ny * sizeof(int), s);
    hipError_t e = launch_kappa<real>(l, m, r, nx, ny, c->L.pitch[g], kc, d_bad, d_rows, s);
    if (e != hipSuccess) { rc = fail(LBM_E_DEVICE, hipGetErrorString(e)); break; }
    int bad = 0;
    std::vector<int> varies(ny);
    hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(varies.data(), d_rows, ny * sizeof(int), hipMemcpyDeviceToHost, s);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) { rc = fail(LBM_E_DEVICE, hipGetErrorString(e)); break; }
    if (bad) {
      char buf[200];
      snprintf(buf, sizeof buf,
               "grid %d: %d cells violate mu > 0, rho > 0, lambda >= 0, nu < 5/11", g, bad);
      rc = fail(LBM_E_INVALID, buf);
      break;
    }
    bool rows_const = std::none_of(varies.begin(), varies.end(), [](int v) { return v != 0; });
    if (rows_const) {
      std::vector<real> kr(ny);
      real *d_tmp = nullptr;
      HIP_TRY(hipMalloc((void **)&d_tmp, ny * sizeof(real)));
      launch_kappa_rows<real>(kc, ny, c->L.pitch[g], d_tmp, s);
      hipMemcpyAsync(kr.data(), d_tmp, ny * sizeof(real), hipMemcpyDeviceToHost, s);
      hipStreamSynchronize(s);
      hipFree(d_tmp);
      const bool all_same = std::all_of(kr.begin(), kr.end(), [&](real v) { return v == kr[0]; });
      if (all_same) {
        c->kmode[g] = kKappaScalar;
        c->kscalar[g] = (double)kr[0];
      } else {
        c->kmode[g] = kKappaRows;
      }
      c->krow_off[g] = (int64_t)krows_all.size();
      krows_all.insert(krows_all.end(), kr.begin(), kr.end());
      for (real k : kr) c->nu_seen.push_back(nu_of_kappa((double)k));
    } else {
      c->kmode[g] = kKappaCells;
      c->krow_off[g] = 0;
      // the range of the cell-wise moduli, sampled evenly
      const int nb = (int)std::min<int64_t>(1024, ((int64_t)nx * ny + 255) / 256);
      real *d_mm = nullptr;
      HIP_TRY(hipMalloc((void **)&d_mm, 2 * nb * sizeof(real)));
      std::vector<real> mm(2 * nb);
      e = launch_kappa_range<real>(kc, nx, ny, c->L.pitch[g], d_mm, nb, s);
      if (e == hipSuccess) e = hipMemcpyAsync(mm.data(), d_mm, 2 * nb * sizeof(real), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      hipFree(d_mm);
      if (e != hipSuccess) { rc = fail(LBM_E_DEVICE, hipGetErrorString(e)); break; }
      double klo = 1e300, khi = -1e300;
      for (int b = 0; b < nb; ++b) {
        klo = std::min(klo, (double)mm[2 * b]);
        khi = std::max(khi, (double)mm[2 * b + 1]);
      }
      for (int q = 0; q <= 8; ++q) c->nu_seen.push_back(nu_of_kappa(klo + (khi - klo) * q / 8.0));
    }
    cell_off += (int64_t)nx * ny;
  }
  hipFree(d_bad);
  hipFree(d_rows);
  if (rc) return rc;
  if (krows_all.empty()) krows_all.push_back(real(0));
  std::vector<char> kb(krows_all.size() * sizeof(real));
  memcpy(kb.data(), krows_all.data(), kb.size());
  HIP_TRY(c->d_krows.upload(kb, s));
  return LBM_OK;
}

// 1/rho0 at the receiver cells, read from the caller's density field.
template <typename real>
int gather_scale(lbm_ctx *c, int g, RecHost &R) {
  const int n = (int)R.xy.size() / 2;
  const int nx = c->grids[g].nx;
  std::vector<int64_t> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = c->cell_off[g] + (int64_t)R.xy[2 * i + 1] * nx + R.xy[2 * i];
  int64_t *d_idx = nullptr;
  real *d_val = nullptr;
  HIP_TRY(hipMalloc((void **)&d_idx, n * sizeof(int64_t)));
  hipError_t e = hipMalloc((void **)&d_val, n * sizeof(real));
  std::vector<real> h(n);
  if (e == hipSuccess) e = hipMemcpyAsync(d_idx, idx.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_gather<real>(reinterpret_cast<const real *>(c->rho), d_idx, n, d_val, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_val, n * sizeof(real), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(d_idx);
  if (d_val) hipFree(d_val);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, hipGetErrorString(e));
  R.scale.resize(n);
  for (int i = 0; i < n; ++i) R.scale[i] = 1.0 / (double)h[i];
  return LBM_OK;
}


// ---- adjoint -------------------------------------------------------------

size_t adj_fbytes(const lbm_ctx *c) { return (size_t)round_up(c->L.f_elems * (int64_t)c->L.esize, 256); }
size_t adj_cbytes(const lbm_ctx *c) { return (size_t)round_up(c->L.k_elems * (int64_t)c->L.esize, 256); }

size_t adj_ws_bytes(const lbm_ctx *c, int32_t seg, int64_t nsteps) {
  const int64_t nseg = (nsteps + seg - 1) / seg;
  return (size_t)nseg * adj_fbytes(c) + 4 * adj_fbytes(c) + (size_t)seg * adj_cbytes(c) + 256;
}

// Steps of the last r segments of a recording (the last one may be short).
int64_t trailing_steps(int32_t seg, int64_t nsteps, int64_t r) {
  const int64_t nseg = (nsteps + seg - 1) / seg;
  r = std::min(r, nseg);
  return r <= 0 ? 0 : nsteps - (nseg - r) * seg;
}

// The most whole trailing segments whose steps fit in `steps` density planes.
int64_t resident_segments(int32_t seg, int64_t nsteps, int64_t steps) {
  const int64_t nseg = (nsteps + seg - 1) / seg;
  int64_t r = 0;
  while (r < nseg && trailing_steps(seg, nsteps, r + 1) <= steps) ++r;
  return r;
}

// Forward steps while an adjoint recording is open: the state at every
// segment start t_begin + m * seg is copied to checkpoint m.
int step_recording(lbm_ctx *c, int64_t n) {
  auto &A = c->adj;
  auto take = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(A.ckpt + (size_t)A.taken * A.fbytes, c->fbuf[c->cur], A.fbytes,
                           hipMemcpyDeviceToDevice, c->stream));
    A.taken += 1;
    return LBM_OK;
  };
  while (n > 0) {
    int64_t m = n;
    if (A.taken < A.nseg) {
      const int64_t next = A.t_begin + A.taken * A.seg;
      if (c->t == next) {
        int rc = take();
        if (rc) return rc;
        continue;
      }
      m = std::min(n, next - c->t);
    }
    int rc = c->dtype == LBM_F64 ? step_impl<double>(c, m) : step_impl<float>(c, m);
    if (rc) return rc;
    n -= m;
  }
  if (A.taken < A.nseg && c->t == A.t_begin + A.taken * A.seg) return take();
  return LBM_OK;
}

// Recompute segment m from its checkpoint in the adjoint's own ping-pong
// buffers, writing rho(t) of each step to the stash.
template <typename real>
int recompute_segment(lbm_ctx *c, int64_t m) {
  auto &A = c->adj;
  const int64_t tm = A.t_begin + m * A.seg;
  const int64_t len = std::min<int64_t>(A.seg, A.t_begin + A.nsteps - tm);
  HIP_TRY(hipMemcpyAsync(A.rbuf[0], A.ckpt + (size_t)m * A.fbytes, A.fbytes, hipMemcpyDeviceToDevice,
                         c->stream));
  auto stash = [&](int64_t s) { return reinterpret_cast<real *>(A.stash + (size_t)s * A.cbytes); };
  int cur = 0;
  int64_t s = 0;
  if (use_fused(c)) {
    for (; s + 2 <= len; s += 2) {
      StepArgs<real> a = make_args<real>(c, 0);
      a.fin = reinterpret_cast<const real *>(A.rbuf[cur]);
      a.fout = reinterpret_cast<real *>(A.rbuf[cur ^ 1]);
      a.t = tm + s;
      HIP_TRY(launch_two_steps<real>(c, a, c->stream, stash(s), stash(s + 1)));
      cur ^= 1;
    }
  }
  for (; s < len; ++s, cur ^= 1) {
    StepArgs<real> a = make_args<real>(c, 0);
    a.fin = reinterpret_cast<const real *>(A.rbuf[cur]);
    a.fout = reinterpret_cast<real *>(A.rbuf[cur ^ 1]);
    a.t = tm + s;
    a.rho_out = stash(s);
    StepArgs<real> ai = a;
    ai.tiles = c->d_tiles_int.p;
    HIP_TRY(launch_pair(
        c, c->stream, c->ntiles_int > 0, c->ntiles > 0,
        [&](hipStream_t q) { return launch_step<real>(a, c->gen_waves, 1, c->ntiles, kModeStash, q); },
        [&](hipStream_t q) { return launch_interior<real>(ai, c->launch.waves, 0, c->ntiles_int, q); }));
  }
  A.stash_seg = m;
  return LBM_OK;
}

// Rows from a two-step adjoint block's own rows to the farthest row whose
// adjoint state its first step forms (three: the second step's gradient
// reads rows one out, whose pulls read fh(t) two out, whose gradient reads
// the first step's rows three out).
constexpr int kAdjRecReach = 3;

// The order of the dL/damp sums over the general adjoint kernel's workgroups
// for one launch or a pair of launches (lists, their slots one after the
// other): for each grid with sources and each of its first kMaxAdjSources
// sources, every workgroup of a tile of that grid that is not a border strip,
// in list order.
int build_amp_plan(lbm_ctx *c, std::initializer_list<const std::vector<TileDev> *> lists,
                   lbm_ctx::AmpPlan &plan) {
  std::vector<std::vector<int32_t>> per_grid(c->nbatch);
  int32_t base = 0;
  for (const std::vector<TileDev> *l : lists) {
    for (size_t i = 0; i < l->size(); ++i) {
      const TileDev &t = (*l)[i];
      if (t.g < 0 || (t.g & kStripTile)) continue;
      per_grid[t.g].push_back(base + (int32_t)i);
    }
    base += (int32_t)l->size();
  }
  std::vector<int32_t> tiles, off{0}, pairs;
  for (int g = 0; g < c->nbatch; ++g) {
    const int ns = std::min((int)c->sources[g].size(), kMaxAdjSources);
    for (int si = 0; si < ns && !per_grid[g].empty(); ++si) {
      tiles.insert(tiles.end(), per_grid[g].begin(), per_grid[g].end());
      off.push_back((int32_t)tiles.size());
      pairs.push_back(g);
      pairs.push_back(si);
    }
  }
  plan.npairs = (int)pairs.size() / 2;
  HIP_TRY(plan.tiles.upload(tiles, c->stream));
  HIP_TRY(plan.off.upload(off, c->stream));
  HIP_TRY(plan.pairs.upload(pairs, c->stream));
  return LBM_OK;
}

// The adjoint's tile lists: the forward's interior tiles whose rows y0-1 and
// y1 also hold no receiver, and every other tile. Built from the real tiles
// of the two (die-ordered, padded) forward lists in their logical order
// (grid, row, column) and die-ordered again.
int build_adjoint_tiles(lbm_ctx *c) {
  std::vector<TileDev> li, lg;
  for (const TileDev &t : c->h_tiles_gen)
    if (t.g >= 0) lg.push_back(t);
  for (const TileDev &t : c->h_tiles_int) {
    if (t.g < 0) continue;
    bool rec = false;
    const std::vector<int32_t> &xy = c->recs[t.g].xy;
    for (size_t r = 1; r < xy.size() && !rec; r += 2) rec = xy[r] == t.y0 - 1 || xy[r] == t.y1;
    if (!rec) {
      li.push_back(t);
    } else {
      const int Wg = 64 * c->gen_waves, W = 64 * c->launch.waves;
      for (int xs = t.x0; xs < std::min(t.x0 + W, c->grids[t.g].nx); xs += Wg)
        lg.push_back(TileDev{t.g, xs, t.y0, t.y1});
    }
  }
  auto logical = [](const TileDev &a, const TileDev &b) {
    return a.g != b.g ? a.g < b.g : (a.y0 != b.y0 ? a.y0 < b.y0 : a.x0 < b.x0);
  };
  std::sort(li.begin(), li.end(), logical);
  std::sort(lg.begin(), lg.end(), logical);
  auto cover = [&](const std::vector<TileDev> &v, int W) {
    int64_t n = 0;
    for (const auto &t : v)
      if (t.g >= 0) n += (int64_t)std::min(W, c->grids[t.g & ~kStripTile].nx - t.x0) * (t.y1 - t.y0);
    return n;
  };
  c->cells_adj_int = cover(li, 64 * c->launch.waves);
  c->cells_adj_gen = cover(lg, 64 * c->gen_waves);
  const std::vector<TileDev> ai = order_for_dies(li), ag = order_for_dies(lg);
  c->n_adj_int = (int)ai.size();
  c->n_adj_gen = (int)ag.size();
  HIP_TRY(c->d_adj_int.upload(ai, c->stream));
  HIP_TRY(c->d_adj_gen.upload(ag, c->stream));
  int rc = build_amp_plan(c, {&ag}, c->amp_single);
  if (rc) return rc;
  size_t part_slots = ag.size();
  c->n_adj_f = c->n_adj_g2 = c->n_adj_g1 = 0;
  c->cells_adj_f = c->cells_adj_g2 = 0;
  c->amp_pair.npairs = 0;
  if (c->launch.fuse_rows > 0) {
    // FP64 blocks of 512 columns would need more than the 168 registers a
    // lane has at three waves per SIMD: 256 columns
    c->adj_fwaves = c->dtype == LBM_F64 ? std::min(fused_waves(c), 4) : fused_waves(c);
    std::vector<FusedTileDev> tf;
    std::vector<TileDev> tg2, tg1;
    int64_t cells = 0;
    build_fused_tiles(c, c->launch.fuse_rows, c->adj_fwaves, kAdjRecReach, kStripTile, tf, tg2,
                      tg1, cells);
    if (cells > 0) {
      c->cells_adj_f = cells;
      c->cells_adj_g2 = cover(tg2, 64);
      c->n_adj_f = (int)tf.size();
      c->n_adj_g2 = (int)tg2.size();
      c->n_adj_g1 = (int)tg1.size();
      HIP_TRY(c->d_adj_ftiles.upload(tf, c->stream));
      HIP_TRY(c->d_adj_g2.upload(tg2, c->stream));
      HIP_TRY(c->d_adj_g1.upload(tg1, c->stream));
      rc = build_amp_plan(c, {&tg1, &tg2}, c->amp_pair);
      if (rc) return rc;
      part_slots = std::max(part_slots, tg1.size() + tg2.size());
    }
  }
  HIP_TRY(c->d_amp_part.reserve(part_slots * kMaxAdjSources));
  c->adj_tiles_ok = true;
  return LBM_OK;
}

// With `out`, every adjoint-kernel launch goes directly to the context's
// stream between a HIP event pair and the mean durations land in *out (the
// recompute of a segment runs as without, untimed); the adjoint state and
// dL/dkappa are the same bit for bit.
template <typename real>
int adjoint_impl(lbm_ctx *c, int64_t n, lbm_kernel_times *out = nullptr) {
  auto &A = c->adj;
  hipEvent_t ev[2] = {nullptr, nullptr};
  double sum[3] = {0.0, 0.0, 0.0};   // interior, general, two-step
  int64_t cnt[3] = {0, 0, 0};
  struct EvGuard {
    hipEvent_t *ev;
    ~EvGuard() {
      for (int i = 0; i < 2; ++i)
        if (ev[i]) hipEventDestroy(ev[i]);
    }
  } guard{ev};
  if (out)
    for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreate(&ev[i]));
  auto timed = [&](int kind, auto &&launch) -> hipError_t {
    hipError_t e = hipEventRecord(ev[0], c->stream);
    if (e == hipSuccess) e = launch(c->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e == hipSuccess) {
      sum[kind] += ms;
      cnt[kind] += 1;
    }
    return e;
  };
  // dL/damp of the launches just queued, after them on the context's stream
  auto reduce_amp = [&](const lbm_ctx::AmpPlan &p) {
    return launch_amp_reduce(c->d_amp_part.p, p.tiles.p, p.off.p, p.pairs.p, p.npairs,
                             c->d_adj_io.p, c->stream);
  };
  // the two kernels of one launch: overlapped as in a step, or timed in turn
  auto run = [&](bool has_int, bool has_gen, int kind_int, auto &&general, auto &&interior) {
    if (!out) return launch_pair(c, c->stream, has_int, has_gen, general, interior);
    hipError_t e = has_int ? timed(kind_int, interior) : hipSuccess;
    if (e == hipSuccess && has_gen) e = general(c->stream);
    return e;
  };
  if (!c->adj_tiles_ok) {
    int rc = build_adjoint_tiles(c);
    if (rc) return rc;
  }
  if (A.io_dirty) {
    HIP_TRY(c->d_adj_io.upload(A.io, c->stream));
    A.io_dirty = false;
  }
  auto stash = [&](int64_t s) { return reinterpret_cast<const real *>(A.stash + (size_t)s * A.cbytes); };
  // rho(s): kept from the recorded forward, or from the segment's recompute
  auto kept = [&](int64_t s) { return A.res_steps > 0 && s >= A.res_t0; };
  for (int64_t k = 0; k < n;) {
    const int64_t t = A.t_adj - 1;
    const int64_t m = (t - A.t_begin) / A.seg;
    if (!kept(t) && A.stash_seg != m) {
      int rc = recompute_segment<real>(c, m);
      if (rc) return rc;
    }
    const int64_t tm = A.t_begin + m * A.seg;
    auto rho_at = [&](int64_t s) {
      return kept(s) ? reinterpret_cast<const real *>(A.res + (size_t)(s - A.res_t0) * A.cbytes)
                     : stash(s - tm);
    };
    AdjArgs<real> a;
    memset(&a, 0, sizeof a);
    a.fin = reinterpret_cast<const real *>(A.abuf[A.cur]);
    a.fout = reinterpret_cast<real *>(A.abuf[A.cur ^ 1]);
    a.grids = c->d_grids.p;
    a.io = c->d_adj_io.p;
    a.kappa_rows = reinterpret_cast<const real *>(c->d_krows.p);
    a.kappa_cells = reinterpret_cast<const real *>(c->kcells);
    a.sponge = reinterpret_cast<const real *>(c->d_sponge.p);
    a.sources = c->d_src.p;
    a.itab = c->d_itab.p;
    a.rtab = reinterpret_cast<const real *>(c->d_rtab.p);
    a.rho = rho_at(t);
    a.t = t;
    a.omega = (real)(1.0 / c->tau);
    a.cforce = (real)(1.0 - 0.5 / c->tau);
    if (c->n_adj_f > 0 && n - k >= 2 && (t - 1 >= tm || (kept(t) && kept(t - 1)))) {
      // Steps t and t-1 of one recomputed segment: g1 takes the general
      // tiles and the blocks' border strips to fh(t) in the recompute's
      // first buffer (free until the next segment is recomputed), g2 the
      // general tiles from there to fh(t-1); the two-step kernel takes its
      // blocks from fh(t+1) to fh(t-1) directly.
      real *mid = reinterpret_cast<real *>(A.rbuf[0]);
      AdjArgs<real> g1 = a, f2 = a, g2 = a;
      g1.fout = mid;
      g1.tiles = c->d_adj_g1.p;
      f2.ftiles = c->d_adj_ftiles.p;
      f2.rho2 = rho_at(t - 1);
      f2.f_elems = c->L.f_elems;
      g2.fin = mid;
      g2.tiles = c->d_adj_g2.p;
      g2.t = t - 1;
      g2.rho = rho_at(t - 1);
      g1.amp_part = c->d_amp_part.p;
      g2.amp_part = c->d_amp_part.p + (size_t)c->n_adj_g1 * kMaxAdjSources;
      HIP_TRY(run(
          true, c->n_adj_g1 > 0, 2,
          [&](hipStream_t q) {
            auto l1 = [&](hipStream_t r) { return launch_adjoint<real>(g1, 1, c->n_adj_g1, r); };
            auto l2 = [&](hipStream_t r) { return launch_adjoint<real>(g2, 1, c->n_adj_g2, r); };
            hipError_t e = out ? timed(1, l1) : l1(q);
            if (e == hipSuccess && c->n_adj_g2 > 0) e = out ? timed(1, l2) : l2(q);
            return e;
          },
          [&](hipStream_t q) { return launch_adjoint_fused2<real>(f2, c->adj_fwaves, c->n_adj_f, q); }));
      HIP_TRY(reduce_amp(c->amp_pair));
      A.cur ^= 1;
      A.t_adj = t - 1;
      k += 2;
      continue;
    }
    AdjArgs<real> ag = a;
    a.tiles = c->d_adj_int.p;
    ag.tiles = c->d_adj_gen.p;
    ag.amp_part = c->d_amp_part.p;
    HIP_TRY(run(
        c->n_adj_int > 0, c->n_adj_gen > 0, 0,
        [&](hipStream_t q) {
          auto lg = [&](hipStream_t r) { return launch_adjoint<real>(ag, c->gen_waves, c->n_adj_gen, r); };
          return out ? timed(1, lg) : lg(q);
        },
        [&](hipStream_t q) { return launch_adjoint_interior<real>(a, c->launch.waves, c->n_adj_int, q); }));
    HIP_TRY(reduce_amp(c->amp_single));
    A.cur ^= 1;
    A.t_adj = t;
    k += 1;
  }
  if (out) {
    out->steps = n;
    out->interior_ms = cnt[0] ? sum[0] / (double)cnt[0] : 0.0;
    out->general_ms = cnt[1] ? sum[1] / (double)cnt[1] : 0.0;
    out->fused_ms = cnt[2] ? sum[2] / (double)cnt[2] : 0.0;
    out->interior_cells = c->cells_adj_int;
    out->general_cells = cnt[2] ? c->cells_adj_g2 : c->cells_adj_gen;
    out->fused_cells = cnt[2] ? c->cells_adj_f : 0;
    out->fused_steps = cnt[2] ? 2 : 0;
  }
  return LBM_OK;
}

int check_ctx(const lbm_ctx *c) {
  if (!c) return fail(LBM_E_INVALID, "null context");
  return LBM_OK;
}

// LBM_OK, or LBM_WARN_UNSTABLE with the reason in the error text: a bulk mode
// grows (the media's Poisson ratios at tau, Sec. 4), or an edge uses the
// printed free-surface rule, whose surface modes grow for every tau.
int stability_verdict(const lbm_ctx *c) {
  if (c->vn_growth > 1.0 + 1e-6) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "unstable: a bulk mode grows by %.6f per step for Poisson ratios %.4f..%.4f at tau %.4f",
             c->vn_growth, *std::min_element(c->nu_seen.begin(), c->nu_seen.end()),
             *std::max_element(c->nu_seen.begin(), c->nu_seen.end()), c->tau);
    return fail(LBM_WARN_UNSTABLE, buf);
  }
  for (const lbm_bc &b : c->bc)
    for (int e = 0; e < 4; ++e)
      if (b.edge[e] == LBM_FREE)
        return fail(LBM_WARN_UNSTABLE, "unstable: the printed free-surface rule (LBM_FREE) lets "
                                       "surface modes grow; LBM_FREE0 does not");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_abi_version(void) { return LBM_ABI_VERSION; }



const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_workspace_bytes(const lbm_grid *grids, int32_t nbatch, int32_t dtype, size_t *bytes) {
  if (!grids || nbatch <= 0 || !bytes) return fail(LBM_E_INVALID, "grids, nbatch > 0 and bytes required");
  if (dtype != LBM_F32 && dtype != LBM_F64) return fail(LBM_E_INVALID, "dtype must be LBM_F32 or LBM_F64");
  for (int g = 0; g < nbatch; ++g) {
    if (grids[g].nx < 3 || grids[g].ny < 3) return fail(LBM_E_INVALID, "nx and ny must be >= 3");
    if (!reach_error({grids[g]}, dtype, kMinTileRows, 0).empty())
      return fail(LBM_E_INVALID, "grid too wide: 8 rows of nine population runs must stay below 2 GiB");
  }
  *bytes = make_layout(grids, nbatch, dtype).bytes();
  return LBM_OK;
}

int lbm_init(lbm_ctx **out, const lbm_grid *grids, int32_t nbatch, int32_t dtype, const void *lam,
             const void *mu, const void *rho, double tau, const lbm_bc *bc, const lbm_sponge *sponge,
             void *workspace, size_t ws_bytes, void *hip_stream) {
  g_err.clear();
  if (!out) return fail(LBM_E_INVALID, "ctx pointer is null");
  *out = nullptr;
  if (!grids || nbatch <= 0) return fail(LBM_E_INVALID, "need nbatch >= 1 grids");
  if (dtype != LBM_F32 && dtype != LBM_F64) return fail(LBM_E_INVALID, "dtype must be LBM_F32 or LBM_F64");
  if (!lam || !mu || !rho) return fail(LBM_E_INVALID, "lam, mu and rho must be device arrays");
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(LBM_E_INVALID, "tau must be > 1/2");
  if (!bc) return fail(LBM_E_INVALID, "bc array is null");
  for (int g = 0; g < nbatch; ++g) {
    int rc = validate_grid(grids[g], bc[g], sponge ? &sponge[g] : nullptr, g, dtype);
    if (rc) return rc;
  }
  Layout L = make_layout(grids, nbatch, dtype);
  if (!workspace) return fail(LBM_E_INVALID, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(LBM_E_INVALID, "workspace must be 256-byte aligned");
  if (ws_bytes < L.bytes()) {
    char buf[128];
    snprintf(buf, sizeof buf, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes());
    return fail(LBM_E_NOMEM, buf);
  }
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_E_NOMEM, "host allocation failed");
  c->dtype = dtype;
  c->nbatch = nbatch;
  c->tau = tau;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->L = L;
  c->grids.assign(grids, grids + nbatch);
  c->bc.assign(bc, bc + nbatch);
  c->sponge.resize(nbatch);
  c->sp_thick.resize(nbatch);
  for (int g = 0; g < nbatch; ++g) {
    for (int e = 0; e < 4; ++e) {
      const int th = sponge ? sponge[g].thick[e] : 0;
      c->sp_thick[g][e] = th;
      for (int k = 0; k < th; ++k) c->sponge[g].push_back(sponge[g].profile[e][k]);
    }
  }
  c->sources.resize(nbatch);
  c->recs.resize(nbatch);
  c->kmode.assign(nbatch, kKappaScalar);
  c->kscalar.assign(nbatch, 0.0);
  c->krow_off.assign(nbatch, 0);
  c->rscale_off.assign(nbatch, 0);
  c->rho = rho;
  {
    int64_t off = 0;
    for (int g = 0; g < nbatch; ++g) {
      c->cell_off.push_back(off);
      off += (int64_t)grids[g].nx * grids[g].ny;
    }
  }
  c->ws = reinterpret_cast<char *>(workspace);
  c->fbuf[0] = c->ws;
  c->fbuf[1] = c->ws + round_up(L.f_elems * (int64_t)L.esize, 256);
  c->kcells = c->fbuf[1] + round_up(L.f_elems * (int64_t)L.esize, 256);
  c->fmid = c->kcells + round_up(L.k_elems * (int64_t)L.esize, 256);
  auto bail = [&](int rc) {
    lbm_destroy(c);
    return rc;
  };
  hipError_t e = hipMemsetAsync(c->fbuf[0], 0, 2 * round_up(L.f_elems * (int64_t)L.esize, 256), c->stream);
  if (e != hipSuccess) return bail(fail(LBM_E_DEVICE, hipGetErrorString(e)));
  int rc = dtype == LBM_F64 ? init_fields<double>(c, lam, mu, rho) : init_fields<float>(c, lam, mu, rho);
  if (rc) return bail(rc);
  std::vector<int64_t> zero_time(1, 0);
  e = c->d_time.upload(zero_time, c->stream);
  if (e != hipSuccess) return bail(fail(LBM_E_DEVICE, hipGetErrorString(e)));
  c->rtab_host.assign(L.esize, 0);
  std::vector<char> r0(c->rtab_host);
  e = c->d_rtab.upload(r0, c->stream);
  if (e != hipSuccess) return bail(fail(LBM_E_DEVICE, hipGetErrorString(e)));
  c->launch = default_launch(c);
  rc = rebuild_tiles(c);
  if (rc) return bail(rc);
  c->vn_growth = context_vn_growth(c);
  rc = commit(c);
  if (rc) return bail(rc);
  *out = c;
  return stability_verdict(c);
}

int lbm_vn_growth(double nu, double tau, int32_t nk, double *growth) {
  if (!growth) return fail(LBM_E_INVALID, "growth is null");
  if (!(nu >= 0.0 && nu < 0.5) || !(tau > 0.5) || !std::isfinite(tau))
    return fail(LBM_E_INVALID, "need 0 <= nu < 1/2 and tau > 1/2");
  if (nk < 2 || nk > 1025) return fail(LBM_E_INVALID, "nk must be in [2, 1025]");
  *growth = vn_growth(nu, tau, nk);
  return LBM_OK;
}

int lbm_stability(const lbm_ctx *c, double *growth) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!growth) return fail(LBM_E_INVALID, "growth is null");
  *growth = c->vn_growth;
  return stability_verdict(c);
}

int lbm_set_sources(lbm_ctx *c, int32_t g, const lbm_source *src, int32_t n) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch) return fail(LBM_E_INVALID, "grid index out of range");
  if (n < 0 || (n > 0 && !src)) return fail(LBM_E_INVALID, "bad source array");
  const lbm_grid &G = c->grids[g];
  for (int i = 0; i < n; ++i) {
    const lbm_source &q = src[i];
    if (!(q.x >= 0 && q.x <= G.nx - 1 && q.y >= 0 && q.y <= G.ny - 1))
      return fail(LBM_E_INVALID, "source outside the grid");
    if (!(q.sigma > 0) || !(q.period > 0) || !std::isfinite(q.amp) || !std::isfinite(q.t0) ||
        !std::isfinite(q.dir_x) || !std::isfinite(q.dir_y))
      return fail(LBM_E_INVALID, "source needs sigma > 0, period > 0 and finite values");
  }
  c->sources[g].assign(src, src + n);
  c->tables_dirty = true;   // committed by the next call that launches work
  return LBM_OK;
}

int lbm_set_receivers(lbm_ctx *c, int32_t g, const int32_t *xy, int32_t n, int32_t comp_mask,
                      void *traces, int64_t max_steps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch) return fail(LBM_E_INVALID, "grid index out of range");
  if (n < 0 || (n > 0 && (!xy || !traces))) return fail(LBM_E_INVALID, "bad receiver arrays");
  if (n > 0 && (comp_mask < 1 || comp_mask > 3)) return fail(LBM_E_INVALID, "comp_mask must be 1, 2 or 3");
  if (max_steps < 0) return fail(LBM_E_INVALID, "max_steps must be >= 0");
  const lbm_grid &G = c->grids[g];
  for (int i = 0; i < n; ++i)
    if (xy[2 * i] < 0 || xy[2 * i] >= G.nx || xy[2 * i + 1] < 0 || xy[2 * i + 1] >= G.ny)
      return fail(LBM_E_INVALID, "receiver outside the grid");
  RecHost R;
  R.xy.assign(xy, xy + 2 * n);
  R.comp_mask = n > 0 ? comp_mask : 0;
  R.trace = n > 0 ? traces : nullptr;
  R.max_steps = n > 0 ? max_steps : 0;
  R.t0 = c->t;
  if (n > 0) {
    rc = c->dtype == LBM_F64 ? gather_scale<double>(c, g, R) : gather_scale<float>(c, g, R);
    if (rc) return rc;
  }
  c->recs[g] = R;
  c->tables_dirty = true;   // committed by the next call that launches work
  return LBM_OK;
}

// A failure the periodic finite check has recorded (visible once the check
// has run), or LBM_OK.
int watch_verdict(const lbm_ctx *c) {
  if (!c->watch_host) return LBM_OK;
  const int64_t bad = *static_cast<volatile int64_t *>(c->watch_host);
  if (bad < 0) return LBM_OK;
  char buf[160];
  snprintf(buf, sizeof buf, "the periodic finite check found NaN or Inf in the state at t = %lld",
           (long long)bad);
  return fail(LBM_E_NONFINITE, buf);
}

// A recording is open until its forward run has taken every checkpoint and
// reached its last step: until then steps must go through it (checkpoints,
// kept densities).
static bool recording_open(const lbm_ctx *c) {
  const auto &A = c->adj;
  return A.begun && (A.taken < A.nseg || c->t < A.t_begin + A.nsteps);
}

int lbm_step(lbm_ctx *c, int64_t n) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (n < 0) return fail(LBM_E_INVALID, "n must be >= 0");
  rc = watch_verdict(c);
  if (rc) return rc;
  if (n == 0) return LBM_OK;
  if (recording_open(c)) {
    rc = commit(c);
    if (rc) return rc;
    return step_recording(c, n);
  }
  return c->dtype == LBM_F64 ? step_impl<double>(c, n) : step_impl<float>(c, n);
}

int lbm_step_timed(lbm_ctx *c, int64_t n, lbm_kernel_times *out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (n < 0) return fail(LBM_E_INVALID, "n must be >= 0");
  if (!out) return fail(LBM_E_INVALID, "out is null");
  if (recording_open(c))
    return fail(LBM_E_STATE, "an adjoint recording is open: advance it with lbm_step");
  rc = commit(c);
  if (rc) return rc;
  return c->dtype == LBM_F64 ? step_timed<double>(c, n, out) : step_timed<float>(c, n, out);
}

int lbm_moments(lbm_ctx *c, int32_t g, void *out6) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch) return fail(LBM_E_INVALID, "grid index out of range");
  if (!out6) return fail(LBM_E_INVALID, "out6 is null");
  rc = commit(c);
  if (rc) return rc;
  // The general kernel in moments mode over both tile lists.
  if (c->dtype == LBM_F64) {
    StepArgs<double> a = make_args<double>(c, c->cur);
    a.fout = nullptr;
    a.mom = reinterpret_cast<double *>(out6);
    a.mom_grid = g;
    HIP_TRY(launch_step<double>(a, c->gen_waves, 1, c->ntiles, kModeMoments, c->stream));
    a.tiles = c->d_tiles_int.p;
    HIP_TRY(launch_step<double>(a, c->launch.waves, 1, c->ntiles_int, kModeMoments, c->stream));
  } else {
    StepArgs<float> a = make_args<float>(c, c->cur);
    a.fout = nullptr;
    a.mom = reinterpret_cast<float *>(out6);
    a.mom_grid = g;
    HIP_TRY(launch_step<float>(a, c->gen_waves, 1, c->ntiles, kModeMoments, c->stream));
    a.tiles = c->d_tiles_int.p;
    HIP_TRY(launch_step<float>(a, c->launch.waves, 1, c->ntiles_int, kModeMoments, c->stream));
  }
  return LBM_OK;
}

int lbm_get_time(const lbm_ctx *c, int64_t *t) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!t) return fail(LBM_E_INVALID, "t is null");
  *t = c->t;
  return LBM_OK;
}

int lbm_get_state(lbm_ctx *c, int32_t g, void *dst) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch || !dst) return fail(LBM_E_INVALID, "bad grid index or dst");
  const lbm_grid &G = c->grids[g];
  const int64_t n = (int64_t)G.nx * G.ny;
  const int64_t ps = c->L.pitch[g], ys = 9 * (int64_t)c->L.pitch[g];
  if (c->dtype == LBM_F64) {
    HIP_TRY(launch_copy_planes<double>(reinterpret_cast<const double *>(c->fbuf[c->cur]) + c->L.f_off[g],
                                       ps, ys, reinterpret_cast<double *>(dst), n, G.nx, G.nx, G.ny,
                                       9, c->stream));
  } else {
    HIP_TRY(launch_copy_planes<float>(reinterpret_cast<const float *>(c->fbuf[c->cur]) + c->L.f_off[g],
                                      ps, ys, reinterpret_cast<float *>(dst), n, G.nx, G.nx, G.ny, 9,
                                      c->stream));
  }
  return LBM_OK;
}

int lbm_set_state(lbm_ctx *c, int32_t g, const void *src, int64_t t) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch || !src) return fail(LBM_E_INVALID, "bad grid index or src");
  if (t < 0) return fail(LBM_E_INVALID, "t must be >= 0");
  c->adj.begun = false;   // the recorded forward run no longer describes the state
  if (c->watch_host) {     // a new state: a recorded failure no longer applies
    HIP_TRY(hipStreamSynchronize(c->stream));
    *static_cast<volatile int64_t *>(c->watch_host) = -1;
  }
  const lbm_grid &G = c->grids[g];
  const int64_t n = (int64_t)G.nx * G.ny;
  const int64_t ps = c->L.pitch[g], ys = 9 * (int64_t)c->L.pitch[g];
  if (c->dtype == LBM_F64) {
    HIP_TRY(launch_copy_planes<double>(reinterpret_cast<const double *>(src), n, G.nx,
                                       reinterpret_cast<double *>(c->fbuf[c->cur]) + c->L.f_off[g],
                                       ps, ys, G.nx, G.ny, 9, c->stream));
  } else {
    HIP_TRY(launch_copy_planes<float>(reinterpret_cast<const float *>(src), n, G.nx,
                                      reinterpret_cast<float *>(c->fbuf[c->cur]) + c->L.f_off[g],
                                      ps, ys, G.nx, G.ny, 9, c->stream));
  }
  if (t != c->t) {
    // The context moves to time t: every grid's trace restarts at row 0 = t.
    c->t = t;
    for (auto &R : c->recs) R.t0 = t;
    c->tables_dirty = true;
    return commit(c);
  }
  return LBM_OK;
}

int lbm_filter(lbm_ctx *c, double sigma) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!(sigma > 0.0 && sigma <= 1.0 / 16.0)) return fail(LBM_E_INVALID, "sigma must be in (0, 1/16]");
  if (recording_open(c))
    return fail(LBM_E_STATE, "an adjoint recording is open: it assumes unfiltered steps");
  rc = commit(c);
  if (rc) return rc;
  const void *fin = c->fbuf[c->cur];
  void *fout = c->fbuf[c->cur ^ 1];
  hipError_t e = c->dtype == LBM_F64
                     ? launch_filter<double>(reinterpret_cast<const double *>(fin), reinterpret_cast<double *>(fout),
                                             c->d_grids.p, c->d_filt_tiles.p, c->nfilt_tiles, sigma, c->stream)
                     : launch_filter<float>(reinterpret_cast<const float *>(fin), reinterpret_cast<float *>(fout),
                                            c->d_grids.p, c->d_filt_tiles.p, c->nfilt_tiles, (float)sigma,
                                            c->stream);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, hipGetErrorString(e));
  c->cur ^= 1;
  return LBM_OK;
}

int lbm_vn_growth_filtered(double nu, double tau, double sigma, int32_t every, int32_t nk,
                           double *growth) {
  if (!growth) return fail(LBM_E_INVALID, "growth is null");
  if (!(nu >= 0.0 && nu < 0.5) || !(tau > 0.5) || !std::isfinite(tau))
    return fail(LBM_E_INVALID, "need 0 <= nu < 1/2 and tau > 1/2");
  if (!(sigma >= 0.0 && sigma <= 1.0 / 16.0)) return fail(LBM_E_INVALID, "sigma must be in [0, 1/16]");
  if (every < 1 || every > 1000) return fail(LBM_E_INVALID, "every must be in [1, 1000]");
  if (nk < 2 || nk > 1025) return fail(LBM_E_INVALID, "nk must be in [2, 1025]");
  *growth = vn_growth_filtered(nu, tau, sigma, every, nk);
  return LBM_OK;
}

int lbm_check_finite(lbm_ctx *c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  int *d = nullptr;
  HIP_TRY(hipMalloc((void **)&d, sizeof(int)));
  hipMemsetAsync(d, 0, sizeof(int), c->stream);
  hipError_t e;
  if (c->dtype == LBM_F64)
    e = launch_count_nonfinite<double>(reinterpret_cast<const double *>(c->fbuf[c->cur]), c->L.f_elems, d, c->stream);
  else
    e = launch_count_nonfinite<float>(reinterpret_cast<const float *>(c->fbuf[c->cur]), c->L.f_elems, d, c->stream);
  int h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(d);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, hipGetErrorString(e));
  if (h) return fail(LBM_E_NONFINITE, "state holds NaN or Inf");
  return LBM_OK;
}

int lbm_set_finite_check(lbm_ctx *c, int64_t every) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (every < 0) return fail(LBM_E_INVALID, "every must be >= 0");
  if (every > 0 && !c->watch_host) {
    void *h = nullptr;
    HIP_TRY(hipHostMalloc(&h, sizeof(int64_t), hipHostMallocMapped));
    void *d = nullptr;
    hipError_t e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess) {
      hipHostFree(h);
      return fail(LBM_E_DEVICE, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e));
    }
    c->watch_host = static_cast<int64_t *>(h);
    c->watch_dev = static_cast<int64_t *>(d);
  }
  // re-arm: work already enqueued may still record into the flag
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->watch_host) *static_cast<volatile int64_t *>(c->watch_host) = -1;
  c->watch_every = every;
  return LBM_OK;
}

int lbm_finite_status(lbm_ctx *c, int64_t *t_bad) {
  int rc = check_ctx(c);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  const int64_t bad = c->watch_host ? *static_cast<volatile int64_t *>(c->watch_host) : -1;
  if (t_bad) *t_bad = bad;
  return watch_verdict(c);
}

int lbm_check_finite_noalloc(lbm_ctx *c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->nbatch > kScratchGrids)
    return fail(LBM_E_INVALID,
                "lbm_check_finite_noalloc: at most 4096 grids (its static device scratch holds "
                "one flag per grid); use lbm_check_finite");
  int64_t max_elems = 0;
  for (int g = 0; g < c->nbatch; ++g)
    max_elems = std::max<int64_t>(max_elems, 9 * (int64_t)c->L.pitch[g] * c->grids[g].ny);
  // The descriptor table holds every grid's offset, pitch and height since
  // lbm_init; those never change, so no commit (which may allocate) is needed.
  uint32_t out[2] = {0u, 0u};
  hipError_t e;
  if (c->dtype == LBM_F64)
    e = check_nonfinite_scratch<double>(reinterpret_cast<const double *>(c->fbuf[c->cur]),
                                        c->d_grids.p, c->nbatch, max_elems, c->stream, out);
  else
    e = check_nonfinite_scratch<float>(reinterpret_cast<const float *>(c->fbuf[c->cur]),
                                       c->d_grids.p, c->nbatch, max_elems, c->stream, out);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, hipGetErrorString(e));
  if (out[0]) {
    char buf[128];
    snprintf(buf, sizeof buf, "state holds NaN or Inf (%u grid(s), the first is grid %u)", out[0],
             out[1]);
    return fail(LBM_E_NONFINITE, buf);
  }
  return LBM_OK;
}

int lbm_get_launch(const lbm_ctx *c, lbm_launch *out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!out) return fail(LBM_E_INVALID, "out is null");
  *out = c->launch;
  return LBM_OK;
}

int lbm_set_launch(lbm_ctx *c, const lbm_launch *cfg) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!cfg) return fail(LBM_E_INVALID, "cfg is null");
  if (cfg->waves != 1 && cfg->waves != 2 && cfg->waves != 4 && cfg->waves != 8)
    return fail(LBM_E_INVALID, "waves must be 1, 2, 4 or 8");
  if (cfg->rows < 1) return fail(LBM_E_INVALID, "rows must be >= 1");
  if (cfg->graph_chunk < 0) return fail(LBM_E_INVALID, "graph_chunk must be >= 0");
  if (cfg->prefetch < 0 || cfg->prefetch > 2) return fail(LBM_E_INVALID, "prefetch must be 1 or 2");
  if (cfg->fuse_rows != 0 && (cfg->fuse_rows < 4 || cfg->fuse_rows > kFusedMaxRows))
    return fail(LBM_E_INVALID, "fuse_rows must be 0 or in [4, 248]");
  if (cfg->fuse_steps != 0 && cfg->fuse_steps != 2 && cfg->fuse_steps != 3)
    return fail(LBM_E_INVALID, "fuse_steps must be 2 or 3 (0 means 2)");
  if (cfg->tri_waves != 0 && (cfg->tri_waves < 2 || cfg->tri_waves > 4))
    return fail(LBM_E_INVALID, "tri_waves must be 0, 2, 3 or 4");
  const int fsteps = cfg->fuse_steps == 3 ? 3 : 2;
  {
    const std::string why = reach_error(c->grids, c->dtype, cfg->rows, cfg->fuse_rows, fsteps);
    if (!why.empty()) return fail(LBM_E_INVALID, why);
  }
  const bool retile = cfg->waves != c->launch.waves || cfg->rows != c->launch.rows ||
                      cfg->split != c->launch.split || cfg->fuse_rows != c->launch.fuse_rows ||
                      fsteps != c->launch.fuse_steps || cfg->tri_waves != c->launch.tri_waves;
  if (cfg->split < 0 || cfg->split > 1 || cfg->pair < 0 || cfg->pair > 1 || cfg->overlap < 0 ||
      cfg->overlap > 1)
    return fail(LBM_E_INVALID, "split, pair and overlap must be 0 or 1");
  const bool regraph = retile || cfg->prefetch != c->launch.prefetch || cfg->pair != c->launch.pair ||
                       cfg->overlap != c->launch.overlap;
  const lbm_launch before = c->launch;
  c->launch = *cfg;
  c->launch.fuse_steps = fsteps;
  c->launch_set = true;
  if (c->launch.prefetch == 0) c->launch.prefetch = 1;
  if (regraph) drop_graphs(c);
  // whole pairs, or whole triples on the three-step path
  const int unit = c->launch.fuse_rows > 0 && fsteps == 3 ? 3 : 2;
  c->launch.graph_chunk = (c->launch.graph_chunk + unit - 1) / unit * unit;
  if (retile) {
    const int rc2 = rebuild_tiles(c);
    if (rc2 != LBM_OK) {   // keep the previous launch
      const std::string why = g_err;
      c->launch = before;
      rebuild_tiles(c);
      return fail(rc2, why);
    }
    return LBM_OK;
  }
  if (c->gchunk != c->launch.graph_chunk) drop_graphs(c);
  return LBM_OK;
}

}  // extern "C"

namespace {

// Tuning results per (GPU architecture, dtype, boundary class, size class,
// path), kept for the life of the process and, when the environment variable
// LBM_TUNE_CACHE names a file, across processes: one line
// "key|waves rows prefetch pair fuse_rows tri_waves" per result (lines
// without the last field, from before it existed, read it as 0), read the first time
// the file is named and appended to after each tuning run (the last line of a
// key wins). Lines that do not parse or hold an invalid launch are skipped.
struct TuneCache {
  std::mutex mu;
  std::map<std::string, lbm_launch> map;
  std::set<std::string> files_read;
};

TuneCache &tune_cache() {
  static TuneCache tc;
  return tc;
}

bool tuned_launch_ok(const lbm_launch &l) {
  return (l.waves == 1 || l.waves == 2 || l.waves == 4 || l.waves == 8) && l.rows >= 1 &&
         l.rows <= 4096 && l.prefetch >= 1 && l.prefetch <= 2 && (l.pair == 0 || l.pair == 1) &&
         (l.fuse_rows == 0 || (l.fuse_rows >= 4 && l.fuse_rows <= kFusedMaxRows)) &&
         (l.tri_waves == 0 || (l.tri_waves >= 2 && l.tri_waves <= 4));
}

int floor_log2(int64_t v) {
  int k = 0;
  while (k < 62 && ((int64_t)1 << (k + 1)) <= v) ++k;
  return k;
}

// The key: the architecture name without its feature suffix, the dtype, the
// distinct boundary classes of the grids (edge kinds, internal rigid row,
// sources, receivers), powers of two of the total cells, of the tallest grid
// and of the number of grids, and the path (triples, pairs or single steps).
std::string tune_key(const lbm_ctx *c) {
  std::string arch = "unknown";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  int64_t cells = 0;
  int max_ny = 0;
  std::set<std::string> cls;
  for (int g = 0; g < c->nbatch; ++g) {
    cells += (int64_t)c->grids[g].nx * c->grids[g].ny;
    max_ny = std::max(max_ny, c->grids[g].ny);
    const lbm_bc &b = c->bc[g];
    char buf[64];
    snprintf(buf, sizeof buf, "%d%d%d%d%c%c%c", b.edge[0], b.edge[1], b.edge[2], b.edge[3],
             b.rigid_row > 0 ? 'r' : '-', c->sources[g].empty() ? '-' : 's',
             c->recs[g].xy.empty() ? '-' : 'v');
    cls.insert(buf);
  }
  std::string key = arch + (c->dtype == LBM_F64 ? " f64 " : " f32 ");
  for (const std::string &k : cls) key += k + ",";
  key += " cells 2^" + std::to_string(floor_log2(cells)) + " rows 2^" +
         std::to_string(floor_log2(max_ny)) + " grids 2^" + std::to_string(floor_log2(c->nbatch)) +
         (c->launch.fuse_rows > 0 ? (c->launch.fuse_steps == 3 ? " triples" : " pairs") : " single");
  return key;
}

// Reads the file LBM_TUNE_CACHE names, once per file name. Caller holds mu.
void tune_cache_load(TuneCache &tc) {
  const char *path = std::getenv("LBM_TUNE_CACHE");
  if (!path || !*path || tc.files_read.count(path)) return;
  tc.files_read.insert(path);
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char *bar = std::strrchr(line, '|');
    if (!bar) continue;
    lbm_launch l{};
    const int got = std::sscanf(bar + 1, "%d %d %d %d %d %d", &l.waves, &l.rows, &l.prefetch,
                                &l.pair, &l.fuse_rows, &l.tri_waves);
    if (got < 5 || !tuned_launch_ok(l)) continue;
    if (got == 5) l.tri_waves = 0;
    tc.map[std::string(line, bar - line)] = l;
  }
  std::fclose(f);
}

// Records a result in the process and appends it to the named file, if any.
// Caller holds mu.
void tune_cache_store(TuneCache &tc, const std::string &key, const lbm_launch &l) {
  tc.map[key] = l;
  const char *path = std::getenv("LBM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s|%d %d %d %d %d %d\n", key.c_str(), l.waves, l.rows, l.prefetch, l.pair,
               l.fuse_rows, l.tri_waves);
  std::fclose(f);
}

// Installs the shape fields of l (the caller's graph chunk, split and overlap
// are kept).
int apply_tuned(lbm_ctx *c, const lbm_launch &l, lbm_launch *chosen) {
  lbm_launch next = c->launch;
  next.waves = l.waves;
  next.rows = l.rows;
  next.prefetch = l.prefetch;
  next.pair = l.pair;
  next.fuse_rows = l.fuse_rows;
  next.tri_waves = l.tri_waves;
  c->launch = next;
  c->launch_set = true;
  const int rc = rebuild_tiles(c);
  if (rc) return rc;
  if (chosen) *chosen = next;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_autotune(lbm_ctx *c, int32_t steps, lbm_launch *chosen) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (steps < 0) return fail(LBM_E_INVALID, "steps must be >= 0");
  rc = commit(c);
  if (rc) return rc;
  const std::string key = tune_key(c);
  TuneCache &tc = tune_cache();
  if (steps == 0) {
    lbm_launch hit{};
    bool found = false;
    {
      std::lock_guard<std::mutex> lock(tc.mu);
      tune_cache_load(tc);
      auto it = tc.map.find(key);
      if (it != tc.map.end()) {
        hit = it->second;
        found = true;
      }
    }
    if (found && reach_error(c->grids, c->dtype, hit.rows, hit.fuse_rows, c->launch.fuse_steps).empty())
      return apply_tuned(c, hit, chosen);
    steps = kDefaultTuneSteps;
  }
  const bool pairs = c->launch.fuse_rows > 0;
  const int unit = pairs ? (c->launch.fuse_steps == 3 ? 3 : 2) : 1;
  steps = (steps + unit - 1) / unit * unit;   // whole pairs or triples
  // Save the state; every candidate restarts from it.
  const size_t bytes = (size_t)c->L.f_elems * c->L.esize;
  void *save = nullptr;
  HIP_TRY(hipMalloc(&save, bytes));
  const int cur0 = c->cur;
  const int64_t t0 = c->t;
  const lbm_launch keep = c->launch;
  hipError_t e = hipMemcpyAsync(save, c->fbuf[cur0], bytes, hipMemcpyDeviceToDevice, c->stream);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  int64_t cells = 0;
  for (auto &g : c->grids) cells += (int64_t)g.nx * g.ny;
  // Candidates. On the two- and three-step paths: the block width (waves,
  // or tri_waves for three-step blocks) and height (fuse_rows), the
  // single-step shape kept for leftover steps. Otherwise the
  // single-step tile width, height, prefetch depth and column pairing.
  std::vector<lbm_launch> cands;
  if (pairs) {
    const std::vector<int> heights = unit == 3 ? std::vector<int>{16, 32, 48, 64, 96, 128, 160}
                                               : std::vector<int>{16, 24, 29, 32, 44, 48, 64};
    for (int w : {2, 3, 4, 8})
      for (int fr : heights) {
        if (unit == 3 && w == 8) continue;   // three-step blocks are at most 4 waves wide
        if (unit == 2 && w == 3) continue;   // two-step blocks: 2, 4 or 8
        lbm_launch cand = keep;
        if (unit == 3) {
          cand.tri_waves = w;
        } else {
          cand.waves = w;
        }
        cand.fuse_rows = fr;
        if (reach_error(c->grids, c->dtype, cand.rows, fr, keep.fuse_steps).empty()) cands.push_back(cand);
      }
  } else {
    bool even = true;
    for (auto &g : c->grids) even = even && (g.nx % 2 == 0);
    for (int pair = 0; pair <= (even ? 1 : 0); ++pair)
      for (int pf = 1; pf <= 2; ++pf)
        for (int w : {1, 2, 4, 8})
          for (int r : {2, 4, 8, 16, 32, 64}) {
            lbm_launch cand{w, r, 0, pf, keep.split, pair, keep.overlap, 0, keep.fuse_steps,
                            keep.tri_waves};
            if (pair && w == 1) continue;
            const int64_t tiles = cells / ((int64_t)64 * w * r);
            if (tiles < 512 && !(w == 1 && r == 4)) continue;
            if (!reach_error(c->grids, c->dtype, r, 0).empty()) continue;
            cands.push_back(cand);
          }
  }
  lbm_launch best = keep;
  float best_ms = 1e30f;
  for (size_t k = 0; k < cands.size() && e == hipSuccess && rc == LBM_OK; ++k) {
    c->launch = cands[k];
    rc = rebuild_tiles(c);
    if (rc) break;
    c->cur = cur0;
    c->t = t0;
    e = hipMemcpyAsync(c->fbuf[cur0], save, bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) break;
    rc = c->dtype == LBM_F64 ? step_direct<double>(c, std::max(unit, 2)) : step_direct<float>(c, std::max(unit, 2));  // warm-up
    if (rc) break;
    e = hipEventRecord(ev0, c->stream);
    if (e != hipSuccess) break;
    rc = c->dtype == LBM_F64 ? step_direct<double>(c, steps) : step_direct<float>(c, steps);
    if (rc) break;
    e = hipEventRecord(ev1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (e == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = cands[k];
    }
  }
  // Restore the state and install the winner (keeping the graph chunk).
  c->cur = cur0;
  c->t = t0;
  if (e == hipSuccess) e = hipMemcpyAsync(c->fbuf[cur0], save, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(save);
  if (ev0) hipEventDestroy(ev0);
  if (ev1) hipEventDestroy(ev1);
  c->launch = keep;
  if (rc) {
    rebuild_tiles(c);
    return rc;
  }
  if (e != hipSuccess) {
    rebuild_tiles(c);
    return fail(LBM_E_DEVICE, hipGetErrorString(e));
  }
  {
    std::lock_guard<std::mutex> lock(tc.mu);
    tune_cache_load(tc);
    tune_cache_store(tc, key, best);
  }
  return apply_tuned(c, best, chosen);
}


int lbm_adjoint_workspace_bytes(const lbm_ctx *c, int32_t seg_steps, int64_t nsteps, size_t *bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (seg_steps < 1 || nsteps < 1 || !bytes) return fail(LBM_E_INVALID, "need seg_steps >= 1, nsteps >= 1 and bytes");
  *bytes = adj_ws_bytes(c, seg_steps, nsteps);
  return LBM_OK;
}

int lbm_adjoint_workspace_bytes_resident(const lbm_ctx *c, int32_t seg_steps, int64_t nsteps,
                                         int64_t resident_steps, size_t *bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!bytes) return fail(LBM_E_INVALID, "bytes is null");
  if (seg_steps < 1 || nsteps < 1 || resident_steps < 0)
    return fail(LBM_E_INVALID, "need seg_steps >= 1, nsteps >= 1 and resident_steps >= 0");
  const int64_t kept = trailing_steps(seg_steps, nsteps, resident_segments(seg_steps, nsteps, resident_steps));
  *bytes = adj_ws_bytes(c, seg_steps, nsteps) + (size_t)kept * adj_cbytes(c);
  return LBM_OK;
}

int lbm_adjoint_begin(lbm_ctx *c, int32_t seg_steps, int64_t nsteps, void *ws, size_t ws_bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (seg_steps < 1 || nsteps < 1) return fail(LBM_E_INVALID, "need seg_steps >= 1 and nsteps >= 1");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(LBM_E_INVALID, "workspace must be 256-byte aligned device memory");
  if (ws_bytes < adj_ws_bytes(c, seg_steps, nsteps)) return fail(LBM_E_NOMEM, "adjoint workspace too small");
  for (int g = 0; g < c->nbatch; ++g)
    if ((int)c->sources[g].size() > kMaxAdjSources)
      return fail(LBM_E_INVALID, "at most 16 sources per grid in an adjoint run");
  rc = commit(c);
  if (rc) return rc;
  auto &A = c->adj;
  A.seg = seg_steps;
  A.nsteps = nsteps;
  A.nseg = (nsteps + seg_steps - 1) / seg_steps;
  A.fbytes = adj_fbytes(c);
  A.cbytes = adj_cbytes(c);
  char *p = reinterpret_cast<char *>(ws);
  A.ckpt = p;
  p += (size_t)A.nseg * A.fbytes;
  for (int i = 0; i < 2; ++i) { A.rbuf[i] = p; p += A.fbytes; }
  for (int i = 0; i < 2; ++i) { A.abuf[i] = p; p += A.fbytes; }
  A.stash = p;
  p += (size_t)seg_steps * A.cbytes;
  // room beyond the minimum keeps the densities of whole trailing segments
  const size_t used = (size_t)(p - reinterpret_cast<char *>(ws));
  const int64_t planes = ws_bytes > used ? (int64_t)((ws_bytes - used) / A.cbytes) : 0;
  A.res_steps = trailing_steps(seg_steps, nsteps, resident_segments(seg_steps, nsteps, planes));
  A.res = A.res_steps > 0 ? p : nullptr;
  A.res_t0 = c->t + nsteps - A.res_steps;
  A.t_begin = c->t;
  A.t_adj = c->t + nsteps;
  A.taken = 0;
  A.cur = 0;
  A.stash_seg = -1;
  A.io.assign(c->nbatch, AdjGridDev{nullptr, nullptr, nullptr});
  A.io_dirty = true;
  HIP_TRY(hipMemsetAsync(A.abuf[0], 0, 2 * A.fbytes, c->stream));
  HIP_TRY(hipMemcpyAsync(A.ckpt, c->fbuf[c->cur], A.fbytes, hipMemcpyDeviceToDevice, c->stream));
  A.taken = 1;
  A.begun = true;
  return LBM_OK;
}

int lbm_adjoint_set_io(lbm_ctx *c, int32_t g, const void *residual, double *grad_kappa,
                       double *grad_amp) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->adj.begun) return fail(LBM_E_STATE, "call lbm_adjoint_begin first");
  if (g < 0 || g >= c->nbatch) return fail(LBM_E_INVALID, "grid index out of range");
  c->adj.io[g] = AdjGridDev{residual, grad_kappa, grad_amp};
  c->adj.io_dirty = true;
  return LBM_OK;
}

int lbm_adjoint_step(lbm_ctx *c, int64_t n) {
  int rc = check_ctx(c);
  if (rc) return rc;
  auto &A = c->adj;
  if (!A.begun) return fail(LBM_E_STATE, "call lbm_adjoint_begin first");
  if (A.taken < A.nseg || c->t < A.t_begin + A.nsteps)
    return fail(LBM_E_STATE, "the recorded forward run has not reached its last step yet");
  if (n < 0 || n > A.t_adj - A.t_begin) return fail(LBM_E_INVALID, "n must be in [0, adjoint time - start time]");
  if (n == 0) return LBM_OK;
  rc = commit(c);
  if (rc) return rc;
  return c->dtype == LBM_F64 ? adjoint_impl<double>(c, n) : adjoint_impl<float>(c, n);
}

int lbm_adjoint_step_timed(lbm_ctx *c, int64_t n, lbm_kernel_times *out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!out) return fail(LBM_E_INVALID, "out is null");
  auto &A = c->adj;
  if (!A.begun) return fail(LBM_E_STATE, "call lbm_adjoint_begin first");
  if (A.taken < A.nseg || c->t < A.t_begin + A.nsteps)
    return fail(LBM_E_STATE, "the recorded forward run has not reached its last step yet");
  if (n < 0 || n > A.t_adj - A.t_begin) return fail(LBM_E_INVALID, "n must be in [0, adjoint time - start time]");
  rc = commit(c);
  if (rc) return rc;
  if (n == 0) {
    *out = lbm_kernel_times{};
    return LBM_OK;
  }
  return c->dtype == LBM_F64 ? adjoint_impl<double>(c, n, out) : adjoint_impl<float>(c, n, out);
}

int lbm_adjoint_time(const lbm_ctx *c, int64_t *t) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!t) return fail(LBM_E_INVALID, "t is null");
  if (!c->adj.begun) return fail(LBM_E_STATE, "call lbm_adjoint_begin first");
  *t = c->adj.t_adj;
  return LBM_OK;
}

static int adj_copy(lbm_ctx *c, int32_t g, void *dst, const void *src, bool out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->adj.begun) return fail(LBM_E_STATE, "call lbm_adjoint_begin first");
  if (g < 0 || g >= c->nbatch || !(out ? dst : src)) return fail(LBM_E_INVALID, "bad grid index or pointer");
  const lbm_grid &G = c->grids[g];
  const int64_t n = (int64_t)G.nx * G.ny;
  const int64_t ps = c->L.pitch[g], ys = 9 * (int64_t)c->L.pitch[g];
  char *buf = c->adj.abuf[c->adj.cur];
  if (c->dtype == LBM_F64) {
    double *b = reinterpret_cast<double *>(buf) + c->L.f_off[g];
    if (out) HIP_TRY(launch_copy_planes<double>(b, ps, ys, reinterpret_cast<double *>(dst), n, G.nx, G.nx, G.ny, 9, c->stream));
    else HIP_TRY(launch_copy_planes<double>(reinterpret_cast<const double *>(src), n, G.nx, b, ps, ys, G.nx, G.ny, 9, c->stream));
  } else {
    float *b = reinterpret_cast<float *>(buf) + c->L.f_off[g];
    if (out) HIP_TRY(launch_copy_planes<float>(b, ps, ys, reinterpret_cast<float *>(dst), n, G.nx, G.nx, G.ny, 9, c->stream));
    else HIP_TRY(launch_copy_planes<float>(reinterpret_cast<const float *>(src), n, G.nx, b, ps, ys, G.nx, G.ny, 9, c->stream));
  }
  return LBM_OK;
}

int lbm_adjoint_get_state(lbm_ctx *c, int32_t g, void *dst) { return adj_copy(c, g, dst, nullptr, true); }
int lbm_adjoint_set_state(lbm_ctx *c, int32_t g, const void *src) { return adj_copy(c, g, nullptr, src, false); }

int lbm_misfit(lbm_ctx *c, int32_t g, const void *d_obs, void *residual, int64_t nrows, double *misfit) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch) return fail(LBM_E_INVALID, "grid index out of range");
  const RecHost &R = c->recs[g];
  if (!R.trace) return fail(LBM_E_STATE, "grid has no receivers");
  if (!d_obs || !misfit) return fail(LBM_E_INVALID, "d_obs and misfit are required");
  if (nrows < 0 || nrows > R.max_steps) return fail(LBM_E_INVALID, "nrows must be in [0, max_steps]");
  const int ncomp = (R.comp_mask & 1) + ((R.comp_mask >> 1) & 1);
  const int64_t n = nrows * (int64_t)(R.xy.size() / 2) * ncomp;
  HIP_TRY(c->d_misfit_part.reserve(kMisfitParts));
  if (c->dtype == LBM_F64)
    HIP_TRY(launch_misfit<double>(reinterpret_cast<const double *>(R.trace), reinterpret_cast<const double *>(d_obs),
                                  reinterpret_cast<double *>(residual), n, misfit, c->d_misfit_part.p, c->stream));
  else
    HIP_TRY(launch_misfit<float>(reinterpret_cast<const float *>(R.trace), reinterpret_cast<const float *>(d_obs),
                                 reinterpret_cast<float *>(residual), n, misfit, c->d_misfit_part.p, c->stream));
  return LBM_OK;
}

int lbm_lame_gradient(lbm_ctx *c, int32_t g, const void *lam, const void *mu, const double *grad_kappa,
                      double *grad_lam, double *grad_mu) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (g < 0 || g >= c->nbatch) return fail(LBM_E_INVALID, "grid index out of range");
  if (!lam || !mu || !grad_kappa) return fail(LBM_E_INVALID, "lam, mu and grad_kappa are required");
  const int64_t n = (int64_t)c->grids[g].nx * c->grids[g].ny;
  if (c->dtype == LBM_F64)
    HIP_TRY(launch_lame_gradient<double>(reinterpret_cast<const double *>(lam), reinterpret_cast<const double *>(mu),
                                         grad_kappa, grad_lam, grad_mu, n, c->stream));
  else
    HIP_TRY(launch_lame_gradient<float>(reinterpret_cast<const float *>(lam), reinterpret_cast<const float *>(mu),
                                        grad_kappa, grad_lam, grad_mu, n, c->stream));
  return LBM_OK;
}

int lbm_destroy(lbm_ctx *c) {
  if (!c) return LBM_OK;
  drop_graphs(c);
  if (c->side) {
    hipStreamSynchronize(c->side);
    hipStreamDestroy(c->side);
  }
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->watch_host) {
    hipStreamSynchronize(c->stream);
    hipHostFree(c->watch_host);
  }
  c->d_adj_io.release();
  c->d_adj_int.release();
  c->d_adj_gen.release();
  c->d_adj_ftiles.release();
  c->d_adj_g2.release();
  c->d_adj_g1.release();
  c->d_amp_part.release();
  for (lbm_ctx::AmpPlan *p : {&c->amp_single, &c->amp_pair}) {
    p->tiles.release();
    p->off.release();
    p->pairs.release();
  }
  c->d_misfit_part.release();
  c->d_grids.release();
  c->d_tiles.release();
  c->d_ftiles.release();
  c->d_filt_tiles.release();
  c->d_gtiles2.release();
  c->d_gtiles1.release();
  c->d_ttiles.release();
  for (int k = 0; k < 3; ++k) c->d_tgen[k].release();
  c->d_fmid2.release();
  c->d_tiles_int.release();
  c->d_krows.release();
  c->d_sponge.release();
  c->d_src.release();
  c->d_itab.release();
  c->d_rtab.release();
  c->d_time.release();
  delete c;
  return LBM_OK;
}

}  // extern "C"
