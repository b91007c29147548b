// CPU stand-in for the HIP runtime and the kernel launchers of liblbm.so, for
// testing the library's host code without a GPU: "device" memory is host
// memory (allocations are recorded), copies and fills are performed, graph and
// event calls are inert, and every kernel launch checks that each tile and
// each address range its kernel would touch lies inside a recorded
// allocation (it aborts otherwise). The initialisation kernels are evaluated
// on the host so the host code takes the same branches as on the device.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <cmath>
#include <vector>
#include "lbm_internal.h"

static std::map<uintptr_t, size_t> g_alloc;   // base -> bytes
extern "C" void sim_register(void *p, size_t n) { g_alloc[(uintptr_t)p] = n; }
extern "C" void sim_unregister(void *p) { g_alloc.erase((uintptr_t)p); }
static void check_range(const void *p, size_t n, const char *what) {
  uintptr_t a = (uintptr_t)p;
  auto it = g_alloc.upper_bound(a);
  if (it == g_alloc.begin()) { fprintf(stderr, "OOB %s: %p not in any allocation\n", what, p); abort(); }
  --it;
  if (a + n > it->first + it->second) {
    fprintf(stderr, "OOB %s: [%p, +%zu) exceeds allocation [%p, +%zu)\n", what, p, n, (void *)it->first, it->second);
    abort();
  }
}

extern "C" void sim_check_range(const void *p, size_t n, const char *what) { check_range(p, n, what); }

hipError_t hipMalloc(void **p, size_t n) { *p = malloc(n ? n : 1); g_alloc[(uintptr_t)*p] = n ? n : 1; return hipSuccess; }
hipError_t hipFree(void *p) { if (p) { g_alloc.erase((uintptr_t)p); free(p); } return hipSuccess; }
namespace lbm { static void times_forget(const void *p, size_t n); }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
  if (k != hipMemcpyHostToDevice) check_range(s, n, "memcpy src");
  if (k != hipMemcpyDeviceToHost) check_range(d, n, "memcpy dst");
  if (k != hipMemcpyDeviceToHost) lbm::times_forget(d, n);
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
  check_range(d, n, "memset");
  lbm::times_forget(d, n);
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { *p = malloc(n ? n : 1); g_alloc[(uintptr_t)*p] = n ? n : 1; return hipSuccess; }
hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned int) { *d = h; return hipSuccess; }
hipError_t hipHostFree(void *p) { g_alloc.erase((uintptr_t)p); free(p); return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "sim error"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t)malloc(8); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { free(e); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = (hipEvent_t)malloc(8); return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t)malloc(8); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { free(s); return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = (hipGraph_t)malloc(8); return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, hipGraphNode_t *, char *, size_t) { *e = (hipGraphExec_t)malloc(8); return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { free(g); return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
  memset(p, 0, sizeof *p);
  strcpy(p->gcnArchName, "sim:feature");
  return hipSuccess;
}

namespace lbm {
template <typename real>
static void check_tiles(const TileDev *tiles, int ntiles, const GridDev *grids, int W, bool interior,
                        const char *what) {
  check_range(tiles, sizeof(TileDev) * ntiles, what);
  for (int i = 0; i < ntiles; ++i) {
    TileDev t = tiles[i];
    if (t.g < 0) continue;   // padding entries: the kernels return at once
    t.g &= ~kStripTile;      // the adjoint's border strips
    check_range(&grids[t.g], sizeof(GridDev), "grid desc");
    const GridDev &g = grids[t.g];
    if (t.x0 < 0 || t.x0 >= g.nx || t.y0 < 0 || t.y1 > g.ny || t.y0 >= t.y1) { fprintf(stderr, "bad tile %s\n", what); abort(); }
    if (interior && (t.y0 - 2 < 0 || t.y1 + 1 > g.ny - 1)) { fprintf(stderr, "interior tile rows out of range %s y0=%d y1=%d ny=%d\n", what, t.y0, t.y1, g.ny); abort(); }
    (void)W;
  }
}
template <typename real>
static void check_pop(const real *base, const GridDev &g, const char *what) {
  check_range(base + g.f_off, sizeof(real) * 9 * (size_t)g.pitch * g.ny, what);
}
// State times: for each population buffer (by base address) and grid, the
// time of the state every cell holds, -1 where unknown (not written by a step
// launch since the last copy or fill over it), -2 where poisoned (computed
// from cells of another time). A launch of S steps from time a.t (fin holding
// the state of time a.t, fout receiving a.t + S) reads the cells within 2 S
// of each cell it writes: all must hold time a.t. Only the second general
// launch of a triple may read others: its 64-column strip tiles compute
// cells beyond the two-deep strips the third launch reads, from intermediate
// cells no launch wrote; those cells are poisoned, and a triple's output must
// hold none.
struct TimeMap {
  uintptr_t lo = 0, hi = 0;   // the grid's population bytes in the buffer
  std::vector<int64_t> t;
};
static std::map<const void *, std::map<int, TimeMap>> g_time;
static int64_t g_time_reads = 0;
extern "C" int64_t sim_time_reads() { return g_time_reads; }
static void times_forget(const void *p, size_t n) {
  const uintptr_t a = (uintptr_t)p, b = a + n;
  for (auto &kv : g_time)
    for (auto &gv : kv.second)
      if (gv.second.lo < b && a < gv.second.hi) std::fill(gv.second.t.begin(), gv.second.t.end(), -1);
}
template <typename real>
static std::vector<int64_t> &times(const real *buf, int gi, const GridDev &g) {
  TimeMap &m = g_time[(const void *)buf][gi];
  if (m.t.empty()) {
    m.t.assign((size_t)g.nx * g.ny, -1);
    m.lo = (uintptr_t)(buf + g.f_off);
    m.hi = m.lo + sizeof(real) * 9 * (size_t)g.pitch * g.ny;
  }
  return m.t;
}
// Check the reads of a launch of `steps` steps writing cell (x, y) of grid gi,
// then record the cell's new time in fout.
template <typename real>
static void time_step_cell(const StepArgs<real> &a, int gi, const GridDev &g, int x, int y, int steps,
                           const char *what) {
  const std::vector<int64_t> &in = times(a.fin, gi, g);
  const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
  const int R = 2 * steps;
  for (int dy = -R; dy <= R; ++dy)
    for (int dx = -R; dx <= R; ++dx) {
      int xx = x + dx, yy = y + dy;
      if (xx < 0 || xx >= g.nx) { if (!px) continue; xx = (xx + g.nx) % g.nx; }
      if (yy < 0 || yy >= g.ny) { if (!py) continue; yy = (yy + g.ny) % g.ny; }
      const int64_t h = in[(size_t)yy * g.nx + xx];
      ++g_time_reads;
      if (h == -2 || (h >= 0 && h != a.t)) {
        if (a.tri_step == 2) {
          times(a.fout, gi, g)[(size_t)y * g.nx + x] = -2;
          return;
        }
        fprintf(stderr, "%s of time %lld at g=%d (%d,%d) reads (%d,%d) holding %s %lld\n", what,
                (long long)a.t, gi, x, y, xx, yy, h == -2 ? "poison" : "time", (long long)h);
        abort();
      }
    }
  times(a.fout, gi, g)[(size_t)y * g.nx + x] = a.t + steps;
}
// A triple: the three-step kernel and the third general launch (in either
// order) write every cell of the triple's output once, and the output then
// holds the state of the triple's end everywhere.
static std::map<int, std::vector<int>> g_tri_cov;
static const void *g_tri_out = nullptr;
static bool g_tri_seen_f3 = false, g_tri_seen_g3 = false;
static int64_t g_tri_end = -1;
static int64_t g_triples_checked = 0;
extern "C" int64_t sim_triples_checked() { return g_triples_checked; }
static int g_ngrids = 0;
static const GridDev *g_tri_grids = nullptr;
template <typename real>
static std::vector<int64_t> &times(const real *buf, int gi, const GridDev &g);
static void tri_begin(const void *out, int64_t end, const GridDev *grids) {
  if (!g_tri_seen_f3 && !g_tri_seen_g3) {
    g_tri_out = out;
    g_tri_end = end;
    g_tri_cov.clear();
  }
  if (out != g_tri_out || end != g_tri_end) {
    fprintf(stderr, "three-step launch and third general step of different triples\n");
    abort();
  }
  g_tri_grids = grids;
}
template <typename real>
static void tri_done() {
  if (!(g_tri_seen_f3 && g_tri_seen_g3)) return;
  for (int gi = 0; gi < g_ngrids; ++gi) {
    const GridDev &g = g_tri_grids[gi];
    const std::vector<int64_t> &tv = times((const real *)g_tri_out, gi, g);
    for (size_t i = 0; i < tv.size(); ++i)
      if (tv[i] != g_tri_end) {
        fprintf(stderr, "triple output cell %zu of grid %d holds time %lld, not %lld\n", i, gi,
                (long long)tv[i], (long long)g_tri_end);
        abort();
      }
    std::vector<int> &v = g_tri_cov[gi];
    if (v.size() != (size_t)g.nx * g.ny) { fprintf(stderr, "triple wrote nothing of grid %d\n", gi); abort(); }
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] != 1) {
        fprintf(stderr, "triple wrote cell %zu of grid %d %d times\n", i, gi, v[i]);
        abort();
      }
  }
  g_tri_cov.clear();
  g_tri_out = nullptr;
  g_tri_seen_f3 = g_tri_seen_g3 = false;
  ++g_triples_checked;
}
// Two-step path bookkeeping. Each launch gets a sequence number and stamps
// the cells it writes in its output buffer. A pair is: the general kernel's
// first step (g1: its tiles and the two-step blocks' border strips, into the
// intermediate buffer), its second step (g2: out of the intermediate buffer)
// and the two-step kernel (f2), which needs nothing from g1 or g2. So g2 must
// find every cell it may read (within two cells of its tiles) stamped by the
// g1 launched just before it, and f2 plus g2 must write every cell of every
// grid exactly once, in either order.
static int64_t g_seq = 0, g_g1_seq = -10;
static const void *g_fmid = nullptr, *g_pair_out = nullptr;
static std::map<const void *, std::map<int, std::vector<int64_t>>> g_stamps;
static std::map<int, std::vector<int>> g_cov;   // per grid and cell: writes of the pending pair
// Density planes: the time whose rho a forward launch last wrote to each
// plane (by base address), checked against the time the adjoint reads it for.
static std::map<const void *, int64_t> g_plane_t;
static void plane_written(const void *p, int64_t t) { g_plane_t[p] = t; }
static void plane_read(const void *p, int64_t t, const char *what) {
  auto it = g_plane_t.find(p);
  if (it == g_plane_t.end() || it->second != t) {
    fprintf(stderr, "%s: density plane %p read for time %lld holds %s%lld\n", what, p, (long long)t,
            it == g_plane_t.end() ? "nothing " : "time ", it == g_plane_t.end() ? 0LL : (long long)it->second);
    abort();
  }
}

static bool g_seen_f2 = false, g_seen_g2 = false;
static int64_t g_pairs_checked = 0;

static std::vector<int64_t> &stamps(const void *buf, int g, const GridDev &G) {
  std::vector<int64_t> &v = g_stamps[buf][g];
  if (v.empty()) v.assign((size_t)G.nx * G.ny, -100);
  return v;
}
static void pair_start(const void *out) {
  if (g_seen_f2 || g_seen_g2) return;   // the pair has begun
  g_pair_out = out;
  g_cov.clear();
}
static void pair_check_done() {
  if (!(g_seen_f2 && g_seen_g2)) return;
  for (int g = 0; g < g_ngrids; ++g) {
    const std::vector<int> &v = g_cov[g];
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] != 1) {
        fprintf(stderr, "two-step pair wrote cell %zu of grid %d %d times\n", i, g, v[i]);
        abort();
      }
  }
  g_seen_f2 = g_seen_g2 = false;
  ++g_pairs_checked;
}
extern "C" int64_t sim_pairs_checked() { pair_check_done(); return g_pairs_checked; }
static std::vector<int> &cov(int g, const GridDev &G) {
  std::vector<int> &v = g_cov[g];
  if (v.empty()) v.assign((size_t)G.nx * G.ny, 0);
  return v;
}

template <typename real>
hipError_t launch_step(const StepArgs<real> &a, int waves, int, int ntiles, int mode, hipStream_t) {
  if (ntiles <= 0) return hipSuccess;
  check_tiles<real>(a.tiles, ntiles, a.grids, 64 * waves, false, "step tiles");
  const int64_t seq = g_seq++;
  const int W = 64 * waves;
  if (a.fmid) g_fmid = a.fmid;
  const bool first = !a.tri_step && g_fmid && (const void *)a.fout == g_fmid;
  const bool second = !a.tri_step && g_fmid && (const void *)a.fin == g_fmid;
  if (a.tri_step == 3) {
    if (g_tri_seen_g3) { fprintf(stderr, "two third general steps in one triple\n"); abort(); }
    tri_begin(a.fout, a.t + 1, a.grids);
  }
  if (first) g_g1_seq = seq;
  if (second) {
    if (g_seen_g2) { fprintf(stderr, "two second general steps in one pair\n"); abort(); }
    pair_start(a.fout);
    if ((const void *)a.fout != g_pair_out) { fprintf(stderr, "second general step writes another buffer than its pair\n"); abort(); }
  }
  for (int i = 0; i < ntiles && mode != kModeMoments; ++i) {
    const TileDev t = a.tiles[i];
    if (t.g < 0) continue;
    const GridDev &g = a.grids[t.g];
    const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
    std::vector<int64_t> &out = stamps(a.fout, t.g, g);
    std::vector<int64_t> *mid = second ? &stamps(g_fmid, t.g, g) : nullptr;
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x0 + W && x < g.nx; ++x) {
        out[(size_t)y * g.nx + x] = seq;
        time_step_cell(a, t.g, g, x, y, 1, "general step");
        if (a.tri_step == 3) {
          std::vector<int> &v = g_tri_cov[t.g];
          if (v.empty()) v.assign((size_t)g.nx * g.ny, 0);
          v[(size_t)y * g.nx + x] += 1;
        }
        if (!second) continue;
        cov(t.g, g)[(size_t)y * g.nx + x] += 1;
        for (int dy = -2; dy <= 2; ++dy)
          for (int dx = -2; dx <= 2; ++dx) {
            int xx = x + dx, yy = y + dy;
            if (xx < 0 || xx >= g.nx) { if (!px) continue; xx = (xx + g.nx) % g.nx; }
            if (yy < 0 || yy >= g.ny) { if (!py) continue; yy = (yy + g.ny) % g.ny; }
            if ((*mid)[(size_t)yy * g.nx + xx] < g_g1_seq) {
              fprintf(stderr, "second general step reads a cell the first did not write: g=%d (%d,%d) from (%d,%d)\n",
                      t.g, xx, yy, x, y);
              abort();
            }
          }
      }
  }
  for (int i = 0; i < ntiles; ++i) {
    if (a.tiles[i].g < 0) continue;
    const GridDev &g = a.grids[a.tiles[i].g];
    check_pop(a.fin, g, "step fin");
    if (mode != kModeMoments) check_pop(a.fout, g, "step fout");
    if (a.rho_out) check_range(a.rho_out + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "stash out");
  }
  if (a.rho_out && mode != kModeMoments) plane_written(a.rho_out, a.t);
  if (second) {
    g_seen_g2 = true;
    pair_check_done();
  }
  if (a.tri_step == 3) {
    g_tri_seen_g3 = true;
    tri_done<real>();
  }
  return hipSuccess;
}
template <typename real>
hipError_t launch_interior(const StepArgs<real> &a, int waves, int, int ntiles, hipStream_t) {
  if (ntiles <= 0) return hipSuccess;
  check_tiles<real>(a.tiles, ntiles, a.grids, 64 * waves, true, "interior tiles");
  for (int i = 0; i < ntiles; ++i) {
    if (a.tiles[i].g < 0) continue;
    const GridDev &g = a.grids[a.tiles[i].g];
    check_pop(a.fin, g, "int fin");
    check_pop(a.fout, g, "int fout");
    if (a.rho_out) check_range(a.rho_out + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "int stash out");
    const TileDev t = a.tiles[i];
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x0 + 64 * waves && x < g.nx; ++x) time_step_cell(a, t.g, g, x, y, 1, "interior step");
  }
  if (a.rho_out) plane_written(a.rho_out, a.t);
  return hipSuccess;
}
template <typename real>
hipError_t launch_fused2(const StepArgs<real> &a, int waves, int ntiles, hipStream_t) {
  if (ntiles <= 0) return hipSuccess;
  const int W = 64 * waves;
  check_range(a.ftiles, sizeof(FusedTileDev) * ntiles, "fused tiles");
  // every grid's population block lies inside f_elems: count the grids
  g_ngrids = 0;
  for (int64_t fe = 0; fe < a.f_elems; ++g_ngrids)
    fe = a.grids[g_ngrids].f_off + 9 * (int64_t)a.grids[g_ngrids].pitch * a.grids[g_ngrids].ny;
  const int64_t seq = g_seq++;
  g_fmid = a.fmid;
  if (g_seen_f2) { fprintf(stderr, "two two-step launches in one pair\n"); abort(); }
  pair_start(a.fout);
  if ((const void *)a.fout != g_pair_out) { fprintf(stderr, "two-step launch writes another buffer than its pair\n"); abort(); }
  for (int g = 0; g < g_ngrids; ++g) cov(g, a.grids[g]);
  for (int i = 0; i < ntiles; ++i) {
    const FusedTileDev t = a.ftiles[i];
    if (t.g < 0) continue;
    if (t.g >= g_ngrids) { fprintf(stderr, "fused tile grid %d out of range\n", t.g); abort(); }
    const GridDev &g = a.grids[t.g];
    if (t.x0 < 0 || t.x1 > g.nx || t.x1 <= t.x0 || t.x1 - t.x0 > W || t.y0 - 4 < 0 ||
        t.y1 + 3 > g.ny - 1 || t.y0 >= t.y1 || t.y1 - t.y0 > kFusedMaxRows) {
      fprintf(stderr, "bad fused tile g=%d x0=%d x1=%d y0=%d y1=%d (nx=%d ny=%d)\n", t.g, t.x0, t.x1, t.y0, t.y1, g.nx, g.ny);
      abort();
    }
    check_pop(a.fin, g, "fused fin");
    check_pop(a.fout, g, "fused fout");
    if (a.rho_out) {
      check_range(a.rho_out + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "fused stash t");
      check_range(a.rho_out2 + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "fused stash t+1");
    }
    // what the two-step kernel does not handle must lie outside its reach:
    // rigid-row links and side walls among the pulled cells, source disks
    // within four cells, receivers in its own rows
    const int rr = g.rigid_row;
    if (rr > 0 && t.y0 - 3 <= rr && t.y1 + 2 >= rr - 1) { fprintf(stderr, "fused tile pulls across the rigid row\n"); abort(); }
    const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
    if (!px && (t.x0 - 5 < 0 || t.x1 + 4 > g.nx - 1)) { fprintf(stderr, "fused tile pulls across a side wall\n"); abort(); }
    for (int si = 0; si < g.nsrc; ++si) {
      const SourceDev q = a.sources[g.src_off + si];
      for (int y = t.y0 - 3; y <= t.y1 + 2; ++y)
        for (int x = t.x0 - 4; x <= t.x1 + 3; ++x) {
          double dx = x - q.x, dy = y - q.y;
          if (px) { if (dx > 0.5 * g.nx) dx -= g.nx; else if (dx < -0.5 * g.nx) dx += g.nx; }
          if (py) { if (dy > 0.5 * g.ny) dy -= g.ny; else if (dy < -0.5 * g.ny) dy += g.ny; }
          if (dx * dx + dy * dy <= 81.0 * q.sigma * q.sigma) { fprintf(stderr, "source reaches a fused tile\n"); abort(); }
        }
    }
    if (g.nrec > 0)
      for (int y = t.y0; y < t.y1; ++y)
        if (a.itab[g.rowtab_off + y] >= 0) { fprintf(stderr, "receiver row %d in a fused tile\n", y); abort(); }
    std::vector<int64_t> &out = stamps(a.fout, t.g, g);
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x1; ++x) {
        const size_t c = (size_t)y * g.nx + x;
        g_cov[t.g][c] += 1;
        out[c] = seq;
        time_step_cell(a, t.g, g, x, y, 2, "two-step block");
      }
  }
  if (a.rho_out) {
    plane_written(a.rho_out, a.t);
    plane_written(a.rho_out2, a.t + 1);
  }
  g_seen_f2 = true;
  pair_check_done();
  return hipSuccess;
}
// The three-step kernel: its blocks inside the grid with six rows and
// columns of reach clear of walls, the y-wrap, the rigid row, source disks
// (over the cells its first stages compute: 5 beyond the block) and
// receivers in its rows; each block's cells read only cells of time a.t
// within six and become a.t + 3.
template <typename real>
hipError_t launch_fused3(const StepArgs<real> &a, int waves, int ntiles, hipStream_t) {
  if (ntiles <= 0) return hipSuccess;
  if (waves < 2 || waves > 4) { fprintf(stderr, "three-step waves %d\n", waves); abort(); }
  if (a.fmid || a.rho_out || a.tri_step) { fprintf(stderr, "three-step launch with pair or stash fields set\n"); abort(); }
  const int W = 64 * waves;
  check_range(a.ftiles, sizeof(FusedTileDev) * ntiles, "three-step tiles");
  g_ngrids = 0;
  for (int64_t fe = 0; fe < a.f_elems; ++g_ngrids)
    fe = a.grids[g_ngrids].f_off + 9 * (int64_t)a.grids[g_ngrids].pitch * a.grids[g_ngrids].ny;
  if (g_tri_seen_f3) { fprintf(stderr, "two three-step launches in one triple\n"); abort(); }
  tri_begin(a.fout, a.t + 3, a.grids);
  for (int gi = 0; gi < g_ngrids; ++gi)
    if (g_tri_cov[gi].empty()) g_tri_cov[gi].assign((size_t)a.grids[gi].nx * a.grids[gi].ny, 0);
  for (int i = 0; i < ntiles; ++i) {
    const FusedTileDev t = a.ftiles[i];
    if (t.g < 0) continue;
    if (t.g >= g_ngrids) { fprintf(stderr, "three-step tile grid %d out of range\n", t.g); abort(); }
    const GridDev &g = a.grids[t.g];
    if (t.x0 < 0 || t.x1 > g.nx || t.x1 <= t.x0 || t.x1 - t.x0 > W || t.y0 - 6 < 0 ||
        t.y1 + 5 > g.ny - 1 || t.y0 >= t.y1 || t.y1 - t.y0 > kFusedMaxRows) {
      fprintf(stderr, "bad three-step tile g=%d x0=%d x1=%d y0=%d y1=%d (nx=%d ny=%d)\n", t.g, t.x0, t.x1, t.y0, t.y1, g.nx, g.ny);
      abort();
    }
    check_pop(a.fin, g, "three-step fin");
    check_pop(a.fout, g, "three-step fout");
    const int rr = g.rigid_row;
    if (rr > 0 && t.y0 - 5 <= rr && t.y1 + 4 >= rr - 1) { fprintf(stderr, "three-step tile pulls across the rigid row\n"); abort(); }
    const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
    if (!px && (t.x0 - 6 < 0 || t.x1 + 5 > g.nx - 1)) { fprintf(stderr, "three-step tile pulls across a side wall\n"); abort(); }
    for (int si = 0; si < g.nsrc; ++si) {
      const SourceDev q = a.sources[g.src_off + si];
      for (int y = t.y0 - 5; y <= t.y1 + 4; ++y)
        for (int x = t.x0 - 5; x <= t.x1 + 4; ++x) {
          double dx = x - q.x, dy = y - q.y;
          if (px) { if (dx > 0.5 * g.nx) dx -= g.nx; else if (dx < -0.5 * g.nx) dx += g.nx; }
          if (py) { if (dy > 0.5 * g.ny) dy -= g.ny; else if (dy < -0.5 * g.ny) dy += g.ny; }
          if (dx * dx + dy * dy <= 81.0 * q.sigma * q.sigma) { fprintf(stderr, "source reaches a three-step tile\n"); abort(); }
        }
    }
    if (g.nrec > 0)
      for (int y = t.y0; y < t.y1; ++y)
        if (a.itab[g.rowtab_off + y] >= 0) { fprintf(stderr, "receiver row %d in a three-step tile\n", y); abort(); }
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x1; ++x) {
        g_tri_cov[t.g][(size_t)y * g.nx + x] += 1;
        time_step_cell(a, t.g, g, x, y, 3, "three-step block");
      }
  }
  g_tri_seen_f3 = true;
  tri_done<real>();
  return hipSuccess;
}
template <typename real>
hipError_t launch_filter(const real *fin, real *fout, const GridDev *grids, const TileDev *tiles, int ntiles,
                         real, hipStream_t) {
  if (ntiles <= 0) return hipSuccess;
  check_tiles<real>(tiles, ntiles, grids, 256, false, "filter tiles");
  for (int i = 0; i < ntiles; ++i) {
    if (tiles[i].g < 0) continue;
    check_pop(fin, grids[tiles[i].g], "filter in");
    check_pop(fout, grids[tiles[i].g], "filter out");
  }
  // the filter keeps the time: each cell it writes (it reads two cells along
  // each axis) takes the time of fin's cell
  for (int i = 0; i < ntiles; ++i) {
    const TileDev t = tiles[i];
    if (t.g < 0) continue;
    const GridDev &g = grids[t.g];
    const std::vector<int64_t> &in = times(fin, t.g, g);
    std::vector<int64_t> &out = times(fout, t.g, g);
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x0 + 256 && x < g.nx; ++x) out[(size_t)y * g.nx + x] = in[(size_t)y * g.nx + x];
  }
  return hipSuccess;
}
// Adjoint pairs, checked as the forward's: the general kernel's first step
// (g1, its tile list holding the blocks' border strips) writes the
// intermediate buffer, its second (g2) reads only cells within two of its
// tiles that g1 wrote, and the two-step kernel (f2) plus g2 write every cell
// of every grid exactly once.
static int64_t g_adj_g1_seq = -10;
static const void *g_adj_mid = nullptr;
static bool g_adj_seen_f2 = false, g_adj_seen_g2 = false;
static std::map<int, std::vector<int>> g_adj_cov;
static int g_adj_ngrids = 0;
static int64_t g_adj_pairs_checked = 0;
static std::map<const double *, int64_t> g_amp_slot;   // partial-sum slot -> launch that wrote it
static int64_t g_amp_reduced = 0;                      // launches before the last reduction
static std::vector<int> &adj_cov(int g, const GridDev &G) {
  std::vector<int> &v = g_adj_cov[g];
  if (v.empty()) v.assign((size_t)G.nx * G.ny, 0);
  return v;
}
static void adj_pair_check_done() {
  if (!(g_adj_seen_f2 && g_adj_seen_g2)) return;
  for (int g = 0; g < g_adj_ngrids; ++g) {
    const std::vector<int> &v = g_adj_cov[g];
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] != 1) {
        fprintf(stderr, "adjoint pair wrote cell %zu of grid %d %d times\n", i, g, v[i]);
        abort();
      }
  }
  g_adj_cov.clear();
  g_adj_seen_f2 = g_adj_seen_g2 = false;
  ++g_adj_pairs_checked;
}
extern "C" int64_t sim_adjoint_pairs_checked() { adj_pair_check_done(); return g_adj_pairs_checked; }

template <typename real>
static hipError_t adj_common(const AdjArgs<real> &a, int waves, int ntiles, bool interior) {
  if (ntiles <= 0) return hipSuccess;
  check_tiles<real>(a.tiles, ntiles, a.grids, 64 * waves, interior, interior ? "adj int tiles" : "adj gen tiles");
  const int64_t seq = g_seq++;
  bool strips = false;
  for (int i = 0; i < ntiles; ++i) strips = strips || (a.tiles[i].g >= 0 && (a.tiles[i].g & kStripTile));
  if (strips && interior) { fprintf(stderr, "border strips in the interior adjoint list\n"); abort(); }
  if (strips) {
    g_adj_g1_seq = seq;
    g_adj_mid = a.fout;
  }
  const bool second = !interior && g_adj_mid && (const void *)a.fin == g_adj_mid;
  plane_read(a.rho, a.t, interior ? "adjoint interior launch" : "adjoint general launch");
  if (second && g_adj_seen_g2) { fprintf(stderr, "two second adjoint steps in one pair\n"); abort(); }
  const int W = 64 * waves;
  for (int i = 0; i < ntiles; ++i) {
    TileDev t = a.tiles[i];
    if (t.g < 0) continue;
    t.g &= ~kStripTile;
    const GridDev &g = a.grids[t.g];
    check_range(&a.io[t.g], sizeof(AdjGridDev), "adj io");
    const AdjGridDev io = a.io[t.g];
    check_pop(a.fin, g, "adj fin");
    check_pop(a.fout, g, "adj fout");
    check_range(a.rho + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "adj rho");
    if (io.grad_kappa) check_range(io.grad_kappa, sizeof(double) * (size_t)g.nx * g.ny, "grad_kappa");
    if (io.grad_amp && g.nsrc) check_range(io.grad_amp, sizeof(double) * (g.nsrc < kMaxAdjSources ? g.nsrc : kMaxAdjSources), "grad_amp");
    if (!interior && io.grad_amp && g.nsrc && !(a.tiles[i].g & kStripTile)) {
      check_range(a.amp_part + (size_t)i * kMaxAdjSources, sizeof(double) * kMaxAdjSources, "dL/damp partial sums");
      g_amp_slot[a.amp_part + (size_t)i * kMaxAdjSources] = g_seq;   // written by this launch
    }
    if (io.residual && g.nrec) check_range(io.residual, sizeof(real) * (size_t)g.trace_max * g.nrec * g.ncomp, "residual");
    std::vector<int64_t> &out = stamps(a.fout, t.g, g);
    std::vector<int64_t> *mid = second ? &stamps(g_adj_mid, t.g, g) : nullptr;
    const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x0 + W && x < g.nx; ++x) {
        out[(size_t)y * g.nx + x] = seq;
        if (!second) continue;
        adj_cov(t.g, g)[(size_t)y * g.nx + x] += 1;
        for (int dy = -2; dy <= 2; ++dy)
          for (int dx = -2; dx <= 2; ++dx) {
            int xx = x + dx, yy = y + dy;
            if (xx < 0 || xx >= g.nx) { if (!px) continue; xx = (xx + g.nx) % g.nx; }
            if (yy < 0 || yy >= g.ny) { if (!py) continue; yy = (yy + g.ny) % g.ny; }
            if ((*mid)[(size_t)yy * g.nx + xx] < g_adj_g1_seq) {
              fprintf(stderr, "second adjoint step reads a cell the first did not write: g=%d (%d,%d) from (%d,%d)\n",
                      t.g, xx, yy, x, y);
              abort();
            }
          }
      }
  }
  if (second) {
    g_adj_seen_g2 = true;
    adj_pair_check_done();
  }
  return hipSuccess;
}
template <typename real>
hipError_t launch_adjoint(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t) { return adj_common(a, waves, ntiles, false); }
// every slot the reduction reads was written by a general launch since the
// previous reduction
hipError_t launch_amp_reduce(const double *part, const int32_t *tiles, const int32_t *off,
                             const int32_t *pairs, int npairs, const AdjGridDev *io, hipStream_t) {
  if (npairs <= 0) return hipSuccess;
  check_range(off, sizeof(int32_t) * (npairs + 1), "amp plan offsets");
  check_range(pairs, sizeof(int32_t) * 2 * npairs, "amp plan pairs");
  for (int k = 0; k < npairs; ++k) {
    check_range(&io[pairs[2 * k]], sizeof(AdjGridDev), "amp io");
    if (!io[pairs[2 * k]].grad_amp) continue;
    check_range(tiles + off[k], sizeof(int32_t) * (off[k + 1] - off[k]), "amp plan tiles");
    for (int i = off[k]; i < off[k + 1]; ++i) {
      const double *slot = part + (size_t)tiles[i] * kMaxAdjSources;
      auto it = g_amp_slot.find(slot);
      if (it == g_amp_slot.end() || it->second <= g_amp_reduced) {
        fprintf(stderr, "dL/damp reduction reads a slot no general launch wrote since the last one\n");
        abort();
      }
    }
  }
  g_amp_reduced = g_seq;
  return hipSuccess;
}
template <typename real>
hipError_t launch_adjoint_interior(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t) { return adj_common(a, waves, ntiles, true); }
template <typename real>
hipError_t launch_adjoint_fused2(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t) {
  if (ntiles <= 0) return hipSuccess;
  if (waves != 2 && waves != 4 && waves != 8) { fprintf(stderr, "adjoint two-step waves %d\n", waves); abort(); }
  if (sizeof(real) == 8 && waves == 8) { fprintf(stderr, "FP64 adjoint two-step blocks of 512 columns\n"); abort(); }
  const int W = 64 * waves;
  check_range(a.ftiles, sizeof(FusedTileDev) * ntiles, "adjoint fused tiles");
  g_adj_ngrids = 0;
  for (int64_t fe = 0; fe < a.f_elems; ++g_adj_ngrids)
    fe = a.grids[g_adj_ngrids].f_off + 9 * (int64_t)a.grids[g_adj_ngrids].pitch * a.grids[g_adj_ngrids].ny;
  if (g_adj_seen_f2) { fprintf(stderr, "two adjoint two-step launches in one pair\n"); abort(); }
  plane_read(a.rho, a.t, "adjoint two-step launch, rho(t)");
  plane_read(a.rho2, a.t - 1, "adjoint two-step launch, rho(t-1)");
  const int64_t seq = g_seq++;
  for (int g = 0; g < g_adj_ngrids; ++g) adj_cov(g, a.grids[g]);
  for (int i = 0; i < ntiles; ++i) {
    const FusedTileDev t = a.ftiles[i];
    if (t.g < 0) continue;
    if (t.g >= g_adj_ngrids) { fprintf(stderr, "adjoint fused tile grid %d out of range\n", t.g); abort(); }
    const GridDev &g = a.grids[t.g];
    if (t.x0 < 0 || t.x1 > g.nx || t.x1 <= t.x0 || t.x1 - t.x0 > W || t.y0 - 4 < 0 ||
        t.y1 + 3 > g.ny - 1 || t.y0 >= t.y1 || t.y1 - t.y0 > kFusedMaxRows) {
      fprintf(stderr, "bad adjoint fused tile g=%d x0=%d x1=%d y0=%d y1=%d\n", t.g, t.x0, t.x1, t.y0, t.y1);
      abort();
    }
    check_pop(a.fin, g, "adj fused fin");
    check_pop(a.fout, g, "adj fused fout");
    check_range(a.rho + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "adj fused rho(t)");
    check_range(a.rho2 + g.c_off, sizeof(real) * (size_t)g.pitch * g.ny, "adj fused rho(t-1)");
    check_range(&a.io[t.g], sizeof(AdjGridDev), "adj io");
    if (a.io[t.g].grad_kappa) check_range(a.io[t.g].grad_kappa, sizeof(double) * (size_t)g.nx * g.ny, "grad_kappa");
    // what the kernel does not handle lies outside its reach: walls and the
    // rigid row among the pulled rows and columns, receivers within three
    // rows of an own row, source disks over its own cells
    const int rr = g.rigid_row;
    if (rr > 0 && t.y0 - 3 <= rr && t.y1 + 2 >= rr - 1) { fprintf(stderr, "adjoint fused tile pulls across the rigid row\n"); abort(); }
    const bool px = g.bc[kEdgeLeft] == kPeriodic, py = g.bc[kEdgeTop] == kPeriodic;
    if (!px && (t.x0 - 5 < 0 || t.x1 + 4 > g.nx - 1)) { fprintf(stderr, "adjoint fused tile pulls across a side wall\n"); abort(); }
    if (g.nrec > 0)
      for (int y = t.y0 - 3; y <= t.y1 + 2; ++y)
        if (a.itab[g.rowtab_off + y] >= 0) { fprintf(stderr, "receiver row %d within reach of an adjoint fused tile\n", y); abort(); }
    for (int si = 0; si < g.nsrc; ++si) {
      const SourceDev q = a.sources[g.src_off + si];
      for (int y = t.y0; y < t.y1; ++y)
        for (int x = t.x0; x < t.x1; ++x) {
          double dx = x - q.x, dy = y - q.y;
          if (px) { if (dx > 0.5 * g.nx) dx -= g.nx; else if (dx < -0.5 * g.nx) dx += g.nx; }
          if (py) { if (dy > 0.5 * g.ny) dy -= g.ny; else if (dy < -0.5 * g.ny) dy += g.ny; }
          if (dx * dx + dy * dy <= 81.0 * q.sigma * q.sigma) { fprintf(stderr, "source reaches an adjoint fused tile\n"); abort(); }
        }
    }
    std::vector<int64_t> &out = stamps(a.fout, t.g, g);
    for (int y = t.y0; y < t.y1; ++y)
      for (int x = t.x0; x < t.x1; ++x) {
        adj_cov(t.g, g)[(size_t)y * g.nx + x] += 1;
        out[(size_t)y * g.nx + x] = seq;
      }
  }
  g_adj_seen_f2 = true;
  adj_pair_check_done();
  return hipSuccess;
}
template <typename real>
hipError_t launch_misfit(const real *tr, const real *d, real *r, int64_t n, double *m, double *part, hipStream_t) {
  check_range(tr, n * sizeof(real), "misfit tr"); check_range(d, n * sizeof(real), "misfit d");
  if (r) check_range(r, n * sizeof(real), "misfit r");
  int64_t nb = (n + 255) / 256;
  nb = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
  check_range(part, nb * sizeof(double), "misfit partial sums");
  check_range(m, 8, "misfit m"); return hipSuccess;
}
template <typename real>
hipError_t launch_lame_gradient(const real *l, const real *m, const double *gk, double *gl, double *gm, int64_t n, hipStream_t) {
  check_range(l, n * sizeof(real), "lame l"); check_range(m, n * sizeof(real), "lame m"); check_range(gk, n * 8, "lame gk");
  if (gl) check_range(gl, n * 8, "lame gl"); if (gm) check_range(gm, n * 8, "lame gm"); return hipSuccess;
}
template <typename real>
hipError_t launch_kappa(const real *lam, const real *mu, const real *rho, int nx, int ny, int pitch, real *kappa, int *bad, int *row_varies, hipStream_t) {
  const int64_t n = (int64_t)nx * ny;
  check_range(lam, n * sizeof(real), "kappa lam"); check_range(mu, n * sizeof(real), "kappa mu"); check_range(rho, n * sizeof(real), "kappa rho");
  check_range(kappa, (size_t)pitch * ny * sizeof(real), "kappa out"); check_range(bad, 4, "bad"); check_range(row_varies, 4 * ny, "rows");
  for (int64_t k = 0; k < n; ++k) {
    const int y = k / nx, x = k % nx;
    double l = lam[k], m = mu[k], r = rho[k];
    bool ok = m > 0 && r > 0 && l >= 0 && l / (2 * (l + m)) < 5.0 / 11.0;
    if (!ok) bad[0]++;
    kappa[(int64_t)y * pitch + x] = ok ? (real)((1.0 / 3.0) * (m - l) / m) : real(0);
    if (x > 0 && (lam[(int64_t)y * nx] != lam[k] || mu[(int64_t)y * nx] != mu[k])) row_varies[y] = 1;
  }
  return hipSuccess;
}
template <typename real>
hipError_t launch_kappa_range(const real *kappa, int nx, int ny, int pitch, real *minmax, int nblocks, hipStream_t) {
  if (nblocks < 1 || nblocks > 1024) { fprintf(stderr, "kappa range blocks %d\n", nblocks); abort(); }
  check_range(kappa, sizeof(real) * (size_t)pitch * ny, "kappa range in");
  check_range(minmax, sizeof(real) * 2 * nblocks, "kappa range out");
  real lo = kappa[0], hi = kappa[0];
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) { lo = std::min(lo, kappa[(int64_t)y * pitch + x]); hi = std::max(hi, kappa[(int64_t)y * pitch + x]); }
  for (int b = 0; b < nblocks; ++b) { minmax[2 * b] = lo; minmax[2 * b + 1] = hi; }
  return hipSuccess;
}
template <typename real>
hipError_t launch_kappa_rows(const real *kappa, int ny, int pitch, real *rows, hipStream_t) {
  check_range(rows, ny * sizeof(real), "krows"); for (int y = 0; y < ny; ++y) rows[y] = kappa[(int64_t)y * pitch]; return hipSuccess;
}
template <typename real>
hipError_t launch_gather(const real *src, const int64_t *idx, int n, real *dst, hipStream_t) {
  for (int i = 0; i < n; ++i) { check_range(src + idx[i], sizeof(real), "gather"); dst[i] = src[idx[i]]; } return hipSuccess;
}
template <typename real>
hipError_t launch_count_nonfinite(const real *f, int64_t n, int *count, hipStream_t) { check_range(f, n * sizeof(real), "nonfinite"); return hipSuccess; }
template <typename real>
hipError_t launch_finite_watch(const real *f, int64_t n, int64_t, int64_t *first_bad, hipStream_t) {
  check_range(f, n * sizeof(real), "finite watch");
  if (!first_bad) { fprintf(stderr, "finite watch without a flag\n"); abort(); }
  return hipSuccess;
}
// the scratch-backed finite check: every grid's populations inside the
// descriptor table's ranges; no scratch exists here, so it reports none
template <typename real>
hipError_t check_nonfinite_scratch(const real *f, const GridDev *grids, int nbatch, int64_t max_elems,
                                   hipStream_t, uint32_t out[2]) {
  if (nbatch < 1 || nbatch > kScratchGrids) return hipErrorInvalidValue;
  check_range(grids, sizeof(GridDev) * nbatch, "scratch grids");
  for (int g = 0; g < nbatch; ++g) {
    if (9 * (int64_t)grids[g].pitch * grids[g].ny > max_elems) { fprintf(stderr, "max_elems too small\n"); abort(); }
    check_range(f + grids[g].f_off, sizeof(real) * 9 * (size_t)grids[g].pitch * grids[g].ny, "scratch check");
  }
  out[0] = 0u;
  out[1] = 0xffffffffu;
  return hipSuccess;
}
template <typename real>
hipError_t launch_copy_planes(const real *src, int64_t sps, int64_t sys, real *dst, int64_t dps, int64_t dys, int nx, int ny, int np, hipStream_t) {
  for (int p = 0; p < np; ++p) for (int y = 0; y < ny; ++y) {
    check_range(src + p * sps + y * sys, nx * sizeof(real), "copy src"); check_range(dst + p * dps + y * dys, nx * sizeof(real), "copy dst");
    memcpy(dst + p * dps + y * dys, src + p * sps + y * sys, nx * sizeof(real));
  }
  return hipSuccess;
}
hipError_t launch_set_time(int64_t *t, int64_t v, hipStream_t) { check_range(t, 8, "time"); *t = v; return hipSuccess; }
hipError_t launch_add_time(int64_t *t, int64_t v, hipStream_t) { check_range(t, 8, "time"); *t += v; return hipSuccess; }

#define INST(real) \
  template hipError_t launch_step<real>(const StepArgs<real> &, int, int, int, int, hipStream_t); \
  template hipError_t launch_interior<real>(const StepArgs<real> &, int, int, int, hipStream_t); \
  template hipError_t launch_fused2<real>(const StepArgs<real> &, int, int, hipStream_t); \
  template hipError_t launch_fused3<real>(const StepArgs<real> &, int, int, hipStream_t); \
  template hipError_t launch_filter<real>(const real *, real *, const GridDev *, const TileDev *, int, real, hipStream_t); \
  template hipError_t launch_adjoint<real>(const AdjArgs<real> &, int, int, hipStream_t); \
  template hipError_t launch_adjoint_interior<real>(const AdjArgs<real> &, int, int, hipStream_t); \
  template hipError_t launch_adjoint_fused2<real>(const AdjArgs<real> &, int, int, hipStream_t); \
  template hipError_t launch_misfit<real>(const real *, const real *, real *, int64_t, double *, double *, hipStream_t); \
  template hipError_t launch_lame_gradient<real>(const real *, const real *, const double *, double *, double *, int64_t, hipStream_t); \
  template hipError_t launch_kappa<real>(const real *, const real *, const real *, int, int, int, real *, int *, int *, hipStream_t); \
  template hipError_t launch_kappa_rows<real>(const real *, int, int, real *, hipStream_t); \
  template hipError_t launch_kappa_range<real>(const real *, int, int, int, real *, int, hipStream_t); \
  template hipError_t launch_gather<real>(const real *, const int64_t *, int, real *, hipStream_t); \
  template hipError_t launch_count_nonfinite<real>(const real *, int64_t, int *, hipStream_t); \
  template hipError_t check_nonfinite_scratch<real>(const real *, const GridDev *, int, int64_t, hipStream_t, uint32_t *); \
  template hipError_t launch_finite_watch<real>(const real *, int64_t, int64_t, int64_t *, hipStream_t); \
  template hipError_t launch_copy_planes<real>(const real *, int64_t, int64_t, real *, int64_t, int64_t, int, int, int, hipStream_t);
INST(float)
INST(double)
}  // namespace lbm
