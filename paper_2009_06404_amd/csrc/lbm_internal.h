// Internal device-side descriptors shared by the kernels and the host API of
// liblbm.so. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D2Q9, direction order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
constexpr int kQ = 9;
constexpr int kEdgeTop = 0, kEdgeBottom = 1, kEdgeLeft = 2, kEdgeRight = 3;
constexpr int kPeriodic = 0, kFree = 1, kRigid = 2, kFree0 = 3;
constexpr int kKappaScalar = 0, kKappaRows = 1, kKappaCells = 2;

// One grid of a (possibly batched) context. Offsets are in elements of the
// context's dtype unless stated otherwise.
// Populations of a grid: population i of cell (x, y) at
// f_off + (y * 9 + i) * pitch + x of a population buffer.
struct GridDev {
  int32_t nx, ny, pitch, kmode;   // pitch: elements per stored population run
  int64_t f_off;                  // offset of the grid inside a population buffer
  int64_t plane;                  // ny * pitch (size of the kappa cell plane)
  int32_t bc[4];
  int32_t rigid_row;              // -1 none
  int32_t nsrc, src_off;          // sources [src_off, src_off + nsrc)
  int32_t nrec;                   // receivers of this grid
  double kscalar;                 // kappa when kmode == scalar
  int64_t k_off;                  // kappa rows: offset into the row table;
                                  // kappa cells: offset into the cell plane
  int32_t sp_thick[4];
  int32_t sp_off[4];              // offsets into the sponge profile table
  int64_t rowtab_off;             // int table: ny entries, receiver row slot or -1
  int64_t rmap_off;               // int table: slots * nx entries, receiver id or -1
  int64_t rnext_off;              // int table: nrec entries, next receiver in the same cell
  int64_t rscale_off;             // real table: 1/rho0 per receiver
  void *trace;                    // [max_steps][nrec][ncomp] of dtype
  int64_t trace_t0, trace_max;
  int32_t ncomp, comp_mask;
  int64_t c_off;                  // offset of the grid in a packed plane of one value
                                  // per cell (same pitch), e.g. the density stash
};

struct SourceDev {
  double x, y, sigma, dir_x, dir_y, amp, period, t0;
};

// A tile is one workgroup's work: grid g, columns [x0, x0 + 64*waves),
// rows [y0, y1).
struct TileDev {
  int32_t g, x0, y0, y1;
};

// Largest block height of the two-step kernel (its per-row table in LDS).
constexpr int kFusedMaxRows = 248;

// A tile of the two-step kernel: grid g, columns [x0, x1) with
// 0 < x1 - x0 <= 64*NW, rows [y0, y1) with y1 - y0 <= kFusedMaxRows.
struct FusedTileDev {
  int32_t g, x0, x1, y0, y1;
};

template <typename real>
struct StepArgs {
  const real *fin;       // state f*(t-1), all grids
  real *fout;            // state f*(t)
  const GridDev *grids;
  const TileDev *tiles;
  const real *kappa_rows;
  const real *kappa_cells;
  const real *sponge;
  const SourceDev *sources;
  const int32_t *itab;
  const real *rtab;
  int64_t t;             // step index (plus *t_dev when t_dev is set)
  const int64_t *t_dev;  // device time base used by captured graphs, or null
  real omega;            // 1 / tau
  real cforce;           // 1 - 1/(2 tau)
  real *mom;             // moments mode: [6][ny][nx] of grid mom_grid
  int32_t mom_grid;
  real *rho_out;         // stash mode: rho(t) of every cell at c_off + y * pitch + x
  real *rho_out2;        // two-step kernel in stash mode: rho(t+1), same layout
  const FusedTileDev *ftiles;  // two-step kernel: its tiles
  real *fmid;            // two-step path: the pair's intermediate buffer f*(t), fout of its
                         // first general launch and fin of its second (set on each launch of
                         // a pair so the host-side checks can tell them apart; no kernel reads it)
  int64_t f_elems;       // elements of one population buffer (bounds of fin/fout)
  int32_t tri_step;      // three-step path: 1, 2 or 3 on the general kernel's launches of a
                         // triple, 0 otherwise (for the host-side checks; no kernel reads it)
};

// kModeStash: the step plus the density of every cell written to rho_out,
// without the receivers (the forward recompute of the adjoint). kModeStep
// with rho_out set writes the densities too, receivers included (a recorded
// forward step whose densities the adjoint keeps).
enum Mode { kModeStep = 0, kModeMoments = 1, kModeStash = 2 };

// The adjoint's per-grid inputs and outputs (device pointers, caller-owned).
struct AdjGridDev {
  const void *residual;   // e(t) in the traces' layout [steps][nrec][ncomp], or null
  double *grad_kappa;     // [ny][nx] dL/dkappa, accumulated, or null
  double *grad_amp;       // [nsrc] dL/damp, accumulated, or null
};

constexpr int kMaxAdjSources = 16;   // sources per grid with an amplitude gradient

template <typename real>
struct AdjArgs {
  const real *fin;        // fh(t+1), all grids (population-buffer layout)
  real *fout;             // fh(t)
  const GridDev *grids;
  const AdjGridDev *io;
  const TileDev *tiles;
  const real *kappa_rows;
  const real *kappa_cells;
  const real *sponge;
  const SourceDev *sources;
  const int32_t *itab;
  const real *rtab;
  const real *rho;        // rho(t) of every cell (stash layout), for the gradient
  int64_t t;
  real omega, cforce;
  // two adjoint steps per pass (adjoint_fused2_kernel): its blocks, rho(t-1)
  // of every cell, and the size of one population buffer (elements)
  const FusedTileDev *ftiles;
  const real *rho2;
  int64_t f_elems;
  // the general kernel's per-workgroup dL/damp sums: kMaxAdjSources doubles
  // at the workgroup's index (read by launch_amp_reduce)
  double *amp_part;
};

template <typename real>
hipError_t launch_adjoint(const AdjArgs<real> &a, int waves, int ntiles, hipStream_t stream);
// Interior tiles whose rows y0-1 .. y1 also hold no receiver.
template <typename real>
hipError_t launch_adjoint_interior(const AdjArgs<real> &a, int waves, int ntiles,
                                   hipStream_t stream);
// Two adjoint steps (t and t-1) of the blocks a.ftiles in one pass, from
// fh(t+1) in a.fin to fh(t-1) in a.fout, with rho(t) in a.rho and rho(t-1)
// in a.rho2; blocks of 64 * waves columns (waves 2, 4 or 8).
template <typename real>
hipError_t launch_adjoint_fused2(const AdjArgs<real> &a, int waves, int ntiles,
                                 hipStream_t stream);
// Tiles of the first general launch of an adjoint pair that are border
// strips of two-step blocks carry this bit in their grid index: they advance
// the adjoint state only, the gradients of their cells being the two-step
// kernel's.
constexpr int32_t kStripTile = 1 << 30;
// Adds to grad_amp of each listed (grid, source) pair (pairs: g, si) the
// partial sums part[tiles[i] * kMaxAdjSources + si], i in off[k] .. off[k+1],
// in that order.
hipError_t launch_amp_reduce(const double *part, const int32_t *tiles, const int32_t *off,
                             const int32_t *pairs, int npairs, const AdjGridDev *io,
                             hipStream_t stream);
// The misfit's per-workgroup sums go to part (at least kMisfitParts doubles)
// and are then added to *misfit in order.
constexpr int kMisfitParts = 4096;
template <typename real>
hipError_t launch_misfit(const real *trace, const real *d_obs, real *residual, int64_t n,
                         double *misfit, double *part, hipStream_t stream);
template <typename real>
hipError_t launch_lame_gradient(const real *lam, const real *mu, const double *grad_kappa,
                                double *grad_lam, double *grad_mu, int64_t n, hipStream_t stream);

template <typename real>
hipError_t launch_step(const StepArgs<real> &a, int waves, int prefetch, int ntiles, int mode,
                       hipStream_t stream);

// Two steps (t and t+1) of the interior tiles in a.ftiles: reads a.fin =
// f*(t-1), writes a.fout = f*(t+1) (f*(t) stays on chip);
// with a.rho_out set also rho(t) and rho(t+1) of its cells to a.rho_out and
// a.rho_out2.
template <typename real>
hipError_t launch_fused2(const StepArgs<real> &a, int waves, int ntiles, hipStream_t stream);

// Three steps (t, t+1, t+2) of the interior tiles in a.ftiles: reads a.fin =
// f*(t-1), writes a.fout = f*(t+2); tiles of 64 x waves columns (2 or 4).
template <typename real>
hipError_t launch_fused3(const StepArgs<real> &a, int waves, int ntiles, hipStream_t stream);

// The high-wavenumber filter (lbm_filter.hip): fout = fin - sigma (d4x + d4y)
// fin for the cells of the 256-column tiles in tiles.
template <typename real>
hipError_t launch_filter(const real *fin, real *fout, const GridDev *grids, const TileDev *tiles,
                         int ntiles, real sigma, hipStream_t stream);

// Interior tiles; with a.rho_out set, the one-column kernel also writes rho(t).
template <typename real>
hipError_t launch_interior(const StepArgs<real> &a, int waves, int pair, int ntiles,
                           hipStream_t stream);

// Initialisation and utility kernels (lbm_util.hip).
template <typename real>
hipError_t launch_kappa(const real *lam, const real *mu, const real *rho, int nx, int ny,
                        int pitch, real *kappa, int *bad, int *row_varies,
                        hipStream_t stream);
template <typename real>
hipError_t launch_kappa_rows(const real *kappa, int ny, int pitch, real *rows,
                             hipStream_t stream);
template <typename real>
hipError_t launch_gather(const real *src, const int64_t *idx, int n, real *dst,
                         hipStream_t stream);
template <typename real>
hipError_t launch_count_nonfinite(const real *f, int64_t n, int *count, hipStream_t stream);
// The periodic finite check of lbm_step: records t in *first_bad (mapped host
// memory, -1 while none) when the n values at f hold NaN or Inf and no time
// is recorded yet.
template <typename real>
hipError_t launch_finite_watch(const real *f, int64_t n, int64_t t, int64_t *first_bad,
                               hipStream_t stream);
// The finite check in the library's static device scratch (no allocation):
// grids [nbatch] is the device descriptor table, at most kScratchGrids grids,
// max_elems the largest grid's population count (9 x pitch x ny). On return
// (the stream synchronised) out[0] holds the number of grids whose state
// holds NaN or Inf and out[1] the lowest such grid index (0xffffffff if none).
constexpr int kScratchGrids = 4096;
template <typename real>
hipError_t check_nonfinite_scratch(const real *f, const GridDev *grids, int nbatch,
                                   int64_t max_elems, hipStream_t stream, uint32_t out[2]);
template <typename real>
hipError_t launch_copy_planes(const real *src, int64_t src_ps, int64_t src_ys, real *dst,
                              int64_t dst_ps, int64_t dst_ys, int nx, int ny, int nplanes,
                              hipStream_t stream);
// Per-block minimum and maximum of the kappa cells of one grid:
// minmax[2*b], minmax[2*b+1] for b < nblocks (nblocks <= 1024).
template <typename real>
hipError_t launch_kappa_range(const real *kappa, int nx, int ny, int pitch, real *minmax,
                              int nblocks, hipStream_t stream);
hipError_t launch_set_time(int64_t *t_dev, int64_t value, hipStream_t stream);

// Largest von Neumann amplification factor of one step of the bulk scheme
// over an nk x nk grid of wavenumbers in [0, pi]^2 (lbm_stability.cpp).
double vn_growth(double nu, double tau, int nk);
// The same for `every` steps followed by the filter of strength sigma, per step.
double vn_growth_filtered(double nu, double tau, double sigma, int every, int nk);
hipError_t launch_add_time(int64_t *t_dev, int64_t delta, hipStream_t stream);

}  // namespace lbm
