// Internal descriptors of the three-dimensional (D3Q19 / D3Q27) step, shared
// by its kernels and its host API. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm3 {

constexpr int kQ19 = 19, kQ27 = 27;   // the two velocity sets
constexpr int kFaceTop = 0, kFaceBottom = 1, kFaceLeft = 2, kFaceRight = 3, kFaceFront = 4,
              kFaceBack = 5;
constexpr int kPeriodic = 0, kFree = 1, kRigid = 2, kFree0 = 3;
constexpr int kMaxSources = 256;

struct Src3Dev {
  double x, y, z, sigma, dir_x, dir_y, dir_z, amp, period, t0;
};

// One volume on the q-velocity set. Populations: population i of cell
// (x, y, z) at z * zplane + (y * q + i) * pitch + x of a population buffer;
// kappa of the cell at (z * ny + y) * pitch + x of the kappa plane.
struct Vol3Dev {
  int32_t nx, ny, nz, pitch;
  int32_t q;               // 19 or 27
  int32_t face[6];
  int32_t kcells;          // 1: kappa per cell, 0: kscalar
  int32_t nsrc;
  double kscalar;
  double omega;            // 1 / tau
  int64_t zplane;          // ny * q * pitch
  const void *kappa;       // real plane (kcells)
  const void *damp;        // real [nx + ny + nz]: sponge damping per x, then y, then z
  const Src3Dev *src;
  // receivers, sorted by (z, y, x): rec_row[z * ny + y] .. rec_row[z * ny + y + 1]
  const int32_t *rec_row;  // nz * ny + 1 entries, or null without receivers
  const int32_t *rec_plane;// nz flags: the plane holds receivers
  const int32_t *rec_x;    // x of each sorted receiver
  const int32_t *rec_id;   // its index in the caller's list
  const void *rec_scale;   // real 1 / rho0 per sorted receiver
  void *trace;             // [trace_max][nrec][ncomp] of dtype
  int64_t trace_t0, trace_max;
  int32_t nrec, comp_mask;
};

// One workgroup's work: columns [x0, x0 + tx) (tx = 64, or 128 for wide lean
// tiles) and rows [y0, y0 + rows_y) of the volume (clipped to it), planes
// [z0, z1).
struct Tile3Dev {
  int32_t x0, y0, z0, z1;
};

// Launchers return the hipError_t of the launch (0 on success).

// Launch of one pass over the tiles of a list. mode 0: a step (fin -> fout);
// mode 1: the macroscopic fields of fin's time into out10 (dense
// [10][nz][ny][nx]). general = false: the lean kernel, for tiles none of whose
// pulled cells lies on a non-periodic face and which hold no receiver cell;
// with src = false their cells are also beyond every source's reach, with
// src = true (mode 0 only) the lean kernel adds the sources' body force.
// general = true: the kernel with every rule (mode 1 always; src must be
// false). tx: tile width, 64, or 128 for the lean FP32 steps in tiles of 2 or
// 6 rows (hipErrorInvalidValue otherwise).
int launch_step3(bool f64, bool general, bool src, int rows_y, int tx, const Tile3Dev *tiles,
                 int ntiles, const void *fin, void *fout, void *out10, const Vol3Dev &v, int64_t t,
                 int mode, hipStream_t s);

// kappa = b^2 (mu - lambda) / mu into the kappa plane. The count of cells
// outside 0 <= nu < 1/2, mu > 0, rho > 0 (NaN included) is added to *bad
// (zeroed by the caller); block b of the *nblocks <= kKappaBlocks launched
// writes the min / max of its kappa values to minmax[2b], minmax[2b + 1].
constexpr int kKappaBlocks = 1024;
int launch_kappa3(bool f64, const void *lam, const void *mu, const void *rho, void *kappa,
                  int nx, int ny, int nz, int pitch, unsigned int *bad, double *minmax,
                  int *nblocks, hipStream_t s);

// out[k] = 1 / rho[z*ny*nx + y*nx + x] for the k-th (x, y, z) triple.
int launch_gather_inv3(bool f64, const void *rho, const int32_t *xyz, int n, int nx, int ny,
                       void *out, hipStream_t s);

// Largest von Neumann amplification factor of the bulk step on the q-velocity
// set over an nk^3 grid of wavenumbers in [0, pi]^3 (host code).
double vn_growth3(int q, double nu, double tau, int nk);

// Dense [q][nz][ny][nx] <-> pitched population buffer.
int launch_pack3(bool f64, int q, const void *src, void *dst, int nx, int ny, int nz, int pitch,
                 bool to_pitched, hipStream_t s);

}  // namespace lbm3
