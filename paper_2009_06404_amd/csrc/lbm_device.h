// Device helpers shared by the forward step kernels (lbm_kernels.hip) and the
// adjoint kernels (lbm_adjoint.hip): the D2Q9 tables, the row and column
// classification of the wall rules, population addressing, raw buffer
// accesses, the source wavelet and the per-cell coefficient and sponge
// look-ups. Not part of the public ABI.
#pragma once

#include "lbm_internal.h"

namespace lbm {
namespace dev {

constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// v / 36 for the integer-coefficient combinations: 1/36 split into a
// rounded head and the rounded remainder, hi + lo = 1/36 to about twice the
// working precision, and v*hi + v*lo formed with a single rounding (the
// small v*lo is added inside the FMA). The quotient is the correctly
// rounded one except in rare near-ties, so it carries no systematic bias
// (a bare multiply by the rounded 1/36 would scale every equilibrium term
// by the same 1 + delta).
template <typename real>
struct Inv36;
template <>
struct Inv36<float> {
  static constexpr float hi = 0x1.c71c72p-6f, lo = -0x1.c71c72p-33f;
};
template <>
struct Inv36<double> {
  static constexpr double hi = 0x1.c71c71c71c71cp-6, lo = 0x1.c71c71c71c71cp-60;
};
template <typename real>
__device__ __forceinline__ real div36(real v) {
  return fma(v, Inv36<real>::hi, v * Inv36<real>::lo);
}

// Row classification for the pull of row y (uniform across the workgroup).
struct Row {
  int y;
  int up, dn;           // source rows of links arriving with c_y = +1 / -1
  int wall_up, wall_dn; // 0, kFree, kFree0 or kRigid: the wall those links cross
};

__device__ __forceinline__ Row make_row(const GridDev &g, int y) {
  Row r;
  r.y = y;
  r.wall_up = 0;
  r.wall_dn = 0;
  r.up = y - 1;
  r.dn = y + 1;
  if (y == 0) {
    if (g.bc[kEdgeTop] == kPeriodic) r.up = g.ny - 1;
    else { r.wall_up = g.bc[kEdgeTop]; r.up = y; }
  } else if (y == g.rigid_row) {
    r.wall_up = kRigid;
    r.up = y;
  }
  if (y == g.ny - 1) {
    if (g.bc[kEdgeBottom] == kPeriodic) r.dn = 0;
    else { r.wall_dn = g.bc[kEdgeBottom]; r.dn = y; }
  } else if (g.rigid_row > 0 && y == g.rigid_row - 1) {
    r.wall_dn = kRigid;
    r.dn = y;
  }
  return r;
}

// The row after y in the marching order, or -1 past a non-periodic bottom.
__device__ __forceinline__ int row_after(const GridDev &g, int y) {
  if (y + 1 < g.ny) return y + 1;
  return g.bc[kEdgeBottom] == kPeriodic ? 0 : -1;
}

// Column classification for one lane (left/right edges: periodic or rigid).
struct Col {
  int x, xl, xr;  // own column, source column for c_x = +1 and c_x = -1
  bool wl, wr;    // links with c_x = +1 / -1 cross a rigid edge
};

__device__ __forceinline__ Col make_col(const GridDev &g, int x) {
  Col c;
  c.x = x;
  c.wl = false;
  c.wr = false;
  c.xl = x - 1;
  c.xr = x + 1;
  if (x == 0) {
    if (g.bc[kEdgeLeft] == kPeriodic) c.xl = g.nx - 1;
    else { c.wl = true; c.xl = x; }
  }
  if (x == g.nx - 1) {
    if (g.bc[kEdgeRight] == kPeriodic) c.xr = 0;
    else { c.wr = true; c.xr = x; }
  }
  return c;
}

// Offset of population i of cell (x, y): rows of nine population runs.
__device__ __forceinline__ int64_t qidx(const GridDev &g, int i, int y, int x) {
  return ((int64_t)y * 9 + i) * g.pitch + x;
}

template <typename real>
__device__ __forceinline__ real sum9(const real f[9]) {
  return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

__device__ __forceinline__ double ricker(double t, double period, double t0) {
  const double a = 3.14159265358979323846 * (t - t0) / period;
  return (1.0 - 2.0 * a * a) * exp(-a * a);
}

__device__ __forceinline__ double min_image(double d, int n, bool periodic) {
  if (periodic) {
    if (d > 0.5 * n) d -= n;
    else if (d < -0.5 * n) d += n;
  }
  return d;
}

// Raw buffer access: the tile's rows live behind one buffer descriptor
// (scalar registers), row and population select a scalar byte offset, and
// the lane's column a 32-bit vector byte offset, so the interior loads and all
// stores carry no per-row vector address arithmetic. 0x00020000 is the
// descriptor's format word for raw accesses on gfx9-family targets.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, 0x7fffffff, 0x00020000);
}

// Buffer descriptor covering [base, base + bytes) (capped at 4 GiB - 1):
// accesses past the end read zero and drop their stores instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t range_rsrc(const void *base, uint64_t bytes) {
  const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)n, 0x00020000);
}

// Cache policy of the raw buffer stores (gfx950 bits): kStoreNT marks the
// populations non-temporal; kStoreNTDevice adds the device scope (sc1). The
// two-dimensional forward kernels store faster with both: 240.0 against
// 237.5 us per two-step launch at 4096^2 FP32, 150.5 against 154.2 GLUPS at
// 16384^2, FP64 73.3-73.8 against 74.1. The adjoint, filter and 3-D kernels
// measured no gain (0.4-1.7% slower) and keep kStoreNT.
constexpr int kStoreNT = 2, kStoreNTDevice = 18;

template <typename real>
struct Buf;

template <>
struct Buf<float> {
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  static __device__ __forceinline__ void store_nt(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                  uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, kStoreNT);
  }
  static __device__ __forceinline__ void store_nt_device(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                         uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, kStoreNTDevice);
  }
};

template <>
struct Buf<double> {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  static __device__ __forceinline__ void store_nt(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                  uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, kStoreNT);
  }
  static __device__ __forceinline__ void store_nt_device(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                         uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, kStoreNTDevice);
  }
};

// Pair access for the kernels with two columns per lane: two consecutive
// elements of one population run (dword-aligned multi-dword buffer accesses;
// stores with the two-dimensional forward kernels' policy, kStoreNTDevice).
template <typename real>
struct Pair {
  real a, b;
};

template <typename real>
struct Buf2;

template <>
struct Buf2<float> {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ Pair<float> load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                     uint32_t soff) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return {__uint_as_float(v.x), __uint_as_float(v.y)};
  }
  static __device__ __forceinline__ void store_nt(float a, float b, __amdgpu_buffer_rsrc_t r,
                                                  uint32_t voff, uint32_t soff) {
    u32x2 v;
    v.x = __float_as_uint(a);
    v.y = __float_as_uint(b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, kStoreNTDevice);
  }
};

template <>
struct Buf2<double> {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ Pair<double> load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                      uint32_t soff) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    u32x2 lo, hi;
    lo.x = v.x; lo.y = v.y;
    hi.x = v.z; hi.y = v.w;
    return {__builtin_bit_cast(double, lo), __builtin_bit_cast(double, hi)};
  }
  static __device__ __forceinline__ void store_nt(double a, double b, __amdgpu_buffer_rsrc_t r,
                                                  uint32_t voff, uint32_t soff) {
    const u32x2 lo = __builtin_bit_cast(u32x2, a), hi = __builtin_bit_cast(u32x2, b);
    u32x4 v;
    v.x = lo.x; v.y = lo.y; v.z = hi.x; v.w = hi.y;
    __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, kStoreNTDevice);
  }
};

// Elastic coefficient of cell (x, y).
template <typename real>
__device__ __forceinline__ real cell_kappa(const real *kappa_rows, const real *kappa_cells,
                                           const GridDev &g, int y, int x) {
  if (g.kmode == kKappaScalar) return (real)g.kscalar;
  if (g.kmode == kKappaRows) return kappa_rows[g.k_off + y];
  return kappa_cells[g.k_off + (int64_t)y * g.pitch + x];
}

// The fields of a grid descriptor that the per-cell look-ups read, moved to
// scalar registers (the descriptor is uniform across the workgroup). A loop
// that stores to memory otherwise keeps re-reading them, or keeps them in
// vector registers whose loads the compiler cannot prove complete inside the
// loop, and waits for all outstanding loads at every use.
__device__ __forceinline__ int32_t sreg(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t sreg(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double sreg(double v) {
  return __builtin_bit_cast(double, sreg(__builtin_bit_cast(int64_t, v)));
}
__device__ __forceinline__ GridDev uniform_lookup_fields(const GridDev &src) {
  GridDev g;
  g.nx = sreg(src.nx);
  g.ny = sreg(src.ny);
  g.pitch = sreg(src.pitch);
  g.kmode = sreg(src.kmode);
  g.f_off = sreg(src.f_off);
  g.kscalar = sreg(src.kscalar);
  g.k_off = sreg(src.k_off);
  g.c_off = sreg(src.c_off);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    g.bc[e] = sreg(src.bc[e]);
    g.sp_thick[e] = sreg(src.sp_thick[e]);
    g.sp_off[e] = sreg(src.sp_off[e]);
  }
  return g;
}

// Sponge pair (A, 1/(1 + A/2)) along x for column x (left/right layers). The
// table holds the pairs; the second decreases with the first, so the largest
// A of overlapping layers pairs with the smallest reciprocal.
template <typename real>
__device__ __forceinline__ void sponge_x(const real *sponge, const GridDev &g, int x, real &A,
                                         real &inv) {
  A = real(0);
  inv = real(1);
  const int dl = x, dr = g.nx - 1 - x;
  if (dl < g.sp_thick[kEdgeLeft]) {
    A = sponge[g.sp_off[kEdgeLeft] + 2 * dl];
    inv = sponge[g.sp_off[kEdgeLeft] + 2 * dl + 1];
  }
  if (dr < g.sp_thick[kEdgeRight]) {
    A = max(A, sponge[g.sp_off[kEdgeRight] + 2 * dr]);
    inv = min(inv, sponge[g.sp_off[kEdgeRight] + 2 * dr + 1]);
  }
}

// Add the top/bottom layers of row y to a column's sponge pair.
template <typename real>
__device__ __forceinline__ void sponge_y(const real *sponge, const GridDev &g, int y, real &A,
                                         real &inv) {
  const int dt_ = y, db = g.ny - 1 - y;
  if (dt_ < g.sp_thick[kEdgeTop]) {
    A = max(A, sponge[g.sp_off[kEdgeTop] + 2 * dt_]);
    inv = min(inv, sponge[g.sp_off[kEdgeTop] + 2 * dt_ + 1]);
  }
  if (db < g.sp_thick[kEdgeBottom]) {
    A = max(A, sponge[g.sp_off[kEdgeBottom] + 2 * db]);
    inv = min(inv, sponge[g.sp_off[kEdgeBottom] + 2 * db + 1]);
  }
}

}  // namespace dev
}  // namespace lbm
