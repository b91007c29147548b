// D3Q19 / D3Q27 elastic-wave step on gfx950: one kernel per step (or per
// evaluation of the macroscopic fields), HBM-bound at 2 x Q population words
// per cell. Q, the velocity set, is a template parameter of every kernel.
//
// Work decomposition. A workgroup owns a tile of TX columns (64, or 128 for
// the wide FP32 lean tiles) by TY rows and a segment of planes in z, and
// marches the segment plane by plane. It runs TX x (TY + 2) lanes: lane
// (lx, ly) with 1 <= ly <= TY owns cell (x0 + lx, y0 + ly - 1); the rows
// ly = 0 and TY + 1 are halo lanes that compute the density of the rows just
// outside the tile (and, in their first TY lanes, of the columns just left
// and right of it). The density of each plane is gathered in a
// (TY + 2) x (TX + 2) LDS tile, double-buffered by plane parity, for the x
// and y differences of eq. FDrho; the z difference uses the
// density of the planes before and after, kept in registers. Each lane pulls
// the populations of plane z + 1 (streaming of eq. LBGK, with the face rules)
// while the tile's LDS holds plane z, so one barrier per plane suffices.
//
// Addressing: the three planes a pull reads are uniform base pointers; within
// a plane, 32-bit element offsets (y * 19 + i) * pitch + x.
#include <hip/hip_runtime.h>

#include "lbm3d_internal.h"
#include "lbm_device.h"

namespace lbm3 {
namespace {

// Velocities in the order of the public header: D3Q19 is the first 19 of
// D3Q27's. Weights by speed class.
__host__ __device__ constexpr int cxv(int i) {
  constexpr int t[kQ27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                           1, -1, 1, -1, 1, -1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int cyv(int i) {
  constexpr int t[kQ27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                           1, -1, 1, -1, -1, 1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int czv(int i) {
  constexpr int t[kQ27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                           1, -1, -1, 1, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int oppv(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr int speed2(int i) {
  return cxv(i) * cxv(i) + cyv(i) * cyv(i) + czv(i) * czv(i);
}

template <typename real, int Q>
__device__ __forceinline__ real wgt(int i) {
  if (Q == kQ19)
    return speed2(i) == 0 ? real(1) / real(3) : (speed2(i) == 1 ? real(1) / real(18) : real(1) / real(36));
  return speed2(i) == 0 ? real(8) / real(27)
                        : (speed2(i) == 1 ? real(2) / real(27)
                                          : (speed2(i) == 2 ? real(1) / real(54) : real(1) / real(216)));
}

// Link kinds, ordered by precedence: a link that leaves through a rigid face
// bounces back even if it also crosses a free one.
constexpr int kIn = 0, kLinkFree = 1, kLinkRigid = 2;

__device__ __forceinline__ int face_link_kind(int face_kind) {
  return face_kind == kRigid ? kLinkRigid : (face_kind == kPeriodic ? kIn : kLinkFree);
}

__device__ __forceinline__ double ricker3(double t, double period, double t0) {
  const double a = 3.14159265358979323846 * (t - t0) / period;
  return (1.0 - 2.0 * a * a) * exp(-a * a);
}

__device__ __forceinline__ double min_image(double d, int n, bool periodic) {
  if (!periodic) return d;
  const double h = 0.5 * n;
  while (d > h) d -= n;
  while (d < -h) d += n;
  return d;
}

// Pull of a cell none of whose links leaves through a non-periodic face:
// every population arrives from a neighbour (periodic axes already wrapped).
// The three planes sit behind buffer descriptors (scalar registers); a load's
// vector offset is the byte offset of its source row and column inside the
// plane, its scalar offset the population's run (i * pitch elements).
using lbm::dev::Buf;
using rsrc_t = __amdgpu_buffer_rsrc_t;

template <typename real, int Q>
__device__ __forceinline__ real pull_inner(rsrc_t R0, rsrc_t R1, rsrc_t R2, const uint32_t (&xb)[3],
                                           const uint32_t (&rb)[3], uint32_t run, real (&f)[Q]) {
  real rho = real(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int dx = 1 - cxv(i), dy = 1 - cyv(i), dz = 1 - czv(i);
    const rsrc_t R = dz == 0 ? R0 : (dz == 1 ? R1 : R2);
    f[i] = Buf<real>::load(R, rb[dy] + xb[dx], (uint32_t)i * run);
    rho += f[i];
  }
  return rho;
}

// A cell a task of a lane pulls every plane: the byte offsets of its wrapped
// neighbours' columns (x-1, x, x+1) and rows (y-1, y, y+1) inside a plane,
// and the link kind of a source beyond each of its x and y faces (kIn where
// the cell is not on that face or the face is periodic).
struct Task {
  uint32_t xb[3];
  uint32_t rb[3];
  int kx0, kx2, ky0, ky2;
};

template <typename real, int Q>
__device__ __forceinline__ Task make_task(const Vol3Dev &v, int x, int y) {
  Task k;
  const int nx = v.nx, ny = v.ny;
  const uint32_t es = sizeof(real), rp = (uint32_t)(Q * v.pitch) * es;
  k.xb[0] = (uint32_t)(x > 0 ? x - 1 : nx - 1) * es;
  k.xb[1] = (uint32_t)x * es;
  k.xb[2] = (uint32_t)(x < nx - 1 ? x + 1 : 0) * es;
  k.rb[0] = (uint32_t)(y > 0 ? y - 1 : ny - 1) * rp;
  k.rb[1] = (uint32_t)y * rp;
  k.rb[2] = (uint32_t)(y < ny - 1 ? y + 1 : 0) * rp;
  k.kx0 = x == 0 ? face_link_kind(v.face[kFaceLeft]) : kIn;
  k.kx2 = x == nx - 1 ? face_link_kind(v.face[kFaceRight]) : kIn;
  k.ky0 = y == 0 ? face_link_kind(v.face[kFaceFront]) : kIn;
  k.ky2 = y == ny - 1 ? face_link_kind(v.face[kFaceBack]) : kIn;
  return k;
}

// Face rules for a cell some of whose links leave through a non-periodic
// face: f holds what the wrapped pull loaded; the links whose source lies
// beyond a rigid face take the bounce-back f*_opp(i) of the cell itself (eq.
// BB), those beyond a free face (and no rigid one) the anti-bounce-back
// toward the air state (Sec. 6.2): -f*_opp(i) + 2 w_i (rho_air + P^n_air :
// (c_i c_i - b^2 I) / (2 b^4)) with P_air n = 0. The air state's density and
// tangential stress (P_xx, P_xy, P_yy) are the cell's (FREE0) or 3/2 the
// cell's - 1/2 the inner neighbour's (FREE): moments of the post-collision
// populations, which the collision leaves unchanged. Returns the new rho.
template <typename real, int Q>
__device__ __forceinline__ real apply_faces(const Vol3Dev &v, rsrc_t R0, rsrc_t R1, rsrc_t R2,
                                            const Task &T, int kz0, int kz2, uint32_t run,
                                            real (&f)[Q]) {
  const uint32_t own = T.rb[1] + T.xb[1];
  real rho_air = real(0), pxx = real(0), pxy = real(0), pyy = real(0);
  if (kz0 == kLinkFree || kz2 == kLinkFree) {
    const int kind = v.face[kz0 == kLinkFree ? kFaceTop : kFaceBottom];
    const real wb = kind == kFree ? real(1.5) : real(1), wi = kind == kFree ? real(-0.5) : real(0);
    const rsrc_t Rin = kz0 == kLinkFree ? R2 : R0;
    // rolled: few loads in flight on this rare path (free-surface planes)
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      real g = wb * Buf<real>::load(R1, own, (uint32_t)i * run);
      if (kind == kFree) g += wi * Buf<real>::load(Rin, own, (uint32_t)i * run);
      rho_air += g;
      const int cx = cxv(i), cy = cyv(i);
      if (cx != 0) pxx += g;
      if (cy != 0) pyy += g;
      pxy += real(cx * cy) * g;
    }
  }
  const real b2 = real(1) / real(3);
  const real pn_xx = pxx - b2 * rho_air, pn_yy = pyy - b2 * rho_air, pn_zz = -b2 * rho_air;
  real rho = real(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    // the population arrives from x - c_i
    const int kxi = cxv(i) > 0 ? T.kx0 : (cxv(i) < 0 ? T.kx2 : kIn);
    const int kyi = cyv(i) > 0 ? T.ky0 : (cyv(i) < 0 ? T.ky2 : kIn);
    const int kzi = czv(i) > 0 ? kz0 : (czv(i) < 0 ? kz2 : kIn);
    int kind = kxi > kyi ? kxi : kyi;
    kind = kind > kzi ? kind : kzi;
    if (kind != kIn) {
      const real back = Buf<real>::load(R1, own, (uint32_t)oppv(i) * run);
      if (kind == kLinkRigid) {
        f[i] = back;
      } else {
        const real cx = real(cxv(i)), cy = real(cyv(i)), cz = real(czv(i));
        const real q = pn_xx * (cx * cx - b2) + pn_yy * (cy * cy - b2) + pn_zz * (cz * cz - b2) +
                       real(2) * pxy * cx * cy;
        f[i] = -back + real(2) * wgt<real, Q>(i) * (rho_air + real(4.5) * q);
      }
    }
    rho += f[i];
  }
  return rho;
}

// Moments of a cell's pulled populations: the first (m) and the second (P).
template <typename real>
struct Mom3 {
  real mx, my, mz, pxx, pxy, pxz, pyy, pyz, pzz;
};

template <typename real, int Q>
__device__ __forceinline__ Mom3<real> moments3(const real (&f)[Q]) {
  Mom3<real> m;
  m.mx = m.my = m.mz = m.pxx = m.pxy = m.pxz = m.pyy = m.pyz = m.pzz = real(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const real fi = f[i];
    if (cxv(i) != 0) { m.mx += real(cxv(i)) * fi; m.pxx += fi; }
    if (cyv(i) != 0) { m.my += real(cyv(i)) * fi; m.pyy += fi; }
    if (czv(i) != 0) { m.mz += real(czv(i)) * fi; m.pzz += fi; }
    if (cxv(i) * cyv(i) != 0) m.pxy += real(cxv(i) * cyv(i)) * fi;
    if (cxv(i) * czv(i) != 0) m.pxz += real(cxv(i) * czv(i)) * fi;
    if (cyv(i) * czv(i) != 0) m.pyz += real(cyv(i) * czv(i)) * fi;
  }
  return m;
}

// Flux with the implicit sponge (eq. MomentChainAbsorbing): j = (m + G/2) / (1 + A/2).
template <typename real>
__device__ __forceinline__ void flux3(const Mom3<real> &m, real Gx, real Gy, real Gz, real A, real &jx,
                                      real &jy, real &jz) {
  const real inv = real(1) / (real(1) + real(0.5) * A);
  jx = (m.mx + real(0.5) * Gx) * inv;
  jy = (m.my + real(0.5) * Gy) * inv;
  jz = (m.mz + real(0.5) * Gz) * inv;
}

// What the collision of a cell needs besides its populations: rho, j, the
// source S = G - A j, and P^n = P - rho b^2 I (eq. Pn) with its trace part.
template <typename real>
struct Coll3 {
  real rc, jx, jy, jz, Sx, Sy, Sz, nxx, nyy, nzz, pxy, pxz, pyz, btr;
};

template <typename real>
__device__ __forceinline__ Coll3<real> coll3(const Mom3<real> &m, real rc, real jx, real jy, real jz,
                                             real Gx, real Gy, real Gz, real A) {
  Coll3<real> c;
  c.rc = rc;
  c.jx = jx;
  c.jy = jy;
  c.jz = jz;
  c.Sx = Gx - A * jx;
  c.Sy = Gy - A * jy;
  c.Sz = Gz - A * jz;
  const real b2 = real(1) / real(3);
  c.nxx = m.pxx - b2 * rc;
  c.nyy = m.pyy - b2 * rc;
  c.nzz = m.pzz - b2 * rc;
  c.btr = b2 * (c.nxx + c.nyy + c.nzz);
  c.pxy = m.pxy;
  c.pxz = m.pxz;
  c.pyz = m.pyz;
  return c;
}

// Post-collision population i: BGK (eq. LBGK) toward the equilibrium of eq.
// equilibrium-solid, w (rho + j.c / b^2 + P^n:(c c - b^2 I) / (2 b^4)), with
// the source of eq. Si. The products with a zero velocity component are left
// out of the sums (they would add exact zeros): the nonzero terms are summed
// in the order of the full expressions.
template <typename real>
__device__ __forceinline__ void sum_in(real &acc, bool &any, real t) {
  acc = any ? acc + t : t;
  any = true;
}

template <typename real, int Q>
__device__ __forceinline__ real post3(int i, real f, const Coll3<real> &c, real om, real src_w) {
  const int ix = cxv(i), iy = cyv(i), iz = czv(i);
  const real cx = real(ix), cy = real(iy), cz = real(iz);
  // P^n : (c c - b^2 I) = sum of P^n_ab c_a c_b - b^2 tr P^n
  real d = real(0), o = real(0);
  bool hd = false, ho = false;
  if (ix != 0) sum_in(d, hd, c.nxx * cx * cx);
  if (iy != 0) sum_in(d, hd, c.nyy * cy * cy);
  if (iz != 0) sum_in(d, hd, c.nzz * cz * cz);
  if (ix * iy != 0) sum_in(o, ho, c.pxy * cx * cy);
  if (ix * iz != 0) sum_in(o, ho, c.pxz * cx * cz);
  if (iy * iz != 0) sum_in(o, ho, c.pyz * cy * cz);
  if (ho) d = d + real(2) * o;
  const real q = hd ? d - c.btr : -c.btr;
  real jc = real(0), sc = real(0);
  bool hj = false, hs = false;
  if (ix != 0) { sum_in(jc, hj, c.jx * cx); sum_in(sc, hs, c.Sx * cx); }
  if (iy != 0) { sum_in(jc, hj, c.jy * cy); sum_in(sc, hs, c.Sy * cy); }
  if (iz != 0) { sum_in(jc, hj, c.jz * cz); sum_in(sc, hs, c.Sz * cz); }
  const real wi = wgt<real, Q>(i);
  const real feq = hj ? wi * (c.rc + real(3) * jc + real(4.5) * q) : wi * (c.rc + real(4.5) * q);
  const real relaxed = f - om * (f - feq);
  return hs ? relaxed + src_w * wi * real(3) * sc : relaxed;
}

// GENERAL = false: the lean kernel (no face rules, sources or receivers; the
// host gives it only tiles that need none); with SRC it adds the body force of
// the sources (tiles clear of faces and receivers but near a source). MODE 1
// (fields) is general only.
// TX = 128 (lean FP32 tiles only): two wavefronts per row, so a workgroup
// reads each population row of a plane as 512 contiguous bytes, not 256.
template <typename real, int Q, int TY, int MODE, bool GENERAL, int TX = 64, bool SRC = GENERAL>
__global__ void __launch_bounds__(TX * (TY + 2))
step3_kernel(const real *__restrict__ fin, real *__restrict__ fout, real *__restrict__ out10,
             const Vol3Dev v, int64_t t, const Tile3Dev *__restrict__ tiles, int ntiles) {
  __shared__ real srho[2][TY + 2][TX + 2];

  // die-aware order: workgroup b runs on die b % 8; each die takes a
  // contiguous run of the list (ordered by plane segment, row, column), so
  // the tiles sharing halo rows and planes share an L2
  const int per_die = (ntiles + 7) / 8;
  const int lin = (int)(blockIdx.x % 8) * per_die + (int)(blockIdx.x / 8);
  if (lin >= ntiles) return;
  const Tile3Dev tile = tiles[lin];

  const int nx = v.nx, ny = v.ny, nz = v.nz, pitch = v.pitch;
  const int x0 = tile.x0, y0 = tile.y0;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int zb = tile.z0, ze = tile.z1;
  const bool zper = v.face[kFaceTop] == kPeriodic;
  const bool xper = v.face[kFaceLeft] == kPeriodic, yper = v.face[kFaceFront] == kPeriodic;

  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  const bool interior = ly >= 1 && ly <= TY;
  const bool active = interior && lx < w && ly <= h;
  const int x = x0 + lx;
  const int y = y0 + ly - 1;

  // Task A: interior lanes their own cell; the halo rows (ly = 0, TY + 1) the
  // cell just above / below the tile in their column. Task B: in the halo
  // rows' first h lanes, the cell just left / right of the tile in row lx.
  bool hasA = active, hasB = false;
  int ax = x, ay = y, arow = ly, acol = lx + 1;
  int bx = 0, by = 0, brow = 0, bcol = 0;
  if (ly == 0 || ly == TY + 1) {
    const bool top = ly == 0;
    int yy = top ? y0 - 1 : y0 + h;
    if (yy < 0 || yy >= ny) yy = yper ? (yy + ny) % ny : -1;
    hasA = lx < w && yy >= 0;
    ay = yy;
    arow = top ? 0 : h + 1;
    if (lx < h) {
      int xx = top ? x0 - 1 : x0 + w;
      if (xx < 0 || xx >= nx) xx = xper ? (xx + nx) % nx : -1;
      hasB = xx >= 0;
      bx = xx;
      by = y0 + lx;
      brow = lx + 1;
      bcol = top ? 0 : w + 1;
    }
  }
  const int tax = hasA ? ax : 0, tay = hasA ? ay : 0, tbx = hasB ? bx : 0, tby = hasB ? by : 0;

  const real *__restrict__ kap = reinterpret_cast<const real *>(v.kappa);
  const real *__restrict__ damp = reinterpret_cast<const real *>(v.damp);
  real Axy = real(0);
  if (active) {
    const real a = damp[x], b = damp[nx + y];
    Axy = a > b ? a : b;
  }

  const uint32_t run = (uint32_t)pitch * (uint32_t)sizeof(real);   // bytes of one population run
  // pull of task T at plane p (0 <= p < nz)
  auto pull_task = [&](const Task &T, int p, real(&f)[Q]) -> real {
    const int zm = p > 0 ? p - 1 : nz - 1;
    const int zp = p < nz - 1 ? p + 1 : 0;
    const rsrc_t R0 = lbm::dev::tile_rsrc(fin + (int64_t)zm * v.zplane);
    const rsrc_t R1 = lbm::dev::tile_rsrc(fin + (int64_t)p * v.zplane);
    const rsrc_t R2 = lbm::dev::tile_rsrc(fin + (int64_t)zp * v.zplane);
    real rho = pull_inner<real, Q>(R0, R1, R2, T.xb, T.rb, run, f);
    if (GENERAL) {
      const int kz0 = p == 0 ? face_link_kind(v.face[kFaceTop]) : kIn;
      const int kz2 = p == nz - 1 ? face_link_kind(v.face[kFaceBottom]) : kIn;
      if ((T.kx0 | T.kx2 | T.ky0 | T.ky2 | kz0 | kz2) != kIn)
        rho = apply_faces<real, Q>(v, R0, R1, R2, T, kz0, kz2, run, f);
    }
    return rho;
  };

  const real om = real(v.omega), src_w = real(1) - real(0.5) * om;
  real cur[Q], nxt[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) cur[i] = real(0);
  real rp = real(0), rc = real(0), rn = real(0);

  // Plane zl + 1 is pulled while plane zl is updated: task A from plane
  // zb - 1 (its density only) to ze (its density only, for the z difference),
  // task B from zb to ze - 1. Planes beyond a non-periodic face are skipped.
  for (int zl = zb - 2; zl < ze; ++zl) {
    const int p = zl + 1;
    const bool inside = (p >= 0 && p < nz) || zper;
    const int pw = p < 0 ? p + nz : (p >= nz ? p - nz : p);
    const int nslot = p & 1, slot = zl & 1;
    rn = real(0);
    if (hasA && inside && p <= ze) {
      // rebuilt every plane: a few integer operations instead of a dozen
      // registers held across the loop
      int cx_ = tax, cy_ = tay;
      asm volatile("" : "+v"(cx_), "+v"(cy_));
      rn = pull_task(make_task<real, Q>(v, cx_, cy_), pw, nxt);
    }
    if (!active && hasA && p >= zb && p < ze) srho[nslot][arow][acol] = rn;
    if (hasB && p >= zb && p < ze) {
      int cx_ = tbx, cy_ = tby;
      asm volatile("" : "+v"(cx_), "+v"(cy_));
      srho[nslot][brow][bcol] = pull_task(make_task<real, Q>(v, cx_, cy_), pw, nxt);
    }

    if (active && zl >= zb) {
      const int z = zl;
      // centred density differences (eq. FDrho), ghosts beyond non-periodic faces
      real rl = srho[slot][ly][lx], rr = srho[slot][ly][lx + 2];
      real ru = srho[slot][ly - 1][lx + 1], rd = srho[slot][ly + 1][lx + 1];
      if (!xper && x == 0) rl = real(2) * rc - rr;
      if (!xper && x == nx - 1) rr = real(2) * rc - rl;
      if (!yper && y == 0) ru = real(2) * rc - rd;
      if (!yper && y == ny - 1) rd = real(2) * rc - ru;
      real rzm = rp, rzp = rn;
      if (!zper && z == 0) rzm = real(2) * rc - rzp;
      if (!zper && z == nz - 1) rzp = real(2) * rc - rzm;
      const real gx = real(0.5) * (rr - rl), gy = real(0.5) * (rd - ru), gz = real(0.5) * (rzp - rzm);

      const Mom3<real> m = moments3<real, Q>(cur);
      // source G = kappa grad(rho) + F (eq. S, Sec. 5)
      const real kap_c = v.kcells ? kap[((int64_t)z * ny + y) * pitch + x] : real(v.kscalar);
      real Gx = kap_c * gx, Gy = kap_c * gy, Gz = kap_c * gz;
      for (int s = 0; s < (SRC ? v.nsrc : 0); ++s) {
        const Src3Dev sd = v.src[s];
        const double dz = min_image((double)z - sd.z, nz, zper);
        const double cut = 81.0 * sd.sigma * sd.sigma;
        if (dz * dz > cut) continue;
        const double dx = min_image((double)x - sd.x, nx, xper);
        const double dy = min_image((double)y - sd.y, ny, yper);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > cut) continue;
        const double mag = sd.amp * exp(-r2 / (2.0 * sd.sigma * sd.sigma)) *
                           ricker3((double)t, sd.period, sd.t0);
        Gx += real(mag * sd.dir_x);
        Gy += real(mag * sd.dir_y);
        Gz += real(mag * sd.dir_z);
      }
      const real az = damp[nx + ny + z];
      const real A = Axy > az ? Axy : az;
      real jx, jy, jz;
      flux3(m, Gx, Gy, Gz, A, jx, jy, jz);

      if (GENERAL && MODE == 0 && v.rec_row && v.rec_plane[z]) {
        const int64_t row = t - v.trace_t0;
        if (row >= 0 && row < v.trace_max) {
          const int rb = v.rec_row[z * ny + y], re = v.rec_row[z * ny + y + 1];
          const real *sc = reinterpret_cast<const real *>(v.rec_scale);
          real *tr = reinterpret_cast<real *>(v.trace);
          const int nc = __builtin_popcount(v.comp_mask);
          // the row's receivers are sorted by x: binary search for the first
          // at or after this column, then take every one at it
          int lo = rb, hi = re;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (v.rec_x[mid] < x) lo = mid + 1;
            else hi = mid;
          }
          for (int r = lo; r < re && v.rec_x[r] == x; ++r) {
            real *o = tr + (row * v.nrec + v.rec_id[r]) * nc;
            int k = 0;
            if (v.comp_mask & 1) o[k++] = jx * sc[r];
            if (v.comp_mask & 2) o[k++] = jy * sc[r];
            if (v.comp_mask & 4) o[k++] = jz * sc[r];
          }
        }
      }

      if (MODE == 1) {
        const int64_t N = (int64_t)nx * ny * nz;
        real *o = out10 + ((int64_t)z * ny + y) * nx + x;
        o[0] = rc;
        o[N] = jx;
        o[2 * N] = jy;
        o[3 * N] = jz;
        o[4 * N] = m.pxx;
        o[5 * N] = m.pxy;
        o[6 * N] = m.pxz;
        o[7 * N] = m.pyy;
        o[8 * N] = m.pyz;
        o[9 * N] = m.pzz;
      } else {
        const Coll3<real> c = coll3(m, rc, jx, jy, jz, Gx, Gy, Gz, A);
        const rsrc_t O = lbm::dev::tile_rsrc(fout + (int64_t)z * v.zplane);
        const uint32_t own = (uint32_t)(y * Q * pitch + x) * (uint32_t)sizeof(real);
#pragma unroll
        for (int i = 0; i < Q; ++i)
          Buf<real>::store_nt(post3<real, Q>(i, cur[i], c, om, src_w), O, own, (uint32_t)i * run);
      }
    }
    if (active && p >= zb && p < ze) srho[nslot][ly][lx + 1] = rn;
#pragma unroll
    for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    rp = rc;
    rc = rn;
    __syncthreads();
  }
}

template <typename real>
__global__ void kappa3_kernel(const real *__restrict__ lam, const real *__restrict__ mu,
                              const real *__restrict__ rho, real *__restrict__ kappa, int nx,
                              int ny, int nz, int pitch, unsigned int *bad, double *minmax) {
  __shared__ double smin[256], smax[256];
  const int64_t N = (int64_t)nx * ny * nz;
  double lo = 1e300, hi = -1e300;
  unsigned int nbad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double l = (double)lam[k], m = (double)mu[k], r = (double)rho[k];
    const double nu = l / (2.0 * (l + m));
    if (!(m > 0.0) || !(r > 0.0) || !(nu >= 0.0) || !(nu < 0.5)) ++nbad;
    const real kv = real(1) / real(3) * (mu[k] - lam[k]) / mu[k];
    const int64_t x = k % nx, yz = k / nx;
    kappa[yz * pitch + x] = kv;
    lo = fmin(lo, (double)kv);
    hi = fmax(hi, (double)kv);
  }
  if (nbad) atomicAdd(bad, nbad);
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    minmax[2 * blockIdx.x] = smin[0];
    minmax[2 * blockIdx.x + 1] = smax[0];
  }
}

template <typename real>
__global__ void gather_inv3_kernel(const real *__restrict__ rho, const int32_t *__restrict__ xyz,
                                   int n, int nx, int ny, real *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t c = ((int64_t)xyz[3 * k + 2] * ny + xyz[3 * k + 1]) * nx + xyz[3 * k];
  out[k] = real(1) / rho[c];
}

template <typename real>
__global__ void pack3_kernel(const real *__restrict__ src, real *__restrict__ dst, int q, int nx,
                             int ny, int nz, int pitch, int to_pitched) {
  // one row (i, z, y) per block.y index, columns over threads
  const int64_t rowid = blockIdx.y + (int64_t)blockIdx.z * 65535;
  const int64_t nrows = (int64_t)q * nz * ny;
  if (rowid >= nrows) return;
  const int i = (int)(rowid / ((int64_t)nz * ny));
  const int64_t zy = rowid % ((int64_t)nz * ny);
  const int z = (int)(zy / ny), y = (int)(zy % ny);
  const int64_t d = (int64_t)i * nz * ny * nx + zy * nx;
  const int64_t p = (int64_t)z * ny * q * pitch + ((int64_t)y * q + i) * pitch;
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < nx; x += gridDim.x * blockDim.x) {
    if (to_pitched)
      dst[p + x] = src[d + x];
    else
      dst[d + x] = src[p + x];
  }
}

template <typename real, int Q, int TY>
hipError_t launch_tile(bool general, bool src, int tx, const Tile3Dev *tiles, int ntiles,
                       const void *fin, void *fout, void *out10, const Vol3Dev &v, int64_t t,
                       int mode, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (general && src) return hipErrorInvalidValue;   // the general kernel always adds sources
  if (tx == 128) {
    // wide lean tiles: FP32 steps, 2 or 6 rows (at most 1024 lanes)
    if constexpr (sizeof(real) == 4 && TY != 14) {
      if (general || mode != 0) return hipErrorInvalidValue;
      if (src)
        hipLaunchKernelGGL((step3_kernel<real, Q, TY, 0, false, 128, true>), dim3((ntiles + 7) / 8 * 8),
                           dim3(128 * (TY + 2)), 0, s, reinterpret_cast<const real *>(fin),
                           reinterpret_cast<real *>(fout), nullptr, v, t, tiles, ntiles);
      else
        hipLaunchKernelGGL((step3_kernel<real, Q, TY, 0, false, 128>), dim3((ntiles + 7) / 8 * 8),
                           dim3(128 * (TY + 2)), 0, s, reinterpret_cast<const real *>(fin),
                           reinterpret_cast<real *>(fout), nullptr, v, t, tiles, ntiles);
      return hipSuccess;
    }
    return hipErrorInvalidValue;
  }
  // general tiles of 14 rows are never built (the host cuts them to 2 rows):
  // that kernel would spill
  if constexpr (TY == 14) {
    if (general || mode == 1) return hipErrorInvalidValue;
  }
  const dim3 grid((ntiles + 7) / 8 * 8), block(64 * (TY + 2));
  const real *in = reinterpret_cast<const real *>(fin);
  real *out = reinterpret_cast<real *>(fout);
  real *o10 = reinterpret_cast<real *>(out10);
  if constexpr (TY != 14) {
    if (mode == 1) {
      hipLaunchKernelGGL((step3_kernel<real, Q, TY, 1, true>), grid, block, 0, s, in, out, o10, v, t,
                         tiles, ntiles);
      return hipSuccess;
    }
    if (general) {
      hipLaunchKernelGGL((step3_kernel<real, Q, TY, 0, true>), grid, block, 0, s, in, out, o10, v, t,
                         tiles, ntiles);
      return hipSuccess;
    }
  }
  if (mode != 0) return hipErrorInvalidValue;
  if (src)
    hipLaunchKernelGGL((step3_kernel<real, Q, TY, 0, false, 64, true>), grid, block, 0, s, in, out, o10,
                       v, t, tiles, ntiles);
  else
    hipLaunchKernelGGL((step3_kernel<real, Q, TY, 0, false>), grid, block, 0, s, in, out, o10, v, t,
                       tiles, ntiles);
  return hipSuccess;
}

template <typename real, int Q>
hipError_t launch_rows(bool general, bool src, int rows_y, int tx, const Tile3Dev *tiles, int ntiles,
                       const void *fin, void *fout, void *out10, const Vol3Dev &v, int64_t t, int mode,
                       hipStream_t s) {
  if (rows_y == 2)
    return launch_tile<real, Q, 2>(general, src, tx, tiles, ntiles, fin, fout, out10, v, t, mode, s);
  if (rows_y == 14)
    return launch_tile<real, Q, 14>(general, src, tx, tiles, ntiles, fin, fout, out10, v, t, mode, s);
  return launch_tile<real, Q, 6>(general, src, tx, tiles, ntiles, fin, fout, out10, v, t, mode, s);
}

template <typename real>
hipError_t launch_lattice(bool general, bool src, int rows_y, int tx, const Tile3Dev *tiles,
                          int ntiles, const void *fin, void *fout, void *out10, const Vol3Dev &v,
                          int64_t t, int mode, hipStream_t s) {
  if (v.q == kQ27)
    return launch_rows<real, kQ27>(general, src, rows_y, tx, tiles, ntiles, fin, fout, out10, v, t,
                                   mode, s);
  return launch_rows<real, kQ19>(general, src, rows_y, tx, tiles, ntiles, fin, fout, out10, v, t,
                                 mode, s);
}

}  // namespace

int launch_step3(bool f64, bool general, bool src, int rows_y, int tx, const Tile3Dev *tiles,
                 int ntiles, const void *fin, void *fout, void *out10, const Vol3Dev &v, int64_t t,
                 int mode, hipStream_t s) {
  const hipError_t e =
      f64 ? launch_lattice<double>(general, src, rows_y, tx, tiles, ntiles, fin, fout, out10, v, t,
                                   mode, s)
          : launch_lattice<float>(general, src, rows_y, tx, tiles, ntiles, fin, fout, out10, v, t,
                                  mode, s);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int launch_kappa3(bool f64, const void *lam, const void *mu, const void *rho, void *kappa,
                  int nx, int ny, int nz, int pitch, unsigned int *bad, double *minmax,
                  int *nblocks, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int nb = (int)std::min<int64_t>(kKappaBlocks, (N + 255) / 256);
  *nblocks = nb;
  if (f64)
    hipLaunchKernelGGL(kappa3_kernel<double>, dim3(nb), dim3(256), 0, s,
                       static_cast<const double *>(lam), static_cast<const double *>(mu),
                       static_cast<const double *>(rho), static_cast<double *>(kappa), nx, ny, nz,
                       pitch, bad, minmax);
  else
    hipLaunchKernelGGL(kappa3_kernel<float>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float *>(lam), static_cast<const float *>(mu),
                       static_cast<const float *>(rho), static_cast<float *>(kappa), nx, ny, nz,
                       pitch, bad, minmax);
  return (int)hipGetLastError();
}

int launch_gather_inv3(bool f64, const void *rho, const int32_t *xyz, int n, int nx, int ny,
                       void *out, hipStream_t s) {
  if (n <= 0) return 0;
  const int nb = (n + 255) / 256;
  if (f64)
    hipLaunchKernelGGL(gather_inv3_kernel<double>, dim3(nb), dim3(256), 0, s,
                       static_cast<const double *>(rho), xyz, n, nx, ny, static_cast<double *>(out));
  else
    hipLaunchKernelGGL(gather_inv3_kernel<float>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float *>(rho), xyz, n, nx, ny, static_cast<float *>(out));
  return (int)hipGetLastError();
}

int launch_pack3(bool f64, int q, const void *src, void *dst, int nx, int ny, int nz, int pitch,
                 bool to_pitched, hipStream_t s) {
  const int64_t nrows = (int64_t)q * nz * ny;
  const dim3 grid((nx + 255) / 256 < 4 ? (nx + 255) / 256 : 4, 65535,
                  (unsigned)((nrows + 65534) / 65535));
  const dim3 g2(grid.x, nrows < 65535 ? (unsigned)nrows : 65535u, grid.z);
  if (f64)
    hipLaunchKernelGGL(pack3_kernel<double>, g2, dim3(256), 0, s, static_cast<const double *>(src),
                       static_cast<double *>(dst), q, nx, ny, nz, pitch, to_pitched ? 1 : 0);
  else
    hipLaunchKernelGGL(pack3_kernel<float>, g2, dim3(256), 0, s, static_cast<const float *>(src),
                       static_cast<float *>(dst), q, nx, ny, nz, pitch, to_pitched ? 1 : 0);
  return (int)hipGetLastError();
}

}  // namespace lbm3
