// Initialisation and utility kernels of liblbm.so: the per-cell elastic
// coefficient, field validation, receiver gathers, state copies, the finite
// check and the device time base used by captured graphs.
#include <algorithm>
#include <mutex>

#include "lbm_internal.h"

// Scratch memory of the allocation-free finite check: a flag per grid, then
// the number of grids found non-finite and the lowest such grid index. Each
// GPU holds its own copy for the life of the process. In host code this name
// is only a stand-in for the symbol: host code reaches the memory through the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint32_t scratch[lbm::kScratchGrids + 2];

namespace lbm {
namespace {

// kappa = (mu - lambda)/rho0 with mu/rho0 = b^2, i.e. b^2 (mu - lambda)/mu
// (Sec. 4). A cell is rejected unless mu > 0, rho > 0, lambda >= 0 and the
// Poisson ratio lambda / (2 (lambda + mu)) < 5/11 (Sec. 4).
template <typename real>
__global__ void kappa_kernel(const real *__restrict__ lam, const real *__restrict__ mu,
                             const real *__restrict__ rho, int nx, int ny, int pitch,
                             real *__restrict__ kappa, int *bad, int *row_varies) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(k / nx), x = (int)(k % nx);
    const double l = (double)lam[k], m = (double)mu[k], r = (double)rho[k];
    const bool ok = m > 0.0 && r > 0.0 && l >= 0.0 && (l / (2.0 * (l + m))) < 5.0 / 11.0;
    if (!ok) atomicAdd(bad, 1);
    const real kv = ok ? (real)((1.0 / 3.0) * (m - l) / m) : real(0);
    kappa[(int64_t)y * pitch + x] = kv;
    if (x > 0) {
      const double l0 = (double)lam[(int64_t)y * nx], m0 = (double)mu[(int64_t)y * nx];
      if (l0 != l || m0 != m) row_varies[y] = 1;
    }
  }
}

template <typename real>
__global__ void kappa_range_kernel(const real *__restrict__ kappa, int nx, int ny, int pitch,
                                   real *__restrict__ minmax) {
  __shared__ real lo[256], hi[256];
  const int64_t n = (int64_t)nx * ny;
  real a = real(1e30), b = real(-1e30);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const real v = kappa[(k / nx) * pitch + k % nx];
    a = min(a, v);
    b = max(b, v);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + s]);
      hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    minmax[2 * blockIdx.x] = lo[0];
    minmax[2 * blockIdx.x + 1] = hi[0];
  }
}

template <typename real>
__global__ void kappa_rows_kernel(const real *__restrict__ kappa, int ny, int pitch,
                                  real *__restrict__ rows) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y < ny) rows[y] = kappa[(int64_t)y * pitch];
}

template <typename real>
__global__ void gather_kernel(const real *__restrict__ src, const int64_t *__restrict__ idx,
                              int n, real *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

template <typename real>
__global__ void nonfinite_kernel(const real *__restrict__ f, int64_t n, int *count) {
  int local = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const real v = f[k];
    if (!(v - v == real(0))) local = 1;
  }
  if (local) atomicAdd(count, 1);
}

// The watch of lbm_set_finite_check: if any of the n values at f is NaN or
// Inf and no earlier check has recorded a time, record t in *first_bad
// (host memory mapped into the device; -1 until then). Every writer of one
// launch writes the same t.
template <typename real>
__global__ void finite_watch_kernel(const real *__restrict__ f, int64_t n, int64_t t,
                                    volatile int64_t *first_bad) {
  int bad = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const real v = f[k];
    if (!(v - v == real(0))) bad = 1;
  }
  // only blocks that found one touch the host word (one read, one write)
  if (__syncthreads_or(bad) && threadIdx.x == 0 && *first_bad < 0) *first_bad = t;
}

// Clears the scratch of the allocation-free finite check for nflags grids:
// flags and count to 0, the lowest bad grid to 0xffffffff.
__global__ void scratch_reset_kernel(uint32_t *s, int nflags) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nflags; k += gridDim.x * blockDim.x)
    s[k] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s[kScratchGrids] = 0u;
    s[kScratchGrids + 1] = 0xffffffffu;
  }
}

// Grid blockIdx.y's populations (9 x pitch x ny from its offset) scanned by
// gridDim.x blocks; a block that finds NaN or Inf raises the grid's flag, and
// the first block to raise it counts the grid and lowers the minimum index.
template <typename real>
__global__ void nonfinite_grids_kernel(const real *__restrict__ f, const GridDev *__restrict__ grids,
                                       uint32_t *s) {
  const int g = blockIdx.y;
  const int64_t off = grids[g].f_off;
  const int64_t n = (int64_t)9 * grids[g].pitch * grids[g].ny;
  int bad = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const real v = f[off + k];
    if (!(v - v == real(0))) bad = 1;
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) {
    if (atomicOr(&s[g], 1u) == 0u) {
      atomicAdd(&s[kScratchGrids], 1u);
      atomicMin(&s[kScratchGrids + 1], (uint32_t)g);
    }
  }
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// The current device's address of the scratch array, taken once per device
// with that device current.
hipError_t scratch_address(uint32_t **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = static_cast<uint32_t *>(g_scratch_addr[dev]);
  return hipSuccess;
}

// Copy nplanes planes of an nx x ny grid between two layouts given by their
// strides (elements) between planes and between rows.
template <typename real>
__global__ void copy_planes_kernel(const real *__restrict__ src, int64_t src_ps, int64_t src_ys,
                                   real *__restrict__ dst, int64_t dst_ps, int64_t dst_ys,
                                   int nx, int ny, int nplanes) {
  const int64_t n = (int64_t)nx * ny * nplanes;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = k / ((int64_t)nx * ny);
    const int64_t rem = k - p * (int64_t)nx * ny;
    const int64_t y = rem / nx, x = rem % nx;
    dst[p * dst_ps + y * dst_ys + x] = src[p * src_ps + y * src_ys + x];
  }
}

__global__ void set_time_kernel(int64_t *t_dev, int64_t value) { t_dev[0] = value; }
__global__ void add_time_kernel(int64_t *t_dev, int64_t delta) { t_dev[0] += delta; }

inline int blocks_for(int64_t n, int per_block = 256, int cap = 8192) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

}  // namespace

template <typename real>
hipError_t launch_kappa(const real *lam, const real *mu, const real *rho, int nx, int ny,
                        int pitch, real *kappa, int *bad, int *row_varies, hipStream_t stream) {
  hipLaunchKernelGGL(kappa_kernel<real>, dim3(blocks_for((int64_t)nx * ny)), dim3(256), 0, stream,
                     lam, mu, rho, nx, ny, pitch, kappa, bad, row_varies);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_kappa_range(const real *kappa, int nx, int ny, int pitch, real *minmax,
                              int nblocks, hipStream_t stream) {
  if (nblocks < 1 || nblocks > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kappa_range_kernel<real>, dim3(nblocks), dim3(256), 0, stream, kappa, nx, ny,
                     pitch, minmax);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_kappa_rows(const real *kappa, int ny, int pitch, real *rows, hipStream_t stream) {
  hipLaunchKernelGGL(kappa_rows_kernel<real>, dim3((ny + 255) / 256), dim3(256), 0, stream, kappa,
                     ny, pitch, rows);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_gather(const real *src, const int64_t *idx, int n, real *dst, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel<real>, dim3((n + 255) / 256), dim3(256), 0, stream, src, idx, n,
                     dst);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_count_nonfinite(const real *f, int64_t n, int *count, hipStream_t stream) {
  hipLaunchKernelGGL(nonfinite_kernel<real>, dim3(blocks_for(n)), dim3(256), 0, stream, f, n, count);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_finite_watch(const real *f, int64_t n, int64_t t, int64_t *first_bad,
                               hipStream_t stream) {
  hipLaunchKernelGGL(finite_watch_kernel<real>, dim3(blocks_for(n, 256, 2048)), dim3(256), 0,
                     stream, f, n, t, first_bad);
  return hipGetLastError();
}

template <typename real>
hipError_t check_nonfinite_scratch(const real *f, const GridDev *grids, int nbatch,
                                   int64_t max_elems, hipStream_t stream, uint32_t out[2]) {
  if (nbatch < 1 || nbatch > kScratchGrids || max_elems < 1) return hipErrorInvalidValue;
  uint32_t *s = nullptr;
  hipError_t e = scratch_address(&s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scratch_reset_kernel, dim3((nbatch + 255) / 256), dim3(256), 0, stream, s,
                     nbatch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // blocks per grid: enough to cover the largest grid in a few passes, and
  // at most 65535 grids along y (nbatch <= kScratchGrids)
  const int bx = blocks_for(max_elems, 256, std::max(1, 16384 / nbatch));
  hipLaunchKernelGGL(nonfinite_grids_kernel<real>, dim3(bx, nbatch), dim3(256), 0, stream, f,
                     grids, s);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(out, s + kScratchGrids, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(stream);
}

template <typename real>
hipError_t launch_copy_planes(const real *src, int64_t src_ps, int64_t src_ys, real *dst,
                              int64_t dst_ps, int64_t dst_ys, int nx, int ny, int nplanes,
                              hipStream_t stream) {
  hipLaunchKernelGGL(copy_planes_kernel<real>, dim3(blocks_for((int64_t)nx * ny * nplanes)),
                     dim3(256), 0, stream, src, src_ps, src_ys, dst, dst_ps, dst_ys, nx, ny,
                     nplanes);
  return hipGetLastError();
}

hipError_t launch_set_time(int64_t *t_dev, int64_t value, hipStream_t stream) {
  hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(1), 0, stream, t_dev, value);
  return hipGetLastError();
}

hipError_t launch_add_time(int64_t *t_dev, int64_t delta, hipStream_t stream) {
  hipLaunchKernelGGL(add_time_kernel, dim3(1), dim3(1), 0, stream, t_dev, delta);
  return hipGetLastError();
}

#define LBM_INST(real)                                                                          \
  template hipError_t launch_kappa<real>(const real *, const real *, const real *, int, int, int, \
                                         real *, int *, int *, hipStream_t);                      \
  template hipError_t launch_kappa_rows<real>(const real *, int, int, real *, hipStream_t);      \
  template hipError_t launch_kappa_range<real>(const real *, int, int, int, real *, int,         \
                                               hipStream_t);                                     \
  template hipError_t launch_gather<real>(const real *, const int64_t *, int, real *,            \
                                          hipStream_t);                                          \
  template hipError_t launch_count_nonfinite<real>(const real *, int64_t, int *, hipStream_t);   \
  template hipError_t launch_finite_watch<real>(const real *, int64_t, int64_t, int64_t *,      \
                                                hipStream_t);                                    \
  template hipError_t check_nonfinite_scratch<real>(const real *, const GridDev *, int, int64_t,  \
                                                    hipStream_t, uint32_t *);                    \
  template hipError_t launch_copy_planes<real>(const real *, int64_t, int64_t, real *, int64_t,  \
                                               int64_t, int, int, int, hipStream_t);
LBM_INST(float)
LBM_INST(double)
#undef LBM_INST

}  // namespace lbm
