// Von Neumann stability of the three-dimensional step (Sec. 4's analysis on
// the D3Q19 / D3Q27 lattices): the amplification of a plane wave exp(i k.x)
// over one step of the bulk scheme (periodic, no sponge, no source), and its
// largest factor over a grid of wavenumbers in [0, pi]^3 for a Poisson ratio
// and a relaxation time. Host code only.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "lbm3d_internal.h"

namespace lbm3 {
namespace {

using cplx = std::complex<double>;
constexpr int kMaxQ = 27;
constexpr double kB2 = 1.0 / 3.0;

// The velocity set in the public order (D3Q19 is the first 19 of D3Q27).
constexpr int VX[kMaxQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                           1, -1, 1, -1, 1, -1, -1, 1};
constexpr int VY[kMaxQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                           1, -1, 1, -1, -1, 1, 1, -1};
constexpr int VZ[kMaxQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                           1, -1, -1, 1, 1, -1, 1, -1};

double weight(int q, int i) {
  const int n = std::abs(VX[i]) + std::abs(VY[i]) + std::abs(VZ[i]);
  if (q == kQ19) return n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  return n == 0 ? 8.0 / 27.0 : (n == 1 ? 2.0 / 27.0 : (n == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
}

// One step applied to the mode with amplitudes a: moments, the centred
// density gradient i sin(k) rho, G = kappa grad rho, j = m + G/2, BGK toward
// the elastic equilibrium with the forcing populations, then the pull
// f_i(x) <- f*_i(x - c_i), a factor exp(-i k.c_i).
void step_mode(int q, const double k[3], double kap, double omega, const cplx *a, cplx *out) {
  cplx rho = 0.0, m[3] = {0.0, 0.0, 0.0}, P[3][3] = {};
  for (int i = 0; i < q; ++i) {
    const int c[3] = {VX[i], VY[i], VZ[i]};
    rho += a[i];
    for (int u = 0; u < 3; ++u) {
      m[u] += a[i] * (double)c[u];
      for (int w = 0; w < 3; ++w) P[u][w] += a[i] * (double)(c[u] * c[w]);
    }
  }
  cplx G[3], j[3];
  for (int u = 0; u < 3; ++u) {
    G[u] = kap * cplx(0.0, std::sin(k[u])) * rho;
    j[u] = m[u] + 0.5 * G[u];
  }
  for (int u = 0; u < 3; ++u) P[u][u] -= kB2 * rho;   // P^n
  const double cf = 1.0 - 0.5 * omega;
  for (int i = 0; i < q; ++i) {
    const int c[3] = {VX[i], VY[i], VZ[i]};
    cplx jc = 0.0, gc = 0.0, pq = 0.0;
    for (int u = 0; u < 3; ++u) {
      jc += j[u] * (double)c[u];
      gc += G[u] * (double)c[u];
      for (int w = 0; w < 3; ++w) pq += P[u][w] * ((double)(c[u] * c[w]) - (u == w ? kB2 : 0.0));
    }
    const double wi = weight(q, i);
    const cplx feq = wi * (rho + jc / kB2 + pq / (2.0 * kB2 * kB2));
    const cplx post = (1.0 - omega) * a[i] + omega * feq + cf * wi * gc / kB2;
    out[i] = post * std::exp(cplx(0.0, -(k[0] * c[0] + k[1] * c[1] + k[2] * c[2])));
  }
}

// Spectral radius of the q x q step matrix: ||M^(2^s)||^(2^-s) by repeated
// squaring with rescaling.
double spectral_radius(int q, std::vector<cplx> M) {
  std::vector<cplx> T((size_t)q * q);
  double logacc = 0.0;
  constexpr int kSquarings = 30;
  for (int s = 0; s < kSquarings; ++s) {
    double big = 0.0;
    for (int r = 0; r < q; ++r)
      for (int c = 0; c < q; ++c) {
        cplx v = 0.0;
        for (int t = 0; t < q; ++t) v += M[(size_t)r * q + t] * M[(size_t)t * q + c];
        T[(size_t)r * q + c] = v;
        big = std::max(big, std::abs(v));
      }
    if (big == 0.0) return 0.0;
    logacc = 2.0 * logacc + std::log(big);
    for (size_t e = 0; e < M.size(); ++e) M[e] = T[e] / big;
  }
  double nrm = 0.0;
  for (const cplx &v : M) nrm = std::max(nrm, std::abs(v));
  return std::exp((logacc + std::log(nrm)) / std::ldexp(1.0, kSquarings));
}

}  // namespace

double vn_growth3(int q, double nu, double tau, int nk) {
  const double r = 2.0 * nu / (1.0 - 2.0 * nu);   // lambda / mu
  const double kap = kB2 * (1.0 - r);              // b^2 (mu - lambda) / mu
  const double omega = 1.0 / tau;
  double best = 0.0;
  std::vector<cplx> M((size_t)q * q);
  cplx v[kMaxQ], w[kMaxQ];
  // the step is symmetric under permutations of the axes: kx >= ky >= kz
  for (int ix = 0; ix < nk; ++ix)
    for (int iy = 0; iy <= ix; ++iy)
      for (int iz = 0; iz <= iy; ++iz) {
        const double k[3] = {M_PI * ix / (nk - 1), M_PI * iy / (nk - 1), M_PI * iz / (nk - 1)};
        for (int jc = 0; jc < q; ++jc) {
          for (int i = 0; i < q; ++i) v[i] = i == jc ? 1.0 : 0.0;
          step_mode(q, k, kap, omega, v, w);
          for (int i = 0; i < q; ++i) M[(size_t)i * q + jc] = w[i];
        }
        best = std::max(best, spectral_radius(q, M));
      }
  return best;
}

}  // namespace lbm3
