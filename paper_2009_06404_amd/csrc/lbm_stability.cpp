// Von Neumann stability of the step (Sec. 4) for the library's own checks:
// the amplification of a plane wave exp(i k.x) over one step of the bulk
// scheme (periodic, no sponge, no source), and its largest factor over the
// wavenumbers for a given Poisson ratio and relaxation time, alone or with
// the high-wavenumber filter applied every few steps. Host code only.
#include <cmath>
#include <complex>

#include "lbm_internal.h"

namespace lbm {
namespace {

using cplx = std::complex<double>;
constexpr int SX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int SY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double SW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
constexpr double kB2 = 1.0 / 3.0;

// One step applied to the mode with amplitudes a: moments (eq. MomentsFeq),
// the centred density gradient i sin(k) rho (eq. FDrho), the source
// G = kappa grad rho and j = m + G/2 (eq. S), BGK toward the elastic
// equilibrium with the forcing populations (eqs. Pn, Si, LBGK), then the
// pull f_i(x) <- f*_i(x - c_i), a factor exp(-i k.c_i).
void step_mode(double kx, double ky, double kap, double omega, const cplx a[9], cplx out[9]) {
  cplx rho = 0.0, mx = 0.0, my = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho += a[i];
    mx += a[i] * (double)SX[i];
    my += a[i] * (double)SY[i];
    pxx += a[i] * (double)(SX[i] * SX[i]);
    pxy += a[i] * (double)(SX[i] * SY[i]);
    pyy += a[i] * (double)(SY[i] * SY[i]);
  }
  const cplx gx = kap * cplx(0.0, std::sin(kx)) * rho, gy = kap * cplx(0.0, std::sin(ky)) * rho;
  const cplx jx = mx + 0.5 * gx, jy = my + 0.5 * gy;
  const cplx nxx = pxx - kB2 * rho, nyy = pyy - kB2 * rho;
  const double cf = 1.0 - 0.5 * omega;
  for (int i = 0; i < 9; ++i) {
    const double cx = SX[i], cy = SY[i];
    const cplx feq = SW[i] * (rho + (jx * cx + jy * cy) / kB2 +
                              (nxx * (cx * cx - kB2) + 2.0 * pxy * cx * cy + nyy * (cy * cy - kB2)) /
                                  (2.0 * kB2 * kB2));
    const cplx force = SW[i] * (gx * cx + gy * cy) / kB2;
    const cplx post = (1.0 - omega) * a[i] + omega * feq + cf * force;
    out[i] = post * std::exp(cplx(0.0, -(kx * cx + ky * cy)));
  }
}

// Spectral radius of the 9x9 step matrix: ||M^(2^s)||^(2^-s) by repeated
// squaring with rescaling.
double spectral_radius(const cplx M0[9][9]) {
  cplx M[9][9], T[9][9];
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) M[r][c] = M0[r][c];
  double logacc = 0.0;   // log of the scale taken out of M^(2^s)
  constexpr int kSquarings = 30;
  for (int s = 0; s < kSquarings; ++s) {
    double big = 0.0;
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 9; ++c) {
        cplx v = 0.0;
        for (int k = 0; k < 9; ++k) v += M[r][k] * M[k][c];
        T[r][c] = v;
        big = std::max(big, std::abs(v));
      }
    if (big == 0.0) return 0.0;
    logacc = 2.0 * logacc + std::log(big);
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 9; ++c) M[r][c] = T[r][c] / big;
  }
  double nrm = 0.0;
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) nrm = std::max(nrm, std::abs(M[r][c]));
  return std::exp((logacc + std::log(nrm)) / std::ldexp(1.0, kSquarings));
}

}  // namespace

double vn_growth_filtered(double nu, double tau, double sigma, int every, int nk) {
  const double r = 2.0 * nu / (1.0 - 2.0 * nu);   // lambda / mu
  const double kap = kB2 * (1.0 - r);              // b^2 (mu - lambda) / mu
  const double omega = 1.0 / tau;
  double best = 0.0;
  for (int ix = 0; ix < nk; ++ix)
    for (int iy = 0; iy <= ix; ++iy) {   // the step is symmetric under kx <-> ky
      const double kx = M_PI * ix / (nk - 1), ky = M_PI * iy / (nk - 1);
      // columns of (filter) x (step)^every applied to the unit vectors
      const double sx = std::sin(0.5 * kx), sy = std::sin(0.5 * ky);
      const double filt = 1.0 - 16.0 * sigma * (sx * sx * sx * sx + sy * sy * sy * sy);
      cplx M[9][9], v[9], w[9];
      for (int j = 0; j < 9; ++j) {
        for (int i = 0; i < 9; ++i) v[i] = i == j ? 1.0 : 0.0;
        for (int s = 0; s < every; ++s) {
          step_mode(kx, ky, kap, omega, v, w);
          for (int i = 0; i < 9; ++i) v[i] = w[i];
        }
        for (int i = 0; i < 9; ++i) M[i][j] = filt * v[i];
      }
      best = std::max(best, std::pow(spectral_radius(M), 1.0 / every));
    }
  return best;
}

double vn_growth(double nu, double tau, int nk) { return vn_growth_filtered(nu, tau, 0.0, 1, nk); }

}  // namespace lbm
