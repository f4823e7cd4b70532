// Host check of the shared 32-point transforms of cf_fft32.h: the two threads of a
// pair are run one after the other with an explicit exchange, and their outputs
// are compared with the one-thread fft32 and with a direct DFT in double.
#define __host__
#define __device__
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "cf_fft32.h"

static double dft_err(const float *xr, const float *xi, const float *Xr, const float *Xi, bool inv) {
  double e = 0.0;
  for (int k = 0; k < 32; ++k) {
    double sr = 0.0, si = 0.0;
    for (int n = 0; n < 32; ++n) {
      const double a = (inv ? 2.0 : -2.0) * M_PI * n * k / 32.0;
      sr += xr[n] * std::cos(a) - xi[n] * std::sin(a);
      si += xr[n] * std::sin(a) + xi[n] * std::cos(a);
    }
    e = std::fmax(e, std::fmax(std::fabs(sr - Xr[k]), std::fabs(si - Xi[k])));
  }
  return e;
}

template <bool INV>
static bool check(unsigned seed) {
  std::srand(seed);
  float xr[32], xi[32];
  for (int n = 0; n < 32; ++n) {
    xr[n] = (float)std::rand() / RAND_MAX - 0.5f;
    xi[n] = (float)std::rand() / RAND_MAX - 0.5f;
  }
  float rr[32], ri[32];
  for (int n = 0; n < 32; ++n) rr[n] = xr[n], ri[n] = xi[n];
  cf::fft32<INV>(rr, ri);
  // decimation in time: thread h holds x[2n + h] and ends with X[16 h + k]
  float ar[2][16], ai[2][16];
  for (int h = 0; h < 2; ++h)
    for (int n = 0; n < 16; ++n) ar[h][n] = xr[2 * n + h], ai[h][n] = xi[2 * n + h];
  float sr[2][16], si[2][16];  // what each thread sends: its values when the exchange happens
  {
    // run both threads up to the exchange, then each reads the other's values
    float tr[2][16], ti[2][16];
    for (int h = 0; h < 2; ++h) {
      for (int n = 0; n < 16; ++n) tr[h][n] = ar[h][n], ti[h][n] = ai[h][n];
      cf::fft16<INV>(tr[h], ti[h]);
      if (h)
        for (int k = 1; k < 16; ++k) cf::twiddle32<INV>(tr[h][k], ti[h][k], k);
      for (int k = 0; k < 16; ++k) sr[h][k] = tr[h][k], si[h][k] = ti[h][k];
    }
  }
  float Xr[32], Xi[32];
  for (int h = 0; h < 2; ++h) {
    int idx = 0;
    // the partner is called with re[k] then im[k] for k = 0..15, in that order
    auto partner = [&](float) {
      const int k = idx >> 1, part = idx & 1;
      ++idx;
      return part ? si[1 - h][k] : sr[1 - h][k];
    };
    cf::fft32_pair_dit<INV>(ar[h], ai[h], h, partner);
    for (int k = 0; k < 16; ++k) Xr[16 * h + k] = ar[h][k], Xi[16 * h + k] = ai[h][k];
  }
  double e1 = 0.0;
  for (int k = 0; k < 32; ++k) e1 = std::fmax(e1, std::fmax(std::fabs(Xr[k] - rr[k]), std::fabs(Xi[k] - ri[k])));
  const double e2 = dft_err(xr, xi, Xr, Xi, INV);
  // decimation in frequency: thread h holds x[16 h + n] and ends with X[2k + h]
  float br[2][16], bi[2][16];
  for (int h = 0; h < 2; ++h)
    for (int n = 0; n < 16; ++n) br[h][n] = xr[16 * h + n], bi[h][n] = xi[16 * h + n];
  float Yr[32], Yi[32];
  for (int h = 0; h < 2; ++h) {
    int idx = 0;
    auto partner = [&](float) {
      const int n = idx >> 1, part = idx & 1;
      ++idx;
      return part ? bi[1 - h][n] : br[1 - h][n];
    };
    float cr[16], ci[16];
    for (int n = 0; n < 16; ++n) cr[n] = br[h][n], ci[n] = bi[h][n];
    cf::fft32_pair_dif<INV>(cr, ci, h, partner);
    for (int k = 0; k < 16; ++k) Yr[2 * k + h] = cr[k], Yi[2 * k + h] = ci[k];
  }
  double e3 = 0.0;
  for (int k = 0; k < 32; ++k) e3 = std::fmax(e3, std::fmax(std::fabs(Yr[k] - rr[k]), std::fabs(Yi[k] - ri[k])));
  const double e4 = dft_err(xr, xi, Yr, Yi, INV);
  const bool ok = e1 < 1e-5 && e2 < 1e-5 && e3 < 1e-5 && e4 < 1e-5;
  if (!ok) std::printf("seed %u inv %d: %g %g %g %g\n", seed, (int)INV, e1, e2, e3, e4);
  return ok;
}

int main() {
  bool ok = true;
  for (unsigned s = 1; s <= 50; ++s) ok = check<false>(s) && check<true>(s) && ok;
  std::printf(ok ? "OK\n" : "FAIL\n");
  return ok ? 0 : 1;
}
