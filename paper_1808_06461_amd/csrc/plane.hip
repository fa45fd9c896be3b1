// Plane phase: staging checks and schedule helpers (kernels and launch helpers in plane.hpp).
#include "plane.hpp"

namespace chn {

bool staging_fits(const FftPlan& pl, int nlines, int nt, int m) {
  for (int p = 0; p < pl.npass; ++p) {
    const int R = pl.radix[p];
    const long need = ((long)nlines * (pl.n / R) + nt - 1) / nt;
    if (m / R < need) return false;
  }
  return true;
}

int xrow_threads(int p1, int bytes_per_value) {
  const int qx = bytes_per_value == 8 ? 12 : 6;
  for (int nt = 256; nt <= 1024; nt *= 2)
    if (p1 <= nt * qx) return nt;
  return 0;
}
bool xpass_two_rows(int p1, int bytes_per_value) {
  return 6 * p1 <= (bytes_per_value == 8 ? 48 : 24) * 256;
}

int staging_for(const FftPlan& pl, int nlines, int bytes_per_value) {
  return bytes_per_value == 8 ? pick_staging<float>(pl, nlines, 256) : pick_staging<double>(pl, nlines, 256);
}
int z_staging(const FftPlan& pl, int K, int bytes_per_value) {
  const bool f = bytes_per_value == 8;
  if (z_threads(pl, K) == 1024) return f ? pick_staging<float>(pl, 1, 1024) : pick_staging<double>(pl, 1, 1024);
  return f ? pick_staging<float>(pl, K, 256) : pick_staging<double>(pl, K, 256);
}
bool xrow_fits(const FftPlan& pl, int bytes_per_value) {
  const int nt = xrow_threads(pl.n, bytes_per_value);
  if (nt == 0) return false;
  return staging_fits(pl, 1, nt, bytes_per_value == 8 ? XrowCfg<float>::MV : XrowCfg<double>::MV);
}



}  // namespace chn
