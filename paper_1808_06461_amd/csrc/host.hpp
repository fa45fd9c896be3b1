// Host-side table builders (quad precision), see coeffs.cpp.
#pragma once
#include <vector>

namespace chn {

// mirrors the device-side FftPlan (common.hpp); kept free of HIP headers so
// coeffs.cpp compiles as plain C++
#ifndef CHN_FFTPLAN_DEFINED
#define CHN_FFTPLAN_DEFINED
struct FftPlan {
  int n;
  int npass;
  int radix[16];
  int twoff[16];  // pass p twiddles: tw[twoff + (r - 1) * Ns + k], r = 1..R-1, k < Ns
};
constexpr int kMaxPass = 16;
#endif

namespace host {
// row i of the banded (A, B) pair: Ar[3 + o] = A[i][i + o], o = -3..3
bool compact_row(int n2, const double* y, int i, int p, double* Ar, double* Br);
bool compact_bands(int n2, const double* y, int p, double* A, double* B);
void quadrature(int n2, const double* y, double* w);
bool band_lu(int n, const double* band, int dir, double* L, double* U);
bool wall_rows(int n, const double* A1, const double* B1, double* clo, double* chi);
bool fft_plan(int n, FftPlan* pl, std::vector<double>* tw);
void default_mesh(int n2, double* y);
}  // namespace host
}  // namespace chn
