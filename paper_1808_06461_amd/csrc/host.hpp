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
// Stockham plan of a length-n transform and its twiddle table.  Radix sets:
// kRadixClassic takes 8s, then 4, 2, 3 (at most radix 8 per pass);
// kRadixComposite the fewest passes over radices up to 16 (6, 9, 12, 16 are
// computed in registers), so each element makes fewer LDS round trips.
// kRadixUpTo6 the fewest passes over radices up to 6 (one radix-6 butterfly
// stages six values per thread, fewer than the classic radix-8 passes need).
constexpr int kRadixClassic = 0, kRadixComposite = 1, kRadixUpTo6 = 2;
bool fft_plan(int n, FftPlan* pl, std::vector<double>* tw, int radices = kRadixClassic);
// 1-norm condition number ||A||_1 ||A^-1||_1 of a [n][7] band (inf if singular)
double band_cond1(int n, const double* A);
// cond_1 of A1 and of A2 with its end rows replaced by Dirichlet rows (the
// implicit steps' matrix at vanishing time step); false if a band is singular
bool operator_conditioning(int n2, const double* y, double* c1, double* c2);
// Default wall-normal mesh: y_j = tanh(g s_j) / tanh(g), s_j uniform on
// [-1, 1], with the largest g in {2, 1.75, ..., 0.5} whose compact operators
// have cond_1(A2, Dirichlet rows) <= 1e4 and cond_1(A1) <= 1e5 (g = 0.5 if
// none); *gamma receives g
void default_mesh(int n2, double* y, double* gamma = nullptr);
}  // namespace host
}  // namespace chn
