// Host-side tables of the wall-normal discretisation and of the FFT plans.
//
// Compiled as plain host C++ (quad precision via __float128).
//
// Compact finite differences (Appendix B of the paper): for each mesh row i
// the coefficients of A f^(p) = B f over the stencil {i-3 .. i+3} (truncated
// at the walls) solve one small linear system making the scheme exact for
// the monomials (y - y_i)^k, k = 0 .. 2w-2, with A_ii = 1 (maximum order).
// The system is solved in quad precision on the scaled offsets (y_j - y_i)/h,
// the analogue of the paper's row premultiplication for conditioning, and
// rounded to float64.
#include <cmath>
#include <cstring>
#include <vector>

#include "host.hpp"

namespace chn {
namespace host {

using q = __float128;

static q qabs(q x) { return x < 0 ? -x : x; }

// Dense Gaussian elimination with partial pivoting (n <= 16).
static bool solve_dense(int n, q* M, q* r) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int k = c + 1; k < n; ++k)
      if (qabs(M[k * n + c]) > qabs(M[p * n + c])) p = k;
    if (M[p * n + c] == 0) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        q t = M[c * n + j];
        M[c * n + j] = M[p * n + j];
        M[p * n + j] = t;
      }
      q t = r[c];
      r[c] = r[p];
      r[p] = t;
    }
    for (int k = c + 1; k < n; ++k) {
      const q f = M[k * n + c] / M[c * n + c];
      if (f == 0) continue;
      for (int j = c; j < n; ++j) M[k * n + j] -= f * M[c * n + j];
      r[k] -= f * r[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    q s = r[c];
    for (int j = c + 1; j < n; ++j) s -= M[c * n + j] * r[j];
    r[c] = s / M[c * n + c];
  }
  return true;
}

bool compact_row(int n2, const double* y, int i, int p, double* Ar, double* Br) {
  for (int o = 0; o < 7; ++o) Ar[o] = Br[o] = 0.0;
  const int lo = i - 3 < 0 ? 0 : i - 3;
  const int hi = i + 3 > n2 - 1 ? n2 - 1 : i + 3;
  const int w = hi - lo + 1;
  const int nu = 2 * w;
  const q h = (i + 2 < n2) ? qabs((q)y[i + 2] - (q)y[i]) : qabs((q)y[i] - (q)y[i - 2]);
  q d[7];
  for (int j = 0; j < w; ++j) d[j] = ((q)y[lo + j] - (q)y[i]) / h;
  q M[14 * 14], r[14];
  for (int e = 0; e < nu * nu; ++e) M[e] = 0;
  for (int k = 0; k < nu - 1; ++k) {
    r[k] = 0;
    for (int j = 0; j < w; ++j) {
      q dk = 1;
      for (int e = 0; e < k; ++e) dk *= d[j];
      M[k * nu + j] = dk;
      if (k >= p) {
        q dkp = 1;
        for (int e = 0; e < k - p; ++e) dkp *= d[j];
        const q fac = p == 2 ? (q)(k * (k - 1)) : (q)k;
        M[k * nu + w + j] = -fac * dkp;
      }
    }
  }
  M[(nu - 1) * nu + w + (i - lo)] = 1;
  r[nu - 1] = 1;
  if (!solve_dense(nu, M, r)) return false;
  q hp = p == 2 ? h * h : h;
  for (int j = 0; j < w; ++j) {
    const int o = lo + j - i + 3;
    Br[o] = (double)(r[j] / hp);
    Ar[o] = (double)r[w + j];
  }
  return true;
}

bool compact_bands(int n2, const double* y, int p, double* A, double* B) {
  for (int i = 0; i < n2; ++i)
    if (!compact_row(n2, y, i, p, A + 7 * i, B + 7 * i)) return false;
  return true;
}

void quadrature(int n2, const double* y, double* wout) {
  std::vector<q> w(n2, (q)0);
  for (int j = 0; j < n2 - 1; ++j) {
    int lo = j - 2;
    if (lo < 0) lo = 0;
    if (lo > n2 - 6) lo = n2 - 6;
    const q a = y[j], b = y[j + 1];
    for (int m = lo; m < lo + 6; ++m) {
      // integral over [a, b] of the Lagrange basis polynomial of node m
      q coef[6] = {1, 0, 0, 0, 0, 0};
      int deg = 0;
      q den = 1;
      for (int k = lo; k < lo + 6; ++k) {
        if (k == m) continue;
        // multiply by (t - y_k)
        for (int e = deg + 1; e >= 1; --e) coef[e] = coef[e - 1] - (q)y[k] * coef[e];
        coef[0] = -(q)y[k] * coef[0];
        ++deg;
        den *= ((q)y[m] - (q)y[k]);
      }
      q integ = 0, ap = a, bp = b;
      for (int e = 0; e <= deg; ++e) {
        integ += coef[e] * (bp - ap) / (q)(e + 1);
        ap *= a;
        bp *= b;
      }
      w[m] += integ / den;
    }
  }
  for (int j = 0; j < n2; ++j) wout[j] = (double)w[j];
}

// LU (no pivoting) of a band processed in direction dir (+1: rows 0..n-1,
// -1: rows n-1..0).  L[i][3-d] multiplies the row at processing distance d;
// U[i] = {1/pivot, u1, u2, u3}, u_t at processing-forward distance t.
bool band_lu(int n, const double* band, int dir, double* L, double* U) {
  std::vector<q> Uq((size_t)n * 4, (q)0);
  for (int t = 0; t < n; ++t) {
    const int i = dir > 0 ? t : n - 1 - t;
    q row[7];
    for (int o = -3; o <= 3; ++o) row[3 + o] = (q)band[i * 7 + 3 + dir * o];
    for (int d = 3; d >= 1; --d) {
      const int prev = i - dir * d;
      q l = 0;
      if (prev >= 0 && prev < n) {
        const q* Up = &Uq[(size_t)prev * 4];
        l = row[3 - d] / Up[0];
        for (int s = 1; s <= 3; ++s) row[3 - d + s] -= l * Up[s];
      }
      L[i * 3 + (3 - d)] = (double)l;
    }
    if (row[3] == 0) return false;
    q* Ui = &Uq[(size_t)i * 4];
    Ui[0] = row[3];
    for (int s = 1; s <= 3; ++s) Ui[s] = row[3 + s];
    U[i * 4 + 0] = (double)(1 / row[3]);
    for (int s = 1; s <= 3; ++s) U[i * 4 + s] = (double)row[3 + s];
  }
  return true;
}

// Wall rows of D1 = A1^{-1} B1: c_lo = B1^T A1^{-T} e_0, c_hi = B1^T A1^{-T} e_{n-1}.
bool wall_rows(int n, const double* A1, const double* B1, double* clo, double* chi) {
  // transposed band of A1, solved in quad with banded elimination (no pivoting)
  for (int side = 0; side < 2; ++side) {
    std::vector<q> T((size_t)n * 7, (q)0), z(n, (q)0);
    for (int i = 0; i < n; ++i)
      for (int o = -3; o <= 3; ++o) {
        const int j = i + o;
        if (j >= 0 && j < n) T[(size_t)i * 7 + 3 + o] = (q)A1[j * 7 + 3 - o];
      }
    z[side == 0 ? 0 : n - 1] = 1;
    for (int i = 0; i < n; ++i) {  // forward elimination
      q* ri = &T[(size_t)i * 7];
      for (int c = i - 3; c < i; ++c) {
        if (c < 0) continue;
        const q* rc = &T[(size_t)c * 7];
        const q l = ri[3 + c - i] / rc[3];
        for (int s = 1; s <= 3; ++s) ri[3 + c - i + s] -= l * rc[3 + s];
        ri[3 + c - i] = 0;
        z[i] -= l * z[c];
      }
      if (ri[3] == 0) return false;
    }
    for (int i = n - 1; i >= 0; --i) {
      const q* ri = &T[(size_t)i * 7];
      q s = z[i];
      for (int t = 1; t <= 3; ++t)
        if (i + t < n) s -= ri[3 + t] * z[i + t];
      z[i] = s / ri[3];
    }
    double* out = side == 0 ? clo : chi;
    for (int j = 0; j < n; ++j) {
      q s = 0;
      for (int i = j - 3; i <= j + 3; ++i)
        if (i >= 0 && i < n) s += z[i] * (q)B1[i * 7 + 3 + (j - i)];
      out[j] = (double)s;
    }
  }
  return true;
}

namespace {
// Fewest passes over the radices {16, 12, 9, 8, 6, 4, 3, 2}, ties to the
// smallest largest radix (lighter butterflies), passes in non-increasing
// radix order.  Depth-first over non-increasing sequences.
struct RadixSearch {
  int best_np = 1 << 30, best_max = 1 << 30;
  int best[kMaxPass] = {}, cur[kMaxPass] = {};
  void run(int m, int np, int maxr) {
    static const int rads[8] = {16, 12, 9, 8, 6, 4, 3, 2};
    if (m == 1) {
      const int mx = np ? cur[0] : 1;
      if (np < best_np || (np == best_np && mx < best_max)) {
        best_np = np;
        best_max = mx;
        for (int p = 0; p < np; ++p) best[p] = cur[p];
      }
      return;
    }
    if (np + 1 > best_np || np >= kMaxPass) return;
    for (int r : rads)
      if (r <= maxr && m % r == 0) {
        cur[np] = r;
        run(m / r, np + 1, r);
      }
  }
};
}  // namespace

bool fft_plan(int n, FftPlan* pl, std::vector<double>* tw, int radices) {
  std::memset(pl, 0, sizeof(*pl));
  pl->n = n;
  int m = n, np = 0;
  if (radices == kRadixComposite || radices == kRadixUpTo6) {
    if (n < 1) return false;
    RadixSearch rs;
    rs.run(n, 0, radices == kRadixUpTo6 ? 6 : 16);
    if (rs.best_np > kMaxPass) return false;
    np = rs.best_np;
    for (int p = 0; p < np; ++p) pl->radix[p] = rs.best[p];
  } else {
    const int rads[4] = {8, 4, 2, 3};
    for (int ri = 0; ri < 4; ++ri) {
      while (m % rads[ri] == 0) {
        if (np >= kMaxPass) return false;
        pl->radix[np++] = rads[ri];
        m /= rads[ri];
      }
    }
    if (m != 1) return false;
  }
  pl->npass = np;
  tw->clear();
  int Ns = 1;
  for (int p = 0; p < np; ++p) {
    const int R = pl->radix[p];
    pl->twoff[p] = (int)(tw->size() / 2);
    // r-major, so that lanes with consecutive k read consecutive twiddles
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < Ns; ++k) {
        const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)(r * k) /
                                (long double)(Ns * R);
        tw->push_back((double)cosl(ang));
        tw->push_back((double)sinl(ang));
      }
    Ns *= R;
  }
  return true;
}

bool operator_conditioning(int n2, const double* y, double* c1, double* c2) {
  std::vector<double> A((size_t)n2 * 7), B((size_t)n2 * 7);
  if (!compact_bands(n2, y, 1, A.data(), B.data())) return false;
  *c1 = band_cond1(n2, A.data());
  if (!compact_bands(n2, y, 2, A.data(), B.data())) return false;
  for (int o = 0; o < 7; ++o) {
    A[o] = o == 3 ? 1.0 : 0.0;
    A[(size_t)(n2 - 1) * 7 + o] = o == 3 ? 1.0 : 0.0;
  }
  *c2 = band_cond1(n2, A.data());
  return std::isfinite(*c1) && std::isfinite(*c2);
}

static void tanh_mesh(int n2, long double g, double* y) {
  const long double tg = tanhl(g);
  for (int j = 0; j < n2; ++j) {
    const long double s = -1.0L + 2.0L * j / (n2 - 1);
    y[j] = (double)(tanhl(g * s) / tg);
  }
  // exact mirror symmetry, walls at -1 and 1
  for (int j = 0; j < n2 / 2; ++j) y[n2 - 1 - j] = -y[j];
  if (n2 % 2) y[n2 / 2] = 0.0;
  y[0] = -1.0;
  y[n2 - 1] = 1.0;
}

void default_mesh(int n2, double* y, double* gamma) {
  for (int k = 0; k < 7; ++k) {
    const double g = 2.0 - 0.25 * k;
    tanh_mesh(n2, g, y);
    double c1, c2;
    if (g == 0.5 || (operator_conditioning(n2, y, &c1, &c2) && c2 <= 1e4 && c1 <= 1e5)) {
      if (gamma) *gamma = g;
      return;
    }
  }
}

}  // namespace host
}  // namespace chn
