// Near-wall mesh optimisation for the homogeneous Helmholtz solutions
// (Appendix B of the paper), host C++.
//
// The implicit step's homogeneous problem (B2 - k* A2) g = 0, g = 1 at the
// lower wall and 0 at the upper one, has the analytic solution
// sinh(q (1 - y)) / sinh(2 q), q = sqrt(k*).  When the layer 1/q is thinner
// than the first cells, the compact solution departs from it near the wall
// by an amount the near-wall coefficients of A2 fix (as k* grows the rows
// tend to A2 g = 0).  The first m interior nodes (and their mirror images at
// the upper wall) are moved to minimise
//   L = ||g - g_ana||_2 + C ||mu - mu_ref||_2,   mu = (y_1 .. y_m),
// by steepest descent in spacing-scaled coordinates (the step in y_j is
// -t s_j^2 dL/dy_j, s_j = y_ref[j+1] - y_ref[j]); the gradient by central
// differences with step 1e-6 s_j; the step length by halving from twice the
// last accepted one (t starts at 1, so the first trial is 2) until the mesh
// is strictly increasing, L strictly decreases, the Armijo condition
// L_new <= L + 1e-4 t (grad . d) holds, every ratio of adjacent spacings of
// the trial mesh lies in [1/2, 2] (the nodes move without changing much the
// individual spacings), and the trial mesh's A2 and A1 each have a 1-norm
// condition number at most ten times the reference mesh's (the functional
// sees only B2 - k* A2; without the bound the descent can reach
// stretchings on which the maximum-order stencils make A2 singular, and A1,
// which the velocity recovery and the forcing use, degrades the same way).
// It stops after max_iter steps or when t < 1e-30.
//
// A moved node changes only the compact rows whose stencils hold it, so a
// gradient component recomputes 14 rows (quad precision, compact_row) and
// solves one banded system; the solve is a banded LU with partial pivoting
// (three sub-diagonals, the upper band growing from three to six).
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "../../include/chn.h"
#include "host.hpp"

namespace chn {
namespace host {
namespace {

constexpr int kW = 10;  // stored columns per row: i-3 .. i+6

struct MeshProblem {
  int n, m;
  double ks, C;
  std::vector<double> yref, xref, s;
  std::vector<double> A, B;  // [n][7] operators at the current mesh
  std::vector<double> M7, g;  // Dirichlet-row matrix [n][7], solution
  std::vector<double> A1, B1;  // first-derivative operators (conditioning check)
  double cond_max, cond1_max;  // bounds on cond_1(A2), cond_1(A1)
};

constexpr double kSpacingRatio = 2.0;

bool spacing_ratio_ok(int n, const double* y) {
  for (int i = 1; i + 1 < n; ++i) {
    const double r = (y[i + 1] - y[i]) / (y[i] - y[i - 1]);
    if (!(r <= kSpacingRatio && r >= 1.0 / kSpacingRatio)) return false;
  }
  return true;
}

double g_analytic(double y, double ks) {
  const double qk = std::sqrt(ks);
  return std::exp(-qk * (1.0 + y)) * (-std::expm1(-2.0 * qk * (1.0 - y))) / (-std::expm1(-4.0 * qk));
}

// Banded LU with partial pivoting of an n x n matrix with three sub- and
// three super-diagonals: row i stores columns i-3 .. i+6 (the upper band
// grows to six with the row exchanges); the multipliers of column c stay in
// (k, c), k = c+1..c+3, which later steps never touch.
struct BandLU {
  int n = 0;
  std::vector<double> W;
  std::vector<int> piv;
  double& at(int row, int col) { return W[(size_t)row * kW + (col - row + 3)]; }
  void load(int n_, const double* M7) {  // M7: [n][7], row i holds M[i][i-3..i+3]
    n = n_;
    W.assign((size_t)n * kW, 0.0);
    piv.assign(n, 0);
    for (int i = 0; i < n; ++i)
      for (int o = -3; o <= 3; ++o)
        if (i + o >= 0 && i + o < n) at(i, i + o) = M7[i * 7 + 3 + o];
  }
  bool factor() {
    for (int c = 0; c < n; ++c) {
      const int last = c + 3 < n - 1 ? c + 3 : n - 1;
      const int cend = c + 6 < n - 1 ? c + 6 : n - 1;
      int p = c;
      for (int k = c + 1; k <= last; ++k)
        if (std::fabs(at(k, c)) > std::fabs(at(p, c))) p = k;
      piv[c] = p;
      if (at(p, c) == 0.0) return false;
      if (p != c)
        for (int col = c; col <= cend; ++col) std::swap(at(c, col), at(p, col));
      for (int k = c + 1; k <= last; ++k) {
        const double f = at(k, c) / at(c, c);
        at(k, c) = f;
        if (f == 0.0) continue;
        for (int col = c + 1; col <= cend; ++col) at(k, col) -= f * at(c, col);
      }
    }
    return true;
  }
  void solve(double* b) {
    for (int c = 0; c < n; ++c) {
      if (piv[c] != c) std::swap(b[c], b[piv[c]]);
      const int last = c + 3 < n - 1 ? c + 3 : n - 1;
      for (int k = c + 1; k <= last; ++k) b[k] -= at(k, c) * b[c];
    }
    for (int c = n - 1; c >= 0; --c) {
      double acc = b[c];
      const int cend = c + 6 < n - 1 ? c + 6 : n - 1;
      for (int col = c + 1; col <= cend; ++col) acc -= at(c, col) * b[col];
      b[c] = acc / at(c, c);
    }
  }
};

// ||g - g_ana||_2 for mesh y and operators A, B.
bool homogeneous_error(MeshProblem& P, const double* y, const double* A, const double* B, double* err) {
  const int n = P.n;
  std::vector<double>& M = P.M7;
  M.assign((size_t)n * 7, 0.0);
  M[3] = 1.0;
  M[(size_t)(n - 1) * 7 + 3] = 1.0;
  for (int i = 1; i < n - 1; ++i)
    for (int o = 0; o < 7; ++o) M[i * 7 + o] = B[i * 7 + o] - P.ks * A[i * 7 + o];
  BandLU lu;
  lu.load(n, M.data());
  if (!lu.factor()) return false;
  std::vector<double>& g = P.g;
  g.assign(n, 0.0);
  g[0] = 1.0;
  lu.solve(g.data());
  double ss = 0.0;
  for (int i = 0; i < n; ++i) {
    const double e = g[i] - g_analytic(y[i], P.ks);
    ss += e * e;
  }
  *err = std::sqrt(ss);
  return std::isfinite(*err);
}

// 1-norm condition number of the banded A ([n][7]): ||A||_1 ||A^-1||_1, the
// inverse's column sums from n banded solves.
double cond1(int n, const double* A) {
  double na = 0.0;
  for (int j = 0; j < n; ++j) {
    double cs = 0.0;
    for (int i = j - 3; i <= j + 3; ++i)
      if (i >= 0 && i < n) cs += std::fabs(A[i * 7 + 3 + (j - i)]);
    na = cs > na ? cs : na;
  }
  BandLU lu;
  lu.load(n, A);
  if (!lu.factor()) return INFINITY;
  std::vector<double> e(n);
  double ni = 0.0;
  for (int j = 0; j < n; ++j) {
    std::fill(e.begin(), e.end(), 0.0);
    e[j] = 1.0;
    lu.solve(e.data());
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += std::fabs(e[i]);
    ni = cs > ni ? cs : ni;
  }
  return na * ni;
}

void place(const MeshProblem& P, const double* x, double* y) {
  for (int i = 0; i < P.n; ++i) y[i] = P.yref[i];
  for (int j = 0; j < P.m; ++j) {
    y[1 + j] = x[j];
    y[P.n - 2 - j] = -x[j];
  }
}

double penalty_term(const MeshProblem& P, const double* x) {
  double ss = 0.0;
  for (int j = 0; j < P.m; ++j) ss += (x[j] - P.xref[j]) * (x[j] - P.xref[j]);
  return P.C * std::sqrt(ss);
}

// Operators of order p of mesh y: the rows within reach of a moved node recomputed.
bool near_wall_rows(const MeshProblem& P, const double* y, double* A, double* B, int p = 2) {
  for (int i = 0; i < P.n; ++i)
    if (i <= P.m + 3 || i >= P.n - 1 - P.m - 3)
      if (!compact_row(P.n, y, i, p, A + 7 * i, B + 7 * i)) return false;
  return true;
}

// The trial-mesh conditions besides the descent: spacing ratios, and the
// conditioning of A2 (given) and of A1 (recomputed near the walls).
bool admissible(const MeshProblem& P, const double* y, const double* A2) {
  if (!spacing_ratio_ok(P.n, y) || !(cond1(P.n, A2) <= P.cond_max)) return false;
  std::vector<double> A1(P.A1), B1(P.B1);
  return near_wall_rows(P, y, A1.data(), B1.data(), 1) && cond1(P.n, A1.data()) <= P.cond1_max;
}

}  // namespace

double band_cond1(int n, const double* A) { return cond1(n, A); }

}  // namespace host
}  // namespace chn

using namespace chn::host;

extern "C" chn_status chn_optimise_mesh(const double* y_ref, int n2, int m, double kstar, double penalty,
                                        int max_iter, double* y_out, double* err_ref, double* err_opt,
                                        int* iterations) {
  if (!y_ref || !y_out || n2 < 9 || m < 1 || 2 * m + 2 > n2 || !(kstar > 0.0) || !std::isfinite(kstar) ||
      !(penalty >= 0.0) || !std::isfinite(penalty) || max_iter < 0)
    return CHN_EINVAL;
  if (y_ref[0] != -1.0 || y_ref[n2 - 1] != 1.0) return CHN_EINVAL;
  for (int i = 0; i + 1 < n2; ++i)
    if (!(y_ref[i + 1] > y_ref[i])) return CHN_EINVAL;
  for (int i = 0; i < n2; ++i)
    if (y_ref[n2 - 1 - i] != -y_ref[i]) return CHN_EINVAL;

  MeshProblem P;
  P.n = n2;
  P.m = m;
  P.ks = kstar;
  P.C = penalty;
  P.yref.assign(y_ref, y_ref + n2);
  P.xref.assign(y_ref + 1, y_ref + 1 + m);
  P.s.resize(m);
  for (int j = 0; j < m; ++j) P.s[j] = y_ref[j + 2] - y_ref[j + 1];
  P.A.resize((size_t)n2 * 7);
  P.B.resize((size_t)n2 * 7);
  if (!compact_bands(n2, y_ref, 2, P.A.data(), P.B.data())) return CHN_EINVAL;
  P.cond_max = 10.0 * cond1(n2, P.A.data());
  if (!std::isfinite(P.cond_max)) return CHN_EINVAL;
  P.A1.resize((size_t)n2 * 7);
  P.B1.resize((size_t)n2 * 7);
  if (!compact_bands(n2, y_ref, 1, P.A1.data(), P.B1.data())) return CHN_EINVAL;
  P.cond1_max = 10.0 * cond1(n2, P.A1.data());
  if (!std::isfinite(P.cond1_max)) return CHN_EINVAL;

  std::vector<double> x = P.xref, yt(n2), xt(m), grad(m), d(m);
  std::vector<double> At(P.A), Bt(P.B), An(P.A), Bn(P.B);
  double e0;
  if (!homogeneous_error(P, y_ref, P.A.data(), P.B.data(), &e0)) return CHN_EUNSTABLE;
  double f = e0, e = e0;

  // L with node j+1 (and its mirror) moved by h, from the operators at x
  auto L_moved = [&](int j, double h, double* out) -> bool {
    xt = x;
    xt[j] += h;
    place(P, xt.data(), yt.data());
    const int i0 = j + 1;  // At, Bt equal the operators at x on entry
    bool ok = true;
    for (int i = i0 - 3; i <= i0 + 3 && ok; ++i) {
      if (i < 0 || i >= n2) continue;
      ok = compact_row(n2, yt.data(), i, 2, &At[i * 7], &Bt[i * 7]) &&
           compact_row(n2, yt.data(), n2 - 1 - i, 2, &At[(n2 - 1 - i) * 7], &Bt[(n2 - 1 - i) * 7]);
    }
    double err = 0.0;
    ok = ok && homogeneous_error(P, yt.data(), At.data(), Bt.data(), &err);
    *out = err + penalty_term(P, xt.data());
    // restore the scratch rows to the operators at x
    for (int i = i0 - 3; i <= i0 + 3; ++i) {
      if (i < 0 || i >= n2) continue;
      for (int row : {i, n2 - 1 - i})
        for (int o = 0; o < 7; ++o) {
          At[row * 7 + o] = P.A[row * 7 + o];
          Bt[row * 7 + o] = P.B[row * 7 + o];
        }
    }
    return ok;
  };

  double t = 1.0;
  int it = 0;
  while (it < max_iter) {
    for (int j = 0; j < m; ++j) {
      const double h = 1e-6 * P.s[j];
      double lp, lm;
      if (!L_moved(j, h, &lp) || !L_moved(j, -h, &lm)) return CHN_EUNSTABLE;
      grad[j] = (lp - lm) / (2.0 * h);
    }
    double slope = 0.0;
    for (int j = 0; j < m; ++j) {
      d[j] = -P.s[j] * P.s[j] * grad[j];
      slope += grad[j] * d[j];
    }
    t *= 2.0;
    bool accepted = false;
    double fn = f, en = e;
    while (t >= 1e-30) {
      for (int j = 0; j < m; ++j) xt[j] = x[j] + t * d[j];
      place(P, xt.data(), yt.data());
      bool increasing = true;
      for (int i = 0; i + 1 < n2 && increasing; ++i) increasing = yt[i + 1] > yt[i];
      if (increasing) {
        An = P.A;
        Bn = P.B;
        double err;
        if (near_wall_rows(P, yt.data(), An.data(), Bn.data()) &&
            homogeneous_error(P, yt.data(), An.data(), Bn.data(), &err)) {
          fn = err + penalty_term(P, xt.data());
          if (fn < f && fn <= f + 1e-4 * t * slope && admissible(P, yt.data(), An.data())) {
            en = err;
            accepted = true;
            break;
          }
        }
      }
      t *= 0.5;
    }
    if (!accepted) break;
    x = xt;
    P.A.swap(An);
    P.B.swap(Bn);
    At = P.A;
    Bt = P.B;
    f = fn;
    e = en;
    ++it;
  }
  place(P, x.data(), y_out);
  if (err_ref) *err_ref = e0;
  if (err_opt) *err_opt = e;
  if (iterations) *iterations = it;
  return CHN_OK;
}
