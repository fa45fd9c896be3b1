// Pencil phase of the RK3 sub-step: everything along the wall-normal lines.
//
// Two lanes per Fourier mode (the real and the imaginary part; the banded
// matrices are real), consecutive lanes on consecutive modes, so every
// wall-normal row of a field is one coalesced [n2][M] complex access.  Each
// banded solve is a forward elimination sweep followed by a back-substitution
// sweep in the opposite direction; the eliminated right-hand sides (and, for
// mode-dependent matrices, the factor rows, computed on the fly) go to a
// scratch buffer between sweeps.  Consecutive solves alternate sweep
// direction so that one sweep finishes a solve and starts the next.
//
//   k_recover : u1, u3 from v and omega2 (continuity), omega1, omega3
//               (Appendix C: velocities and vorticities before the transforms)
//   k_advance : non-linear forcings N_omega2, N_chi, explicit viscous terms,
//               implicit Helmholtz steps for omega2 and chi, Poisson step for v,
//               influence-matrix combination enforcing dv/dy = 0 at the walls
//               (Appendix A eqs. for chi and omega2, Appendix B), plus one
//               extra workgroup for the mean profiles with constant mass flux.
//   k_chi_from_v : chi = (D2 - k^2) v for a new state.
#include "kernels.hpp"

namespace chn {

struct Lane {
  size_t col;   // lane column in [n2][2M] arrays (= 2 m + c)
  int m, c;
  bool act, live, mean;
  double A, B, k2, ik2;
};

__device__ __forceinline__ Lane lane_setup(const PencilGeom& g) {
  Lane L;
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  int m = gl >> 1;
  L.c = gl & 1;
  L.act = m < g.M;
  if (!L.act) m = g.M - 1;
  L.m = m;
  L.col = 2 * (size_t)m + L.c;
  const int kx = m / g.n3, s = m - kx * g.n3, half = g.n3 / 2;
  const int kz = s < half ? s : s - g.n3;
  L.A = g.ka * kx;
  L.B = g.kb * kz;
  L.k2 = L.A * L.A + L.B * L.B;
  L.mean = L.act && m == 0;
  L.live = L.act && m != 0 && s != half;
  L.ik2 = L.live ? 1.0 / L.k2 : 0.0;
  return L;
}

template <int N> __device__ __forceinline__ void push_back(double (&w)[N], double v) {
#pragma unroll
  for (int k = 0; k < N - 1; ++k) w[k] = w[k + 1];
  w[N - 1] = v;
}
template <int N> __device__ __forceinline__ void push_front(double (&w)[N], double v) {
#pragma unroll
  for (int k = N - 1; k > 0; --k) w[k] = w[k - 1];
  w[0] = v;
}
__device__ __forceinline__ double dot7(const double* __restrict__ b, const double (&w)[7]) {
  double r = 0.0;
#pragma unroll
  for (int o = 0; o < 7; ++o) r = fma(b[o], w[o], r);
  return r;
}
// eliminated value with a precomputed L row: r - L0 y(dist 3) - L1 y(dist 2) - L2 y(dist 1)
__device__ __forceinline__ double elim3(double r, const double* __restrict__ l, const double (&yb)[3]) {
  return r - l[0] * yb[0] - l[1] * yb[1] - l[2] * yb[2];
}
// back-substitution: (y - U1 x(dist 1) - U2 x(dist 2) - U3 x(dist 3)) / pivot
__device__ __forceinline__ double back3(double y, const double* __restrict__ U, const double (&xb)[3]) {
  return (y - U[1] * xb[0] - U[2] * xb[1] - U[3] * xb[2]) * U[0];
}
__device__ __forceinline__ void push_x(double (&xb)[3], double x) {
  xb[2] = xb[1];
  xb[1] = xb[0];
  xb[0] = x;
}

template <typename T> __device__ __forceinline__ double2 load_c(const T* p, size_t idx);
template <> __device__ __forceinline__ double2 load_c<double>(const double* p, size_t idx) {
  return reinterpret_cast<const double2*>(p)[idx];
}
template <> __device__ __forceinline__ double2 load_c<float>(const float* p, size_t idx) {
  const float2 f = reinterpret_cast<const float2*>(p)[idx];
  return make_double2((double)f.x, (double)f.y);
}

// ---------------------------------------------------------------- recovery
template <typename TP>
__global__ void __launch_bounds__(256) k_recover(RecoverArgs<TP> a) {
  const PencilGeom& g = a.g;
  const Lane L = lane_setup(g);
  const int n = g.n2;
  const size_t st = 2 * (size_t)g.M;
  const size_t col = L.col;

  // R1, downward: eliminate A1 (dv) = B1 v; copy v for the transforms
  {
    double w[7] = {0, 0, 0, 0, 0, 0, 0};
    double yb[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) w[3 + k] = a.v[k * st + col];
    for (int i = 0; i < n; ++i) {
      w[6] = (i + 3 < n) ? a.v[(i + 3) * st + col] : 0.0;
      const double yi = elim3(dot7(g.B1 + i * 7, w), g.L1d + i * 3, yb);
      if (L.act) {
        a.S0[i * st + col] = yi;
        a.out[1][i * st + col] = (TP)w[3];
      }
      yb[0] = yb[1];
      yb[1] = yb[2];
      yb[2] = yi;
      push_back(w, 0.0);
    }
  }
  // R2, upward: finish dv; u1, u3; eliminate A1 (du) = B1 u for both
  {
    double xb[3] = {0, 0, 0};
    double w1[7] = {0, 0, 0, 0, 0, 0, 0}, w3[7] = {0, 0, 0, 0, 0, 0, 0};
    double y1b[3] = {0, 0, 0}, y3b[3] = {0, 0, 0};
    for (int i = n - 1; i >= -3; --i) {
      double u1 = 0.0, u3 = 0.0;
      if (i >= 0) {
        const double dv = back3(a.S0[i * st + col], g.U1d + i * 4, xb);
        push_x(xb, dv);
        const double dvo = __shfl_xor(dv, 1);
        const double dre = L.c ? dvo : dv, dim = L.c ? dv : dvo;
        const double2 om = reinterpret_cast<const double2*>(a.om2)[(size_t)i * g.M + L.m];
        if (L.live) {
          u1 = L.c == 0 ? -(L.A * dim - L.B * om.y) * L.ik2 : (L.A * dre - L.B * om.x) * L.ik2;
          u3 = L.c == 0 ? -(L.B * dim + L.A * om.y) * L.ik2 : (L.B * dre + L.A * om.x) * L.ik2;
        } else if (L.mean && L.c == 0) {
          u1 = a.U1[i];
          u3 = a.U3[i];
        }
        if (L.act) {
          a.out[0][i * st + col] = (TP)u1;
          a.out[2][i * st + col] = (TP)u3;
        }
      }
      push_front(w1, u1);
      push_front(w3, u3);
      const int r = i + 3;
      if (r <= n - 1) {
        const double* b = g.B1 + r * 7;
        const double* l = g.L1u + r * 3;
        const double y1 = elim3(dot7(b, w1), l, y1b);
        const double y3 = elim3(dot7(b, w3), l, y3b);
        if (L.act) {
          a.S1[r * st + col] = y1;
          a.S2[r * st + col] = y3;
        }
        y1b[0] = y1b[1]; y1b[1] = y1b[2]; y1b[2] = y1;
        y3b[0] = y3b[1]; y3b[1] = y3b[2]; y3b[2] = y3;
      }
    }
  }
  // R3, downward: finish du1, du3; omega1 = du3 - i b v, omega3 = i a v - du1
  {
    double x1[3] = {0, 0, 0}, x3[3] = {0, 0, 0};
    for (int r = 0; r < n; ++r) {
      const double* U = g.U1u + r * 4;
      const double du1 = back3(a.S1[r * st + col], U, x1);
      const double du3 = back3(a.S2[r * st + col], U, x3);
      push_x(x1, du1);
      push_x(x3, du3);
      const double2 v = reinterpret_cast<const double2*>(a.v)[(size_t)r * g.M + L.m];
      const double o1 = L.c == 0 ? du3 + L.B * v.y : du3 - L.B * v.x;
      const double o3 = L.c == 0 ? -L.A * v.y - du1 : L.A * v.x - du1;
      if (L.act) {
        a.out[3][r * st + col] = (TP)o1;
        a.out[4][r * st + col] = (TP)o3;
      }
    }
  }
}

// ---------------------------------------------------------------- mean modes
template <typename TH>
__device__ void mean_block(const AdvanceArgs<TH>& a) {
  const PencilGeom& g = a.g;
  const int n = g.n2;
  const int t = threadIdx.x;
  double* NU = a.mean_scr + 3 * (size_t)n * 5;
  double* NW = NU + n;
  // plane means of H1 and H3: float64 sums of the per-row sums over x
  if (t < 64) {
    for (int r = t; r < n; r += 64) {
      double s1 = 0.0, s3 = 0.0;
      const double* p1 = a.rowsum + (size_t)r * a.p3;
      const double* p3 = a.rowsum + ((size_t)n + r) * a.p3;
      for (int z = 0; z < a.p3; ++z) {
        s1 += p1[z];
        s3 += p3[z];
      }
      NU[r] = s1 * a.inv_p1p3;
      NW[r] = s3 * a.inv_p1p3;
    }
  }
  __syncthreads();
  // three serial solves with M0 = A2 - cb B2 (Dirichlet end rows): role 0 the
  // particular U1, role 1 the mass-flux influence function (rhs 1), role 2 U3
  const double cb = a.dt * a.be * a.nu, f2 = a.al * a.dt * a.nu;
  if (t < 3) {
    const double* X = t == 2 ? a.U3 : a.U1;
    const double* Nn = t == 2 ? NW : NU;
    const double* No = t == 2 ? a.nw_old : a.nu_old;
    double* scr = a.mean_scr + (size_t)t * n * 5;
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    double yb[3] = {0, 0, 0};
    for (int r = 0; r < n; ++r) {
      double m7[7], rhs = 0.0;
      if (r == 0 || r == n - 1) {
        for (int o = 0; o < 7; ++o) m7[o] = o == 3 ? 1.0 : 0.0;
      } else {
        const double* A2r = g.A2 + r * 7;
        const double* B2r = g.B2 + r * 7;
        for (int o = 0; o < 7; ++o) {
          m7[o] = A2r[o] - cb * B2r[o];
          const int j = r + o - 3;
          if (j < 0 || j >= n) continue;
          if (t == 1) {
            rhs += A2r[o];
          } else {
            const double q = X[j] + a.dt * (a.ga * Nn[j] + a.ze * No[j]);
            rhs += A2r[o] * q + f2 * B2r[o] * X[j];
          }
        }
      }
      for (int d = 3; d >= 1; --d) {
        const double* U = uh[3 - d];
        const double lm = m7[3 - d] * U[0];
        m7[4 - d] -= lm * U[1];
        m7[5 - d] -= lm * U[2];
        m7[6 - d] -= lm * U[3];
        rhs -= lm * yb[3 - d];
      }
      double* s = scr + (size_t)r * 5;
      s[0] = 1.0 / m7[3];
      s[1] = m7[4];
      s[2] = m7[5];
      s[3] = m7[6];
      s[4] = rhs;
      for (int q = 0; q < 2; ++q)
        for (int k = 0; k < 4; ++k) uh[q][k] = uh[q + 1][k];
      for (int k = 0; k < 4; ++k) uh[2][k] = s[k];
      yb[0] = yb[1];
      yb[1] = yb[2];
      yb[2] = rhs;
    }
    double xb[3] = {0, 0, 0};
    for (int r = n - 1; r >= 0; --r) {
      double* s = scr + (size_t)r * 5;
      const double x = (s[4] - s[1] * xb[0] - s[2] * xb[1] - s[3] * xb[2]) * s[0];
      s[4] = x;
      push_x(xb, x);
    }
  }
  __syncthreads();
  // constant mass flux: U1 = U_p + phi U_h with w.U1 = Q
  if (t < 64) {
    double wp = 0.0, wh = 0.0;
    for (int r = t; r < n; r += 64) {
      wp += g.quad[r] * a.mean_scr[(size_t)r * 5 + 4];
      wh += g.quad[r] * a.mean_scr[((size_t)n + r) * 5 + 4];
    }
    for (int off = 32; off > 0; off >>= 1) {
      wp += __shfl_xor(wp, off);
      wh += __shfl_xor(wh, off);
    }
    const double phi = (a.mass_flux - wp) / wh;
    for (int r = t; r < n; r += 64) {
      a.U1[r] = a.mean_scr[(size_t)r * 5 + 4] + phi * a.mean_scr[((size_t)n + r) * 5 + 4];
      a.U3[r] = a.mean_scr[(2 * (size_t)n + r) * 5 + 4];
      a.nu_old[r] = NU[r];
      a.nw_old[r] = NW[r];
    }
    if (t == 0) a.mean_out[0] = phi / (a.dt * (a.al + a.be));
  }
}

// ---------------------------------------------------------------- advance
template <typename TH>
__global__ void __launch_bounds__(256) k_advance(AdvanceArgs<TH> a) {
  if (blockIdx.x == gridDim.x - 1) {
    mean_block(a);
    return;
  }
  const PencilGeom& g = a.g;
  const Lane L = lane_setup(g);
  const int n = g.n2;
  const size_t st = 2 * (size_t)g.M;
  const size_t M = g.M;
  const size_t col = L.col;
  const double cb = a.dt * a.be * a.nu;
  const double f1 = 1.0 - a.al * a.dt * a.nu * L.k2;
  const double f2 = a.al * a.dt * a.nu;
  const double dga = a.dt * a.ga, dze = a.dt * a.ze;
  const double hk = 1.0 + cb * L.k2;

  auto gval = [&](int i) -> double {
    if (!L.live) return 0.0;
    const double2 h1 = load_c<TH>(a.H[0], (size_t)i * M + L.m);
    const double2 h3 = load_c<TH>(a.H[2], (size_t)i * M + L.m);
    return L.c == 0 ? -(L.A * h1.y + L.B * h3.y) : (L.A * h1.x + L.B * h3.x);
  };

  // S1, downward: G = i(a H1 + b H3); eliminate A1 (dG) = B1 G
  {
    double w[7] = {0, 0, 0, 0, 0, 0, 0};
    double yb[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) w[3 + k] = gval(k);
    for (int i = 0; i < n; ++i) {
      w[6] = (i + 3 < n) ? gval(i + 3) : 0.0;
      const double yi = elim3(dot7(g.B1 + i * 7, w), g.L1d + i * 3, yb);
      if (L.act) a.S[0][i * st + col] = yi;
      yb[0] = yb[1];
      yb[1] = yb[2];
      yb[2] = yi;
      push_back(w, 0.0);
    }
  }
  // S2, upward: finish dG; N_chi, N_omega2; right-hand sides of the implicit
  // steps (lag 3 rows); eliminate the Helmholtz matrix (factored on the fly)
  // for chi_p, omega2 and the homogeneous chi_h (lane c = 0: 1 at the lower
  // wall, lane c = 1: 1 at the upper wall)
  {
    double xb[3] = {0, 0, 0};
    double qc[7] = {0, 0, 0, 0, 0, 0, 0}, xc[7] = {0, 0, 0, 0, 0, 0, 0};
    double qo[7] = {0, 0, 0, 0, 0, 0, 0}, xo[7] = {0, 0, 0, 0, 0, 0, 0};
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    double ycb[3] = {0, 0, 0}, yob[3] = {0, 0, 0}, yhb[3] = {0, 0, 0};
    for (int i = n - 1; i >= -3; --i) {
      double qcv = 0.0, xcv = 0.0, qov = 0.0, xov = 0.0;
      if (i >= 0) {
        const double dG = back3(a.S[0][i * st + col], g.U1d + i * 4, xb);
        push_x(xb, dG);
        double nchi = 0.0, nom = 0.0;
        if (L.live) {
          const size_t mi = (size_t)i * M + L.m;
          const double2 h1 = load_c<TH>(a.H[0], mi);
          const double2 h2 = load_c<TH>(a.H[1], mi);
          const double2 h3 = load_c<TH>(a.H[2], mi);
          nchi = -dG - L.k2 * (L.c == 0 ? h2.x : h2.y);
          nom = L.c == 0 ? (-L.B * h1.y + L.A * h3.y) : (L.B * h1.x - L.A * h3.x);
        }
        const size_t ix = i * st + col;
        xcv = a.chi[ix];
        xov = a.om2[ix];
        qcv = f1 * xcv + dga * nchi + dze * a.nchi_old[ix];
        qov = f1 * xov + dga * nom + dze * a.nom_old[ix];
        if (L.act) {
          a.nchi_old[ix] = nchi;
          a.nom_old[ix] = nom;
        }
      }
      push_front(qc, qcv);
      push_front(xc, xcv);
      push_front(qo, qov);
      push_front(xo, xov);
      const int r = i + 3;
      if (r <= n - 1) {
        double m7[7], rc = 0.0, ro = 0.0, rh = 0.0;
        if (r == 0 || r == n - 1) {
#pragma unroll
          for (int o = 0; o < 7; ++o) m7[o] = o == 3 ? 1.0 : 0.0;
          rh = (r == 0) == (L.c == 0) ? 1.0 : 0.0;
        } else {
          const double* A2r = g.A2 + r * 7;
          const double* B2r = g.B2 + r * 7;
#pragma unroll
          for (int o = 0; o < 7; ++o) {
            rc += A2r[o] * qc[o] + f2 * B2r[o] * xc[o];
            ro += A2r[o] * qo[o] + f2 * B2r[o] * xo[o];
            m7[o] = hk * A2r[o] - cb * B2r[o];
          }
        }
        // upward elimination of columns r+3, r+2, r+1
#pragma unroll
        for (int d = 3; d >= 1; --d) {
          const double lm = m7[3 + d] * uh[3 - d][0];
          m7[2 + d] -= lm * uh[3 - d][1];
          m7[1 + d] -= lm * uh[3 - d][2];
          m7[0 + d] -= lm * uh[3 - d][3];
          rc -= lm * ycb[3 - d];
          ro -= lm * yob[3 - d];
          rh -= lm * yhb[3 - d];
        }
        const double u0 = 1.0 / m7[3];
        const size_t mr = (size_t)r * M + L.m;
        if (L.act && L.c == 0) {
          a.SU[0][mr] = u0;
          a.SU[1][mr] = m7[2];
          a.SU[2][mr] = m7[1];
          a.SU[3][mr] = m7[0];
        }
        const size_t ix = r * st + col;
        if (L.act) {
          a.S[1][ix] = rc;
          a.S[2][ix] = ro;
          a.S[3][ix] = rh;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          uh[0][k] = uh[1][k];
          uh[1][k] = uh[2][k];
        }
        uh[2][0] = u0; uh[2][1] = m7[2]; uh[2][2] = m7[1]; uh[2][3] = m7[0];
        ycb[0] = ycb[1]; ycb[1] = ycb[2]; ycb[2] = rc;
        yob[0] = yob[1]; yob[1] = yob[2]; yob[2] = ro;
        yhb[0] = yhb[1]; yhb[1] = yhb[2]; yhb[2] = rh;
      }
    }
  }
  // S3, downward: finish chi_p, omega2 (final), chi_h; right-hand sides of
  // the Poisson step (lag 3); eliminate P = B2 - k^2 A2 (on the fly) for v_p, v_h
  {
    double xcb[3] = {0, 0, 0}, xob[3] = {0, 0, 0}, xhb[3] = {0, 0, 0};
    double wcp[7] = {0, 0, 0, 0, 0, 0, 0}, wch[7] = {0, 0, 0, 0, 0, 0, 0};
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    double yvb[3] = {0, 0, 0}, yhb[3] = {0, 0, 0};
    for (int i = 0; i <= n + 2; ++i) {
      double cp = 0.0, ch = 0.0;
      if (i < n) {
        const size_t mi = (size_t)i * M + L.m;
        const double U[4] = {a.SU[0][mi], a.SU[1][mi], a.SU[2][mi], a.SU[3][mi]};
        const size_t ix = i * st + col;
        cp = back3(a.S[1][ix], U, xcb);
        const double om = back3(a.S[2][ix], U, xob);
        ch = back3(a.S[3][ix], U, xhb);
        push_x(xcb, cp);
        push_x(xob, om);
        push_x(xhb, ch);
        if (L.act) {
          a.om2[ix] = L.live ? om : 0.0;
          a.chi[ix] = cp;
          a.S[4][ix] = ch;
        }
      }
      push_back(wcp, cp);
      push_back(wch, ch);
      const int r = i - 3;
      if (r >= 0) {
        double p7[7], rv = 0.0, rhv = 0.0;
        if (r == 0 || r == n - 1) {
#pragma unroll
          for (int o = 0; o < 7; ++o) p7[o] = o == 3 ? 1.0 : 0.0;
        } else {
          const double* A2r = g.A2 + r * 7;
          const double* B2r = g.B2 + r * 7;
#pragma unroll
          for (int o = 0; o < 7; ++o) {
            rv += A2r[o] * wcp[o];
            rhv += A2r[o] * wch[o];
            p7[o] = B2r[o] - L.k2 * A2r[o];
          }
        }
        // downward elimination of columns r-3, r-2, r-1
#pragma unroll
        for (int d = 3; d >= 1; --d) {
          const double lm = p7[3 - d] * uh[3 - d][0];
          p7[4 - d] -= lm * uh[3 - d][1];
          p7[5 - d] -= lm * uh[3 - d][2];
          p7[6 - d] -= lm * uh[3 - d][3];
          rv -= lm * yvb[3 - d];
          rhv -= lm * yhb[3 - d];
        }
        const double u0 = 1.0 / p7[3];
        const size_t mr = (size_t)r * M + L.m;
        if (L.act && L.c == 0) {
          a.SU[4][mr] = u0;
          a.SU[5][mr] = p7[4];
          a.SU[6][mr] = p7[5];
          a.SU[7][mr] = p7[6];
        }
        const size_t ix = r * st + col;
        if (L.act) {
          a.S[5][ix] = rv;
          a.S[6][ix] = rhv;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          uh[0][k] = uh[1][k];
          uh[1][k] = uh[2][k];
        }
        uh[2][0] = u0; uh[2][1] = p7[4]; uh[2][2] = p7[5]; uh[2][3] = p7[6];
        yvb[0] = yvb[1]; yvb[1] = yvb[2]; yvb[2] = rv;
        yhb[0] = yhb[1]; yhb[1] = yhb[2]; yhb[2] = rhv;
      }
    }
  }
  // S4, upward: finish v_p, v_h; wall derivatives (D1 v)_{0, n2-1} by the
  // dense wall rows of D1; 2x2 influence system for c_lo, c_hi
  double clo_c = 0.0, chi_c = 0.0;
  {
    double xvb[3] = {0, 0, 0}, xhb[3] = {0, 0, 0};
    double gplo = 0.0, gphi = 0.0, ghlo = 0.0, ghhi = 0.0;
    for (int r = n - 1; r >= 0; --r) {
      const size_t mr = (size_t)r * M + L.m;
      const double U[4] = {a.SU[4][mr], a.SU[5][mr], a.SU[6][mr], a.SU[7][mr]};
      const size_t ix = r * st + col;
      const double vp = back3(a.S[5][ix], U, xvb);
      const double vh = back3(a.S[6][ix], U, xhb);
      push_x(xvb, vp);
      push_x(xhb, vh);
      if (L.act) {
        a.v[ix] = vp;
        a.S[7][ix] = vh;
      }
      gplo = fma(g.clo[r], vp, gplo);
      gphi = fma(g.chi[r], vp, gphi);
      ghlo = fma(g.clo[r], vh, ghlo);
      ghhi = fma(g.chi[r], vh, ghhi);
    }
    const double oglo = __shfl_xor(ghlo, 1), oghi = __shfl_xor(ghhi, 1);
    const double m00 = L.c == 0 ? ghlo : oglo;  // lower-wall homogeneous solution, lower wall
    const double m10 = L.c == 0 ? ghhi : oghi;  // ... upper wall
    const double m01 = L.c == 0 ? oglo : ghlo;  // upper-wall homogeneous solution, lower wall
    const double m11 = L.c == 0 ? oghi : ghhi;
    if (L.live) {
      const double det = m00 * m11 - m01 * m10;
      clo_c = (-gplo * m11 + gphi * m01) / det;
      chi_c = (-gphi * m00 + gplo * m10) / det;
    }
  }
  // S5: v = v_p + c_lo v_lo + c_hi v_hi, chi likewise
  for (int r = 0; r < n; ++r) {
    const size_t ix = r * st + col;
    const double vh = a.S[7][ix], ch = a.S[4][ix];
    const double vho = __shfl_xor(vh, 1), cho = __shfl_xor(ch, 1);
    const double vlo = L.c == 0 ? vh : vho, vhi = L.c == 0 ? vho : vh;
    const double clo = L.c == 0 ? ch : cho, chh = L.c == 0 ? cho : ch;
    if (L.act) {
      const double v = a.v[ix] + clo_c * vlo + chi_c * vhi;
      const double c = a.chi[ix] + clo_c * clo + chi_c * chh;
      a.v[ix] = L.live ? v : 0.0;
      a.chi[ix] = L.live ? c : 0.0;
    }
  }
}

// ---------------------------------------------------------------- set state
__global__ void __launch_bounds__(256) k_chi_from_v(ChiArgs a) {
  const PencilGeom& g = a.g;
  const Lane L = lane_setup(g);
  const int n = g.n2;
  const size_t st = 2 * (size_t)g.M;
  const size_t col = L.col;
  auto vin = [&](int i) -> double { return L.live ? a.vin[i * st + col] : 0.0; };
  double w[7] = {0, 0, 0, 0, 0, 0, 0};
  double yb[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) w[3 + k] = vin(k);
  for (int i = 0; i < n; ++i) {
    w[6] = (i + 3 < n) ? vin(i + 3) : 0.0;
    const double yi = elim3(dot7(g.B2 + i * 7, w), g.L2d + i * 3, yb);
    if (L.act) {
      a.S0[i * st + col] = yi;
      a.v[i * st + col] = w[3];
      a.om2[i * st + col] = L.live ? a.omin[i * st + col] : 0.0;
    }
    yb[0] = yb[1];
    yb[1] = yb[2];
    yb[2] = yi;
    push_back(w, 0.0);
  }
  double xb[3] = {0, 0, 0};
  for (int i = n - 1; i >= 0; --i) {
    const double d2 = back3(a.S0[i * st + col], g.U2d + i * 4, xb);
    push_x(xb, d2);
    if (L.act) a.chi[i * st + col] = L.live ? d2 - L.k2 * vin(i) : 0.0;
  }
}

// ---------------------------------------------------------------- diagnostics
__global__ void __launch_bounds__(256) k_info(InfoArgs a) {
  __shared__ double red[3][4];
  const int n = a.g.n2;
  double cm = 0.0, wm = 0.0;
  bool bad = false;
  for (size_t e = threadIdx.x; e < (size_t)n * a.p3; e += blockDim.x) {
    const float c = a.rowcfl[e];
    if (!isfinite(c)) bad = true;
    cm = fmax(cm, (double)c);
  }
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    wm += a.g.quad[r] * a.U1[r];
    if (!isfinite(a.U1[r])) bad = true;
  }
  double b = bad ? 1.0 : 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    cm = fmax(cm, __shfl_xor(cm, off));
    wm += __shfl_xor(wm, off);
    b = fmax(b, __shfl_xor(b, off));
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wid] = cm;
    red[1][wid] = wm;
    red[2][wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double c = 0.0, m = 0.0, bb = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      c = fmax(c, red[0][w]);
      m += red[1][w];
      bb = fmax(bb, red[2][w]);
    }
    double dlo = 0.0, dhi = 0.0;
    for (int r = 0; r < n; ++r) {
      dlo += a.g.clo[r] * a.U1[r];
      dhi += a.g.chi[r] * a.U1[r];
    }
    a.out[0] = c * a.dt;
    a.out[1] = m;
    a.out[2] = sqrt(a.nu * fabs(dlo));
    a.out[3] = sqrt(a.nu * fabs(dhi));
    a.out[4] = a.mean_out[0];
    a.out[5] = bb;
  }
}

__global__ void k_d2f(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void k_f2d(const float* __restrict__ in, double* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

// ---------------------------------------------------------------- launchers
static inline unsigned pencil_blocks(int M) { return (unsigned)((2 * (size_t)M + 255) / 256); }

template <typename TP> hipError_t launch_recover(const RecoverArgs<TP>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_recover<TP>), dim3(pencil_blocks(a.g.M)), dim3(256), 0, st, a);
  return hipGetLastError();
}
template <typename TH> hipError_t launch_advance(const AdvanceArgs<TH>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_advance<TH>), dim3(pencil_blocks(a.g.M) + 1), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_chi_from_v(const ChiArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_chi_from_v, dim3(pencil_blocks(a.g.M)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_info(const InfoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_info, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_convert_d2f(const double* in, float* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_d2f, dim3(1024), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}
hipError_t launch_convert_f2d(const float* in, double* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_f2d, dim3(1024), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

template hipError_t launch_recover<double>(const RecoverArgs<double>&, hipStream_t);
template hipError_t launch_recover<float>(const RecoverArgs<float>&, hipStream_t);
template hipError_t launch_advance<double>(const AdvanceArgs<double>&, hipStream_t);
template hipError_t launch_advance<float>(const AdvanceArgs<float>&, hipStream_t);

}  // namespace chn
