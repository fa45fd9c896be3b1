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
//               extra workgroup for the mean profiles with constant mass flux;
//               fused with the recovery of the next sub-step's fields.
//   k_homog   : per time step size, the factor tables, homogeneous solutions
//               and wall-derivative vectors k_advance reads.
//   k_pressure : the filtered pressure of the low-storage database (Section 3.1).
//   k_chi_from_v : chi = (D2 - k^2) v for a new state.
#include "kernels.hpp"

namespace chn {

struct Lane {
  size_t col;   // lane column in [n2][2M] arrays (= 2 m + c)
  int m, c;
  bool act, live, mean;
  double A, B, k2, ik2;
};

__device__ __forceinline__ Lane lane_setup(const PencilGeom& g, int bx) {
  Lane L;
  const int gl = bx * blockDim.x + threadIdx.x;
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

template <typename T, int N> __device__ __forceinline__ void push_back(T (&w)[N], T v) {
#pragma unroll
  for (int k = 0; k < N - 1; ++k) w[k] = w[k + 1];
  w[N - 1] = v;
}
template <typename T, int N> __device__ __forceinline__ void push_front(T (&w)[N], T v) {
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

// Row r of the Helmholtz matrix (1 + cb k^2) A2 - cb B2 (hk = 1 + cb k^2),
// and of the Poisson matrix B2 - k^2 A2; Dirichlet rows at the walls.  Band
// order: m[3] diagonal, m[3 + d] the entry d columns to the right.
__device__ __forceinline__ void helm_row(double (&m)[7], const double* __restrict__ A2r,
                                         const double* __restrict__ B2r, bool wall, double hk, double cb) {
#pragma unroll
  for (int o = 0; o < 7; ++o) m[o] = wall ? (o == 3 ? 1.0 : 0.0) : hk * A2r[o] - cb * B2r[o];
}
__device__ __forceinline__ void pois_row(double (&m)[7], const double* __restrict__ A2r,
                                         const double* __restrict__ B2r, bool wall, double k2) {
#pragma unroll
  for (int o = 0; o < 7; ++o) m[o] = wall ? (o == 3 ? 1.0 : 0.0) : B2r[o] - k2 * A2r[o];
}
// One row of an LU factorisation on the fly, upward (rows processed from
// n - 1 to 0): eliminates the entries m[4..6] with the U rows uh[2], uh[1],
// uh[0] of rows r + 1, r + 2, r + 3 (uh = {1/pivot, u1, u2, u3}, u_t the
// entry at distance t towards row 0).  lm[3 - d] is the multiplier of the
// row at distance d; the caller applies the same multipliers to its
// right-hand sides.  The advance and homogeneous-solution kernels both
// factor through these two functions, so their factors agree to the bit.
__device__ __forceinline__ void factor_up(double (&m)[7], const double (&uh)[3][4], double (&lm)[3]) {
#pragma unroll
  for (int d = 3; d >= 1; --d) {
    lm[3 - d] = m[3 + d] * uh[3 - d][0];
    m[2 + d] -= lm[3 - d] * uh[3 - d][1];
    m[1 + d] -= lm[3 - d] * uh[3 - d][2];
    m[0 + d] -= lm[3 - d] * uh[3 - d][3];
  }
}
// The same downward (rows 0 to n - 1): eliminates m[0..2].
__device__ __forceinline__ void factor_down(double (&m)[7], const double (&uh)[3][4], double (&lm)[3]) {
#pragma unroll
  for (int d = 3; d >= 1; --d) {
    lm[3 - d] = m[3 - d] * uh[3 - d][0];
    m[4 - d] -= lm[3 - d] * uh[3 - d][1];
    m[5 - d] -= lm[3 - d] * uh[3 - d][2];
    m[6 - d] -= lm[3 - d] * uh[3 - d][3];
  }
}
// shift the U-row history by one row
__device__ __forceinline__ void push_u(double (&uh)[3][4], double u0, double u1, double u2, double u3) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uh[0][k] = uh[1][k];
    uh[1][k] = uh[2][k];
  }
  uh[2][0] = u0; uh[2][1] = u1; uh[2][2] = u2; uh[2][3] = u3;
}

template <typename T> __device__ __forceinline__ double2 load_c(const T* p, size_t idx);
template <> __device__ __forceinline__ double2 load_c<double>(const double* p, size_t idx) {
  return reinterpret_cast<const double2*>(p)[idx];
}
template <> __device__ __forceinline__ double2 load_c<float>(const float* p, size_t idx) {
  const float2 f = reinterpret_cast<const float2*>(p)[idx];
  return make_double2((double)f.x, (double)f.y);
}


// Element at a byte offset from a (wave-uniform) base.  These are the
// streaming accesses of the sweeps: every field row a sweep touches is used
// again only a whole sweep later, far beyond the caches, so loads and stores
// carry the non-temporal hint.
template <typename T> __device__ __forceinline__ T ldn(const T* base, unsigned boff) {
  return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff));
}
template <typename T> __device__ __forceinline__ void stn(T* base, unsigned boff, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff));
}

// one real component (c = 0: real part, 1: imaginary part) of a complex entry
template <typename T> __device__ __forceinline__ double load_r(const T* p, size_t idx, int c) {
  return (double)p[2 * idx + c];
}

// ---------------------------------------------------------------- recovery
template <typename TP>
__global__ void __launch_bounds__(256) k_recover(RecoverArgs<TP> a, const double* __restrict__ B1,
                                                 const double* __restrict__ L1d, const double* __restrict__ U1d,
                                                 const double* __restrict__ L1u, const double* __restrict__ U1u) {
  // tables as noalias parameters: wave-uniform row reads through the scalar cache
  const PencilGeom& g = a.g;
  const Lane L = lane_setup(g, blockIdx.x);
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
      const double yi = elim3(dot7(B1 + i * 7, w), L1d + i * 3, yb);
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
        const double dv = back3(a.S0[i * st + col], U1d + i * 4, xb);
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
      if (!a.omega) continue;  // velocities only
      push_front(w1, u1);
      push_front(w3, u3);
      const int r = i + 3;
      if (r <= n - 1) {
        const double* b = B1 + r * 7;
        const double* l = L1u + r * 3;
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
  if (a.omega) {
    double x1[3] = {0, 0, 0}, x3[3] = {0, 0, 0};
    for (int r = 0; r < n; ++r) {
      const double* U = U1u + r * 4;
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

// ---------------------------------------------------------------- pipelining
// Software pipeline over T steps of a sweep: the loads of step t + D are
// issued right after step t is processed, so D rows of loads are in flight
// while the recurrence advances (the sweeps are otherwise latency-bound:
// one dependent row per iteration).  load(t, buf) must accept every t >= 0
// (rows outside the line are clamped, their values unused) and load
// unconditionally: a load under a branch makes the compiler wait for all
// outstanding loads where the branch joins, which serialises the pipeline.
// The steady state runs whole groups of D steps with no bounds test; the
// last T mod D steps follow without loads.
template <int D, typename B, typename LoadF, typename StepF>
__device__ __forceinline__ void pipeline(int T, LoadF&& load, StepF&& step) {
  B buf[D];
#pragma unroll
  for (int k = 0; k < D; ++k) load(k, buf[k]);
  int t0 = 0;
  for (; t0 + D <= T; t0 += D) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      step(t0 + k, buf[k]);
      load(t0 + k + D, buf[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < D - 1; ++k)
    if (t0 + k < T) step(t0 + k, buf[k]);
}

template <typename T> __device__ __forceinline__ void store_c(T* p, size_t idx, double x, double y);
template <> __device__ __forceinline__ void store_c<double>(double* p, size_t idx, double x, double y) {
  reinterpret_cast<double2*>(p)[idx] = make_double2(x, y);
}
template <> __device__ __forceinline__ void store_c<float>(float* p, size_t idx, double x, double y) {
  reinterpret_cast<float2*>(p)[idx] = make_float2((float)x, (float)y);
}

// ---------------------------------------------------------------- guard
// True when the sub-step must leave the state untouched: an earlier sub-step
// failed, or this one's CFL number (the x pass's maximum times dt) is not
// finite or above the limit.  Uniform over the launch.
template <typename TH, typename TP> __device__ __forceinline__ bool unstable(const AdvanceArgs<TH, TP>& a) {
  if (!a.guard) return false;
  const unsigned bits = __hip_atomic_load(a.guard, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned fail = __hip_atomic_load(a.guard + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return fail != 0u || bits >= kGuardNonFinite || (double)__uint_as_float(bits) * a.dt > a.cfl_limit;
}

// ---------------------------------------------------------------- mean modes
// One workgroup: U1 with constant mass flux and U3 (float64, Section 2.1),
// then the (0,0) entries of the next sub-step's velocity/vorticity fields.
// It also keeps the guard's books: the fail code of an unstable sub-step,
// the count of completed steps.
template <typename TH, typename TP>
__device__ void mean_block(const AdvanceArgs<TH, TP>& a) {
  const PencilGeom& g = a.g;
  const int n = g.n2;
  const int t = threadIdx.x;
  if (unstable(a)) {
    if (t == 0 && a.guard[1] == 0u) a.guard[1] = 1u + 3u * a.guard[2] + (unsigned)a.substep;
    return;
  }
  if (a.guard && t == 0 && a.substep == 2) a.guard[2] += 1u;
  double* NU = a.mean_scr + 3 * (size_t)n * 5;
  double* NW = NU + n;
  double* DU = NW + n;  // D1 U1, D1 U3
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
  // particular U1, role 1 the mass-flux influence function (rhs A2 1), role 2 U3
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
      double* sr = scr + (size_t)r * 5;
      sr[0] = 1.0 / m7[3];
      sr[1] = m7[4];
      sr[2] = m7[5];
      sr[3] = m7[6];
      sr[4] = rhs;
      for (int q = 0; q < 2; ++q)
        for (int k = 0; k < 4; ++k) uh[q][k] = uh[q + 1][k];
      for (int k = 0; k < 4; ++k) uh[2][k] = sr[k];
      yb[0] = yb[1];
      yb[1] = yb[2];
      yb[2] = rhs;
    }
    double xb[3] = {0, 0, 0};
    for (int r = n - 1; r >= 0; --r) {
      double* sr = scr + (size_t)r * 5;
      const double x = (sr[4] - sr[1] * xb[0] - sr[2] * xb[1] - sr[3] * xb[2]) * sr[0];
      sr[4] = x;
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
  __syncthreads();
  // D1 U1 (lane 0) and D1 U3 (lane 1) with the precomputed LU of A1
  if (t < 2) {
    const double* X = t == 0 ? a.U1 : a.U3;
    double* Y = DU + (size_t)t * n;
    double yb[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
      double r = 0.0;
      for (int o = 0; o < 7; ++o) {
        const int j = i + o - 3;
        if (j >= 0 && j < n) r += g.B1[i * 7 + o] * X[j];
      }
      const double yi = elim3(r, g.L1d + i * 3, yb);
      Y[i] = yi;
      yb[0] = yb[1];
      yb[1] = yb[2];
      yb[2] = yi;
    }
    double xb[3] = {0, 0, 0};
    for (int i = n - 1; i >= 0; --i) {
      const double x = back3(Y[i], g.U1d + i * 4, xb);
      Y[i] = x;
      push_x(xb, x);
    }
  }
  __syncthreads();
  // (0,0) entries of the next sub-step's fields: u1 = U1, u3 = U3,
  // omega1 = D1 U3, omega3 = -D1 U1, u2 = 0
  if (t < 64) {
    for (int r = t; r < n; r += 64) {
      const size_t m0 = (size_t)r * g.M;
      store_c<TP>(a.ph[0], m0, a.U1[r], 0.0);
      store_c<TP>(a.ph[1], m0, 0.0, 0.0);
      store_c<TP>(a.ph[2], m0, a.U3[r], 0.0);
      store_c<TP>(a.ph[3], m0, DU[n + r], 0.0);
      store_c<TP>(a.ph[4], m0, -DU[r], 0.0);
    }
  }
}

// ---------------------------------------------------------------- advance
// One Fourier mode per lane, its real and imaginary parts together (the
// banded matrices are real, so both go through the same factorisations):
// every wall-normal row of a field is one 16-byte access per lane, 1 KB
// contiguous per wave.  Lanes l and l + 32 of a wave hold the modes (kx, kz)
// and (kx, -kz) of one pair; they share k^2, so every per-dt table (factor
// rows, homogeneous solutions, wall-derivative vectors) is stored per pair
// and the two lanes read the same entries.  Pair q = kx n3/2 + p,
// p = 0 .. n3/2 - 1, holds kz = +p (slot p) and kz = -p (slot n3 - p; for
// p = 0 the Nyquist slot n3/2, which carries no mode).
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ dv2 zi(dv2 z) { return (dv2){-z.y, z.x}; }  // i z
__device__ __forceinline__ dv2 zz() { return (dv2){0.0, 0.0}; }

// complex element at a byte offset from a wave-uniform row base
// (non-temporal, like the real accesses of the sweeps)
__device__ __forceinline__ dv2 ldz(const double* base, unsigned boff) {
  return __builtin_nontemporal_load(reinterpret_cast<const dv2*>(reinterpret_cast<const char*>(base) + boff));
}
__device__ __forceinline__ dv2 ldz(const float* base, unsigned boff) {
  const fv2 f = __builtin_nontemporal_load(reinterpret_cast<const fv2*>(reinterpret_cast<const char*>(base) + boff));
  return __builtin_convertvector(f, dv2);
}
__device__ __forceinline__ void stz(double* base, unsigned boff, dv2 v) {
  __builtin_nontemporal_store(v, reinterpret_cast<dv2*>(reinterpret_cast<char*>(base) + boff));
}
__device__ __forceinline__ void stz(float* base, unsigned boff, dv2 v) {
  __builtin_nontemporal_store(__builtin_convertvector(v, fv2),
                              reinterpret_cast<fv2*>(reinterpret_cast<char*>(base) + boff));
}
// complex element in its stored precision (converted where it is used)
template <typename T> struct NV2;
template <> struct NV2<double> { using t = dv2; };
template <> struct NV2<float> { using t = fv2; };
template <typename T> __device__ __forceinline__ typename NV2<T>::t ldr(const T* base, unsigned boff) {
  using V = typename NV2<T>::t;
  return __builtin_nontemporal_load(reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + boff));
}
__device__ __forceinline__ dv2 cvt(dv2 v) { return v; }
__device__ __forceinline__ dv2 cvt(fv2 v) { return __builtin_convertvector(v, dv2); }
__device__ __forceinline__ dv2 dot7z(const double* __restrict__ b, const dv2 (&w)[7]) {
  dv2 r = zz();
#pragma unroll
  for (int o = 0; o < 7; ++o) r += b[o] * w[o];
  return r;
}
__device__ __forceinline__ dv2 elim3z(dv2 r, const double* __restrict__ l, const dv2 (&yb)[3]) {
  return r - l[0] * yb[0] - l[1] * yb[1] - l[2] * yb[2];
}
__device__ __forceinline__ dv2 back3z(dv2 y, const double* __restrict__ U, const dv2 (&xb)[3]) {
  return (y - U[1] * xb[0] - U[2] * xb[1] - U[3] * xb[2]) * U[0];
}
__device__ __forceinline__ void shift3(dv2 (&b)[3], dv2 x) {
  b[0] = b[1];
  b[1] = b[2];
  b[2] = x;
}
__device__ __forceinline__ void push_xz(dv2 (&xb)[3], dv2 x) {
  xb[2] = xb[1];
  xb[1] = xb[0];
  xb[0] = x;
}

struct PairLane {
  unsigned m, q;     // mode slot in [n2][M] arrays, pair in [n2][Q] tables
  bool act, live, wph;
  double A, B, k2, ik2;
};
// Lane gl of the launch: wave gl / 64 holds pairs 32 (gl / 64) .. + 31;
// lanes 0..31 of the wave the +kz modes, 32..63 the -kz ones.
__device__ __forceinline__ PairLane pair_lane(const PencilGeom& g, int bx) {
  PairLane L;
  const int gl = bx * blockDim.x + threadIdx.x;
  const int n3h = g.n3 >> 1, Q = g.n1h * n3h;
  int q = 32 * (gl >> 6) + (gl & 31);
  const bool neg = (gl >> 5) & 1;
  L.act = q < Q;
  if (!L.act) q = Q - 1;  // in-bounds reads; nothing is written
  const int kx = q / n3h, p = q - kx * n3h;
  const int slot = neg ? (p == 0 ? n3h : g.n3 - p) : p;
  L.q = q;
  L.m = kx * g.n3 + slot;
  L.A = g.ka * kx;
  L.B = g.kb * (neg ? -p : p);
  L.k2 = L.A * L.A + L.B * L.B;
  L.live = L.act && slot != n3h && L.m != 0;
  L.wph = L.act && L.m != 0;  // the (0,0) phase entries come from the mean block
  L.ik2 = L.live ? 1.0 / L.k2 : 0.0;
  return L;
}

// One sub-step of the pencil phase, fused with the recovery of the next
// sub-step's velocities and vorticities:
//   S1 down : G = i(a H1 + b H3); eliminate A1 (dG) = B1 G
//   S2 up   : finish dG; N_chi, N_omega2, histories; implicit right-hand
//             sides of chi and omega2 (lag 3); Helmholtz factor on the fly;
//             eliminate chi_p, omega2; the wall values of D1 v_p as dot
//             products with the chi right-hand side, then the 2x2 influence
//             system (Appendix B)
//   S3 down : finish chi_p, omega2; chi = chi_p + c_lo, c_hi homogeneous;
//             Poisson rhs (lag 3); P factor on the fly; eliminate v
//   S4 up   : finish v; eliminate A1 (dv) = B1 v
//   R2 down : finish dv; u1, u3 by continuity; eliminate A1 (du) = B1 u
//   R3 up   : finish du1, du3; omega1 = du3 - i b v, omega3 = i a v - du1
// Scratch rows between sweeps are float64; the histories N_old are stored in
// the phase precision TP (float32 on the mixed path: they are products of
// the float32 transforms, rounded once after their float64 assembly).
template <typename TH, typename TP>
__device__ __forceinline__ void advance_body(const AdvanceArgs<TH, TP>& a, int bx,
                                             // read-only tables as noalias parameters, so the wave-uniform
                                             // row loads go through the scalar cache, not vector registers
                                             const double* __restrict__ B1, const double* __restrict__ A2,
                                             const double* __restrict__ B2, const double* __restrict__ L1d,
                                             const double* __restrict__ U1d, const double* __restrict__ L1u,
                                             const double* __restrict__ U1u) {
  constexpr int D = 5, DS1 = 8, D2 = 2, D3 = 3;
  if (unstable(a)) return;
  const PencilGeom& g = a.g;
  const PairLane L = pair_lane(g, bx);
  const int n = g.n2;
  const size_t M = g.M, Q = M / 2;
  const double cb = a.dt * a.be * a.nu;
  const double f1 = 1.0 - a.al * a.dt * a.nu * L.k2;
  const double f2 = a.al * a.dt * a.nu;
  const double dga = a.dt * a.ga, dze = a.dt * a.ze;
  const double hk = 1.0 + cb * L.k2;
  // Row bases are wave-uniform (scalar registers); per-lane offsets are
  // 32-bit byte offsets, so every access is one scalar base + one shared VGPR.
  const unsigned zo = 16u * L.m;                                 // complex float64 rows [n2][M]
  const unsigned ho = 2u * (unsigned)sizeof(TH) * L.m;           // complex TH rows
  const unsigned po = 2u * (unsigned)sizeof(TP) * L.m;           // complex TP rows
  const unsigned qo = 8u * L.q, qo2 = 16u * L.q;                 // pair tables: one value, (lo, hi)
  auto ZR = [&](auto* p, int i) { return p + 2 * (size_t)i * M; };   // row i of a complex [n2][M] array
  auto QR = [&](const double* p, int i) { return p + (size_t)i * Q; };       // [n2][Q]
  auto Q2R = [&](const double* p, int i) { return p + 2 * (size_t)i * Q; };  // [n2][Q][2]
  // histories N_old (phase precision): rows read at stride hist_rs, written
  // at hist_ws (0: one row)
  auto HRD = [&](const TP* p, int i) { return p + (size_t)i * a.hist_rs; };
  auto HWR = [&](TP* p, int i) { return p + (size_t)i * a.hist_ws; };
  const TP* nchi_rd = reinterpret_cast<const TP*>(a.nchi_rd);
  const TP* nom_rd = reinterpret_cast<const TP*>(a.nom_rd);
  TP* nchi_wr = reinterpret_cast<TP*>(a.nchi_wr);
  TP* nom_wr = reinterpret_cast<TP*>(a.nom_wr);
  // Scratch rows between sweeps stay float64 on both paths: an eliminated
  // right-hand side of the A1 solves rounded to float32 loses about four
  // digits in the back-substitution (cond(A1) ~ 1e4), and the influence
  // coefficients amplify that error much further at the wall rows of chi.
  double* S0r = a.S[0];
  double* S1r = a.S[1];
  double* S2r = a.S[2];
  double* S5r = a.S[5];
  // The scratch rows are stored per wave ([wave][n2][64 lanes], 1 KB per row
  // of a wave), so each wave walks one contiguous region of n2 KB per array
  // instead of striding across the whole mode plane from row to row.
  const size_t wv = (size_t)bx * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const unsigned so = 16u * (threadIdx.x & 63u);
  auto SR = [&](double* p, int i) { return p + 2 * ((size_t)wv * n + i) * 64; };

  // ---- S1 (down): G = i(a H1 + b H3), eliminate A1 (dG) = B1 G (look-ahead 3)
  {
    struct B { typename NV2<TH>::t h1, h3; };
    dv2 w[7], yb[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) w[k] = zz();
    yb[0] = yb[1] = yb[2] = zz();
    auto loadcol = [&](int j, B& b) {  // rows j >= n are clamped (used only for j < n)
      j = min(j, n - 1);
      b.h1 = ldr(ZR(a.H[0], j), ho);
      b.h3 = ldr(ZR(a.H[2], j), ho);
    };
    auto gval = [&](const B& b) -> dv2 { return L.live ? zi(L.A * cvt(b.h1) + L.B * cvt(b.h3)) : zz(); };
    for (int j = 0; j < 3; ++j) {
      B b;
      loadcol(j, b);
      w[3 + j] = gval(b);
    }
    pipeline<DS1, B>(
        n, [&](int t, B& b) { loadcol(t + 3, b); },
        [&](int t, B& b) {
          w[6] = (t + 3 < n) ? gval(b) : zz();
          const dv2 yi = elim3z(dot7z(B1 + t * 7, w), L1d + t * 3, yb);
          if (L.act) stz(SR(S0r, t), so, yi);
          shift3(yb, yi);
          push_back(w, zz());
        });
  }
  // ---- S2 (up): finish dG; N_chi = -dG - k^2 H2 and N_omega2 = i b H1 - i a H3;
  // the right-hand sides A2 q + f2 B2 x, q = f1 x + dt (gamma N + zeta N_old),
  // of chi and omega2 accumulated as columns arrive (acc[k] is row i + 3 - k,
  // complete at lag 3; zero on the wall rows); histories; Helmholtz matrix
  // factored on the fly; eliminate chi_p and omega2.  The wall values of
  // D1 v_p are linear in the chi right-hand side r: D1 v_p(wall c) = w_c . r
  // with w_c tabulated per sub-step (k_homog), so the influence coefficients
  // c_lo, c_hi are known when this sweep ends.
  dv2 clo_c = zz(), chi_c = zz();
  {
    struct B {
      typename NV2<TP>::t nco, noo;
      typename NV2<TH>::t h1, h2, h3;
      dv2 s0, chi, om, w;
    };
    dv2 xb[3], ac[7], ao[7], ycb[3], yob[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) ac[k] = ao[k] = zz();
#pragma unroll
    for (int k = 0; k < 3; ++k) xb[k] = ycb[k] = yob[k] = zz();
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    dv2 glo = zz(), ghi = zz();
    pipeline<D2, B>(
        n + 3,
        [&](int t, B& b) {  // rows clamped; the step uses them only inside the line
          const int i = max(n - 1 - t, 0), r = min(max(n + 2 - t, 0), n - 1);
          b.s0 = ldz(SR(S0r, i), so);
          b.h1 = ldr(ZR(a.H[0], i), ho);
          b.h2 = ldr(ZR(a.H[1], i), ho);
          b.h3 = ldr(ZR(a.H[2], i), ho);
          b.chi = ldz(ZR(a.chi, i), zo);
          b.om = ldz(ZR(a.om2, i), zo);
          b.nco = ldr(HRD(nchi_rd, i), po);
          b.noo = ldr(HRD(nom_rd, i), po);
          b.w = ldz(Q2R(a.hw, r), qo2);
        },
        [&](int t, B& b) {
          const int i = n - 1 - t;
          if (i >= 0) {
            const dv2 dG = back3z(b.s0, U1d + i * 4, xb);
            push_xz(xb, dG);
            const dv2 h1 = cvt(b.h1), h3 = cvt(b.h3);
            const dv2 nchi = L.live ? -dG - L.k2 * cvt(b.h2) : zz();
            const dv2 nom = L.live ? zi(L.B * h1 - L.A * h3) : zz();
            const dv2 qc = f1 * b.chi + dga * nchi + dze * cvt(b.nco);
            const dv2 qo = f1 * b.om + dga * nom + dze * cvt(b.noo);
            if (L.act) {
              stz(HWR(nchi_wr, i), po, nchi);
              stz(HWR(nom_wr, i), po, nom);
            }
#pragma unroll
            for (int k = 0; k < 7; ++k) {
              const int r = i + 3 - k;
              if (r >= 1 && r <= n - 2) {
                const double a2 = A2[r * 7 + k], b2 = f2 * B2[r * 7 + k];
                ac[k] += a2 * qc + b2 * b.chi;
                ao[k] += a2 * qo + b2 * b.om;
              }
            }
          }
          const int r = i + 3;
          if (r <= n - 1) {
            // the factor rows themselves are tabulated per sub-step (k_homog)
            double m7[7], lm[3];
            dv2 rc = ac[0], ro = ao[0];
            glo += b.w.x * rc;  // (w_lo, w_hi) of row r
            ghi += b.w.y * rc;
            helm_row(m7, A2 + r * 7, B2 + r * 7, r == 0 || r == n - 1, hk, cb);
            factor_up(m7, uh, lm);
#pragma unroll
            for (int d = 3; d >= 1; --d) {
              rc -= lm[3 - d] * ycb[3 - d];
              ro -= lm[3 - d] * yob[3 - d];
            }
            const double u0 = 1.0 / m7[3];
            if (L.act) {
              stz(SR(S1r, r), so, rc);
              stz(SR(S2r, r), so, ro);
            }
            push_u(uh, u0, m7[2], m7[1], m7[0]);
            shift3(ycb, rc);
            shift3(yob, ro);
          }
          push_back(ac, zz());
          push_back(ao, zz());
        });
    // 2x2 influence system: D1 v = 0 at both walls, with the wall derivatives
    // of the homogeneous v (tabulated)
    const double* hm = a.hm + 4 * (size_t)L.q;
    const double m00 = hm[0];  // lower-wall homogeneous solution, D1 at the lower wall
    const double m10 = hm[1];  // ... at the upper wall
    const double m01 = hm[2];  // upper-wall homogeneous solution, lower wall
    const double m11 = hm[3];
    if (L.live) {
      const double det = m00 * m11 - m01 * m10;
      clo_c = (m01 * ghi - m11 * glo) / det;
      chi_c = (m10 * glo - m00 * ghi) / det;
    }
  }
  // ---- S3 (down): finish chi_p and omega2; chi = chi_p + c_lo chi_lo +
  // c_hi chi_hi (homogeneous solutions tabulated); Poisson right-hand side
  // A2 chi (lag 3), Poisson matrix factored on the fly; eliminate v.  The
  // Poisson step is linear, so this v is v_p + c_lo v_lo + c_hi v_hi.
  {
    struct B { double u[4]; dv2 s1, s2, hc; };
    dv2 xcb[3], xob[3], wch[7], yvb[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) wch[k] = zz();
#pragma unroll
    for (int k = 0; k < 3; ++k) xcb[k] = xob[k] = yvb[k] = zz();
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    pipeline<D3, B>(
        n + 3,
        [&](int i, B& b) {
          i = min(i, n - 1);
#pragma unroll
          for (int k = 0; k < 4; ++k) b.u[k] = ldn(QR(a.SU[k], i), qo);
          b.s1 = ldz(SR(S1r, i), so);
          b.s2 = ldz(SR(S2r, i), so);
          b.hc = ldz(Q2R(a.hc, i), qo2);
        },
        [&](int i, B& b) {
          dv2 cn = zz();
          if (i < n) {
            const dv2 cp = back3z(b.s1, b.u, xcb);
            const dv2 om = back3z(b.s2, b.u, xob);
            push_xz(xcb, cp);
            push_xz(xob, om);
            cn = L.live ? cp + b.hc.x * clo_c + b.hc.y * chi_c : zz();  // hc = (chi_lo, chi_hi) of row i
            if (L.act) {
              stz(ZR(a.om2, i), zo, L.live ? om : zz());
              stz(ZR(a.chi, i), zo, cn);
            }
          }
          push_back(wch, cn);
          const int r = i - 3;
          if (r >= 0) {
            // the Poisson factor rows are tabulated once (k_homog)
            const bool wall = r == 0 || r == n - 1;
            double p7[7], lm[3];
            dv2 rv = zz();
            if (!wall) rv = dot7z(A2 + r * 7, wch);
            pois_row(p7, A2 + r * 7, B2 + r * 7, wall, L.k2);
            factor_down(p7, uh, lm);
#pragma unroll
            for (int d = 3; d >= 1; --d) rv -= lm[3 - d] * yvb[3 - d];
            const double u0 = 1.0 / p7[3];
            if (L.act) stz(SR(S5r, r), so, rv);
            push_u(uh, u0, p7[4], p7[5], p7[6]);
            shift3(yvb, rv);
          }
        });
  }
  // ---- S4 (up): finish v; eliminate A1 (dv) = B1 v upward (lag 3)
  {
    struct B { double u[4]; dv2 s5; };
    dv2 xvb[3], wv[7], yb[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) wv[k] = zz();
#pragma unroll
    for (int k = 0; k < 3; ++k) xvb[k] = yb[k] = zz();
    pipeline<D, B>(
        n + 3,
        [&](int t, B& b) {
          const int r = max(n - 1 - t, 0);
#pragma unroll
          for (int k = 0; k < 4; ++k) b.u[k] = ldn(QR(a.SU[4 + k], r), qo);
          b.s5 = ldz(SR(S5r, r), so);
        },
        [&](int t, B& b) {
          const int i = n - 1 - t;
          dv2 vn = zz();
          if (i >= 0) {
            vn = back3z(b.s5, b.u, xvb);
            push_xz(xvb, vn);
            if (L.act) stz(ZR(a.v, i), zo, vn);
            if (L.wph) stz(ZR(a.ph[1], i), po, vn);
          }
          push_front(wv, vn);
          const int r = i + 3;
          if (r <= n - 1) {
            const dv2 yr = elim3z(dot7z(B1 + r * 7, wv), L1u + r * 3, yb);
            if (L.act) stz(SR(S0r, r), so, yr);
            shift3(yb, yr);
          }
        });
  }
  // ---- R2 (down): finish dv; u1, u3 by continuity; eliminate A1 (du) = B1 u
  // downward (lag 3)
  {
    struct B { dv2 s0, om; };
    dv2 xb[3], w1[7], w3[7], y1b[3], y3b[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) w1[k] = w3[k] = zz();
#pragma unroll
    for (int k = 0; k < 3; ++k) xb[k] = y1b[k] = y3b[k] = zz();
    pipeline<D, B>(
        n + 3,
        [&](int i, B& b) {
          i = min(i, n - 1);
          b.s0 = ldz(SR(S0r, i), so);
          b.om = ldz(ZR(a.om2, i), zo);
        },
        [&](int i, B& b) {
          dv2 u1 = zz(), u3 = zz();
          if (i < n) {
            const dv2 dv = back3z(b.s0, U1u + i * 4, xb);
            push_xz(xb, dv);
            if (L.live) {
              // u1 = i(a dv - b omega2)/k^2, u3 = i(b dv + a omega2)/k^2
              u1 = zi(L.A * dv - L.B * b.om) * L.ik2;
              u3 = zi(L.B * dv + L.A * b.om) * L.ik2;
            }
            if (L.wph) {
              stz(ZR(a.ph[0], i), po, u1);
              stz(ZR(a.ph[2], i), po, u3);
            }
          }
          push_back(w1, u1);
          push_back(w3, u3);
          const int r = i - 3;
          if (r >= 0) {
            const double* bb = B1 + r * 7;
            const double* l = L1d + r * 3;
            const dv2 y1 = elim3z(dot7z(bb, w1), l, y1b);
            const dv2 y3 = elim3z(dot7z(bb, w3), l, y3b);
            if (L.act) {
              stz(SR(S1r, r), so, y1);
              stz(SR(S2r, r), so, y3);
            }
            shift3(y1b, y1);
            shift3(y3b, y3);
          }
        });
  }
  // ---- R3 (up): finish du1, du3; omega1 = du3 - i b v, omega3 = i a v - du1
  {
    struct B { dv2 s1, s2, v; };
    dv2 x1[3], x3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) x1[k] = x3[k] = zz();
    pipeline<D, B>(
        n,
        [&](int t, B& b) {
          const int r = max(n - 1 - t, 0);
          b.s1 = ldz(SR(S1r, r), so);
          b.s2 = ldz(SR(S2r, r), so);
          b.v = ldz(ZR(a.v, r), zo);
        },
        [&](int t, B& b) {
          const int r = n - 1 - t;
          const double* U = U1d + r * 4;
          const dv2 du1 = back3z(b.s1, U, x1);
          const dv2 du3 = back3z(b.s2, U, x3);
          push_xz(x1, du1);
          push_xz(x3, du3);
          if (L.wph) {
            stz(ZR(a.ph[3], r), po, du3 - zi(L.B * b.v));
            stz(ZR(a.ph[4], r), po, zi(L.A * b.v) - du1);
          }
        });
  }
}

// The mesh's operator rows (B1, A2, B2 and the A1 factors L1d, U1d, L1u,
// U1u: 35 values per row) staged in LDS once per workgroup.  Every sweep
// step reads one or two rows of several of them, wave-uniform; from LDS they
// return in about a hundred cycles, where the scalar cache, missing to L2 on
// each new row, made every step wait on a chain of scalar loads.
constexpr int kTableRow = 35;
__device__ __forceinline__ void stage_table(double* dst, const double* __restrict__ src, int cnt) {
  constexpr int G = 6;  // loads per thread in flight together
  for (int e0 = threadIdx.x; e0 < cnt; e0 += G * (int)blockDim.x) {
    double v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int e = e0 + u * blockDim.x;
      v[u] = src[e < cnt ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < cnt) dst[e] = v[u];
    }
  }
}
template <typename TH, typename TP>
__device__ __forceinline__ void advance_lds(const AdvanceArgs<TH, TP>& a, int bx, const double* __restrict__ B1,
                                            const double* __restrict__ A2, const double* __restrict__ B2,
                                            const double* __restrict__ L1d, const double* __restrict__ U1d,
                                            const double* __restrict__ L1u, const double* __restrict__ U1u) {
  extern __shared__ double tbl[];
  const int n = a.g.n2;
  double* t = tbl;
  stage_table(t, B1, 7 * n);
  stage_table(t + 7 * n, A2, 7 * n);
  stage_table(t + 14 * n, B2, 7 * n);
  stage_table(t + 21 * n, L1d, 3 * n);
  stage_table(t + 24 * n, U1d, 4 * n);
  stage_table(t + 28 * n, L1u, 3 * n);
  stage_table(t + 31 * n, U1u, 4 * n);
  __syncthreads();
  advance_body(a, bx, t, t + 7 * n, t + 14 * n, t + 21 * n, t + 24 * n, t + 28 * n, t + 31 * n);
}

// Workgroups of 128 pairs (256 modes); at most 256 VGPRs (two waves per
// SIMD): the 384 x 384 mode plane gives 289 workgroups, resident in one round.
// LT: operator rows from LDS (meshes whose tables fit), else from the scalar cache.
template <typename TH, typename TP, bool LT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
    k_advance(AdvanceArgs<TH, TP> a, const double* __restrict__ B1, const double* __restrict__ A2,
              const double* __restrict__ B2, const double* __restrict__ L1d, const double* __restrict__ U1d,
              const double* __restrict__ L1u, const double* __restrict__ U1u) {
  if (blockIdx.x == gridDim.x - 1) {
    mean_block(a);
    return;
  }
  if constexpr (LT) advance_lds(a, blockIdx.x, B1, A2, B2, L1d, U1d, L1u, U1u);
  else advance_body(a, blockIdx.x, B1, A2, B2, L1d, U1d, L1u, U1u);
}

// Batched over contexts: work item (context, block, -, mean flag).
template <typename TH, typename TP, bool LT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_advance_batch(const AdvanceArgs<TH, TP>* __restrict__ d,
                                                       const int4* __restrict__ w) {
  const int4 q = w[blockIdx.x];
  const AdvanceArgs<TH, TP>& a = d[q.x];
  if (q.w) {
    mean_block(a);
    return;
  }
  const PencilGeom& g = a.g;
  if constexpr (LT) advance_lds(a, q.y, g.B1, g.A2, g.B2, g.L1d, g.U1d, g.L1u, g.U1u);
  else advance_body(a, q.y, g.B1, g.A2, g.B2, g.L1d, g.U1d, g.L1u, g.U1u);
}

// ---------------------------------------------------------------- homogeneous solutions
// Row i of the transpose of a 7-band matrix with Dirichlet rows 0 and n - 1,
// in band order: mt[3 + d] = M[i + d][i]; ent(j, o) is entry o of interior row j.
template <typename F>
__device__ __forceinline__ void transposed_row(double (&mt)[7], int i, int n, F&& ent) {
#pragma unroll
  for (int d = -3; d <= 3; ++d) {
    const int j = i + d;
    mt[3 + d] = (j < 0 || j > n - 1) ? 0.0 : (j == 0 || j == n - 1) ? (d == 0 ? 1.0 : 0.0) : ent(j, 3 - d);
  }
}

// Solve M^T x = b for a 7-band M given by rows mrow (transposed_row): LU
// factored on the fly downward (U rows to the mode-indexed scratch Q, the
// eliminated right-hand side to the lane-indexed Y), back-substitution
// upward; out(i, x) receives x_i from row n - 1 to 0.  rhs(i) must accept
// every row of the line (it is read ahead by the pipeline).
template <typename RowF, typename RhsF, typename OutF>
__device__ __forceinline__ void solve_transposed(const Lane& L, int n, size_t st, size_t M, double* const (&Q)[4],
                                                 double* Y, RowF&& mrow, RhsF&& rhs, OutF&& out) {
  constexpr int D = 4;
  const size_t col = L.col, m = L.m;
  {
    struct B { double b; };
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    double yb[3] = {0, 0, 0};
    pipeline<D, B>(
        n, [&](int i, B& b) { b.b = rhs(min(i, n - 1)); },
        [&](int i, B& b) {
          double mt[7], lm[3];
          mrow(mt, i);
          factor_down(mt, uh, lm);
          double y = b.b;
#pragma unroll
          for (int d = 3; d >= 1; --d) y -= lm[3 - d] * yb[3 - d];
          const double u0 = 1.0 / mt[3];
          if (L.act && L.c == 0) {
            Q[0][i * M + m] = u0;
            Q[1][i * M + m] = mt[4];
            Q[2][i * M + m] = mt[5];
            Q[3][i * M + m] = mt[6];
          }
          if (L.act) Y[i * st + col] = y;
          push_u(uh, u0, mt[4], mt[5], mt[6]);
          yb[0] = yb[1]; yb[1] = yb[2]; yb[2] = y;
        });
  }
  {
    struct B { double u[4]; double y; };
    double xb[3] = {0, 0, 0};
    pipeline<D, B>(
        n,
        [&](int t, B& b) {
          const int i = max(n - 1 - t, 0);
#pragma unroll
          for (int k = 0; k < 4; ++k) b.u[k] = Q[k][i * M + m];
          b.y = Y[i * st + col];
        },
        [&](int t, B& b) {
          const int i = n - 1 - t;
          const double x = back3(b.y, b.u, xb);
          push_x(xb, x);
          out(i, x);
        });
  }
}

// For each sub-step s of a time step dt, per mode: chi_h with chi = 1 at wall
// c (lane c) and zero forcing from the Helmholtz step, v_h from the Poisson
// step with right-hand side A2 chi_h, and D1 v_h at both walls.  The same
// sweeps (directions, on-the-fly factorisation, operation order) as the
// particular solutions in k_advance.  Also the vectors w_c that give the wall
// derivatives of the particular v from the chi right-hand side r of
// k_advance: D1 v_p(wall c) = d_c . P^-1 E A2 H^-1 r = w_c . r with
// w_c = H^-T A2^T E P^-T d_c (d_c the compact D1 row at wall c, E zeroing the
// Dirichlet rows of the Poisson right-hand side).
// Read-only tables as noalias parameters: wave-uniform row reads through the
// scalar cache, and no ordering against the kernel's stores.
// Lane pair of a (kx, +-kz) pair of modes for the per-pair tables: lane c
// carries the homogeneous solution of wall c; k^2 from kz = p >= 0.
__device__ __forceinline__ Lane pair_wall_lane(const PencilGeom& g, int bx) {
  Lane L;
  const int gl = bx * blockDim.x + threadIdx.x;
  const int n3h = g.n3 >> 1, Q = g.n1h * n3h;
  int q = gl >> 1;
  L.c = gl & 1;
  L.act = q < Q;
  if (!L.act) q = Q - 1;
  L.m = q;
  L.col = 2 * (size_t)q + L.c;
  const int kx = q / n3h, p = q - kx * n3h;
  L.A = g.ka * kx;
  L.B = g.kb * p;
  L.k2 = L.A * L.A + L.B * L.B;
  L.mean = L.act && q == 0;
  L.live = L.act && q != 0;
  L.ik2 = L.live ? 1.0 / L.k2 : 0.0;
  return L;
}

__device__ __forceinline__ void homog_body(const HomogArgs& a, const double* __restrict__ A2,
                                           const double* __restrict__ B2, const double* __restrict__ dlo,
                                           const double* __restrict__ dhi) {
  const PencilGeom& g = a.g;
  const Lane L = pair_wall_lane(g, blockIdx.x);
  const int n = g.n2;
  // per-pair tables: [n2][2Q] lane-indexed (lane c: wall c), [n2][Q] pair-indexed
  const size_t M = g.M / 2, st = 2 * M;
  const size_t col = L.col, m = L.m;
  // t_c = A2^T E P^-T d_c (independent of dt), to a.T; z_c = E P^-T d_c is
  // consumed row by row (lag 3)
  {
    double wz[7] = {0, 0, 0, 0, 0, 0, 0};
    auto emit_t = [&](int r) {  // t at row r from wz[o] = (E z) at row r - 3 + o
      double tr = 0.0;
#pragma unroll
      for (int o = 0; o < 7; ++o) {
        const int j = r - 3 + o;
        if (j >= 1 && j <= n - 2) tr += A2[j * 7 + 6 - o] * wz[o];
      }
      if (L.act) a.T[r * st + col] = tr;
    };
    solve_transposed(
        L, n, st, M, a.Q, a.S0,
        [&](double(&mt)[7], int i) {
          transposed_row(mt, i, n, [&](int j, int o) { return B2[j * 7 + o] - L.k2 * A2[j * 7 + o]; });
        },
        [&](int i) { return L.c == 0 ? dlo[i] : dhi[i]; },
        [&](int i, double z) {
          push_front(wz, (i == 0 || i == n - 1) ? 0.0 : z);
          if (i + 3 <= n - 1) emit_t(i + 3);
        });
    for (int r = 2; r >= 0; --r) {
      push_front(wz, 0.0);
      emit_t(r);
    }
  }
  for (int s = 0; s < 3; ++s) {
    const double cb = a.dt * a.be[s] * a.nu;
    const double hk = 1.0 + cb * L.k2;
    // Helmholtz, upward: factor rows, eliminate the wall forcing
    {
      double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
      double yhb[3] = {0, 0, 0};
      for (int r = n - 1; r >= 0; --r) {
        const bool wall = r == 0 || r == n - 1;
        double m7[7], lm[3];
        double rh = wall && (r == 0) == (L.c == 0) ? 1.0 : 0.0;
        helm_row(m7, A2 + r * 7, B2 + r * 7, wall, hk, cb);
        factor_up(m7, uh, lm);
#pragma unroll
        for (int d = 3; d >= 1; --d) rh -= lm[3 - d] * yhb[3 - d];
        const double u0 = 1.0 / m7[3];
        if (L.act && L.c == 0) {  // the factor table of sub-step s (read by k_advance)
          a.hu[s][0][r * M + m] = u0;
          a.hu[s][1][r * M + m] = m7[2];
          a.hu[s][2][r * M + m] = m7[1];
          a.hu[s][3][r * M + m] = m7[0];
        }
        if (L.act) a.S0[r * st + col] = rh;
        push_u(uh, u0, m7[2], m7[1], m7[0]);
        yhb[0] = yhb[1]; yhb[1] = yhb[2]; yhb[2] = rh;
      }
    }
    // Helmholtz back-substitution, downward: chi_h; Poisson right-hand side
    // A2 chi_h (lag 3), Poisson rows factored, eliminated
    {
      struct B { double u[4]; double s0; };
      double xhb[3] = {0, 0, 0};
      double wch[7] = {0, 0, 0, 0, 0, 0, 0};
      double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
      double yhb[3] = {0, 0, 0};
      pipeline<4, B>(
          n + 3,
          [&](int i, B& b) {
            i = min(i, n - 1);
#pragma unroll
            for (int k = 0; k < 4; ++k) b.u[k] = a.hu[s][k][i * M + m];
            b.s0 = a.S0[i * st + col];
          },
          [&](int i, B& b) {
        double ch = 0.0;
        if (i < n) {
          ch = back3(b.s0, b.u, xhb);
          push_x(xhb, ch);
          if (L.act) a.hc[s][i * st + col] = ch;
        }
        push_back(wch, ch);
        const int r = i - 3;
        if (r >= 0) {
          const bool wall = r == 0 || r == n - 1;
          double p7[7], lm[3], rhv = 0.0;
          if (!wall) {
#pragma unroll
            for (int o = 0; o < 7; ++o) rhv += A2[r * 7 + o] * wch[o];
          }
          pois_row(p7, A2 + r * 7, B2 + r * 7, wall, L.k2);
          factor_down(p7, uh, lm);
#pragma unroll
          for (int d = 3; d >= 1; --d) rhv -= lm[3 - d] * yhb[3 - d];
          const double u0 = 1.0 / p7[3];
          if (L.act && L.c == 0) {  // the Poisson factor table (independent of dt)
            a.SU[4][r * M + m] = u0;
            a.SU[5][r * M + m] = p7[4];
            a.SU[6][r * M + m] = p7[5];
            a.SU[7][r * M + m] = p7[6];
          }
          if (L.act) a.S1[r * st + col] = rhv;
          push_u(uh, u0, p7[4], p7[5], p7[6]);
          yhb[0] = yhb[1]; yhb[1] = yhb[2]; yhb[2] = rhv;
        }
          });
    }
    // Poisson back-substitution, upward: v_h and D1 v_h at both walls
    {
      struct B { double u[4]; double s1; };
      double xhb[3] = {0, 0, 0};
      double glo = 0.0, ghi = 0.0;
      pipeline<4, B>(
          n,
          [&](int t, B& b) {
            const int r = max(n - 1 - t, 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) b.u[k] = a.SU[4 + k][r * M + m];
            b.s1 = a.S1[r * st + col];
          },
          [&](int t, B& b) {
            const int r = n - 1 - t;
            const double vh = back3(b.s1, b.u, xhb);
            push_x(xhb, vh);
            glo = fma(dlo[r], vh, glo);
            ghi = fma(dhi[r], vh, ghi);
          });
      const double olo = __shfl_xor(glo, 1), ohi = __shfl_xor(ghi, 1);
      if (L.act && L.c == 0) {
        double* hm = a.hm[s] + 4 * m;
        hm[0] = glo;
        hm[1] = ghi;
        hm[2] = olo;
        hm[3] = ohi;
      }
    }
    // w_c = H^-T t_c
    {
      const double* T = a.T;
      double* W = a.hw[s];
      solve_transposed(
          L, n, st, M, a.Q, a.S0,
          [&](double(&mt)[7], int i) {
            transposed_row(mt, i, n, [&](int j, int o) { return hk * A2[j * 7 + o] - cb * B2[j * 7 + o]; });
          },
          [&](int i) { return T[i * st + col]; }, [&](int i, double w) {
            if (L.act) W[i * st + col] = w;
          });
    }
  }
}

__global__ void __launch_bounds__(256) k_homog(HomogArgs a, const double* __restrict__ A2,
                                               const double* __restrict__ B2, const double* __restrict__ dlo,
                                               const double* __restrict__ dhi) {
  homog_body(a, A2, B2, dlo, dhi);
}

// ---------------------------------------------------------------- filtered pressure
// Section 3.1: d_kk p = -d_i d_j F(u_i u_j) on every retained mode, from the
// filtered stresses and the filtered wall-normal velocity.  Per mode: the
// right-hand side in the A-form of the implicit steps (B2 - k^2 A2) p = A2 r,
// the wall rows D1 p = nu D2 F(v) (full compact rows) through the influence
// matrix (particular solution with p = 0 at the walls, plus the homogeneous
// ones with p = 1 at one wall, tabulated nowhere: computed alongside), mode
// (0,0) as P = -F(u_2 u_2).  Lanes as in the pencil kernels: two per mode
// (real, imaginary part); lane c also carries the homogeneous solution of
// wall c.
//   S1 down : eliminate A1 d = B1 F(u1u2), A1 d = B1 F(u2u3), A2 d = B2 F(v)
//   S2 up   : finish them (D2 F(v) only at the walls)
//   S3 down : A2 r (lag 3); factor B2 - k^2 A2 on the fly; eliminate p_0, p_h
//   S4 up   : finish p_0, p_h; wall rows of D1; 2x2 influence system
//   S5      : p = p_0 + c_lo p_lo + c_hi p_hi
__device__ __forceinline__ void pressure_body(const PressureArgs& a, const double* __restrict__ A2,
                                              const double* __restrict__ B2, const double* __restrict__ B1,
                                              const double* __restrict__ L1d, const double* __restrict__ U1d,
                                              const double* __restrict__ L2d, const double* __restrict__ U2d,
                                              const double* __restrict__ dlo, const double* __restrict__ dhi) {
  const int n = a.g.n2;
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  int r = gl >> 1;
  const int c = gl & 1;
  const bool act = r < a.R;
  if (!act) r = a.R - 1;
  const int kx = r / a.nz, s = r - kx * a.nz;
  const int kz = s <= a.kcz ? s : s - a.nz;
  const double A = a.g.ka * kx, B = a.g.kb * kz, k2 = A * A + B * B;
  const bool mean = r == 0;
  const double sg = c == 0 ? -1.0 : 1.0;  // (i z)_c = sg z_other
  const size_t st = 2 * (size_t)a.R, R = a.R;
  const size_t col = 2 * (size_t)r + c;
  const size_t fs = (size_t)n * st;      // one field of uu
  auto U = [&](int q, int i) { return a.uu[q * fs + (size_t)i * st + col]; };
  double* T0 = a.T[0];
  double* T1 = a.T[1];
  double* T2 = a.T[2];
  double* T3 = a.T[3];
  // ---- S1 (down)
  {
    double w12[7] = {0, 0, 0, 0, 0, 0, 0}, w23[7] = {0, 0, 0, 0, 0, 0, 0}, wv[7] = {0, 0, 0, 0, 0, 0, 0};
    double y12[3] = {0, 0, 0}, y23[3] = {0, 0, 0}, yv[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
      w12[3 + k] = U(1, k);
      w23[3 + k] = U(4, k);
      wv[3 + k] = a.vb[(size_t)k * st + col];
    }
    for (int i = 0; i < n; ++i) {
      const bool more = i + 3 < n;
      w12[6] = more ? U(1, i + 3) : 0.0;
      w23[6] = more ? U(4, i + 3) : 0.0;
      wv[6] = more ? a.vb[(size_t)(i + 3) * st + col] : 0.0;
      const double e12 = elim3(dot7(B1 + i * 7, w12), L1d + i * 3, y12);
      const double e23 = elim3(dot7(B1 + i * 7, w23), L1d + i * 3, y23);
      const double ev = elim3(dot7(B2 + i * 7, wv), L2d + i * 3, yv);
      if (act) {
        T0[i * st + col] = e12;
        T1[i * st + col] = e23;
        T2[i * st + col] = ev;
      }
      y12[0] = y12[1]; y12[1] = y12[2]; y12[2] = e12;
      y23[0] = y23[1]; y23[1] = y23[2]; y23[2] = e23;
      yv[0] = yv[1]; yv[1] = yv[2]; yv[2] = ev;
      push_back(w12, 0.0);
      push_back(w23, 0.0);
      push_back(wv, 0.0);
    }
  }
  // ---- S2 (up): D1 F(u1u2), D1 F(u2u3) in place; nu D2 F(v) at the walls
  double g_lo = 0.0, g_hi = 0.0;
  {
    double x12[3] = {0, 0, 0}, x23[3] = {0, 0, 0}, xv[3] = {0, 0, 0};
    for (int i = n - 1; i >= 0; --i) {
      const double d12 = back3(T0[i * st + col], U1d + i * 4, x12);
      const double d23 = back3(T1[i * st + col], U1d + i * 4, x23);
      const double dv = back3(T2[i * st + col], U2d + i * 4, xv);
      push_x(x12, d12);
      push_x(x23, d23);
      push_x(xv, dv);
      if (act) {
        T0[i * st + col] = d12;
        T1[i * st + col] = d23;
      }
      if (i == n - 1) g_hi = a.nu * dv;
      if (i == 0) g_lo = a.nu * dv;
    }
  }
  // ---- S3 (down): rhs = -(A2 q + B2 F(u2u2)) on interior rows, q = -a^2 u11
  // + 2a (i d12) - 2ab u13 + 2b (i d23) - b^2 u33; Dirichlet rows: 0 for p_0,
  // 1 at wall c for p_h
  {
    double wq[7] = {0, 0, 0, 0, 0, 0, 0}, wu[7] = {0, 0, 0, 0, 0, 0, 0};
    double uh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    double y0[3] = {0, 0, 0}, yh[3] = {0, 0, 0};
    for (int i = 0; i < n + 3; ++i) {
      double q = 0.0, u22 = 0.0;
      if (i < n) {
        const double d12 = T0[i * st + col], d23 = T1[i * st + col];
        const double d12o = __shfl_xor(d12, 1), d23o = __shfl_xor(d23, 1);
        q = -A * A * U(0, i) + 2.0 * A * sg * d12o - 2.0 * A * B * U(2, i) + 2.0 * B * sg * d23o - B * B * U(5, i);
        u22 = U(3, i);
      }
      push_back(wq, q);
      push_back(wu, u22);
      const int rr = i - 3;
      if (rr >= 0) {
        const bool wall = rr == 0 || rr == n - 1;
        double rhs = 0.0, rh = 0.0;
        if (!wall) {
#pragma unroll
          for (int o = 0; o < 7; ++o) rhs -= A2[rr * 7 + o] * wq[o] + B2[rr * 7 + o] * wu[o];
        } else {
          rh = (rr == 0) == (c == 0) ? 1.0 : 0.0;
        }
        double p7[7], lm[3];
        pois_row(p7, A2 + rr * 7, B2 + rr * 7, wall, k2);
        factor_down(p7, uh, lm);
#pragma unroll
        for (int d = 3; d >= 1; --d) {
          rhs -= lm[3 - d] * y0[3 - d];
          rh -= lm[3 - d] * yh[3 - d];
        }
        const double u0 = 1.0 / p7[3];
        if (act && c == 0) {
          a.Q[0][rr * R + r] = u0;
          a.Q[1][rr * R + r] = p7[4];
          a.Q[2][rr * R + r] = p7[5];
          a.Q[3][rr * R + r] = p7[6];
        }
        if (act) {
          T2[rr * st + col] = rhs;
          T3[rr * st + col] = rh;
        }
        push_u(uh, u0, p7[4], p7[5], p7[6]);
        y0[0] = y0[1]; y0[1] = y0[2]; y0[2] = rhs;
        yh[0] = yh[1]; yh[1] = yh[2]; yh[2] = rh;
      }
    }
  }
  // ---- S4 (up): p_0, p_h; D1 at the walls (full compact rows)
  double c_lo = 0.0, c_hi = 0.0;
  {
    double x0[3] = {0, 0, 0}, xh[3] = {0, 0, 0};
    double l0 = 0.0, h0 = 0.0, lh = 0.0, hh = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double u[4] = {a.Q[0][i * R + r], a.Q[1][i * R + r], a.Q[2][i * R + r], a.Q[3][i * R + r]};
      const double p0 = back3(T2[i * st + col], u, x0);
      const double ph = back3(T3[i * st + col], u, xh);
      push_x(x0, p0);
      push_x(xh, ph);
      if (act) {
        T2[i * st + col] = p0;
        T3[i * st + col] = ph;
      }
      l0 = fma(dlo[i], p0, l0);
      h0 = fma(dhi[i], p0, h0);
      lh = fma(dlo[i], ph, lh);
      hh = fma(dhi[i], ph, hh);
    }
    // lane c holds D1 p_h of wall c at (lower, upper); the other lane the other wall's
    const double lo_ = __shfl_xor(lh, 1), ho_ = __shfl_xor(hh, 1);
    const double m00 = c == 0 ? lh : lo_, m10 = c == 0 ? hh : ho_;  // p_lo at the lower, upper wall
    const double m01 = c == 0 ? lo_ : lh, m11 = c == 0 ? ho_ : hh;  // p_hi
    if (!mean) {
      const double f0 = g_lo - l0, f1 = g_hi - h0;
      const double det = m00 * m11 - m01 * m10;
      c_lo = (f0 * m11 - f1 * m01) / det;
      c_hi = (f1 * m00 - f0 * m10) / det;
    }
  }
  // ---- S5: combine and write
  for (int i = 0; i < n; ++i) {
    const double ph = T3[i * st + col], pho = __shfl_xor(ph, 1);
    const double plo = c == 0 ? ph : pho, phi = c == 0 ? pho : ph;
    const double v = mean ? (c == 0 ? -U(3, i) : 0.0) : T2[i * st + col] + c_lo * plo + c_hi * phi;
    if (act) a.p[(size_t)i * st + col] = v;
  }
}

__global__ void __launch_bounds__(256) k_pressure(PressureArgs a, const double* __restrict__ A2,
                                                  const double* __restrict__ B2, const double* __restrict__ B1,
                                                  const double* __restrict__ L1d, const double* __restrict__ U1d,
                                                  const double* __restrict__ L2d, const double* __restrict__ U2d,
                                                  const double* __restrict__ dlo, const double* __restrict__ dhi) {
  pressure_body(a, A2, B2, B1, L1d, U1d, L2d, U2d, dlo, dhi);
}

// ---------------------------------------------------------------- set state
__global__ void __launch_bounds__(256) k_chi_from_v(ChiArgs a) {
  const PencilGeom& g = a.g;
  const Lane L = lane_setup(g, blockIdx.x);
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
// Divergence i a u1 + D1 u2 + i b u3 of the phase velocities, per mode and
// node: A1 (D1 u2) = B1 u2 eliminated downward, finished upward; the lane
// pair of a mode forms the complex divergence and its modulus.
template <typename TP>
__global__ void __launch_bounds__(256) k_div(DivArgs<TP> a, const double* __restrict__ B1,
                                             const double* __restrict__ L1d, const double* __restrict__ U1d) {
  const PencilGeom& g = a.g;
  const Lane L = lane_setup(g, blockIdx.x);
  const int n = g.n2;
  const size_t st = 2 * (size_t)g.M, col = L.col;
  auto u = [&](int f, int i) { return (double)a.u[f][(size_t)i * st + col]; };
  {
    double w[7] = {0, 0, 0, 0, 0, 0, 0};
    double yb[3] = {0, 0, 0};
    for (int k = 0; k < 3 && k < n; ++k) w[3 + k] = u(1, k);
    for (int i = 0; i < n; ++i) {
      w[6] = (i + 3 < n) ? u(1, i + 3) : 0.0;
      const double yi = elim3(dot7(B1 + i * 7, w), L1d + i * 3, yb);
      if (L.act) a.S0[i * st + col] = yi;
      yb[0] = yb[1];
      yb[1] = yb[2];
      yb[2] = yi;
      push_back(w, 0.0);
    }
  }
  double dmax = 0.0;
  double xb[3] = {0, 0, 0};
  const double sg = L.c == 0 ? -1.0 : 1.0;  // component c of i z is sg times the other component of z
  for (int i = n - 1; i >= 0; --i) {
    const double dv = back3(a.S0[i * st + col], U1d + i * 4, xb);
    push_x(xb, dv);
    const double u1o = __shfl_xor(u(0, i), 1), u3o = __shfl_xor(u(2, i), 1);
    const double dc = dv + sg * (L.A * u1o + L.B * u3o);
    const double m2 = dc * dc + __shfl_xor(dc * dc, 1);
    if (L.act) dmax = nanmax(dmax, sqrt(m2));
  }
  for (int off = 32; off > 0; off >>= 1) dmax = nanmax(dmax, __shfl_xor(dmax, off));
  if ((threadIdx.x & 63) == 0)
    atomicMax(a.maxbits, (unsigned long long)__double_as_longlong(dmax != dmax ? __longlong_as_double(0x7ff8000000000000ll) : dmax));
}

__global__ void __launch_bounds__(256) k_info(InfoArgs a) {
  __shared__ double red[3][4];
  const int n = a.g.n2;
  double cm = 0.0, wm = 0.0;
  bool bad = false;
  for (size_t e = threadIdx.x; e < (size_t)n * a.p3; e += blockDim.x) {
    const double c = a.rowcfl[e];
    if (!isfinite(c)) bad = true;
    cm = nanmax(cm, c);
  }
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    wm += a.g.quad[r] * a.U1[r];
    if (!isfinite(a.U1[r])) bad = true;
  }
  double b = bad ? 1.0 : 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    cm = nanmax(cm, __shfl_xor(cm, off));
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
      c = nanmax(c, red[0][w]);
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
// k_advance: 128 (kx, +-kz) pairs (256 modes) per workgroup, plus the mean workgroup
int advance_blocks(int M) { return (int)(((size_t)M / 2 + 127) / 128); }

template <typename TP> hipError_t launch_recover(const RecoverArgs<TP>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_recover<TP>), dim3(pencil_blocks(a.g.M)), dim3(256), 0, st, a, a.g.B1, a.g.L1d, a.g.U1d,
                     a.g.L1u, a.g.U1u);
  return hipGetLastError();
}
hipError_t launch_homog(const HomogArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_homog, dim3(pencil_blocks(a.g.M / 2)), dim3(256), 0, st, a, a.g.A2, a.g.B2, a.g.clo,
                     a.g.chi);
  return hipGetLastError();
}

// Operator rows in LDS on the mixed path up to this many bytes per workgroup
// (two workgroups per CU keep their tables; 193 rows take 54 KB), else from
// the scalar cache.  Measured on 384x193x384: mixed 2.12 -> 2.03 ms per
// launch; float64 2.24 -> 2.40 ms (the rows then occupy vector registers the
// float64 sweeps need), so the float64 path keeps the scalar cache.
constexpr size_t kTableLdsMax = 64 << 10;
size_t advance_table_bytes(int n2) { return (size_t)kTableRow * n2 * sizeof(double); }
template <typename TH, typename TP> hipError_t launch_advance(const AdvanceArgs<TH, TP>& a, hipStream_t st) {
  const size_t tb = advance_table_bytes(a.g.n2);
  if (sizeof(TP) == 4 && tb <= kTableLdsMax)
    hipLaunchKernelGGL((k_advance<TH, TP, true>), dim3(advance_blocks(a.g.M) + 1), dim3(256), tb, st, a, a.g.B1,
                       a.g.A2, a.g.B2, a.g.L1d, a.g.U1d, a.g.L1u, a.g.U1u);
  else
    hipLaunchKernelGGL((k_advance<TH, TP, false>), dim3(advance_blocks(a.g.M) + 1), dim3(256), 0, st, a, a.g.B1,
                       a.g.A2, a.g.B2, a.g.L1d, a.g.U1d, a.g.L1u, a.g.U1u);
  return hipGetLastError();
}
hipError_t launch_pressure(const PressureArgs& a, hipStream_t st) {
  const unsigned nb = (unsigned)((2 * (size_t)a.R + 255) / 256);
  const PencilGeom& g = a.g;
  hipLaunchKernelGGL(k_pressure, dim3(nb), dim3(256), 0, st, a, g.A2, g.B2, g.B1, g.L1d, g.U1d, g.L2d, g.U2d, g.clo,
                     g.chi);
  return hipGetLastError();
}
hipError_t launch_chi_from_v(const ChiArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_chi_from_v, dim3(pencil_blocks(a.g.M)), dim3(256), 0, st, a);
  return hipGetLastError();
}
template <typename TP> hipError_t launch_div(const DivArgs<TP>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_div<TP>), dim3(pencil_blocks(a.g.M)), dim3(256), 0, st, a, a.g.B1, a.g.L1d, a.g.U1d);
  return hipGetLastError();
}
template hipError_t launch_div<double>(const DivArgs<double>&, hipStream_t);
template hipError_t launch_div<float>(const DivArgs<float>&, hipStream_t);
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
template <typename T>
hipError_t launch_advance_batch(const AdvanceArgs<T, T>* d, const int4* w, int nblocks, int n2max, hipStream_t st) {
  const size_t tb = advance_table_bytes(n2max);
  if (sizeof(T) == 4 && tb <= kTableLdsMax)
    hipLaunchKernelGGL((k_advance_batch<T, T, true>), dim3(nblocks), dim3(256), tb, st, d, w);
  else hipLaunchKernelGGL((k_advance_batch<T, T, false>), dim3(nblocks), dim3(256), 0, st, d, w);
  return hipGetLastError();
}
template hipError_t launch_advance_batch<double>(const AdvanceArgs<double, double>*, const int4*, int, int, hipStream_t);
template hipError_t launch_advance_batch<float>(const AdvanceArgs<float, float>*, const int4*, int, int, hipStream_t);

template hipError_t launch_advance<double, double>(const AdvanceArgs<double, double>&, hipStream_t);
template hipError_t launch_advance<float, float>(const AdvanceArgs<float, float>&, hipStream_t);

}  // namespace chn
