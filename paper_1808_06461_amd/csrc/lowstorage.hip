// Low-storage database stage (Section 3.1 of the paper): sharp Fourier cut-off
// in x and z, the filtered products F(u_i u_j) and the sub-grid stress
// tau_ij = F(u_i u_j) - F(u_i) F(u_j) on a q1 x q3 grid of every plane.
//
// The plane means U_i(y) are removed before the products (u' = u - U, by
// zeroing the (0,0) coefficient), so the transforms carry only fluctuations:
//   F(u_i u_j) = F(u'_i u'_j) + U_i F(u'_j) + U_j F(u'_i) + U_i U_j delta_k0,
//   tau_ij     = F(u'_i u'_j) - F(u'_i) F(u'_j)      (the plane means cancel).
// The inputs are the velocity (or vorticity) coefficients the time step
// keeps in its phase precision (float32 on the mixed path), widened to
// float64 as they are loaded; every transform, product, sum and stress is
// float64.  (Float32 inverse transforms with float64 products and forward
// sums leave F(u'_i u'_j) at 2.5e-6 but tau_ij, which is 40 times smaller
// near the wall, at 1.1e-4 of itself on the 1536 x 385 x 1152 field.)
// The products live on an f1 x f3 grid, the smallest 2,3-smooth sizes above
// 2 h + kc (h the highest stored wavenumber, kc the cut-off), on which every
// retained mode of a product is exact.
//
//   k_zinv (plane.hip) : the three fields with zero (0,0) mode, padded to f3, float64 inverse in z
//   k_xfilter : inverse in x to f1 points, products, float64 forward in x, keep kx <= kcx
//   k_zfilter : float64 forward in z, keep |kz| <= kcz; F(u_i), F(u_i u_j)
//   k_zinv_q  : the nine retained fields padded to q3, inverse in z
//   k_xtau    : inverse in x on q1 points, tau_ij = pp_ij - ub_i ub_j
#include "fft.hpp"
#include "kernels.hpp"

namespace chn {

// pairs (11, 12, 13, 22, 23, 33)
__device__ __constant__ int kPairI[6] = {0, 0, 0, 1, 1, 2};
__device__ __constant__ int kPairJ[6] = {0, 1, 2, 1, 2, 2};

// Per (y, z row): inverse x transforms of u1 + i u2 and u3, the six
// products in float64, forward float64 transforms of
// (11, 22), (12, 13), (23, 33) as two real signals per complex line, kx <=
// kcx kept.  Trace mode: one product, u1^2 + u2^2 + u3^2, one forward line.
// One line in LDS at a time (the physical values stay in registers), so
// several workgroups share a CU.
template <typename T, int NQ, int FN = kFnComposite>
__global__ void __launch_bounds__(256) k_xfilter(XfilterArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  c2<T>* lt = reinterpret_cast<c2<T>*>(smem_raw);      // one phase-precision line
  double2* ld = reinterpret_cast<double2*>(smem_raw);  // one float64 line (the same space)
  const int y = blockIdx.y, z = blockIdx.x;
  const int n1h = a.n1h, f1 = a.f1, f3 = a.f3;
  const c2<T> zero = mk<T>(T(0), T(0));
  T ph[3][NQ];  // u1, u2, u3 at x = threadIdx.x + q * blockDim.x (f1 <= NQ * 256)
  // inverse transforms: line 0 = u1 + i u2 (two real signals), line 1 = u3
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    for (int e = threadIdx.x; e < f1; e += blockDim.x) lt[e] = zero;
    __syncthreads();
    // kG coefficients per thread loaded together (clamped addresses), then
    // written to LDS
    constexpr int kG = 4;
    for (int k0 = threadIdx.x; k0 < n1h; k0 += kG * blockDim.x) {
      c2<T> X[kG], Y[kG];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int k = k0 + u * blockDim.x;
        const size_t base = ((size_t)(y * 3 + 2 * l) * f3 + z) * n1h + (k < n1h ? k : 0);
        X[u] = a.buf[base];
        Y[u] = l == 0 ? a.buf[base + (size_t)f3 * n1h] : zero;
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int k = k0 + u * blockDim.x;
        if (k == 0) {
          lt[0] = mk<T>(X[u].x, Y[u].x);
        } else if (k < n1h) {
          lt[k] = mk<T>(X[u].x - Y[u].y, X[u].y + Y[u].x);
          lt[f1 - k] = mk<T>(X[u].x + Y[u].y, Y[u].x - X[u].y);
        }
      }
    }
    __syncthreads();
    fft_lines<T, 16, FN>(lt, a.lst, 1, a.plan, a.tw, +1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int x = threadIdx.x + q * blockDim.x;
      const c2<T> v = keep_if<T>(x < f1, lt[x < f1 ? x : 0]);
      if (l == 0) {
        ph[0][q] = v.x;
        ph[1][q] = v.y;
      } else {
        ph[2][q] = v.x;
      }
    }
    __syncthreads();
  }
  const int kc1 = a.kcx + 1;
  double2* out = a.out + ((size_t)y * a.plane_stride) + (size_t)z * kc1;
  if (a.trace) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int x = threadIdx.x + q * blockDim.x;
      const double u = ph[0][q], v = ph[1][q], w = ph[2][q];
      if (x < f1) ld[x] = make_double2(u * u + v * v + w * w, 0.0);
    }
    __syncthreads();
    fft_lines<double, 16, FN>(ld, a.lsd, 1, a.plan, a.tw_d, -1);
    for (int k = threadIdx.x; k < kc1; k += blockDim.x) out[k] = ld[k];
    return;
  }
  // one float64 line of two products at a time: (11, 22), (12, 13), (23, 33);
  // then kx <= kcx of both spectra
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int ia = l == 0 ? 0 : (l == 1 ? 0 : 1), ja = l == 0 ? 0 : (l == 1 ? 1 : 2);
    const int ib = l == 0 ? 1 : (l == 1 ? 0 : 2), jb = l == 0 ? 1 : (l == 1 ? 2 : 2);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int x = threadIdx.x + q * blockDim.x;
      if (x < f1)
        ld[x] = make_double2((double)ph[ia][q] * (double)ph[ja][q], (double)ph[ib][q] * (double)ph[jb][q]);
    }
    __syncthreads();
    fft_lines<double, 16, FN>(ld, a.lsd, 1, a.plan, a.tw_d, -1);
    // pairs of the line: 0 (11) and 3 (22); 1 (12) and 2 (13); 4 (23) and 5 (33)
    const int pa = l == 0 ? 0 : (l == 1 ? 1 : 4);
    const int pb = l == 0 ? 3 : (l == 1 ? 2 : 5);
    for (int k = threadIdx.x; k < kc1; k += blockDim.x) {
      const double2 W = ld[k];
      const double2 Wm = ld[k == 0 ? 0 : f1 - k];
      const double2 P = make_double2(0.5 * (W.x + Wm.x), 0.5 * (W.y - Wm.y));   // (W_k + conj W_m)/2
      const double2 Q = make_double2(0.5 * (W.y + Wm.y), -0.5 * (W.x - Wm.x));  // (W_k - conj W_m)/(2i)
      out[(size_t)pa * f3 * kc1 + k] = P;
      out[(size_t)pb * f3 * kc1 + k] = Q;
    }
    __syncthreads();
  }
}

// Coefficient idx of field i, widened to float64 where it is stored in float32.
__device__ __forceinline__ double2 ldu(const FieldsIn& u, int i, size_t idx) {
  if ((u.f32 >> i) & 1u) {
    const float2 v = reinterpret_cast<const float2*>(u.u[i])[idx];
    return make_double2((double)v.x, (double)v.y);
  }
  return reinterpret_cast<const double2*>(u.u[i])[idx];
}

// Per (y, tile of retained kx): forward z transform of the six products,
// F(u'_i u'_j) on |kz| <= kcz -> pp; F(u_i u_j) with the mean terms -> uubar;
// F(u_i) -> ubar.  Trace mode: the one product u'_i u'_i, with the mean
// terms 2 U_i F(u'_i) (+ U_i U_i at k = 0), -> trace (fed the vorticity, the
// filtered enstrophy of Section 3.1).  uubar and ubar are optional.
__global__ void __launch_bounds__(256) k_zfilter(ZfilterArgs a) {
  extern __shared__ unsigned char smem_raw[];
  double2* lds = reinterpret_cast<double2*>(smem_raw);
  const int y = blockIdx.y;
  const int kx0 = blockIdx.x * a.K;
  const int n3 = a.n3, f3 = a.f3, K = a.K, LS = a.lstride;
  const int kc1 = a.kcx + 1, nz = 2 * a.kcz + 1;
  const int nk = min(K, kc1 - kx0);
  const size_t M = (size_t)a.n1h * n3;
  const double2* in = a.xout + (size_t)y * a.plane_stride;
  // plane means U_i = Re u_i(0, 0)
  const double U[3] = {ldu(a.u, 0, (size_t)y * M).x, ldu(a.u, 1, (size_t)y * M).x, ldu(a.u, 2, (size_t)y * M).x};
  auto slot = [&](int s) { return s <= a.kcz ? s : n3 - (nz - s); };  // retained slot -> stored slot
  // F(u_i) on the retained set
  for (int e = threadIdx.x; a.ubar && e < 3 * nk * nz; e += blockDim.x) {
    const int i = e / (nk * nz), r = e - i * nk * nz, l = r / nz, s = r - l * nz;
    const double2 v = ldu(a.u, i, (size_t)y * M + (size_t)(kx0 + l) * n3 + slot(s));
    a.ubar[(((size_t)i * a.n2 + y) * kc1 + kx0 + l) * nz + s] = v;
  }
  const int nf = a.trace_only ? 1 : 6;
  for (int f = 0; f < nf; ++f) {
    const double2* src = in + (size_t)f * f3 * kc1 + kx0;
    for (int e = threadIdx.x; e < K * f3; e += blockDim.x) {
      const int z = e / K, l = e - z * K;
      lds[l * LS + z] = l < nk ? src[(size_t)z * kc1 + l] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    fft_lines<double, 24, kFnComposite>(lds, LS, K, a.plan, a.tw, -1);
    for (int e = threadIdx.x; e < nk * nz; e += blockDim.x) {
      const int l = e / nz, s = e - l * nz;
      const int kz = s <= a.kcz ? s : s - nz;
      const double2 w = lds[l * LS + (kz >= 0 ? kz : f3 + kz)];
      const double2 pp = make_double2(w.x * a.scale, w.y * a.scale);
      const bool k0 = (kx0 + l == 0) && kz == 0;
      const size_t mi = (size_t)y * M + (size_t)(kx0 + l) * n3 + slot(s);
      if (a.trace_only) {
        double2 t = pp;
        if (k0) {
          t.x += U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const double2 ui = ldu(a.u, i, mi);
            t.x += 2.0 * U[i] * ui.x;
            t.y += 2.0 * U[i] * ui.y;
          }
        }
        a.trace[((size_t)y * kc1 + kx0 + l) * nz + s] = t;
        continue;
      }
      const size_t o = (((size_t)f * a.n2 + y) * kc1 + kx0 + l) * nz + s;
      a.pp[o] = pp;
      if (!a.uubar) continue;
      // mean terms: U_i F(u'_j) + U_j F(u'_i) (+ U_i U_j at k = 0)
      const int i = kPairI[f], j = kPairJ[f];
      double2 uj = make_double2(0.0, 0.0), ui = make_double2(0.0, 0.0);
      if (!k0) {
        ui = ldu(a.u, i, mi);
        uj = ldu(a.u, j, mi);
      }
      double2 uu = make_double2(pp.x + U[i] * uj.x + U[j] * ui.x, pp.y + U[i] * uj.y + U[j] * ui.y);
      if (k0) uu.x += U[i] * U[j];
      a.uubar[o] = uu;
    }
    __syncthreads();
  }
}

// Per (y, tile of retained kx): the nine retained fields (six pp, three
// F(u'_i) with zero (0,0) mode) padded from 2 kcz + 1 to q3 slots, inverse in
// z, stored [y][9][q3][kcx+1].
__global__ void __launch_bounds__(256) k_zinv_q(ZinvQArgs a) {
  extern __shared__ unsigned char smem_raw[];
  double2* lds = reinterpret_cast<double2*>(smem_raw);
  const int y = blockIdx.y;
  const int kx0 = blockIdx.x * a.K;
  const int n3 = a.n3, q3 = a.q3, K = a.K, LS = a.lstride;
  const int kc1 = a.kcx + 1, nz = 2 * a.kcz + 1;
  const int nk = min(K, kc1 - kx0);
  const size_t M = (size_t)a.n1h * n3;
  for (int f = 0; f < 9; ++f) {
    for (int e = threadIdx.x; e < K * q3; e += blockDim.x) {
      const int l = e / q3;
      lds[l * LS + (e - l * q3)] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nk * nz; e += blockDim.x) {
      const int l = e / nz, s = e - l * nz;
      const int kz = s <= a.kcz ? s : s - nz;
      double2 v;
      if (f < 6) {
        v = a.pp[(((size_t)f * a.n2 + y) * kc1 + kx0 + l) * nz + s];
      } else {
        const int kx = kx0 + l;
        const int st = kz >= 0 ? kz : n3 + kz;
        v = (kx == 0 && kz == 0) ? make_double2(0.0, 0.0) : ldu(a.u, f - 6, (size_t)y * M + (size_t)kx * n3 + st);
      }
      lds[l * LS + (kz >= 0 ? kz : q3 + kz)] = v;
    }
    __syncthreads();
    fft_lines<double, 24, kFnComposite>(lds, LS, K, a.plan, a.tw, +1);
    double2* out = a.out + ((size_t)(y * 9 + f) * q3) * kc1 + kx0;
    for (int e = threadIdx.x; e < nk * q3; e += blockDim.x) {
      const int z = e / nk, l = e - z * nk;
      out[(size_t)z * kc1 + l] = lds[l * LS + z];
    }
    __syncthreads();
  }
}

// Per (y, z row of the q grid): inverse in x of the nine fields (two real
// fields per complex line, Hermitian-extended from kcx + 1 modes to q1
// points), tau_ij = pp_ij - ub_i ub_j.
__global__ void __launch_bounds__(256) k_xtau(XtauArgs a) {
  extern __shared__ unsigned char smem_raw[];
  double2* lds = reinterpret_cast<double2*>(smem_raw);
  const int y = blockIdx.y, z = blockIdx.x;
  const int q1 = a.q1, q3 = a.q3, LS = a.lstride;
  const int kc1 = a.kcx + 1;
  // line L holds field 2L + i field 2L+1 (fields 0..5 pp, 6..8 ub; field 9 = 0)
  for (int e = threadIdx.x; e < 5 * q1; e += blockDim.x) {
    const int l = e / q1;
    lds[l * LS + (e - l * q1)] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 5 * kc1; e += blockDim.x) {
    const int l = e / kc1, k = e - l * kc1;
    const double2* src = a.in + ((size_t)(y * 9) * q3 + z) * kc1 + k;
    const size_t fs = (size_t)q3 * kc1;
    const double2 X = src[(size_t)(2 * l) * fs];
    const double2 Y = (2 * l + 1 < 9) ? src[(size_t)(2 * l + 1) * fs] : make_double2(0.0, 0.0);
    double2* line = lds + l * LS;
    if (k == 0) {
      line[0] = make_double2(X.x, Y.x);
    } else {
      line[k] = make_double2(X.x - Y.y, X.y + Y.x);
      line[q1 - k] = make_double2(X.x + Y.y, Y.x - X.y);
    }
  }
  __syncthreads();
  fft_lines<double, 24, kFnComposite>(lds, LS, 5, a.plan, a.tw, +1);
  for (int x = threadIdx.x; x < q1; x += blockDim.x) {
    double f[10];
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      const double2 v = lds[l * LS + x];
      f[2 * l] = v.x;
      f[2 * l + 1] = v.y;
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double t = f[p] - f[6 + kPairI[p]] * f[6 + kPairJ[p]];
      a.tau[(((size_t)p * a.n2 + y) * q3 + z) * q1 + x] = t;
    }
  }
}

// ---------------------------------------------------------------- statistics
// One thread per mode-point: the running sums of the two-dimensional spectra
// E_ii(kx, y, kz) = |u_i|^2 (the mean mode (0,0) left out: fluctuations) and,
// on the first mode of each plane, of the mean profiles U1(y), U3(y).
template <typename TP>
__global__ void __launch_bounds__(256) k_stats(StatsArgs<TP> a) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.NP) return;
  const size_t y = idx / a.M, m = idx - y * a.M;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const c2<TP> u = a.u[i][idx];
    const double re = (double)u.x, im = (double)u.y;
    a.spec[(size_t)i * a.NP + idx] += m == 0 ? 0.0 : re * re + im * im;
  }
  if (m == 0) {
    a.mean[y] += a.U1[y];
    a.mean[a.n2 + y] += a.U3[y];
  }
}

// ---------------------------------------------------------------- launchers
template <typename TP> hipError_t launch_stats(const StatsArgs<TP>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_stats<TP>, dim3((unsigned)((a.NP + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_stats<double>(const StatsArgs<double>&, hipStream_t);
template hipError_t launch_stats<float>(const StatsArgs<float>&, hipStream_t);

template <typename T>
hipError_t launch_xfilter(const XfilterArgs<T>& a, size_t lds_bytes, hipStream_t st) {
  // one line of f1 <= 3072 points per transform: 16 staged values per thread
  // hold every radix pass (radix 8: 2 butterflies, 4: 4, 3: 5, 2: 8 per thread);
  // physical values per thread: the fewest of 3, 6, 9, 12 that cover f1
  const dim3 grid(a.f3, a.n2);
  if (!staging_fits(a.plan, 1, 256, 16)) return hipErrorInvalidValue;
  if (a.f1 <= 3 * 256) hipLaunchKernelGGL((k_xfilter<T, 3>), grid, dim3(256), lds_bytes, st, a);
  else if (a.f1 <= 6 * 256) hipLaunchKernelGGL((k_xfilter<T, 6>), grid, dim3(256), lds_bytes, st, a);
  else if (a.f1 <= 9 * 256 && plan_is_1728c(a.plan))  // compile-time 12, 12, 12
    hipLaunchKernelGGL((k_xfilter<T, 9, kFn1728Composite>), grid, dim3(256), lds_bytes, st, a);
  else if (a.f1 <= 9 * 256) hipLaunchKernelGGL((k_xfilter<T, 9>), grid, dim3(256), lds_bytes, st, a);
  else if (a.f1 <= 12 * 256) hipLaunchKernelGGL((k_xfilter<T, 12>), grid, dim3(256), lds_bytes, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_zfilter(const ZfilterArgs& a, size_t lds_bytes, hipStream_t st) {
  if (!staging_fits(a.plan, a.K, 256, 24)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zfilter, dim3((a.kcx + 1 + a.K - 1) / a.K, a.n2), dim3(256), lds_bytes, st, a);
  return hipGetLastError();
}
hipError_t launch_zinv_q(const ZinvQArgs& a, size_t lds_bytes, hipStream_t st) {
  if (!staging_fits(a.plan, a.K, 256, 24)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zinv_q, dim3((a.kcx + 1 + a.K - 1) / a.K, a.n2), dim3(256), lds_bytes, st, a);
  return hipGetLastError();
}
hipError_t launch_xtau(const XtauArgs& a, size_t lds_bytes, hipStream_t st) {
  if (!staging_fits(a.plan, 5, 256, 24)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_xtau, dim3(a.q3, a.n2), dim3(256), lds_bytes, st, a);
  return hipGetLastError();
}

template hipError_t launch_xfilter<double>(const XfilterArgs<double>&, size_t, hipStream_t);

}  // namespace chn
