// Batched in-LDS Stockham FFT for wave64 workgroups (gfx950).
//
// A workgroup transforms `nlines` lines of length N held in LDS (line l at
// lds[l * lstride + e]).  Each pass of radix R reads R strided values per
// butterfly into registers, the whole workgroup synchronises, and the
// twiddled radix-R DFTs are written back in place in Stockham (self-sorting)
// order, so the result is in natural order with no bit reversal.  sgn = -1
// is the forward (analysis) transform, sgn = +1 the unscaled inverse.
#pragma once
#include "common.hpp"

namespace chn {

template <typename T> __device__ __forceinline__ void dft2(c2<T>* v) {
  c2<T> a = v[0], b = v[1];
  v[0] = cadd<T>(a, b);
  v[1] = csub<T>(a, b);
}

template <typename T> __device__ __forceinline__ void dft3(c2<T>* v, int sgn) {
  const T c = T(-0.5);
  const T s = T(0.866025403784438646763723170752936) * T(sgn);
  c2<T> t = cadd<T>(v[1], v[2]);
  c2<T> d = csub<T>(v[1], v[2]);
  c2<T> m = mk<T>(v[0].x + c * t.x, v[0].y + c * t.y);
  v[0] = cadd<T>(v[0], t);
  v[1] = mk<T>(m.x - s * d.y, m.y + s * d.x);
  v[2] = mk<T>(m.x + s * d.y, m.y - s * d.x);
}

template <typename T> __device__ __forceinline__ void dft4(c2<T>& x0, c2<T>& x1, c2<T>& x2, c2<T>& x3, int sgn) {
  c2<T> a = cadd<T>(x0, x2), b = csub<T>(x0, x2);
  c2<T> c = cadd<T>(x1, x3), d = cmuli<T>(csub<T>(x1, x3), sgn);
  x0 = cadd<T>(a, c);
  x2 = csub<T>(a, c);
  x1 = cadd<T>(b, d);
  x3 = csub<T>(b, d);
}

template <typename T> __device__ __forceinline__ void dft8(c2<T>* v, int sgn) {
  const T r2 = T(0.707106781186547524400844362104849);
  c2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  c2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T>(e0, e1, e2, e3, sgn);
  dft4<T>(o0, o1, o2, o3, sgn);
  const T s = T(sgn);
  // o_q *= exp(sgn 2 pi i q / 8)
  o1 = mk<T>(r2 * (o1.x - s * o1.y), r2 * (o1.y + s * o1.x));
  o2 = cmuli<T>(o2, sgn);
  o3 = mk<T>(r2 * (-o3.x - s * o3.y), r2 * (-o3.y + s * o3.x));
  v[0] = cadd<T>(e0, o0); v[4] = csub<T>(e0, o0);
  v[1] = cadd<T>(e1, o1); v[5] = csub<T>(e1, o1);
  v[2] = cadd<T>(e2, o2); v[6] = csub<T>(e2, o2);
  v[3] = cadd<T>(e3, o3); v[7] = csub<T>(e3, o3);
}

// (cos, sin)(2 pi m / R) at compile time: the angle is reduced to the
// nearest multiple q pi / 2 (exact integer arithmetic) plus |rho| <= pi / 4,
// whose Taylor series converges to double rounding in a dozen terms; the
// quadrant rotates the result exactly (so multiples of pi / 2 give 0, +-1).
struct Cis {
  double c, s;
};
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr Cis cis_const(int m, int R) {
  m %= R;
  if (m < 0) m += R;
  const int q = (8 * m + R) / (2 * R);  // nearest integer to 4 m / R
  const double rho = (kPiD / 2) * (double)(4 * m - q * R) / (double)R;
  double c = 1.0, s = rho, tc = 1.0, ts = rho;
  for (int k = 1; k < 12; ++k) {
    tc *= -rho * rho / (double)((2 * k - 1) * (2 * k));
    ts *= -rho * rho / (double)((2 * k) * (2 * k + 1));
    c += tc;
    s += ts;
  }
  switch (q & 3) {
    case 0: return Cis{c, s};
    case 1: return Cis{-s, c};
    case 2: return Cis{-c, -s};
    default: return Cis{s, -c};
  }
}

template <typename T, int R> __device__ __forceinline__ void dft(c2<T>* v, int sgn);

// v * exp(sgn 2 pi i m / R), m and R known at compile time: multiples of a
// quarter turn are exact swaps and negations, the rest one complex product.
template <typename T, int M, int R> __device__ __forceinline__ c2<T> rot(c2<T> v, int sgn) {
  constexpr int m = M % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr ((4 * m) % R == 0) {
    constexpr int q = 4 * m / R;  // quarter turns: 1, 2, 3
    if constexpr (q == 2) return mk<T>(-v.x, -v.y);
    else if constexpr (q == 1) return cmuli<T>(v, sgn);
    else return cmuli<T>(v, -sgn);
  } else {
    constexpr Cis w = cis_const(m, R);
    const T c = T(w.c), s = T(w.s) * T(sgn);
    return mk<T>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// Radix R = R1 R2 in registers (Cooley-Tukey with n = R2 n1 + n2, k = k1 +
// R1 k2): R2 DFTs of length R1, the twiddles exp(sgn 2 pi i n2 k1 / R), R1
// DFTs of length R2, outputs in natural order.
template <typename T, int R1, int R2, int N2, int K1 = 0>
__device__ __forceinline__ void comp_twiddle(const c2<T>* t, c2<T>* w, int sgn) {
  w[N2 * R1 + K1] = rot<T, N2 * K1, R1 * R2>(t[K1], sgn);
  if constexpr (K1 + 1 < R1) comp_twiddle<T, R1, R2, N2, K1 + 1>(t, w, sgn);
}
template <typename T, int R1, int R2, int N2 = 0>
__device__ __forceinline__ void comp_stage1(const c2<T>* v, c2<T>* w, int sgn) {
  c2<T> t[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + N2];
  dft<T, R1>(t, sgn);
  comp_twiddle<T, R1, R2, N2>(t, w, sgn);
  if constexpr (N2 + 1 < R2) comp_stage1<T, R1, R2, N2 + 1>(v, w, sgn);
}
template <typename T, int R1, int R2> __device__ __forceinline__ void dft_comp(c2<T>* v, int sgn) {
  c2<T> w[R1 * R2];
  comp_stage1<T, R1, R2>(v, w, sgn);
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    c2<T> t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = w[n2 * R1 + k1];
    dft<T, R2>(t, sgn);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
  }
}

// Radices of the Stockham passes: 2, 3, 4, 8 directly; 6, 9, 12, 16 as
// compositions held in registers (one LDS round trip for the whole radix).
template <typename T, int R> __device__ __forceinline__ void dft(c2<T>* v, int sgn) {
  if constexpr (R == 2) dft2<T>(v);
  else if constexpr (R == 3) dft3<T>(v, sgn);
  else if constexpr (R == 4) dft4<T>(v[0], v[1], v[2], v[3], sgn);
  else if constexpr (R == 8) dft8<T>(v, sgn);
  else if constexpr (R == 6) dft_comp<T, 2, 3>(v, sgn);
  else if constexpr (R == 9) dft_comp<T, 3, 3>(v, sgn);
  else if constexpr (R == 12) dft_comp<T, 4, 3>(v, sgn);
  else if constexpr (R == 16) dft_comp<T, 4, 4>(v, sgn);
  else static_assert(R == 2, "unsupported radix");
}

// x / d as a multiply-high with m = ceil(2^32 / d) (m = 0 for d = 1): exact
// while x * d < 2^32, which holds for the element indices of a workgroup
__device__ __forceinline__ unsigned qmagic(unsigned d) { return d <= 1 ? 0u : 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ unsigned qdiv(unsigned x, unsigned d, unsigned m) {
  return m == 0 ? x : __umulhi(x, m);
}

// LDS element index within a line: with PAD one slot is skipped after every 8
// elements, which spreads the stride-R and stride-R Ns accesses of the
// Stockham writes over the banks (lines are then lx(N - 1) + 1 long at least).
template <bool PAD> __device__ __forceinline__ int lx(int i) { return PAD ? i + (i >> 3) : i; }

// One radix-R pass over all lines.  NB = butterflies per thread (compile
// time, so the staging array lives in registers); the caller guarantees
// nlines * N / R <= NB * blockDim.x.
template <typename T, int R, int NB, bool PAD = false>
__device__ __forceinline__ void stockham_pass(c2<T>* lds, int lstride, int nlines, int N, int Ns, unsigned mb,
                                              unsigned mk, const c2<T>* __restrict__ tw, int sgn) {
  const int nbl = N / R;
  const int total = nbl * nlines;
  const int nt = blockDim.x;
  c2<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int g = threadIdx.x + q * nt;
    if (g < total) {
      const int line = (int)qdiv((unsigned)g, (unsigned)nbl, mb);
      const int j = g - line * nbl;
      const c2<T>* src = lds + line * lstride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[lx<PAD>(j + r * nbl)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int g = threadIdx.x + q * nt;
    if (g < total) {
      const int line = (int)qdiv((unsigned)g, (unsigned)nbl, mb);
      const int j = g - line * nbl;
      const int k = j - (int)qdiv((unsigned)j, (unsigned)Ns, mk) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          c2<T> t = tw[(r - 1) * Ns + k];
          if (sgn > 0) t.y = -t.y;
          v[q][r] = cmul<T>(v[q][r], t);
        }
      }
      dft<T, R>(v[q], sgn);
      c2<T>* dst = lds + line * lstride;
      const int d0 = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[lx<PAD>(d0 + r * Ns)] = v[q][r];
    }
  }
  __syncthreads();
}

// The same pass with the line length and Ns known at compile time: divisions
// by constants, LDS and twiddle offsets folded into the instructions.  Same
// arithmetic, in the same order, as the runtime pass.
template <typename T, int R, int NB, int N, int NS, bool PAD = false>
__device__ __forceinline__ void stockham_pass_c(c2<T>* lds, int lstride, int nlines, const c2<T>* __restrict__ tw,
                                                int sgn) {
  constexpr int nbl = N / R;
  const int total = nbl * nlines;
  const int nt = blockDim.x;
  c2<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int g = threadIdx.x + q * nt;
    if (g < total) {
      const int line = (unsigned)g / (unsigned)nbl;
      const int j = g - line * nbl;
      if constexpr (!PAD || nbl % 8 == 0) {  // lx(j + r nbl) = lx(j) + r lx(nbl)
        const c2<T>* src = lds + line * lstride + lx<PAD>(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = src[r * (PAD ? nbl + nbl / 8 : nbl)];
      } else {
        const c2<T>* src = lds + line * lstride;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = src[lx<PAD>(j + r * nbl)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int g = threadIdx.x + q * nt;
    if (g < total) {
      const int line = (unsigned)g / (unsigned)nbl;
      const int j = g - line * nbl;
      const int k = (unsigned)j % (unsigned)NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          c2<T> t = tw[(r - 1) * NS + k];
          if (sgn > 0) t.y = -t.y;
          v[q][r] = cmul<T>(v[q][r], t);
        }
      }
      dft<T, R>(v[q], sgn);
      const int d0 = (j - k) * R + k;
      if constexpr (!PAD || NS % 8 == 0) {  // lx(d0 + r NS) = lx(d0) + r lx(NS)
        c2<T>* dst = lds + line * lstride + lx<PAD>(d0);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * (PAD ? NS + NS / 8 : NS)] = v[q][r];
      } else if constexpr (NS == 1 && R == 8) {  // d0 = 8 j: lx(d0 + r) = lx(d0) + r
        c2<T>* dst = lds + line * lstride + lx<PAD>(d0);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = v[q][r];
      } else {
        c2<T>* dst = lds + line * lstride;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[lx<PAD>(d0 + r * NS)] = v[q][r];
      }
    }
  }
  __syncthreads();
}

// FN value of a runtime plan that may hold the composite radices 6, 9, 12,
// 16 (FN = 0: radices 2, 3, 4, 8 only, which keeps the register allocation of
// those kernels to the classic passes).
constexpr int kFnComposite = 1;
// FN of the batched kernels of ensembles: the short composite lines of
// minimal channels (48 = 8 x 6, 72 = 9 x 8, 96 = 12 x 8) take compile-time
// schedules, any other plan the runtime composite passes.
constexpr int kFnShort = 2;
// FN of the compile-time schedule of 576-point lines in the composite radix
// set (9, 8, 8); FN = 576 is the classic one (8, 8, 3, 3).
constexpr int kFn576Composite = 10576;
// FN of the 1728-point schedule in the composite set (12, 12, 12).
constexpr int kFn1728Composite = 11728;

// Full transform of nlines lines of length pl.n.  MAXV = complex values
// staged per thread; every pass must hold nlines * pl.n / R butterflies in
// (MAXV / R) * blockDim.x (the host checks this with the plan).
template <typename T, int MAXV, int FN = 0, bool PAD = false>
__device__ __forceinline__ void fft_lines(c2<T>* lds, int lstride, int nlines, const FftPlan& pl,
                          const c2<T>* __restrict__ tw, int sgn) {
  // 576 = 3/2 x 384 (the 384-mode directions): radices 8, 8, 3, 3 at compile time
  if constexpr (FN == 576) {
    stockham_pass_c<T, 8, MAXV / 8, 576, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
    stockham_pass_c<T, 8, MAXV / 8, 576, 8, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
    stockham_pass_c<T, 3, MAXV / 3, 576, 64, PAD>(lds, lstride, nlines, tw + pl.twoff[2], sgn);
    stockham_pass_c<T, 3, MAXV / 3, 576, 192, PAD>(lds, lstride, nlines, tw + pl.twoff[3], sgn);
    return;
  } else if constexpr (FN == kFn576Composite) {  // 576 in three passes: radices 9, 8, 8
    // (the host never stages this plan in fewer than 9 values per thread)
    if constexpr (MAXV >= 9) {
      stockham_pass_c<T, 9, MAXV / 9, 576, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
      stockham_pass_c<T, 8, MAXV / 8, 576, 9, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
      stockham_pass_c<T, 8, MAXV / 8, 576, 72, PAD>(lds, lstride, nlines, tw + pl.twoff[2], sgn);
    }
    return;
  } else if constexpr (FN == kFn1728Composite) {  // the low-storage product grid in x: 12, 12, 12
    if constexpr (MAXV >= 12) {
      stockham_pass_c<T, 12, MAXV / 12, 1728, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
      stockham_pass_c<T, 12, MAXV / 12, 1728, 12, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
      stockham_pass_c<T, 12, MAXV / 12, 1728, 144, PAD>(lds, lstride, nlines, tw + pl.twoff[2], sgn);
    }
    return;
  } else if constexpr (FN == kFnShort) {
    if constexpr (MAXV >= 12) {
      if (pl.npass == 2 && pl.n == 48 && pl.radix[0] == 8 && pl.radix[1] == 6) {
        stockham_pass_c<T, 8, MAXV / 8, 48, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
        stockham_pass_c<T, 6, MAXV / 6, 48, 8, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
        return;
      }
      if (pl.npass == 2 && pl.n == 72 && pl.radix[0] == 9 && pl.radix[1] == 8) {
        stockham_pass_c<T, 9, MAXV / 9, 72, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
        stockham_pass_c<T, 8, MAXV / 8, 72, 9, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
        return;
      }
      if (pl.npass == 2 && pl.n == 96 && pl.radix[0] == 12 && pl.radix[1] == 8) {
        stockham_pass_c<T, 12, MAXV / 12, 96, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
        stockham_pass_c<T, 8, MAXV / 8, 96, 12, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
        return;
      }
    }
    fft_lines<T, MAXV, kFnComposite, PAD>(lds, lstride, nlines, pl, tw, sgn);
    return;
  } else if constexpr (FN == 9216) {  // 3/2 x 6144: radices 8, 8, 8, 2, 3, 3
    stockham_pass_c<T, 8, MAXV / 8, 9216, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
    stockham_pass_c<T, 8, MAXV / 8, 9216, 8, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
    stockham_pass_c<T, 8, MAXV / 8, 9216, 64, PAD>(lds, lstride, nlines, tw + pl.twoff[2], sgn);
    stockham_pass_c<T, 2, MAXV / 2, 9216, 512, PAD>(lds, lstride, nlines, tw + pl.twoff[3], sgn);
    stockham_pass_c<T, 3, MAXV / 3, 9216, 1024, PAD>(lds, lstride, nlines, tw + pl.twoff[4], sgn);
    stockham_pass_c<T, 3, MAXV / 3, 9216, 3072, PAD>(lds, lstride, nlines, tw + pl.twoff[5], sgn);
    return;
  } else if constexpr (FN == 12288) {  // 3/2 x 8192: radices 8, 8, 8, 8, 3
    stockham_pass_c<T, 8, MAXV / 8, 12288, 1, PAD>(lds, lstride, nlines, tw + pl.twoff[0], sgn);
    stockham_pass_c<T, 8, MAXV / 8, 12288, 8, PAD>(lds, lstride, nlines, tw + pl.twoff[1], sgn);
    stockham_pass_c<T, 8, MAXV / 8, 12288, 64, PAD>(lds, lstride, nlines, tw + pl.twoff[2], sgn);
    stockham_pass_c<T, 8, MAXV / 8, 12288, 512, PAD>(lds, lstride, nlines, tw + pl.twoff[3], sgn);
    stockham_pass_c<T, 3, MAXV / 3, 12288, 4096, PAD>(lds, lstride, nlines, tw + pl.twoff[4], sgn);
    return;
  } else {
  int Ns = 1;
  for (int p = 0; p < pl.npass; ++p) {
    const c2<T>* twp = tw + pl.twoff[p];
    const int R = pl.radix[p];
    const unsigned mb = qmagic((unsigned)(pl.n / R)), mk = qmagic((unsigned)Ns);
    if constexpr (FN == kFnComposite) {
      // composite radices only where the staging holds one butterfly (the
      // host's staging check never plans them otherwise)
      switch (R) {
        case 16:
          if constexpr (MAXV >= 16) stockham_pass<T, 16, MAXV / 16, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn);
          break;
        case 12:
          if constexpr (MAXV >= 12) stockham_pass<T, 12, MAXV / 12, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn);
          break;
        case 9:
          if constexpr (MAXV >= 9) stockham_pass<T, 9, MAXV / 9, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn);
          break;
        case 6:
          if constexpr (MAXV >= 6) stockham_pass<T, 6, MAXV / 6, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn);
          break;
        default: break;
      }
    }
    switch (R) {
      case 8: stockham_pass<T, 8, MAXV / 8, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      case 4: stockham_pass<T, 4, MAXV / 4, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      case 3: stockham_pass<T, 3, MAXV / 3, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      case 2: stockham_pass<T, 2, MAXV / 2, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      default: break;
    }
    Ns *= R;
  }
  }
}

}  // namespace chn
