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

template <typename T, int R> __device__ __forceinline__ void dft(c2<T>* v, int sgn) {
  if constexpr (R == 2) dft2<T>(v);
  else if constexpr (R == 3) dft3<T>(v, sgn);
  else if constexpr (R == 4) dft4<T>(v[0], v[1], v[2], v[3], sgn);
  else dft8<T>(v, sgn);
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

// Full transform of nlines lines of length pl.n.  MAXV = complex values
// staged per thread (a multiple of 24); requires nlines * pl.n <= MAXV * blockDim.x.
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
    switch (R) {
      case 8: stockham_pass<T, 8, MAXV / 8, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      case 4: stockham_pass<T, 4, MAXV / 4, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      case 3: stockham_pass<T, 3, MAXV / 3, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
      default: stockham_pass<T, 2, MAXV / 2, PAD>(lds, lstride, nlines, pl.n, Ns, mb, mk, twp, sgn); break;
    }
    Ns *= R;
  }
  }
}

}  // namespace chn
