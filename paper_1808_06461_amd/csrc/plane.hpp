// Plane phase of the RK3 sub-step: dealiased u x omega on every x-z plane.
// Kernel bodies and launch helpers; the launchers are split over plane*.hip
// (one translation unit per kernel family and precision, compiled in parallel).
//
// Three passes over a [n2][6][p3][n1/2] intermediate (z-major, kx contiguous):
//   k_zinv : per (y, tile of kx lines): zero-pad kz from n3 to p3 = 3 n3 / 2
//            slots, form omega2 = i b u1 - i a u3 in Fourier space, inverse
//            FFT in z, store transposed so kx is contiguous.
//   k_xpass: per (y, pair of z rows): pad kx to p1 = 3 n1 / 2 (Hermitian
//            extension), two real inverse transforms per complex FFT, products
//            H = u x omega, float64 row sums of H1 and H3 (mean modes) and the
//            row CFL maximum, forward FFT (two real signals per complex FFT),
//            truncate to kx < n1/2, write back in place.
//   k_zfwd : per (y, tile of kx lines): forward FFT in z, keep |kz| < n3/2,
//            scale by 1/(p1 p3), write [n2][n1/2][n3].
// Section 2.1 / Appendix A of the paper (3/2-rule zero padding, rotational
// form of the non-linear term).
#pragma once
#include "fft.hpp"
#include "kernels.hpp"

namespace chn {

static constexpr double kTwoPi = 6.283185307179586476925286766559;

// The z passes and the x pass skip one LDS slot after every 8 elements of a
// line (bank spreading, see lx in fft.hpp); their line stride on the host is
// plane_lds_stride(p) = p + p / 8 + 1.
constexpr bool kPad = true;

// Values of one field staged per thread by the pipelined z passes: the next
// field's loads are issued before the current field's transform, so their
// latency hides behind it.  Fields with more values per thread than this take
// the unpipelined loop.
constexpr int kZinvStage = 8;
constexpr int kZfwdStage = 12;
// Loads per thread issued together by the unpipelined element loops (the
// x pass's coefficient loads, the z passes' fields): a group's values are
// all in flight before the first is written to LDS.
constexpr int kGroup = 6;

// Input coefficient idx of field f; float32 data widened where in_f32 says so.
template <typename T> __device__ __forceinline__ c2<T> ldin(const ZinvArgs<T>& a, int f, size_t idx) {
  if constexpr (sizeof(T) == 8) {
    if ((a.in_f32 >> f) & 1u) {
      const float2 v = reinterpret_cast<const float2*>(a.in[f])[idx];
      return mk<T>((T)v.x, (T)v.y);
    }
  }
  return a.in[f][idx];
}

template <typename T, int MAXV, int FN = 0, bool PIPE = false>
__device__ __forceinline__ void zinv_body(const ZinvArgs<T>& a, int bx, int by) {
  extern __shared__ unsigned char smem_raw[];
  c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
  const int y = a.y0 + by;  // plane of the inputs; `by` indexes `out`
  const int kx0 = bx * a.K;
  const int n1h = a.d.n1h, n3 = a.d.n3, p3 = a.d.p3, K = a.K, LS = a.lstride;
  const int nk = min(K, n1h - kx0);
  const int half = n3 / 2;
  const int npad = p3 - 2 * half + 1;
  // element loops divide by multiply-high (exact: every index times its
  // divisor stays below 2^32)
  const unsigned mnp = qmagic(npad), mn3 = qmagic(n3), mnk = qmagic(nk);
  const double tpx = kTwoPi / a.d.lx, tpz = kTwoPi / a.d.lz;
  const c2<T> zero = mk<T>(T(0), T(0));
  // the first launch of a sub-step's plane phase starts the CFL maximum
  if (a.guard && a.y0 == 0 && bx == 0 && by == 0 && threadIdx.x == 0) a.guard[0] = 0u;
  const int nt = blockDim.x, tot = K * n3;
  if (PIPE && tot <= kZinvStage * nt) {
    // Pipelined: field f's values sit in registers (st) while field f - 1 is
    // transformed.  omega2 = i b u1 - i a u3, when not given, is accumulated
    // in ws from the u1 and u3 values already loaded, so it costs no loads.
    const bool form_w = a.in[4] == nullptr && a.nfields == 6;
    int order[6], loads[6], nl = 0;
    for (int i = 0; i < a.nfields; ++i) order[i] = i;
    if (form_w) {
      const int o[6] = {0, 2, 4, 1, 3, 5};
      for (int i = 0; i < 6; ++i) order[i] = o[i];
    }
    for (int i = 0; i < a.nfields; ++i)
      if (!(form_w && order[i] == 4)) loads[nl++] = order[i];
    c2<T> st[kZinvStage], ws[kZinvStage];
    auto fetch = [&](int f) {
#pragma unroll
      for (int q = 0; q < kZinvStage; ++q) {
        const int e = threadIdx.x + q * nt;
        const int l = (int)qdiv(e, n3, mn3), s = e - l * n3;
        st[q] = zero;
        if (e < tot && l < nk && s != half && !(a.zero_mean && kx0 + l == 0 && s == 0))
          st[q] = ldin(a, f, ((size_t)y * n1h + kx0 + l) * n3 + s);
      }
    };
    fetch(loads[0]);
    int next = 1;
    for (int i = 0; i < a.nfields; ++i) {
      const int f = order[i];
      for (int e = threadIdx.x; e < K * npad; e += nt) {
        const int l = (int)qdiv(e, npad, mnp);
        lds[l * LS + lx<kPad>(half + (e - l * npad))] = zero;
      }
#pragma unroll
      for (int q = 0; q < kZinvStage; ++q) {
        const int e = threadIdx.x + q * nt;
        const int l = (int)qdiv(e, n3, mn3), s = e - l * n3;
        if (e >= tot || s == half) continue;
        c2<T> v = st[q];
        if (form_w) {
          const int kz = s < half ? s : s - n3;
          const T ka = T(tpx * (kx0 + l)), kb = T(tpz * kz);
          if (f == 0) ws[q] = mk<T>(-kb * v.y, kb * v.x);                    // i b u1
          if (f == 2) ws[q] = mk<T>(ws[q].x + ka * v.y, ws[q].y - ka * v.x);  // - i a u3
          if (f == 4) v = ws[q];
        }
        lds[l * LS + lx<kPad>(s < half ? s : p3 - (n3 - s))] = v;
      }
      // the next loaded field's values, in flight during this transform
      if (!(form_w && f == 4) && next < nl) fetch(loads[next++]);
      __syncthreads();
      fft_lines<T, MAXV, FN, kPad>(lds, LS, K, a.plan, a.tw, +1);
      c2<T>* out = a.out + ((size_t)(by * a.nslot + f) * p3) * n1h + kx0;
      for (int e = threadIdx.x; e < nk * p3; e += nt) {
        const int z = (int)qdiv(e, nk, mnk), l = e - z * nk;
        out[(size_t)z * n1h + l] = lds[l * LS + lx<kPad>(z)];
      }
      __syncthreads();
    }
    return;
  }

  for (int f = 0; f < a.nfields; ++f) {
    for (int e = threadIdx.x; e < K * npad; e += blockDim.x) {
      const int l = (int)qdiv(e, npad, mnp);
      lds[l * LS + lx<kPad>(half + (e - l * npad))] = zero;
    }
    // kGroup values per thread loaded together (addresses clamped in
    // bounds, values masked after), then written to LDS
    const bool wform = f == 4 && a.in[4] == nullptr;
    const int tot = K * n3;
    for (int e0 = threadIdx.x; e0 < tot; e0 += kGroup * (int)blockDim.x) {
      c2<T> A[kGroup], B[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int e = e0 + u * blockDim.x;
        const int l = (int)qdiv(e, n3, mn3), s = e - l * n3;
        const bool ok = e < tot && l < nk && s != half && !(a.zero_mean && kx0 + l == 0 && s == 0);
        const size_t idx = ok ? ((size_t)y * n1h + kx0 + l) * n3 + s : 0;
        if (wform) {
          A[u] = ldin(a, 0, idx);
          B[u] = ldin(a, 2, idx);
        } else {
          A[u] = ldin(a, f, idx);
          B[u] = zero;
        }
      }
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int e = e0 + u * blockDim.x;
        const int l = (int)qdiv(e, n3, mn3), s = e - l * n3;
        const bool keep = l < nk && !(a.zero_mean && kx0 + l == 0 && s == 0);
        c2<T> v = keep_if<T>(keep, A[u]);
        if (wform) {  // omega2 = i (b u1 - a u3)
          const int kz = s < half ? s : s - n3;
          const T ka = T(tpx * (kx0 + l)), kb = T(tpz * kz);
          const c2<T> u1 = v, u3 = keep_if<T>(keep, B[u]);
          const c2<T> t = mk<T>(kb * u1.x - ka * u3.x, kb * u1.y - ka * u3.y);
          v = mk<T>(-t.y, t.x);
        }
        if (e < tot && s != half) lds[l * LS + lx<kPad>(s < half ? s : p3 - (n3 - s))] = v;
      }
    }
    __syncthreads();
    fft_lines<T, MAXV, FN, kPad>(lds, LS, K, a.plan, a.tw, +1);
    c2<T>* out = a.out + ((size_t)(by * a.nslot + f) * p3) * n1h + kx0;
    for (int e = threadIdx.x; e < nk * p3; e += blockDim.x) {
      const int z = (int)qdiv(e, nk, mnk), l = e - z * nk;
      out[(size_t)z * n1h + l] = lds[l * LS + lx<kPad>(z)];
    }
    __syncthreads();
  }
}

// x pass over RZ rows (z0 .. z0 + RZ - 1) of one plane per workgroup: line
// 3 row + pair holds field(2 pair) + i field(2 pair + 1), Hermitian-extended;
// after the products, line row holds H1 + i H2 of that row and line RZ + j
// holds H3 of rows 2j (real part) and 2j + 1 (imaginary part).  Rows beyond
// p3 (a ragged last group) are zero and not stored.
template <typename T, int MAXV, int FN = 0, int RZ = 2>
__device__ __forceinline__ void xpass_body(const XpassArgs<T>& a, int bx, int by) {
  extern __shared__ unsigned char smem_raw[];
  c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
  const int y = by;         // plane of buf
  const int yg = a.y0 + by;  // global plane (row sums, CFL, mesh)
  const int z0 = bx * RZ;
  const int n1h = a.d.n1h, p1 = a.d.p1, p3 = a.d.p3, LS = a.lstride;
  const int npad = p1 - 2 * n1h + 1;
  const unsigned mnp = qmagic(npad), mnh = qmagic(n1h);  // exact multiply-high divisions
  const c2<T> zero = mk<T>(T(0), T(0));
  // --- load
  for (int e = threadIdx.x; e < 3 * RZ * npad; e += blockDim.x) {
    const int l = (int)qdiv(e, npad, mnp);
    lds[l * LS + lx<kPad>(n1h + (e - l * npad))] = zero;
  }
  // coefficients fetched kGroup per thread at a time, every load of a group
  // in flight together (addresses clamped in bounds, values masked after)
  const int tot = 3 * RZ * n1h, nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < tot; e0 += kGroup * nt) {
    c2<T> X[kGroup], Y[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int e = e0 + u * nt;
      const int l = (int)qdiv(e, n1h, mnh), k = e - l * n1h;
      const int row = l / 3, pr = l - row * 3;
      const bool ok = e < tot && z0 + row < p3;
      const size_t base = ok ? ((size_t)(y * 6 + 2 * pr) * p3 + z0 + row) * n1h + k : 0;
      X[u] = a.buf[base];
      Y[u] = a.buf[base + (size_t)p3 * n1h];
    }
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int e = e0 + u * nt;
      const int l = (int)qdiv(e, n1h, mnh), k = e - l * n1h;
      const c2<T> Xu = keep_if<T>(z0 + l / 3 < p3, X[u]), Yu = keep_if<T>(z0 + l / 3 < p3, Y[u]);
      c2<T>* line = lds + l * LS;
      if (e < tot && k == 0) {
        line[0] = mk<T>(Xu.x, Yu.x);
      } else if (e < tot) {
        line[lx<kPad>(k)] = mk<T>(Xu.x - Yu.y, Xu.y + Yu.x);
        line[lx<kPad>(p1 - k)] = mk<T>(Xu.x + Yu.y, Yu.x - Xu.y);
      }
    }
  }
  __syncthreads();
  fft_lines<T, MAXV, FN, kPad>(lds, LS, 3 * RZ, a.plan, a.tw, +1);
  // --- products, row sums and CFL
  const T idx_ = T(a.inv_dx), idy = T(a.inv_dy[yg]), idz = T(a.inv_dz);
  // (the compile-time 576-point schedules never take the short-row branch)
  constexpr bool kLong = FN == 576 || FN == kFn576Composite;
  if (!kLong && p1 < 256) {
    // Short rows: one wave per row (rows dealt to the waves in turn), lane l
    // summing x = l, l + 64, ... in order, then a wave reduction: every
    // thread is busy and the order of the sums depends on the row length
    // only (the same bits for any rows per workgroup).  The products stay in
    // registers until every input line has been read.
    constexpr int RW = (RZ + 3) / 4, PL = 4;  // rows per wave (four waves), points per lane
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T hv[RW][PL][3];
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const int row = wid + 4 * j;
      double t1 = 0.0, t3 = 0.0;
      T c = T(0);
#pragma unroll
      for (int q = 0; q < PL; ++q) {
        const int x = lane + 64 * q;
        hv[j][q][0] = hv[j][q][1] = hv[j][q][2] = T(0);
        if (row < RZ && x < p1) {
          const int px = lx<kPad>(x);
          const c2<T> Z0 = lds[(3 * row + 0) * LS + px];
          const c2<T> Z1 = lds[(3 * row + 1) * LS + px];
          const c2<T> Z2 = lds[(3 * row + 2) * LS + px];
          const T u1 = Z0.x, u2 = Z0.y, u3 = Z1.x, o1 = Z1.y, o2 = Z2.x, o3 = Z2.y;
          hv[j][q][0] = u2 * o3 - u3 * o2;
          hv[j][q][1] = u3 * o1 - u1 * o3;
          hv[j][q][2] = u1 * o2 - u2 * o1;
          t1 += (double)hv[j][q][0];
          t3 += (double)hv[j][q][2];
          c = nanmax(c, fabs(u1) * idx_ + fabs(u2) * idy + fabs(u3) * idz);
        }
      }
      double tc = (double)c;
      for (int off = 32; off > 0; off >>= 1) {
        t1 += __shfl_xor(t1, off);
        t3 += __shfl_xor(t3, off);
        tc = nanmax(tc, __shfl_xor(tc, off));
      }
      if (lane == 0 && row < RZ && z0 + row < p3) {
        const size_t o = (size_t)yg * p3 + z0 + row;
        a.rowsum[o] = t1;
        a.rowsum[(size_t)a.d.n2 * p3 + o] = t3;
        a.rowcfl[o] = tc;
        if (a.guard) atomicMax(a.guard, __float_as_uint(fabsf((float)tc)) | (tc != tc ? kGuardNonFinite : 0u));
      }
    }
    __syncthreads();
    // line row <- H1 + i H2 of the row; line RZ + row / 2 <- H3 of rows 2j (real) and 2j + 1 (imaginary)
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const int row = wid + 4 * j;
#pragma unroll
      for (int q = 0; q < PL; ++q) {
        const int x = lane + 64 * q;
        if (row < RZ && x < p1) {
          const int px = lx<kPad>(x);
          lds[row * LS + px] = mk<T>(hv[j][q][0], hv[j][q][1]);
          reinterpret_cast<T*>(&lds[(RZ + row / 2) * LS + px])[row & 1] = hv[j][q][2];
        }
      }
    }
    __syncthreads();
  } else {
  double s1[RZ], s3[RZ];
  T cf[RZ];  // CFL numbers in the transform precision (they only report)
#pragma unroll
  for (int row = 0; row < RZ; ++row) {
    s1[row] = s3[row] = 0.0;
    cf[row] = T(0);
  }
  for (int x = threadIdx.x; x < p1; x += blockDim.x) {
    const int px = lx<kPad>(x);
    T h3[RZ];
#pragma unroll
    for (int row = 0; row < RZ; ++row) {
      const c2<T> Z0 = lds[(3 * row + 0) * LS + px];
      const c2<T> Z1 = lds[(3 * row + 1) * LS + px];
      const c2<T> Z2 = lds[(3 * row + 2) * LS + px];
      const T u1 = Z0.x, u2 = Z0.y, u3 = Z1.x, o1 = Z1.y, o2 = Z2.x, o3 = Z2.y;
      const T H1 = u2 * o3 - u3 * o2;
      const T H2 = u3 * o1 - u1 * o3;
      h3[row] = u1 * o2 - u2 * o1;
      s1[row] += (double)H1;
      s3[row] += (double)h3[row];
      const T c = fabs(u1) * idx_ + fabs(u2) * idy + fabs(u3) * idz;
      cf[row] = nanmax(cf[row], c);
      // line `row` belongs to row row / 3 <= row, already read at this x
      lds[row * LS + px] = mk<T>(H1, H2);
    }
#pragma unroll
    for (int j = 0; j < RZ / 2; ++j) lds[(RZ + j) * LS + px] = mk<T>(h3[2 * j], h3[2 * j + 1]);
  }
  // block reductions: wave64 shuffles, then across the waves through LDS
  __shared__ double red[3 * RZ][4];
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 3 * RZ; ++q) {
    const int row = q % RZ, kind = q / RZ;
    double v = kind == 0 ? s1[row] : (kind == 1 ? s3[row] : (double)cf[row]);
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off);
      v = kind < 2 ? v + o : nanmax(v, o);
    }
    if ((threadIdx.x & 63) == 0) red[q][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < RZ && z0 + (int)threadIdx.x < p3) {
    const int row = threadIdx.x;
    const int nw = blockDim.x >> 6;
    double t1 = 0.0, t3 = 0.0, tc = 0.0;
    for (int w = 0; w < nw; ++w) {
      t1 += red[row][w];
      t3 += red[RZ + row][w];
      tc = nanmax(tc, red[2 * RZ + row][w]);
    }
    const size_t o = (size_t)yg * p3 + z0 + row;
    a.rowsum[o] = t1;
    a.rowsum[(size_t)a.d.n2 * p3 + o] = t3;
    a.rowcfl[o] = tc;
    if (a.guard) atomicMax(a.guard, __float_as_uint(fabsf((float)tc)) | (tc != tc ? kGuardNonFinite : 0u));
  }
  }
  fft_lines<T, MAXV, FN, kPad>(lds, LS, RZ + RZ / 2, a.plan, a.tw, -1);
  // --- unpack two real spectra per line, truncate, store in place over fields 0..2
  for (int e = threadIdx.x; e < (RZ + RZ / 2) * n1h; e += blockDim.x) {
    const int l = (int)qdiv(e, n1h, mnh), k = e - l * n1h;
    const c2<T> W = lds[l * LS + lx<kPad>(k)];
    const c2<T> Wm = lds[l * LS + lx<kPad>(k == 0 ? 0 : p1 - k)];
    const c2<T> P = mk<T>(T(0.5) * (W.x + Wm.x), T(0.5) * (W.y - Wm.y));   // (W_k + conj W_m)/2
    const c2<T> Q = mk<T>(T(0.5) * (W.y + Wm.y), T(-0.5) * (W.x - Wm.x));  // (W_k - conj W_m)/(2i)
    if (l < RZ) {  // row l: H1 = P, H2 = Q
      if (z0 + l < p3) {
        a.buf[((size_t)(y * 6 + 0) * p3 + z0 + l) * n1h + k] = P;
        a.buf[((size_t)(y * 6 + 1) * p3 + z0 + l) * n1h + k] = Q;
      }
    } else {       // H3 of rows 2j and 2j + 1
      const int r0 = 2 * (l - RZ);
      if (z0 + r0 < p3) a.buf[((size_t)(y * 6 + 2) * p3 + z0 + r0) * n1h + k] = P;
      if (z0 + r0 + 1 < p3) a.buf[((size_t)(y * 6 + 2) * p3 + z0 + r0 + 1) * n1h + k] = Q;
    }
  }
}

// Long rows (one row per workgroup, NT threads): the three input lines go
// through LDS one at a time and the physical values stay in registers
// (thread t owns x = t + NT q, q < QX); the products are formed in registers,
// then H1 + i H2 and H3 are transformed forward one line at a time.  Used
// when six lines of the row do not fit the two-row kernel.
template <typename T, int NT, int QX, int MAXV, int FN = 0>
__device__ __forceinline__ void xrow_body(const XpassArgs<T>& a, int z, int y) {
  static_assert(FN == 0 || FN == kFnComposite || FN == 12288, "compile-time schedules of long rows: 12288 points");
  extern __shared__ unsigned char smem_raw[];
  c2<T>* line = reinterpret_cast<c2<T>*>(smem_raw);
  const int n1h = a.d.n1h, p1 = a.d.p1, p3 = a.d.p3;
  const c2<T> zero = mk<T>(T(0), T(0));
  // line l (fields 2l + i 2l+1, Hermitian-extended) -> physical values of this thread
  auto inverse = [&](int l, c2<T>(&r)[QX]) {
    for (int x = n1h + threadIdx.x; x <= p1 - n1h; x += NT) line[x] = zero;
    const size_t base = ((size_t)(y * 6 + 2 * l) * p3 + z) * n1h;
    for (int k = threadIdx.x; k < n1h; k += NT) {
      const c2<T> X = a.buf[base + k];
      const c2<T> Y = a.buf[base + (size_t)p3 * n1h + k];
      if (k == 0) {
        line[0] = mk<T>(X.x, Y.x);
      } else {
        line[k] = mk<T>(X.x - Y.y, X.y + Y.x);
        line[p1 - k] = mk<T>(X.x + Y.y, Y.x - X.y);
      }
    }
    __syncthreads();
    fft_lines<T, MAXV, FN>(line, p1, 1, a.plan, a.tw, +1);
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int x = threadIdx.x + q * NT;
      r[q] = keep_if<T>(x < p1, line[x < p1 ? x : 0]);
    }
    __syncthreads();
  };
  c2<T> r0[QX], r1[QX], r2[QX];
  inverse(0, r0);
  inverse(1, r1);
  inverse(2, r2);
  // products (r0 <- H1 + i H2, r1 <- H3), row sums and CFL
  double s1 = 0.0, s3 = 0.0, cf = 0.0;
  const double idy = a.inv_dy[a.y0 + y];
#pragma unroll
  for (int q = 0; q < QX; ++q) {
    const T u1 = r0[q].x, u2 = r0[q].y, u3 = r1[q].x, o1 = r1[q].y, o2 = r2[q].x, o3 = r2[q].y;
    const T H1 = u2 * o3 - u3 * o2;
    const T H2 = u3 * o1 - u1 * o3;
    const T H3 = u1 * o2 - u2 * o1;
    if (threadIdx.x + q * NT < p1) {
      s1 += (double)H1;
      s3 += (double)H3;
      cf = nanmax(cf, fabs((double)u1) * a.inv_dx + fabs((double)u2) * idy + fabs((double)u3) * a.inv_dz);
    }
    r0[q] = mk<T>(H1, H2);
    r1[q] = mk<T>(H3, T(0));
  }
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_xor(s1, off);
    s3 += __shfl_xor(s3, off);
    cf = nanmax(cf, __shfl_xor(cf, off));
  }
  __shared__ double red[3][NT / 64];
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wid] = s1;
    red[1][wid] = s3;
    red[2][wid] = cf;
  }
  // forward transforms: line 0 = H1 + i H2 (two real spectra), line 1 = H3
  auto forward = [&](int l, const c2<T>(&r)[QX]) {
#pragma unroll
    for (int q = 0; q < QX; ++q) {
      const int x = threadIdx.x + q * NT;
      if (x < p1) line[x] = r[q];
    }
    __syncthreads();
    if (l == 0 && threadIdx.x == 0) {
      double t1 = 0.0, t3 = 0.0, tc = 0.0;
      for (int w = 0; w < NT / 64; ++w) {
        t1 += red[0][w];
        t3 += red[1][w];
        tc = nanmax(tc, red[2][w]);
      }
      const size_t o = (size_t)(a.y0 + y) * p3 + z;
      a.rowsum[o] = t1;
      a.rowsum[(size_t)a.d.n2 * p3 + o] = t3;
      a.rowcfl[o] = tc;
      if (a.guard) atomicMax(a.guard, __float_as_uint(fabsf((float)tc)) | (tc != tc ? kGuardNonFinite : 0u));
    }
    fft_lines<T, MAXV, FN>(line, p1, 1, a.plan, a.tw, -1);
    for (int k = threadIdx.x; k < n1h; k += NT) {
      const c2<T> W = line[k];
      if (l == 0) {
        const c2<T> Wm = line[k == 0 ? 0 : p1 - k];
        a.buf[((size_t)(y * 6 + 0) * p3 + z) * n1h + k] = mk<T>(T(0.5) * (W.x + Wm.x), T(0.5) * (W.y - Wm.y));
        a.buf[((size_t)(y * 6 + 1) * p3 + z) * n1h + k] = mk<T>(T(0.5) * (W.y + Wm.y), T(-0.5) * (W.x - Wm.x));
      } else {
        a.buf[((size_t)(y * 6 + 2) * p3 + z) * n1h + k] = W;
      }
    }
    __syncthreads();
  };
  forward(0, r0);
  forward(1, r1);
}

template <typename T, typename TO, int MAXV, int FN = 0, bool PIPE = false>
__device__ __forceinline__ void zfwd_body(const ZfwdArgs<T, TO>& a, int bx, int by) {
  extern __shared__ unsigned char smem_raw[];
  c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
  const int y = by;
  const int kx0 = bx * a.K;
  const int n1h = a.d.n1h, n3 = a.d.n3, p3 = a.d.p3, K = a.K, LS = a.lstride;
  const int nk = min(K, n1h - kx0);
  const int half = n3 / 2;
  const unsigned mK = qmagic(K), mn3 = qmagic(n3);  // exact multiply-high divisions
  const T scale = T(a.scale);
  const c2<T> zero = mk<T>(T(0), T(0));
  const int nt = blockDim.x, tot = K * p3;
  auto store = [&](int f) {
    c2<TO>* out = a.out[f] + ((size_t)(a.y0 + y) * n1h + kx0) * n3;
    for (int e = threadIdx.x; e < nk * n3; e += nt) {
      const int l = (int)qdiv(e, n3, mn3), s = e - l * n3;
      c2<TO> v = mk<TO>(TO(0), TO(0));
      if (s != half) {
        const c2<T> w = lds[l * LS + lx<kPad>(s < half ? s : p3 - (n3 - s))];
        v = mk<TO>(TO(w.x * scale), TO(w.y * scale));
      }
      out[(size_t)l * n3 + s] = v;
    }
  };
  if (PIPE && tot <= kZfwdStage * nt) {
    // Pipelined: the next field's transposed lines are loaded into registers
    // while this one is transformed.
    c2<T> st[kZfwdStage];
    auto fetch = [&](int f) {
      const c2<T>* in = a.buf + ((size_t)(y * 6 + f) * p3) * n1h + kx0;
#pragma unroll
      for (int q = 0; q < kZfwdStage; ++q) {
        const int e = threadIdx.x + q * nt;
        const int z = (int)qdiv(e, K, mK), l = e - z * K;
        const bool ok = e < tot && l < nk;
        st[q] = keep_if<T>(ok, in[ok ? (size_t)z * n1h + l : 0]);
      }
    };
    fetch(0);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
      for (int q = 0; q < kZfwdStage; ++q) {
        const int e = threadIdx.x + q * nt;
        const int z = (int)qdiv(e, K, mK), l = e - z * K;
        if (e < tot) lds[l * LS + lx<kPad>(z)] = st[q];
      }
      if (f < 2) fetch(f + 1);
      __syncthreads();
      fft_lines<T, MAXV, FN, kPad>(lds, LS, K, a.plan, a.tw, -1);
      store(f);
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const c2<T>* in = a.buf + ((size_t)(y * 6 + f) * p3) * n1h + kx0;
    for (int e0 = threadIdx.x; e0 < tot; e0 += kGroup * nt) {
      c2<T> v[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int e = e0 + u * nt;
        const int z = (int)qdiv(e, K, mK), l = e - z * K;
        v[u] = in[e < tot && l < nk ? (size_t)z * n1h + l : 0];
      }
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int e = e0 + u * nt;
        const int z = (int)qdiv(e, K, mK), l = e - z * K;
        if (e < tot) lds[l * LS + lx<kPad>(z)] = keep_if<T>(l < nk, v[u]);
      }
    }
    __syncthreads();
    fft_lines<T, MAXV, FN, kPad>(lds, LS, K, a.plan, a.tw, -1);
    store(f);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- entry points
// Single-context launches index blocks by (blockIdx.x, blockIdx.y); batched
// launches (ensembles) read (context, bx, by) from a work list and the
// context's arguments from a descriptor array.
// z passes: tiles of K kx lines; the logical tile order is XCD-aware so that
// tiles sharing the cache lines of the transposed intermediate meet in one L2
__device__ __forceinline__ int2 z_tile() {
  const int n = gridDim.x * gridDim.y;
  const int t = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, n);
  return make_int2(t % gridDim.x, t / gridDim.x);
}
template <typename T, int MAXV, int FN, int NT = 256, bool PIPE = false>
__global__ void __launch_bounds__(NT) k_zinv(ZinvArgs<T> a) {
  const int2 t = z_tile();
  zinv_body<T, MAXV, FN, PIPE>(a, t.x, t.y);
}
template <typename T, int MAXV, int FN, int RZ>
__global__ void __launch_bounds__(256) k_xpass(XpassArgs<T> a) { xpass_body<T, MAXV, FN, RZ>(a, blockIdx.x, blockIdx.y); }
template <typename T, int NT, int QX, int MAXV, int FN = 0>
__global__ void __launch_bounds__(NT) k_xrow(XpassArgs<T> a) { xrow_body<T, NT, QX, MAXV, FN>(a, blockIdx.x, blockIdx.y); }
template <typename T, typename TO, int MAXV, int FN, int NT = 256, bool PIPE = false>
__global__ void __launch_bounds__(NT) k_zfwd(ZfwdArgs<T, TO> a) {
  const int2 t = z_tile();
  zfwd_body<T, TO, MAXV, FN, PIPE>(a, t.x, t.y);
}

template <typename T, int MAXV, int FN = 0>
__global__ void __launch_bounds__(256) k_zinv_batch(const ZinvArgs<T>* __restrict__ d, const int4* __restrict__ w) {
  const int4 q = w[blockIdx.x];
  zinv_body<T, MAXV, FN>(d[q.x], q.y, q.z);
}
template <typename T, int MAXV, int RZ, int FN = 0>
__global__ void __launch_bounds__(256) k_xpass_batch(const XpassArgs<T>* __restrict__ d, const int4* __restrict__ w) {
  const int4 q = w[blockIdx.x];
  xpass_body<T, MAXV, FN, RZ>(d[q.x], q.y, q.z);
}
template <typename T, int MAXV, int FN = 0>
__global__ void __launch_bounds__(256) k_zfwd_batch(const ZfwdArgs<T, T>* __restrict__ d, const int4* __restrict__ w) {
  const int4 q = w[blockIdx.x];
  zfwd_body<T, T, MAXV, FN>(d[q.x], q.y, q.z);
}

// ---------------------------------------------------------------- launchers
template <typename T> struct FftMaxv;
template <> struct FftMaxv<double> { static constexpr int v = 24; };
template <> struct FftMaxv<float> { static constexpr int v = 48; };

// Staging registers of the transforms: the smallest MAXV (complex values
// per thread) that holds every pass of nlines lines over nt threads.  The
// register allocation of a kernel follows its largest radix path, so a
// tight MAXV raises occupancy.
template <typename T> int pick_staging(const FftPlan& pl, int nlines, int nt) {
  static const int cf[4] = {16, 24, 32, 48}, cd[4] = {8, 12, 16, 24};
  const int* c = sizeof(T) == 4 ? cf : cd;
  for (int i = 0; i < 4; ++i)
    if (staging_fits(pl, nlines, nt, c[i])) return c[i];
  return 0;
}

#define CHN_STAGED(T, m, ...)                                 \
  do {                                                           \
    if constexpr (sizeof(T) == 4) {                              \
      if (m == 16) { constexpr int MV = 16; __VA_ARGS__; }            \
      else if (m == 24) { constexpr int MV = 24; __VA_ARGS__; }       \
      else if (m == 32) { constexpr int MV = 32; __VA_ARGS__; }       \
      else if (m == 48) { constexpr int MV = 48; __VA_ARGS__; }       \
      else return hipErrorInvalidValue;                          \
    } else {                                                     \
      if (m == 8) { constexpr int MV = 8; __VA_ARGS__; }              \
      else if (m == 12) { constexpr int MV = 12; __VA_ARGS__; }       \
      else if (m == 16) { constexpr int MV = 16; __VA_ARGS__; }       \
      else if (m == 24) { constexpr int MV = 24; __VA_ARGS__; }       \
      else return hipErrorInvalidValue;                          \
    }                                                            \
  } while (0)

// Long z lines (one line per workgroup) get 1024 threads: LDS then admits
// one workgroup per CU, and 16 waves keep it busy.
inline int z_threads(const FftPlan& pl, int K) { return K == 1 && pl.n >= 4096 ? 1024 : 256; }

// Rows of p1 points: two rows per workgroup while six lines fit the
// staging registers, otherwise one row per workgroup of 256 / 512 / 1024
// threads holding QX points each (xrow_limit gives the largest p1).
template <typename T> struct XrowCfg;
template <> struct XrowCfg<float> { static constexpr int QX = 12, MV = 16; };
template <> struct XrowCfg<double> { static constexpr int QX = 6, MV = 8; };

#define CHN_ROWS(rz, ...)                                   \
  do {                                                      \
    if (rz == 2) { constexpr int RZ = 2; __VA_ARGS__; }     \
    else if (rz == 4) { constexpr int RZ = 4; __VA_ARGS__; } \
    else if (rz == 8) { constexpr int RZ = 8; __VA_ARGS__; } \
    else return hipErrorInvalidValue;                       \
  } while (0)

}  // namespace chn
