// Device-side helpers shared by the HIP kernels: complex arithmetic for the
// plan's real type, accurate exp(i pi a/b) for integer a, b, and the
// in-LDS FFTs used by the ring transforms.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace arkcos {

template <typename R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };
template <typename R> using cx_t = typename Cx<R>::T;

template <typename C> __device__ __forceinline__ C cmake(decltype(C{}.x) a, decltype(C{}.x) b) {
  C c; c.x = a; c.y = b; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C{}.x) s) { return cmake<C>(a.x * s, a.y * s); }

// exp(i pi num / den) for integers 0 <= num < 2^24, 0 < den < 2^24.  The
// quotient is rounded once; its rounding residual, obtained exactly with an
// FMA, is applied as a first-order rotation, so the phase is accurate to a
// few ulp for every num/den.
__device__ __forceinline__ float2 expipi_frac(float, int num, int den) {
  float fn = (float)num, fd = (float)den;
  float q = fn / fd;
  float res = fmaf(-q, fd, fn) / fd;
  float s, c;
  sincospif(q, &s, &c);
  float pr = 3.14159265358979f * res;
  return make_float2(fmaf(-pr, s, c), fmaf(pr, c, s));
}
__device__ __forceinline__ double2 expipi_frac(double, int num, int den) {
  double s, c;
  sincospi((double)num / (double)den, &s, &c);
  return make_double2(c, s);
}
template <typename R> __device__ __forceinline__ cx_t<R> expipi(int num, int den) {
  return expipi_frac(R(0), num, den);
}

// e^{-i pi l^2 / n}, the Bluestein chirp, with l^2 reduced modulo 2n exactly
// (l < 65536, so l^2 fits 32 bits).
template <typename R> __device__ __forceinline__ cx_t<R> chirp(int l, int n) {
  uint32_t t = ((uint32_t)l * (uint32_t)l) % (2u * (uint32_t)n);
  return cconj(expipi<R>((int)t, n));
}

// ---------------------------------------------------------------------------
// In-place power-of-two complex FFT of length M in LDS, Stockham formulation
// with radix-16 passes (plus one radix-2/4/8 pass for the leftover factor).
// Each butterfly keeps its R points in registers; its twiddles are the powers
// of one table value w = exp(-2 pi i k / (Ns R)), formed by at most four
// multiplications.  The LDS buffer is padded by one element every 32
// (index i lives at lidx(i)) so the strided writes of the first pass do not
// collide in the same banks.  All threads of the block take part; the block
// is synchronised on entry and exit.  INV = true gives the unnormalised
// inverse.  tw: exp(-2 pi i k / TN) for k < TN, TN a multiple of M.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lidx(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int lds_elems(int m) { return m + (m >> 5) + 1; }

// Unnormalised forward (INV = false) or inverse DFT of R points in registers.
template <typename C, bool INV> __device__ __forceinline__ C mul_mi(C a) {
  // forward: multiply by -i; inverse: by +i
  return INV ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

template <typename C, bool INV> __device__ __forceinline__ void dft2(C& a, C& b) {
  C t = csub(a, b);
  a = cadd(a, b);
  b = t;
}

template <typename C, bool INV> __device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
  C a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = mul_mi<C, INV>(csub(x1, x3));
  x0 = cadd(a0, a2);
  x2 = csub(a0, a2);
  x1 = cadd(a1, a3);
  x3 = csub(a1, a3);
}

// v[k] <- sum_n v[n] W_R^{nk}, natural order in and out.
template <typename C, bool INV, int R> __device__ __forceinline__ void dft_reg(C* v) {
  using T = decltype(C{}.x);
  if constexpr (R == 2) {
    dft2<C, INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<C, INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // n = 2 n1 + n2, k = k1 + 4 k2
    dft4<C, INV>(v[0], v[2], v[4], v[6]);
    dft4<C, INV>(v[1], v[3], v[5], v[7]);
    const T h = T(0.70710678118654752440);
    // twiddles W8^{k1} on the odd half
    C t1 = v[3], t2 = v[5], t3 = v[7];
    v[3] = INV ? cmake<C>(h * (t1.x - t1.y), h * (t1.x + t1.y)) : cmake<C>(h * (t1.x + t1.y), h * (t1.y - t1.x));
    v[5] = mul_mi<C, INV>(t2);
    v[7] = INV ? cmake<C>(-h * (t3.x + t3.y), h * (t3.x - t3.y)) : cmake<C>(h * (t3.y - t3.x), -h * (t3.x + t3.y));
    C o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C a = v[2 * k1], b = v[2 * k1 + 1];
      o[k1] = cadd(a, b);
      o[k1 + 4] = csub(a, b);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = o[k];
  } else {
    static_assert(R == 16, "radix");
    // n = 4 n1 + n2, k = k1 + 4 k2
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<C, INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // now v[4 k1 + n2] = Y[n2][k1]; multiply by W16^{n2 k1}
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173), h = T(0.70710678118654752440);
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
#pragma unroll
      for (int n2 = 1; n2 < 4; ++n2) {
        const int e = k1 * n2;  // exponent of W16 in 1..9
        T wc, ws;               // cos, -sin of 2 pi e / 16
        switch (e) {
          case 1: wc = c1; ws = -s1; break;
          case 2: wc = h; ws = -h; break;
          case 3: wc = s1; ws = -c1; break;
          case 4: wc = 0; ws = -1; break;
          case 6: wc = -h; ws = -h; break;
          case 9: wc = -c1; ws = s1; break;
          default: wc = 1; ws = 0; break;
        }
        if (INV) ws = -ws;
        v[4 * k1 + n2] = cmul(v[4 * k1 + n2], cmake<C>(wc, ws));
      }
    }
    C o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
      dft4<C, INV>(a0, a1, a2, a3);
      o[k1] = a0;
      o[k1 + 4] = a1;
      o[k1 + 8] = a2;
      o[k1 + 12] = a3;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = o[k];
  }
}

// powers w^r, r = 1 .. R-1, each formed by at most four multiplications
template <typename C, int R> __device__ __forceinline__ void twiddle_powers(C w, C* p) {
  p[1] = w;
  if constexpr (R > 2) {
    p[2] = cmul(w, w);
    p[3] = cmul(p[2], w);
  }
  if constexpr (R > 4) {
    p[4] = cmul(p[2], p[2]);
    p[5] = cmul(p[4], w);
    p[6] = cmul(p[4], p[2]);
    p[7] = cmul(p[4], p[3]);
  }
  if constexpr (R > 8) {
    p[8] = cmul(p[4], p[4]);
#pragma unroll
    for (int r = 1; r < 8; ++r) p[8 + r] = cmul(p[8], p[r]);
  }
}

// The ring transforms run NT = 256 or 512 threads per block; a block handles
// FFT lengths up to kFftCap<NT> = 16 NT, so every thread holds one radix-16
// butterfly per pass and at most 16 points in any phase.
template <int NT> constexpr int kFftCap = 16 * NT;

// One Stockham pass of radix RAD over the M points in LDS (butterflies
// j = threadIdx.x + b NT, b < MAXB).  w: the butterfly's twiddle base
// (unused when Ns = 1).
template <typename R, bool INV, int RAD, int MAXB, int NT>
__device__ __forceinline__ void stockham_pass(cx_t<R>* buf, int M, int Ns, cx_t<R> w) {
  using C = cx_t<R>;
  const int Q = M / RAD;
  C v[MAXB][RAD];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < Q) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b][r] = buf[lidx(j + r * Q)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < Q) {
      const int k = j & (Ns - 1);
      if (Ns > 1) {
        C p[RAD];
        twiddle_powers<C, RAD>(INV ? cconj(w) : w, p);
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[b][r] = cmul(v[b][r], p[r]);
      }
      dft_reg<C, INV, RAD>(v[b]);
      const int o = (j - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[lidx(o + r * Ns)] = v[b][r];
    }
  }
  __syncthreads();
}

// Power-of-two FFT of length M <= kFftCap<NT> in LDS: one radix-2, 4 or 8
// pass for the leftover factor (its Ns is 1: no twiddles), then radix-16
// passes.  The twiddles of the radix-16 passes are loaded from the table
// before the first pass so their latency is paid once.
template <typename R, bool INV, int NT>
__device__ void lds_fft(cx_t<R>* buf, int M, const cx_t<R>* __restrict__ tw, int TN) {
  using C = cx_t<R>;
  constexpr int CAP = kFftCap<NT>;
  const int lg = 31 - __clz(M);
  const int rest = lg & 3, n16 = lg >> 2;
  const int j = threadIdx.x;
  auto tw_at = [&](int t) {
    const int Ns = (1 << rest) << (4 * t);
    return (t < n16 && Ns > 1 && j < M / 16) ? tw[(j & (Ns - 1)) * (TN / (Ns * 16))] : cmake<C>(R(1), R(0));
  };
  const C w0 = tw_at(0), w1 = tw_at(1), w2 = tw_at(2);
  if (rest == 1) stockham_pass<R, INV, 2, CAP / 2 / NT, NT>(buf, M, 1, w0);
  else if (rest == 2) stockham_pass<R, INV, 4, CAP / 4 / NT, NT>(buf, M, 1, w0);
  else if (rest == 3) stockham_pass<R, INV, 8, CAP / 8 / NT, NT>(buf, M, 1, w0);
  if (n16 > 0) stockham_pass<R, INV, 16, 1, NT>(buf, M, 1 << rest, w0);
  if (n16 > 1) stockham_pass<R, INV, 16, 1, NT>(buf, M, (1 << rest) << 4, w1);
  if (n16 > 2) stockham_pass<R, INV, 16, 1, NT>(buf, M, (1 << rest) << 8, w2);
}

// ---------------------------------------------------------------------------
// The same FFT for a length M known at compile time (the long rings: M =
// 16 NT, one radix-16 butterfly per thread and pass).  All LDS addresses of a
// butterfly are its base address plus compile-time offsets: the reads
// j + r Q of a pass sit r (Q + Q/32) slots apart (Q a multiple of 32), and
// the writes o + r Ns (o = (j - j mod Ns) RAD + j mod Ns) a constant distance
// out_gap(r) apart (Ns and RAD powers of two).
// ---------------------------------------------------------------------------
template <int NS, int RAD> __device__ __forceinline__ constexpr int out_gap(int r) {
  // o = (j - k) RAD + k with k < NS and j - k a multiple of NS: if NS RAD >= 32,
  // o mod 32 = k mod 32 and o + r NS crosses exactly the 32-slot rows r NS
  // does; if NS RAD <= 32, o mod 32 is a multiple of NS RAD plus k and the
  // RAD outputs stay in one row
  static_assert((NS & (NS - 1)) == 0 && (RAD & (RAD - 1)) == 0, "pass shape");
  return r * NS + ((r * NS) >> 5);
}

// HIN (first pass, NS = 1): the points M/2 .. M-1 are zero and not read.
// HOUT (last pass, NS = M/RAD): only the outputs 0 .. M/2-1 are written.
// REGIN (first pass): the inputs come from io instead of LDS, io[e] being
// point threadIdx.x + e NT (e < 16): thread j's butterfly b takes points
// j + b NT + r Q = io[b + (16 / RAD) r].  REGOUT (last pass, Q = NT): the
// outputs j + r NT stay in io[r] instead of going to LDS; the pass then
// ends without a barrier.
template <typename R, bool INV, int RAD, int NT, int M, int NS, bool HIN = false, bool HOUT = false,
          bool REGIN = false, bool REGOUT = false>
__device__ __forceinline__ void stockham_ct(cx_t<R>* buf, cx_t<R> w, cx_t<R>* io = nullptr) {
  using C = cx_t<R>;
  constexpr int Q = M / RAD;
  constexpr int MAXB = Q / NT;
  static_assert(Q % NT == 0 && Q % 32 == 0 && NT % 32 == 0, "pass shape");
  static_assert((!HIN || NS == 1) && (!HOUT || NS == Q), "pruned pass");
  static_assert((!REGIN || (NS == 1 && M == 16 * NT)) && (!REGOUT || (NS == Q && MAXB == 1)), "register pass");
  constexpr int RG = Q + Q / 32;
  C v[MAXB][RAD];
  if constexpr (REGIN) {
#pragma unroll
    for (int b = 0; b < MAXB; ++b)
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b][r] = (HIN && 2 * r >= RAD) ? cmake<C>(R(0), R(0)) : io[b + MAXB * r];
  } else {
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const C* src = buf + lidx(threadIdx.x + b * NT);
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b][r] = (HIN && 2 * r >= RAD) ? cmake<C>(R(0), R(0)) : src[r * RG];
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * NT;
    const int k = j & (NS - 1);
    if constexpr (NS > 1) {
      C p[RAD];
      twiddle_powers<C, RAD>(INV ? cconj(w) : w, p);
#pragma unroll
      for (int r = 1; r < RAD; ++r) v[b][r] = cmul(v[b][r], p[r]);
    }
    dft_reg<C, INV, RAD>(v[b]);
    if constexpr (REGOUT) {
#pragma unroll
      for (int r = 0; r < RAD; ++r)
        if (!HOUT || 2 * r < RAD) io[r] = v[b][r];
    } else {
      C* dst = buf + lidx((j - k) * RAD + k);
#pragma unroll
      for (int r = 0; r < RAD; ++r)
        if (!HOUT || 2 * r < RAD) dst[out_gap<NS, RAD>(r)] = v[b][r];
    }
  }
  if constexpr (!REGOUT) __syncthreads();
}

template <int M> struct Log2 { static constexpr int value = 1 + Log2<M / 2>::value; };
template <> struct Log2<1> { static constexpr int value = 0; };

// HIN: the input's upper half is zero; HOUT: only the lower half of the
// output is wanted (the two halves of a Bluestein convolution).  REGIN /
// REGOUT: the input / output point threadIdx.x + e NT is io[e] (e < 16)
// instead of LDS (see stockham_ct); with REGIN the block need not be
// synchronised on entry, with REGOUT the call ends without a barrier.
template <typename R, bool INV, int NT, int M, bool HIN = false, bool HOUT = false, bool REGIN = false,
          bool REGOUT = false>
__device__ __forceinline__ void lds_fft_ct(cx_t<R>* buf, const cx_t<R>* __restrict__ tw, int TN,
                                           cx_t<R>* io = nullptr) {
  using C = cx_t<R>;
  constexpr int LG = Log2<M>::value, REST = LG & 3, N16 = LG >> 2;
  static_assert(M == 16 * NT && N16 <= 3 && N16 >= 1, "length");
  constexpr int NS0 = 1 << REST, NS1 = NS0 << 4, NS2 = NS0 << 8;
  constexpr bool H16 = HIN && REST == 0;  // the first radix-16 pass is the first pass
  constexpr bool R16 = REGIN && REST == 0;
  const int j = threadIdx.x;
  auto tw_at = [&](int ns) {
    return ns > 1 ? tw[(j & (ns - 1)) * (TN / (ns * 16))] : cmake<C>(R(1), R(0));
  };
  const C w0 = tw_at(NS0), w1 = tw_at(NS1), w2 = N16 > 2 ? tw_at(NS2) : cmake<C>(R(1), R(0));
  if constexpr (REST == 1) stockham_ct<R, INV, 2, NT, M, 1, HIN, false, REGIN>(buf, w0, io);
  else if constexpr (REST == 2) stockham_ct<R, INV, 4, NT, M, 1, HIN, false, REGIN>(buf, w0, io);
  else if constexpr (REST == 3) stockham_ct<R, INV, 8, NT, M, 1, HIN, false, REGIN>(buf, w0, io);
  stockham_ct<R, INV, 16, NT, M, NS0, H16, HOUT && N16 == 1, R16, REGOUT && N16 == 1>(buf, w0, io);
  if constexpr (N16 > 1) stockham_ct<R, INV, 16, NT, M, NS1, false, HOUT && N16 == 2, false, REGOUT && N16 == 2>(buf, w1, io);
  if constexpr (N16 > 2) stockham_ct<R, INV, 16, NT, M, NS2, false, HOUT, false, REGOUT>(buf, w2, io);
}

// Bluestein's chirp convolution: the length-n DFT of buf[0..n) (padded
// layout) through power-of-two FFTs of length M >= 2n - 1, M <= kFftCap<NT>,
// in place.  filt: FFT_M of the conjugate chirp, followed by the chirp
// e^{-i pi l^2 / n} for l < n.  INV gives the unnormalised inverse DFT.  The
// block is synchronised on entry and on exit; the global loads of each phase
// are issued together before their first use.
template <typename R, bool INV, int NT, int MF = 0>
__device__ __forceinline__ void bluestein(cx_t<R>* buf, int n, int M_, const cx_t<R>* __restrict__ filt,
                                          const cx_t<R>* __restrict__ tw, int TN) {
  const int M = MF > 0 ? MF : M_;
  using C = cx_t<R>;
  constexpr int EPT = kFftCap<NT> / NT;
  const int tid = threadIdx.x;
  {
    C c[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int l = tid + e * NT;
      if (l < n) c[e] = filt[M + l];
    }
    // n <= M/2: the compile-time FFTs skip the zero upper half of the input
    // and the unused upper half of the output
    const int lim = MF > 0 ? M / 2 : M;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int l = tid + e * NT;
      if (l < lim) {
        C v = cmake<C>(R(0), R(0));
        if (l < n) {
          v = buf[lidx(l)];
          if (INV) v = cconj(v);
          v = cmul(v, c[e]);
        }
        buf[lidx(l)] = v;
      }
    }
  }
  __syncthreads();
  if constexpr (MF > 0) lds_fft_ct<R, false, NT, MF, true, false>(buf, tw, TN);
  else lds_fft<R, false, NT>(buf, M, tw, TN);
  {
    C f[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int k = tid + e * NT;
      if (k < M) f[e] = filt[k];
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int k = tid + e * NT;
      if (k < M) buf[lidx(k)] = cmul(buf[lidx(k)], f[e]);
    }
  }
  __syncthreads();
  if constexpr (MF > 0) lds_fft_ct<R, true, NT, MF, false, true>(buf, tw, TN);
  else lds_fft<R, true, NT>(buf, M, tw, TN);
  {
    const R inv = R(1) / R(M);
    C c[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int k = tid + e * NT;
      if (k < n) c[e] = filt[M + k];
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int k = tid + e * NT;
      if (k < n) {
        C v = cscale(cmul(buf[lidx(k)], c[e]), inv);
        if (INV) v = cconj(v);
        buf[lidx(k)] = v;
      }
    }
  }
  __syncthreads();
}

// The same for a compile-time length M = MF = 16 NT, with the phases that
// act point by point kept in registers: io[e] is point threadIdx.x + e NT.
// The chirp product feeds the forward FFT's first pass, the filter product
// sits between the forward FFT's last pass and the inverse FFT's first pass,
// and the final chirp product takes the inverse FFT's last pass.  REGIN:
// the input is io (points >= n zero) instead of buf; REGOUT: the result is
// left in io[e] (e < 8, points < M/2 >= n) instead of buf, and the call ends
// without a barrier.
template <typename R, bool INV, int NT, int MF, bool REGIN, bool REGOUT>
__device__ __forceinline__ void bluestein_ct(cx_t<R>* buf, int n, const cx_t<R>* __restrict__ filt,
                                             const cx_t<R>* __restrict__ tw, int TN, cx_t<R>* io) {
  using C = cx_t<R>;
  constexpr int M = MF;
  constexpr int EPT = 16;
  static_assert(M == EPT * NT, "length");
  const int tid = threadIdx.x;
  C x[EPT];
  {
    C c[EPT / 2];
#pragma unroll
    for (int e = 0; e < EPT / 2; ++e) {
      const int l = tid + e * NT;
      c[e] = l < n ? filt[M + l] : cmake<C>(R(0), R(0));
    }
#pragma unroll
    for (int e = 0; e < EPT / 2; ++e) {
      const int l = tid + e * NT;
      C v = cmake<C>(R(0), R(0));
      if (l < n) v = REGIN ? io[e] : buf[lidx(l)];
      if (INV) v = cconj(v);
      x[e] = cmul(v, c[e]);
      x[e + EPT / 2] = cmake<C>(R(0), R(0));  // n <= M/2: the upper half is zero
    }
  }
  if constexpr (!REGIN) __syncthreads();  // every read of buf done before the first pass writes it
  lds_fft_ct<R, false, NT, M, true, false, true, true>(buf, tw, TN, x);
#pragma unroll
  for (int e = 0; e < EPT; ++e) x[e] = cmul(x[e], filt[tid + e * NT]);
  lds_fft_ct<R, true, NT, M, false, true, true, true>(buf, tw, TN, x);
  const R inv = R(1) / R(M);
#pragma unroll
  for (int e = 0; e < EPT / 2; ++e) {
    const int k = tid + e * NT;
    if (k < n) {
      C v = cscale(cmul(x[e], filt[M + k]), inv);
      if (INV) v = cconj(v);
      if constexpr (REGOUT) io[e] = v;
      else buf[lidx(k)] = v;
    }
  }
  if constexpr (!REGOUT) __syncthreads();
}

// ---------------------------------------------------------------------------
// Mixed-radix FFT in LDS for lengths n = 2^a 3^b 5^c 7^d (n <= 16 NT): a
// Stockham pass per factor (radix 16, 8, 4, 2 for the power of two, then 3,
// 5 and 7), each butterfly's twiddles exp(-/+ 2 pi i k r / (Ns R)) formed
// from one exactly reduced sincospi value by products, the butterflies' R
// points in registers and written back in place after a barrier (the whole
// pass's inputs are read first).  Same padded layout and conventions as
// lds_fft: synchronised on entry and exit, INV = unnormalised inverse.
// ---------------------------------------------------------------------------

// DFT of odd radix R in registers: y_k = sum_r v_r W_R^{rk} from the pairs
// a_r = v_r + v_{R-r}, b_r = v_r - v_{R-r} (exact cosines and sines of 2 pi
// r k / R).
template <typename C, bool INV, int RAD> __device__ __forceinline__ void dft_odd(C* v) {
  using T = decltype(C{}.x);
  static_assert(RAD == 3 || RAD == 5 || RAD == 7, "odd radix");
  constexpr int H = (RAD - 1) / 2;
  // cos / sin of 2 pi q / RAD, q = 1 .. H
  const T cs3[1] = {T(-0.5)}, sn3[1] = {T(0.86602540378443864676)};
  const T cs5[2] = {T(0.30901699437494742410), T(-0.80901699437494742410)};
  const T sn5[2] = {T(0.95105651629515357212), T(0.58778525229247312917)};
  const T cs7[3] = {T(0.62348980185873353053), T(-0.22252093395631440429), T(-0.90096886790241912624)};
  const T sn7[3] = {T(0.78183148246802980871), T(0.97492791218182360702), T(0.43388373911755812048)};
  const T* cs = RAD == 3 ? cs3 : (RAD == 5 ? cs5 : cs7);
  const T* sn = RAD == 3 ? sn3 : (RAD == 5 ? sn5 : sn7);
  C a[H], b[H];
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    a[r - 1] = cadd(v[r], v[RAD - r]);
    b[r - 1] = csub(v[r], v[RAD - r]);
  }
  C y[RAD];
  C s0 = v[0];
#pragma unroll
  for (int r = 0; r < H; ++r) s0 = cadd(s0, a[r]);
  y[0] = s0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    C re = v[0], im = cmake<C>(T(0), T(0));
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      const int q = (r * k) % RAD;                   // W^{rk} = cos(2 pi q / R) - i sin(2 pi q / R)
      const int qq = q <= H ? q : RAD - q;
      const T c = cs[qq - 1], sg = q <= H ? sn[qq - 1] : -sn[qq - 1];
      re = cadd(re, cscale(a[r - 1], c));
      im = cadd(im, cscale(b[r - 1], sg));
    }
    // forward: y_k = re - i im, y_{R-k} = re + i im (inverse: the opposite)
    const C mi = cmake<C>(im.y, -im.x);               // -i im
    y[k] = INV ? csub(re, mi) : cadd(re, mi);
    y[RAD - k] = INV ? cadd(re, mi) : csub(re, mi);
  }
#pragma unroll
  for (int k = 0; k < RAD; ++k) v[k] = y[k];
}

template <typename C, bool INV, int RAD> __device__ __forceinline__ void dft_any(C* v) {
  if constexpr (RAD == 3 || RAD == 5 || RAD == 7) dft_odd<C, INV, RAD>(v);
  else dft_reg<C, INV, RAD>(v);
}

// One mixed-radix Stockham pass of radix RAD over the n points (n / RAD
// butterflies, j = threadIdx.x + b NT), the product of the radices of the
// earlier passes being Ns.
template <typename R, bool INV, int RAD, int NT>
__device__ __forceinline__ void mixed_pass(cx_t<R>* buf, int n, int Ns) {
  using C = cx_t<R>;
  constexpr int MAXB = (16 * NT / RAD + NT - 1) / NT;
  const int Q = n / RAD;
  C v[MAXB][RAD];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < Q) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b][r] = buf[lidx(j + r * Q)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < Q) {
      const int k = j % Ns;
      if (Ns > 1) {
        // w = exp(-2 pi i k / (Ns RAD)) = exp(i pi 2 (Ns RAD - k) / (Ns RAD))
        C w = expipi<R>(2 * (Ns * RAD - k), Ns * RAD);
        if (INV) w = cconj(w);
        C p = w;
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          v[b][r] = cmul(v[b][r], p);
          p = cmul(p, w);
        }
      }
      dft_any<C, INV, RAD>(v[b]);
      const int o = (j - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[lidx(o + r * Ns)] = v[b][r];
    }
  }
  __syncthreads();
}

// The passes of n = 2^a 3^b 5^c 7^d: radix 16 while 16 divides the rest,
// then 8, 4 or 2 once, then the odd factors.
template <typename R, bool INV, int NT>
__device__ void mixed_fft(cx_t<R>* buf, int n) {
  int rest = n, Ns = 1;
  while ((rest & 15) == 0) {
    mixed_pass<R, INV, 16, NT>(buf, n, Ns);
    Ns *= 16;
    rest >>= 4;
  }
  if ((rest & 7) == 0) {
    mixed_pass<R, INV, 8, NT>(buf, n, Ns);
    Ns *= 8;
    rest >>= 3;
  } else if ((rest & 3) == 0) {
    mixed_pass<R, INV, 4, NT>(buf, n, Ns);
    Ns *= 4;
    rest >>= 2;
  } else if ((rest & 1) == 0) {
    mixed_pass<R, INV, 2, NT>(buf, n, Ns);
    Ns *= 2;
    rest >>= 1;
  }
  while (rest % 3 == 0) {
    mixed_pass<R, INV, 3, NT>(buf, n, Ns);
    Ns *= 3;
    rest /= 3;
  }
  while (rest % 5 == 0) {
    mixed_pass<R, INV, 5, NT>(buf, n, Ns);
    Ns *= 5;
    rest /= 5;
  }
  while (rest % 7 == 0) {
    mixed_pass<R, INV, 7, NT>(buf, n, Ns);
    Ns *= 7;
    rest /= 7;
  }
}

// ---------------------------------------------------------------------------
// Wide kernel rows by FFT.  A real sequence x_q, q < 2P, packed as
// z_l = x_2l + i x_2l+1 (l < P) and transformed in place by an LDS FFT of P
// points gives the 2P-point transform of x at any k in [0, 2P):
//   X(k) = E(k) + wk O(k),  E = (Z(k) + conj Z(-k)) / 2,  O = (Z(k) - conj Z(-k)) / 2i,
// with wk = exp(-i pi k / P) for the forward transform and exp(+i pi k / P)
// for the inverse (Z, E, O of period P).  buf: padded layout (lidx).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ cx_t<R> real_from_packed(const cx_t<R>* buf, int P, int k, cx_t<R> wk) {
  using C = cx_t<R>;
  const int k1 = k & (P - 1), k2 = (P - k1) & (P - 1);
  const C z1 = buf[lidx(k1)], z2 = cconj(buf[lidx(k2)]);
  const C e = cscale(cadd(z1, z2), R(0.5));
  const C d = csub(z1, z2);
  const C o = cmake<C>(R(0.5) * d.y, R(-0.5) * d.x);  // d / 2i
  return cadd(e, cmul(wk, o));
}

// Loads and stores through the global address space.  Pointers read from
// memory (per-map argument blocks of the batched kernels) are otherwise
// generic, and generic (flat) accesses count against the LDS wait counter
// as well, which serialises LDS reads behind outstanding global loads.
template <typename T> __device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T> __device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef double d2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gload(const float2* p) {
  const f2v_t v = gload(reinterpret_cast<const f2v_t*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 gload(const double2* p) {
  const d2v_t v = gload(reinterpret_cast<const d2v_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gstore(float2* p, float2 v) {
  f2v_t w;
  w.x = v.x;
  w.y = v.y;
  gstore(reinterpret_cast<f2v_t*>(p), w);
}
__device__ __forceinline__ void gstore(double2* p, double2 v) {
  d2v_t w;
  w.x = v.x;
  w.y = v.y;
  gstore(reinterpret_cast<d2v_t*>(p), w);
}

template <typename T> __device__ __forceinline__ T uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// A~(m) of a ring of N pixels (N even) from the modes 0 .. N/2 that head its
// extended spectrum (a mode m folds to an index no larger than m):
// A~(qN + r) = s^q A~(r) for r <= N/2 and A~(qN + N - k) = s^(q+1) conj(A~(k)),
// s = -1 for rings whose first pixel is offset by half a pixel, 1 otherwise.
// The knot gradient reads spectra this way: a row's correlation then touches
// a few KB per ring, which stay in cache across the rows of a unit, instead
// of the whole extension.
// inv = 1/N in FP32: the quotient m / N (m < 2^24) from the float product is
// off by at most one, then corrected.  ext_index gives the stored mode k and
// the signs of the real and imaginary parts, A~(m) = (sre A(k).x, sim A(k).y);
// a ring and its mirror share them.
struct ExtIdx {
  uint32_t k;
  float sre, sim;
};

__device__ __forceinline__ ExtIdx ext_index(uint32_t N, float inv, bool shifted, uint32_t m) {
  int qi = (int)((float)m * inv);
  int ri = (int)m - qi * (int)N;
  if (ri < 0) {
    ri += (int)N;
    --qi;
  } else if (ri >= (int)N) {
    ri -= (int)N;
    ++qi;
  }
  const uint32_t q = (uint32_t)qi, r = (uint32_t)ri;
  const bool up = 2 * r > N;
  const bool neg = shifted && ((q + (up ? 1u : 0u)) & 1u);
  const float sg = neg ? -1.f : 1.f;
  return ExtIdx{up ? N - r : r, sg, up ? -sg : sg};
}

template <typename C> __device__ __forceinline__ C ext_at(const C* __restrict__ base, const ExtIdx& e) {
  using T = decltype(base->x);
  const C v = base[e.k];
  return cmake<C>(T(e.sre) * v.x, T(e.sim) * v.y);
}

template <typename C>
__device__ __forceinline__ C ext_mode(const C* __restrict__ base, uint32_t N, float inv, bool shifted, uint32_t m) {
  return ext_at(base, ext_index(N, inv, shifted, m));
}

}  // namespace arkcos
