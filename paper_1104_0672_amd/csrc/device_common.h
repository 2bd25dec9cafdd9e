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

// e^{-i pi l^2 / n}, the Bluestein chirp, with l^2 reduced modulo 2n exactly.
template <typename R> __device__ __forceinline__ cx_t<R> chirp(int l, int n) {
  int64_t t = ((int64_t)l * (int64_t)l) % (2 * (int64_t)n);
  return cconj(expipi<R>((int)t, n));
}

// ---------------------------------------------------------------------------
// In-place power-of-two complex FFT of length M in LDS (Stockham formulation,
// radix-4 passes and one radix-2 pass when log2 M is odd).  All threads of the
// block take part; on entry and exit the data are in natural order and the
// block is synchronised.  INV = true computes the unnormalised inverse.
// tw: exp(-2 pi i k / TN) for k < TN, TN a multiple of M.
// ---------------------------------------------------------------------------
template <typename R> struct FftLimits;
template <> struct FftLimits<float> { static constexpr int kMaxM = 8192; };
template <> struct FftLimits<double> { static constexpr int kMaxM = 4096; };

template <typename R, bool INV>
__device__ void lds_fft(cx_t<R>* buf, int M, const cx_t<R>* __restrict__ tw, int TN) {
  using C = cx_t<R>;
  constexpr int MAXB4 = FftLimits<R>::kMaxM / 4 / 256;
  constexpr int MAXB2 = FftLimits<R>::kMaxM / 2 / 256;
  const int tid = threadIdx.x, nth = blockDim.x;
  int lg = 31 - __clz(M);
  int Ns = 1;
  while (lg >= 2) {
    const int Q = M >> 2;
    const int tstep = TN / (Ns * 4);
    C v[MAXB4][4];
#pragma unroll
    for (int b = 0; b < MAXB4; ++b) {
      int j = tid + b * nth;
      if (j < Q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[b][r] = buf[j + r * Q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB4; ++b) {
      int j = tid + b * nth;
      if (j < Q) {
        int k = j & (Ns - 1);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          C t = tw[(k * r) * tstep];
          if (INV) t = cconj(t);
          v[b][r] = cmul(v[b][r], t);
        }
        C a0 = cadd(v[b][0], v[b][2]), a1 = csub(v[b][0], v[b][2]);
        C a2 = cadd(v[b][1], v[b][3]), d = csub(v[b][1], v[b][3]);
        // forward: multiply d by -i; inverse: by +i
        C a3 = INV ? cmake<C>(-d.y, d.x) : cmake<C>(d.y, -d.x);
        int o = (j - k) * 4 + k;
        buf[o] = cadd(a0, a2);
        buf[o + Ns] = cadd(a1, a3);
        buf[o + 2 * Ns] = csub(a0, a2);
        buf[o + 3 * Ns] = csub(a1, a3);
      }
    }
    __syncthreads();
    Ns <<= 2;
    lg -= 2;
  }
  if (lg == 1) {
    const int Q = M >> 1;
    const int tstep = TN / (Ns * 2);
    C v[MAXB2][2];
#pragma unroll
    for (int b = 0; b < MAXB2; ++b) {
      int j = tid + b * nth;
      if (j < Q) { v[b][0] = buf[j]; v[b][1] = buf[j + Q]; }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB2; ++b) {
      int j = tid + b * nth;
      if (j < Q) {
        int k = j & (Ns - 1);
        C t = tw[k * tstep];
        if (INV) t = cconj(t);
        C x1 = cmul(v[b][1], t);
        int o = (j - k) * 2 + k;
        buf[o] = cadd(v[b][0], x1);
        buf[o + Ns] = csub(v[b][0], x1);
      }
    }
    __syncthreads();
  }
}

// Complex DFT of length n held in buf[0..n), in place, by the ring's method:
// power of two directly, otherwise Bluestein's chirp convolution of length M
// (buf must hold M elements; filt = FFT_M of the conjugate chirp).  INV gives
// the unnormalised inverse DFT.  Synchronises the block on exit.
template <typename R, bool INV>
__device__ void ring_dft(cx_t<R>* buf, int n, int kind, int M, const cx_t<R>* __restrict__ filt,
                         const cx_t<R>* __restrict__ tw, int TN) {
  using C = cx_t<R>;
  if (kind == 1) {
    lds_fft<R, INV>(buf, n, tw, TN);
    return;
  }
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int l = tid; l < M; l += nth) {
    C v = cmake<C>(R(0), R(0));
    if (l < n) {
      v = buf[l];
      if (INV) v = cconj(v);
      v = cmul(v, chirp<R>(l, n));
    }
    buf[l] = v;
  }
  __syncthreads();
  lds_fft<R, false>(buf, M, tw, TN);
  for (int k = tid; k < M; k += nth) buf[k] = cmul(buf[k], filt[k]);
  __syncthreads();
  lds_fft<R, true>(buf, M, tw, TN);
  const R inv = R(1) / R(M);
  for (int k = tid; k < n; k += nth) {
    C v = cscale(cmul(buf[k], chirp<R>(k, n)), inv);
    if (INV) v = cconj(v);
    buf[k] = v;
  }
  __syncthreads();
}

template <typename T> __device__ __forceinline__ T uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace arkcos
