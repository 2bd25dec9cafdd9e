// Ring transforms: step (a) and step (d) of the hybrid method (paper
// Sect. 4.1, with the artifact suppression of Sect. 4.3).
//
// Step (a), per input ring j of N_j pixels at longitudes phi0_j + 2 pi k / N_j:
//   A_j(m) = sum_k x_jk exp(-2 pi i m k / N_j),  m = 0 .. N_j/2,
// then the phase shift to absolute longitude (eq. "fftrot") and the periodic
// extension past the ring's Nyquist mode:
//   A~_j(m) = A_j(m mod N_j) exp(-i m phi0_j),  m = 0 .. spec_len_j - 1,
// where A_j(N_j - r) = conj(A_j(r)).
//
// Step (d), per output ring i:
//   G_i(r) = sum_{m = r mod N_i} B_i(m) e^{i m phi0_i} + sum_{m = -r mod N_i, m > 0} conj(B_i(m) e^{i m phi0_i}),
//   y_ik   = sum_{r < N_i} G_i(r) exp(2 pi i r k / N_i)     (inverse real FFT),
// i.e. the reverse phase shift and the aliasing of super-Nyquist modes onto
// the ring's own modes.
//
// A real ring of even length N is transformed as a complex sequence of length
// N/2 (even samples in the real part, odd samples in the imaginary part) with
// the usual split; the complex DFT is a power-of-two LDS FFT or, for other
// lengths, Bluestein's chirp convolution through a power-of-two FFT.  Rings of
// up to 64 pixels use a plain DFT.  One block transforms one ring.
#include "arkcos_internal.h"
#include "device_common.h"

namespace arkcos {

template <typename R> struct RingArgs {
  const int32_t* n;
  const int64_t* start;
  const int32_t* phase_den;
  const int32_t* fft_kind;
  const int32_t* fft_m;
  const int64_t* bl_off;
  const int64_t* off;    // spectrum (step a) or B (step d) offsets
  const int32_t* len;
  const double* w;
  const cx_t<R>* bl;
  const cx_t<R>* tw;
  int32_t TN;
  int32_t nrings;
  int32_t adjoint;
  int32_t zero_pole_rings;
};

// exp(-i m phi0) for phi0 = pi / den (den = 0: no offset).
template <typename R> __device__ __forceinline__ cx_t<R> unshift(int m, int den) {
  using C = cx_t<R>;
  if (den == 0) return cmake<C>(R(1), R(0));
  int t = (int)((uint32_t)m % (2u * (uint32_t)den));
  return cconj(expipi<R>(t, den));
}

// Step (a) for ring j of one plan; x and spec are that plan's map and
// spectrum buffer.  buf: dynamic LDS, nyq: one shared slot.
template <typename R>
__device__ __forceinline__ void r2c_ring(const RingArgs<R>& a, const int j, const R* __restrict__ x,
                                         cx_t<R>* __restrict__ spec, cx_t<R>* buf, cx_t<R>& nyq) {
  using C = cx_t<R>;
  const int N = a.n[j], half = N / 2, kind = a.fft_kind[j];
  const int den = a.phase_den[j], len = a.len[j];
  C* out = spec + a.off[j];
  const int tid = threadIdx.x, nth = blockDim.x;
  if (a.zero_pole_rings && (j == 0 || j == a.nrings - 1)) {
    for (int m = tid; m < len; m += nth) out[m] = cmake<C>(R(0), R(0));
    return;
  }
  const R scale = a.adjoint ? R(1.0 / a.w[j]) : R(1);
  const R* xr = x + a.start[j];
  if (kind == FFT_DIRECT) {
    C* tab = buf + lds_elems(half);
    R* xs = reinterpret_cast<R*>(tab + N);
    for (int t = tid; t < N; t += nth) {
      tab[t] = cconj(expipi<R>(2 * t, N));  // exp(-2 pi i t / N)
      xs[t] = xr[t] * scale;
    }
    __syncthreads();
    for (int m = tid; m <= half; m += nth) {
      C acc = cmake<C>(R(0), R(0));
      int idx = 0;
      for (int k = 0; k < N; ++k) {
        acc = cadd(acc, cscale(tab[idx], xs[k]));
        idx += m;
        if (idx >= N) idx -= N;
      }
      if (m < half) buf[lidx(m)] = acc;
      else nyq = acc;
    }
    __syncthreads();
  } else {
    const int n = half;
    for (int l = tid; l < n; l += nth) buf[lidx(l)] = cmake<C>(xr[2 * l] * scale, xr[2 * l + 1] * scale);
    __syncthreads();
    if (kind == FFT_POW2)
      ring_dft<R, false>(buf, n, 1, n, nullptr, a.tw, a.TN);
    else
      ring_dft<R, false>(buf, n, 2, a.fft_m[j], a.bl + a.bl_off[j], a.tw, a.TN);
    // split Z into A(r) = E(r) + exp(-2 pi i r / N) O(r), in place, pairing r with n - r
    for (int r = tid; r <= n / 2; r += nth) {
      const int r2 = n - r;
      const C z1 = buf[lidx(r)], z2 = buf[lidx(r2 == n ? 0 : r2)];
      C e = cscale(cadd(z1, cconj(z2)), R(0.5));
      C o = cscale(csub(z1, cconj(z2)), R(0.5));
      C ar = cadd(e, cmul(cconj(expipi<R>(2 * r, N)), cmake<C>(o.y, -o.x)));
      C e2 = cscale(cadd(z2, cconj(z1)), R(0.5));
      C o2 = cscale(csub(z2, cconj(z1)), R(0.5));
      C ar2 = cadd(e2, cmul(cconj(expipi<R>(2 * r2, N)), cmake<C>(o2.y, -o2.x)));
      buf[lidx(r)] = ar;
      if (r2 == n) nyq = ar2;
      else if (r2 != r) buf[lidx(r2)] = ar2;
    }
    __syncthreads();
  }
  // periodic extension with the phase shift to absolute longitude
  for (int m = tid; m < len; m += nth) {
    const int r = m % N;
    C v;
    if (r == half) v = nyq;
    else if (r < half) v = buf[lidx(r)];
    else v = cconj(buf[lidx(N - r)]);
    out[m] = cmul(v, unshift<R>(m, den));
  }
}

// Step (d) for ring i of one plan.
template <typename R>
__device__ __forceinline__ void c2r_ring(const RingArgs<R>& a, const int i, const cx_t<R>* __restrict__ bin,
                                         R* __restrict__ y, cx_t<R>* buf, cx_t<R>& nyq) {
  using C = cx_t<R>;
  const int N = a.n[i], half = N / 2, kind = a.fft_kind[i];
  const int den = a.phase_den[i], len = a.len[i];
  const C* b = bin + a.off[i];
  const int tid = threadIdx.x, nth = blockDim.x;
  const R scale = a.adjoint ? R(a.w[i]) : R(1);
  // fold: reverse phase shift and aliasing onto m mod N
  for (int r = tid; r <= half; r += nth) {
    C g = cmake<C>(R(0), R(0));
    for (int m = r; m < len; m += N) g = cadd(g, cmul(b[m], cconj(unshift<R>(m, den))));
    for (int m = (r == 0 ? N : N - r); m < len; m += N)
      g = cadd(g, cconj(cmul(b[m], cconj(unshift<R>(m, den)))));
    g = cscale(g, scale);
    if (r < half) buf[lidx(r)] = g;
    else nyq = g;
  }
  __syncthreads();
  R* yr = y + a.start[i];
  if (kind == FFT_DIRECT) {
    C* tab = buf + lds_elems(half);
    for (int t = tid; t < N; t += nth) tab[t] = expipi<R>(2 * t, N);  // exp(+2 pi i t / N)
    __syncthreads();
    const C g0 = buf[lidx(0)];
    for (int k = tid; k < N; k += nth) {
      R acc = g0.x + ((k & 1) ? -nyq.x : nyq.x);
      int idx = k;
      for (int r = 1; r < half; ++r) {
        const C t = tab[idx], g = buf[lidx(r)];
        acc += R(2) * (g.x * t.x - g.y * t.y);
        idx += k;
        if (idx >= N) idx -= N;
      }
      yr[k] = acc;
    }
    return;
  }
  const int n = half;
  // Z(r) = E(r) + i O(r), E(r) = G(r) + conj(G(n-r)), O(r) = e^{2 pi i r/N} (G(r) - conj(G(n-r)))
  for (int r = tid; r <= n / 2; r += nth) {
    const int r2 = n - r;
    const C g1 = buf[lidx(r)], g2 = r2 == n ? nyq : buf[lidx(r2)];
    const C e1 = cadd(g1, cconj(g2));
    const C o1 = cmul(expipi<R>(2 * r, N), csub(g1, cconj(g2)));
    buf[lidx(r)] = cadd(e1, cmake<C>(-o1.y, o1.x));
    if (r2 < n && r2 != r) {
      const C e2 = cadd(g2, cconj(g1));
      const C o2 = cmul(expipi<R>(2 * r2, N), csub(g2, cconj(g1)));
      buf[lidx(r2)] = cadd(e2, cmake<C>(-o2.y, o2.x));
    }
  }
  __syncthreads();
  if (kind == FFT_POW2)
    ring_dft<R, true>(buf, n, 1, n, nullptr, a.tw, a.TN);
  else
    ring_dft<R, true>(buf, n, 2, a.fft_m[i], a.bl + a.bl_off[i], a.tw, a.TN);
  for (int l = tid; l < n; l += nth) {
    const C z = buf[lidx(l)];
    yr[2 * l] = z.x;
    yr[2 * l + 1] = z.y;
  }
}


template <typename R>
__global__ void __launch_bounds__(kBlock) r2c_kernel(RingArgs<R> a, const int32_t* __restrict__ list,
                                                     const R* __restrict__ x, cx_t<R>* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx_t<R> nyq;  // A(N/2), kept outside the padded buffer
  r2c_ring<R>(a, list[blockIdx.x], x, spec, reinterpret_cast<cx_t<R>*>(smem), nyq);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) c2r_kernel(RingArgs<R> a, const int32_t* __restrict__ list,
                                                     const cx_t<R>* __restrict__ bin, R* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx_t<R> nyq;  // G(N/2)
  c2r_ring<R>(a, list[blockIdx.x], bin, y, reinterpret_cast<cx_t<R>*>(smem), nyq);
}

// Batched forms: entry (map, ring); per-map arguments, maps and workspace
// offsets in device arrays.
template <typename R>
__global__ void __launch_bounds__(kBlock) r2c_batch_kernel(const RingArgs<R>* __restrict__ args,
                                                           const int2* __restrict__ entries,
                                                           const R* const* __restrict__ xs,
                                                           cx_t<R>* __restrict__ ws, const int64_t* __restrict__ base) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx_t<R> nyq;
  const int2 e = entries[blockIdx.x];
  const RingArgs<R> a = args[e.x];
  r2c_ring<R>(a, e.y, xs[e.x], ws + base[e.x], reinterpret_cast<cx_t<R>*>(smem), nyq);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) c2r_batch_kernel(const RingArgs<R>* __restrict__ args,
                                                           const int2* __restrict__ entries,
                                                           const cx_t<R>* __restrict__ ws,
                                                           const int64_t* __restrict__ base, R* const* __restrict__ ys) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx_t<R> nyq;
  const int2 e = entries[blockIdx.x];
  const RingArgs<R> a = args[e.x];
  c2r_ring<R>(a, e.y, ws + base[e.x], ys[e.x], reinterpret_cast<cx_t<R>*>(smem), nyq);
}

template <typename R> RingArgs<R> ring_args(arkcos_plan_s* P, bool out_side, int adjoint,
                                                   int zero_pole) {
  RingArgs<R> a{};
  a.n = P->rt.n;
  a.start = P->rt.start;
  a.phase_den = P->rt.phase_den;
  a.fft_kind = P->rt.fft_kind;
  a.fft_m = P->rt.fft_m;
  a.bl_off = P->rt.bl_off;
  a.off = out_side ? P->rt.out_off : P->rt.spec_off;
  a.len = out_side ? P->rt.out_len : P->rt.spec_len;
  a.w = P->rt.w;
  a.bl = (const cx_t<R>*)P->d_bl;
  a.tw = (const cx_t<R>*)P->d_twiddle;
  a.TN = P->twiddle_n;
  a.nrings = (int32_t)P->nrings;
  a.adjoint = adjoint;
  a.zero_pole_rings = zero_pole;
  return a;
}

hipError_t configure_fft_kernels(arkcos_plan_s* P) {
  // dynamic LDS above 64 KiB (plus the static Nyquist slot) needs the attribute
  hipError_t e;
  if (P->dtype == ARKCOS_F32) {
    e = hipFuncSetAttribute((const void*)r2c_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, P->max_fft_lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)c2r_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, P->max_fft_lds);
  } else {
    e = hipFuncSetAttribute((const void*)r2c_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, P->max_fft_lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)c2r_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, P->max_fft_lds);
  }
  return e;
}

hipError_t launch_r2c(arkcos_plan_s* P, const void* x, void* spec, int32_t adjoint,
                      int32_t zero_pole_rings, hipStream_t s) {
  for (const FftClass& c : P->fft_classes) {
    if (P->dtype == ARKCOS_F32)
      r2c_kernel<float><<<(unsigned)c.count, kBlock, c.lds, s>>>(
          ring_args<float>(P, false, adjoint, zero_pole_rings), c.d_rings, (const float*)x, (float2*)spec);
    else
      r2c_kernel<double><<<(unsigned)c.count, kBlock, c.lds, s>>>(
          ring_args<double>(P, false, adjoint, zero_pole_rings), c.d_rings, (const double*)x, (double2*)spec);
  }
  return hipGetLastError();
}

size_t ring_args_size() { return sizeof(RingArgs<float>); }

void fill_ring_args(arkcos_plan_s* P, bool out_side, int32_t adjoint, int32_t zero_pole, void* out) {
  if (P->dtype == ARKCOS_F32)
    *reinterpret_cast<RingArgs<float>*>(out) = ring_args<float>(P, out_side, adjoint, zero_pole);
  else
    *reinterpret_cast<RingArgs<double>*>(out) = ring_args<double>(P, out_side, adjoint, zero_pole);
}

// Batched ring transforms: forward (R2C of maps[m] into ws + base[m]) or
// inverse (C2R of ws + base[m] into maps[m]).
hipError_t launch_ring_batch(arkcos_dtype_t dt, bool inverse, const void* args, const void* entries, int32_t count,
                             int32_t lds, const void* maps, void* ws, const int64_t* base, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipError_t e;
  if (dt == ARKCOS_F32) {
    if (!inverse) {
      e = hipFuncSetAttribute((const void*)r2c_batch_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      r2c_batch_kernel<float><<<count, kBlock, lds, s>>>((const RingArgs<float>*)args, (const int2*)entries,
                                                         (const float* const*)maps, (float2*)ws, base);
    } else {
      e = hipFuncSetAttribute((const void*)c2r_batch_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      c2r_batch_kernel<float><<<count, kBlock, lds, s>>>((const RingArgs<float>*)args, (const int2*)entries,
                                                         (const float2*)ws, base, (float* const*)maps);
    }
  } else {
    if (!inverse) {
      e = hipFuncSetAttribute((const void*)r2c_batch_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      r2c_batch_kernel<double><<<count, kBlock, lds, s>>>((const RingArgs<double>*)args, (const int2*)entries,
                                                          (const double* const*)maps, (double2*)ws, base);
    } else {
      e = hipFuncSetAttribute((const void*)c2r_batch_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      c2r_batch_kernel<double><<<count, kBlock, lds, s>>>((const RingArgs<double>*)args, (const int2*)entries,
                                                          (const double2*)ws, base, (double* const*)maps);
    }
  }
  return hipGetLastError();
}

// Step (a) into the output-ring layout (lengths out_len): the extended
// spectra of a map on the output rings, for the kernel-profile gradient.
hipError_t launch_r2c_layout(arkcos_plan_s* P, const void* x, void* spec, bool out_layout, int32_t zero_pole,
                             hipStream_t s) {
  for (const FftClass& c : P->fft_classes) {
    if (P->dtype == ARKCOS_F32)
      r2c_kernel<float><<<(unsigned)c.count, kBlock, c.lds, s>>>(
          ring_args<float>(P, out_layout, 0, zero_pole), c.d_rings, (const float*)x, (float2*)spec);
    else
      r2c_kernel<double><<<(unsigned)c.count, kBlock, c.lds, s>>>(
          ring_args<double>(P, out_layout, 0, zero_pole), c.d_rings, (const double*)x, (double2*)spec);
  }
  return hipGetLastError();
}

hipError_t launch_c2r(arkcos_plan_s* P, const void* bout, void* y, int32_t adjoint, hipStream_t s) {
  for (const FftClass& c : P->fft_classes) {
    if (P->dtype == ARKCOS_F32)
      c2r_kernel<float><<<(unsigned)c.count, kBlock, c.lds, s>>>(
          ring_args<float>(P, true, adjoint, 0), c.d_rings, (const float2*)bout, (float*)y);
    else
      c2r_kernel<double><<<(unsigned)c.count, kBlock, c.lds, s>>>(
          ring_args<double>(P, true, adjoint, 0), c.d_rings, (const double2*)bout, (double*)y);
  }
  return hipGetLastError();
}

}  // namespace arkcos
