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
// the usual split; the complex DFT is a power-of-two LDS FFT, a mixed-radix
// one (radices 2-16, 3, 5, 7) for lengths with no other prime factors, or,
// for the rest, Bluestein's chirp convolution through a power-of-two FFT.
// Rings of up to 64 pixels use a plain DFT.  One block transforms one ring.
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

// Every ring offset in longitude has phi0 = pi / N (HEALPix polar rings and
// every other equatorial ring), so the phase factors of one ring are powers
// of w = exp(-i pi / N).  With w_r = w^r:
//   A~(m + N) = s A~(m),  A~(N - r) = s conj(A~(r)),  s = -1 (offset), +1,
// so a ring needs w_r only for r <= N/2, and the split of the half-length
// complex FFT needs w_r^2 = exp(-2 pi i r / N).  Power-of-two rings read w_r
// from the twiddle table (TN a multiple of 2N), Bluestein rings from the
// table stored after their filter (ph), the short rings compute it.
template <typename R>
__device__ __forceinline__ cx_t<R> half_twiddle(int r, int N, int kind, const cx_t<R>* __restrict__ ph,
                                                const cx_t<R>* __restrict__ tw, int TN) {
  if (kind == FFT_POW2) return tw[r * (TN / (2 * N))];
  if (kind == FFT_BLUESTEIN) return ph[r];
  return cconj(expipi<R>(r, N));
}

// The half-angle phase table of a Bluestein ring: after its filter (M values)
// and chirp (n values).
template <typename R>
__device__ __forceinline__ const cx_t<R>* phase_table(const RingArgs<R>& a, int ring, int kind, int n) {
  return kind == FFT_BLUESTEIN ? a.bl + a.bl_off[ring] + a.fft_m[ring] + n : nullptr;
}

// (r, n - r) pairs per thread per batch of loads
template <typename R> struct PairBatch { static constexpr int value = sizeof(R) == 4 ? 4 : 2; };

// Step (a) for ring j of one plan; x and spec are that plan's map and
// spectrum buffer.  buf: dynamic LDS (A(n) is kept in the slot after the n
// points).
template <typename R, int NT, int MF>
__device__ __forceinline__ void r2c_ring(const RingArgs<R>& a, const int j, const R* __restrict__ x,
                                         cx_t<R>* __restrict__ spec, cx_t<R>* buf) {
  using C = cx_t<R>;
  constexpr int EPT = kFftCap<NT> / NT;
  const int N = a.n[j], n = N / 2, kind = a.fft_kind[j];
  const bool shifted = a.phase_den[j] != 0;
  const int len = a.len[j];
  C* out = spec + a.off[j];
  const int tid = threadIdx.x;
  if (a.zero_pole_rings && (j == 0 || j == a.nrings - 1)) {
    for (int m = tid; m < len; m += NT) out[m] = cmake<C>(R(0), R(0));
    return;
  }
  const R scale = a.adjoint ? R(1.0 / a.w[j]) : R(1);
  const R* xr = x + a.start[j];
  const C* ph = phase_table(a, j, kind, n);
  if (kind == FFT_DIRECT) {
    C* tab = buf + lds_elems(n);
    R* xs = reinterpret_cast<R*>(tab + N);
    for (int t = tid; t < N; t += NT) {
      tab[t] = cconj(expipi<R>(2 * t, N));  // exp(-2 pi i t / N)
      xs[t] = xr[t] * scale;
    }
    __syncthreads();
    for (int m = tid; m <= n; m += NT) {
      C acc = cmake<C>(R(0), R(0));
      int idx = 0;
      for (int k = 0; k < N; ++k) {
        acc = cadd(acc, cscale(tab[idx], xs[k]));
        idx += m;
        if (idx >= N) idx -= N;
      }
      if (shifted) acc = cmul(acc, half_twiddle<R>(m, N, FFT_DIRECT, ph, a.tw, a.TN));
      buf[lidx(m)] = acc;  // A(n) in the slot after the n points
    }
    __syncthreads();
  } else {
    // the ring as n complex samples (x_2l, x_2l+1), all loads issued at
    // once; z[e] is sample tid + e NT.  The compile-time transforms take
    // them from registers, the others from LDS.
    const int M = a.fft_m[j];
    const cx_t<R>* xc = reinterpret_cast<const cx_t<R>*>(xr);
    C z[EPT];
    if constexpr (MF > 0) {
      auto load = [&](int e0, int e1) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int l = tid + e * NT;
          if (e >= e0 && e < e1) z[e] = l < n ? cscale(xc[l], scale) : cmake<C>(R(0), R(0));
        }
      };
      if (kind == FFT_POW2) {  // n == MF
        load(0, EPT);
        lds_fft_ct<R, false, NT, (MF > 0 ? MF : 16 * NT), false, false, true, false>(buf, a.tw, a.TN, z);
      } else {  // Bluestein, M == MF >= 2 n
        load(0, EPT / 2);
        bluestein_ct<R, false, NT, (MF > 0 ? MF : 16 * NT), true, false>(buf, n, a.bl + a.bl_off[j], a.tw, a.TN,
                                                                            z);
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int l = tid + e * NT;
        if (l < n) z[e] = xc[l];
      }
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int l = tid + e * NT;
        if (l < n) buf[lidx(l)] = cscale(z[e], scale);
      }
      __syncthreads();
      if constexpr (MF < 0) mixed_fft<R, false, NT>(buf, n);  // the mixed-radix classes hold only FFT_MIXED rings
      else if (kind == FFT_POW2) lds_fft<R, false, NT>(buf, n, a.tw, a.TN);
      else bluestein<R, false, NT>(buf, n, M, a.bl + a.bl_off[j], a.tw, a.TN);
    }
    constexpr int kPairBatch = PairBatch<R>::value;
    // A~(k), 0 <= k <= n, to every mode of the periodic extension:
    // A~(qN + k) = s^q A~(k) and, for 0 < k < n, A~(qN + N - k) = s^(q+1) conj(A~(k))
    auto emit = [&](int k, C v) {
      for (int m = k, q = 0; m < len; m += N, ++q) out[m] = (shifted && (q & 1)) ? cscale(v, R(-1)) : v;
      if (k > 0 && k < n) {
        const C vc = cconj(v);
        for (int m = N - k, q = 1; m < len; m += N, ++q) out[m] = (shifted && (q & 1)) ? cscale(vc, R(-1)) : vc;
      }
    };
    // split Z into A(r) = E(r) - i exp(-2 pi i r / N) O(r) for the pair
    // (r, n - r), then the phase shift A~(r) = A(r) w_r, w_{n-r} = -i conj(w_r),
    // and the results straight to the spectrum
    for (int base = 0; base <= n / 2; base += NT * kPairBatch) {
      C wr[kPairBatch];
#pragma unroll
      for (int u = 0; u < kPairBatch; ++u) {
        const int r = base + tid + u * NT;
        if (r <= n / 2) wr[u] = half_twiddle<R>(r, N, kind, ph, a.tw, a.TN);
      }
#pragma unroll
      for (int u = 0; u < kPairBatch; ++u) {
        const int r = base + tid + u * NT;
        if (r <= n / 2) {
          const int r2 = n - r;
          const C z1 = buf[lidx(r)], z2 = buf[lidx(r2 == n ? 0 : r2)];
          const C t = cmul(wr[u], wr[u]);                 // exp(-2 pi i r / N)
          const C t2 = cmake<C>(-t.x, t.y);               // exp(-2 pi i (n - r) / N) = -conj(t)
          const C e1 = cscale(cadd(z1, cconj(z2)), R(0.5)), o1 = cscale(csub(z1, cconj(z2)), R(0.5));
          const C e2 = cscale(cadd(z2, cconj(z1)), R(0.5)), o2 = cscale(csub(z2, cconj(z1)), R(0.5));
          C a1 = cadd(e1, cmul(t, cmake<C>(o1.y, -o1.x)));
          C a2 = cadd(e2, cmul(t2, cmake<C>(o2.y, -o2.x)));
          if (shifted) {
            a1 = cmul(a1, wr[u]);
            const C w2 = cmake<C>(-wr[u].y, -wr[u].x);    // -i conj(w_r)
            a2 = cmul(a2, w2);
          }
          emit(r, a1);
          if (r2 != r) emit(r2, a2);  // r = 0: A(n)
        }
      }
    }
    return;
  }
  // (short rings) periodic extension: A~(qN + r) = s^q A~(r),
  // A~(N - r) = s conj(A~(r)), m = q N + r advanced by NT per step
  int q = tid / N, r = tid - q * N;
  const int dq = NT / N, dr = NT - dq * N;
  for (int m = tid; m < len; m += NT) {
    const bool up = r > n;
    const C c = buf[lidx(up ? N - r : r)];
    const R sg = (shifted && ((q + (up ? 1 : 0)) & 1)) ? R(-1) : R(1);
    out[m] = cmake<C>(sg * c.x, (up ? -sg : sg) * c.y);
    r += dr;
    q += dq;
    if (r >= N) {
      r -= N;
      ++q;
    }
  }
}

// Step (d) for ring i of one plan.  With P(r) = sum_q s^q B(qN + r) the
// fold onto the ring's own modes is
//   G(r) = conj(w_r) (P(r) - conj(P(N - r)))   (offset rings),
//   G(r) = P(r) + conj(P(N - r))               (others),
// for 0 <= r <= N/2 (P(N) collects the modes qN, q >= 1).
template <typename R, int NT, int MF>
__device__ __forceinline__ void c2r_ring(const RingArgs<R>& a, const int i, const cx_t<R>* __restrict__ bin,
                                         R* __restrict__ y, cx_t<R>* buf, cx_t<R>& nyq) {
  using C = cx_t<R>;
  constexpr int EPT = kFftCap<NT> / NT;
  const int N = a.n[i], n = N / 2, kind = a.fft_kind[i];
  const bool shifted = a.phase_den[i] != 0;
  const int len = a.len[i];
  const C* b = bin + a.off[i];
  const int tid = threadIdx.x;
  const R scale = a.adjoint ? R(a.w[i]) : R(1);
  const C* ph = phase_table(a, i, kind, n);
  const bool direct = kind == FFT_DIRECT;
  constexpr int kPairBatch = PairBatch<R>::value;
  const int nq = (len + N - 1) / N;
  // the fold's results for the pair (r, n - r), from pp = P at r, N - r,
  // n - r and n + r: G(r), G(n - r), then the split for the half-length FFT
  auto finish = [&](int r, const C (&pp)[4]) {
    const int r2 = n - r;
    const C w = half_twiddle<R>(r, N, kind, ph, a.tw, a.TN);
    C g1, g2;
    if (shifted) {
      g1 = cmul(cconj(w), csub(pp[0], cconj(pp[1])));
      g2 = cmul(cmake<C>(-w.y, w.x), csub(pp[2], cconj(pp[3])));   // conj(w_{n-r}) = i w_r
    } else {
      g1 = cadd(pp[0], cconj(pp[1]));
      g2 = cadd(pp[2], cconj(pp[3]));
    }
    g1 = cscale(g1, scale);
    g2 = cscale(g2, scale);
    if (direct) {
      buf[lidx(r)] = g1;
      if (r2 == n) nyq = g2;
      else if (r2 != r) buf[lidx(r2)] = g2;
      return;
    }
    // Z(r) = E(r) + i O(r), E(r) = G(r) + conj(G(n-r)), O(r) = exp(2 pi i r/N) (G(r) - conj(G(n-r)))
    const C t = cconj(cmul(w, w));                      // exp(2 pi i r / N)
    const C t2 = cmake<C>(-t.x, t.y);                   // exp(2 pi i (n - r) / N)
    const C e1 = cadd(g1, cconj(g2)), o1 = cmul(t, csub(g1, cconj(g2)));
    buf[lidx(r)] = cadd(e1, cmake<C>(-o1.y, o1.x));
    if (r2 < n && r2 != r) {
      const C e2 = cadd(g2, cconj(g1)), o2 = cmul(t2, csub(g2, cconj(g1)));
      buf[lidx(r2)] = cadd(e2, cmake<C>(-o2.y, o2.x));
    }
  };
  const int npr = n / 2 + 1;  // pairs (r, n - r), r <= n / 2
  if (NT >= kFoldThreads && 2 * npr <= kFoldThreads) {
    // a short ring: the periods q are shared out over G groups of threads
    // (thread t: pair t mod npr, periods q = t / npr + k G), the groups'
    // partial sums are added in group order through LDS
    const int G = kFoldThreads / npr;
    const int u = tid % npr, grp = tid / npr;
    C pp[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pp[c] = cmake<C>(R(0), R(0));
    if (grp < G) {
      for (int q = grp; q < nq; q += G) {
        const R sg = (shifted && (q & 1)) ? R(-1) : R(1);
        const int m0 = q * N;
        const int ms[4] = {m0 + u, m0 + N - u, m0 + n - u, m0 + n + u};
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (ms[c] < len) pp[c] = cadd(pp[c], cscale(b[ms[c]], sg));
      }
    }
    C* scr = buf;  // G npr 4 <= 4 kFoldThreads values: the ring's LDS holds them
    if (grp < G) {
#pragma unroll
      for (int c = 0; c < 4; ++c) scr[(grp * npr + u) * 4 + c] = pp[c];
    }
    __syncthreads();
    C fin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) fin[c] = cmake<C>(R(0), R(0));
    if (tid < npr) {
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) fin[c] = cadd(fin[c], scr[(k * npr + tid) * 4 + c]);
    }
    __syncthreads();
    if (tid < npr) finish(tid, fin);
  } else {
    for (int base = 0; base <= n / 2; base += NT * kPairBatch) {
      // P at r, N - r, n - r and n + r for each pair (r, n - r)
      C p[kPairBatch][4];
#pragma unroll
      for (int u = 0; u < kPairBatch; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) p[u][c] = cmake<C>(R(0), R(0));
      for (int q = 0; q < nq; ++q) {
        const R sg = (shifted && (q & 1)) ? R(-1) : R(1);
        const int m0 = q * N;
        C v[kPairBatch][4];
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
          const int r = base + tid + u * NT;
          const int ms[4] = {m0 + r, m0 + N - r, m0 + n - r, m0 + n + r};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            v[u][c] = cmake<C>(R(0), R(0));
            if (r <= n / 2 && ms[c] < len) v[u][c] = b[ms[c]];
          }
        }
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) p[u][c] = cadd(p[u][c], cscale(v[u][c], sg));
      }
#pragma unroll
      for (int u = 0; u < kPairBatch; ++u) {
        const int r = base + tid + u * NT;
        if (r <= n / 2) finish(r, p[u]);
      }
    }
  }
  __syncthreads();
  R* yr = y + a.start[i];
  if (direct) {
    C* tab = buf + lds_elems(n);
    for (int t = tid; t < N; t += NT) tab[t] = expipi<R>(2 * t, N);  // exp(+2 pi i t / N)
    __syncthreads();
    const C g0 = buf[lidx(0)];
    for (int k = tid; k < N; k += NT) {
      R acc = g0.x + ((k & 1) ? -nyq.x : nyq.x);
      int idx = k;
      for (int r = 1; r < n; ++r) {
        const C t = tab[idx], g = buf[lidx(r)];
        acc += R(2) * (g.x * t.x - g.y * t.y);
        idx += k;
        if (idx >= N) idx -= N;
      }
      yr[k] = acc;
    }
    return;
  }
  const int M = a.fft_m[i];
  cx_t<R>* yc = reinterpret_cast<cx_t<R>*>(yr);
  if constexpr (MF > 0) {
    // the compile-time transforms leave point tid + e NT in z[e]
    C z[EPT];
    if (kind == FFT_POW2) {  // n == MF
      lds_fft_ct<R, true, NT, (MF > 0 ? MF : 16 * NT), false, false, false, true>(buf, a.tw, a.TN, z);
#pragma unroll
      for (int e = 0; e < EPT; ++e) yc[tid + e * NT] = z[e];
    } else {  // Bluestein, M == MF >= 2 n
      bluestein_ct<R, true, NT, (MF > 0 ? MF : 16 * NT), false, true>(buf, n, a.bl + a.bl_off[i], a.tw, a.TN, z);
#pragma unroll
      for (int e = 0; e < EPT / 2; ++e) {
        const int l = tid + e * NT;
        if (l < n) yc[l] = z[e];
      }
    }
    return;
  }
  if constexpr (MF < 0) mixed_fft<R, true, NT>(buf, n);
  else if (kind == FFT_POW2) lds_fft<R, true, NT>(buf, n, a.tw, a.TN);
  else bluestein<R, true, NT>(buf, n, M, a.bl + a.bl_off[i], a.tw, a.TN);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = tid + e * NT;
    if (l < n) yc[l] = buf[lidx(l)];
  }
}


// Minimum waves per SIMD the ring kernels are compiled for: four blocks of
// 256 threads (or two of 512) per CU in FP32, whose LDS also fits four.
template <typename R> struct FftWaves { static constexpr int value = sizeof(R) == 4 ? 4 : 2; };

template <typename R, int NT, int MF>
__global__ void __launch_bounds__(NT, FftWaves<R>::value) r2c_kernel(RingArgs<R> a, const int32_t* __restrict__ list,
                                                 const R* __restrict__ x, cx_t<R>* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char smem[];
  r2c_ring<R, NT, MF>(a, list[blockIdx.x], x, spec, reinterpret_cast<cx_t<R>*>(smem));
}

template <typename R, int NT, int MF>
__global__ void __launch_bounds__(NT, FftWaves<R>::value) c2r_kernel(RingArgs<R> a, const int32_t* __restrict__ list,
                                                 const cx_t<R>* __restrict__ bin, R* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx_t<R> nyq;  // G(N/2)
  c2r_ring<R, NT, MF>(a, list[blockIdx.x], bin, y, reinterpret_cast<cx_t<R>*>(smem), nyq);
}

// Batched forms: entry (map, ring); per-map arguments, maps and workspace
// offsets in device arrays.
template <typename R, int NT, int MF>
__global__ void __launch_bounds__(NT, FftWaves<R>::value) r2c_batch_kernel(const RingArgs<R>* __restrict__ args,
                                                       const int2* __restrict__ entries,
                                                       const R* const* __restrict__ xs,
                                                       cx_t<R>* __restrict__ ws, const int64_t* __restrict__ base) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int2 e = entries[blockIdx.x];
  const RingArgs<R> a = args[e.x];
  r2c_ring<R, NT, MF>(a, e.y, xs[e.x], ws + base[e.x], reinterpret_cast<cx_t<R>*>(smem));
}

template <typename R, int NT, int MF>
__global__ void __launch_bounds__(NT, FftWaves<R>::value) c2r_batch_kernel(const RingArgs<R>* __restrict__ args,
                                                       const int2* __restrict__ entries,
                                                       const cx_t<R>* __restrict__ ws,
                                                       const int64_t* __restrict__ base, R* const* __restrict__ ys) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx_t<R> nyq;
  const int2 e = entries[blockIdx.x];
  const RingArgs<R> a = args[e.x];
  c2r_ring<R, NT, MF>(a, e.y, ws + base[e.x], ys[e.x], reinterpret_cast<cx_t<R>*>(smem), nyq);
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

// Threads per block for a ring class whose longest FFT has length fft_len:
// at least 256, and enough for 16 points per thread (FP32 up to 16384 points
// in 1024 threads, FP64 up to 8192 in 512: 135 KB of LDS either way).
int fft_threads(arkcos_dtype_t dt, int32_t fft_len) {
  (void)dt;
  int nt = 256;
  while (16 * nt < fft_len) nt *= 2;
  return nt;
}

int32_t ct_fft_length(arkcos_dtype_t dt, int32_t fft_len, int64_t rings) {
  if (dt != ARKCOS_F32) return 0;
  if (fft_len == 4096 || fft_len == 8192) return fft_len;
  if ((fft_len == 1024 || fft_len == 2048) && rings >= kCtMinRings) return fft_len;
  return 0;
}

template <typename K> static hipError_t allow_lds(K* k, int32_t bytes) {
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t configure_fft_kernels(arkcos_plan_s* P) {
  // dynamic LDS above 64 KiB (plus the static Nyquist slot) needs the attribute
  hipError_t e = hipSuccess;
  const int32_t b = P->max_fft_lds;
  if (P->dtype == ARKCOS_F32) {
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 256, 0>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 512, 0>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 256, 4096>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 512, 8192>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 128, 2048>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 64, 1024>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 256, 0>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 512, 0>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 256, 4096>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 512, 8192>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 128, 2048>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 64, 1024>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 1024, 0>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 1024, 0>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 256, -1>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 512, -1>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<float, 1024, -1>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 256, -1>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 512, -1>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<float, 1024, -1>, b);
  } else {
    if (e == hipSuccess) e = allow_lds(r2c_kernel<double, 256, 0>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<double, 256, 0>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<double, 512, 0>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<double, 512, 0>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<double, 256, -1>, b);
    if (e == hipSuccess) e = allow_lds(r2c_kernel<double, 512, -1>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<double, 256, -1>, b);
    if (e == hipSuccess) e = allow_lds(c2r_kernel<double, 512, -1>, b);
  }
  return e;
}

// The launches of one class: a kernel compiled for the class's FFT length
// when every ring of the class has the same one (a compile-time length).
template <typename R>
static void r2c_class(const FftClass& c, const RingArgs<R>& a, const void* x, void* spec, hipStream_t s) {
  const R* xi = (const R*)x;
  cx_t<R>* so = (cx_t<R>*)spec;
  if (c.mf < 0) {  // mixed-radix rings
    if constexpr (sizeof(R) == 4) {
      if (c.threads == 1024) {
        r2c_kernel<R, 1024, -1><<<(unsigned)c.count, 1024, c.lds, s>>>(a, c.d_rings, xi, so);
        return;
      }
    }
    if (c.threads == 512)
      r2c_kernel<R, 512, -1><<<(unsigned)c.count, 512, c.lds, s>>>(a, c.d_rings, xi, so);
    else
      r2c_kernel<R, 256, -1><<<(unsigned)c.count, 256, c.lds, s>>>(a, c.d_rings, xi, so);
    return;
  }
  if constexpr (sizeof(R) == 4) {
    if (c.threads == 512 && c.mf == 8192) {
      r2c_kernel<R, 512, 8192><<<(unsigned)c.count, 512, c.lds, s>>>(a, c.d_rings, xi, so);
      return;
    }
    if (c.threads == 256 && c.mf == 4096) {
      r2c_kernel<R, 256, 4096><<<(unsigned)c.count, 256, c.lds, s>>>(a, c.d_rings, xi, so);
      return;
    }
    if (c.threads == 128 && c.mf == 2048) {
      r2c_kernel<R, 128, 2048><<<(unsigned)c.count, 128, c.lds, s>>>(a, c.d_rings, xi, so);
      return;
    }
    if (c.threads == 64 && c.mf == 1024) {
      r2c_kernel<R, 64, 1024><<<(unsigned)c.count, 64, c.lds, s>>>(a, c.d_rings, xi, so);
      return;
    }
    if (c.threads == 1024) {
      r2c_kernel<R, 1024, 0><<<(unsigned)c.count, 1024, c.lds, s>>>(a, c.d_rings, xi, so);
      return;
    }
  }
  if (c.threads == 512) {
    r2c_kernel<R, 512, 0><<<(unsigned)c.count, 512, c.lds, s>>>(a, c.d_rings, xi, so);
    return;
  }
  r2c_kernel<R, 256, 0><<<(unsigned)c.count, 256, c.lds, s>>>(a, c.d_rings, xi, so);
}

template <typename R>
static void c2r_class(const FftClass& c, const RingArgs<R>& a, const void* b, void* y, hipStream_t s) {
  const cx_t<R>* bi = (const cx_t<R>*)b;
  R* yo = (R*)y;
  if (c.mf < 0) {  // mixed-radix rings
    if constexpr (sizeof(R) == 4) {
      if (c.threads == 1024) {
        c2r_kernel<R, 1024, -1><<<(unsigned)c.count, 1024, c.lds, s>>>(a, c.d_rings, bi, yo);
        return;
      }
    }
    if (c.threads == 512)
      c2r_kernel<R, 512, -1><<<(unsigned)c.count, 512, c.lds, s>>>(a, c.d_rings, bi, yo);
    else
      c2r_kernel<R, 256, -1><<<(unsigned)c.count, 256, c.lds, s>>>(a, c.d_rings, bi, yo);
    return;
  }
  if constexpr (sizeof(R) == 4) {
    if (c.threads == 512 && c.mf == 8192) {
      c2r_kernel<R, 512, 8192><<<(unsigned)c.count, 512, c.lds, s>>>(a, c.d_rings, bi, yo);
      return;
    }
    if (c.threads == 256 && c.mf == 4096) {
      c2r_kernel<R, 256, 4096><<<(unsigned)c.count, 256, c.lds, s>>>(a, c.d_rings, bi, yo);
      return;
    }
    if (c.threads == 128 && c.mf == 2048) {
      c2r_kernel<R, 128, 2048><<<(unsigned)c.count, 128, c.lds, s>>>(a, c.d_rings, bi, yo);
      return;
    }
    if (c.threads == 64 && c.mf == 1024) {
      c2r_kernel<R, 64, 1024><<<(unsigned)c.count, 64, c.lds, s>>>(a, c.d_rings, bi, yo);
      return;
    }
    if (c.threads == 1024) {
      c2r_kernel<R, 1024, 0><<<(unsigned)c.count, 1024, c.lds, s>>>(a, c.d_rings, bi, yo);
      return;
    }
  }
  if (c.threads == 512) {
    c2r_kernel<R, 512, 0><<<(unsigned)c.count, 512, c.lds, s>>>(a, c.d_rings, bi, yo);
    return;
  }
  c2r_kernel<R, 256, 0><<<(unsigned)c.count, 256, c.lds, s>>>(a, c.d_rings, bi, yo);
}

hipError_t launch_r2c(arkcos_plan_s* P, const void* x, void* spec, int32_t adjoint,
                      int32_t zero_pole_rings, hipStream_t s) {
  for (const FftClass& c : P->fft_classes) {
    if (P->dtype == ARKCOS_F32)
      r2c_class<float>(c, ring_args<float>(P, false, adjoint, zero_pole_rings), x, spec, s);
    else
      r2c_class<double>(c, ring_args<double>(P, false, adjoint, zero_pole_rings), x, spec, s);
  }
  return hipGetLastError();
}

size_t ring_args_size() { return sizeof(RingArgs<float>); }

void fill_ring_args(arkcos_plan_s* P, bool out_side, int32_t adjoint, int32_t zero_pole, void* out,
                    const int64_t* off, const int32_t* len) {
  if (P->dtype == ARKCOS_F32) {
    RingArgs<float> a = ring_args<float>(P, out_side, adjoint, zero_pole);
    if (off) a.off = off;
    if (len) a.len = len;
    *reinterpret_cast<RingArgs<float>*>(out) = a;
  } else {
    RingArgs<double> a = ring_args<double>(P, out_side, adjoint, zero_pole);
    if (off) a.off = off;
    if (len) a.len = len;
    *reinterpret_cast<RingArgs<double>*>(out) = a;
  }
}

// Batched ring transforms: forward (R2C of maps[m] into ws + base[m]) or
// inverse (C2R of ws + base[m] into maps[m]).
template <typename R, int NT, int MF>
static hipError_t ring_batch(bool inverse, const void* args, const void* entries, int32_t count, int32_t lds,
                             const void* maps, void* ws, const int64_t* base, hipStream_t s) {
  hipError_t e;
  if (!inverse) {
    e = allow_lds(r2c_batch_kernel<R, NT, MF>, lds);
    if (e != hipSuccess) return e;
    r2c_batch_kernel<R, NT, MF><<<count, NT, lds, s>>>((const RingArgs<R>*)args, (const int2*)entries,
                                                       (const R* const*)maps, (cx_t<R>*)ws, base);
  } else {
    e = allow_lds(c2r_batch_kernel<R, NT, MF>, lds);
    if (e != hipSuccess) return e;
    c2r_batch_kernel<R, NT, MF><<<count, NT, lds, s>>>((const RingArgs<R>*)args, (const int2*)entries,
                                                       (const cx_t<R>*)ws, base, (R* const*)maps);
  }
  return hipGetLastError();
}

hipError_t launch_ring_batch(arkcos_dtype_t dt, bool inverse, const void* args, const void* entries, int32_t count,
                             int32_t lds, int32_t threads, int32_t mf, const void* maps, void* ws,
                             const int64_t* base, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (mf < 0) {  // mixed-radix rings
    if (dt == ARKCOS_F32) {
      if (threads == 1024) return ring_batch<float, 1024, -1>(inverse, args, entries, count, lds, maps, ws, base, s);
      return threads == 512 ? ring_batch<float, 512, -1>(inverse, args, entries, count, lds, maps, ws, base, s)
                            : ring_batch<float, 256, -1>(inverse, args, entries, count, lds, maps, ws, base, s);
    }
    return threads == 512 ? ring_batch<double, 512, -1>(inverse, args, entries, count, lds, maps, ws, base, s)
                          : ring_batch<double, 256, -1>(inverse, args, entries, count, lds, maps, ws, base, s);
  }
  if (dt == ARKCOS_F32) {
    if (threads == 512 && mf == 8192)
      return ring_batch<float, 512, 8192>(inverse, args, entries, count, lds, maps, ws, base, s);
    if (threads == 256 && mf == 4096)
      return ring_batch<float, 256, 4096>(inverse, args, entries, count, lds, maps, ws, base, s);
    if (threads == 128 && mf == 2048)
      return ring_batch<float, 128, 2048>(inverse, args, entries, count, lds, maps, ws, base, s);
    if (threads == 64 && mf == 1024)
      return ring_batch<float, 64, 1024>(inverse, args, entries, count, lds, maps, ws, base, s);
    if (threads == 1024) return ring_batch<float, 1024, 0>(inverse, args, entries, count, lds, maps, ws, base, s);
    return threads == 512 ? ring_batch<float, 512, 0>(inverse, args, entries, count, lds, maps, ws, base, s)
                          : ring_batch<float, 256, 0>(inverse, args, entries, count, lds, maps, ws, base, s);
  }
  return threads == 512 ? ring_batch<double, 512, 0>(inverse, args, entries, count, lds, maps, ws, base, s)
                        : ring_batch<double, 256, 0>(inverse, args, entries, count, lds, maps, ws, base, s);
}

// Step (a) into the output-ring layout (lengths out_len): the extended
// spectra of a map on the output rings, for the kernel-profile gradient.
hipError_t launch_r2c_layout(arkcos_plan_s* P, const void* x, void* spec, bool out_layout, int32_t zero_pole,
                             hipStream_t s) {
  for (const FftClass& c : P->fft_classes) {
    if (P->dtype == ARKCOS_F32)
      r2c_class<float>(c, ring_args<float>(P, out_layout, 0, zero_pole), x, spec, s);
    else
      r2c_class<double>(c, ring_args<double>(P, out_layout, 0, zero_pole), x, spec, s);
  }
  return hipGetLastError();
}

hipError_t launch_c2r(arkcos_plan_s* P, const void* bout, void* y, int32_t adjoint, hipStream_t s) {
  for (const FftClass& c : P->fft_classes) {
    if (P->dtype == ARKCOS_F32)
      c2r_class<float>(c, ring_args<float>(P, true, adjoint, 0), bout, y, s);
    else
      c2r_class<double>(c, ring_args<double>(P, true, adjoint, 0), bout, y, s);
  }
  return hipGetLastError();
}

}  // namespace arkcos
