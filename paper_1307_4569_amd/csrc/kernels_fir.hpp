// FIR-window algorithm (Sec. 4: the weighted-overlap-add DGT for windows of
// short support, cost 8 L L_g / a + 4 N M log2 M; on a nonseparable lattice
// the multiwindow route of Table 1 with FIR separable transforms).  For a
// window supported on the L_g samples start, ..., start + L_g - 1 (mod L),
// eq. (DGT) reads, per time position n,
//     y_n(j) = f(l_j) conj(g(l_j - n a)) exp(-2 pi i l_j w(n) / M),
//              l_j = (n a + start + j) mod L, j in Z_{L_g},
//     c(m, n) = sum_k Y_n(k) exp(-2 pi i k m / M),  Y_n(k) = sum_{l_j = k mod M} y_n(j),
// with w(n) = (n lambda1 mod lambda2) / lambda2: the windowed samples are
// folded modulo M and one length-M DFT gives column n.  No intermediate
// array: the signal is read (each sample by about L_g / a time positions,
// from cache) and the coefficients written once.
//
// The adjoint f(l) = sum_n g(l - n a) exp(2 pi i l w(n) / M) y_n(l mod M),
// y_n = unnormalised inverse DFT of c(., n), runs as the inverse DFTs of the
// columns into Y[n][k] and a gather over the time positions whose window
// covers each sample.
#pragma once
#include "kernels.hpp"
#include "wave_fft.hpp"

namespace dgtns {

template <typename C> struct FirArgs {
  const void* x;
  long long xs;
  int real_in;
  int list;
  const void* xl[kListMax];
  C* c;
  long long cs;
  C* cl[kListMax];
  const C* gw;     // conj(g(start + j)), j in Z_{L_g}
  const C* ph;     // exp(-2 pi i e / (lambda2 M)), e in Z_{lambda2 M} (lambda2 > 1)
  const C* twm;    // length-M stage twiddles
  long long L, start;
  int a, M, Lg, lam1, lam2, N, R, Sm;
  FftSched fm;
  CoefLayout lay;  // coefficient layout (c, cs and cl follow it)
  int real_out;    // the adjoint writes real samples
  // floor((2^64 - 1) / m) for m = M, lambda2 and lambda2 M (Barrett)
  unsigned long long muM, muL2, muPM;
};

// Per-time-position constants of the folding: base = (n a + start) mod L
// (index of support sample 0), bm = base mod M, kn = n lambda1 mod lambda2
// and eb = (base kn) mod (lambda2 M), the phase index of sample 0.  Phase
// indices then advance without divisions: lambda2 M divides L, so the
// index (l kn) mod (lambda2 M) of sample l = base + j is eb + j kn reduced.
// n a + start < 2 L (n a <= L - a, start < L): one conditional subtraction;
// the other reductions are Barrett reductions with host reciprocals.  With n
// the same on every lane (one transform per wavefront) all of it runs on the
// scalar unit.
struct FirPos {
  long long base;
  int bm, kn, eb;
};

template <typename C>
__device__ __forceinline__ FirPos fir_pos(const FirArgs<C>& A, int n) {
  using U = unsigned long long;
  FirPos q;
  q.base = (long long)n * A.a + A.start;
  if (q.base >= A.L) q.base -= A.L;
  q.bm = int(mod_b(U(q.base), U(A.M), A.muM));
  q.kn = A.lam2 > 1 ? int(mod_b(U(n) * U(A.lam1), U(A.lam2), A.muL2)) : 0;
  const U PM = U(A.lam2) * U(A.M);
  q.eb = q.kn ? int(mod_b(mod_b(U(q.base), PM, A.muPM) * U(q.kn), PM, A.muPM)) : 0;
  return q;
}

// Windowed, modulated and folded bin k of time position n: the sum over the
// support samples j = jk + t M, jk = (k - base) mod M.
template <typename C>
__device__ __forceinline__ C fir_bin(const FirArgs<C>& A, const void* xsrc, long long xoff, const FirPos& q, int k) {
  const int M = A.M, PM = A.lam2 * A.M, step = M * q.kn;   // step < PM
  int jk = k - q.bm;
  if (jk < 0) jk += M;
  int e = q.eb + jk * q.kn;                                // jk kn < PM
  if (e >= PM) e -= PM;
  C acc = czero<C>();
  long long idx = q.base + jk;
  if (idx >= A.L) idx -= A.L;
  for (int j = jk; j < A.Lg; j += M) {
    C v = cmul(load_sig<C>(xsrc, A.real_in, xoff + idx), A.gw[j]);
    if (q.kn) v = cmul(v, A.ph[e]);
    acc = cadd(acc, v);
    idx += M;
    if (idx >= A.L) idx -= A.L;
    e += step;
    if (e >= PM) e -= PM;
  }
  return acc;
}

// fir_bin with at most NT samples per bin (L_g <= NT M), fully unrolled so
// that the loads of all bins of a lane are issued together.
template <int NT, typename C>
__device__ __forceinline__ C fir_bin_n(const FirArgs<C>& A, const void* xsrc, long long xoff, const FirPos& q,
                                       int k) {
  const int M = A.M, PM = A.lam2 * A.M, step = M * q.kn;
  int jk = k - q.bm;
  if (jk < 0) jk += M;
  int e = q.eb + jk * q.kn;
  if (e >= PM) e -= PM;
  long long idx = q.base + jk;
  if (idx >= A.L) idx -= A.L;
  C acc = czero<C>();
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = jk + t * M;
    if (j < A.Lg) {
      C v = cmul(load_sig<C>(xsrc, A.real_in, xoff + idx), A.gw[j]);
      if (q.kn) v = cmul(v, A.ph[e]);
      acc = cadd(acc, v);
    }
    idx += M;
    if (idx >= A.L) idx -= A.L;
    e += step;
    if (e >= PM) e -= PM;
  }
  return acc;
}

// ----------------------------------------------------------------------------
// Forward, power-of-two M = MI in [32, 1024]: one wave transform per time
// position; a work-group handles 8 TPW consecutive positions.
// grid (ceil(N / (8 TPW)), B), 512 threads.
// HS: streaming stores of the coefficients.
// ----------------------------------------------------------------------------
// NT: samples per bin (L_g <= NT M), 0 for any L_g.
template <typename C, int MI, bool HS, int NT>
__global__ void __launch_bounds__(kThreads) k_fir_fwd_w(FirArgs<C> A) {
  using I = WInfo<MI>;
  constexpr int E = I::E, T = I::T, TPW = I::TPW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  // the same n on every lane of a wavefront when TPW = 1
  const int n = (blockIdx.x * 8 + (TPW == 1 ? __builtin_amdgcn_readfirstlane(wave) : wave)) * TPW + tt;
  const FirPos q = fir_pos(A, n < A.N ? n : A.N - 1);
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if constexpr (NT > 0)
      v[e] = fir_bin_n<NT>(A, xsrc, xoff, q, l + T * e);
    else
      v[e] = fir_bin(A, xsrc, xoff, q, l + T * e);
  }
  WTw<C, MI> tw;
  tw.load(A.twm, l);
  C* ex = lds + (wave * TPW + tt) * WEx<C, MI>::EX;
  wave_fft<C, MI, false>(v, ex, l, tw);
  if (n < A.N) {
    int cnt, ee;
    C* row = (A.list ? pick(A.cl, int(bo)) : A.c + bo * A.cs) + coef_col(A.lay, n, &cnt, &ee);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (l + T * e < cnt) {
        if constexpr (HS)
          st_stream(row + l + T * e, v[e]);
        else
          row[l + T * e] = v[e];
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Forward, power-of-two M = MI, with the work-group's signal span and the
// window staged in LDS.  The P = 8 TPW positions of a work-group read the
// S = (P - 1) a + L_g samples from (n_first a + start) mod L on, so the span
// is loaded once, coalesced, and every wave folds from LDS.  The phase
// exp(-2 pi i (eb + j kn) / (lambda2 M)) of sample j = jk + t M of bin k
// splits into the bin factor exp(-2 pi i (eb + jk kn) / (lambda2 M)), applied
// once to the folded sum, and the tap factor exp(-2 pi i t kn / lambda2),
// the same for every bin of a transform.  The span and window alias the FFT
// exchange areas: a barrier separates the fold from the transforms.
// grid (ceil(N / (8 TPW)), B), 512 threads; LDS max(exchange, (S + L_g) C).
// ----------------------------------------------------------------------------
// FP32 with M = 1024: the half-size exchange (wave_fft_h, 36352 bytes of LDS
// for the eight wavefronts instead of 73216) and at most 80 VGPRs, so that
// three work-groups share a compute unit and one's loads overlap another's
// transforms (forward, whose staged span and window may need a little more
// LDS, and the inverse DFTs of the adjoint).
template <typename C, int MI> struct FirWs {
  static constexpr bool HALF = MI == 1024 && sizeof(C) == 8;
  static constexpr int EX = HALF ? WExH<C>::EX : WEx<C, MI>::EX;   // per transform
  static constexpr int WAVES_PER_EU = HALF ? 6 : 4;
};

template <typename C, int MI, bool HS, int NT>
__global__ void __launch_bounds__(kThreads, (FirWs<C, MI>::WAVES_PER_EU)) k_fir_fwd_ws(FirArgs<C> A) {
  using I = WInfo<MI>;
  using F = FirWs<C, MI>;
  constexpr int E = I::E, T = I::T, TPW = I::TPW, P = 8 * TPW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  const int nf = blockIdx.x * P, S = (P - 1) * A.a + A.Lg;
  // 1. span f((base0 + i) mod L), i < S, and window gw[j], j < L_g; each
  // thread issues U loads before it waits for the first
  {
    constexpr int U = 4;
    using T = decltype(C::x);
    long long base0 = (long long)nf * A.a + A.start;   // < 2 L
    if (base0 >= A.L) base0 -= A.L;
    C* span = lds;
    // spans that do not wrap (all but the last few of a signal): one
    // uniform base address and 32-bit lane offsets.  Indices beyond the span
    // load its last sample (not stored), so the U loads carry no branch.
    auto stage = [&](auto ld) {
      for (unsigned i0 = tid; i0 < unsigned(S); i0 += U * kThreads) {
        C v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const unsigned i = i0 + u * kThreads;
          v[u] = ld(i < unsigned(S) ? i : unsigned(S - 1));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (i0 + u * kThreads < unsigned(S)) span[i0 + u * kThreads] = v[u];
      }
    };
    if (base0 + S <= A.L) {
      if (A.real_in) {
        const T* xp = reinterpret_cast<const T*>(xsrc) + xoff + base0;
        stage([&](unsigned i) { return mk<C>(xp[i], T(0)); });
      } else {
        const C* xp = reinterpret_cast<const C*>(xsrc) + xoff + base0;
        stage([&](unsigned i) { return xp[i]; });
      }
    } else {
      stage([&](unsigned i) {
        long long idx = base0 + i;
        if (idx >= A.L) {
          idx -= A.L;
          if (idx >= A.L) idx %= A.L;   // spans longer than L (short signals)
        }
        return load_sig<C>(xsrc, A.real_in, xoff + idx);
      });
    }
    C* win = lds + S;
    for (unsigned j0 = tid; j0 < unsigned(A.Lg); j0 += U * kThreads) {
      C v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned j = j0 + u * kThreads;
        v[u] = A.gw[j < unsigned(A.Lg) ? j : unsigned(A.Lg - 1)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (j0 + u * kThreads < unsigned(A.Lg)) win[j0 + u * kThreads] = v[u];
    }
  }
  __syncthreads();
  // 2. fold: bin k = l + T e of position n
  // the same p on every lane of a wavefront when TPW = 1
  const int p = TPW == 1 ? __builtin_amdgcn_readfirstlane(wave) : wave * TPW + tt, n = nf + p;
  const FirPos q = fir_pos(A, n < A.N ? n : A.N - 1);
  const int M = A.M, PM = A.lam2 * A.M, tstep = M * q.kn;   // tap phase step, < PM
  const C* sp = lds + p * A.a;
  const C* win = lds + S;
  C v[E];
  if constexpr (NT > 0) {
    C wt[NT];
    wt[0] = mk<C>(1, 0);
    {
      int te = 0;
#pragma unroll
      for (int t = 1; t < NT; ++t) {
        te += tstep;
        if (te >= PM) te -= PM;
        wt[t] = q.kn ? A.ph[te] : mk<C>(1, 0);
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jk = (l + T * e - q.bm) & (MI - 1);
      C acc = jk < A.Lg ? cmul(sp[jk], win[jk]) : czero<C>();
#pragma unroll
      for (int t = 1; t < NT; ++t) {
        const int j = jk + t * MI;
        if (j < A.Lg) acc = cadd(acc, cmul(cmul(sp[j], win[j]), wt[t]));
      }
      v[e] = acc;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jk = (l + T * e - q.bm) & (MI - 1);
      C acc = czero<C>();
      int te = 0;
      for (int j = jk; j < A.Lg; j += MI) {
        C u = cmul(sp[j], win[j]);
        if (te) u = cmul(u, A.ph[te]);
        acc = cadd(acc, u);
        te += tstep;
        if (te >= PM) te -= PM;
      }
      v[e] = acc;
    }
  }
  if (q.kn) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jk = (l + T * e - q.bm) & (MI - 1);
      int be = q.eb + jk * q.kn;                          // jk kn < PM
      if (be >= PM) be -= PM;
      v[e] = cmul(v[e], A.ph[be]);
    }
  }
  C* ex = lds + (wave * TPW + tt) * F::EX;
  if constexpr (F::HALF) {
    __syncthreads();   // the exchange areas alias the span and the window
    wave_fft_h<C, false>(v, ex, l, A.twm);
  } else {
    WTw<C, MI> tw;
    tw.load(A.twm, l);
    __syncthreads();
    wave_fft<C, MI, false>(v, ex, l, tw);
  }
  if (n < A.N) {
    int cnt, ee;
    C* row = (A.list ? pick(A.cl, int(bo)) : A.c + bo * A.cs) + coef_col(A.lay, n, &cnt, &ee);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (l + T * e < cnt) {
        if constexpr (HS)
          st_stream(row + l + T * e, v[e]);
        else
          row[l + T * e] = v[e];
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Forward, any in-LDS M: R time positions per work-group, LDS transforms.
// grid (ceil(N / R), B), 512 threads.
// ----------------------------------------------------------------------------
template <typename C>
__global__ void __launch_bounds__(kThreads) k_fir_fwd(FirArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int M = A.M, R = A.R, Sm = A.Sm;
  C* buf = tw + M;
  for (int e = threadIdx.x; e < M; e += kThreads) tw[e] = A.twm[e];
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  const int n0 = blockIdx.x * R;
  for (int e = threadIdx.x; e < R * M; e += kThreads) {
    const int r = e / M, k = e - r * M, n = n0 + r;
    C v = czero<C>();
    if (n < A.N) v = fir_bin(A, xsrc, xoff, fir_pos(A, n), k);
    buf[r * Sm + k] = v;
  }
  __syncthreads();
  fft_lds<C, false>(buf, Sm, A.fm, R, tw);
  C* cb = A.list ? pick(A.cl, int(bo)) : A.c + bo * A.cs;
  for (int e = threadIdx.x; e < R * M; e += kThreads) {
    const int r = e / M, m = e - r * M, n = n0 + r;
    if (n >= A.N) continue;
    int cnt, ee;
    const long long col = coef_col(A.lay, n, &cnt, &ee);
    if (m < cnt) cb[col + m] = buf[r * Sm + m];
  }
}

// ----------------------------------------------------------------------------
// Adjoint, first pass for power-of-two M = MI in [32, 1024]: one inverse wave
// transform per time position, Y[n][k] = sum_m c(m, n) exp(2 pi i k m / M).
// grid (ceil(N / (8 TPW)), B), 512 threads.
// ----------------------------------------------------------------------------
template <typename C, int MI>
__global__ void __launch_bounds__(kThreads, (FirWs<C, MI>::WAVES_PER_EU)) k_fir_adj_rows_w(FirArgs<C> A, C* Y,
                                                                                long long ys) {
  using I = WInfo<MI>;
  using F = FirWs<C, MI>;
  constexpr int E = I::E, T = I::T, TPW = I::TPW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const long long bo = blockIdx.y;
  const int n = (blockIdx.x * 8 + wave) * TPW + tt;
  const bool ok = n < A.N;
  int cnt, ee;
  const long long col = coef_col(A.lay, ok ? n : 0, &cnt, &ee);
  const C* cb = A.c + bo * A.cs;
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = coef_load(cb, MI, col, cnt, ee, l + T * e);
  C* ex = lds + (wave * TPW + tt) * F::EX;
  if constexpr (F::HALF) {
    wave_fft_h<C, true>(v, ex, l, A.twm);
  } else {
    WTw<C, MI> tw;
    tw.load(A.twm, l);
    wave_fft<C, MI, true>(v, ex, l, tw);
  }
  if (ok) {
    C* yr = Y + bo * ys + (long long)n * MI;
#pragma unroll
    for (int e = 0; e < E; ++e) yr[l + T * e] = v[e];
  }
}

// ----------------------------------------------------------------------------
// Adjoint, first pass: Y[n][k] = sum_m c(m, n) exp(2 pi i k m / M).
// grid (ceil(N / R), B), 512 threads.
// ----------------------------------------------------------------------------
template <typename C>
__global__ void __launch_bounds__(kThreads) k_fir_adj_rows(FirArgs<C> A, C* Y, long long ys) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int M = A.M, R = A.R, Sm = A.Sm;
  C* buf = tw + M;
  for (int e = threadIdx.x; e < M; e += kThreads) tw[e] = A.twm[e];
  const long long bo = blockIdx.y;
  const int n0 = blockIdx.x * R;
  const C* cb = A.c + bo * A.cs;
  for (int e = threadIdx.x; e < R * M; e += kThreads) {
    const int r = e / M, m = e - r * M, n = n0 + r;
    C v = czero<C>();
    if (n < A.N) {
      int cnt, ee;
      const long long col = coef_col(A.lay, n, &cnt, &ee);
      v = coef_load(cb, M, col, cnt, ee, m);
    }
    buf[r * Sm + m] = v;
  }
  __syncthreads();
  fft_lds<C, true>(buf, Sm, A.fm, R, tw);
  for (int e = threadIdx.x; e < R * M; e += kThreads) {
    const int r = e / M, k = e - r * M, n = n0 + r;
    if (n < A.N) Y[bo * ys + (long long)n * M + k] = buf[r * Sm + k];
  }
}

// ----------------------------------------------------------------------------
// Adjoint, gather: f(l) = sum over the time positions n whose window covers
// l (u = (l - start) mod L, n = floor(u / a) - t, j = u mod a + t a < L_g)
// of g(l - n a) exp(2 pi i l w(n) / M) Y[n][l mod M].  One sample per thread.
// grid (ceil(L / 512), B).
// ----------------------------------------------------------------------------
template <typename C>
__global__ void __launch_bounds__(kThreads) k_fir_adj_gather(FirArgs<C> A, const C* Y, long long ys, C* f) {
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= A.L) return;
  const long long bo = blockIdx.y;
  const int M = A.M, PM = A.lam2 * A.M, l2 = A.lam2;
  long long u = idx - A.start;
  if (u < 0) u += A.L;
  const long long nt = u / A.a;
  const int j0 = int(u - nt * A.a);
  const int i0 = int(idx % PM), km = i0 % M;
  const C* Yb = Y + bo * ys + km;
  const long long N = A.N, step = (long long)l2 * M, wrap = N * M;
  // taps t = 0, 1, ... (position n = nt - t mod N, window sample j = j0 + t a)
  // in lambda2 classes t = cl mod lambda2: lambda2 divides N, so a class has
  // one kn = (n lambda1) mod lambda2 and one phase exp(2 pi i l kn / (lambda2 M))
  C acc = czero<C>();
  for (int cl = 0; cl < l2; ++cl) {
    long long j = j0 + (long long)cl * A.a;     // 64-bit: l2 a may exceed 2^31 - L_g
    if (j >= A.Lg) break;
    long long n = nt - cl;
    if (n < 0) n += N;
    const int kn = int((n * A.lam1) % l2);
    long long o = n * M;
    C s = czero<C>();
    const long long ja = (long long)l2 * A.a;
#pragma unroll 4
    for (; j < A.Lg; j += ja) {
      s = cadd(s, cmulc(Yb[o], A.gw[j]));      // times g(l - n a) = conj(gw[j])
      o -= step;
      if (o < 0) o += wrap;
    }
    if (kn) {
      const int e = int(((long long)i0 * kn) % PM);
      s = cmulc(s, A.ph[e]);
    }
    acc = cadd(acc, s);
  }
  st_out(f, bo * A.L + idx, acc, A.real_out);
}

// Window support for the FIR algorithm: gw[j] = conj(g((start + j) mod L))
// in the plan precision, from the FP64 window.
template <typename CO>
__global__ void __launch_bounds__(kThreads) k_fir_window(const double2* g, CO* gw, long long L, long long start,
                                                         int Lg) {
  using TO = decltype(CO::x);
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= Lg) return;
  long long idx = start + j;
  if (idx >= L) idx -= L;
  gw[j] = mk<CO>(TO(g[idx].x), TO(-g[idx].y));
}

}  // namespace dgtns
