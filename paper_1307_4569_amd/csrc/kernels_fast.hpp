// Wave-FFT versions of the four hot kernels for power-of-two transform
// lengths (p = 1): forward factorisation ("cols"), channel DFT with the
// post-processing of Alg. 1 ("rows"), and their adjoints.
//
// Intermediate layout (shared with the generic kernels): per signal
//   h[n0][r][t'] = h_{n0 + q t'}(r),   n0 in Z_q, r in Z_Mi, t' in Z_d,
// so a factorisation column writes d contiguous values per time offset n0,
// and a row kernel reads, for each channel r, a contiguous run of time
// positions t' (one work-group handles RB consecutive t' of one n0).
#pragma once
#include "kernels.hpp"
#include "wave_fft.hpp"

namespace dgtns {

// elements per work-group: 8192 (FP32) or 4096 (FP64)
template <typename C> struct Budget { static constexpr int value = sizeof(C) == 8 ? 8192 : 4096; };

// Columns per work-group of the fast factorisation kernels for length D
// (KF > 0: that many wave transforms per wavefront; the adjoint uses one, as
// its accumulators stay live across the loop over n0).
template <typename C, int D, int KF = 0> struct FastCols {
  static constexpr int TPW = WInfo<D>::TPW;
  static constexpr int K0 = Budget<C>::value / (8 * TPW * D);
  static constexpr int K = KF > 0 ? KF : (K0 < 1 ? 1 : K0);   // wave transforms per wavefront
  static constexpr int W = 8 * TPW * K;           // columns per work-group (8 wavefronts)
  static constexpr int SD = D + 1;                // padded column stride of the LDS tile
  static constexpr int TILE = W * SD;
  static constexpr int EXW = TPW * WEx<C, D>::EX;  // exchange elements per wavefront
  static constexpr int LDS = (TILE > 8 * EXW ? TILE : 8 * EXW);
  // forward with h[n0][t][r]: the [t][column] staging tile of stride W + 1
  static constexpr int SW = W + 1;
  static constexpr int LDS_T = (LDS > D * SW ? LDS : D * SW);
  // KF = 1: the staging tile after the exchange areas instead of aliasing them
  static constexpr int LDS_TS = (TILE > 8 * EXW + D * SW ? TILE : 8 * EXW + D * SW);
};

// Rows per work-group of the fast row kernels for length MI: half the element
// budget, so that four work-groups (32 wavefronts) fit on a compute unit; the
// adjoint (ADJ) takes the whole budget, so that its strided stores of h
// cover whole 128-byte lines in FP32.
// The [Mi][RB] tile of the adjoint (strided stores, row-wise loads) uses the
// padded stride RB + 1; the forward tile (row-wise stores, strided loads)
// stores element (m, i) at m RB + i + m / PD, which keeps both its stores
// (128 bytes per cycle) and its column loads (256 bytes per cycle) free of
// LDS bank conflicts when RB is below the 256 bytes a load serves.
template <typename C, int MI, bool ADJ = false> struct FastRows {
  static constexpr int TPW = WInfo<MI>::TPW;
  static constexpr int K0 = Budget<C>::value / ((ADJ ? 8 : 16) * TPW * MI);
  static constexpr int K = K0 < 1 ? 1 : K0;
  static constexpr int RB = 8 * TPW * K;          // rows (time positions t') per work-group
  static constexpr int SR = RB + 1;               // padded stride of the adjoint tile
  static constexpr int LR = 256 / int(sizeof(C)); // elements one LDS load cycle serves
  static constexpr int PD = RB >= LR ? 1 : LR / RB;
  static __device__ __forceinline__ int fwd_at(int m, int i) { return m * RB + i + m / PD; }
  static constexpr int TILE_F = MI * RB + MI / PD;
  static constexpr int TILE = MI * SR > TILE_F ? MI * SR : TILE_F;
  static constexpr int EXW = TPW * WEx<C, MI>::EX;
  static constexpr int LDS = (TILE > 8 * EXW ? TILE : 8 * EXW);
};

// ----------------------------------------------------------------------------
// Forward factorisation, p = 1, compile-time d = D.
// grid (ceil(Mi / W) * nsplit, B), 512 threads; the nsplit work-groups of a
// column block each compute the column DFTs and a share of the q offsets n0
// (more work-groups for small batches).
// ----------------------------------------------------------------------------
// HS: streaming stores of h (chosen at launch from the size of h, stream_h).
// HT: h is written as h[n0][t][r] (time-major), which lets the row kernel read
// each row of Mi channels as one contiguous run; otherwise h[n0][r][t].
// KF: wave transforms per wavefront (0: as many as the element budget allows;
// 1: one, for the chunks of a sequential batch, whose h stays in the
// last-level cache, so that the half-line rows of 8 columns cost nothing in
// HBM and the lower register count lets more waves hide latency).
template <typename C, int D, bool HS, bool HT, int KF = 0>
__global__ void __launch_bounds__(kThreads) k_fwd_cols_w(ColArgs<C> A) {
  using F = FastCols<C, D, KF>;
  using I = WInfo<D>;
  constexpr int E = I::E, T = I::T, K = F::K, W = F::W, SD = F::SD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const int Mi = A.Mi;
  // column block and the share of time offsets n0 of this work-group
  const int bx = xcd_block_x();
  const int cb = bx / A.nsplit, part = bx - cb * A.nsplit;
  const int qper = (A.q + A.nsplit - 1) / A.nsplit;
  const int n0_begin = part * qper, n0_end = min(A.q, n0_begin + qper);
  const int r0 = cb * W;
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  // 1. coalesced load of W adjacent columns (d values each), chirp applied
  {
    constexpr int NL = (W * D) / kThreads;
    static_assert(NL * kThreads == W * D, "column tile is a whole number of passes");
    long long li[NL];
    bool ok[NL];
    C v[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = tid + i * kThreads, t = e / W, cc = e - t * W, r = r0 + cc;
      ok[i] = r < Mi;
      li[i] = ok[i] ? r + (long long)t * Mi : 0;
    }
    load_chirped<C, NL>(xsrc, A.real_in, xoff, A.chirp, li, ok, v);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = tid + i * kThreads, t = e / W, cc = e - t * W;
      lds[cc * SD + t] = v[i];
    }
  }
  WTw<C, D> tw;
  tw.load(A.twd, l);
  __syncthreads();
  C X[K][E];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int cc = (wave * K + k) * I::TPW + tt;
#pragma unroll
    for (int e = 0; e < E; ++e) X[k][e] = lds[cc * SD + l + T * e];
  }
  __syncthreads();
  C* ex = lds + wave * F::EXW + tt * WEx<C, D>::EX;
#pragma unroll
  for (int k = 0; k < K; ++k) wave_fft<C, D, false>(X[k], ex, l, tw);
  if constexpr (HT) {
    // The W columns of each n0 are staged through LDS as [t][column] rows
    // (stride SW) and leave as W contiguous values per time position.  A row
    // index u = r - n0 ai below zero multiplies the window Zak by
    // exp(2 pi i nu / d); after the inverse DFT that is the cyclic shift
    // h(t) = y(t + 1), applied here as a shifted staging index.
    // SEP (KF = 1): the staging tile has LDS of its own, after the exchange
    // areas, which saves one barrier per offset; the window rows of the next
    // offset are loaded while the current one is transformed and stored, and
    // each thread reads all its staged values before it stores them.
    constexpr int SW = F::SW;
    constexpr bool SEP = KF == 1;
    C* stg = SEP ? lds + 8 * F::EXW : lds;
    C Z[K][E];
    int sh[K];
    auto zload = [&](int n0) {
      int n0w;
      const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int r = r0 + (wave * K + k) * I::TPW + tt;
        const int v0 = r - n0w * A.ai;
        const int u = v0 >= 0 ? v0 : v0 + Mi;
        sh[k] = v0 < 0 ? D - 1 : 0;
        const C* zrow = zc + (long long)(r < Mi ? u : 0) * D;
#pragma unroll
        for (int e = 0; e < E; ++e) Z[k][e] = zrow[l + T * e];
      }
    };
    if (SEP && n0_begin < n0_end) zload(n0_begin);
    for (int n0 = n0_begin; n0 < n0_end; ++n0) {
      if (!SEP) zload(n0);
      C Y[K][E];
      int shc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        shc[k] = sh[k];
#pragma unroll
        for (int e = 0; e < E; ++e) Y[k][e] = cmul(X[k][e], Z[k][e]);
      }
      if (SEP) zload(n0 + 1 < n0_end ? n0 + 1 : n0);   // unconditional: no register copies of Z
#pragma unroll
      for (int k = 0; k < K; ++k) wave_fft<C, D, true>(Y[k], ex, l, tw);
      // SEP: every thread has read the previous offset's tile; otherwise the
      // exchange areas alias the tile
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int cc = (wave * K + k) * I::TPW + tt;
#pragma unroll
        for (int e = 0; e < E; ++e) stg[((l + T * e + shc[k]) & (D - 1)) * SW + cc] = Y[k][e];
      }
      __syncthreads();
      C* hb = A.H + bo * A.hs + (long long)n0 * D * Mi + r0;
      if constexpr (SEP) {
        constexpr int NS = (W * D) / kThreads;
        static_assert(NS * kThreads == W * D, "staging tile is a whole number of passes");
        C sv[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int e = tid + i * kThreads, t = e / W, c = e - t * W;
          sv[i] = stg[t * SW + c];
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int e = tid + i * kThreads, t = e / W, c = e - t * W;
          if (r0 + c < Mi) {
            if constexpr (HS)
              st_stream(hb + (long long)t * Mi + c, sv[i]);
            else
              hb[(long long)t * Mi + c] = sv[i];
          }
        }
      } else {
        for (int e = tid; e < W * D; e += kThreads) {
          const int t = e / W, c = e - t * W;
          if (r0 + c < Mi) {
            if constexpr (HS)
              st_stream(hb + (long long)t * Mi + c, stg[t * SW + c]);
            else
              hb[(long long)t * Mi + c] = stg[t * SW + c];
          }
        }
        __syncthreads();
      }
    }
    return;
  }
  const C* tw_d = A.twd;
  for (int n0 = n0_begin; n0 < n0_end; ++n0) {
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = r0 + (wave * K + k) * I::TPW + tt;
      const bool ok = r < Mi;
      const int v0 = r - n0w * A.ai;
      const int u = v0 >= 0 ? v0 : v0 + Mi;
      const C* zrow = zc + (long long)(ok ? u : 0) * D;
      C Y[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int nu = l + T * e;
        C z = zrow[nu];
        if (v0 < 0) z = cmulc(z, tw_d[nu]);
        Y[e] = cmul(X[k][e], z);
      }
      wave_fft<C, D, true>(Y, ex, l, tw);
      if (ok) {
        C* hb = A.H + bo * A.hs + ((long long)n0 * Mi + r) * D;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if constexpr (HS)
            st_stream(hb + l + T * e, Y[e]);
          else
            hb[l + T * e] = Y[e];
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Adjoint factorisation, p = 1, compile-time d = D.
// ----------------------------------------------------------------------------
// FP32: at least four waves per SIMD (two work-groups per compute unit).
template <typename C, int D>
__global__ void __launch_bounds__(kThreads, sizeof(C) == 8 ? 4 : 1) k_adj_cols_w(ColAdjArgs<C> A) {
  using F = FastCols<C, D, 1>;
  using I = WInfo<D>;
  constexpr int E = I::E, T = I::T, K = F::K, W = F::W, SD = F::SD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const int Mi = A.Mi;
  const int r0 = blockIdx.x * W;
  const long long bo = blockIdx.y;
  WTw<C, D> tw;
  tw.load(A.twd, l);
  C* ex = lds + wave * F::EXW + tt * WEx<C, D>::EX;
  C acc[K][E];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[k][e] = czero<C>();
  for (int n0 = 0; n0 < A.q; ++n0) {
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = r0 + (wave * K + k) * I::TPW + tt;
      const bool ok = r < Mi;
      C Y[E];
      const C* hb = A.H + bo * A.hs + ((long long)n0 * Mi + (ok ? r : 0)) * D;
#pragma unroll
      for (int e = 0; e < E; ++e) Y[e] = hb[l + T * e];
      wave_fft<C, D, false>(Y, ex, l, tw);
      const int v0 = r - n0w * A.ai;
      const int u = v0 >= 0 ? v0 : v0 + Mi;
      const C* zrow = zc + (long long)(ok ? u : 0) * D;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int nu = l + T * e;
        C z = zrow[nu];
        if (v0 < 0) z = cmulc(z, A.twd[nu]);
        acc[k][e] = cadd(acc[k][e], cmulc(Y[e], z));
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) wave_fft<C, D, true>(acc[k], ex, l, tw);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int cc = (wave * K + k) * I::TPW + tt;
#pragma unroll
    for (int e = 0; e < E; ++e) lds[cc * SD + l + T * e] = acc[k][e];
  }
  __syncthreads();
  for (int e = tid; e < W * D; e += kThreads) {
    const int t = e / W, cc = e - t * W, r = r0 + cc;
    if (r < Mi) {
      const long long li = r + (long long)t * Mi;
      st_out(A.y, bo * A.ys + li, apply_chirp(A.chirp, lds[cc * SD + t], li), A.real_out);
    }
  }
}

// ----------------------------------------------------------------------------
// Window gradient, p = 1, compile-time d = D.
// k_col_spectra_w: X_r = DFT_d of the (chirped) signal column r, stored as
// one contiguous row X[r][nu] per column; grid (ceil(Mi / W), B).
// k_grad_cols_w: for window column u and time offset n0 the signal column is
// r = (u + n0 ai) mod Mi, and in the Zak domain
//   grad Zg_u(nu) = (1/d) sum_n0 X_r(nu) conj(Hhat_{n0,r}(nu)) w(nu),
// with Hhat the DFT over t' of the adjoint-row output h[n0][r][.] and
// w(nu) = exp(2 pi i nu / d) where the column index wrapped (else 1); the
// gradient column is the unnormalised inverse DFT of grad Zg_u.  One wave
// transform per window column accumulates over n0 in registers; grid
// (ceil(Mi / W), B), one partial per signal, summed in a fixed order after.
// ----------------------------------------------------------------------------
template <typename C, int D>
__global__ void __launch_bounds__(kThreads) k_col_spectra_w(ColArgs<C> A) {
  using F = FastCols<C, D>;
  using I = WInfo<D>;
  constexpr int E = I::E, T = I::T, K = F::K, W = F::W, SD = F::SD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const int Mi = A.Mi;
  const int r0 = blockIdx.x * W;
  const long long bo = blockIdx.y;
  for (int e = tid; e < W * D; e += kThreads) {
    const int t = e / W, cc = e - t * W, r = r0 + cc;
    C v = czero<C>();
    if (r < Mi) {
      const long long li = r + (long long)t * Mi;
      v = apply_chirp(A.chirp, load_sig<C>(A.x, A.real_in, bo * A.xs + li), li);
    }
    lds[cc * SD + t] = v;
  }
  WTw<C, D> tw;
  tw.load(A.twd, l);
  __syncthreads();
  C X[K][E];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int cc = (wave * K + k) * I::TPW + tt;
#pragma unroll
    for (int e = 0; e < E; ++e) X[k][e] = lds[cc * SD + l + T * e];
  }
  __syncthreads();
  C* ex = lds + wave * F::EXW + tt * WEx<C, D>::EX;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    wave_fft<C, D, false>(X[k], ex, l, tw);
    const int r = r0 + (wave * K + k) * I::TPW + tt;
    if (r < Mi) {
      C* xo = A.H + bo * A.hs + (long long)r * D;
#pragma unroll
      for (int e = 0; e < E; ++e) xo[l + T * e] = X[k][e];
    }
  }
}

template <typename C> struct GradWArgs {
  const C* X;          // column spectra X[r][nu], xs values per signal
  long long xs;
  const C* H;          // adjoint-row output h[n0][r][t'], hs values per signal
  long long hs;
  C* part;             // per-signal window gradient, ps values per signal
  long long ps;
  const C* twd;
  int Mi, ai, q;
};

template <typename C, int D>
__global__ void __launch_bounds__(kThreads, sizeof(C) == 8 ? 4 : 1) k_grad_cols_w(GradWArgs<C> A) {
  using F = FastCols<C, D, 1>;
  using I = WInfo<D>;
  constexpr int E = I::E, T = I::T, W = F::W, SD = F::SD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const int Mi = A.Mi;
  const int u0 = blockIdx.x * W;
  const long long bo = blockIdx.y;
  WTw<C, D> tw;
  tw.load(A.twd, l);
  C* ex = lds + wave * F::EXW + tt * WEx<C, D>::EX;
  const int cc = wave * I::TPW + tt, u = u0 + cc;
  const int uc = u < Mi ? u : 0;
  C acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = czero<C>();
  for (int n0 = 0; n0 < A.q; ++n0) {
    int r = uc + n0 * A.ai;   // n0 ai < Mi for p = 1
    const bool wrap = r >= Mi;
    if (wrap) r -= Mi;
    C Y[E];
    const C* hb = A.H + bo * A.hs + ((long long)n0 * Mi + r) * D;
#pragma unroll
    for (int e = 0; e < E; ++e) Y[e] = hb[l + T * e];
    wave_fft<C, D, false>(Y, ex, l, tw);
    const C* xb = A.X + bo * A.xs + (long long)r * D;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int nu = l + T * e;
      C pr = cmulc(xb[nu], Y[e]);
      if (wrap) pr = cmulc(pr, A.twd[nu]);
      acc[e] = cadd(acc[e], pr);
    }
  }
  using R = decltype(C::x);
  const R inv_d = R(1) / R(D);
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = cscale(acc[e], inv_d);
  wave_fft<C, D, true>(acc, ex, l, tw);
  __syncthreads();   // the exchange areas alias the output tile
#pragma unroll
  for (int e = 0; e < E; ++e) lds[cc * SD + l + T * e] = acc[e];
  __syncthreads();
  for (int e = tid; e < W * D; e += kThreads) {
    const int t = e / W, c = e - t * W, uu = u0 + c;
    if (uu < Mi) A.part[bo * A.ps + uu + (long long)t * Mi] = lds[c * SD + t];
  }
}

// ----------------------------------------------------------------------------
// Row kernels, compile-time Mi = MI.  A work-group handles the RB
// intermediate rows (n0, t0 + i), i in Z_RB, n0 = blockIdx.x mod q, whose
// time positions are n = row_time(n0, t0 + i) (n0 + q (t0 + i) for the shear
// algorithm).
// grid (q * ceil(d / RB), B), 512 threads.
// ----------------------------------------------------------------------------
// HS: streaming stores of the coefficients (a launch whose output cannot stay
// in the last-level cache; otherwise its dirty lines are written back while
// the next kernel runs).
// HT: h[n0][t][r] (written by k_fwd_cols_w<.., true>): each wave transform
// loads its row of MI channels straight into registers, with no LDS tile.
template <typename C, int MI, int MODE, bool HS, bool HT>
__global__ void __launch_bounds__(kThreads) k_fwd_rows_w(RowArgs<C> A) {
  using F = FastRows<C, MI>;
  using I = WInfo<MI>;
  constexpr int E = I::E, T = I::T, K = F::K, RB = F::RB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const int q = A.q, d = A.d;
  const int n0 = blockIdx.x % q, t0 = (blockIdx.x / q) * RB;
  const long long bo = blockIdx.y;
  C v[K][E];
  WTw<C, MI> tw;
  if constexpr (HT) {
    const C* hb = A.H + bo * A.hs + (long long)n0 * MI * d;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int t = t0 + (wave * K + k) * I::TPW + tt;
      const C* hr = hb + (long long)(t < d ? t : 0) * MI;
#pragma unroll
      for (int e = 0; e < E; ++e) v[k][e] = hr[l + T * e];
    }
    tw.load(A.twm, l);
  } else {
    const C* hb = A.H + bo * A.hs + (long long)n0 * MI * d + t0;
    for (int e = tid; e < RB * MI; e += kThreads) {
      const int m = e / RB, i = e - m * RB;
      lds[F::fwd_at(m, i)] = t0 + i < d ? hb[(long long)m * d + i] : czero<C>();
    }
    tw.load(A.twm, l);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = (wave * K + k) * I::TPW + tt;
#pragma unroll
      for (int e = 0; e < E; ++e) v[k][e] = lds[F::fwd_at(l + T * e, i)];
    }
    __syncthreads();
  }
  C* ex = lds + wave * F::EXW + tt * WEx<C, MI>::EX;
  C* cb = A.list ? pick(A.cl, int(bo)) : A.c + bo * A.cs;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    wave_fft<C, MI, false>(v[k], ex, l, tw);
    const int i = (wave * K + k) * I::TPW + tt;
    const int n = row_time(n0, t0 + i, A.qw, A.nw);
    if (t0 + i >= d) {
      // time position beyond d in the last work-group: nothing to store
    } else if (MODE == 0) {
      const C En = A.postE[n];
      const int rho = A.rho[n];
      int cnt, ee;
      C* row = cb + coef_col(A.lay, n, &cnt, &ee);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int mo = l + T * e + rho;
        if (mo >= MI) mo -= MI;
        if (mo < cnt) {
          if constexpr (HS)
            st_stream(row + mo, cmul(En, v[k][e]));
          else
            row[mo] = cmul(En, v[k][e]);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int kp = l + T * e;
        const long long kk = kp == 0 ? 0 : MI - kp;
        long long nt, kt;
        C Ev;
        shear_map(A, n, kk, &nt, &kt, &Ev);
        int cnt, ee;
        const long long col = coef_col(A.lay, nt, &cnt, &ee);
        if (kt < cnt) {
          if constexpr (HS)
            st_stream(cb + col + kt, cmul(Ev, v[k][e]));
          else
            cb[col + kt] = cmul(Ev, v[k][e]);
        }
      }
    }
  }
}

template <typename C, int MI, int MODE, bool HS>
__global__ void __launch_bounds__(kThreads) k_adj_rows_w(RowArgs<C> A) {
  using F = FastRows<C, MI, true>;
  using I = WInfo<MI>;
  constexpr int E = I::E, T = I::T, K = F::K, RB = F::RB, SR = F::SR;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  // the wave index through readfirstlane: when one transform fills the
  // wavefront, its row indices, phase and rotation loads and row addresses
  // stay on the scalar unit
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, tt = lane / T, l = lane - tt * T;
  const int q = A.q, d = A.d;
  const int n0 = blockIdx.x % q, t0 = (blockIdx.x / q) * RB;
  const long long bo = blockIdx.y;
  WTw<C, MI> tw;
  tw.load(A.twm, l);
  C* ex = lds + wave * F::EXW + tt * WEx<C, MI>::EX;
  const C* cb = A.c + bo * A.cs;
  C v[K][E];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = (wave * K + k) * I::TPW + tt;
    const bool ok = t0 + i < d;
    const int n = row_time(n0, ok ? t0 + i : 0, A.qw, A.nw);
    if (MODE == 0) {
      const C En = A.postE[n];
      const int rho = A.rho[n];
      int cnt, ee;
      const long long col = coef_col(A.lay, n, &cnt, &ee);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int mo = l + T * e + rho;
        if (mo >= MI) mo -= MI;
        v[k][e] = cmulc(coef_load(cb, MI, col, cnt, ee, mo), En);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int kp = l + T * e;
        const long long kk = kp == 0 ? 0 : MI - kp;
        long long nt, kt;
        C Ev;
        shear_map(A, n, kk, &nt, &kt, &Ev);
        int cnt, ee;
        const long long col = coef_col(A.lay, nt, &cnt, &ee);
        v[k][e] = cmulc(coef_load(cb, int(A.M), col, cnt, ee, int(kt)), Ev);
      }
    }
  }
  // every row of the thread is loaded before the first transform
#pragma unroll
  for (int k = 0; k < K; ++k) wave_fft<C, MI, true>(v[k], ex, l, tw);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = (wave * K + k) * I::TPW + tt;
#pragma unroll
    for (int e = 0; e < E; ++e) lds[(l + T * e) * SR + i] = v[k][e];
  }
  __syncthreads();
  // all staged values of a thread are read before the first store
  C* hb = const_cast<C*>(A.H) + bo * A.hs + (long long)n0 * MI * d + t0;
  constexpr int NS = (RB * MI) / kThreads;
  static_assert(NS * kThreads == RB * MI, "row tile is a whole number of passes");
  C sv[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int e = tid + j * kThreads, m = e / RB, i = e - m * RB;
    sv[j] = lds[m * SR + i];
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int e = tid + j * kThreads, m = e / RB, i = e - m * RB;
    if (t0 + i < d) {
      if constexpr (HS)
        st_stream(hb + (long long)m * d + i, sv[j]);
      else
        hb[(long long)m * d + i] = sv[j];
    }
  }
}

}  // namespace dgtns
