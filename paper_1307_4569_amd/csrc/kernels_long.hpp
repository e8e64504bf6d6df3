// Factorisation with columns longer than one in-LDS transform (Sec. 4,
// full-window algorithm): the length-d DFTs of the column step are split as
// d = d1 d2 (Cooley-Tukey).  With t = t1 d2 + t2, nu = k1 + d1 k2 and
// W_n = exp(-2 pi i / n):
//   forward   X(k1 + d1 k2) = sum_t2 W_d2^{t2 k2} W_d^{t2 k1} sum_t1 x(t1 d2 + t2) W_d1^{t1 k1}
//   inverse   h(s2 + d2 s1) = sum_k1 W_d1^{-s1 k1} W_d^{-s2 k1} sum_k2 Y(k1 + d1 k2) W_d2^{-s2 k2}
// (the inverse unnormalised).  Spectra are kept digit-reversed: value nu at
// position k1 d2 + k2, the window Zak tables too, so the products read
// contiguous rows.
//
// A signal of length L = ncol d has ncol = Mi p sub-columns cid = r + Mi j0
// (column r, polyphase index j0) with samples x(cid + ncol t); viewed as the
// row-major [d1][d2 ncol] matrix its element (t1, t2 ncol + cid) is
// x(cid + ncol (t1 d2 + t2)).  Three passes per direction:
//   k_long_col   length-d1 transforms down the columns of such matrices
//                (signal <-> U, and V <-> h), with the inter-pass twiddle;
//   k_long_mid   forward: per (k1, block of columns r) the length-d2 DFTs of
//                the sub-columns, the q window products and the length-d2
//                inverse DFTs, writing V[n0][k1][r d2 + s2];
//   k_long_mid_adj  the adjoint: per n0 the length-d2 DFT of V, products with
//                the conjugate window accumulated over n0, one inverse DFT
//                per sub-column, writing U.
#pragma once
#include "kernels.hpp"

namespace dgtns {

// ----------------------------------------------------------------------------
// Column pass.  Transforms of length n = d1 down the columns c in Z_ncols of
// per-signal (and per-n0, grid z) matrices.  Element (j, c):
//   inmode 0: in[j ncols + c] (+ pre-chirp at that index: the signal, list)
//   inmode 1: h layout, in[r d + s2 + d2 j] with c = r d2 + s2
// and the output element (k, c):
//   outmode 0: out[k ncols + c]
//   outmode 1: h layout, out[r d + s2 + d2 k]
//   outmode 2: out[k ncols + c] times the conjugate post-chirp at that index
// twmode: 0 none; 1 times W_d^{(c / tdiv) k}; 2 times W_d^{(c mod tdiv) k}
// (conjugated for INV).  grid (ceil(ncols / W), B, q), 512 threads.
// ----------------------------------------------------------------------------
template <typename C> struct LongColArgs {
  const void* x;
  long long xs, xz;            // per-signal and per-grid-z strides of the input
  int real_in;
  int list;
  const void* xl[kListMax];
  ChirpSrc<C> pre, post;
  C* y;
  long long ys, yz;
  const C* tws;                // length-n stage twiddles
  const C* twd;                // exp(-2 pi i e / d), e in Z_d
  int n, ncols, W, Sn;
  int inmode, outmode, twmode;
  int tdiv, d, d2;
  FftSched fs;
  int real_out;                // write the real part of y only (outmode 0 and 2)
};

template <typename C, bool INV>
__global__ void __launch_bounds__(kThreads) k_long_col(LongColArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int n = A.n, W = A.W, Sn = A.Sn, nc = A.ncols, d = A.d, d2 = A.d2;
  C* buf = tw + n;
  for (int e = threadIdx.x; e < n; e += kThreads) tw[e] = A.tws[e];
  const int c0 = blockIdx.x * W;
  const long long bo = blockIdx.y, z = blockIdx.z;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = (A.list ? 0 : bo * A.xs) + z * A.xz;
  batched_for<4, C>(
      threadIdx.x, W * n, kThreads,
      [&](int e) {
        const int j = e / W, cc = e - j * W, col = c0 + cc;
        C v = czero<C>();
        if (col < nc) {
          if (A.inmode == 0) {
            const long long idx = (long long)j * nc + col;
            v = apply_chirp(A.pre, load_sig<C>(xsrc, A.real_in, xoff + idx), idx);
          } else {
            const int r = col / d2, s2 = col - r * d2;
            v = load_sig<C>(xsrc, 0, xoff + (long long)r * d + s2 + (long long)d2 * j);
          }
        }
        return v;
      },
      [&](int e, C v) {
        const int j = e / W, cc = e - j * W;
        buf[cc * Sn + j] = v;
      });
  __syncthreads();
  fft_lds<C, INV>(buf, Sn, A.fs, W, tw);
  const long long yoff = bo * A.ys + z * A.yz;
  for (int e = threadIdx.x; e < W * n; e += kThreads) {
    const int k = e / W, cc = e - k * W, col = c0 + cc;
    if (col >= nc) continue;
    C v = buf[cc * Sn + k];
    if (A.twmode) {
      const long long m = A.twmode == 1 ? col / A.tdiv : col % A.tdiv;
      const C w = A.twd[(m * k) % d];
      v = INV ? cmulc(v, w) : cmul(v, w);
    }
    if (A.outmode == 1) {
      const int r = col / d2, s2 = col - r * d2;
      A.y[yoff + (long long)r * d + s2 + (long long)d2 * k] = v;
    } else {
      const long long idx = (long long)k * nc + col;
      st_out(A.y, yoff + idx, A.outmode == 2 ? apply_chirp(A.post, v, idx) : v, A.real_out);
    }
  }
}

// Window coefficient of the long factorisation: as zc_coef, with the tables
// stored digit-reversed (nu = k1 + d1 k2 at k1 d2 + k2) and the twiddle
// exp(+2 pi i nu / d) from the global length-d table.
template <typename C>
__device__ __forceinline__ C zc_coef_long(const C* zc, const C* twd, int r, int n0, int j0, int k1, int k2, int ai,
                                          int Mi, int p, int d, int d1, int d2) {
  const int v = r - n0 * ai + Mi * j0;
  int u = v % Mi;
  if (u < 0) u += Mi;
  const int j1 = (v - u) / Mi;
  int j0p = j1 % p;
  if (j0p < 0) j0p += p;
  C z = zc[((long long)u * p + j0p) * d + (long long)k1 * d2 + k2];
  if (j1 < 0) z = cmulc(z, twd[k1 + d1 * k2]);
  return z;
}

// ----------------------------------------------------------------------------
// Middle pass, forward.  grid (d1 ceil(Mi / W), B), 512 threads; block
// x = rb d1 + k1 handles columns r0 = rb W ... of spectral row k1.
//   U: per signal [d1][d2 ncol] (output of the first column pass)
//   V: per signal [q][d1][Mi d2]
// ----------------------------------------------------------------------------
template <typename C> struct LongMidArgs {
  const C* U;
  long long us;
  C* V;
  long long vs;
  const C* zc;
  long long zs;
  const C* twd;
  const C* tw2;
  int Mi, ai, p, q, qw, d, d1, d2, W, Sd2, ncol;
  FftSched fs2;
};

template <typename C>
__global__ void __launch_bounds__(kThreads) k_long_mid(LongMidArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int d1 = A.d1, d2 = A.d2, W = A.W, S = A.Sd2, p = A.p, Mi = A.Mi, ncol = A.ncol;
  C* xb = tw + d2;               // [W p][S]
  C* yb = xb + W * p * S;        // [W][S]
  for (int e = threadIdx.x; e < d2; e += kThreads) tw[e] = A.tw2[e];
  const int k1 = blockIdx.x % d1, r0 = (blockIdx.x / d1) * W;
  const long long bo = blockIdx.y;
  const C* Ub = A.U + bo * A.us + (long long)k1 * d2 * ncol;
  for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
    const int t2 = e / (W * p), rem = e - t2 * (W * p), j0 = rem / W, cc = rem - j0 * W, r = r0 + cc;
    xb[(cc * p + j0) * S + t2] = r < Mi ? Ub[(long long)t2 * ncol + r + Mi * j0] : czero<C>();
  }
  __syncthreads();
  fft_lds<C, false>(xb, S, A.fs2, W * p, tw);
  for (int n0 = 0; n0 < A.q; ++n0) {
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
    for (int e = threadIdx.x; e < W * d2; e += kThreads) {
      const int cc = e / d2, k2 = e - cc * d2, r = r0 + cc;
      C y = czero<C>();
      if (r < Mi) {
        for (int j0 = 0; j0 < p; ++j0)
          y = cadd(y, cmul(xb[(cc * p + j0) * S + k2],
                           zc_coef_long(zc, A.twd, r, n0w, j0, k1, k2, A.ai, Mi, p, A.d, d1, d2)));
      }
      yb[cc * S + k2] = y;
    }
    __syncthreads();
    fft_lds<C, true>(yb, S, A.fs2, W, tw);
    C* Vb = A.V + bo * A.vs + ((long long)n0 * d1 + k1) * Mi * d2;
    for (int e = threadIdx.x; e < W * d2; e += kThreads) {
      const int cc = e / d2, s2 = e - cc * d2, r = r0 + cc;
      if (r < Mi) Vb[(long long)r * d2 + s2] = cmulc(yb[cc * S + s2], A.twd[((long long)s2 * k1) % A.d]);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// Middle pass, adjoint.  Same grid.  V: per signal [q][d1][Mi d2] (the
// forward DFT over s1 of h with its twiddle); U: per signal [d1][d2 ncol].
// ----------------------------------------------------------------------------
template <typename C>
__global__ void __launch_bounds__(kThreads) k_long_mid_adj(LongMidArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int d1 = A.d1, d2 = A.d2, W = A.W, S = A.Sd2, p = A.p, Mi = A.Mi, ncol = A.ncol;
  C* acc = tw + d2;              // [W p][S]
  C* yb = acc + W * p * S;       // [W][S]
  for (int e = threadIdx.x; e < d2; e += kThreads) tw[e] = A.tw2[e];
  for (int e = threadIdx.x; e < W * p * S; e += kThreads) acc[e] = czero<C>();
  const int k1 = blockIdx.x % d1, r0 = (blockIdx.x / d1) * W;
  const long long bo = blockIdx.y;
  for (int n0 = 0; n0 < A.q; ++n0) {
    const C* Vb = A.V + bo * A.vs + ((long long)n0 * d1 + k1) * Mi * d2;
    __syncthreads();
    for (int e = threadIdx.x; e < W * d2; e += kThreads) {
      const int cc = e / d2, s2 = e - cc * d2, r = r0 + cc;
      yb[cc * S + s2] = r < Mi ? Vb[(long long)r * d2 + s2] : czero<C>();
    }
    __syncthreads();
    fft_lds<C, false>(yb, S, A.fs2, W, tw);
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
    for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
      const int cc = e / (p * d2), rem = e - cc * (p * d2), j0 = rem / d2, k2 = rem - j0 * d2, r = r0 + cc;
      if (r < Mi) {
        C& a = acc[(cc * p + j0) * S + k2];
        a = cadd(a, cmulc(yb[cc * S + k2], zc_coef_long(zc, A.twd, r, n0w, j0, k1, k2, A.ai, Mi, p, A.d, d1, d2)));
      }
    }
  }
  __syncthreads();
  fft_lds<C, true>(acc, S, A.fs2, W * p, tw);
  C* Ub = const_cast<C*>(A.U) + bo * A.us + (long long)k1 * d2 * ncol;
  for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
    const int t2 = e / (W * p), rem = e - t2 * (W * p), j0 = rem / W, cc = rem - j0 * W, r = r0 + cc;
    if (r < Mi)
      Ub[(long long)t2 * ncol + r + Mi * j0] = cmulc(acc[(cc * p + j0) * S + t2], A.twd[((long long)t2 * k1) % A.d]);
  }
}

// ----------------------------------------------------------------------------
// Window Zak transform, long columns (FP64): from U64 (the first column pass
// of the prepared window) the length-d2 DFTs of every sub-column, stored
// digit-reversed as conj(Zg)/d in the plan precision and, if z64, as Zg.
// grid (d1 ceil(Mi / W)), 512 threads.
// ----------------------------------------------------------------------------
template <typename CO>
__global__ void __launch_bounds__(kThreads) k_long_zak(const double2* U, CO* zc, double2* z64, const double2* tw2,
                                                       int Mi, int p, int d, int d1, int d2, int W, int S,
                                                       FftSched fs2) {
  using TO = decltype(CO::x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* tw = reinterpret_cast<double2*>(smem_raw);
  double2* xb = tw + d2;
  const int ncol = Mi * p;
  for (int e = threadIdx.x; e < d2; e += kThreads) tw[e] = tw2[e];
  const int k1 = blockIdx.x % d1, r0 = (blockIdx.x / d1) * W;
  const double2* Ub = U + (long long)k1 * d2 * ncol;
  for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
    const int t2 = e / (W * p), rem = e - t2 * (W * p), j0 = rem / W, cc = rem - j0 * W, r = r0 + cc;
    xb[(cc * p + j0) * S + t2] = r < Mi ? Ub[(long long)t2 * ncol + r + Mi * j0] : make_double2(0, 0);
  }
  __syncthreads();
  fft_lds<double2, false, 8>(xb, S, fs2, W * p, tw);
  const double inv_d = 1.0 / d;
  for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
    const int cc = e / (p * d2), rem = e - cc * (p * d2), j0 = rem / d2, k2 = rem - j0 * d2, r = r0 + cc;
    if (r < Mi) {
      const double2 z = xb[(cc * p + j0) * S + k2];
      const long long o = ((long long)r * p + j0) * d + (long long)k1 * d2 + k2;
      if (zc) zc[o] = mk<CO>(TO(z.x * inv_d), TO(-z.y * inv_d));
      if (z64) z64[o] = z;
    }
  }
}

// Inverse window Zak of the long factorisation (FP64), first pass: with
// nu = k1 + d1 k2 and t = t2 + d2 t1,
//   x(r + Mi (j0 + p t)) = (1/d) sum_k1 exp(2 pi i k1 t1 / d1) V_k1(t2),
//   V_k1(t2) = exp(2 pi i k1 t2 / d) sum_k2 Z_{r,j0}(nu) exp(2 pi i k2 t2 / d2).
// This kernel forms V / d from the digit-reversed tables (one k1 and W
// residues r per work-group) into U[k1][t2][r + Mi j0]; the length-d1 inverse
// DFTs over k1 are a k_long_col pass.
template <int Unused = 0>
__global__ void __launch_bounds__(kThreads) k_long_zak_inv(const double2* z, double2* U, const double2* tw2,
                                                           const double2* twd, int Mi, int p, int d, int d1,
                                                           int d2, int W, int S, FftSched fs2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* tw = reinterpret_cast<double2*>(smem_raw);
  double2* xb = tw + d2;
  const int ncol = Mi * p;
  for (int e = threadIdx.x; e < d2; e += kThreads) tw[e] = tw2[e];
  const int k1 = blockIdx.x % d1, r0 = (blockIdx.x / d1) * W;
  for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
    const int cc = e / (p * d2), rem = e - cc * (p * d2), j0 = rem / d2, k2 = rem - j0 * d2, r = r0 + cc;
    xb[(cc * p + j0) * S + k2] =
        r < Mi ? z[((long long)r * p + j0) * d + (long long)k1 * d2 + k2] : make_double2(0, 0);
  }
  __syncthreads();
  fft_lds<double2, true, 8>(xb, S, fs2, W * p, tw);
  const double inv_d = 1.0 / d;
  double2* Ub = U + (long long)k1 * d2 * ncol;
  for (int e = threadIdx.x; e < W * p * d2; e += kThreads) {
    const int t2 = e / (W * p), rem = e - t2 * (W * p), j0 = rem / W, cc = rem - j0 * W, r = r0 + cc;
    if (r < Mi) {
      const double2 v = cmulc(xb[(cc * p + j0) * S + t2], twd[(long long)k1 * t2 % d]);
      Ub[(long long)t2 * ncol + r + Mi * j0] = cscale(v, inv_d);
    }
  }
}

// ----------------------------------------------------------------------------
// Middle pass of the window gradient (long columns).  grid (d1 ceil(Mp / W),
// B), Mp = Mi p window columns; block x = ub d1 + k1 handles the window
// columns u0 = ub W ... of spectral row k1.  For each n0 the signal column
// w = (u + n0 ai) mod Mp (first column pass in U) and the column (n0, w mod Mi)
// of h (first pass of the adjoint in V) are transformed over their second
// digit, and
//   acc(nu) += X_w(nu) conj(Y(nu)) exp(2 pi i k nu / d),  k = (u + n0 ai) div Mp,
// nu = k1 + d1 k2 (the window's Zak columns wrap into the next period); then
// the length-d2 inverse DFTs with the twiddle exp(2 pi i k1 t2 / d) and 1/d
// into G[k1][t2][u] (per signal [d1][d2 Mp]); a length-d1 inverse column pass
// finishes the gradient's polyphase columns.
// ----------------------------------------------------------------------------
template <typename C> struct LongGradArgs {
  const C* U;   // per signal [d1][d2 Mp]
  long long us;
  const C* V;   // per signal [q][d1][Mi d2]
  long long vs;
  C* G;         // per signal [d1][d2 Mp]
  long long gs;
  const C* twd;
  const C* tw2;
  int Mi, ai, p, q, d, d1, d2, W, Sd2;
  FftSched fs2;
};

template <typename C>
__global__ void __launch_bounds__(kThreads) k_long_mid_grad(LongGradArgs<C> A) {
  using T = decltype(C::x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int d1 = A.d1, d2 = A.d2, d = A.d, W = A.W, S = A.Sd2, Mi = A.Mi, Mp = A.Mi * A.p;
  C* xb = tw + d2;       // [W][S] signal spectra
  C* yb = xb + W * S;    // [W][S] spectra of h
  C* acc = yb + W * S;   // [W][S]
  for (int e = threadIdx.x; e < d2; e += kThreads) tw[e] = A.tw2[e];
  for (int e = threadIdx.x; e < W * S; e += kThreads) acc[e] = czero<C>();
  const int k1 = blockIdx.x % d1, u0 = (blockIdx.x / d1) * W;
  const long long bo = blockIdx.y;
  const C* Ub = A.U + bo * A.us + (long long)k1 * d2 * Mp;
  for (int n0 = 0; n0 < A.q; ++n0) {
    const C* Vb = A.V + bo * A.vs + ((long long)n0 * d1 + k1) * Mi * d2;
    __syncthreads();
    for (int e = threadIdx.x; e < W * d2; e += kThreads) {
      const int cc = e / d2, t = e - cc * d2, u = u0 + cc;
      C x = czero<C>(), y = czero<C>();
      if (u < Mp) {
        const int w = int((u + (long long)n0 * A.ai) % Mp);
        x = Ub[(long long)t * Mp + w];
        y = Vb[(long long)(w % Mi) * d2 + t];
      }
      xb[cc * S + t] = x;
      yb[cc * S + t] = y;
    }
    __syncthreads();
    fft_lds<C, false>(xb, S, A.fs2, 2 * W, tw);
    for (int e = threadIdx.x; e < W * d2; e += kThreads) {
      const int cc = e / d2, k2 = e - cc * d2, u = u0 + cc;
      if (u < Mp) {
        C pr = cmulc(xb[cc * S + k2], yb[cc * S + k2]);
        const long long k = (u + (long long)n0 * A.ai) / Mp;
        if (k) pr = cmulc(pr, A.twd[(k * (k1 + (long long)d1 * k2)) % d]);
        acc[cc * S + k2] = cadd(acc[cc * S + k2], pr);
      }
    }
  }
  __syncthreads();
  fft_lds<C, true>(acc, S, A.fs2, W, tw);
  const T inv_d = T(1) / T(d);
  C* Gb = A.G + bo * A.gs + (long long)k1 * d2 * Mp;
  for (int e = threadIdx.x; e < W * d2; e += kThreads) {
    const int t2 = e / W, cc = e - t2 * W, u = u0 + cc;
    if (u < Mp) Gb[(long long)t2 * Mp + u] = cscale(cmulc(acc[cc * S + t2], A.twd[((long long)t2 * k1) % d]), inv_d);
  }
}

}  // namespace dgtns
