// HIP kernels of the shear DGT (gfx950).
//
// Notation: the factorised separable DGT runs on the lattice with time step
// ai and Mi channels (Alg. 1: (a, M) when s0 = 0, (b_r, N_r) when s0 != 0),
// L = Mi * bi, c = gcd(ai, Mi), p = ai / c, q = Mi / c, d = bi / p, Ni = d q.
//
// Factorisation (the full-window algorithm of Section 4, derived from
// eq. (DGT) with lambda = 0).  Column r in Z_Mi of the signal is split into p
// polyphase sub-columns x(r + Mi (j0 + p t)), t in Z_d.  With X_{r,j0} their
// length-d DFTs and Zg_{u,j0} those of the window,
//   h_{n0 + q t'}(r) = sum_nu exp(2 pi i nu t'/d) sum_{j0} X_{r,j0}(nu)
//                       conj(Zg_{u,j0'}(nu)) exp(-2 pi i nu delta/d) / d,
// where r - n0 ai + Mi j0 = u + Mi (j0' + p delta), u in Z_Mi, j0' in Z_p,
// and c_r(m, n) = sum_r h_n(r) exp(-2 pi i r m / Mi).  The intermediate h is
// stored per signal as h[n0][r][t'] (t' fastest).  The plan stores
// Zc = conj(Zg) / d.  Kernel "cols" computes h (all q time offsets n0 of one
// block of W adjacent columns per work-group, the DFT of the signal columns
// kept in registers), kernel "rows" the channel DFT of each time position and
// the post-processing of Alg. 1.
#pragma once
#include "fft_core.hpp"

namespace dgtns {

// Largest batch of the list-batched forward call (per-signal pointers in the
// kernel arguments).
constexpr int kListMax = 16;

// a[i] for a work-group-uniform i, with constant indices only (a dynamic
// index into a by-value kernel argument would move the whole argument block
// to scratch memory)
template <typename T, int N> __device__ __forceinline__ T pick(const T (&a)[N], int i) {
  T r = a[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = i == k ? a[k] : r;
  return r;
}

template <typename C> struct ChirpSrc {
  const C* tab;   // pchirp values per sample (plan precision), or null
  long long K;    // s (L+1) mod 2L for exact on-the-fly FP64 evaluation when tab is null
  long long L;    // K == 0 and tab == null: identity
  int conj;       // multiply by the conjugate chirp
};

template <typename C> __device__ __forceinline__ C chirp_val(const ChirpSrc<C>& cs, long long l) {
  using T = decltype(C::x);
  if (cs.tab) return cs.tab[l];
  // exp(pi i r / L), r = K (l^2 mod 2L) mod 2L (Lemma 1), exact in integers
  const long long twoL = 2 * cs.L;
  const long long l2 = (l * l) % twoL;
  const long long r = (long long)(((unsigned long long)cs.K * (unsigned long long)l2) % (unsigned long long)twoL);
  return phase_pi(r, cs.L, T());
}

template <typename C> __device__ __forceinline__ C apply_chirp(const ChirpSrc<C>& cs, C v, long long l) {
  if (!cs.tab && cs.K == 0) return v;
  C p = chirp_val(cs, l);
  if (cs.conj) p = cconj(p);
  return cmul_comp(v, p);
}

// Streaming (non-temporal) accesses for the intermediate h, which is read
// once.  Stores stream only when the launch's h cannot stay in the 256 MB
// last-level cache anyway (hstream): a smaller h is re-read from that cache by
// the next kernel.  The element is moved as one native 2-vector.
template <typename T> struct NVec;
template <> struct NVec<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct NVec<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename C> __device__ __forceinline__ void st_stream(C* p, C v) {
  using T = decltype(C::x);
  typename NVec<T>::type w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<typename NVec<T>::type*>(p));
}
template <typename C> __device__ __forceinline__ void st_h(C* p, C v, int hstream) {
  if (hstream)
    st_stream(p, v);
  else
    *p = v;
}
// Signal output of the synthesis: complex, or the real part only (the
// real-signal variant's synthesis writes real samples).
template <typename C> __device__ __forceinline__ void st_out(C* y, long long idx, C v, int real_out) {
  using T = decltype(C::x);
  if (real_out)
    reinterpret_cast<T*>(y)[idx] = v.x;
  else
    y[idx] = v;
}

// Coefficient layout of a call.  Full: column n of a signal at n M, all M
// channels.  Real-signal variant (Section 4.4's real-signal entry point, for
// a real signal and window): a column whose offset w(n) is 0 or 1/2 is
// conjugate symmetric, c((-m - 2 w(n)) mod M, n) = conj(c(m, n)), and keeps
// channels 0 .. M/2 only; the other columns are kept whole.  w(n) depends on
// n mod lambda2, and the half columns are n = 0 and, for even lambda2,
// n = lambda2/2 (mod lambda2); the columns are grouped by n div lambda2 into
// rows of S values.
struct CoefLayout {
  int real;        // 1: real-signal layout
  int lam2, M, M2; // M2 = M/2 + 1
  long long S;     // values per group of lambda2 columns
};
// Offset of column n within a signal's coefficients; *cnt: its stored
// channels; *e: 2 w(n) of a half-stored column.
__device__ __forceinline__ long long coef_col(const CoefLayout& R, long long n, int* cnt, int* e) {
  if (!R.real) {
    *cnt = R.M;
    *e = 0;
    return n * R.M;
  }
  const long long j = n / R.lam2;
  const int k = int(n - j * R.lam2), h = R.lam2 >> 1;
  const bool even = (R.lam2 & 1) == 0;
  const bool half1 = even && k == h;
  *cnt = (k == 0 || half1) ? R.M2 : R.M;
  *e = half1 ? 1 : 0;
  const int before = (k > 0 ? 1 : 0) + (even && k > h ? 1 : 0);
  return j * R.S + (long long)k * R.M - (long long)(R.M - R.M2) * before;
}
// Channel m of a column at col (coef_col): stored, or the conjugate of the
// stored channel (-m - e) mod M.
template <typename C>
__device__ __forceinline__ C coef_load(const C* cb, int M, long long col, int cnt, int e, int m) {
  if (m < cnt) return cb[col + m];
  return cconj(cb[col + (M - m - e)]);
}

template <typename C> __device__ __forceinline__ C ld_stream(const C* p) {
  using T = decltype(C::x);
  const typename NVec<T>::type w = __builtin_nontemporal_load(reinterpret_cast<const typename NVec<T>::type*>(p));
  return mk<C>(w.x, w.y);
}

template <typename C> __device__ __forceinline__ C load_sig(const void* x, int real_in, long long idx) {
  using T = decltype(C::x);
  if (real_in) return mk<C>(reinterpret_cast<const T*>(x)[idx], T(0));
  return reinterpret_cast<const C*>(x)[idx];
}

// The NL samples x[xoff + li[i]] (zero where !ok[i]; li[i] is then 0) times
// the chirp at li[i]: every load of the thread is issued before the first is
// used, so their latencies overlap (the precision and chirp source are
// uniform per launch and tested once).
template <typename C, int NL>
__device__ __forceinline__ void load_chirped(const void* x, int real_in, long long xoff, const ChirpSrc<C>& ch,
                                             const long long (&li)[NL], const bool (&ok)[NL], C (&v)[NL]) {
  using T = decltype(C::x);
  if (real_in) {
    const T* xr = reinterpret_cast<const T*>(x) + xoff;
#pragma unroll
    for (int i = 0; i < NL; ++i) v[i] = mk<C>(ok[i] ? xr[li[i]] : T(0), T(0));
  } else {
    const C* xc = reinterpret_cast<const C*>(x) + xoff;
#pragma unroll
    for (int i = 0; i < NL; ++i) v[i] = ok[i] ? xc[li[i]] : czero<C>();
  }
  if (ch.tab) {
    C p[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) p[i] = ch.tab[li[i]];
#pragma unroll
    for (int i = 0; i < NL; ++i) v[i] = cmul_comp(v[i], ch.conj ? cconj(p[i]) : p[i]);
  } else if (ch.K) {
#pragma unroll
    for (int i = 0; i < NL; ++i) v[i] = apply_chirp(ch, v[i], li[i]);
  }
}

// XCD-aware order of a launch's x blocks: work-groups are dealt to the 8
// XCDs in turn by linear id, so with gridDim.x a multiple of 8 the x blocks
// of one XCD are those of one residue mod 8.  They get consecutive logical
// indices here, so neighbouring column blocks (which share cache lines of
// the signal and of h) run behind the same L2.
__device__ __forceinline__ int xcd_block_x() {
  const int G = gridDim.x, x = blockIdx.x;
  if (G & 7) return x;
  return (x & 7) * (G >> 3) + (x >> 3);
}

// exp(-2 pi i e / n) (sign = -1) or its conjugate, from a table or on the fly
template <typename C> __device__ __forceinline__ C root_at(const C* tab, long long e, long long n, int inv) {
  using T = decltype(C::x);
  C w;
  if (tab) {
    w = tab[e];
  } else {
    w = cconj(phase_pi(2 * e, n, T()));  // exp(-2 pi i e / n)
  }
  return inv ? cconj(w) : w;
}

// Window-Zak coefficient used by the factorisation for output column r, time
// offset n0 and polyphase index j0: Zc_{u,j0'}(nu) exp(-2 pi i nu delta / d).
template <typename C>
__device__ __forceinline__ C zc_coef(const C* zc, const C* tw, int r, int n0, int j0, int nu, int ai, int Mi,
                                     int p, int d) {
  const int v = r - n0 * ai + Mi * j0;  // in (-Mi p, Mi p)
  int u = v % Mi;
  if (u < 0) u += Mi;
  const int j1 = (v - u) / Mi;          // in [-p, p)
  int j0p = j1 % p;
  if (j0p < 0) j0p += p;
  C z = zc[((long long)u * p + j0p) * d + nu];
  if (j1 < 0) z = cmulc(z, tw[nu]);     // delta = -1: multiply by exp(+2 pi i nu / d)
  return z;
}

// ----------------------------------------------------------------------------
// Forward factorisation kernel ("cols").  grid (ceil(Mi/W), B), 512 threads.
// ----------------------------------------------------------------------------
template <typename C> struct ColArgs {
  const void* x;
  long long xs;
  int real_in;
  int list;                    // 1: signal k at xl[k] instead of x + k xs
  const void* xl[kListMax];
  ChirpSrc<C> chirp;
  const C* zc;                 // window tables: nw of zs values each
  C* H;
  long long hs;
  const C* twd;
  int Mi, ai, d, p, q, W, Sd;
  int qw;                      // time offsets per window (q = nw qw)
  long long zs;
  int hstream;                 // stream the h stores (st_h)
  int ht;                      // h[n0][t][r] layout (fast forward kernels only)
  int nsplit;                  // work-groups sharing one column block (split of Z_q)
  FftSched fd;
};

// Offset n0 in Z_q of the factorisation: window mu = n0 / qw (its table at
// zc + mu zs) and time offset n0 mod qw of that window's separable lattice.
// The shear algorithm has one window (qw = q).
template <typename C>
__device__ __forceinline__ const C* window_of(const C* zc, long long zs, int qw, int n0, int* n0w) {
  const int mu = n0 / qw;
  *n0w = n0 - mu * qw;
  return zc + mu * zs;
}

// Time position of intermediate row (n0, t'): n0 + q t' for the shear
// algorithm (qw = q, nw = 1); for the multiwindow algorithm (Prop. 5) the
// separable lattice of window mu = n0 / qw has position nt = n0 mod qw + qw t',
// which is coefficient column nt nw + mu.
__device__ __forceinline__ int row_time(int n0, int t, int qw, int nw) {
  const int mu = n0 / qw;
  return (n0 - mu * qw + qw * t) * nw + mu;
}

// Runtime-schedule factorisation: grid (ceil(Mi / W) * nsplit, B); the
// nsplit work-groups of a column block each compute the column DFTs and a
// share of the q offsets n0 (more work-groups for small batches).
template <typename C, bool GENP>
__global__ void __launch_bounds__(kThreads) k_fwd_cols(ColArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int d = A.d, p = GENP ? A.p : 1, W = A.W, Sd = A.Sd, Mi = A.Mi;
  C* xb = tw + d;
  C* yb = GENP ? xb + W * p * Sd : xb;
  for (int e = threadIdx.x; e < d; e += kThreads) tw[e] = A.twd[e];
  const int cb = blockIdx.x / A.nsplit, part = blockIdx.x - cb * A.nsplit;
  const int qper = (A.q + A.nsplit - 1) / A.nsplit;
  const int n0_begin = part * qper, n0_end = min(A.q, n0_begin + qper);
  const int r0 = cb * W;
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  const int b = p * d;
  const float rW = 1.0f / float(W), rd = 1.0f / float(d);   // W b, W d < 2^15
  batched_for<4, C>(
      threadIdx.x, W * b, kThreads,
      [&](int e) {
        const int j = qdiv(e, rW), cc = e - j * W, r = r0 + cc;
        C v = czero<C>();
        if (r < Mi) {
          const long long l = r + (long long)j * Mi;
          v = apply_chirp(A.chirp, load_sig<C>(xsrc, A.real_in, xoff + l), l);
        }
        return v;
      },
      [&](int e, C v) {
        const int j = qdiv(e, rW), cc = e - j * W;
        const int j0 = GENP ? j % p : 0, t = GENP ? j / p : j;
        xb[(cc * p + j0) * Sd + t] = v;
      });
  __syncthreads();
  fft_lds<C, false>(xb, Sd, A.fd, W * p, tw);
  const int WD = W * d;
  constexpr int KX = GENP ? 1 : MaxE<C>::value;
  C X[KX];
  if (!GENP) {
#pragma unroll
    for (int i = 0; i < KX; ++i) {
      const int e = threadIdx.x + i * kThreads;
      if (e < WD) {
        const int cc = qdiv(e, rd), nu = e - cc * d;
        X[i] = xb[cc * Sd + nu];
      }
    }
  }
  for (int n0 = n0_begin; n0 < n0_end; ++n0) {
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
    __syncthreads();
    if (!GENP) {
#pragma unroll
      for (int i = 0; i < KX; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < WD) {
          const int cc = qdiv(e, rd), nu = e - cc * d, r = r0 + cc;
          C y = czero<C>();
          if (r < Mi) {
            const int v = r - n0w * A.ai;
            C z;
            if (v >= 0) {
              z = zc[(long long)v * d + nu];
            } else {
              z = cmulc(zc[(long long)(v + Mi) * d + nu], tw[nu]);
            }
            y = cmul(X[i], z);
          }
          yb[cc * Sd + nu] = y;
        }
      }
    } else {
      for (int e = threadIdx.x; e < WD; e += kThreads) {
        const int cc = qdiv(e, rd), nu = e - cc * d, r = r0 + cc;
        C y = czero<C>();
        if (r < Mi) {
          for (int j0 = 0; j0 < p; ++j0)
            y = cadd(y, cmul(xb[(cc * p + j0) * Sd + nu], zc_coef(zc, tw, r, n0w, j0, nu, A.ai, Mi, p, d)));
        }
        yb[cc * Sd + nu] = y;
      }
    }
    __syncthreads();
    fft_lds<C, true>(yb, Sd, A.fd, W, tw);
    for (int e = threadIdx.x; e < WD; e += kThreads) {
      const int cc = qdiv(e, rd), t = e - cc * d, r = r0 + cc;
      if (r < Mi) st_h(A.H + bo * A.hs + ((long long)n0 * Mi + r) * d + t, yb[cc * Sd + t], A.hstream);
    }
  }
}

// ----------------------------------------------------------------------------
// Adjoint factorisation kernel: h*[Ni][Mi] -> signal domain.  Reverse of
// k_fwd_cols: per n0 a forward DFT over t' of the h* column, multiplied by
// conj of the window coefficient and accumulated per sub-column, then one
// unnormalised inverse DFT per sub-column and the conjugate chirp.
// ----------------------------------------------------------------------------
template <typename C> struct ColAdjArgs {
  const C* H;
  long long hs;
  const C* zc;
  const C* twd;
  ChirpSrc<C> chirp;
  C* y;
  long long ys;
  int Mi, ai, d, p, q, W, Sd;
  int qw;                      // time offsets per window (q = nw qw), tables zs apart
  long long zs;
  FftSched fd;
  int real_out;                // write the real part of y only (real samples)
};

// Factorisation for p = 1 and any 7-smooth d <= 64 MV, one column per
// wavefront: the 8 columns of a work-group arrive through one coalesced LDS
// tile, after which each wavefront transforms its own column in place
// (fft_wave_rt) with no further work-group barrier.  The column spectrum
// stays in registers (MV values per lane) across the q window products.
// TWL: the twiddle table is copied into LDS after the tile (when it fits).
// NW: wavefronts (columns) per work-group.
// grid (ceil(Mi / NW) * nsplit, B), 64 NW threads.
template <typename C, int MV, bool TWL, int NW = kThreads / 64>
__global__ void __launch_bounds__(64 * NW) k_fwd_cols_wr(ColArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  constexpr int W = NW, NT = 64 * NW;
  const int d = A.d, Sd = A.Sd, Mi = A.Mi;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int cb = blockIdx.x / A.nsplit, part = blockIdx.x - cb * A.nsplit;
  const int qper = (A.q + A.nsplit - 1) / A.nsplit;
  const int n0_begin = part * qper, n0_end = min(A.q, n0_begin + qper);
  const int r0 = cb * W;
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  batched_for<4, C>(
      tid, W * d, NT,
      [&](int e) {
        const int t = e / W, cc = e - t * W, r = r0 + cc;
        C v = czero<C>();
        if (r < Mi) {
          const long long l = r + (long long)t * Mi;
          v = apply_chirp(A.chirp, load_sig<C>(xsrc, A.real_in, xoff + l), l);
        }
        return v;
      },
      [&](int e, C v) {
        const int t = e / W, cc = e - t * W;
        lds[cc * Sd + t] = v;
      });
  const C* twl = A.twd;
  if constexpr (TWL) {
    C* t = lds + W * Sd;
    for (int e = tid; e < d; e += NT) t[e] = A.twd[e];
    twl = t;
  }
  __syncthreads();
  const int r = r0 + wave;
  const int rr = r < Mi ? r : 0;
  C* buf = lds + wave * Sd;
  fft_wave_rt<C, false, MV>(buf, A.fd, twl, lane);
  C X[MV];
#pragma unroll
  for (int e = 0; e < MV; ++e) {
    const int nu = lane + 64 * e;
    X[e] = nu < d ? buf[nu] : czero<C>();
  }
  for (int n0 = n0_begin; n0 < n0_end; ++n0) {
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
    const int v0 = rr - n0w * A.ai;
    const C* zrow = zc + (long long)(v0 >= 0 ? v0 : v0 + Mi) * d;
#pragma unroll
    for (int e = 0; e < MV; ++e) {
      const int nu = lane + 64 * e;
      if (nu < d) {
        C z = zrow[nu];
        if (v0 < 0) z = cmulc(z, twl[nu]);
        buf[nu] = cmul(X[e], z);
      }
    }
    fft_wave_rt<C, true, MV>(buf, A.fd, twl, lane);
    if (r < Mi) {
      C* hb = A.H + bo * A.hs + ((long long)n0 * Mi + r) * d;
#pragma unroll
      for (int e = 0; e < MV; ++e) {
        const int t = lane + 64 * e;
        if (t < d) st_h(hb + t, buf[t], A.hstream);
      }
    }
  }
}

template <typename C, bool GENP>
__global__ void __launch_bounds__(kThreads) k_adj_cols(ColAdjArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int d = A.d, p = GENP ? A.p : 1, W = A.W, Sd = A.Sd, Mi = A.Mi;
  C* xb = tw + d;
  // p = 1 accumulates in registers and fills xb only after the loop over n0,
  // so the h columns can take the same LDS
  C* yb = GENP ? xb + W * p * Sd : xb;
  for (int e = threadIdx.x; e < d; e += kThreads) tw[e] = A.twd[e];
  const int r0 = blockIdx.x * W;
  const long long bo = blockIdx.y;
  const int WD = W * d;
  const float rW = 1.0f / float(W), rd = 1.0f / float(d);   // W p d < 2^15
  constexpr int KX = GENP ? 1 : MaxE<C>::value;
  C acc[KX];
#pragma unroll
  for (int i = 0; i < KX; ++i) acc[i] = czero<C>();
  if (GENP)
    for (int e = threadIdx.x; e < W * p * Sd; e += kThreads) xb[e] = czero<C>();
  for (int n0 = 0; n0 < A.q; ++n0) {
    __syncthreads();
    batched_for<4, C>(
        threadIdx.x, WD, kThreads,
        [&](int e) {
          const int cc = qdiv(e, rd), t = e - cc * d, r = r0 + cc;
          return r < Mi ? A.H[bo * A.hs + ((long long)n0 * Mi + r) * d + t] : czero<C>();
        },
        [&](int e, C v) {
          const int cc = qdiv(e, rd), t = e - cc * d;
          yb[cc * Sd + t] = v;
        });
    __syncthreads();
    fft_lds<C, false>(yb, Sd, A.fd, W, tw);
    int n0w;
    const C* zc = window_of(A.zc, A.zs, A.qw, n0, &n0w);
    if (!GENP) {
#pragma unroll
      for (int i = 0; i < KX; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < WD) {
          const int cc = qdiv(e, rd), nu = e - cc * d, r = r0 + cc;
          if (r < Mi) {
            const int v = r - n0w * A.ai;
            C z;
            if (v >= 0) {
              z = zc[(long long)v * d + nu];
            } else {
              z = cmulc(zc[(long long)(v + Mi) * d + nu], tw[nu]);
            }
            acc[i] = cadd(acc[i], cmulc(yb[cc * Sd + nu], z));
          }
        }
      }
    } else {
      for (int e = threadIdx.x; e < WD; e += kThreads) {
        const int cc = qdiv(e, rd), nu = e - cc * d, r = r0 + cc;
        if (r < Mi) {
          const C yv = yb[cc * Sd + nu];
          for (int j0 = 0; j0 < p; ++j0) {
            C& a = xb[(cc * p + j0) * Sd + nu];
            a = cadd(a, cmulc(yv, zc_coef(zc, tw, r, n0w, j0, nu, A.ai, Mi, p, d)));
          }
        }
      }
    }
  }
  __syncthreads();
  if (!GENP) {
#pragma unroll
    for (int i = 0; i < KX; ++i) {
      const int e = threadIdx.x + i * kThreads;
      if (e < WD) {
        const int cc = qdiv(e, rd), nu = e - cc * d;
        xb[cc * Sd + nu] = acc[i];
      }
    }
    __syncthreads();
  }
  fft_lds<C, true>(xb, Sd, A.fd, W * p, tw);
  const int b = p * d;
  for (int e = threadIdx.x; e < W * b; e += kThreads) {
    const int j = qdiv(e, rW), cc = e - j * W, r = r0 + cc;
    if (r < Mi) {
      const long long l = r + (long long)j * Mi;
      const int j0 = GENP ? j % p : 0, t = GENP ? j / p : j;
      st_out(A.y, bo * A.ys + l, apply_chirp(A.chirp, xb[(cc * p + j0) * Sd + t], l), A.real_out);
    }
  }
}

// ----------------------------------------------------------------------------
// Row kernels: channel DFT per time position plus the post-processing of
// Alg. 1, and the adjoint.  A work-group handles the R time positions
// n = n0 + q (t0 + i), i in Z_R (n0 = blockIdx.x mod q), whose intermediate
// values h[n0][r][t0 + i] are contiguous in i.  grid (q ceil(d/R), B), 512
// threads.
//   MODE 0 (s0 = 0): c((m + rho_n) mod M, n) = E_n c_r(m, n), tables E, rho.
//   MODE 1 (s0 != 0): row = inner position m in Z_{M_r}, FFT over the N_r
//     inner channels k'; with k = -k' mod N_r,
//       sq = C1 k + C2 m mod 2N,
//       E  = exp(pi i ((C3 sq^2 - m (C4 m + C5 k)) mod 2N) / N),
//       m~ = C1 k + C2 m mod N (time position of c),
//       k~ = floor(((-s1 a_r k + C6 m) mod L) / b) (channel of c),
//     and c(k~, m~) = E c_r(k', m).
// ----------------------------------------------------------------------------
template <typename C> struct RowArgs {
  const C* H;
  long long hs;
  C* c;
  long long cs;
  const C* twm;
  const C* postE;
  const int* rho;
  int list;                    // forward: coefficients of signal k at cl[k] instead of c + k cs
  C* cl[kListMax];
  int Mi, Ni, R, Sm, q, d;
  int qw, nw;                  // time offsets per window, windows (row_time)
  int hstream;                 // stream the stores: h (adjoint) or the coefficients (forward)
  int ht;                      // h[n0][t][r] layout (fast forward kernels only)
  FftSched fm;
  long long N, L, b, M, K1, K2, K3, K4, K5, C1n, C2n, Kt1, Kt6;
  // floor((2^64 - 1) / m) for the moduli 2N, N, L and the divisor b (Barrett)
  unsigned long long mu2N, muN, muL, mub;
  CoefLayout lay;              // coefficient layout (c, cs and cl follow it)
};

// x mod m for any 64-bit x by Barrett reduction with mu = floor((2^64 - 1) /
// m), m >= 1: q = floor(x mu / 2^64) is floor(x / m) or at most 2 below it,
// so r = x - q m needs at most two corrections.  A few 32-bit products
// instead of a 64-bit integer division.
__device__ __forceinline__ unsigned long long mod_b(unsigned long long x, unsigned long long m,
                                                    unsigned long long mu) {
  const unsigned long long q = __umul64hi(x, mu);
  unsigned long long r = x - q * m;
  if (r >= m) r -= m;
  if (r >= m) r -= m;
  return r;
}
// floor(x / m) by the same reduction
__device__ __forceinline__ unsigned long long div_b(unsigned long long x, unsigned long long m,
                                                    unsigned long long mu) {
  unsigned long long q = __umul64hi(x, mu);
  unsigned long long r = x - q * m;
  if (r >= m) { r -= m; ++q; }
  if (r >= m) ++q;
  return q;
}

// Frequency-shear post-processing of Alg. 1 for intermediate position m and
// channel k: the phase *E and the coefficient's time position *nt and
// channel *kt.
template <typename C>
__device__ __forceinline__ void shear_map(const RowArgs<C>& A, long long m, long long k, long long* nt,
                                          long long* kt, C* E) {
  using T = decltype(C::x);
  // every constant is reduced into [0, modulus) on the host and m, k are
  // non-negative, so each product below stays under 2^63
  using U = unsigned long long;
  const U twoN = U(2 * A.N), um = U(m), uk = U(k);
  const U sq = mod_b(U(A.K1) * uk + U(A.K2) * um, twoN, A.mu2N);
  const U sq2 = mod_b(sq * sq, twoN, A.mu2N);
  const U e1 = mod_b(U(A.K3) * sq2, twoN, A.mu2N);
  const U inner = mod_b(U(A.K4) * um + U(A.K5) * uk, twoN, A.mu2N);
  const U mi = mod_b(um * inner, twoN, A.mu2N);
  const long long e = (long long)(e1 >= mi ? e1 - mi : e1 + twoN - mi);
  *E = phase_pi(e, A.N, T());
  *nt = (long long)mod_b(U(A.C1n) * uk + U(A.C2n) * um, U(A.N), A.muN);
  *kt = (long long)div_b(mod_b(U(A.Kt1) * uk + U(A.Kt6) * um, U(A.L), A.muL), U(A.b), A.mub);
}

template <typename C, int MODE>
__global__ void __launch_bounds__(kThreads) k_fwd_rows(RowArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int Mi = A.Mi, R = A.R, Sm = A.Sm;
  C* buf = tw + Mi;
  for (int e = threadIdx.x; e < Mi; e += kThreads) tw[e] = A.twm[e];
  const int q = A.q, d = A.d, n0 = blockIdx.x % q, t0 = (blockIdx.x / q) * R;
  const long long bo = blockIdx.y;
  const C* Hb = A.H + bo * A.hs + (long long)n0 * Mi * d + t0;
  for (int e = threadIdx.x; e < R * Mi; e += kThreads) {
    const int m = e / R, i = e - m * R;
    buf[i * Sm + m] = t0 + i < d ? Hb[(long long)m * d + i] : czero<C>();
  }
  __syncthreads();
  fft_lds<C, false>(buf, Sm, A.fm, R, tw);
  C* cb = A.list ? pick(A.cl, int(bo)) : A.c + bo * A.cs;
  for (int e = threadIdx.x; e < R * Mi; e += kThreads) {
    const int row = e / Mi, mo = e - row * Mi;
    if (t0 + row >= d) continue;
    const int n = row_time(n0, t0 + row, A.qw, A.nw);
    if (MODE == 0) {
      int cnt, ee;
      const long long col = coef_col(A.lay, n, &cnt, &ee);
      if (mo >= cnt) continue;
      int mi = mo - A.rho[n];
      if (mi < 0) mi += Mi;
      st_h(cb + col + mo, cmul(A.postE[n], buf[row * Sm + mi]), A.hstream);
    } else {
      const long long k = mo == 0 ? 0 : Mi - mo;
      long long nt, kt;
      C E;
      shear_map(A, n, k, &nt, &kt, &E);
      int cnt, ee;
      const long long col = coef_col(A.lay, nt, &cnt, &ee);
      if (kt < cnt) st_h(cb + col + kt, cmul(E, buf[row * Sm + mo]), A.hstream);
    }
  }
}

template <typename C, int MODE>
__global__ void __launch_bounds__(kThreads) k_adj_rows(RowArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int Mi = A.Mi, R = A.R, Sm = A.Sm;
  C* buf = tw + Mi;
  for (int e = threadIdx.x; e < Mi; e += kThreads) tw[e] = A.twm[e];
  const int q = A.q, d = A.d, n0 = blockIdx.x % q, t0 = (blockIdx.x / q) * R;
  const long long bo = blockIdx.y;
  const C* cb = A.c + bo * A.cs;
  for (int e = threadIdx.x; e < R * Mi; e += kThreads) {
    const int row = e / Mi, m = e - row * Mi;
    C v = czero<C>();
    if (t0 + row < d) {
      const int n = row_time(n0, t0 + row, A.qw, A.nw);
      if (MODE == 0) {
        int mo = m + A.rho[n];
        if (mo >= Mi) mo -= Mi;
        int cnt, ee;
        const long long col = coef_col(A.lay, n, &cnt, &ee);
        v = cmulc(coef_load(cb, Mi, col, cnt, ee, mo), A.postE[n]);
      } else {
        const long long k = m == 0 ? 0 : Mi - m;
        long long nt, kt;
        C E;
        shear_map(A, n, k, &nt, &kt, &E);
        int cnt, ee;
        const long long col = coef_col(A.lay, nt, &cnt, &ee);
        v = cmulc(coef_load(cb, int(A.M), col, cnt, ee, int(kt)), E);
      }
    }
    buf[row * Sm + m] = v;
  }
  __syncthreads();
  fft_lds<C, true>(buf, Sm, A.fm, R, tw);
  C* Hb = const_cast<C*>(A.H) + bo * A.hs + (long long)n0 * Mi * d + t0;
  for (int e = threadIdx.x; e < R * Mi; e += kThreads) {
    const int m = e / R, i = e - m * R;
    if (t0 + i < d) st_h(Hb + (long long)m * d + i, buf[i * Sm + m], A.hstream);
  }
}

// ----------------------------------------------------------------------------
// Two-pass transform of length L = L1 L2 (frequency shear).  Column pass:
// transform along the row index of an [n][ncols] array, W adjacent columns per
// work-group, with a pre-multiplication (chirp) and the inter-pass twiddle
// exp(-+ 2 pi i k col / L).  Row pass: transform along contiguous rows of an
// [nrows][n] array and store transposed, out[k nrows + row], with a
// post-multiplication and a scale.
// ----------------------------------------------------------------------------
template <typename C> struct ColFftArgs {
  const void* x;
  long long xs;
  int real_in;
  int list;
  const void* xl[kListMax];
  C* y;
  long long ys;
  ChirpSrc<C> pre;
  const C* twL;   // length-L table exp(-2 pi i e / L) or null (on the fly)
  long long L;
  const C* tws;   // length-n stage twiddles
  int n, ncols, W, Sn;
  FftSched fs;
};

template <typename C, bool INV>
__global__ void __launch_bounds__(kThreads) k_col_fft(ColFftArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int n = A.n, W = A.W, Sn = A.Sn, nc = A.ncols;
  C* buf = tw + n;
  for (int e = threadIdx.x; e < n; e += kThreads) tw[e] = A.tws[e];
  const int c0 = blockIdx.x * W;
  const long long bo = blockIdx.y;
  const void* xsrc = A.list ? pick(A.xl, int(bo)) : A.x;
  const long long xoff = A.list ? 0 : bo * A.xs;
  batched_for<4, C>(
      threadIdx.x, W * n, kThreads,
      [&](int e) {
        const int j = e / W, cc = e - j * W, col = c0 + cc;
        C v = czero<C>();
        if (col < nc) {
          const long long idx = (long long)j * nc + col;
          v = apply_chirp(A.pre, load_sig<C>(xsrc, A.real_in, xoff + idx), idx);
        }
        return v;
      },
      [&](int e, C v) {
        const int j = e / W, cc = e - j * W;
        buf[cc * Sn + j] = v;
      });
  __syncthreads();
  fft_lds<C, INV>(buf, Sn, A.fs, W, tw);
  for (int e = threadIdx.x; e < W * n; e += kThreads) {
    const int k = e / W, cc = e - k * W, col = c0 + cc;
    if (col < nc) {
      const long long ex = (long long)k * col;   // k < n, col < ncols, n ncols = L: below L
      A.y[bo * A.ys + (long long)k * nc + col] = cmul(buf[cc * Sn + k], root_at(A.twL, ex, A.L, INV ? 1 : 0));
    }
  }
}

template <typename C> struct RowFftArgs {
  const C* x;
  long long xs;
  C* y;
  long long ys;
  ChirpSrc<C> post;
  decltype(C::x) scale;
  const C* tws;
  int n, nrows, R, Sn;
  FftSched fs;
  int real_out;   // write the real part of y only (real samples)
};

template <typename C, bool INV>
__global__ void __launch_bounds__(kThreads) k_row_fft(RowFftArgs<C> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  const int n = A.n, R = A.R, Sn = A.Sn, nr = A.nrows;
  C* buf = tw + n;
  for (int e = threadIdx.x; e < n; e += kThreads) tw[e] = A.tws[e];
  const int row0 = blockIdx.x * R;
  const long long bo = blockIdx.y;
  const float rn = 1.0f / float(n);   // R n < 2^15
  batched_for<4, C>(
      threadIdx.x, R * n, kThreads,
      [&](int e) {
        const int rr = qdiv(e, rn), j = e - rr * n, row = row0 + rr;
        return row < nr ? A.x[bo * A.xs + (long long)row * n + j] : czero<C>();
      },
      [&](int e, C v) {
        const int rr = qdiv(e, rn), j = e - rr * n;
        buf[rr * Sn + j] = v;
      });
  __syncthreads();
  fft_lds<C, INV>(buf, Sn, A.fs, R, tw);
  for (int e = threadIdx.x; e < R * n; e += kThreads) {
    const int k = e / R, rr = e - k * R, row = row0 + rr;
    if (row < nr) {
      const long long idx = (long long)k * nr + row;
      st_out(A.y, bo * A.ys + idx, cscale(apply_chirp(A.post, buf[rr * Sn + k], idx), A.scale), A.real_out);
    }
  }
}

// ----------------------------------------------------------------------------
// Window Zak transform (FP64 in; plan precision conj(Z)/d and/or FP64 Z out).
// ----------------------------------------------------------------------------
template <typename CO> struct ZakArgs {
  const double2* x;
  ChirpSrc<double2> chirp;
  // source sample l is exp(pi i (mod2 l mod 2L) / L) x[(l - shift) mod L]
  // (coset window of the multiwindow algorithm; shift = mod2 = 0 otherwise)
  long long L, shift, mod2;
  CO* zc;
  double2* z64;
  const double2* twd;
  int Mi, d, p, W, Sd;
  FftSched fd;
};

template <typename CO>
__global__ void __launch_bounds__(kThreads) k_zak_fwd(ZakArgs<CO> A) {
  using TO = decltype(CO::x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* tw = reinterpret_cast<double2*>(smem_raw);
  const int d = A.d, p = A.p, W = A.W, Sd = A.Sd, Mi = A.Mi;
  double2* xb = tw + d;
  for (int e = threadIdx.x; e < d; e += kThreads) tw[e] = A.twd[e];
  const int r0 = blockIdx.x * W;
  const int b = p * d;
  for (int e = threadIdx.x; e < W * b; e += kThreads) {
    const int j = e / W, cc = e - j * W, r = r0 + cc;
    double2 v = make_double2(0, 0);
    if (r < Mi) {
      const long long l = r + (long long)j * Mi;
      if (A.shift == 0 && A.mod2 == 0) {
        v = apply_chirp(A.chirp, A.x[l], l);
      } else {
        long long ls = l - A.shift;
        if (ls < 0) ls += A.L;
        const long long e = (long long)(((unsigned long long)A.mod2 * (unsigned long long)l) %
                                        (unsigned long long)(2 * A.L));
        v = cmul(A.x[ls], phase_pi(e, A.L, 0.0));
      }
    }
    xb[(cc * p + j % p) * Sd + j / p] = v;
  }
  __syncthreads();
  // at most MaxE * kThreads values per transform call (4096 in FP64)
  const int per = (MaxE<double2>::value * kThreads) / d;
  for (int t0 = 0; t0 < W * p; t0 += per) fft_lds<double2, false>(xb + t0 * Sd, Sd, A.fd, min(per, W * p - t0), tw);
  const double inv_d = 1.0 / d;
  for (int e = threadIdx.x; e < W * b; e += kThreads) {
    const int cc = e / b, rem = e - cc * b, j0 = rem / d, nu = rem - j0 * d, r = r0 + cc;
    if (r < Mi) {
      const double2 z = xb[(cc * p + j0) * Sd + nu];
      const long long o = ((long long)r * p + j0) * d + nu;
      if (A.zc) A.zc[o] = mk<CO>(TO(z.x * inv_d), TO(-z.y * inv_d));
      if (A.z64) A.z64[o] = z;
    }
  }
}

// Inverse window Zak (FP64): x(r + Mi (j0 + p t)) = (1/d) sum_nu Z_{r,j0}(nu) exp(2 pi i nu t / d),
// followed by a chirp multiplication.
struct ZakInvArgs {
  const double2* z;
  ChirpSrc<double2> chirp;
  double2* x;
  const double2* twd;
  int Mi, d, p, W, Sd;
  FftSched fd;
};

template <int Unused = 0>
__global__ void __launch_bounds__(kThreads) k_zak_inv(ZakInvArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* tw = reinterpret_cast<double2*>(smem_raw);
  const int d = A.d, p = A.p, W = A.W, Sd = A.Sd, Mi = A.Mi;
  double2* xb = tw + d;
  for (int e = threadIdx.x; e < d; e += kThreads) tw[e] = A.twd[e];
  const int r0 = blockIdx.x * W;
  const int b = p * d;
  for (int e = threadIdx.x; e < W * b; e += kThreads) {
    const int cc = e / b, rem = e - cc * b, j0 = rem / d, nu = rem - j0 * d, r = r0 + cc;
    xb[(cc * p + j0) * Sd + nu] = r < Mi ? A.z[((long long)r * p + j0) * d + nu] : make_double2(0, 0);
  }
  __syncthreads();
  // at most MaxE * kThreads values per transform call (4096 in FP64)
  const int per = (MaxE<double2>::value * kThreads) / d;
  for (int t0 = 0; t0 < W * p; t0 += per) fft_lds<double2, true>(xb + t0 * Sd, Sd, A.fd, min(per, W * p - t0), tw);
  const double inv_d = 1.0 / d;
  for (int e = threadIdx.x; e < W * b; e += kThreads) {
    const int j = e / W, cc = e - j * W, r = r0 + cc;
    if (r < Mi) {
      const long long l = r + (long long)j * Mi;
      A.x[l] = apply_chirp(A.chirp, cscale(xb[(cc * p + j % p) * Sd + j / p], inv_d), l);
    }
  }
}

// ----------------------------------------------------------------------------
// Canonical dual and tight windows in the Zak domain (p = 1): the frame
// operator of the separable system is diagonal there with entries
//   D(u, nu) = Mi sum_{n0 in Z_q} |Zg_{(u - n0 ai) mod Mi}(nu)|^2,
// so the dual S^{-1} g has Zak Zg / D and the tight window S^{-1/2} g has
// Zak Zg / sqrt(D) (tight != 0).  Each block also writes its min and max of D.
// ----------------------------------------------------------------------------
template <int Unused = 0>
__global__ void __launch_bounds__(kThreads) k_dual_div(const double2* z, double2* zd, double* part, int Mi, int d,
                                                      int ai, int q, double scale_bounds, int tight) {
  __shared__ double smin[kThreads], smax[kThreads];
  const long long tot = (long long)Mi * d;
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  double mn = 1e308, mx = 0;
  if (i < tot) {
    const int u = int(i / d), nu = int(i - (long long)u * d);
    double D = 0;
    for (int n0 = 0; n0 < q; ++n0) {
      int uu = u - n0 * ai;
      uu %= Mi;
      if (uu < 0) uu += Mi;
      const double2 v = z[(long long)uu * d + nu];
      D += v.x * v.x + v.y * v.y;
    }
    D *= Mi;
    const double2 v = z[i];
    const double den = tight ? sqrt(D) : D;
    zd[i] = D > 0 ? make_double2(v.x / den, v.y / den) : make_double2(0, 0);
    mn = D * scale_bounds;
    mx = D * scale_bounds;
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

// ----------------------------------------------------------------------------
// Canonical dual and tight windows for p > 1 of the sheared lattice.  In the
// Zak domain the analysis operator takes the p values Zf_{r,j0}(nu), j0 in
// Z_p, of a signal to its q coefficients at (r, nu) through the q x p matrix
//   A(n0, j0) = conj(Zg_{u,j1 mod p}(nu)) / d,  u + Mi j1 = r - n0 ai + Mi j0,
// times exp(2 pi i nu / d) where j1 < 0 (the index wraps one period of the
// window's polyphase sequence), so the frame operator is block diagonal with
// p x p blocks S(r, nu) = Mi d^2 A^H A; for p = 1 this is the scalar D of
// k_dual_div.  The dual window has Zak S^{-1} Zg, the tight window S^{-1/2} Zg
// (Section 4.2), and the optimal frame bounds are the extreme eigenvalues of
// the blocks.  Each thread diagonalises one Hermitian block by cyclic Jacobi
// rotations; eigenvalues that are not positive (no frame) contribute zero.
// d2 != 0: the tables are those of the long factorisation (digit-reversed).
// ----------------------------------------------------------------------------
constexpr int kDualMaxP = 8;

template <int PM>
__global__ void __launch_bounds__(kThreads) k_dual_block(const double2* z, double2* zd, double* part, int Mi, int d,
                                                        int p, int ai, int q, double scale_bounds, int tight,
                                                        int d2) {
  __shared__ double smin[kThreads], smax[kThreads];
  const long long tot = (long long)Mi * d;
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  double mn = 1e308, mx = 0;
  if (i < tot) {
    const int r = int(i / d), nu = int(i - (long long)r * d);
    double2 S[PM][PM], V[PM][PM];
    for (int j = 0; j < p; ++j)
      for (int k = 0; k < p; ++k) {
        S[j][k] = make_double2(0, 0);
        V[j][k] = make_double2(j == k ? 1.0 : 0.0, 0);
      }
    // tables of the long factorisation hold nu = k1 + d1 k2 at k1 d2 + k2
    const int nut = d2 ? nu / d2 + (d / d2) * (nu % d2) : nu;
    double sw, cw;
    sincospi(2.0 * nut / d, &sw, &cw);
    const double2 wrap = make_double2(cw, sw);
    // S = Mi d^2 A^H A = Mi sum_{n0} conj(a) a^T with a = d A(n0, .)
    for (int n0 = 0; n0 < q; ++n0) {
      double2 row[PM];
      for (int j0 = 0; j0 < p; ++j0) {
        const long long v = r - (long long)n0 * ai + (long long)Mi * j0;
        long long u = v % Mi;
        if (u < 0) u += Mi;
        const long long j1 = (v - u) / Mi;
        const long long jp = ((j1 % p) + p) % p;
        double2 t = z[(u * p + jp) * d + nu];
        t.y = -t.y;
        if (j1 < 0) t = cmul(t, wrap);
        row[j0] = t;
      }
      for (int j = 0; j < p; ++j)
        for (int k = 0; k < p; ++k) {
          const double2 a = row[j], b = row[k];
          S[j][k].x += a.x * b.x + a.y * b.y;   // conj(a) b
          S[j][k].y += a.x * b.y - a.y * b.x;
        }
    }
    for (int j = 0; j < p; ++j)
      for (int k = 0; k < p; ++k) S[j][k] = cscale(S[j][k], double(Mi));
    // cyclic Jacobi: S <- U^H S U, V <- V U, U = diag(1, conj(e)) R(c, s) on (j, k)
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0, dia = 0;
      for (int j = 0; j < p; ++j) {
        dia += S[j][j].x * S[j][j].x;
        for (int k = j + 1; k < p; ++k) off += S[j][k].x * S[j][k].x + S[j][k].y * S[j][k].y;
      }
      if (off <= 1e-32 * dia) break;
      for (int j = 0; j < p - 1; ++j)
        for (int k = j + 1; k < p; ++k) {
          const double2 h = S[j][k];
          const double ah = hypot(h.x, h.y);
          if (ah == 0) continue;
          const double2 e = make_double2(h.x / ah, h.y / ah);
          const double2 ec = make_double2(e.x, -e.y);
          const double tau = (S[k][k].x - S[j][j].x) / (2 * ah);
          const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
          const double c = 1 / sqrt(1 + t * t), s = t * c;
          for (int m = 0; m < p; ++m) {   // columns j, k
            const double2 x = S[m][j], y = cmul(S[m][k], ec);
            S[m][j] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
            S[m][k] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
            const double2 vx = V[m][j], vy = cmul(V[m][k], ec);
            V[m][j] = make_double2(c * vx.x - s * vy.x, c * vx.y - s * vy.y);
            V[m][k] = make_double2(s * vx.x + c * vy.x, s * vx.y + c * vy.y);
          }
          for (int m = 0; m < p; ++m) {   // rows j, k
            const double2 x = S[j][m], y = cmul(S[k][m], e);
            S[j][m] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
            S[k][m] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
          }
          S[j][k] = make_double2(0, 0);
          S[k][j] = make_double2(0, 0);
          S[j][j].y = 0;
          S[k][k].y = 0;
        }
    }
    // out = V diag(lambda^-1 or lambda^-1/2) V^H Zg(r, ., nu)
    double2 w[PM];
    for (int k = 0; k < p; ++k) {
      double2 acc = make_double2(0, 0);
      for (int j = 0; j < p; ++j) {
        const double2 vj = V[j][k], g = z[((long long)r * p + j) * d + nu];
        acc.x += vj.x * g.x + vj.y * g.y;   // conj(V) g
        acc.y += vj.x * g.y - vj.y * g.x;
      }
      const double lam = S[k][k].x;
      mn = fmin(mn, fmax(lam, 0.0) * scale_bounds);
      mx = fmax(mx, lam * scale_bounds);
      const double f = lam > 0 ? (tight ? 1 / sqrt(lam) : 1 / lam) : 0.0;
      w[k] = cscale(acc, f);
    }
    for (int j = 0; j < p; ++j) {
      double2 acc = make_double2(0, 0);
      for (int k = 0; k < p; ++k) {
        const double2 t = cmul(V[j][k], w[k]);
        acc.x += t.x;
        acc.y += t.y;
      }
      zd[((long long)r * p + j) * d + nu] = acc;
    }
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

// ----------------------------------------------------------------------------
// The same dual and tight windows for 8 < p <= kDualLdsMaxP: one wavefront per
// (r, nu) block (grid-stride over the blocks), the Hermitian block S and its
// eigenvectors V in LDS.  The cyclic Jacobi rotations are those of
// k_dual_block; each one changes two columns, then two rows, of S (and two
// columns of V), and lane m updates the entries of row (column) m, so the
// lanes apply one rotation together.  part receives one (min, max) pair per
// work-group.
// ----------------------------------------------------------------------------
constexpr int kDualLdsMaxP = 64;
constexpr int kDualLdsGroups = 8192;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int Unused = 0>
__global__ void __launch_bounds__(64) k_dual_block_lds(const double2* z, double2* zd, double* part, int Mi, int d,
                                                       int p, int ai, int q, double scale_bounds, int tight,
                                                       int d2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* S = reinterpret_cast<double2*>(smem_raw);   // [p][p]
  double2* V = S + p * p;                               // [p][p]
  __shared__ double2 vec[kDualLdsMaxP];
  __shared__ double2 rot[2];                            // (c, s), e
  const int m = threadIdx.x;
  const long long tot = (long long)Mi * d;
  double mn = 1e308, mx = 0;
  for (long long i = blockIdx.x; i < tot; i += gridDim.x) {
    const int r = int(i / d), nu = int(i - (long long)r * d);
    const int nut = d2 ? nu / d2 + (d / d2) * (nu % d2) : nu;
    double sw, cw;
    sincospi(2.0 * nut / d, &sw, &cw);
    const double2 wrap = make_double2(cw, sw);
    __syncthreads();
    for (int e = m; e < p * p; e += 64) {
      S[e] = make_double2(0, 0);
      V[e] = make_double2(e / p == e % p ? 1.0 : 0.0, 0);
    }
    // S = Mi sum_{n0} conj(a) a^T with a = d A(n0, .); lane m owns row m
    for (int n0 = 0; n0 < q; ++n0) {
      __syncthreads();
      if (m < p) {
        const long long v = r - (long long)n0 * ai + (long long)Mi * m;
        long long u = v % Mi;
        if (u < 0) u += Mi;
        const long long j1 = (v - u) / Mi;
        const long long jp = ((j1 % p) + p) % p;
        double2 t = z[(u * p + jp) * d + nu];
        t.y = -t.y;
        if (j1 < 0) t = cmul(t, wrap);
        vec[m] = t;
      }
      __syncthreads();
      if (m < p) {
        const double2 a = vec[m];
        for (int k = 0; k < p; ++k) {
          const double2 b = vec[k];
          double2& sk = S[m * p + k];
          sk.x += Mi * (a.x * b.x + a.y * b.y);
          sk.y += Mi * (a.x * b.y - a.y * b.x);
        }
      }
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
      __syncthreads();
      double off = 0, dia = 0;
      if (m < p) {
        dia = S[m * p + m].x * S[m * p + m].x;
        for (int k = m + 1; k < p; ++k) off += S[m * p + k].x * S[m * p + k].x + S[m * p + k].y * S[m * p + k].y;
      }
      off = wave_sum(off);
      dia = wave_sum(dia);
      if (off <= 1e-32 * dia) break;
      for (int j = 0; j < p - 1; ++j)
        for (int k = j + 1; k < p; ++k) {
          __syncthreads();
          if (m == 0) {
            const double2 h = S[j * p + k];
            const double ah = hypot(h.x, h.y);
            double c = 1, sn = 0;
            double2 e = make_double2(1, 0);
            if (ah != 0) {
              e = make_double2(h.x / ah, h.y / ah);
              const double tau = (S[k * p + k].x - S[j * p + j].x) / (2 * ah);
              const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
              c = 1 / sqrt(1 + t * t);
              sn = t * c;
            }
            rot[0] = make_double2(c, sn);
            rot[1] = ah != 0 ? e : make_double2(0, 0);
          }
          __syncthreads();
          const double2 e = rot[1];
          if (e.x == 0 && e.y == 0) continue;   // uniform: S[j][k] is already zero
          const double c = rot[0].x, sn = rot[0].y;
          const double2 ec = make_double2(e.x, -e.y);
          if (m < p) {   // columns j, k of S and V
            const double2 x = S[m * p + j], y = cmul(S[m * p + k], ec);
            S[m * p + j] = make_double2(c * x.x - sn * y.x, c * x.y - sn * y.y);
            S[m * p + k] = make_double2(sn * x.x + c * y.x, sn * x.y + c * y.y);
            const double2 vx = V[m * p + j], vy = cmul(V[m * p + k], ec);
            V[m * p + j] = make_double2(c * vx.x - sn * vy.x, c * vx.y - sn * vy.y);
            V[m * p + k] = make_double2(sn * vx.x + c * vy.x, sn * vx.y + c * vy.y);
          }
          __syncthreads();
          if (m < p) {   // rows j, k of S
            const double2 x = S[j * p + m], y = cmul(S[k * p + m], e);
            S[j * p + m] = make_double2(c * x.x - sn * y.x, c * x.y - sn * y.y);
            S[k * p + m] = make_double2(sn * x.x + c * y.x, sn * x.y + c * y.y);
          }
          __syncthreads();
          if (m == 0) {
            S[j * p + k] = make_double2(0, 0);
            S[k * p + j] = make_double2(0, 0);
            S[j * p + j].y = 0;
            S[k * p + k].y = 0;
          }
        }
    }
    __syncthreads();
    // out = V diag(lambda^-1 or lambda^-1/2) V^H Zg(r, ., nu)
    if (m < p) {
      double2 acc = make_double2(0, 0);
      for (int j = 0; j < p; ++j) {
        const double2 vj = V[j * p + m], g = z[((long long)r * p + j) * d + nu];
        acc.x += vj.x * g.x + vj.y * g.y;
        acc.y += vj.x * g.y - vj.y * g.x;
      }
      const double lam = S[m * p + m].x;
      mn = fmin(mn, fmax(lam, 0.0) * scale_bounds);
      mx = fmax(mx, lam * scale_bounds);
      const double f = lam > 0 ? (tight ? 1 / sqrt(lam) : 1 / lam) : 0.0;
      vec[m] = cscale(acc, f);
    }
    __syncthreads();
    if (m < p) {
      double2 acc = make_double2(0, 0);
      for (int k = 0; k < p; ++k) {
        const double2 t = cmul(V[m * p + k], vec[k]);
        acc.x += t.x;
        acc.y += t.y;
      }
      zd[((long long)r * p + m) * d + nu] = acc;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  if (m == 0) {
    part[2 * blockIdx.x] = mn;
    part[2 * blockIdx.x + 1] = mx;
  }
}

template <int Unused = 0>
__global__ void __launch_bounds__(kThreads) k_minmax_final(const double* part, int nparts, double* out) {
  __shared__ double smin[kThreads], smax[kThreads];
  double mn = 1e308, mx = 0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) {
    mn = fmin(mn, part[2 * i]);
    mx = fmax(mx, part[2 * i + 1]);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
  }
}

// ----------------------------------------------------------------------------
// Window gradient.  The window's Zak transform has Mi p columns u (window
// samples u + Mi p t, t in Z_d); the factorisation multiplies signal column
// (r, j0) (samples r + Mi j0 + Mi p t) by conj(Zg_u) with u = r + Mi j0 - n0 ai
// (mod Mi p, a wrap multiplying by exp(-2 pi i nu / d)).  For a given u and
// time offset n0 exactly one pair (r, j0) contributes: w = u + n0 ai mod Mi p,
// j0 = w div Mi, r = w mod Mi.  In the Zak domain
//   grad Zg_u(nu) += X_w(nu) conj(Hhat_{n0,r}(nu)) exp(-2 pi i nu delta/d) / d,
// with X_w the DFT over t of the signal column w, Hhat the DFT over t' of
// h*_{n0 + q t'}(r) and delta = -1 when w wrapped.  (p = 1: w = r.)  The
// window gradient is the unnormalised inverse DFT of grad Zg.  grid
// (ceil(Mi p / W), B): one partial per signal, summed by k_batch_sum
// (deterministic, no atomics).
// ----------------------------------------------------------------------------
template <typename C> struct GradArgs {
  const void* x;
  long long xs;
  int real_in;
  ChirpSrc<C> chirp;
  const C* H;
  long long hs;
  C* part;
  long long ps;
  const C* twd;
  int Mi, ai, d, q, W, Sd;
  int p;                       // columns of the window's Zak transform: Mi p
  FftSched fd;
};

// TWG: twiddles read from global memory, which leaves the whole LDS to the
// 2 W column transforms (FP64 columns above 3412 values).
template <typename C, bool TWG>
__global__ void __launch_bounds__(kThreads) k_grad_cols(GradArgs<C> A) {
  using T = decltype(C::x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* twl = lds;
  const C* tw = TWG ? A.twd : twl;
  const int d = A.d, W = A.W, Sd = A.Sd, Mi = A.Mi, Mp = A.Mi * A.p;
  C* xb = TWG ? lds : lds + d;   // W transforms of the signal columns, then W of h*
  C* yb = xb + W * Sd;
  if (!TWG)
    for (int e = threadIdx.x; e < d; e += kThreads) twl[e] = A.twd[e];
  const int u0 = blockIdx.x * W;
  const long long bo = blockIdx.y;
  const int WD = W * d;
  constexpr int KX = MaxE<C>::value;
  C acc[KX];
#pragma unroll
  for (int i = 0; i < KX; ++i) acc[i] = czero<C>();
  for (int n0 = 0; n0 < A.q; ++n0) {
    __syncthreads();
    for (int e = threadIdx.x; e < WD; e += kThreads) {
      const int t = e / W, cc = e - t * W, u = u0 + cc;
      C v = czero<C>();
      if (u < Mp) {
        int w = u + n0 * A.ai;
        if (w >= Mp) w -= Mp;
        const long long l = w + (long long)t * Mp;
        v = apply_chirp(A.chirp, load_sig<C>(A.x, A.real_in, bo * A.xs + l), l);
      }
      xb[cc * Sd + t] = v;
    }
    for (int e = threadIdx.x; e < WD; e += kThreads) {
      const int cc = e / d, t = e - cc * d, u = u0 + cc;
      C h = czero<C>();
      if (u < Mp) {
        int w = u + n0 * A.ai;
        if (w >= Mp) w -= Mp;
        const int r = w - (w / Mi) * Mi;
        h = A.H[bo * A.hs + ((long long)n0 * Mi + r) * d + t];
      }
      yb[cc * Sd + t] = h;
    }
    __syncthreads();
    // one call transforms at most MaxE * kThreads values
    if (2 * WD <= MaxE<C>::value * kThreads) {
      fft_lds<C, false>(xb, Sd, A.fd, 2 * W, tw);
    } else {
      fft_lds<C, false>(xb, Sd, A.fd, W, tw);
      fft_lds<C, false>(yb, Sd, A.fd, W, tw);
    }
#pragma unroll
    for (int i = 0; i < KX; ++i) {
      const int e = threadIdx.x + i * kThreads;
      if (e < WD) {
        const int cc = e / d, nu = e - cc * d, u = u0 + cc;
        if (u < Mp) {
          C pr = cmulc(xb[cc * Sd + nu], yb[cc * Sd + nu]);
          if (u + n0 * A.ai >= Mp) pr = cmulc(pr, tw[nu]);
          acc[i] = cadd(acc[i], pr);
        }
      }
    }
  }
  __syncthreads();
  const T inv_d = T(1) / T(d);
#pragma unroll
  for (int i = 0; i < KX; ++i) {
    const int e = threadIdx.x + i * kThreads;
    if (e < WD) {
      const int cc = e / d, nu = e - cc * d;
      xb[cc * Sd + nu] = cscale(acc[i], inv_d);
    }
  }
  __syncthreads();
  fft_lds<C, true>(xb, Sd, A.fd, W, tw);
  for (int e = threadIdx.x; e < WD; e += kThreads) {
    const int t = e / W, cc = e - t * W, u = u0 + cc;
    if (u < Mp) A.part[bo * A.ps + u + (long long)t * Mp] = xb[cc * Sd + t];
  }
}

// out[l] = chirp(l) * sum_k part[k][l]  (fixed summation order)
template <typename C>
__global__ void __launch_bounds__(kThreads) k_batch_sum(const C* part, long long ps, int B, long long L,
                                                       ChirpSrc<C> chirp, C* out) {
  const long long l = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (l >= L) return;
  C s = czero<C>();
  for (int k = 0; k < B; ++k) s = cadd(s, part[k * ps + l]);
  out[l] = apply_chirp(chirp, s, l);
}

// precision conversion of a complex vector
template <typename CI, typename CO>
__global__ void __launch_bounds__(kThreads) k_convert(const CI* x, CO* y, long long n) {
  using TO = decltype(CO::x);
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = mk<CO>(TO(x[i].x), TO(x[i].y));
}

}  // namespace dgtns
