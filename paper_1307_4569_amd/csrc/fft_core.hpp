// Device-side building blocks: complex arithmetic and an in-LDS mixed-radix
// Stockham FFT executed cooperatively by one 512-thread work-group.
//
// A transform of length n = prod(radices) runs as one radix-R pass per
// factor.  Pass s with radix R and Ns = product of the earlier radices maps
// element j + r n/R (r in Z_R) of the current sequence to position
// (j - j mod Ns) R + j mod Ns + r Ns after multiplying by the twiddle
// exp(-+ 2 pi i r (j mod Ns) / (Ns R)) and an R-point DFT, which sorts the
// output into natural order without a bit-reversal pass.  Twiddles come from
// a length-n table exp(-2 pi i e / n) computed on the host from exactly
// reduced integer indices; the inverse direction conjugates them.
//
// Each thread keeps the R inputs of up to ceil(MAXE / R) butterflies in
// registers between the read and the write half of a pass, so a pass works
// in place: read all, barrier, write all, barrier.  The caller guarantees
// ntr * n <= MAXE * kThreads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgtns {

constexpr int kThreads = 512;
// elements per thread held in registers by a pass: 16 complex (FP32) or 8
// (FP64), i.e. 8192 or 4096 elements per work-group
template <typename C> struct MaxE { static constexpr int value = sizeof(C) == 8 ? 16 : 8; };
constexpr int kMaxE = 16;

template <typename T> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) re, decltype(C::x) im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
template <typename C> __device__ __forceinline__ C czero() { return mk<C>(0, 0); }
// multiply by -i (forward) or +i (inverse)
template <typename C, bool INV> __device__ __forceinline__ C mul_mi(C a) {
  return INV ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}

// Compensated complex product for the chirp multiplications: each real part
// a*b - c*d is evaluated with one rounding error term recovered by FMA
// (Kahan's difference-of-products), so the product carries an error of about
// one rounding of the result instead of the cancellation error of the plain
// formula.
template <typename T> __device__ __forceinline__ T diff_prod(T a, T b, T c, T d) {
  T w = c * d;
  T e = fma(-c, d, w);
  T f = fma(a, b, -w);
  return f + e;
}
template <typename C> __device__ __forceinline__ C cmul_comp(C a, C b) {
  return mk<C>(diff_prod(a.x, b.x, a.y, b.y), diff_prod(a.x, b.y, -a.y, b.x));
}

struct FftSched {
  int n;
  int nst;
  int8_t rad[20];
};

// ---- R-point DFTs on registers ----
template <typename C, int R, bool INV> struct Bfly;

template <typename C, bool INV> struct Bfly<C, 2, INV> {
  static __device__ __forceinline__ void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename C, bool INV> struct Bfly<C, 4, INV> {
  static __device__ __forceinline__ void run(C* v) {
    C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C c = cadd(v[1], v[3]), d = mul_mi<C, INV>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <typename C, bool INV> struct Bfly<C, 8, INV> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(C::x);
    const T h = T(0.70710678118654752440);
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<C, 4, INV>::run(e);
    Bfly<C, 4, INV>::run(o);
    // o[k] *= W8^k (forward W8 = (1 - i)/sqrt2; inverse conjugate)
    C o1 = INV ? mk<C>(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : mk<C>(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    C o2 = mul_mi<C, INV>(o[2]);
    C o3 = INV ? mk<C>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : mk<C>(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// odd prime radices: y_k = x_0 + sum_{j=1}^{(R-1)/2} [ (x_j + x_{R-j}) cos(2 pi jk/R)
//                                 -+ i (x_j - x_{R-j}) sin(2 pi jk/R) ]
template <int R> struct OddConst;
template <> struct OddConst<3> {
  static __device__ __forceinline__ double c(int k) { (void)k; return -0.5; }
  static __device__ __forceinline__ double s(int k) { (void)k; return 0.86602540378443864676; }
};
template <> struct OddConst<5> {
  static __device__ __forceinline__ double c(int k) { return k == 1 ? 0.30901699437494742410 : -0.80901699437494742410; }
  static __device__ __forceinline__ double s(int k) { return k == 1 ? 0.95105651629515357212 : 0.58778525229247312917; }
};
template <> struct OddConst<7> {
  static __device__ __forceinline__ double c(int k) {
    return k == 1 ? 0.62348980185873353053 : (k == 2 ? -0.22252093395631440429 : -0.90096886790241912624);
  }
  static __device__ __forceinline__ double s(int k) {
    return k == 1 ? 0.78183148246802980871 : (k == 2 ? 0.97492791218182360702 : 0.43388373911755812048);
  }
};

template <typename C, int R, bool INV> struct BflyOdd {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(C::x);
    constexpr int H = (R - 1) / 2;
    C s[H], d[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      s[j - 1] = cadd(v[j], v[R - j]);
      d[j - 1] = csub(v[j], v[R - j]);
    }
    C x0 = v[0];
    C y0 = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) y0 = cadd(y0, s[j]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      C re = x0, im = czero<C>();
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const int jk = (j * k) % R;
        const int kk = jk <= H ? jk : R - jk;
        const T cs = T(OddConst<R>::c(kk));
        const T sn = T(jk <= H ? OddConst<R>::s(kk) : -OddConst<R>::s(kk));
        re = cadd(re, cscale(s[j - 1], cs));
        im = cadd(im, cscale(d[j - 1], sn));
      }
      // forward: y_k = re - i im, y_{R-k} = re + i im
      C mi = mul_mi<C, INV>(im);
      v[k] = cadd(re, mi);
      v[R - k] = csub(re, mi);
    }
    v[0] = y0;
  }
};
template <typename C, bool INV> struct Bfly<C, 3, INV> : BflyOdd<C, 3, INV> {};
template <typename C, bool INV> struct Bfly<C, 5, INV> : BflyOdd<C, 5, INV> {};
template <typename C, bool INV> struct Bfly<C, 7, INV> : BflyOdd<C, 7, INV> {};

// Quotient x / d of integers 0 <= x < 2^15 and 1 <= d <= 4096 from the
// correctly rounded reciprocal inv = 1.0f / d: (x + 1/2) / d lies at least
// 1 / (2 d) from every integer, far more than the error of one rounded
// product, so truncation gives the exact quotient (checked for every such
// pair).  Three vector instructions instead of a runtime integer division.
__device__ __forceinline__ int qdiv(int x, float inv) { return int((float(x) + 0.5f) * inv); }

// for (e = e0; e < n; e += step) st(e, ld(e)), in batches of U trips whose
// loads are all issued before the first is used (so their latencies overlap
// instead of one load and wait per trip).
template <int U, typename V, typename LD, typename ST>
__device__ __forceinline__ void batched_for(int e0, int n, int step, LD ld, ST st) {
  for (int b = e0; b < n; b += U * step) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b + u * step;
      if (e < n) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b + u * step;
      if (e < n) st(e, v[u]);
    }
  }
}

// One in-place Stockham pass over `ntr` transforms of length n stored at
// buf + t * tstride (t in Z_ntr).
template <typename C, int R, bool INV, int MAXE>
__device__ __noinline__ void fft_pass(C* buf, int tstride, int n, int ntr, int Ns, const C* tw) {
  constexpr int KB = (MAXE + R - 1) / R;
  const int nb = n / R;
  const int total = nb * ntr;
  const int twstep = n / (Ns * R);
  const float inb = 1.0f / float(nb), ins = 1.0f / float(Ns);   // total < 2^15, n <= 4096
  C v[KB][R];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int bf = threadIdx.x + i * kThreads;
    if (bf < total) {
      const int t = qdiv(bf, inb), j = bf - t * nb;
      const C* src = buf + t * tstride + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int bf = threadIdx.x + i * kThreads;
    if (bf < total) {
      const int t = qdiv(bf, inb), j = bf - t * nb;
      const int k = j - Ns * qdiv(j, ins);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[r * k * twstep];
          v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
        }
      }
      Bfly<C, R, INV>::run(v[i]);
      C* dst = buf + t * tstride + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform (all passes).  Must be called by all threads of the block.
// INV = false: X(k) = sum_j x(j) exp(-2 pi i jk/n); INV = true: the same with
// +i, unnormalised.
template <typename C, bool INV, int MAXE = MaxE<C>::value>
__device__ void fft_lds(C* buf, int tstride, const FftSched& fs, int ntr, const C* tw) {
  int Ns = 1;
  for (int s = 0; s < fs.nst; ++s) {
    const int R = fs.rad[s];
    switch (R) {
      case 8: fft_pass<C, 8, INV, MAXE>(buf, tstride, fs.n, ntr, Ns, tw); break;
      case 4: fft_pass<C, 4, INV, MAXE>(buf, tstride, fs.n, ntr, Ns, tw); break;
      case 2: fft_pass<C, 2, INV, MAXE>(buf, tstride, fs.n, ntr, Ns, tw); break;
      case 3: fft_pass<C, 3, INV, MAXE>(buf, tstride, fs.n, ntr, Ns, tw); break;
      case 5: fft_pass<C, 5, INV, MAXE>(buf, tstride, fs.n, ntr, Ns, tw); break;
      case 7: fft_pass<C, 7, INV, MAXE>(buf, tstride, fs.n, ntr, Ns, tw); break;
      default: break;
    }
    Ns *= R;
  }
}

// ---- one wavefront, one transform: runtime-schedule Stockham in LDS ----
// Pass of radix R over n <= 64 MV values at buf, executed by the 64 lanes of
// one wavefront: every lane loads all its butterflies before storing any, so
// the pass can run in place (a wavefront's LDS accesses complete in program
// order) and needs no work-group barrier.  tw: the length-n twiddle table
// exp(-2 pi i k / n) (in LDS for the factorisation kernel).
template <typename C, int R, bool INV, int MV>
__device__ __forceinline__ void wrt_pass(C* buf, int n, int Ns, const C* tw, int lane) {
  constexpr int KB = MV / R + 1;   // butterflies per lane: ceil(n / (64 R)) <= KB
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  const float ins = 1.0f / float(Ns);
  C v[KB][R];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int j = lane + 64 * i;
    if (j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[j + r * nb];
    }
  }
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int j = lane + 64 * i;
    if (j < nb) {
      const int k = j - Ns * qdiv(j, ins);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const C w = tw[r * k * twstep];
          v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
        }
      }
      Bfly<C, R, INV>::run(v[i]);
      C* dst = buf + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[i][r];
    }
  }
}

template <typename C, bool INV, int MV>
__device__ void fft_wave_rt(C* buf, const FftSched& fs, const C* tw, int lane) {
  int Ns = 1;
  for (int s = 0; s < fs.nst; ++s) {
    const int R = fs.rad[s];
    switch (R) {
      case 8: wrt_pass<C, 8, INV, MV>(buf, fs.n, Ns, tw, lane); break;
      case 4: wrt_pass<C, 4, INV, MV>(buf, fs.n, Ns, tw, lane); break;
      case 2: wrt_pass<C, 2, INV, MV>(buf, fs.n, Ns, tw, lane); break;
      case 3: wrt_pass<C, 3, INV, MV>(buf, fs.n, Ns, tw, lane); break;
      case 5: wrt_pass<C, 5, INV, MV>(buf, fs.n, Ns, tw, lane); break;
      case 7: wrt_pass<C, 7, INV, MV>(buf, fs.n, Ns, tw, lane); break;
      default: break;
    }
    Ns *= R;
  }
}

// exp(i pi e / N) for an exactly reduced integer e in [0, 2N): the argument
// e / N is formed after shifting e into [-N, N), so its rounding error is at
// most half an ulp of a number below 1.
__device__ __forceinline__ float2 phase_pi(long long e, long long N, float) {
  long long r = e >= N ? e - 2 * N : e;
  float s, c;
  sincospif(float(r) / float(N), &s, &c);
  return make_float2(c, s);
}
__device__ __forceinline__ double2 phase_pi(long long e, long long N, double) {
  long long r = e >= N ? e - 2 * N : e;
  double s, c;
  sincospi(double(r) / double(N), &s, &c);
  return make_double2(c, s);
}

__device__ __forceinline__ long long fmodll(long long x, long long m) {
  long long r = x % m;
  return r < 0 ? r + m : r;
}

}  // namespace dgtns
