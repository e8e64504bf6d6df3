// Wave-level FFT for compile-time power-of-two lengths N in [32, 1024].
//
// A transform is owned by T = N / E lanes of one 64-lane wavefront (64 / T
// transforms per wavefront); lane position l in Z_T holds the E elements
// x[l + T e] (e in Z_E) in registers.  The transform runs as Stockham passes
// whose radices divide E: in a pass of radix R each lane computes E / R
// butterflies, butterfly j = l + T i reading x[j + r N / R] = v[i + r E / R].
// Results of all passes but the last go through a wave-private LDS region
// (no work-group barrier: a wavefront issues its LDS instructions in order),
// and the last pass leaves X[l + T e] in v[e], i.e. the same strided layout,
// so global loads and stores of a transform are fully coalesced.
//
// Each exchange stores element x of the pass output at x + c (x >> s), with
// (c, s) chosen per pass and element size so that the strided stores of the
// pass ((j - k) R + k + r Ns for lanes j, k = j mod Ns) and the contiguous
// loads that follow spread over the LDS banks.  On gfx950 a store serves 128
// bytes per cycle (32 banks: 16 lanes of 8-byte or 8 lanes of 16-byte
// elements) and a load 256 bytes (64 banks), as measured with the
// SQ_LDS_BANK_CONFLICT counter; the offsets stay affine in the element index,
// so every access of a lane is one base register plus an immediate offset.
//
// Twiddles exp(-+ 2 pi i r k / (Ns R)) are read once per lane from the exact
// length-N table exp(-2 pi i e / N) and kept in registers (they depend only on
// the lane, not on the data), so a wavefront that transforms many rows pays
// for them once.
#pragma once
#include "fft_core.hpp"

namespace dgtns {

template <int N> struct WSched;
template <> struct WSched<32> {
  static constexpr int E = 8, NP = 2;
  static constexpr int rad(int p) { return p == 0 ? 8 : 4; }
};
template <> struct WSched<64> {
  static constexpr int E = 8, NP = 2;
  static constexpr int rad(int) { return 8; }
};
template <> struct WSched<128> {
  static constexpr int E = 8, NP = 3;
  static constexpr int rad(int p) { return p < 2 ? 8 : 2; }
};
template <> struct WSched<256> {
  static constexpr int E = 8, NP = 3;
  static constexpr int rad(int p) { return p < 2 ? 8 : 4; }
};
template <> struct WSched<512> {
  static constexpr int E = 8, NP = 3;
  static constexpr int rad(int) { return 8; }
};
template <> struct WSched<1024> {
  static constexpr int E = 16, NP = 3;
  static constexpr int rad(int p) { return p < 2 ? 8 : 16; }
};

// radix-16 DFT: radix-8 DFTs of the even and odd elements, combined with W16^k
template <typename C, bool INV> struct Bfly<C, 16, INV> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(C::x);
    C e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    }
    Bfly<C, 8, INV>::run(e);
    Bfly<C, 8, INV>::run(o);
    // W16^k = cos(pi k / 8) -+ i sin(pi k / 8)
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    const T h = T(0.70710678118654752440);
    const T cs[8] = {T(1), c1, h, s1, T(0), -s1, -h, -c1};
    const T sn[8] = {T(0), s1, h, c1, T(1), c1, h, s1};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const C w = mk<C>(cs[k], INV ? sn[k] : -sn[k]);
      const C t = k == 0 ? o[0] : cmul(o[k], w);
      v[k] = cadd(e[k], t);
      v[k + 8] = csub(e[k], t);
    }
  }
};

template <int N> struct WInfo {
  using S = WSched<N>;
  static constexpr int E = S::E;
  static constexpr int T = N / E;       // lanes per transform
  static constexpr int TPW = 64 / T;    // transforms per wavefront
  static constexpr int ns(int p) { return p == 0 ? 1 : ns(p - 1) * S::rad(p - 1); }
  static constexpr int ntw_upto(int p) {  // twiddles used by passes 1 .. p-1
    return p <= 1 ? 0 : ntw_upto(p - 1) + (E / S::rad(p - 1)) * (S::rad(p - 1) - 1);
  }
  static constexpr int NTW = ntw_upto(S::NP);
};

// Exchange offset of a pass of stride Ns for ES-byte elements: element x of
// the pass output lives at x + c (x >> s).  Ns = 1 (stores of stride R = 8):
// one pad element per 16 (8-byte elements, N >= 128) or per 8; Ns = 8 (runs
// of 8 at stride 64): 8 pad elements per 64 for 8-byte elements, none for
// 16-byte ones (8 lanes per store cycle already hit distinct banks).  Later
// passes store runs of at least 64 contiguous elements and are unpadded.
template <int ES, int N, int Ns> struct XPad {
  static constexpr int s = Ns == 1 ? ((ES >= 16 || N <= 64) ? 3 : 4) : 6;
  static constexpr int c = Ns == 1 ? 1 : (Ns == 8 && ES == 8 ? 8 : 0);
  static constexpr int need = N + c * ((N - 1) >> s);  // elements spanned
  static __device__ __forceinline__ int at(int x) { return x + c * (x >> s); }
};

// Exchange region per transform (elements of type C).  Transforms that share
// a wavefront (N <= 128) are N + N / 8 apart so that their loads do not
// collide.
template <typename C, int N> struct WEx {
  using I = WInfo<N>;
  static constexpr int ES = sizeof(C);
  static constexpr int n0 = XPad<ES, N, 1>::need;
  static constexpr int n1 = WSched<N>::NP > 2 ? XPad<ES, N, I::ns(1)>::need : 0;
  static constexpr int need = n0 > n1 ? n0 : n1;
  static constexpr int EX = (N <= 128 && need < N + N / 8) ? N + N / 8 : need;
};

// Per-lane twiddles of all passes after the first.
template <typename C, int N> struct WTw {
  C w[WInfo<N>::NTW > 0 ? WInfo<N>::NTW : 1];

  template <int P>
  __device__ __forceinline__ void fill(const C* tab, int l) {
    if constexpr (P < WSched<N>::NP) {
      using I = WInfo<N>;
      constexpr int R = WSched<N>::rad(P), Ns = I::ns(P), NB = I::E / R, step = N / (Ns * R);
      constexpr int off = I::ntw_upto(P);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int k = (l + I::T * i) & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[off + i * (R - 1) + r - 1] = tab[r * k * step];
      }
      fill<P + 1>(tab, l);
    }
  }
  __device__ __forceinline__ void load(const C* tab, int l) { fill<1>(tab, l); }
};

template <typename C, int N, bool INV, int P>
__device__ __forceinline__ void wave_pass(C (&v)[WInfo<N>::E], C* ex, int l, const WTw<C, N>& tw) {
  using I = WInfo<N>;
  constexpr int E = I::E, T = I::T, R = WSched<N>::rad(P), Ns = I::ns(P), NB = E / R;
  constexpr bool LAST = P == WSched<N>::NP - 1;
  constexpr int off = I::ntw_upto(P);
  using XP = XPad<int(sizeof(C)), N, Ns>;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    C u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[i + r * NB];
    if constexpr (P > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tw.w[off + i * (R - 1) + r - 1];
        u[r] = INV ? cmulc(u[r], w) : cmul(u[r], w);
      }
    }
    Bfly<C, R, INV>::run(u);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i + r * NB] = u[r];
    } else {
      const int j = l + T * i;
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) ex[XP::at(base + r * Ns)] = u[r];
    }
  }
  if constexpr (!LAST) {
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ex[XP::at(l + T * e)];
    __builtin_amdgcn_wave_barrier();
    wave_pass<C, N, INV, P + 1>(v, ex, l, tw);
  }
}

// In-register transform of the N elements held by this lane's transform
// group; ex: wave-private LDS region of WEx<C, N>::EX elements for this
// transform.  INV: unnormalised inverse.
template <typename C, int N, bool INV>
__device__ __forceinline__ void wave_fft(C (&v)[WInfo<N>::E], C* ex, int l, const WTw<C, N>& tw) {
  wave_pass<C, N, INV, 0>(v, ex, l, tw);
}

// Length-1024 transform with a half-size exchange region and the twiddles of
// each pass read when the pass runs, for kernels that need the LDS and the
// registers for more resident work-groups (one transform per wavefront).  In
// the two exchanges of this schedule (radix 8, 8, 16; two butterflies per
// lane) butterfly i of every lane fills exactly half i of the pass output
// (positions [512 i, 512 i + 512)), and elements e < 8 of the next pass are
// read from half 0, e >= 8 from half 1: the halves go through one region
// of WExH elements in turn.
template <typename C> struct WExH {
  static constexpr int ES = sizeof(C);
  using X0 = XPad<ES, 1024, 1>;
  using X1 = XPad<ES, 1024, 8>;
  static constexpr int n0 = 512 + X0::c * (511 >> X0::s);
  static constexpr int n1 = 512 + X1::c * (511 >> X1::s);
  static constexpr int EX = n0 > n1 ? n0 : n1;
};

template <typename C, bool INV, int P>
__device__ __forceinline__ void wave_pass_h(C (&v)[16], C* ex, int l, const C* tab) {
  constexpr int N = 1024, E = 16, T = 64;
  using S = WSched<N>;
  constexpr int R = S::rad(P), Ns = WInfo<N>::ns(P), NB = E / R, step = N / (Ns * R);
  constexpr bool LAST = P == S::NP - 1;
  static_assert(LAST || NB == 2, "two butterflies per lane before the last pass");
  using XP = XPad<int(sizeof(C)), N, Ns>;
  C u[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int r = 0; r < R; ++r) u[i][r] = v[i + r * NB];
    if constexpr (P > 0) {
      const int k = (l + T * i) & (Ns - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tab[r * k * step];
        u[i][r] = INV ? cmulc(u[i][r], w) : cmul(u[i][r], w);
      }
    }
    Bfly<C, R, INV>::run(u[i]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = u[0][r];
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = l + T * h, k = j & (Ns - 1);
      const int base = (j - k) * R + k - h * (N / 2);
#pragma unroll
      for (int r = 0; r < R; ++r) ex[XP::at(base + r * Ns)] = u[h][r];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int e = 0; e < E / 2; ++e) v[h * (E / 2) + e] = ex[XP::at(l + T * e)];
      __builtin_amdgcn_wave_barrier();
    }
    wave_pass_h<C, INV, P + 1>(v, ex, l, tab);
  }
}

// tab: the length-1024 table exp(-2 pi i e / 1024); ex: WExH<C>::EX elements
template <typename C, bool INV>
__device__ __forceinline__ void wave_fft_h(C (&v)[16], C* ex, int l, const C* tab) {
  wave_pass_h<C, INV, 0>(v, ex, l, tab);
}

}  // namespace dgtns
