// Shear-OLA algorithm (Section 4): the shear algorithm on blocks of the
// signal, combined by overlap-add.  For a window supported on
// n a + s + [0, L_g) (mod L) the coefficients of eq. (DGT) split by blocks of
// L_b samples:
//     c(m, n) = sum_b sum_{l in block b} f(l) conj(g(l - n a)) exp(-2 pi i l (m + w(n)) / M).
// Block b is zero-extended into a signal x_b of length L_x whose sample j is
// global sample o_b + j, o_b = b L_b - J0, the block itself at j in
// [J0, J0 + L_b).  Its DGT on the same lattice at length L_x, with the window
// g_loc(i) = g(s + i) for i < L_g (0 up to L_x), gives at local position n'
// (global n = b L_b / a - P0 + n') exactly the block's share of c(m, n)
// times exp(2 pi i o_b (m + w(n)) / M), since P0 and L_b / a are multiples of
// lambda2 (so w(n') = w(n)) and J0 >= L_g - a keeps windows that wrap around
// L_x off the block's samples.
#pragma once
#include "kernels.hpp"

namespace dgtns {

template <typename C> struct OlaArgs {
  const void* x;       // signals, xs samples apart
  long long xs;
  int real_in;
  C* X;                // zero-extended blocks [B Nb][Lx]
  const C* cl;         // block coefficients [B Nb][Nx][M]
  C* c;                // coefficients [B][N][M], cs values apart
  long long cs;
  const C* ph;         // exp(-2 pi i e / (lambda2 M)), e in Z_{lambda2 M}
  long long L, Lb, Lx, J0;
  int a, M, N, Nb, Nx, P0, lam1, lam2;
  CoefLayout lay;      // layout of c (cs values per signal)
};

// X[k Nb + b][j] = f_k(b L_b - J0 + j) for j in [J0, J0 + L_b), else 0.
// grid (ceil(Lx / kThreads), B Nb).
template <typename C>
__global__ void __launch_bounds__(kThreads) k_ola_gather(OlaArgs<C> A) {
  const long long j = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (j >= A.Lx) return;
  const long long kb = blockIdx.y;
  const long long k = kb / A.Nb, b = kb - k * A.Nb;
  C v = czero<C>();
  if (j >= A.J0 && j < A.J0 + A.Lb) v = load_sig<C>(A.x, A.real_in, k * A.xs + b * A.Lb + (j - A.J0));
  A.X[kb * A.Lx + j] = v;
}

// c_k(m, n) = sum over the blocks b whose local positions n' = (n + P0 -
// b L_b / a) mod N lie in Z_Nx of exp(-2 pi i o_b (m lambda2 + kn) /
// (lambda2 M)) cl[k Nb + b][n'][m], kn = n lambda1 mod lambda2, in a fixed
// order (no atomics).  One work-group per time position n and signal k
// (grid (N, B), kOlaThreads threads): the covering blocks, their rows and
// position phases are found once per work-group, and the phase index of
// channel m advances by a constant step between a thread's channels.
constexpr int kOlaThreads = 256;
constexpr int kOlaPer = 16;   // channels per thread and slice

template <typename C>
__global__ void __launch_bounds__(kOlaThreads) k_ola_combine(OlaArgs<C> A) {
  const int n = blockIdx.x, tid = threadIdx.x;
  const long long k = blockIdx.y;
  int cnt, ee;
  const long long col = coef_col(A.lay, n, &cnt, &ee);
  const int Q = int(A.Lb / A.a);
  int t = n + A.P0;
  if (t >= A.N) t -= A.N;
  const int bh = t / Q, n00 = t - bh * Q;
  const unsigned long long PM = (unsigned long long)A.lam2 * A.M;
  const unsigned long long kn = (unsigned long long)(((long long)n * A.lam1) % A.lam2);
  // channels in slices of kOlaThreads kOlaPer (one slice for M <= 4096)
  for (int m0 = 0; m0 < cnt; m0 += kOlaThreads * kOlaPer) {
    C acc[kOlaPer];
#pragma unroll
    for (int j = 0; j < kOlaPer; ++j) acc[j] = czero<C>();
    for (int i = 0;; ++i) {
      const int np = n00 + i * Q;   // np < Nx < N = Nb Q, so i < Nb
      if (np >= A.Nx) break;
      int b = bh - i;
      if (b < 0) b += A.Nb;
      long long ob = ((long long)b * A.Lb - A.J0) % (long long)PM;
      if (ob < 0) ob += PM;
      // phase index of channel m: (ob (m lambda2 + kn)) mod PM = (e0 + m st) mod PM
      const unsigned long long e0 = ((unsigned long long)ob * kn) % PM;
      const unsigned long long st = ((unsigned long long)ob * A.lam2) % PM;
      const unsigned long long est = (st * kOlaThreads) % PM;
      unsigned long long e = (e0 + st * (unsigned long long)(m0 + tid)) % PM;
      const C* src = A.cl + ((k * A.Nb + b) * A.Nx + np) * (long long)A.M;
#pragma unroll
      for (int j = 0; j < kOlaPer; ++j) {
        const int m = m0 + tid + j * kOlaThreads;
        if (m < cnt) acc[j] = cadd(acc[j], cmul(A.ph[e], src[m]));
        e += est;
        if (e >= PM) e -= PM;
      }
    }
    C* dst = A.c + k * A.cs + col;
#pragma unroll
    for (int j = 0; j < kOlaPer; ++j) {
      const int m = m0 + tid + j * kOlaThreads;
      if (m < cnt) dst[m] = acc[j];
    }
  }
}

// Adjoint of the overlap-add: block b's coefficient at local position n' is
// the global coefficient c(m, n) of the position n it adds to, times the
// conjugate of the combine's phase:
//     cl[k Nb + b][n'][m] = conj(exp(-2 pi i o_b (m lambda2 + kn) / (lambda2 M))) c_k(m, n),
// with i = n' div Q, n00 = n' mod Q (Q = L_b / a), n = ((b + i) mod Nb) Q +
// n00 - P0 (mod N).  grid (Nx, B Nb), kOlaThreads threads.
template <typename C>
__global__ void __launch_bounds__(kOlaThreads) k_ola_split(OlaArgs<C> A) {
  // one work-group per local position n' (blockIdx.x) of block kb: the
  // global position, its column and the block phase are uniform
  const int np = blockIdx.x, tid = threadIdx.x;
  const long long NxM = (long long)A.Nx * A.M;
  const long long kb = blockIdx.y;
  const long long k = kb / A.Nb;
  const int b = int(kb - k * A.Nb);
  const int Q = int(A.Lb / A.a);
  const int i = np / Q, n00 = np - i * Q;
  int bh = b + i;
  if (bh >= A.Nb) bh -= A.Nb;   // i < Nb (np < Nx < N)
  int n = bh * Q + n00 - A.P0;
  if (n < 0) n += A.N;
  const unsigned long long PM = (unsigned long long)A.lam2 * A.M;
  const unsigned long long kn = (unsigned long long)(((long long)n * A.lam1) % A.lam2);
  long long ob = ((long long)b * A.Lb - A.J0) % (long long)PM;
  if (ob < 0) ob += PM;
  const unsigned long long e0 = ((unsigned long long)ob * kn) % PM;
  const unsigned long long st = ((unsigned long long)ob * A.lam2) % PM;
  const unsigned long long est = (st * kOlaThreads) % PM;
  unsigned long long e = (e0 + st * tid) % PM;
  int cnt, ee;
  const long long col = coef_col(A.lay, n, &cnt, &ee);
  const C* cb = A.c + k * A.cs;
  C* dst = const_cast<C*>(A.cl) + kb * NxM + (long long)np * A.M;
  for (int m = tid; m < A.M; m += kOlaThreads) {
    dst[m] = cmulc(coef_load(cb, A.M, col, cnt, ee, m), A.ph[e]);
    e += est;
    if (e >= PM) e -= PM;
  }
}

// Adjoint of the block gather: sample j of block b's synthesis, j in
// [J0, J0 + L_b), is global sample b L_b + j - J0 (each sample in one block).
// grid (ceil(L / kThreads), B).
template <typename C>
__global__ void __launch_bounds__(kThreads) k_ola_scatter(OlaArgs<C> A, C* f, int real_out) {
  const long long l = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (l >= A.L) return;
  const long long k = blockIdx.y;
  const long long b = l / A.Lb, j = l - b * A.Lb + A.J0;
  st_out(f, k * A.L + l, A.X[(k * A.Nb + b) * A.Lx + j], real_out);
}

// Block window g_loc(i) = g((s + i) mod L) for i < L_g, 0 for i in [L_g, L_x)
// (FP64).  grid ceil(Lx / kThreads).
template <int Unused = 0>
__global__ void __launch_bounds__(kThreads) k_ola_window(const double2* g, double2* gl, long long L, long long s,
                                                        long long Lg, long long Lx) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (i >= Lx) return;
  double2 v = make_double2(0, 0);
  if (i < Lg) {
    long long l = (s + i) % L;
    if (l < 0) l += L;
    v = g[l];
  }
  gl[i] = v;
}

}  // namespace dgtns
