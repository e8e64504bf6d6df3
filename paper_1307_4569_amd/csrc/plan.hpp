// Host-side lattice planner for the shear DGT (exact int64 arithmetic).
//
// Given (L, a, M, lambda1, lambda2) the planner
//   * validates the lattice (Prop. 1 normal form; feasible lengths, Prop. 8),
//   * finds the shear factorisation A = U_{s0,s1} D V (Thm. 2): first a time
//     shear alone (a | s + k b for some k, Prop. 9), otherwise the
//     constructive proof of Thm. 2 (choice of s1 from prime exponents,
//     Bezout for k1, s0 from the exponents of k1, check of eq. (modcond)),
//   * derives the separable lattice the factorised DGT runs on and the
//     constants of Alg. 1 (C1 ... C6), or, for the multiwindow algorithm
//     (Prop. 4, Prop. 5), the separable lattice (lambda2 a, M) shared by the
//     lambda2 coset windows,
//   * builds the FFT radix schedules and all twiddle/chirp/phase tables in
//     FP64 (rounded to FP32 for single-precision plans).
#pragma once
#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

namespace dgtns {

constexpr int kMaxStages = 20;
constexpr int64_t kMaxFft = 4096;     // largest in-LDS transform length
constexpr int64_t kMaxL = int64_t(1) << 30;

struct FftSchedule {
  int n = 1;
  int nst = 0;
  int8_t rad[kMaxStages] = {0};
};

// Floor modulus for possibly negative values.
inline int64_t fmod64(int64_t x, int64_t m) {
  int64_t r = x % m;
  return r < 0 ? r + m : r;
}

// (x * y) mod m without overflow for 0 <= x, y < m < 2^62.
inline int64_t mulmod(int64_t x, int64_t y, int64_t m) {
  return int64_t((__int128)x * y % m);
}

struct Shear {
  int64_t s0 = 0, s1 = 0, br = 0;   // frequency shear, time shear, b_r
  bool constructed = false;          // true if the Thm. 2 construction was used
};

// Number theory helpers (exposed for tests through the C-ABI).
int64_t gcd64(int64_t a, int64_t b);
int64_t lcm64(int64_t a, int64_t b);
bool fft_schedule(int64_t n, FftSchedule* out);
Shear shearfind(int64_t L, int64_t a, int64_t M, int64_t s, int64_t b, std::string* err);

enum Branch { kSeparable = 0, kTimeShear = 1, kFreqShear = 2, kMultiwindow = 3, kFir = 4, kShearOla = 5 };
enum Algorithm { kAlgShear = 0, kAlgMultiwindow = 1, kAlgFir = 2, kAlgShearOla = 3, kAlgAuto = 4 };

// Automatic choice between the shear and the multiwindow algorithm: the
// multiwindow plan when the shear factorisation needs a frequency shear and
// the multiwindow lattice (lambda2 a, M) has p <= kAutoMaxP.
constexpr int64_t kAutoMaxP = 15;

struct Plan {
  // lattice
  int64_t L, a, M, lam1, lam2, b, N, s;
  Shear sh;
  int branch;
  int dtype;           // 0 = complex64, 1 = complex128
  int64_t max_batch;
  // separable lattice the factorised DGT runs on (time step ai, channels Mi).
  // The factorisation runs over qi = nw * qw time offsets n0: nw windows with
  // qw = Mi / ci offsets each (nw = 1 for the shear algorithm; nw = lambda2
  // coset windows for the multiwindow algorithm, window mu = n0 / qw).
  int64_t ai, Mi, bi, Ni, ci, pi, qi, di;
  int64_t qw = 0, nw = 1;
  // frequency-shear branch constants of Alg. 1 (reduced mod 2N or mod L)
  int64_t ar, Mr, Nr;
  int64_t K1, K2, K3, K4, K5;     // C1, C2, C3, C4, C5 mod 2N
  int64_t Kt1, Kt6;               // (-s1 a_r) mod L and C6 mod L
  int64_t C1n, C2n;               // C1, C2 mod N
  // FFT schedules
  FftSchedule fd, fm, f1, f2;     // length di, Mi, and L = L1 * L2 (freq shear)
  int64_t L1, L2;
  // Columns longer than one in-LDS transform: d = d1 d2 (two-level column
  // transforms); Wl columns per work-group of the length-d1 passes and Wm
  // columns r per work-group of the middle pass.
  bool longd = false;
  // FIR-window algorithm: window support start, ..., start + fir_len - 1 (mod L)
  int64_t fir_start = 0, fir_len = 0;
  // Shear-OLA (Section 4): ola_Nb blocks of ola_Lb samples, each zero-extended
  // into a DGT of length ola_Lx = ola_Nx a on the same lattice (the inner
  // plan).  Block b covers local time positions n' in Z_{ola_Nx}, global
  // position n = b ola_Lb / a - ola_P0 + n' (ola_P0 a multiple of lambda2), and
  // local sample j is global sample (b ola_Lb - ola_J0 + j) mod L; the block's
  // own samples sit at j in [ola_J0, ola_J0 + ola_Lb).  ola_s: signed window
  // start.
  int64_t ola_Lb = 0, ola_Nb = 0, ola_Lx = 0, ola_Nx = 0, ola_P0 = 0, ola_J0 = 0, ola_s = 0;
  std::shared_ptr<Plan> inner;
  int64_t d1 = 0, d2 = 0;
  FftSchedule fd1, fd2;
  int Wl = 1, Wm = 1;
  // column-block width of the factorisation kernels
  int W;
  // host tables (FP64, interleaved re/im); uploaded by bind
  std::vector<double> tw_d, tw_m, tw_1, tw_2, tw_L, chirp1, chirp0, post_E, tw_d1, tw_d2, fir_ph;
  std::vector<int32_t> post_rho;
  // device memory map (byte offsets into the persistent block)
  struct Off {
    size_t tw_d, tw_m, tw_1, tw_2, tw_L, chirp1, chirp0, post_E, post_rho, zc;   // plan dtype
    size_t tw_d64, tw_m64, tw_1_64, tw_2_64, tw_L64;                             // FP64 copies
    size_t tw_d1, tw_d2, tw_d1_64, tw_d2_64;                                     // long columns
    size_t fir_ph;                                                               // FIR, OLA: lambda2 M phases
    size_t inner;                                                                // OLA: inner plan's block
    size_t bounds;  // 2 doubles
    size_t total;
  } off;
  void* dev = nullptr;       // bound persistent memory
  bool window_set = false;
  bool generic = false;   // force the runtime-schedule kernels (DGTNS_GENERIC=1)
  // Signals per chunk of the optional two-stream pipeline of the time-shear
  // branch (DGTNS_CHUNK_MIB): the workspace then holds two chunks of h
  // instead of the whole batch.  0: one launch per stage.
  int64_t chunk = 0;
  // Signals per chunk of the sequential forward and adjoint (time-shear and
  // separable branches, columns in one in-LDS transform): both stages of a
  // chunk run back to back on the caller's stream through one h buffer of
  // that many signals, small enough to stay in the last-level cache between
  // the two kernels.  Used when the whole batch's h would not stay there.
  // 0: one launch per stage.
  int64_t seq = 0;
};

// Returns 0 on success, else an error status with a message in *err.
int plan_make(int64_t L, int64_t a, int64_t M, int64_t lam1, int64_t lam2, int dtype,
              int64_t max_batch, int algorithm, Plan* p, std::string* err, int64_t fir_start = 0,
              int64_t fir_len = 0, int64_t ola_block = 0, int ola_inner = kAlgAuto);

// Coset window mu of the multiwindow algorithm: g_mu(l) = exp(2 pi i l sigma / L)
// g(l - mu a) with sigma = (mu s) mod b (Prop. 5).
inline int64_t mw_sigma(const Plan& p, int64_t mu) { return int64_t((__int128)mu * p.s % p.b); }

// exp(2 pi i num / den), accurate to about one ulp (num reduced exactly first).
void unit_root(int64_t num, int64_t den, double* re, double* im);

}  // namespace dgtns
