// Lattice planner: normal form checks, shear factorisation and tables.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <utility>
#include <map>

namespace dgtns {

int64_t gcd64(int64_t a, int64_t b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

int64_t lcm64(int64_t a, int64_t b) { return a / gcd64(a, b) * b; }

// Extended Euclid: returns g = gcd(|x|, |y|) >= 0 and u, v with u x + v y = g.
static int64_t egcd(int64_t x, int64_t y, int64_t* u, int64_t* v) {
  int64_t r0 = x, r1 = y, s0 = 1, s1 = 0, t0 = 0, t1 = 1;
  while (r1 != 0) {
    int64_t qq = r0 / r1;
    int64_t t;
    t = r0 - qq * r1; r0 = r1; r1 = t;
    t = s0 - qq * s1; s0 = s1; s1 = t;
    t = t0 - qq * t1; t0 = t1; t1 = t;
  }
  if (r0 < 0) { r0 = -r0; s0 = -s0; t0 = -t0; }
  *u = s0;
  *v = t0;
  return r0;
}

static std::map<int64_t, int> factorize(int64_t n) {
  std::map<int64_t, int> f;
  for (int64_t p = 2; p * p <= n; ++p)
    while (n % p == 0) { f[p]++; n /= p; }
  if (n > 1) f[n]++;
  return f;
}

// Exponent of prime p in x (x != 0).
static int vexp(int64_t x, int64_t p) {
  if (x < 0) x = -x;
  int e = 0;
  while (x != 0 && x % p == 0) { x /= p; ++e; }
  return e;
}

static int64_t ipow(int64_t p, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= p;
  return r;
}

// Shear factorisation of the lattice [[a, 0], [s, b]] (Thm. 2 and Prop. 9).
Shear shearfind(int64_t L, int64_t a, int64_t M, int64_t s, int64_t b, std::string* err) {
  (void)M;
  Shear r;
  if (s == 0) {           // separable lattice: no shear at all
    r.br = b;
    return r;
  }
  // A time shear alone suffices iff a | s + k b for some k (Prop. 9); then
  // s1 = -(s + k b) / a makes [[1,0],[s1,1]] A = [[a,0],[-k b, b]] separable.
  // Residues of s + k b mod a repeat with period a / gcd(a, b).
  for (int64_t k = 0; k <= a; ++k) {
    if ((s + k * b) % a == 0) {
      r.s0 = 0;
      r.s1 = -((s + k * b) / a);
      r.br = b;
      return r;
    }
  }
  // Constructive proof of Thm. 2.
  auto primes = factorize(L);
  int64_t s1 = 1;
  for (auto& pe : primes)
    if (vexp(a, pe.first) == vexp(s, pe.first)) s1 *= pe.first;
  int64_t k1, k2;
  int64_t X = egcd(s1 * a + s, b, &k1, &k2);
  const int64_t modulus = a * b / X;
  int64_t s0 = 0;
  bool ok = false;
  if (k1 != 0) {
    int64_t lrest = k1;
    int64_t t1 = 1, t2 = 1;
    bool overflow = false;
    for (auto& pe : primes) {
      int64_t p = pe.first;
      int kap = 0;
      while (lrest % p == 0) { lrest /= p; ++kap; }
      int al = vexp(a, p), be = vexp(b, p), ga = vexp(X, p);
      int e1 = be - ga - kap;
      if (e1 < 0) e1 = 0;
      int e2 = al + kap - ga;
      if (e2 < 0 || e1 > 62 || e2 > 62) { overflow = true; break; }
      t1 *= ipow(p, e1);
      t2 *= ipow(p, e2);
    }
    if (!overflow) {
      __int128 cand = (__int128)(t1 - lrest) * t2;
      // reduce the candidate mod the period of the chirp, 2L, keeping its class
      int64_t c = int64_t(cand % (__int128)(2 * L));
      __int128 chk = (__int128)c * X + (__int128)a * k1;
      if (chk % modulus == 0) {
        s0 = c;
        ok = true;
      }
    }
  }
  if (!ok) {
    // Fallback: solve s0 X = -a k1 (mod a b / X) directly.
    int64_t u, v;
    int64_t gX = egcd(X % modulus, modulus, &u, &v);
    int64_t rhs = fmod64(-mulmod(a % modulus, fmod64(k1, modulus), modulus), modulus);
    if (rhs % gX != 0) {
      if (err) *err = "shear factorisation failed (eq. modcond has no solution)";
      r.br = 0;
      return r;
    }
    int64_t m2 = modulus / gX;
    s0 = fmod64(mulmod(fmod64(u, m2), (rhs / gX) % m2, m2), m2);
  }
  // keep s0 in (-L, L]: the chirps depend on s0 mod 2L only, and the
  // post-processing constants are reduced with the same representative
  s0 = fmod64(s0, 2 * L);
  if (s0 > L) s0 -= 2 * L;
  if (s0 == 0) {
    // s0 = 0 would mean a time shear alone works, which was ruled out above
    if (err) *err = "internal: frequency shear reduced to zero";
    r.br = 0;
    return r;
  }
  r.s0 = s0;
  r.s1 = s1;
  r.br = X;
  r.constructed = true;
  return r;
}

bool fft_schedule(int64_t n, FftSchedule* out) {
  FftSchedule fs;
  fs.n = int(n);
  if (n < 1 || n > kMaxFft) return false;
  int64_t m = n;
  int e2 = 0, e3 = 0, e5 = 0, e7 = 0;
  while (m % 2 == 0) { m /= 2; ++e2; }
  while (m % 3 == 0) { m /= 3; ++e3; }
  while (m % 5 == 0) { m /= 5; ++e5; }
  while (m % 7 == 0) { m /= 7; ++e7; }
  if (m != 1) return false;
  int r8 = e2 / 3, rem = e2 % 3;
  auto push = [&](int r) { fs.rad[fs.nst++] = int8_t(r); };
  if (rem == 1 && r8 > 0) {
    for (int i = 0; i < r8 - 1; ++i) push(8);
    push(4);
    push(4);
  } else {
    for (int i = 0; i < r8; ++i) push(8);
    if (rem == 1) push(2);
    if (rem == 2) push(4);
  }
  for (int i = 0; i < e7; ++i) push(7);
  for (int i = 0; i < e5; ++i) push(5);
  for (int i = 0; i < e3; ++i) push(3);
  if (fs.nst > kMaxStages) return false;
  *out = fs;
  return true;
}

void unit_root(int64_t num, int64_t den, double* re, double* im) {
  num = fmod64(num, den);
  // reduce to the first octant with exact integer comparisons
  const long double twopi = 6.283185307179586476925286766559005768L;
  long double x = (long double)num / (long double)den;
  long double s = sinl(twopi * x), c = cosl(twopi * x);
  // exact values on the axes
  if (4 * num == 0) { s = 0; c = 1; }
  else if (4 * num == den) { s = 1; c = 0; }
  else if (2 * num == den) { s = 0; c = -1; }
  else if (4 * num == 3 * den) { s = -1; c = 0; }
  *re = double(c);
  *im = double(s);
}

static void fill_twiddles(int64_t n, std::vector<double>* v) {
  v->resize(2 * n);
  for (int64_t e = 0; e < n; ++e) unit_root(-e, n, &(*v)[2 * e], &(*v)[2 * e + 1]);
}

// pchirp(L, s)(l) = exp(pi i s (L+1) l^2 / L) = exp(2 pi i r / (2L)),
// r = s (L+1) l^2 mod 2L, reduced exactly factor by factor (Lemma 1).
static void fill_chirp(int64_t L, int64_t s, std::vector<double>* v) {
  const int64_t twoL = 2 * L;
  const int64_t K = mulmod(fmod64(s, twoL), fmod64(L + 1, twoL), twoL);
  v->resize(2 * L);
  for (int64_t l = 0; l < L; ++l) {
    int64_t l2 = mulmod(l, l, twoL);
    int64_t r = mulmod(K, l2, twoL);
    unit_root(r, twoL, &(*v)[2 * l], &(*v)[2 * l + 1]);
  }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int plan_make(int64_t L, int64_t a, int64_t M, int64_t lam1, int64_t lam2, int dtype,
              int64_t max_batch, int algorithm, Plan* P, std::string* err, int64_t fir_start, int64_t fir_len,
              int64_t ola_block, int ola_inner) {
  // status codes mirror include/dgtns.h
  const int kEInval = 1, kELattice = 2, kEUnsupported = 4;
  if (dtype != 0 && dtype != 1) { *err = "dtype must be DGTNS_C64 or DGTNS_C128"; return kEInval; }
  if (algorithm != kAlgShear && algorithm != kAlgMultiwindow && algorithm != kAlgFir &&
      algorithm != kAlgShearOla && algorithm != kAlgAuto) {
    *err = "algorithm must be DGTNS_ALG_SHEAR, DGTNS_ALG_MULTIWINDOW, DGTNS_ALG_FIR, DGTNS_ALG_SHEAR_OLA or DGTNS_ALG_AUTO";
    return kEInval;
  }
  if (algorithm == kAlgAuto) {
    // The shear plan, unless it needs a frequency shear (a length-L
    // transform pair and Alg. 1's scattered output permutation, measured at
    // 2.3-3.3x the multiwindow plan on such lattices) and the multiwindow
    // lattice keeps p small enough (measured faster up to p = 15).
    int rc = plan_make(L, a, M, lam1, lam2, dtype, max_batch, kAlgShear, P, err);
    if (rc != 0 || P->branch != kFreqShear) return rc;
    const int64_t ai = lam2 * a, pmw = ai / gcd64(ai, M);
    if (pmw > kAutoMaxP) return rc;
    Plan mw;
    std::string e2;
    if (plan_make(L, a, M, lam1, lam2, dtype, max_batch, kAlgMultiwindow, &mw, &e2) == 0) *P = std::move(mw);
    return 0;
  }
  if (L < 1 || a < 1 || M < 1 || max_batch < 1) { *err = "L, a, M and max_batch must be positive"; return kEInval; }
  if (L > kMaxL) { *err = "L above 2^30 is not supported"; return kEUnsupported; }
  if (L % a || L % M) { *err = "a and M must divide L"; return kELattice; }
  if (lam2 < 1 || lam1 < 0 || lam1 >= lam2 || gcd64(lam1, lam2) != 1) {
    *err = "lattice offset must be lambda1/lambda2 with 0 <= lambda1 < lambda2 and gcd 1 (0/1 for separable)";
    return kELattice;
  }
  // feasible lengths are the multiples of lambda2 lcm(a, M) (Prop. 8)
  if (L % (lam2 * lcm64(a, M)) != 0) {
    *err = "L is not a multiple of lambda2 * lcm(a, M) (minimal feasible length)";
    return kELattice;
  }
  Plan& p = *P;
  p = Plan();
  p.L = L; p.a = a; p.M = M; p.lam1 = lam1; p.lam2 = lam2;
  p.b = L / M; p.N = L / a;
  p.s = p.b * lam1 / lam2;   // absolute shear in normal form (Section 2.1)
  p.dtype = dtype;
  p.max_batch = max_batch;
  {
    const char* gen = std::getenv("DGTNS_GENERIC");
    p.generic = gen && gen[0] == '1';
  }
  if (algorithm == kAlgShearOla) {
    // Shear-OLA (Section 4): blocks of ola_block samples, each zero-extended
    // and transformed by the shear algorithm at a length L_x on the same
    // lattice, then overlap-added with the phase of the block's position
    if (fir_len < 1 || fir_len > L) { *err = "window support length must be in [1, L]"; return kEInval; }
    if (ola_inner != kAlgShear && ola_inner != kAlgMultiwindow && ola_inner != kAlgAuto) {
      *err = "the block transform's algorithm must be DGTNS_ALG_SHEAR, DGTNS_ALG_MULTIWINDOW or DGTNS_ALG_AUTO";
      return kEInval;
    }
    const int64_t Lb = ola_block;
    if (Lb < 1 || L % Lb) { *err = "block length must divide L"; return kEInval; }
    if (Lb % (lam2 * a)) { *err = "block length must be a multiple of lambda2 a"; return kEInval; }
    const int64_t Nb = L / Lb;
    if (max_batch * Nb > 65535) { *err = "max_batch * L / block above 65535"; return kEInval; }
    // signed window start s: the support of position n is n a + s + [0, g_len)
    int64_t sg = fmod64(fir_start, L);
    if (2 * sg >= L) sg -= L;
    // local positions before the block, P0 (a multiple of lambda2 so that the
    // offsets w(n) of the block's DGT are the global ones); the block starts
    // at local sample J0 = P0 a - s >= g_len - a, so no window that wraps
    // around the block DGT's length reaches the block's samples
    const int64_t need = std::max<int64_t>(fir_len - a, 0) + sg;
    int64_t P0 = need > 0 ? (need + a - 1) / a : 0;
    P0 = (P0 + lam2 - 1) / lam2 * lam2;
    const int64_t J0 = P0 * a - sg;
    // the least feasible length L_x = N_x a >= J0 + L_b of the block DGT
    const int64_t step = lam2 * lcm64(a, M) / a;   // N_x steps between feasible lengths
    int64_t Nx = (J0 + Lb + a - 1) / a;
    Nx = (Nx + step - 1) / step * step;
    auto in = std::make_shared<Plan>();
    bool ok = false;
    std::string e2;
    // L_x + g_len <= L: a window offset in (-L_x, L_x) cannot alias the
    // support of the global window modulo L.  The block DGT's algorithm is
    // ola_inner (by default the automatic choice: the shear plan, or the
    // multiwindow plan where the shear plan needs a frequency shear).
    for (int k = 0; k < 64 && Nx * a + fir_len <= L; ++k, Nx += step) {
      if (plan_make(Nx * a, a, M, lam1, lam2, dtype, max_batch * Nb, ola_inner, in.get(), &e2) == 0) {
        ok = true;
        break;
      }
    }
    if (!ok) {
      *err = "no feasible block DGT length below L for this block length (" + e2 + ")";
      return kEUnsupported;
    }
    p.branch = kShearOla;
    p.sh = in->sh;
    p.ai = in->ai; p.Mi = in->Mi; p.bi = in->bi; p.Ni = in->Ni;
    p.ci = in->ci; p.pi = in->pi; p.qw = in->qw; p.qi = in->qi; p.di = in->di; p.nw = in->nw;
    p.fir_start = fmod64(fir_start, L);
    p.fir_len = fir_len;
    p.ola_Lb = Lb; p.ola_Nb = Nb; p.ola_Nx = Nx; p.ola_Lx = Nx * a; p.ola_P0 = P0; p.ola_J0 = J0; p.ola_s = sg;
    p.fir_ph.resize(2 * lam2 * M);
    for (int64_t e = 0; e < lam2 * M; ++e) unit_root(-e, lam2 * M, &p.fir_ph[2 * e], &p.fir_ph[2 * e + 1]);
    const size_t es = dtype == 0 ? 8 : 16;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    p.off = Plan::Off();
    p.off.inner = take(in->off.total);
    p.off.fir_ph = take(es * lam2 * M);
    p.off.bounds = take(16);
    p.off.total = o;
    p.inner = in;
    return 0;
  }
  if (algorithm == kAlgFir) {
    // FIR-window algorithm: per time position the windowed samples folded
    // modulo M and one length-M DFT; needs the M-point transform and the
    // lambda2 M phases exp(-2 pi i e / (lambda2 M)) of the offsets w(n)
    if (fir_len < 1 || fir_len > L) { *err = "window support length must be in [1, L]"; return kEInval; }
    if (!fft_schedule(M, &p.fm)) {
      *err = "channel count M = " + std::to_string(M) + " must be 7-smooth and at most 4096";
      return kEUnsupported;
    }
    p.branch = kFir;
    p.sh.br = p.b;
    p.ai = a; p.Mi = M; p.bi = p.b; p.Ni = p.N;
    p.ci = p.pi = p.qw = p.qi = p.di = 0;
    p.fir_start = fmod64(fir_start, L);
    p.fir_len = fir_len;
    fill_twiddles(M, &p.tw_m);
    if (lam2 > 1) {
      p.fir_ph.resize(2 * lam2 * M);
      for (int64_t e = 0; e < lam2 * M; ++e) unit_root(-e, lam2 * M, &p.fir_ph[2 * e], &p.fir_ph[2 * e + 1]);
    }
    const size_t es = dtype == 0 ? 8 : 16;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    p.off = Plan::Off();
    p.off.tw_m = take(es * M);
    p.off.tw_m64 = dtype == 0 ? take(16 * M) : p.off.tw_m;   // FP64 copy, uploaded for every FP32 plan
    p.off.fir_ph = p.fir_ph.empty() ? 0 : take(es * lam2 * M);
    p.off.zc = take(es * fir_len);   // conj of the window support
    p.off.bounds = take(16);
    p.off.total = o;
    return 0;
  }
  if (algorithm == kAlgMultiwindow) {
    // Prop. 4: the lattice is the union of lambda2 cosets of the separable
    // lattice (lambda2 a, M); no shear is used
    p.branch = kMultiwindow;
    p.sh.br = p.b;
  } else {
    p.sh = shearfind(L, a, M, p.s, p.b, err);
    if (p.sh.br == 0) return kELattice;
    if (p.s == 0) p.branch = kSeparable;
    else if (p.sh.s0 == 0) p.branch = kTimeShear;
    else p.branch = kFreqShear;
  }

  const int64_t N = p.N, b = p.b;
  if (p.branch == kMultiwindow) {
    p.ai = lam2 * a; p.Mi = M;
  } else if (p.branch != kFreqShear) {
    p.ai = a; p.Mi = M;
  } else {
    // Alg. 1, frequency-shear branch: separable DGT with time step b_r and
    // N_r channels on the Fourier transform of the chirped signal
    p.ar = a * b / p.sh.br;
    p.Mr = L / p.sh.br;
    p.Nr = L / p.ar;
    p.ai = p.sh.br; p.Mi = p.Nr;
    const int64_t twoN = 2 * N;
    int64_t C1 = p.ar / a;
    if (((__int128)p.sh.s0 * p.sh.br) % a != 0) {
      *err = "internal: s0 b_r not divisible by a";
      return kELattice;
    }
    __int128 C2 = -(__int128)p.sh.s0 * p.sh.br / a;
    __int128 C3 = (__int128)a * p.sh.s1 * (L + 1);
    __int128 C4 = C2 * p.sh.br * (L + 1);
    __int128 C5 = (__int128)2 * C1 * p.sh.br;
    __int128 C6 = ((__int128)p.sh.s0 * p.sh.s1 + 1) * p.sh.br;
    auto red = [](__int128 x, int64_t m) { __int128 r = x % m; if (r < 0) r += m; return int64_t(r); };
    p.K1 = red(C1, twoN); p.K2 = red(C2, twoN); p.K3 = red(C3, twoN);
    p.K4 = red(C4, twoN); p.K5 = red(C5, twoN);
    p.C1n = red(C1, N); p.C2n = red(C2, N);
    p.Kt1 = red(-(__int128)p.sh.s1 * p.ar, L);
    p.Kt6 = red(C6, L);
  }
  p.bi = L / p.Mi;
  p.Ni = L / p.ai;
  p.ci = gcd64(p.ai, p.Mi);
  p.pi = p.ai / p.ci;
  p.qw = p.Mi / p.ci;
  p.nw = p.branch == kMultiwindow ? lam2 : 1;
  p.qi = p.nw * p.qw;
  p.di = p.bi / p.pi;
  if (p.branch != kFreqShear && p.di <= kMaxFft) {
    // opt-in (DGTNS_CHUNK_MIB): chunks of about that many MiB of h, two in flight
    const int64_t per_sig = p.qi * p.Mi * p.di * (dtype == 0 ? 8 : 16);
    const char* cm = std::getenv("DGTNS_CHUNK_MIB");
    if (cm && std::atoi(cm) > 0) {
      p.chunk = (int64_t(std::atoi(cm)) << 20) / per_sig;
      if (p.chunk < 1) p.chunk = 1;
    }
    // Sequential chunks of about 128 MiB of h (DGTNS_SEQ_MIB overrides; 0
    // turns them off): used by calls whose whole h would not stay in the
    // 256 MB last-level cache, while one chunk of h does.
    const char* sm = std::getenv("DGTNS_SEQ_MIB");
    const int64_t seq_mib = sm ? std::atoi(sm) : 128;
    if (seq_mib > 0 && !p.chunk) p.seq = (seq_mib << 20) / per_sig;
  }

  // LDS element budget per work-group: 8192 complex elements (FP32) or 4096 (FP64)
  const int64_t budget = dtype == 0 ? 8192 : 4096;
  if (!fft_schedule(p.Mi, &p.fm)) {
    *err = "channel count M = " + std::to_string(p.Mi) + " must be 7-smooth and at most 4096";
    return kEUnsupported;
  }
  int64_t W = 1;
  // in-LDS columns: the p sub-columns of a column within the element budget,
  // and within the LDS of the FP64 window Zak transform (16 bytes per value)
  if (fft_schedule(p.di, &p.fd) && p.pi * p.di <= budget && 16 * (p.di + p.pi * (p.di | 1)) <= (160 << 10)) {
    const int64_t Sd = p.di | 1;
    W = 16;
    while (W > 1 && (W * p.pi * p.di > budget || W * (p.pi * Sd + (p.pi > 1 ? Sd : 0)) > budget + 64 * W))
      --W;
  } else {
    // long columns: d = d1 d2, both 7-smooth in-LDS lengths, the middle pass
    // holding p sub-columns of length d2 per column (p d2 <= 4096, the FP64
    // capacity used by the window transform); the most balanced split
    int64_t best = 0;
    double bestq = 1e300;
    for (int64_t a2 = 2; a2 <= kMaxFft && a2 <= p.di; ++a2) {
      if (p.di % a2) continue;
      const int64_t a1 = p.di / a2;
      FftSchedule s1, s2;
      if (a1 < 2 || a1 > kMaxFft || p.pi * a2 > 4096) continue;
      if (!fft_schedule(a1, &s1) || !fft_schedule(a2, &s2)) continue;
      const double qd = std::fabs(std::log(double(a1)) - std::log(double(a2)));
      if (qd < bestq) { bestq = qd; best = a2; }
    }
    if (best == 0) {
      *err = "column length d = " + std::to_string(p.di) + " (p = " + std::to_string(p.pi) +
             ") has no split d1 d2 into 7-smooth in-LDS lengths";
      return kEUnsupported;
    }
    if (p.branch == kMultiwindow) {
      *err = "multiwindow plans need columns of at most 4096 values (d = " + std::to_string(p.di) + ")";
      return kEUnsupported;
    }
    p.longd = true;
    p.d2 = best;
    p.d1 = p.di / best;
    fft_schedule(p.d1, &p.fd1);
    fft_schedule(p.d2, &p.fd2);
    const int64_t es = dtype == 0 ? 8 : 16, S2 = p.d2 | 1;
    int64_t wm = 16;
    while (wm > 1 && (wm * p.pi * p.d2 > budget || es * (p.d2 + wm * (p.pi + 1) * S2) > (64 << 10))) --wm;
    p.Wm = int(wm);
    const int64_t wl = budget / (p.d1 | 1);
    p.Wl = int(wl > 16 ? 16 : (wl < 1 ? 1 : wl));
    p.chunk = 0;
    p.seq = 0;
  }
  if (p.Mi > budget) {
    *err = "channel count exceeds the in-LDS limit";
    return kEUnsupported;
  }
  p.W = int(W);
  if (p.branch == kFreqShear) {
    // L = L1 * L2 for the two-pass transform of length L
    int64_t best = 0;
    for (int64_t d1 = 1; d1 * d1 <= L; ++d1) {
      if (L % d1) continue;
      int64_t d2 = L / d1;
      FftSchedule t1, t2;
      if (d2 <= budget && d1 <= kMaxFft && d2 <= kMaxFft && fft_schedule(d1, &t1) && fft_schedule(d2, &t2))
        best = d1;
    }
    if (best == 0) {
      *err = "signal length cannot be split into two in-LDS transform lengths";
      return kEUnsupported;
    }
    p.L1 = best;
    p.L2 = L / best;
    fft_schedule(p.L1, &p.f1);
    fft_schedule(p.L2, &p.f2);
  }

  // ---- host tables (FP64) ----
  fill_twiddles(p.di, &p.tw_d);
  fill_twiddles(p.Mi, &p.tw_m);
  if (p.longd) {
    fill_twiddles(p.d1, &p.tw_d1);
    fill_twiddles(p.d2, &p.tw_d2);
  }
  if (p.branch == kTimeShear || p.branch == kFreqShear) fill_chirp(L, p.sh.s1, &p.chirp1);
  if (p.branch == kMultiwindow) {
    // Prop. 5: c(m, nt lambda2 + mu) = exp(-2 pi i nt (lambda2 a) sigma_mu / L)
    // c_mu(m, nt), c_mu the separable DGT of f with the coset window g_mu
    p.post_E.resize(2 * N);
    p.post_rho.assign(N, 0);
    for (int64_t n = 0; n < N; ++n) {
      const int64_t nt = n / lam2, mu = n % lam2;
      const int64_t e = mulmod(mulmod(nt, p.ai, L), mw_sigma(p, mu), L);
      unit_root(fmod64(-e, L), L, &p.post_E[2 * n], &p.post_E[2 * n + 1]);
    }
  } else if (p.branch == kFreqShear) {
    fill_twiddles(p.L1, &p.tw_1);
    fill_twiddles(p.L2, &p.tw_2);
    fill_twiddles(L, &p.tw_L);
    fill_chirp(L, -p.sh.s0, &p.chirp0);
  } else {
    // Alg. 1, time-shear branch: c((m + rho_n) mod M, n) = E_n c_r(m, n) with
    // E_n = exp(pi i (C1 n^2 mod 2N) / N), C1 = s1 a (L+1) mod 2N,
    // rho_n = floor(((-s1 n a) mod L) / b)
    const int64_t twoN = 2 * N;
    int64_t C1 = int64_t(((__int128)p.sh.s1 * a % twoN * ((L + 1) % twoN)) % twoN);
    C1 = fmod64(C1, twoN);
    p.post_E.resize(2 * N);
    p.post_rho.resize(N);
    const int64_t ms1a = fmod64(-(int64_t)((__int128)p.sh.s1 * a % L), L);
    for (int64_t n = 0; n < N; ++n) {
      int64_t e = mulmod(C1, mulmod(n, n, twoN), twoN);
      unit_root(e, twoN, &p.post_E[2 * n], &p.post_E[2 * n + 1]);
      p.post_rho[n] = int32_t(mulmod(ms1a, n, L) / b);
    }
  }

  // ---- device memory map ----
  const size_t es = dtype == 0 ? 8 : 16;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  p.off.tw_d = take(es * p.di);
  p.off.tw_m = take(es * p.Mi);
  p.off.tw_d1 = p.off.tw_d2 = p.off.tw_d1_64 = p.off.tw_d2_64 = 0;
  if (p.longd) {
    p.off.tw_d1 = take(es * p.d1);
    p.off.tw_d2 = take(es * p.d2);
    p.off.tw_d1_64 = dtype == 0 ? take(16 * p.d1) : p.off.tw_d1;
    p.off.tw_d2_64 = dtype == 0 ? take(16 * p.d2) : p.off.tw_d2;
  }
  p.off.chirp1 = p.chirp1.empty() ? 0 : take(es * L);
  p.off.tw_1 = p.off.tw_2 = p.off.tw_L = p.off.chirp0 = 0;
  p.off.tw_1_64 = p.off.tw_2_64 = p.off.tw_L64 = 0;
  if (p.branch == kFreqShear) {
    p.off.tw_1 = take(es * p.L1);
    p.off.tw_2 = take(es * p.L2);
    p.off.tw_L = take(es * L);
    p.off.chirp0 = take(es * L);
  }
  p.off.post_E = p.post_E.empty() ? 0 : take(es * N);
  p.off.post_rho = p.post_rho.empty() ? 0 : take(4 * N);
  p.off.zc = take(es * L * p.nw);   // one Zak table of L values per window
  if (dtype == 0) {
    p.off.tw_d64 = take(16 * p.di);
    p.off.tw_m64 = take(16 * p.Mi);
    if (p.branch == kFreqShear) {
      p.off.tw_1_64 = take(16 * p.L1);
      p.off.tw_2_64 = take(16 * p.L2);
      p.off.tw_L64 = take(16 * L);
    }
  } else {
    p.off.tw_d64 = p.off.tw_d;
    p.off.tw_m64 = p.off.tw_m;
    p.off.tw_1_64 = p.off.tw_1;
    p.off.tw_2_64 = p.off.tw_2;
    p.off.tw_L64 = p.off.tw_L;
  }
  p.off.bounds = take(16);
  p.off.total = o;
  return 0;
}

}  // namespace dgtns
