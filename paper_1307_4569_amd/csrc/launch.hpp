// Host-side launchers of libdgtns: workspace layout, per-stage kernel
// launches and the compositions of Alg. 1 (forward), its adjoint, the window
// gradient, the window preparation and the dual window (Alg. 2).  Included by
// one translation unit per precision.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dgtns.h"
#include "kernels.hpp"
#include "kernels_fast.hpp"
#include "kernels_long.hpp"
#include "kernels_fir.hpp"
#include "kernels_ola.hpp"
#include "plan.hpp"

namespace dgtns {
namespace host {

// records the message of the last error of the calling thread
void set_last_error(const std::string& msg);

inline int fail(int status, const std::string& msg) {
  set_last_error(msg);
  return status;
}

inline int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(DGTNS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return DGTNS_OK;
}

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Dry run of a call (per thread): every launcher checks its launch (LDS
// request, workspace pointers, supported sizes) and returns without
// enqueueing anything.  Each entry point runs its body dry first, so every
// refusal is reported before the first kernel of the call is enqueued.
bool dry_run();

// ---------------------------------------------------------------------------
// Two-stream pipeline over chunks of the batch (time-shear branch): stage 1
// of chunk k runs on the caller's stream into h buffer k mod 2, stage 2 of
// chunk k on a helper stream of the device as soon as stage 1 is done, so
// stage 1 of chunk k+1 overlaps stage 2 of chunk k and each h buffer is read
// back while it is still in the last-level cache.  The caller's stream waits
// for the last stage 2 before the call returns.
// ---------------------------------------------------------------------------
hipStream_t helper_stream();          // per device, created once (default priority)
hipEvent_t take_sync_event();
void give_sync_event(hipEvent_t e);

// True while a call that must not create streams or events runs (per
// thread): the two-stream pipeline is then not used.
bool no_pipeline();

// True while a call of the real-signal variant runs (per thread): the
// launchers then read and write coefficients in the real-signal layout and
// the synthesis writes real samples.  A scope that must use the full layout
// (the inner blocks of shear-OLA) sets it with FullLayoutScope.
bool real_call();
void set_real_call(bool on);
struct FullLayoutScope {
  bool saved;
  FullLayoutScope() : saved(real_call()) { set_real_call(false); }
  ~FullLayoutScope() { set_real_call(saved); }
};

// Values per group of lambda2 columns in the real-signal layout: lambda2 M
// minus the omitted channels of the one or two half-stored columns.
inline long long real_row(const Plan& P) {
  const long long M2 = P.M / 2 + 1;
  return P.lam2 * P.M - (P.M - M2) * (P.lam2 % 2 == 0 ? 2 : 1);
}
// Coefficients per signal in the layout of the current call.
inline long long coef_per_signal(const Plan& P) { return real_call() ? P.N / P.lam2 * real_row(P) : P.M * P.N; }
inline CoefLayout coef_layout(const Plan& P) {
  CoefLayout R;
  R.real = real_call() ? 1 : 0;
  R.lam2 = int(P.lam2);
  R.M = int(P.M);
  R.M2 = int(P.M / 2 + 1);
  R.S = real_call() ? real_row(P) : P.M;
  return R;
}

inline bool pipelined(const Plan& P, long long B, int op) {
  return op == DGTNS_OP_FORWARD && P.chunk > 0 && B >= 2 * P.chunk && !no_pipeline();
}

// Sequential chunks of the forward and the adjoint: one h buffer of P.seq
// signals, reused, when the whole batch's h is at least 256 MiB.  Only for
// FP32 columns of 32 to 512 values on the wave kernels, whose factorisation
// kernels hold two work-groups per compute unit: with one (FP64, or FP32
// d = 1024) a chunk's launch fills the GPU once or twice with work-groups in
// the same phase, and the chunks were measured slower than one launch.
inline bool seq_chunked(const Plan& P, long long B, int op) {
  if (op != DGTNS_OP_FORWARD && op != DGTNS_OP_ADJOINT) return false;
  if (P.seq < 1 || B <= P.seq || P.branch == kFreqShear || P.longd || P.branch == kFir || P.branch == kShearOla)
    return false;
  if (P.dtype != 0 || P.pi != 1 || P.generic || P.di < 32 || P.di > 512 || (P.di & (P.di - 1)) != 0) return false;
  const double h_bytes = double(P.qi) * double(P.Mi) * double(P.di) * double(B) * (P.dtype == 0 ? 8.0 : 16.0);
  return h_bytes >= double(256ll << 20);
}

template <typename S1, typename S2>
int run_pipeline(long long B, long long chunk, hipStream_t st, S1 stage1, S2 stage2) {
  const long long nch = (B + chunk - 1) / chunk;
  if (dry_run()) {   // the stages of every chunk, no streams or events
    for (long long k = 0; k < nch; ++k) {
      const long long b0 = k * chunk, nb = B - b0 < chunk ? B - b0 : chunk;
      int rc = stage1(b0, nb, int(k & 1), st);
      if (!rc) rc = stage2(b0, nb, int(k & 1), st);
      if (rc) return rc;
    }
    return DGTNS_OK;
  }
  hipStream_t hs = helper_stream();
  if (!hs) return fail(DGTNS_EDEVICE, "could not create the helper stream");
  hipEvent_t eA[2] = {take_sync_event(), take_sync_event()};
  hipEvent_t eB[2] = {take_sync_event(), take_sync_event()};
  int rc = DGTNS_OK;
  long long last = -1;
  for (long long k = 0; k < nch && rc == DGTNS_OK; ++k) {
    const long long b0 = k * chunk, nb = B - b0 < chunk ? B - b0 : chunk;
    const int buf = int(k & 1);
    if (k >= 2) rc = check_hip(hipStreamWaitEvent(st, eB[buf], 0), "pipeline wait");
    if (!rc) rc = stage1(b0, nb, buf, st);
    if (!rc) rc = check_hip(hipEventRecord(eA[buf], st), "pipeline record");
    if (!rc) rc = check_hip(hipStreamWaitEvent(hs, eA[buf], 0), "pipeline wait");
    if (!rc) rc = stage2(b0, nb, buf, hs);
    if (!rc) rc = check_hip(hipEventRecord(eB[buf], hs), "pipeline record");
    if (!rc) last = k;
  }
  if (last >= 0) {
    int rc2 = check_hip(hipStreamWaitEvent(st, eB[last & 1], 0), "pipeline wait");
    if (!rc) rc = rc2;
  }
  for (int i = 0; i < 2; ++i) {
    give_sync_event(eA[i]);
    give_sync_event(eB[i]);
  }
  return rc;
}



// Optional per-kernel timing: every launch bracketed by two HIP events on
// the launch stream; dgtns_timing_collect() waits for them and aggregates.
struct Timing {
  std::mutex mu;
  bool on = false;
  struct Rec { std::string name; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  struct Agg { long long n = 0; double ms = 0; };
  std::vector<std::pair<std::string, Agg>> agg;
};
Timing& timing();
inline hipEvent_t take_event(Timing& t) {
  if (!t.pool.empty()) { hipEvent_t e = t.pool.back(); t.pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

template <typename K, typename... A>
int launch_raw(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st, const char* name, A... args) {
  if (dry_run()) return DGTNS_OK;
  Timing& t = timing();
  hipEvent_t ea = nullptr, eb = nullptr;
  if (t.on) {
    std::lock_guard<std::mutex> g(t.mu);
    ea = take_event(t);
    eb = take_event(t);
  }
  if (ea) hipEventRecord(ea, st);
  hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
  int rc = check_hip(hipGetLastError(), name);
  if (eb) {
    hipEventRecord(eb, st);
    std::lock_guard<std::mutex> g(t.mu);
    t.recs.push_back({name, ea, eb});
  }
  return rc;
}

// 512-thread launch with any kernel arguments: empty grids are no-ops, LDS
// requests above 64 KiB are granted up to the 160 KiB of a compute unit.
template <typename K, typename... A>
int launch_v(K kernel, dim3 grid, size_t lds, hipStream_t st, const char* name, A... args) {
  if (grid.x == 0 || grid.y == 0) return DGTNS_OK;
  if (lds > 160 * 1024) return fail(DGTNS_EUNSUPPORTED, std::string(name) + ": LDS request above 160 KiB");
  if (dry_run()) return DGTNS_OK;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return check_hip(e, name);
  }
  return launch_raw(kernel, grid, dim3(kThreads), lds, st, name, args...);
}

template <typename K, typename A>
int launch(K kernel, dim3 grid, size_t lds, hipStream_t st, const A& args, const char* name) {
  return launch_v(kernel, grid, lds, st, name, args);
}

// launch with `threads` threads per work-group (the kernel's launch bounds)
template <typename K, typename A>
int launch_t(K kernel, dim3 grid, unsigned threads, size_t lds, hipStream_t st, const A& args, const char* name) {
  if (grid.x == 0 || grid.y == 0) return DGTNS_OK;
  if (lds > 160 * 1024) return fail(DGTNS_EUNSUPPORTED, std::string(name) + ": LDS request above 160 KiB");
  if (dry_run()) return DGTNS_OK;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return check_hip(e, name);
  }
  return launch_raw(kernel, grid, dim3(threads), lds, st, name, args);
}

inline unsigned cdiv(long long a, long long b) { return unsigned((a + b - 1) / b); }

// Device address of a table in the plan's persistent block (integer
// arithmetic: a dry run of an unbound plan computes addresses it never uses).
template <typename C> const C* tab(const Plan& P, size_t off) {
  return reinterpret_cast<const C*>(reinterpret_cast<uintptr_t>(P.dev) + off);
}
template <typename C> C* mtab(const Plan& P, size_t off) {
  return reinterpret_cast<C*>(reinterpret_cast<uintptr_t>(P.dev) + off);
}

inline FftSched sched(const FftSchedule& s) {
  FftSched f;
  f.n = s.n;
  f.nst = s.nst;
  for (int i = 0; i < 20; ++i) f.rad[i] = s.rad[i];
  return f;
}

inline long long chirpK(const Plan& P, long long s) {
  const long long twoL = 2 * P.L;
  return mulmod(fmod64(s, twoL), fmod64(P.L + 1, twoL), twoL);
}

// elements per work-group for column/row transforms of length n
inline int block_width(long long n, int es, int maxw = 16) {
  const long long budget = es == 8 ? 8192 : 4096;
  long long w = budget / n;
  if (w > maxw) w = maxw;
  if (w < 1) w = 1;
  return int(w);
}

struct Layout {
  size_t H = 0, F = 0, Y = 0, part = 0, G = 0, U = 0, V = 0, total = 0;
  // shear-OLA: zero-extended blocks, their coefficients, the inner workspace
  size_t ola_x = 0, ola_c = 0, inner = 0;
};

// Values of the intermediate h per signal: q offsets x Mi columns x d
// (= Mi Ni for the shear algorithm, nw Mi Ni for nw coset windows).
inline long long h_per_signal(const Plan& P) { return P.qi * P.Mi * P.di; }

// Stream the stores of h when a launch's h (B signals) cannot stay in the
// 256 MB last-level cache for the kernel that reads it next; the same for a
// launch's coefficients (their dirty lines would otherwise be written back
// while the next kernel runs).
inline int stream_h(const Plan& P, long long B, size_t es) {
  return double(h_per_signal(P)) * double(B) * double(es) >= double(256ll << 20) ? 1 : 0;
}
inline int stream_c(const Plan& P, long long B, size_t es) {
  return double(P.M) * double(P.N) * double(B) * double(es) >= double(256ll << 20) ? 1 : 0;
}

inline Layout ws_layout(const Plan& P, int op, long long B) {
  const size_t es = P.dtype == 0 ? 8 : 16;
  const size_t MN = size_t(h_per_signal(P));
  const size_t L = size_t(P.L);
  Layout l;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al256(o + bytes); return r; };
  const bool fs = P.branch == kFreqShear;
  if (P.branch == kShearOla) {
    // blocks and block coefficients, then the inner plan's own workspace
    const long long Bi = B * P.ola_Nb;
    if (op == DGTNS_OP_FORWARD || op == DGTNS_OP_ADJOINT) {
      l.ola_x = take(es * size_t(P.ola_Lx) * Bi);
      l.ola_c = take(es * size_t(P.ola_Nx) * size_t(P.M) * Bi);
      l.inner = take(ws_layout(*P.inner, op, Bi).total);
    } else if (op == DGTNS_OP_SET_WINDOW) {
      l.ola_x = take(16 * size_t(P.ola_Lx));   // the block window, FP64
      l.inner = take(ws_layout(*P.inner, op, 1).total);
    }
    l.total = o < 256 ? 256 : o;
    return l;
  }
  switch (op) {
    case DGTNS_OP_FORWARD:
    case DGTNS_OP_ADJOINT:
      if (P.branch == kFir) {   // the adjoint's inverse DFTs of the columns
        if (op == DGTNS_OP_ADJOINT) l.H = take(es * size_t(P.M) * size_t(P.N) * B);
        break;
      }
      if (pipelined(P, B, op)) {
        l.H = take(es * MN * P.chunk);
        l.F = take(es * MN * P.chunk);   // second h buffer
      } else if (seq_chunked(P, B, op)) {
        l.H = take(es * MN * P.seq);
      } else {
        l.H = take(es * MN * B);
        if (fs) { l.F = take(es * L * B); l.Y = take(es * L * B); }
        if (P.longd) { l.U = take(es * L * B); l.V = take(es * MN * B); }   // two-level column passes
      }
      break;
    case DGTNS_OP_WINDOW_GRAD:
      l.H = take(es * MN * B);
      l.part = take(es * L * B);
      l.U = take(es * L * B);   // column spectra of the wave-kernel path, or first column pass
      if (P.longd) l.V = take(es * MN * B);   // first column pass of h (long columns)
      if (fs) { l.F = take(es * L * B); l.Y = take(es * L * B); l.G = take(es * L); }
      break;
    case DGTNS_OP_SET_WINDOW:
      if (fs) { l.Y = take(16 * L); l.G = take(16 * L); }
      if (P.longd) l.U = take(16 * L);
      break;
    case DGTNS_OP_DUAL:
      l.H = take(16 * L);   // Zak of the sheared window
      l.F = take(16 * L);   // divided Zak
      l.G = take(16 * L);   // separable dual / frequency-domain dual
      if (fs) l.Y = take(16 * L);
      if (P.longd) l.U = take(16 * L);   // between the two inverse column passes
      l.part = take(16 * (size_t(std::max<long long>(cdiv((long long)P.Mi * P.di, kThreads),
                                                      std::min<long long>(P.Mi * P.di, kDualLdsGroups))) + 1));
      break;
    default:
      break;
  }
  l.total = o < 256 ? 256 : o;
  return l;
}


// ---------------------------------------------------------------------------
// stage launchers (templated on precision)
// ---------------------------------------------------------------------------

// Wave-kernel sizes: powers of two from 32 to 1024.
inline bool wave_len(long long n) { return n >= 32 && n <= 1024 && (n & (n - 1)) == 0; }

// The forward runs the wave kernels in both stages, so h can take the
// time-major layout h[n0][t][r] that only those two kernels use.
template <typename C> bool h_time_major(const Plan& P) {
  const bool cols = P.pi == 1 && !P.generic && !P.longd && P.di * long(sizeof(C)) <= 8192 && wave_len(P.di);
  const bool rows = !P.generic && wave_len(P.Mi);
  return cols && rows;
}

// The q offsets of a column block are split over several work-groups (each
// repeats the block's column DFTs) until the launch has about min_wg
// work-groups.
template <typename C, int D, int KF>
int run_cols_fast_k(const Plan& P, const ColArgs<C>& A, long long B, hipStream_t st, long long min_wg) {
  using F = FastCols<C, D, KF>;
  const long long nblk = cdiv(P.Mi, F::W);
  long long ns = (min_wg + nblk * B - 1) / (nblk * B);
  if (ns > P.qi) ns = P.qi;
  if (ns < 1) ns = 1;
  ColArgs<C> A2 = A;
  A2.nsplit = int(ns);
  dim3 grid(unsigned(nblk * ns), unsigned(B));
  if (A2.ht) {
    const size_t lds = sizeof(C) * (KF == 1 ? F::LDS_TS : F::LDS_T);
    if (A2.hstream) return launch(k_fwd_cols_w<C, D, true, true, KF>, grid, lds, st, A2, "factorisation kernel");
    return launch(k_fwd_cols_w<C, D, false, true, KF>, grid, lds, st, A2, "factorisation kernel");
  }
  const size_t lds = sizeof(C) * F::LDS;
  if (A2.hstream) return launch(k_fwd_cols_w<C, D, true, false, KF>, grid, lds, st, A2, "factorisation kernel");
  return launch(k_fwd_cols_w<C, D, false, false, KF>, grid, lds, st, A2, "factorisation kernel");
}

// chunk: the launch is a chunk of a sequential batch (FP32, d <= 512, h in the
// last-level cache): one wave transform per wavefront (8 columns per
// work-group) and at least 512 work-groups, two per compute unit.  Otherwise
// as many transforms per wavefront as fit and at least about 2048
// work-groups (8 per compute unit) for a small batch.
template <typename C, int D>
int run_cols_fast(const Plan& P, const ColArgs<C>& A, long long B, hipStream_t st, bool chunk) {
  if constexpr (sizeof(C) == 8 && D <= 512) {
    if (chunk && !A.hstream) return run_cols_fast_k<C, D, 1>(P, A, B, st, 512);
  }
  return run_cols_fast_k<C, D, 0>(P, A, B, st, 2048);
}

template <typename C, int D>
int run_adj_cols_fast(const Plan& P, const ColAdjArgs<C>& A, long long B, hipStream_t st) {
  using F = FastCols<C, D, 1>;   // as in k_adj_cols_w
  dim3 grid(cdiv(P.Mi, F::W), unsigned(B));
  return launch(k_adj_cols_w<C, D>, grid, sizeof(C) * F::LDS, st, A, "adjoint factorisation kernel");
}

template <typename C, int MI>
int run_rows_fast(const Plan& P, const RowArgs<C>& A, long long B, bool adjoint, hipStream_t st) {
  using F = FastRows<C, MI>;
  using FA = FastRows<C, MI, true>;   // as in k_adj_rows_w
  dim3 grid(unsigned(P.qi) * cdiv(P.di, adjoint ? FA::RB : F::RB), unsigned(B));
  const size_t lds = sizeof(C) * (adjoint ? FA::LDS : F::LDS);
  const bool fs = P.branch == kFreqShear;
  if (!adjoint && A.ht) {
    // rows come straight from h[n0][t][r]: LDS only for the wave exchanges
    const size_t lt = sizeof(C) * 8 * F::EXW;
    if (A.hstream) {
      if (fs) return launch(k_fwd_rows_w<C, MI, 1, true, true>, grid, lt, st, A, "channel DFT + shear post-processing");
      return launch(k_fwd_rows_w<C, MI, 0, true, true>, grid, lt, st, A, "channel DFT + phase correction");
    }
    if (fs) return launch(k_fwd_rows_w<C, MI, 1, false, true>, grid, lt, st, A, "channel DFT + shear post-processing");
    return launch(k_fwd_rows_w<C, MI, 0, false, true>, grid, lt, st, A, "channel DFT + phase correction");
  }
  if (!adjoint) {
    if (A.hstream) {
      if (fs) return launch(k_fwd_rows_w<C, MI, 1, true, false>, grid, lds, st, A, "channel DFT + shear post-processing");
      return launch(k_fwd_rows_w<C, MI, 0, true, false>, grid, lds, st, A, "channel DFT + phase correction");
    }
    if (fs) return launch(k_fwd_rows_w<C, MI, 1, false, false>, grid, lds, st, A, "channel DFT + shear post-processing");
    return launch(k_fwd_rows_w<C, MI, 0, false, false>, grid, lds, st, A, "channel DFT + phase correction");
  }
  if (A.hstream) {
    if (fs) return launch(k_adj_rows_w<C, MI, 1, true>, grid, lds, st, A, "adjoint channel DFT (shear)");
    return launch(k_adj_rows_w<C, MI, 0, true>, grid, lds, st, A, "adjoint channel DFT");
  }
  if (fs) return launch(k_adj_rows_w<C, MI, 1, false>, grid, lds, st, A, "adjoint channel DFT (shear)");
  return launch(k_adj_rows_w<C, MI, 0, false>, grid, lds, st, A, "adjoint channel DFT");
}

// ---------------------------------------------------------------------------
// Two-level column passes (kernels_long.hpp) for columns longer than one
// in-LDS transform; U and V are workspace buffers of L and q Mi d values per
// signal.
// ---------------------------------------------------------------------------
template <typename C>
LongColArgs<C> long_col_args(const Plan& P) {
  LongColArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.pre.L = A.post.L = P.L;
  A.tws = tab<C>(P, P.off.tw_d1);
  A.twd = tab<C>(P, P.off.tw_d);
  A.n = int(P.d1); A.Sn = int(P.d1 | 1); A.W = P.Wl;
  A.d = int(P.di); A.d2 = int(P.d2);
  A.fs = sched(P.fd1);
  return A;
}

template <typename C>
LongMidArgs<C> long_mid_args(const Plan& P, C* U, C* V) {
  LongMidArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.U = U; A.us = P.L; A.V = V; A.vs = h_per_signal(P);
  A.zc = tab<C>(P, P.off.zc); A.zs = P.L;
  A.twd = tab<C>(P, P.off.tw_d); A.tw2 = tab<C>(P, P.off.tw_d2);
  A.Mi = int(P.Mi); A.ai = int(P.ai); A.p = int(P.pi); A.q = int(P.qi); A.qw = int(P.qw);
  A.d = int(P.di); A.d1 = int(P.d1); A.d2 = int(P.d2); A.W = P.Wm; A.Sd2 = int(P.d2 | 1);
  A.ncol = int(P.Mi * P.pi);
  A.fs2 = sched(P.fd2);
  return A;
}

template <typename C>
int run_cols_long(const Plan& P, const void* x, long long xs, int real_in, ChirpSrc<C> ch, C* H, long long B,
                  hipStream_t st, const void* const* xlist, C* U, C* V) {
  if (!U || !V) return fail(DGTNS_EINVAL, "internal: no workspace for the two-level column passes");
  const long long ncol = P.Mi * P.pi, Md = P.Mi * P.di;
  const size_t es = sizeof(C);
  // 1: length-d1 DFTs of the signal with the chirp, twiddle W_d^{t2 k1}
  LongColArgs<C> A = long_col_args<C>(P);
  A.x = x; A.xs = xs; A.real_in = real_in; A.pre = ch;
  if (xlist) {
    A.list = 1;
    for (long long k = 0; k < B; ++k) A.xl[k] = xlist[k];
  }
  A.y = U; A.ys = P.L;
  A.ncols = int(P.d2 * ncol); A.inmode = 0; A.outmode = 0; A.twmode = 1; A.tdiv = int(ncol);
  size_t lds = es * (P.d1 + size_t(A.W) * A.Sn);
  int rc = launch(k_long_col<C, false>, dim3(cdiv(A.ncols, A.W), unsigned(B), 1), lds, st, A,
                  "factorisation, first column pass");
  if (rc) return rc;
  // 2: length-d2 DFTs, window products, inverse length-d2 DFTs
  LongMidArgs<C> M = long_mid_args<C>(P, U, V);
  lds = es * (P.d2 + size_t(M.W) * (P.pi + 1) * M.Sd2);
  rc = launch(k_long_mid<C>, dim3(unsigned(P.d1) * cdiv(P.Mi, M.W), unsigned(B)), lds, st, M,
              "factorisation, middle pass");
  if (rc) return rc;
  // 3: inverse length-d1 DFTs into h[n0][r][t']
  LongColArgs<C> A3 = long_col_args<C>(P);
  A3.x = V; A3.xs = h_per_signal(P); A3.xz = Md;
  A3.pre.K = 0;
  A3.y = H; A3.ys = h_per_signal(P); A3.yz = Md;
  A3.ncols = int(P.Mi * P.d2); A3.inmode = 0; A3.outmode = 1; A3.twmode = 0;
  lds = es * (P.d1 + size_t(A3.W) * A3.Sn);
  return launch(k_long_col<C, true>, dim3(cdiv(A3.ncols, A3.W), unsigned(B), unsigned(P.qi)), lds, st, A3,
                "factorisation, last column pass");
}

template <typename C>
int run_adj_cols_long(const Plan& P, const C* H, ChirpSrc<C> ch, C* y, long long B, hipStream_t st, C* U, C* V,
                      int real_out) {
  if (!U || !V) return fail(DGTNS_EINVAL, "internal: no workspace for the two-level column passes");
  const long long ncol = P.Mi * P.pi, Md = P.Mi * P.di;
  const size_t es = sizeof(C);
  // 1: length-d1 DFTs over s1 of h, twiddle W_d^{s2 k1}
  LongColArgs<C> A = long_col_args<C>(P);
  A.x = H; A.xs = h_per_signal(P); A.xz = Md;
  A.y = V; A.ys = h_per_signal(P); A.yz = Md;
  A.ncols = int(P.Mi * P.d2); A.inmode = 1; A.outmode = 0; A.twmode = 2; A.tdiv = int(P.d2);
  size_t lds = es * (P.d1 + size_t(A.W) * A.Sn);
  int rc = launch(k_long_col<C, false>, dim3(cdiv(A.ncols, A.W), unsigned(B), unsigned(P.qi)), lds, st, A,
                  "adjoint factorisation, first column pass");
  if (rc) return rc;
  // 2: per n0 length-d2 DFTs and conjugate window products, accumulated;
  //    inverse length-d2 DFTs with twiddle
  LongMidArgs<C> M = long_mid_args<C>(P, U, V);
  lds = es * (P.d2 + size_t(M.W) * (P.pi + 1) * M.Sd2);
  rc = launch(k_long_mid_adj<C>, dim3(unsigned(P.d1) * cdiv(P.Mi, M.W), unsigned(B)), lds, st, M,
              "adjoint factorisation, middle pass");
  if (rc) return rc;
  // 3: inverse length-d1 DFTs into the signal with the conjugate chirp
  LongColArgs<C> A3 = long_col_args<C>(P);
  A3.x = U; A3.xs = P.L;
  A3.post = ch;
  A3.y = y; A3.ys = P.L;
  A3.ncols = int(P.d2 * ncol); A3.inmode = 0; A3.outmode = 2; A3.twmode = 0;
  A3.real_out = real_out;
  lds = es * (P.d1 + size_t(A3.W) * A3.Sn);
  return launch(k_long_col<C, true>, dim3(cdiv(A3.ncols, A3.W), unsigned(B), 1), lds, st, A3,
                "adjoint factorisation, last column pass");
}

// chunk: the launch is a chunk of a sequential batch (run_cols_fast).
template <typename C>
int run_cols(const Plan& P, const void* x, long long xs, int real_in, ChirpSrc<C> ch, C* H, long long B,
             hipStream_t st, const void* const* xlist = nullptr, C* U = nullptr, C* V = nullptr,
             bool chunk = false) {
  if (P.longd) return run_cols_long<C>(P, x, xs, real_in, ch, H, B, st, xlist, U, V);
  ColArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.x = x; A.xs = xs; A.real_in = real_in; A.chirp = ch;
  if (xlist) {
    A.list = 1;
    for (long long k = 0; k < B; ++k) A.xl[k] = xlist[k];
  }
  A.zc = tab<C>(P, P.off.zc);
  A.H = H; A.hs = h_per_signal(P);
  A.twd = tab<C>(P, P.off.tw_d);
  A.Mi = int(P.Mi); A.ai = int(P.ai); A.d = int(P.di); A.p = int(P.pi); A.q = int(P.qi);
  A.qw = int(P.qw); A.zs = P.L;
  A.hstream = stream_h(P, B, sizeof(C));
  A.ht = h_time_major<C>(P);
  A.W = P.W; A.Sd = int(P.di | 1); A.fd = sched(P.fd);
  A.nsplit = 1;
  const size_t es = sizeof(C);
  // wave kernels up to d = 1024 (FP32) or 512 (FP64; d = 1024 would spill registers)
  if (P.pi == 1 && !P.generic && P.di * long(sizeof(C)) <= 8192) {
    switch (P.di) {
      case 32: return run_cols_fast<C, 32>(P, A, B, st, chunk);
      case 64: return run_cols_fast<C, 64>(P, A, B, st, chunk);
      case 128: return run_cols_fast<C, 128>(P, A, B, st, chunk);
      case 256: return run_cols_fast<C, 256>(P, A, B, st, chunk);
      case 512: return run_cols_fast<C, 512>(P, A, B, st, chunk);
      case 1024: return run_cols_fast<C, 1024>(P, A, B, st, chunk);
      default: break;
    }
  }
  // other 7-smooth d up to 1152 (p = 1): one wavefront per column
  if (P.pi == 1 && !P.generic && P.di <= 1152) {
    // FP32 columns above 576 values: 4 columns per work-group, so that three
    // work-groups (12 wavefronts at 142 VGPRs) share a compute unit instead of
    // one 8-column work-group holding 83 KB of LDS (batches of 8 serving
    // requests, L = 294912: 159 -> 138 us; at d = 576 the 4-column form was
    // slower on one plan and faster on another, so it keeps 8 columns)
    const int nw = (sizeof(C) == 8 && P.di > 576) ? 4 : 8;
    // the twiddle table joins the tile in LDS when both fit in 160 KiB
    const size_t lt = es * nw * size_t(A.Sd), lw = lt + es * size_t(P.di);
    const bool twl = lw <= 160 * 1024;
    const long long nblk = cdiv(P.Mi, nw);
    // small batches: split the q offsets until every work-group slot is used once
    long long ns = (512 + nblk * B - 1) / (nblk * B);
    if (ns > P.qi) ns = P.qi;
    if (ns < 1) ns = 1;
    A.nsplit = int(ns);
    dim3 gw(unsigned(nblk * ns), unsigned(B));
    if (nw == 4) {
      if (twl) return launch_t(k_fwd_cols_wr<C, 18, true, 4>, gw, 256, lw, st, A, "factorisation kernel");
      return launch_t(k_fwd_cols_wr<C, 18, false, 4>, gw, 256, lt, st, A, "factorisation kernel");
    }
    if (!twl) return launch(k_fwd_cols_wr<C, 18, false>, gw, lt, st, A, "factorisation kernel");
    // values per lane: as few as hold d, so that short columns do not run
    // masked iterations (d = 36: one value per lane instead of five)
    if (P.di <= 64) return launch(k_fwd_cols_wr<C, 1, true>, gw, lw, st, A, "factorisation kernel");
    if (P.di <= 128) return launch(k_fwd_cols_wr<C, 2, true>, gw, lw, st, A, "factorisation kernel");
    if (P.di <= 192) return launch(k_fwd_cols_wr<C, 3, true>, gw, lw, st, A, "factorisation kernel");
    if (P.di <= 320) return launch(k_fwd_cols_wr<C, 5, true>, gw, lw, st, A, "factorisation kernel");
    if (P.di <= 576) return launch(k_fwd_cols_wr<C, 9, true>, gw, lw, st, A, "factorisation kernel");
    return launch(k_fwd_cols_wr<C, 18, true>, gw, lw, st, A, "factorisation kernel");
  }
  const size_t lds = P.pi == 1 ? es * (P.di + size_t(P.W) * A.Sd)
                               : es * (P.di + size_t(P.W) * A.Sd * (P.pi + 1));
  dim3 grid(cdiv(P.Mi, P.W), unsigned(B));
  if (P.pi == 1) return launch(k_fwd_cols<C, false>, grid, lds, st, A, "factorisation kernel");
  return launch(k_fwd_cols<C, true>, grid, lds, st, A, "factorisation kernel (p > 1)");
}

template <typename C>
int run_adj_cols(const Plan& P, const C* H, ChirpSrc<C> ch, C* y, long long B, hipStream_t st, C* U = nullptr,
                 C* V = nullptr, int real_out = 0) {
  if (P.longd) return run_adj_cols_long<C>(P, H, ch, y, B, st, U, V, real_out);
  ColAdjArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.real_out = real_out;
  A.H = H; A.hs = h_per_signal(P);
  A.zc = tab<C>(P, P.off.zc);
  A.twd = tab<C>(P, P.off.tw_d);
  A.chirp = ch; A.y = y; A.ys = P.L;
  A.Mi = int(P.Mi); A.ai = int(P.ai); A.d = int(P.di); A.p = int(P.pi); A.q = int(P.qi);
  A.qw = int(P.qw); A.zs = P.L;
  A.W = P.W; A.Sd = int(P.di | 1); A.fd = sched(P.fd);
  const size_t es = sizeof(C);
  // adjoint wave kernels up to d = 512 (larger d would spill registers)
  if (P.pi == 1 && !P.generic && P.di <= 512) {
    switch (P.di) {
      case 32: return run_adj_cols_fast<C, 32>(P, A, B, st);
      case 64: return run_adj_cols_fast<C, 64>(P, A, B, st);
      case 128: return run_adj_cols_fast<C, 128>(P, A, B, st);
      case 256: return run_adj_cols_fast<C, 256>(P, A, B, st);
      case 512: return run_adj_cols_fast<C, 512>(P, A, B, st);
      default: break;
    }
  }
  dim3 grid(cdiv(P.Mi, P.W), unsigned(B));
  size_t lds = es * (P.di + size_t(P.W) * A.Sd * (P.pi > 1 ? P.pi + 1 : 1));
  if (P.pi == 1) return launch(k_adj_cols<C, false>, grid, lds, st, A, "adjoint factorisation kernel");
  return launch(k_adj_cols<C, true>, grid, lds, st, A, "adjoint factorisation kernel (p > 1)");
}

template <typename C>
RowArgs<C> row_args(const Plan& P, const C* H, C* c) {
  RowArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.H = H; A.hs = h_per_signal(P);
  A.c = c; A.cs = coef_per_signal(P);
  A.lay = coef_layout(P);
  A.twm = tab<C>(P, P.off.tw_m);
  A.Mi = int(P.Mi); A.Ni = int(P.Ni);
  A.qw = int(P.qw); A.nw = int(P.nw);
  // rows per work-group of the runtime-schedule row kernels: enough rows that
  // a work-group has work for its 512 threads when Mi is small
  A.R = block_width(P.Mi | 1, sizeof(C), P.Mi < 32 ? 256 : 64);
  A.Sm = int(P.Mi | 1);
  A.fm = sched(P.fm);
  A.q = int(P.qi);
  A.d = int(P.di);
  if (P.branch != kFreqShear) {
    A.postE = tab<C>(P, P.off.post_E);
    A.rho = reinterpret_cast<const int*>(tab<C>(P, P.off.post_rho));
  } else {
    A.N = P.N; A.L = P.L; A.b = P.b; A.M = P.M;
    A.K1 = P.K1; A.K2 = P.K2; A.K3 = P.K3; A.K4 = P.K4; A.K5 = P.K5;
    A.C1n = P.C1n; A.C2n = P.C2n; A.Kt1 = P.Kt1; A.Kt6 = P.Kt6;
    const unsigned long long all = ~0ull;
    A.mu2N = all / (unsigned long long)(2 * P.N);
    A.muN = all / (unsigned long long)P.N;
    A.muL = all / (unsigned long long)P.L;
    A.mub = all / (unsigned long long)P.b;
  }
  return A;
}

// Bc: the batch whose coefficients the call writes in all (a sequential
// chunk of a larger batch streams its stores when the whole output would not
// stay in the last-level cache); 0: B.
template <typename C>
int run_rows(const Plan& P, const C* H, C* c, long long B, bool adjoint, hipStream_t st,
             void* const* clist = nullptr, long long Bc = 0) {
  RowArgs<C> A = row_args<C>(P, H, c);
  // the adjoint writes h, the forward the coefficients
  // the forward of the frequency-shear branch scatters single coefficients
  // (Alg. 1's output permutation): plain stores let the cache merge them
  A.hstream = adjoint ? stream_h(P, B, sizeof(C))
                      : (P.branch == kFreqShear ? 0 : stream_c(P, Bc > 0 ? Bc : B, sizeof(C)));
  A.ht = !adjoint && h_time_major<C>(P);
  if (clist) {
    A.list = 1;
    for (long long k = 0; k < B; ++k) A.cl[k] = static_cast<C*>(clist[k]);
  }
  if (!P.generic) {
    switch (P.Mi) {
      case 32: return run_rows_fast<C, 32>(P, A, B, adjoint, st);
      case 64: return run_rows_fast<C, 64>(P, A, B, adjoint, st);
      case 128: return run_rows_fast<C, 128>(P, A, B, adjoint, st);
      case 256: return run_rows_fast<C, 256>(P, A, B, adjoint, st);
      case 512: return run_rows_fast<C, 512>(P, A, B, adjoint, st);
      case 1024: return run_rows_fast<C, 1024>(P, A, B, adjoint, st);
      default: break;
    }
  }
  dim3 grid(unsigned(P.qi) * cdiv(P.di, A.R), unsigned(B));
  size_t lds = sizeof(C) * (P.Mi + size_t(A.R) * A.Sm);
  const bool fs = P.branch == kFreqShear;
  if (!adjoint) {
    if (fs) return launch(k_fwd_rows<C, 1>, grid, lds, st, A, "channel DFT + shear post-processing");
    return launch(k_fwd_rows<C, 0>, grid, lds, st, A, "channel DFT + phase correction");
  }
  if (fs) return launch(k_adj_rows<C, 1>, grid, lds, st, A, "adjoint channel DFT (shear)");
  return launch(k_adj_rows<C, 0>, grid, lds, st, A, "adjoint channel DFT");
}

// Length-L transform as column pass (length n1 over n2 columns) + row pass
// (length n2 over n1 rows, transposed store).  Forward: n1 = L1, n2 = L2;
// inverse: n1 = L2, n2 = L1.
template <typename C>
int run_four_step(const Plan& P, const void* x, int real_in, C* tmp, C* y, long long B, bool inv,
                  ChirpSrc<C> pre, ChirpSrc<C> post, decltype(C::x) scale, const C* twL,
                  const C* tw1, const C* tw2, hipStream_t st, const void* const* xlist = nullptr) {
  const long long n1 = inv ? P.L2 : P.L1, n2 = inv ? P.L1 : P.L2;
  const FftSched s1 = sched(inv ? P.f2 : P.f1), s2 = sched(inv ? P.f1 : P.f2);
  ColFftArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  if (xlist) {
    A.list = 1;
    for (long long k = 0; k < B; ++k) A.xl[k] = xlist[k];
  }
  A.x = x; A.xs = P.L; A.real_in = real_in; A.y = tmp; A.ys = P.L; A.pre = pre;
  A.twL = twL; A.L = P.L; A.tws = inv ? tw2 : tw1;
  A.n = int(n1); A.ncols = int(n2); A.Sn = int(n1 | 1); A.W = block_width(A.Sn, sizeof(C)); A.fs = s1;
  size_t lds = sizeof(C) * (n1 + size_t(A.W) * A.Sn);
  dim3 g1(cdiv(n2, A.W), unsigned(B));
  int rc = inv ? launch(k_col_fft<C, true>, g1, lds, st, A, "length-L transform, column pass")
               : launch(k_col_fft<C, false>, g1, lds, st, A, "length-L transform, column pass");
  if (rc) return rc;
  RowFftArgs<C> R;
  std::memset(&R, 0, sizeof(R));
  R.x = tmp; R.xs = P.L; R.y = y; R.ys = P.L; R.post = post; R.scale = scale;
  R.real_out = inv && real_call() ? 1 : 0;   // the synthesis' last pass writes the signal
  R.tws = inv ? tw1 : tw2;
  R.n = int(n2); R.nrows = int(n1); R.Sn = int(n2 | 1); R.R = block_width(R.Sn, sizeof(C)); R.fs = s2;
  lds = sizeof(C) * (n2 + size_t(R.R) * R.Sn);
  dim3 g2(cdiv(n1, R.R), unsigned(B));
  return inv ? launch(k_row_fft<C, true>, g2, lds, st, R, "length-L transform, row pass")
             : launch(k_row_fft<C, false>, g2, lds, st, R, "length-L transform, row pass");
}

template <typename C> ChirpSrc<C> no_chirp(const Plan& P) {
  ChirpSrc<C> c;
  c.tab = nullptr; c.K = 0; c.L = P.L; c.conj = 0;
  return c;
}
template <typename C> ChirpSrc<C> chirp_tab(const Plan& P, size_t off, int conj) {
  ChirpSrc<C> c;
  c.tab = off ? tab<C>(P, off) : nullptr; c.K = 0; c.L = P.L; c.conj = conj;
  return c;
}
inline ChirpSrc<double2> chirp_fly(const Plan& P, long long s, int conj) {
  ChirpSrc<double2> c;
  c.tab = nullptr; c.K = chirpK(P, s); c.L = P.L; c.conj = conj;
  return c;
}

// ---------------------------------------------------------------------------
// FIR-window algorithm (kernels_fir.hpp)
// ---------------------------------------------------------------------------
template <typename C>
FirArgs<C> fir_args(const Plan& P) {
  FirArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.gw = tab<C>(P, P.off.zc);
  A.ph = P.off.fir_ph ? tab<C>(P, P.off.fir_ph) : nullptr;
  A.twm = tab<C>(P, P.off.tw_m);
  A.L = P.L; A.start = P.fir_start;
  A.a = int(P.a); A.M = int(P.M); A.Lg = int(P.fir_len); A.lam1 = int(P.lam1); A.lam2 = int(P.lam2);
  A.N = int(P.N);
  A.R = block_width(P.M | 1, sizeof(C)); A.Sm = int(P.M | 1);
  A.fm = sched(P.fm);
  A.lay = coef_layout(P);
  const unsigned long long all = ~0ULL;
  A.muM = all / (unsigned long long)P.M;
  A.muL2 = all / (unsigned long long)P.lam2;
  A.muPM = all / ((unsigned long long)P.lam2 * (unsigned long long)P.M);
  return A;
}

template <typename C, int MI, bool HS>
int run_fir_fwd_w2(const FirArgs<C>& A, const Plan& P, long long B, hipStream_t st) {
  using I = WInfo<MI>;
  dim3 grid(cdiv(P.N, 8 * I::TPW), unsigned(B));
  const size_t lds = sizeof(C) * 8 * I::TPW * WEx<C, MI>::EX;
  // samples per folded bin: unrolled for up to four
  const long long nt = (P.fir_len + MI - 1) / MI;
  // span and window in LDS when they fit beside the exchange areas' size
  const size_t need = sizeof(C) * size_t((8 * I::TPW - 1) * P.a + 2 * P.fir_len);
  if (need <= std::max(lds, size_t(40960))) {
    const size_t lw = std::max(sizeof(C) * 8 * I::TPW * FirWs<C, MI>::EX, need);
    if (nt <= 1) return launch(k_fir_fwd_ws<C, MI, HS, 1>, grid, lw, st, A, "FIR DGT");
    if (nt <= 2) return launch(k_fir_fwd_ws<C, MI, HS, 2>, grid, lw, st, A, "FIR DGT");
    if (nt <= 4) return launch(k_fir_fwd_ws<C, MI, HS, 4>, grid, lw, st, A, "FIR DGT");
    return launch(k_fir_fwd_ws<C, MI, HS, 0>, grid, lw, st, A, "FIR DGT");
  }
  if (nt <= 1) return launch(k_fir_fwd_w<C, MI, HS, 1>, grid, lds, st, A, "FIR DGT");
  if (nt <= 2) return launch(k_fir_fwd_w<C, MI, HS, 2>, grid, lds, st, A, "FIR DGT");
  if (nt <= 4) return launch(k_fir_fwd_w<C, MI, HS, 4>, grid, lds, st, A, "FIR DGT");
  return launch(k_fir_fwd_w<C, MI, HS, 0>, grid, lds, st, A, "FIR DGT");
}

template <typename C, int MI>
int run_fir_fwd_w(const FirArgs<C>& A, const Plan& P, long long B, hipStream_t st) {
  if (stream_c(P, B, sizeof(C))) return run_fir_fwd_w2<C, MI, true>(A, P, B, st);
  return run_fir_fwd_w2<C, MI, false>(A, P, B, st);
}

template <typename C>
int run_fir_fwd(const Plan& P, const void* f, int real_in, C* c, long long B, hipStream_t st,
                const void* const* flist, void* const* clist) {
  FirArgs<C> A = fir_args<C>(P);
  A.x = f; A.xs = P.L; A.real_in = real_in; A.c = c; A.cs = coef_per_signal(P);
  if (flist) {
    A.list = 1;
    for (long long k = 0; k < B; ++k) {
      A.xl[k] = flist[k];
      A.cl[k] = static_cast<C*>(clist[k]);
    }
  }
  if (!P.generic && P.M * long(sizeof(C)) <= 8192) {
    switch (P.M) {
      case 32: return run_fir_fwd_w<C, 32>(A, P, B, st);
      case 64: return run_fir_fwd_w<C, 64>(A, P, B, st);
      case 128: return run_fir_fwd_w<C, 128>(A, P, B, st);
      case 256: return run_fir_fwd_w<C, 256>(A, P, B, st);
      case 512: return run_fir_fwd_w<C, 512>(A, P, B, st);
      case 1024: return run_fir_fwd_w<C, 1024>(A, P, B, st);
      default: break;
    }
  }
  const size_t lds = sizeof(C) * (P.M + size_t(A.R) * A.Sm);
  return launch(k_fir_fwd<C>, dim3(cdiv(P.N, A.R), unsigned(B)), lds, st, A, "FIR DGT");
}

template <typename C, int MI>
int run_fir_adj_rows_w(const FirArgs<C>& A, const Plan& P, long long B, C* Y, long long ys, hipStream_t st) {
  using I = WInfo<MI>;
  const size_t lds = sizeof(C) * 8 * I::TPW * FirWs<C, MI>::EX;
  return launch_v(k_fir_adj_rows_w<C, MI>, dim3(cdiv(P.N, 8 * I::TPW), unsigned(B)), lds, st,
                       "FIR adjoint, inverse DFTs", A, Y, ys);
}

template <typename C>
int run_fir_adj_rows(const FirArgs<C>& A, const Plan& P, long long B, C* Y, long long ys, hipStream_t st) {
  if (!P.generic && P.M * long(sizeof(C)) <= 8192) {
    switch (P.M) {
      case 32: return run_fir_adj_rows_w<C, 32>(A, P, B, Y, ys, st);
      case 64: return run_fir_adj_rows_w<C, 64>(A, P, B, Y, ys, st);
      case 128: return run_fir_adj_rows_w<C, 128>(A, P, B, Y, ys, st);
      case 256: return run_fir_adj_rows_w<C, 256>(A, P, B, Y, ys, st);
      case 512: return run_fir_adj_rows_w<C, 512>(A, P, B, Y, ys, st);
      case 1024: return run_fir_adj_rows_w<C, 1024>(A, P, B, Y, ys, st);
      default: break;
    }
  }
  const size_t lds = sizeof(C) * (P.M + size_t(A.R) * A.Sm);
  return launch_v(k_fir_adj_rows<C>, dim3(cdiv(P.N, A.R), unsigned(B)), lds, st,
                       "FIR adjoint, inverse DFTs", A, Y, ys);
}

template <typename C>
int run_fir_adj(const Plan& P, const C* c, C* f, long long B, C* Y, hipStream_t st) {
  FirArgs<C> A = fir_args<C>(P);
  A.c = const_cast<C*>(c); A.cs = coef_per_signal(P);
  A.real_out = real_call() ? 1 : 0;
  const long long ys = P.M * P.N;
  int rc = run_fir_adj_rows<C>(A, P, B, Y, ys, st);
  if (rc) return rc;
  return launch_raw(k_fir_adj_gather<C>, dim3(cdiv(P.L, kThreads), unsigned(B)), dim3(kThreads), 0, st,
                    "FIR adjoint, gather", A, (const C*)Y, ys, f);
}

template <typename C>
int run_ola_fwd(const Plan& P, const void* f, int real_in, C* c, long long B, char* ws, const Layout& l,
                hipStream_t st);

template <typename C>
int forward_impl(const Plan& P, const void* f, int real_in, C* c, long long B, char* ws, const Layout& l,
                 hipStream_t st, const void* const* flist = nullptr, void* const* clist = nullptr) {
  if (P.branch == kFir) return run_fir_fwd<C>(P, f, real_in, c, B, st, flist, clist);
  if (P.branch == kShearOla) {
    if (flist || clist) return fail(DGTNS_EUNSUPPORTED, "shear-OLA plans have no list-batched forward");
    return run_ola_fwd<C>(P, f, real_in, c, B, ws, l, st);
  }
  C* H = reinterpret_cast<C*>(ws + l.H);
  int rc;
  // the workspace layout of this batch size decides the path (ws_layout):
  // pipelined batches only have room for two chunks of h
  if (pipelined(P, B, DGTNS_OP_FORWARD)) {
    C* Hb[2] = {H, reinterpret_cast<C*>(ws + l.F)};
    const size_t sig_bytes = size_t(P.L) * (real_in ? sizeof(C) / 2 : sizeof(C));
    const long long MN = coef_per_signal(P);
    return run_pipeline(
        B, P.chunk, st,
        [&](long long b0, long long nb, int buf, hipStream_t s) {
          if (flist)
            return run_cols<C>(P, nullptr, P.L, real_in, chirp_tab<C>(P, P.off.chirp1, 0), Hb[buf], nb, s,
                               flist + b0);
          return run_cols<C>(P, static_cast<const char*>(f) + b0 * sig_bytes, P.L, real_in,
                             chirp_tab<C>(P, P.off.chirp1, 0), Hb[buf], nb, s);
        },
        [&](long long b0, long long nb, int buf, hipStream_t s) {
          if (clist) return run_rows<C>(P, Hb[buf], nullptr, nb, false, s, clist + b0);
          return run_rows<C>(P, Hb[buf], c + b0 * MN, nb, false, s);
        });
  }
  if (seq_chunked(P, B, DGTNS_OP_FORWARD)) {
    const size_t sig_bytes = size_t(P.L) * (real_in ? sizeof(C) / 2 : sizeof(C));
    const long long MN = coef_per_signal(P);
    for (long long b0 = 0; b0 < B; b0 += P.seq) {
      const long long nb = B - b0 < P.seq ? B - b0 : P.seq;
      if (flist)
        rc = run_cols<C>(P, nullptr, P.L, real_in, chirp_tab<C>(P, P.off.chirp1, 0), H, nb, st, flist + b0,
                         nullptr, nullptr, true);
      else
        rc = run_cols<C>(P, static_cast<const char*>(f) + b0 * sig_bytes, P.L, real_in,
                         chirp_tab<C>(P, P.off.chirp1, 0), H, nb, st, nullptr, nullptr, nullptr, true);
      if (!rc) rc = run_rows<C>(P, H, clist ? nullptr : c + b0 * MN, nb, false, st, clist ? clist + b0 : nullptr, B);
      if (rc) return rc;
    }
    return DGTNS_OK;
  }
  if (P.branch != kFreqShear) {
    rc = run_cols<C>(P, f, P.L, real_in, chirp_tab<C>(P, P.off.chirp1, 0), H, B, st, flist,
                     reinterpret_cast<C*>(ws + l.U), reinterpret_cast<C*>(ws + l.V));
  } else {
    C* F = reinterpret_cast<C*>(ws + l.F);
    C* Y = reinterpret_cast<C*>(ws + l.Y);
    rc = run_four_step<C>(P, f, real_in, Y, F, B, false, chirp_tab<C>(P, P.off.chirp1, 0),
                          chirp_tab<C>(P, P.off.chirp0, 0), 1, tab<C>(P, P.off.tw_L), tab<C>(P, P.off.tw_1),
                          tab<C>(P, P.off.tw_2), st, flist);
    if (rc) return rc;
    rc = run_cols<C>(P, F, P.L, 0, no_chirp<C>(P), H, B, st, nullptr, reinterpret_cast<C*>(ws + l.U),
                     reinterpret_cast<C*>(ws + l.V));
  }
  if (rc) return rc;
  return run_rows<C>(P, H, c, B, false, st, clist);
}

// Shear-OLA block window g_loc (FP64, L_x values at gl) from the length-L
// window g.
inline int ola_block_window(const Plan& P, const double2* g, double2* gl, hipStream_t st) {
  return launch_raw(k_ola_window<>, dim3(cdiv(P.ola_Lx, kThreads)), dim3(kThreads), 0, st, "OLA block window", g, gl,
                    (long long)P.L, (long long)P.ola_s, (long long)P.fir_len, (long long)P.ola_Lx);
}

// Shear-OLA forward (kernels_ola.hpp): zero-extended blocks, the shear
// algorithm on all of them as one batch of the inner plan, overlap-add.
template <typename C>
int run_ola_fwd(const Plan& P, const void* f, int real_in, C* c, long long B, char* ws, const Layout& l,
                hipStream_t st) {
  const Plan& Q = *P.inner;
  OlaArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.x = f; A.xs = P.L; A.real_in = real_in;
  A.X = reinterpret_cast<C*>(ws + l.ola_x);
  A.cl = reinterpret_cast<C*>(ws + l.ola_c);
  A.c = c; A.cs = coef_per_signal(P);
  A.lay = coef_layout(P);
  A.ph = tab<C>(P, P.off.fir_ph);
  A.L = P.L; A.Lb = P.ola_Lb; A.Lx = P.ola_Lx; A.J0 = P.ola_J0;
  A.a = int(P.a); A.M = int(P.M); A.N = int(P.N); A.Nb = int(P.ola_Nb); A.Nx = int(P.ola_Nx);
  A.P0 = int(P.ola_P0); A.lam1 = int(P.lam1); A.lam2 = int(P.lam2);
  const long long Bi = B * P.ola_Nb;
  int rc = launch_raw(k_ola_gather<C>, dim3(cdiv(P.ola_Lx, kThreads), unsigned(Bi)), dim3(kThreads), 0, st,
                      "OLA blocks", A);
  if (rc) return rc;
  {
    FullLayoutScope full;   // block coefficients: full layout
    rc = forward_impl<C>(Q, A.X, 0, const_cast<C*>(A.cl), Bi, ws + l.inner, ws_layout(Q, DGTNS_OP_FORWARD, Bi), st);
  }
  if (rc) return rc;
  return launch_raw(k_ola_combine<C>, dim3(unsigned(P.N), unsigned(B)), dim3(kOlaThreads), 0, st,
                    "OLA overlap-add", A);
}

template <typename C>
int adjoint_impl(const Plan& P, const C* c, C* f, long long B, char* ws, const Layout& l, hipStream_t st);

// Shear-OLA adjoint: the adjoint of each forward stage in reverse order.  The
// global coefficients are split into the blocks' coefficients with the
// conjugate position phases, the inner plan synthesises all blocks as one
// batch, and each block's own samples are written back to the signal.
template <typename C>
int run_ola_adj(const Plan& P, const C* c, C* f, long long B, char* ws, const Layout& l, hipStream_t st) {
  const Plan& Q = *P.inner;
  OlaArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.X = reinterpret_cast<C*>(ws + l.ola_x);
  A.cl = reinterpret_cast<C*>(ws + l.ola_c);
  A.c = const_cast<C*>(c); A.cs = coef_per_signal(P);
  A.lay = coef_layout(P);
  A.ph = tab<C>(P, P.off.fir_ph);
  A.L = P.L; A.Lb = P.ola_Lb; A.Lx = P.ola_Lx; A.J0 = P.ola_J0;
  A.a = int(P.a); A.M = int(P.M); A.N = int(P.N); A.Nb = int(P.ola_Nb); A.Nx = int(P.ola_Nx);
  A.P0 = int(P.ola_P0); A.lam1 = int(P.lam1); A.lam2 = int(P.lam2);
  const long long Bi = B * P.ola_Nb;
  int rc = launch_raw(k_ola_split<C>, dim3(unsigned(P.ola_Nx), unsigned(Bi)), dim3(kOlaThreads), 0, st,
                      "OLA split", A);
  if (rc) return rc;
  const int real_out = real_call() ? 1 : 0;
  {
    FullLayoutScope full;   // block coefficients and block signals: full layout, complex
    rc = adjoint_impl<C>(Q, A.cl, A.X, Bi, ws + l.inner, ws_layout(Q, DGTNS_OP_ADJOINT, Bi), st);
  }
  if (rc) return rc;
  return launch_raw(k_ola_scatter<C>, dim3(cdiv(P.L, kThreads), unsigned(B)), dim3(kThreads), 0, st,
                    "OLA block scatter", A, f, real_out);
}

template <typename C>
int adjoint_impl(const Plan& P, const C* c, C* f, long long B, char* ws, const Layout& l, hipStream_t st) {
  if (P.branch == kShearOla) return run_ola_adj<C>(P, c, f, B, ws, l, st);
  C* H = reinterpret_cast<C*>(ws + l.H);
  if (P.branch == kFir) return run_fir_adj<C>(P, c, f, B, H, st);
  if (pipelined(P, B, DGTNS_OP_ADJOINT)) {
    C* Hb[2] = {H, reinterpret_cast<C*>(ws + l.F)};
    const long long MN = coef_per_signal(P);
    return run_pipeline(
        B, P.chunk, st,
        [&](long long b0, long long nb, int buf, hipStream_t s) {
          return run_rows<C>(P, Hb[buf], const_cast<C*>(c) + b0 * MN, nb, true, s);
        },
        [&](long long b0, long long nb, int buf, hipStream_t s) {
          return run_adj_cols<C>(P, Hb[buf], chirp_tab<C>(P, P.off.chirp1, 1), f + b0 * P.L, nb, s, nullptr,
                                 nullptr, real_call() ? 1 : 0);
        });
  }
  if (seq_chunked(P, B, DGTNS_OP_ADJOINT)) {
    const long long MN = coef_per_signal(P);
    const size_t sig_bytes = size_t(P.L) * (real_call() ? sizeof(C) / 2 : sizeof(C));
    for (long long b0 = 0; b0 < B; b0 += P.seq) {
      const long long nb = B - b0 < P.seq ? B - b0 : P.seq;
      C* fb = reinterpret_cast<C*>(reinterpret_cast<char*>(f) + b0 * sig_bytes);
      int rc = run_rows<C>(P, H, const_cast<C*>(c) + b0 * MN, nb, true, st);
      if (!rc)
        rc = run_adj_cols<C>(P, H, chirp_tab<C>(P, P.off.chirp1, 1), fb, nb, st, nullptr, nullptr,
                             real_call() ? 1 : 0);
      if (rc) return rc;
    }
    return DGTNS_OK;
  }
  int rc = run_rows<C>(P, H, const_cast<C*>(c), B, true, st);
  if (rc) return rc;
  C* U = reinterpret_cast<C*>(ws + l.U);
  C* V = reinterpret_cast<C*>(ws + l.V);
  if (P.branch != kFreqShear)
    return run_adj_cols<C>(P, H, chirp_tab<C>(P, P.off.chirp1, 1), f, B, st, U, V, real_call() ? 1 : 0);
  C* F = reinterpret_cast<C*>(ws + l.F);
  C* Y = reinterpret_cast<C*>(ws + l.Y);
  rc = run_adj_cols<C>(P, H, no_chirp<C>(P), F, B, st, U, V);
  if (rc) return rc;
  return run_four_step<C>(P, F, 0, Y, f, B, true, chirp_tab<C>(P, P.off.chirp0, 1),
                          chirp_tab<C>(P, P.off.chirp1, 1), 1, tab<C>(P, P.off.tw_L), tab<C>(P, P.off.tw_1),
                          tab<C>(P, P.off.tw_2), st);
}

// Window gradient columns: wave kernels (column spectra, then one wave
// transform per window column) or the runtime-schedule kernel.
template <typename C, int D>
int run_grad_cols_w(const Plan& P, const void* x, ChirpSrc<C> ch, const C* H, C* X, C* part, long long B,
                    hipStream_t st) {
  ColArgs<C> A;
  std::memset(&A, 0, sizeof(A));
  A.x = x; A.xs = P.L; A.real_in = 0; A.chirp = ch;
  A.H = X; A.hs = P.L;
  A.twd = tab<C>(P, P.off.tw_d);
  A.Mi = int(P.Mi); A.d = int(P.di);
  using F = FastCols<C, D>;
  int rc = launch(k_col_spectra_w<C, D>, dim3(cdiv(P.Mi, F::W), unsigned(B)), sizeof(C) * F::LDS, st, A,
                  "column spectra");
  if (rc) return rc;
  GradWArgs<C> G;
  G.X = X; G.xs = P.L;
  G.H = H; G.hs = h_per_signal(P);
  G.part = part; G.ps = P.L;
  G.twd = tab<C>(P, P.off.tw_d);
  G.Mi = int(P.Mi); G.ai = int(P.ai); G.q = int(P.qi);
  using F1 = FastCols<C, D, 1>;
  return launch(k_grad_cols_w<C, D>, dim3(cdiv(P.Mi, F1::W), unsigned(B)), sizeof(C) * F1::LDS, st, G,
                "window gradient");
}

template <typename C>
int run_grad_cols_fast(const Plan& P, const void* x, ChirpSrc<C> ch, const C* H, C* X, C* part, long long B,
                       hipStream_t st) {
  switch (P.di) {
    case 32: return run_grad_cols_w<C, 32>(P, x, ch, H, X, part, B, st);
    case 64: return run_grad_cols_w<C, 64>(P, x, ch, H, X, part, B, st);
    case 128: return run_grad_cols_w<C, 128>(P, x, ch, H, X, part, B, st);
    case 256: return run_grad_cols_w<C, 256>(P, x, ch, H, X, part, B, st);
    default: return run_grad_cols_w<C, 512>(P, x, ch, H, X, part, B, st);
  }
}

template <typename C>
int run_grad_cols_generic(const Plan& P, const void* x, ChirpSrc<C> ch, const C* H, C* part, long long B,
                          hipStream_t st) {
  GradArgs<C> A;
  A.x = x; A.xs = P.L; A.real_in = 0; A.chirp = ch;
  A.H = H; A.hs = h_per_signal(P);
  A.part = part; A.ps = P.L;
  A.twd = tab<C>(P, P.off.tw_d);
  A.Mi = int(P.Mi); A.ai = int(P.ai); A.d = int(P.di); A.q = int(P.qi);
  A.p = int(P.pi);
  A.Sd = int(P.di | 1);
  A.W = block_width(2 * A.Sd, sizeof(C));
  A.fd = sched(P.fd);
  const size_t lds = sizeof(C) * (P.di + 2 * size_t(A.W) * A.Sd), lcols = sizeof(C) * 2 * size_t(A.W) * A.Sd;
  const dim3 grid(cdiv(P.Mi * P.pi, A.W), unsigned(B));
  if (lds <= 160 * 1024) return launch(k_grad_cols<C, false>, grid, lds, st, A, "window gradient");
  return launch(k_grad_cols<C, true>, grid, lcols, st, A, "window gradient");
}

// Window gradient columns with long columns (d = d1 d2): the first column
// pass of the signal (as the forward's) into U and of h (as the adjoint's)
// into V, the middle pass into part, then the length-d1 inverse DFTs in place.
template <typename C>
int run_grad_cols_long(const Plan& P, const void* x, ChirpSrc<C> ch, const C* H, C* U, C* V, C* part, long long B,
                       hipStream_t st) {
  const long long Mp = P.Mi * P.pi, Md = P.Mi * P.di;
  const size_t es = sizeof(C);
  LongColArgs<C> A = long_col_args<C>(P);
  A.x = x; A.xs = P.L; A.pre = ch;
  A.y = U; A.ys = P.L;
  A.ncols = int(P.d2 * Mp); A.inmode = 0; A.outmode = 0; A.twmode = 1; A.tdiv = int(Mp);
  int rc = launch(k_long_col<C, false>, dim3(cdiv(A.ncols, A.W), unsigned(B), 1), es * (P.d1 + size_t(A.W) * A.Sn),
                  st, A, "window gradient, signal column pass");
  if (rc) return rc;
  LongColArgs<C> A1 = long_col_args<C>(P);
  A1.x = H; A1.xs = h_per_signal(P); A1.xz = Md;
  A1.y = V; A1.ys = h_per_signal(P); A1.yz = Md;
  A1.ncols = int(P.Mi * P.d2); A1.inmode = 1; A1.outmode = 0; A1.twmode = 2; A1.tdiv = int(P.d2);
  rc = launch(k_long_col<C, false>, dim3(cdiv(A1.ncols, A1.W), unsigned(B), unsigned(P.qi)),
              es * (P.d1 + size_t(A1.W) * A1.Sn), st, A1, "window gradient, h column pass");
  if (rc) return rc;
  LongGradArgs<C> G;
  G.U = U; G.us = P.L; G.V = V; G.vs = h_per_signal(P); G.G = part; G.gs = P.L;
  G.twd = tab<C>(P, P.off.tw_d); G.tw2 = tab<C>(P, P.off.tw_d2);
  G.Mi = int(P.Mi); G.ai = int(P.ai); G.p = int(P.pi); G.q = int(P.qi);
  G.d = int(P.di); G.d1 = int(P.d1); G.d2 = int(P.d2); G.Sd2 = int(P.d2 | 1);
  G.fs2 = sched(P.fd2);
  const long long budget = MaxE<C>::value * kThreads;
  int W = 16;
  while (W > 1 && (2 * W * P.d2 > budget || es * (P.d2 + 3 * size_t(W) * G.Sd2) > (64u << 10))) --W;
  G.W = W;
  rc = launch(k_long_mid_grad<C>, dim3(unsigned(P.d1) * cdiv(Mp, W), unsigned(B)),
              es * (P.d2 + 3 * size_t(W) * G.Sd2), st, G, "window gradient, middle pass");
  if (rc) return rc;
  LongColArgs<C> A3 = long_col_args<C>(P);
  A3.x = part; A3.xs = P.L;
  A3.y = part; A3.ys = P.L;
  A3.ncols = int(P.d2 * Mp); A3.inmode = 0; A3.outmode = 0; A3.twmode = 0;
  return launch(k_long_col<C, true>, dim3(cdiv(A3.ncols, A3.W), unsigned(B), 1), es * (P.d1 + size_t(A3.W) * A3.Sn),
                st, A3, "window gradient, last column pass");
}

template <typename C>
int grad_impl(const Plan& P, const C* f, const C* gc, C* gg, long long B, char* ws, const Layout& l,
              hipStream_t st) {
  if (P.branch == kMultiwindow || P.branch == kFir)
    return fail(DGTNS_EUNSUPPORTED, "the window gradient is implemented for shear-algorithm plans only");
  C* H = reinterpret_cast<C*>(ws + l.H);
  C* part = reinterpret_cast<C*>(ws + l.part);
  int rc = run_rows<C>(P, H, const_cast<C*>(gc), B, true, st);
  if (rc) return rc;
  const void* x = f;
  ChirpSrc<C> ch = chirp_tab<C>(P, P.off.chirp1, 0);
  const bool fs = P.branch == kFreqShear;
  if (fs) {
    C* F = reinterpret_cast<C*>(ws + l.F);
    C* Y = reinterpret_cast<C*>(ws + l.Y);
    rc = run_four_step<C>(P, f, 0, Y, F, B, false, chirp_tab<C>(P, P.off.chirp1, 0),
                          chirp_tab<C>(P, P.off.chirp0, 0), 1, tab<C>(P, P.off.tw_L), tab<C>(P, P.off.tw_1),
                          tab<C>(P, P.off.tw_2), st);
    if (rc) return rc;
    x = F;
    ch = no_chirp<C>(P);
  }
  const bool wave = P.pi == 1 && !P.generic && wave_len(P.di) && P.di <= 512;
  if (P.longd) {
    rc = run_grad_cols_long<C>(P, x, ch, H, reinterpret_cast<C*>(ws + l.U), reinterpret_cast<C*>(ws + l.V), part,
                               B, st);
  } else if (wave) {
    rc = run_grad_cols_fast<C>(P, x, ch, H, reinterpret_cast<C*>(ws + l.U), part, B, st);
  } else {
    rc = run_grad_cols_generic<C>(P, x, ch, H, part, B, st);
  }
  if (rc) return rc;
  if (!fs) {
    return launch_raw(k_batch_sum<C>, dim3(cdiv(P.L, kThreads)), dim3(kThreads), 0, st, "batch sum", part,
                      (long long)P.L, int(B), (long long)P.L, chirp_tab<C>(P, P.off.chirp1, 1), gg);
  }
  C* G = reinterpret_cast<C*>(ws + l.G);
  rc = launch_raw(k_batch_sum<C>, dim3(cdiv(P.L, kThreads)), dim3(kThreads), 0, st, "batch sum", part,
                  (long long)P.L, int(B), (long long)P.L, no_chirp<C>(P), G);
  if (rc) return rc;
  // the frequency-domain window is p0 FFT(p1 g) / L: its adjoint is
  // conj(p1) IFFT_unnormalised(conj(p0) .) / L
  C* Y = reinterpret_cast<C*>(ws + l.Y);
  using T = decltype(C::x);
  return run_four_step<C>(P, G, 0, Y, gg, 1, true, chirp_tab<C>(P, P.off.chirp0, 1),
                          chirp_tab<C>(P, P.off.chirp1, 1), T(1) / T(P.L), tab<C>(P, P.off.tw_L),
                          tab<C>(P, P.off.tw_1), tab<C>(P, P.off.tw_2), st);
}

// FP64 window preparation: Zak of the sheared window; writes the plan-dtype
// conj(Z)/d table (zc_out) and/or the FP64 Zak (z64_out).
template <typename CO>
int window_zak(const Plan& P, const double2* g, CO* zc_out, double2* z64_out, char* ws, const Layout& l,
               hipStream_t st) {
  if (P.branch == kFir) {
    if (!zc_out) return fail(DGTNS_EUNSUPPORTED, "FIR plans keep only the window support");
    return launch_raw(k_fir_window<CO>, dim3(cdiv(P.fir_len, kThreads)), dim3(kThreads), 0, st,
                      "FIR window support", g, zc_out, (long long)P.L, (long long)P.fir_start, int(P.fir_len));
  }
  const double2* src = g;
  ChirpSrc<double2> ch = chirp_fly(P, P.sh.s1, 0);
  if (P.branch == kSeparable) ch = no_chirp<double2>(P);
  if (P.branch == kFreqShear) {
    double2* Y = reinterpret_cast<double2*>(ws + l.Y);
    double2* G = reinterpret_cast<double2*>(ws + l.G);
    int rc = run_four_step<double2>(P, g, 0, Y, G, 1, false, chirp_fly(P, P.sh.s1, 0), chirp_fly(P, -P.sh.s0, 0),
                                    1.0 / double(P.L), nullptr, tab<double2>(P, P.off.tw_1_64),
                                    tab<double2>(P, P.off.tw_2_64), st);
    if (rc) return rc;
    src = G;
    ch = no_chirp<double2>(P);
  }
  if (P.longd) {
    // long columns: first column pass of the prepared window in FP64, then
    // the length-d2 DFTs into the digit-reversed tables (one window: the
    // planner refuses multiwindow plans with long columns)
    double2* U = reinterpret_cast<double2*>(ws + l.U);
    LongColArgs<double2> A;
    std::memset(&A, 0, sizeof(A));
    A.x = src; A.pre = ch; A.post.L = P.L;
    A.y = U; A.ys = P.L;
    A.tws = tab<double2>(P, P.off.tw_d1_64); A.twd = tab<double2>(P, P.off.tw_d64);
    A.n = int(P.d1); A.Sn = int(P.d1 | 1); A.W = block_width(A.Sn, 16);
    A.ncols = int(P.d2 * P.Mi * P.pi); A.inmode = 0; A.outmode = 0; A.twmode = 1; A.tdiv = int(P.Mi * P.pi);
    A.d = int(P.di); A.d2 = int(P.d2); A.fs = sched(P.fd1);
    int rc = launch(k_long_col<double2, false>, dim3(cdiv(A.ncols, A.W), 1, 1), 16 * (P.d1 + size_t(A.W) * A.Sn), st,
                    A, "window Zak, first column pass");
    if (rc) return rc;
    const int S = int(P.d2 | 1);
    int W = 16;
    while (W > 1 && (W * P.pi * P.d2 > 4096 || 16 * (P.d2 + size_t(W) * P.pi * S) > (64u << 10))) --W;
    const size_t zl = 16 * (P.d2 + size_t(W) * P.pi * S);
    if (zl > 160 * 1024) return fail(DGTNS_EUNSUPPORTED, "window Zak: LDS request above 160 KiB");
    if (zl > 64 * 1024 && !dry_run()) {
      rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_long_zak<CO>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(zl)),
                     "window Zak");
      if (rc) return rc;
    }
    return launch_raw(k_long_zak<CO>, dim3(unsigned(P.d1) * cdiv(P.Mi, W)), dim3(kThreads),
                      zl, st, "window Zak, middle pass", (const double2*)U, zc_out,
                      z64_out, tab<double2>(P, P.off.tw_d2_64), int(P.Mi), int(P.pi), int(P.di), int(P.d1),
                      int(P.d2), W, S, sched(P.fd2));
  }
  ZakArgs<CO> Z;
  Z.x = src; Z.chirp = ch; Z.zc = zc_out; Z.z64 = z64_out;
  Z.L = P.L; Z.shift = 0; Z.mod2 = 0;
  Z.twd = tab<double2>(P, P.off.tw_d64);
  Z.Mi = int(P.Mi); Z.d = int(P.di); Z.p = int(P.pi); Z.Sd = int(P.di | 1);
  Z.W = block_width(P.pi * Z.Sd, 16);
  Z.fd = sched(P.fd);
  size_t lds = 16 * (P.di + size_t(Z.W) * P.pi * Z.Sd);
  // one table per window: the multiwindow algorithm's coset windows
  // g_mu(l) = exp(2 pi i l sigma_mu / L) g(l - mu a) (Prop. 5), each L values
  for (long long mu = 0; mu < P.nw; ++mu) {
    ZakArgs<CO> Zm = Z;
    if (P.branch == kMultiwindow) {
      Zm.shift = mu * P.a;
      Zm.mod2 = 2 * mw_sigma(P, mu) % (2 * P.L);
      if (zc_out) Zm.zc = zc_out + mu * P.L;
      if (z64_out) Zm.z64 = z64_out + mu * P.L;
    }
    int rc = launch(k_zak_fwd<CO>, dim3(cdiv(P.Mi, Z.W), 1), lds, st, Zm, "window Zak transform");
    if (rc) return rc;
  }
  return DGTNS_OK;
}



// Canonical dual window in FP64 (Alg. 2, with the time shear undone at the
// end): Zak of the sheared window, division by the diagonal of the frame
// operator (p = 1) or inversion of its p x p blocks (p > 1), inverse Zak, and
// for s0 != 0 the inverse frequency shear.
// tight: the canonical tight window S^{-1/2} g by the same steps (Section
// 4.2), dividing by the square root of the diagonal; with a frequency shear
// the window transform scaled by 1/L is undone by sqrt(L) instead of L, as
// S^{-1/2} of a positive multiple of a window is that of the window itself.
inline int dual_impl(const Plan& P, const double2* g_dev, double2* gd_dev, double* bounds_dev, char* w,
                     const Layout& l, hipStream_t st, bool tight = false) {
  int rc;
  double2* Z = reinterpret_cast<double2*>(w + l.H);
  double2* Zd = reinterpret_cast<double2*>(w + l.F);
  double2* Gd = reinterpret_cast<double2*>(w + l.G);
  double* part = reinterpret_cast<double*>(w + l.part);
  // the Zak of the frequency-sheared window uses the Y/G scratch of set_window:
  // map it onto this layout (Y = l.Y, G = Gd before it is overwritten)
  Layout lw;
  lw.Y = l.Y;
  lw.G = l.G;
  lw.U = l.U;
  rc = window_zak<double2>(P, g_dev, nullptr, Z, w, lw, st);
  if (rc) return rc;
  const long long tot = P.Mi * P.di;
  unsigned nb = cdiv(tot, kThreads);
  const double sb = P.branch == kFreqShear ? double(P.L) : 1.0;
  if (P.pi == 1)
    rc = launch_raw(k_dual_div<>, dim3(nb), dim3(kThreads), 0, st, "dual division", Z, Zd, part, int(P.Mi),
                    int(P.di), int(P.ai), int(P.qi), sb, tight ? 1 : 0);
  else if (P.pi > kDualMaxP) {
    // one wavefront per block, S and its eigenvectors in LDS
    nb = unsigned(std::min<long long>(tot, kDualLdsGroups));
    const size_t lds = 32 * size_t(P.pi) * size_t(P.pi);
    if (lds > 64 * 1024 && !dry_run()) {
      rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_dual_block_lds<>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)),
                     "dual block inversion");
      if (rc) return rc;
    }
    rc = launch_raw(k_dual_block_lds<>, dim3(nb), dim3(64), lds, st, "dual block inversion", (const double2*)Z, Zd,
                    part, int(P.Mi), int(P.di), int(P.pi), int(P.ai), int(P.qi), sb, tight ? 1 : 0,
                    P.longd ? int(P.d2) : 0);
  } else {
    auto kern = P.pi <= 2 ? k_dual_block<2> : P.pi <= 4 ? k_dual_block<4> : k_dual_block<kDualMaxP>;
    rc = launch_raw(kern, dim3(nb), dim3(kThreads), 0, st, "dual block inversion", (const double2*)Z, Zd, part,
                    int(P.Mi), int(P.di), int(P.pi), int(P.ai), int(P.qi), sb, tight ? 1 : 0,
                    P.longd ? int(P.d2) : 0);
  }
  if (rc) return rc;
  rc = launch_raw(k_minmax_final<>, dim3(1), dim3(kThreads), 0, st, "frame bounds", (const double*)part, int(nb),
                  bounds_dev);
  if (rc) return rc;
  const ChirpSrc<double2> post = P.branch == kFreqShear ? no_chirp<double2>(P)
                                 : P.branch == kSeparable ? no_chirp<double2>(P)
                                                          : chirp_fly(P, P.sh.s1, 1);
  double2* xout = P.branch == kFreqShear ? Gd : gd_dev;
  if (P.longd) {
    // two-level inverse Zak: length-d2 inverse DFTs of the digit-reversed
    // tables with the twiddles and 1/d, then the length-d1 inverse DFTs
    double2* U = reinterpret_cast<double2*>(w + l.U);
    const int S = int(P.d2 | 1);
    int W = 16;
    while (W > 1 && (W * P.pi * P.d2 > 4096 || 16 * (P.d2 + size_t(W) * P.pi * S) > (64u << 10))) --W;
    const size_t zl = 16 * (P.d2 + size_t(W) * P.pi * S);
    if (zl > 160 * 1024) return fail(DGTNS_EUNSUPPORTED, "inverse Zak: LDS request above 160 KiB");
    if (zl > 64 * 1024 && !dry_run()) {
      rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_long_zak_inv<>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(zl)),
                     "inverse Zak");
      if (rc) return rc;
    }
    rc = launch_raw(k_long_zak_inv<>, dim3(unsigned(P.d1) * cdiv(P.Mi, W)), dim3(kThreads), zl, st,
                    "inverse Zak, middle pass", (const double2*)Zd, U, tab<double2>(P, P.off.tw_d2_64),
                    tab<double2>(P, P.off.tw_d64), int(P.Mi), int(P.pi), int(P.di), int(P.d1), int(P.d2), W, S,
                    sched(P.fd2));
    if (rc) return rc;
    LongColArgs<double2> A;
    std::memset(&A, 0, sizeof(A));
    A.x = U; A.pre = no_chirp<double2>(P); A.post = post;
    A.y = xout; A.ys = P.L;
    A.tws = tab<double2>(P, P.off.tw_d1_64); A.twd = tab<double2>(P, P.off.tw_d64);
    A.n = int(P.d1); A.Sn = int(P.d1 | 1); A.W = block_width(A.Sn, 16);
    A.ncols = int(P.d2 * P.Mi * P.pi); A.inmode = 0; A.outmode = 2; A.twmode = 0;
    A.d = int(P.di); A.d2 = int(P.d2); A.fs = sched(P.fd1);
    rc = launch(k_long_col<double2, true>, dim3(cdiv(A.ncols, A.W), 1, 1), 16 * (P.d1 + size_t(A.W) * A.Sn), st,
                A, "inverse Zak, last column pass");
    if (rc) return rc;
  } else {
    ZakInvArgs Zi;
    Zi.z = Zd;
    Zi.twd = tab<double2>(P, P.off.tw_d64);
    Zi.Mi = int(P.Mi); Zi.d = int(P.di); Zi.p = int(P.pi); Zi.Sd = int(P.di | 1);
    Zi.W = block_width(P.pi * Zi.Sd, 16);
    Zi.fd = sched(P.fd);
    const size_t lds = 16 * (P.di + size_t(Zi.W) * P.pi * Zi.Sd);
    Zi.chirp = post;
    Zi.x = xout;
    rc = launch(k_zak_inv<>, dim3(cdiv(P.Mi, Zi.W), 1), lds, st, Zi, "inverse Zak");
    if (rc) return rc;
  }
  if (P.branch != kFreqShear) return DGTNS_OK;
  // g_d = conj(p1) IFFT(conj(p0) dual_sep(G))  (Alg. 2 with the time shear undone)
  double2* Y = reinterpret_cast<double2*>(w + l.Y);
  return run_four_step<double2>(P, Gd, 0, Y, gd_dev, 1, true, chirp_fly(P, -P.sh.s0, 1),
                                chirp_fly(P, P.sh.s1, 1), tight ? 1.0 / std::sqrt(double(P.L)) : 1.0 / double(P.L),
                                nullptr,
                                tab<double2>(P, P.off.tw_1_64), tab<double2>(P, P.off.tw_2_64), st);
}

// per-precision entry points (launch_c64.hip, launch_c128.hip)
int forward_c64(const Plan& P, const void* f, int real_in, void* c, long long B, char* ws, const Layout& l,
                hipStream_t st);
int forward_c128(const Plan& P, const void* f, int real_in, void* c, long long B, char* ws, const Layout& l,
                 hipStream_t st);
int forward_list_c64(const Plan& P, const void* const* f, int real_in, void* const* c, long long B, char* ws,
                     const Layout& l, hipStream_t st);
int forward_list_c128(const Plan& P, const void* const* f, int real_in, void* const* c, long long B, char* ws,
                      const Layout& l, hipStream_t st);
int adjoint_c64(const Plan& P, const void* c, void* f, long long B, char* ws, const Layout& l, hipStream_t st);
int adjoint_c128(const Plan& P, const void* c, void* f, long long B, char* ws, const Layout& l, hipStream_t st);
int grad_c64(const Plan& P, const void* f, const void* gc, void* gg, long long B, char* ws, const Layout& l,
             hipStream_t st);
int grad_c128(const Plan& P, const void* f, const void* gc, void* gg, long long B, char* ws, const Layout& l,
              hipStream_t st);
int set_window_c64(const Plan& P, const double2* g, char* ws, const Layout& l, hipStream_t st);
int set_window_c128(const Plan& P, const double2* g, char* ws, const Layout& l, hipStream_t st);
int dual_c128(const Plan& P, const double2* g, double2* gd, double* bounds, char* ws, const Layout& l, bool tight,
              hipStream_t st);

}  // namespace host
}  // namespace dgtns
