"""Throughput benchmark of the shear DGT on one MI355X.

One step = the forward transform of one batch of the quincunx workload
(64 complex signals, L = 2^18, a = 64, M = 512, lambda = 1/2, redundancy 8) in
FP32 with plan tables and window resident in HBM: chirp (time shear),
factorisation kernel, channel DFT + phase correction.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join("paper_1307_4569_amd", "csrc")


def kernel_sources():
    """Every source of the native library: stored HBM-counter readings are
    valid only for the exact code they were taken on."""
    d = os.path.join(ROOT, CSRC)
    return sorted(os.path.join(CSRC, n) for n in os.listdir(d) if n.endswith((".hpp", ".hip", ".cpp", ".h")))


def sources_hash() -> str:
    h = hashlib.sha256()
    for p in kernel_sources():
        h.update(p.encode())
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel_err(got, ref) -> float:
    import numpy as np
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))


def sample_columns(N: int, n: int = 12):
    """Time positions spread over Z_N, first and last included."""
    import numpy as np
    return sorted(set(np.linspace(0, N - 1, n).astype(int).tolist()))


class Deferred:
    """Comparisons of GPU results with the oracle.  The GPU sections copy
    what a comparison needs (inputs, sampled GPU outputs) to the host and
    register it here; the comparisons run only in the CPU-baseline leg, the
    one part of the benchmark that runs the oracle (none run with
    --no-cpu-baseline).  Each result lands at target[key]."""

    def __init__(self):
        self.items = []

    def add(self, target: dict, key: str, fn):
        self.items.append((target, key, fn))

    def run(self):
        for target, key, fn in self.items:
            try:
                target[key] = fn()
            except Exception as e:      # noqa: BLE001 - reported in the output line
                target[key] = f"error: {type(e).__name__}: {e}"
        self.items = []


CHECKS = Deferred()


def forward_check(c_dev, f_host, g_host, lat, signals, cols=None, channels=None):
    """Largest relative l2 error of the GPU coefficients c_dev (B, N, M) of the
    given signals against the oracle's eq. (DGT) on sampled time positions
    (the GPU values are copied now, the oracle runs later).  channels: only
    the first that many channels are stored (real-signal layout, lambda2 <= 2)."""
    L, a, M, l1, l2 = lat
    cols = cols or sample_columns(L // a)
    got = {k: c_dev[k, cols].cpu().numpy() for k in signals}
    fs = {k: f_host[k] for k in signals}
    nch = channels or M

    def fn():
        import oracle
        return max(rel_err(got[k], oracle.dgt_fold(fs[k], g_host, a, M, l1, l2, columns=cols)[:, :nch])
                   for k in signals)
    return fn


def adjoint_check(fa_dev, c_dev, g_host, lat, signals, nsamp=2048):
    """Largest relative l2 error of the GPU synthesis fa_dev (B, L) of the
    coefficients c_dev against the oracle at nsamp sampled samples."""
    import numpy as np
    import torch
    L, a, M, l1, l2 = lat
    samples = np.unique(np.linspace(0, L - 1, nsamp).astype(np.int64))
    idx = torch.tensor(samples, device=fa_dev.device)
    got = {k: fa_dev[k, idx].cpu().numpy() for k in signals}
    cin = {k: c_dev[k].cpu().numpy().astype(np.complex128) for k in signals}

    def fn():
        import oracle
        return max(rel_err(got[k], oracle.idgt_adjoint(cin[k], g_host, a, M, l1, l2, samples=samples))
                   for k in signals)
    return fn


def algorithmic_bytes_per_step(kernel: str, es: int, L: int, MN: int, B: int) -> int:
    """Bytes a kernel must move per step (whole batch): its inputs and outputs
    once.  factorisation kernel: read the signals (L each) and write h (M N
    each); channel DFT: read h and write the coefficients (2 M N each).  A
    launch that processes a chunk of the batch moves its share."""
    if kernel.startswith("factorisation"):
        return es * (L + MN) * B
    if kernel.startswith("channel DFT"):
        return 2 * es * MN * B
    return 0


def rotating(f, nbytes_min=3 << 28):
    """Copies of the input batch at distinct addresses, enough that together
    they exceed the 256 MB last-level cache: the timed steps cycle through
    them, so every step reads its input from HBM as a new batch would."""
    n = max(2, -(-nbytes_min // (f.numel() * f.element_size())))
    return [f] + [f.clone() for _ in range(n - 1)]


def time_forward(plan, f, c, steps, warmup, torch, B_mod):
    """Milliseconds per forward (HIP events around exactly `steps` steps,
    no other events in between), host wall milliseconds per step, and the
    per-kernel times of a second pass of `steps` steps with every library
    launch bracketed by events on its stream (those events cost a few
    microseconds per launch, so they stay out of the first pass)."""
    fl = f if isinstance(f, list) else [f]
    for i in range(warmup):
        plan.forward(fl[i % len(fl)], out=c)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for i in range(steps):
        plan.forward(fl[i % len(fl)], out=c)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B_mod.dgtns_timing_reset()
    B_mod.dgtns_timing_enable(1)
    for i in range(steps):
        plan.forward(fl[i % len(fl)], out=c)
    torch.cuda.synchronize()
    B_mod.dgtns_timing_enable(0)
    kt = B_mod.kernel_times()
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3, kt


def time_adjoint(plan, c, fa, steps, torch, B_mod, warmup=3):
    """Milliseconds per adjoint of the batch c into fa (no events between the
    steps), and per-kernel times from a second, instrumented pass."""
    for _ in range(warmup):
        plan.adjoint(c, out=fa)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.adjoint(c, out=fa)
    e1.record()
    torch.cuda.synchronize()
    B_mod.dgtns_timing_reset()
    B_mod.dgtns_timing_enable(1)
    for _ in range(steps):
        plan.adjoint(c, out=fa)
    torch.cuda.synchronize()
    B_mod.dgtns_timing_enable(0)
    return e0.elapsed_time(e1) / steps, B_mod.kernel_times()


def crossover_bench(torch, dev, steps=5):
    """Shear versus multiwindow algorithm as the lattice complexity lambda2
    grows (the experiment of Section 4.4, Fig. 2): lambda = 1/lambda2,
    lambda2 = 1..10, L = lcm(a, M) 2520 (the least length feasible for all of
    them), (a, M) = (32, 64), (40, 60), (60, 80); FP32 forward on a batch of
    about 2^22 samples, milliseconds per signal."""
    import math

    import numpy as np

    from dgt_inputs import complex_normal_batch, gaussian_window
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bm
    rows = []
    for (a, M) in ((32, 64), (40, 60), (60, 80)):
        L = a * M // math.gcd(a, M) * 2520
        B = max(1, (1 << 22) // L)
        f = torch.tensor(complex_normal_batch(B, L, 5).astype(np.complex64), device=dev)
        fr = rotating(f)
        g = torch.tensor(gaussian_window(L, a, M))
        f_host = f[:1].cpu().numpy().astype(np.complex128)
        g_host = gaussian_window(L, a, M).astype(np.complex64).astype(np.complex128)
        for lam2 in range(1, 11):
            lam1 = 1 if lam2 > 1 else 0
            row = {"a": a, "M": M, "L": L, "lambda": f"{lam1}/{lam2}", "batch": B}
            for alg in ("shear", "multiwindow"):
                try:
                    plan = Plan(L, a, M, lam1, lam2, dtype=torch.complex64, max_batch=B, device=dev,
                                algorithm=alg)
                except Bm.DgtnsError as e:
                    row[alg] = {"unsupported": str(e)}
                    continue
                plan.set_window(g)
                c = torch.empty((B, L // a, M), dtype=torch.complex64, device=dev)
                ms, _, _ = time_forward(plan, fr, c, steps, 2, torch, Bm)
                row[alg] = {"ms_per_signal": round(ms / B, 5), "branch": plan.info.branch, "p": plan.info.p,
                            "q": plan.info.q, "d": plan.info.d,
                            }
                CHECKS.add(row[alg], "rel_err_vs_oracle",
                           forward_check(c, f_host, g_host, (L, a, M, lam1, lam2), [0], sample_columns(L // a, 6)))
                del c, plan
            if "ms_per_signal" in row.get("shear", {}) and "ms_per_signal" in row.get("multiwindow", {}):
                row["faster"] = ("shear" if row["shear"]["ms_per_signal"] < row["multiwindow"]["ms_per_signal"]
                                 else "multiwindow")
                ap = Plan(L, a, M, lam1, lam2, dtype=torch.complex64, max_batch=1, device=dev, algorithm="auto")
                row["auto_choice"] = "multiwindow" if ap.info.branch == Bm.DGTNS_MULTIWINDOW else "shear"
                del ap
            rows.append(row)
            log(f"crossover a={a} M={M} lambda={lam1}/{lam2}: "
                + ", ".join(f"{k} {v.get('ms_per_signal')}" for k, v in row.items() if isinstance(v, dict)))
        del f, fr
    return rows


def gradient_bench(torch, dev, steps=20):
    """One training step of the differentiation workload (L = 65536, a = 32,
    M = 256, lambda = 1/2, 32 signals, FP32): c = DGT_g(f), loss
    sum((|c|^2 - T)^2), then gradients for f (the adjoint) and for a
    full-length trainable window g (the window gradient)."""
    import numpy as np

    from dgt_inputs import GRADIENT, complex_normal, complex_normal_batch, gaussian_window
    from paper_1307_4569_amd import DGTFunction, Plan
    from paper_1307_4569_amd import _binding as Bm
    w = GRADIENT
    plan = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=torch.complex64, max_batch=w.batch, device=dev)
    g0 = gaussian_window(w.L, w.a, w.M)
    plan.set_window(torch.tensor(g0))
    T = plan.forward(torch.tensor(complex_normal(w.L, 4000).astype(np.complex64), device=dev)).abs() ** 2
    f = torch.tensor(complex_normal_batch(w.batch, w.L, 4).astype(np.complex64), device=dev, requires_grad=True)
    g = torch.tensor(g0.astype(np.complex64), device=dev, requires_grad=True)

    def step():
        f.grad = None
        g.grad = None
        c = DGTFunction.apply(f, g, plan)
        loss = ((c.abs() ** 2 - T) ** 2).sum()
        loss.backward()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    Bm.dgtns_timing_reset()
    Bm.dgtns_timing_enable(1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    Bm.dgtns_timing_enable(0)
    kt = Bm.kernel_times()
    coeffs = w.batch * w.M * w.N
    lib_ms = sum(t for _, t in kt.values()) / steps
    res = {"workload": f"{w.name} FP32, loss sum((|c|^2 - T)^2), gradients for f and g",
           "ms_per_step": round(ms, 4), "coeffs_per_s": coeffs / (ms * 1e-3),
           "library_ms_per_step": round(lib_ms, 4),
           "kernels": {k: {"launches_per_step": n / steps, "avg_ms": round(t / n, 4)} for k, (n, t) in kt.items()}}
    # the last step's grad_f of signal 0 against the oracle; the batch's window
    # gradient sums all 32 signals, so a step on signals 0 and 1 alone checks
    # grad_g within the time budget
    T_h = T.cpu().numpy().astype(np.float64)
    f_h = f.detach()[:2].cpu().numpy().astype(np.complex128)
    g_h = g.detach().cpu().numpy().astype(np.complex128)
    gf_gpu = f.grad[0].cpu().numpy()
    f2 = f.detach()[:2].clone().requires_grad_(True)
    g2 = g.detach().clone().requires_grad_(True)
    plan2 = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=torch.complex64, max_batch=2, device=dev)
    c2 = DGTFunction.apply(f2, g2, plan2)
    ((c2.abs() ** 2 - T) ** 2).sum().backward()
    gg_gpu = g2.grad.cpu().numpy()

    def check():
        import oracle
        lat = (w.a, w.M, w.lam1, w.lam2)
        _, gf0, gg0 = oracle.loss_and_grads(f_h[0], g_h, T_h, *lat)
        _, _, gg1 = oracle.loss_and_grads(f_h[1], g_h, T_h, *lat)
        return {"grad_f_signal0": rel_err(gf_gpu, gf0), "grad_g_signals0_1": rel_err(gg_gpu, gg0 + gg1)}
    CHECKS.add(res, "rel_err_vs_oracle", check)
    return res


def fir_bench(torch, dev, steps=20, with_shear=True, with_adjoint=True):
    """Precision workload: L = 2^20, a = 128, M = 1024, lambda = 1/4, 16 real
    chirp signals (FP32).  The periodic Hann window of length 2048 centred at
    0 (support L - 1024 ... L + 1023 mod L) under the FIR-window, shear and
    shear-OLA algorithms, and the unit-norm Gaussian under the shear
    algorithm; the real-signal variant (non-redundant channels only) of the
    FIR and shear forwards; each with its error against the oracle on
    sampled time positions of the first and last signal, and the
    reconstruction through the canonical dual window computed in FP64 on the
    GPU.  The FIR kernel's compulsory traffic is the real signal (4 bytes
    per sample) and the coefficients (8 bytes each)."""
    import numpy as np

    from dgt_inputs import PRECISION, chirp_mixture, gaussian_window, hann_window, seed_for
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bm
    w = PRECISION
    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    x = np.stack([chirp_mixture(w.L, seed_for(3, k)) for k in range(w.batch)]).real.astype(np.float32)
    x_host = x.astype(np.complex128)
    xt = torch.tensor(x, device=dev)
    xr = rotating(xt)
    windows = {"hann": hann_window(w.L, 2048), "gaussian": gaussian_window(w.L, w.a, w.M)}
    g_host = {k: v.astype(np.complex64).astype(np.complex128) for k, v in windows.items()}
    coeffs = w.batch * w.M * w.N
    last = w.batch - 1
    out = {"workload": f"precision L={w.L} a={w.a} M={w.M} lambda={w.lam1}/{w.lam2} B={w.batch} real chirps, "
                       "Hann window of length 2048 and unit-norm Gaussian"}
    algs = [("fir", "hann", {"algorithm": "fir", "support": (w.L - 1024, 2048)})]
    if with_shear:
        algs += [("shear", "hann", {}), ("shear_gaussian", "gaussian", {})]
        # the shear algorithm on overlap-added blocks (Section 4)
        # (block transforms by the automatic plan, multiwindow here, and by
        # the shear plan, which needs a frequency shear at these lengths)
        algs += [(f"shear_ola_block{blk}", "hann", {"algorithm": "shear-ola", "support": (w.L - 1024, 2048),
                                                    "block": blk}) for blk in (32768, 131072)]
        algs += [("shear_ola_shear_block32768", "hann", {"algorithm": "shear-ola", "support": (w.L - 1024, 2048),
                                                         "block": 32768, "inner": "shear"})]
    for name, win, kw in algs:
        plan = Plan(*lat, dtype=torch.complex64, max_batch=w.batch, device=dev, **kw)
        plan.set_window(torch.tensor(g_host[win]))
        c = torch.empty((w.batch, w.N, w.M), dtype=torch.complex64, device=dev)
        ms, _, kt = time_forward(plan, xr, c, steps, 3, torch, Bm)
        out[name] = {"window": win, "ms_per_step": ms, "coeffs_per_s": coeffs / (ms * 1e-3),
                     "kernels": {k: round(t / n, 4) for k, (n, t) in kt.items()}}
        CHECKS.add(out[name], "rel_err_vs_oracle", forward_check(c, x_host, g_host[win], lat, [0, last]))
        if kw.get("algorithm") == "fir" and with_adjoint:
            # adjoint of the FIR transform: inverse DFTs of the columns, then the gather
            fa = torch.empty((w.batch, w.L), dtype=torch.complex64, device=dev)
            ams, akt = time_adjoint(plan, c, fa, steps, torch, Bm)
            out[name]["adjoint"] = {"ms_per_step": ams, "coeffs_per_s": coeffs / (ams * 1e-3),
                                    "kernels": {k: round(t / n, 4) for k, (n, t) in akt.items()}}
            CHECKS.add(out[name]["adjoint"], "rel_err_vs_oracle", adjoint_check(fa, c, g_host[win], lat, [0, last]))
            del fa
        if kw.get("algorithm") == "shear-ola":
            Lx = plan.info.block_dgt_length
            out[name]["block_dgt_length"] = Lx
            out[name]["rho"] = Lx / kw["block"]
            out[name]["block_transform"] = "multiwindow" if plan.info.windows > 1 else "shear"
        if name in ("fir", "shear_gaussian") and with_shear:
            # real-signal variant: the non-redundant channels (two half and two
            # whole columns per group of four), real samples back
            cr = torch.empty((w.batch,) + plan.real_shape, dtype=torch.complex64, device=dev)
            for _ in range(3):
                plan.forward_real(xt, out=cr)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(steps):
                plan.forward_real(xr[i % len(xr)], out=cr)
            e1.record()
            torch.cuda.synchronize()
            rms = e0.elapsed_time(e1) / steps
            groups = [0, 1, 517, w.N // w.lam2 - 1]
            got = {k: cr[k, groups].cpu().numpy() for k in (0, last)}

            def real_check(got=got, groups=groups, gw=g_host[win]):
                import oracle
                from oracle.real import pack_real
                cols = [4 * j + i for j in groups for i in range(4)]
                errs = []
                for k in (0, last):
                    full = np.zeros((w.N, w.M), complex)
                    full[cols] = oracle.dgt_fold(x_host[k], gw, w.a, w.M, w.lam1, w.lam2, columns=cols)
                    errs.append(rel_err(got[k], pack_real(full, w.M, w.lam1, w.lam2)[groups]))
                return max(errs)
            # reconstruction through the canonical dual (FP64 on the GPU) and the
            # real-signal synthesis
            dplan = Plan(*lat, dtype=torch.complex64, max_batch=w.batch, device=dev)
            gd, bounds = dplan.dual(torch.tensor(g_host[win]))
            dplan.set_window(gd)
            xrec = dplan.adjoint_real(cr)
            rec = float(torch.linalg.vector_norm(xrec - xt) / torch.linalg.vector_norm(xt))
            vals = cr.numel()
            out[name]["real_variant"] = {
                "ms_per_step": rms, "stored_coeffs_per_step": vals, "stored_coeffs_per_s": vals / (rms * 1e-3),
                "full_coeffs_per_s": coeffs / (rms * 1e-3),
                "reconstruction_rel_err_via_gpu_fp64_dual": rec,
                "frame_bounds": [float(v) for v in bounds.cpu()]}
            CHECKS.add(out[name]["real_variant"], "rel_err_vs_oracle", real_check)
            del cr, dplan, xrec
        del plan, c
    fb = w.batch * (4 * w.L + 8 * w.M * w.N)
    out["fir"]["compulsory_GBps"] = round(fb / (out["fir"]["ms_per_step"] * 1e-3) / 1e9, 1)
    if with_shear:
        out["fir_speedup"] = out["shear"]["ms_per_step"] / out["fir"]["ms_per_step"]
        log(f"FIR {out['fir']['coeffs_per_s'] / 1e9:.1f} Gcoeff/s, shear {out['shear']['coeffs_per_s'] / 1e9:.1f} "
            f"Gcoeff/s on the precision workload")
    return out


def cpu_baseline(w, f_host, g_host, c_gpu_fn, budget_s=12.0):
    """Time the FP64 oracle (per-column fold form, single-threaded NumPy) on a
    bounded sample of the workload: whole signals of the batch, in order,
    until the time budget is used.  Also returns the relative l2 error of the
    GPU coefficients of those signals against the oracle."""
    import numpy as np

    import oracle
    el = 0.0
    err_num = err_den = 0.0
    k = 0
    while k < len(f_host) and (k == 0 or el < budget_s):
        t0 = time.perf_counter()
        ref = oracle.dgt_fold(f_host[k], g_host, w.a, w.M, w.lam1, w.lam2)
        el += time.perf_counter() - t0
        got = c_gpu_fn(k)
        err_num += float(np.linalg.norm(got - ref) ** 2)
        err_den += float(np.linalg.norm(ref) ** 2)
        k += 1
    coeffs = k * w.N * w.M
    return {"value": coeffs / el, "unit": "coeffs/s", "cores": 1, "kind": "oracle",
            "sample": f"signals 0..{k - 1} of the batch, all {w.N}x{w.M} coefficients each "
                      f"({coeffs} coefficients, {el:.1f} s, single-threaded NumPy FP64 fold form)",
            "host": host_cpu()}, \
        (err_num / err_den) ** 0.5


def host_cpu():
    """The host the oracle ran on: logical cores and CPU model."""
    import os
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"logical_cores": os.cpu_count(), "usable_cores": usable, "model": model}


def _oracle_signal(args):
    """One signal through the FP64 oracle in a worker process; returns its
    coefficients' squared norm (the values stay in the worker)."""
    import numpy as np

    import oracle
    f, g, a, M, l1, l2 = args
    return float(np.linalg.norm(oracle.dgt_fold(f, g, a, M, l1, l2)) ** 2)


def cpu_baseline_parallel(w, f_host, g_host, max_workers=16, timeout_s=120.0):
    """The same oracle, one signal per worker process, P = min(16, usable
    host cores) processes (started and warmed up before the clock runs): the
    host's multi-process rate beside the single-threaded one.  16 is the CPU
    share of one GPU on the benchmark host, whatever its total core count.
    Any failure or a run past timeout_s ends the pool and is reported, not
    raised."""
    import multiprocessing as mp
    import os
    P = max(1, min(max_workers, host_cpu()["usable_cores"] or 1, len(f_host)))
    tasks = [(f_host[k], g_host, w.a, w.M, w.lam1, w.lam2) for k in range(P)]
    small = (f_host[0][:2 * w.M], g_host[:2 * w.M], 1, w.M, 0, 1)
    pool = mp.get_context("spawn").Pool(P)
    try:
        pool.map_async(_oracle_signal, [small] * P, chunksize=1).get(timeout_s)   # workers up, modules imported
        t0 = time.perf_counter()
        pool.map_async(_oracle_signal, tasks, chunksize=1).get(timeout_s)
        el = time.perf_counter() - t0
    except Exception as e:      # noqa: BLE001 - reported in the output line
        return {"error": f"{type(e).__name__}: {e}", "processes": P}
    finally:
        pool.terminate()
        pool.join()
    coeffs = P * w.N * w.M
    return {"value": coeffs / el, "unit": "coeffs/s", "processes": P, "cores": P,
            "sample": f"signals 0..{P - 1}, one per process ({coeffs} coefficients, {el:.1f} s wall)"}


def serve_bench(nreq, torch, dev):
    """Serving workload: a seeded stream of nreq requests over the 24 plans
    (L in {36864, 73728, 147456, 294912}, (a, M) in {(32,256), (64,512)},
    lambda in {1/2, 1/3, 2/3}), signals CN(0,1) pre-staged in HBM.  The FP32
    continuous-batching server (4 streams, list batches of up to 8) and the
    plain FP64 per-request server (1 stream, batch 1, shear algorithm) are
    each measured closed loop (capacity mu) and open loop with Poisson
    arrivals at 0.5, 0.8 and 0.95 mu.  The FP32 server's plans choose their
    algorithm (DGTNS_ALG_AUTO: multiwindow for the six lattices whose shear
    needs a frequency shear)."""
    import numpy as np

    from dgt_inputs import gaussian_window, poisson_arrivals, serving_plans, serving_requests, seed_for
    from paper_1307_4569_amd.serve import GpuExecutor, Request, Server, latency_stats

    plans = serving_plans()
    spec = serving_requests(nreq)
    # pre-stage signals: one seeded pool per signal length
    by_len = {}
    for j, (_, key, _) in enumerate(spec):
        by_len.setdefault(key[0], []).append(j)
    sig32 = [None] * nreq
    for L, idx in sorted(by_len.items()):
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed_for(5, L))
        pool = torch.randn((len(idx), L), dtype=torch.complex64, generator=gen, device=dev)
        for t, j in enumerate(idx):
            sig32[j] = pool[t]
    coeffs = lambda r: (r.key[0] // r.key[1]) * r.key[2]
    out = {"workload": f"serving mix: {nreq} requests over 24 plans (6 with a frequency shear)",
           "total_coeffs": int(sum((k[0] // k[1]) * k[2] for _, k, _ in spec))}

    def check(ex, sigs, tol_name):
        """Error against the oracle of 12 requests (two per (a, M) and shear
        kind, every plan family) served in one mix, on sampled time positions."""
        pick = []
        per_family = {}
        for j, (_, key, _) in enumerate(spec):
            fam = (key[1], key[2], key[4], ex.plan(key).info.branch)
            if per_family.get(fam, 0) < 2:
                per_family[fam] = per_family.get(fam, 0) + 1
                pick.append(j)
            if len(pick) >= 12:
                break
        srv = Server(ex, hbm_budget=16 << 30, max_inflight_per_slot=2, keep_outputs=True)
        reqs = srv.run([Request(j, spec[j][1], sigs[j], 0.0) for j in pick])
        torch.cuda.synchronize()
        cases = []
        for r in reqs:
            L, a, M, l1, l2 = r.key
            cols = sample_columns(L // a, 6)
            g = torch.tensor(gaussian_window(L, a, M)).to(ex.dtype).cpu().numpy().astype(np.complex128)
            cases.append((r.key, r.f.cpu().numpy().astype(np.complex128), g, cols, r.c[cols].cpu().numpy()))
        res = {"requests_checked": len(reqs), "bar": tol_name}

        def fn():
            import oracle
            return max(rel_err(got, oracle.dgt_fold(f, g, k[1], k[2], k[3], k[4], columns=cols))
                       for k, f, g, cols, got in cases)
        CHECKS.add(res, "max_rel_err_vs_oracle", fn)
        return res

    def run_server(name, dtype, streams, max_batch, inflight, sigs, rates=None, algorithm="auto"):
        ex = GpuExecutor(lambda k: torch.tensor(gaussian_window(k[0], k[1], k[2])), dtype=dtype, streams=streams,
                         max_batch=max_batch, device=dev, algorithm=algorithm)
        ex.prepare(plans)
        mk = lambda: [Request(j, key, sigs[j], 0.0) for j, (_, key, _) in enumerate(spec)]
        srv = Server(ex, hbm_budget=16 << 30, max_inflight_per_slot=inflight, keep_outputs=False)
        srv.run(mk()[: min(500, nreq)])
        torch.cuda.synchronize()
        srv = Server(ex, hbm_budget=16 << 30, max_inflight_per_slot=inflight, keep_outputs=False)
        cap = latency_stats(srv.run(mk()), coeffs)
        res = {"capacity": cap}
        mu = cap["req_per_s"]
        loads = [(f"load_{frac}", frac * mu) for frac in (0.5, 0.8, 0.95)]
        loads += [(f"at_{k}_req_per_s", v) for k, v in (rates or {}).items()]
        for label, rate in loads:
            arr = list(poisson_arrivals(nreq, rate, seed_for(5, int(rate) % 997)))
            srv = Server(ex, hbm_budget=16 << 30, max_inflight_per_slot=inflight, keep_outputs=False)
            st = latency_stats(srv.run(mk(), arr), coeffs)
            st["offered_req_per_s"] = rate
            res[label] = st
        res["oracle_check"] = check(ex, sigs, "1e-5" if dtype == torch.complex64 else "1e-12")
        del ex
        torch.cuda.synchronize()
        log(f"serve {name}: capacity {mu:.0f} req/s, p50/p99 at 0.8 mu: "
            f"{res['load_0.8']['p50_ms']:.3f}/{res['load_0.8']['p99_ms']:.3f} ms")
        failed = {k: v["failed"] for k, v in res.items() if isinstance(v, dict) and v.get("failed")}
        if failed:
            log(f"WARNING: serve {name}: failed requests {failed}")
        return res

    sig64 = [x.to(torch.complex128) for x in sig32]
    out["fp64_per_request"] = run_server("fp64", torch.complex128, 1, 1, 4, sig64, algorithm="shear")
    del sig64
    # the FP32 server also at the FP64 server's offered rates, for latencies
    # measured under the same load
    mu64 = out["fp64_per_request"]["capacity"]["req_per_s"]
    same = {f"fp64_{frac}": frac * mu64 for frac in (0.5, 0.8, 0.95)}
    out["fp32_batched"] = run_server("fp32", torch.complex64, 4, 8, 2, sig32, rates=same)
    a, b = out["fp32_batched"]["load_0.8"], out["fp64_per_request"]["load_0.8"]
    a_same = out["fp32_batched"]["at_fp64_0.8_req_per_s"]
    out["headline"] = {"p50_ms": a["p50_ms"], "p99_ms": a["p99_ms"], "coeffs_per_s": a["coeffs_per_s"],
                       "load": "0.8 of measured capacity",
                       "fp64_baseline_p50_ms": b["p50_ms"], "fp64_baseline_p99_ms": b["p99_ms"],
                       "fp32_at_fp64_rate_p50_ms": a_same["p50_ms"], "fp32_at_fp64_rate_p99_ms": a_same["p99_ms"],
                       "same_offered_req_per_s": a_same["offered_req_per_s"],
                       "capacity_speedup_vs_fp64": out["fp32_batched"]["capacity"]["coeffs_per_s"]
                       / out["fp64_per_request"]["capacity"]["coeffs_per_s"]}
    return out


def serve_profile(nreq, rate, torch, dev):
    """The FP32 continuous-batching server alone, open loop at `rate`
    requests/s (Poisson), for a kernel trace of the serving run."""
    from dgt_inputs import gaussian_window, poisson_arrivals, serving_plans, serving_requests, seed_for
    from paper_1307_4569_amd.serve import GpuExecutor, Request, Server, latency_stats
    spec = serving_requests(nreq)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed_for(5, 1))
    sigs = [torch.randn(key[0], dtype=torch.complex64, generator=gen, device=dev) for _, key, _ in spec]
    ex = GpuExecutor(lambda k: torch.tensor(gaussian_window(k[0], k[1], k[2])), dtype=torch.complex64, streams=4,
                     max_batch=8, device=dev)
    ex.prepare(serving_plans())
    torch.cuda.synchronize()
    arr = list(poisson_arrivals(nreq, rate, seed_for(5, 80)))
    srv = Server(ex, hbm_budget=16 << 30, max_inflight_per_slot=2, keep_outputs=False)
    st = latency_stats(srv.run([Request(j, key, sigs[j], 0.0) for j, (_, key, _) in enumerate(spec)], arr),
                       lambda r: (r.key[0] // r.key[1]) * r.key[2])
    torch.cuda.synchronize()
    log(f"serve profile at {rate:.0f} req/s offered: {json.dumps(st)}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--no-multiwindow", action="store_true")
    ap.add_argument("--no-crossover", action="store_true")
    ap.add_argument("--no-fir", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the FP32 forward loop (for rocprofv3)")
    ap.add_argument("--profile-fir", action="store_true",
                    help="run only the FIR forward loop of the precision workload (for rocprofv3)")
    ap.add_argument("--profile-serve", type=float, default=0.0, metavar="RATE",
                    help="run only the FP32 server open loop at RATE requests/s (for rocprofv3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (batches and requests shard across "
                                   "GPUs with no exchange, one process per GPU); use --gpus 1"}))
        sys.exit(2)
    if args.profile_serve > 0:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        serve_profile(args.serve_requests, args.profile_serve, torch, dev)
        return
    if args.profile_fir:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        r = fir_bench(torch, dev, steps=args.steps, with_shear=False, with_adjoint=False)
        log(f"FIR forward {r['fir']['ms_per_step']:.3f} ms/step")
        return

    import numpy as np
    import torch

    from dgt_inputs import LARGE, complex_normal_batch, gaussian_window
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bm

    w = LARGE
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"inputs: {w.name}")
    f64 = complex_normal_batch(w.batch, w.L, 2)
    g = gaussian_window(w.L, w.a, w.M)
    f32 = torch.tensor(f64.astype(np.complex64), device=dev)
    g32 = g.astype(np.complex64).astype(np.complex128)

    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    f_host32 = f32.cpu().numpy().astype(np.complex128)
    plan = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=torch.complex64, max_batch=w.batch, device=dev)
    plan.set_window(torch.tensor(g32))
    c = torch.empty((w.batch, w.N, w.M), dtype=torch.complex64, device=dev)
    MN = w.M * w.N
    coeffs = w.batch * MN
    log("fp32 forward timing")
    f32r = rotating(f32)
    ms, wall_ms, kt = time_forward(plan, f32r, c, args.steps, args.warmup, torch, Bm)
    if args.profile_only:
        log(f"fp32 forward {ms:.3f} ms/step")
        return
    value = coeffs / (ms * 1e-3)

    # dominant kernel and its roofline: bytes per launch = bytes per step
    # divided by the launches per step (the batch may run in chunks)
    dom = max(kt.items(), key=lambda kv: kv[1][1])
    dname, (dn, dms) = dom
    avg_ms = dms / dn
    per_step = dn / args.steps
    abytes = algorithmic_bytes_per_step(dname, 8, w.L, MN, w.batch) / per_step
    achieved = abytes / (avg_ms * 1e-3) / 1e9
    kernels = {}
    for k, (n, t) in kt.items():
        b = algorithmic_bytes_per_step(k, 8, w.L, MN, w.batch) / (n / args.steps)
        kernels[k] = {"launches_per_step": n / args.steps, "avg_ms": round(t / n, 4),
                      "algorithmic_bytes_per_launch": int(b),
                      "algorithmic_GBps": round(b / (t / n * 1e-3) / 1e9, 1)}
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath))
        ent = tr.get("kernels", {}).get(dname)
        if ent and tr.get("sources") == sources_hash():
            traffic = ent["bytes_per_launch"]

    out = {
        "metric": "nonsep DGT coeffs/s FP32 vs FP64 (rel err \u22641e-5); serve p50/p99 latency",
        "value": value,
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded complex normal signals, unit-norm periodic Gaussian window); "
                "timed steps cycle through copies of the batch at distinct addresses larger than the "
                "256 MB last-level cache together, so each step reads its input from HBM",
        "config": {"workload": w.name, "L": w.L, "a": w.a, "M": w.M, "lambda": f"{w.lam1}/{w.lam2}",
                   "batch": w.batch, "coeffs_per_step": coeffs, "branch": "time shear (s0=0, s1=-4)"},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(abytes), "avg_launch_ms": round(avg_ms, 4)},
        "kernels": kernels,
        "wall_ms_per_step": wall_ms,
        "whole_path": {"compulsory_bytes_per_coeff": 9.0,
                       "compulsory_GBps": round(9.0 * value / 1e9, 1),
                       "frac_of_compulsory_bound": round(9.0 * value / 1e9 / HBM_PEAK_GBS, 4),
                       # read f, write and read back h, write c: the two-kernel design's bytes
                       # if h made the round trip through HBM (here it stays in the Infinity Cache)
                       "two_kernel_bytes_per_coeff": 25.0,
                       "frac_of_two_kernel_bound": round(25.0 * value / 1e9 / HBM_PEAK_GBS, 4)},
    }

    # practical HBM ceiling: a plain device copy of the same size as the
    # coefficient array (read + write)
    cc = torch.empty_like(c)
    for _ in range(3):
        cc.copy_(c)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cc.copy_(c)
    e1.record()
    torch.cuda.synchronize()
    out["copy_GBps"] = round(2 * c.numel() * 8 / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9, 1)
    del cc

    # adjoint (synthesis) on the same batch, FP32
    log("fp32 adjoint timing")
    fa = torch.empty_like(f32)
    na = max(5, args.steps // 5)
    ams, akt = time_adjoint(plan, c, fa, na, torch, Bm)
    out["adjoint"] = {"ms_per_step": ams, "coeffs_per_s": coeffs / (ams * 1e-3),
                      "kernels": {k: {"launches_per_step": n / na, "avg_ms": round(t / n, 4)}
                                  for k, (n, t) in akt.items()}}
    CHECKS.add(out["adjoint"], "rel_err_vs_oracle", adjoint_check(fa, c, g32, lat, [0, w.batch - 1]))
    del fa

    # real-signal variant on real signals of the same lattice (lambda = 1/2:
    # every column conjugate symmetric, channels 0 .. M/2 stored)
    log("fp32 real-signal forward timing")
    xr32 = f32.real.contiguous()
    cr = torch.empty((w.batch,) + plan.real_shape, dtype=torch.complex64, device=dev)
    xrr = rotating(xr32)
    for i in range(3):
        plan.forward_real(xrr[i % len(xrr)], out=cr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        plan.forward_real(xrr[i % len(xrr)], out=cr)
    e1.record()
    torch.cuda.synchronize()
    rms = e0.elapsed_time(e1) / args.steps
    out["real_variant"] = {"ms_per_step": rms, "stored_coeffs_per_s": cr.numel() / (rms * 1e-3),
                           "full_coeffs_per_s": coeffs / (rms * 1e-3),
                           "compulsory_GBps": round(w.batch * (4 * w.L + 8 * cr[0].numel()) / (rms * 1e-3) / 1e9, 1)}
    # lambda = 1/2: the stored channels of column n are its first M/2 + 1
    CHECKS.add(out["real_variant"], "rel_err_vs_oracle",
               forward_check(cr.reshape(w.batch, w.N, w.M // 2 + 1), xr32[:1].cpu().numpy().astype(np.complex128),
                             g32, lat, [0], channels=w.M // 2 + 1))
    del cr, xrr, xr32

    if not args.no_fp64:
        log("fp64 forward timing")
        plan64 = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=torch.complex128, max_batch=w.batch, device=dev)
        plan64.set_window(torch.tensor(g))
        f64d = torch.tensor(f64, device=dev)
        c64 = torch.empty((w.batch, w.N, w.M), dtype=torch.complex128, device=dev)
        ms64, _, _ = time_forward(plan64, rotating(f64d), c64, max(5, args.steps // 5), 2, torch, Bm)
        out["fp64"] = {"ms_per_step": ms64, "value": coeffs / (ms64 * 1e-3),
                       "fp32_speedup": ms64 / ms,
                       }
        CHECKS.add(out["fp64"], "rel_err_vs_oracle", forward_check(c64, f64, g, lat, [0, w.batch - 1]))
        del c64, f64d, plan64
        torch.cuda.synchronize()

    if not args.no_multiwindow:
        # the same workload by the multiwindow algorithm (Section 3.1)
        log("fp32 forward timing, multiwindow algorithm")
        pmw = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=torch.complex64, max_batch=w.batch, device=dev,
                   algorithm="multiwindow")
        pmw.set_window(torch.tensor(g32))
        cmw = torch.empty_like(c)
        msm, _, ktm = time_forward(pmw, f32r, cmw, max(10, args.steps // 2), 3, torch, Bm)
        out["multiwindow"] = {"ms_per_step": msm, "coeffs_per_s": coeffs / (msm * 1e-3),
                              "vs_shear": ms / msm,

                              "kernels": {k: {"launches_per_step": n / max(10, args.steps // 2),
                                              "avg_ms": round(t / n, 4)} for k, (n, t) in ktm.items()}}
        CHECKS.add(out["multiwindow"], "rel_err_vs_oracle", forward_check(cmw, f_host32, g32, lat, [0, w.batch - 1]))
        del cmw, pmw
        torch.cuda.synchronize()
    if not args.no_crossover:
        log("shear versus multiwindow over lambda2")
        out["crossover"] = crossover_bench(torch, dev)
    if not args.no_fir:
        log("FIR-window algorithm on the precision workload")
        out["fir"] = fir_bench(torch, dev)
    if not args.no_gradient:
        log("training step of the differentiation workload")
        out["gradient"] = gradient_bench(torch, dev)

    if not args.no_serve:
        log("serving workload")
        torch.cuda.empty_cache()
        out["serve"] = serve_bench(args.serve_requests, torch, dev)
    if not args.no_cpu_baseline:
        # the CPU-baseline leg: the oracle timed on the host, then every
        # comparison of a GPU result with the oracle registered above
        log("cpu baseline (oracle)")
        f_host = f_host32

        def gpu_signal(k):
            return c[k].cpu().numpy().astype(np.complex128)

        cb, err = cpu_baseline(w, f_host, g32, gpu_signal)
        log("cpu baseline, one signal per process")
        cb["parallel"] = cpu_baseline_parallel(w, f_host, g32)
        out["cpu_baseline"] = cb
        out["rel_err_fp32_vs_oracle"] = err
        log(f"oracle comparisons of {len(CHECKS.items)} GPU results")
        t0 = time.perf_counter()
        CHECKS.run()
        log(f"oracle comparisons done in {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
