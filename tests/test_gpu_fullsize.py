"""GPU parity at the sizes the benchmark times, element by element against
the FP64 oracle: the adjoint of the quincunx workload on complete signals
(FP32 and FP64, batch 64), the adjoint of the precision workload on sampled
output samples (shear and FIR plans, Gaussian and Hann windows), and every
row of the shear-versus-multiwindow crossover (the Fig. 2 lattices of
Section 4.4) under both algorithms."""
import functools

import numpy as np
import pytest

import oracle
from dgt_inputs import (LARGE, PRECISION, complex_normal, crossover_batch, crossover_lattices, gaussian_window,
                        hann_window, round_to, seed_for)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}


def rel(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1307_4569_amd import _binding
    _binding.lib()
    return torch.device("cuda", 0)


def coefficient_pair(w, seed0):
    """Two seeded coefficient arrays (N, M), rounded to FP32 so that the same
    values feed the FP32 and the FP64 runs and one oracle result serves both."""
    return [round_to(complex_normal(w.N * w.M, seed0 + k).reshape(w.N, w.M), True) for k in range(2)]


# ---------------------------------------------------------------------------
# Quincunx workload (L = 2^18, a = 64, M = 512, lambda = 1/2, batch 64)
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def large_adjoint_reference():
    w = LARGE
    g = round_to(gaussian_window(w.L, w.a, w.M), True)
    cs = coefficient_pair(w, seed_for(2, 500))
    refs = [oracle.idgt_adjoint(c, g, w.a, w.M, w.lam1, w.lam2) for c in cs]
    return g, cs, refs


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_large_workload_adjoint_complete_signals(dtype):
    """Adjoint of a batch of 64 coefficient arrays, as the benchmark times it:
    signals 0 and 63 compared with the oracle's synthesis at every sample."""
    from paper_1307_4569_amd import Plan
    w = LARGE
    g, cs, refs = large_adjoint_reference()
    plan = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=dtype, max_batch=w.batch)
    plan.set_window(torch.tensor(g))
    pair = torch.stack([torch.tensor(c) for c in cs]).to(dtype).cuda()
    cin = pair.repeat(w.batch // 2, 1, 1)            # signal k holds cs[k % 2]
    fa = plan.adjoint(cin)
    torch.cuda.synchronize()
    errs = [rel(fa[0].cpu().numpy(), refs[0]), rel(fa[w.batch - 1].cpu().numpy(), refs[1])]
    print("large workload adjoint", dtype, "complete signals 0 and 63:", errs)
    assert max(errs) < TOL[dtype]
    # every other signal of the batch equals the one with the same input
    assert torch.equal(fa[2], fa[0]) and torch.equal(fa[w.batch - 3], fa[w.batch - 1])


# ---------------------------------------------------------------------------
# Precision workload (L = 2^20, a = 128, M = 1024, lambda = 1/4, batch 16)
# ---------------------------------------------------------------------------

PRECISION_SAMPLES = np.concatenate([(127 * np.arange(8192)) % PRECISION.L, [PRECISION.L - 1]])


@functools.lru_cache(maxsize=None)
def precision_adjoint_reference(window):
    w = PRECISION
    g = gaussian_window(w.L, w.a, w.M) if window == "gaussian" else hann_window(w.L, 2048)
    g = round_to(g, True)
    cs = coefficient_pair(w, seed_for(3, 500))
    refs = [oracle.idgt_adjoint(c, g, w.a, w.M, w.lam1, w.lam2, samples=PRECISION_SAMPLES) for c in cs]
    return g, cs, refs


@pytest.mark.parametrize("window,algorithm", [("gaussian", "shear"), ("hann", "shear"), ("hann", "fir")])
def test_precision_workload_adjoint_sampled(window, algorithm):
    """FP32 adjoint of a batch of 16 at L = 2^20: signals 0 and 15 at 8193
    samples (stride 127, every residue mod M) against the oracle.  The FIR
    plan's support (L - 1024, 2048 samples) holds the whole Hann window, so
    it is compared with the same reference."""
    from paper_1307_4569_amd import Plan
    w = PRECISION
    g, cs, refs = precision_adjoint_reference(window)
    kw = {"algorithm": "fir", "support": (w.L - 1024, 2048)} if algorithm == "fir" else {}
    plan = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=torch.complex64, max_batch=w.batch, **kw)
    plan.set_window(torch.tensor(g))
    pair = torch.stack([torch.tensor(c) for c in cs]).to(torch.complex64).cuda()
    fa = plan.adjoint(pair.repeat(w.batch // 2, 1, 1))
    idx = torch.tensor(PRECISION_SAMPLES, device="cuda")
    got = [fa[0, idx].cpu().numpy(), fa[w.batch - 1, idx].cpu().numpy()]
    errs = [rel(got[0], refs[0]), rel(got[1], refs[1])]
    print("precision workload adjoint", window, algorithm, errs)
    assert max(errs) < 1e-5


# ---------------------------------------------------------------------------
# Crossover rows (Fig. 2 lattices), both algorithms
# ---------------------------------------------------------------------------

CROSSOVER = crossover_lattices()


def crossover_columns(N):
    return sorted({0, 1, N // 7, N // 3, N // 2, (2 * N) // 3, N - 2, N - 1})


@functools.lru_cache(maxsize=None)
def crossover_reference(lat):
    L, a, M, l1, l2 = lat
    N = L // a
    f = [round_to(complex_normal(L, seed_for(6, 10 * k + l2)), True) for k in range(2)]
    g = round_to(gaussian_window(L, a, M), True)
    cols = crossover_columns(N)
    fwd = [oracle.dgt_fold(x, g, a, M, l1, l2, columns=cols) for x in f]
    cin = round_to(complex_normal(N * M, seed_for(6, 500 + l2)).reshape(N, M), True)
    pts = np.linspace(0, L - 1, 48).astype(np.int64)
    adj = oracle.idgt_adjoint(cin, g, a, M, l1, l2, samples=pts)
    return f, g, cols, fwd, cin, pts, adj


@pytest.mark.parametrize("algorithm", ["shear", "multiwindow"])
@pytest.mark.parametrize("lat", CROSSOVER, ids=[f"{l[1]}-{l[2]}-{l[3]}_{l[4]}" for l in CROSSOVER])
def test_crossover_row(lat, algorithm):
    """One crossover lattice at its own length, FP32, the benchmark's batch
    size: sampled time positions of the first and last signal against the
    oracle's eq. (DGT), the adjoint at 48 samples, and adjointness over the
    whole batch."""
    from paper_1307_4569_amd import Plan
    L, a, M, l1, l2 = lat
    N = L // a
    B = crossover_batch(L)
    f, g, cols, fwd, cin, pts, adj = crossover_reference(lat)
    plan = Plan(*lat, dtype=torch.complex64, max_batch=B, algorithm=algorithm)
    plan.set_window(torch.tensor(g))
    ft = torch.stack([torch.tensor(f[k % 2]) for k in range(B)]).to(torch.complex64).cuda()
    c = plan.forward(ft)
    last = (B - 1) % 2
    errs = [rel(c[0, cols].cpu().numpy(), fwd[0]), rel(c[B - 1, cols].cpu().numpy(), fwd[last])]
    ca = torch.tensor(cin).to(torch.complex64).cuda().unsqueeze(0).repeat(B, 1, 1)
    fa = plan.adjoint(ca)
    e_adj = rel(fa[B - 1, torch.tensor(pts, device="cuda")].cpu().numpy(), adj)
    lhs = torch.vdot(c.flatten().to(torch.complex128), ca.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(ft.flatten().to(torch.complex128), fa.flatten().to(torch.complex128)).item()
    e_dot = abs(lhs - rhs) / (c.norm().item() * ca.norm().item())
    print("crossover", lat, algorithm, "branch", plan.info.branch, "p", plan.info.p, "d", plan.info.d,
          "forward", errs, "adjoint", e_adj, "adjointness", e_dot)
    assert max(errs) < 1e-5 and e_adj < 1e-5 and e_dot < 1e-6


# ---------------------------------------------------------------------------
# Sequential chunks against one launch per stage
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.complex64])
def test_sequential_chunks_equal_single_launch(dtype, monkeypatch):
    """The quincunx workload's forward and adjoint in sequential chunks (the
    default for FP32 batches whose h exceeds the last-level cache) give the
    coefficients and signals of one launch per stage bit for bit, with a
    ragged last chunk (61 signals)."""
    from paper_1307_4569_amd import Plan
    w = LARGE
    g = torch.tensor(round_to(gaussian_window(w.L, w.a, w.M), dtype == torch.complex64))
    plans = {}
    for env in ("128", "0"):
        monkeypatch.setenv("DGTNS_SEQ_MIB", env)
        plans[env] = Plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype=dtype, max_batch=w.batch)
        plans[env].set_window(g)
    nb = 61
    f = torch.stack([torch.tensor(round_to(complex_normal(w.L, seed_for(2, 700 + k)), True)) for k in range(4)])
    f = f.to(dtype).cuda().repeat(16, 1)[:nb]
    c1, c0 = plans["128"].forward(f), plans["0"].forward(f)
    f1, f0 = plans["128"].adjoint(c0), plans["0"].adjoint(c0)
    torch.cuda.synchronize()
    assert torch.equal(c1, c0)
    assert torch.equal(f1, f0)
    # and one chunk's signal against the oracle's eq. (DGT) on sampled columns
    cols = [0, 1, w.N // 3, w.N - 1]
    ref = oracle.dgt_fold(f[60].cpu().to(torch.complex128).numpy(), g.numpy(), w.a, w.M, w.lam1, w.lam2,
                          columns=cols)
    assert rel(c1[60, cols].cpu().numpy(), ref) < TOL[dtype]
