"""Serving loop on the GPU: each result is the same alone and in the mix of
all 24 plans of the serving workload, and admission keeps the in-flight HBM
footprint within a small budget."""
import numpy as np
import pytest

import oracle
from dgt_inputs import complex_normal, gaussian_window, serving_plans

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1307_4569_amd.serve import GpuExecutor
    plans = serving_plans()
    ex = GpuExecutor(lambda k: torch.tensor(gaussian_window(k[0], k[1], k[2])), streams=4, max_batch=8)
    ex.prepare(plans)
    rng = np.random.default_rng(99)
    keys = [plans[i] for i in rng.integers(0, len(plans), 96)] + plans
    sig = {}
    for i, k in enumerate(keys):
        sig[i] = torch.tensor(complex_normal(k[0], 7000 + i).astype(np.complex64), device="cuda")
    torch.cuda.synchronize()
    return ex, keys, sig


def test_results_same_alone_and_in_mix(setup):
    from paper_1307_4569_amd.serve import Request, Server, latency_stats
    ex, keys, sig = setup
    srv = Server(ex, hbm_budget=8 << 30, max_inflight_per_slot=2)
    reqs = srv.run([Request(i, k, sig[i], 0.0) for i, k in enumerate(keys)])
    torch.cuda.synchronize()
    assert all(r.error is None for r in reqs)
    assert max(r.batch_size for r in reqs) > 1
    for r in reqs:
        alone = ex.plan(r.key).forward(r.f)
        assert torch.equal(alone, r.c), r.key
    # a few against the oracle
    for r in reqs[:: len(reqs) // 6]:
        L, a, M, l1, l2 = r.key
        f = r.f.cpu().numpy().astype(np.complex128)
        g = gaussian_window(L, a, M).astype(np.complex64).astype(np.complex128)
        cols = list(range(0, L // a, L // a // 7))
        ref = oracle.dgt_fold(f, g, a, M, l1, l2, columns=cols)
        got = r.c[cols].cpu().numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print("serve", r.key, "batch", r.batch_size, "err", e)
        assert e < 1e-5
    print(latency_stats(reqs, lambda r: r.key[0] // r.key[1] * r.key[2]))


def test_admission_under_small_budget(setup):
    from paper_1307_4569_amd.serve import Request, Server
    ex, keys, sig = setup
    budget = 64 << 20
    srv = Server(ex, hbm_budget=budget, max_inflight_per_slot=4)
    reqs = srv.run([Request(i, k, sig[i], 0.0) for i, k in enumerate(keys)])
    torch.cuda.synchronize()
    assert all(r.error is None for r in reqs)
    assert 0 < srv.peak_bytes <= budget
    for r in reqs[::9]:
        assert torch.equal(ex.plan(r.key).forward(r.f), r.c)


def test_signals_produced_without_synchronising(setup):
    """Signals written by torch work still pending on the current stream are
    submitted without a synchronisation: each batch's stream waits for that
    work, so the results equal the transforms computed afterwards.  The
    coefficients handed out stay valid while the consumer's own work on them
    runs and other batches allocate."""
    from paper_1307_4569_amd.serve import Request, Server
    ex, keys, _ = setup
    sel = keys[:24]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4321)
    # a long queue of work on the current stream ahead of the signals
    x = torch.randn((2048, 2048), device="cuda", generator=gen)
    for _ in range(8):
        x = x @ x / 2048.0
    sigs = [torch.randn(k[0], dtype=torch.complex64, generator=gen, device="cuda") + x[0, 0] * 0 for k in sel]
    srv = Server(ex, hbm_budget=8 << 30, max_inflight_per_slot=2)
    reqs = srv.run([Request(i, k, sigs[i], 0.0) for i, k in enumerate(sel)])
    # consumer work on the handed-out coefficients, then more batches that allocate
    norms = [r.c.abs().sum() for r in reqs]
    srv2 = Server(ex, hbm_budget=8 << 30, max_inflight_per_slot=2)
    srv2.run([Request(100 + i, k, sigs[i], 0.0) for i, k in enumerate(sel)])
    torch.cuda.synchronize()
    for r, nrm in zip(reqs, norms):
        alone = ex.plan(r.key).forward(r.f)
        assert torch.equal(alone, r.c), r.key
        assert torch.equal(nrm, alone.abs().sum())
