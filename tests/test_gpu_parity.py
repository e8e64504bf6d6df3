"""GPU parity of libdgtns against the FP64 oracle, element by element on the
same seeded inputs.  Bar: relative l2 error per signal <= 1e-12 (FP64) and
<= 1e-5 (FP32)."""
import math

import numpy as np
import pytest

import oracle
from dgt_inputs import (GRADIENT, LARGE, PRECISION, SMALL, chirp_mixture, complex_normal, complex_normal_batch,
                        gaussian_window, hann_window, round_to)
from tests.conftest import DEGENERATE_LATTICES, feasible_lattices

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}


@pytest.fixture(params=["fast", "generic"])
def kernel_path(request, monkeypatch):
    """Run a test with the wave-FFT kernels (power-of-two lengths) and with the
    runtime-schedule kernels forced by DGTNS_GENERIC=1."""
    if request.param == "generic":
        monkeypatch.setenv("DGTNS_GENERIC", "1")
    else:
        monkeypatch.delenv("DGTNS_GENERIC", raising=False)
    return request.param


def rel(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1307_4569_amd import _binding
    _binding.lib()   # fail loudly if the library is missing
    return torch.device("cuda", 0)


def make_plan(L, a, M, l1, l2, dtype, B=4):
    from paper_1307_4569_amd import Plan
    return Plan(L, a, M, l1, l2, dtype=dtype, max_batch=B)


def inputs(L, a, M, B, single, seed=0):
    f = np.stack([complex_normal(L, 1000 + seed + i) for i in range(B)])
    g = gaussian_window(L, a, M)
    return round_to(f, single), round_to(g, single)


def run_forward(lat, dtype, B=2, g=None, seed=0):
    L, a, M, l1, l2 = lat
    single = dtype == torch.complex64
    f, g0 = inputs(L, a, M, B, single, seed)
    g = g0 if g is None else round_to(g, single)
    plan = make_plan(L, a, M, l1, l2, dtype, B)
    plan.set_window(torch.tensor(g))
    c = plan.forward(torch.tensor(f)).cpu().numpy()
    return plan, f, g, c


# ---------------------------------------------------------------------------
# Small workload and random lattices
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_small_workload(dtype, kernel_path):
    lat = (SMALL.L, SMALL.a, SMALL.M, SMALL.lam1, SMALL.lam2)
    plan, f, g, c = run_forward(lat, dtype, B=1)
    assert c.shape == (1, 24, 12)
    ref = oracle.dgt_direct(f[0], g, *lat[1:])
    print("small workload", dtype, rel(c[0], ref))
    assert rel(c[0], ref) < TOL[dtype]


POW2_LATTICES = [(2048, 16, 64, 1, 2), (4096, 32, 128, 1, 2), (4096, 8, 64, 1, 4), (8192, 32, 256, 1, 2),
                 (16384, 64, 512, 3, 4), (32768, 64, 1024, 1, 2), (4096, 16, 32, 1, 2),
                 (12288, 16, 64, 1, 3), (6144, 32, 64, 2, 3), (65536, 64, 256, 0, 1), (1024, 8, 32, 1, 2),
                 (2048, 64, 64, 1, 2), (18432, 32, 256, 1, 2), (9216, 8, 64, 1, 2)]


def sample_lattices(p1_only):
    lats = [l for l in feasible_lattices(max_L=240, max_lam2=4) if l[0] >= 24]
    rng = np.random.default_rng(7)
    idx = rng.choice(len(lats), 400, replace=False)
    out = []
    from paper_1307_4569_amd import _binding as B
    for i in idx:
        L, a, M, l1, l2 = lats[i]
        try:
            h = B.dgtns_plan_create(L, a, M, l1, l2, 1, 2)
        except B.DgtnsError:
            continue
        info = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        if p1_only and info.p != 1:
            continue
        out.append((lats[i], info.branch, info.p))
    return out


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_random_lattices_forward_and_adjoint(dtype, kernel_path):
    lats = sample_lattices(False)
    seen = {"fs": 0, "ts": 0, "sep": 0, "p>1": 0}
    worst_f = worst_a = 0.0
    from paper_1307_4569_amd import _binding as Bb
    extra = []
    for lat in POW2_LATTICES:
        h = Bb.dgtns_plan_create(*lat, 1, 2)
        info = Bb.dgtns_plan_info(h)
        Bb.dgtns_plan_destroy(h)
        extra.append((lat, info.branch, info.p))
    for (lat, branch, p) in extra + lats[:120]:
        L, a, M, l1, l2 = lat
        plan, f, g, c = run_forward(lat, dtype, B=2, g=complex_normal(L, 77))
        for k in range(2):
            e = rel(c[k], oracle.dgt_fold(f[k], g, a, M, l1, l2))
            worst_f = max(worst_f, e)
            assert e < TOL[dtype], (lat, branch, p, e)
        cin = np.stack([complex_normal(L // a * M, 500 + k).reshape(L // a, M) for k in range(2)])
        cin = round_to(cin, dtype == torch.complex64)
        fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
        for k in range(2):
            e = rel(fa[k], oracle.idgt_adjoint(cin[k], g, a, M, l1, l2))
            worst_a = max(worst_a, e)
            assert e < TOL[dtype], ("adjoint", lat, branch, p, e)
        seen[["sep", "ts", "fs"][branch]] += 1
        seen["p>1"] += p > 1
    print("random lattices", kernel_path, dtype, seen, "worst forward", worst_f, "worst adjoint", worst_a)
    assert seen["fs"] >= 5 and seen["ts"] >= 20 and seen["p>1"] >= 5


def test_ragged_blocks_and_batch_sizes():
    """Column blocks that do not divide M, batch 1 and the maximal batch."""
    lat = (5 * 7 * 8, 5, 70, 0, 1)      # M = 70 channels: 70 = 4 * 16 + 6 columns
    dt = torch.complex128
    L, a, M, l1, l2 = lat
    plan = make_plan(L, a, M, l1, l2, dt, B=5)
    g = complex_normal(L, 3)
    plan.set_window(torch.tensor(g))
    f = np.stack([complex_normal(L, 10 + i) for i in range(5)])
    c5 = plan.forward(torch.tensor(f)).cpu().numpy()
    c1 = plan.forward(torch.tensor(f[3])).cpu().numpy()
    assert np.array_equal(c5[3], c1)           # batch position does not change the result
    for k in range(5):
        assert rel(c5[k], oracle.dgt_fold(f[k], g, a, M, l1, l2)) < 1e-12


# The largest in-LDS transforms: rows of M = 4096 channels, columns of
# d = 4096, and a frequency-shear plan with M = 8192 channels (its rows run on
# the N_r inner channels).
MAXIMA = [(65536, 64, 4096, 0, 1), (65536, 16, 16, 1, 2), (32768, 8, 8, 0, 1), (65536, 64, 4096, 1, 2),
          (131072, 64, 8192, 1, 2)]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("lat", MAXIMA)
def test_maximum_in_lds_sizes(lat, dtype):
    L, a, M, l1, l2 = lat
    plan, f, g, c = run_forward(lat, dtype, B=2, g=complex_normal(L, 78), seed=40)
    for k in range(2):
        e = rel(c[k], oracle.dgt_fold(f[k], g, a, M, l1, l2))
        assert e < TOL[dtype], (lat, k, e)
    cin = round_to(complex_normal(L // a * M, 541).reshape(1, L // a, M), dtype == torch.complex64)
    fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
    e = rel(fa[0], oracle.idgt_adjoint(cin[0], g, a, M, l1, l2))
    assert e < TOL[dtype], ("adjoint", lat, e)
    if plan.info.d == 4096:
        gg = plan.window_grad(torch.tensor(f), torch.tensor(round_to(
            np.stack([complex_normal(L // a * M, 542 + k).reshape(L // a, M) for k in range(2)]),
            dtype == torch.complex64))).cpu().numpy()
        Gs = round_to(np.stack([complex_normal(L // a * M, 542 + k).reshape(L // a, M) for k in range(2)]),
                      dtype == torch.complex64)
        ref = sum(oracle.window_gradient(f[k], Gs[k], a, M, l1, l2) for k in range(2))
        assert rel(gg, ref) < TOL[dtype], ("window gradient", lat, rel(gg, ref))
        gw = gaussian_window(L, a, M)
        gd, _ = plan.dual(torch.tensor(gw))
        pts = np.linspace(0, L - 1, 16).astype(np.int64)
        sg = oracle.frame_operator_apply(gd.cpu().numpy(), gw, a, M, l1, l2, pts)
        assert rel(sg, gw[pts]) < 1e-11, ("dual", lat, rel(sg, gw[pts]))


# p > 1 (p sub-columns per column) at the LDS element budget: p d = 4096 is
# the FP64 in-LDS limit, p d = 8192 the FP32 one; beyond it the columns take
# the two-level passes (d = d1 d2).
BLOCK_BUDGET = [(49152, 8, 12, 0, 1), (49152, 8, 12, 1, 2), (98304, 8, 12, 1, 2), (36864, 12, 8, 0, 1),
                (73728, 12, 8, 0, 1)]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("lat", BLOCK_BUDGET)
def test_block_columns_at_the_budget(lat, dtype):
    L, a, M, l1, l2 = lat
    plan, f, g, c = run_forward(lat, dtype, B=2, g=complex_normal(L, 79), seed=60)
    assert plan.info.p > 1
    N = L // a
    cols = sorted(set(range(0, N, N // 40)) | {N - 1})      # sampled time positions
    for k in range(2):
        e = rel(c[k][cols], oracle.dgt_fold(f[k], g, a, M, l1, l2, columns=cols))
        assert e < TOL[dtype], (lat, k, e)
    # adjoint: <C f, c'> = <f, C* c'> with the forward checked above
    cin = round_to(complex_normal(N * M, 561).reshape(1, N, M), dtype == torch.complex64)
    fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
    lhs = np.vdot(c[0].astype(np.complex128), cin[0].astype(np.complex128))
    rhs = np.vdot(f[0].astype(np.complex128), fa[0].astype(np.complex128))
    scale = np.linalg.norm(c[0]) * np.linalg.norm(cin[0])
    assert abs(lhs - rhs) < TOL[dtype] * scale, ("adjoint", lat, abs(lhs - rhs) / scale)
    # the dual window, in one in-LDS transform or in two passes
    gw = gaussian_window(L, a, M)
    gd, _ = plan.dual(torch.tensor(gw))
    pts = np.linspace(0, L - 1, 4).astype(np.int64)
    sg = oracle.frame_operator_apply(gd.cpu().numpy(), gw, a, M, l1, l2, pts)
    assert rel(sg, gw[pts]) < 1e-11, ("dual", lat, rel(sg, gw[pts]))
    # the window gradient of the two signals at sampled time positions
    G = round_to(complex_normal(2 * N * M, 562).reshape(2, N, M), dtype == torch.complex64)
    gg = plan.window_grad(torch.tensor(f), torch.tensor(G)).cpu().numpy()
    pts = np.array(sorted(set(range(0, L, L // 24)) | {L - 1}), dtype=np.int64)
    ref = sum(oracle.window_gradient(f[k], G[k], a, M, l1, l2, points=pts) for k in range(2))
    assert rel(gg[pts], ref) < TOL[dtype], ("window gradient", lat, rel(gg[pts], ref))


def test_real_input_matches_complex():
    lat = (240, 6, 12, 1, 2)
    L, a, M, l1, l2 = lat
    dt = torch.complex128
    plan = make_plan(*lat, dt, B=2)
    g = gaussian_window(L, a, M)
    plan.set_window(torch.tensor(g))
    x = np.stack([chirp_mixture(L, 5), chirp_mixture(L, 6)])
    cr = plan.forward(torch.tensor(x)).cpu().numpy()
    cc = plan.forward(torch.tensor(x.astype(np.complex128))).cpu().numpy()
    assert np.array_equal(cr, cc)
    assert rel(cr[1], oracle.dgt_fold(x[1], g, a, M, l1, l2)) < 1e-12


def test_errors_are_reported():
    from paper_1307_4569_amd import _binding as B
    plan = make_plan(144, 6, 12, 1, 2, torch.complex64, B=2)
    f = torch.zeros(2, 144, dtype=torch.complex64, device="cuda")
    with pytest.raises(B.DgtnsError) as e:
        plan.forward(f)                           # window not set
    assert e.value.status == B.DGTNS_ESTATE
    plan.set_window(torch.tensor(gaussian_window(144, 6, 12)))
    c = torch.empty(3, 24, 12, dtype=torch.complex64, device="cuda")
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_forward(plan._h, f.data_ptr(), 0, c.data_ptr(), 3, c.data_ptr(), 10 ** 9, 0)   # B > max_batch
    assert e.value.status == B.DGTNS_EINVAL
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_forward(plan._h, f.data_ptr(), 0, c.data_ptr(), 2, ws.data_ptr(), 16, 0)
    assert e.value.status == B.DGTNS_EWORKSPACE


# ---------------------------------------------------------------------------
# Full-size workloads: all signals transformed, sampled time positions
# compared with the oracle, plus invariants that hold at any size.
# ---------------------------------------------------------------------------

def full_size(w, dtype, B, columns, real=False, window=None):
    single = dtype == torch.complex64
    if real:
        f = np.stack([chirp_mixture(w.L, 13074569 + 3000 + i) for i in range(B)])
    else:
        f = complex_normal_batch(B, w.L, 2)
    f = round_to(f, single)
    g = round_to(gaussian_window(w.L, w.a, w.M) if window is None else window, single)
    plan = make_plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype, B)
    plan.set_window(torch.tensor(g))
    ft = torch.tensor(f).cuda()
    c = plan.forward(ft)
    torch.cuda.synchronize()
    errs = []
    for k in sorted({0, B - 1}):
        ref = oracle.dgt_fold(f[k], g, w.a, w.M, w.lam1, w.lam2, columns=columns)
        got = c[k, columns].cpu().numpy()
        errs.append(rel(got, ref))
    return plan, ft, c, errs


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_large_workload_sampled(dtype, kernel_path):
    w = LARGE
    B = w.batch
    cols = list(range(0, w.N, 97)) + [w.N - 1]
    plan, f, c, errs = full_size(w, dtype, B, cols)
    print("large workload", kernel_path, dtype, "B", B, "errors", errs)
    assert max(errs) < TOL[dtype]
    # every signal: Parseval-type invariant ||c||^2 = <S f, f> is not cheap; check
    # adjointness <C f, c'> = <f, C* c'> on the whole batch instead
    cp = torch.randn_like(c)
    fa = plan.adjoint(cp)
    lhs = torch.vdot(c.flatten().to(torch.complex128), cp.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(f.flatten().to(torch.complex128), fa.flatten().to(torch.complex128)).item()
    print("adjointness", abs(lhs - rhs) / abs(lhs))
    # measured 3e-7 to 6e-7 (FP32) and 1e-16 to 1e-15 (FP64)
    assert abs(lhs - rhs) <= TOL[dtype] * abs(lhs)


def test_precision_workload_real_signals(kernel_path):
    w = PRECISION
    cols = list(range(0, w.N, 331)) + [w.N - 1]
    for name, win in (("gaussian", None), ("hann", hann_window(w.L, 2048))):
        plan, f, c, errs = full_size(w, torch.complex64, w.batch, cols, real=True, window=win)
        print("precision workload", kernel_path, name, errs)
        assert max(errs) < 1e-5


def test_gradient_workload_sampled(kernel_path):
    w = GRADIENT
    cols = list(range(0, w.N, 53))
    plan, f, c, errs = full_size(w, torch.complex64, w.batch, cols)
    print("gradient workload forward", errs)
    assert max(errs) < 1e-5


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_pipelined_batches_match_single_launch(dtype, monkeypatch):
    """The optional two-stream chunk pipeline (DGTNS_CHUNK_MIB; ragged last
    chunk) gives the same coefficients and adjoints, bit for bit, as one
    launch per stage, with a smaller workspace."""
    w = LARGE
    B = 11
    f = torch.tensor(complex_normal_batch(B, w.L, 2).astype(np.complex64)).to(dtype).cuda()
    g = torch.tensor(gaussian_window(w.L, w.a, w.M))
    out = {}
    for mode in ("pipeline", "single"):
        if mode == "single":
            monkeypatch.delenv("DGTNS_CHUNK_MIB", raising=False)
            monkeypatch.setenv("DGTNS_SEQ_MIB", "0")    # one launch per stage
        else:
            monkeypatch.setenv("DGTNS_CHUNK_MIB", "64")
        plan = make_plan(w.L, w.a, w.M, w.lam1, w.lam2, dtype, B)
        plan.set_window(g)
        c = plan.forward(f)
        fa = plan.adjoint(c)
        torch.cuda.synchronize()
        from paper_1307_4569_amd import _binding as Bm
        out[mode] = (c, fa, Bm.dgtns_workspace_bytes(plan._h, Bm.DGTNS_OP_FORWARD, B))
    # the pipeline needs two chunks of the intermediate instead of the whole batch
    assert out["pipeline"][2] < out["single"][2]
    assert torch.equal(out["pipeline"][0], out["single"][0])
    assert torch.equal(out["pipeline"][1], out["single"][1])
    ref = oracle.dgt_fold(f[B - 1].cpu().numpy().astype(np.complex128),
                          g.numpy().astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else g.numpy(),
                          w.a, w.M, w.lam1, w.lam2, columns=[0, 1000, 4095])
    assert rel(out["pipeline"][0][B - 1, [0, 1000, 4095]].cpu().numpy(), ref) < TOL[dtype]


# Column lengths d = 9 2^k (72 to 1152) of the serving plans: the one-wavefront
# runtime-schedule factorisation (FP64 at d = 1152 keeps its twiddle table in
# global memory, as the LDS tile then fills the work-group's 160 KiB).
SERVING_D = [(36864, 64, 512, 1, 3), (73728, 64, 512, 2, 3), (147456, 64, 512, 1, 3), (294912, 64, 512, 2, 3),
             (294912, 32, 256, 1, 3), (294912, 32, 256, 1, 2)]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_serving_column_lengths_sampled(dtype, kernel_path):
    single = dtype == torch.complex64
    B = 2
    for lat in SERVING_D:
        L, a, M, l1, l2 = lat
        plan = make_plan(*lat, dtype, B)
        f, g = inputs(L, a, M, B, single, seed=7)
        plan.set_window(torch.tensor(g))
        c = plan.forward(torch.tensor(f)).cpu().numpy()
        N = L // a
        cols = list(range(0, N, max(1, N // 24))) + [N - 1]
        e = max(rel(c[k, cols], oracle.dgt_fold(f[k], g, a, M, l1, l2, columns=cols)) for k in range(B))
        print("serving d", kernel_path, dtype, lat, plan.info.branch, plan.info.d, e)
        assert e < TOL[dtype], (lat, e)


# Real input (4 bytes per FP32 sample) on every route that reads the signal:
# the factorisation loads of each column kernel, the length-L transform of
# the frequency shear, the two-level column passes, the multiwindow, FIR and
# shear-OLA algorithms.  The result must equal that of the same samples
# passed as complex numbers with zero imaginary part, bit for bit.
REAL_ROUTES = [((262144, 64, 512, 1, 2), {}),                      # time shear, wave columns d = 512
               ((73728, 64, 512, 1, 3), {}),                       # time shear, d = 144 (one wavefront per column)
               ((36864, 32, 256, 1, 2), {}),                       # frequency shear, d = 576
               ((20160, 3, 6, 1, 3), {}),                          # frequency shear, two-level columns
               ((1 << 20, 32, 64, 1, 2), {}),                      # time shear, two-level columns
               ((65536, 32, 32, 1, 2), {"algorithm": "multiwindow"}),
               ((8192, 32, 256, 1, 2), {"algorithm": "fir", "support": (8000, 200)}),
               ((65536, 64, 1024, 1, 2), {"algorithm": "fir", "support": (65000, 2048)}),
               ((6144, 16, 64, 1, 2), {"algorithm": "shear-ola", "support": (6000, 300), "block": 1024})]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("lat,kw", REAL_ROUTES)
def test_real_input_on_every_route(lat, kw, dtype, kernel_path):
    from paper_1307_4569_amd import Plan
    L, a, M, l1, l2 = lat
    single = dtype == torch.complex64
    x = np.stack([chirp_mixture(L, 71 + k) for k in range(2)]).real
    x = x.astype(np.float32 if single else np.float64)
    plan = Plan(*lat, dtype=dtype, max_batch=2, **kw)
    plan.set_window(torch.tensor(round_to(gaussian_window(L, a, M), single)))
    cr = plan.forward(torch.tensor(x)).cpu().numpy()
    cc = plan.forward(torch.tensor(x.astype(np.complex64 if single else np.complex128))).cpu().numpy()
    assert np.array_equal(cr, cc), (lat, kw, float(np.abs(cr - cc).max()))


@pytest.mark.parametrize("lat,kw", REAL_ROUTES)
def test_list_batch_on_every_route(lat, kw, kernel_path):
    """dgtns_forward_batch (signals and outputs at separate addresses, up to
    16 per launch) gives the batched forward's coefficients bit for bit on
    every route; shear-OLA plans refuse it."""
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bb
    L, a, M, l1, l2 = lat
    B = 3
    plan = Plan(*lat, dtype=torch.complex64, max_batch=B, **kw)
    plan.set_window(torch.tensor(round_to(gaussian_window(L, a, M), True)))
    fs = [torch.tensor(complex_normal(L, 90 + k).astype(np.complex64)).cuda() for k in range(B)]
    c = plan.forward(torch.stack(fs))
    outs = [torch.empty_like(c[0]) for _ in range(B)]
    wsb = Bb.dgtns_workspace_bytes(plan._h, Bb.DGTNS_OP_FORWARD, B)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    call = lambda: Bb.dgtns_forward_batch(plan._h, [x.data_ptr() for x in fs], 0,   # noqa: E731
                                          [o.data_ptr() for o in outs], ws.data_ptr(), wsb, st)
    if kw.get("algorithm") == "shear-ola":
        with pytest.raises(Bb.DgtnsError) as e:
            call()
        assert e.value.status == Bb.DGTNS_EUNSUPPORTED
        return
    call()
    torch.cuda.synchronize()
    for k in range(B):
        assert torch.equal(outs[k], c[k]), (lat, kw, k)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_degenerate_lattices(dtype, kernel_path):
    """a = L (one time position), M = 1, a = 1, M = L, p = 48 with columns of
    one value, and L = 1: forward and adjoint against the oracle."""
    for lat in DEGENERATE_LATTICES:
        L, a, M, l1, l2 = lat
        plan, f, g, c = run_forward(lat, dtype, B=2, g=complex_normal(L, 81), seed=80)
        for k in range(2):
            e = rel(c[k], oracle.dgt_fold(f[k], g, a, M, l1, l2))
            assert e < TOL[dtype], (lat, k, e)
        cin = round_to(complex_normal(L // a * M, 591).reshape(1, L // a, M), dtype == torch.complex64)
        fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
        e = rel(fa[0], oracle.idgt_adjoint(cin[0], g, a, M, l1, l2))
        assert e < TOL[dtype], ("adjoint", lat, e)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_degenerate_lattices_other_algorithms(dtype, kernel_path):
    """The multiwindow and FIR algorithms on the degenerate lattices (the FIR
    window on the first half of the samples, wrapping from L - 1 for L = 1):
    forward and adjoint against the oracle on the same (truncated) window."""
    from paper_1307_4569_amd import Plan
    single = dtype == torch.complex64
    for lat in DEGENERATE_LATTICES:
        L, a, M, l1, l2 = lat
        N = L // a
        f = round_to(np.stack([complex_normal(L, 600 + k) for k in range(2)]), single)
        g = round_to(complex_normal(L, 610), single)
        support = (L - 1, max(1, L // 2))
        gt = np.zeros_like(g)
        idx = (support[0] + np.arange(support[1])) % L
        gt[idx] = g[idx]
        for kw, gw in (({"algorithm": "multiwindow"}, g), ({"algorithm": "fir", "support": support}, gt)):
            plan = Plan(*lat, dtype=dtype, max_batch=2, **kw)
            plan.set_window(torch.tensor(g))
            c = plan.forward(torch.tensor(f)).cpu().numpy()
            for k in range(2):
                e = rel(c[k], oracle.dgt_fold(f[k], gw, a, M, l1, l2))
                assert e < TOL[dtype], (lat, kw, k, e)
            cin = round_to(complex_normal(N * M, 620).reshape(1, N, M), single)
            fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
            e = rel(fa[0], oracle.idgt_adjoint(cin[0], gw, a, M, l1, l2))
            assert e < TOL[dtype], ("adjoint", lat, kw, e)


def test_degenerate_lattices_dual_and_tight():
    """Dual and tight windows on the degenerate lattices: the oracle's windows
    and frame bounds where the Gaussian gives a frame, and a lower bound of
    zero (not a frame) for the undercomplete ones, among them a = L, M = 1
    with p = 48 (one wavefront per frame-operator block)."""
    from paper_1307_4569_amd import Plan
    seen_p = set()
    for lat in DEGENERATE_LATTICES:
        L, a, M, l1, l2 = lat
        g = gaussian_window(L, a, M)
        plan = Plan(*lat, dtype=torch.complex128, max_batch=1)
        seen_p.add(plan.info.p)
        lo, hi = oracle.frame_bounds(g, a, M, l1, l2)
        gd, bounds = plan.dual(torch.tensor(g))
        gt, _ = plan.tight(torch.tensor(g))
        A, B = bounds.cpu().numpy()
        assert abs(B - hi) < 1e-10 * hi, (lat, B, hi)
        if lo < 1e-9 * hi:                     # a = L or M = 1 with fewer atoms than samples
            assert A < 1e-9 * hi, (lat, A)
            continue
        assert abs(A - lo) < 1e-10 * hi, (lat, A, lo)
        assert rel(gd.cpu().numpy(), oracle.dual_window(g, a, M, l1, l2)) < 1e-12, lat
        assert rel(gt.cpu().numpy(), oracle.tight_window(g, a, M, l1, l2)) < 1e-12, lat
    assert max(seen_p) > 8
