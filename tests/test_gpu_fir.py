"""GPU parity of the FIR-window algorithm (Sec. 4, weighted overlap-add;
Table 1's multiwindow FIR row): coefficients and adjoint of eq. (DGT) for a
window truncated to its support, against the FP64 oracle applied to the
truncated window, on sampled feasible lattices with random supports (wrapping
ones, the full length, fewer samples than a), both kernel paths, and on the
precision workload's Hann window of length 2048 at L = 2^20, lambda = 1/4."""
import numpy as np
import pytest

import oracle
from dgt_inputs import PRECISION, chirp_mixture, complex_normal, complex_normal_batch, hann_window, round_to
from tests.conftest import feasible_lattices

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1307_4569_amd import _binding
    _binding.lib()
    return torch.device("cuda", 0)


@pytest.fixture(params=["fast", "generic"])
def kernel_path(request, monkeypatch):
    if request.param == "generic":
        monkeypatch.setenv("DGTNS_GENERIC", "1")
    else:
        monkeypatch.delenv("DGTNS_GENERIC", raising=False)
    return request.param


def rel(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


def truncate(g, start, length):
    L = g.shape[-1]
    out = np.zeros_like(g)
    idx = (start + np.arange(length)) % L
    out[idx] = g[idx]
    return out


def fir_plan(lat, support, dtype, B):
    from paper_1307_4569_amd import Plan
    return Plan(*lat, dtype=dtype, max_batch=B, algorithm="fir", support=support)


POW2 = [(4096, 32, 128, 1, 2), (8192, 32, 256, 1, 2), (16384, 64, 512, 3, 4), (32768, 64, 1024, 1, 2),
        (2048, 16, 64, 1, 2), (4096, 8, 32, 1, 4)]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_fir_lattices_forward_and_adjoint(dtype, kernel_path):
    rng = np.random.default_rng(21)
    lats = [l for l in feasible_lattices(max_L=240, max_lam2=4) if l[0] >= 24 and l[2] >= 2]
    picks = [lats[i] for i in rng.choice(len(lats), 60, replace=False)] + POW2
    single = dtype == torch.complex64
    worst = [0.0, 0.0]
    for n, lat in enumerate(picks):
        L, a, M, l1, l2 = lat
        N = L // a
        kind = n % 4
        length = [L, max(1, a // 2), int(rng.integers(1, L)), min(L, 2 * M + 3)][kind]
        start = int(rng.integers(0, L))
        f = round_to(np.stack([complex_normal(L, 900 + n + k) for k in range(2)]), single)
        g = round_to(complex_normal(L, 950 + n), single)
        from paper_1307_4569_amd import _binding as Bb
        try:
            plan = fir_plan(lat, (start, length), dtype, 2)
        except Bb.DgtnsError as e:      # M not 7-smooth
            assert e.status == Bb.DGTNS_EUNSUPPORTED
            continue
        assert plan.branch == 4
        plan.set_window(torch.tensor(g))
        gt = truncate(g, start, length)
        c = plan.forward(torch.tensor(f)).cpu().numpy()
        ef = max(rel(c[k], oracle.dgt_fold(f[k], gt, a, M, l1, l2)) for k in range(2))
        cin = round_to(complex_normal(N * M, 990 + n).reshape(N, M), single)
        fa = plan.adjoint(torch.tensor(cin[None])).cpu().numpy()[0]
        ea = rel(fa, oracle.idgt_adjoint(cin, gt, a, M, l1, l2))
        worst = [max(worst[0], ef), max(worst[1], ea)]
        assert ef < TOL[dtype] and ea < TOL[dtype], (lat, start, length, ef, ea)
    print("FIR lattices", kernel_path, dtype, len(picks), "worst forward/adjoint", worst)


def test_fir_precision_workload():
    """Hann window of length 2048 centred at 0 (support start L - 1024),
    L = 2^20, a = 128, M = 1024, lambda = 1/4, 16 real chirp signals in FP32:
    sampled time positions against the oracle, and the shear plan with the
    same (full-length, zero-padded) window gives the same coefficients."""
    from paper_1307_4569_amd import Plan
    w = PRECISION
    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    g = round_to(hann_window(w.L, 2048), True)
    x = round_to(np.stack([chirp_mixture(w.L, 13074569 + 3000 + k) for k in range(w.batch)]), True).real
    plan = fir_plan(lat, (w.L - 1024, 2048), torch.complex64, w.batch)
    plan.set_window(torch.tensor(g))
    xt = torch.tensor(x.astype(np.complex64)).cuda()
    c = plan.forward(xt)
    cols = list(range(0, w.N, 331)) + [w.N - 1]
    errs = [rel(c[k, cols].cpu().numpy(), oracle.dgt_fold(x[k].astype(complex), g, w.a, w.M, w.lam1, w.lam2,
                                                          columns=cols)) for k in (0, w.batch - 1)]
    sh = Plan(*lat, dtype=torch.complex64, max_batch=w.batch)
    sh.set_window(torch.tensor(g))
    cs = sh.forward(xt)
    d = (torch.linalg.vector_norm(c - cs) / torch.linalg.vector_norm(cs)).item()
    cp = torch.randn_like(c)
    fa = plan.adjoint(cp)
    lhs = torch.vdot(c.flatten().to(torch.complex128), cp.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(xt.flatten().to(torch.complex128), fa.flatten().to(torch.complex128)).item()
    print("FIR precision workload", errs, "vs shear", d, "adjointness", abs(lhs - rhs) / abs(lhs))
    assert max(errs) < 1e-5 and d < 2e-5 and abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_fir_list_batch_and_refusals():
    from paper_1307_4569_amd import _binding as Bb
    lat = (8192, 32, 256, 1, 2)
    L, a, M, _, _ = lat
    B = 4
    plan = fir_plan(lat, (L - 300, 600), torch.complex64, B)
    g = torch.tensor(complex_normal(L, 3))
    plan.set_window(g)
    f = torch.tensor(complex_normal_batch(B, L, 7).astype(np.complex64)).cuda()
    c = plan.forward(f)
    out = torch.empty_like(c)
    wsb = Bb.dgtns_workspace_bytes(plan._h, Bb.DGTNS_OP_FORWARD, B)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    stride = plan.N * M * 8
    Bb.dgtns_forward_batch(plan._h, [f[k].data_ptr() for k in range(B)], 0,
                           [out.data_ptr() + k * stride for k in range(B)], ws.data_ptr(), wsb,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(out, c)
    for fn in (lambda: plan.dual(g), lambda: plan.tight(g), lambda: plan.window_grad(f, c)):
        with pytest.raises(Bb.DgtnsError) as e:
            fn()
        assert e.value.status == Bb.DGTNS_EUNSUPPORTED


# Power-of-two M: the forward stages the work-group's signal span and the
# window in LDS when they fit (one, two, up to four or any number of samples
# per folded bin), else every wave reads them from global memory.
FORMS = [((8192, 32, 256, 1, 2), (8000, 200), False),     # span form, 1 sample per bin, wrapping
         ((8192, 32, 256, 1, 2), (5, 511), False),        # span form, 2 samples per bin
         ((8192, 32, 256, 3, 4), (8100, 1000), True),     # span form, 4 samples per bin, lambda = 3/4
         ((4096, 16, 64, 1, 2), (0, 2048), False),        # span form, 32 samples per bin
         ((8192, 32, 256, 1, 2), (100, 8000), True),      # global form: span beyond the LDS budget
         ((16384, 64, 1024, 1, 4), (16000, 3000), True)]  # M = 1024, span form


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("lat,support,real", FORMS)
def test_fir_forward_forms(lat, support, real, dtype):
    L, a, M, l1, l2 = lat
    single = dtype == torch.complex64
    B = 3
    f = round_to(complex_normal_batch(B, L, 31), single)
    if real:
        f = f.real.copy()
    g = round_to(complex_normal(L, 32), single)
    plan = fir_plan(lat, support, dtype, B)
    plan.set_window(torch.tensor(g))
    c = plan.forward(torch.tensor(f)).cpu().numpy()
    gt = truncate(g, *support)
    err = max(rel(c[k], oracle.dgt_fold(f[k].astype(complex), gt, a, M, l1, l2)) for k in range(B))
    assert err < TOL[dtype], (lat, support, err)


# M = 4096 (the longest in-LDS channel DFT) and FP64 with M = 1024, both on
# the work-group transform form of the FIR kernels.
FIR_WIDE = [((65536, 64, 4096, 1, 2), (63536, 4000)), ((65536, 64, 1024, 1, 2), (65000, 2048))]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("lat,support", FIR_WIDE)
def test_fir_wide_channel_counts(lat, support, dtype):
    L, a, M, l1, l2 = lat
    N = L // a
    single = dtype == torch.complex64
    f = round_to(complex_normal_batch(2, L, 33), single)
    g = round_to(complex_normal(L, 34), single)
    plan = fir_plan(lat, support, dtype, 2)
    plan.set_window(torch.tensor(g))
    gt = truncate(g, *support)
    c = plan.forward(torch.tensor(f)).cpu().numpy()
    ef = max(rel(c[k], oracle.dgt_fold(f[k], gt, a, M, l1, l2)) for k in range(2))
    cin = round_to(complex_normal(N * M, 35).reshape(1, N, M), single)
    fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
    ea = rel(fa[0], oracle.idgt_adjoint(cin[0], gt, a, M, l1, l2))
    assert ef < TOL[dtype] and ea < TOL[dtype], (lat, ef, ea)


def test_fir_start_is_taken_mod_L():
    """The support start is reduced modulo L: starts -24, L - 24 and 2 L - 24
    give the same coefficients, bit for bit, and match the oracle."""
    lat = (4096, 32, 128, 1, 2)
    L, a, M, l1, l2 = lat
    f = round_to(complex_normal_batch(2, L, 36), True)
    g = round_to(complex_normal(L, 37), True)
    out = []
    for start in (-24, L - 24, 2 * L - 24):
        plan = fir_plan(lat, (start, 48), torch.complex64, 2)
        plan.set_window(torch.tensor(g))
        out.append(plan.forward(torch.tensor(f)).cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[1], out[2])
    gt = truncate(g, L - 24, 48)
    assert rel(out[0][1], oracle.dgt_fold(f[1], gt, a, M, l1, l2)) < 1e-5
