"""GPU parity of the multiwindow algorithm (Section 3.1, Prop. 4, Prop. 5):
plans created with algorithm "multiwindow" must give the coefficients of
eq. (DGT) and their adjoint, checked against the FP64 oracle on sampled
feasible lattices (both kernel paths, p = 1 and p > 1 of the lattice
(lambda2 a, M)) and on sampled time positions of the full-size quincunx
workload."""
import numpy as np
import pytest

import oracle
from dgt_inputs import LARGE, complex_normal, complex_normal_batch, gaussian_window, round_to
from tests.conftest import feasible_lattices

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}


@pytest.fixture(params=["fast", "generic"])
def kernel_path(request, monkeypatch):
    if request.param == "generic":
        monkeypatch.setenv("DGTNS_GENERIC", "1")
    else:
        monkeypatch.delenv("DGTNS_GENERIC", raising=False)
    return request.param


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1307_4569_amd import _binding
    _binding.lib()
    return torch.device("cuda", 0)


def rel(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


def mw_plan(lat, dtype, B):
    from paper_1307_4569_amd import Plan
    return Plan(*lat, dtype=dtype, max_batch=B, algorithm="multiwindow")


def mw_info(lat):
    from paper_1307_4569_amd import _binding as Bb
    try:
        h = Bb.dgtns_plan_create_alg(*lat, 1, 2, Bb.DGTNS_ALG_MULTIWINDOW)
    except Bb.DgtnsError:
        return None
    info = Bb.dgtns_plan_info(h)
    Bb.dgtns_plan_destroy(h)
    return info


# power-of-two lattices (wave kernels for p = 1 of the lattice (lambda2 a, M))
MW_POW2 = [(2048, 16, 64, 1, 2), (4096, 8, 64, 1, 4), (4096, 32, 128, 1, 2), (8192, 32, 256, 1, 2),
           (16384, 64, 512, 3, 4), (65536, 64, 256, 0, 1), (12288, 16, 64, 1, 3), (6144, 32, 64, 2, 3),
           (18432, 32, 256, 1, 2), (9216, 8, 64, 1, 2)]


def check_lattice(lat, dtype, seed):
    L, a, M, l1, l2 = lat
    single = dtype == torch.complex64
    f = round_to(np.stack([complex_normal(L, seed + k) for k in range(2)]), single)
    g = round_to(complex_normal(L, seed + 7), single)
    plan = mw_plan(lat, dtype, 2)
    plan.set_window(torch.tensor(g))
    c = plan.forward(torch.tensor(f)).cpu().numpy()
    ef = max(rel(c[k], oracle.dgt_fold(f[k], g, a, M, l1, l2)) for k in range(2))
    cin = round_to(np.stack([complex_normal(L // a * M, seed + 20 + k).reshape(L // a, M) for k in range(2)]),
                   single)
    fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
    ea = max(rel(fa[k], oracle.idgt_adjoint(cin[k], g, a, M, l1, l2)) for k in range(2))
    return ef, ea


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_multiwindow_random_lattices(dtype, kernel_path):
    lats = [l for l in feasible_lattices(max_L=240, max_lam2=4) if l[0] >= 24 and l[4] > 1]
    rng = np.random.default_rng(11)
    seen = {"lam2=2": 0, "lam2=3": 0, "lam2=4": 0, "p>1": 0, "pow2": 0}
    worst = [0.0, 0.0]
    picks = [lats[i] for i in rng.choice(len(lats), 150, replace=False)]
    n = 0
    for lat in MW_POW2 + picks:
        info = mw_info(lat)
        if info is None:
            continue
        ef, ea = check_lattice(lat, dtype, 300 + n)
        n += 1
        worst = [max(worst[0], ef), max(worst[1], ea)]
        assert ef < TOL[dtype] and ea < TOL[dtype], (lat, info.p, info.windows, ef, ea)
        assert info.branch == 3 and info.windows == lat[4]
        if lat[4] > 1:
            seen[f"lam2={lat[4]}"] += 1
        seen["p>1"] += info.p > 1
        seen["pow2"] += lat in MW_POW2
    print("multiwindow lattices", kernel_path, dtype, n, seen, "worst forward/adjoint", worst)
    assert n >= 80 and min(seen.values()) >= 5


def test_multiwindow_equals_paper_route_and_shear():
    """Same coefficients as the oracle's multiwindow route (Prop. 5, written
    with separable DGTs of the coset windows) and as the shear plan."""
    from paper_1307_4569_amd import Plan
    lat = (4320, 24, 40, 2, 3)     # multiwindow lattice (72, 40): p = 9; shear plan: time shear, p = 3
    L, a, M, l1, l2 = lat
    f = complex_normal(L, 5)
    g = gaussian_window(L, a, M)
    mw = mw_plan(lat, torch.complex128, 1)
    sh = Plan(*lat, dtype=torch.complex128, max_batch=1)
    for p in (mw, sh):
        p.set_window(torch.tensor(g))
    cm = mw.forward(torch.tensor(f)).cpu().numpy()
    cs = sh.forward(torch.tensor(f)).cpu().numpy()
    ref = oracle.dgt_multiwindow(f, g, a, M, l1, l2)
    print("multiwindow vs paper route", rel(cm, ref), "vs shear plan", rel(cm, cs), mw.info.p)
    assert mw.info.p == 9 and rel(cm, ref) < 1e-12 and rel(cs, ref) < 1e-12


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_multiwindow_large_workload_sampled(dtype, kernel_path):
    w = LARGE
    B = w.batch if dtype == torch.complex64 else 8
    single = dtype == torch.complex64
    f = round_to(complex_normal_batch(B, w.L, 2), single)
    g = round_to(gaussian_window(w.L, w.a, w.M), single)
    plan = mw_plan((w.L, w.a, w.M, w.lam1, w.lam2), dtype, B)
    assert plan.info.p == 1 and plan.info.windows == 2 and plan.info.inner_a == 2 * w.a
    plan.set_window(torch.tensor(g))
    ft = torch.tensor(f).cuda()
    c = plan.forward(ft)
    cols = list(range(0, w.N, 89)) + [w.N - 1]
    errs = [rel(c[k, cols].cpu().numpy(), oracle.dgt_fold(f[k], g, w.a, w.M, w.lam1, w.lam2, columns=cols))
            for k in sorted({0, B - 1})]
    print("multiwindow large workload", kernel_path, dtype, errs)
    assert max(errs) < TOL[dtype]
    cp = torch.randn_like(c)
    fa = plan.adjoint(cp)
    lhs = torch.vdot(c.flatten().to(torch.complex128), cp.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(ft.flatten().to(torch.complex128), fa.flatten().to(torch.complex128)).item()
    assert abs(lhs - rhs) <= (1e-4 if single else 1e-11) * abs(lhs)


def test_multiwindow_list_batch_pipeline_and_window_grad(monkeypatch):
    """List-batched forward and the optional chunk pipeline give the same
    coefficients as one launch; the window gradient is refused."""
    from paper_1307_4569_amd import _binding as Bb
    lat = (8192, 32, 256, 1, 2)
    L, a, M, l1, l2 = lat
    B = 5
    f = torch.tensor(complex_normal_batch(B, L, 3).astype(np.complex64)).cuda()
    g = torch.tensor(gaussian_window(L, a, M))
    plan = mw_plan(lat, torch.complex64, B)
    plan.set_window(g)
    c = plan.forward(f)
    out = torch.empty_like(c)
    wsb = Bb.dgtns_workspace_bytes(plan._h, Bb.DGTNS_OP_FORWARD, B)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    stride = plan.N * M * 8
    Bb.dgtns_forward_batch(plan._h, [f[k].data_ptr() for k in range(B)], 0,
                           [out.data_ptr() + k * stride for k in range(B)], ws.data_ptr(), wsb,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(out, c)
    monkeypatch.setenv("DGTNS_CHUNK_MIB", "1")   # chunks of 2 signals
    pp = mw_plan(lat, torch.complex64, B)
    pp.set_window(g)
    cpipe = pp.forward(f)
    assert torch.equal(cpipe, c)
    ref = oracle.dgt_fold(f[B - 1].cpu().numpy(), g.numpy().astype(np.complex64), a, M, l1, l2)
    assert rel(c[B - 1].cpu().numpy(), ref) < 1e-5
    with pytest.raises(Bb.DgtnsError) as e:
        plan.window_grad(f, c)
    assert e.value.status == Bb.DGTNS_EUNSUPPORTED


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_multiwindow_largest_columns(dtype):
    """p_mw d_mw = 4096 on the (lambda2 a, M) lattice: the FP64 in-LDS limit
    of the multiwindow factorisation, forward and adjoint against the oracle."""
    lat = (32768, 8, 8, 1, 2)
    i = mw_info(lat)
    assert i.p * i.d == 4096
    ef, ea = check_lattice(lat, dtype, 870)
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert ef < tol and ea < tol, (ef, ea)


def test_automatic_plans_on_serving_lattices():
    """DGTNS_ALG_AUTO on the serving lattices whose shear needs a frequency
    shear gives multiwindow plans: FP32 forward of two signals on sampled
    time positions and the adjoint at sampled samples against the oracle."""
    from dgt_inputs import complex_normal, gaussian_window, round_to, serving_plans
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bb
    seen = 0
    for lat in serving_plans():
        L, a, M, l1, l2 = lat
        plan = Plan(*lat, dtype=torch.complex64, max_batch=2, algorithm="auto")
        if plan.info.branch != Bb.DGTNS_MULTIWINDOW:
            assert plan.info.branch != Bb.DGTNS_FREQ_SHEAR
            continue
        seen += 1
        N = L // a
        g = round_to(gaussian_window(L, a, M), True)
        f = round_to(np.stack([complex_normal(L, 300 + k) for k in range(2)]), True)
        plan.set_window(torch.tensor(g))
        c = plan.forward(torch.tensor(f).cuda())
        cols = sorted({0, 1, N // 3, N // 2, N - 1})
        ef = max(rel(c[k, cols].cpu().numpy(), oracle.dgt_fold(f[k], g, a, M, l1, l2, columns=cols)) for k in range(2))
        cin = round_to(complex_normal(N * M, 310).reshape(N, M), True)
        fa = plan.adjoint(torch.tensor(cin[None]).cuda())
        pts = np.linspace(0, L - 1, 64).astype(np.int64)
        ea = rel(fa[0, torch.tensor(pts, device="cuda")].cpu().numpy(),
                 oracle.idgt_adjoint(cin, g, a, M, l1, l2, samples=pts))
        print("auto plan", lat, "p", plan.info.p, "d", plan.info.d, "forward", ef, "adjoint", ea)
        assert ef < 1e-5 and ea < 1e-5
    assert seen == 6
