"""GPU parity of the factorisation with columns longer than one in-LDS
transform (d = d1 d2, two-level column transforms; Sec. 4 full-window
algorithm): separable, time-shear and frequency-shear plans with p = 1 and
p = 3, against the FP64 oracle, and the frequency-shear lattice of Fig. 2's
first shape (L = 161280, a = 32, M = 64, lambda = 1/2, d = 20160).  The p = 3
lattices have p d = 5040: FP64 plans take the two-level path, FP32 plans the
in-LDS one with the window's FP64 Zak transform split into calls of at most
4096 values."""
import numpy as np
import pytest

import oracle
from dgt_inputs import complex_normal, complex_normal_batch, gaussian_window, round_to

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}

# (lattice, branch, p of the sheared lattice)
LONG_LATTICES = [((20160, 2, 4, 0, 1), 0, 1), ((20160, 3, 4, 0, 1), 0, 3), ((20160, 2, 4, 1, 2), 1, 1),
                 ((20160, 3, 4, 1, 2), 1, 3), ((20160, 3, 6, 1, 3), 2, 1), ((20160, 12, 16, 1, 4), 2, 3)]


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


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("case", LONG_LATTICES, ids=lambda c: "-".join(map(str, c[0])))
def test_long_columns_forward_and_adjoint(case, dtype):
    from paper_1307_4569_amd import Plan
    lat, branch, p = case
    L, a, M, l1, l2 = lat
    N = L // a
    single = dtype == torch.complex64
    plan = Plan(*lat, dtype=dtype, max_batch=2)
    assert plan.branch == branch and plan.info.p == p and (plan.info.d > 4096 or p * plan.info.d > 4096)
    f = round_to(np.stack([complex_normal(L, 700 + k) for k in range(2)]), single)
    g = round_to(gaussian_window(L, a, M) + 0.05j * complex_normal(L, 9), single)
    plan.set_window(torch.tensor(g))
    c = plan.forward(torch.tensor(f)).cpu().numpy()
    cols = list(range(0, N, 7)) + [N - 1]
    ef = max(rel(c[k][cols], oracle.dgt_fold(f[k], g, a, M, l1, l2, columns=cols)) for k in range(2))
    cin = round_to(complex_normal(N * M, 800).reshape(N, M), single)
    fa = plan.adjoint(torch.tensor(cin[None])).cpu().numpy()[0]
    ea = rel(fa, oracle.idgt_adjoint(cin, g, a, M, l1, l2))
    print("long columns", lat, dtype, "d", plan.info.d, "forward", ef, "adjoint", ea)
    assert ef < TOL[dtype] and ea < TOL[dtype]


def test_fig2_frequency_shear_lattice():
    """L = lcm(32, 64) 2520, lambda = 1/2: frequency shear with N_r = 8 inner
    channels and columns of d = 20160; FP32 batch of 16, sampled time
    positions against the oracle and whole-batch adjointness."""
    from paper_1307_4569_amd import Plan
    lat = (161280, 32, 64, 1, 2)
    L, a, M, l1, l2 = lat
    B = 16
    plan = Plan(*lat, dtype=torch.complex64, max_batch=B)
    assert plan.branch == 2 and plan.info.d == 20160
    f = round_to(complex_normal_batch(B, L, 6), True)
    g = round_to(gaussian_window(L, a, M), True)
    plan.set_window(torch.tensor(g))
    ft = torch.tensor(f).cuda()
    c = plan.forward(ft)
    cols = list(range(0, L // a, 113)) + [L // a - 1]
    errs = [rel(c[k, cols].cpu().numpy(), oracle.dgt_fold(f[k], g, a, M, l1, l2, columns=cols)) for k in (0, B - 1)]
    cp = torch.randn_like(c)
    fa = plan.adjoint(cp)
    lhs = torch.vdot(c.flatten().to(torch.complex128), cp.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(ft.flatten().to(torch.complex128), fa.flatten().to(torch.complex128)).item()
    print("fig2 lattice", errs, abs(lhs - rhs) / abs(lhs))
    assert max(errs) < 1e-5 and abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_long_columns_list_batch():
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bb
    lat = (20160, 3, 6, 1, 3)
    L, a, M, _, _ = lat
    B = 3
    plan = Plan(*lat, dtype=torch.complex64, max_batch=B)
    g = torch.tensor(gaussian_window(L, a, M))
    plan.set_window(g)
    f = torch.tensor(complex_normal_batch(B, L, 7).astype(np.complex64)).cuda()
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


# (lattice, branch, p, dtype): the long-column lattices of the forward tests
# in the precisions whose plans split the columns (FP32 plans hold p d = 5040
# in one transform)
GRAD_LONG = [((20160, 2, 4, 0, 1), 0, 1, torch.complex128), ((20160, 2, 4, 0, 1), 0, 1, torch.complex64),
             ((20160, 3, 4, 1, 2), 1, 3, torch.complex128), ((20160, 3, 6, 1, 3), 2, 1, torch.complex128),
             ((20160, 3, 6, 1, 3), 2, 1, torch.complex64), ((20160, 12, 16, 1, 4), 2, 3, torch.complex128)]


@pytest.mark.parametrize("case", GRAD_LONG, ids=lambda c: "-".join(map(str, c[0])) + "-" + str(c[3])[-3:])
def test_long_columns_window_gradient(case):
    """Window gradient with the column transforms in two passes, summed over
    a batch of 2, against the oracle's gradient (eq. (DGT) differentiated in
    the window)."""
    from paper_1307_4569_amd import Plan
    lat, branch, p, dtype = case
    L, a, M, l1, l2 = lat
    N = L // a
    single = dtype == torch.complex64
    B = 2
    plan = Plan(*lat, dtype=dtype, max_batch=B)
    assert plan.branch == branch and plan.info.p == p
    assert plan.info.d > 4096 or p * plan.info.d > (8192 if single else 4096)
    g = round_to(complex_normal(L, 31), single)
    f = round_to(np.stack([complex_normal(L, 32 + k) for k in range(B)]), single)
    G = round_to(np.stack([complex_normal(N * M, 34 + k).reshape(N, M) for k in range(B)]), single)
    plan.set_window(torch.tensor(g))
    gg = plan.window_grad(torch.tensor(f), torch.tensor(G)).cpu().numpy()
    ref = sum(oracle.window_gradient(f[k], G[k], a, M, l1, l2) for k in range(B))
    e = rel(gg, ref)
    print("long window gradient", lat, dtype, "d", plan.info.d, e)
    assert e < TOL[dtype]


# (lattice, plan dtype, branch, p): FP64 plans with p = 3 split p d = 5040 in
# two passes; Fig. 2's first shape has d = 20160 in both precisions
DUAL_LONG = [((20160, 3, 4, 1, 2), torch.complex128, 1, 3), ((20160, 12, 16, 1, 4), torch.complex128, 2, 3),
             ((20160, 3, 4, 0, 1), torch.complex128, 0, 3), ((161280, 32, 64, 1, 2), torch.complex64, 2, 1)]


@pytest.mark.parametrize("case", DUAL_LONG, ids=lambda c: "-".join(map(str, c[0])))
def test_long_columns_dual_and_tight(case):
    """Canonical dual and tight windows with the window Zak and its inverse
    in two passes (Alg. 2 on long columns): S g_d = g and S_gt = I at sampled
    points through the oracle's Walnut form, the frame bounds of both calls
    agree, and they bracket S's Rayleigh quotient on the dual window."""
    from paper_1307_4569_amd import Plan
    lat, dtype, branch, p = case
    L, a, M, l1, l2 = lat
    plan = Plan(*lat, dtype=dtype, max_batch=1)
    assert plan.branch == branch and plan.info.p == p and plan.info.d * p > 4096
    g = gaussian_window(L, a, M) + 0.05j * complex_normal(L, 12)
    gd, bd = plan.dual(torch.tensor(g))
    gt, bt = plan.tight(torch.tensor(g))
    gd, gt = gd.cpu().numpy(), gt.cpu().numpy()
    bd, bt = bd.cpu().numpy(), bt.cpu().numpy()
    assert 0 < bd[0] <= bd[1] and np.allclose(bd, bt, rtol=1e-12)
    pts = np.concatenate([np.linspace(0, L - 1, 3).astype(np.int64), [1, L // 2 + 3]])
    es = rel(oracle.frame_operator_apply(gd, g, a, M, l1, l2, pts), g[pts])
    x = complex_normal(L, 13)
    et = rel(oracle.frame_operator_apply(x, gt, a, M, l1, l2, pts), x[pts])
    print("long dual/tight", lat, "S g_d = g", es, "S_gt = I", et, "bounds", bd)
    assert es < 1e-11 and et < 1e-11


def test_long_dual_matches_the_one_pass_path():
    """The lattice L = 20160, a = 3, M = 4, lambda = 1/2 has p d = 5040: the
    FP64 plan takes the two-pass Zak, the FP32 plan the in-LDS one (both
    compute the window in FP64), so the two dual and tight windows and
    frame bounds agree to FP64 rounding."""
    from paper_1307_4569_amd import Plan
    lat = (20160, 3, 4, 1, 2)
    L, a, M, _, _ = lat
    g = torch.tensor(gaussian_window(L, a, M) + 0.05j * complex_normal(L, 14))
    p64 = Plan(*lat, dtype=torch.complex128, max_batch=1)
    p32 = Plan(*lat, dtype=torch.complex64, max_batch=1)
    for fn in ("dual", "tight"):
        w64, b64 = getattr(p64, fn)(g)
        w32, b32 = getattr(p32, fn)(g)
        e = rel(w64.cpu().numpy(), w32.cpu().numpy())
        print(fn, "two-pass against in-LDS", e)
        assert e < 1e-12 and np.allclose(b64.cpu().numpy(), b32.cpu().numpy(), rtol=1e-12)


def test_fig2_lattice_window_gradient():
    """Window gradient on Fig. 2's first shape (L = 161280, a = 32, M = 64,
    lambda = 1/2, columns of d = 20160 in two passes), FP32 batch of 4:
    sampled time positions against the oracle, summed over the batch."""
    from paper_1307_4569_amd import Plan
    lat = (161280, 32, 64, 1, 2)
    L, a, M, l1, l2 = lat
    N = L // a
    B = 4
    plan = Plan(*lat, dtype=torch.complex64, max_batch=B)
    assert plan.info.d == 20160
    g = round_to(gaussian_window(L, a, M), True)
    f = round_to(complex_normal_batch(B, L, 41), True)
    G = round_to(complex_normal_batch(B, N * M, 42).reshape(B, N, M), True)
    plan.set_window(torch.tensor(g))
    gg = plan.window_grad(torch.tensor(f), torch.tensor(G)).cpu().numpy()
    pts = np.concatenate([np.arange(0, L, 9973), [L - 1]])
    ref = sum(oracle.window_gradient(f[k], G[k], a, M, l1, l2, points=pts) for k in range(B))
    e = rel(gg[pts], ref)
    print("fig2 window gradient", e)
    assert e < 1e-5
