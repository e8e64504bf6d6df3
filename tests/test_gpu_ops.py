"""GPU checks of the operations beside the forward transform: window
gradient, canonical dual window (FP64) and the autograd function, against
the FP64 oracle, finite differences and reconstruction."""
import numpy as np
import pytest

import oracle
from dgt_inputs import (GRADIENT, PRECISION, chirp_mixture, complex_normal, complex_normal_batch, gaussian_window,
                        hann_window, round_to)

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


@pytest.fixture(params=["fast", "generic"])
def kernel_path(request, monkeypatch):
    if request.param == "generic":
        monkeypatch.setenv("DGTNS_GENERIC", "1")
    else:
        monkeypatch.delenv("DGTNS_GENERIC", raising=False)
    return request.param


def plan_for(lat, dtype, B):
    from paper_1307_4569_amd import Plan
    return Plan(*lat, dtype=dtype, max_batch=B)


# lattices of both shear branches and the separable one
GRAD_LATTICES = [(144, 6, 12, 1, 2), (16, 4, 8, 1, 2), (72, 6, 12, 1, 3), (2048, 16, 64, 1, 2),
                 (4096, 32, 128, 1, 2), (18432, 32, 256, 1, 2), (1152, 8, 64, 2, 3), (576, 4, 32, 0, 1),
                 # d = 32 and 64 with Mi = 12: ragged work-groups of the wave-kernel gradient
                 (384, 2, 12, 1, 2), (768, 2, 12, 0, 1),
                 # p > 1 of the sheared lattice: time shear, frequency shear and separable
                 # plans with p = 2, 3, 5, 7 and a Fig. 2 shape (a, M) = (40, 60)
                 (48, 4, 6, 1, 2), (48, 4, 6, 1, 4), (48, 6, 8, 0, 1), (72, 6, 8, 1, 3), (120, 10, 12, 1, 2),
                 (224, 7, 8, 1, 2), (2400, 40, 60, 1, 2), (3600, 40, 60, 1, 3)]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_window_gradient_matches_oracle(dtype, kernel_path):
    single = dtype == torch.complex64
    seen = set()
    for lat in GRAD_LATTICES:
        L, a, M, l1, l2 = lat
        N = L // a
        B = 3
        plan = plan_for(lat, dtype, B)
        seen.add(plan.branch)
        g = round_to(complex_normal(L, 11), single)
        f = round_to(np.stack([complex_normal(L, 20 + k) for k in range(B)]), single)
        G = round_to(np.stack([complex_normal(N * M, 40 + k).reshape(N, M) for k in range(B)]), single)
        plan.set_window(torch.tensor(g))
        gg = plan.window_grad(torch.tensor(f), torch.tensor(G)).cpu().numpy()
        ref = sum(oracle.window_gradient(f[k], G[k], a, M, l1, l2) for k in range(B))
        e = rel(gg, ref)
        print("window gradient", kernel_path, dtype, lat, e)
        assert e < TOL[dtype], (lat, e)
    assert {1, 2} <= seen


DUAL_LATTICES = [(144, 6, 12, 1, 2), (16, 4, 8, 1, 2), (2048, 16, 64, 1, 2), (4096, 32, 128, 1, 2),
                 (1152, 8, 64, 2, 3), (576, 4, 32, 0, 1), (240, 6, 12, 1, 2)]
# p > 1 of the sheared lattice (p x p frame-operator blocks): time shear,
# frequency shear and separable plans, p = 2, 3, 5, 7, 8
DUAL_LATTICES_BLOCK = [(48, 4, 6, 1, 2), (48, 4, 6, 1, 4), (48, 6, 8, 0, 1), (72, 6, 8, 1, 3),
                       (120, 10, 12, 1, 2), (180, 10, 12, 1, 3), (224, 7, 8, 1, 2), (288, 8, 9, 1, 2),
                       (1200, 40, 60, 1, 2)]


@pytest.mark.parametrize("lat", DUAL_LATTICES + DUAL_LATTICES_BLOCK)
def test_dual_window_matches_oracle(lat):
    L, a, M, l1, l2 = lat
    plan = plan_for(lat, torch.complex64, 1)
    g = gaussian_window(L, a, M)
    gd, bounds = plan.dual(torch.tensor(g))
    gd = gd.cpu().numpy()
    A, Bb = bounds.cpu().numpy()
    if L <= 2048:
        ref = oracle.dual_window(g, a, M, l1, l2)
        lo, hi = oracle.frame_bounds(g, a, M, l1, l2)
        print("dual", lat, rel(gd, ref), (A, lo), (Bb, hi))
        assert rel(gd, ref) < 1e-12
        assert abs(A - lo) < 1e-10 * hi and abs(Bb - hi) < 1e-10 * hi
    # S g_d = g at sampled points
    pts = np.linspace(0, L - 1, 16).astype(np.int64)
    sg = oracle.frame_operator_apply(gd, g, a, M, l1, l2, pts)
    assert rel(sg, g[pts]) < 1e-11


@pytest.mark.parametrize("lat", DUAL_LATTICES + DUAL_LATTICES_BLOCK + [(24, 2, 6, 1, 4), (18, 3, 6, 2, 3)])
def test_tight_window_matches_oracle(lat):
    """Canonical tight window S^{-1/2} g (time shear, frequency shear and
    separable plans): oracle values, the frame bounds, and tightness S_gt = I
    at sampled points."""
    L, a, M, l1, l2 = lat
    plan = plan_for(lat, torch.complex64, 1)
    g = gaussian_window(L, a, M) + 0.1j * complex_normal(L, 8)
    gt, bounds = plan.tight(torch.tensor(g))
    gt = gt.cpu().numpy()
    A, Bb = bounds.cpu().numpy()
    _, bounds_d = plan.dual(torch.tensor(g))
    assert np.allclose(bounds.cpu().numpy(), bounds_d.cpu().numpy(), rtol=1e-12)
    if L <= 2048:
        ref = oracle.tight_window(g, a, M, l1, l2)
        lo, hi = oracle.frame_bounds(g, a, M, l1, l2)
        print("tight", lat, plan.branch, rel(gt, ref), (A, lo), (Bb, hi))
        assert rel(gt, ref) < 1e-12
        assert abs(A - lo) < 1e-10 * hi and abs(Bb - hi) < 1e-10 * hi
    pts = np.linspace(0, L - 1, 16).astype(np.int64)
    x = complex_normal(L, 9)
    st = oracle.frame_operator_apply(x, gt, a, M, l1, l2, pts)
    assert rel(st, x[pts]) < 1e-11


def test_dual_and_tight_on_a_crossover_lattice():
    """Fig. 2 shape a = 40, M = 60 at L = 302400, lambda = 1/2: the sheared
    lattice has p = 2 and columns of 2520.  S g_d = g and S_gt = I at sampled
    points, and both calls report the same frame bounds."""
    lat = (302400, 40, 60, 1, 2)
    L, a, M, l1, l2 = lat
    plan = plan_for(lat, torch.complex64, 1)
    assert plan.info.p == 2
    g = gaussian_window(L, a, M)
    gd, bd = plan.dual(torch.tensor(g))
    gt, bt = plan.tight(torch.tensor(g))
    bd, bt = bd.cpu().numpy(), bt.cpu().numpy()
    assert 0 < bd[0] <= bd[1] and np.allclose(bd, bt, rtol=1e-12)
    pts = np.linspace(0, L - 1, 4).astype(np.int64)
    sg = oracle.frame_operator_apply(gd.cpu().numpy(), g, a, M, l1, l2, pts)
    assert rel(sg, g[pts]) < 1e-11
    x = complex_normal(L, 3)
    st = oracle.frame_operator_apply(x, gt.cpu().numpy(), a, M, l1, l2, pts)
    assert rel(st, x[pts]) < 1e-11


# p > 8 of the sheared lattice (one wavefront per p x p block, in LDS):
# separable, time-shear and frequency-shear plans, p = 9 ... 64
DUAL_LATTICES_WIDE = [(90, 9, 10, 0, 1), (180, 9, 10, 1, 2), (720, 18, 20, 1, 4), (810, 27, 30, 1, 3),
                      (480, 15, 16, 1, 2), (1728, 27, 32, 1, 2), (2520, 35, 36, 1, 2), (4032, 63, 64, 0, 1),
                      (4032, 64, 63, 0, 1), (8064, 63, 64, 1, 2)]


@pytest.mark.parametrize("lat", DUAL_LATTICES_WIDE)
def test_dual_and_tight_with_wide_blocks(lat):
    """Canonical dual and tight windows and the frame bounds for p from 9 to
    64 against the oracle's Walnut-block solve and eigendecomposition (L up
    to 4032), S g_d = g and S_gt = I at sampled points.  a = 64, M = 63 is
    not a frame: the lower bound is zero.  The window is a modulated Gaussian
    with a small complex perturbation (frame bound ratio below 40, so the
    FP64 solve keeps the 1e-12 bar)."""
    L, a, M, l1, l2 = lat
    plan = plan_for(lat, torch.complex128, 1)
    assert plan.info.p > 8
    l = np.arange(L)
    g = gaussian_window(L, a, M) * np.exp(2j * np.pi * 5 * l / L) + 0.002j * complex_normal(L, 18)
    gd, bd = plan.dual(torch.tensor(g))
    gt, bt = plan.tight(torch.tensor(g))
    gd, gt = gd.cpu().numpy(), gt.cpu().numpy()
    bd, bt = bd.cpu().numpy(), bt.cpu().numpy()
    assert np.allclose(bd, bt, rtol=1e-12)
    if a > M:
        assert bd[0] == 0 and bd[1] > 0
        return
    if L <= 4032:
        lo, hi = oracle.frame_bounds(g, a, M, l1, l2)
        ed = rel(gd, oracle.dual_window(g, a, M, l1, l2))
        et = rel(gt, oracle.tight_window(g, a, M, l1, l2))
        print("wide blocks", lat, plan.branch, plan.info.p, ed, et, (bd[0], lo), (bd[1], hi))
        assert ed < 1e-12 and et < 1e-12
        assert abs(bd[0] - lo) < 1e-10 * hi and abs(bd[1] - hi) < 1e-10 * hi
    pts = np.linspace(0, L - 1, 8).astype(np.int64)
    assert rel(oracle.frame_operator_apply(gd, g, a, M, l1, l2, pts), g[pts]) < 1e-11
    x = complex_normal(L, 19)
    assert rel(oracle.frame_operator_apply(x, gt, a, M, l1, l2, pts), x[pts]) < 1e-11


def test_functional_dual_and_tight():
    """paper_1307_4569_amd.dual(g, a, M, lambda1, lambda2) builds the plan
    itself: the same windows and bounds as the plan calls and the oracle."""
    import paper_1307_4569_amd as dgtns
    lat = (144, 6, 12, 1, 2)
    L, a, M, l1, l2 = lat
    g = torch.tensor(gaussian_window(L, a, M) + 0.1j * complex_normal(L, 21))
    gd, bd = dgtns.dual(g, a, M, l1, l2)
    gt, bt = dgtns.dual(g, a, M, l1, l2, tight=True)
    gn = g.numpy()
    assert rel(gd.cpu().numpy(), oracle.dual_window(gn, a, M, l1, l2)) < 1e-12
    assert rel(gt.cpu().numpy(), oracle.tight_window(gn, a, M, l1, l2)) < 1e-12
    lo, hi = oracle.frame_bounds(gn, a, M, l1, l2)
    for b in (bd, bt):
        A, Bb = b.cpu().numpy()
        assert abs(A - lo) < 1e-10 * hi and abs(Bb - hi) < 1e-10 * hi


def test_dual_refuses_p_above_64():
    from paper_1307_4569_amd import _binding as Bb
    plan = plan_for((4160, 65, 64, 0, 1), torch.complex64, 1)
    assert plan.info.p == 65
    g = torch.tensor(gaussian_window(4160, 65, 64))
    for fn in (plan.dual, plan.tight):
        with pytest.raises(Bb.DgtnsError) as e:
            fn(g)
        assert e.value.status == Bb.DGTNS_EUNSUPPORTED


def test_multiwindow_plans_refuse_dual_and_tight():
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as Bb
    plan = Plan(144, 6, 12, 1, 2, dtype=torch.complex64, max_batch=1, algorithm="multiwindow")
    g = torch.tensor(gaussian_window(144, 6, 12))
    for fn in (plan.dual, plan.tight):
        with pytest.raises(Bb.DgtnsError) as e:
            fn(g)
        assert e.value.status == Bb.DGTNS_EUNSUPPORTED


def test_precision_workload_tight_and_reconstruction():
    """FP64 tight windows of the Gaussian and the Hann window at L = 2^20,
    lambda = 1/4: S_gt = I at sampled points, and f = C*_gt C_gt f through the
    FP64 forward and adjoint transforms."""
    w = PRECISION
    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    plan = plan_for(lat, torch.complex128, 2)
    pts = np.linspace(0, w.L - 1, 12).astype(np.int64)
    for name, g in (("gaussian", gaussian_window(w.L, w.a, w.M)), ("hann", hann_window(w.L, 2048))):
        gt, bounds = plan.tight(torch.tensor(g))
        x1 = complex_normal(w.L, 5)
        e_s = rel(oracle.frame_operator_apply(x1, gt.cpu().numpy(), w.a, w.M, w.lam1, w.lam2, pts), x1[pts])
        x = np.stack([chirp_mixture(w.L, 13074569 + 3000 + k) for k in range(2)])
        plan.set_window(gt)
        rec = plan.adjoint(plan.forward(torch.tensor(x))).cpu().numpy()
        e_r = rel(rec, x)
        print("precision tight", name, "bounds", bounds.cpu().numpy(), "S_gt err", e_s, "reconstruction err", e_r)
        assert e_s < 1e-11 and e_r < 1e-12


def test_precision_workload_dual_and_reconstruction():
    """FP64 dual of the Gaussian and of the Hann window at L = 2^20, lambda =
    1/4; S g_d = g at sampled points and perfect reconstruction of real chirp
    signals through the FP64 forward and adjoint transforms."""
    w = PRECISION
    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    plan = plan_for(lat, torch.complex128, 2)
    pts = np.linspace(0, w.L - 1, 12).astype(np.int64)
    for name, g in (("gaussian", gaussian_window(w.L, w.a, w.M)), ("hann", hann_window(w.L, 2048))):
        gd, bounds = plan.dual(torch.tensor(g))
        A, Bb = bounds.cpu().numpy()
        sg = oracle.frame_operator_apply(gd.cpu().numpy(), g, w.a, w.M, w.lam1, w.lam2, pts)
        e_s = rel(sg, g[pts])
        x = np.stack([chirp_mixture(w.L, 13074569 + 3000 + k) for k in range(2)])
        plan.set_window(torch.tensor(g))
        c = plan.forward(torch.tensor(x))
        plan.set_window(gd)
        rec = plan.adjoint(c).cpu().numpy()
        e_r = rel(rec, x)
        print("precision dual", name, "bounds", A, Bb, "S gd err", e_s, "reconstruction err", e_r)
        assert A > 0 and e_s < 1e-11 and e_r < 1e-12


def test_autograd_gradcheck_fp64():
    from paper_1307_4569_amd import DGTFunction
    lat = (144, 6, 12, 1, 2)
    plan = plan_for(lat, torch.complex128, 2)
    rng = np.random.default_rng(5)
    f = torch.tensor(rng.standard_normal((2, 144)) + 1j * rng.standard_normal((2, 144)), device="cuda",
                     requires_grad=True)
    g = torch.tensor(gaussian_window(144, 6, 12) + 0.1j * rng.standard_normal(144), device="cuda",
                     requires_grad=True)
    fn = lambda f_, g_: DGTFunction.apply(f_, g_, plan)
    assert torch.autograd.gradcheck(fn, (f, g), eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)


@pytest.mark.parametrize("lat", [(144, 6, 12, 1, 2), (4096, 32, 128, 1, 2), (2400, 40, 60, 1, 2)])
def test_autograd_matches_oracle_gradients(lat):
    from paper_1307_4569_amd import DGTFunction
    L, a, M, l1, l2 = lat
    plan = plan_for(lat, torch.complex128, 2)
    f = np.stack([complex_normal(L, 60 + k) for k in range(2)])
    g = gaussian_window(L, a, M)
    T = np.stack([np.abs(oracle.dgt_fold(complex_normal(L, 90 + k), g, a, M, l1, l2)) ** 2 for k in range(2)])
    ft = torch.tensor(f, device="cuda", requires_grad=True)
    gt = torch.tensor(g, device="cuda", requires_grad=True)
    c = DGTFunction.apply(ft, gt, plan)
    loss = ((c.abs() ** 2 - torch.tensor(T, device="cuda")) ** 2).sum()
    loss.backward()
    gf_ref = []
    gg_ref = np.zeros(L, complex)
    l_ref = 0.0
    for k in range(2):
        lk, gf, gg = oracle.loss_and_grads(f[k], g, T[k], a, M, l1, l2)
        l_ref += lk
        gf_ref.append(gf)
        gg_ref += gg
    assert abs(loss.item() - l_ref) < 1e-12 * l_ref
    assert rel(ft.grad.cpu().numpy(), np.stack(gf_ref)) < 1e-12
    assert rel(gt.grad.cpu().numpy(), gg_ref) < 1e-12
    # the window was prepared once for the forward and backward of this step
    assert plan.window_serial == 1


def test_autograd_prepares_the_window_once_per_step():
    """DGTFunction prepares the plan's window once per forward, and prepares
    it again in backward only if another window was set after the forward."""
    from paper_1307_4569_amd import DGTFunction
    lat = (144, 6, 12, 1, 2)
    plan = plan_for(lat, torch.complex128, 1)
    f = torch.tensor(complex_normal(144, 70), device="cuda", requires_grad=True)
    g = torch.tensor(gaussian_window(144, 6, 12), device="cuda", requires_grad=True)
    opt = torch.optim.SGD([g], lr=1e-3)
    for step in range(3):
        opt.zero_grad()
        c = DGTFunction.apply(f, g, plan)
        (c.abs() ** 2).sum().backward()
        assert plan.window_serial == step + 1
        opt.step()
    # a window set between forward and backward is replaced by the saved one
    c = DGTFunction.apply(f, g, plan)
    other = torch.tensor(complex_normal(144, 71), device="cuda")
    plan.set_window(other)
    g.grad = None
    (c.abs() ** 2).sum().backward()
    assert plan.window_serial == 6
    f_np, g_np = f.detach().cpu().numpy(), g.detach().cpu().numpy()
    c_ref = oracle.dgt_fold(f_np, g_np, 6, 12, 1, 2)
    gg_ref = oracle.window_gradient(f_np, 2 * c_ref, 6, 12, 1, 2)
    assert rel(g.grad.cpu().numpy(), gg_ref) < 1e-12


def test_gradient_workload():
    """Differentiation workload: FP32 forward and hand-written backward at
    L = 65536, a = 32, M = 256, lambda = 1/2, batch 32; gradients checked
    against the oracle gradient on two signals and, in FP64, against central
    finite differences (h = 1e-6) along seeded directions."""
    from paper_1307_4569_amd import DGTFunction
    w = GRADIENT
    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    g0 = gaussian_window(w.L, w.a, w.M)
    fT = complex_normal(w.L, 4000)
    f = complex_normal_batch(w.batch, w.L, 4)
    # target spectrogram of a seeded signal through the initial window
    plan32 = plan_for(lat, torch.complex64, w.batch)
    plan32.set_window(torch.tensor(g0))
    T = (plan32.forward(torch.tensor(fT.astype(np.complex64))).abs() ** 2).double()
    ft = torch.tensor(f.astype(np.complex64), device="cuda", requires_grad=True)
    gt = torch.tensor(g0.astype(np.complex64), device="cuda", requires_grad=True)
    c = DGTFunction.apply(ft, gt, plan32)
    loss = ((c.abs() ** 2 - T.float()) ** 2).sum()
    loss.backward()
    # oracle gradients of the first two signals (window gradient of that sub-batch)
    Tn = T.cpu().numpy()
    f32 = f.astype(np.complex64).astype(np.complex128)
    g32 = g0.astype(np.complex64).astype(np.complex128)
    gf_err = []
    for k in (0, w.batch - 1):
        _, gf, _ = oracle.loss_and_grads(f32[k], g32, Tn, w.a, w.M, w.lam1, w.lam2)
        gf_err.append(rel(ft.grad[k].cpu().numpy(), gf))
    print("gradient workload grad_f rel err vs oracle", gf_err)
    assert max(gf_err) < 1e-5
    sub = torch.tensor(f32[:2].astype(np.complex64), device="cuda", requires_grad=True)
    gsub = torch.tensor(g0.astype(np.complex64), device="cuda", requires_grad=True)
    plan2 = plan_for(lat, torch.complex64, 2)
    csub = DGTFunction.apply(sub, gsub, plan2)
    ((csub.abs() ** 2 - T.float()) ** 2).sum().backward()
    gg_ref = sum(oracle.loss_and_grads(f32[k], g32, Tn, w.a, w.M, w.lam1, w.lam2)[2] for k in range(2))
    e_gg = rel(gsub.grad.cpu().numpy(), gg_ref)
    print("gradient workload grad_g rel err vs oracle", e_gg)
    assert e_gg < 1e-5
    # FP64 central differences on the full batch
    plan64 = plan_for(lat, torch.complex128, w.batch)
    f64 = torch.tensor(f, device="cuda", requires_grad=True)
    g64 = torch.tensor(g0, device="cuda", requires_grad=True)

    def loss_fn(ff, gg):
        cc = DGTFunction.apply(ff, gg, plan64)
        return ((cc.abs() ** 2 - T) ** 2).sum()

    L0 = loss_fn(f64, g64)
    L0.backward()
    rng = np.random.default_rng(123)
    h = 1e-6
    for i in range(16):
        df = torch.tensor(rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape), device="cuda")
        dg = torch.tensor(rng.standard_normal(w.L) + 1j * rng.standard_normal(w.L), device="cuda") * 1e-2
        with torch.no_grad():
            fd_f = (loss_fn(f64 + h * df, g64) - loss_fn(f64 - h * df, g64)).item() / (2 * h)
            fd_g = (loss_fn(f64, g64 + h * dg) - loss_fn(f64, g64 - h * dg)).item() / (2 * h)
        an_f = torch.vdot(f64.grad.flatten(), df.flatten()).real.item()
        an_g = torch.vdot(g64.grad.flatten(), dg.flatten()).real.item()
        print("finite differences", i, fd_f, an_f, fd_g, an_g)
        assert abs(fd_f - an_f) < 1e-5 * abs(an_f)
        assert abs(fd_g - an_g) < 1e-5 * abs(an_g)
