"""GPU parity of the shear-OLA algorithm (Section 4: the shear algorithm on
blocks of the signal, combined by overlap-add): coefficients of eq. (DGT) for
a window truncated to its support, against the FP64 oracle applied to the
truncated window, on small lattices (separable, time-shear and
frequency-shear inner plans, signed and wrapping supports, several blocks per
window), both kernel paths, and on the precision workload's Hann window of
length 2048 at L = 2^20, lambda = 1/4 against the oracle and the FIR-window
algorithm; the adjoint (synthesis) of the same plans against the oracle's
synthesis with the truncated window."""
import numpy as np
import pytest

import oracle
from dgt_inputs import PRECISION, chirp_mixture, complex_normal, complex_normal_batch, hann_window, round_to

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


def ola_plan(lat, support, block, dtype, B, inner="auto"):
    from paper_1307_4569_amd import Plan
    return Plan(*lat, dtype=dtype, max_batch=B, algorithm="shear-ola", support=support, block=block, inner=inner)


# (L, a, M, lambda1, lambda2), (support start, length), block
CASES = [((1536, 8, 16, 1, 2), (1536 - 24, 48), 192),
         ((3456, 12, 24, 1, 3), (0, 60), 288),
         ((2304, 16, 32, 1, 4), (2304 - 32, 64), 256),
         ((1536, 8, 16, 0, 1), (5, 40), 96),
         ((4096, 32, 128, 1, 2), (4096 - 96, 192), 512),     # window longer than a block
         ((6144, 16, 64, 1, 2), (6000, 300), 1024)]          # support wrapping past L


@pytest.mark.parametrize("inner", ["shear", "auto"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_shear_ola_matches_oracle(dtype, kernel_path, inner):
    """Block transforms by the shear algorithm (separable, time-shear and
    frequency-shear inner plans) or the automatic choice (multiwindow where
    the shear plan needs a frequency shear)."""
    single = dtype == torch.complex64
    seen, windows, shears = set(), set(), set()
    for lat, support, block in CASES:
        L, a, M, l1, l2 = lat
        B = 3
        plan = ola_plan(lat, support, block, dtype, B, inner)
        seen.add(plan.info.branch)
        windows.add(plan.info.windows)
        shears.add(plan.info.s0 != 0)
        g = round_to(complex_normal(L, 21), single)
        f = round_to(np.stack([complex_normal(L, 30 + k) for k in range(B)]), single)
        plan.set_window(torch.tensor(g))
        c = plan.forward(torch.tensor(f)).cpu().numpy()
        gt = truncate(g, *support)
        e = max(rel(c[k], oracle.dgt_fold(f[k], gt, a, M, l1, l2)) for k in range(B))
        # adjoint: each stage's adjoint in reverse order, against the oracle's
        # synthesis with the truncated window
        N = L // a
        cin = round_to(np.stack([complex_normal(N * M, 60 + k).reshape(N, M) for k in range(B)]), single)
        fa = plan.adjoint(torch.tensor(cin)).cpu().numpy()
        ea = max(rel(fa[k], oracle.idgt_adjoint(cin[k], gt, a, M, l1, l2)) for k in range(B))
        print("shear-OLA", inner, kernel_path, dtype, lat, support, block, plan.info.block_dgt_length, e,
              "adjoint", ea)
        assert e < TOL[dtype] and ea < TOL[dtype], (lat, e, ea)
    assert seen == {5}
    if inner == "shear":
        assert windows == {1} and shears == {False, True}
    else:
        assert windows > {1} and shears == {False}


@pytest.mark.parametrize("inner", ["shear", "auto"])
def test_shear_ola_precision_workload(inner):
    """Hann window of length 2048 centred at 0, L = 2^20, a = 128, M = 1024,
    lambda = 1/4, real chirp signals in FP32, blocks of 32768 samples, block
    transforms by the shear and by the automatic (multiwindow) plan: sampled
    time positions against the oracle, and the FIR-window algorithm with the
    same window gives the same coefficients."""
    w = PRECISION
    lat = (w.L, w.a, w.M, w.lam1, w.lam2)
    B = 4
    g = round_to(hann_window(w.L, 2048), True)
    x = round_to(np.stack([chirp_mixture(w.L, 13074569 + 3000 + k) for k in range(B)]), True).real
    xt = torch.tensor(x.astype(np.complex64)).cuda()
    plan = ola_plan(lat, (w.L - 1024, 2048), 32768, torch.complex64, B, inner)
    assert plan.info.windows == (1 if inner == "shear" else w.lam2)
    plan.set_window(torch.tensor(g))
    c = plan.forward(xt)
    cols = list(range(0, w.N, 331)) + [w.N - 1]
    errs = [rel(c[k, cols].cpu().numpy(), oracle.dgt_fold(x[k].astype(complex), g, w.a, w.M, w.lam1, w.lam2,
                                                          columns=cols)) for k in (0, B - 1)]
    from paper_1307_4569_amd import Plan
    fir = Plan(*lat, dtype=torch.complex64, max_batch=B, algorithm="fir", support=(w.L - 1024, 2048))
    fir.set_window(torch.tensor(g))
    cf = fir.forward(xt)
    d = (torch.linalg.vector_norm(c - cf) / torch.linalg.vector_norm(cf)).item()
    print("shear-OLA precision workload", inner, plan.info.block_dgt_length, errs, "vs FIR", d)
    assert max(errs) < 1e-5 and d < 2e-5
    # adjoint of the batch against the FIR algorithm's adjoint and the oracle
    # at sampled samples
    fa, fa_fir = plan.adjoint(cf), fir.adjoint(cf)
    da = (torch.linalg.vector_norm(fa - fa_fir) / torch.linalg.vector_norm(fa_fir)).item()
    samples = np.arange(0, w.L, 509)
    ref = oracle.idgt_adjoint(cf[B - 1].cpu().numpy().astype(np.complex128), g, w.a, w.M, w.lam1, w.lam2,
                              samples=samples)
    ea = rel(fa[B - 1, torch.tensor(samples, device="cuda")].cpu().numpy(), ref)
    print("shear-OLA precision workload adjoint: vs FIR", da, "sampled vs oracle", ea)
    assert da < 2e-5 and ea < 1e-5


def test_shear_ola_refusals():
    from paper_1307_4569_amd import _binding as Bb
    lat, support, block = CASES[0]
    L = lat[0]
    plan = ola_plan(lat, support, block, torch.complex64, 2)
    g = torch.tensor(complex_normal(L, 3))
    plan.set_window(g)
    f = torch.tensor(complex_normal_batch(2, L, 7).astype(np.complex64)).cuda()
    c = plan.forward(f)
    for call in (lambda: plan.window_grad(f, c), lambda: plan.dual(g), lambda: plan.tight(g)):
        with pytest.raises(Bb.DgtnsError) as e:
            call()
        assert e.value.status == Bb.DGTNS_EUNSUPPORTED
    wsb = Bb.dgtns_workspace_bytes(plan._h, Bb.DGTNS_OP_FORWARD, 2)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(c)
    with pytest.raises(Bb.DgtnsError) as e:
        Bb.dgtns_forward_batch(plan._h, [f[k].data_ptr() for k in range(2)], 0,
                               [out[k].data_ptr() for k in range(2)], ws.data_ptr(), wsb,
                               torch.cuda.current_stream().cuda_stream)
    assert e.value.status == Bb.DGTNS_EUNSUPPORTED
