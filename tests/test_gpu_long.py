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


def test_long_columns_list_batch_and_refusals():
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
    for fn in (lambda: plan.dual(g), lambda: plan.tight(g), lambda: plan.window_grad(f, c)):
        with pytest.raises(Bb.DgtnsError) as e:
            fn()
        assert e.value.status == Bb.DGTNS_EUNSUPPORTED
