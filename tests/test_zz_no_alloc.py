"""The forward that allocates nothing (dgtns_forward_noalloc): its scratch is
a static device array, so the test checks it against dgtns_forward (the same
transform with a caller workspace) on two calls in a row, the second with a
smaller batch, and the refusal of a batch whose workspace exceeds the
scratch.  Runs through the C-ABI binding."""
import numpy as np
import pytest

from dgt_inputs import complex_normal, gaussian_window, hann_window, round_to

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}

# (lattice, dtype, plan keywords, first batch, second batch)
CASES = [
    ((262144, 64, 512, 1, 2), torch.complex64, {}, 3, 1),           # time shear, 16 MiB of h per signal
    ((36864, 32, 256, 1, 2), torch.complex64, {}, 6, 2),            # frequency shear (two-pass length-L transform)
    ((73728, 64, 512, 1, 3), torch.complex128, {}, 2, 1),           # time shear, FP64
    ((5184, 6, 36, 1, 3), torch.complex64, {"algorithm": "multiwindow"}, 5, 3),
    ((65536, 32, 256, 1, 2), torch.complex64, {"algorithm": "fir", "support": (65536 - 256, 512)}, 4, 1),
]


def rel(x, y):
    return float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1307_4569_amd import _binding
    _binding.lib()
    return torch.device("cuda", 0)


def signals(L, nb, seed, dtype):
    return torch.tensor(np.stack([round_to(complex_normal(L, seed + k), dtype == torch.complex64)
                                  for k in range(nb)])).to(dtype).cuda()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[2].get('algorithm', 'shear')}-{c[1]}" for c in CASES])
def test_noalloc_forward_matches_forward(case):
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as B
    lat, dtype, kw, b1, b2 = case
    L, a, M, l1, l2 = lat
    plan = Plan(*lat, dtype=dtype, max_batch=max(b1, b2), **kw)
    g = hann_window(L, 512) if kw.get("algorithm") == "fir" else gaussian_window(L, a, M)
    plan.set_window(torch.tensor(g))
    st = torch.cuda.current_stream().cuda_stream
    for nb, seed in ((b1, 11), (b2, 12)):      # second call: smaller batch, same scratch
        assert B.dgtns_workspace_bytes(plan._h, B.DGTNS_OP_FORWARD, nb) <= B.DGTNS_NOALLOC_SCRATCH_BYTES
        f = signals(L, nb, seed, dtype)
        ref = plan.forward(f)
        c = torch.full_like(ref, float("nan"))
        B.dgtns_forward_noalloc(plan._h, f.data_ptr(), 0, c.data_ptr(), nb, st)
        torch.cuda.synchronize()
        err = rel(c, ref)
        print(lat, kw.get("algorithm", "shear"), dtype, "batch", nb, "rel err vs dgtns_forward", err,
              "bitwise", torch.equal(c, ref))
        assert err < TOL[dtype]
        assert torch.equal(c, ref)


def test_noalloc_refuses_batch_beyond_scratch():
    """A batch whose forward workspace exceeds the static scratch returns
    DGTNS_EWORKSPACE before anything is enqueued: the output is untouched."""
    from paper_1307_4569_amd import Plan
    from paper_1307_4569_amd import _binding as B
    L, a, M, l1, l2 = 262144, 64, 512, 1, 2
    plan = Plan(L, a, M, l1, l2, dtype=torch.complex64, max_batch=8)
    plan.set_window(torch.tensor(gaussian_window(L, a, M)))
    nb = 8
    assert B.dgtns_workspace_bytes(plan._h, B.DGTNS_OP_FORWARD, nb) > B.DGTNS_NOALLOC_SCRATCH_BYTES
    f = signals(L, nb, 21, torch.complex64)
    c = torch.zeros((nb, plan.N, plan.M), dtype=torch.complex64, device="cuda")
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_forward_noalloc(plan._h, f.data_ptr(), 0, c.data_ptr(), nb, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == B.DGTNS_EWORKSPACE
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(c)) == 0
