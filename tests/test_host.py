"""Host-side checks of libdgtns that need no GPU: exported symbols, the
lattice planner against brute force and the paper's number-theory results,
and the synchronous error paths of the C-ABI."""
import ctypes
import math
import os
import re

import pytest

from tests.conftest import ROOT, feasible_lattices

B = pytest.importorskip("paper_1307_4569_amd._binding")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libdgtns.so not built")
    return B.lib()


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "dgtns.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dgtns_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_header_symbol(lib):
    syms = header_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(n for n, _, _ in B.SIGNATURES) == syms


def test_status_strings(lib):
    for code, name in B.STATUS_NAMES.items():
        assert B.dgtns_status_string(code) == name


# ---------------------------------------------------------------------------
# Planner
# ---------------------------------------------------------------------------

def lattice(L, a, M, l1, l2):
    b = L // M
    s = b * l1 // l2
    return {((a * k1) % L, (s * k1 + b * k2) % L) for k1 in range(L // a) for k2 in range(L // b)}


def is_closed_lattice(L, a, M, l1, l2):
    """Brute-force lattice condition (proof of Prop. 1): s = b l1/l2 is an
    integer and N steps of (a, s) land in {0} x bZ."""
    b = L // M
    if (b * l1) % l2:
        return False
    s = b * l1 // l2
    return ((L // a) * s) % b == 0


def test_prop8_feasible_lengths(lib):
    """The planner accepts exactly the lengths that form a lattice, which
    are the multiples of lambda2 * lcm(a, M) (Prop. 8)."""
    n = 0
    for L in range(2, 97):
        divs = [d for d in range(1, L + 1) if L % d == 0]
        for a in divs:
            for M in divs:
                for l2 in range(1, 5):
                    for l1 in range(l2):
                        if math.gcd(l1, l2) != 1:
                            continue
                        ok = is_closed_lattice(L, a, M, l1, l2)
                        assert ok == (L % (l2 * (a * M // math.gcd(a, M))) == 0)
                        h = ctypes.c_void_p()
                        st = lib.dgtns_plan_create(ctypes.byref(h), L, a, M, l1, l2, 0, 1)
                        if ok:
                            assert st in (B.DGTNS_OK, B.DGTNS_EUNSUPPORTED), (L, a, M, l1, l2)
                        else:
                            assert st == B.DGTNS_ELATTICE, (L, a, M, l1, l2)
                        if st == B.DGTNS_OK:
                            lib.dgtns_plan_destroy(h)
                        n += 1
    assert n > 5000


@pytest.mark.parametrize("chunk", range(4))
def test_shearfind_makes_lattice_separable(lib, chunk):
    """U^{-1} A Z_L^2 is the separable lattice (ab/b_r) Z x b_r Z, where
    U^{-1} = [[1 + s0 s1, s0], [s1, 1]] (proof of Thm. 2)."""
    lats = feasible_lattices(max_L=90, max_lam2=4)[chunk::4]
    nfs = 0
    for (L, a, M, l1, l2) in lats:
        s0, s1, br = B.dgtns_shearfind(L, a, M, l1, l2)
        b = L // M
        ar = a * b // br
        assert (a * b) % br == 0 and L % br == 0 and L % ar == 0
        img = {(((1 + s0 * s1) * x + s0 * w) % L, (s1 * x + w) % L) for (x, w) in lattice(L, a, M, l1, l2)}
        sep = {((ar * i) % L, (br * j) % L) for i in range(L // ar) for j in range(L // br)}
        assert img == sep, (L, a, M, l1, l2, s0, s1, br)
        # a time shear alone is used exactly when a | s + k b for some k (Prop. 9)
        s = b * l1 // l2
        time_only = any((s + k * b) % a == 0 for k in range(a + 1))
        assert (s0 == 0) == time_only
        nfs += s0 != 0
    assert nfs > 20


def test_remark_values(lib):
    path = os.path.join(ROOT, "tests", "golden", "remark_quincunx.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for a, M, l1, l2, expect in (map(int, r) for r in rows):
        lmin = l2 * (a * M // math.gcd(a, M))
        assert lmin * B.dgtns_noshear_factor(a, M, l1, l2) == expect
        # at that length the planner needs no frequency shear ...
        assert B.dgtns_shearfind(expect, a, M, l1, l2)[0] == 0
        # ... and shorter feasible lengths do need one
        for L in range(lmin, expect, lmin):
            assert B.dgtns_shearfind(L, a, M, l1, l2)[0] != 0


def test_prop9_lengths_need_no_frequency_shear(lib):
    for (L, a, M, l1, l2) in feasible_lattices(max_L=120, max_lam2=4):
        lmin = l2 * (a * M // math.gcd(a, M))
        if L % (lmin * B.dgtns_noshear_factor(a, M, l1, l2)) == 0:
            assert B.dgtns_shearfind(L, a, M, l1, l2)[0] == 0


SERVING_FREQ_SHEAR = {(36864, 32, 256), (73728, 32, 256), (36864, 64, 512), (73728, 64, 512),
                      (147456, 64, 512), (294912, 64, 512)}


def test_workload_plans(lib):
    from dgt_inputs import GRADIENT, LARGE, PRECISION, SMALL, serving_plans
    # the small workload has q = 2 (c = 6, d = 12); the others q = 8
    for w, q in ((SMALL, 2), (LARGE, 8), (PRECISION, 8), (GRADIENT, 8)):
        h = B.dgtns_plan_create(w.L, w.a, w.M, w.lam1, w.lam2, 0, 1)
        i = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        assert (i.branch, i.s0, i.p, i.q) == (B.DGTNS_TIME_SHEAR, 0, 1, q), (w, i.branch, i.s0, i.p, i.q)
    h = B.dgtns_plan_create(SMALL.L, SMALL.a, SMALL.M, SMALL.lam1, SMALL.lam2, 1, 1)
    i = B.dgtns_plan_info(h)
    B.dgtns_plan_destroy(h)
    assert (i.s1, i.c, i.d) == (-1, 6, 12)
    nfs = 0
    for (L, a, M, l1, l2) in serving_plans():
        h = B.dgtns_plan_create(L, a, M, l1, l2, 0, 8)
        i = B.dgtns_plan_info(h)
        fs = i.branch == B.DGTNS_FREQ_SHEAR
        assert fs == ((L, a, M) in SERVING_FREQ_SHEAR and (l1, l2) == (1, 2))
        nfs += fs
        B.dgtns_plan_destroy(h)
    assert nfs == 6


def test_multiwindow_plans(lib):
    """Multiwindow plans (Prop. 4): no shear, the separable lattice
    (lambda2 a, M) with its constants (eq. (cd), eq. (pq)) and lambda2 windows
    whose lambda2 q d intermediate rows cover the N coefficient columns."""
    n = 0
    for (L, a, M, l1, l2) in feasible_lattices(max_L=120, max_lam2=4):
        try:
            h = B.dgtns_plan_create_alg(L, a, M, l1, l2, 0, 2, B.DGTNS_ALG_MULTIWINDOW)
        except B.DgtnsError as e:
            assert e.status == B.DGTNS_EUNSUPPORTED, (L, a, M, l1, l2)
            continue
        i = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        c = math.gcd(l2 * a, M)
        assert i.branch == B.DGTNS_MULTIWINDOW and i.s0 == 0 and i.s1 == 0
        assert (i.inner_a, i.inner_M, i.c, i.p, i.q, i.windows) == (l2 * a, M, c, l2 * a // c, M // c, l2)
        assert i.d * i.p == L // M and i.windows * i.q * i.d == L // a
        n += 1
    assert n > 1000
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create_alg(144, 6, 12, 1, 2, 0, 1, 7)
    assert e.value.status == B.DGTNS_EINVAL
    h = B.dgtns_plan_create_alg(144, 6, 12, 1, 2, 0, 1, B.DGTNS_ALG_SHEAR)
    assert B.dgtns_plan_info(h).branch == B.DGTNS_TIME_SHEAR and B.dgtns_plan_info(h).windows == 1
    B.dgtns_plan_destroy(h)


def test_long_column_plans(lib):
    """Columns longer than one in-LDS transform plan as d = d1 d2 (every
    branch, p = 1 and p = 3, the Fig. 2 lengths); a column length with a
    prime factor above 7 is still refused."""
    cases = [((20160, 2, 4, 0, 1), 0, 5040), ((20160, 3, 4, 1, 2), 1, 1680), ((20160, 3, 6, 1, 3), 2, 10080),
             ((161280, 32, 64, 1, 2), 2, 20160), ((302400, 40, 60, 1, 4), 2, 5040), ((1 << 20, 32, 64, 1, 2), 1, 16384)]
    for lat, branch, d in cases:
        h = B.dgtns_plan_create(*lat, 0, 2)
        i = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        assert (i.branch, i.d) == (branch, d), (lat, i.branch, i.d)
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create(4099 * 4, 2, 4, 0, 1, 0, 1)        # d = 4099 is prime
    assert e.value.status == B.DGTNS_EUNSUPPORTED
    with pytest.raises(B.DgtnsError) as e:                      # multiwindow plans keep d <= 4096
        B.dgtns_plan_create_alg(20160, 2, 4, 1, 2, 0, 1, B.DGTNS_ALG_MULTIWINDOW)
    assert e.value.status == B.DGTNS_EUNSUPPORTED


def test_channel_count_limit(lib):
    """Rows are in-LDS transforms of at most 4096 channels: a separable or
    time-shear lattice with M = 8192 is refused, while a frequency-shear plan
    with M = 8192 runs its rows on the N_r inner channels."""
    for dt in (0, 1):
        with pytest.raises(B.DgtnsError) as e:
            B.dgtns_plan_create(131072, 64, 8192, 0, 1, dt, 1)
        assert e.value.status == B.DGTNS_EUNSUPPORTED
        h = B.dgtns_plan_create(131072, 64, 8192, 1, 2, dt, 1)
        i = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        assert (i.branch, i.d) == (2, 128)


def test_fir_plans(lib):
    """FIR-window plans: branch, no factorisation constants, and the errors."""
    h = B.dgtns_plan_create_fir(144, 6, 12, 1, 2, 0, 2, 140, 20)
    i = B.dgtns_plan_info(h)
    B.dgtns_plan_destroy(h)
    assert i.branch == B.DGTNS_FIR and (i.c, i.d, i.p, i.q) == (0, 0, 0, 0) and i.N == 24
    for args, status in (((144, 6, 12, 1, 2, 0, 1, 0, 0), B.DGTNS_EINVAL),
                         ((144, 6, 12, 1, 2, 0, 1, 0, 145), B.DGTNS_EINVAL),
                         ((242, 2, 11, 0, 1, 0, 1, 0, 10), B.DGTNS_EUNSUPPORTED),   # M = 11 is not 7-smooth
                         ((100, 6, 12, 1, 2, 0, 1, 0, 10), B.DGTNS_ELATTICE)):
        with pytest.raises(B.DgtnsError) as e:
            B.dgtns_plan_create_fir(*args)
        assert e.value.status == status, args
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create_alg(144, 6, 12, 1, 2, 0, 1, B.DGTNS_ALG_FIR)
    assert e.value.status == B.DGTNS_EINVAL


def test_shear_ola_plans(lib):
    """Shear-OLA plans (Section 4): the block DGT length is the least feasible
    one of at least block + window support, the inner plan's constants are
    reported, and the errors."""
    from math import gcd
    L, a, M, l1, l2 = 1048576, 128, 1024, 1, 4
    for block in (32768, 65536, 131072):
        h = B.dgtns_plan_create_ola(L, a, M, l1, l2, 0, 4, L - 1024, 2048, block)
        i = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        Lx = i.block_dgt_length
        assert i.branch == B.DGTNS_SHEAR_OLA and i.block == block
        step = l2 * a * M // gcd(a, M)
        assert Lx % step == 0 and Lx >= block + 2048
        # the least such length: shorter candidates have no shear plan
        for cand in range(-(-(block + 2048) // step) * step, Lx, step):
            with pytest.raises(B.DgtnsError):
                B.dgtns_plan_create(cand, a, M, l1, l2, 0, 1)
        # the inner plan is the automatic plan at that length: here the shear
        # plan needs a frequency shear, so the multiwindow plan
        hi = B.dgtns_plan_create_alg(Lx, a, M, l1, l2, 0, 1, B.DGTNS_ALG_AUTO)
        ii = B.dgtns_plan_info(hi)
        B.dgtns_plan_destroy(hi)
        assert ii.windows == l2
        assert (ii.s0, ii.s1, ii.c, ii.d, ii.p, ii.q, ii.windows) == (i.s0, i.s1, i.c, i.d, i.p, i.q, i.windows)
        # with the shear algorithm asked for: the frequency-shear plan at that length
        h = B.dgtns_plan_create_ola_alg(L, a, M, l1, l2, 0, 4, L - 1024, 2048, block, B.DGTNS_ALG_SHEAR)
        i = B.dgtns_plan_info(h)
        B.dgtns_plan_destroy(h)
        hi = B.dgtns_plan_create(i.block_dgt_length, a, M, l1, l2, 0, 1)
        ii = B.dgtns_plan_info(hi)
        B.dgtns_plan_destroy(hi)
        assert i.block_dgt_length == Lx and i.windows == 1 and i.s0 != 0
        assert (ii.s0, ii.s1, ii.c, ii.d, ii.p, ii.q) == (i.s0, i.s1, i.c, i.d, i.p, i.q)
    for alg in (B.DGTNS_ALG_FIR, B.DGTNS_ALG_SHEAR_OLA, 7):
        with pytest.raises(B.DgtnsError) as e:
            B.dgtns_plan_create_ola_alg(L, a, M, l1, l2, 0, 4, L - 1024, 2048, 32768, alg)
        assert e.value.status == B.DGTNS_EINVAL
    h = B.dgtns_plan_create_fir(L, a, M, l1, l2, 0, 1, 0, 10)
    assert B.dgtns_plan_info(h).block == 0
    B.dgtns_plan_destroy(h)
    for args, status in (((L, a, M, l1, l2, 0, 4, 0, 2048, 3000), B.DGTNS_EINVAL),      # does not divide L
                         ((L, a, M, l1, l2, 0, 4, 0, 2048, 256), B.DGTNS_EINVAL),       # not a multiple of 4 a
                         ((L, a, M, l1, l2, 0, 4, 0, 0, 32768), B.DGTNS_EINVAL),        # empty support
                         ((L, a, M, l1, l2, 0, 40000, 0, 2048, 512), B.DGTNS_EINVAL),   # batch x blocks
                         ((4096, 8, 32, 1, 2, 0, 1, 0, 64, 4096), B.DGTNS_EUNSUPPORTED)):  # one block
        with pytest.raises(B.DgtnsError) as e:
            B.dgtns_plan_create_ola(*args)
        assert e.value.status == status, args
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create_alg(144, 6, 12, 1, 2, 0, 1, B.DGTNS_ALG_SHEAR_OLA)
    assert e.value.status == B.DGTNS_EINVAL


def test_error_paths_without_device(lib):
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create(100, 6, 12, 1, 2, 0, 1)
    assert e.value.status == B.DGTNS_ELATTICE
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create(144, 6, 12, 2, 4, 0, 1)        # not coprime
    assert e.value.status == B.DGTNS_ELATTICE
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create(144, 6, 12, 1, 2, 7, 1)        # bad dtype
    assert e.value.status == B.DGTNS_EINVAL
    with pytest.raises(B.DgtnsError) as e:
        B.dgtns_plan_create(242, 2, 2, 0, 1, 0, 1)         # d = 121 is not 7-smooth
    assert e.value.status == B.DGTNS_EUNSUPPORTED
    h = B.dgtns_plan_create(144, 6, 12, 1, 2, 1, 4)
    dummy = ctypes.c_void_p(4096)
    # not bound: every device call is refused before touching the device
    assert lib.dgtns_forward(h, dummy, 0, dummy, 1, dummy, 1 << 20, None) == B.DGTNS_ESTATE
    assert lib.dgtns_set_window(h, dummy, dummy, 1 << 20, None) == B.DGTNS_ESTATE
    assert lib.dgtns_plan_bind(h, None, 0, None) == B.DGTNS_EINVAL
    assert B.dgtns_workspace_bytes(h, B.DGTNS_OP_FORWARD, 4) >= 16 * 144 * 4 * 2
    with pytest.raises(B.DgtnsError):
        B.dgtns_workspace_bytes(h, 99, 1)
    B.dgtns_plan_destroy(h)


OPS = (B.DGTNS_OP_FORWARD, B.DGTNS_OP_ADJOINT, B.DGTNS_OP_WINDOW_GRAD, B.DGTNS_OP_SET_WINDOW, B.DGTNS_OP_DUAL)


def check_op(h, op, batch=1):
    """Status of dgtns_check_op (host only) and its message."""
    try:
        B.dgtns_check_op(h, op, batch)
        return B.DGTNS_OK, ""
    except B.DgtnsError as e:
        return e.status, str(e)


# (plan constructor arguments, operation, phrase of the refusal message):
# every DGTNS_EUNSUPPORTED refusal of a device call, found on the host
REFUSALS = [
    (("ola", 6144, 16, 64, 1, 2, 0, 2, 6000, 300, 1024), B.DGTNS_OP_WINDOW_GRAD, "shear-algorithm plans only"),
    (("ola", 6144, 16, 64, 1, 2, 0, 2, 6000, 300, 1024), B.DGTNS_OP_DUAL, "shear-algorithm plans"),
    (("fir", 144, 6, 12, 1, 2, 0, 2, 140, 20), B.DGTNS_OP_WINDOW_GRAD, "shear-algorithm plans"),
    (("fir", 144, 6, 12, 1, 2, 0, 2, 140, 20), B.DGTNS_OP_DUAL, "shear-algorithm plans"),
    (("mw", 144, 6, 12, 1, 2, 0, 2), B.DGTNS_OP_WINDOW_GRAD, "shear-algorithm plans"),
    (("mw", 144, 6, 12, 1, 2, 0, 2), B.DGTNS_OP_DUAL, "shear-algorithm plans"),
    (("shear", 4160, 65, 64, 0, 1, 0, 2), B.DGTNS_OP_DUAL, "p <= 64"),                 # p = 65
]


def make(args):
    kind, rest = args[0], args[1:]
    if kind == "ola":
        return B.dgtns_plan_create_ola(*rest)
    if kind == "fir":
        return B.dgtns_plan_create_fir(*rest)
    if kind == "mw":
        return B.dgtns_plan_create_alg(*rest, B.DGTNS_ALG_MULTIWINDOW)
    return B.dgtns_plan_create(*rest)


@pytest.mark.parametrize("args,op,phrase", REFUSALS)
def test_every_refusal_is_found_on_the_host(lib, args, op, phrase):
    """dgtns_check_op runs a call's per-launch checks on the host, on an
    unbound plan: each unsupported operation is refused with its reason, and
    the device call runs the same checks before it enqueues anything."""
    h = make(args)
    try:
        st, msg = check_op(h, op)
        assert st == B.DGTNS_EUNSUPPORTED and phrase in msg, (args, op, st, msg)
        # the transforms of the plan pass the same checks
        for other in (B.DGTNS_OP_FORWARD, B.DGTNS_OP_SET_WINDOW, B.DGTNS_OP_ADJOINT):
            assert check_op(h, other) == (B.DGTNS_OK, ""), (args, other)
    finally:
        B.dgtns_plan_destroy(h)


def test_check_op_arguments(lib):
    h = B.dgtns_plan_create(144, 6, 12, 1, 2, 0, 4)
    try:
        assert check_op(h, 99)[0] == B.DGTNS_EINVAL
        assert check_op(h, B.DGTNS_OP_FORWARD, 0)[0] == B.DGTNS_EINVAL
        assert check_op(h, B.DGTNS_OP_FORWARD, 5)[0] == B.DGTNS_EINVAL       # above max_batch
        assert check_op(h, B.DGTNS_OP_FORWARD, 4)[0] == B.DGTNS_OK
    finally:
        B.dgtns_plan_destroy(h)
    assert lib.dgtns_check_op(None, 0, 1) == B.DGTNS_EINVAL


# the largest sizes of the GPU tests: rows of 4096 channels, columns of 4096
# values, p d at the element budgets and beyond (two-level columns)
LARGE_LATTICES = [(65536, 64, 4096, 0, 1), (65536, 16, 16, 1, 2), (32768, 8, 8, 0, 1), (65536, 64, 4096, 1, 2),
                  (131072, 64, 8192, 1, 2), (49152, 8, 12, 0, 1), (49152, 8, 12, 1, 2), (98304, 8, 12, 1, 2),
                  (36864, 12, 8, 0, 1), (73728, 12, 8, 0, 1), (1 << 20, 128, 1024, 1, 4), (262144, 64, 512, 1, 2),
                  (302400, 40, 60, 1, 4), (604800, 60, 80, 1, 5), (161280, 32, 64, 1, 2)]


def test_check_op_sweep(lib):
    """Every operation on every small feasible lattice (both precisions, the
    shear and multiwindow algorithms, FIR plans) and on the largest sizes:
    the host check either passes or refuses with DGTNS_EUNSUPPORTED, and the
    forward and adjoint transforms of shear and multiwindow plans always
    pass."""
    seen = {B.DGTNS_OK: 0, B.DGTNS_EUNSUPPORTED: 0}
    lats = feasible_lattices(max_L=72, max_lam2=3) + LARGE_LATTICES
    for lat in lats:
        for dt in (0, 1):
            for alg in (B.DGTNS_ALG_SHEAR, B.DGTNS_ALG_MULTIWINDOW, B.DGTNS_ALG_FIR):
                try:
                    if alg == B.DGTNS_ALG_FIR:
                        h = B.dgtns_plan_create_fir(*lat, dt, 3, lat[0] - 1, max(1, lat[0] // 3))
                    else:
                        h = B.dgtns_plan_create_alg(*lat, dt, 3, alg)
                except B.DgtnsError as e:
                    assert e.status in (B.DGTNS_EUNSUPPORTED, B.DGTNS_ELATTICE), (lat, alg, e)
                    continue
                try:
                    for op in OPS:
                        for batch in (1, 3):
                            st, msg = check_op(h, op, batch)
                            assert st in seen, (lat, dt, alg, op, st, msg)
                            seen[st] += 1
                            if op in (B.DGTNS_OP_FORWARD, B.DGTNS_OP_ADJOINT, B.DGTNS_OP_SET_WINDOW):
                                assert st == B.DGTNS_OK, (lat, dt, alg, op, msg)
                finally:
                    B.dgtns_plan_destroy(h)
    assert seen[B.DGTNS_OK] > 1000 and seen[B.DGTNS_EUNSUPPORTED] > 100


def test_sequential_chunk_workspace(lib, monkeypatch):
    """A forward or adjoint whose whole h would not stay in the 256 MB
    last-level cache runs in sequential chunks of about 128 MiB of h through
    one buffer: the workspace then holds one chunk (8 signals of the quincunx
    workload, 16 MiB of h each), not the batch.  DGTNS_SEQ_MIB=0 at plan
    creation turns the chunks off."""
    from dgt_inputs import LARGE as w
    per_sig = 8 * w.N * w.M
    for env, chunk_ws in ((None, True), ("0", False)):
        if env is None:
            monkeypatch.delenv("DGTNS_SEQ_MIB", raising=False)
        else:
            monkeypatch.setenv("DGTNS_SEQ_MIB", env)
        h = B.dgtns_plan_create(w.L, w.a, w.M, w.lam1, w.lam2, 0, 64)
        try:
            for op in (B.DGTNS_OP_FORWARD, B.DGTNS_OP_ADJOINT):
                ws64 = B.dgtns_workspace_bytes(h, op, 64)
                # 16 signals: 256 MiB of h, chunked; 8 signals: 128 MiB, one launch
                ws16 = B.dgtns_workspace_bytes(h, op, 16)
                ws8 = B.dgtns_workspace_bytes(h, op, 8)
                assert ws8 >= 8 * per_sig
                if chunk_ws:
                    assert 8 * per_sig <= ws64 < 9 * per_sig and ws16 == ws64, (op, ws64)
                else:
                    assert ws64 >= 64 * per_sig and ws16 >= 16 * per_sig
            # the window gradient never chunks
            assert B.dgtns_workspace_bytes(h, B.DGTNS_OP_WINDOW_GRAD, 64) >= 64 * per_sig
        finally:
            B.dgtns_plan_destroy(h)
    # FP64 plans and FP32 columns of 1024 values (one factorisation work-group
    # per compute unit) run one launch per stage
    monkeypatch.delenv("DGTNS_SEQ_MIB", raising=False)
    from dgt_inputs import PRECISION as p
    for lat, dtype, per in (((w.L, w.a, w.M, w.lam1, w.lam2), 1, 2 * per_sig),
                            ((p.L, p.a, p.M, p.lam1, p.lam2), 0, 8 * p.L * 8)):
        h = B.dgtns_plan_create(*lat, dtype, 16)
        try:
            assert B.dgtns_workspace_bytes(h, B.DGTNS_OP_FORWARD, 16) >= 16 * per
        finally:
            B.dgtns_plan_destroy(h)


def test_automatic_algorithm_choice(lib):
    """DGTNS_ALG_AUTO keeps the shear plan unless it needs a frequency shear
    and the multiwindow lattice (lambda2 a, M) has p <= 15: on the serving
    lattices the six frequency-shear ones become multiwindow plans; on the
    Fig. 2 lattices the choice follows the same rule."""
    from dgt_inputs import crossover_lattices, serving_plans
    nmw = 0
    for lat in serving_plans() + crossover_lattices():
        L, a, M, l1, l2 = lat
        hs = B.dgtns_plan_create(*lat, 0, 1)
        ha = B.dgtns_plan_create_alg(*lat, 0, 1, B.DGTNS_ALG_AUTO)
        try:
            s_branch = B.dgtns_plan_info(hs).branch
            a_branch = B.dgtns_plan_info(ha).branch
            pmw = l2 * a // math.gcd(l2 * a, M)
            want_mw = s_branch == B.DGTNS_FREQ_SHEAR and pmw <= 15
            assert a_branch == (B.DGTNS_MULTIWINDOW if want_mw else s_branch), (lat, s_branch, a_branch, pmw)
            nmw += lat in serving_plans() and want_mw
        finally:
            B.dgtns_plan_destroy(hs)
            B.dgtns_plan_destroy(ha)
    assert nmw == 6


def test_float_reciprocal_quotient_is_exact():
    """The runtime-schedule kernels divide small integers through a float
    reciprocal: for 0 <= x < 2^15 and 1 <= d <= 4096, truncating
    (x + 1/2) * fl(1/d) in IEEE single precision gives x // d exactly."""
    import numpy as np
    x = np.arange(0, 1 << 15, dtype=np.int64)
    xf = x.astype(np.float32) + np.float32(0.5)
    for d in range(1, 4097):
        inv = np.float32(1.0) / np.float32(d)
        q = (xf * inv).astype(np.int64)
        assert np.array_equal(q, x // d), d


def test_barrett_reduction_of_the_index_maps():
    """The frequency-shear index map reduces 64-bit products modulo 2N, N
    and L and divides by b, and the FIR positions reduce modulo M, lambda2
    and lambda2 M, through Barrett reduction with mu = floor((2^64 - 1) /
    m): the quotient estimate floor(x mu / 2^64) is at most 2 below
    floor(x / m), so two corrections give x mod m and x // m exactly.  The
    same steps in Python integers, on the edge cases and random dividends."""
    import random
    M64 = (1 << 64) - 1

    def mod_b(x, m, mu):
        q = (x * mu) >> 64
        r = x - q * m
        if r >= m:
            r -= m
        if r >= m:
            r -= m
        return r

    def div_b(x, m, mu):
        q = (x * mu) >> 64
        r = x - q * m
        if r >= m:
            r -= m
            q += 1
        if r >= m:
            q += 1
        return q

    rng = random.Random(13074569)
    moduli = [1, 2, 3, 7, 64, 1000, 4096, 36864, 2 * 147456, (1 << 30) - 1, 1 << 30, 2 * (1 << 30), 3 ** 19]
    for m in moduli:
        mu = M64 // m
        xs = [0, 1, m - 1, m, m + 1, 2 * m - 1, (1 << 62) - 1, (1 << 63) - 1, M64] + \
             [rng.randrange(0, 1 << 63) for _ in range(2000)]
        for x in xs:
            assert mod_b(x, m, mu) == x % m, (x, m)
            assert div_b(x, m, mu) == x // m, (x, m)
