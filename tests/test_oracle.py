"""Pins of the CPU oracle against things other than itself: brute force over
the lattice points with explicit time-frequency shift operators, full-length
library FFTs, closed forms, the multi-window identity, adjointness, the dense
frame operator, finite differences and torch autograd."""
import math

import numpy as np
import pytest

import oracle
from dgt_inputs import complex_normal, gaussian_window
from tests.conftest import DEGENERATE_LATTICES, feasible_lattices

RNG = np.random.default_rng(20240611)


def rand_c(*shape):
    return (RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)) / math.sqrt(2)


def rel(x, y):
    return float(np.linalg.norm(np.ravel(x - y)) / max(np.linalg.norm(np.ravel(y)), 1e-300))


# ---------------------------------------------------------------------------
# Brute force: enumerate the lattice A Z_L^2 with A = [[a, 0], [s, b]]
# (Prop. 1), build each atom M_omega T_x g from the operator definitions
# (Section 2.1) and index the frequencies of each time position upward from
# the lowest non-negative one (eq. (DGT)).
# ---------------------------------------------------------------------------

def lattice_points(L, a, M, lam1, lam2):
    b = L // M
    s = b * lam1 // lam2
    pts = set()
    for k1 in range(L):
        for k2 in range(L // b + 1):
            pts.add(((a * k1) % L, (s * k1 + b * k2) % L))
    return pts


def brute_force_atoms(g, L, a, M, lam1, lam2):
    """Matrix whose column (n, m) is the atom M_omega T_{na} g, with omega the
    m-th smallest lattice frequency above time position n a."""
    pts = lattice_points(L, a, M, lam1, lam2)
    N = L // a
    assert len(pts) == L * L // (a * (L // M))  # |Lambda| = L^2/(ab)
    l = np.arange(L)
    T = lambda x: np.eye(L)[(l - x) % L]               # (T_x f)(l) = f(l - x)
    Mo = lambda w: np.diag(np.exp(2j * np.pi * l * w / L))
    atoms = np.zeros((L, N, M), dtype=np.complex128)
    for n in range(N):
        freqs = sorted(w for (x, w) in pts if x == (n * a) % L)
        assert len(freqs) == M
        for m, w in enumerate(freqs):
            atoms[:, n, m] = Mo(w) @ (T(n * a) @ g)
    return atoms


FIG1 = [(36, 6, 6, 0, 1), (36, 6, 6, 1, 2), (36, 6, 6, 1, 3), (36, 6, 6, 2, 3)]
SMALL_LATTICES = FIG1 + [(16, 4, 8, 1, 2), (60, 5, 6, 1, 2), (72, 6, 4, 1, 3),
                         (64, 4, 8, 1, 4), (24, 2, 6, 1, 2), (144, 6, 12, 1, 2)]


@pytest.mark.parametrize("lat", SMALL_LATTICES)
def test_direct_and_fold_match_brute_force(lat):
    L, a, M, l1, l2 = lat
    f, g = rand_c(L), rand_c(L)
    A = brute_force_atoms(g, L, a, M, l1, l2)
    c_bf = np.einsum("l,lnm->nm", f, np.conj(A))       # <f, atom>
    assert rel(oracle.dgt_direct(f, g, a, M, l1, l2), c_bf) < 1e-13
    assert rel(oracle.dgt_fold(f, g, a, M, l1, l2), c_bf) < 1e-13
    assert rel(oracle.dgt_multiwindow(f, g, a, M, l1, l2), c_bf) < 1e-13


@pytest.mark.parametrize("lat", DEGENERATE_LATTICES)
def test_degenerate_lattices_match_brute_force(lat):
    """One time position, one channel, a = 1, M = L and L = 1: both
    evaluation orders against the explicit atoms, and the adjoint identity."""
    L, a, M, l1, l2 = lat
    f, g = rand_c(L), rand_c(L)
    A = brute_force_atoms(g, L, a, M, l1, l2)
    c_bf = np.einsum("l,lnm->nm", f, np.conj(A))
    assert rel(oracle.dgt_direct(f, g, a, M, l1, l2), c_bf) < 1e-13
    assert rel(oracle.dgt_fold(f, g, a, M, l1, l2), c_bf) < 1e-13
    c = rand_c(L // a * M).reshape(L // a, M)
    fa = oracle.idgt_adjoint(c, g, a, M, l1, l2)
    assert rel(fa, np.einsum("nm,lnm->l", c, A)) < 1e-13


def test_plus_one_reading_is_rejected():
    """The window argument read literally as l - a n + 1 disagrees with the
    brute-force STFT samples; the 0-based reading l - a n agrees."""
    L, a, M, l1, l2 = 36, 6, 6, 1, 2
    f, g = rand_c(L), rand_c(L)
    c_bf = np.einsum("l,lnm->nm", f, np.conj(brute_force_atoms(g, L, a, M, l1, l2)))
    shifted = np.roll(g, -1)  # shifted(x) = g(x + 1), so shifted(l - a n) = g(l - a n + 1)
    assert rel(oracle.dgt_fold(f, shifted, a, M, l1, l2), c_bf) > 0.1


def test_frequency_index_matches_lattice():
    for (L, a, M, l1, l2) in SMALL_LATTICES:
        pts = lattice_points(L, a, M, l1, l2)
        N, b = L // a, L // M
        fr = oracle.coefficient_frequencies(N, M, b, l1, l2)
        for n in range(N):
            assert sorted(w for (x, w) in pts if x == n * a % L) == list(fr[n])


@pytest.mark.parametrize("lat", feasible_lattices(max_L=48, max_lam2=4)[::7])
def test_fold_equals_full_length_fft_samples(lat):
    """c(m, n) is the STFT sample V_g f(n a, b m + sigma_n); each column of the
    STFT is a length-L library FFT of the windowed signal."""
    L, a, M, l1, l2 = lat
    f, g = rand_c(L), rand_c(L)
    N, b = L // a, L // M
    fr = oracle.coefficient_frequencies(N, M, b, l1, l2)
    ref = np.empty((N, M), dtype=np.complex128)
    for n in range(N):
        ref[n] = np.fft.fft(f * np.conj(np.roll(g, n * a)))[fr[n]]
    assert rel(oracle.dgt_fold(f, g, a, M, l1, l2), ref) < 1e-13
    assert rel(oracle.dgt_multiwindow(f, g, a, M, l1, l2), ref) < 1e-13


def test_separable_is_subsampled_stft():
    for (L, a, M) in [(48, 4, 12), (60, 6, 10), (64, 1, 64), (30, 5, 6)]:
        f, g = rand_c(L), rand_c(L)
        N, b = L // a, L // M
        ref = np.array([np.fft.fft(f * np.conj(np.roll(g, n * a)))[::b] for n in range(N)])
        assert rel(oracle.dgt_separable(f, g, a, M), ref) < 1e-13


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lat", SMALL_LATTICES)
def test_closed_forms(lat):
    L, a, M, l1, l2 = lat
    N, b = L // a, L // M
    f = rand_c(L)
    sig = (b * oracle.offsets(N, l1, l2)) // l2
    n = np.arange(N)[:, None]
    m = np.arange(M)[None, :]
    # g = delta_0: c(m, n) = f(n a) exp(-2 pi i n a (b m + sigma_n) / L)
    delta = np.zeros(L, complex)
    delta[0] = 1
    ref = f[(n * a) % L] * np.exp(-2j * np.pi * (((n * a) * (b * m + sig[:, None])) % L) / L)
    assert rel(oracle.dgt_fold(f, delta, a, M, l1, l2), ref) < 1e-13
    # g constant 1/sqrt(L): c(m, n) = fhat(b m + sigma_n) / sqrt(L)
    const = np.full(L, 1 / math.sqrt(L), complex)
    ref = np.fft.fft(f)[b * m + sig[:, None]] / math.sqrt(L)
    assert rel(oracle.dgt_fold(f, const, a, M, l1, l2), ref) < 1e-13
    # f = delta_{l0}: c(m, n) = conj(g(l0 - n a)) exp(-2 pi i l0 (b m + sigma_n) / L)
    g = rand_c(L)
    l0 = L // 3
    d = np.zeros(L, complex)
    d[l0] = 1
    ref = np.conj(g[(l0 - n * a) % L]) * np.exp(-2j * np.pi * ((l0 * (b * m + sig[:, None])) % L) / L)
    assert rel(oracle.dgt_fold(d, g, a, M, l1, l2), ref) < 1e-13


def test_lattice_covariance():
    """Shifting the signal by a lattice point (a, s) permutes coefficients:
    c_{M_s T_a f}(m, n) = exp(-2 pi i a (b m' + sigma_{n-1}) / L) c_f(m', n-1)
    with m' = m + (sigma_n - s - sigma_{n-1}) / b mod M."""
    for (L, a, M, l1, l2) in SMALL_LATTICES:
        N, b = L // a, L // M
        s = b * l1 // l2
        f, g = rand_c(L), rand_c(L)
        l = np.arange(L)
        fs = np.exp(2j * np.pi * (l * s % L) / L) * np.roll(f, a)
        c0 = oracle.dgt_fold(f, g, a, M, l1, l2)
        c1 = oracle.dgt_fold(fs, g, a, M, l1, l2)
        sig = (b * oracle.offsets(N, l1, l2)) // l2
        for n in range(N):
            nm = (n - 1) % N
            dm = sig[n] - s - sig[nm]
            assert dm % b == 0
            mp = (np.arange(M) + dm // b) % M
            ph = np.exp(-2j * np.pi * ((a * (b * mp + sig[nm])) % L) / L)
            assert rel(c1[n], ph * c0[nm, mp]) < 1e-12


# ---------------------------------------------------------------------------
# Adjoint, frame operator, dual window
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lat", SMALL_LATTICES)
def test_adjoint(lat):
    L, a, M, l1, l2 = lat
    N = L // a
    g = rand_c(L)
    A = brute_force_atoms(g, L, a, M, l1, l2)
    c = rand_c(N, M)
    ref = np.einsum("lnm,nm->l", A, c)          # synthesis = sum c(m,n) atom
    assert rel(oracle.idgt_adjoint(c, g, a, M, l1, l2), ref) < 1e-13
    # the evaluation at chosen samples (any order, repeats allowed) against
    # the same brute-force synthesis
    pts = RNG.integers(0, L, size=L // 2 + 3)
    assert rel(oracle.idgt_adjoint(c, g, a, M, l1, l2, samples=pts), ref[pts]) < 1e-13
    f = rand_c(L)
    lhs = np.vdot(c, oracle.dgt_fold(f, g, a, M, l1, l2))       # <Cf, c>^*
    rhs = np.vdot(oracle.idgt_adjoint(c, g, a, M, l1, l2), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("lat", SMALL_LATTICES)
def test_frame_operator_and_dual(lat):
    L, a, M, l1, l2 = lat
    g = gaussian_window(L, a, M)
    A = brute_force_atoms(g, L, a, M, l1, l2).reshape(L, -1)
    S = A @ A.conj().T                          # dense frame operator
    b = L // M
    blocks = oracle.frame_blocks(g, a, M, l1, l2)
    i = np.arange(b)
    for r in range(M):
        assert np.allclose(blocks[r], S[np.ix_(r + i * M, r + i * M)], atol=1e-13)
    x = rand_c(L)
    assert rel(oracle.frame_operator_apply(x, g, a, M, l1, l2), S @ x) < 1e-13
    ev = np.linalg.eigvalsh(S)
    lo, hi = oracle.frame_bounds(g, a, M, l1, l2)
    assert abs(lo - ev.min()) < 1e-10 * ev.max() and abs(hi - ev.max()) < 1e-10 * ev.max()
    if lo < 1e-8 * hi:
        return  # not a frame (redundancy 1 lattices can be singular)
    gd = oracle.dual_window(g, a, M, l1, l2)
    assert rel(S @ gd, g) < 1e-12
    f = rand_c(L)
    rec = oracle.idgt_adjoint(oracle.dgt_fold(f, g, a, M, l1, l2), gd, a, M, l1, l2)
    assert rel(rec, f) < 1e-11
    # ||C f||^2 = <S f, f>
    c = oracle.dgt_fold(f, g, a, M, l1, l2)
    assert abs(np.vdot(c, c).real - np.vdot(f, S @ f).real) < 1e-11 * np.vdot(c, c).real


@pytest.mark.parametrize("lat", SMALL_LATTICES)
def test_tight_window(lat):
    """Canonical tight window S^{-1/2} g: its Gabor system is a tight frame
    with bound 1 (dense frame operator from brute-force atoms is the
    identity), and it equals S^{-1/2} g computed from the dense L x L frame
    operator (no Walnut blocks)."""
    L, a, M, l1, l2 = lat
    g = gaussian_window(L, a, M) + 0.2j * rand_c(L)
    A = brute_force_atoms(g, L, a, M, l1, l2).reshape(L, -1)
    S = A @ A.conj().T
    ev, V = np.linalg.eigh(S)
    if ev.min() < 1e-8 * ev.max():
        with pytest.raises(ValueError):
            oracle.tight_window(g, a, M, l1, l2)
        return
    gt = oracle.tight_window(g, a, M, l1, l2)
    At = brute_force_atoms(gt, L, a, M, l1, l2).reshape(L, -1)
    assert np.abs(At @ At.conj().T - np.eye(L)).max() < 1e-12
    dense = V @ ((V.conj().T @ g) / np.sqrt(ev))
    assert rel(gt, dense) < 1e-12
    # painless reconstruction with the tight window alone
    f = rand_c(L)
    assert rel(oracle.idgt_adjoint(oracle.dgt_fold(f, gt, a, M, l1, l2), gt, a, M, l1, l2), f) < 1e-11


def test_painless_tight_closed_form():
    """Separable lattice, window supported in [0, M): S is diagonal with
    entries M sum_n |g(l - n a)|^2, so the tight window is g / sqrt of it."""
    L, a, M = 48, 4, 12
    g = np.zeros(L, complex)
    g[:M] = RNG.uniform(0.5, 1.5, M) + 0.3j * RNG.uniform(-1, 1, M)
    diag = M * sum(np.abs(np.roll(g, n * a)) ** 2 for n in range(L // a))
    assert rel(oracle.tight_window(g, a, M, 0, 1), g / np.sqrt(diag)) < 1e-13


def test_painless_dual_closed_form():
    """Separable lattice and a window supported in [0, M): S is diagonal with
    entries M sum_n |g(l - n a)|^2, so the dual is g / that diagonal."""
    L, a, M = 48, 4, 12
    g = np.zeros(L, complex)
    g[:M] = RNG.uniform(0.5, 1.5, M) + 0.3j * RNG.uniform(-1, 1, M)
    diag = M * sum(np.abs(np.roll(g, n * a)) ** 2 for n in range(L // a))
    assert rel(oracle.dual_window(g, a, M, 0, 1), g / diag) < 1e-13


# ---------------------------------------------------------------------------
# Gradients
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lat", [(36, 6, 6, 1, 2), (72, 6, 4, 1, 3), (64, 4, 8, 1, 4)])
def test_gradients_finite_differences(lat):
    L, a, M, l1, l2 = lat
    f, g = rand_c(L), rand_c(L)
    T = np.abs(oracle.dgt_fold(rand_c(L), g, a, M, l1, l2)) ** 2
    loss0, gf, gg = oracle.loss_and_grads(f, g, T, a, M, l1, l2)
    h = 1e-6
    for _ in range(4):
        d = rand_c(L)
        lp = oracle.loss_and_grads(f + h * d, g, T, a, M, l1, l2)[0]
        lm = oracle.loss_and_grads(f - h * d, g, T, a, M, l1, l2)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.vdot(gf, d).real) < 1e-6 * max(1.0, abs(fd))
        lp = oracle.loss_and_grads(f, g + h * d, T, a, M, l1, l2)[0]
        lm = oracle.loss_and_grads(f, g - h * d, T, a, M, l1, l2)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.vdot(gg, d).real) < 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("lat", [(36, 6, 6, 1, 2), (72, 6, 4, 1, 3), (64, 4, 8, 1, 4), (48, 4, 6, 0, 1)])
def test_window_gradient_at_points_matches_the_whole_gradient(lat):
    """The sampled form of the window gradient (used at sizes where the
    whole one is too slow) agrees with the whole gradient, which the finite
    differences and the dense-atom autograd pin."""
    L, a, M, l1, l2 = lat
    f = rand_c(L)
    G = rand_c(L // a * M).reshape(L // a, M)
    whole = oracle.window_gradient(f, G, a, M, l1, l2)
    pts = np.array([0, 1, L // 3, L - 1], dtype=np.int64)
    assert rel(oracle.window_gradient(f, G, a, M, l1, l2, points=pts), whole[pts]) < 1e-13
    assert rel(oracle.window_gradient(f, G, a, M, l1, l2, points=np.arange(L)), whole) < 1e-13


def test_gradients_match_torch_autograd_on_dense_atoms():
    torch = pytest.importorskip("torch")
    L, a, M, l1, l2 = 36, 6, 6, 1, 3
    f, g = rand_c(L), rand_c(L)
    T = np.abs(oracle.dgt_fold(rand_c(L), g, a, M, l1, l2)) ** 2
    _, gf, gg = oracle.loss_and_grads(f, g, T, a, M, l1, l2)
    # coefficients as an explicit sum over lattice points: c = sum_l f(l) conj(atom(l))
    pts = sorted(lattice_points(L, a, M, l1, l2))
    ft = torch.tensor(f, requires_grad=True)
    gt = torch.tensor(g, requires_grad=True)
    l = torch.arange(L)
    Tt = torch.tensor(T)
    loss = 0
    N = L // a
    for n in range(N):
        freqs = sorted(w for (x, w) in pts if x == n * a)
        shifted = gt[(l - n * a) % L]
        for m, w in enumerate(freqs):
            mod = torch.exp(2j * math.pi * ((l * w) % L).double() / L)
            c = torch.sum(ft * torch.conj(mod * shifted))
            loss = loss + (c.abs() ** 2 - Tt[n, m]) ** 2
    loss.backward()
    assert rel(ft.grad.numpy(), gf) < 1e-12
    assert rel(gt.grad.numpy(), gg) < 1e-12


# ---------------------------------------------------------------------------
# Sweep: the three evaluation orders agree on every feasible small lattice
# ---------------------------------------------------------------------------

def test_sweep_orders_agree():
    lats = feasible_lattices(max_L=40, max_lam2=4)
    assert len(lats) > 200
    for (L, a, M, l1, l2) in lats[::3]:
        f, g = rand_c(L), rand_c(L)
        c1 = oracle.dgt_direct(f, g, a, M, l1, l2)
        assert rel(oracle.dgt_fold(f, g, a, M, l1, l2), c1) < 1e-12
        assert rel(oracle.dgt_multiwindow(f, g, a, M, l1, l2), c1) < 1e-12


def test_small_workload_shape():
    from dgt_inputs import SMALL
    f = complex_normal(SMALL.L, 1)
    g = gaussian_window(SMALL.L, SMALL.a, SMALL.M)
    c = oracle.dgt_fold(f, g, SMALL.a, SMALL.M, SMALL.lam1, SMALL.lam2)
    assert c.shape == (24, 12)
    assert abs(np.linalg.norm(g) - 1) < 1e-14


# ---------------------------------------------------------------------------
# Real-signal variant: conjugate symmetry of the columns with w(n) in {0, 1/2}
# ---------------------------------------------------------------------------

REAL_LATTICES = [(36, 6, 6, 0, 1), (36, 6, 6, 1, 2), (36, 6, 6, 1, 3), (36, 6, 6, 2, 3), (64, 4, 8, 1, 4),
                 (60, 5, 6, 1, 2), (72, 6, 4, 1, 3), (144, 6, 12, 1, 2), (60, 6, 5, 1, 2), (72, 4, 9, 1, 2),
                 (144, 4, 9, 1, 4), (64, 2, 8, 3, 4)]


@pytest.mark.parametrize("lat", REAL_LATTICES)
def test_real_signal_symmetry_from_atoms(lat):
    """For a real signal and a real window, the explicit atoms give
    c((-m - e) mod M, n) = conj(c(m, n)) in every column whose offset w(n) is
    0 or 1/2 (e = 2 w(n)), and not in the other columns; the layout keeps
    exactly the channels that determine each column (even and odd M)."""
    from oracle.real import real_layout
    L, a, M, l1, l2 = lat
    f, g = RNG.standard_normal(L), RNG.standard_normal(L)
    A = brute_force_atoms(g.astype(np.complex128), L, a, M, l1, l2)
    c = np.einsum("l,lnm->nm", f, np.conj(A))
    N = L // a
    S, off, count, e = real_layout(M, l1, l2)
    nsym = 0
    for n in range(N):
        k = n % l2
        w2 = (2 * ((n * l1) % l2))
        m = np.arange(M)
        if w2 % l2 == 0:
            nsym += 1
            assert e[k] == w2 // l2 and count[k] == M // 2 + 1
            assert np.allclose(c[n, (-m - e[k]) % M], np.conj(c[n]), atol=1e-12)
            # every orbit {m, -m - e} has a member among the stored channels
            assert set(np.minimum(m, (-m - e[k]) % M)) <= set(range(count[k]))
        else:
            assert e[k] is None and count[k] == M
            # the negated frequencies are off the lattice: no symmetry
            assert not np.allclose(c[n, (-m) % M], np.conj(c[n]), atol=1e-6)
            assert not np.allclose(c[n, (-m - 1) % M], np.conj(c[n]), atol=1e-6)
    assert S == sum(count) and nsym == N // l2 * (1 + (l2 % 2 == 0))


@pytest.mark.parametrize("lat", REAL_LATTICES)
def test_real_signal_pack_unpack_and_synthesis(lat):
    """The stored channels determine the transform of a real signal (unpack
    restores the brute-force coefficients); the synthesis of real-signal
    coefficients is the adjoint of the transform under the real inner
    product (Re <C f, E c> = <f, synthesis(c)> with E the expansion); with
    the canonical dual window it reconstructs the signal."""
    from oracle.real import dgtreal, idgtreal, pack_real, real_layout, unpack_real
    L, a, M, l1, l2 = lat
    N = L // a
    f, g = RNG.standard_normal(L), RNG.standard_normal(L)
    A = brute_force_atoms(g.astype(np.complex128), L, a, M, l1, l2)
    c_bf = np.einsum("l,lnm->nm", f, np.conj(A))
    cr = dgtreal(f, g, a, M, l1, l2)
    S, off, count, e = real_layout(M, l1, l2)
    assert cr.shape == (N // l2, S)
    assert rel(unpack_real(cr, N, M, l1, l2), c_bf) < 1e-13
    assert np.array_equal(pack_real(unpack_real(cr, N, M, l1, l2), M, l1, l2), cr)
    # adjoint under the real inner product, against the explicit atoms
    z = rand_c(N // l2, S)
    lhs = np.real(np.vdot(c_bf, unpack_real(z, N, M, l1, l2)))
    synth = np.real(np.einsum("lnm,nm->l", A, unpack_real(z, N, M, l1, l2)))
    assert rel(idgtreal(z, g, a, M, l1, l2), synth) < 1e-13
    assert abs(lhs - np.dot(f, idgtreal(z, g, a, M, l1, l2))) < 1e-12 * abs(lhs) + 1e-12
    # reconstruction through the canonical dual window (frame lattices only)
    if L * L // (a * (L // M)) >= L:
        gd = oracle.dual_window(g.astype(np.complex128), a, M, l1, l2)
        if np.all(np.isfinite(gd)):
            assert rel(idgtreal(cr, gd, a, M, l1, l2), f) < 1e-10


def test_real_layout_separable_and_quincunx_shapes():
    """lam2 <= 2: an (N, floor(M/2) + 1) array; lam2 = 4 (the precision
    workload's lattice): two half and two whole columns per group of four."""
    from oracle.real import real_layout
    assert real_layout(12, 0, 1)[0] == 7
    assert real_layout(12, 1, 2)[0] == 14
    assert real_layout(1024, 1, 4)[0] == 2 * 513 + 2 * 1024
    assert real_layout(9, 1, 3)[0] == 5 + 9 + 9
    S, off, count, e = real_layout(1024, 1, 4)
    assert list(count) == [513, 1024, 513, 1024] and e == [0, None, 1, None] and list(off) == [0, 513, 1537, 2050]
