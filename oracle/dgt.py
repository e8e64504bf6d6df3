"""Plain FP64 reference for the discrete Gabor transform on a nonseparable
lattice (test infrastructure only).

Conventions (Section 2.1, eq. (DGT)):

* ``f`` and ``g`` are complex vectors of length L; indices are taken mod L.
* The lattice is given by the time step ``a``, the number of channels ``M``
  (frequency step b = L/M) and the relative shear lambda = lam1/lam2, with
  lam1, lam2 coprime and 0 <= lam1 < lam2 (lam1 = 0 means lam2 = 1).
* The coefficient at time position n in Z_N (N = L/a) and channel m in Z_M is

      c(m, n) = sum_l f(l) conj(g(l - n a)) exp(-2 pi i l (m + w(n)) / M),
      w(n) = (n lam1 mod lam2) / lam2.

  The paper prints the window argument as ``l - an + 1``; the ``+1`` is the
  1-based indexing of its MATLAB implementation and is read here as the
  0-based ``g((l - n a) mod L)``.
* Arrays of coefficients are returned as ``c[n, m]`` (time position major,
  channel fastest), i.e. the transpose of the paper's M x N array.

Every phase is reduced exactly in integers before the exponential is taken:
with K = M lam2, exp(-2 pi i l (m + w(n)) / M) = exp(-2 pi i k / K) where
k = l (m lam2 + (n lam1 mod lam2)) mod K.
"""
from __future__ import annotations

import numpy as np


def _check(L, a, M, lam1, lam2):
    if L % a or L % M:
        raise ValueError("a and M must divide L")
    if lam2 < 1 or not (0 <= lam1 < lam2) or np.gcd(lam1, lam2) != 1:
        raise ValueError("need 0 <= lam1 < lam2 with gcd(lam1, lam2) = 1")
    if (L // M) * lam1 % lam2:
        # the absolute shear s = b lam1 / lam2 must be an integer
        raise ValueError("b * lam1 / lam2 is not an integer: not a lattice")
    if (L // a) * lam1 % lam2:
        raise ValueError("N * lam1 / lam2 is not an integer: not a lattice")


def offsets(N: int, lam1: int, lam2: int) -> np.ndarray:
    """Numerators of the frequency offsets, (n lam1 mod lam2), n in Z_N, so
    that w(n) = offsets[n] / lam2 (eq. (DGT))."""
    return (np.arange(N, dtype=np.int64) * lam1) % lam2


def _unit_root(k: np.ndarray, K: int, sign: int) -> np.ndarray:
    """exp(sign * 2 pi i k / K) for exact integers k (reduced mod K first)."""
    k = np.mod(k, K)
    return np.exp(sign * 2j * np.pi * (k.astype(np.float64) / K))


def dgt_direct(f, g, a, M, lam1, lam2):
    """Direct O(L M N) evaluation of eq. (DGT); for small L only."""
    f = np.asarray(f, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    L = f.shape[-1]
    _check(L, a, M, lam1, lam2)
    N = L // a
    K = M * lam2
    off = offsets(N, lam1, lam2)
    l = np.arange(L, dtype=np.int64)
    m = np.arange(M, dtype=np.int64)
    c = np.empty((N, M), dtype=np.complex128)
    for n in range(N):
        u = f * np.conj(np.roll(g, n * a))  # f(l) conj(g(l - n a))
        k = (l[None, :] * (m[:, None] * lam2 + off[n])) % K
        c[n] = _unit_root(k, K, -1) @ u
    return c


def dgt_fold(f, g, a, M, lam1, lam2, columns=None):
    """Per-column evaluation of eq. (DGT): modulate by the fractional offset,
    fold the L samples onto M bins, then one length-M DFT per column.

    For column n, u_n(l) = f(l) conj(g(l - n a)) exp(-2 pi i l w(n)/M); since
    exp(-2 pi i l m / M) is M-periodic in l, c(., n) is the DFT of the fold
    h_n(r) = sum_j u_n(r + j M).  The offset modulation must be applied
    before folding because it is not M-periodic.  ``columns`` restricts the
    evaluation to the given time positions (the result then has one row per
    requested column).
    """
    f = np.asarray(f, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    L = f.shape[-1]
    _check(L, a, M, lam1, lam2)
    N = L // a
    b = L // M
    K = M * lam2
    off = offsets(N, lam1, lam2)
    l = np.arange(L, dtype=np.int64)
    # one modulation vector per distinct offset numerator
    mods = [_unit_root(l * o, K, -1) for o in range(lam2)]
    cols = range(N) if columns is None else list(columns)
    c = np.empty((len(cols), M), dtype=np.complex128)
    for i, n in enumerate(cols):
        u = f * np.conj(np.roll(g, n * a)) * mods[off[n]]
        h = u.reshape(b, M).sum(axis=0)
        c[i] = np.fft.fft(h)
    return c


def dgt_separable(f, g, a, M):
    """Textbook DGT on the separable lattice aZ x bZ:
    c(m, n) = sum_l f(l) conj(g(l - n a)) exp(-2 pi i l m / M), as c[n, m]."""
    f = np.asarray(f, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    L = f.shape[-1]
    if L % a or L % M:
        raise ValueError("a and M must divide L")
    N = L // a
    b = L // M
    c = np.empty((N, M), dtype=np.complex128)
    for n in range(N):
        u = f * np.conj(np.roll(g, n * a))
        c[n] = np.fft.fft(u.reshape(b, M).sum(axis=0))
    return c


def dgt_multiwindow(f, g, a, M, lam1, lam2):
    """Multi-window route (Prop. 4, Prop. 5, eq. (mw_phases)).

    The lattice splits into lam2 cosets of the separable lattice with time
    step lam2*a and frequency step b.  With n = nt*lam2 + mu (mu = n mod lam2;
    the paper prints ``m = n - nt`` where n - lam2*nt is meant), the coset
    window is g_mu = M_{sigma} T_{mu a} g with sigma = (mu s) mod b, s = b
    lam1/lam2, and

        c(k, n) = exp(-2 pi i nt (lam2 a) sigma / L) * DGT_sep(f, g_mu; lam2 a, M)(k, nt).
    """
    f = np.asarray(f, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    L = f.shape[-1]
    _check(L, a, M, lam1, lam2)
    N = L // a
    b = L // M
    s = b * lam1 // lam2
    at = lam2 * a
    Nt = N // lam2
    l = np.arange(L, dtype=np.int64)
    c = np.empty((N, M), dtype=np.complex128)
    for mu in range(lam2):
        sigma = (mu * s) % b
        g_mu = _unit_root(l * sigma, L, +1) * np.roll(g, mu * a)
        cs = dgt_separable(f, g_mu, at, M)
        nt = np.arange(Nt, dtype=np.int64)
        phase = _unit_root(nt * at * sigma, L, -1)
        c[nt * lam2 + mu] = phase[:, None] * cs
    return c


def idgt_adjoint(c, g, a, M, lam1, lam2, samples=None):
    """Adjoint (synthesis) operator of eq. (DGT):
    f(l) = sum_{m,n} c(m, n) g(l - n a) exp(+2 pi i l (m + w(n)) / M).

    Per column: y_n(l) = sum_m c(m, n) exp(2 pi i l (m + w(n))/M) is an
    M-periodic inverse DFT times the offset modulation, then the windowed
    columns are summed.  ``samples`` restricts the evaluation to the given
    sample indices l (the result then has one value per requested sample);
    each value is the same sum over all N columns."""
    c = np.asarray(c, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    N, M_ = c.shape
    if M_ != M:
        raise ValueError("coefficient array must be (N, M)")
    L = N * a
    _check(L, a, M, lam1, lam2)
    b = L // M
    K = M * lam2
    off = offsets(N, lam1, lam2)
    if samples is not None:
        l = np.asarray(samples, dtype=np.int64)
        y = M * np.fft.ifft(c, axis=1)           # y[n, r] = sum_m c(m, n) e^{2 pi i r m / M}
        mods = [_unit_root(l * o, K, +1) for o in range(lam2)]
        f = np.zeros(len(l), dtype=np.complex128)
        for n in range(N):
            f += g[(l - n * a) % L] * y[n, l % M] * mods[off[n]]
        return f
    l = np.arange(L, dtype=np.int64)
    mods = [_unit_root(l * o, K, +1) for o in range(lam2)]
    f = np.zeros(L, dtype=np.complex128)
    for n in range(N):
        y = np.tile(M * np.fft.ifft(c[n]), b) * mods[off[n]]
        f += np.roll(g, n * a) * y
    return f


def coefficient_frequencies(N, M, b, lam1, lam2):
    """Integer frequency (in Z_L) of coefficient (m, n): b m + (n s mod b),
    the lattice frequencies of column n counted upward from the lowest
    non-negative one (eq. (DGT)); returned as an (N, M) int64 array."""
    off = offsets(N, lam1, lam2)
    sigma = (b * off) // lam2
    return np.arange(M, dtype=np.int64)[None, :] * b + sigma[:, None]
