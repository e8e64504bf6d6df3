"""Plain FP64 reference for the frame operator and the canonical dual window
(test infrastructure only).

The frame operator of the Gabor system on the lattice (eq. (frameop),
Section 2.1) is S f = sum_{m,n} <f, g_{m,n}> g_{m,n} with atoms
g_{m,n}(l) = g(l - n a) exp(2 pi i l (m + w(n)) / M).  Summing over the
channel index m first gives M times the indicator of l = l' mod M, so S only
couples samples that are a multiple of M apart (Walnut form):

    (S f)(l) = sum_{j in Z_b} W_j(l) f(l - j M),
    W_j(l)   = M sum_n exp(2 pi i j (n lam1 mod lam2)/lam2) g(l - n a) conj(g(l - n a - j M)).

For every r in Z_M this is a b x b matrix acting on the samples
f(r), f(r + M), ..., f(r + (b-1) M): S_r[i, i'] = W_{(i - i') mod b}(r + i M).
The canonical dual window is S^{-1} g (Section 2.1), obtained here by one
dense FP64 solve per block, and the canonical tight window S^{-1/2} g
(Section 4.2) by the inverse square root of each Hermitian block.
"""
from __future__ import annotations

import numpy as np

from .dgt import _check, offsets


def walnut_weights(g, a, M, lam1, lam2, points=None):
    """W_j(l) for j in Z_b and l in ``points`` (default: all of Z_L); returns
    an array of shape (b, len(points))."""
    g = np.asarray(g, dtype=np.complex128)
    L = g.shape[-1]
    _check(L, a, M, lam1, lam2)
    N = L // a
    b = L // M
    pts = np.arange(L, dtype=np.int64) if points is None else np.asarray(points, dtype=np.int64)
    off = offsets(N, lam1, lam2)
    n = np.arange(N, dtype=np.int64)
    j = np.arange(b, dtype=np.int64)
    # phase exp(2 pi i j off_n / lam2), exact in integers
    ph = np.exp(2j * np.pi * (((j[:, None] * off[None, :]) % lam2) / lam2))  # (b, N)
    W = np.empty((b, len(pts)), dtype=np.complex128)
    for i, l in enumerate(pts):
        g1 = g[(l - n * a) % L]                                   # (N,)
        g2 = g[(l - n[None, :] * a - j[:, None] * M) % L]         # (b, N)
        W[:, i] = M * np.sum(ph * g1[None, :] * np.conj(g2), axis=1)
    return W


def frame_blocks(g, a, M, lam1, lam2):
    """The M Walnut blocks S_r (array of shape (M, b, b))."""
    g = np.asarray(g, dtype=np.complex128)
    L = g.shape[-1]
    b = L // M
    W = walnut_weights(g, a, M, lam1, lam2)         # (b, L)
    i = np.arange(b)
    S = np.empty((M, b, b), dtype=np.complex128)
    for r in range(M):
        rows = r + i * M
        S[r] = W[(i[:, None] - i[None, :]) % b, rows[:, None]]
    return S


def frame_operator_apply(x, g, a, M, lam1, lam2, points=None):
    """(S x)(l) at the given points via the Walnut form."""
    x = np.asarray(x, dtype=np.complex128)
    L = x.shape[-1]
    b = L // M
    pts = np.arange(L, dtype=np.int64) if points is None else np.asarray(points, dtype=np.int64)
    W = walnut_weights(g, a, M, lam1, lam2, pts)
    j = np.arange(b, dtype=np.int64)
    xs = x[(pts[None, :] - j[:, None] * M) % L]
    return np.sum(W * xs, axis=0)


def dual_window(g, a, M, lam1, lam2):
    """Canonical dual window S^{-1} g (one dense solve per Walnut block).
    Raises numpy.linalg.LinAlgError if a block is singular (not a frame)."""
    g = np.asarray(g, dtype=np.complex128)
    L = g.shape[-1]
    b = L // M
    S = frame_blocks(g, a, M, lam1, lam2)
    gd = np.empty(L, dtype=np.complex128)
    i = np.arange(b)
    for r in range(M):
        gd[r + i * M] = np.linalg.solve(S[r], g[r + i * M])
    return gd


def tight_window(g, a, M, lam1, lam2):
    """Canonical tight window S^{-1/2} g: each Walnut block is Hermitian
    positive definite for a frame, S_r = V diag(ev) V^H, and its inverse
    square root is V diag(ev^{-1/2}) V^H.  Raises ValueError if a block is
    singular (not a frame)."""
    g = np.asarray(g, dtype=np.complex128)
    L = g.shape[-1]
    b = L // M
    S = frame_blocks(g, a, M, lam1, lam2)
    gt = np.empty(L, dtype=np.complex128)
    i = np.arange(b)
    for r in range(M):
        ev, V = np.linalg.eigh(S[r])
        if ev.min() <= 1e-14 * max(ev.max(), 1e-300):
            raise ValueError("frame operator is singular: no tight window")
        gt[r + i * M] = V @ ((V.conj().T @ g[r + i * M]) / np.sqrt(ev))
    return gt


def frame_bounds(g, a, M, lam1, lam2):
    """Optimal frame bounds (smallest and largest eigenvalue of S)."""
    S = frame_blocks(g, a, M, lam1, lam2)
    ev = np.linalg.eigvalsh(S)
    return float(ev.min()), float(ev.max())
