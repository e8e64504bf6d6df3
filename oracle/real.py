"""Real-signal variant of the DGT (test infrastructure only).

Section 4.4 names two entry points of the toolbox the algorithms live in,
one for complex and one for real signals (``dgtreal``), without specifying
the second.  Reading (documented with the other readings of the paper):
for a real signal f and a real window g, complex conjugation of eq. (DGT)
gives

    conj(c(m, n)) = sum_l f(l) g(l - n a) exp(+2 pi i l (m + w(n)) / M),

which is the coefficient of frequency -(m + w(n)) at time position n.  That
frequency lies on the lattice column n exactly when e(n) = 2 w(n) is an
integer (w(n) in {0, 1/2}); then

    c((-m - e(n)) mod M, n) = conj(c(m, n)),

and channels 0 .. floor(M/2) determine the whole column.  Columns with any
other offset are not redundant and are kept whole.  Since w(n) depends on
n mod lam2 only, the symmetric columns are those with n = 0 (mod lam2) and,
for even lam2, n = lam2/2 (mod lam2).

Layout of the real-signal coefficients of one signal: the N columns are
grouped by j = n div lam2 into N/lam2 rows of S values; column
n = j lam2 + k sits at j S + off(k) and holds count(k) channels 0 .. count(k)-1,
count(k) = floor(M/2) + 1 for the symmetric residues k, M otherwise.  For
lam2 <= 2 this is an (N, floor(M/2) + 1) array, as on a separable lattice.

The synthesis of real-signal coefficients expands them to the full array
(the omitted channels of a symmetric column are the conjugates of stored
ones) and returns the real part of the adjoint of eq. (DGT).  With the
canonical dual window this inverts the real-signal transform.
"""
from __future__ import annotations

import numpy as np

from .dgt import dgt_fold, idgt_adjoint, offsets


def real_layout(M: int, lam1: int, lam2: int):
    """(S, off, count, e) of the real-signal layout: values per group of lam2
    columns, offset and stored channel count of residue k = n mod lam2, and
    e(k) = 2 w(k) for the symmetric residues (None for the others)."""
    w2 = 2 * offsets(lam2, lam1, lam2)            # 2 (k lam1 mod lam2), k in Z_lam2
    e = [int(x // lam2) if x % lam2 == 0 else None for x in w2]
    count = [M // 2 + 1 if ek is not None else M for ek in e]
    off = np.concatenate([[0], np.cumsum(count)]).astype(np.int64)
    return int(off[-1]), off[:-1], count, e


def pack_real(c, M: int, lam1: int, lam2: int):
    """Real-signal layout (N/lam2, S) of a full coefficient array c[n, m]:
    channels 0 .. count(n mod lam2) - 1 of every column."""
    c = np.asarray(c)
    N = c.shape[0]
    S, off, count, _ = real_layout(M, lam1, lam2)
    out = np.empty((N // lam2, S), dtype=c.dtype)
    for n in range(N):
        j, k = divmod(n, lam2)
        out[j, off[k]:off[k] + count[k]] = c[n, :count[k]]
    return out


def unpack_real(cr, N: int, M: int, lam1: int, lam2: int):
    """Full array c[n, m] from real-signal coefficients: a symmetric column's
    channel m >= count holds conj(c((-m - e) mod M, n))."""
    cr = np.asarray(cr, dtype=np.complex128)
    S, off, count, e = real_layout(M, lam1, lam2)
    c = np.empty((N, M), dtype=np.complex128)
    for n in range(N):
        j, k = divmod(n, lam2)
        col = cr[j, off[k]:off[k] + count[k]]
        c[n, :count[k]] = col
        if count[k] < M:
            m = np.arange(count[k], M)
            c[n, count[k]:] = np.conj(col[(-m - e[k]) % M])
    return c


def dgtreal(f, g, a, M, lam1, lam2):
    """Coefficients of eq. (DGT) of a real signal f with a real window g, in
    the real-signal layout (N/lam2, S)."""
    f = np.asarray(f)
    g = np.asarray(g)
    if np.iscomplexobj(f) and np.any(np.imag(f)):
        raise ValueError("dgtreal needs a real signal")
    if np.iscomplexobj(g) and np.any(np.imag(g)):
        raise ValueError("dgtreal needs a real window")
    return pack_real(dgt_fold(np.real(f), np.real(g), a, M, lam1, lam2), M, lam1, lam2)


def idgtreal(cr, g, a, M, lam1, lam2, N=None, samples=None):
    """Real part of the synthesis (adjoint of eq. (DGT)) of the expanded
    real-signal coefficients cr (N/lam2, S); any window g."""
    cr = np.asarray(cr)
    if N is None:
        N = cr.shape[0] * lam2
    c = unpack_real(cr, N, M, lam1, lam2)
    return np.real(idgt_adjoint(c, g, a, M, lam1, lam2, samples=samples))
