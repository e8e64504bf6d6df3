"""Plain FP64 reference gradients of a spectrogram-matching loss
(test infrastructure only).

Gradients follow the convention of complex autograd: for a real loss l of a
complex variable z the gradient is dl/dRe(z) + i dl/dIm(z), so that the first
order change is dl = Re(sum conj(grad) dz).

For c = C_g f (eq. (DGT)):

* grad_f = C_g^* grad_c, because c is linear in f;
* c is conjugate-linear in g; writing y_n(l) = sum_m grad_c(m, n)
  exp(2 pi i l (m + w(n)) / M), the change of the loss is
  Re sum_{n,l} f(l) conj(dg(l - n a)) conj(y_n(l)), hence
  grad_g(j) = sum_n f(j + n a) conj(y_n(j + n a)).
"""
from __future__ import annotations

import numpy as np

from .dgt import _check, _unit_root, dgt_fold, idgt_adjoint, offsets


def spectrogram_loss(c, T):
    """sum (|c|^2 - T)^2 and its gradient with respect to c."""
    p = np.abs(c) ** 2 - T
    return float(np.sum(p * p)), 4.0 * p * c


def window_gradient(f, G, a, M, lam1, lam2, points=None):
    """grad_g(j) = sum_n f(j + n a) conj(y_n(j + n a)) for a coefficient
    gradient G given as G[n, m]; at the time positions ``points`` only if
    given (each position then costs N M instead of the whole L N)."""
    f = np.asarray(f, dtype=np.complex128)
    G = np.asarray(G, dtype=np.complex128)
    L = f.shape[-1]
    _check(L, a, M, lam1, lam2)
    N = L // a
    b = L // M
    K = M * lam2
    off = offsets(N, lam1, lam2)
    if points is not None:
        # y_n(l) = Y[n, l mod M] exp(2 pi i l w(n)), Y = M ifft(G[n]) (period M in l)
        j = np.asarray(points, dtype=np.int64)
        n = np.arange(N, dtype=np.int64)
        Y = M * np.fft.ifft(G, axis=1)
        ln = (j[:, None] + n[None, :] * a) % L
        y = Y[n[None, :], ln % M] * _unit_root(ln * off[None, :], K, +1)
        return np.sum(f[ln] * np.conj(y), axis=1)
    l = np.arange(L, dtype=np.int64)
    mods = [_unit_root(l * o, K, +1) for o in range(lam2)]
    gg = np.zeros(L, dtype=np.complex128)
    for n in range(N):
        y = np.tile(M * np.fft.ifft(G[n]), b) * mods[off[n]]
        gg += np.roll(f * np.conj(y), -n * a)
    return gg


def loss_and_grads(f, g, T, a, M, lam1, lam2):
    """Loss sum(|C_g f|^2 - T)^2 with gradients with respect to f and g."""
    c = dgt_fold(f, g, a, M, lam1, lam2)
    loss, G = spectrogram_loss(c, T)
    gf = idgt_adjoint(G, g, a, M, lam1, lam2)
    gg = window_gradient(f, G, a, M, lam1, lam2)
    return loss, gf, gg
