"""CPU oracle: plain, slow, FP64 NumPy definitions of what the GPU path
computes.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code,
tables or constants with the HIP library and never imports it; the two only
share the seeded input generators in ``dgt_inputs``.

Contents and the passages they follow:

* ``dgt_direct``, ``dgt_fold`` -- eq. (DGT) of Section 2.1 (direct triple sum,
  and the per-column modulate/fold/DFT order of the same sum);
* ``dgt_separable`` -- the textbook DGT on a separable lattice;
* ``dgt_multiwindow`` -- the multi-window decomposition, Prop. 4 and Prop. 5
  (eq. (mw_phases));
* ``idgt_adjoint`` -- the synthesis operator, the adjoint of eq. (DGT);
* ``dual.*`` -- frame operator eq. (frameop) in Walnut form, canonical dual
  window S^{-1} g, canonical tight window S^{-1/2} g (Section 4.2), frame
  bounds;
* ``grad.*`` -- gradients of a spectrogram loss with respect to the signal and
  the window;
* ``real.*`` -- the real-signal variant named in Section 4.4: the
  non-redundant channels of the conjugate-symmetric columns of eq. (DGT) for a
  real signal and window, and the synthesis of such coefficients.

Every function is pinned by tests in ``tests/test_oracle.py`` against
brute force, closed forms, library routines and invariants.
"""
from .dgt import (coefficient_frequencies, dgt_direct, dgt_fold, dgt_multiwindow,
                  dgt_separable, idgt_adjoint, offsets)
from .dual import (dual_window, frame_blocks, frame_bounds, frame_operator_apply, tight_window,
                   walnut_weights)
from .grad import loss_and_grads, spectrogram_loss, window_gradient
from .real import dgtreal, idgtreal, pack_real, real_layout, unpack_real

__all__ = [
    "coefficient_frequencies", "dgt_direct", "dgt_fold", "dgt_multiwindow", "dgt_separable",
    "idgt_adjoint", "offsets", "dual_window", "frame_blocks", "frame_bounds",
    "frame_operator_apply", "tight_window", "walnut_weights", "loss_and_grads", "spectrogram_loss",
    "window_gradient", "dgtreal", "idgtreal", "pack_real", "real_layout", "unpack_real",
]
