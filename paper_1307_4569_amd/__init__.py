"""MI355X-native discrete Gabor transform on nonseparable lattices by the
shear method (Wiesmeyr, Holighaus, Sondergaard).

All computation runs in the HIP library libdgtns.so (built in-tree by
``python -m paper_1307_4569_amd.build``); this package only marshals
arguments and provides device memory and streams through PyTorch.  Importing
the package does not load the library; the first call that needs it raises if
it is missing.
"""
from ._binding import DgtnsError  # noqa: F401

__all__ = ["Plan", "dgt", "idgt", "dual", "DGTFunction", "DgtnsError"]


def __getattr__(name):
    if name in ("Plan", "dgt", "idgt", "dual", "DGTFunction"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
