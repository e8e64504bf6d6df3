"""Torch-facing API over the C-ABI: PyTorch provides device memory and
streams, libdgtns does all the computation.

    plan = Plan(L, a, M, lam1, lam2, dtype=torch.complex64, max_batch=64)
    plan.set_window(g)            # any complex/real tensor of length L
    c = plan.forward(f)           # f: (B, L) -> c: (B, N, M), c[k, n, m] = c_k(m, n)
    f2 = plan.adjoint(c)          # synthesis (adjoint) operator
    gd, (A, B) = plan.dual(g)     # canonical dual window (FP64) and frame bounds
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import torch

from . import _binding as B

_DT = {torch.complex64: B.DGTNS_C64, torch.complex128: B.DGTNS_C128}
_REAL = {torch.complex64: torch.float32, torch.complex128: torch.float64}


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


_ALG = {"shear": B.DGTNS_ALG_SHEAR, "multiwindow": B.DGTNS_ALG_MULTIWINDOW, "fir": B.DGTNS_ALG_FIR,
        "shear-ola": B.DGTNS_ALG_SHEAR_OLA, "auto": B.DGTNS_ALG_AUTO}


class Plan:
    """A lattice plan with its tables and window resident in device memory.

    algorithm: "shear" (Alg. 1), "multiwindow" (lambda2 coset windows on the
    separable lattice (lambda2 a, M), Prop. 4 and Prop. 5), "fir" (windows of
    short support, support=(start, length): the window is taken to be zero
    outside samples start, ..., start + length - 1 mod L), "shear-ola" (the
    same truncated window; blocks of block samples transformed on the lattice
    and combined by overlap-add, Section 4; inner: the block transform's
    algorithm, "auto" (default), "shear" or "multiwindow") or "auto" (the
    shear plan, or the multiwindow plan where the shear plan would need a
    frequency shear).  All compute the coefficients of eq. (DGT).  Window
    gradients, dual and tight windows need a shear plan."""

    def __init__(self, L: int, a: int, M: int, lam1: int = 0, lam2: int = 1,
                 dtype: torch.dtype = torch.complex64, max_batch: int = 64, device=None,
                 algorithm: str = "shear", support: Optional[Tuple[int, int]] = None,
                 block: Optional[int] = None, inner: str = "auto"):
        if dtype not in _DT:
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        if algorithm not in _ALG:
            raise ValueError("algorithm must be 'shear', 'multiwindow', 'fir', 'shear-ola' or 'auto'")
        if (algorithm in ("fir", "shear-ola")) != (support is not None):
            raise ValueError("support=(start, length) is given exactly for algorithms 'fir' and 'shear-ola'")
        if (algorithm == "shear-ola") != (block is not None):
            raise ValueError("block is given exactly for algorithm 'shear-ola'")
        if inner not in ("auto", "shear", "multiwindow"):
            raise ValueError("inner must be 'auto', 'shear' or 'multiwindow'")
        if not torch.cuda.is_available():
            raise RuntimeError("libdgtns needs a HIP device")
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        self.algorithm = algorithm
        if algorithm == "fir":
            self._h = B.dgtns_plan_create_fir(L, a, M, lam1, lam2, _DT[dtype], max_batch, int(support[0]),
                                              int(support[1]))
        elif algorithm == "shear-ola":
            self._h = B.dgtns_plan_create_ola_alg(L, a, M, lam1, lam2, _DT[dtype], max_batch, int(support[0]),
                                                  int(support[1]), int(block), _ALG[inner])
        else:
            self._h = B.dgtns_plan_create_alg(L, a, M, lam1, lam2, _DT[dtype], max_batch, _ALG[algorithm])
        self.info = B.dgtns_plan_info(self._h)
        self.L, self.a, self.M, self.lam1, self.lam2 = L, a, M, lam1, lam2
        self.N = self.info.N
        self.max_batch = max_batch
        nbytes = self.info.persistent_bytes
        # 256-byte alignment: allocate with slack and offset
        self._persist = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._persist.data_ptr()
        self._pptr = base + ((-base) % 256)
        with torch.cuda.device(self.device):
            B.dgtns_plan_bind(self._h, self._pptr, nbytes, _stream_handle(self.device))
        self._ws: Dict[Tuple[int, int], torch.Tensor] = {}
        self.window: Optional[torch.Tensor] = None
        # changes with every set_window
        self.window_serial = 0

    # ------------------------------------------------------------------
    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                B.dgtns_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def branch(self) -> int:
        return self.info.branch

    @property
    def shear(self) -> Tuple[int, int, int]:
        return self.info.s0, self.info.s1, self.info.b_r

    def workspace(self, op: int, batch: int, stream: Optional[int] = None) -> Tuple[int, int]:
        """Workspace pointer and size for op, cached per (op, stream)."""
        need = B.dgtns_workspace_bytes(self._h, op, batch)
        key = (op, stream if stream is not None else _stream_handle(self.device))
        buf = self._ws.get(key)
        if buf is None or buf.numel() < need:
            buf = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[key] = buf
        return buf.data_ptr(), buf.numel()

    # ------------------------------------------------------------------
    def set_window(self, g: torch.Tensor) -> None:
        g64 = g.detach().to(device=self.device, dtype=torch.complex128).contiguous()
        if g64.shape != (self.L,):
            raise ValueError(f"window must have shape ({self.L},)")
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_SET_WINDOW, 1, st)
        B.dgtns_set_window(self._h, g64.data_ptr(), ws, wsb, st)
        self.window = g64
        self.window_serial += 1

    def _signals(self, f: torch.Tensor):
        if f.dim() == 1:
            f = f.unsqueeze(0)
        if f.dim() != 2 or f.shape[1] != self.L:
            raise ValueError(f"signals must have shape (B, {self.L})")
        if f.is_complex():
            f = f.to(device=self.device, dtype=self.dtype).contiguous()
            return f, 0
        f = f.to(device=self.device, dtype=_REAL[self.dtype]).contiguous()
        return f, 1

    def forward(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Coefficients c[k, n, m] = c_k(m, n) of eq. (DGT) for signals f (B, L)
        (real or complex)."""
        squeeze = f.dim() == 1
        f, real = self._signals(f)
        nb = f.shape[0]
        if out is None:
            out = torch.empty((nb, self.N, self.M), dtype=self.dtype, device=self.device)
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_FORWARD, nb, st)
        B.dgtns_forward(self._h, f.data_ptr(), real, out.data_ptr(), nb, ws, wsb, st)
        return out[0] if squeeze else out

    def adjoint(self, c: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Synthesis f(l) = sum_{m,n} c(m, n) g(l - n a) exp(2 pi i l (m + w(n))/M)."""
        squeeze = c.dim() == 2
        if squeeze:
            c = c.unsqueeze(0)
        if c.shape[1:] != (self.N, self.M):
            raise ValueError(f"coefficients must have shape (B, {self.N}, {self.M})")
        c = c.to(device=self.device, dtype=self.dtype).contiguous()
        nb = c.shape[0]
        if out is None:
            out = torch.empty((nb, self.L), dtype=self.dtype, device=self.device)
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_ADJOINT, nb, st)
        B.dgtns_adjoint(self._h, c.data_ptr(), out.data_ptr(), nb, ws, wsb, st)
        return out[0] if squeeze else out

    @property
    def real_shape(self) -> Tuple[int, int]:
        """Per-signal shape (N / lambda2, real_row) of real-signal coefficients."""
        return (self.N // self.info.lambda2, self.info.real_row)

    def forward_real(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Real-signal variant: the non-redundant channels of eq. (DGT) of real
        signals f (B, L), as (B, N / lambda2, real_row) (see dgtns_forward_real)."""
        squeeze = f.dim() == 1
        if f.is_complex():
            raise ValueError("forward_real takes real signals")
        if f.dim() == 1:
            f = f.unsqueeze(0)
        if f.dim() != 2 or f.shape[1] != self.L:
            raise ValueError(f"signals must have shape (B, {self.L})")
        f = f.to(device=self.device, dtype=_REAL[self.dtype]).contiguous()
        nb = f.shape[0]
        if out is None:
            out = torch.empty((nb,) + self.real_shape, dtype=self.dtype, device=self.device)
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_FORWARD, nb, st)
        B.dgtns_forward_real(self._h, f.data_ptr(), out.data_ptr(), nb, ws, wsb, st)
        return out[0] if squeeze else out

    def adjoint_real(self, c: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Real part of the synthesis of real-signal coefficients c
        (B, N / lambda2, real_row), expanded by conjugate symmetry: real (B, L)."""
        squeeze = c.dim() == 2
        if squeeze:
            c = c.unsqueeze(0)
        if tuple(c.shape[1:]) != self.real_shape:
            raise ValueError(f"coefficients must have shape (B, {self.real_shape[0]}, {self.real_shape[1]})")
        c = c.to(device=self.device, dtype=self.dtype).contiguous()
        nb = c.shape[0]
        if out is None:
            out = torch.empty((nb, self.L), dtype=_REAL[self.dtype], device=self.device)
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_ADJOINT, nb, st)
        B.dgtns_adjoint_real(self._h, c.data_ptr(), out.data_ptr(), nb, ws, wsb, st)
        return out[0] if squeeze else out

    def window_grad(self, f: torch.Tensor, gc: torch.Tensor) -> torch.Tensor:
        """Gradient of a real loss with respect to the window, summed over the
        batch, given the coefficient gradient gc (B, N, M)."""
        if f.dim() == 1:
            f = f.unsqueeze(0)
            gc = gc.unsqueeze(0)
        f = f.to(device=self.device, dtype=self.dtype).contiguous()
        gc = gc.to(device=self.device, dtype=self.dtype).contiguous()
        nb = f.shape[0]
        out = torch.empty(self.L, dtype=self.dtype, device=self.device)
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_WINDOW_GRAD, nb, st)
        B.dgtns_window_grad(self._h, f.data_ptr(), gc.data_ptr(), out.data_ptr(), nb, ws, wsb, st)
        return out

    def _dual_or_tight(self, fn, g):
        g64 = (self.window if g is None else g).detach().to(device=self.device, dtype=torch.complex128).contiguous()
        out = torch.empty(self.L, dtype=torch.complex128, device=self.device)
        bounds = torch.empty(2, dtype=torch.float64, device=self.device)
        st = _stream_handle(self.device)
        ws, wsb = self.workspace(B.DGTNS_OP_DUAL, 1, st)
        fn(self._h, g64.data_ptr(), out.data_ptr(), bounds.data_ptr(), ws, wsb, st)
        return out, bounds

    def dual(self, g: Optional[torch.Tensor] = None):
        """Canonical dual window S^{-1} g (complex128) and the frame bounds (A, B)."""
        return self._dual_or_tight(B.dgtns_dual_window, g)

    def tight(self, g: Optional[torch.Tensor] = None):
        """Canonical tight window S^{-1/2} g (complex128) and the frame bounds (A, B)."""
        return self._dual_or_tight(B.dgtns_tight_window, g)


def dgt(f: torch.Tensor, plan: Plan) -> torch.Tensor:
    return plan.forward(f)


def idgt(c: torch.Tensor, plan: Plan) -> torch.Tensor:
    return plan.adjoint(c)


def dual(g: torch.Tensor, a: int, M: int, lam1: int = 0, lam2: int = 1, tight: bool = False, device=None):
    """Canonical dual window S^{-1} g (tight=True: the canonical tight window
    S^{-1/2} g) of the Gabor frame of g (length L) on the lattice (a, M,
    lambda1/lambda2), in FP64 on the GPU, with the optimal frame bounds
    (A, B) (A = 0: not a frame).  A shear plan of the lattice is built for
    the call (its tables hold the shear factorisation the computation uses)."""
    L = int(g.shape[-1])
    plan = Plan(L, a, M, lam1, lam2, dtype=torch.complex64, max_batch=1, device=device)
    return plan.tight(g) if tight else plan.dual(g)


class DGTFunction(torch.autograd.Function):
    """c = DGT_g(f) with gradients for both the signal and the window.

    Backward: grad_f = C_g^* grad_c (the synthesis operator) and
    grad_g(j) = sum_k sum_n f_k(j + n a) conj(y_{k,n}(j + n a)), both computed
    by libdgtns.

    The plan's resident window is prepared (dgtns_set_window) once per
    forward, from the values g holds at that moment (a tensor's values can
    change without a version bump, e.g. through .data), and not again in
    backward unless another window was set on the plan in between.  The
    function sets the window of the plan it is given, so one plan must not
    serve two graphs with different windows on different streams at once
    (give each its own plan)."""

    @staticmethod
    def forward(ctx, f, g, plan: Plan):
        plan.set_window(g)
        c = plan.forward(f)
        ctx.plan = plan
        ctx.serial = plan.window_serial
        ctx.save_for_backward(f, g)
        return c

    @staticmethod
    def backward(ctx, gc):
        f, g = ctx.saved_tensors
        plan = ctx.plan
        # autograd has checked that g is unchanged since forward; the window
        # is prepared again only if another window was set in between
        if plan.window_serial != ctx.serial:
            plan.set_window(g)
        gf = gg = None
        if ctx.needs_input_grad[0]:
            gf = plan.adjoint(gc)
            if f.dim() == 1:
                gf = gf.reshape(-1)
            gf = gf.to(f.dtype)
        if ctx.needs_input_grad[1]:
            fc = f if f.is_complex() else f.to(plan.dtype)
            gg = plan.window_grad(fc, gc).to(g.dtype)
        return gf, gg, None
