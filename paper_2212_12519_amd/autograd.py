"""Differentiable Joseph projectors (the paper's deep-learning use, Sec. 1 and 4).

``JosephOperator`` binds a ray list (sinogram LORs or listmode events) to an
image grid; calling it applies the forward projector A and ``.T`` applies the
back projector A^T.  Both are torch.autograd.Functions whose backward pass is
the other hand-written kernel: d(Ax)/dx^T g = A^T g and d(A^T y)/dy^T g = A g,
so the pair is exactly adjoint and double backward works.  Leading batch
dimensions (images [..., n0, n1, n2] <-> projections [..., n] or [..., n,
n_bins]) go through the batched listmode forward and back projections (one
pass over the events for all images) for the TOF listmode kind, and are
looped over otherwise.
"""
from __future__ import annotations

import torch

from ._lib import as_geom, as_tof
from . import projectors as P

KINDS = ("nontof", "tof_sino", "tof_lm")


class JosephOperator:
    """A: images on `geom` -> projections of the rays (xstart[i], xend[i]).

    kind: "nontof" (p[n]), "tof_sino" (p[n, n_bins]) or "tof_lm" (p[n], tof_bin required).
    presort: listmode kinds only -- process rays in pp_lm_presort order (faster, same result
    up to float summation order in A^T).
    """

    def __init__(self, xstart, xend, geom, kind="nontof", tof=None, tof_bin=None, presort=False):
        if kind not in KINDS:
            raise ValueError(f"kind must be one of {KINDS}")
        if kind != "nontof" and tof is None:
            raise ValueError("TOF kinds need tof parameters")
        if kind == "tof_lm" and tof_bin is None:
            raise ValueError("tof_lm needs tof_bin")
        self.xs, self.xe = xstart.contiguous(), xend.contiguous()
        self.geom = as_geom(geom)
        self.kind = kind
        self.tof = as_tof(tof) if tof is not None else None
        self.bins = tof_bin.contiguous() if tof_bin is not None else None
        self.order = None
        if presort and kind != "tof_sino" and self.xs.shape[0] > 0:
            self.order = P.presort(self.xs, self.xe, self.geom, self.bins, self.tof)

    @property
    def n(self):
        return self.xs.shape[0]

    @property
    def proj_shape(self):
        return (self.n, self.tof.n_bins) if self.kind == "tof_sino" else (self.n,)

    # raw (non-autograd) applications, batched over leading dims
    def _fwd1(self, x):
        x = x.contiguous()
        if self.kind == "nontof":
            return P.fwd(self.xs, self.xe, self.geom, x, self.order)
        if self.kind == "tof_sino":
            return P.fwd_tof_sino(self.xs, self.xe, self.geom, self.tof, x)
        return P.fwd_tof_lm(self.xs, self.xe, self.bins, self.geom, self.tof, x, self.order)

    def _back1(self, y):
        y = y.contiguous()
        if self.kind == "nontof":
            return P.back(self.xs, self.xe, self.geom, y, order=self.order)
        if self.kind == "tof_sino":
            return P.back_tof_sino(self.xs, self.xe, self.geom, self.tof, y)
        return P.back_tof_lm(self.xs, self.xe, self.bins, self.geom, self.tof, y, order=self.order)

    def apply_raw(self, x):
        lead = x.shape[:-3]
        if tuple(x.shape[-3:]) != self.geom.dim:
            raise ValueError(f"image shape {tuple(x.shape[-3:])} != grid {self.geom.dim}")
        xf = x.reshape(-1, *self.geom.dim)
        if self.kind == "tof_lm" and xf.shape[0] > 1:  # one batched projection of all images
            out = P.fwd_tof_lm_batch(self.xs, self.xe, self.bins, self.geom, self.tof, xf.contiguous(), self.order)
        else:
            out = torch.stack([self._fwd1(xf[b]) for b in range(xf.shape[0])]) if xf.shape[0] else \
                x.new_empty((0, *self.proj_shape))
        return out.reshape(*lead, *self.proj_shape)

    def adjoint_raw(self, y):
        k = len(self.proj_shape)
        lead = y.shape[:-k]
        if tuple(y.shape[-k:]) != self.proj_shape:
            raise ValueError(f"projection shape {tuple(y.shape[-k:])} != {self.proj_shape}")
        yf = y.reshape(-1, *self.proj_shape)
        if self.kind == "tof_lm" and yf.shape[0] > 1:  # one batched back projection of all value arrays
            out = P.back_tof_lm_batch(self.xs, self.xe, self.bins, self.geom, self.tof, yf.contiguous(), self.order)
        else:
            out = torch.stack([self._back1(yf[b]) for b in range(yf.shape[0])]) if yf.shape[0] else \
                y.new_empty((0, *self.geom.dim))
        return out.reshape(*lead, *self.geom.dim)

    # differentiable applications
    def __call__(self, x):
        return JosephFwd.apply(x, self)

    def T(self, y):
        return JosephBack.apply(y, self)


class JosephFwd(torch.autograd.Function):
    """y = A x; backward: grad_x = A^T grad_y (hand-written back projection kernel)."""

    @staticmethod
    def forward(ctx, x, op):
        ctx.op = op
        return op.apply_raw(x)

    @staticmethod
    def backward(ctx, g):
        return JosephBack.apply(g, ctx.op), None


class JosephBack(torch.autograd.Function):
    """x = A^T y; backward: grad_y = A grad_x (hand-written forward projection kernel)."""

    @staticmethod
    def forward(ctx, y, op):
        ctx.op = op
        return op.adjoint_raw(y)

    @staticmethod
    def backward(ctx, g):
        return JosephFwd.apply(g, ctx.op), None


class PoissonNLL(torch.autograd.Function):
    """L = sum(ybar - y log ybar), ybar = p + bg: the loss and its gradient 1 - y / ybar in one pass of
    the library's kernel (float64 per element, the gradient stored as float32).  A backward that is
    itself differentiated (create_graph) recomputes the gradient with torch operations instead."""

    @staticmethod
    def forward(ctx, p, y, bg):
        pc = p.contiguous()
        yc = y.to(device=p.device, dtype=torch.float32).contiguous()
        grad = torch.empty_like(pc)
        n_partial = max(1, min(2048, (pc.numel() + 255) // 256))
        partial = torch.empty(n_partial, dtype=torch.float64, device=p.device)
        P.pp_poisson_nll(pc, bg, yc, grad, partial)
        ctx.save_for_backward(pc, yc, grad)
        ctx.bg = bg
        return partial.sum()

    @staticmethod
    def backward(ctx, g):
        p, y, grad = ctx.saved_tensors
        if torch.is_grad_enabled():  # differentiable form for higher derivatives
            ybar = (p + ctx.bg).double()
            return (g * (1.0 - y.double() / ybar)).to(p.dtype), None, None
        return grad * g.to(grad.dtype), None, None


def poisson_nll(ybar, y, bg=0.0):
    """Poisson negative log-likelihood (up to a constant) of the expectation ybar + bg against the data
    y: sum(ybar + bg - y log(ybar + bg)), accumulated in float64 (float32 ybar; the constant background
    is added inside the kernel, in float32, as ``ybar + bg`` would)."""
    if ybar.dtype != torch.float32:
        raise TypeError("ybar must be float32")
    return PoissonNLL.apply(ybar, y, float(bg))
