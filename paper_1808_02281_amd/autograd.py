"""Differentiable access to the Symanzik action.

``symanzik_action(U, L, u0, beta)`` returns S_G (a 0-d float64 CUDA tensor) for a link
field in the SoA even-odd layout; its gradient comes from the force kernels
(sym_action_grad, run in the forward when a backward can follow), which return 2 G U
per link: the gradient of S_G with respect to
the link matrices, projected on the tangent space of SU(3) at U. Derivatives along
any parametrisation that keeps the links in SU(3) -- for instance
U = exp(i omega.T) U0 built with torch ops -- are therefore exact, and
dS/domega^a = -2i tr(T_a G) at omega = 0 (arXiv:1808.02281 Sec. II, eq. 18_7_25_1 with
dU/domega = iTU). Components normal to the group (moving U off SU(3)) are not
represented.

``pack``/``unpack`` are the layout kernels as differentiable permutations, so a
canonical complex field built in torch can be fed to the action and differentiated.
"""
import torch

from . import api


class _Pack(torch.autograd.Function):
    @staticmethod
    def forward(ctx, aos, L):
        ctx.L = tuple(L)
        return api.pack(aos.contiguous(), ctx.L)

    @staticmethod
    def backward(ctx, g):
        # the real SoA gradient holds dL/dRe and dL/dIm; unpacking it gives the complex
        # gradient dL/dRe + i dL/dIm that torch expects for complex inputs
        return api.unpack(g.contiguous(), ctx.L), None


class _Unpack(torch.autograd.Function):
    @staticmethod
    def forward(ctx, soa, L):
        ctx.L = tuple(L)
        return api.unpack(soa.contiguous(), ctx.L)

    @staticmethod
    def backward(ctx, g):
        return api.pack(g.contiguous(), ctx.L), None


class SymanzikAction(torch.autograd.Function):
    """S_G(U). When a backward can follow, the forward runs the force kernels once
    (sym_action_grad with the fused action: S from the same staple sums) and keeps
    2 G U for the backward; otherwise it runs the action kernel alone."""

    @staticmethod
    def forward(ctx, U, L, u0, beta, with_grad):
        L = tuple(L)
        if with_grad:
            grad, S = api.action_grad(U, L, u0, beta, with_action=True)
            ctx.save_for_backward(grad)
            return S[0]
        ctx.save_for_backward(None)
        return api.action(U, L, u0, beta)[0]

    @staticmethod
    def backward(ctx, gS):
        (grad,) = ctx.saved_tensors
        return grad * gS.to(grad.dtype), None, None, None, None


def pack(aos, L):
    return _Pack.apply(aos, L)


def unpack(soa, L):
    return _Unpack.apply(soa, L)


def symanzik_action(U, L, u0, beta):
    return SymanzikAction.apply(U, L, u0, beta, torch.is_grad_enabled() and U.requires_grad)


class FatSmear(torch.autograd.Function):
    """(V, W) = fat and Naik links of U; backward = the path-force kernels (sym_fat_force).
    When a backward can follow, the forward fills a private workspace that is kept
    until the backward, which then reuses its intermediates (SYM_FAT_REUSE_LINKS)
    instead of recomputing the two forward passes."""

    @staticmethod
    def forward(ctx, U, L, c, with_grad):
        ctx.save_for_backward(U)
        ctx.args = (tuple(L), tuple(float(v) for v in c))
        ctx.ws = api.new_fat_workspace(ctx.args[0], api.prec_of(U.dtype), U.device) if with_grad else None
        return api.fat_links(U, ctx.args[0], ctx.args[1], with_naik=True, ws=ctx.ws)

    @staticmethod
    def backward(ctx, gV, gW):
        (U,) = ctx.saved_tensors
        L, c = ctx.args
        if gV is None:
            gV = torch.zeros_like(U)
        gW = None if gW is None else gW.contiguous()
        if ctx.ws is not None:
            grad = api.fat_force(U, L, c, gV.contiguous(), gW, mode="grad", ws=ctx.ws, reuse_links=True)
        else:
            grad = api.fat_force(U, L, c, gV.contiguous(), gW, mode="grad")
        return grad, None, None, None


def fat_smear(U, L, c):
    """Differentiable asqtad/HISQ smearing: (V, W) with V the fat links and W the Naik
    links of the SoA link field U (real gradient layout as for the fields: the gradient
    of a real function with respect to the re and im parts of every element)."""
    return FatSmear.apply(U, L, c, torch.is_grad_enabled() and U.requires_grad)
