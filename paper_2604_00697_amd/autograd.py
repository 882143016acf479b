"""torch.autograd.Function around the library's bound and hand-written backward.

The forward evaluates F (eq. rsvgp_precond) at the given factor L; the
backward calls the library's backward kernels (K_uf tiles recomputed, T held
fixed as in Section 3.1), scaled in-kernel by the incoming adjoint.  Gradients
flow to the lengthscales, signal variance, noise variance, Z and m~.
"""
import torch

from .lib import Context


class _Bound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ell, sf2, noise, Z, m, X, y, s, L, N, lib):
        F, terms = lib.bound(X, y, N, ell, sf2, noise, Z, m, s, L)
        ctx.lib = lib
        ctx.gen = lib.generation
        ctx.N = N
        ctx.save_for_backward(ell, sf2, noise if noise is not None else sf2, Z, m, X, y, s, L)
        ctx.has_noise = noise is not None
        ctx.mark_non_differentiable(terms)
        return F.reshape(()), terms

    @staticmethod
    def backward(ctx, gF, gterms):
        lib = ctx.lib
        if lib.generation != ctx.gen:
            raise RuntimeError("another forward ran on this library context since this "
                               "bound was evaluated; use one context per graph in flight")
        ell, sf2, noise, Z, m, X, y, s, L = ctx.saved_tensors
        noise = noise if ctx.has_noise else None
        scale = gF.detach().to(torch.float64).reshape(1).contiguous()
        g = lib.bound_bwd(X, y, ctx.N, ell, sf2, noise, Z, m, s, L, grad_scale=scale)
        return (g["ell"], g["sf2"], g.get("noise_var") if ctx.has_noise else None,
                g["Z"], g["m"], None, None, None, None, None, None)


def ifsvgp_bound(lib: Context, X, y, N, ell, sf2, noise, Z, m, s, L):
    """F (0-dim fp64 tensor, differentiable w.r.t. ell, sf2, noise, Z, m) and terms."""
    return _Bound.apply(ell, sf2, noise, Z, m, X, y, s, L, float(N), lib)
