"""torch.autograd.Function around the library's bound and hand-written backward.

The forward evaluates F (eq. rsvgp_precond) at the given factor L; the
backward calls the library's backward kernels (K_uf tiles recomputed, T held
fixed as in Section 3.1), scaled in-kernel by the incoming adjoint.  Gradients
flow to the lengthscales, signal variance, noise variance, Z, m~ and s~; only
those whose inputs require grad are computed (s~ costs one more M^3 product).
The multi-output form (Q outputs sharing Z, the kernel, S~ and T) does the
same for the per-output inducing means Mt; it has no s~ gradient.
"""
import torch

from .lib import Context


_GRAD_NAMES = ("ell", "sf2", "noise_var", "Z", "m", "s")


class _Bound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ell, sf2, noise, Z, m, s, X, y, L, N, lib):
        F, terms = lib.bound(X, y, N, ell, sf2, noise, Z, m, s, L)
        ctx.lib = lib
        ctx.gen = lib.generation
        ctx.N = N
        ctx.save_for_backward(ell, sf2, noise if noise is not None else sf2, Z, m, s, X, y, L)
        ctx.has_noise = noise is not None
        ctx.mark_non_differentiable(terms)
        return F.reshape(()), terms

    @staticmethod
    def backward(ctx, gF, gterms):
        lib = ctx.lib
        if lib.generation != ctx.gen:
            raise RuntimeError("another forward ran on this library context since this "
                               "bound was evaluated; use one context per graph in flight")
        ell, sf2, noise, Z, m, s, X, y, L = ctx.saved_tensors
        noise = noise if ctx.has_noise else None
        want = tuple(n for n, need in zip(_GRAD_NAMES, ctx.needs_input_grad[:6])
                     if need and (n != "noise_var" or ctx.has_noise))
        scale = gF.detach().to(torch.float64).reshape(1).contiguous()
        g = lib.bound_bwd(X, y, ctx.N, ell, sf2, noise, Z, m, s, L, grad_scale=scale, want=want)
        return tuple(g.get(n) for n in _GRAD_NAMES) + (None,) * 5


def ifsvgp_bound(lib: Context, X, y, N, ell, sf2, noise, Z, m, s, L):
    """F (0-dim fp64 tensor, differentiable w.r.t. ell, sf2, noise, Z, m, s) and terms."""
    return _Bound.apply(ell, sf2, noise, Z, m, s, X, y, L, float(N), lib)


_MULTI_GRAD_NAMES = ("ell", "sf2", "noise_var", "Z", "m")


class _MultiBound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ell, sf2, noise, Z, Mt, s, X, Y, L, N, lib):
        F, terms = lib.bound_multi(X, Y, N, ell, sf2, noise, Z, Mt, s, L)
        ctx.lib = lib
        ctx.gen = lib.generation
        ctx.N = N
        ctx.save_for_backward(ell, sf2, noise if noise is not None else sf2, Z, Mt, s, X, Y, L)
        ctx.has_noise = noise is not None
        ctx.mark_non_differentiable(terms)
        return F.reshape(()), terms

    @staticmethod
    def backward(ctx, gF, gterms):
        lib = ctx.lib
        if lib.generation != ctx.gen:
            raise RuntimeError("another forward ran on this library context since this "
                               "bound was evaluated; use one context per graph in flight")
        if ctx.needs_input_grad[5]:
            raise RuntimeError("the multi-output bound has no gradient with respect to s~")
        ell, sf2, noise, Z, Mt, s, X, Y, L = ctx.saved_tensors
        noise = noise if ctx.has_noise else None
        want = tuple(n for n, need in zip(_MULTI_GRAD_NAMES, ctx.needs_input_grad[:5])
                     if need and (n != "noise_var" or ctx.has_noise))
        scale = gF.detach().to(torch.float64).reshape(1).contiguous()
        g = lib.bound_multi_bwd(X, Y, ctx.N, ell, sf2, noise, Z, Mt, s, L, grad_scale=scale,
                                want=want)
        return tuple(g.get(n) for n in _MULTI_GRAD_NAMES) + (None,) * 6


def ifsvgp_bound_multi(lib: Context, X, Y, N, ell, sf2, noise, Z, Mt, s, L):
    """Multi-output F (0-dim fp64 tensor, differentiable w.r.t. ell, sf2, noise,
    Z and the inducing means Mt (Q, M)) and terms; Y is (B, Q)."""
    return _MultiBound.apply(ell, sf2, noise, Z, Mt, s, X, Y, L, float(N), lib)
