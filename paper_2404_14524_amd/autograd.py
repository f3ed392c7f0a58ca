"""torch.autograd.Function around ipm_solve / ipm_adjoint.

forward(A, b, c, q) -> x* solves (P) with Nys-IP-PMM on the GPU; backward(g)
runs the KKT adjoint (a Nystrom-PCG solve of the adjoint normal equations)
and returns dL/d(A, b, c, q) for the inputs that need a gradient only; the
gradient of A (m x n) is produced only when A requires grad.
"""

from __future__ import annotations

import warnings

import torch

from .nysipm import NYS_OK, ipm_adjoint, ipm_solve


class NysConvergenceWarning(RuntimeWarning):
    """A solve behind NysQP stopped at its iteration limit: its output (the
    forward solution or the gradients) comes from the last iterate."""


class NysQP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, b, c, q, opts):
        opts = dict(opts)
        A_lo = opts.pop("A_lo", None)
        ell = opts.pop("ell")
        x, y, z, info = ipm_solve(A.detach(), b.detach(), c.detach(), q.detach(), ell, A_lo=A_lo, **opts)
        if info.status != NYS_OK:
            warnings.warn(f"NysQP forward: ipm_solve stopped at its iteration limit after {info.iters} "
                          f"iterations (KKT {info.kkt_rel:.2e}); x is the last iterate",
                          NysConvergenceWarning, stacklevel=2)
        ctx.save_for_backward(A, b, c, q, x, y, z)
        ctx.ell, ctx.A_lo, ctx.opts = ell, A_lo, opts
        ctx.rho, ctx.delta = info.rho, info.delta
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        A, b, c, q, x, y, z = ctx.saved_tensors
        names = ("A", "b", "c", "q")
        want = tuple(nm for nm, need in zip(names, ctx.needs_input_grad[:4]) if need)
        if not want:
            return None, None, None, None, None
        opts = {k: v for k, v in ctx.opts.items() if k not in ("tol", "max_iter")}
        grads, pinfo = ipm_adjoint(A.detach(), b.detach(), c.detach(), q.detach(), x, y, z, ctx.rho, ctx.delta,
                                   gx.detach().to(torch.float64).contiguous(), ctx.ell, A_lo=ctx.A_lo,
                                   want=want, **opts)
        if pinfo.status != NYS_OK:
            warnings.warn(f"NysQP backward: the adjoint PCG solve stopped at its iteration limit after "
                          f"{pinfo.iters} iterations (relative residual {pinfo.rel_res:.2e}); the gradients "
                          "come from its last iterate", NysConvergenceWarning, stacklevel=2)
        gA = grads.get("A")
        if gA is not None:
            gA = gA.to(A.dtype)
        return gA, grads.get("b"), grads.get("c"), grads.get("q"), None


def nys_qp(A, b, c, q, ell: int, **opts):
    """x*(A, b, c, q) with autograd support.  Keyword options as for ipm_solve
    (tol, seed, sketch_dtype, A_lo, ...)."""
    return NysQP.apply(A, b, c, q, dict(opts, ell=ell))
