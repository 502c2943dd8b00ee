"""MI355X (gfx950) implementation of the gp2Scale hot path (arXiv 2512.06143).

The compute lives in libgp2s.so (HIP kernels behind the C ABI of include/gp2s.h);
this package only marshals arguments. `GP2SLML` exposes the log marginal
likelihood (Sec. 3) as a differentiable torch function of the kernel
hyperparameters (r, bump weights, noise variance).
"""
from __future__ import annotations

import numpy as np

from .gp2s import (GP2S_FP64, GP2S_MIXED, Batch, GP2SError, Context, HostParams, Matrix, Report, SolveOpts,
                   default_context, default_opts, gp2s_assemble, gp2s_lml, gp2s_lml_grad,
                   gp2s_matrix_import, gp2s_predict, gp2s_solve, gp2s_spmv, gp2s_spmv_noalloc, lib)

from .mcmc import BlockMH  # noqa: E402

__all__ = ["BlockMH", "GP2S_FP64", "GP2S_MIXED", "Batch", "GP2SError", "Context", "HostParams", "Matrix", "Report", "SolveOpts",
           "default_context", "default_opts", "gp2s_assemble", "gp2s_lml", "gp2s_lml_grad",
           "gp2s_matrix_import", "gp2s_predict", "gp2s_solve", "gp2s_spmv", "gp2s_spmv_noalloc", "GP2SLML", "lml"]


def _autograd_function():
    import torch

    class GP2SLML(torch.autograd.Function):
        """LML(x, y; r, a_1..a_P, sigma_n^2) with the hand-written gradient kernel.

        forward(x, y, radius, weights, noise_var, centers, bump_width, precision, opts)
        radius, weights and noise_var may require grad; x, y, centers and bump_width
        are data / fixed geometry. The gradient comes from gp2s_lml_grad, which runs
        the probe solves the log-determinant needs anyway and contracts dK/dtheta
        over the stored pattern.
        """

        @staticmethod
        def forward(ctx, x, y, radius, weights, noise_var, centers, bump_width, precision="mixed", opts=None):
            params = HostParams(int(x.shape[1]), float(radius), float(bump_width), float(noise_var),
                                np.asarray(centers.detach().cpu() if hasattr(centers, "detach") else centers,
                                           dtype=np.float64),
                                weights.detach().cpu().double().numpy())
            m = gp2s_assemble(x, params, precision)
            try:
                need = any(ctx.needs_input_grad[2:5])
                if need:
                    rep, grad, _ = gp2s_lml_grad(m, y, opts, want_a=False)
                    ctx.grad = torch.as_tensor(grad)
                else:
                    rep, _ = gp2s_lml(m, y, opts, want_a=False)
                    ctx.grad = None
            finally:
                m.free()
            ctx.P = int(weights.shape[0])
            ctx.report = rep.as_dict()
            # each hyperparameter's gradient goes back on that input's device and dtype
            ctx.like = [(v.device, v.dtype) if torch.is_tensor(v) else (None, None)
                        for v in (radius, weights, noise_var)]
            dev = weights.device if torch.is_tensor(weights) else None
            return torch.tensor(rep.lml, dtype=torch.float64, device=dev)

        @staticmethod
        def backward(ctx, g):
            if ctx.grad is None:
                return (None,) * 9
            G = ctx.grad * g.detach().to("cpu", torch.float64)
            P = ctx.P
            parts = [G[0].reshape(()), G[1:P + 1].clone(), G[P + 1].reshape(())]
            out = [t.to(device=d, dtype=dt) if d is not None else t for t, (d, dt) in zip(parts, ctx.like)]
            return (None, None, out[0], out[1], out[2], None, None, None, None)

    return GP2SLML


try:
    GP2SLML = _autograd_function()
except ImportError:  # torch missing: the ctypes binding still works
    GP2SLML = None


def lml(x, y, radius, weights, noise_var, centers, bump_width, precision="mixed", opts=None):
    """Differentiable LML; see GP2SLML."""
    return GP2SLML.apply(x, y, radius, weights, noise_var, centers, bump_width, precision, opts)
