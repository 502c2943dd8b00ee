"""CPU float64 oracle for the gp2Scale hot path (test infrastructure, not product code).

This package is a plain, slow, obviously correct restatement of what the GPU path
computes, written from the paper (arXiv 2512.06143):

* the compactly supported kernel k(x_i, x_j) = g(x_i) g(x_j) W(||x_i - x_j|| / r),
  the product construction of Sec. 4.1 with g a sum of bump functions (Sec. 4.3,
  Eq. bump) and W the C^2 member of the Wendland family (a variant of Eq. wendland,
  which Sec. 4.1 allows);
* its sparsity pattern, by brute force and by a k-d tree;
* the log marginal likelihood of Sec. 3 (first displayed equation, zero prior
  mean, noise on the diagonal) through a dense Cholesky factorisation;
* its exact gradient with respect to the hyperparameters, and the same-probe
  stochastic estimators (Hutchinson trace, probe log-determinant) that the GPU
  path approximates with conjugate gradients and Lanczos quadrature;
* the counter-based SplitMix64 probe signs;
* the preconditioners of the solves (diagonal, and block diagonal over runs of the
  binned point order) that the estimators are defined with;
* the posterior mean and variance of the latent function at test points (Sec. 3,
  Eq. posterior);
* the block Metropolis-Hastings sampler of the hyperparameters (Sec. 4.6, App. D);
* the non-stationary convolution Wendland kernel (Sec. 4.2, Eq. wendconv) with an
  axis-anisotropic, bump-driven length-scale field (``oracle.wendconv``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never calls it, and it
shares no code with the HIP path.

Every function documents the passage it follows, and states the reading it takes
where the paper is silent or garbled.
"""
from .kernel import (wendland_c2, wendland_c2_dr, wendland_c6, wendland_c6_dr, wendland, wendland_dr,
                     wendland_dlog, KERNELS, bump_values, kernel_params_check)
from . import wendconv
from .pattern import (pairwise_sqdist, pattern_bruteforce, pattern_kdtree, mean_row_count,
                      boundary_exempt_pairs, boundary_exempt_points)
from .dense import covariance_dense, dcov_dense, lml_dense, grad_exact, LMLResult
from .probes import splitmix64, rademacher_probes, probe_sign_masks
from .estimators import logdet_same_probe, grad_same_probe, lml_same_probe, hutchinson_variance
from .sparse import (covariance_csr, covariance_rows, residual_rel, pcg_jacobi, dcov_csr, lml_components,
                     lanczos_logquad, lml_grad_sparse)
from .posterior import cross_covariance, posterior_dense
from .mcmc import block_mh
from .precond import (BLOCK, BLOCK_SMALL, BATCH_BLOCK, grid, bin_coords, bin_order, block_partition, jacobi_partition, block_factor,
                      morton, sub_cell_codes)

__all__ = [
    "wendland_c2", "wendland_c2_dr", "wendland_c6", "wendland_c6_dr", "wendland", "wendland_dr", "wendland_dlog",
    "KERNELS", "wendconv",
    "bump_values", "kernel_params_check",
    "pairwise_sqdist", "pattern_bruteforce", "pattern_kdtree", "mean_row_count",
    "boundary_exempt_pairs", "boundary_exempt_points",
    "covariance_dense", "dcov_dense", "lml_dense", "grad_exact", "LMLResult",
    "splitmix64", "rademacher_probes", "probe_sign_masks",
    "logdet_same_probe", "grad_same_probe", "lml_same_probe", "hutchinson_variance",
    "cross_covariance", "posterior_dense", "block_mh",
    "BLOCK", "BLOCK_SMALL", "BATCH_BLOCK", "grid", "bin_coords", "bin_order", "block_partition", "jacobi_partition", "block_factor",
    "morton", "sub_cell_codes",
    "covariance_csr", "covariance_rows", "residual_rel", "pcg_jacobi", "dcov_csr", "lml_components",
    "lanczos_logquad", "lml_grad_sparse",
]
