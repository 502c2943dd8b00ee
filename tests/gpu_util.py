"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and
bring its outputs back into user order for comparison with the oracle."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def params_of(prob):
    import paper_2512_06143_amd as G
    return G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights)


def oracle_blocks(x, radius, precond="block"):
    """The preconditioner blocks the oracle's estimators need for a handle assembled
    from x with support radius r: None (diagonal) or runs of 128 (block) or 64 (block64) points of the binned
    order, computed by the oracle from its own definition."""
    import oracle
    if precond in ("jacobi", 0):
        return None
    size = oracle.BLOCK_SMALL if precond in ("block64", 2) else oracle.BLOCK
    return oracle.block_partition(oracle.bin_order(x, radius), size)


def imported_blocks(n, precond="block"):
    """The same for an imported handle (its order is the given one)."""
    import oracle
    if precond in ("jacobi", 0):
        return None
    size = oracle.BLOCK_SMALL if precond in ("block64", 2) else oracle.BLOCK
    return oracle.block_partition(np.arange(n), size)


def exported_user_csr(m):
    """The handle's CSR as a scipy matrix in user order (values promoted to float64)."""
    rp, col, val, perm = m.export()
    rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy().astype(np.float64)
    n = m.n
    rows_int = np.repeat(np.arange(n), np.diff(rp))
    if perm is not None:
        perm = perm.cpu().numpy().astype(np.int64)
        rows, cols = perm[rows_int], perm[col]
    else:
        rows, cols = rows_int, col.astype(np.int64)
    K = sp.csr_matrix((val, (rows, cols)), shape=(n, n))
    K.sort_indices()
    return K, dict(rp=rp, col=col, val=val, perm=perm)


def pattern_pairs(K):
    coo = K.tocoo()
    pairs = np.stack([coo.row, coo.col], 1).astype(np.int64)
    return pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]


def compare_patterns(got, want, x, prob, gamma_exempt_pts):
    """Exact set equality except pairs within 1e-6 of the support boundary or
    touching a point within 1e-6 of a bump boundary. Returns (n_mismatch, n_exempt)."""
    import oracle
    gs = set(map(tuple, got))
    ws = set(map(tuple, want))
    diff = np.array(sorted(gs ^ ws), dtype=np.int64).reshape(-1, 2)
    if diff.size == 0:
        return 0, 0
    ex = oracle.boundary_exempt_pairs(x, prob.radius, diff)
    ex |= gamma_exempt_pts[diff[:, 0]] | gamma_exempt_pts[diff[:, 1]]
    return int((~ex).sum()), int(ex.sum())


def rel_entry_errors(Kgot, Kwant, floor_rel=1e-30):
    """Max relative error over entries present in both with |K| >= floor * max diag."""
    A = Kgot.tocoo()
    W = Kwant.tocsr()
    want = np.asarray(W[A.row, A.col]).ravel()
    scale = floor_rel * np.abs(Kwant.diagonal()).max()
    mask = np.abs(want) >= scale
    err = np.abs(A.data[mask] - want[mask]) / np.abs(want[mask])
    return float(err.max()) if err.size else 0.0, int((~mask).sum())
