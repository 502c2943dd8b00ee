"""The allocation-free product gp2s_spmv_noalloc through the C ABI: equal to gp2s_spmv
(to 1e-12 relative; both sum in float64) on two calls in a row, the second with a
smaller input, with no allocator call; inputs past its fixed workspace and far-field
handles are refused with GP2S_E_INVALID."""
import numpy as np
import pytest

import workloads
from gpu_util import params_of

pytestmark = pytest.mark.gpu


def _allocs(torch):
    return torch.cuda.memory_stats()["allocation.all.allocated"]


def test_noalloc_product_matches_spmv(gpu):
    import torch
    import paper_2512_06143_amd as G
    cases = [(workloads.make_problem("c1"), "mixed", 16),
             (workloads.make_random_problem(77, 900, 3, 0.12, n_bumps=3, bump_width=0.5), "fp64", 5),
             (workloads.make_random_problem(78, 300, 2, 0.1, n_bumps=2, bump_width=0.5), "mixed", 1)]
    for prob, prec, nrhs in cases:
        print(f"[noalloc] n={prob.n} {prec} nrhs={nrhs}", flush=True)
        m = G.gp2s_assemble(prob.x, params_of(prob), prec)
        shape = (prob.n, nrhs) if nrhs > 1 else (prob.n,)
        X = torch.as_tensor(np.random.default_rng(nrhs).standard_normal(shape), device="cuda")
        ref = G.gp2s_spmv(m, X).cpu().numpy()
        Y = torch.full_like(X, float("nan"))
        torch.cuda.synchronize()
        before = _allocs(torch)
        G.gp2s_spmv_noalloc(m, X, Y)
        assert _allocs(torch) == before
        got = Y.cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        m.free()


def test_noalloc_limits(gpu):
    import torch
    import paper_2512_06143_amd as G
    prob = workloads.make_random_problem(79, 70_000, 2, 0.004, n_bumps=2, bump_width=0.6)
    m = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    X = torch.zeros((prob.n, 64), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(G.GP2SError) as e:  # 70 000 x 64 > 2^22 values
        G.gp2s_spmv_noalloc(m, X, Y)
    assert e.value.status == 1
    X1, Y1 = X[:, :32].contiguous(), Y[:, :32].contiguous()  # 70 000 x 32 <= 2^22
    G.gp2s_spmv_noalloc(m, X1, Y1)
    assert float(Y1.abs().max()) == 0.0
    ff = G.HostParams(2, 0.05, 0.5, 1e-3, np.array([[0.3, 0.3], [0.7, 0.6]]), np.array([1.0, 0.8]),
                      ff_groups=np.array([0, 1]))
    small = workloads.make_random_problem(80, 500, 2, 0.05, n_bumps=2, bump_width=0.5)
    mf = G.gp2s_assemble(small.x, ff, "fp64")
    Xf = torch.ones((small.n, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_spmv_noalloc(mf, Xf, torch.zeros_like(Xf))
    assert e.value.status == 1
