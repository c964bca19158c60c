"""hodlr_solve_refined_noalloc (the refined solve on the library's fixed scratch array,
no allocation) against hodlr_solve_refined on the same inputs, through the C ABI: two
calls in a row, the second with a smaller input, each matching the allocating entry
point to the solve's own bar (the same PCG arithmetic: iterations equal, solutions to
1e-12 relative); and the size limit is enforced."""
import numpy as np
import pytest

from workloads import small_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


def _case(n, nrhs, ell, alpha, seed):
    x, _ = small_1d(n=n, seed=seed)
    dev = torch.device("cuda:0")
    K = fg().Hodlr(torch.tensor(x, device=dev), ell, nugget=1e-6, leaf=64, tol=1e-10)
    F = fg().Factor(K, alpha, 1.0, precision=fg().MIXED)
    b = torch.tensor(np.random.default_rng(seed).normal(size=(nrhs, n)), device=dev)
    return K, F, b.reshape(-1) if nrhs == 1 else b


def test_noalloc_matches_allocating_solve_twice():
    for n, nrhs, ell, alpha, seed in [(3001, 2, 0.03, 400.0, 1), (1200, 1, 0.05, 50.0, 2)]:
        K, F, b = _case(n, nrhs, ell, alpha, seed)
        ref, it_ref, rr_ref = fg().solve_refined(K, F, alpha, 1.0, b)
        out = torch.empty_like(b)
        got, it, rr = fg().solve_refined(K, F, alpha, 1.0, b, noalloc=True, out=out)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
        print(f"n={n} nrhs={nrhs}: {it} iterations (allocating: {it_ref}), relres {rr:.1e}, "
              f"difference {err:.1e}")
        assert it == it_ref and rr <= 1e-10
        assert err <= 1e-12


def test_noalloc_rejects_inputs_beyond_its_array():
    n = 300_000  # 4 right-hand sides exceed 2^20 entries
    x = np.sort(np.random.default_rng(0).uniform(0, 1, n))
    dev = torch.device("cuda:0")
    K = fg().Hodlr(torch.tensor(x, device=dev), 0.05, nugget=1e-6, leaf=128, tol=1e-8)
    F = fg().Factor(K, 10.0, 1.0)
    b = torch.zeros((4, n), dtype=torch.float64, device=dev)
    with pytest.raises(fg().FgError, match="scratch"):
        fg().solve_refined(K, F, 10.0, 1.0, b, noalloc=True)
