"""The exact discrete length-scale conditional (gibbs_chain_create_grid) against the
oracle's grid chain (oracle/exact_rho.py), sweep by sweep.

The drawn grid index is an FP64 decision on both sides (same log-weights up to the q bar,
same uniform, same cumulative order): it must agree unless the uniform falls within the
log-weights' bar of a cumulative boundary, which is checked and reported.  f, tau, sigma_f^2
and the log-likelihood take the plain chain's 1e-9; q_h takes 2.5 times the W-operator bar
max(1e-9, 2 u kappa(leaf)); the drawn index's log-probability takes that bar times the
spread of the q_h / (2 sigma_f^2) terms."""
import numpy as np
import pytest

from oracle import exact_rho, kernels, sampler
from workloads import SMALL_1D, small_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


G, CENTER = 15, 7


def _pair(n, seed):
    c = SMALL_1D
    x, y = small_1d(n, seed)
    dev = torch.device("cuda:0")
    g = fg().Chain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0=c["ell0"],
                   tau0=c["tau0"], sigf2_0=c["sigf2_0"], nugget=c["nugget"], leaf=c["leaf"],
                   tol=c["tol"], seed=seed, grid_size=G, grid_center=CENTER, exact_rho=True)
    grid = sampler.ell_grid(c["ell0"], G, CENTER)  # the library's grid values
    o = exact_rho.ExactGridChain(x, y, kernels.SE, c["ell0"], c["nugget"], c["leaf"], c["tol"],
                                 c["tau0"], c["sigf2_0"], seed, grid=grid)
    return g, o


@pytest.mark.parametrize("n,seed", [(1000, 0), (2500, 3)])
def test_grid_chain_matches_oracle(n, seed):
    g, o = _pair(n, seed)
    moved = 0
    for it in range(10):
        kap = max(np.linalg.cond(o.H.leaf_block(lo, hi)) for lo, hi in o.H.tree.leaves())
        b = max(1e-9, 2.0 * 2.0 ** -53 * kap)
        g.step(1)
        s = g.state(with_vectors=True)
        k_before = o.k
        r = o.step()
        assert s["status"] == 0
        if s["k"] != r["k"]:
            lp = r["lp"]
            w = np.exp(lp - lp.max())
            c = np.cumsum(w)
            margin = np.min(np.abs(c - r["u_rho"] * c[-1])) / c[-1]
            spread = 2.5 * b * np.max(np.abs(r["q_all"])) / (2.0 * r["sigf2"])
            assert margin < 4.0 * spread, (it, s["k"], r["k"], margin)
            print(f"sweep {it}: near-tie of the inverse CDF (margin {margin:.2e}); stopping")
            return
        moved += r["k"] != k_before
        assert s["last_accept"] == int(r["k"] != k_before)
        for key in ["tau", "sigf2", "loglik"]:
            assert abs(s[key] - r[key]) <= 1e-9 * abs(r[key]), (it, key, s[key], r[key])
        f = s["f"].cpu().numpy()
        assert np.linalg.norm(f - o.f) <= 1e-9 * np.linalg.norm(o.f)
        qk = r["q_all"][r["k"]]
        assert abs(s["q"] - qk) <= 2.5 * b * qk, (it, s["q"], qk)
        spread = 2.5 * b * np.max(np.abs(r["q_all"])) / (2.0 * r["sigf2"])
        assert abs(s["mh_log_ratio"] - r["mh_log_ratio"]) <= 2.0 * spread + 1e-12
    assert moved > 0, "the length-scale never moved"


def test_grid_chains_batched_with_graphs_equal_eager():
    a, _ = _pair(800, 5)
    b, _ = _pair(800, 6)
    a2, _ = _pair(800, 5)
    b2, _ = _pair(800, 6)
    fg().step_batch([a, b], iters=6, nstreams=2, graphs=True)
    a2.step(6)
    b2.step(6)
    for u, v in [(a, a2), (b, b2)]:
        su, sv = u.state(with_vectors=True), v.state(with_vectors=True)
        assert su["k"] == sv["k"] and su["tau"] == sv["tau"] and su["accepts"] == sv["accepts"]
        assert torch.equal(su["f"], sv["f"])
