"""Mixed precision (leaf factor of M~ = alpha K~_1 + I computed and held in FP32, levels
and node factors FP64, solves refined by PCG in FP64), against the FP64 oracle.  Every
output's error is printed and held to a bound derived from the arithmetic:

  * solves refined by PCG to a relative residual rtol = 1e-10: the forward error is at
    most kappa(M~) rtol (relative);
  * the mixed factor is an FP64-exact factor of A + E, E block-diagonal over the leaves:
    each leaf's entries are rounded to FP32 (|dA| <= u32 |A|) and its Cholesky has the
    componentwise backward error |dA| <= gamma_(m+1) |L||L'| (Higham, Thm 10.3).  Its
    log-det moves by tr(A^-1 E) to first order, at most
    sum_leaves sum |A^-1|_(leaf,leaf) (u32 |A_leaf| + gamma_(m+1) |L||L'|), with A^-1 the
    inverse of the whole matrix;  u32 = 2^-24;
  * chain outputs: the Metropolis step uses only the FP64 factor of K~_1, so grid
    indices and accept flags are exact; tau and sigma_f^2 follow f (bounded like the
    solves); the log-likelihood carries the log-det bound.
"""
import math

import numpy as np
import pytest

from oracle import hodlr as oh, kernels, sampler
from workloads import SMALL_1D, small_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U32 = 2.0 ** -24


def fg():
    import paper_2006_06537_amd as m
    return m


def logdet_bound(H, alpha, OF):
    """First-order bound on the log-det error of a factor of alpha K~_1 + I whose leaf
    Choleskys are FP32 (everything else exact)."""
    Minv = np.abs(np.linalg.inv(alpha * H.dense() + np.eye(H.n)))
    b = 0.0
    for (lo, hi), Lb in zip(H.tree.leaves(), OF.leafL):
        m = hi - lo
        A = alpha * H.leaf_block(lo, hi) + np.eye(m)
        g = (m + 1) * U32 / (1.0 - (m + 1) * U32)
        E = U32 * np.abs(A) + g * (np.abs(Lb) @ np.abs(Lb).T)
        b += float(np.sum(Minv[lo:hi, lo:hi] * E))
    return b


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [(1000, 64, 0.1, 1e-12, 0, 100.0), (3001, 64, 0.03, 1e-10, 1, 400.0),
         (1537, 32, 0.01, 1e-10, 3, 50.0), (2048, 128, 0.02, 1e-10, 2, 400.0)]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}-B{c[1]}-a{c[5]:g}" for c in CASES])
def test_fp32_factor_refined_solve_and_logdet(case):
    n, leaf, ell, tol, seed, alpha = case
    x, _ = small_1d(n=n, seed=seed)
    dev = torch.device("cuda:0")
    K = fg().Hodlr(torch.tensor(x, device=dev), ell, nugget=1e-6, leaf=leaf, tol=tol)
    F32 = fg().Factor(K, alpha, 1.0, precision=fg().MIXED)
    assert F32.status() == 0
    H = oh.HODLR(x, kernels.SE, ell, 1e-6, leaf, tol)
    OF = oh.Factor(H, alpha, 1.0)
    M = alpha * H.dense() + np.eye(n)
    kappa = np.linalg.cond(M)
    b = np.random.default_rng(5).normal(size=(2, n))
    xs, its, rr = fg().solve_refined(K, F32, alpha, 1.0, torch.tensor(b, device=dev))
    ref = OF.solve(b.T).T
    err = rel(xs.cpu().numpy(), ref)
    ld = float(F32.logdet().cpu()[0])
    dld = abs(ld - OF.logdet())
    lb = logdet_bound(H, alpha, OF)
    print(f"n={n} alpha={alpha:g}: PCG {its} it, relres {rr:.2e}, solve err {err:.2e} "
          f"(bound {kappa * 1e-10:.1e}), logdet err {dld:.2e} (bound {lb:.1e})")
    assert rr <= 1e-10
    assert err <= kappa * 1e-10
    assert dld <= lb


def test_fp64_factor_refined_solve_converges_at_once():
    x, _ = small_1d(n=1200, seed=4)
    dev = torch.device("cuda:0")
    K = fg().Hodlr(torch.tensor(x, device=dev), 0.05, nugget=1e-6, leaf=64, tol=1e-10)
    F = fg().Factor(K, 30.0, 1.0)
    b = torch.tensor(np.random.default_rng(1).normal(size=1200), device=dev)
    xs, its, rr = fg().solve_refined(K, F, 30.0, 1.0, b)
    assert its <= 2 and rr <= 1e-10
    assert rel(xs.cpu().numpy(), F.solve(b).cpu().numpy()) <= 1e-9


def test_mixed_chain_against_fp64_oracle():
    c = SMALL_1D
    x, y = small_1d(c["n"], c["seed"])
    dev = torch.device("cuda:0")
    g = fg().Chain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0=c["ell0"],
                   tau0=c["tau0"], sigf2_0=c["sigf2_0"], nugget=c["nugget"], leaf=c["leaf"],
                   tol=c["tol"], seed=c["seed"], precision=fg().MIXED)
    o = sampler.Chain(x, y, kernels.SE, c["ell0"], c["nugget"], c["leaf"], c["tol"], c["tau0"],
                      c["sigf2_0"], c["seed"])
    worst = {}
    for it in range(10):
        tau_draw, s2_draw, Hprev = o.tau, o.sigf2, o.H
        g.step(1)
        s = g.state(with_vectors=(it == 9))
        r = o.step()
        assert s["status"] == 0 and s["pcg_relres"] <= 1e-10 and s["pcg_iters"] >= 1
        assert s["k"] == r["k"] and s["last_accept"] == int(r["accept"])
        Hd = Hprev  # K~_1 of the f-draw (before this sweep's Metropolis step)
        a = tau_draw * s2_draw
        M = a * Hd.dense() + np.eye(c["n"])
        kappa = np.linalg.cond(M)
        worst["kappa"] = max(worst.get("kappa", 0.0), kappa)
        lb = logdet_bound(Hd, a, oh.Factor(Hd, a, 1.0))
        for key in ["tau", "sigf2"]:
            e = abs(s[key] - r[key]) / abs(r[key])
            worst[key] = max(worst.get(key, 0.0), e)
            assert e <= kappa * 1e-10, (it, key, e)
        dl = abs(s["loglik"] - r["loglik"])
        worst["loglik"] = max(worst.get("loglik", 0.0), dl)
        # loglik = -n/2 log 2 pi - 1/2 (log|M~| - n log tau) - 1/2 y'r
        assert dl <= 0.5 * lb + 0.5 * kappa * 1e-10 * abs(r["yr"]), (it, dl, lb)
    f = s["f"].cpu().numpy()
    worst["f"] = rel(f, o.f)
    print("mixed chain vs FP64 oracle, worst errors:", worst)
    assert worst["f"] <= worst["kappa"] * 1e-10


def _lambda_max(H, its=12, seed=0):
    """Largest eigenvalue of the oracle's K~_1 by power iteration (a slight
    underestimate; the bars below double it)."""
    v = np.random.default_rng(seed).normal(size=H.n)
    lam = 0.0
    for _ in range(its):
        w = H.matvec(v)
        lam = float(v @ w) / float(v @ v)
        v = w / np.linalg.norm(w)
    return lam


def test_mixed_chain_large_n_stays_mixed():
    """n = 2^17 at tau sigma_f^2 = 400, where kappa(M~) u32 > 1 (an all-FP32 factor breaks
    down here): with FP32 leaves and FP64 levels the chain stays in mixed precision, every
    PCG solve reaches 1e-10, and two sweeps match the FP64 oracle's chain -- the same grid
    moves, f, tau and sigma_f^2 within kappa(M~) 1e-10."""
    from workloads import sinusoid_1d
    n = 1 << 17
    x, y = sinusoid_1d(n, seed=7)
    dev = torch.device("cuda:0")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    kw = dict(ell0=0.02, tau0=400.0, leaf=128, tol=1e-10, seed=7)
    m = fg().Chain(xt, yt, precision=fg().MIXED, **kw)
    o = sampler.Chain(x, y, kernels.SE, 0.02, 1e-6, 128, 1e-10, 400.0, 1.0, 7)
    for it in range(2):
        a_draw = o.tau * o.sigf2
        kappa = 1.0 + 2.0 * a_draw * _lambda_max(o.H)
        m.step(1)
        s = m.state(with_vectors=True)
        r = o.step()
        ef = rel(s["f"].cpu().numpy(), o.f)
        print(f"sweep {it}: kappa(M~) <= {kappa:.2e}, PCG {s['pcg_iters']} it, relres "
              f"{s['pcg_relres']:.1e}; f err {ef:.2e}, tau err "
              f"{abs(s['tau'] - r['tau']) / r['tau']:.2e}, sigf2 err "
              f"{abs(s['sigf2'] - r['sigf2']) / r['sigf2']:.2e}, D {r.get('mh_log_ratio')}")
        assert s["precision_used"] == fg().MIXED and s["status"] == 0
        assert 1 <= s["pcg_iters"] and s["pcg_relres"] <= 1e-10
        assert (s["k"], s["last_proposal"], s["last_accept"]) == (r["k"], r["proposal"], int(r["accept"]))
        assert ef <= kappa * 1e-10 + 1e-8
        e = np.linalg.norm(y - o.f)
        assert abs(s["tau"] - r["tau"]) <= (2.0 * (kappa * 1e-10 + 1e-8) * np.linalg.norm(o.f) / e
                                            + 1e-9) * r["tau"]
