"""Function posterior at new inputs (gibbs_predict_inputs / gibbs_predict) against the
oracle (oracle/predict.py) on the chain's state after each sweep.

Bars.  mu*_j = Z_j . z and s2*_j = sigma_f^2 (1 + eta - |Z_j|^2) are sums whose terms
come from W_1^-1, held elsewhere to the W-operator bar b_W = max(1e-9, 2 u kappa(leaf))
(plus four times the oracle's reproducibility band, measured here by redoing the
prediction with the oracle's unblocked-leaf variant and with its panels perturbed by a few
rounding units).  A relative error b_W in Z_j and z
moves mu*_j by at most 2 b_W |Z_j||z| and s2*_j by 2 b_W sigma_f^2 |Z_j|^2; sqrt moves
by at most the square root of its argument's change, which bounds f*."""
import numpy as np
import pytest

from oracle import hodlr as oh, kernels, predict, rng, sampler
from workloads import SMALL_1D, small_1d
from bands import InvLeafFactor, perturbed_panels

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


def _bars(o, xs, xi, ref):
    H, W1 = o.H, o.W1
    kap = max(np.linalg.cond(H.leaf_block(lo, hi)) for lo, hi in H.tree.leaves())
    bw = max(1e-9, 2.0 * 2.0 ** -53 * kap)
    var_mu, var_s2 = np.zeros(xs.size), np.zeros(xs.size)
    for Hv, Wv in [(H, InvLeafFactor(H, 1.0, 0.0))] + [
            (Hp, oh.Factor(Hp, 1.0, 0.0)) for Hp in [perturbed_panels(H, seed=s_) for s_ in (1, 2)]]:
        v = predict.predict(Hv, Wv, o.f, o.sigf2, xs, xi)
        var_mu = np.maximum(var_mu, np.abs(v[1] - ref[1]))
        var_s2 = np.maximum(var_s2, np.abs(v[2] - ref[2]))
    Kx = kernels.k1(H.kind, H.ell, H.x, xs)
    zn = np.linalg.norm(W1.apply_Winv(Kx), axis=0)
    zf = np.linalg.norm(W1.apply_Winv(o.f))
    b_mu = 2.0 * bw * zn * zf + 4.0 * var_mu + 1e-15
    b_s2 = 2.0 * bw * o.sigf2 * (1.0 + zn ** 2) + 4.0 * var_s2 + 1e-15
    b_f = b_mu + np.sqrt(b_s2) * np.abs(xi)
    return b_mu, b_s2, b_f


def _check(g, o, xs, seed, stream=0):
    fs, mu, s2 = (t.cpu().numpy() for t in g.predict())
    xi = rng.normals(xs.size, seed, rng.TAG_PRED, o.it, stream)
    ref = predict.predict(o.H, o.W1, o.f, o.sigf2, xs, xi)
    b_mu, b_s2, b_f = _bars(o, xs, xi, ref)
    assert np.all(np.abs(mu - ref[1]) <= b_mu), np.max(np.abs(mu - ref[1]) / b_mu)
    assert np.all(np.abs(s2 - ref[2]) <= b_s2), np.max(np.abs(s2 - ref[2]) / b_s2)
    assert np.all(np.abs(fs - ref[0]) <= b_f), np.max(np.abs(fs - ref[0]) / b_f)
    return ref


def _chain(x, y, c, seed):
    dev = torch.device("cuda:0")
    g = fg().Chain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0=c["ell0"],
                   tau0=c["tau0"], sigf2_0=c["sigf2_0"], nugget=c["nugget"], leaf=c["leaf"],
                   tol=c["tol"], seed=seed)
    o = sampler.Chain(x, y, kernels.SE, c["ell0"], c["nugget"], c["leaf"], c["tol"], c["tau0"],
                      c["sigf2_0"], seed)
    return g, o


def test_predict_follows_the_chain():
    """37 new inputs (ragged: several 16-lane groups and a tail) -- inside the data,
    outside its range, repeated, and equal to training inputs -- after each of eight
    sweeps; Z is kept while the length-scale stays and rebuilt when it moves."""
    c = SMALL_1D
    x, y = small_1d(c["n"], c["seed"])
    g, o = _chain(x, y, c, c["seed"])
    rs = np.random.default_rng(4)
    xs = np.concatenate([rs.uniform(0, 1, 25), [-0.3, 1.4, 7.0], x[[0, 10, 500, -1]],
                         [0.5, 0.5], rs.uniform(0.2, 0.3, 3)])
    assert xs.size == 37
    g.predict_inputs(torch.tensor(xs, device="cuda"), max_grid_points=2)
    ks = []
    for it in range(12):
        g.step(1)
        o.step()
        ks.append(o.k)
        ref = _check(g, o, xs, c["seed"])
        # the prior far from the data
        assert ref[1][27] == 0.0 and ref[2][27] == pytest.approx(o.sigf2 * (1 + c["nugget"]))
        cached, builds = g.predict_stats()
        assert cached == min(2, len(set(ks)))
    assert len(set(ks)) > 2, "the length-scale visited too few grid points to evict"
    assert builds >= len(set(ks))


def test_predict_before_a_sweep_and_single_point():
    """Before any sweep f = 0, so mu* = 0; a single new input (no full 16-lane group)."""
    c = SMALL_1D
    x, y = small_1d(300, 8)
    g, o = _chain(x, y, c, 11)
    g.predict_inputs(torch.tensor([0.42], dtype=torch.float64, device="cuda"))
    fs, mu, s2 = (t.cpu().numpy() for t in g.predict())
    assert mu[0] == 0.0
    ref = predict.predict(o.H, o.W1, o.f, o.sigf2, np.array([0.42]),
                          rng.normals(1, 11, rng.TAG_PRED, 0, 0))
    assert abs(s2[0] - ref[2][0]) <= 1e-9 * o.sigf2
    g.step(2)
    o.step(); o.step()
    _check(g, o, np.array([0.42]), 11)
    # new inputs replace the old ones
    g.predict_inputs(torch.tensor([0.1, 0.9, 0.95], dtype=torch.float64, device="cuda"))
    _check(g, o, np.array([0.1, 0.9, 0.95]), 11)


def test_cache_size_does_not_change_the_draws():
    """Z rebuilt on every move (one slot) and Z kept for every grid point give bitwise
    equal draws: each build is the same deterministic computation."""
    c = SMALL_1D
    x, y = small_1d(700, 5)
    xs = torch.tensor(np.linspace(-0.05, 1.05, 19), device="cuda")
    out = []
    for cap in (1, 8):
        g, _ = _chain(x, y, c, 21)
        g.predict_inputs(xs, max_grid_points=cap)
        draws = []
        for it in range(10):
            g.step(1)
            draws.append(torch.stack(g.predict()).cpu())
        out.append((torch.stack(draws), g.predict_stats()))
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1][1] >= out[1][1][1]


def test_predict_errors():
    c = SMALL_1D
    x, y = small_1d(200, 3)
    g, _ = _chain(x, y, c, 1)
    with pytest.raises(fg().FgError):
        g.predict()  # no inputs set
    g.predict_inputs(torch.tensor([0.5], dtype=torch.float64, device="cuda"))
    g.predict_inputs(None)
    with pytest.raises(fg().FgError):
        g.predict()
