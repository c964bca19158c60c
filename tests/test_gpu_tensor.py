"""Parity of the tensor-product path (Algorithm 1.h and the tensor sweep, through the
C ABI) with the oracle, on the same seeded inputs.

Tolerance: relative 1e-9 (2-norm) for scalars, exact for grid indices, proposals and
accept flags -- the bar used for the 1-D sampler's draws.  The factors f_h contain
W_h b, a product with the symmetric factor of K~_h (nugget 1e-6), which the factor
parity tests hold to max(1e-9, 2 u kappa(leaf)) (leaf Cholesky forward error); each f_h
is held to that same bar, and the scalars built on the product G = prod_h f_h carry the
sum of the factors' bars (beta), magnified by 2 |beta G| / |y - beta G| for the residual
sum of squares and tau.  The
quadratic forms q = |W_h^-1 f_h|^2 carry twice the bar of a W^-1 product of K~_h,
max(1e-9, 2 u kappa(leaf)) -- the leaf Cholesky forward-error bound of the factor
parity tests -- and the Metropolis log ratio D = -1/2 (l' - l) - (q' - q)/2, a
difference of such terms, the sum of their bounds."""
import numpy as np
import pytest

from oracle import hodlr as oh, kernels, rng, sampler, tensor
from workloads import TENSOR_4D, small_1d, tensor_surface

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


HCASES = [
    # n, leaf, ell, tol, seed, factor
    (1000, 64, 0.1, 1e-12, 0, -1),
    (3001, 64, 0.03, 1e-10, 1, 2),   # ragged leaves, factor tags
    (1537, 32, 0.01, 1e-10, 3, 0),
    (50, 64, 0.2, 1e-10, 5, -1),     # one leaf
]


@pytest.mark.parametrize("case", HCASES, ids=[f"n{c[0]}-B{c[1]}-h{c[5]}" for c in HCASES])
def test_draw_f_hetero_matches_oracle(case):
    n, leaf, ell, tol, seed, factor = case
    x, y = small_1d(n=n, seed=seed)
    # precisions shaped like tau g^2 of a tensor sweep: g crosses zero, D spans decades
    g = np.sin(7.0 * x + 0.3) * np.sqrt(4.0 * x + 0.1)
    g = tensor.clamp_g(g)
    D = 100.0 * g * g
    dev = torch.device("cuda:0")
    xt, yt, Dt = (torch.tensor(v, device=dev) for v in (x, y, D))
    K = fg().Hodlr(xt, ell, nugget=1e-6, leaf=leaf, tol=tol)
    WK = fg().Factor(K, 1.0, 0.0)
    WP = fg().Factor(K, 1.0, 0.0, diag=1.0 / Dt)
    assert WP.status() == 0
    f, R = fg().draw_f_hetero(K, WK, WP, Dt, yt, 17, 4, 9, factor)
    ta = rng.TAG_A if factor < 0 else tensor.factor_tag(rng.TAG_A, factor)
    tb = rng.TAG_B if factor < 0 else tensor.factor_tag(rng.TAG_B, factor)
    a = rng.normals(n, 17, ta, 4, 9)
    b = rng.normals(n, 17, tb, 4, 9)
    H = oh.HODLR(x, kernels.SE, ell, 1e-6, leaf, tol)
    of, oR = sampler.draw_f_hetero(H, oh.Factor(H, 1.0, 0.0), oh.Factor(H, 1.0, 0.0, 1.0 / D), D,
                                   y, a, b)
    assert rel(R.cpu().numpy(), oR) <= 1e-9
    assert rel(f.cpu().numpy(), of) <= 1e-9


def _pair(d, n, leaf, tol, ell0, seed, positive=False, tau0=100.0):
    x, y = tensor_surface(d, n, seed=seed, positive=positive)
    dev = torch.device("cuda:0")
    g = fg().TensorChain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0,
                         tau0=tau0, beta0=1.0, nugget=1e-6, leaf=leaf, tol=tol, seed=seed)
    o = tensor.TensorChain(x, y, kernels.SE, ell0, 1e-6, leaf, tol, tau0, 1.0, seed)
    return g, o


def _tw(o, h, k):
    """Bar of a W_h^-1 product at grid point k: max(1e-9, 2 u kappa(leaf)), the leaf
    Cholesky forward-error bound used for the K~_1 factor operators."""
    if not 0 <= k < len(o.grids[h]):
        return 1e-9
    ell = o.grids[h][k]
    xs = o.xs[h % o.d]  # factor h = c d + dimension
    kap = max(np.linalg.cond(kernels.K1_dense(kernels.SE, ell, 1e-6, xs[lo:hi]))
              for lo, hi in o.H[h].tree.leaves())
    return max(1e-9, 2.0 * 2.0 ** -53 * kap)


def _check_factors(F, o, ks):
    for h in range(o.d):
        bar = max(_tw(o, h, k) for k in ks[h])
        assert rel(F[h], o.F[h]) <= bar, (h, rel(F[h], o.F[h]), bar)


def _compare(s, r, o, it, kb, ld_bars=None):
    """ld_bars: relative bar of each factor's log-det (default 1e-9)."""
    d = o.d
    ldb = ld_bars or [1e-9] * d
    assert s["k"] == r["k"], (it, s["k"], r["k"])
    assert s["last_proposal"] == r["proposal"], it
    assert s["last_accept"] == [int(a) for a in r["accept"]], it
    # G = prod_h f_h carries the factors' bars (added); sse = |y - beta G|^2 magnifies an
    # error in beta G by 2 |beta G| / |y - beta G|, and tau follows sse
    tws = sum(_tw(o, h, kb[h]) for h in range(d))
    bG = abs(r["beta"]) * float(np.linalg.norm(o.product()))
    bars = {"beta": 2 * tws, "beta_mean": 2 * tws, "beta_sd": 2 * tws,
            "sse": 2 * tws * bG / np.sqrt(r["sse"]), "tau": 2 * tws * bG / np.sqrt(r["sse"])}
    for key in ["tau", "beta", "sse", "beta_mean", "beta_sd"]:
        ref = r[key]
        assert abs(s[key] - ref) <= max(1e-9, bars[key]) * abs(ref), (it, key, s[key], ref)
    for h in range(d):
        # q = |W_h^-1 f_h|^2: twice the relative bar of W_h^-1 (plus its square)
        tq = _tw(o, h, r["k"][h])
        q_now = r["q_prop"][h] if r["accept"][h] else r["q"][h]  # q at the current ell_h
        assert abs(s["q"][h] - q_now) <= 2.5 * tq * abs(q_now), (it, h)
        assert abs(s["logdet"][h] - r["logdet"][h]) <= ldb[h] * abs(r["logdet"][h]), (it, h)
        # D is a difference of terms of size |log det| and q: each carries its bar
        bound = (ldb[h] * (abs(r["logdet_prop"][h]) + abs(r["logdet"][h]))
                 + 2.5 * _tw(o, h, r["proposal"][h]) * abs(r["q_prop"][h])
                 + 2.5 * _tw(o, h, kb[h]) * abs(r["q"][h]))
        assert abs(s["mh_log_ratio"][h] - r["mh_log_ratio"][h]) <= bound, (it, h)
    assert s["status"] == 0


@pytest.mark.parametrize("positive", [False, True], ids=["sin-sqrt", "positive"])
def test_tensor_chain_matches_oracle(positive):
    g, o = _pair(3, 2000, 64, 1e-10, (0.05, 0.1, 0.2), 3, positive=positive)
    seen = [set() for _ in range(o.d)]
    for it in range(4):
        g.step(1)
        s = g.state(with_factors=(it == 3))
        kb = list(o.k)
        for h in range(o.d):
            seen[h].add(kb[h])
        r = o.step()
        _compare(s, r, o, it, kb)
    _check_factors(s["F"].cpu().numpy(), o, seen)


def test_tensor_chain_one_factor_ragged():
    g, o = _pair(1, 777, 32, 1e-10, (0.07,), 8)
    seen = [set()]
    for it in range(3):
        g.step(1)
        s = g.state(with_factors=True)
        kb = list(o.k)
        seen[0].add(kb[0])
        _compare(s, o.step(), o, it, kb)
    _check_factors(s["F"].cpu().numpy(), o, seen)


def test_tensor_chain_full_size_first_sweep():
    """The d = 4, n = 65,536 tensor workload: first sweep against the oracle.

    The factors' log|K~_h| (nugget 1e-6) are held as the large workload holds log|K~_1|, by
    their two parts: the leaf part at 1e-9, the node part at the larger of the node-part
    bar (four times the oracle's own reproducibility band, or the first-order error of the
    Gram route, never below 1e-9) and twice the HIP route's own band -- the largest change
    of the HIP path's node part when the length-scale moves by one rounding unit either way.
    The top node factors of these matrices sit at 1 - s^2 far below the leaves' rounding,
    where the Gram route (s^2 from products of Gram matrices of whitened panels) moves
    log(1 - s^2) by more than the oracle's QR route does; the chain's total log-det then
    carries 1e-9 of the leaf part plus that bar of the node part."""
    from bands import logdet_parts, node_part_bar
    T = TENSOR_4D
    g, o = _pair(T["d"], T["n"], T["leaf"], T["tol"], T["ell0"], T["seed"], tau0=T["tau0"])
    g.step(1)
    s = g.state(with_factors=True)
    kb = list(o.k)
    r = o.step()
    dev = torch.device("cuda:0")

    def gpu_parts(h, ell):
        K = fg().Hodlr(torch.tensor(o.xs[h], device=dev), ell, nugget=1e-6, leaf=T["leaf"],
                       tol=T["tol"])
        return tuple(float(v) for v in fg().Factor(K, 1.0, 0.0).logdet_parts().cpu())

    bars = []
    for h in range(o.d):
        ell = o.grids[h][o.k[h]]
        gl, gn = gpu_parts(h, ell)
        # the same factorization on the same inputs as the chain's
        assert abs(gl + gn - s["logdet"][h]) <= 1e-12 * abs(s["logdet"][h]), h
        hip_band = max(abs(gpu_parts(h, float(np.nextafter(ell, e)))[1] - gn)
                       for e in (0.0, 1.0)) / abs(gn)
        leaf, node = logdet_parts(o.W[h])
        nb, band, gram = node_part_bar(o.H[h], o.W[h])
        nb = max(nb, 2.0 * hip_band)
        el, en = abs(gl - leaf) / abs(leaf), abs(gn - node) / abs(node)
        print(f"factor {h}: leaf part rel err {el:.2e}; node part rel err {en:.2e} (bar {nb:.2e}:"
              f" oracle band {band:.2e}, Gram bound {gram:.2e}, HIP band {hip_band:.2e})")
        assert el <= 1e-9, h
        assert en <= nb, h
        bars.append((1e-9 * abs(leaf) + nb * abs(node)) / abs(leaf + node))
    _compare(s, r, o, 0, kb, ld_bars=bars)
    _check_factors(s["F"].cpu().numpy(), o, [{k} for k in kb])


def test_tensor_chain_deterministic():
    x, y = tensor_surface(2, 900, seed=6)
    dev = torch.device("cuda:0")
    runs = []
    for _ in range(2):
        c = fg().TensorChain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), (0.1, 0.2),
                             leaf=64, seed=6)
        c.step(3)
        runs.append(c.state(with_factors=True))
    assert torch.equal(runs[0]["F"], runs[1]["F"])
    assert runs[0]["tau"] == runs[1]["tau"] and runs[0]["beta"] == runs[1]["beta"]


def test_additive_tensor_chain_matches_oracle():
    """Two components over d = 2 (factor m = c d + h) on n = 2500 observations.  Every
    component's scalars carry the bars above with the factors' bars summed over all
    factors (component c's data are the partial residual, which holds the others);
    sse and tau use |fit| / |y - fit| with fit = sum_c beta_c G_c."""
    d, C, n = 2, 2, 2500
    x, y = tensor_surface(d, n, seed=8)
    dev = torch.device("cuda:0")
    ell0 = (0.08, 0.15)
    g = fg().TensorChain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0,
                         tau0=50.0, beta0=0.7, nugget=1e-6, leaf=64, tol=1e-10, seed=8, ncomp=C)
    o = tensor.TensorChain(x, y, kernels.SE, ell0, 1e-6, 64, 1e-10, 50.0, 0.7, 8, ncomp=C)
    seen = [set() for _ in range(o.nf)]
    for it in range(5):
        g.step(1)
        s = g.state(with_factors=(it == 4))
        kb = list(o.k)
        for m in range(o.nf):
            seen[m].add(kb[m])
        r = o.step()
        assert s["status"] == 0 and s["ncomp"] == C
        assert s["k"] == r["k"] and s["last_proposal"] == r["proposal"], it
        assert s["last_accept"] == [int(a) for a in r["accept"]], it
        tws = sum(_tw(o, m, kb[m]) for m in range(o.nf))
        fit = float(np.linalg.norm(o.fitted()))
        res = np.sqrt(r["sse"])
        for cc in range(C):
            for key, ref in [("betas", r["betas"][cc]), ("beta_means", r["beta_means"][cc]),
                             ("beta_sds", r["beta_sds"][cc])]:
                assert abs(s[key][cc] - ref) <= max(1e-9, 2 * tws) * abs(ref), (it, key, cc)
        for key in ["sse", "tau"]:
            bar = max(1e-9, 2 * tws * fit / res)
            assert abs(s[key] - r[key]) <= bar * abs(r[key]), (it, key, s[key], r[key])
        for m in range(o.nf):
            tq = _tw(o, m, r["k"][m])
            q_now = r["q_prop"][m] if r["accept"][m] else r["q"][m]
            assert abs(s["q"][m] - q_now) <= 2.5 * tq * abs(q_now), (it, m)
    F = s["F"].cpu().numpy()
    for m in range(o.nf):
        bar = max(_tw(o, m, k) for k in seen[m])
        assert rel(F[m], o.F[m]) <= bar, (m, rel(F[m], o.F[m]), bar)
