"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element on
the same seeded inputs.

Tolerances
  * integers (ranks, grid indices, accept flags): exact;
  * K~_1 entries, matrix-vector products, everything built on M~ = alpha K~_1 + I and
    the outputs the sampler reports (log-determinants, posterior mean, draws): relative
    1e-9 (2-norm);
  * the symmetric factor of K~_1 itself (alpha = 1, beta = 0, nugget 1e-6): two FP64
    evaluations of the same canonical W differ by more than 1e-9 because its node
    factors sit at 1 - sigma^2 ~ 1e-7.  The bound used is the oracle's own
    reproducibility band -- the distance between the oracle and the same oracle with
    its leaf Cholesky computed column by column and its leaf triangular solves replaced by
    explicit inverses -- times 4, and never below 1e-9; for the operators W, W', W^-1,
    W^-T and the solve also never below the Cholesky forward-error bound 2 u kappa(leaf).
"""
import numpy as np
import pytest

from oracle import hodlr as oh, kernels, kalman, rng, sampler
from workloads import small_1d, sinusoid_1d
from bands import InvLeafFactor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    # n, leaf, ell, tol, kernel, seed
    (1000, 64, 0.1, 1e-12, kernels.SE, 0),    # small 1-D workload shape
    (3001, 64, 0.03, 1e-10, kernels.SE, 1),   # ragged leaves 93/94
    (2048, 128, 0.3, 1e-8, kernels.SE, 2),    # smooth kernel, large leaves
    (1537, 32, 0.01, 1e-10, kernels.SE, 3),   # many levels, small leaves
    (1200, 64, 0.05, 1e-10, kernels.EXP, 4),  # exponential kernel: rank-one blocks
    (50, 64, 0.2, 1e-10, kernels.SE, 5),      # one leaf: W = Cholesky factor
    (900, 16, 1e-4, 1e-10, kernels.SE, 6),    # empty windows: rank-zero nodes
    (1500, 64, 0.05, 1e-10, kernels.MATERN32, 7),
    (2000, 64, 0.08, 1e-10, kernels.MATERN52, 8),
]
IDS = [f"n{c[0]}-B{c[1]}-ell{c[2]}-k{c[4]}" for c in CASES]


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def case(request):
    n, leaf, ell, tol, kind, seed = request.param
    x, y = small_1d(n=n, seed=seed)
    dev = torch.device("cuda:0")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    K1 = fg().Hodlr(xt, ell, nugget=1e-6, leaf=leaf, tol=tol, kind=kind)
    H = oh.HODLR(x, kind, ell, 1e-6, leaf, tol)
    return dict(n=n, x=x, y=y, xt=xt, yt=yt, K1=K1, H=H, ell=ell, kind=kind, dev=dev)


def test_normals_bitwise_stream():
    z = fg().normals(4099, 11, 2, 7, 3).cpu().numpy()
    ref = rng.normals(4099, 11, 2, 7, 3)
    assert np.abs(z - ref).max() < 4 * np.finfo(float).eps * np.abs(ref).max()


def test_ranks_match(case):
    H, K1 = case["H"], case["K1"]
    assert K1.status() == 0
    got = K1.ranks()
    ref = [H.blocks[(l, j)].k for l in range(H.tree.L) for j in range(1 << l)]
    assert len(got) == len(ref)
    diff = [h for h in range(len(ref)) if got[h] != ref[h]]
    # a mismatch is only acceptable at a documented near-tie of the rank rule
    for h in diff:
        l = int(np.log2(h + 1))
        b = H.blocks[(l, h - (1 << l) + 1)]
        margin = np.min(np.abs(b.sv / b.thr - 1.0))
        assert margin < 1e-9, (h, got[h], ref[h], margin)


def test_entries_match_dense(case):
    n, H, K1 = case["n"], case["H"], case["K1"]
    dev = case["dev"]
    ii = torch.arange(n, device=dev).repeat_interleave(n)
    jj = torch.arange(n, device=dev).repeat(n)
    E = K1.entries(ii, jj).reshape(n, n).cpu().numpy()
    A = H.dense()
    assert np.abs(E - A).max() <= 1e-9 * np.abs(A).max()
    # the matrix the GPU holds meets the max-norm bound too
    K = kernels.K1_dense(case["kind"], case["ell"], 1e-6, case["x"])
    assert np.abs(E - K).max() <= case["H"].tol


def test_singular_values_match(case):
    H, K1 = case["H"], case["K1"]
    sv = K1.singular_values()
    for (l, j), b in H.blocks.items():
        h = (1 << l) - 1 + j
        m = min(len(b.sv), 60)
        if m == 0:
            continue
        g = np.array(sv[h][:m])
        assert np.abs(g - b.sv[:m]).max() <= 1e-12 * b.sv[0] + 1e-300


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (100.0, 1.0)])
def test_factor_logdet_apply_solve(case, alpha, beta):
    n, H, K1 = case["n"], case["H"], case["K1"]
    F = fg().Factor(K1, alpha, beta)
    assert F.status() == 0
    OF = oh.Factor(H, alpha, beta)
    v = np.random.default_rng(1).normal(size=(2, n))
    vt = torch.tensor(v, device=case["dev"])
    ld = float(F.logdet().cpu()[0])
    band = {}
    if beta == 0.0:
        OV = InvLeafFactor(H, alpha, beta)
        band["logdet"] = abs(OV.logdet() - OF.logdet()) / abs(OF.logdet())
        for nm, fn in [("W", "apply_W"), ("WT", "apply_WT"), ("Winv", "apply_Winv"),
                       ("WinvT", "apply_WinvT"), ("solve", "solve")]:
            band[nm] = rel(getattr(OV, fn)(v.T), getattr(OF, fn)(v.T))

    # forward-error bound of a Cholesky factor: ~ u kappa(leaf) (relative), whatever the
    # summation order; leaves of alpha K~_1 + beta I with a 1e-6 nugget reach kappa ~ 1e7
    kap = max(np.linalg.cond(alpha * H.leaf_block(lo, hi) + beta * np.eye(hi - lo))
              for lo, hi in H.tree.leaves())
    u = 2.0 ** -53

    def tol(nm):
        t = max(1e-9, 4.0 * band.get(nm, 0.0))
        if nm != "logdet":
            t = max(t, 2.0 * u * kap)
        return t

    assert abs(ld - OF.logdet()) <= tol("logdet") * abs(OF.logdet()) + 1e-12
    for nm, t, i, fn in [("W", 0, 0, "apply_W"), ("WT", 1, 0, "apply_WT"),
                         ("Winv", 0, 1, "apply_Winv"), ("WinvT", 1, 1, "apply_WinvT")]:
        g = F.apply(vt, transpose=bool(t), inverse=bool(i)).cpu().numpy().T
        assert rel(g, getattr(OF, fn)(v.T)) <= tol(nm), nm
    s = F.solve(vt).cpu().numpy().T
    assert rel(s, OF.solve(v.T)) <= tol("solve")


def test_factor_heteroskedastic_diagonal(case):
    n, H, K1 = case["n"], case["H"], case["K1"]
    d = np.random.default_rng(7).uniform(0.05, 2.0, n)
    F = fg().Factor(K1, 1.0, 0.0, diag=torch.tensor(d, device=case["dev"]))
    OF = oh.Factor(H, 1.0, 0.0, d)
    assert abs(float(F.logdet().cpu()[0]) - OF.logdet()) <= 1e-9 * abs(OF.logdet())
    b = np.random.default_rng(8).normal(size=n)
    s = F.solve(torch.tensor(b, device=case["dev"])).cpu().numpy()
    assert rel(s, OF.solve(b)) <= 1e-9


def test_matvec(case):
    n, H, K1 = case["n"], case["H"], case["K1"]
    v = np.random.default_rng(2).normal(size=(3, n))
    y = K1.matvec(torch.tensor(v, device=case["dev"]), 2.5, 0.75).cpu().numpy().T
    assert rel(y, H.matvec(v.T, 2.5, 0.75)) <= 1e-12


def test_draw_f_algorithm1(case):
    n, H, K1 = case["n"], case["H"], case["K1"]
    tau, s2 = 40.0, 1.7
    W1 = fg().Factor(K1, 1.0, 0.0)
    WM = fg().Factor(K1, tau * s2, 1.0)
    f, r, mu = fg().draw_f(K1, W1, WM, s2, tau, case["yt"], 21, 3, 5)
    a = rng.normals(n, 21, rng.TAG_A, 3, 5)
    b = rng.normals(n, 21, rng.TAG_B, 3, 5)
    of, orr, omu = sampler.draw_f(H, oh.Factor(H, 1.0, 0.0), oh.Factor(H, tau * s2, 1.0), s2,
                                  tau, case["y"], a, b)
    assert rel(mu.cpu().numpy(), omu) <= 1e-9
    assert rel(r.cpu().numpy(), orr) <= 1e-9
    assert rel(f.cpu().numpy(), of) <= 1e-9


def test_exponential_kernel_exact_at_large_n():
    """Exponential kernel, n = 2^18: HODLR is exact (rank-one blocks) and the O(n)
    state-space recursion gives the exact log-det and solve of a K_1 + s I."""
    n = 1 << 18
    x, _ = sinusoid_1d(n, seed=12)
    b = np.random.default_rng(3).normal(size=n)
    dev = torch.device("cuda:0")
    K1 = fg().Hodlr(torch.tensor(x, device=dev), 0.01, nugget=1e-6, leaf=128, tol=1e-13,
                    kind=fg().KERNEL_EXP)
    assert set(K1.ranks()) <= {1}
    F = fg().Factor(K1, 2.0, 0.5)
    ld, xs = kalman.exp_kernel_logdet_solve(x, 0.01, 2.0, 2.0 * 1e-6 + 0.5, b)
    assert abs(float(F.logdet().cpu()[0]) - ld) <= 1e-11 * abs(ld)
    s = F.solve(torch.tensor(b, device=dev)).cpu().numpy()
    assert rel(s, xs) <= 1e-9
