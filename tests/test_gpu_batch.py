"""Batched stepping of many chains (gibbs_step_batch): library streams, one host
synchronisation per batched sweep, captured and replayed HIP graphs, grouped launches
(every chain's kernels at the same point issued as one launch) and the autotuner that
chooses among them.  Every batched result must equal the per-chain result bit for bit
(chains share no buffers, every reduction is deterministic and each block of a grouped
launch runs the same code on the same data), on every graph replay and in every mode,
for chains of different sizes, FP64 and mixed precision in one batch."""
import numpy as np
import pytest

from oracle import kernels, sampler
from workloads import sinusoid_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


SPECS = [  # n, ell0, seed
    (700, 0.05, 11), (1000, 0.02, 12), (1333, 0.1, 13), (512, 0.2, 14), (900, 0.03, 15),
    (1200, 0.07, 16),
]


def make(spec, precision=0):
    n, ell0, seed = spec
    x, y = sinusoid_1d(n, seed=seed)
    dev = torch.device("cuda:0")
    return fg().Chain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0=ell0,
                      tau0=400.0, leaf=64, tol=1e-10, seed=seed, stream_id=seed,
                      precision=precision)


def snap(c):
    s = c.state(with_vectors=True)
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in s.items()}


def same(a, b):
    for k in ["iteration", "tau", "sigf2", "k", "accepts", "loglik", "q", "logdet1", "status"]:
        assert a[k] == b[k], (k, a[k], b[k])
    for k in ["f", "r", "mu"]:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("mode,nstreams", [(1, 4), (0, 2), (2, 1), (3, 4)],
                         ids=["graphs", "eager", "grouped", "auto"])
def test_batch_equals_sequential(mode, nstreams):
    # chains of six sizes, every other one in mixed precision
    eager = [make(s, precision=i % 2) for i, s in enumerate(SPECS)]
    batch = [make(s, precision=i % 2) for i, s in enumerate(SPECS)]
    # later rounds replay captured sweeps, interleaved with acceptances that swap slots
    for rnd, iters in enumerate([3, 2, 4, 6, 5]):
        for c in eager:
            c.step(iters)
        fg().step_batch(batch, iters, nstreams=nstreams, mode=mode)
        torch.cuda.synchronize()
        for a, b in zip(eager, batch):
            same(snap(a), snap(b))
    if mode == 3:  # 20 sweeps: the autotuner has tried every candidate and chosen
        name, ns, ms = fg().batch_tuning(batch)
        assert name in ("eager", "graphs", "grouped") and ns >= 1 and ms > 0.0


def test_batch_matches_oracle():
    specs = SPECS[:2]
    batch = [make(s) for s in specs]
    orc = []
    for n, ell0, seed in specs:
        x, y = sinusoid_1d(n, seed=seed)
        orc.append(sampler.Chain(x, y, kernels.SE, ell0, 1e-6, 64, 1e-10, 400.0, 1.0, seed,
                                 stream=seed))
    for it in range(4):
        fg().step_batch(batch, 1)
        for c, o in zip(batch, orc):
            r = o.step()
            s = c.state()
            assert s["k"] == r["k"] and s["last_accept"] == int(r["accept"])
            for key in ["tau", "sigf2", "loglik"]:
                assert abs(s[key] - r[key]) <= 1e-9 * abs(r[key]), (it, key)


def test_batch_rejects_repeated_chain():
    c = make(SPECS[3])
    with pytest.raises(fg().FgError):
        fg().step_batch([c, c], 1)


def test_grouped_batch_of_equal_chains_matches_oracle():
    """Sixteen chains of one size (the shape of the 64 x 32 768 batch, scaled down), grouped:
    each chain against the oracle's chain at 1e-9, grid moves exact."""
    specs = [(1024, 0.02 + 0.002 * i, 100 + i) for i in range(16)]
    batch = [make(s) for s in specs]
    fg().step_batch(batch, 3, mode=fg().BATCH_GROUPED)
    for (n, ell0, seed), c in zip(specs, batch):
        x, y = sinusoid_1d(n, seed=seed)
        o = sampler.Chain(x, y, kernels.SE, ell0, 1e-6, 64, 1e-10, 400.0, 1.0, seed, stream=seed)
        for _ in range(3):
            r = o.step()
        s = c.state(with_vectors=True)
        assert s["status"] == 0
        assert s["k"] == r["k"] and s["last_accept"] == int(r["accept"])
        for key in ["tau", "sigf2", "loglik"]:
            assert abs(s[key] - r[key]) <= 1e-9 * abs(r[key]), key
        f = s["f"].cpu().numpy()
        assert np.linalg.norm(f - o.f) <= 1e-9 * np.linalg.norm(o.f)


def test_eager_batch_of_served_jobs_equals_alone():
    """48 jobs of the serving workload (n from 1e3 to 2e5) stepped 60 sweeps as one eager
    batch on four streams, where the kernels of different chains run side by side on the
    device and the waves of one work-group drift apart, against each chain stepped alone:
    every chain must end in the same state bit for bit, with no failed factorization.  The
    list includes jobs whose node factors pivot often (the pivoted Cholesky of a node's
    Gram block must give one decision to every wave of its work-group)."""
    from workloads import served_jobs
    jobs = served_jobs(512, seed=5)
    pick = list(range(40)) + [44, 76, 128, 170, 233, 273, 357, 439]
    dev = torch.device("cuda:0")

    def chain(j):
        job = jobs[j]
        return fg().Chain(torch.tensor(job["x"], device=dev), torch.tensor(job["y"], device=dev),
                          job["ell0"], job["tau0"], leaf=128, tol=1e-10, seed=job["seed"],
                          stream_id=j)

    batch = [chain(j) for j in pick]
    fg().step_batch(batch, 60, nstreams=4, mode=fg().BATCH_EAGER)
    torch.cuda.synchronize()
    got = [snap(c) for c in batch]
    del batch
    for j, b in zip(pick, got):
        assert b["status"] == 0, (j, b["status"])
        a = chain(j)
        a.step(60)
        same(snap(a), b)
        del a
