"""Serving loop: jobs of mixed n submitted while others run are admitted by memory
footprint, advanced together one sweep at a time, and each job's result equals the
same chain run alone, bit for bit (chains share no buffers, reductions are
deterministic)."""
import time

import numpy as np
import pytest

from workloads import sinusoid_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


JOBS = [  # n, ell0, iters, seed
    (600, 0.05, 4, 21), (1500, 0.02, 3, 22), (3000, 0.1, 5, 23), (900, 0.03, 6, 24),
    (2200, 0.2, 3, 25), (1200, 0.07, 4, 26), (2600, 0.01, 5, 27),
]


def alone(n, ell0, iters, seed):
    x, y = sinusoid_1d(n, seed=seed)
    dev = torch.device("cuda:0")
    c = fg().Chain(torch.tensor(x, device=dev), torch.tensor(y, device=dev), ell0=ell0,
                   tau0=400.0, leaf=64, tol=1e-10, seed=seed, stream_id=seed)
    c.step(iters)
    return c.state(with_vectors=True)


def test_served_jobs_equal_alone_and_respect_the_budget():
    est = {}
    for n, ell0, iters, seed in JOBS:
        x, _ = sinusoid_1d(n, seed=seed)
        est[seed] = fg().footprint_bytes(x, ell0, leaf=64)
    # room for about three of the jobs at a time
    budget = int(sorted(est.values())[-1] + sorted(est.values())[-2] + min(est.values()))
    srv = fg().Server(budget, max_active=8, nstreams=4, graphs=True)
    ids = {}
    for k, (n, ell0, iters, seed) in enumerate(JOBS):
        x, y = sinusoid_1d(n, seed=seed)
        ids[srv.submit(x, y, ell0, iters, tau0=400.0, leaf=64, seed=seed, stream_id=seed)] = k
        if k == 2:
            time.sleep(0.05)  # later jobs arrive while the first ones run
    srv.drain(300.0)
    res = srv.poll()
    stats = srv.stats()
    srv.close()
    assert len(res) == len(JOBS)
    assert stats["peak_bytes"] <= budget
    by_k = {ids[r["id"]]: r for r in res}
    # admission is first come, first served
    admits = [by_k[k]["t_admit"] for k in range(len(JOBS))]
    assert admits == sorted(admits)
    # the budget held some jobs back while others ran, and several ran at once
    assert any(by_k[k]["t_admit"] > by_k[k]["t_submit"] + 1e-4 for k in range(len(JOBS)))
    overlap = any(by_k[a]["t_admit"] < by_k[b]["t_done"] and by_k[b]["t_admit"] < by_k[a]["t_done"]
                  for a in range(len(JOBS)) for b in range(a + 1, len(JOBS)))
    assert overlap
    for k, (n, ell0, iters, seed) in enumerate(JOBS):
        r = by_k[k]
        assert r["status"] == 0 and r["iteration"] == iters
        assert r["bytes"] == est[seed], (r["bytes"], est[seed])
        s = alone(n, ell0, iters, seed)
        assert np.array_equal(r["f"], s["f"].cpu().numpy()), k
        for key in ["tau", "sigf2", "k", "accepts", "loglik"]:
            assert r[key] == s[key], (k, key)


def test_serve_rejects_unsorted_inputs():
    srv = fg().Server(1 << 30, max_active=2)
    x = np.array([0.3, 0.1, 0.2])
    with pytest.raises(fg().FgError):
        srv.submit(x, x, 0.1, 2)
    srv.close()
