"""Live kernel timer (fg_timer_start/stop) through the C ABI: the algorithmic bytes it
reports for the level reduce depend on the per-level ranks of the matrix being factored.
One rank snapshot serves every timed launch until that matrix is built again or freed, so
repeated factorizations, two matrices in one window, and a matrix freed and replaced by a
new build inside the window must each give the bytes of the same work timed alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fg():
    import paper_2006_06537_amd as m
    return m


N = 1 << 15


def xs(seed):
    return torch.tensor(np.sort(np.random.default_rng(seed).uniform(0.0, 1.0, N)),
                        dtype=torch.float64, device="cuda")


def timed(work):
    """(launches, bytes) of the level reduce over work()"""
    m = fg()
    t = m.KernelTimer(m.KID_REDUCE)
    t.start()
    keep = work()
    torch.cuda.synchronize()
    _, launches, by = t.stop()
    del keep
    return launches, by


def test_timer_bytes_follow_the_factored_matrix():
    m = fg()
    x = xs(3)
    Ka = m.Hodlr(x, 0.02)
    Kb = m.Hodlr(x, 0.2)
    torch.cuda.synchronize()
    L = Ka.levels()
    assert Kb.levels() == L and L > 3
    ra, rb = np.asarray(Ka.ranks()), np.asarray(Kb.ranks())
    assert ra.max() != rb.max()  # different ranks, hence different bytes

    na, ba = timed(lambda: m.Factor(Ka, 1.0, 0.0))
    nb, bb = timed(lambda: m.Factor(Kb, 1.0, 0.0))
    assert na == L and nb == L
    assert ba > 0 and bb > 0 and ba != bb

    # the same matrix twice: the snapshot is reused
    n2, b2 = timed(lambda: (m.Factor(Ka, 1.0, 0.0), m.Factor(Ka, 1.0, 0.0)))
    assert n2 == 2 * L
    assert b2 == pytest.approx(2 * ba, rel=1e-12)

    # two matrices in one window
    n3, b3 = timed(lambda: (m.Factor(Kb, 1.0, 0.0), m.Factor(Ka, 1.0, 0.0)))
    assert n3 == 2 * L
    assert b3 == pytest.approx(ba + bb, rel=1e-12)

    # a matrix freed and a new one built inside the window: the new build's ranks count
    def replace():
        nonlocal Kb
        F = m.Factor(Kb, 1.0, 0.0)
        torch.cuda.synchronize()
        del F
        Kb = None
        Kc = m.Hodlr(x, 0.02)
        return m.Factor(Kc, 1.0, 0.0), Kc

    n4, b4 = timed(replace)
    assert n4 == 2 * L
    assert b4 == pytest.approx(bb + ba, rel=1e-12)
