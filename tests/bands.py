"""A second, equally valid FP64 evaluation of the oracle's canonical factor, used to
measure the oracle's own reproducibility band where a bar is derived from it."""
import numpy as np
import scipy.linalg as sla

from oracle import hodlr as oh


class InvLeafFactor(oh.Factor):
    """The oracle factor with an unblocked column-by-column leaf Cholesky and explicit
    leaf inverses: an equally valid FP64 evaluation of the same W, used only to measure
    the oracle's reproducibility band."""

    @staticmethod
    def _leaf_chol(A):
        A = np.array(A, dtype=np.float64, copy=True)
        m = A.shape[0]
        for j in range(m):
            if not A[j, j] > 0.0:
                raise np.linalg.LinAlgError("not positive definite")
            A[j, j] = np.sqrt(A[j, j])
            A[j + 1:, j] /= A[j, j]
            A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j + 1:, j])
        return np.tril(A)

    def _leaf_solve(self, start, Y, trans=False):
        Y = np.array(Y, dtype=np.float64, copy=True)
        for a, c, Lb in self._leaf_iter(start, Y.shape[0]):
            Li = sla.solve_triangular(Lb, np.eye(Lb.shape[0]), lower=True)
            Y[a:c] = (Li.T if trans else Li) @ Y[a:c]
        return Y


def perturbed_panels(H, rel=4.0 * 2.0 ** -53, seed=0):
    """A copy of the oracle's HODLR whose off-diagonal factors U, V carry independent
    relative perturbations of `rel` (a few units of rounding): the compressed matrix as a
    different, equally valid FP64 compression would store it.  Leaves are shared."""
    import copy
    g = np.random.default_rng(seed)
    H2 = copy.copy(H)
    H2.blocks = {}
    for key, b in H.blocks.items():
        b2 = copy.copy(b)
        b2.U = b.U * (1.0 + rel * g.standard_normal(b.U.shape))
        b2.V = b.V * (1.0 + rel * g.standard_normal(b.V.shape))
        H2.blocks[key] = b2
    return H2


def logdet_parts(OF):
    """(leaf part, node part) of an oracle factor's log-determinant: 2 sum log diag L of the
    leaf Choleskys, and sum log(1 - s^2) over the node factors."""
    leaf = sum(2.0 * float(np.sum(np.log(np.diag(Lb)))) for Lb in OF.leafL)
    node = sum(float(np.sum(np.log((1.0 - nf.sig) * (1.0 + nf.sig)))) for nf in OF.nodes.values())
    return leaf, node


def node_part_bar(H, OF, alpha=1.0, beta=0.0):
    """Relative bar of the node part of log det(alpha K~ + beta I), the larger of
      * four times the oracle's own reproducibility band: the largest distance between the
        oracle's node part and the same factor (a) with unblocked leaf Choleskys and
        explicit leaf inverses, (b) on compressed panels perturbed by 4 u, as another FP64
        compression would store them -- never below 1e-9;
      * the first-order error of the Gram route the HIP path takes for the node factors
        (s^2 are eigenvalues of products of Gram matrices summed over the m rows of the
        node): |d s_i^2| <= 2 s_i^2 sqrt(m) u, so |d node part| <= sum_nodes sum_i
        2 s_i^2 sqrt(m) u / (1 - s_i^2).
    The top node factors of a small-nugget K~ sit at 1 - s^2 ~ 1e-7, where a rounding-level
    change of s^2 moves log(1 - s^2) by |d s^2| / (1 - s^2).  Returns (bar, band, gram)."""
    node = logdet_parts(OF)[1]
    alts = [InvLeafFactor(H, alpha, beta)] + [oh.Factor(perturbed_panels(H, seed=s_), alpha, beta)
                                              for s_ in (1, 2)]
    band = max(abs(logdet_parts(v)[1] - node) / abs(node) for v in alts)
    u = 2.0 ** -53
    gram = 0.0
    for (l, j), nf in OF.nodes.items():
        lo, mid, hi = H.tree.node(l, j)
        s2 = nf.sig ** 2
        gram += float(np.sum(2.0 * s2 / (1.0 - s2))) * np.sqrt(hi - lo) * u
    gram /= abs(node)
    return max(1e-9, 4.0 * band, gram), band, gram
