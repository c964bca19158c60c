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
