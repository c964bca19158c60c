"""O2: canonical HODLR matrix, symmetric factor W W' = A, solve and log-det, on the
CPU in FP64 (test infrastructure only).

What the paper fixes and what this file reads into it
-----------------------------------------------------
* HODLR format (Section 3.2, SI 'HODLR decomposition and factorization'): recursive
  2x2 partition of the sorted inputs, dense diagonal leaves, low-rank off-diagonal
  blocks U V', leaves no larger than the maximum block size B (Algorithm 1 input).
  Reading: a node of m rows splits into floor(m/2) and m - floor(m/2) rows; all leaves
  sit at depth L = min{L : ceil(n / 2^L) <= B}.
* Off-diagonal blocks are approximated so that the max-norm error is bounded by the
  tolerance by construction (Section 3.2; Theorem 4.2 needs only that bound).
  Reading (deterministic, so that two implementations build the same matrix):
    - window: rows of the left child farther than R from the first right-child input
      are dropped (and symmetrically); there every kernel entry is below tol/3;
    - interpolant: p-point first-kind Chebyshev interpolation in each variable on the
      window's input range, p the smallest count whose a-priori error bound is within
      tol/6 per variable (when a window holds no more inputs than p, the inputs
      themselves are the nodes and that side is exact);
    - recompression: the truncated SVD of the interpolant, keeping singular values
      above max(tol/3, 8 u s_1); spectral norm bounds max norm, so the total max-norm
      error is below tol.
* Symmetric factorization A = W W' (SI 'HODLR decomposition and factorization'):
  W = A_L ... A_0 with A_L the block-diagonal Cholesky factor of the leaves and each
  further factor an identity-plus-low-rank matrix per tree node.  The paper defers the
  node factor to Ambikasaran (2014); the reading used here is the canonical one:
  after whitening, the node's diagonal block is T = [[I, C], [C', I]] with C = U~ V~';
  W_nu = [[I, 0], [C', (I - C'C)^(1/2)]] with the symmetric square root.  With
  C = P Sigma R' (SVD), (I - C'C)^(1/2) = I + R (Delta - I) R', Delta =
  diag(sqrt(1 - sigma_i^2)).  W_nu W_nu' = T, and W_nu depends on C only, so W is a
  function of A alone.
* Log-determinant (SI 'Determinant computation speedup'): product of block
  determinants and Sylvester's theorem:
      log det A = 2 sum log diag(L_leaf) + sum_nodes sum_i log(1 - sigma_i^2).
"""
from __future__ import annotations

import math
import numpy as np
import scipy.linalg as sla

from . import kernels

U_ROUND = 2.0 ** -53
KAPPA_H = 1.086435          # Cramer's bound: |H_n(x)| e^{-x^2/2} <= KAPPA_H 2^{n/2} sqrt(n!)
PMAX = 64                   # largest interpolation-node count per side


class NotSPD(Exception):
    pass


class TolTooSmall(Exception):
    pass


# ---------------------------------------------------------------------------------
# tree
# ---------------------------------------------------------------------------------
class Tree:
    """Levels 0..L; level l holds 2^l nodes given by their [lo, hi) row ranges."""

    def __init__(self, n: int, leaf: int):
        L = 0
        while -(-n // (1 << L)) > leaf:
            L += 1
        self.n, self.leaf, self.L = n, leaf, L
        self.ranges = [[(0, n)]]
        for _ in range(L):
            nxt = []
            for lo, hi in self.ranges[-1]:
                mid = lo + (hi - lo) // 2
                nxt += [(lo, mid), (mid, hi)]
            self.ranges.append(nxt)

    def node(self, l, j):
        lo, hi = self.ranges[l][j]
        return lo, lo + (hi - lo) // 2, hi

    def leaves(self):
        return self.ranges[self.L]


# ---------------------------------------------------------------------------------
# interpolation error bounds (choice of p)
# ---------------------------------------------------------------------------------
def window_radius(kind, ell, tol):
    """Distance beyond which k_1 < tol/3."""
    if kind == kernels.SE:
        return ell * math.sqrt(2.0 * math.log(3.0 / tol))
    if kind == kernels.EXP:
        return ell * math.log(3.0 / tol)
    # Matern: P(u) exp(-u) = tol/3 with P increasing, solved by u = log(3 P(u) / tol) from
    # below (the iterates increase to the root)
    c = math.sqrt(3.0) if kind == kernels.MATERN32 else math.sqrt(5.0)
    poly = (lambda u: 1.0 + u) if kind == kernels.MATERN32 else (lambda u: 1.0 + u + u * u / 3.0)
    u = math.log(3.0 / tol)
    for _ in range(200):
        u_new = math.log(3.0 * poly(u) / tol)
        if abs(u_new - u) <= 1e-14 * u_new:
            u = u_new
            break
        u = u_new
    return ell * u / c


def interp_bound(kind, p, h, ell):
    """Bound on the max error of p-node first-kind Chebyshev interpolation in one
    variable over an interval of half-width h:  h^p / (2^(p-1) p!) * max|d^p k_1|.
    SE: |d^p exp(-t^2/(2 ell^2))| <= KAPPA_H ell^-p sqrt(p!)  (Hermite functions).
    EXP on separated intervals: |d^p exp(-t/ell)| <= ell^-p.
    Matern on separated intervals (t >= 0), with a = sqrt(3)/ell, resp. sqrt(5)/ell and
    u = a t:  d^p/du^p [(1+u) e^-u] = (-1)^p e^-u (1 + u - p), bounded by max(p - 1, 1);
    d^p/du^p [(1+u+u^2/3) e^-u] = (-1)^p e^-u (1 + u + u^2/3 - p (1 + 2u/3) + p(p-1)/3),
    bounded by p^2/3 + p + 1; so |d^p k_1| <= a^p times those."""
    if h <= 0.0:
        return 0.0
    if kind in (kernels.MATERN32, kernels.MATERN52):
        a = (math.sqrt(3.0) if kind == kernels.MATERN32 else math.sqrt(5.0)) / ell
        m = max(p - 1.0, 1.0) if kind == kernels.MATERN32 else p * p / 3.0 + p + 1.0
        return math.exp(math.log(2.0 * m) + p * math.log(h * a / 2.0) - math.lgamma(p + 1.0))
    r = math.log(h / (2.0 * ell))
    if kind == kernels.SE:
        return math.exp(math.log(2.0 * KAPPA_H) + p * r - 0.5 * math.lgamma(p + 1.0))
    return math.exp(math.log(2.0) + p * r - math.lgamma(p + 1.0))


def lebesgue_bound(p):
    """Lebesgue constant bound of p first-kind Chebyshev nodes."""
    return 2.0 / math.pi * math.log(p + 1.0) + 1.0


def choose_p(kind, h, ell, target, factor=1.0):
    for p in range(1, PMAX + 1):
        if factor * interp_bound(kind, p, h, ell) <= target:
            return p
    raise TolTooSmall(f"interpolation needs more than {PMAX} nodes (h={h}, ell={ell})")


def cheb_nodes(p, a, b):
    s = np.arange(p)
    t = np.cos((2 * s + 1) * math.pi / (2 * p))
    return 0.5 * (a + b) + 0.5 * (b - a) * t, (-1.0) ** s * np.sin((2 * s + 1) * math.pi / (2 * p))


def lagrange_matrix(xs, nodes, wts):
    """Barycentric Lagrange basis values L[i, s] = l_s(xs[i])."""
    d = xs[:, None] - nodes[None, :]
    hit = d == 0.0
    d = np.where(hit, 1.0, d)
    t = wts[None, :] / d
    Lm = t / t.sum(axis=1, keepdims=True)
    rows = hit.any(axis=1)
    Lm[rows] = hit[rows].astype(np.float64)
    return Lm


# ---------------------------------------------------------------------------------
# HODLR build
# ---------------------------------------------------------------------------------
class NodeBlock:
    __slots__ = ("lo", "mid", "hi", "U", "V", "k", "sv", "thr", "pI", "pJ", "exactI",
                 "exactJ", "i0", "j1")


class HODLR:
    """K~_1 of unit amplitude with the nugget on the diagonal."""

    def __init__(self, x, kind, ell, nugget, leaf, tol):
        x = np.asarray(x, dtype=np.float64)
        if np.any(np.diff(x) < 0):
            raise ValueError("x must be sorted ascending")
        self.x, self.kind, self.ell, self.nugget, self.tol = x, kind, ell, nugget, tol
        self.tree = Tree(x.size, leaf)
        self.R = window_radius(kind, ell, tol)
        self.blocks = {}
        for l in range(self.tree.L):
            for j in range(1 << l):
                self.blocks[(l, j)] = self._compress(*self.tree.node(l, j))

    def _compress(self, lo, mid, hi):
        x, kind, ell, tol = self.x, self.kind, self.ell, self.tol
        b = NodeBlock()
        b.lo, b.mid, b.hi = lo, mid, hi
        i0 = lo + int(np.searchsorted(x[lo:mid], x[mid] - self.R, side="left"))
        j1 = mid + int(np.searchsorted(x[mid:hi], x[mid - 1] + self.R, side="right"))
        b.i0, b.j1 = i0, j1
        mI, mJ = mid - i0, j1 - mid
        b.U = np.zeros((mid - lo, 0))
        b.V = np.zeros((hi - mid, 0))
        b.k, b.sv, b.thr = 0, np.zeros(0), 0.0
        b.pI = b.pJ = 0
        b.exactI = b.exactJ = False
        if mI == 0 or mJ == 0:
            return b
        xI, xJ = x[i0:mid], x[mid:j1]
        hI = 0.5 * (xI[-1] - xI[0])
        hJ = 0.5 * (xJ[-1] - xJ[0])
        pI = choose_p(kind, hI, ell, tol / 6.0)
        exactI = mI <= pI
        lam = 1.0 if exactI else lebesgue_bound(pI)
        pJ = choose_p(kind, hJ, ell, tol / 6.0, factor=lam)
        exactJ = mJ <= pJ
        if exactI:
            LI, nI = np.eye(mI), xI
        else:
            nI, wI = cheb_nodes(pI, xI[0], xI[-1])
            LI = lagrange_matrix(xI, nI, wI)
        if exactJ:
            LJ, nJ = np.eye(mJ), xJ
        else:
            nJ, wJ = cheb_nodes(pJ, xJ[0], xJ[-1])
            LJ = lagrange_matrix(xJ, nJ, wJ)
        C = kernels.k1(kind, ell, nI, nJ)
        QI, RI = np.linalg.qr(LI)
        QJ, RJ = np.linalg.qr(LJ)
        Uh, s, Vh = np.linalg.svd(RI @ C @ RJ.T)
        thr = max(tol / 3.0, 8.0 * U_ROUND * s[0]) if s.size else tol / 3.0
        k = int(np.sum(s > thr))
        sq = np.sqrt(s[:k])
        b.U = np.zeros((mid - lo, k))
        b.V = np.zeros((hi - mid, k))
        b.U[i0 - lo:, :] = (QI @ Uh[:, :k]) * sq
        b.V[:mJ, :] = (QJ @ Vh[:k, :].T) * sq
        b.k, b.sv, b.thr = k, s, thr
        b.pI, b.pJ = LI.shape[1], LJ.shape[1]
        b.exactI, b.exactJ = exactI, exactJ
        return b

    # -- queries ----------------------------------------------------------------------
    @property
    def n(self):
        return self.x.size

    def ranks(self):
        return [[self.blocks[(l, j)].k for j in range(1 << l)] for l in range(self.tree.L)]

    def tie_margin(self):
        """Smallest relative distance |s_i / thr - 1| over all nodes (rank decisions
        closer than rounding to their threshold can differ between implementations)."""
        m = math.inf
        for b in self.blocks.values():
            if b.sv.size:
                m = min(m, float(np.min(np.abs(b.sv / b.thr - 1.0))))
        return m

    def leaf_block(self, lo, hi):
        K = kernels.k1(self.kind, self.ell, self.x[lo:hi], self.x[lo:hi])
        K[np.diag_indices_from(K)] += self.nugget
        return K

    def dense(self):
        """K~_1 as a dense matrix (small n only)."""
        n = self.n
        A = np.zeros((n, n))
        for lo, hi in self.tree.leaves():
            A[lo:hi, lo:hi] = self.leaf_block(lo, hi)
        for b in self.blocks.values():
            blk = b.U @ b.V.T
            A[b.lo:b.mid, b.mid:b.hi] = blk
            A[b.mid:b.hi, b.lo:b.mid] = blk.T
        return A

    def entries(self, ii, jj):
        """K~_1[ii[t], jj[t]] without forming the matrix."""
        out = np.empty(len(ii))
        for t, (i, j) in enumerate(zip(ii, jj)):
            i, j = int(i), int(j)
            if i > j:
                i, j = j, i
            val = None
            for l in range(self.tree.L):
                for jn in range(1 << l):
                    lo, mid, hi = self.tree.node(l, jn)
                    if lo <= i < mid <= j < hi:
                        b = self.blocks[(l, jn)]
                        val = float(b.U[i - lo] @ b.V[j - mid])
                        break
                if val is not None:
                    break
            if val is None:      # same leaf
                val = float(kernels.k1(self.kind, self.ell, self.x[[i]], self.x[[j]])[0, 0])
                if i == j:
                    val += self.nugget
            out[t] = val
        return out

    def matvec(self, v, alpha=1.0, beta=0.0):
        """(alpha K~_1 + beta I) v for a vector or an n x m array."""
        v = np.asarray(v, dtype=np.float64)
        y = beta * v
        for lo, hi in self.tree.leaves():
            y[lo:hi] += alpha * (self.leaf_block(lo, hi) @ v[lo:hi])
        for b in self.blocks.values():
            if b.k == 0:
                continue
            y[b.lo:b.mid] += alpha * (b.U @ (b.V.T @ v[b.mid:b.hi]))
            y[b.mid:b.hi] += alpha * (b.V @ (b.U.T @ v[b.lo:b.mid]))
        return y


# ---------------------------------------------------------------------------------
# symmetric factorization of alpha K~_1 + beta I + diag(d)
# ---------------------------------------------------------------------------------
class NodeFactor:
    __slots__ = ("P", "R", "sig", "delta")


class Factor:
    """W with W W' = alpha K~_1 + beta I + diag(d), W = L_D W_(L-1) ... W_(0)."""

    def __init__(self, H: HODLR, alpha: float, beta: float, d=None):
        self.H, self.alpha, self.beta = H, alpha, beta
        tree = H.tree
        self.leafL = []
        for lo, hi in tree.leaves():
            A = alpha * H.leaf_block(lo, hi) + beta * np.eye(hi - lo)
            if d is not None:
                A[np.diag_indices_from(A)] += d[lo:hi]
            try:
                self.leafL.append(self._leaf_chol(A))
            except np.linalg.LinAlgError as e:
                raise NotSPD(f"leaf [{lo},{hi}) not positive definite") from e
        # whitened panels: U~ = L_D^-1 sqrt(alpha) U, V~ likewise
        sa = math.sqrt(alpha)
        self.Ut, self.Vt = {}, {}
        for key, b in H.blocks.items():
            self.Ut[key] = self._leaf_solve(b.lo, sa * b.U)
            self.Vt[key] = self._leaf_solve(b.mid, sa * b.V)
        self.nodes = {}
        for l in range(tree.L - 1, -1, -1):
            for j in range(1 << l):
                nf = self._node_factor(self.Ut[(l, j)], self.Vt[(l, j)])
                self.nodes[(l, j)] = nf
                lo, mid, hi = tree.node(l, j)
                # W_nu^-1 on every coarser panel restricted to this node's rows
                for la in range(l):
                    ja = j >> (l - la)
                    alo, amid, ahi = tree.node(la, ja)
                    if hi <= amid:
                        Y = self.Ut[(la, ja)][lo - alo:hi - alo]
                    else:
                        Y = self.Vt[(la, ja)][lo - amid:hi - amid]
                    self._inv_node(nf, mid - lo, Y)

    @staticmethod
    def _leaf_chol(A):
        return sla.cholesky(A, lower=True)

    # leaf block-diagonal helpers (rows starting at `start`)
    def _leaf_iter(self, start, m):
        for (lo, hi), Lb in zip(self.H.tree.leaves(), self.leafL):
            if lo >= start and hi <= start + m:
                yield lo - start, hi - start, Lb

    def _leaf_solve(self, start, Y, trans=False):
        Y = np.array(Y, dtype=np.float64, copy=True)
        for a, c, Lb in self._leaf_iter(start, Y.shape[0]):
            Y[a:c] = sla.solve_triangular(Lb, Y[a:c], lower=True, trans=1 if trans else 0)
        return Y

    def _leaf_mul(self, start, Y, trans=False):
        Y = np.array(Y, dtype=np.float64, copy=True)
        for a, c, Lb in self._leaf_iter(start, Y.shape[0]):
            Y[a:c] = (Lb.T if trans else Lb) @ Y[a:c]
        return Y

    @staticmethod
    def _node_factor(Ut, Vt):
        nf = NodeFactor()
        k = Ut.shape[1]
        if k == 0:
            nf.P, nf.R = np.zeros((Ut.shape[0], 0)), np.zeros((Vt.shape[0], 0))
            nf.sig = nf.delta = np.zeros(0)
            return nf
        QU, RU = np.linalg.qr(Ut)
        QV, RV = np.linalg.qr(Vt)
        Ph, sig, Rht = np.linalg.svd(RU @ RV.T)
        if sig.size and sig[0] >= 1.0:
            raise NotSPD(f"node singular value {sig[0]} >= 1")
        nf.P, nf.R, nf.sig = QU @ Ph, QV @ Rht.T, sig
        nf.delta = np.sqrt((1.0 - sig) * (1.0 + sig))
        return nf

    # node operators on Y (rows of the node, any number of columns), in place
    @staticmethod
    def _inv_node(nf, mI, Y):
        if nf.sig.size == 0:
            return
        YI, YJ = Y[:mI], Y[mI:]
        RtYJ = nf.R.T @ YJ
        t = RtYJ - nf.sig[:, None] * (nf.P.T @ YI)
        YJ += nf.R @ (t / nf.delta[:, None] - RtYJ)

    @staticmethod
    def _fwd_node(nf, mI, Y):
        if nf.sig.size == 0:
            return
        YI, YJ = Y[:mI], Y[mI:]
        RtYJ = nf.R.T @ YJ
        YJ += nf.R @ (nf.sig[:, None] * (nf.P.T @ YI) + (nf.delta - 1.0)[:, None] * RtYJ)

    @staticmethod
    def _fwdT_node(nf, mI, Y):
        if nf.sig.size == 0:
            return
        YI, YJ = Y[:mI], Y[mI:]
        RtYJ = nf.R.T @ YJ
        YI += nf.P @ (nf.sig[:, None] * RtYJ)
        YJ += nf.R @ ((nf.delta - 1.0)[:, None] * RtYJ)

    @staticmethod
    def _invT_node(nf, mI, Y):
        if nf.sig.size == 0:
            return
        YI, YJ = Y[:mI], Y[mI:]
        RtYJ = nf.R.T @ YJ
        YJ += nf.R @ ((1.0 / nf.delta - 1.0)[:, None] * RtYJ)
        YI -= nf.P @ (nf.sig[:, None] * (nf.R.T @ YJ))

    def _level(self, l, Y, op):
        for j in range(1 << l):
            lo, mid, hi = self.H.tree.node(l, j)
            op(self.nodes[(l, j)], mid - lo, Y[lo:hi])

    # public operators --------------------------------------------------------------
    @staticmethod
    def _as2d(v):
        v = np.asarray(v, dtype=np.float64)
        return (v.reshape(-1, 1) if v.ndim == 1 else np.array(v, copy=True)), v.ndim == 1

    def apply_W(self, v):
        """W v = L_D W_(L-1) ... W_(0) v."""
        Y, vec = self._as2d(v)
        Y = np.array(Y, copy=True)
        for l in range(self.H.tree.L):
            self._level(l, Y, self._fwd_node)
        Y = self._leaf_mul(0, Y)
        return Y[:, 0] if vec else Y

    def apply_Winv(self, v):
        """W^-1 v = W_(0)^-1 ... W_(L-1)^-1 L_D^-1 v."""
        Y, vec = self._as2d(v)
        Y = self._leaf_solve(0, Y)
        for l in range(self.H.tree.L - 1, -1, -1):
            self._level(l, Y, self._inv_node)
        return Y[:, 0] if vec else Y

    def apply_WT(self, v):
        """W' v = W_(0)' ... W_(L-1)' L_D' v."""
        Y, vec = self._as2d(v)
        Y = self._leaf_mul(0, Y, trans=True)
        for l in range(self.H.tree.L - 1, -1, -1):
            self._level(l, Y, self._fwdT_node)
        return Y[:, 0] if vec else Y

    def apply_WinvT(self, v):
        """W^-T v = L_D^-T W_(L-1)^-T ... W_(0)^-T v."""
        Y, vec = self._as2d(v)
        Y = np.array(Y, copy=True)
        for l in range(self.H.tree.L):
            self._level(l, Y, self._invT_node)
        Y = self._leaf_solve(0, Y, trans=True)
        return Y[:, 0] if vec else Y

    def solve(self, b):
        """A^-1 b = W^-T W^-1 b."""
        return self.apply_WinvT(self.apply_Winv(b))

    def logdet(self):
        ld = 0.0
        for Lb in self.leafL:
            ld += 2.0 * float(np.sum(np.log(np.diag(Lb))))
        for nf in self.nodes.values():
            ld += float(np.sum(np.log((1.0 - nf.sig) * (1.0 + nf.sig))))
        return ld

    def dense_W(self):
        return self.apply_W(np.eye(self.H.n))
