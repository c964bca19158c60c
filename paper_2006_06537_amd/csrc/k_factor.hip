// Symmetric factorization W W' = alpha K~_1 + beta I + diag(d) (gfx950 kernels).
//
// W = L_D W_(L-1) ... W_(0): L_D is the block-diagonal Cholesky factor of the leaves;
// W_(l) holds, for each level-l node, the canonical factor of its whitened diagonal
// block T = [[I, C], [C', I]], C = U~ V~' (U~, V~ = panels whitened by all finer
// factors):  W_nu = [[I, 0], [C', S^(1/2)]],  S = I - C'C.
// Node arithmetic works on Gram matrices only.  With G_U = U~'U~ = S_U'S_U,
// H = S_U G_V S_U' = P diag(s^2) P', B = S_U' P:
//   S^(+-1/2) = I + V~ B g(s^2) B' V~'  with  g_+(s2) = -1/(1 + sqrt(1-s2)),
//   g_-(s2) = 1/(sqrt(1-s2) (1 + sqrt(1-s2))),  F1 = B g_+ B',  F2 = B g_- B'.
// W_nu^-1 on the rows of a coarser panel Y:  Y_J += V~ (-S + F2 (T - G_V S)),
// S = U~'Y_I, T = V~'Y_J.  log det W W' = 2 sum log diag L_D + sum_nodes sum log(1-s2).
#include <cfloat>

#include "fg_internal.h"
#include "fg_timer.h"

namespace fg {

__device__ __forceinline__ double kern1(int kind, double ell, double a, double b) {
  const double d = a - b;
  if (kind == FG_KERNEL_SE) return exp(-(d * d) / (2.0 * ell * ell));
  return exp(-fabs(d) / ell);
}

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------
// leaves: Cholesky, its inverse, log-det and the whitening of every panel row
//
// One work-group of 256 threads per leaf (m <= 128 rows).  The leaf matrix lives in
// registers in a 16 x 16 thread grid: thread (tr, tc) holds the 8 x 8 elements
// (tr + 16 i, tc + 16 j).  Right-looking Cholesky, forward substitution and the
// inverse (substitution on identity columns) all run as column steps: the owners of
// column j (and of row j of the right-hand sides) publish it through a double-
// buffered LDS vector, one barrier per step, and every thread updates its elements.
// ---------------------------------------------------------------------------------
constexpr int LG = 16;        // thread grid side
constexpr int LE = BMAX / LG; // elements per thread per dimension (8)
constexpr int YQ = 4;         // right-hand-side columns per thread (64 per pass)

template <int N>
__device__ __forceinline__ double pick(const double (&v)[N], int idx) {
  double r = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) r = (t == idx) ? v[t] : r;
  return r;
}

// y (rows tr + 16 i, columns tc + 16 q of a 64-column block) <- L^-1 y, steps j0..m-1.
__device__ __forceinline__ void leaf_trsm(const double (&a)[LE][LE], double (&y)[LE][YQ], int m,
                                          int j0, double (*colL)[BMAX], double (*rowY)[64],
                                          int tr, int tc) {
  for (int j = j0; j < m; ++j) {
    const int buf = j & 1, js = j >> 4;
    if (tc == (j & 15)) {
#pragma unroll
      for (int i = 0; i < LE; ++i) {
        const int r = tr + LG * i;
        if (r >= j && r < m) colL[buf][r] = pick(a[i], js);
      }
    }
    if (tr == (j & 15)) {
#pragma unroll
      for (int q = 0; q < YQ; ++q) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < LE; ++i) v = (i == js) ? y[i][q] : v;
        rowY[buf][tc + LG * q] = v;
      }
    }
    __syncthreads();
    const double dinv = 1.0 / colL[buf][j];
    double yj[YQ];
#pragma unroll
    for (int q = 0; q < YQ; ++q) yj[q] = rowY[buf][tc + LG * q] * dinv;
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      const int r = tr + LG * i;
      const double lr = (r > j && r < m) ? colL[buf][r] : 0.0;
#pragma unroll
      for (int q = 0; q < YQ; ++q) y[i][q] -= lr * yj[q];
      if (r == j) {
#pragma unroll
        for (int q = 0; q < YQ; ++q) y[i][q] = yj[q];
      }
    }
  }
}

__global__ void __launch_bounds__(NTHREADS, 2) k_leaf(
    const int* __restrict__ leaf_lo, int nleaf, const double* __restrict__ x, int kind, double ell,
    double nugget, double alpha_v, const double* __restrict__ alpha_p, double beta_v,
    const double* __restrict__ beta_p, const double* __restrict__ diag, int Bc,
    double* __restrict__ leafL, double* __restrict__ leafLinv, double* __restrict__ leaf_ld,
    int* __restrict__ status, const double* __restrict__ src, double* __restrict__ dst, int ld,
    const int* __restrict__ coff, const int* __restrict__ kmax, int L) {
  const int b = blockIdx.x;
  if (b >= nleaf) return;
  const int lo = leaf_lo[b], m = leaf_lo[b + 1] - lo;
  const double alpha = alpha_p ? *alpha_p : alpha_v;
  const double beta = beta_p ? *beta_p : beta_v;
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  __shared__ double xs[BMAX];
  __shared__ double colL[2][BMAX];
  __shared__ double rowY[2][64];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int r = threadIdx.x; r < m; r += NTHREADS) xs[r] = x[lo + r];
  __syncthreads();
  double a[LE][LE];
#pragma unroll
  for (int i = 0; i < LE; ++i) {
    const int r = tr + LG * i;
#pragma unroll
    for (int jj = 0; jj < LE; ++jj) {
      const int c = tc + LG * jj;
      double v = (r == c) ? 1.0 : 0.0;
      if (r < m && c < m) {
        v = alpha * kern1(kind, ell, xs[r], xs[c]);
        if (r == c) v += alpha * nugget + beta + (diag ? diag[lo + r] : 0.0);
      }
      a[i][jj] = v;
    }
  }
  // Cholesky: column j of L = (column j of the updated matrix) / sqrt(pivot)
  double ldsum = 0.0;
  bool mybad = false;
  for (int j = 0; j < m; ++j) {
    const int buf = j & 1, js = j >> 4;
    if (tc == (j & 15)) {
#pragma unroll
      for (int i = 0; i < LE; ++i) {
        const int r = tr + LG * i;
        if (r >= j && r < m) colL[buf][r] = pick(a[i], js);
      }
    }
    __syncthreads();
    const double d = colL[buf][j];
    const bool ok = d > 0.0;
    mybad |= !ok;
    const double inv = ok ? 1.0 / sqrt(d) : 1.0;
    if (threadIdx.x == 0) ldsum += ok ? log(d) : 0.0;
    double lr[LE], lc[LE];
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      const int r = tr + LG * i;
      lr[i] = (r > j && r < m) ? colL[buf][r] * inv : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < LE; ++jj) {
      const int c = tc + LG * jj;
      lc[jj] = (c > j && c < m) ? colL[buf][c] * inv : 0.0;
    }
#pragma unroll
    for (int i = 0; i < LE; ++i)
#pragma unroll
      for (int jj = 0; jj < LE; ++jj) a[i][jj] -= lr[i] * lc[jj];
    if (tc == (j & 15)) {
#pragma unroll
      for (int i = 0; i < LE; ++i) {
        const int r = tr + LG * i;
        const double v = (r >= j && r < m) ? colL[buf][r] * inv : 0.0;
#pragma unroll
        for (int jj = 0; jj < LE; ++jj)
          if (jj == js) a[i][jj] = v;
      }
    }
  }
  if (mybad) atomicOr(&bad, 1);
  if (threadIdx.x == 0) leaf_ld[b] = ldsum;  // sum log(pivot) = 2 sum log diag(L)
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(status, ST_NOTSPD);
  // L to global (lower triangle, column-major, ld = Bc)
  double* Lg = leafL + (size_t)b * Bc * Bc;
#pragma unroll
  for (int jj = 0; jj < LE; ++jj) {
    const int c = tc + LG * jj;
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      const int r = tr + LG * i;
      if (r < m && c < m) Lg[r + (size_t)c * Bc] = (c <= r) ? a[i][jj] : 0.0;
    }
  }
  // L^-1 by substitution on identity columns, 64 columns per pass
  double* Lig = leafLinv + (size_t)b * Bc * Bc;
  for (int c0 = 0; c0 < m; c0 += 64) {
    double y[LE][YQ];
#pragma unroll
    for (int i = 0; i < LE; ++i)
#pragma unroll
      for (int q = 0; q < YQ; ++q) y[i][q] = (tr + LG * i == c0 + tc + LG * q) ? 1.0 : 0.0;
    leaf_trsm(a, y, m, c0, colL, rowY, tr, tc);
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int c = c0 + tc + LG * q;
#pragma unroll
      for (int i = 0; i < LE; ++i) {
        const int r = tr + LG * i;
        if (r < m && c < m) Lig[r + (size_t)c * Bc] = (c <= r) ? y[i][q] : 0.0;
      }
    }
    __syncthreads();
  }
  // whitening of all panel rows of this leaf: dst = sqrt(alpha) L^-1 src.  The active
  // columns of all levels are numbered 0..total-1 and handled 64 per pass.
  const double sa = sqrt(alpha);
  int total = 0;
  for (int l = 0; l < L; ++l) total += kmax[l];
  for (int p0 = 0; p0 < total; p0 += 64) {
    int gcq[YQ];
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      int f = p0 + tc + LG * q;
      gcq[q] = -1;
      if (f < total) {
        for (int l = 0; l < L; ++l) {
          const int km = kmax[l];
          if (f < km) { gcq[q] = coff[l] + f; break; }
          f -= km;
        }
      }
    }
    double y[LE][YQ];
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
#pragma unroll
      for (int i = 0; i < LE; ++i) {
        const int r = tr + LG * i;
        y[i][q] = (gcq[q] >= 0 && r < m) ? src[(size_t)gcq[q] * ld + lo + r] : 0.0;
      }
    }
    __syncthreads();
    leaf_trsm(a, y, m, 0, colL, rowY, tr, tc);
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      if (gcq[q] < 0) continue;
#pragma unroll
      for (int i = 0; i < LE; ++i) {
        const int r = tr + LG * i;
        if (r < m) dst[(size_t)gcq[q] * ld + lo + r] = sa * y[i][q];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// level reduce (panel x panel): Z[a][b] = sum_i P[i, coff_l + a] R[i, rcols_l[b]]
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(NTHREADS) k_reduce_panel(
    const Task* __restrict__ tasks, int tbase, int ntask, int l, const int* __restrict__ coff,
    const int* __restrict__ kmax, const int* __restrict__ rcols, const int* __restrict__ rcount,
    int Ktot, const double* __restrict__ P, int ld, double* __restrict__ zpart, int zs_a,
    int zs_task) {
  const int t = blockIdx.x;
  if (t >= ntask) return;
  const Task tk = tasks[tbase + t];
  const int c0 = coff[l], kl = kmax[l], W = rcount[l];
  const int* rc = rcols + (size_t)l * Ktot;
  __shared__ double Ls[PMAX][64];
  __shared__ double Rs[64][65];
  const int bb = threadIdx.x & 63, a0 = threadIdx.x >> 6;
  for (int b0 = 0; b0 < W; b0 += 64) {
    const int bw = min(64, W - b0);
    double acc[15];
#pragma unroll
    for (int m = 0; m < 15; ++m) acc[m] = 0.0;
    for (int r = tk.r0; r < tk.r1; r += 64) {
      const int rw = min(64, tk.r1 - r);
      for (int idx = threadIdx.x; idx < kl * 64; idx += NTHREADS) {
        const int row = idx & 63, col = idx >> 6;
        Ls[col][row] = row < rw ? P[(size_t)(c0 + col) * ld + r + row] : 0.0;
      }
      for (int idx = threadIdx.x; idx < bw * 64; idx += NTHREADS) {
        const int row = idx & 63, col = idx >> 6;
        Rs[row][col] = row < rw ? P[(size_t)rc[b0 + col] * ld + r + row] : 0.0;
      }
      __syncthreads();
      if (bb < bw) {
        for (int i = 0; i < rw; ++i) {
          const double rv = Rs[i][bb];
#pragma unroll
          for (int m = 0; m < 15; ++m) {
            const int a = a0 + 4 * m;
            if (a < kl) acc[m] += Ls[a][i] * rv;
          }
        }
      }
      __syncthreads();
    }
    if (bb < bw) {
#pragma unroll
      for (int m = 0; m < 15; ++m) {
        const int a = a0 + 4 * m;
        if (a < kl) zpart[(size_t)t * zs_task + (size_t)a * zs_a + b0 + bb] = acc[m];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// symmetric Jacobi eigen-decomposition of an m x m LDS matrix (A <- diag, E <- vectors)
// ---------------------------------------------------------------------------------
__device__ bool lds_sym_eig(double* A, double* E, int m, int lda) {
  __shared__ int perm[PMAX + 1];
  __shared__ double cs[PMAX / 2 + 1], sn[PMAX / 2 + 1];
  __shared__ double red[NTHREADS / 64][2];
  __shared__ int done;
  for (int idx = threadIdx.x; idx < m * m; idx += NTHREADS)
    E[idx % m + (idx / m) * lda] = (idx % m == idx / m) ? 1.0 : 0.0;
  __syncthreads();
  if (m < 2) return true;
  const int me = m + (m & 1), np = me / 2;
  bool conv = false;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = threadIdx.x; idx < m * m; idx += NTHREADS) {
      const double v = A[idx % m + (idx / m) * lda];
      tot += v * v;
      if (idx % m != idx / m) off += v * v;
    }
    off = wsum(off);
    tot = wsum(tot);
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6][0] = off; red[threadIdx.x >> 6][1] = tot; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double o = 0.0, s = 0.0;
      for (int w = 0; w < NTHREADS / 64; ++w) { o += red[w][0]; s += red[w][1]; }
      // converged once the off-diagonal part is at the rounding level of the matrix
      const double lim = 4.0 * m * DBL_EPSILON;
      done = (o <= lim * lim * s) ? 1 : 0;
    }
    __syncthreads();
    if (done) { conv = true; break; }
    for (int step = 0; step < me - 1; ++step) {
      if (threadIdx.x < me) {
        const int j = threadIdx.x;
        perm[j] = (j == 0) ? 0 : 1 + ((j - 1 + step) % (me - 1));
      }
      __syncthreads();
      if (threadIdx.x < np) {
        int p = perm[threadIdx.x], q = perm[me - 1 - threadIdx.x];
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[p + q * lda];
          if (apq != 0.0) {
            const double th = (A[q + q * lda] - A[p + p * lda]) / (2.0 * apq);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
          }
        }
        cs[threadIdx.x] = c;
        sn[threadIdx.x] = s;
      }
      __syncthreads();
      // rows p, q  (A <- J' A)
      for (int idx = threadIdx.x; idx < np * m; idx += NTHREADS) {
        const int pr = idx / m, col = idx % m;
        int p = perm[pr], q = perm[me - 1 - pr];
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (q >= m) continue;
        const double c = cs[pr], s = sn[pr];
        const double ap = A[p + col * lda], aq = A[q + col * lda];
        A[p + col * lda] = c * ap - s * aq;
        A[q + col * lda] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q  (A <- A J, E <- E J)
      for (int idx = threadIdx.x; idx < np * m; idx += NTHREADS) {
        const int pr = idx / m, row = idx % m;
        int p = perm[pr], q = perm[me - 1 - pr];
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (q >= m) continue;
        const double c = cs[pr], s = sn[pr];
        const double ap = A[row + p * lda], aq = A[row + q * lda];
        A[row + p * lda] = c * ap - s * aq;
        A[row + q * lda] = s * ap + c * aq;
        const double ep = E[row + p * lda], eq = E[row + q * lda];
        E[row + p * lda] = c * ep - s * eq;
        E[row + q * lda] = s * ep + c * eq;
      }
      __syncthreads();
    }
  }
  return conv;
}

// ---------------------------------------------------------------------------------
// node factor of one level (factorization): Gram blocks -> (G_V, F1, F2), log-det
// and the update coefficients of the coarser panels
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(NTHREADS) k_node_factor(
    int l, const int* __restrict__ rank, const int* __restrict__ kmax,
    const int* __restrict__ rcount, const int* __restrict__ node_task_off, int tbase,
    const double* __restrict__ zpart, int zs_a, int zs_task, double* __restrict__ zfin,
    int zf_side, double* __restrict__ nodemat, const int* __restrict__ nodemat_off,
    double* __restrict__ node_ld, double* __restrict__ coef, int cs_node, int cs_a,
    int* __restrict__ status, int kc) {
  const int j = blockIdx.x;
  const int h = (1 << l) - 1 + j;
  const int k = rank[h], kl = kmax[l], W = rcount[l], Wc = W - kl;
  if (k == 0) {
    if (threadIdx.x == 0) node_ld[h] = 0.0;
    return;
  }
  // final Gram blocks Z_side[a][b] (a < k, b < W), summed over tasks in order
  double* ZI = zfin + (size_t)j * 2 * zf_side;
  double* ZJ = ZI + zf_side;
  for (int side = 0; side < 2; ++side) {
    const int t0 = node_task_off[2 * h + side] - tbase, t1 = node_task_off[2 * h + side + 1] - tbase;
    double* Z = side ? ZJ : ZI;
    for (int idx = threadIdx.x; idx < k * W; idx += NTHREADS) {
      const int a = idx / W, b = idx % W;
      double s = 0.0;
      for (int t = t0; t < t1; ++t) s += zpart[(size_t)t * zs_task + (size_t)a * zs_a + b];
      Z[(size_t)a * W + b] = s;
    }
  }
  __syncthreads();
  extern __shared__ double lds[];
  double* GU = lds;
  double* GV = GU + kc * kc;
  double* E = GV + kc * kc;
  double* Hm = E + kc * kc;
  double* X = Hm + kc * kc;
  __shared__ double lam[PMAX], g1[PMAX], g2[PMAX];
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    GU[a + b * kc] = 0.5 * (ZI[(size_t)a * W + b] + ZI[(size_t)b * W + a]);
    GV[a + b * kc] = 0.5 * (ZJ[(size_t)a * W + b] + ZJ[(size_t)b * W + a]);
  }
  __syncthreads();
  bool ok = lds_sym_eig(GU, E, k, kc);
  if (threadIdx.x < k) lam[threadIdx.x] = sqrt(fmax(GU[threadIdx.x + threadIdx.x * kc], 0.0));
  __syncthreads();
  // S_U = diag(sqrt(lambda)) E'  -> X
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    X[a + b * kc] = lam[a] * E[b + a * kc];
  }
  __syncthreads();
  // E <- S_U G_V ; Hm <- E S_U'
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += X[a + c * kc] * GV[c + b * kc];
    E[a + b * kc] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += E[a + c * kc] * X[b + c * kc];
    Hm[a + b * kc] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {  // symmetrise
    const int a = idx % k, b = idx / k;
    if (a < b) {
      const double v = 0.5 * (Hm[a + b * kc] + Hm[b + a * kc]);
      Hm[a + b * kc] = v;
      Hm[b + a * kc] = v;
    }
  }
  __syncthreads();
  ok = lds_sym_eig(Hm, E, k, kc) && ok;
  if (threadIdx.x == 0) {
    double s = 0.0;
    bool spd = true;
    for (int a = 0; a < k; ++a) {
      double s2 = fmax(Hm[a + a * kc], 0.0);
      if (!(s2 < 1.0)) { spd = false; s2 = 1.0 - DBL_EPSILON; }
      const double d = sqrt(1.0 - s2);
      g1[a] = -1.0 / (1.0 + d);
      g2[a] = 1.0 / (d * (1.0 + d));
      s += log1p(-s2);
    }
    node_ld[h] = s;
    if (!spd) atomicOr(status, ST_NOTSPD);
    if (!ok) atomicOr(status, ST_NOTCONV);
  }
  __syncthreads();
  // B = S_U' P  -> GU
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += X[c + a * kc] * E[c + b * kc];
    GU[a + b * kc] = acc;
  }
  __syncthreads();
  // F1 -> Hm, F2 -> E ; store G_V, F1, F2
  double* out = nodemat + nodemat_off[h];
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    double f1 = 0.0, f2 = 0.0;
    for (int c = 0; c < k; ++c) {
      const double pr = GU[a + c * kc] * GU[b + c * kc];
      f1 += pr * g1[c];
      f2 += pr * g2[c];
    }
    out[a + b * k] = GV[a + b * kc];
    out[k * k + a + b * k] = f1;
    out[2 * k * k + a + b * k] = f2;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * k; idx += NTHREADS) {
    const int a = idx % k, b = idx / k;
    E[a + b * kc] = out[2 * k * k + a + b * k];
  }
  __syncthreads();
  // coefficients of the coarser panels: U = T - G_V S (into ZJ), A = -S + F2 U
  for (int idx = threadIdx.x; idx < k * Wc; idx += NTHREADS) {
    const int a = idx / Wc, b = kl + idx % Wc;
    double acc = ZJ[(size_t)a * W + b];
    for (int d = 0; d < k; ++d) acc -= GV[a + d * kc] * ZI[(size_t)d * W + b];
    ZJ[(size_t)a * W + b] = acc;
  }
  __syncthreads();
  double* cf = coef + (size_t)j * cs_node;
  for (int idx = threadIdx.x; idx < k * Wc; idx += NTHREADS) {
    const int a = idx / Wc, bc = idx % Wc, b = kl + bc;
    double acc = -ZI[(size_t)a * W + b];
    for (int c = 0; c < k; ++c) acc += E[a + c * kc] * ZJ[(size_t)c * W + b];
    cf[(size_t)a * cs_a + bc] = acc;
  }
}

// ---------------------------------------------------------------------------------
// level update (factorization): coarser columns of right-child rows += V~ A
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(NTHREADS) k_update_panel(
    const Task* __restrict__ tasks, int tbase, int ntask, int l, const int* __restrict__ rank,
    const int* __restrict__ coff, const int* __restrict__ kmax, const int* __restrict__ rcols,
    const int* __restrict__ rcount, int Ktot, double* __restrict__ P, int ld,
    const double* __restrict__ coef, int cs_node, int cs_a) {
  const int t = blockIdx.x;
  if (t >= ntask) return;
  const Task tk = tasks[tbase + t];
  if (tk.side == 0) return;
  const int k = rank[tk.h];
  const int kl = kmax[l], Wc = rcount[l] - kl;
  if (k == 0 || Wc <= 0) return;
  const int c0 = coff[l];
  const int j = tk.h - ((1 << l) - 1);
  const int* yc = rcols + (size_t)l * Ktot + kl;
  const double* cf = coef + (size_t)j * cs_node;
  __shared__ double As[PMAX][64];
  __shared__ double Vs[PMAX][64];
  const int i = threadIdx.x & 63, bg = threadIdx.x >> 6;
  for (int b0 = 0; b0 < Wc; b0 += 64) {
    const int bw = min(64, Wc - b0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < k * 64; idx += NTHREADS) {
      const int a = idx >> 6, b = idx & 63;
      As[a][b] = b < bw ? cf[(size_t)a * cs_a + b0 + b] : 0.0;
    }
    for (int r = tk.r0; r < tk.r1; r += 64) {
      const int rw = min(64, tk.r1 - r);
      __syncthreads();
      for (int idx = threadIdx.x; idx < k * 64; idx += NTHREADS) {
        const int a = idx >> 6, row = idx & 63;
        Vs[a][row] = row < rw ? P[(size_t)(c0 + a) * ld + r + row] : 0.0;
      }
      __syncthreads();
      if (i < rw) {
        for (int b = bg; b < bw; b += 4) {
          double acc = 0.0;
          for (int a = 0; a < k; ++a) acc += Vs[a][i] * As[a][b];
          double* y = P + (size_t)yc[b0 + b] * ld + r + i;
          *y += acc;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// log-det: sum of leaf and node parts in a fixed order
// ---------------------------------------------------------------------------------
__global__ void k_logdet_sum(const double* __restrict__ leaf_ld, int nleaf,
                             const double* __restrict__ node_ld, int nint, double* __restrict__ out) {
  __shared__ double red[NTHREADS / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nleaf; i += NTHREADS) s += leaf_ld[i];
  for (int i = threadIdx.x; i < nint; i += NTHREADS) s += node_ld[i];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) t += red[w];
    *out = t;
  }
}

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
void launch_factor(FactorData& F, const double* alpha_dev, const double* beta_dev,
                   const double* diag, hipStream_t s) {
  const HodlrData& H = *F.H;
  const HostPlan& P = H.pk->P;
  const DevPlan& D = H.pk->D;
  const int Bc = P.B;
  timer_before(KID_LEAF, s, -1, P, H.kmax, 0);
  k_leaf<<<P.nleaf, NTHREADS, 0, s>>>(
      D.leaf_lo, P.nleaf, H.x, P.kind, P.ell, P.nugget, F.alpha, alpha_dev, F.beta, beta_dev,
      diag, Bc, F.leafL, F.leafLinv, F.leaf_ld, F.status, H.panel, F.panel, H.ld, D.coff, H.kmax,
      P.L);
  timer_after(KID_LEAF, s);
  const int kc = std::max(P.kcapmax, 1);
  const size_t lds_node = sizeof(double) * 5 * (size_t)kc * kc;
  if (lds_node > 65536)
    (void)hipFuncSetAttribute((const void*)k_node_factor,
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_node));
  for (int l = P.L - 1; l >= 0; --l) {
    const int tb = P.ltask_off[l], nt = P.ltask_off[l + 1] - tb;
    const int Wcap = P.coff[l + 1];  // columns of levels <= l (capacity)
    const int zs_a = Wcap, zs_task = P.kcap[l] * Wcap;
    timer_before(KID_REDUCE, s, l, P, H.kmax, nt);
    k_reduce_panel<<<nt, NTHREADS, 0, s>>>(D.ltasks, tb, nt, l, D.coff, H.kmax, H.rcols,
                                           H.rcount, P.Ktot, F.panel, H.ld, F.zpart, zs_a, zs_task);
    timer_after(KID_REDUCE, s);
    const int cs_node = P.kcap[l] * Wcap, cs_a = Wcap;
    k_node_factor<<<1 << l, NTHREADS, lds_node, s>>>(
        l, H.rank, H.kmax, H.rcount, D.node_task_off, tb, F.zpart, zs_a, zs_task, F.zfin,
        P.kcap[l] * Wcap, F.nodemat, D.nodemat_off, F.node_ld, F.coef, cs_node, cs_a, F.status,
        kc);
    if (l > 0) {
      timer_before(KID_UPDATE, s, l, P, H.kmax, nt);
      k_update_panel<<<nt, NTHREADS, 0, s>>>(D.ltasks, tb, nt, l, H.rank, D.coff, H.kmax,
                                             H.rcols, H.rcount, P.Ktot, F.panel, H.ld, F.coef,
                                             cs_node, cs_a);
      timer_after(KID_UPDATE, s);
    }
  }
  launch_logdet_sum(F, s);
}

void launch_logdet_sum(FactorData& F, hipStream_t s) {
  const HostPlan& P = F.H->pk->P;
  k_logdet_sum<<<1, NTHREADS, 0, s>>>(F.leaf_ld, P.nleaf, F.node_ld, P.nint, F.logdet);
}

}  // namespace fg
