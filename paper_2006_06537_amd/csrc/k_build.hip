// HODLR construction kernels (gfx950): interpolation moments, per-node compression
// (Cholesky-QR of the Chebyshev basis, then a one-sided Jacobi SVD of the p x p core
// preconditioned by a column-pivoted QR), rank bookkeeping and panel generation.
//
// Off-diagonal block of node (I, J) on its windows: the first-kind Chebyshev
// interpolant in both variables, written in the Chebyshev polynomial basis:
//   K(x, y) ~ T_I(x) C_T T_J(y)',  C_T = A_I C A_J',  C[s,t] = k_1(xi_s, eta_t),
//   A[k,s] = (2 - [k=0]) / p cos(k (2s+1) pi / (2p))        (discrete cosine transform).
// G_I = T_I' T_I over the window rows follows from the moments mu_m = sum_i T_m(t_i)
// through T_j T_k = (T_{j+k} + T_{|j-k|}) / 2, so the basis is never stored.
// With G = R'R (Cholesky), X = R_I C_T R_J' has the singular values of the interpolant;
// the block is truncated to the singular values above max(tol/3, 8 u s_1) and stored
// as U = T_I(x) T_U, V = T_J(y) T_V with T_U = R_I^-1 U_X sqrt(S), T_V = R_J^-1 V_X sqrt(S).
#include <cfloat>

#include "fg_group.h"
#include "fg_internal.h"
#include "fg_timer.h"

namespace fg {

// ---------------------------------------------------------------------------------
// moments: partial sums of T_m(t_i), m < 2p-1, over the rows of one task; one wave per
// task, so that the many short tasks of the deep levels take no block barriers.  Each
// lane keeps the three-term recurrence of its MRPT rows in registers across the chunks
// of MB moments, so every T_m(t_i) is formed once; rows past the end of the task start
// at zero and stay zero.  The wave reduces its MB sums by recursive halving: at the step
// with lane offset o, the lanes with bit o set keep the upper half of their values and
// the others the lower half, each adding its partner's copy of the half it keeps.
// ---------------------------------------------------------------------------------
constexpr int MRPT = MCHM / 64;  // rows per lane
constexpr int MB = 16;           // moments per chunk
static_assert(MRPT * 64 == MCHM, "a moment task must fit the lanes of one wave");

// arguments of k_moments (one struct, so that grouped launches can stage one per member)
struct k_moments_args {
  const Task* tasks;
  int ntask;
  const NodePlan* nodes;
  const double* x;
  double* mpart;
  int stride;
};
__device__ __forceinline__ void k_moments_body(const k_moments_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const Task* __restrict__ tasks = a_.tasks;
  int ntask = a_.ntask;
  const NodePlan* __restrict__ nodes = a_.nodes;
  const double* __restrict__ x = a_.x;
  double* __restrict__ mpart = a_.mpart;
  int stride = a_.stride;
  (void)by_;
  (void)gy_;

  const int lane = threadIdx.x & 63;
  const int t = bx_ * (NTHREADS / 64) + (threadIdx.x >> 6);
  if (t >= ntask) return;  // whole waves: no barrier below
  const Task tk = tasks[t];
  const NodePlan q = nodes[tk.h];
  const int p = tk.side ? q.pJ : q.pI;
  const double a = tk.side ? q.aJ : q.aI, b = tk.side ? q.bJ : q.bI;
  const double c = 0.5 * (a + b), hw = 0.5 * (b - a);
  const int nm = 2 * p - 1;
  double t2[MRPT], tc[MRPT], tn[MRPT];  // 2 t, T_m(t), T_{m+1}(t)
#pragma unroll
  for (int k = 0; k < MRPT; ++k) {
    const int r = tk.r0 + lane + k * 64;
    const bool in = r < tk.r1;
    const double tt = (in && hw > 0.0) ? (x[r] - c) / hw : 0.0;
    t2[k] = 2.0 * tt;
    tc[k] = in ? 1.0 : 0.0;
    tn[k] = tt;
  }
  // rows per lane that the task reaches (wave-uniform): short tasks skip the rest
  const int kn = (tk.r1 - tk.r0 + 63) / 64;
  // the element of the chunk that this lane holds after the four halving steps
  const int e = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                ((lane >> 2) & 1);
  double* out = mpart + (size_t)t * stride;
  for (int mb = 0; mb < nm; mb += MB) {
    double v[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) v[j] = 0.0;
#pragma unroll
    for (int g = 0; g < MRPT; g += 4) {
      if (g < kn) {
#pragma unroll
        for (int j = 0; j < MB; ++j) {
#pragma unroll
          for (int k = g; k < g + 4; ++k) {
            v[j] += tc[k];
            const double nx = t2[k] * tn[k] - tc[k];
            tc[k] = tn[k];
            tn[k] = nx;
          }
        }
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int o = 32 >> st;
      const int half = MB >> (st + 1);
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const double send = up ? v[i] : v[i + half];
        const double keep = up ? v[i + half] : v[i];
        v[i] = keep + __shfl_xor(send, o, 64);
      }
    }
    double sum = v[0];
    sum += __shfl_xor(sum, 2, 64);
    sum += __shfl_xor(sum, 1, 64);
    if ((lane & 3) == 0 && mb + e < nm) out[mb + e] = sum;
  }
}
__global__ void __launch_bounds__(NTHREADS) k_moments(const k_moments_args a_) {
  k_moments_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_moments_g(const k_moments_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_moments_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_moments_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_moments_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_moments_args* a, const int* st, const int* gy, int mm) {
    k_moments_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_moments now, or records it while a recorder is open on this thread
static void k_moments_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_moments_args& a) {
  if (recording())
    record_group(k_moments_grp, group_key((const void*)k_moments_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_moments<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// small dense helpers on LDS matrices (column-major, leading dimension ldm)
// ---------------------------------------------------------------------------------
// Cholesky with diagonal pivoting of an m x m positive semidefinite Gram matrix G (full
// symmetric storage): P G P' = L L', taking the largest remaining diagonal at each step and
// stopping once it falls to the rounding level 64 m u max diag(G) (the stopping rule for
// semidefinite matrices, Higham 1990).  Repeated inputs make G singular: a window with
// more data points than interpolation nodes but fewer distinct values has rank < m.  On
// return A holds F = P' L (row i: basis function i; column a: step a; columns >= rank are
// zero), so that G = F F', and perm[a] is the basis function pivoted at step a.  tmp is an
// m x m LDS scratch.  Returns the rank, or -1 on a NaN diagonal.
__device__ int lds_pchol(double* A, int m, int ldm, int* perm, double* tmp) {
  __shared__ int rk, piv, bad;
  __shared__ double dfloor;
  // wave 0 reduces over the diagonal (m <= PMAX < 64: one entry per lane)
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const double d = lane < m ? A[lane + lane * ldm] : 0.0;
    double dmax = d;
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    const bool nan = __ballot(lane < m && d != d) != 0;
    if (lane < m) perm[lane] = lane;
    if (lane == 0) {
      bad = nan ? 1 : 0;
      dfloor = 64.0 * m * (DBL_EPSILON * 0.5) * dmax;
      rk = m;
    }
  }
  __syncthreads();
  if (bad) return -1;
  for (int j = 0; j < m; ++j) {
    if (threadIdx.x < 64) {
      // largest remaining diagonal entry, first index on ties
      const int lane = threadIdx.x;
      double v = (lane >= j && lane < m) ? A[lane + lane * ldm] : -DBL_MAX;
      int iv = lane;
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o, 64);
        const int i2 = __shfl_xor(iv, o, 64);
        if (v2 > v || (v2 == v && i2 < iv)) {
          v = v2;
          iv = i2;
        }
      }
      if (lane == 0) {
        if (v > dfloor) {
          piv = iv;
          const int t = perm[j]; perm[j] = perm[iv]; perm[iv] = t;
        } else {
          piv = -1;
          rk = j;
        }
      }
    }
    __syncthreads();
    const int k = piv;
    if (k < 0) break;
    if (k != j) {  // symmetric interchange of rows and columns j and k
      for (int i = threadIdx.x; i < m; i += NTHREADS) {
        const double t = A[j + i * ldm]; A[j + i * ldm] = A[k + i * ldm]; A[k + i * ldm] = t;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += NTHREADS) {
        const double t = A[i + j * ldm]; A[i + j * ldm] = A[i + k * ldm]; A[i + k * ldm] = t;
      }
      __syncthreads();
    }
    const double ljj = sqrt(A[j + j * ldm]);
    __syncthreads();
    if (threadIdx.x == 0) A[j + j * ldm] = ljj;
    for (int r = j + 1 + threadIdx.x; r < m; r += NTHREADS) A[r + j * ldm] /= ljj;
    __syncthreads();
    const int w = m - j - 1;
    for (int idx = threadIdx.x; idx < w * w; idx += NTHREADS) {
      const int r = j + 1 + idx % w, cc = j + 1 + idx / w;
      A[r + cc * ldm] -= A[r + j * ldm] * A[cc + j * ldm];
    }
    __syncthreads();
  }
  const int r = rk;
  // F[perm[a], b] = L[a, b] for b <= a, b < rank
  for (int idx = threadIdx.x; idx < m * m; idx += NTHREADS) {
    const int a = idx % m, b = idx / m;
    tmp[perm[a] + b * m] = (b <= a && b < r) ? A[a + b * ldm] : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < m * m; idx += NTHREADS)
    A[idx % m + (idx / m) * ldm] = tmp[idx];
  __syncthreads();
  return r;
}

// One-sided Jacobi on the columns of M (mr x qc, mr >= qc) with right vectors Q (qc x qc).
// A pair is rotated unless its columns are orthogonal to working precision, or both of
// them are below nu = min(1e-13 max|col|, thr_lo / 8), thr_lo = max(tol/3, 8 (u/2) max|col|)
// (max over the columns at the start of the sweep).  Such columns stay under the
// truncation threshold max(tol/3, 8 (u/2) s_max) >= thr_lo, so every column that is kept
// is still orthogonalised against all others, and a discarded singular value is off by at
// most nu.  Returns false if 40 sweeps did not converge.
__device__ bool lds_jacobi_svd(double* M, int mr, int qc, int ldm, double* Q, int ldq,
                               double tol) {
  __shared__ double nu2s;
  // per sweep parity; the next sweep's flag (the one read at the end of the previous
  // sweep) is reset after this sweep's first barrier, when every thread has read it
  __shared__ int rotated[2];
  for (int idx = threadIdx.x; idx < qc * qc; idx += NTHREADS)
    Q[idx % qc + (idx / qc) * ldq] = (idx % qc == idx / qc) ? 1.0 : 0.0;
  const int qe = qc + (qc & 1);  // even number of players
  const int npair = qe / 2;
  const int g = threadIdx.x >> 3, gl = threadIdx.x & 7;  // 8 lanes per pair
  if (threadIdx.x == 0) rotated[0] = 0;
  __syncthreads();
  if (qc < 2) return true;
  bool conv = false;
  for (int sweep = 0; sweep < 40 && !conv; ++sweep) {
    if (threadIdx.x < 64) {  // the largest column norm (qc <= PMAX < 64 columns)
      double n2 = 0.0;
      if (threadIdx.x < qc)
        for (int r = 0; r < mr; ++r) n2 += M[r + threadIdx.x * ldm] * M[r + threadIdx.x * ldm];
      for (int o = 32; o > 0; o >>= 1) n2 = fmax(n2, __shfl_xor(n2, o, 64));
      if (threadIdx.x == 0) {
        const double mx = sqrt(n2);
        const double thr_lo = fmax(tol / 3.0, 8.0 * (DBL_EPSILON * 0.5) * mx);
        const double nu = fmin(1e-13 * mx, thr_lo / 8.0);
        nu2s = nu * nu;
      }
    }
    __syncthreads();
    const double nu2 = nu2s;
    for (int step = 0; step < qe - 1; ++step) {
      if (g < npair) {
        // pair g of this step of the round-robin order
        int i = rr_index(g, step, qe), k = rr_index(qe - 1 - g, step, qe);
        if (i > k) { const int tmp = i; i = k; k = tmp; }
        // this lane's rows (gl, gl + 8, ...) of columns i and k of M and Q, loaded at once
        constexpr int RPL = (PMAX + 7) / 8;
        double mu[RPL], mv[RPL], qu[RPL], qv[RPL];
        const bool live = k < qc;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = gl + 8 * t;
          mu[t] = (live && r < mr) ? M[r + i * ldm] : 0.0;
          mv[t] = (live && r < mr) ? M[r + k * ldm] : 0.0;
          qu[t] = (live && r < qc) ? Q[r + i * ldq] : 0.0;
          qv[t] = (live && r < qc) ? Q[r + k * ldq] : 0.0;
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          if (gl + 8 * t < mr) {
            al += mu[t] * mu[t]; be += mv[t] * mv[t]; ga += mu[t] * mv[t];
          }
        }
        for (int o = 4; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 8);
          be += __shfl_xor(be, o, 8);
          ga += __shfl_xor(ga, o, 8);
        }
        if (live && (al >= nu2 || be >= nu2) && fabs(ga) > 2.0 * DBL_EPSILON * sqrt(al * be) &&
            ga != 0.0) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const int r = gl + 8 * t;
            if (r < mr) {
              M[r + i * ldm] = cs * mu[t] - sn * mv[t];
              M[r + k * ldm] = sn * mu[t] + cs * mv[t];
            }
            if (r < qc) {
              Q[r + i * ldq] = cs * qu[t] - sn * qv[t];
              Q[r + k * ldq] = sn * qu[t] + cs * qv[t];
            }
          }
          if (gl == 0) rotated[sweep & 1] = 1;
        }
      }
      __syncthreads();
      if (step == 0 && threadIdx.x == 0) rotated[(sweep + 1) & 1] = 0;
    }
    conv = (rotated[sweep & 1] == 0);
  }
  return conv;
}

// One-sided Jacobi SVD preconditioned by a column-pivoted QR (Drmac and Veselic): with
// M P = Q_h R (Householder, largest remaining column first) the Jacobi method runs on the
// rows of R, R' W = G, which are graded and converge in a few sweeps where the columns
// of M took twenty.  On return, as from lds_jacobi_svd, M holds U S (= Q_h W S, columns
// orthogonal with norms s = |G_j|) and Q holds V with M = M_in V: V = P G S^-1 (a column
// with s = 0 is set to zero; it is never used).  T is a scratch of qc x qc (leading
// dimension ld).  Returns false if the Jacobi sweeps did not converge.
__device__ bool lds_svd_qr(double* M, int mr, int qc, int ld, double* Q, double* T, double tol) {
  __shared__ double tau[PMAX], nrm[PMAX], sg[PMAX];
  __shared__ int perm[PMAX], piv_s;
  const int tid = threadIdx.x;
  const int g = tid >> 3, gl = tid & 7;  // 8 lanes per column
  for (int j = tid; j < qc; j += NTHREADS) {
    double s = 0.0;
    for (int r = 0; r < mr; ++r) s += M[r + j * ld] * M[r + j * ld];
    nrm[j] = s;
    perm[j] = j;
  }
  __syncthreads();
  for (int k = 0; k < qc; ++k) {
    if (tid < 64) {  // pivot: the largest remaining column (first index on ties)
      double v = (tid >= k && tid < qc) ? nrm[tid] : -1.0;
      int iv = tid;
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o, 64);
        const int i2 = __shfl_xor(iv, o, 64);
        if (v2 > v || (v2 == v && i2 < iv)) {
          v = v2;
          iv = i2;
        }
      }
      if (tid == 0) piv_s = iv;
    }
    __syncthreads();
    const int piv = piv_s;
    if (piv != k) {
      for (int r = tid; r < mr; r += NTHREADS) {
        const double x = M[r + k * ld];
        M[r + k * ld] = M[r + piv * ld];
        M[r + piv * ld] = x;
      }
      if (tid == 0) {
        const double x = nrm[k]; nrm[k] = nrm[piv]; nrm[piv] = x;
        const int i = perm[k]; perm[k] = perm[piv]; perm[piv] = i;
      }
      __syncthreads();
    }
    if (tid < 64) {  // Householder vector of column k, rows k.. (v_k = 1 implicit)
      const int r = k + tid;
      const double x = r < mr ? M[r + k * ld] : 0.0;
      double s2 = x * x;
      for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
      const double x0 = __shfl(x, 0, 64);
      const double al = sqrt(s2);
      double beta = 0.0, t = 0.0, scale = 0.0;
      if (al > 0.0) {
        beta = x0 >= 0.0 ? -al : al;
        t = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      if (r < mr) M[r + k * ld] = (tid == 0) ? beta : x * scale;
      if (tid == 0) tau[k] = t;
    }
    __syncthreads();
    // H_k on the columns right of k, and their norms over the rows below k
    const double tk = tau[k];
    for (int j0 = k + 1; j0 < qc; j0 += NTHREADS / 8) {
      const int j = j0 + g;
      if (j >= qc) break;  // uniform over the 8 lanes of a column
      double w = 0.0;
      for (int r = k + gl; r < mr; r += 8) w += (r == k ? 1.0 : M[r + k * ld]) * M[r + j * ld];
      for (int o = 4; o > 0; o >>= 1) w += __shfl_xor(w, o, 8);
      double n2 = 0.0;
      for (int r = k + gl; r < mr; r += 8) {
        const double y = M[r + j * ld] - tk * w * (r == k ? 1.0 : M[r + k * ld]);
        M[r + j * ld] = y;
        if (r > k) n2 += y * y;
      }
      for (int o = 4; o > 0; o >>= 1) n2 += __shfl_xor(n2, o, 8);
      if (gl == 0) nrm[j] = n2;
    }
    __syncthreads();
  }
  // R' (lower triangular) into T
  for (int e = tid; e < qc * qc; e += NTHREADS) {
    const int a = e % qc, b = e / qc;
    T[a + b * ld] = (b <= a) ? M[b + a * ld] : 0.0;
  }
  __syncthreads();
  // explicit Q_h (mr x qc) in place, last reflector first
  for (int k = qc - 1; k >= 0; --k) {
    const double tk = tau[k];
    for (int j0 = k + 1; j0 < qc; j0 += NTHREADS / 8) {
      const int j = j0 + g;
      if (j >= qc) break;
      double w = 0.0;
      for (int r = k + gl; r < mr; r += 8) w += (r == k ? 1.0 : M[r + k * ld]) * M[r + j * ld];
      for (int o = 4; o > 0; o >>= 1) w += __shfl_xor(w, o, 8);
      for (int r = k + gl; r < mr; r += 8)
        M[r + j * ld] -= tk * w * (r == k ? 1.0 : M[r + k * ld]);
    }
    __syncthreads();
    for (int r = tid; r < mr; r += NTHREADS)
      M[r + k * ld] = r < k ? 0.0 : (r == k ? 1.0 - tk : -tk * M[r + k * ld]);
    __syncthreads();
  }
  // one-sided Jacobi on the rows of R, W accumulated in Q
  const bool conv = lds_jacobi_svd(T, qc, qc, ld, Q, ld, tol);
  for (int j = tid; j < qc; j += NTHREADS) {
    double s = 0.0;
    for (int a = 0; a < qc; ++a) s += T[a + j * ld] * T[a + j * ld];
    sg[j] = sqrt(s);
  }
  __syncthreads();
  // M <- Q_h W S (each thread's entries in registers until every read is done)
  constexpr int EPT = (PMAX * PMAX + NTHREADS - 1) / NTHREADS;
  double acc[EPT];
#pragma unroll
  for (int t = 0; t < EPT; ++t) {
    const int e = tid + t * NTHREADS;
    acc[t] = 0.0;
    if (e < mr * qc) {
      const int r = e % mr, j = e / mr;
      double s = 0.0;
      for (int a = 0; a < qc; ++a) s += M[r + a * ld] * Q[a + j * ld];
      acc[t] = s * sg[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < EPT; ++t) {
    const int e = tid + t * NTHREADS;
    if (e < mr * qc) M[e % mr + (e / mr) * ld] = acc[t];
  }
  // Q <- P G S^-1
  __syncthreads();
  for (int e = tid; e < qc * qc; e += NTHREADS) {
    const int a = e % qc, j = e / qc;
    Q[perm[a] + j * ld] = sg[j] > 0.0 ? T[a + j * ld] / sg[j] : 0.0;
  }
  __syncthreads();
  return conv;
}

// ---------------------------------------------------------------------------------
// compression: one work-group per internal node
// ---------------------------------------------------------------------------------
// arguments of k_compress (one struct, so that grouped launches can stage one per member)
struct k_compress_args {
  const NodePlan* nodes;
  int nint;
  const double* x;
  int kind;
  double ell;
  double tol;
  const double* mpart;
  int mstride;
  const int* mtask_off;
  const int* kcap;
  double* tbuf;
  double* sv;
  int* rank;
  int* status;
  int pm;
  int h0;
  int h1;
};
__device__ __forceinline__ void k_compress_body(const k_compress_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const NodePlan* __restrict__ nodes = a_.nodes;
  int nint = a_.nint;
  const double* __restrict__ x = a_.x;
  int kind = a_.kind;
  double ell = a_.ell;
  double tol = a_.tol;
  const double* __restrict__ mpart = a_.mpart;
  int mstride = a_.mstride;
  const int* __restrict__ mtask_off = a_.mtask_off;
  const int* __restrict__ kcap = a_.kcap;
  double* __restrict__ tbuf = a_.tbuf;
  double* __restrict__ sv = a_.sv;
  int* __restrict__ rank = a_.rank;
  int* __restrict__ status = a_.status;
  int pm = a_.pm;
  int h0 = a_.h0;
  int h1 = a_.h1;
  (void)by_;
  (void)gy_;

  // nodes h0 .. h1-1, each with interpolation orders of at most pm
  const int h = h0 + bx_;
  if (h >= h1 || h >= nint) return;
  const NodePlan q = nodes[h];
  const int pI = q.pI, pJ = q.pJ;
  if (threadIdx.x < PMAX) sv[(size_t)h * PMAX + threadIdx.x] = 0.0;
  if (pI == 0 || pJ == 0) {
    if (threadIdx.x == 0) rank[h] = 0;
    return;
  }
  extern __shared__ double lds[];
  const int ld = pm;
  double* GI = lds;
  double* GJ = GI + pm * pm;
  double* Cm = GJ + pm * pm;
  double* Tm = Cm + pm * pm;
  double* Vm = Tm + pm * pm;
  __shared__ double sig[PMAX];
  __shared__ int order[PMAX];
  __shared__ int kk;
  // Gram matrices of the two bases
  for (int side = 0; side < 2; ++side) {
    double* G = side ? GJ : GI;
    const int p = side ? pJ : pI;
    const int exact = side ? q.exactJ : q.exactI;
    if (exact) {
      for (int idx = threadIdx.x; idx < p * p; idx += NTHREADS)
        G[idx % p + (idx / p) * ld] = (idx % p == idx / p) ? 1.0 : 0.0;
    } else {
      // final moments: sum the task partials in task order
      __shared__ double mom[2 * PMAX];
      const int t0 = mtask_off[2 * h + side], t1 = mtask_off[2 * h + side + 1];
      for (int m = threadIdx.x; m < 2 * p - 1; m += NTHREADS) {
        double s = 0.0;
        for (int t = t0; t < t1; ++t) s += mpart[(size_t)t * mstride + m];
        mom[m] = s;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < p * p; idx += NTHREADS) {
        const int r = idx % p, cc = idx / p;
        G[r + cc * ld] = 0.5 * (mom[r + cc] + mom[r > cc ? r - cc : cc - r]);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  __shared__ int permI[PMAX], permJ[PMAX];
  const int rkI = lds_pchol(GI, pI, ld, permI, Tm);
  const int rkJ = lds_pchol(GJ, pJ, ld, permJ, Tm);
  if (rkI < 0 || rkJ < 0) {
    if (threadIdx.x == 0) { atomicOr(status, ST_NOTSPD); rank[h] = 0; }
    return;
  }
  // kernel values at the interpolation nodes
  const double cI = 0.5 * (q.aI + q.bI), hI = 0.5 * (q.bI - q.aI);
  const double cJ = 0.5 * (q.aJ + q.bJ), hJ = 0.5 * (q.bJ - q.aJ);
  for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS) {
    const int s = idx % pI, t = idx / pI;
    const double xs = q.exactI ? x[q.i0 + s] : cI + hI * cos((2 * s + 1) * M_PI / (2.0 * pI));
    const double yt = q.exactJ ? x[q.mid + t] : cJ + hJ * cos((2 * t + 1) * M_PI / (2.0 * pJ));
    Cm[s + t * ld] = k1_value(kind, ell, xs, yt);
  }
  __syncthreads();
  // C_T = A_I C A_J'
  if (!q.exactI) {
    for (int idx = threadIdx.x; idx < pI * pI; idx += NTHREADS) {
      const int k = idx % pI, s = idx / pI;
      Vm[k + s * ld] = (k == 0 ? 1.0 : 2.0) / pI * cos(k * (2 * s + 1) * M_PI / (2.0 * pI));
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS) {
      const int k = idx % pI, t = idx / pI;
      double acc = 0.0;
      for (int s = 0; s < pI; ++s) acc += Vm[k + s * ld] * Cm[s + t * ld];
      Tm[k + t * ld] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS)
      Cm[idx % pI + (idx / pI) * ld] = Tm[idx % pI + (idx / pI) * ld];
    __syncthreads();
  }
  if (!q.exactJ) {
    for (int idx = threadIdx.x; idx < pJ * pJ; idx += NTHREADS) {
      const int k = idx % pJ, s = idx / pJ;
      Vm[k + s * ld] = (k == 0 ? 1.0 : 2.0) / pJ * cos(k * (2 * s + 1) * M_PI / (2.0 * pJ));
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS) {
      const int s = idx % pI, k = idx / pI;
      double acc = 0.0;
      for (int t = 0; t < pJ; ++t) acc += Cm[s + t * ld] * Vm[k + t * ld];
      Tm[s + k * ld] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS)
      Cm[idx % pI + (idx / pI) * ld] = Tm[idx % pI + (idx / pI) * ld];
    __syncthreads();
  }
  // X = F_I' C_T F_J   (G = F F', F = P' L)
  for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS) {
    const int r = idx % pI, t = idx / pI;
    double acc = 0.0;
    for (int s = 0; s < pI; ++s) acc += GI[s + r * ld] * Cm[s + t * ld];
    Tm[r + t * ld] = acc;
  }
  __syncthreads();
  const bool trans = pJ > pI;  // SVD of the taller orientation
  const int mr = trans ? pJ : pI, qc = trans ? pI : pJ;
  for (int idx = threadIdx.x; idx < pI * pJ; idx += NTHREADS) {
    const int r = idx % pI, t = idx / pI;
    double acc = 0.0;
    for (int s = 0; s < pJ; ++s) acc += Tm[r + s * ld] * GJ[s + t * ld];
    if (trans) Cm[t + r * ld] = acc; else Cm[r + t * ld] = acc;
  }
  __syncthreads();
  const bool conv = lds_svd_qr(Cm, mr, qc, ld, Vm, Tm, tol);
  if (!conv && threadIdx.x == 0) atomicOr(status, ST_NOTCONV);
  // singular values, descending order, rank
  if (threadIdx.x < qc) {
    double s = 0.0;
    for (int r = 0; r < mr; ++r) s += Cm[r + threadIdx.x * ld] * Cm[r + threadIdx.x * ld];
    sig[threadIdx.x] = sqrt(s);
  }
  __syncthreads();
  // descending order of the singular values (ties by index): thread j finds its place
  if (threadIdx.x < qc) {
    const int j = threadIdx.x;
    const double sj = sig[j];
    int pos = 0;
    for (int b = 0; b < qc; ++b) pos += (sig[b] > sj || (sig[b] == sj && b < j)) ? 1 : 0;
    order[pos] = j;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double thr = fmax(tol / 3.0, 8.0 * (DBL_EPSILON * 0.5) * sig[order[0]]);
    int k = 0;
    while (k < qc && sig[order[k]] > thr) ++k;
    kk = k;
    rank[h] = k;
  }
  __syncthreads();
  if (threadIdx.x < qc) sv[(size_t)h * PMAX + threadIdx.x] = sig[order[threadIdx.x]];
  // T_U = F_I^-T (U_X sqrt s), T_V = F_J^-T (V_X sqrt s); F' is upper triangular in the
  // pivot order, and the unknowns of steps at or beyond the rank are zero
  const int k = kk;
  const int kc = kcap[q.level];
  double* TU = tbuf + q.toff_u;
  double* TV = tbuf + q.toff_v;
  // column c of U_X sqrt(s) and V_X sqrt(s) for sorted index c: 8 lanes per column, lane gl
  // holding the unknowns of pivot positions gl, gl + 8, ... in registers
  constexpr int RPL = (PMAX + 7) / 8;
  const int gq = threadIdx.x >> 3, gl = threadIdx.x & 7;
  for (int idx0 = 0; idx0 < 2 * k; idx0 += NTHREADS / 8) {
    const int idx = idx0 + gq;
    if (idx >= 2 * k) break;  // uniform over the 8 lanes of a column
    const int c = idx % k, side = idx / k;
    const int j = order[c];
    const double sj = sig[j], rs = sqrt(sj);
    const int p = side ? pJ : pI;
    const int rkp = side ? rkJ : rkI;
    const int* pv = side ? permJ : permI;
    const double* F = side ? GJ : GI;
    double* out = side ? (TV + (size_t)c * pJ) : (TU + (size_t)c * pI);
    // no transpose: U_X = M[:,j]/s_j (length pI), V_X = Q[:,j] (length pJ)
    // transpose   : U_X = Q[:,j] (length pI),   V_X = M[:,j]/s_j (length pJ)
    const bool fromM = (side == 0) != trans;
    double sol[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) sol[t] = 0.0;
    for (int a = rkp - 1; a >= 0; --a) {
      double part = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int b = gl + 8 * t;
        if (b > a && b < rkp) part += F[pv[b] + a * ld] * sol[t];
      }
      for (int o = 4; o > 0; o >>= 1) part += __shfl_xor(part, o, 8);
      const double rhs = fromM ? Cm[a + j * ld] / sj * rs : Vm[a + j * ld] * rs;
      const double val = (rhs - part) / F[pv[a] + a * ld];
#pragma unroll
      for (int t = 0; t < RPL; ++t)
        if (gl + 8 * t == a) sol[t] = val;
    }
    // unknowns at or beyond the rank stay zero
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int b = gl + 8 * t;
      if (b < p) out[pv[b]] = sol[t];
    }
  }
  (void)kc;
}
__global__ void __launch_bounds__(NTHREADS) k_compress(const k_compress_args a_) {
  k_compress_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_compress_g(const k_compress_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_compress_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_compress_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_compress_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_compress_args* a, const int* st, const int* gy, int mm) {
    k_compress_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_compress now, or records it while a recorder is open on this thread
static void k_compress_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_compress_args& a) {
  if (recording())
    record_group(k_compress_grp, group_key((const void*)k_compress_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_compress<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// per-level maximum rank and the right-column lists used by the factorization
// ---------------------------------------------------------------------------------
constexpr int RL_THREADS = 1024;
// arguments of k_rank_levels (one struct, so that grouped launches can stage one per member)
struct k_rank_levels_args {
  const int* rank;
  int L;
  const int* coff;
  int Ktot;
  int* kmax;
  int* rcols;
  int* rcount;
};
__device__ __forceinline__ void k_rank_levels_body(const k_rank_levels_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const int* __restrict__ rank = a_.rank;
  int L = a_.L;
  const int* __restrict__ coff = a_.coff;
  int Ktot = a_.Ktot;
  int* __restrict__ kmax = a_.kmax;
  int* __restrict__ rcols = a_.rcols;
  int* __restrict__ rcount = a_.rcount;
  (void)by_;
  (void)gy_;

  if (bx_ != 0) return;
  __shared__ int km[32];
  if (threadIdx.x < 32) km[threadIdx.x] = 0;
  __syncthreads();
  // heap node h sits on level floor(log2(h + 1)); the tree is complete, 2^L - 1 nodes
  const int nint = (1 << L) - 1;
  for (int h = threadIdx.x; h < nint; h += RL_THREADS) atomicMax(&km[31 - __clz(h + 1)], rank[h]);
  __syncthreads();
  if (threadIdx.x < L) {
    const int l = threadIdx.x;
    kmax[l] = km[l];
    int c = km[l];
    for (int lp = 0; lp < l; ++lp) c += km[lp];
    rcount[l] = c;
  }
  // right-column list of level l: its own km[l] columns, then those of levels 0 .. l-1
  for (int idx = threadIdx.x; idx < L * Ktot; idx += RL_THREADS) {
    const int l = idx / Ktot;
    int rem = idx - l * Ktot;
    if (rem < km[l]) {
      rcols[idx] = coff[l] + rem;
      continue;
    }
    rem -= km[l];
    for (int lp = 0; lp < l; ++lp) {
      if (rem < km[lp]) {
        rcols[idx] = coff[lp] + rem;
        break;
      }
      rem -= km[lp];
    }
  }
}
__global__ void __launch_bounds__(RL_THREADS) k_rank_levels(const k_rank_levels_args a_) {
  k_rank_levels_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(RL_THREADS) k_rank_levels_g(const k_rank_levels_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_rank_levels_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_rank_levels_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_rank_levels_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_rank_levels_args* a, const int* st, const int* gy, int mm) {
    k_rank_levels_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_rank_levels now, or records it while a recorder is open on this thread
static void k_rank_levels_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_rank_levels_args& a) {
  if (recording())
    record_group(k_rank_levels_grp, group_key((const void*)k_rank_levels_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_rank_levels<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// panel generation: U rows of left children, V rows of right children (all levels)
// ---------------------------------------------------------------------------------
// arguments of k_panel_gen (one struct, so that grouped launches can stage one per member)
struct k_panel_gen_args {
  const Task* tasks;
  int ntask;
  const NodePlan* nodes;
  const double* x;
  const double* tbuf;
  const int* rank;
  const int* kmax;
  const int* coff;
  double* panel;
  int K;
};
__device__ __forceinline__ void k_panel_gen_body(const k_panel_gen_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const Task* __restrict__ tasks = a_.tasks;
  int ntask = a_.ntask;
  const NodePlan* __restrict__ nodes = a_.nodes;
  const double* __restrict__ x = a_.x;
  const double* __restrict__ tbuf = a_.tbuf;
  const int* __restrict__ rank = a_.rank;
  const int* __restrict__ kmax = a_.kmax;
  const int* __restrict__ coff = a_.coff;
  double* __restrict__ panel = a_.panel;
  int K = a_.K;
  (void)by_;
  (void)gy_;

  const int t = bx_;
  if (t >= ntask) return;
  const Task tk = tasks[t];
  const NodePlan q = nodes[tk.h];
  const int l = q.level;
  const int k = rank[tk.h], kl = kmax[l];
  const int p = tk.side ? q.pJ : q.pI;
  const int exact = tk.side ? q.exactJ : q.exactI;
  const int w0 = tk.side ? q.mid : q.i0, w1 = tk.side ? q.j1 : q.mid;
  const double a = tk.side ? q.aJ : q.aI, b = tk.side ? q.bJ : q.bI;
  const double c = 0.5 * (a + b), hw = 0.5 * (b - a);
  const double* T = tbuf + (tk.side ? q.toff_v : q.toff_u);
  // exact windows: T as stored (column cc at cc * p); interpolated windows: T transposed,
  // row m at m * kp, zero-padded to kp columns so that a chunk of PCB columns needs no guard
  constexpr int PCB = 8;
  __shared__ __align__(16) double Ts[PMAX * ((PMAX + PCB - 1) / PCB * PCB)];
  const int kp = (k + PCB - 1) / PCB * PCB;
  if (exact) {
    for (int idx = threadIdx.x; idx < p * k; idx += NTHREADS) Ts[idx] = T[idx];
  } else {
    for (int idx = threadIdx.x; idx < p * kp; idx += NTHREADS) {
      const int m = idx / kp, cc = idx - m * kp;
      Ts[idx] = cc < k ? T[cc * p + m] : 0.0;
    }
  }
  __syncthreads();
  const int cb = coff[l];
  for (int r = tk.r0 + threadIdx.x; r < tk.r1; r += NTHREADS) {
    const bool inwin = (r >= w0 && r < w1);
    if (!inwin || k == 0) {
      for (int cc = 0; cc < kl; ++cc) panel[pix(r, cb + cc, K)] = 0.0;
      continue;
    }
    if (exact) {
      const int e = r - w0;
      for (int cc = 0; cc < k; ++cc) panel[pix(r, cb + cc, K)] = Ts[cc * p + e];
    } else {
      // the recurrence T_m(t) runs once per chunk of PCB columns; each column sums its
      // terms in the order m = 0, 1, ..., p-1
      const double tt = hw > 0.0 ? (x[r] - c) / hw : 0.0;
      for (int c0 = 0; c0 < k; c0 += PCB) {
        double acc[PCB];
#pragma unroll
        for (int j = 0; j < PCB; ++j) acc[j] = Ts[c0 + j];
        if (p > 1) {
#pragma unroll
          for (int j = 0; j < PCB; ++j) acc[j] += tt * Ts[kp + c0 + j];
        }
        double tm2 = 1.0, tm1 = tt;
        for (int m = 2; m < p; ++m) {
          const double tn = 2.0 * tt * tm1 - tm2;
          const double* row = Ts + m * kp + c0;
#pragma unroll
          for (int j = 0; j < PCB; ++j) acc[j] += tn * row[j];
          tm2 = tm1;
          tm1 = tn;
        }
#pragma unroll
        for (int j = 0; j < PCB; ++j)
          if (c0 + j < k) panel[pix(r, cb + c0 + j, K)] = acc[j];
      }
    }
    for (int cc = k; cc < kl; ++cc) panel[pix(r, cb + cc, K)] = 0.0;
  }
}
__global__ void __launch_bounds__(NTHREADS) k_panel_gen(const k_panel_gen_args a_) {
  k_panel_gen_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_panel_gen_g(const k_panel_gen_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_panel_gen_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_panel_gen_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_panel_gen_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_panel_gen_args* a, const int* st, const int* gy, int mm) {
    k_panel_gen_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_panel_gen now, or records it while a recorder is open on this thread
static void k_panel_gen_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_panel_gen_args& a) {
  if (recording())
    record_group(k_panel_gen_grp, group_key((const void*)k_panel_gen_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_panel_gen<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// sampled entries of K~_1
// ---------------------------------------------------------------------------------
__global__ void k_entries(const NodePlan* __restrict__ nodes, int nint,
                          const double* __restrict__ x, int kind, double ell, double nugget,
                          const int* __restrict__ kmax, const int* __restrict__ coff,
                          const double* __restrict__ panel, int K, const int64_t* __restrict__ ii,
                          const int64_t* __restrict__ jj, int64_t count, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int i = (int)ii[t], j = (int)jj[t];
  if (i > j) { const int tmp = i; i = j; j = tmp; }
  int h = 0;
  while (h < nint) {
    const NodePlan q = nodes[h];
    if (j < q.mid) h = 2 * h + 1;
    else if (i >= q.mid) h = 2 * h + 2;
    else {
      double acc = 0.0;
      const int cb = coff[q.level];
      for (int c = 0; c < kmax[q.level]; ++c) acc += panel[pix(i, cb + c, K)] * panel[pix(j, cb + c, K)];
      out[t] = acc;
      return;
    }
  }
  out[t] = k1_value(kind, ell, x[i], x[j]) + (i == j ? nugget : 0.0);
}

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
void launch_build(HodlrData& H, hipStream_t s) {
  const HostPlan& P = H.pk->P;
  const DevPlan D = H.pk->D;
  timer_forget(H.kmax);  // the ranks change below
  if (P.L == 0) return;
  // the plan's scalars (launches recorded for a grouped replay copy what they use)
  const int nm = P.nmt, nint = P.nint, kind = P.kind, mstride = P.mpart_stride, L = P.L;
  const int Ktot = P.Ktot;
  const double ell = P.ell, tol = P.tol;
  const HodlrData Hc = H;
  if (nm > 0)
    k_moments_launch(dim3((nm + NTHREADS / 64 - 1) / (NTHREADS / 64)), dim3(NTHREADS), 0, s,
                     k_moments_args{D.mtasks, nm, D.nodes, Hc.x, Hc.mpart, mstride});
  // A work-group holds five p x p matrices in LDS, p the largest order of its launch.  The
  // top levels set the largest order; when every level from ls down needs at most half
  // that LDS and those levels hold far more nodes than the GPU keeps resident at the top
  // size (about 512 work-groups), they run in a second launch sized for their own order,
  // so that they do not hold LDS and CU slots at the size of the few top nodes.  With
  // fewer nodes the second launch would only add the top nodes' latency in series.
  constexpr int SPLIT_MIN_NODES = 2048;
  const int pm = std::max(P.pmax, 1);
  int ls = 0, pm_lo = pm;
  for (int l = P.L - 1, suf = 0; l >= 1; --l) {
    suf = std::max(suf, P.lpmax[l]);
    if (2 * suf * suf > pm * pm) break;
    ls = l;
    pm_lo = std::max(suf, 1);
  }
  if (ls > 0 && P.nint - ((1 << ls) - 1) < SPLIT_MIN_NODES) ls = 0;
  const int h_split = ls > 0 ? (1 << ls) - 1 : P.nint;
  // raised once to the largest size any plan can ask for (a function-local static is
  // initialised exactly once, whichever host thread builds first)
  static const bool lds_set = [] {
    (void)hipFuncSetAttribute((const void*)k_compress, hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(sizeof(double) * 5 * PMAX * PMAX));
    (void)hipFuncSetAttribute((const void*)k_compress_g,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(sizeof(double) * 5 * PMAX * PMAX));
    return true;
  }();
  (void)lds_set;

  k_compress_launch(dim3(h_split), dim3(NTHREADS), (uint32_t)(sizeof(double) * 5 * pm * pm), s,
                    k_compress_args{D.nodes, nint, Hc.x, kind, ell, tol, Hc.mpart, mstride,
                                    D.mtask_off, D.kcap, Hc.tbuf, Hc.sv, Hc.rank, Hc.status, pm,
                                    0, h_split});
  if (h_split < nint)
    k_compress_launch(dim3(nint - h_split), dim3(NTHREADS),
                      (uint32_t)(sizeof(double) * 5 * pm_lo * pm_lo), s,
                      k_compress_args{D.nodes, nint, Hc.x, kind, ell, tol, Hc.mpart, mstride,
                                      D.mtask_off, D.kcap, Hc.tbuf, Hc.sv, Hc.rank, Hc.status,
                                      pm_lo, h_split, nint});
  k_rank_levels_launch(dim3(1), dim3(RL_THREADS), 0, s,
                       k_rank_levels_args{Hc.rank, L, D.coff, Ktot, Hc.kmax, Hc.rcols, Hc.rcount});
  const int ng = P.ngt;
  k_panel_gen_launch(dim3(ng), dim3(NTHREADS), 0, s,
                     k_panel_gen_args{D.gtasks, ng, D.nodes, Hc.x, Hc.tbuf, Hc.rank, Hc.kmax,
                                      D.coff, Hc.panel, Ktot});
}

void launch_entries(const HodlrData& H, const int64_t* i, const int64_t* j, int64_t count,
                    double* out, hipStream_t s) {
  if (count <= 0) return;
  const int nb = int((count + 255) / 256);
  const HostPlan& P = H.pk->P;
  k_entries<<<nb, 256, 0, s>>>(H.pk->D.nodes, P.nint, H.x, P.kind, P.ell, P.nugget, H.kmax,
                               H.pk->D.coff, H.panel, P.Ktot, i, j, count, out);
}

}  // namespace fg
