// Vector operators of a HODLR matrix and of its symmetric factor (gfx950 kernels):
// W v, W' v, W^-1 v, W^-T v (level sweeps over the canonical node factors) and the
// product (alpha K~_1 + beta I) v (dense leaves evaluated on the fly + low-rank
// blocks, all levels in one pass).
//
// Per node, with s = U~' v_I and t = V~' v_J (level reduce) the node operators are
//   W      : v_J += V~ (s + F1 t)
//   W'     : v_I += U~ t,                 v_J += V~ F1 t
//   W^-1   : v_J += V~ (-s + F2 (t - G_V s))
//   W^-T   : w = F2 t; v_I -= U~ (t + G_V w); v_J += V~ w
// and the order of levels follows W = L_D W_(L-1) ... W_(0).
#include "fg_group.h"
#include "fg_internal.h"

namespace fg {

constexpr int NRHS_MAX = 4;

__device__ __forceinline__ double wave_red(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// leaf block operators L v (op 0) and L^-1 v (op 2), in place on v.  L is the leaf's
// lower triangle (column-major, leading dimension Bc); Dinv holds the inverses of its
// 16 x 16 diagonal blocks (in the diagonal blocks of the slot).  One work-group of BMAX
// threads per leaf; thread r owns row r of the leaf's vector block (nrhs columns in
// registers), so a wave's load of one column of L covers 64 consecutive rows.
//   L v:    row r sums L[r][s] v_s over s <= r, 16 columns per batch of loads.
//   L^-1 v: right-looking blocked substitution over the 16-row diagonal blocks:
//           v_j = D_j^-1 t_j, then every row below takes t_r -= L_rj v_j, j = 0, 1, ...;
//           a row's 16 coefficients of a step are loaded at the start of the step.
// (Factor data of precision T; vectors and arithmetic in FP64.)
// arguments of k_leaf_apply (one struct, so that grouped launches can stage one per member)
template <typename T>
struct k_leaf_apply_args {
  const int* leaf_lo;
  int nleaf;
  const T* Lm;
  const T* Dinv;
  int Bc;
  int op;
  double* v;
  int nrhs;
  int ld;
};
template <typename T>
__device__ __forceinline__ void k_leaf_apply_body(const k_leaf_apply_args<T>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const int* __restrict__ leaf_lo = a_.leaf_lo;
  int nleaf = a_.nleaf;
  const T* __restrict__ Lm = a_.Lm;
  const T* __restrict__ Dinv = a_.Dinv;
  int Bc = a_.Bc;
  int op = a_.op;
  double* __restrict__ v = a_.v;
  int nrhs = a_.nrhs;
  int ld = a_.ld;
  (void)by_;
  (void)gy_;

  const int b = bx_;
  if (b >= nleaf) return;
  const int lo = leaf_lo[b], m = leaf_lo[b + 1] - lo;
  const int r = threadIdx.x;
  const bool live = r < m;
  const T* Mb = Lm + (size_t)b * Bc * Bc;
  double x[NRHS_MAX];
#pragma unroll
  for (int c = 0; c < NRHS_MAX; ++c)
    x[c] = (live && c < nrhs) ? v[(size_t)c * ld + lo + r] : 0.0;
  if (op == 0) {
    __shared__ double vs[NRHS_MAX][BMAX];  // rows >= m hold zeros
#pragma unroll
    for (int c = 0; c < NRHS_MAX; ++c) vs[c][r] = x[c];
    __syncthreads();
    if (!live) return;
    double acc[NRHS_MAX] = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 <= r; s0 += 16) {
      double p[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        p[u] = (s0 + u <= r) ? (double)Mb[r + (size_t)(s0 + u) * Bc] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int c = 0; c < NRHS_MAX; ++c)
          if (c < nrhs) acc[c] += p[u] * vs[c][(s0 + u) & (BMAX - 1)];
    }
#pragma unroll
    for (int c = 0; c < NRHS_MAX; ++c)
      if (c < nrhs) v[(size_t)c * ld + lo + r] = acc[c];
    return;
  }
  __shared__ double ts[NRHS_MAX][16], vj[NRHS_MAX][16];
  // zeros where a ragged block has no rows (they meet zero coefficients)
  if (r < NRHS_MAX * 16) {
    ts[r >> 4][r & 15] = 0.0;
    vj[r >> 4][r & 15] = 0.0;
  }
  __syncthreads();
  const T* Db = Dinv + (size_t)b * Bc * Bc;
  const int nb = (m + 15) >> 4;
  const int jr = r >> 4, rr = r & 15;
  for (int j = 0; j < nb; ++j) {
    const int r0 = j * 16, mj = min(16, m - r0);
    const bool inb = live && jr == j;
    const bool upd = live && jr > j;
    // a row of D_j^-1 on block j's rows, L[r][r0 + u] on the rows below, zeros elsewhere
    double q[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      double w = 0.0;
      if (u < mj) {
        if (inb) {
          if (u <= rr) w = (double)Db[r + (size_t)(r0 + u) * Bc];
        } else if (upd) {
          w = (double)Mb[r + (size_t)(r0 + u) * Bc];
        }
      }
      q[u] = w;
    }
    if (inb)
#pragma unroll
      for (int c = 0; c < NRHS_MAX; ++c)
        if (c < nrhs) ts[c][rr] = x[c];
    __syncthreads();
    if (inb) {
#pragma unroll
      for (int c = 0; c < NRHS_MAX; ++c) {
        if (c < nrhs) {
          double acc = 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) acc += q[u] * ts[c][u];
          x[c] = acc;
          vj[c][rr] = acc;
        }
      }
    }
    __syncthreads();
    if (upd) {
#pragma unroll
      for (int c = 0; c < NRHS_MAX; ++c) {
        if (c < nrhs) {
          double acc = 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) acc += q[u] * vj[c][u];
          x[c] -= acc;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NRHS_MAX; ++c)
    if (live && c < nrhs) v[(size_t)c * ld + lo + r] = x[c];
}
template <typename T>
__global__ void __launch_bounds__(BMAX) k_leaf_apply(const k_leaf_apply_args<T> a_) {
  k_leaf_apply_body<T>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T>
__global__ void __launch_bounds__(BMAX) k_leaf_apply_g(const k_leaf_apply_args<T>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_leaf_apply_body<T>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T>
static void k_leaf_apply_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_leaf_apply_args<T>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_leaf_apply_args<T>* a, const int* st, const int* gy, int mm) {
    k_leaf_apply_g<T><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_leaf_apply now, or records it while a recorder is open on this thread
template <typename T>
static void k_leaf_apply_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_leaf_apply_args<T>& a) {
  if (recording())
    record_group(k_leaf_apply_grp<T>, group_key((const void*)k_leaf_apply_grp<T>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_leaf_apply<T><<<g, b, lds, s>>>(a);
}

// transposed leaf block operators L' v (op 1) and L^-T v (op 3), in place on v.  Their
// reads run along L's columns, so threads take consecutive entries of one column:
//   L' v:   one thread per (row r, vector column) sums L[s][r] v_s over s >= r, 16 rows
//           of column r per batch of loads.
//   L^-T v: left-looking blocked substitution,
//           v_i <- D_i^-T (v_i - sum_{j>i} L_ji' v_j),  i = nb-1, ..., 0,
//           four threads per (row of block i, vector column) reading consecutive rows of
//           L's column, their partial sums combined by shuffles.
// (Factor data of precision T; vectors and arithmetic in FP64.)
// arguments of k_leaf_apply_t (one struct, so that grouped launches can stage one per member)
template <typename T>
struct k_leaf_apply_t_args {
  const int* leaf_lo;
  int nleaf;
  const T* Lm;
  const T* Dinv;
  int Bc;
  int op;
  double* v;
  int nrhs;
  int ld;
};
template <typename T>
__device__ __forceinline__ void k_leaf_apply_t_body(const k_leaf_apply_t_args<T>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const int* __restrict__ leaf_lo = a_.leaf_lo;
  int nleaf = a_.nleaf;
  const T* __restrict__ Lm = a_.Lm;
  const T* __restrict__ Dinv = a_.Dinv;
  int Bc = a_.Bc;
  int op = a_.op;
  double* __restrict__ v = a_.v;
  int nrhs = a_.nrhs;
  int ld = a_.ld;
  (void)by_;
  (void)gy_;

  const int b = bx_;
  if (b >= nleaf) return;
  const int lo = leaf_lo[b], m = leaf_lo[b + 1] - lo;
  __shared__ double vs[NRHS_MAX][BMAX];  // rows >= m hold zeros
  __shared__ double ts[NRHS_MAX][16];
  for (int idx = threadIdx.x; idx < BMAX * nrhs; idx += NTHREADS) {
    const int c = idx / BMAX, r = idx % BMAX;
    vs[c][r] = r < m ? v[(size_t)c * ld + lo + r] : 0.0;
  }
  __syncthreads();
  const T* Mb = Lm + (size_t)b * Bc * Bc;
  if (op == 1) {
    for (int idx = threadIdx.x; idx < m * nrhs; idx += NTHREADS) {
      const int r = idx % m, c = idx / m;
      double acc = 0.0;
      for (int s0 = r; s0 < m; s0 += 16) {  // 16 entries of column r per batch of loads
        double p[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) p[u] = (s0 + u < m) ? (double)Mb[s0 + u + (size_t)r * Bc] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += p[u] * vs[c][(s0 + u) & (BMAX - 1)];
      }
      v[(size_t)c * ld + lo + r] = acc;
    }
    return;
  }
  const T* Db = Dinv + (size_t)b * Bc * Bc;
  const int nb = (m + 15) >> 4;
  const int q = threadIdx.x & 3, e = threadIdx.x >> 2;  // e: 0..63 = row (16) x column (4)
  const int rr = e & 15, c = e >> 4;
  for (int i = nb - 1; i >= 0; --i) {
    const int r = i * 16 + rr;
    double t = 0.0;
    if (c < nrhs && r < m)
      // eight loads in flight, added in the order of s (a row past the leaf reads row 0)
      for (int s0 = (i + 1) * 16 + q; s0 < m; s0 += 32) {
        double p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int s = s0 + 4 * u;
          p[u] = (double)Mb[(s < m ? s : 0) + (size_t)r * Bc];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (s0 + 4 * u < m) t += p[u] * vs[c][s0 + 4 * u];
      }
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    if (q == 0 && c < nrhs) ts[c][rr] = (r < m) ? vs[c][r] - t : 0.0;
    __syncthreads();
    // v_i = D_i^-T t, with D_i^-1 lower triangular
    if (q == 0 && c < nrhs && r < m) {
      double u = 0.0;
      const int r0 = i * 16, mi = min(16, m - r0);
      // the row's entries loaded together, then added in the order of s2
      double p[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int s2 = rr + k;
        p[k] = (double)Db[(r0 + (s2 < mi ? s2 : rr)) + (size_t)(r0 + rr) * Bc];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (rr + k < mi) u += p[k] * ts[c][rr + k];
      vs[c][r] = u;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * nrhs; idx += NTHREADS)
    v[(size_t)(idx / m) * ld + lo + idx % m] = vs[idx / m][idx % m];
}
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_leaf_apply_t(const k_leaf_apply_t_args<T> a_) {
  k_leaf_apply_t_body<T>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_leaf_apply_t_g(const k_leaf_apply_t_args<T>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_leaf_apply_t_body<T>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T>
static void k_leaf_apply_t_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_leaf_apply_t_args<T>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_leaf_apply_t_args<T>* a, const int* st, const int* gy, int mm) {
    k_leaf_apply_t_g<T><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_leaf_apply_t now, or records it while a recorder is open on this thread
template <typename T>
static void k_leaf_apply_t_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_leaf_apply_t_args<T>& a) {
  if (recording())
    record_group(k_leaf_apply_t_grp<T>, group_key((const void*)k_leaf_apply_t_grp<T>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_leaf_apply_t<T><<<g, b, lds, s>>>(a);
}

// level reduce with a vector right operand: z[t][a][c] = sum_rows P[i, coff + a] v[i, c]
//
// The panel stores 16-row groups with each column's 16 rows contiguous, so the level's
// columns of one group are contiguous too.  A wave reads 4 adjacent columns x 16 rows
// (512 contiguous bytes) per load: lane = 16 * (column slot) + (row in group), and the
// group's 16 entries of each v column (read straight from memory).  Waves stride over the
// task's groups; rows outside the task (partial first and last groups) are masked.  Lane
// partials are summed over the 16 row lanes, then over the 4 waves in a fixed order.
// NR >= nrhs bounds the vector columns held in registers.
// arguments of k_reduce_vec (one struct, so that grouped launches can stage one per member)
template <typename T, int NR>
struct k_reduce_vec_args {
  const Task* tasks;
  int tbase;
  int ntask;
  const NodePlan* nodes;
  const int* coff;
  const int* kmax;
  const T* P;
  int K;
  const double* v;
  int nrhs;
  int ldv;
  double* zpart;
  int zs_task;
};
template <typename T, int NR>
__device__ __forceinline__ void k_reduce_vec_body(const k_reduce_vec_args<T, NR>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const Task* __restrict__ tasks = a_.tasks;
  int tbase = a_.tbase;
  int ntask = a_.ntask;
  const NodePlan* __restrict__ nodes = a_.nodes;
  const int* __restrict__ coff = a_.coff;
  const int* __restrict__ kmax = a_.kmax;
  const T* __restrict__ P = a_.P;
  int K = a_.K;
  const double* __restrict__ v = a_.v;
  int nrhs = a_.nrhs;
  int ldv = a_.ldv;
  double* __restrict__ zpart = a_.zpart;
  int zs_task = a_.zs_task;
  (void)by_;
  (void)gy_;

  const int t = bx_;
  if (t >= ntask) return;
  const Task tk = tasks[tbase + t];
  const int l = nodes[tk.h].level;
  const int c0 = coff[l], kl = kmax[l];
  const int gr0 = tk.r0 & ~15;                 // first row of the first group
  const int ng = (tk.r1 - gr0 + 15) >> 4;      // groups touched
  __shared__ double red[NTHREADS / 64][16][NR];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rl = lane & 15, cslot = lane >> 4;
  for (int q0 = 0; q0 < kl; q0 += 16) {
    double acc[4][NR];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < NR; ++c) acc[j][c] = 0.0;
    // 4 groups per pass (g, g + NW, g + 2 NW, g + 3 NW): all their loads are issued
    // before any product
    constexpr int NW = NTHREADS / 64;
    for (int g0 = wv; g0 < ng; g0 += 4 * NW) {
      double p[4][4], vv[4][NR];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int g = g0 + bb * NW;
        const int r = gr0 + g * 16 + rl;
        const bool ok = g < ng && r >= tk.r0 && r < tk.r1;
        const T* pg = P + ((size_t)((gr0 >> 4) + g) * K + c0 + q0) * 16 + lane;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          p[bb][j] = (ok && q0 + 4 * j + cslot < kl) ? (double)pg[64 * j] : 0.0;
#pragma unroll
        for (int c = 0; c < NR; ++c)
          vv[bb][c] = (ok && c < nrhs) ? v[(size_t)c * ldv + r] : 0.0;
      }
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int c = 0; c < NR; ++c)
          if (c < nrhs)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j][c] += p[bb][j] * vv[bb][c];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < NR; ++c)
        if (c < nrhs)
          for (int o = 1; o < 16; o <<= 1) acc[j][c] += __shfl_xor(acc[j][c], o, 64);
    if (rl == 0)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < NR; ++c)
          if (c < nrhs) red[wv][4 * j + cslot][c] = acc[j][c];
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * nrhs; e += NTHREADS) {
      const int aa = e / nrhs, c = e - aa * nrhs, a = q0 + aa;
      if (a < kl)
        zpart[(size_t)t * zs_task + a * nrhs + c] =
            (red[0][aa][c] + red[1][aa][c]) + (red[2][aa][c] + red[3][aa][c]);
    }
    __syncthreads();
  }
}
template <typename T, int NR>
__global__ void __launch_bounds__(NTHREADS) k_reduce_vec(const k_reduce_vec_args<T, NR> a_) {
  k_reduce_vec_body<T, NR>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T, int NR>
__global__ void __launch_bounds__(NTHREADS) k_reduce_vec_g(const k_reduce_vec_args<T, NR>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_reduce_vec_body<T, NR>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T, int NR>
static void k_reduce_vec_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_reduce_vec_args<T, NR>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_reduce_vec_args<T, NR>* a, const int* st, const int* gy, int mm) {
    k_reduce_vec_g<T, NR><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_reduce_vec now, or records it while a recorder is open on this thread
template <typename T, int NR>
static void k_reduce_vec_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_reduce_vec_args<T, NR>& a) {
  if (recording())
    record_group(k_reduce_vec_grp<T, NR>, group_key((const void*)k_reduce_vec_grp<T, NR>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_reduce_vec<T, NR><<<g, b, lds, s>>>(a);
}

// per-node coefficients.  op: 0 W, 1 W', 2 W^-1, 3 W^-T, 4 matvec (alpha scaling)
//
// The two sides' sums S, T of the task partials come from zsum for sides it presummed,
// else from the partials themselves: with E = 2 k nrhs elements, G = blockDim / E groups
// per element sum tasks t0 + g, t0 + g + G, ... (eight loads in flight), and the G group
// sums are added in group order.  A level whose sides hold many tasks runs 1 024 threads.
constexpr int NC_MAX_THREADS = 1024;
// arguments of k_node_coef (one struct, so that grouped launches can stage one per member)
struct k_node_coef_args {
  int op;
  int hbase;
  int nnode;
  const int* rank;
  const int* node_task_off;
  int tbase;
  const double* zpart;
  int zs_task;
  int nrhs;
  const double* nodemat;
  const int* nodemat_off;
  double alpha_v;
  const double* alpha_p;
  double* coef;
  int cs_node;
  const double* zsum;
};
__device__ __forceinline__ void k_node_coef_body(const k_node_coef_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int op = a_.op;
  int hbase = a_.hbase;
  int nnode = a_.nnode;
  const int* __restrict__ rank = a_.rank;
  const int* __restrict__ node_task_off = a_.node_task_off;
  int tbase = a_.tbase;
  const double* __restrict__ zpart = a_.zpart;
  int zs_task = a_.zs_task;
  int nrhs = a_.nrhs;
  const double* __restrict__ nodemat = a_.nodemat;
  const int* __restrict__ nodemat_off = a_.nodemat_off;
  double alpha_v = a_.alpha_v;
  const double* __restrict__ alpha_p = a_.alpha_p;
  double* __restrict__ coef = a_.coef;
  int cs_node = a_.cs_node;
  const double* __restrict__ zsum = a_.zsum;
  (void)by_;
  (void)gy_;

  const int jn = bx_;
  if (jn >= nnode) return;
  const int h = hbase + jn;
  const int k = rank[h];
  if (k == 0) return;
  __shared__ double S[PMAX][NRHS_MAX], T[PMAX][NRHS_MAX], X[PMAX][NRHS_MAX];
  const int kn = k * nrhs, E = 2 * kn;
  const int G = E >= (int)blockDim.x ? 1 : (int)blockDim.x / E;
  __shared__ double red[NC_MAX_THREADS];  // E * G <= max(E, blockDim) <= 1 024
  for (int idx = threadIdx.x; idx < E * G; idx += blockDim.x) {
    const int ei = idx % E, g = idx / E;
    const int side = ei / kn, e = ei % kn;
    double s = 0.0;
    const int t0 = node_task_off[2 * h + side] - tbase;
    const int t1 = node_task_off[2 * h + side + 1] - tbase;
    if (zsum && t1 - t0 > 1) {  // presummed per node side (k_zsum)
      if (g == 0) s = zsum[(size_t)(2 * jn + side) * zs_task + e];
    } else {
      int t = t0 + g;
      for (; t + 7 * G < t1; t += 8 * G) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = zpart[(size_t)(t + u * G) * zs_task + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; t < t1; t += G) s += zpart[(size_t)t * zs_task + e];
    }
    red[idx] = s;
  }
  __syncthreads();
  for (int ei = threadIdx.x; ei < E; ei += blockDim.x) {
    double s = red[ei];
    for (int g = 1; g < G; ++g) s += red[g * E + ei];
    const int side = ei / kn, e = ei % kn;
    if (side) T[e / nrhs][e % nrhs] = s; else S[e / nrhs][e % nrhs] = s;
  }
  __syncthreads();
  double* cI = coef + (size_t)jn * cs_node;
  double* cJ = cI + PMAX * NRHS_MAX;
  if (op == 4) {
    const double al = alpha_p ? *alpha_p : alpha_v;
    for (int e = threadIdx.x; e < kn; e += blockDim.x) {
      cI[e] = al * T[e / nrhs][e % nrhs];
      cJ[e] = al * S[e / nrhs][e % nrhs];
    }
    return;
  }
  const double* GV = nodemat + nodemat_off[h];
  const double* F1 = GV + k * k;
  const double* F2 = GV + 2 * k * k;
  if (op == 0 || op == 1) {
    for (int e = threadIdx.x; e < kn; e += blockDim.x) {
      const int a = e / nrhs, c = e % nrhs;
      double f = 0.0;
      for (int d = 0; d < k; ++d) f += F1[a + d * k] * T[d][c];
      if (op == 0) { cI[e] = 0.0; cJ[e] = S[a][c] + f; }
      else { cI[e] = T[a][c]; cJ[e] = f; }
    }
    return;
  }
  if (op == 2) {
    for (int e = threadIdx.x; e < kn; e += blockDim.x) {
      const int a = e / nrhs, c = e % nrhs;
      double u = T[a][c];
      for (int d = 0; d < k; ++d) u -= GV[a + d * k] * S[d][c];
      X[a][c] = u;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kn; e += blockDim.x) {
      const int a = e / nrhs, c = e % nrhs;
      double f = -S[a][c];
      for (int d = 0; d < k; ++d) f += F2[a + d * k] * X[d][c];
      cI[e] = 0.0;
      cJ[e] = f;
    }
    return;
  }
  // op == 3
  for (int e = threadIdx.x; e < kn; e += blockDim.x) {
    const int a = e / nrhs, c = e % nrhs;
    double w = 0.0;
    for (int d = 0; d < k; ++d) w += F2[a + d * k] * T[d][c];
    X[a][c] = w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kn; e += blockDim.x) {
    const int a = e / nrhs, c = e % nrhs;
    double g = T[a][c];
    for (int d = 0; d < k; ++d) g += GV[a + d * k] * X[d][c];
    cI[e] = -g;
    cJ[e] = X[a][c];
  }
}
__global__ void __launch_bounds__(NC_MAX_THREADS) k_node_coef(const k_node_coef_args a_) {
  k_node_coef_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NC_MAX_THREADS) k_node_coef_g(const k_node_coef_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_node_coef_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_node_coef_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_node_coef_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_node_coef_args* a, const int* st, const int* gy, int mm) {
    k_node_coef_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_node_coef now, or records it while a recorder is open on this thread
static void k_node_coef_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_node_coef_args& a) {
  if (recording())
    record_group(k_node_coef_grp, group_key((const void*)k_node_coef_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_node_coef<<<g, b, lds, s>>>(a);
}

// v[rows of side] += P[rows, coff + a] coef_side[a][c]
// One row per thread (work-group y of a task takes rows r0 + 256 y + thread, stepping by
// 256 gridDim.y); the row's panel columns are loaded 8 at a time before they are used.
// arguments of k_update_vec (one struct, so that grouped launches can stage one per member)
template <typename T>
struct k_update_vec_args {
  const Task* tasks;
  int tbase;
  int ntask;
  const NodePlan* nodes;
  int hbase;
  const int* rank;
  const int* coff;
  const T* P;
  int K;
  double* v;
  int nrhs;
  int ldv;
  const double* coef;
  int cs_node;
  int skip_left;
};
template <typename T>
__device__ __forceinline__ void k_update_vec_body(const k_update_vec_args<T>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const Task* __restrict__ tasks = a_.tasks;
  int tbase = a_.tbase;
  int ntask = a_.ntask;
  const NodePlan* __restrict__ nodes = a_.nodes;
  int hbase = a_.hbase;
  const int* __restrict__ rank = a_.rank;
  const int* __restrict__ coff = a_.coff;
  const T* __restrict__ P = a_.P;
  int K = a_.K;
  double* __restrict__ v = a_.v;
  int nrhs = a_.nrhs;
  int ldv = a_.ldv;
  const double* __restrict__ coef = a_.coef;
  int cs_node = a_.cs_node;
  int skip_left = a_.skip_left;
  (void)by_;
  (void)gy_;

  const int t = bx_;
  if (t >= ntask) return;
  const Task tk = tasks[tbase + t];
  if (skip_left && tk.side == 0) return;
  const int k = rank[tk.h];
  if (k == 0) return;
  const int l = nodes[tk.h].level;
  const double* cf = coef + (size_t)(tk.h - hbase) * cs_node + tk.side * PMAX * NRHS_MAX;
  __shared__ double cs[PMAX * NRHS_MAX];
  for (int e = threadIdx.x; e < k * nrhs; e += NTHREADS) cs[e] = cf[e];
  __syncthreads();
  const int cb = coff[l];
  for (int r = tk.r0 + by_ * NTHREADS + threadIdx.x; r < tk.r1;
       r += NTHREADS * gy_) {
    double acc[NRHS_MAX] = {0.0, 0.0, 0.0, 0.0};
    const T* pr = P + ((size_t)(r >> 4) * K + cb) * 16 + (r & 15);
    int a = 0;
    for (; a + 8 <= k; a += 8) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = (double)pr[(size_t)(a + u) * 16];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < NRHS_MAX; ++c)
          if (c < nrhs) acc[c] += p[u] * cs[(a + u) * nrhs + c];
    }
    for (; a < k; ++a) {
      const double pv = (double)pr[(size_t)a * 16];
#pragma unroll
      for (int c = 0; c < NRHS_MAX; ++c)
        if (c < nrhs) acc[c] += pv * cs[a * nrhs + c];
    }
#pragma unroll
    for (int c = 0; c < NRHS_MAX; ++c)
      if (c < nrhs) v[(size_t)c * ldv + r] += acc[c];
  }
}
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_update_vec(const k_update_vec_args<T> a_) {
  k_update_vec_body<T>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T>
__global__ void __launch_bounds__(NTHREADS) k_update_vec_g(const k_update_vec_args<T>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_update_vec_body<T>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T>
static void k_update_vec_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_update_vec_args<T>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_update_vec_args<T>* a, const int* st, const int* gy, int mm) {
    k_update_vec_g<T><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_update_vec now, or records it while a recorder is open on this thread
template <typename T>
static void k_update_vec_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_update_vec_args<T>& a) {
  if (recording())
    record_group(k_update_vec_grp<T>, group_key((const void*)k_update_vec_grp<T>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_update_vec<T><<<g, b, lds, s>>>(a);
}

// y = alpha (K_leaf + nugget I) v + beta v + sum_levels panel rows x coefficients
// arguments of k_mv_apply (one struct, so that grouped launches can stage one per member)
struct k_mv_apply_args {
  const int* leaf_lo;
  int nleaf;
  int L;
  const double* x;
  int kind;
  double ell;
  double nugget;
  double alpha_v;
  const double* alpha_p;
  double beta_v;
  const double* beta_p;
  const double* v;
  double* y;
  int nrhs;
  int ld;
  const int* rank;
  const int* coff;
  const double* P;
  int K;
  const double* coef;
  int cs_node;
};
__device__ __forceinline__ void k_mv_apply_body(const k_mv_apply_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const int* __restrict__ leaf_lo = a_.leaf_lo;
  int nleaf = a_.nleaf;
  int L = a_.L;
  const double* __restrict__ x = a_.x;
  int kind = a_.kind;
  double ell = a_.ell;
  double nugget = a_.nugget;
  double alpha_v = a_.alpha_v;
  const double* __restrict__ alpha_p = a_.alpha_p;
  double beta_v = a_.beta_v;
  const double* __restrict__ beta_p = a_.beta_p;
  const double* __restrict__ v = a_.v;
  double* __restrict__ y = a_.y;
  int nrhs = a_.nrhs;
  int ld = a_.ld;
  const int* __restrict__ rank = a_.rank;
  const int* __restrict__ coff = a_.coff;
  const double* __restrict__ P = a_.P;
  int K = a_.K;
  const double* __restrict__ coef = a_.coef;
  int cs_node = a_.cs_node;
  (void)by_;
  (void)gy_;

  const int b = bx_;
  if (b >= nleaf) return;
  const int lo = leaf_lo[b], m = leaf_lo[b + 1] - lo;
  const double alpha = alpha_p ? *alpha_p : alpha_v;
  const double beta = beta_p ? *beta_p : beta_v;
  __shared__ double xs[BMAX];
  __shared__ double vs[NRHS_MAX][BMAX];
  for (int r = threadIdx.x; r < m; r += BMAX) {
    xs[r] = x[lo + r];
    for (int c = 0; c < nrhs; ++c) vs[c][r] = v[(size_t)c * ld + lo + r];
  }
  __syncthreads();
  const int r = threadIdx.x;
  if (r >= m) return;
  const int i = lo + r;
  double acc[NRHS_MAX];
  for (int c = 0; c < nrhs; ++c) acc[c] = (beta + alpha * nugget) * vs[c][r];
  const double xr = xs[r];
  double kacc[NRHS_MAX] = {0.0, 0.0, 0.0, 0.0};
  for (int s2 = 0; s2 < m; ++s2) {
    const double kv = k1_value(kind, ell, xr, xs[s2]);
    for (int c = 0; c < nrhs; ++c) kacc[c] += kv * vs[c][s2];
  }
  for (int c = 0; c < nrhs; ++c) acc[c] += alpha * kacc[c];
  for (int l = 0; l < L; ++l) {
    const int h = (1 << l) - 1 + (b >> (L - l));
    const int k = rank[h];
    if (k == 0) continue;
    const int side = (b >> (L - l - 1)) & 1;
    const double* cf = coef + (size_t)h * cs_node + side * PMAX * NRHS_MAX;
    // column cb + a of row i lies a * 16 words after column cb; eight loads are issued
    // before their products so that a wave keeps several in flight
    const double* Pc = P + pix(i, coff[l], K);
    int a = 0;
    for (; a + 8 <= k; a += 8) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = Pc[(size_t)(a + u) * 16];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        for (int c = 0; c < nrhs; ++c) acc[c] += pv[u] * cf[(a + u) * nrhs + c];
    }
    for (; a < k; ++a) {
      const double pv = Pc[(size_t)a * 16];
      for (int c = 0; c < nrhs; ++c) acc[c] += pv * cf[a * nrhs + c];
    }
  }
  for (int c = 0; c < nrhs; ++c) y[(size_t)c * ld + i] = acc[c];
}
__global__ void __launch_bounds__(BMAX) k_mv_apply(const k_mv_apply_args a_) {
  k_mv_apply_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(BMAX) k_mv_apply_g(const k_mv_apply_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_mv_apply_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_mv_apply_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_mv_apply_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_mv_apply_args* a, const int* st, const int* gy, int mm) {
    k_mv_apply_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_mv_apply now, or records it while a recorder is open on this thread
static void k_mv_apply_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_mv_apply_args& a) {
  if (recording())
    record_group(k_mv_apply_grp, group_key((const void*)k_mv_apply_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_mv_apply<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
// workspace: task partials | per-node coefficients | per-node-side presummed partials
size_t apply_work_doubles(const HostPlan& P, int nrhs) {
  (void)nrhs;
  const size_t zp = (size_t)std::max(P.max_ltasks, 1) * PMAX * NRHS_MAX;
  const size_t cf = (size_t)std::max(P.nint, 1) * 2 * PMAX * NRHS_MAX;
  return zp + 2 * cf;
}

size_t matvec_work_doubles(const HostPlan& P, int nrhs) {
  (void)nrhs;
  const size_t zp = (size_t)std::max(P.nlt, 1) * PMAX * NRHS_MAX;
  const size_t cf = (size_t)std::max(P.nint, 1) * 2 * PMAX * NRHS_MAX;
  return zp + 2 * cf;
}

template <typename T>
static void sweep_level(FactorData& F, const T* panel, int op, int l, double* v, int nrhs, int ld,
                        double* work, hipStream_t s) {
  const HodlrData& H = *F.H;
  const HostPlan& P = H.pk->P;
  const DevPlan& D = H.pk->D;
  const int tb = P.ltask_off[l], nt = P.ltask_off[l + 1] - tb;
  const int zs_task = PMAX * NRHS_MAX;
  double* zpart = work;
  double* coef = work + (size_t)std::max(P.max_ltasks, 1) * zs_task;
  const int cs_node = 2 * PMAX * NRHS_MAX;
  const int hbase = (1 << l) - 1;
#define FG_REDUCE_VEC(NR_)                                                                   \
  k_reduce_vec_launch<T, NR_>(dim3(nt), dim3(NTHREADS), 0, s,                                  \
                              k_reduce_vec_args<T, NR_>{D.ltasks, tb, nt, D.nodes, D.coff, H.kmax, \
                                                        panel, P.Ktot, v, nrhs, ld, zpart, zs_task})
  if (nrhs <= 1) FG_REDUCE_VEC(1); else if (nrhs <= 2) FG_REDUCE_VEC(2); else FG_REDUCE_VEC(4);
#undef FG_REDUCE_VEC
  // the node coefficients sum the sides' task partials themselves (no separate pass)
  k_node_coef_launch(dim3(1 << l), dim3(P.max_tps[l] > 1 ? NC_MAX_THREADS : 64), 0, s, k_node_coef_args{
      op, hbase, 1 << l, H.rank, D.node_task_off, tb, zpart, zs_task, nrhs, F.nodemat,
      D.nodemat_off, 0.0, nullptr, coef, cs_node, nullptr});
  const int skip_left = (op == 0 || op == 2) ? 1 : 0;
  const dim3 grid_u(nt, (std::min(P.max_trows[l], RCH) + NTHREADS - 1) / NTHREADS);
  k_update_vec_launch<T>(grid_u, dim3(NTHREADS), 0, s, k_update_vec_args<T>{D.ltasks, tb, nt, D.nodes, hbase, H.rank, D.coff,
                                              panel, P.Ktot, v, nrhs, ld, coef, cs_node,
                                              skip_left});
}

template <typename T>
static void apply_w(FactorData& F, const T* leafL, const T* leafLinv, const double* panel, int op,
                    double* v, int nrhs, int ld, double* work, hipStream_t s) {
  const HostPlan& P = F.H->pk->P;
  const int* leaf_lo = F.H->pk->D.leaf_lo;
  // W = L_D W_(L-1) ... W_(0)
  auto leaf = [&](int lop) {
    if (lop == 0 || lop == 2)
      k_leaf_apply_launch<T>(dim3(P.nleaf), dim3(BMAX), 0, s, k_leaf_apply_args<T>{leaf_lo, P.nleaf, leafL, leafLinv, P.B, lop, v,
                                               nrhs, ld});
    else
      k_leaf_apply_t_launch<T>(dim3(P.nleaf), dim3(NTHREADS), 0, s, k_leaf_apply_t_args<T>{leaf_lo, P.nleaf, leafL, leafLinv, P.B, lop,
                                                     v, nrhs, ld});
  };
  if (op == 0) {          // W v: W_(0) first, then finer levels, then L_D
    for (int l = 0; l < P.L; ++l) sweep_level<double>(F, panel, 0, l, v, nrhs, ld, work, s);
    leaf(0);
  } else if (op == 1) {   // W' v = W_(0)' ... W_(L-1)' L_D' v
    leaf(1);
    for (int l = P.L - 1; l >= 0; --l) sweep_level<double>(F, panel, 1, l, v, nrhs, ld, work, s);
  } else if (op == 2) {   // W^-1 v = W_(0)^-1 ... W_(L-1)^-1 L_D^-1 v
    leaf(2);
    for (int l = P.L - 1; l >= 0; --l) sweep_level<double>(F, panel, 2, l, v, nrhs, ld, work, s);
  } else {                // W^-T v = L_D^-T W_(L-1)^-T ... W_(0)^-T v
    for (int l = 0; l < P.L; ++l) sweep_level<double>(F, panel, 3, l, v, nrhs, ld, work, s);
    leaf(3);
  }
}

void launch_apply_w(FactorData& F, int op, double* v, int nrhs, int ld, double* work,
                    hipStream_t s) {
  if (F.fp32)  // FP32 leaf factor, FP64 levels
    apply_w<float>(F, F.leafLf, F.leafLinvf, F.panel, op, v, nrhs, ld, work, s);
  else
    apply_w<double>(F, F.leafL, F.leafLinv, F.panel, op, v, nrhs, ld, work, s);
}

void launch_matvec(const HodlrData& H, double alpha, double beta, const double* alpha_dev,
                   const double* beta_dev, const double* v, double* y, int nrhs, int ld,
                   double* work, hipStream_t s) {
  const HostPlan& P = H.pk->P;
  const DevPlan& D = H.pk->D;
  const int zs_task = PMAX * NRHS_MAX;
  const int nt = P.nlt;
  double* zpart = work;
  double* coef = work + (size_t)std::max(nt, 1) * zs_task;
  const int cs_node = 2 * PMAX * NRHS_MAX;
  if (P.L > 0) {
#define FG_REDUCE_VEC(NR_)                                                                 \
  k_reduce_vec_launch<double, NR_>(                                                          \
      dim3(nt), dim3(NTHREADS), 0, s,                                                        \
      k_reduce_vec_args<double, NR_>{D.ltasks, 0, nt, D.nodes, D.coff, H.kmax, H.panel, P.Ktot, \
                                     v, nrhs, ld, zpart, zs_task})
    if (nrhs <= 1) FG_REDUCE_VEC(1); else if (nrhs <= 2) FG_REDUCE_VEC(2); else FG_REDUCE_VEC(4);
#undef FG_REDUCE_VEC
    double* zs = coef + (size_t)std::max(P.nint, 1) * cs_node;
    launch_zsum(zpart, zs_task, 0, D.node_task_off, 0, 2 * P.nint, zs_task, zs, zs_task,
                *std::max_element(P.max_tps.begin(), P.max_tps.end()), s);
    k_node_coef_launch(dim3(P.nint), dim3(64), 0, s,
                       k_node_coef_args{4, 0, P.nint, H.rank, D.node_task_off, 0, zpart, zs_task,
                                        nrhs, nullptr, nullptr, alpha, alpha_dev, coef, cs_node,
                                        zs});
  }
  k_mv_apply_launch(dim3(P.nleaf), dim3(BMAX), 0, s,
                    k_mv_apply_args{D.leaf_lo, P.nleaf, P.L, H.x, P.kind, P.ell, P.nugget, alpha,
                                    alpha_dev, beta, beta_dev, v, y, nrhs, ld, H.rank, D.coff,
                                    H.panel, P.Ktot, coef, cs_node});
}

}  // namespace fg
