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

#include "fg_group.h"
#include "fg_internal.h"
#include "fg_timer.h"

namespace fg {

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------
// leaves: Cholesky and the log-det (the panel rows are whitened by k_whiten on matrix
// cores)
//
// One work-group of 256 threads per leaf (m <= 128 rows).  The leaf matrix lives in
// registers in a 16 x 16 thread grid: thread (tr, tc) holds the 8 x 8 elements
// (16 i + tr, 16 j + tc) of the block lower triangle.  Right-looking Cholesky one column
// at a time, with every thread of the work-group in every column step: the 16 threads
// that hold column j (one quarter of one wave) take its pivot from the lane that holds
// it, scale the column and publish it in LDS; after one barrier every thread subtracts
// L[r][j] L[c][j] from its entries right of and below it.  A step is a short chain of
// register operations, one LDS write and read and one barrier, so no wave waits on a
// serial factorization of a diagonal block.  After each 16 columns the finished block
// column is written out and the register tile shifts by one block, so that the current
// block column is always register column 0 and every register index is fixed at
// compile time.  The inverses of the 16 x 16 diagonal blocks of L (used by the
// whitening and the solves) are then formed by forward substitution, one column of one
// block per thread.  Output: L (lower triangle), those inverses and the log-det.
// ---------------------------------------------------------------------------------
constexpr int LG = 16;        // thread grid side
constexpr int LE = BMAX / LG; // 16-row blocks per leaf (8)
constexpr int LPD = 17;       // LDS pitch of a stored 16 x 16 diagonal block

// a value of lane l, as a wave-uniform value (l a compile-time index after unrolling)
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

#ifndef LEAF_OCC
#define LEAF_OCC 4  // work-groups per CU the leaf kernel's registers are sized for
#endif
#define LT(i, j) ((i) * ((i) + 1) / 2 + (j))
// arguments of k_leaf (one struct, so that grouped launches can stage one per member)
template <typename T>
struct k_leaf_args {
  const int* leaf_lo;
  int nleaf;
  const double* x;
  int kind;
  double ell;
  double nugget;
  double alpha_v;
  const double* alpha_p;
  double beta_v;
  const double* beta_p;
  const double* diag;
  int Bc;
  T* leafL;
  T* leafLinv;
  double* leaf_ld;
  int* status;
};
template <typename T>
__device__ __forceinline__ void k_leaf_body(const k_leaf_args<T>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const int* __restrict__ leaf_lo = a_.leaf_lo;
  int nleaf = a_.nleaf;
  const double* __restrict__ x = a_.x;
  int kind = a_.kind;
  double ell = a_.ell;
  double nugget = a_.nugget;
  double alpha_v = a_.alpha_v;
  const double* __restrict__ alpha_p = a_.alpha_p;
  double beta_v = a_.beta_v;
  const double* __restrict__ beta_p = a_.beta_p;
  const double* __restrict__ diag = a_.diag;
  int Bc = a_.Bc;
  T* __restrict__ leafL = a_.leafL;
  T* __restrict__ leafLinv = a_.leafLinv;
  double* __restrict__ leaf_ld = a_.leaf_ld;
  int* __restrict__ status = a_.status;
  (void)by_;
  (void)gy_;

  const int b = bx_;
  if (b >= nleaf) return;
  const int lo = leaf_lo[b], m = leaf_lo[b + 1] - lo;
  const int nb = (m + 15) >> 4;  // 16-row blocks in use
  const double alpha = alpha_p ? *alpha_p : alpha_v;
  const double beta = beta_p ? *beta_p : beta_v;
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  const int wave = threadIdx.x >> 6;
  // LDS: the inputs, column j of L (two buffers: column j + 1 is written while slower
  // waves may still read column j), the pivots and their reciprocals, and the diagonal
  // blocks of L for their inverses (19 KB in FP64)
  __shared__ double xs[BMAX];
  __shared__ T colb[2][BMAX];
  __shared__ T piv_s[BMAX], pinv_s[BMAX];
  __shared__ T Ld[LE][16 * LPD];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int r = threadIdx.x; r < m; r += NTHREADS) xs[r] = x[lo + r];
  colb[threadIdx.x >> 7][threadIdx.x & 127] = T(0);
  __syncthreads();
  // block-lower part only: element (16 i + tr, 16 jj + tc), jj <= i, at a[LT(i, jj)]; after
  // kb block columns are done, a[LT(i, jj)] holds block (kb + i, kb + jj)
  T a[LE * (LE + 1) / 2];
#pragma unroll
  for (int i = 0; i < LE; ++i) {
    const int r = LG * i + tr;
#pragma unroll
    for (int jj = 0; jj <= i; ++jj) {
      const int c = LG * jj + tc;
      double v = (r == c) ? 1.0 : 0.0;
      if (r < m && c < m) {
        v = alpha * k1_value(kind, ell, xs[r], xs[c]);
        if (r == c) v += alpha * nugget + beta + (diag ? diag[lo + r] : 0.0);
      }
      a[LT(i, jj)] = (T)v;  // entries are formed in FP64 and stored in T
    }
  }
  bool mybad = false;
  T* Lg = leafL + (size_t)b * Bc * Bc;
  for (int kb = 0; kb < nb; ++kb) {
    const int nbr = nb - kb;  // block rows from the current one down
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int j = 16 * kb + t;
      if (j < m) {  // (uniform: the last block may be partial)
        T* col = colb[t & 1];
        if (wave == (t >> 2)) {
          // the pivot sits in thread (t, t), the column in threads (., t): one wave
          const T piv = lane_value(a[LT(0, 0)], (17 * t) & 63);
          const bool ok = piv > T(0);
          mybad |= !ok;
          const T sq = ok ? sqrt(piv) : T(1);
          const T inv = T(1) / sq;
          if (tc == t) {
#pragma unroll
            for (int i = 0; i < LE; ++i) {
              if (i < nbr) {
                const int rho = LG * i + tr;  // row within the current block row and below
                if (rho > t) {
                  a[LT(i, 0)] *= inv;
                  col[rho] = a[LT(i, 0)];
                } else {
                  col[rho] = T(0);  // rows up to the pivot take no update
                  if (rho == t) {
                    a[LT(0, 0)] = sq;
                    piv_s[j] = sq;
                    pinv_s[j] = inv;
                  }
                }
              }
            }
          }
        }
        __syncthreads();
        // trailing update: entries (rho, c) with t < c <= rho take -L[rho][j] L[c][j].  The
        // published column is zero at rows up to the pivot, so every entry of the tile can
        // take the product with no test: the finished columns (c <= t) and rows (rho <= t)
        // are multiplied by zero, and the upper triangles of the diagonal blocks, which
        // nothing reads, take the mirror image of their lower triangles' updates.
        T lr[LE], lc[LE];
#pragma unroll
        for (int i = 0; i < LE; ++i) {
          lr[i] = (i < nbr) ? col[LG * i + tr] : T(0);
          lc[i] = (i < nbr) ? col[LG * i + tc] : T(0);
        }
#pragma unroll
        for (int i = 0; i < LE; ++i) {
          if (i < nbr) {
#pragma unroll
            for (int jj = 0; jj <= i; ++jj) a[LT(i, jj)] -= lr[i] * lc[jj];
          }
        }
      }
    }
    // block column kb is final: L to global (lower triangle, column-major, ld = Bc), the
    // diagonal block to LDS for its inverse; then the tile moves up one block
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      const int r = 16 * kb + LG * i + tr, c = 16 * kb + tc;
      if (i < nbr && r < m && c <= r) Lg[r + (size_t)c * Bc] = a[LT(i, 0)];
    }
    Ld[kb][tr * LPD + tc] = (tc <= tr) ? a[LT(0, 0)] : T(0);
#pragma unroll
    for (int i = 0; i + 1 < LE; ++i) {
#pragma unroll
      for (int jj = 0; jj <= i; ++jj) a[LT(i, jj)] = a[LT(i + 1, jj + 1)];
    }
  }
  if (mybad) bad = 1;
  __syncthreads();
  // inverses of the diagonal blocks: thread (block bb, column c) solves L_bb x = e_c by
  // forward substitution (row k: x_k = (e_c,k - sum_{jj<k} L[k][jj] x_jj) / L[k][k], the
  // terms in increasing jj) and writes x into column c of the block's slot
  if (threadIdx.x < 16 * LE) {
    const int bb = threadIdx.x >> 4, c = threadIdx.x & 15;
    if (bb < nb) {
      const T* Lb = Ld[bb];
      T* Lig = leafLinv + (size_t)b * Bc * Bc + (size_t)(16 * bb) * (Bc + 1);
      T xv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        T acc = (k == c) ? T(1) : T(0);
#pragma unroll
        for (int jj = 0; jj < k; ++jj)
          if (jj >= c) acc -= Lb[k * LPD + jj] * xv[jj];
        const int kk = 16 * bb + k;
        xv[k] = (k >= c && kk < m) ? acc * pinv_s[kk] : T(0);
        if (k >= c && kk < m) Lig[k + (size_t)c * Bc] = xv[k];
      }
    }
  }
  // log-det: sum of 2 log L[j][j], wave 0 with two rows per lane, in a fixed order
  if (wave == 0) {
    const int l = threadIdx.x;
    double ls = (l < m && piv_s[l] > T(0)) ? 2.0 * log((double)piv_s[l]) : 0.0;
    if (l + 64 < m && piv_s[l + 64] > T(0)) ls += 2.0 * log((double)piv_s[l + 64]);
    ls = wsum(ls);
    if (l == 0) {
      leaf_ld[b] = ls;  // sum log(pivot) = 2 sum log diag(L)
      if (bad) atomicOr(status, ST_NOTSPD);
    }
  }
}
template <typename T>
__global__ void __launch_bounds__(NTHREADS, LEAF_OCC) k_leaf(const k_leaf_args<T> a_) {
  k_leaf_body<T>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T>
__global__ void __launch_bounds__(NTHREADS, LEAF_OCC) k_leaf_g(const k_leaf_args<T>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_leaf_body<T>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T>
static void k_leaf_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_leaf_args<T>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_leaf_args<T>* a, const int* st, const int* gy, int mm) {
    k_leaf_g<T><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_leaf now, or records it while a recorder is open on this thread
template <typename T>
static void k_leaf_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_leaf_args<T>& a) {
  if (recording())
    record_group(k_leaf_grp<T>, group_key((const void*)k_leaf_grp<T>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_leaf<T><<<g, b, lds, s>>>(a);
}

#undef LT

// ---------------------------------------------------------------------------------
// level reduce (panel x panel): Z[a][b] = sum_i P[i, coff_l + a] P[i, rcols_l[b]]
//
// A tall-skinny product (rows are the reduction dimension) on FP64 matrix cores:
// v_mfma_f64_16x16x4f64 takes A (16 x 4) with lane l holding A[l%16][l/16], B (4 x 16)
// with lane l holding B[l/16][l%16], and accumulates D (16 x 16) with lane l holding
// D[l/16 + 4 v][l%16], v = 0..3 (layout checked on gfx950).  Here M = left columns a, N = right columns b and
// K = rows.  Each wave owns 16 right columns and all left tiles and reads 16 rows of them
// per step straight from the panel (16-byte loads of four rows of a column).
// ---------------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
// global-address-space views, for accesses the compiler would otherwise make flat
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) double gdouble;

// one 16 x 16 x 4 MFMA step in the precision of the panel, and the accumulator row of
// (lane group kg, register v): f64 puts row kg + 4 v in register v, f32 row 4 kg + v
// (both layouts checked on gfx950)
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kg, int v) { return kg + 4 * v; }
  // row of a 16-row block that lane group kg feeds into K-step s; equal to row(kg, s), so
  // accumulator register s of a finished block is the B operand of step s
  static __device__ __forceinline__ int kcol(int kg, int s) { return 4 * s + kg; }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kg, int v) { return 4 * kg + v; }
  static __device__ __forceinline__ int kcol(int kg, int s) { return 4 * kg + s; }
};

// Four consecutive panel rows of one column (16-byte aligned) with 16-byte loads.
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const float4 a = reinterpret_cast<const float4*>(p)[0];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Each wave owns 16 right columns of one task and every 16-column left tile; it walks
// the task's rows 16 at a time with no LDS and no barrier.  For step s (0..3) of a
// 16-row group, K-slot k holds row base + 4k + s, so lane l reads rows base + 4 (l/16)
// .. +3 of its column: 32 contiguous bytes, and the four steps use each 128-byte line
// of the 16-row tile completely.
// arguments of k_reduce_panel (one struct, so that grouped launches can stage one per member)
template <typename T, int NA>
struct k_reduce_panel_args {
  const Task* tasks;
  int tbase;
  int ntask;
  int l;
  const int* coff;
  const int* kmax;
  const int* rcols;
  const int* rcount;
  int K;
  const T* P;
  double* zpart;
  int zs_a;
  int zs_task;
};
template <typename T, int NA>
__device__ __forceinline__ void k_reduce_panel_body(const k_reduce_panel_args<T, NA>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const Task* __restrict__ tasks = a_.tasks;
  int tbase = a_.tbase;
  int ntask = a_.ntask;
  int l = a_.l;
  const int* __restrict__ coff = a_.coff;
  const int* __restrict__ kmax = a_.kmax;
  const int* __restrict__ rcols = a_.rcols;
  const int* __restrict__ rcount = a_.rcount;
  int K = a_.K;
  const T* __restrict__ P = a_.P;
  double* __restrict__ zpart = a_.zpart;
  int zs_a = a_.zs_a;
  int zs_task = a_.zs_task;
  (void)by_;
  (void)gy_;

  typedef typename Mfma<T>::acc_t acc_t;
  const int t = bx_;
  if (t >= ntask) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c0 = coff[l], kl = kmax[l], W = rcount[l];
  const int b0 = by_ * 64 + wv * 16;
  if (b0 >= W || kl == 0) return;
  const Task tk = tasks[tbase + t];
  const int na = min(NA, (kl + 15) >> 4);  // left tiles in use (NA: capacity of the level)
  const int cl = lane & 15, kg = lane >> 4;
  const int bcol = b0 + cl;
  const int gcb = bcol < W ? rcols[(size_t)l * K + bcol] : -1;
  int acol[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acol[q] = (q * 16 + cl < kl) ? c0 + q * 16 + cl : -1;
  acc_t acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = acc_t{T(0), T(0), T(0), T(0)};
  const bool aligned = ((tk.r0 | tk.r1) & 15) == 0;
  // operands of one 16-row group: bv (this wave's 16 right columns) and av[q] (left tile q).
  // A lane's four rows of a column are 16-byte aligned and contiguous: read them with
  // 16-byte loads (8-byte loads leave the kernel at about half the bandwidth).
  auto load = [&](int base, T (&bv)[4], T (&av)[NA][4]) {
    if (aligned) {
      load4(P + pix(base + 4 * kg, gcb < 0 ? 0 : gcb, K), bv);
#pragma unroll
      for (int s = 0; s < 4; ++s) bv[s] = gcb >= 0 ? bv[s] : T(0);
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        load4(P + pix(base + 4 * kg, acol[q] < 0 ? 0 : acol[q], K), av[q]);
#pragma unroll
        for (int s = 0; s < 4; ++s) av[q][s] = (q < na && acol[q] >= 0) ? av[q][s] : T(0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = base + 4 * kg + s;
        bv[s] = (gcb >= 0 && row < tk.r1) ? P[pix(row, gcb, K)] : T(0);
#pragma unroll
        for (int q = 0; q < NA; ++q)
          av[q][s] = (q < na && acol[q] >= 0 && row < tk.r1) ? P[pix(row, acol[q], K)] : T(0);
      }
    }
  };
  for (int base = tk.r0; base < tk.r1; base += 16) {
    T bv[4], av[NA][4];
    load(base, bv, av);
#pragma unroll
    for (int q = 0; q < NA; ++q)
      if (q < na) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[q] = Mfma<T>::step(av[q][s], bv[s], acc[q]);
      }
  }
  if (bcol < W) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      if (q < na) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = q * 16 + Mfma<T>::row(kg, v);
          if (a < kl) zpart[(size_t)t * zs_task + (size_t)a * zs_a + bcol] = (double)acc[q][v];
        }
      }
    }
  }
}
template <typename T, int NA>
__global__ void __launch_bounds__(NTHREADS) k_reduce_panel(const k_reduce_panel_args<T, NA> a_) {
  k_reduce_panel_body<T, NA>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T, int NA>
__global__ void __launch_bounds__(NTHREADS) k_reduce_panel_g(const k_reduce_panel_args<T, NA>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_reduce_panel_body<T, NA>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T, int NA>
static void k_reduce_panel_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_reduce_panel_args<T, NA>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_reduce_panel_args<T, NA>* a, const int* st, const int* gy, int mm) {
    k_reduce_panel_g<T, NA><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_reduce_panel now, or records it while a recorder is open on this thread
template <typename T, int NA>
static void k_reduce_panel_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_reduce_panel_args<T, NA>& a) {
  if (recording())
    record_group(k_reduce_panel_grp<T, NA>, group_key((const void*)k_reduce_panel_grp<T, NA>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_reduce_panel<T, NA><<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// leaf whitening on matrix cores: dst = sqrt(alpha) L^-1 src for every active panel
// column of every level, rows of one leaf per work-group, by blocked forward
// substitution in 16-row blocks:  Y_j = D_j^-1 Y_j;  Y_i -= L_ij Y_j (i > j).  L may be
// stored in FP32 (TL = float, the mixed-precision factor); the substitution is FP64.
//
// The 28 strictly lower 16 x 16 blocks of L (negated) and the 8 diagonal-block inverses
// D_j^-1 are staged in LDS once (pitch 17), with each thread's loads issued in batches.
// Each wave owns two groups of 16 panel columns at a time, keeps the leaf's 8 row blocks
// of both in MFMA accumulators, and feeds every operand read from LDS to both; a finished
// block's register s is exactly the B operand of K-step s (rows Mfma::kcol), so results
// feed the next products without moving.  Every column is read once and written once.
// ---------------------------------------------------------------------------------
constexpr int WB = BMAX / 16;          // 16-row blocks per leaf (8)
constexpr int WTRI = WB * (WB + 1) / 2;  // lower blocks (36)
constexpr int WPD = 17;                // LDS pitch of a staged block

// arguments of k_whiten (one struct, so that grouped launches can stage one per member)
template <typename T, typename TL>
struct k_whiten_args {
  const int* leaf_lo;
  int nleaf;
  const TL* leafL;
  const TL* leafLinv;
  int Bc;
  double alpha_v;
  const double* alpha_p;
  const double* src;
  T* dst;
  int K;
  const int* coff;
  const int* kmax;
  int L;
};
template <typename T, typename TL>
__device__ __forceinline__ void k_whiten_body(const k_whiten_args<T, TL>& a_, const int bx_, const int by_,
                                             const int gy_) {
  const int* __restrict__ leaf_lo = a_.leaf_lo;
  int nleaf = a_.nleaf;
  const TL* __restrict__ leafL = a_.leafL;
  const TL* __restrict__ leafLinv = a_.leafLinv;
  int Bc = a_.Bc;
  double alpha_v = a_.alpha_v;
  const double* __restrict__ alpha_p = a_.alpha_p;
  const double* __restrict__ src = a_.src;
  T* __restrict__ dst = a_.dst;
  int K = a_.K;
  const int* __restrict__ coff = a_.coff;
  const int* __restrict__ kmax = a_.kmax;
  int L = a_.L;
  (void)by_;
  (void)gy_;

  static_assert(sizeof(T) == 8, "the whitening runs in FP64");
  const int b = bx_;
  if (b >= nleaf) return;
  const int lo = __builtin_amdgcn_readfirstlane(leaf_lo[b]);
  const int m = __builtin_amdgcn_readfirstlane(leaf_lo[b + 1]) - lo;
  const int nb = (m + 15) >> 4;
  __shared__ double Ls[WTRI * 16 * WPD];
  const TL* Lg = leafL + (size_t)b * Bc * Bc;
  const TL* Dg = leafLinv + (size_t)b * Bc * Bc;
  int total = 0;
  for (int l = 0; l < L; ++l) total += kmax[l];
  total = __builtin_amdgcn_readfirstlane(total);
  const int ngrp = (total + 15) >> 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cl = lane & 15, kg = lane >> 4;
  // panel entries as byte offsets from the leaf's first row tile (below 2^32: at most 9
  // tiles of K * 128 bytes), wave-uniform base in the global address space
  const gchar* sb = (const gchar*)(src + (size_t)(lo >> 4) * K * 16);
  gchar* db = (gchar*)(dst + (size_t)(lo >> 4) * K * 16);
  const int r0 = lo & 15;
  auto off = [&](int row, int gc) -> unsigned {
    const int rr = r0 + row;
    return (unsigned)((((rr >> 4) * K + gc) * 16 + (rr & 15)) * 8);
  };
  // panel column of group g for this lane (-1 past the last active column)
  auto column = [&](int g) -> int {
    int f = 16 * g + cl;
    if (f >= total) return -1;
    for (int l = 0; l < L; ++l) {
      const int km = kmax[l];
      if (f < km) return coff[l] + f;
      f -= km;
    }
    return -1;
  };
  // rows past the leaf and columns past the last read a valid entry (row 0, column 0) and
  // are replaced by zero; all loads are issued before any is used
  auto load = [&](int gc, d4 (&acc)[WB]) {
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i * 16 + Mfma<double>::row(kg, v);
        const bool ok = gc >= 0 && row < m;
        acc[i][v] = *(const gdouble*)(sb + (ok ? off(row, gc) : off(0, 0)));
      }
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i * 16 + Mfma<double>::row(kg, v);
        acc[i][v] = (gc >= 0 && row < m) ? acc[i][v] : 0.0;
      }
  };
  // Each wave takes column groups w and w + 4 (then w + 8 and w + 12, ...) together: two
  // independent substitutions share every A operand read from LDS.  The first pair's panel
  // reads are issued before the factor is staged, so their latency overlaps the staging.
  int g0 = w;
  int gcA = column(g0), gcB = column(g0 + 4);
  d4 accA[WB], accB[WB];
  load(gcA, accA);
  load(gcB, accB);
  // stage: element (r, c) of block t = (bi, bj) at Ls[t*16*WPD + r*WPD + c]; r runs
  // fastest so that reads of the column-major factors are contiguous.  A factor held in
  // FP32 is widened exactly: the products below are those of that factor, in FP64.  Blocks
  // and rows past the leaf are zero, so the substitution below runs on all WB blocks.
  // Thread x stages element x of every block (WTRI x 256 elements, 256 threads), so each
  // block index is a compile-time constant and the loads go out SB at a time rather than
  // one round trip each.
  static_assert(NTHREADS == 256, "one element of every staged block per thread");
  {
    constexpr int SB = 12;  // loads in flight per thread while staging
    static_assert(WTRI % SB == 0, "staging batches");
    const int r = threadIdx.x & 15, c = threadIdx.x >> 4;
#pragma unroll
    for (int t0 = 0; t0 < WTRI; t0 += SB) {
      double v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int t = t0 + u;
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
        const int bj = t - bi * (bi + 1) / 2;
        const int gr = bi * 16 + r, gcol = bj * 16 + c;
        // entries outside the leaf read entry 0 (always valid) and are replaced by zero
        const bool ok = bi == bj ? (gr < m && c <= r) : (bi < nb && gr < m);
        const size_t e = ok ? gr + (size_t)gcol * Bc : 0;
        v[u] = (double)(bi == bj ? Dg[e] : Lg[e]);
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int t = t0 + u;
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
        const int bj = t - bi * (bi + 1) / 2;
        const int gr = bi * 16 + r;
        const bool ok = bi == bj ? (gr < m && c <= r) : (bi < nb && gr < m);
        Ls[t * 16 * WPD + r * WPD + c] = ok ? (bi == bj ? v[u] : -v[u]) : 0.0;
      }
    }
  }
  __syncthreads();
  const double alpha = alpha_p ? *alpha_p : alpha_v;
  const double sa = sqrt(alpha);
  for (;;) {
    if (g0 >= ngrp) break;
#pragma unroll
    for (int j = 0; j < WB; ++j) {
      // the lane's operand offset is made opaque per block, so that the compiler reads a
      // block's four operands just before its steps rather than all of them up front
      auto opnd = [&](int i, int s4, unsigned lb) -> double {
        return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(Ls) + lb +
                                                (((i * (i + 1) / 2 + j) * 16 * WPD) + 4 * s4) * 8);
      };
      unsigned lb = (unsigned)(cl * WPD + kg) * 8u;
      asm volatile("" : "+v"(lb));
      d4 yA = d4{0.0, 0.0, 0.0, 0.0}, yB = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double d = opnd(j, s4, lb);
        yA = Mfma<double>::step(d, accA[j][s4], yA);
        yB = Mfma<double>::step(d, accB[j][s4], yB);
      }
      accA[j] = yA;
      accB[j] = yB;
#pragma unroll
      for (int i = j + 1; i < WB; ++i) {
        unsigned li = (unsigned)(cl * WPD + kg) * 8u;
        asm volatile("" : "+v"(li));
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const double a = opnd(i, s4, li);
          accA[i] = Mfma<double>::step(a, accA[j][s4], accA[i]);
          accB[i] = Mfma<double>::step(a, accB[j][s4], accB[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i * 16 + Mfma<double>::row(kg, v);
        if (row < m) {
          if (gcA >= 0) *(gdouble*)(db + off(row, gcA)) = sa * accA[i][v];
          if (gcB >= 0) *(gdouble*)(db + off(row, gcB)) = sa * accB[i][v];
        }
      }
    g0 += 8;
    if (g0 >= ngrp) break;
    gcA = column(g0);
    gcB = column(g0 + 4);
    load(gcA, accA);
    load(gcB, accB);
  }
}
template <typename T, typename TL>
__global__ void __launch_bounds__(NTHREADS, 2) k_whiten(const k_whiten_args<T, TL> a_) {
  k_whiten_body<T, TL>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <typename T, typename TL>
__global__ void __launch_bounds__(NTHREADS, 2) k_whiten_g(const k_whiten_args<T, TL>* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_whiten_body<T, TL>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <typename T, typename TL>
static void k_whiten_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_whiten_args<T, TL>>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_whiten_args<T, TL>* a, const int* st, const int* gy, int mm) {
    k_whiten_g<T, TL><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_whiten now, or records it while a recorder is open on this thread
template <typename T, typename TL>
static void k_whiten_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_whiten_args<T, TL>& a) {
  if (recording())
    record_group(k_whiten_grp<T, TL>, group_key((const void*)k_whiten_grp<T, TL>, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_whiten<T, TL><<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// deterministic sum of task partials per node side: zfin[side][e] = sum_t zpart[t][e]
// (4 task lanes per entry, combined in a fixed order).  Sides with a single task are
// skipped: their consumers read zpart[t0] in place.
// ---------------------------------------------------------------------------------
// arguments of k_zsum (one struct, so that grouped launches can stage one per member)
struct k_zsum_args {
  const double* zpart;
  int zs_task;
  int tbase;
  const int* node_task_off;
  int hbase;
  int nsides;
  int esz;
  double* zfin;
  int zf_side;
};
__device__ __forceinline__ void k_zsum_body(const k_zsum_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const double* __restrict__ zpart = a_.zpart;
  int zs_task = a_.zs_task;
  int tbase = a_.tbase;
  const int* __restrict__ node_task_off = a_.node_task_off;
  int hbase = a_.hbase;
  int nsides = a_.nsides;
  int esz = a_.esz;
  double* __restrict__ zfin = a_.zfin;
  int zf_side = a_.zf_side;
  (void)by_;
  (void)gy_;

  const int sd = bx_;
  if (sd >= nsides) return;
  const int h = hbase + (sd >> 1), side = sd & 1;
  const int t0 = node_task_off[2 * h + side] - tbase, t1 = node_task_off[2 * h + side + 1] - tbase;
  if (t1 - t0 <= 1) return;
  const int e = by_ * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  __shared__ double red[4][64];
  // group g sums tasks t0 + g, t0 + g + 4, ... in that order; eight loads are issued
  // before their additions, so a long side does not wait on one load at a time
  double s = 0.0;
  if (e < esz) {
    int t = t0 + g;
    for (; t + 28 < t1; t += 32) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = zpart[(size_t)(t + 4 * u) * zs_task + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; t < t1; t += 4) s += zpart[(size_t)t * zs_task + e];
  }
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && e < esz)
    zfin[(size_t)sd * zf_side + e] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}
__global__ void __launch_bounds__(NTHREADS) k_zsum(const k_zsum_args a_) {
  k_zsum_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_zsum_g(const k_zsum_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_zsum_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_zsum_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_zsum_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_zsum_args* a, const int* st, const int* gy, int mm) {
    k_zsum_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_zsum now, or records it while a recorder is open on this thread
static void k_zsum_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_zsum_args& a) {
  if (recording())
    record_group(k_zsum_grp, group_key((const void*)k_zsum_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_zsum<<<g, b, lds, s>>>(a);
}

// sides of at most four tasks: one element per thread, summed as (z0 + z1) + (z2 + z3),
// the value k_zsum's four groups give, so that both kernels agree to the bit
// arguments of k_zsum_few (one struct, so that grouped launches can stage one per member)
struct k_zsum_few_args {
  const double* zpart;
  int zs_task;
  int tbase;
  const int* node_task_off;
  int hbase;
  int nsides;
  int esz;
  double* zfin;
  int zf_side;
};
__device__ __forceinline__ void k_zsum_few_body(const k_zsum_few_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const double* __restrict__ zpart = a_.zpart;
  int zs_task = a_.zs_task;
  int tbase = a_.tbase;
  const int* __restrict__ node_task_off = a_.node_task_off;
  int hbase = a_.hbase;
  int nsides = a_.nsides;
  int esz = a_.esz;
  double* __restrict__ zfin = a_.zfin;
  int zf_side = a_.zf_side;
  (void)by_;
  (void)gy_;

  const int sd = bx_;
  if (sd >= nsides) return;
  const int h = hbase + (sd >> 1), side = sd & 1;
  const int t0 = node_task_off[2 * h + side] - tbase, t1 = node_task_off[2 * h + side + 1] - tbase;
  const int nt = t1 - t0;
  const int e = by_ * NTHREADS + threadIdx.x;
  if (nt <= 1 || e >= esz) return;
  const double* z = zpart + (size_t)t0 * zs_task + e;
  const double a = z[0] + z[zs_task];
  double b = 0.0;
  if (nt > 2) b = z[2 * (size_t)zs_task];
  if (nt > 3) b += z[3 * (size_t)zs_task];
  zfin[(size_t)sd * zf_side + e] = a + b;
}
__global__ void __launch_bounds__(NTHREADS) k_zsum_few(const k_zsum_few_args a_) {
  k_zsum_few_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_zsum_few_g(const k_zsum_few_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_zsum_few_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_zsum_few_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_zsum_few_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_zsum_few_args* a, const int* st, const int* gy, int mm) {
    k_zsum_few_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_zsum_few now, or records it while a recorder is open on this thread
static void k_zsum_few_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_zsum_few_args& a) {
  if (recording())
    record_group(k_zsum_few_grp, group_key((const void*)k_zsum_few_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_zsum_few<<<g, b, lds, s>>>(a);
}

void launch_zsum(const double* zpart, int zs_task, int tbase, const int* node_task_off, int hbase,
                 int nsides, int esz, double* zfin, int zf_side, int max_tasks, hipStream_t s) {
  if (nsides <= 0 || esz <= 0) return;
  if (max_tasks <= 4) {
    const dim3 grid(nsides, (esz + NTHREADS - 1) / NTHREADS);
    k_zsum_few_launch(grid, dim3(NTHREADS), 0, s,
                      k_zsum_few_args{zpart, zs_task, tbase, node_task_off, hbase, nsides, esz,
                                      zfin, zf_side});
    return;
  }
  const dim3 grid(nsides, (esz + 63) / 64);
  k_zsum_launch(grid, dim3(NTHREADS), 0, s,
                k_zsum_args{zpart, zs_task, tbase, node_task_off, hbase, nsides, esz, zfin, zf_side});
}

// ---------------------------------------------------------------------------------
// symmetric Jacobi eigen-decomposition of an m x m LDS matrix (A <- diag, E <- vectors),
// for a work-group of one wave (64 lanes); lda must be even and at least m
//
// Cyclic Jacobi in the round-robin parallel order: a step rotates the disjoint index
// pairs (p_t, q_t), t < me/2, at once, and me - 1 steps make a sweep (me = m rounded up
// to even; an odd m is padded with a zero row and column, whose rotations are the
// identity).  Lane b owns the 2 x 2 block (pair t) x (pair u), b = t np + u, of A and of
// E.  It computes the rotations of both pairs itself from a_pp, a_qq and a_pq, so a step
// is one pass of reads, one of writes and one barrier.  A is double-buffered (A, T, A,
// ...), E is rotated in place (its blocks are disjoint).  Blocks t < u of A also write
// their transpose (blocks t > u write nothing), so A stays exactly symmetric; a
// diagonal block takes the classical update a_pp - t a_pq, a_qq + t a_pq, a_pq = 0.
// Converged once the off-diagonal part is at most 4 m eps of the Frobenius norm
// (checked before each sweep, at most 30 sweeps); returns false otherwise.
// ---------------------------------------------------------------------------------
struct JRot {
  double c, s, t;
};

__device__ __forceinline__ JRot jacobi_rot(double app, double aqq, double apq) {
  JRot r{1.0, 0.0, 0.0};
  if (apq != 0.0) {
    const double th = (aqq - app) / (2.0 * apq);
    const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
    r.c = 1.0 / sqrt(tt * tt + 1.0);
    r.s = tt * r.c;
    r.t = tt;
  }
  return r;
}

__device__ bool lds_sym_eig(double* A, double* E, double* T, int m, int lda) {
  const int lane = threadIdx.x & 63;
  const int me = m + (m & 1);
  for (int c = 0; c < me; ++c)
    for (int r = lane; r < me; r += 64) {
      E[r + c * lda] = (r == c) ? 1.0 : 0.0;
      if (r == m || c == m) A[r + c * lda] = 0.0;  // padding (odd m)
    }
  __syncthreads();
  if (m < 2) return true;
  const int np = me >> 1, nb = np * np;
  const int t0 = lane / np, u0 = lane - t0 * np;
  double* cur = A;
  double* nxt = T;
  bool conv = false;
  int roff = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int c = 0; c < m; ++c)
      for (int r = lane; r < m; r += 64) {
        const double v = cur[r + c * lda];
        tot += v * v;
        if (r != c) off += v * v;
      }
    off = wsum(off);
    tot = wsum(tot);
    const double lim = 4.0 * m * DBL_EPSILON;
    if (__builtin_amdgcn_readfirstlane((int)(off <= lim * lim * tot))) {
      conv = true;
      break;
    }
#pragma unroll 1
    for (int step = 0; step < me - 1; ++step) {
      int t = t0, u = u0;
#pragma unroll 1
      for (int b = lane; b < nb; b += 64) {
        int pt = rr_index(t, roff, me), qt = rr_index(me - 1 - t, roff, me);
        int pu = rr_index(u, roff, me), qu = rr_index(me - 1 - u, roff, me);
        if (pt > qt) { const int x = pt; pt = qt; qt = x; }
        if (pu > qu) { const int x = pu; pu = qu; qu = x; }
        const int cpt = __umul24(pt, lda), cqt = __umul24(qt, lda);
        const int cpu = __umul24(pu, lda), cqu = __umul24(qu, lda);
        const JRot ru = jacobi_rot(cur[pu + cpu], cur[qu + cqu], cur[pu + cqu]);
        const JRot rt = jacobi_rot(cur[pt + cpt], cur[qt + cqt], cur[pt + cqt]);
        // E <- E J on columns (pu, qu), rows pt and qt
        const double e00 = E[pt + cpu], e01 = E[pt + cqu];
        const double e10 = E[qt + cpu], e11 = E[qt + cqu];
        E[pt + cpu] = ru.c * e00 - ru.s * e01;
        E[pt + cqu] = ru.s * e00 + ru.c * e01;
        E[qt + cpu] = ru.c * e10 - ru.s * e11;
        E[qt + cqu] = ru.s * e10 + ru.c * e11;
        if (t <= u) {
          const double b00 = cur[pt + cpu], b01 = cur[pt + cqu];
          const double b10 = cur[qt + cpu], b11 = cur[qt + cqu];
          double x00, x01, x10, x11;
          if (t == u) {
            x00 = b00 - ru.t * b01;
            x11 = b11 + ru.t * b01;
            x01 = 0.0;
            x10 = 0.0;
          } else {
            // rows (pair t), then columns (pair u)
            const double y00 = rt.c * b00 - rt.s * b10, y10 = rt.s * b00 + rt.c * b10;
            const double y01 = rt.c * b01 - rt.s * b11, y11 = rt.s * b01 + rt.c * b11;
            x00 = ru.c * y00 - ru.s * y01;
            x01 = ru.s * y00 + ru.c * y01;
            x10 = ru.c * y10 - ru.s * y11;
            x11 = ru.s * y10 + ru.c * y11;
          }
          nxt[pt + cpu] = x00;
          nxt[pu + cpt] = x00;
          nxt[pt + cqu] = x01;
          nxt[qu + cpt] = x01;
          nxt[qt + cpu] = x10;
          nxt[pu + cqt] = x10;
          nxt[qt + cqu] = x11;
          nxt[qu + cqt] = x11;
        }
        u += 64;
        while (u >= np) { u -= np; ++t; }
      }
      __syncthreads();
      double* x = cur;
      cur = nxt;
      nxt = x;
      if (++roff == me - 1) roff = 0;
    }
  }
  if (cur != A) {
    for (int c = 0; c < m; ++c)
      for (int r = lane; r < m; r += 64) A[r + c * lda] = cur[r + c * lda];
    __syncthreads();
  }
  return conv;
}

// ---------------------------------------------------------------------------------
// the same eigen-decomposition for a work-group of 256 threads (lda even, >= m + 1 when m
// is odd).  Same round-robin order, rotations and convergence test as lds_sym_eig; a step
// is two phases: the owner thread of each pair computes its rotation once and publishes,
// per index i, its partner i*, the row coefficients (alpha_i, beta_i) (row i of J'A is
// alpha_i row_i + beta_i row_i*) and the signed t of the classical diagonal update; then
// thread e updates entry e of A (into T, double-buffered) as
//   (a1 a_ij + b1 a_i*j*) + (a2 a_ij* + b2 a_i*j),  products of coefficient pairs first,
// which is the same expression for (i, j) and (j, i), so A stays exactly symmetric; and
// thread (r, u) rotates row r of E's column pair u in place.
// ---------------------------------------------------------------------------------
__device__ bool lds_sym_eig256(double* A, double* E, double* T, int m, int lda) {
  __shared__ int partner[PMAX + 2], pp[PMAX / 2 + 1], pq[PMAX / 2 + 1];
  __shared__ double alp[PMAX + 2], bet[PMAX + 2], tsg[PMAX + 2];
  __shared__ double red[4][2];
  const int tid = threadIdx.x;
  const int me = m + (m & 1);
  for (int e = tid; e < me * me; e += blockDim.x) {
    const int r = e % me, c = e / me;
    E[r + c * lda] = (r == c) ? 1.0 : 0.0;
    if (r == m || c == m) A[r + c * lda] = 0.0;  // padding (odd m)
  }
  __syncthreads();
  if (m < 2) return true;
  const int np = me >> 1;
  double* cur = A;
  double* nxt = T;
  bool conv = false;
  int roff = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = e % m, c = e / m;
      const double v = cur[r + c * lda];
      tot += v * v;
      if (r != c) off += v * v;
    }
    off = wsum(off);
    tot = wsum(tot);
    if ((tid & 63) == 0) {
      red[tid >> 6][0] = off;
      red[tid >> 6][1] = tot;
    }
    __syncthreads();
    const double o = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    const double t2 = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    const double lim = 4.0 * m * DBL_EPSILON;
    if (o <= lim * lim * t2) {  // the same sums in every thread
      conv = true;
      break;
    }
#pragma unroll 1
    for (int step = 0; step < me - 1; ++step) {
      if (tid < np) {  // owner of pair tid
        int p = rr_index(tid, roff, me), q = rr_index(me - 1 - tid, roff, me);
        if (p > q) { const int x = p; p = q; q = x; }
        const JRot ro = jacobi_rot(cur[p + p * lda], cur[q + q * lda], cur[p + q * lda]);
        partner[p] = q;
        partner[q] = p;
        alp[p] = ro.c;
        alp[q] = ro.c;
        bet[p] = -ro.s;
        bet[q] = ro.s;
        tsg[p] = -ro.t;
        tsg[q] = ro.t;
        pp[tid] = p;
        pq[tid] = q;
      }
      __syncthreads();
      for (int e = tid; e < me * me; e += blockDim.x) {
        const int i = e % me, j = e / me;
        const int is = partner[i], js = partner[j];
        double x;
        if (i == j) {
          x = cur[i + i * lda] + tsg[i] * cur[i + is * lda];
        } else if (is == j) {
          x = 0.0;
        } else {
          const double ai = alp[i], bi = bet[i], aj = alp[j], bj = bet[j];
          const double w1 = __dmul_rn(__dmul_rn(ai, aj), cur[i + j * lda]);
          const double w4 = __dmul_rn(__dmul_rn(bi, bj), cur[is + js * lda]);
          const double w2 = __dmul_rn(__dmul_rn(ai, bj), cur[i + js * lda]);
          const double w3 = __dmul_rn(__dmul_rn(bi, aj), cur[is + j * lda]);
          x = __dadd_rn(__dadd_rn(w1, w4), __dadd_rn(w2, w3));
        }
        nxt[i + j * lda] = x;
      }
      for (int e = tid; e < me * np; e += blockDim.x) {
        const int r = e % me, u = e / me;
        const int p = pp[u], q = pq[u];
        const double c = alp[p], sn = -bet[p];
        const double ep = E[r + p * lda], eq = E[r + q * lda];
        E[r + p * lda] = c * ep - sn * eq;
        E[r + q * lda] = sn * ep + c * eq;
      }
      __syncthreads();
      double* x = cur;
      cur = nxt;
      nxt = x;
      if (++roff == me - 1) roff = 0;
    }
  }
  if (cur != A) {
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = e % m, c = e / m;
      A[r + c * lda] = cur[r + c * lda];
    }
    __syncthreads();
  }
  return conv;
}

// ---------------------------------------------------------------------------------
// pivoted Cholesky of an m x m LDS Gram matrix G (symmetric positive semi-definite) by
// one wave: Pi' G Pi = L L' with diagonal pivoting (largest remaining diagonal, first
// index on ties), stopped at the first pivot at or below 64 m (u/2) max_i G_ii (Higham's
// floor for semidefinite Cholesky).  Writes the square root S = L' Pi' (r x m, so that
// S'S = G up to the dropped tail) into S (leading dimension lda) and returns the rank r,
// or -1 if the diagonal of G holds a NaN.  G is overwritten.
// ---------------------------------------------------------------------------------
__device__ int wave_pchol(double* G, int m, int lda, double* S, int* perm) {
  const int lane = threadIdx.x & 63;
  // in a work-group of several waves every wave takes the same decisions from the same
  // reads, and wave 0 alone writes.  Every read of G that feeds a decision is separated
  // from wave 0's next write by a barrier: a wave that falls behind (waves of one
  // work-group drift apart when other kernels share the compute unit) must not see a
  // half-swapped diagonal, or it would choose another pivot or rank than wave 0 and the
  // barriers of the two would no longer pair up.
  const bool w0 = threadIdx.x < 64;
  const double d0 = lane < m ? G[lane + lane * lda] : 0.0;
  if (__ballot(d0 != d0) != 0) return -1;
  double dmax = d0;
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  const double dfloor = 64.0 * m * (DBL_EPSILON * 0.5) * dmax;
  if (w0 && lane < m) perm[lane] = lane;
  __syncthreads();
  int r = m;
  for (int j = 0; j < m; ++j) {
    double v = (lane >= j && lane < m) ? G[lane + lane * lda] : -DBL_MAX;
    int iv = lane;
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(v, o, 64);
      const int i2 = __shfl_xor(iv, o, 64);
      if (v2 > v || (v2 == v && i2 < iv)) {
        v = v2;
        iv = i2;
      }
    }
    // every lane holds the same (v, iv): the butterfly's comparisons are symmetric.  All
    // waves have read the diagonal before wave 0 swaps rows and columns.
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane((int)!(v > dfloor))) {
      r = j;
      break;
    }
    const int piv = __builtin_amdgcn_readfirstlane(iv);
    if (piv != j) {  // symmetric interchange of rows and columns j and piv
      if (w0 && lane < m) {
        const double t = G[j + lane * lda];
        G[j + lane * lda] = G[piv + lane * lda];
        G[piv + lane * lda] = t;
      }
      __syncthreads();
      if (w0 && lane < m) {
        const double t = G[lane + j * lda];
        G[lane + j * lda] = G[lane + piv * lda];
        G[lane + piv * lda] = t;
      }
      if (threadIdx.x == 0) {
        const int t = perm[j];
        perm[j] = perm[piv];
        perm[piv] = t;
      }
      __syncthreads();
    }
    // (only wave 0 uses the pivot's root; the other waves do not read G here)
    const double ljj = w0 ? sqrt(G[j + j * lda]) : 1.0;
    double lij = 0.0;
    if (w0 && lane > j && lane < m) {
      lij = G[lane + j * lda] / ljj;
      G[lane + j * lda] = lij;
    }
    if (w0 && lane == j) G[j + j * lda] = ljj;
    __syncthreads();
    if (w0 && lane > j && lane < m)
      for (int c = j + 1; c < m; ++c) G[lane + c * lda] -= lij * G[c + j * lda];
    __syncthreads();
  }
  // S[b][perm[a]] = L[a][b] for b <= a, b < r
  if (w0)
    for (int a = lane; a < m; a += 64)
      for (int b = 0; b < r; ++b) S[b + perm[a] * lda] = (b <= a) ? G[a + b * lda] : 0.0;
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------------
// node factor of one level (factorization): Gram blocks -> (G_V, F1, F2), log-det
// and the update coefficients of the coarser panels
// ---------------------------------------------------------------------------------
// arguments of k_node_factor (one struct, so that grouped launches can stage one per member)
struct k_node_factor_args {
  int l;
  const int* rank;
  const int* kmax;
  const int* rcount;
  const int* node_task_off;
  int tbase;
  double* zpart;
  int zs_a;
  int zs_task;
  double* zfin;
  int zf_side;
  double* nodemat;
  const int* nodemat_off;
  double* node_ld;
  double* coef;
  int cs_node;
  int cs_a;
  int* status;
  int kc;
};
__device__ __forceinline__ void k_node_factor_body(const k_node_factor_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int l = a_.l;
  const int* __restrict__ rank = a_.rank;
  const int* __restrict__ kmax = a_.kmax;
  const int* __restrict__ rcount = a_.rcount;
  const int* __restrict__ node_task_off = a_.node_task_off;
  int tbase = a_.tbase;
  double* __restrict__ zpart = a_.zpart;
  int zs_a = a_.zs_a;
  int zs_task = a_.zs_task;
  double* __restrict__ zfin = a_.zfin;
  int zf_side = a_.zf_side;
  double* __restrict__ nodemat = a_.nodemat;
  const int* __restrict__ nodemat_off = a_.nodemat_off;
  double* __restrict__ node_ld = a_.node_ld;
  double* __restrict__ coef = a_.coef;
  int cs_node = a_.cs_node;
  int cs_a = a_.cs_a;
  int* __restrict__ status = a_.status;
  int kc = a_.kc;
  (void)by_;
  (void)gy_;

  const int j = bx_;
  const int h = (1 << l) - 1 + j;
  const int k = rank[h], kl = kmax[l], W = rcount[l], Wc = W - kl;
  if (k == 0) {
    if (threadIdx.x == 0) node_ld[h] = 0.0;
    return;
  }
  // final Gram blocks Z_side[a][b] = Z[a * zs_a + b]: summed by k_zsum, or the side's
  // only task partial (ZJ is overwritten below, in either place)
  const int tI = node_task_off[2 * h] - tbase, tJ = node_task_off[2 * h + 1] - tbase;
  const int tE = node_task_off[2 * h + 2] - tbase;
  double* ZI = (tJ - tI == 1) ? zpart + (size_t)tI * zs_task : zfin + (size_t)j * 2 * zf_side;
  double* ZJ = (tE - tJ == 1) ? zpart + (size_t)tJ * zs_task : zfin + (size_t)(2 * j + 1) * zf_side;
  const int zW = zs_a;
  extern __shared__ double lds[];
  double* GU = lds;
  double* GV = GU + kc * kc;
  double* E = GV + kc * kc;
  double* Hm = E + kc * kc;
  double* X = Hm + kc * kc;
  __shared__ double g1[PMAX], g2[PMAX];
  __shared__ int perm[PMAX];
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int a = idx % k, b = idx / k;
    GU[a + b * kc] = 0.5 * (ZI[(size_t)a * zW + b] + ZI[(size_t)b * zW + a]);
    GV[a + b * kc] = 0.5 * (ZJ[(size_t)a * zW + b] + ZJ[(size_t)b * zW + a]);
  }
  __syncthreads();
  // S_U (r x k, S_U' S_U = G_U) by pivoted Cholesky; the node's outputs do not depend
  // on which square root of G_U is used
  const int rc = wave_pchol(GU, k, kc, X, perm);
  const int r = rc < 0 ? 0 : rc;
  // E <- S_U G_V (r x k) ; Hm <- E S_U' (r x r)
  for (int idx = threadIdx.x; idx < r * k; idx += blockDim.x) {
    const int a = idx % r, b = idx / r;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += X[a + c * kc] * GV[c + b * kc];
    E[a + b * kc] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int a = idx % r, b = idx / r;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += E[a + c * kc] * X[b + c * kc];
    Hm[a + b * kc] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {  // symmetrise
    const int a = idx % r, b = idx / r;
    if (a < b) {
      const double v = 0.5 * (Hm[a + b * kc] + Hm[b + a * kc]);
      Hm[a + b * kc] = v;
      Hm[b + a * kc] = v;
    }
  }
  __syncthreads();
  // GU is free until B; levels of larger rank run 4 waves per node
  const bool ok = blockDim.x >= 256 ? lds_sym_eig256(Hm, E, GU, r, kc)
                                    : lds_sym_eig(Hm, E, GU, r, kc);
  {
    // lane a: the coefficients of s_a^2 and its log(1 - s_a^2)
    double lg = 0.0;
    bool spd = true;
    for (int a = threadIdx.x; a < r; a += 64) {
      double s2 = fmax(Hm[a + a * kc], 0.0);
      if (!(s2 < 1.0)) {
        spd = false;
        s2 = 1.0 - DBL_EPSILON;
      }
      const double d = sqrt(1.0 - s2);
      g1[a] = -1.0 / (1.0 + d);
      g2[a] = 1.0 / (d * (1.0 + d));
      lg += log1p(-s2);
    }
    lg = wsum(lg);
    const bool notspd = __ballot(!spd) != 0 || rc < 0;
    if (threadIdx.x == 0) {
      node_ld[h] = lg;
      if (notspd) atomicOr(status, ST_NOTSPD);
      if (!ok) atomicOr(status, ST_NOTCONV);
    }
  }
  __syncthreads();
  // B = S_U' P (k x r) -> GU
  for (int idx = threadIdx.x; idx < k * r; idx += blockDim.x) {
    const int a = idx % k, b = idx / k;
    double acc = 0.0;
    for (int c = 0; c < r; ++c) acc += X[c + a * kc] * E[c + b * kc];
    GU[a + b * kc] = acc;
  }
  __syncthreads();
  // F1 -> Hm, F2 -> E ; store G_V, F1, F2
  double* out = nodemat + nodemat_off[h];
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int a = idx % k, b = idx / k;
    double f1 = 0.0, f2 = 0.0;
    for (int c = 0; c < r; ++c) {
      const double pr = GU[a + c * kc] * GU[b + c * kc];
      f1 += pr * g1[c];
      f2 += pr * g2[c];
    }
    out[a + b * k] = GV[a + b * kc];
    out[k * k + a + b * k] = f1;
    out[2 * k * k + a + b * k] = f2;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int a = idx % k, b = idx / k;
    E[a + b * kc] = out[2 * k * k + a + b * k];
  }
  __syncthreads();
  // coefficients of the coarser panels: U = T - G_V S (into ZJ), A = -S + F2 U
  for (int idx = threadIdx.x; idx < k * Wc; idx += blockDim.x) {
    const int a = idx / Wc, b = kl + idx % Wc;
    double acc = ZJ[(size_t)a * zW + b];
    for (int d = 0; d < k; ++d) acc -= GV[a + d * kc] * ZI[(size_t)d * zW + b];
    ZJ[(size_t)a * zW + b] = acc;
  }
  __syncthreads();
  double* cf = coef + (size_t)j * cs_node;
  for (int idx = threadIdx.x; idx < k * Wc; idx += blockDim.x) {
    const int a = idx / Wc, bc = idx % Wc, b = kl + bc;
    double acc = -ZI[(size_t)a * zW + b];
    for (int c = 0; c < k; ++c) acc += E[a + c * kc] * ZJ[(size_t)c * zW + b];
    cf[(size_t)a * cs_a + bc] = acc;
  }
}
__global__ void __launch_bounds__(256) k_node_factor(const k_node_factor_args a_) {
  k_node_factor_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(256) k_node_factor_g(const k_node_factor_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_node_factor_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_node_factor_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_node_factor_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_node_factor_args* a, const int* st, const int* gy, int mm) {
    k_node_factor_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_node_factor now, or records it while a recorder is open on this thread
static void k_node_factor_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_node_factor_args& a) {
  if (recording())
    record_group(k_node_factor_grp, group_key((const void*)k_node_factor_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_node_factor<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// level update (factorization): coarser columns of right-child rows += V~ A
// On FP64 matrix cores with the output transposed: for one 16-row tile and 16 coarser
// columns, Y^T (16 x 16) += A^T (16 x k) V^T (k x 16), in steps of v_mfma_f64_16x16x4f64
// (4 ranks each).  In the row-tiled panel layout every operand a wave reads or writes is
// one 512-byte run (4 ranks x 16 rows of V) or four 128-byte runs (one coarser column
// each), so no entry is touched by more than one lane and the VALU only forms addresses.
// A work-group stages A for up to 16 QB coarser columns in LDS in operand order, and a
// wave updates all of them on a tile in one visit, reading that tile's V once.  Wider
// levels take further work-groups along grid.y, and gy work-groups share one level task
// so that the grid fills the chip.
// ---------------------------------------------------------------------------------
// arguments of k_update_panel (one struct, so that grouped launches can stage one per member)
struct k_update_panel_args {
  const Task* tasks;
  int tbase;
  int ntask;
  int l;
  const int* rank;
  const int* coff;
  const int* kmax;
  const int* rcols;
  const int* rcount;
  int K;
  double* P;
  const double* coef;
  int cs_node;
  int cs_a;
  int gy;  // work-groups per level task and column chunk
};
// This wave's row tiles of one task for one staged chunk of bw <= 16 NQ coarser columns.
// SM: MFMA steps held in registers (4 ranks each; the host picks SM >= ceil(kcap / 4));
// ranks past 4 S read as zero.  Every load of a tile is issued before any of its stores:
// the memory counter that a wave waits on is in order over loads and stores, so a load
// issued behind a store would also wait for that store.
template <int SM, int QB, int NQ>
__device__ __forceinline__ void update_tiles(const double* __restrict__ Acf,
                                             const int* __restrict__ ycol, double* __restrict__ P,
                                             int K, int c0, int k, int S, int bw, int r0, int r1,
                                             int tfirst, int tend, int tstep) {
  const int lane = threadIdx.x & 63, kg = lane >> 4, jr = lane & 15;
  // ycol holds, at [16 q + 4 kg + v], the column of accumulator register v of block q for
  // lane group kg; it is read per tile, four at a time, rather than held in registers
  const uint4* yq = reinterpret_cast<const uint4*>(ycol);
#pragma unroll 1
  for (int tt = tfirst; tt < tend; tt += tstep) {
    const int row = tt * 16 + jr;
    const bool ok = row >= r0 && row < r1;
    // whole row tiles lie inside the panel (its leading dimension is a multiple of 64), so
    // every load is in bounds; entries that are not ours are read and discarded.  The tile
    // base is wave-uniform and in the global address space (a pointer read from a grouped
    // launch's member array would otherwise be accessed as flat).
    gchar* tp = (gchar*)(P + (size_t)tt * K * 16);
    // B operands: ranks 4s + kg of row jr; ranks >= k and rows outside the task give 0
    double vb[SM];
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      const bool va = s < S && ok && 4 * s + kg < k;
      const unsigned o = va ? (unsigned)((c0 + 4 * s) * 16 + lane) : (unsigned)(c0 * 16 + jr);
      vb[s] = *(const gdouble*)(tp + o * 8u);
    }
    // accumulators: register v of block q holds coarser column 16 q + row(kg, v), row jr;
    // byte offsets within the tile are below 2^32 (K * 128 bytes per tile).  The table index
    // is made opaque per tile so that its reads stay in the loop (an index, not a pointer,
    // so that they stay LDS reads).
    int yi = kg;
    asm volatile("" : "+v"(yi));
    d4 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const uint4 c = yq[yi + 4 * q];
      const unsigned cv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[q][v] = *(const gdouble*)(tp + (cv[v] * 16u + (unsigned)jr) * 8u);
    }
#pragma unroll
    for (int s = 0; s < SM; ++s) vb[s] = (s < S && ok && 4 * s + kg < k) ? vb[s] : 0.0;
    // the A operands are read from LDS per tile (an opaque base keeps the compiler from
    // holding all of them in registers across tiles)
    unsigned ab = (unsigned)lane * 8u;
    asm volatile("" : "+v"(ab));
    const char* Ab = reinterpret_cast<const char*>(Acf) + ab;
    // all SM steps run (steps past the rank multiply zeros): a branch here would sink the
    // loads of V into it and serialise their latencies
#pragma unroll
    for (int s = 0; s < SM; ++s)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        acc[q] = Mfma<double>::step(*reinterpret_cast<const double*>(Ab + ((s * QB + q) * 64) * 8),
                                    vb[s], acc[q]);
    // the offsets are read again for the stores rather than kept live across the steps
    int ys = kg;
    asm volatile("" : "+v"(ys));
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const uint4 c = yq[ys + 4 * q];
      const unsigned cv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * q + Mfma<double>::row(kg, v);
        if (ok && i < bw) *(gdouble*)(tp + (cv[v] * 16u + (unsigned)jr) * 8u) = acc[q][v];
      }
    }
  }
}
// QB: 16-column blocks staged per work-group (8 when the A operands fit in 32 KB of LDS)
template <int SM, int QB>
__device__ __forceinline__ void k_update_panel_body(const k_update_panel_args& a_, const int bx_,
                                                    const int by_, const int gy_) {
  static_assert(QB == 4 || QB == 8, "chunks of 64 or 128 columns");
  const Task* __restrict__ tasks = a_.tasks;
  const int K = a_.K;
  const int l = a_.l;
  const int t = bx_;
  (void)gy_;
  if (t >= a_.ntask) return;
  // every scalar below is block-uniform; readfirstlane says so to the compiler (a grouped
  // launch reads them through pointers it cannot see as uniform), so that the tile walk and
  // the tile base stay in scalar registers
  Task tk = tasks[a_.tbase + t];
  tk.h = __builtin_amdgcn_readfirstlane(tk.h);
  tk.side = __builtin_amdgcn_readfirstlane(tk.side);
  tk.r0 = __builtin_amdgcn_readfirstlane(tk.r0);
  tk.r1 = __builtin_amdgcn_readfirstlane(tk.r1);
  if (tk.side == 0) return;
  const int k = __builtin_amdgcn_readfirstlane(a_.rank[tk.h]);
  const int kl = __builtin_amdgcn_readfirstlane(a_.kmax[l]);
  const int Wc = __builtin_amdgcn_readfirstlane(a_.rcount[l]) - kl;
  if (k == 0 || Wc <= 0) return;
  const int S = min((k + 3) >> 2, SM);  // MFMA steps (ranks never exceed the level's cap)
  const int c0 = __builtin_amdgcn_readfirstlane(a_.coff[l]);
  const int j = tk.h - ((1 << l) - 1);
  const int* yc = a_.rcols + (size_t)l * K + kl;
  const double* cf = a_.coef + (size_t)j * a_.cs_node;
  const int cs_a = a_.cs_a;
  constexpr int NW = NTHREADS / 64;
  constexpr int CW = 16 * QB;  // columns per chunk
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform tile walk
  const int T0 = tk.r0 >> 4, T1 = (tk.r1 + 15) >> 4;
  // grid.y = gy x (column chunks): this work-group takes one chunk and every gy-th group of
  // NW tiles of the task, so it stages its A operands once
  const int gy = a_.gy;
  const int chunk = by_ / gy, sub = by_ - chunk * gy;
  const int bt = chunk * CW;
  if (bt >= Wc) return;
  const int bw = min(CW, Wc - bt);
  __shared__ double Acf[SM][QB][64];  // step s, column block q: lane-ordered A operand
  __shared__ __align__(16) int ycol[CW];
  {
    // zeros past step S; each thread's NST loads are issued together (an entry outside
    // reads entry 0 and is replaced by zero)
    constexpr int NST = SM * QB * 64 / NTHREADS;
    static_assert(NST * NTHREADS == SM * QB * 64, "whole staging trips");
    double st[NST];
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int idx = threadIdx.x + u * NTHREADS;
      const int s = idx / (QB * 64), q = (idx >> 6) % QB, ln = idx & 63;
      const int a = 4 * s + (ln >> 4), b = 16 * q + (ln & 15);
      st[u] = cf[(a < k && b < bw) ? (size_t)a * cs_a + bt + b : 0];
    }
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int idx = threadIdx.x + u * NTHREADS;
      const int s = idx / (QB * 64), q = (idx >> 6) % QB, ln = idx & 63;
      const int a = 4 * s + (ln >> 4), b = 16 * q + (ln & 15);
      Acf[s][q][ln] = (a < k && b < bw) ? st[u] : 0.0;
    }
  }
  // column table in accumulator order, entry (q, kg, v) = column 16 q + row(kg, v) of the
  // chunk; a column past the chunk is the first column of V, which this kernel never writes
  // (it is read and masked at the store)
  if (threadIdx.x < CW) {
    const int q = threadIdx.x >> 4, g = (threadIdx.x >> 2) & 3, v = threadIdx.x & 3;
    const int i = 16 * q + Mfma<double>::row(g, v);
    ycol[threadIdx.x] = i < bw ? yc[bt + i] : c0;
  }
  __syncthreads();
  const int t0 = T0 + sub * NW + wv, ts = gy * NW;
  const double* A = &Acf[0][0][0];
#define FG_UPD_TILES(NQ) \
  update_tiles<SM, QB, NQ>(A, ycol, a_.P, K, c0, k, S, bw, tk.r0, tk.r1, t0, T1, ts)
  switch ((bw + 15) >> 4) {
    case 1: FG_UPD_TILES(1); break;
    case 2: FG_UPD_TILES(2); break;
    case 3: FG_UPD_TILES(3); break;
    case 4: FG_UPD_TILES(4); break;
    case 5: if constexpr (QB == 8) FG_UPD_TILES(5); break;
    case 6: if constexpr (QB == 8) FG_UPD_TILES(6); break;
    case 7: if constexpr (QB == 8) FG_UPD_TILES(7); break;
    default: if constexpr (QB == 8) FG_UPD_TILES(8); break;
  }
#undef FG_UPD_TILES
}
template <int SM, int QB>
__global__ void __launch_bounds__(NTHREADS) k_update_panel(const k_update_panel_args a_) {
  k_update_panel_body<SM, QB>(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
template <int SM, int QB>
__global__ void __launch_bounds__(NTHREADS) k_update_panel_g(const k_update_panel_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_update_panel_body<SM, QB>(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
template <int SM, int QB>
static void k_update_panel_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_update_panel_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_update_panel_args* a, const int* st, const int* gy, int mm) {
    k_update_panel_g<SM, QB><<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_update_panel now, or records it while a recorder is open on this thread
template <int SM, int QB>
static void k_update_panel_launch1(int ntask, int wcap, hipStream_t s, k_update_panel_args a) {
  const dim3 g(ntask, a.gy * std::max(1, (wcap + 16 * QB - 1) / (16 * QB))), b(NTHREADS);
  if (recording())
    record_group(k_update_panel_grp<SM, QB>, group_key((const void*)k_update_panel_grp<SM, QB>, b, 0),
                 g, b, 0, &a, sizeof(a));
  else
    k_update_panel<SM, QB><<<g, b, 0, s>>>(a);
}
// The variant whose registers hold ceil(kcap / 4) steps, with 128-column chunks while their
// A operands fit in 32 KB of LDS; wcap bounds the coarser columns and trows the rows of a
// task.  One work-group per task while a task has at most 32 row tiles, two above.
static void k_update_panel_launch(int kcap, int wcap, int trows, int ntask, hipStream_t s,
                                  k_update_panel_args a) {
  a.gy = trows / 16 > 32 ? 2 : 1;
  const int sm = (std::max(kcap, 1) + 3) / 4;
  if (sm <= 4)
    k_update_panel_launch1<4, 8>(ntask, wcap, s, a);
  else if (sm <= 8)
    k_update_panel_launch1<8, 8>(ntask, wcap, s, a);
  else if (sm <= 12)
    k_update_panel_launch1<12, 4>(ntask, wcap, s, a);
  else
    k_update_panel_launch1<16, 4>(ntask, wcap, s, a);
}

// ---------------------------------------------------------------------------------
// log-det: sum of leaf and node parts in a fixed order
// ---------------------------------------------------------------------------------
// s += v[i] for i = tid, tid + NTHREADS, ... < n, in that order, with 8 loads in flight
__device__ __forceinline__ double strided_sum(const double* __restrict__ v, int n, double s) {
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * NTHREADS) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NTHREADS;
      x[u] = i < n ? v[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * NTHREADS < n) s += x[u];
  }
  return s;
}
// arguments of k_logdet_sum (one struct, so that grouped launches can stage one per member)
struct k_logdet_sum_args {
  const double* leaf_ld;
  int nleaf;
  const double* node_ld;
  int nint;
  double* out;
};
__device__ __forceinline__ void k_logdet_sum_body(const k_logdet_sum_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const double* __restrict__ leaf_ld = a_.leaf_ld;
  int nleaf = a_.nleaf;
  const double* __restrict__ node_ld = a_.node_ld;
  int nint = a_.nint;
  double* __restrict__ out = a_.out;
  (void)by_;
  (void)gy_;

  __shared__ double red[NTHREADS / 64];
  double s = strided_sum(leaf_ld, nleaf, 0.0);
  s = strided_sum(node_ld, nint, s);
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) t += red[w];
    *out = t;
  }
}
__global__ void  k_logdet_sum(const k_logdet_sum_args a_) {
  k_logdet_sum_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_logdet_sum_g(const k_logdet_sum_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_logdet_sum_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_logdet_sum_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_logdet_sum_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_logdet_sum_args* a, const int* st, const int* gy, int mm) {
    k_logdet_sum_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_logdet_sum now, or records it while a recorder is open on this thread
static void k_logdet_sum_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_logdet_sum_args& a) {
  if (recording())
    record_group(k_logdet_sum_grp, group_key((const void*)k_logdet_sum_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_logdet_sum<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
// the leaves (Cholesky, diagonal-block inverses, leaf log-dets): they need x and the
// kernel's parameters only, not the compressed panels
template <typename T>
static void factor_leaves(FactorData& F, T* leafL, T* leafLinv, const double* alpha_dev,
                          const double* beta_dev, const double* diag, hipStream_t s) {
  const HodlrData& H = *F.H;
  const HostPlan& P = H.pk->P;
  const DevPlan& D = H.pk->D;
  timer_before(KID_LEAF, s, -1, P, nullptr, 0);  // the leaf bytes do not depend on the ranks
  k_leaf_launch<T>(dim3(P.nleaf), dim3(NTHREADS), 0, s,
                   k_leaf_args<T>{D.leaf_lo, P.nleaf, H.x, P.kind, P.ell, P.nugget, F.alpha,
                                  alpha_dev, F.beta, beta_dev, diag, P.B, leafL, leafLinv,
                                  F.leaf_ld, F.status});
  timer_after(KID_LEAF, s);
}

// everything after the leaves: whitened panels, the levels, the log-det.  The panels,
// Gram blocks, node factors and updates are FP64 whatever the precision of the leaf
// factor: the node gaps 1 - s^2 of a well-conditioned-at-the-leaves matrix can sit far
// below FP32 resolution at the top levels (about 1 / (alpha n ell) for the squared
// exponential), and only the leaf factor can be rounded without changing them by more
// than a relative u32 kappa(leaf).
static void factor_levels(FactorData& F, const double* alpha_dev, hipStream_t s) {
  const HodlrData& H = *F.H;
  const HostPlan& P = H.pk->P;
  const DevPlan& D = H.pk->D;
  const int Bc = P.B;
  double* panel = F.panel;
  if (P.L > 0) {
    timer_before(KID_WHITEN, s, -1, P, H.kmax, 0);
    if (F.fp32)
      k_whiten_launch<double, float>(
          dim3(P.nleaf), dim3(NTHREADS), 0, s,
          k_whiten_args<double, float>{D.leaf_lo, P.nleaf, F.leafLf, F.leafLinvf, Bc, F.alpha,
                                       alpha_dev, H.panel, panel, P.Ktot, D.coff, H.kmax, P.L});
    else
      k_whiten_launch<double, double>(
          dim3(P.nleaf), dim3(NTHREADS), 0, s,
          k_whiten_args<double, double>{D.leaf_lo, P.nleaf, F.leafL, F.leafLinv, Bc, F.alpha,
                                        alpha_dev, H.panel, panel, P.Ktot, D.coff, H.kmax, P.L});
    timer_after(KID_WHITEN, s);
  }
  // raised once to the largest size any plan can ask for (thread-safe one-time init)
  static const bool lds_set = [] {
    (void)hipFuncSetAttribute((const void*)k_node_factor,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(sizeof(double) * 5 * PMAX * PMAX));
    (void)hipFuncSetAttribute((const void*)k_node_factor_g,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(sizeof(double) * 5 * PMAX * PMAX));
    return true;
  }();
  (void)lds_set;
  for (int l = P.L - 1; l >= 0; --l) {
    const int tb = P.ltask_off[l], nt = P.ltask_off[l + 1] - tb;
    const int Wcap = P.coff[l + 1];  // columns of levels <= l (capacity)
    const int zs_a = Wcap, zs_task = P.kcap[l] * Wcap;
    timer_before(KID_REDUCE, s, l, P, H.kmax, nt);
    const dim3 grid_r(nt, (Wcap + 63) / 64);
    const int na_cap = std::max(1, std::min(4, (P.kcap[l] + 15) / 16));
#define FG_REDUCE_PANEL(NA_)                                                                 \
  k_reduce_panel_launch<double, NA_>(                                                        \
      grid_r, dim3(NTHREADS), 0, s,                                                          \
      k_reduce_panel_args<double, NA_>{D.ltasks, tb, nt, l, D.coff, H.kmax, H.rcols, H.rcount, \
                                       P.Ktot, panel, F.zpart, zs_a, zs_task})
    switch (na_cap) {
      case 1: FG_REDUCE_PANEL(1); break;
      case 2: FG_REDUCE_PANEL(2); break;
      case 3: FG_REDUCE_PANEL(3); break;
      default: FG_REDUCE_PANEL(4); break;
    }
#undef FG_REDUCE_PANEL
    timer_after(KID_REDUCE, s);
    const int cs_node = P.kcap[l] * Wcap, cs_a = Wcap;
    if (P.max_tps[l] > 1)
      launch_zsum(F.zpart, zs_task, tb, D.node_task_off, (1 << l) - 1, 2 << l, zs_task, F.zfin,
                  zs_task, P.max_tps[l], s);
    const int kc = std::max(P.kcap[l], 1) + (std::max(P.kcap[l], 1) & 1);  // even pitch
    const size_t lds_node = sizeof(double) * 5 * (size_t)kc * kc;
    k_node_factor_launch(dim3(1 << l), dim3(kc > 8 ? 256 : 64), (uint32_t)lds_node, s, k_node_factor_args{
        l, H.rank, H.kmax, H.rcount, D.node_task_off, tb, F.zpart, zs_a, zs_task, F.zfin,
        P.kcap[l] * Wcap, F.nodemat, D.nodemat_off, F.node_ld, F.coef, cs_node, cs_a, F.status,
        kc});
    if (l > 0) {
      timer_before(KID_UPDATE, s, l, P, H.kmax, nt);
      k_update_panel_launch(P.kcap[l], P.coff[l], P.max_trows[l], nt, s,
                            k_update_panel_args{D.ltasks, tb, nt, l, H.rank, D.coff, H.kmax, H.rcols,
                                                H.rcount, P.Ktot, panel, F.coef, cs_node, cs_a, 1});
      timer_after(KID_UPDATE, s);
    }
  }
  launch_logdet_sum(F, s);
}

void launch_factor_leaves(FactorData& F, const double* alpha_dev, const double* beta_dev,
                          const double* diag, hipStream_t s) {
  if (F.fp32)
    factor_leaves<float>(F, F.leafLf, F.leafLinvf, alpha_dev, beta_dev, diag, s);
  else
    factor_leaves<double>(F, F.leafL, F.leafLinv, alpha_dev, beta_dev, diag, s);
}

void launch_factor_levels(FactorData& F, const double* alpha_dev, hipStream_t s) {
  factor_levels(F, alpha_dev, s);
}

void launch_factor(FactorData& F, const double* alpha_dev, const double* beta_dev,
                   const double* diag, hipStream_t s) {
  launch_factor_leaves(F, alpha_dev, beta_dev, diag, s);
  launch_factor_levels(F, alpha_dev, s);
}

// the two parts of the log-det separately: out[0] = sum of the leaf terms
// (2 sum log diag L_D), out[1] = sum of the node terms (sum log(1 - s^2)), each in the
// fixed order of k_logdet_sum
__global__ void k_logdet_parts(const double* __restrict__ leaf_ld, int nleaf,
                               const double* __restrict__ node_ld, int nint,
                               double* __restrict__ out) {
  __shared__ double red[2][NTHREADS / 64];
  double a = strided_sum(leaf_ld, nleaf, 0.0), b = strided_sum(node_ld, nint, 0.0);
  a = wsum(a);
  b = wsum(b);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) {
      ta += red[0][w];
      tb += red[1][w];
    }
    out[0] = ta;
    out[1] = tb;
  }
}

void launch_logdet_parts(const FactorData& F, double* out, hipStream_t s) {
  const HostPlan& P = F.H->pk->P;
  k_logdet_parts<<<1, NTHREADS, 0, s>>>(F.leaf_ld, P.nleaf, F.node_ld, P.nint, out);
}

void launch_logdet_sum(FactorData& F, hipStream_t s) {
  const HostPlan& P = F.H->pk->P;
  k_logdet_sum_launch(dim3(1), dim3(NTHREADS), 0, s,
                      k_logdet_sum_args{F.leaf_ld, P.nleaf, F.node_ld, P.nint, F.logdet});
}

}  // namespace fg
