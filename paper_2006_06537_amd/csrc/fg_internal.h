// Internal declarations of libfifagp (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fifa_gp.h"

namespace fg {

constexpr int PMAX = 60;          // interpolation nodes per side (and rank cap)
constexpr int BMAX = 128;         // maximum leaf size
constexpr int NTHREADS = 256;     // work-group size of every kernel
constexpr int RCH = 1024;         // rows per level-task (reduce / update)
constexpr int MCH = 4096;         // rows per panel-generation task
constexpr int MCHM = 1024;        // rows per moment task (one wave)
constexpr double KAPPA_H = 1.086435;  // Cramer: |H_n(x)| e^{-x^2/2} <= KAPPA_H 2^{n/2} sqrt(n!)

// kernels selectable for live timing (same values as FG_KID_* in fifa_gp.h)
constexpr int KID_LEAF = 1;
constexpr int KID_REDUCE = 2;
constexpr int KID_UPDATE = 3;
constexpr int KID_WHITEN = 4;
constexpr int KID_PREDICT = 5;

// status bits written by kernels (device word, OR-ed)
constexpr int ST_NOTSPD = 1;
constexpr int ST_NOTCONV = 2;
constexpr int ST_TOL = 4;

// k_1(a, b) without the nugget (Section 2.1; rho = 1 / (2 ell^2) for the squared
// exponential): squared exponential, exponential, Matern-3/2, Matern-5/2.
__device__ __forceinline__ double k1_value(int kind, double ell, double a, double b) {
  const double d = a - b;
  if (kind == FG_KERNEL_SE) return exp(-(d * d) / (2.0 * ell * ell));
  if (kind == FG_KERNEL_EXP) return exp(-fabs(d) / ell);
  if (kind == FG_KERNEL_MATERN32) {
    const double u = 1.7320508075688772 * fabs(d) / ell;  // sqrt(3)
    return (1.0 + u) * exp(-u);
  }
  const double u = 2.23606797749979 * fabs(d) / ell;      // sqrt(5), Matern-5/2
  return (1.0 + u + u * u / 3.0) * exp(-u);
}

// Panels are stored in 16-row tiles: rows of a tile are contiguous (128 bytes per
// column), then the K columns of that tile, then the next tile.  A 16-row segment of
// one column is a single cache line and the columns of a tile are adjacent.
// index at position j (0 <= j < me, me even) of the round-robin pairing schedule of the
// parallel Jacobi methods after `off` < me - 1 steps: position 0 stays, positions 1..me-1
// rotate; the pairs of a step are positions (t, me - 1 - t)
__device__ __forceinline__ int rr_index(int j, int off, int me) {
  if (j == 0) return 0;
  int v = j - 1 + off;
  if (v >= me - 1) v -= me - 1;
  return 1 + v;
}

__host__ __device__ __forceinline__ size_t pix(int r, int c, int K) {
  return ((size_t)(r >> 4) * (size_t)K + (size_t)c) * 16 + (size_t)(r & 15);
}

// One internal tree node: rows [lo, hi) split at mid; window rows [i0, mid) of the
// left child and [mid, j1) of the right child carry the off-diagonal block.
struct NodePlan {
  int lo, mid, hi;
  int i0, j1;
  int pI, pJ;          // basis sizes (Chebyshev nodes, or window size when exact)
  int exactI, exactJ;  // 1: the window's inputs themselves are the nodes
  int level;
  int toff_u, toff_v;  // offsets (doubles) of T_U (pI x kcap) and T_V (pJ x kcap)
  int mom_off_i, mom_off_j;  // offsets (doubles) of the final moments of each side
  int pad;
  double aI, bI, aJ, bJ;     // interpolation intervals
};

// A contiguous row range of one side of one node.
struct Task {
  int h;     // heap index of the internal node
  int side;  // 0: left child rows (U), 1: right child rows (V)
  int r0, r1;
};

// Host-side plan of one HODLR build (tree + windows + interpolation sizes).
struct HostPlan {
  int n = 0, B = 0, L = 0, nint = 0, nleaf = 0;
  int kind = 0;
  double ell = 0, nugget = 0, tol = 0;
  std::vector<int> leaf_lo;              // nleaf + 1
  std::vector<NodePlan> nodes;           // nint
  std::vector<int> kcap, coff;           // per level
  std::vector<int> lpmax;                // per level: largest interpolation order of a side
  int Ktot = 0, kcapmax = 0, pmax = 0;
  int tbuf_size = 0;                     // doubles for all T_U / T_V
  int mom_size = 0;                      // doubles for final moments
  std::vector<Task> mtasks;              // moment tasks (Chebyshev sides, window rows)
  std::vector<int> mtask_off;            // per node side: first moment-task index (2*nint+1)
  int mpart_stride = 0;                  // doubles per moment partial (2*PMAX-1 padded)
  std::vector<Task> gtasks;              // panel-generation tasks (all rows of both sides)
  std::vector<Task> ltasks;              // level tasks, grouped by level
  std::vector<int> ltask_off;            // L + 1
  std::vector<int> node_task_off;        // per node side: first level task (2*nint+1)
  int max_ltasks = 0;
  std::vector<int> max_tps;              // per level: most tasks on one node side
  std::vector<int> max_trows;            // per level: most rows in one level task
  int nmt = 0, ngt = 0, nlt = 0;         // task counts (kept after the vectors are freed)
};

// Builds the plan; returns FG_OK, FG_EINVAL or FG_ETOL (message in err).
fg_status make_plan(const double* xh, int n, int kind, double ell, double nugget, int leaf,
                    double tol, HostPlan& P, std::string& err);

// Device copy of a plan plus per-level device arrays.
struct DevPlan {
  NodePlan* nodes = nullptr;
  int* leaf_lo = nullptr;
  Task* mtasks = nullptr;
  int* mtask_off = nullptr;
  Task* gtasks = nullptr;
  Task* ltasks = nullptr;
  int* node_task_off = nullptr;
  int* coff = nullptr;
  int* kcap = nullptr;
  int* nodemat_off = nullptr;
};

// One plan on host and device, plus the buffer sizes it needs.
struct PlanPack {
  HostPlan P;                    // task vectors are released after upload (counts kept)
  DevPlan D;
  std::vector<int> nodemat_off;  // per node offset (doubles) of G_V, F1, F2
  size_t nodemat_size = 0;
  size_t zpart_size = 0, zfin_size = 0, coef_size = 0;  // factorization scratch (doubles)
  size_t mpart_size = 0;
  size_t mv_work = 0, ap_work = 0;
  std::vector<int> kc_host, co_host;  // upload sources of D.kcap and D.coff
};

// Plans the tree for x (host copy), uploads it; nullptr on error (status, err set).
PlanPack* plan_pack_create(const double* xh, int n, int kind, double ell, double nugget, int leaf,
                           double tol, hipStream_t s, fg_status& st, std::string& err);
// the two halves: the host plan alone (thread-safe, no device call), then its upload on s;
// with sync = false nothing waits and the host task vectors are kept (the uploads may
// still read them) until the pack is destroyed
PlanPack* plan_pack_make(const double* xh, int n, int kind, double ell, double nugget, int leaf,
                         double tol, fg_status& st, std::string& err);
fg_status plan_pack_upload(PlanPack* pk, hipStream_t s, bool sync, std::string& err);
void plan_pack_destroy(PlanPack* pk);
void plan_pack_sizes(PlanPack* pk);  // buffer sizes of pk->P (host only)

// Buffers of one compressed matrix, sized for `cap` (>= the plan it currently holds).
struct HodlrData {
  const PlanPack* pk = nullptr;
  double* x = nullptr;       // n
  double* tbuf = nullptr;    // T_U / T_V
  double* mpart = nullptr;   // moment partials
  double* sv = nullptr;      // nint x PMAX singular values
  int* rank = nullptr;       // nint
  int* kmax = nullptr;       // L (device-decided max rank per level)
  int* rcols = nullptr;      // L x Ktot: right-column lists per level
  int* rcount = nullptr;     // L
  double* panel = nullptr;   // ld x Ktot, column-major (U rows in left children)
  int ld = 0;
  int* status = nullptr;     // device status word
  double* work = nullptr;    // matvec workspace
};

struct FactorData {
  const HodlrData* H = nullptr;
  double alpha = 1, beta = 0;
  bool fp32 = false;           // leaf factor computed and held in FP32 (levels stay FP64)
  float* leafLf = nullptr;     // FP32 leafL / leafLinv (fp32 only; the FP64 ones are unused)
  float* leafLinvf = nullptr;
  double* leafL = nullptr;     // nleaf x B x B
  double* leafLinv = nullptr;  // nleaf x B x B: inverses of L's 16 x 16 diagonal blocks
  double* leaf_ld = nullptr;   // nleaf
  double* panel = nullptr;     // whitened panels, same layout as H->panel
  double* nodemat = nullptr;   // per node: G_V, F1, F2 (k x k each)
  double* node_ld = nullptr;   // nint
  double* zpart = nullptr;     // reduce partials
  double* zfin = nullptr;      // per node final Gram blocks of one level
  double* coef = nullptr;      // per node update coefficients of one level
  double* logdet = nullptr;    // device scalar
  int* status = nullptr;
  double* work = nullptr;      // sweep workspace
};

// capacity of a set of plans
struct Caps {
  int n = 0, B = 0, L = 0, nint = 0, nleaf = 0;
  size_t tbuf = 1, mpart = 1, Ktot = 1, nodemat = 1, zpart = 1, zfin = 1, coef = 1;
  size_t mv_work = 1, ap_work = 1;
  void add(const PlanPack& pk);
};
// device buffers (dev_alloc); the status words and counters they start from are cleared
// by hipMemset, or by hipMemsetAsync on s when async is set
fg_status hodlr_alloc(HodlrData& H, const Caps& c, std::string& err, hipStream_t s = nullptr,
                      bool async = false);
void hodlr_free(HodlrData& H);
fg_status factor_alloc(FactorData& F, const Caps& c, std::string& err, bool fp32 = false,
                       hipStream_t s = nullptr, bool async = false);
void factor_free(FactorData& F);
// device bytes held by a plan upload, a compressed matrix and a factor of capacity c
size_t plan_device_bytes(const PlanPack& pk);
size_t hodlr_bytes(const Caps& c);
size_t factor_bytes(const Caps& c, bool fp32);

// -------- kernels' host launchers (stream-ordered) --------
void launch_build(HodlrData& H, hipStream_t s);
void launch_factor(FactorData& F, const double* alpha_dev, const double* beta_dev,
                   const double* diag, hipStream_t s);
// the two halves of launch_factor: the leaves need x and the kernel's parameters only (not
// the compressed panels), so they may run on another stream than the build; the levels
// need both the leaves and the build
void launch_factor_leaves(FactorData& F, const double* alpha_dev, const double* beta_dev,
                          const double* diag, hipStream_t s);
void launch_factor_levels(FactorData& F, const double* alpha_dev, hipStream_t s);
void launch_logdet_sum(FactorData& F, hipStream_t s);
// out (device, 2): the leaf part and the node part of the log-det
void launch_logdet_parts(const FactorData& F, double* out, hipStream_t s);
// op: 0 = W, 1 = W', 2 = W^-1, 3 = W^-T; in place on v (ld x nrhs)
void launch_apply_w(FactorData& F, int op, double* v, int nrhs, int ld, double* work,
                    hipStream_t s);
// y = alpha K~_1 v + beta v (alpha/beta from device pointers when non-null)
void launch_matvec(const HodlrData& H, double alpha, double beta, const double* alpha_dev,
                   const double* beta_dev, const double* v, double* y, int nrhs, int ld,
                   double* work, hipStream_t s);
void launch_entries(const HodlrData& H, const int64_t* i, const int64_t* j, int64_t count,
                    double* out, hipStream_t s);
// iteration word from iter_dev (device) when given, else `iter`
void launch_normals(uint64_t seed, uint64_t tag, uint64_t iter, uint64_t strm, int64_t n,
                    double* out, hipStream_t s, const uint64_t* iter_dev = nullptr);
// out = scale * sum (a-b)^2 or sum a*b etc (deterministic two-stage)
void launch_dot(const double* a, const double* b, int n, int mode, double* out, double* work,
                hipStream_t s);
// Sums the task partials of every node side with more than one task; a side with one
// task is left to its consumer, which reads that task's partial in place.  max_tasks
// bounds the tasks of any one side (the plan's per-level maximum).
void launch_zsum(const double* zpart, int zs_task, int tbase, const int* node_task_off, int hbase,
                 int nsides, int esz, double* zfin, int zf_side, int max_tasks, hipStream_t s);
// device-to-device copy (a kernel, so that grouped batches can group it)
void launch_copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s);
void launch_axpby(int n, const double* x, const double* y, double* out,
                  const double* ca_dev, double ca, const double* cb_dev, double cb, hipStream_t s);
// non-unique inputs: sum w (a - b)^2, out = x / *den, and the averages' precisions
void launch_wsse(const double* a, const double* b, const double* w, int n, double* out,
                 double* work, hipStream_t s);
void launch_div_scalar(int n, const double* x, const double* den_dev, double* out, hipStream_t s);
void launch_collapsed_weights(int n, const double* w, const double* alpha_dev, double* dprec,
                              double* dinv, hipStream_t s);
// function posterior at new inputs (k_predict.hip)
void launch_cross_cov(const double* x, int n, const double* xstar, int nstar, int kind,
                      double ell, double* Z, int64_t ld, hipStream_t s);
constexpr int PC_PREDICT = 4;         // new points per work-group of the predictive reduction
constexpr int MAX_NSTAR = 65535 * PC_PREDICT;
size_t predict_part_doubles(int n, int nstar);  // partial sums of the predictive reduction
void launch_predict_point(const double* Z, int64_t ld, int n, const double* zf, const double* xi,
                          const double* sigf2_p, double eta, int nstar, double* part,
                          double* fstar, double* mu, double* s2, hipStream_t s);

size_t matvec_work_doubles(const HostPlan& P, int nrhs);
size_t apply_work_doubles(const HostPlan& P, int nrhs);

// error helper
void set_error(const std::string& msg);

// -------- memory (alloc.cpp) --------
// A region of device (or pinned host) memory allocated once and sub-allocated best-fit
// in 256-byte units.  Thread-safe.
class Arena {
 public:
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena();
  fg_status init(size_t bytes, bool pinned_host, std::string& err);
  // an arena over memory that belongs to someone else (a block of another arena); the
  // base address must be 256-byte aligned
  fg_status init_view(void* base, size_t bytes);
  void release();
  void* alloc(size_t bytes);  // nullptr when no free block is large enough
  void free(void* p);
  size_t capacity() const { return cap_; }
  size_t largest_free() const;
  size_t in_use() const;

 private:
  char* base_ = nullptr;
  size_t cap_ = 0;
  bool pinned_ = false;
  bool view_ = false;
  mutable std::mutex mu_;
  std::map<size_t, size_t> free_;  // offset -> size
  std::map<size_t, size_t> used_;
  size_t in_use_ = 0;
};
// While an ArenaScope lives, dev_alloc / host_alloc on this thread take their memory from
// the given arenas (a null arena: the runtime allocator).
class ArenaScope {
 public:
  ArenaScope(Arena* dev, Arena* host);
  ~ArenaScope();

 private:
  Arena* prev_dev_;
  Arena* prev_host_;
};
hipError_t dev_alloc(void** p, size_t bytes);
void dev_free(void* p);   // arena memory goes back to its arena, from any thread
hipError_t host_alloc(void** p, size_t bytes);  // pinned host memory
void host_free(void* p);

}  // namespace fg
