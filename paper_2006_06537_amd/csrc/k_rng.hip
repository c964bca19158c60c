// Random numbers, reductions and the scalar steps of the Gibbs sweep (gfx950).
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by the Weyl constants after each round.  Key (seed, 0), counter
// (block, tag, iteration, stream); uniform ((w >> 12) + 0.5) 2^-52 lies in (0, 1).
// Normals: Box-Muller on (u0, u1) and (u2, u3) of each block, cosine then sine.
// Gamma(a, 1): Marsaglia & Tsang (2000), try t on block t (normal from u0, u1 by the
// cosine branch, acceptance uniform u2), at most 64 tries.
#include "fg_group.h"
#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_pcg.h"

namespace fg {

// arguments of k_normals (one struct, so that grouped launches can stage one per member)
struct k_normals_args {
  uint64_t seed;
  uint64_t tag;
  uint64_t iter;
  const uint64_t* iter_p;
  uint64_t strm;
  int64_t n;
  double* out;
};
__device__ __forceinline__ void k_normals_body(const k_normals_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  uint64_t seed = a_.seed;
  uint64_t tag = a_.tag;
  uint64_t iter = a_.iter;
  const uint64_t* iter_p = a_.iter_p;
  uint64_t strm = a_.strm;
  int64_t n = a_.n;
  double* __restrict__ out = a_.out;
  (void)by_;
  (void)gy_;

  const int64_t j = (int64_t)bx_ * blockDim.x + threadIdx.x;
  const int64_t nb = (n + 3) / 4;
  if (j >= nb) return;
  if (iter_p) iter = *iter_p;
  uint64_t w[4];
  philox4x64_10((uint64_t)j, tag, iter, strm, seed, 0, w);
  const double u0 = to_unit(w[0]), u1 = to_unit(w[1]), u2 = to_unit(w[2]), u3 = to_unit(w[3]);
  const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
  const double z[4] = {r01 * cos(2.0 * M_PI * u1), r01 * sin(2.0 * M_PI * u1),
                       r23 * cos(2.0 * M_PI * u3), r23 * sin(2.0 * M_PI * u3)};
  for (int e = 0; e < 4; ++e) {
    const int64_t i = 4 * j + e;
    if (i < n) out[i] = z[e];
  }
}
__global__ void  k_normals(const k_normals_args a_) {
  k_normals_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_normals_g(const k_normals_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_normals_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_normals_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_normals_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_normals_args* a, const int* st, const int* gy, int mm) {
    k_normals_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_normals now, or records it while a recorder is open on this thread
static void k_normals_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_normals_args& a) {
  if (recording())
    record_group(k_normals_grp, group_key((const void*)k_normals_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_normals<<<g, b, lds, s>>>(a);
}

// ---------------------------------------------------------------------------------
// deterministic two-stage reductions.  mode 0: sum a*b, 1: sum (a-b)^2
// ---------------------------------------------------------------------------------
constexpr int DOT_BLOCKS = 1024;

__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// arguments of k_dot_stage1 (one struct, so that grouped launches can stage one per member)
struct k_dot_stage1_args {
  const double* a;
  const double* b;
  int n;
  int mode;
  double* part;
};
__device__ __forceinline__ void k_dot_stage1_body(const k_dot_stage1_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const double* __restrict__ a = a_.a;
  const double* __restrict__ b = a_.b;
  int n = a_.n;
  int mode = a_.mode;
  double* __restrict__ part = a_.part;
  (void)by_;
  (void)gy_;

  __shared__ double red[NTHREADS / 64];
  double s = 0.0;
  for (int i = bx_ * NTHREADS + threadIdx.x; i < n; i += DOT_BLOCKS * NTHREADS) {
    const double d = (mode == 1) ? a[i] - b[i] : a[i];
    s += (mode == 1) ? d * d : d * b[i];
  }
  s = wsum64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) t += red[w];
    part[bx_] = t;
  }
}
__global__ void __launch_bounds__(NTHREADS) k_dot_stage1(const k_dot_stage1_args a_) {
  k_dot_stage1_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_dot_stage1_g(const k_dot_stage1_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_dot_stage1_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_dot_stage1_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_dot_stage1_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_dot_stage1_args* a, const int* st, const int* gy, int mm) {
    k_dot_stage1_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_dot_stage1 now, or records it while a recorder is open on this thread
static void k_dot_stage1_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_dot_stage1_args& a) {
  if (recording())
    record_group(k_dot_stage1_grp, group_key((const void*)k_dot_stage1_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_dot_stage1<<<g, b, lds, s>>>(a);
}

// arguments of k_dot_stage2 (one struct, so that grouped launches can stage one per member)
struct k_dot_stage2_args {
  const double* part;
  double* out;
};
__device__ __forceinline__ void k_dot_stage2_body(const k_dot_stage2_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const double* __restrict__ part = a_.part;
  double* __restrict__ out = a_.out;
  (void)by_;
  (void)gy_;

  __shared__ double red[NTHREADS / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += NTHREADS) s += part[i];
  s = wsum64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) t += red[w];
    *out = t;
  }
}
__global__ void __launch_bounds__(NTHREADS) k_dot_stage2(const k_dot_stage2_args a_) {
  k_dot_stage2_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void __launch_bounds__(NTHREADS) k_dot_stage2_g(const k_dot_stage2_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_dot_stage2_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_dot_stage2_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_dot_stage2_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_dot_stage2_args* a, const int* st, const int* gy, int mm) {
    k_dot_stage2_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_dot_stage2 now, or records it while a recorder is open on this thread
static void k_dot_stage2_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_dot_stage2_args& a) {
  if (recording())
    record_group(k_dot_stage2_grp, group_key((const void*)k_dot_stage2_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_dot_stage2<<<g, b, lds, s>>>(a);
}

// sum_i w_i (a_i - b_i)^2, stage 1 (stage 2 as for the plain dot)
__global__ void __launch_bounds__(NTHREADS) k_wdot_stage1(const double* __restrict__ a,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ w, int n,
                                                          double* __restrict__ part) {
  __shared__ double red[NTHREADS / 64];
  double s = 0.0;
  for (int i = blockIdx.x * NTHREADS + threadIdx.x; i < n; i += DOT_BLOCKS * NTHREADS) {
    const double d = a[i] - b[i];
    s += w[i] * d * d;
  }
  s = wsum64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int v = 0; v < NTHREADS / 64; ++v) t += red[v];
    part[blockIdx.x] = t;
  }
}

void launch_wsse(const double* a, const double* b, const double* w, int n, double* out,
                 double* work, hipStream_t s) {
  FG_RUN(s, k_wdot_stage1<<<DOT_BLOCKS, NTHREADS, 0, q_>>>(a, b, w, n, work));
  k_dot_stage2_launch(dim3(1), dim3(NTHREADS), 0, s, k_dot_stage2_args{work, out});
}

// out = x / *den
__global__ void k_div_scalar(int n, const double* __restrict__ x, const double* __restrict__ den,
                             double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] / *den;
}
void launch_div_scalar(int n, const double* x, const double* den_dev, double* out, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_div_scalar<<<(n + 255) / 256, 256, 0, q_>>>(n, x, den_dev, out));
}

// precisions of the averages on the sigma_f scale, and their inverses:
// dprec_i = (tau sigma_f^2) |Q_i|, dinv_i = 1 / dprec_i
__global__ void k_collapsed_weights(int n, const double* __restrict__ w,
                                    const double* __restrict__ alpha, double* __restrict__ dprec,
                                    double* __restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = (*alpha) * w[i];
  dprec[i] = d;
  dinv[i] = 1.0 / d;
}
void launch_collapsed_weights(int n, const double* w, const double* alpha_dev, double* dprec,
                              double* dinv, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_collapsed_weights<<<(n + 255) / 256, 256, 0, q_>>>(n, w, alpha_dev, dprec, dinv));
}

void launch_dot(const double* a, const double* b, int n, int mode, double* out, double* work,
                hipStream_t s) {
  k_dot_stage1_launch(dim3(DOT_BLOCKS), dim3(NTHREADS), 0, s, k_dot_stage1_args{a, b, n, mode, work});
  k_dot_stage2_launch(dim3(1), dim3(NTHREADS), 0, s, k_dot_stage2_args{work, out});
}

// out = ca * x + cb * y  (coefficients from device pointers when given)
// arguments of k_axpby (one struct, so that grouped launches can stage one per member)
struct k_axpby_args {
  int n;
  const double* x;
  const double* y;
  double* out;
  const double* ca_p;
  double ca;
  const double* cb_p;
  double cb;
};
__device__ __forceinline__ void k_axpby_body(const k_axpby_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int n = a_.n;
  const double* __restrict__ x = a_.x;
  const double* __restrict__ y = a_.y;
  double* __restrict__ out = a_.out;
  const double* __restrict__ ca_p = a_.ca_p;
  double ca = a_.ca;
  const double* __restrict__ cb_p = a_.cb_p;
  double cb = a_.cb;
  (void)by_;
  (void)gy_;

  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = ca_p ? *ca_p : ca;
  const double b = cb_p ? *cb_p : cb;
  double v = a * x[i];
  if (y) v += b * y[i];
  out[i] = v;
}
__global__ void  k_axpby(const k_axpby_args a_) {
  k_axpby_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_axpby_g(const k_axpby_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_axpby_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_axpby_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_axpby_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_axpby_args* a, const int* st, const int* gy, int mm) {
    k_axpby_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_axpby now, or records it while a recorder is open on this thread
static void k_axpby_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_axpby_args& a) {
  if (recording())
    record_group(k_axpby_grp, group_key((const void*)k_axpby_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_axpby<<<g, b, lds, s>>>(a);
}

void launch_axpby(int n, const double* x, const double* y, double* out, const double* ca_dev,
                  double ca, const double* cb_dev, double cb, hipStream_t s) {
  if (n <= 0) return;
  k_axpby_launch(dim3((n + 255) / 256), dim3(256), 0, s, k_axpby_args{n, x, y, out, ca_dev, ca, cb_dev, cb});
}

void launch_normals(uint64_t seed, uint64_t tag, uint64_t iter, uint64_t strm, int64_t n,
                    double* out, hipStream_t s, const uint64_t* iter_dev) {
  const int64_t nb = (n + 3) / 4;
  if (nb <= 0) return;
  k_normals_launch(dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, k_normals_args{seed, tag, iter, iter_dev, strm, n, out});
}

// ---------------------------------------------------------------------------------
// scalar steps of the sweep (one thread)
// ---------------------------------------------------------------------------------
// derived scalars at the start of a sweep
// arguments of k_sweep_begin (one struct, so that grouped launches can stage one per member)
struct k_sweep_begin_args {
  DevState* st;
  DevState* prev;
};
__device__ __forceinline__ void k_sweep_begin_body(const k_sweep_begin_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  DevState* st = a_.st;
  DevState* prev = a_.prev;
  (void)by_;
  (void)gy_;

  if (prev) *prev = *st;
  st->alphaM = st->tau * st->sigf2;
  st->c_ka = sqrt(st->tau) * st->sigf2;
  st->sigf = sqrt(st->sigf2);
  st->tau_draw = st->tau;
}
__global__ void  k_sweep_begin(const k_sweep_begin_args a_) {
  k_sweep_begin_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_sweep_begin_g(const k_sweep_begin_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_sweep_begin_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_sweep_begin_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_sweep_begin_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_sweep_begin_args* a, const int* st, const int* gy, int mm) {
    k_sweep_begin_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_sweep_begin now, or records it while a recorder is open on this thread
static void k_sweep_begin_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_sweep_begin_args& a) {
  if (recording())
    record_group(k_sweep_begin_grp, group_key((const void*)k_sweep_begin_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_sweep_begin<<<g, b, lds, s>>>(a);
}

__global__ void k_set_draw_scalars(DevState* st, double tau, double sigf2) {
  st->tau = tau;
  st->sigf2 = sigf2;
  st->alphaM = tau * sigf2;
  st->c_ka = sqrt(tau) * sigf2;
  st->sigf = sqrt(sigf2);
  st->tau_draw = tau;
}

// log-likelihood bookkeeping of the f draw and the tau update
// arguments of k_tau_step (one struct, so that grouped launches can stage one per member)
struct k_tau_step_args {
  DevState* st;
  int n;
  double a1;
  double b1;
  uint64_t seed;
  uint64_t strm;
};
__device__ __forceinline__ void k_tau_step_body(const k_tau_step_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  DevState* st = a_.st;
  int n = a_.n;
  double a1 = a_.a1;
  double b1 = a_.b1;
  uint64_t seed = a_.seed;
  uint64_t strm = a_.strm;
  (void)by_;
  (void)gy_;

  const uint64_t iter = st->iter;
  const double tau0 = st->tau_draw;
  st->logdet_sigma = st->logdetM - n * log(tau0);
  st->loglik = -0.5 * n * log(2.0 * M_PI) - 0.5 * st->logdet_sigma - 0.5 * st->yr;
  const double g = gamma_mt(0.5 * (a1 + n), seed, 3, iter, strm, &st->status);
  st->tau = g / (0.5 * (b1 + st->sse));
}
__global__ void  k_tau_step(const k_tau_step_args a_) {
  k_tau_step_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_tau_step_g(const k_tau_step_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_tau_step_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_tau_step_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_tau_step_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_tau_step_args* a, const int* st, const int* gy, int mm) {
    k_tau_step_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_tau_step now, or records it while a recorder is open on this thread
static void k_tau_step_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_tau_step_args& a) {
  if (recording())
    record_group(k_tau_step_grp, group_key((const void*)k_tau_step_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_tau_step<<<g, b, lds, s>>>(a);
}

// collapsed data: the averages' log-likelihood (Sigma = sigma_f^2 (K~_1 + D^-1), st->yr
// holding ybar' P^-1 (ybar / sigma_f)) and tau from the full-data residual
__global__ void k_tau_step_collapsed(DevState* st, int u, int64_t n_obs, double within, double a1,
                                     double b1, uint64_t seed, uint64_t strm) {
  const uint64_t iter = st->iter;
  st->yr = st->yr / st->sigf;
  st->logdet_sigma = st->logdetM + u * log(st->sigf2);
  st->loglik = -0.5 * u * log(2.0 * M_PI) - 0.5 * st->logdet_sigma - 0.5 * st->yr;
  st->sse += within;
  const double g = gamma_mt(0.5 * (a1 + (double)n_obs), seed, 3, iter, strm, &st->status);
  st->tau = g / (0.5 * (b1 + st->sse));
}

// arguments of k_sigf_step (one struct, so that grouped launches can stage one per member)
struct k_sigf_step_args {
  DevState* st;
  int n;
  double a2;
  double b2;
  uint64_t seed;
  uint64_t strm;
};
__device__ __forceinline__ void k_sigf_step_body(const k_sigf_step_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  DevState* st = a_.st;
  int n = a_.n;
  double a2 = a_.a2;
  double b2 = a_.b2;
  uint64_t seed = a_.seed;
  uint64_t strm = a_.strm;
  (void)by_;
  (void)gy_;

  const uint64_t iter = st->iter;
  const double g = gamma_mt(0.5 * (a2 + n), seed, 4, iter, strm, &st->status);
  st->sigf2 = 1.0 / (g / (0.5 * (b2 + st->q)));
}
__global__ void  k_sigf_step(const k_sigf_step_args a_) {
  k_sigf_step_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_sigf_step_g(const k_sigf_step_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_sigf_step_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_sigf_step_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_sigf_step_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_sigf_step_args* a, const int* st, const int* gy, int mm) {
    k_sigf_step_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_sigf_step now, or records it while a recorder is open on this thread
static void k_sigf_step_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_sigf_step_args& a) {
  if (recording())
    record_group(k_sigf_step_grp, group_key((const void*)k_sigf_step_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_sigf_step<<<g, b, lds, s>>>(a);
}

// arguments of k_mh_step (one struct, so that grouped launches can stage one per member)
struct k_mh_step_args {
  DevState* st;
  int kprop;
  int ongrid;
  uint64_t seed;
  uint64_t strm;
  const int* pst_a;
  const int* pst_b;
};
__device__ __forceinline__ void k_mh_step_body(const k_mh_step_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  DevState* st = a_.st;
  int kprop = a_.kprop;
  int ongrid = a_.ongrid;
  uint64_t seed = a_.seed;
  uint64_t strm = a_.strm;
  const int* pst_a = a_.pst_a;
  const int* pst_b = a_.pst_b;
  (void)by_;
  (void)gy_;

  const uint64_t iter = st->iter;
  st->iter = iter + 1;  // this step ends the sweep
  st->kprop = kprop;
  st->accept = 0;
  st->mh = 0.0;
  if (!ongrid) return;
  // a proposal whose matrix is not positive definite on the device is rejected
  if ((pst_a && (*pst_a & ST_NOTSPD)) || (pst_b && (*pst_b & ST_NOTSPD))) return;
  const double D = -0.5 * (st->logdet1p - st->logdet1) - (st->qprop - st->q) / (2.0 * st->sigf2);
  st->mh = D;
  uint64_t w[4];
  philox4x64_10(0, 6, iter, strm, seed, 0, w);
  const double u = to_unit(w[0]);
  if (log(u) < D) {
    st->accept = 1;
    st->accepts += 1;
    st->k = kprop;
    st->logdet1 = st->logdet1p;
    st->q = st->qprop;
  }
}
__global__ void  k_mh_step(const k_mh_step_args a_) {
  k_mh_step_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_mh_step_g(const k_mh_step_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_mh_step_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_mh_step_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_mh_step_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_mh_step_args* a, const int* st, const int* gy, int mm) {
    k_mh_step_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_mh_step now, or records it while a recorder is open on this thread
static void k_mh_step_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_mh_step_args& a) {
  if (recording())
    record_group(k_mh_step_grp, group_key((const void*)k_mh_step_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_mh_step<<<g, b, lds, s>>>(a);
}

// The exact discrete conditional of the length-scale (Section 4.1, uniform prior over the
// grid): log-weights lp_h = -1/2 log det K~_1(s_h) - q_h / (2 sigma_f^2), one uniform (tag 9)
// through the inverse CDF: the first h whose cumulative weight exceeds u times the total.
// Ends the sweep like the Metropolis step.
__global__ void k_rho_exact(DevState* st, const double* __restrict__ ld,
                            const double* __restrict__ q, int G, uint64_t seed, uint64_t strm) {
  const uint64_t iter = st->iter;
  st->iter = iter + 1;
  const double s2 = st->sigf2;
  double m = -INFINITY;
  for (int h = 0; h < G; ++h) m = fmax(m, -0.5 * ld[h] - q[h] / (2.0 * s2));
  double tot = 0.0;
  for (int h = 0; h < G; ++h) tot += exp(-0.5 * ld[h] - q[h] / (2.0 * s2) - m);
  uint64_t w[4];
  philox4x64_10(0, 9, iter, strm, seed, 0, w);
  const double t = to_unit(w[0]) * tot;
  double c = 0.0;
  int pick = G - 1;
  for (int h = 0; h < G; ++h) {
    c += exp(-0.5 * ld[h] - q[h] / (2.0 * s2) - m);
    if (c > t) {
      pick = h;
      break;
    }
  }
  const int old = st->k;
  st->kprop = pick;
  st->accept = pick != old;
  st->accepts += st->accept;
  st->k = pick;
  st->logdet1 = ld[pick];
  st->q = q[pick];
  st->mh = -0.5 * ld[pick] - q[pick] / (2.0 * s2) - (m + log(tot));
}

void launch_rho_exact(DevState* st, const double* ld, const double* q, int G, uint64_t seed,
                      uint64_t strm, hipStream_t s) {
  FG_RUN(s, k_rho_exact<<<1, 1, 0, q_>>>(st, ld, q, G, seed, strm));
}

void launch_sweep_begin(DevState* st, DevState* prev, hipStream_t s) {
  k_sweep_begin_launch(dim3(1), dim3(1), 0, s, k_sweep_begin_args{st, prev});
}
void launch_set_draw_scalars(DevState* st, double tau, double sigf2, hipStream_t s) {
  FG_RUN(s, k_set_draw_scalars<<<1, 1, 0, q_>>>(st, tau, sigf2));
}
void launch_tau_step(DevState* st, int n, double a1, double b1, uint64_t seed, uint64_t strm,
                     hipStream_t s) {
  k_tau_step_launch(dim3(1), dim3(1), 0, s, k_tau_step_args{st, n, a1, b1, seed, strm});
}
void launch_tau_step_collapsed(DevState* st, int u, int64_t n_obs, double within, double a1,
                               double b1, uint64_t seed, uint64_t strm, hipStream_t s) {
  FG_RUN(s, k_tau_step_collapsed<<<1, 1, 0, q_>>>(st, u, n_obs, within, a1, b1, seed, strm));
}
void launch_sigf_step(DevState* st, int n, double a2, double b2, uint64_t seed, uint64_t strm,
                      hipStream_t s) {
  k_sigf_step_launch(dim3(1), dim3(1), 0, s, k_sigf_step_args{st, n, a2, b2, seed, strm});
}
void launch_mh_step(DevState* st, int kprop, int ongrid, uint64_t seed, uint64_t strm,
                    const int* pst_a, const int* pst_b, hipStream_t s) {
  k_mh_step_launch(dim3(1), dim3(1), 0, s, k_mh_step_args{st, kprop, ongrid, seed, strm, pst_a, pst_b});
}

// arguments of k_zero_int (one struct, so that grouped launches can stage one per member)
struct k_zero_int_args {
  int* p;
  int n;
};
__device__ __forceinline__ void k_zero_int_body(const k_zero_int_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int* p = a_.p;
  int n = a_.n;
  (void)by_;
  (void)gy_;

  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
__global__ void  k_zero_int(const k_zero_int_args a_) {
  k_zero_int_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_zero_int_g(const k_zero_int_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_zero_int_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_zero_int_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_zero_int_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_zero_int_args* a, const int* st, const int* gy, int mm) {
    k_zero_int_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_zero_int now, or records it while a recorder is open on this thread
static void k_zero_int_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_zero_int_args& a) {
  if (recording())
    record_group(k_zero_int_grp, group_key((const void*)k_zero_int_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_zero_int<<<g, b, lds, s>>>(a);
}
// device-to-device copy of `words` 32-bit words, one per thread
// arguments of k_copy_words (one struct, so that grouped launches can stage one per member)
struct k_copy_words_args {
  const uint32_t* src;
  uint32_t* dst;
  int64_t words;
};
__device__ __forceinline__ void k_copy_words_body(const k_copy_words_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const uint32_t* __restrict__ src = a_.src;
  uint32_t* __restrict__ dst = a_.dst;
  int64_t words = a_.words;
  (void)by_;
  (void)gy_;

  const int64_t i = (int64_t)bx_ * blockDim.x + threadIdx.x;
  if (i < words) dst[i] = src[i];
}
__global__ void  k_copy_words(const k_copy_words_args a_) {
  k_copy_words_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_copy_words_g(const k_copy_words_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_copy_words_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_copy_words_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_copy_words_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_copy_words_args* a, const int* st, const int* gy, int mm) {
    k_copy_words_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_copy_words now, or records it while a recorder is open on this thread
static void k_copy_words_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_copy_words_args& a) {
  if (recording())
    record_group(k_copy_words_grp, group_key((const void*)k_copy_words_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_copy_words<<<g, b, lds, s>>>(a);
}

void launch_copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(dst) % 4 || reinterpret_cast<uintptr_t>(src) % 4) {
    FG_RUN(s, (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, q_));
    return;
  }
  const int64_t words = (int64_t)(bytes / 4);
  k_copy_words_launch(dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                      k_copy_words_args{static_cast<const uint32_t*>(src),
                                        static_cast<uint32_t*>(dst), words});
}

void launch_zero_int(int* p, int n, hipStream_t s) {
  if (n > 0) k_zero_int_launch(dim3((n + 255) / 256), dim3(256), 0, s, k_zero_int_args{p, n});
}

}  // namespace fg

// ---------------------------------------------------------------------------------
// PCG vector steps (one thread per row, all right-hand sides)
// ---------------------------------------------------------------------------------
namespace fg {

// arguments of k_pcg_init (one struct, so that grouped launches can stage one per member)
struct k_pcg_init_args {
  int n;
  int nrhs;
  const double* b;
  int ld;
  double* x;
  double* r;
  PcgScalars* sc;
};
__device__ __forceinline__ void k_pcg_init_body(const k_pcg_init_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int n = a_.n;
  int nrhs = a_.nrhs;
  const double* __restrict__ b = a_.b;
  int ld = a_.ld;
  double* __restrict__ x = a_.x;
  double* __restrict__ r = a_.r;
  PcgScalars* sc = a_.sc;
  (void)by_;
  (void)gy_;

  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i == 0) {
    sc->done = 0;
    sc->iters = 0;
    sc->relres = INFINITY;
  }
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) {
    r[(size_t)c * n + i] = b[(size_t)c * ld + i];
    x[(size_t)c * ld + i] = 0.0;
  }
}
__global__ void  k_pcg_init(const k_pcg_init_args a_) {
  k_pcg_init_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_init_g(const k_pcg_init_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_init_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_init_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_init_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_init_args* a, const int* st, const int* gy, int mm) {
    k_pcg_init_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_init now, or records it while a recorder is open on this thread
static void k_pcg_init_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_init_args& a) {
  if (recording())
    record_group(k_pcg_init_grp, group_key((const void*)k_pcg_init_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_init<<<g, b, lds, s>>>(a);
}

// arguments of k_pcg_copy (one struct, so that grouped launches can stage one per member)
struct k_pcg_copy_args {
  int n;
  int nrhs;
  const double* a;
  double* o;
};
__device__ __forceinline__ void k_pcg_copy_body(const k_pcg_copy_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int n = a_.n;
  int nrhs = a_.nrhs;
  const double* __restrict__ a = a_.a;
  double* __restrict__ o = a_.o;
  (void)by_;
  (void)gy_;

  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) o[(size_t)c * n + i] = a[(size_t)c * n + i];
}
__global__ void  k_pcg_copy(const k_pcg_copy_args a_) {
  k_pcg_copy_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_copy_g(const k_pcg_copy_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_copy_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_copy_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_copy_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_copy_args* a, const int* st, const int* gy, int mm) {
    k_pcg_copy_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_copy now, or records it while a recorder is open on this thread
static void k_pcg_copy_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_copy_args& a) {
  if (recording())
    record_group(k_pcg_copy_grp, group_key((const void*)k_pcg_copy_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_copy<<<g, b, lds, s>>>(a);
}

// arguments of k_pcg_xr (one struct, so that grouped launches can stage one per member)
struct k_pcg_xr_args {
  int n;
  int nrhs;
  double* x;
  int ld;
  double* r;
  const double* p;
  const double* q;
  const PcgScalars* sc;
};
__device__ __forceinline__ void k_pcg_xr_body(const k_pcg_xr_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int n = a_.n;
  int nrhs = a_.nrhs;
  double* __restrict__ x = a_.x;
  int ld = a_.ld;
  double* __restrict__ r = a_.r;
  const double* __restrict__ p = a_.p;
  const double* __restrict__ q = a_.q;
  const PcgScalars* __restrict__ sc = a_.sc;
  (void)by_;
  (void)gy_;

  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i >= n || sc->done) return;
  for (int c = 0; c < nrhs; ++c) {
    const double a = sc->pq[c] != 0.0 ? sc->rz[c] / sc->pq[c] : 0.0;
    x[(size_t)c * ld + i] += a * p[(size_t)c * n + i];
    r[(size_t)c * n + i] -= a * q[(size_t)c * n + i];
  }
}
__global__ void  k_pcg_xr(const k_pcg_xr_args a_) {
  k_pcg_xr_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_xr_g(const k_pcg_xr_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_xr_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_xr_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_xr_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_xr_args* a, const int* st, const int* gy, int mm) {
    k_pcg_xr_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_xr now, or records it while a recorder is open on this thread
static void k_pcg_xr_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_xr_args& a) {
  if (recording())
    record_group(k_pcg_xr_grp, group_key((const void*)k_pcg_xr_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_xr<<<g, b, lds, s>>>(a);
}

// p = z + (rz_new / rz) p; the ratio is formed before any thread can update rz, which
// is done by a second kernel
// arguments of k_pcg_p (one struct, so that grouped launches can stage one per member)
struct k_pcg_p_args {
  int n;
  int nrhs;
  double* p;
  const double* z;
  const PcgScalars* sc;
};
__device__ __forceinline__ void k_pcg_p_body(const k_pcg_p_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int n = a_.n;
  int nrhs = a_.nrhs;
  double* __restrict__ p = a_.p;
  const double* __restrict__ z = a_.z;
  const PcgScalars* __restrict__ sc = a_.sc;
  (void)by_;
  (void)gy_;

  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i >= n || sc->done) return;
  for (int c = 0; c < nrhs; ++c) {
    const double bt = sc->rz[c] != 0.0 ? sc->rz_new[c] / sc->rz[c] : 0.0;
    p[(size_t)c * n + i] = z[(size_t)c * n + i] + bt * p[(size_t)c * n + i];
  }
}
__global__ void  k_pcg_p(const k_pcg_p_args a_) {
  k_pcg_p_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_p_g(const k_pcg_p_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_p_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_p_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_p_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_p_args* a, const int* st, const int* gy, int mm) {
    k_pcg_p_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_p now, or records it while a recorder is open on this thread
static void k_pcg_p_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_p_args& a) {
  if (recording())
    record_group(k_pcg_p_grp, group_key((const void*)k_pcg_p_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_p<<<g, b, lds, s>>>(a);
}

// arguments of k_pcg_rz (one struct, so that grouped launches can stage one per member)
struct k_pcg_rz_args {
  int nrhs;
  PcgScalars* sc;
};
__device__ __forceinline__ void k_pcg_rz_body(const k_pcg_rz_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int nrhs = a_.nrhs;
  PcgScalars* sc = a_.sc;
  (void)by_;
  (void)gy_;

  const int c = threadIdx.x;
  if (c < nrhs && !sc->done) sc->rz[c] = sc->rz_new[c];
}
__global__ void  k_pcg_rz(const k_pcg_rz_args a_) {
  k_pcg_rz_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_rz_g(const k_pcg_rz_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_rz_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_rz_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_rz_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_rz_args* a, const int* st, const int* gy, int mm) {
    k_pcg_rz_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_rz now, or records it while a recorder is open on this thread
static void k_pcg_rz_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_rz_args& a) {
  if (recording())
    record_group(k_pcg_rz_grp, group_key((const void*)k_pcg_rz_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_rz<<<g, b, lds, s>>>(a);
}

// the convergence test of iteration `it` (rr and bb hold |r|^2 and |b|^2 per column)
// arguments of k_pcg_check (one struct, so that grouped launches can stage one per member)
struct k_pcg_check_args {
  int nrhs;
  double rtol;
  int it;
  PcgScalars* sc;
};
__device__ __forceinline__ void k_pcg_check_body(const k_pcg_check_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  int nrhs = a_.nrhs;
  double rtol = a_.rtol;
  int it = a_.it;
  PcgScalars* sc = a_.sc;
  (void)by_;
  (void)gy_;

  if (threadIdx.x != 0 || sc->done) return;
  double worst = 0.0;
  bool finite = true;
  for (int c = 0; c < nrhs; ++c) {
    const double bn = sc->bb[c], rn = sc->rr[c];
    if (!isfinite(bn) || !isfinite(rn)) finite = false;
    const double rel = bn > 0.0 ? sqrt(rn / bn) : 0.0;
    if (!(rel <= worst)) worst = rel;
  }
  sc->iters = it;
  if (!finite) {
    sc->relres = NAN;
    sc->done = -1;
    return;
  }
  sc->relres = worst;
  if (worst <= rtol) sc->done = 1;
}
__global__ void  k_pcg_check(const k_pcg_check_args a_) {
  k_pcg_check_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_check_g(const k_pcg_check_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_check_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_check_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_check_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_check_args* a, const int* st, const int* gy, int mm) {
    k_pcg_check_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_check now, or records it while a recorder is open on this thread
static void k_pcg_check_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_check_args& a) {
  if (recording())
    record_group(k_pcg_check_grp, group_key((const void*)k_pcg_check_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_check<<<g, b, lds, s>>>(a);
}

static inline unsigned pblk(int n) { return (unsigned)((n + 255) / 256); }

void launch_pcg_init(int n, int nrhs, const double* b, int ld, double* x, double* r,
                     PcgScalars* sc, hipStream_t s) {
  k_pcg_init_launch(dim3(std::max(pblk(n), 1u)), dim3(256), 0, s,
                    k_pcg_init_args{n, nrhs, b, ld, x, r, sc});
}
void launch_pcg_check(int nrhs, double rtol, int it, PcgScalars* sc, hipStream_t s) {
  k_pcg_check_launch(dim3(1), dim3(64), 0, s, k_pcg_check_args{nrhs, rtol, it, sc});
}

// arguments of k_pcg_record (one struct, so that grouped launches can stage one per member)
struct k_pcg_record_args {
  const PcgScalars* sc;
  DevState* st;
  const int* fstatus;  // status word of the preconditioning factor, or null
};
__device__ __forceinline__ void k_pcg_record_body(const k_pcg_record_args& a_, const int bx_, const int by_,
                                             const int gy_) {
  const PcgScalars* sc = a_.sc;
  DevState* st = a_.st;
  const int* fstatus = a_.fstatus;
  (void)by_;
  (void)gy_;

  st->pcg_relres = sc->relres;
  st->pcg_iters = sc->iters;
  // a preconditioner whose Cholesky met a non-positive pivot is no factor of M~ at all:
  // reported as a failed solve, so that the sweep is run again on an FP64 factor
  st->pcg_done = (fstatus && (*fstatus & ST_NOTSPD)) ? -1 : sc->done;
}
__global__ void  k_pcg_record(const k_pcg_record_args a_) {
  k_pcg_record_body(a_, blockIdx.x, blockIdx.y, gridDim.y);
}
// grouped: blocks [st_[j], st_[j+1]) of the grid run member j; gy_[j] is its grid.y
__global__ void  k_pcg_record_g(const k_pcg_record_args* __restrict__ a_,
                                   const int* __restrict__ st_, const int* __restrict__ gyv_,
                                   int m_) {
  const int j = group_member(st_, m_, blockIdx.x);
  if ((int)blockIdx.y >= gyv_[j]) return;
  k_pcg_record_body(a_[j], blockIdx.x - st_[j], blockIdx.y, gyv_[j]);
}
static void k_pcg_record_grp(GroupExec& ex, const RecLaunch* const* mem, int m) {
  grouped_launch<k_pcg_record_args>(ex, mem, m, [](dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                                  const k_pcg_record_args* a, const int* st, const int* gy, int mm) {
    k_pcg_record_g<<<g, b, lds, s>>>(a, st, gy, mm);
  });
}
// launches k_pcg_record now, or records it while a recorder is open on this thread
static void k_pcg_record_launch(dim3 g, dim3 b, uint32_t lds, hipStream_t s,
                             const k_pcg_record_args& a) {
  if (recording())
    record_group(k_pcg_record_grp, group_key((const void*)k_pcg_record_grp, b, lds), g, b, lds, &a,
                 sizeof(a));
  else
    k_pcg_record<<<g, b, lds, s>>>(a);
}
void launch_pcg_record(const PcgScalars* sc, DevState* st, const int* fstatus, hipStream_t s) {
  k_pcg_record_launch(dim3(1), dim3(1), 0, s, k_pcg_record_args{sc, st, fstatus});
}
void launch_pcg_copy(int n, int nrhs, const double* a, double* out, hipStream_t s) {
  if (n > 0) k_pcg_copy_launch(dim3(pblk(n)), dim3(256), 0, s, k_pcg_copy_args{n, nrhs, a, out});
}
void launch_pcg_xr(int n, int nrhs, double* x, int ld, double* r, const double* p, const double* q,
                   const PcgScalars* sc, hipStream_t s) {
  if (n > 0) k_pcg_xr_launch(dim3(pblk(n)), dim3(256), 0, s, k_pcg_xr_args{n, nrhs, x, ld, r, p, q, sc});
}
void launch_pcg_p(int n, int nrhs, double* p, const double* z, PcgScalars* sc, hipStream_t s) {
  if (n > 0) k_pcg_p_launch(dim3(pblk(n)), dim3(256), 0, s, k_pcg_p_args{n, nrhs, p, z, sc});
  k_pcg_rz_launch(dim3(1), dim3(64), 0, s, k_pcg_rz_args{nrhs, sc});
}

}  // namespace fg
