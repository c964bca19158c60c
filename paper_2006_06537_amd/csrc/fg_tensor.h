// Tensor-product sampler internals (device state and launchers).
#pragma once
#include "fg_internal.h"

namespace fg {

constexpr int TP_DMAX = 8;          // most factors of one tensor-product chain
constexpr int TP_CMAX = 4;          // most additive components
constexpr uint64_t TP_TAG_BETA = 7;
constexpr uint64_t TP_TAG_STRIDE = 16;

// tag of the 1-D sampler's draw `tag` for factor h
__host__ __device__ inline uint64_t tp_factor_tag(uint64_t tag, int h) {
  return tag + TP_TAG_STRIDE * (uint64_t)(h + 1);
}
// tag of beta_c's normal
__host__ __device__ inline uint64_t tp_beta_tag(int c) {
  return c == 0 ? TP_TAG_BETA : TP_TAG_BETA + TP_TAG_STRIDE * (uint64_t)(9 + c);
}

struct TpState {
  double tau;
  double beta[TP_CMAX];
  double GG, Gy, sse;               // G_c'G_c, G_c'r_c, |y - sum beta_c G_c|^2
  double beta_mean[TP_CMAX], beta_sd[TP_CMAX];  // moments of the last beta_c draws
  double logdet[TP_DMAX], logdetp[TP_DMAX];
  double q[TP_DMAX], qp[TP_DMAX], mh[TP_DMAX];
  int k[TP_DMAX], kprop[TP_DMAX], accept[TP_DMAX], accepts[TP_DMAX];
  int status, pad;
};

void launch_tp_prepare(int n, int d, int h, const int* perm, const double* F, const double* y,
                       const TpState* st, const double* beta_p, double* D, double* Dinv,
                       double* yt, hipStream_t s);
// r = y - sum_{c' != c} beta_c' G_c'  and  fit = sum_c beta_c G_c  (G: C x n)
void launch_tp_partial(int n, int C, int c, const double* y, const double* G, const TpState* st,
                       double* r, hipStream_t s);
void launch_tp_fit(int n, int C, const double* G, const TpState* st, double* fit, hipStream_t s);
void launch_scale_sqrt(int n, const double* D, double* v, hipStream_t s);
void launch_hetero_finish(int n, const double* R, const double* Zs, const double* D, double* f,
                          const int* perm, double* Fh, hipStream_t s);
void launch_tp_product(int n, int d, const double* F, double* G, hipStream_t s);
void launch_tp_beta_step(TpState* st, int c, double s_beta, uint64_t seed, uint64_t iter,
                         uint64_t strm, hipStream_t s);
void launch_tp_tau_step(TpState* st, int n, double a1, double b1, uint64_t seed, uint64_t iter,
                        uint64_t strm, hipStream_t s);
void launch_tp_mh_step(TpState* st, int h, int kprop, int ongrid, uint64_t seed, uint64_t iter,
                       uint64_t strm, const int* pst_a, const int* pst_b, hipStream_t s);

}  // namespace fg
