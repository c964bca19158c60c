// Tensor-product surface model (Section 4.2) and Algorithm 1.h (Appendix,
// heteroskedastic noise): the per-factor data of a sweep and its scalar steps.
//
// Factor h sees y_i / g_i, g_i = beta prod_{k != h} f_k(x[k, i]), as a noisy
// observation of f_h(x[h, i]) with precision D_i = tau g_i^2.  Vectors of factor h are
// kept in the ascending order of dimension h (perm_h[j] = observation index of sorted
// position j); the factors themselves are kept in observation order.  |g| is floored
// at 1e-150 (sign kept, zero taken as positive) so that 1/D stays finite.
#include "fg_group.h"
#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_tensor.h"

namespace fg {

constexpr double G_FLOOR = 1e-150;

// D, 1/D and y/g of factor h, in the sorted order of dimension h
__global__ void k_tp_prepare(int n, int d, int h, const int* __restrict__ perm,
                             const double* __restrict__ F, const double* __restrict__ y,
                             const TpState* __restrict__ st, const double* __restrict__ beta_p,
                             double* __restrict__ D, double* __restrict__ Dinv,
                             double* __restrict__ yt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = perm[j];
  double g = *beta_p;
  for (int k = 0; k < d; ++k)
    if (k != h) g *= F[(size_t)k * n + i];
  if (fabs(g) < G_FLOOR) g = (g < 0.0) ? -G_FLOOR : G_FLOOR;
  const double dv = st->tau * g * g;
  D[j] = dv;
  Dinv[j] = 1.0 / dv;
  yt[j] = y[i] / g;
}

// a = sqrt(D) a_std  (a ~ N(0, D))
__global__ void k_scale_sqrt(int n, const double* __restrict__ D, double* __restrict__ v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) v[j] *= sqrt(D[j]);
}

// f = R + Z* / D; written in sorted order and scattered to observation order
__global__ void k_hetero_finish(int n, const double* __restrict__ R, const double* __restrict__ Zs,
                                const double* __restrict__ D, double* __restrict__ f,
                                const int* __restrict__ perm, double* __restrict__ Fh) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double v = R[j] + Zs[j] / D[j];
  f[j] = v;
  if (perm) Fh[perm[j]] = v;
}

// partial residual of component c and the fitted sum (observation order)
__global__ void k_tp_partial(int n, int C, int c, const double* __restrict__ y,
                             const double* __restrict__ G, const TpState* __restrict__ st,
                             double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = y[i];
  for (int cc = 0; cc < C; ++cc)
    if (cc != c) v -= st->beta[cc] * G[(size_t)cc * n + i];
  r[i] = v;
}

__global__ void k_tp_fit(int n, int C, const double* __restrict__ G,
                         const TpState* __restrict__ st, double* __restrict__ fit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int cc = 0; cc < C; ++cc) v += st->beta[cc] * G[(size_t)cc * n + i];
  fit[i] = v;
}

// G_i = prod_h f_h(x[h, i])  (observation order)
__global__ void k_tp_product(int n, int d, const double* __restrict__ F, double* __restrict__ G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double g = 1.0;
  for (int k = 0; k < d; ++k) g *= F[(size_t)k * n + i];
  G[i] = g;
}

// beta_c | - ~ N(tau G_c'r_c / prec, 1 / prec), prec = tau G_c'G_c + s_beta^-2; the normal
// is z[0] of the normals stream of beta_c's tag (Box-Muller cosine branch of block 0)
__global__ void k_tp_beta_step(TpState* st, int c, double s_beta, uint64_t seed, uint64_t iter,
                               uint64_t strm) {
  const double prec = st->tau * st->GG + 1.0 / (s_beta * s_beta);
  const double mean = st->tau * st->Gy / prec;
  const double sd = 1.0 / sqrt(prec);
  uint64_t w[4];
  philox4x64_10(0, tp_beta_tag(c), iter, strm, seed, 0, w);
  const double z = sqrt(-2.0 * log(to_unit(w[0]))) * cos(2.0 * M_PI * to_unit(w[1]));
  st->beta_mean[c] = mean;
  st->beta_sd[c] = sd;
  st->beta[c] = mean + sd * z;
}

__global__ void k_tp_tau_step(TpState* st, int n, double a1, double b1, uint64_t seed,
                              uint64_t iter, uint64_t strm) {
  const double g = gamma_mt(0.5 * (a1 + n), seed, 3, iter, strm, &st->status);
  st->tau = g / (0.5 * (b1 + st->sse));
}

// length-scale of factor h: D = -1/2 (log|K~'| - log|K~|) - (q' - q)/2
__global__ void k_tp_mh_step(TpState* st, int h, int kprop, int ongrid, uint64_t seed,
                             uint64_t iter, uint64_t strm, const int* pst_a, const int* pst_b) {
  st->kprop[h] = kprop;
  st->accept[h] = 0;
  st->mh[h] = 0.0;
  if (!ongrid) return;
  if ((pst_a && (*pst_a & ST_NOTSPD)) || (pst_b && (*pst_b & ST_NOTSPD))) return;
  const double D = -0.5 * (st->logdetp[h] - st->logdet[h]) - 0.5 * (st->qp[h] - st->q[h]);
  st->mh[h] = D;
  uint64_t w[4];
  philox4x64_10(0, tp_factor_tag(6, h), iter, strm, seed, 0, w);
  if (log(to_unit(w[0])) < D) {
    st->accept[h] = 1;
    st->accepts[h] += 1;
    st->k[h] = kprop;
    st->logdet[h] = st->logdetp[h];
    st->q[h] = st->qp[h];
  }
}

static inline unsigned nblk(int n) { return (unsigned)((n + 255) / 256); }

void launch_tp_prepare(int n, int d, int h, const int* perm, const double* F, const double* y,
                       const TpState* st, const double* beta_p, double* D, double* Dinv,
                       double* yt, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_tp_prepare<<<nblk(n), 256, 0, q_>>>(n, d, h, perm, F, y, st, beta_p, D, Dinv, yt));
}
void launch_tp_partial(int n, int C, int c, const double* y, const double* G, const TpState* st,
                       double* r, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_tp_partial<<<nblk(n), 256, 0, q_>>>(n, C, c, y, G, st, r));
}
void launch_tp_fit(int n, int C, const double* G, const TpState* st, double* fit, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_tp_fit<<<nblk(n), 256, 0, q_>>>(n, C, G, st, fit));
}
void launch_scale_sqrt(int n, const double* D, double* v, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_scale_sqrt<<<nblk(n), 256, 0, q_>>>(n, D, v));
}
void launch_hetero_finish(int n, const double* R, const double* Zs, const double* D, double* f,
                          const int* perm, double* Fh, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_hetero_finish<<<nblk(n), 256, 0, q_>>>(n, R, Zs, D, f, perm, Fh));
}
void launch_tp_product(int n, int d, const double* F, double* G, hipStream_t s) {
  if (n > 0) FG_RUN(s, k_tp_product<<<nblk(n), 256, 0, q_>>>(n, d, F, G));
}
void launch_tp_beta_step(TpState* st, int c, double s_beta, uint64_t seed, uint64_t iter,
                         uint64_t strm, hipStream_t s) {
  FG_RUN(s, k_tp_beta_step<<<1, 1, 0, q_>>>(st, c, s_beta, seed, iter, strm));
}
void launch_tp_tau_step(TpState* st, int n, double a1, double b1, uint64_t seed, uint64_t iter,
                        uint64_t strm, hipStream_t s) {
  FG_RUN(s, k_tp_tau_step<<<1, 1, 0, q_>>>(st, n, a1, b1, seed, iter, strm));
}
void launch_tp_mh_step(TpState* st, int h, int kprop, int ongrid, uint64_t seed, uint64_t iter,
                       uint64_t strm, const int* pst_a, const int* pst_b, hipStream_t s) {
  FG_RUN(s, k_tp_mh_step<<<1, 1, 0, q_>>>(st, h, kprop, ongrid, seed, iter, strm, pst_a, pst_b));
}

}  // namespace fg
