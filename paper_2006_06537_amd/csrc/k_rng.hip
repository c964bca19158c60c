// Random numbers, reductions and the scalar steps of the Gibbs sweep (gfx950).
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by the Weyl constants after each round.  Key (seed, 0), counter
// (block, tag, iteration, stream); uniform ((w >> 12) + 0.5) 2^-52 lies in (0, 1).
// Normals: Box-Muller on (u0, u1) and (u2, u3) of each block, cosine then sine.
// Gamma(a, 1): Marsaglia & Tsang (2000), try t on block t (normal from u0, u1 by the
// cosine branch, acceptance uniform u2), at most 64 tries.
#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_pcg.h"

namespace fg {

__global__ void k_normals(uint64_t seed, uint64_t tag, uint64_t iter, const uint64_t* iter_p,
                          uint64_t strm, int64_t n, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// ---------------------------------------------------------------------------------
// deterministic two-stage reductions.  mode 0: sum a*b, 1: sum (a-b)^2
// ---------------------------------------------------------------------------------
constexpr int DOT_BLOCKS = 1024;

__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(NTHREADS) k_dot_stage1(const double* __restrict__ a,
                                                         const double* __restrict__ b, int n,
                                                         int mode, double* __restrict__ part) {
  __shared__ double red[NTHREADS / 64];
  double s = 0.0;
  for (int i = blockIdx.x * NTHREADS + threadIdx.x; i < n; i += DOT_BLOCKS * NTHREADS) {
    const double d = (mode == 1) ? a[i] - b[i] : a[i];
    s += (mode == 1) ? d * d : d * b[i];
  }
  s = wsum64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(NTHREADS) k_dot_stage2(const double* __restrict__ part,
                                                         double* __restrict__ out) {
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
  k_wdot_stage1<<<DOT_BLOCKS, NTHREADS, 0, s>>>(a, b, w, n, work);
  k_dot_stage2<<<1, NTHREADS, 0, s>>>(work, out);
}

// out = x / *den
__global__ void k_div_scalar(int n, const double* __restrict__ x, const double* __restrict__ den,
                             double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] / *den;
}
void launch_div_scalar(int n, const double* x, const double* den_dev, double* out, hipStream_t s) {
  if (n > 0) k_div_scalar<<<(n + 255) / 256, 256, 0, s>>>(n, x, den_dev, out);
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
  if (n > 0) k_collapsed_weights<<<(n + 255) / 256, 256, 0, s>>>(n, w, alpha_dev, dprec, dinv);
}

void launch_dot(const double* a, const double* b, int n, int mode, double* out, double* work,
                hipStream_t s) {
  k_dot_stage1<<<DOT_BLOCKS, NTHREADS, 0, s>>>(a, b, n, mode, work);
  k_dot_stage2<<<1, NTHREADS, 0, s>>>(work, out);
}

// out = ca * x + cb * y  (coefficients from device pointers when given)
__global__ void k_axpby(int n, const double* __restrict__ x, const double* __restrict__ y,
                        double* __restrict__ out, const double* __restrict__ ca_p, double ca,
                        const double* __restrict__ cb_p, double cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = ca_p ? *ca_p : ca;
  const double b = cb_p ? *cb_p : cb;
  double v = a * x[i];
  if (y) v += b * y[i];
  out[i] = v;
}

void launch_axpby(int n, const double* x, const double* y, double* out, const double* ca_dev,
                  double ca, const double* cb_dev, double cb, hipStream_t s) {
  if (n <= 0) return;
  k_axpby<<<(n + 255) / 256, 256, 0, s>>>(n, x, y, out, ca_dev, ca, cb_dev, cb);
}

void launch_normals(uint64_t seed, uint64_t tag, uint64_t iter, uint64_t strm, int64_t n,
                    double* out, hipStream_t s, const uint64_t* iter_dev) {
  const int64_t nb = (n + 3) / 4;
  if (nb <= 0) return;
  k_normals<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(seed, tag, iter, iter_dev, strm, n, out);
}

// ---------------------------------------------------------------------------------
// scalar steps of the sweep (one thread)
// ---------------------------------------------------------------------------------
// derived scalars at the start of a sweep
__global__ void k_sweep_begin(DevState* st, DevState* prev) {
  if (prev) *prev = *st;
  st->alphaM = st->tau * st->sigf2;
  st->c_ka = sqrt(st->tau) * st->sigf2;
  st->sigf = sqrt(st->sigf2);
  st->tau_draw = st->tau;
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
__global__ void k_tau_step(DevState* st, int n, double a1, double b1, uint64_t seed,
                           uint64_t strm) {
  const uint64_t iter = st->iter;
  const double tau0 = st->tau_draw;
  st->logdet_sigma = st->logdetM - n * log(tau0);
  st->loglik = -0.5 * n * log(2.0 * M_PI) - 0.5 * st->logdet_sigma - 0.5 * st->yr;
  const double g = gamma_mt(0.5 * (a1 + n), seed, 3, iter, strm, &st->status);
  st->tau = g / (0.5 * (b1 + st->sse));
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

__global__ void k_sigf_step(DevState* st, int n, double a2, double b2, uint64_t seed,
                            uint64_t strm) {
  const uint64_t iter = st->iter;
  const double g = gamma_mt(0.5 * (a2 + n), seed, 4, iter, strm, &st->status);
  st->sigf2 = 1.0 / (g / (0.5 * (b2 + st->q)));
}

__global__ void k_mh_step(DevState* st, int kprop, int ongrid, uint64_t seed, uint64_t strm,
                          const int* pst_a, const int* pst_b) {
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
  k_rho_exact<<<1, 1, 0, s>>>(st, ld, q, G, seed, strm);
}

void launch_sweep_begin(DevState* st, DevState* prev, hipStream_t s) {
  k_sweep_begin<<<1, 1, 0, s>>>(st, prev);
}
void launch_set_draw_scalars(DevState* st, double tau, double sigf2, hipStream_t s) {
  k_set_draw_scalars<<<1, 1, 0, s>>>(st, tau, sigf2);
}
void launch_tau_step(DevState* st, int n, double a1, double b1, uint64_t seed, uint64_t strm,
                     hipStream_t s) {
  k_tau_step<<<1, 1, 0, s>>>(st, n, a1, b1, seed, strm);
}
void launch_tau_step_collapsed(DevState* st, int u, int64_t n_obs, double within, double a1,
                               double b1, uint64_t seed, uint64_t strm, hipStream_t s) {
  k_tau_step_collapsed<<<1, 1, 0, s>>>(st, u, n_obs, within, a1, b1, seed, strm);
}
void launch_sigf_step(DevState* st, int n, double a2, double b2, uint64_t seed, uint64_t strm,
                      hipStream_t s) {
  k_sigf_step<<<1, 1, 0, s>>>(st, n, a2, b2, seed, strm);
}
void launch_mh_step(DevState* st, int kprop, int ongrid, uint64_t seed, uint64_t strm,
                    const int* pst_a, const int* pst_b, hipStream_t s) {
  k_mh_step<<<1, 1, 0, s>>>(st, kprop, ongrid, seed, strm, pst_a, pst_b);
}

__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
void launch_zero_int(int* p, int n, hipStream_t s) {
  if (n > 0) k_zero_int<<<(n + 255) / 256, 256, 0, s>>>(p, n);
}

}  // namespace fg

// ---------------------------------------------------------------------------------
// PCG vector steps (one thread per row, all right-hand sides)
// ---------------------------------------------------------------------------------
namespace fg {

__global__ void k_pcg_init(int n, int nrhs, const double* __restrict__ b, int ld,
                           double* __restrict__ x, double* __restrict__ r, PcgScalars* sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void k_pcg_copy(int n, int nrhs, const double* __restrict__ a, double* __restrict__ o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) o[(size_t)c * n + i] = a[(size_t)c * n + i];
}

__global__ void k_pcg_xr(int n, int nrhs, double* __restrict__ x, int ld, double* __restrict__ r,
                         const double* __restrict__ p, const double* __restrict__ q,
                         const PcgScalars* __restrict__ sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || sc->done) return;
  for (int c = 0; c < nrhs; ++c) {
    const double a = sc->pq[c] != 0.0 ? sc->rz[c] / sc->pq[c] : 0.0;
    x[(size_t)c * ld + i] += a * p[(size_t)c * n + i];
    r[(size_t)c * n + i] -= a * q[(size_t)c * n + i];
  }
}

// p = z + (rz_new / rz) p; the ratio is formed before any thread can update rz, which
// is done by a second kernel
__global__ void k_pcg_p(int n, int nrhs, double* __restrict__ p, const double* __restrict__ z,
                        const PcgScalars* __restrict__ sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || sc->done) return;
  for (int c = 0; c < nrhs; ++c) {
    const double bt = sc->rz[c] != 0.0 ? sc->rz_new[c] / sc->rz[c] : 0.0;
    p[(size_t)c * n + i] = z[(size_t)c * n + i] + bt * p[(size_t)c * n + i];
  }
}

__global__ void k_pcg_rz(int nrhs, PcgScalars* sc) {
  const int c = threadIdx.x;
  if (c < nrhs && !sc->done) sc->rz[c] = sc->rz_new[c];
}

// the convergence test of iteration `it` (rr and bb hold |r|^2 and |b|^2 per column)
__global__ void k_pcg_check(int nrhs, double rtol, int it, PcgScalars* sc) {
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

static inline unsigned pblk(int n) { return (unsigned)((n + 255) / 256); }

void launch_pcg_init(int n, int nrhs, const double* b, int ld, double* x, double* r,
                     PcgScalars* sc, hipStream_t s) {
  k_pcg_init<<<std::max(pblk(n), 1u), 256, 0, s>>>(n, nrhs, b, ld, x, r, sc);
}
void launch_pcg_check(int nrhs, double rtol, int it, PcgScalars* sc, hipStream_t s) {
  k_pcg_check<<<1, 64, 0, s>>>(nrhs, rtol, it, sc);
}

__global__ void k_pcg_record(const PcgScalars* sc, DevState* st) {
  st->pcg_relres = sc->relres;
  st->pcg_iters = sc->iters;
  st->pcg_done = sc->done;
}
void launch_pcg_record(const PcgScalars* sc, DevState* st, hipStream_t s) {
  k_pcg_record<<<1, 1, 0, s>>>(sc, st);
}
void launch_pcg_copy(int n, int nrhs, const double* a, double* out, hipStream_t s) {
  if (n > 0) k_pcg_copy<<<pblk(n), 256, 0, s>>>(n, nrhs, a, out);
}
void launch_pcg_xr(int n, int nrhs, double* x, int ld, double* r, const double* p, const double* q,
                   const PcgScalars* sc, hipStream_t s) {
  if (n > 0) k_pcg_xr<<<pblk(n), 256, 0, s>>>(n, nrhs, x, ld, r, p, q, sc);
}
void launch_pcg_p(int n, int nrhs, double* p, const double* z, PcgScalars* sc, hipStream_t s) {
  if (n > 0) k_pcg_p<<<pblk(n), 256, 0, s>>>(n, nrhs, p, z, sc);
  k_pcg_rz<<<1, 64, 0, s>>>(nrhs, sc);
}

}  // namespace fg
