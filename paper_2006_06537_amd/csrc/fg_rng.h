// Philox4x64-10 and the sampler's device state (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fg_internal.h"

namespace fg {

__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
}

// Philox4x64 with 10 rounds; counter (c0..c3), key (k0, k1); out[4].
__host__ __device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// 52-bit uniform strictly inside (0, 1); every step is exact in FP64.
__host__ __device__ inline double to_unit(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

// Gamma(shape, 1) by Marsaglia & Tsang (ACM TOMS 26(3), 2000): try t uses block t of
// the counter, z from (u0, u1) by the cosine branch, acceptance uniform u2; shape < 1
// takes Gamma(shape + 1) u3^(1/shape).  At most 64 tries (then ST_NOTCONV).
__device__ inline double gamma_mt(double shape, uint64_t seed, uint64_t tag, uint64_t iter,
                           uint64_t strm, int* status) {
  const bool boost = shape < 1.0;
  const double a = boost ? shape + 1.0 : shape;
  const double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
  for (int t = 0; t < 64; ++t) {
    uint64_t w[4];
    philox4x64_10((uint64_t)t, tag, iter, strm, seed, 0, w);
    const double u0 = to_unit(w[0]), u1 = to_unit(w[1]), u2 = to_unit(w[2]), u3 = to_unit(w[3]);
    const double z = sqrt(-2.0 * log(u0)) * cos(2.0 * M_PI * u1);
    double v = 1.0 + c * z;
    if (v <= 0.0) continue;
    v = v * v * v;
    if (log(u2) < 0.5 * z * z + d - d * v + d * log(v)) {
      double g = d * v;
      if (boost) g *= pow(u3, 1.0 / shape);
      return g;
    }
  }
  atomicOr(status, ST_NOTCONV);
  return d;
}

// Scalars of one chain kept in device memory so that a sweep needs no host round trip.
struct DevState {
  double tau, sigf2;          // current tau and sigma_f^2
  double alphaM, c_ka, sigf;  // tau*sigf2, sqrt(tau)*sigf2, sqrt(sigf2) at the f draw
  double tau_draw;            // tau used by the f draw
  double sse, q, qprop, yr;
  double logdetM, logdet1, logdet1p;
  double logdet_sigma, loglik, mh;
  uint64_t iter;              // sweeps completed (the Philox iteration word)
  int k, kprop, accept, accepts, status, pad;
  double pcg_relres;          // mixed precision: the f-draw's PCG record (0 in FP64)
  int pcg_iters, pcg_done;
};

// Starts a sweep (the draw's scalars from tau and sigma_f^2); when `prev` is not null it
// first keeps a copy of the state there, from which the sweep can be run again.
void launch_sweep_begin(DevState* st, DevState* prev, hipStream_t s);
struct PcgScalars;
// copies a PCG solve's convergence record into the state (pcg_done = -1 when the status word
// fstatus of the preconditioning factor, if given, reports a non-positive pivot)
void launch_pcg_record(const PcgScalars* sc, DevState* st, const int* fstatus, hipStream_t s);
void launch_set_draw_scalars(DevState* st, double tau, double sigf2, hipStream_t s);
// the steps below take the iteration word from st->iter; the Metropolis step ends the
// sweep and advances it
void launch_tau_step(DevState* st, int n, double a1, double b1, uint64_t seed, uint64_t strm,
                     hipStream_t s);
void launch_sigf_step(DevState* st, int n, double a2, double b2, uint64_t seed, uint64_t strm,
                      hipStream_t s);
void launch_rho_exact(DevState* st, const double* ld, const double* q, int G, uint64_t seed,
                      uint64_t strm, hipStream_t s);
void launch_tau_step_collapsed(DevState* st, int u, int64_t n_obs, double within, double a1,
                               double b1, uint64_t seed, uint64_t strm, hipStream_t s);
void launch_mh_step(DevState* st, int kprop, int ongrid, uint64_t seed, uint64_t strm,
                    const int* pst_a, const int* pst_b, hipStream_t s);
void launch_zero_int(int* p, int n, hipStream_t s);

}  // namespace fg
