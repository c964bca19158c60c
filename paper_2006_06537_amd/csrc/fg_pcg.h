// Preconditioned conjugate gradients (internal).
#pragma once
#include <string>

#include "fg_internal.h"

namespace fg {

constexpr int NRHS_PCG = 4;

struct PcgScalars {  // per right-hand side, then the solve's convergence record
  double bb[NRHS_PCG], rz[NRHS_PCG], rz_new[NRHS_PCG], pq[NRHS_PCG], rr[NRHS_PCG];
  double relres;      // largest relative residual after the last active iteration
  int done;           // 0 running; 1 converged; -1 stopped on a non-finite residual
  int iters;          // iterations taken (the iteration that converged, or the last one)
};

struct PcgWork {
  int n = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;  // NRHS_PCG x n each
  double* dotwork = nullptr;
  PcgScalars* sc = nullptr;
  PcgScalars* sc_host = nullptr;  // pinned
};

fg_status pcg_alloc(PcgWork& w, int n, std::string& err);
void pcg_free(PcgWork& w);

// Enqueues PCG on (alpha K~_1 + beta I) x = b (nrhs <= 4 columns, ld >= n; alpha from
// alpha_dev when given), preconditioned with M, with no host round trip: the set-up, then
// iterations it0 + 1 .. it0 + count (it0 = 0 starts a new solve).  The convergence test
// runs on the device after each iteration; once every column's relative residual is at
// most rtol (or a residual is not finite) the record in w.sc is closed and the remaining
// iterations leave x untouched, so the result equals that of a solve stopped at the
// converged iteration, whatever `count` is.  Capturable in a graph.  `final`: no chunk
// follows, so the last iteration skips forming the next search direction.
void pcg_enqueue(const HodlrData& H, double alpha, const double* alpha_dev, double beta,
                 FactorData& M, const double* b, double* x, int nrhs, int ld, double rtol,
                 int it0, int count, PcgWork& w, hipStream_t s, bool final);

// The same solve run to convergence from the host: iterations are enqueued in chunks and
// the record read back after each (one synchronisation per chunk).  FG_ENOTCONV if the
// relative residual is still above rtol after maxit iterations.
fg_status pcg_solve(const HodlrData& H, double alpha, const double* alpha_dev, double beta,
                    FactorData& M, const double* b, double* x, int nrhs, int ld, double rtol,
                    int maxit, PcgWork& w, hipStream_t s, int* iters, double* relres,
                    std::string& err);

// vector kernels (k_rng.hip): r and the PCG vectors use leading dimension n; the x, r and
// p updates do nothing once the record says done
void launch_pcg_init(int n, int nrhs, const double* b, int ld, double* x, double* r,
                     PcgScalars* sc, hipStream_t s);
void launch_pcg_copy(int n, int nrhs, const double* a, double* out, hipStream_t s);
void launch_pcg_xr(int n, int nrhs, double* x, int ld, double* r, const double* p, const double* q,
                   const PcgScalars* sc, hipStream_t s);
void launch_pcg_p(int n, int nrhs, double* p, const double* z, PcgScalars* sc, hipStream_t s);
// after iteration `it`: close the record if every column has |r| <= rtol |b|
void launch_pcg_check(int nrhs, double rtol, int it, PcgScalars* sc, hipStream_t s);

}  // namespace fg
