// Preconditioned conjugate gradients (internal).
#pragma once
#include <string>

#include "fg_internal.h"

namespace fg {

constexpr int NRHS_PCG = 4;

struct PcgScalars {  // per right-hand side
  double bb[NRHS_PCG], rz[NRHS_PCG], rz_new[NRHS_PCG], pq[NRHS_PCG], rr[NRHS_PCG];
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

// Solves (alpha K~_1 + beta I) x = b (nrhs <= 4 columns, ld >= n; alpha from alpha_dev when
// given) by PCG preconditioned with M; synchronises the stream once per iteration from
// iteration min_iters on.
// FG_ENOTCONV if the relative residual is still above rtol after maxit iterations.
fg_status pcg_solve(const HodlrData& H, double alpha, const double* alpha_dev, double beta,
                    FactorData& M, const double* b, double* x, int nrhs, int ld, double rtol,
                    int maxit, PcgWork& w, hipStream_t s, int* iters, double* relres,
                    std::string& err, int min_iters = 1);

// vector kernels (k_rng.hip): r and the PCG vectors use leading dimension n
void launch_pcg_init(int n, int nrhs, const double* b, int ld, double* x, double* r, hipStream_t s);
void launch_pcg_copy(int n, int nrhs, const double* a, double* out, hipStream_t s);
void launch_pcg_xr(int n, int nrhs, double* x, int ld, double* r, const double* p, const double* q,
                   const PcgScalars* sc, hipStream_t s);
void launch_pcg_p(int n, int nrhs, double* p, const double* z, PcgScalars* sc, hipStream_t s);

}  // namespace fg
