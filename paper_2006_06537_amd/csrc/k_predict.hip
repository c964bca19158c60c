// Function posterior at new inputs (Appendix, "Function posterior at new inputs").
// With z_f = W_1^-1 f and Z = W_1^-1 k1(X, X*) (K~_1 = W_1 W_1'), each new point j has
//   mu*_j = Z_j . z_f,   s2*_j = sigma_f^2 (1 + eta - |Z_j|^2),
//   f*_j  = mu*_j + sqrt(max(s2*_j, 0)) xi_j.
// The products go through the factor, so K~_1^-1 f (whose entries grow like 1/eta) is
// never formed.
#include "fg_internal.h"
#include "fg_rng.h"

namespace fg {

// Z[i + j ld] = k1(x_i, x*_(j0 + j)) for the columns of one launch (blockIdx.y = j)
__global__ void __launch_bounds__(NTHREADS) k_cross_cov(const double* __restrict__ x, int n,
                                                        const double* __restrict__ xstar,
                                                        int j0, int kind, double ell,
                                                        double* __restrict__ Z, int64_t ld) {
  const int j = j0 + (int)blockIdx.y;
  const double xs = xstar[j];
  double* col = Z + (size_t)j * (size_t)ld;
  for (int i = blockIdx.x * NTHREADS + threadIdx.x; i < n; i += gridDim.x * NTHREADS)
    col[i] = k1_value(kind, ell, x[i], xs);
}

__device__ __forceinline__ double wave_total(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// one work-group per new point: the two length-n reductions in a fixed order
__global__ void __launch_bounds__(NTHREADS) k_predict_point(
    const double* __restrict__ Z, int64_t ld, int n, const double* __restrict__ zf,
    const double* __restrict__ xi, const double* __restrict__ sigf2_p, double eta, int nstar,
    double* __restrict__ fstar, double* __restrict__ mu, double* __restrict__ s2) {
  const int j = blockIdx.x;
  if (j >= nstar) return;
  const double* col = Z + (size_t)j * (size_t)ld;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += NTHREADS) {
    const double z = col[i];
    a += z * zf[i];
    b += z * z;
  }
  a = wave_total(a);
  b = wave_total(b);
  __shared__ double ra[NTHREADS / 64], rb[NTHREADS / 64];
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = a;
    rb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) {
      ta += ra[w];
      tb += rb[w];
    }
    const double v = (*sigf2_p) * (1.0 + eta - tb);
    fstar[j] = ta + sqrt(fmax(v, 0.0)) * xi[j];
    if (mu) mu[j] = ta;
    if (s2) s2[j] = v;
  }
}

void launch_cross_cov(const double* x, int n, const double* xstar, int nstar, int kind,
                      double ell, double* Z, int64_t ld, hipStream_t s) {
  const int gx = std::max(1, std::min((n + NTHREADS * 4 - 1) / (NTHREADS * 4), 4096));
  for (int j0 = 0; j0 < nstar; j0 += 65535) {
    const int nj = std::min(65535, nstar - j0);
    k_cross_cov<<<dim3(gx, nj), NTHREADS, 0, s>>>(x, n, xstar, j0, kind, ell, Z, ld);
  }
}

void launch_predict_point(const double* Z, int64_t ld, int n, const double* zf, const double* xi,
                          const double* sigf2_p, double eta, int nstar, double* fstar,
                          double* mu, double* s2, hipStream_t s) {
  k_predict_point<<<nstar, NTHREADS, 0, s>>>(Z, ld, n, zf, xi, sigf2_p, eta, nstar, fstar, mu, s2);
}

}  // namespace fg
