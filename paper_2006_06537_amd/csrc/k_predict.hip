// Function posterior at new inputs (Appendix, "Function posterior at new inputs").
// With z_f = W_1^-1 f and Z = W_1^-1 k1(X, X*) (K~_1 = W_1 W_1'), each new point j has
//   mu*_j = Z_j . z_f,   s2*_j = sigma_f^2 (1 + eta - |Z_j|^2),
//   f*_j  = mu*_j + sqrt(max(s2*_j, 0)) xi_j.
// The products go through the factor, so K~_1^-1 f (whose entries grow like 1/eta) is
// never formed.
#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_timer.h"

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

// Stage 1: work-group (chunk, group) takes PT_ROWS rows of PC new points, so each
// slice of z_f is read once for PC columns of Z.  Partial sums go to
// part[(chunk * nstar + j) * 2 + {0: Z_j . z_f, 1: |Z_j|^2}].
constexpr int PT_ROWS = 16384;  // measured best with 4 points per work-group (5.9 TB/s at n = 2^20)

template <int PC>
__global__ void __launch_bounds__(NTHREADS) k_predict_partial(
    const double* __restrict__ Z, int64_t ld, int n, const double* __restrict__ zf, int nstar,
    double* __restrict__ part) {
  const int chunk = blockIdx.x, j0 = blockIdx.y * PC;
  const int r0 = chunk * PT_ROWS, r1 = min(r0 + PT_ROWS, n);
  const int pc = min(PC, nstar - j0);
  double a[PC], b[PC];
#pragma unroll
  for (int c = 0; c < PC; ++c) a[c] = b[c] = 0.0;
  const double* col = Z + (size_t)j0 * (size_t)ld;
  for (int i = r0 + threadIdx.x; i < r1; i += NTHREADS) {
    const double z = zf[i];
#pragma unroll
    for (int c = 0; c < PC; ++c) {
      if (c < pc) {
        const double v = col[(size_t)c * (size_t)ld + i];
        a[c] += v * z;
        b[c] += v * v;
      }
    }
  }
  __shared__ double red[NTHREADS / 64][2 * PC];
#pragma unroll
  for (int c = 0; c < PC; ++c) {
    a[c] = wave_total(a[c]);
    b[c] = wave_total(b[c]);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < PC; ++c) {
      red[threadIdx.x >> 6][2 * c] = a[c];
      red[threadIdx.x >> 6][2 * c + 1] = b[c];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * pc) {
    double t = 0.0;
    for (int w = 0; w < NTHREADS / 64; ++w) t += red[w][threadIdx.x];
    part[((size_t)chunk * nstar + j0 + (threadIdx.x >> 1)) * 2 + (threadIdx.x & 1)] = t;
  }
}

// Stage 2: one thread per new point sums its chunk partials in chunk order.
__global__ void __launch_bounds__(NTHREADS) k_predict_final(
    const double* __restrict__ part, int nchunk, int nstar, const double* __restrict__ xi,
    const double* __restrict__ sigf2_p, double eta, double* __restrict__ fstar,
    double* __restrict__ mu, double* __restrict__ s2) {
  const int j = blockIdx.x * NTHREADS + threadIdx.x;
  if (j >= nstar) return;
  double ta = 0.0, tb = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    ta += part[((size_t)c * nstar + j) * 2];
    tb += part[((size_t)c * nstar + j) * 2 + 1];
  }
  const double v = (*sigf2_p) * (1.0 + eta - tb);
  fstar[j] = ta + sqrt(fmax(v, 0.0)) * xi[j];
  if (mu) mu[j] = ta;
  if (s2) s2[j] = v;
}

void launch_cross_cov(const double* x, int n, const double* xstar, int nstar, int kind,
                      double ell, double* Z, int64_t ld, hipStream_t s) {
  const int gx = std::max(1, std::min((n + NTHREADS * 4 - 1) / (NTHREADS * 4), 4096));
  for (int j0 = 0; j0 < nstar; j0 += 65535) {
    const int nj = std::min(65535, nstar - j0);
    k_cross_cov<<<dim3(gx, nj), NTHREADS, 0, s>>>(x, n, xstar, j0, kind, ell, Z, ld);
  }
}

size_t predict_part_doubles(int n, int nstar) {
  return (size_t)((n + PT_ROWS - 1) / PT_ROWS) * (size_t)nstar * 2;
}

void launch_predict_point(const double* Z, int64_t ld, int n, const double* zf, const double* xi,
                          const double* sigf2_p, double eta, int nstar, double* part,
                          double* fstar, double* mu, double* s2, hipStream_t s) {
  const int nchunk = (n + PT_ROWS - 1) / PT_ROWS;
  // algorithmic bytes: Z read once, z_f and the normals read, three outputs written
  timer_before_bytes(KID_PREDICT, s, 8.0 * ((double)n * nstar + n + 4.0 * nstar));
  const int ng = (nstar + PC_PREDICT - 1) / PC_PREDICT;  // <= 65535 (checked by the caller)
  k_predict_partial<PC_PREDICT><<<dim3(nchunk, ng), NTHREADS, 0, s>>>(Z, ld, n, zf, nstar, part);
  timer_after(KID_PREDICT, s);
  k_predict_final<<<(nstar + NTHREADS - 1) / NTHREADS, NTHREADS, 0, s>>>(
      part, nchunk, nstar, xi, sigf2_p, eta, fstar, mu, s2);
}

}  // namespace fg
