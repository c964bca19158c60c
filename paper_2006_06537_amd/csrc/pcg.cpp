// Preconditioned conjugate gradients on A = alpha K~_1 + beta I with the symmetric factor
// of (an approximation of) A as preconditioner, z = W^-T W^-1 r.  With a factor held in
// FP32 this is the refinement that brings an FP32-factored solve back to FP64 accuracy:
// every product with A uses the FP64 HODLR matrix, every residual and inner product is
// FP64, and the iteration stops once |b - A x| <= rtol |b| for every right-hand side.
// The stopping test reads one small vector on the host per iteration, from iteration
// min_iters on (a caller that knows roughly how many iterations it needs skips the
// earlier round trips).
#include <cmath>
#include <string>

#include "fg_internal.h"
#include "fg_pcg.h"

namespace fg {

fg_status pcg_alloc(PcgWork& w, int n, std::string& err) {
  const size_t nv = (size_t)NRHS_PCG * n;
  if (hipMalloc(reinterpret_cast<void**>(&w.r), sizeof(double) * nv) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w.z), sizeof(double) * nv) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w.p), sizeof(double) * nv) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w.q), sizeof(double) * nv) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w.dotwork), sizeof(double) * 1024 * 4 * NRHS_PCG) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w.sc), sizeof(PcgScalars)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&w.sc_host), sizeof(PcgScalars)) != hipSuccess) {
    pcg_free(w);
    err = "PCG workspace allocation failed";
    return FG_ENOMEM;
  }
  w.n = n;
  return FG_OK;
}

void pcg_free(PcgWork& w) {
  double* b[] = {w.r, w.z, w.p, w.q, w.dotwork};
  for (double* p : b)
    if (p) (void)hipFree(p);
  if (w.sc) (void)hipFree(w.sc);
  if (w.sc_host) (void)hipHostFree(w.sc_host);
  w = PcgWork{};
}

fg_status pcg_solve(const HodlrData& H, double alpha, const double* alpha_dev, double beta,
                    FactorData& M, const double* b, double* x, int nrhs, int ld, double rtol,
                    int maxit, PcgWork& w, hipStream_t s, int* iters, double* relres,
                    std::string& err, int min_iters) {
  const int n = H.pk->P.n;
  if (nrhs < 1 || nrhs > NRHS_PCG || ld < n || w.n < n) {
    err = "pcg: bad nrhs, ld or workspace";
    return FG_EINVAL;
  }
  double* const r = w.r;
  double* const z = w.z;
  double* const p = w.p;
  double* const q = w.q;
  auto dots = [&](const double* a, const double* bb, double* out) {
    for (int c = 0; c < nrhs; ++c)
      launch_dot(a + (size_t)c * n, bb + (size_t)c * n, n, 0, out + c, w.dotwork + 1024 * c, s);
  };
  // x = 0, r = b, |b|^2
  launch_pcg_init(n, nrhs, b, ld, x, r, s);
  dots(r, r, w.sc->bb);
  // z = M^-1 r, p = z, rz = r'z
  launch_pcg_copy(n, nrhs, r, z, s);
  launch_apply_w(M, 2, z, nrhs, n, M.work, s);
  launch_apply_w(M, 3, z, nrhs, n, M.work, s);
  launch_pcg_copy(n, nrhs, z, p, s);
  dots(r, z, w.sc->rz);
  int it = 0;
  double worst = 1.0;
  for (it = 1; it <= maxit; ++it) {
    launch_matvec(H, alpha, beta, alpha_dev, nullptr, p, q, nrhs, n, H.work, s);
    dots(p, q, w.sc->pq);
    launch_pcg_xr(n, nrhs, x, ld, r, p, q, w.sc, s);  // x += a p, r -= a q
    dots(r, r, w.sc->rr);
    if (it < min_iters && it < maxit) {  // no residual test yet: keep the stream busy
      launch_pcg_copy(n, nrhs, r, z, s);
      launch_apply_w(M, 2, z, nrhs, n, M.work, s);
      launch_apply_w(M, 3, z, nrhs, n, M.work, s);
      dots(r, z, w.sc->rz_new);
      launch_pcg_p(n, nrhs, p, z, w.sc, s);
      continue;
    }
    hipMemcpyAsync(w.sc_host, w.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
      err = "pcg: device failure";
      return FG_EDEVICE;
    }
    worst = 0.0;
    bool finite = true;
    for (int c = 0; c < nrhs; ++c) {
      const double bn = w.sc_host->bb[c], rn = w.sc_host->rr[c];
      if (!std::isfinite(bn) || !std::isfinite(rn)) finite = false;
      const double rel = bn > 0.0 ? std::sqrt(rn / bn) : 0.0;
      if (!(rel <= worst)) worst = rel;  // NaN propagates
    }
    if (!finite) {
      worst = NAN;
      break;
    }
    if (worst <= rtol) break;
    launch_pcg_copy(n, nrhs, r, z, s);
    launch_apply_w(M, 2, z, nrhs, n, M.work, s);
    launch_apply_w(M, 3, z, nrhs, n, M.work, s);
    dots(r, z, w.sc->rz_new);
    launch_pcg_p(n, nrhs, p, z, w.sc, s);  // p = z + (rz_new / rz) p; rz = rz_new
  }
  if (iters) *iters = std::min(it, maxit);
  if (relres) *relres = worst;
  if (std::isnan(worst) || worst > rtol) {
    err = "pcg: no convergence to the requested residual";
    return FG_ENOTCONV;
  }
  return FG_OK;
}

}  // namespace fg
