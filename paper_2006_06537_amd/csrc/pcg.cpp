// Preconditioned conjugate gradients on A = alpha K~_1 + beta I with the symmetric factor
// of (an approximation of) A as preconditioner, z = W^-T W^-1 r.  With a factor held in
// FP32 this is the refinement that brings an FP32-factored solve back to FP64 accuracy:
// every product with A uses the FP64 HODLR matrix, every residual and inner product is
// FP64, and the iteration stops once |b - A x| <= rtol |b| for every right-hand side.
// The stopping test runs on the device: a solve can be enqueued (and captured) as a
// fixed number of iterations whose updates stop at convergence.
#include <algorithm>
#include <cmath>
#include <string>

#include "fg_internal.h"
#include "fg_pcg.h"

namespace fg {

fg_status pcg_alloc(PcgWork& w, int n, std::string& err) {
  const size_t nv = (size_t)NRHS_PCG * n;
  if (dev_alloc(reinterpret_cast<void**>(&w.r), sizeof(double) * nv) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&w.z), sizeof(double) * nv) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&w.p), sizeof(double) * nv) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&w.q), sizeof(double) * nv) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&w.dotwork), sizeof(double) * 1024 * 4 * NRHS_PCG) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&w.sc), sizeof(PcgScalars)) != hipSuccess ||
      host_alloc(reinterpret_cast<void**>(&w.sc_host), sizeof(PcgScalars)) != hipSuccess) {
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
    if (p) dev_free(p);
  if (w.sc) dev_free(w.sc);
  if (w.sc_host) host_free(w.sc_host);
  w = PcgWork{};
}

void pcg_enqueue(const HodlrData& H, double alpha, const double* alpha_dev, double beta,
                 FactorData& M, const double* b, double* x, int nrhs, int ld, double rtol,
                 int it0, int count, PcgWork& w, hipStream_t s, bool final) {
  const int n = H.pk->P.n;
  double* const r = w.r;
  double* const z = w.z;
  double* const p = w.p;
  double* const q = w.q;
  auto dots = [&](const double* a, const double* bb, double* out) {
    for (int c = 0; c < nrhs; ++c)
      launch_dot(a + (size_t)c * n, bb + (size_t)c * n, n, 0, out + c, w.dotwork + 1024 * c, s);
  };
  auto precondition = [&]() {  // z = M^-1 r = W^-T W^-1 r
    launch_pcg_copy(n, nrhs, r, z, s);
    launch_apply_w(M, 2, z, nrhs, n, M.work, s);
    launch_apply_w(M, 3, z, nrhs, n, M.work, s);
  };
  if (it0 == 0) {
    // x = 0, r = b, |b|^2;  z = M^-1 r, p = z, rz = r'z
    launch_pcg_init(n, nrhs, b, ld, x, r, w.sc, s);
    dots(r, r, w.sc->bb);
    precondition();
    launch_pcg_copy(n, nrhs, z, p, s);
    dots(r, z, w.sc->rz);
  }
  for (int it = it0 + 1; it <= it0 + count; ++it) {
    launch_matvec(H, alpha, beta, alpha_dev, nullptr, p, q, nrhs, n, H.work, s);
    dots(p, q, w.sc->pq);
    launch_pcg_xr(n, nrhs, x, ld, r, p, q, w.sc, s);  // x += a p, r -= a q
    dots(r, r, w.sc->rr);
    launch_pcg_check(nrhs, rtol, it, w.sc, s);
    // the next direction (also after the last iteration of a chunk: a later chunk
    // continues from it; not after the last iteration of a final chunk)
    if (final && it == it0 + count) break;
    precondition();
    dots(r, z, w.sc->rz_new);
    launch_pcg_p(n, nrhs, p, z, w.sc, s);  // p = z + (rz_new / rz) p; rz = rz_new
  }
}

fg_status pcg_solve(const HodlrData& H, double alpha, const double* alpha_dev, double beta,
                    FactorData& M, const double* b, double* x, int nrhs, int ld, double rtol,
                    int maxit, PcgWork& w, hipStream_t s, int* iters, double* relres,
                    std::string& err) {
  const int n = H.pk->P.n;
  if (nrhs < 1 || nrhs > NRHS_PCG || ld < n || w.n < n) {
    err = "pcg: bad nrhs, ld or workspace";
    return FG_EINVAL;
  }
  constexpr int CHUNK = 4;
  int it = 0;
  for (;;) {
    const int cnt = std::min(CHUNK, maxit - it);
    pcg_enqueue(H, alpha, alpha_dev, beta, M, b, x, nrhs, ld, rtol, it, cnt, w, s, false);
    it += cnt;
    hipMemcpyAsync(w.sc_host, w.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
      err = "pcg: device failure";
      return FG_EDEVICE;
    }
    if (w.sc_host->done != 0 || it >= maxit) break;
  }
  if (iters) *iters = w.sc_host->iters;
  if (relres) *relres = w.sc_host->relres;
  if (w.sc_host->done != 1) {
    err = "pcg: no convergence to the requested residual";
    return FG_ENOTCONV;
  }
  return FG_OK;
}

}  // namespace fg
