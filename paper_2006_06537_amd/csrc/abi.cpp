// extern "C" entry points of libfifagp (see include/fifa_gp.h for the contract).
#include <cmath>
#include <string>
#include <vector>

#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_tensor.h"
#include "fg_pcg.h"

namespace fg {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
}  // namespace fg

struct fg_hodlr_s {
  fg::PlanPack* pk = nullptr;
  fg::HodlrData d;
  fg::Caps caps;
};

struct fg_factor_s {
  fg::FactorData d;
  double* vecs = nullptr;  // n x 4 workspace (Algorithm 1 scratch)
  int n = 0;
};

namespace fg {
const HodlrData* hodlr_data(fg_hodlr A) { return &A->d; }
FactorData* factor_data(fg_factor F) { return &F->d; }
int factor_n(fg_factor F) { return F->n; }
}  // namespace fg

using fg::set_error;

static fg_status fail(fg_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static fg_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return FG_OK;
}

static fg_status status_word(int* dev, hipStream_t s) {
  int v = 0;
  if (hipStreamSynchronize(s) != hipSuccess) return fail(FG_EDEVICE, "stream synchronisation failed");
  if (hipMemcpy(&v, dev, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(FG_EDEVICE, "status read failed");
  if (v & fg::ST_NOTSPD) return fail(FG_ENOTSPD, "matrix not positive definite on the device");
  if (v & fg::ST_NOTCONV) return fail(FG_ENOTCONV, "a device iteration did not converge");
  if (v & fg::ST_TOL) return fail(FG_ETOL, "tolerance out of range");
  return FG_OK;
}

static fg_status copy_cols(double* dst, const double* src, int n, int nrhs, int64_t ld,
                           hipStream_t s) {
  if (dst == src) return FG_OK;
  if (hipMemcpy2DAsync(dst, ld * sizeof(double), src, ld * sizeof(double), n * sizeof(double),
                       nrhs, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(FG_EDEVICE, "device copy failed");
  return FG_OK;
}

extern "C" {

const char* fg_last_error(void) { return fg::g_err.c_str(); }

fg_status hodlr_build(const double* x, int64_t n, fg_kernel kernel, int32_t leaf, double tol,
                      fg_stream stream, fg_hodlr* out) {
  if (!out) return fail(FG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!x) return fail(FG_EINVAL, "x is NULL");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(FG_EINVAL, "n out of range");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<double> xh(n);
  if (hipMemcpyAsync(xh.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FG_EDEVICE, "copy of x to the host failed");
  fg_status st;
  std::string err;
  fg::PlanPack* pk = fg::plan_pack_create(xh.data(), int(n), kernel.kind, kernel.lengthscale,
                                          kernel.nugget, leaf, tol, s, st, err);
  if (!pk) return fail(st, err);
  fg_hodlr_s* A = new fg_hodlr_s();
  A->pk = pk;
  A->caps.add(*pk);
  if ((st = fg::hodlr_alloc(A->d, A->caps, err)) != FG_OK) {
    fg::plan_pack_destroy(pk);
    delete A;
    return fail(st, err);
  }
  A->d.pk = pk;
  if (hipMemcpyAsync(A->d.x, x, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    hodlr_destroy(A);
    return fail(FG_EDEVICE, "copy of x failed");
  }
  fg::launch_build(A->d, s);
  if ((st = check_launch("hodlr_build")) != FG_OK) { hodlr_destroy(A); return st; }
  *out = A;
  return FG_OK;
}

fg_status hodlr_info(fg_hodlr A, int32_t* levels, int64_t* n_out) {
  if (!A) return fail(FG_EINVAL, "NULL handle");
  if (levels) *levels = A->pk->P.L;
  if (n_out) *n_out = A->pk->P.n;
  return FG_OK;
}

fg_status hodlr_ranks(fg_hodlr A, int32_t* ranks, int32_t cap, int32_t* count, fg_stream stream) {
  if (!A) return fail(FG_EINVAL, "NULL handle");
  const int nint = A->pk->P.nint;
  if (count) *count = nint;
  if (nint == 0) return FG_OK;
  if (!ranks || cap < nint) return fail(FG_EINVAL, "ranks buffer too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(ranks, A->d.rank, nint * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(FG_EDEVICE, "rank copy failed");
  return FG_OK;
}

fg_status hodlr_singular_values(fg_hodlr A, double* sv, int32_t cap, fg_stream stream) {
  if (!A || !sv || cap < 1) return fail(FG_EINVAL, "bad arguments");
  const int nint = A->pk->P.nint;
  if (nint == 0) return FG_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<double> tmp((size_t)nint * fg::PMAX);
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(tmp.data(), A->d.sv, tmp.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(FG_EDEVICE, "copy failed");
  for (int h = 0; h < nint; ++h)
    for (int j = 0; j < cap; ++j) sv[(size_t)h * cap + j] = j < fg::PMAX ? tmp[(size_t)h * fg::PMAX + j] : 0.0;
  return FG_OK;
}

fg_status hodlr_entries(fg_hodlr A, const int64_t* i, const int64_t* j, int64_t count, double* out,
                        fg_stream stream) {
  if (!A || (count > 0 && (!i || !j || !out))) return fail(FG_EINVAL, "bad arguments");
  fg::launch_entries(A->d, i, j, count, out, reinterpret_cast<hipStream_t>(stream));
  return check_launch("hodlr_entries");
}

fg_status hodlr_matvec(fg_hodlr A, double alpha, double beta, const double* v, double* y,
                       int32_t nrhs, int64_t ld, fg_stream stream) {
  if (!A || !v || !y) return fail(FG_EINVAL, "NULL argument");
  const int n = A->pk->P.n;
  if (nrhs < 1 || ld < n) return fail(FG_EINVAL, "bad nrhs or ld");
  if (v == y) return fail(FG_EINVAL, "v and y must not overlap");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int c = 0; c < nrhs; c += 4) {
    const int nb = std::min(4, nrhs - c);
    fg::launch_matvec(A->d, alpha, beta, nullptr, nullptr, v + (size_t)c * ld, y + (size_t)c * ld,
                      nb, int(ld), A->d.work, s);
  }
  return check_launch("hodlr_matvec");
}

fg_status hodlr_factor_prec(fg_hodlr A, double alpha, double beta, const double* diag,
                            int32_t precision, fg_stream stream, fg_factor* out) {
  if (!out) return fail(FG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!A) return fail(FG_EINVAL, "NULL handle");
  if (precision != FG_FP64 && precision != FG_MIXED) return fail(FG_EINVAL, "bad precision");
  if (!(alpha > 0.0) || !(beta >= 0.0) || !std::isfinite(alpha) || !std::isfinite(beta))
    return fail(FG_EINVAL, "alpha must be > 0 and beta >= 0");
  std::string err;
  fg_factor_s* F = new fg_factor_s();
  fg_status st = fg::factor_alloc(F->d, A->caps, err, precision == FG_MIXED);
  if (st != FG_OK) { delete F; return fail(st, err); }
  F->n = A->pk->P.n;
  if (hipMalloc(reinterpret_cast<void**>(&F->vecs), sizeof(double) * 4 * (size_t)F->n) != hipSuccess) {
    factor_destroy(F);
    return fail(FG_ENOMEM, "workspace allocation failed");
  }
  F->d.H = &A->d;
  F->d.alpha = alpha;
  F->d.beta = beta;
  fg::launch_factor(F->d, nullptr, nullptr, diag, reinterpret_cast<hipStream_t>(stream));
  if ((st = check_launch("hodlr_factor")) != FG_OK) { factor_destroy(F); return st; }
  *out = F;
  return FG_OK;
}

fg_status hodlr_factor(fg_hodlr A, double alpha, double beta, const double* diag,
                       fg_stream stream, fg_factor* out) {
  return hodlr_factor_prec(A, alpha, beta, diag, FG_FP64, stream, out);
}

fg_status hodlr_solve_refined(fg_hodlr A, fg_factor F, double alpha, double beta,
                              const double* b, double* x, int32_t nrhs, int64_t ld, double rtol,
                              int32_t maxit, int32_t* iters, double* relres, fg_stream stream) {
  if (!A || !F || !b || !x) return fail(FG_EINVAL, "NULL argument");
  const int n = A->pk->P.n;
  if (F->n != n || F->d.H != &A->d) return fail(FG_EINVAL, "F is not a factor of A");
  if (nrhs < 1 || nrhs > fg::NRHS_PCG || ld < n) return fail(FG_EINVAL, "bad nrhs or ld");
  if (!(rtol > 0.0) || maxit < 1) return fail(FG_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (!(alpha > 0.0) || !(beta >= 0.0)) return fail(FG_EINVAL, "alpha must be > 0, beta >= 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  fg::PcgWork w;
  std::string err;
  fg_status st = fg::pcg_alloc(w, n, err);
  if (st != FG_OK) return fail(st, err);
  st = fg::pcg_solve(A->d, alpha, nullptr, beta, F->d, b, x, nrhs, int(ld), rtol, maxit, w, s,
                     iters, relres, err);
  (void)hipStreamSynchronize(s);
  fg::pcg_free(w);
  if (st != FG_OK) return fail(st, err);
  return check_launch("hodlr_solve_refined");
}

fg_status hodlr_solve(fg_factor F, const double* b, double* x, int32_t nrhs, int64_t ld,
                      fg_stream stream) {
  if (!F || !b || !x) return fail(FG_EINVAL, "NULL argument");
  const int n = F->n;
  if (nrhs < 1 || ld < n) return fail(FG_EINVAL, "bad nrhs or ld");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  fg_status st = copy_cols(x, b, n, nrhs, ld, s);
  if (st != FG_OK) return st;
  for (int c = 0; c < nrhs; c += 4) {
    const int nb = std::min(4, nrhs - c);
    fg::launch_apply_w(F->d, 2, x + (size_t)c * ld, nb, int(ld), F->d.work, s);
    fg::launch_apply_w(F->d, 3, x + (size_t)c * ld, nb, int(ld), F->d.work, s);
  }
  return check_launch("hodlr_solve");
}

fg_status hodlr_logdet(fg_factor F, double* logdet_dev, fg_stream stream) {
  if (!F || !logdet_dev) return fail(FG_EINVAL, "NULL argument");
  if (hipMemcpyAsync(logdet_dev, F->d.logdet, sizeof(double), hipMemcpyDeviceToDevice,
                     reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(FG_EDEVICE, "copy failed");
  return FG_OK;
}

fg_status hodlr_logdet_parts(fg_factor F, double* parts_dev, fg_stream stream) {
  if (!F || !parts_dev) return fail(FG_EINVAL, "NULL argument");
  fg::launch_logdet_parts(F->d, parts_dev, reinterpret_cast<hipStream_t>(stream));
  return check_launch("hodlr_logdet_parts");
}

fg_status hodlr_apply_w(fg_factor F, int32_t transpose, int32_t inverse, const double* v, double* y,
                        int32_t nrhs, int64_t ld, fg_stream stream) {
  if (!F || !v || !y) return fail(FG_EINVAL, "NULL argument");
  const int n = F->n;
  if (nrhs < 1 || ld < n) return fail(FG_EINVAL, "bad nrhs or ld");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  fg_status st = copy_cols(y, v, n, nrhs, ld, s);
  if (st != FG_OK) return st;
  const int op = (transpose ? 1 : 0) + (inverse ? 2 : 0);
  for (int c = 0; c < nrhs; c += 4) {
    const int nb = std::min(4, nrhs - c);
    fg::launch_apply_w(F->d, op, y + (size_t)c * ld, nb, int(ld), F->d.work, s);
  }
  return check_launch("hodlr_apply_w");
}

fg_status fg_normals(uint64_t seed, uint64_t tag, uint64_t iteration, uint64_t stream_id,
                     int64_t n, double* out, fg_stream stream) {
  if (n < 0 || (n > 0 && !out)) return fail(FG_EINVAL, "bad arguments");
  fg::launch_normals(seed, tag, iteration, stream_id, n, out, reinterpret_cast<hipStream_t>(stream));
  return check_launch("fg_normals");
}

fg_status gp_draw_f(fg_hodlr K1, fg_factor W1, fg_factor WM, double sigf2, double tau,
                    const double* y, uint64_t seed, uint64_t iteration, uint64_t stream_id,
                    double* f, double* r, double* mu, fg_stream stream) {
  if (!K1 || !W1 || !WM || !y || !f || !r) return fail(FG_EINVAL, "NULL argument");
  if (!(sigf2 > 0.0) || !(tau > 0.0)) return fail(FG_EINVAL, "sigf2 and tau must be > 0");
  const int n = K1->pk->P.n;
  if (W1->n != n || WM->n != n) return fail(FG_EINVAL, "size mismatch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* a = WM->vecs;
  double* b = a + n;
  double* z = b + n;  // columns z and z + n form the 2-RHS block [Z, tau y]
  fg::launch_normals(seed, 1, iteration, stream_id, n, a, s);
  fg::launch_normals(seed, 2, iteration, stream_id, n, b, s);
  fg::launch_matvec(K1->d, 1.0, 0.0, nullptr, nullptr, a, z, 1, n, K1->d.work, s);
  fg::launch_apply_w(W1->d, 0, b, 1, n, W1->d.work, s);
  fg::launch_axpby(n, z, b, z, nullptr, std::sqrt(tau) * sigf2, nullptr, std::sqrt(sigf2), s);
  fg::launch_axpby(n, y, nullptr, z + n, nullptr, tau, nullptr, 0.0, s);
  fg::launch_apply_w(WM->d, 2, z, 2, n, WM->d.work, s);
  fg::launch_apply_w(WM->d, 3, z, 2, n, WM->d.work, s);
  double* m = mu ? mu : a;
  fg::launch_matvec(K1->d, sigf2, 0.0, nullptr, nullptr, z + n, m, 1, n, K1->d.work, s);
  fg::launch_axpby(n, z, m, f, nullptr, 1.0, nullptr, 1.0, s);
  if (hipMemcpyAsync(r, z + n, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(FG_EDEVICE, "copy failed");
  return check_launch("gp_draw_f");
}

fg_status gp_draw_f_hetero(fg_hodlr K, fg_factor WK, fg_factor WP, const double* D,
                           const double* y, uint64_t seed, uint64_t iteration,
                           uint64_t stream_id, int32_t factor, double* f, double* R,
                           fg_stream stream) {
  if (!K || !WK || !WP || !D || !y || !f) return fail(FG_EINVAL, "NULL argument");
  if (factor < -1 || factor >= fg::TP_DMAX) return fail(FG_EINVAL, "factor out of range");
  const int n = K->pk->P.n;
  if (WK->n != n || WP->n != n) return fail(FG_EINVAL, "size mismatch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint64_t ta = factor < 0 ? 1 : fg::tp_factor_tag(1, factor);
  const uint64_t tb = factor < 0 ? 2 : fg::tp_factor_tag(2, factor);
  double* a = WP->vecs;
  double* b = a + n;
  double* z = b + n;  // columns z and z + n form the 2-RHS block [Z, y]
  fg::launch_normals(seed, ta, iteration, stream_id, n, a, s);
  fg::launch_scale_sqrt(n, D, a, s);
  fg::launch_normals(seed, tb, iteration, stream_id, n, b, s);
  fg::launch_matvec(K->d, 1.0, 0.0, nullptr, nullptr, a, z, 1, n, K->d.work, s);
  fg::launch_apply_w(WK->d, 0, b, 1, n, WK->d.work, s);
  fg::launch_axpby(n, z, b, z, nullptr, 1.0, nullptr, 1.0, s);
  if (hipMemcpyAsync(z + n, y, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(FG_EDEVICE, "copy failed");
  fg::launch_apply_w(WP->d, 2, z, 2, n, WP->d.work, s);
  fg::launch_apply_w(WP->d, 3, z, 2, n, WP->d.work, s);
  double* r = R ? R : a;
  fg::launch_matvec(K->d, 1.0, 0.0, nullptr, nullptr, z + n, r, 1, n, K->d.work, s);
  fg::launch_hetero_finish(n, r, z, D, f, nullptr, nullptr, s);
  return check_launch("gp_draw_f_hetero");
}

fg_status hodlr_status(fg_hodlr A, fg_stream stream) {
  if (!A) return fail(FG_EINVAL, "NULL handle");
  return status_word(A->d.status, reinterpret_cast<hipStream_t>(stream));
}

fg_status factor_status(fg_factor F, fg_stream stream) {
  if (!F) return fail(FG_EINVAL, "NULL handle");
  return status_word(F->d.status, reinterpret_cast<hipStream_t>(stream));
}

void hodlr_destroy(fg_hodlr A) {
  if (!A) return;
  (void)hipDeviceSynchronize();
  fg::hodlr_free(A->d);
  fg::plan_pack_destroy(A->pk);
  delete A;
}

void factor_destroy(fg_factor F) {
  if (!F) return;
  (void)hipDeviceSynchronize();
  fg::factor_free(F->d);
  if (F->vecs) (void)hipFree(F->vecs);
  delete F;
}

}  // extern "C"
