// Tensor-product surface chain on the device (Section 4.2): y_i = beta prod_h f_h(x[h,i])
// + e_i with unit-variance GP factors, or a sum of C such products (additive tensor
// products, Sections 4.2 and 5.2).  One sweep draws, component by component, the
// factors f_{c,1..d} in turn by Algorithm 1.h (Appendix) on the partial residual and then
// beta_c; then tau; then each factor's length-scale by the grid Metropolis step.  Per
// factor m = c d + h the chain keeps two slots of (K~_m, W_m) -- current length-scale and
// proposal -- and one shared factor of P~ = K~_m + D^-1 (the factors are drawn one after
// the other, so one buffer serves all of them).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_tensor.h"

struct fg_tp_chain_s {
  fg_tp_cfg cfg{};
  int n = 0, d = 0;
  int C = 1, nf = 0;                               // components, factors (C d)
  std::vector<std::vector<double>> grid;           // per factor
  std::vector<std::vector<fg::PlanPack*>> packs;   // per factor, per grid point
  fg::Caps caps;
  fg::HodlrData H[fg::TP_DMAX][2];
  fg::FactorData W[fg::TP_DMAX][2];
  fg::FactorData WP;
  int cur[fg::TP_DMAX] = {};
  int k[fg::TP_DMAX] = {};
  int64_t iter = 0;
  int* perm = nullptr;     // d x n: sorted position -> observation index
  double* F = nullptr;     // nf x n, observation order
  double* fs = nullptr;    // nf x n, sorted order of each factor's dimension
  double* Gc = nullptr;    // C x n: prod_h f_{c,h}, observation order
  double* R = nullptr;     // n: partial residual of the component being drawn
  double* y = nullptr;     // n
  double* vecs = nullptr;  // 8 n: D, Dinv, y~, G, and four work vectors
  double* dotwork = nullptr;
  fg::TpState* st = nullptr;
  fg::TpState* st_host = nullptr;
  hipStream_t aux = nullptr;  // proposals' builds and factors, beside the draws
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

using fg::set_error;

static fg_status tfail(fg_status st, const std::string& m) {
  set_error(m);
  return st;
}

static void tp_free(fg_tp_chain c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  for (int h = 0; h < fg::TP_DMAX; ++h)
    for (int i = 0; i < 2; ++i) { fg::hodlr_free(c->H[h][i]); fg::factor_free(c->W[h][i]); }
  fg::factor_free(c->WP);
  for (auto& v : c->packs)
    for (auto* p : v) fg::plan_pack_destroy(p);
  void* bufs[] = {c->perm, c->F, c->fs, c->y, c->vecs, c->dotwork, c->st, c->Gc, c->R};
  for (void* b : bufs)
    if (b) fg::dev_free(b);
  if (c->st_host) fg::host_free(c->st_host);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
}

extern "C" {

fg_status tp_chain_create(const fg_tp_cfg* cfg, const double* x, const double* y, int64_t n,
                          fg_stream stream, fg_tp_chain* out) {
  if (!out) return tfail(FG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || !x || !y) return tfail(FG_EINVAL, "NULL argument");
  if (cfg->d < 1 || cfg->d > fg::TP_DMAX) return tfail(FG_EINVAL, "d must be in 1..8");
  const int ncomp = cfg->ncomp == 0 ? 1 : cfg->ncomp;
  if (ncomp < 1 || ncomp > fg::TP_CMAX || ncomp * cfg->d > fg::TP_DMAX)
    return tfail(FG_EINVAL, "ncomp must be in 1..4 with ncomp * d <= 8");
  if (n < 1 || n >= (int64_t(1) << 31) / fg::TP_DMAX) return tfail(FG_EINVAL, "n out of range");
  if (cfg->grid_size < 1 || cfg->grid_center < 0 || cfg->grid_center >= cfg->grid_size)
    return tfail(FG_EINVAL, "bad grid");
  if (!(cfg->tau0 > 0) || !std::isfinite(cfg->beta0) || !(cfg->s_beta > 0))
    return tfail(FG_EINVAL, "tau0 and s_beta must be > 0, beta0 finite");
  for (int m = 0; m < ncomp * cfg->d; ++m)
    if (!(cfg->ell0[m] > 0)) return tfail(FG_EINVAL, "ell0 must be > 0 for every factor");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int d = cfg->d, nn = int(n);
  std::vector<double> xh((size_t)d * nn);
  if (hipMemcpyAsync(xh.data(), x, xh.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return tfail(FG_EDEVICE, "copy of x to the host failed");
  for (double v : xh)
    if (!std::isfinite(v)) return tfail(FG_EINVAL, "x must be finite");
  fg_tp_chain c = new fg_tp_chain_s();
  c->cfg = *cfg;
  c->n = nn;
  c->d = d;
  c->C = ncomp;
  c->nf = ncomp * d;
  const int nf = c->nf;
  // per-dimension ascending order (stable, so ties keep observation order)
  std::vector<int> permh((size_t)d * nn);
  std::vector<double> xs((size_t)d * nn);
  for (int h = 0; h < d; ++h) {
    int* p = permh.data() + (size_t)h * nn;
    const double* xr = xh.data() + (size_t)h * nn;
    std::iota(p, p + nn, 0);
    std::stable_sort(p, p + nn, [xr](int a, int b) { return xr[a] < xr[b]; });
    for (int j = 0; j < nn; ++j) xs[(size_t)h * nn + j] = xr[p[j]];
  }
  fg_status st;
  std::string err;
  c->grid.resize(nf);
  c->packs.resize(nf);
  for (int m = 0; m < nf; ++m) {
    const int h = m % d;
    c->grid[m].resize(cfg->grid_size);
    for (int g = 0; g < cfg->grid_size; ++g) {
      c->grid[m][g] = cfg->ell0[m] * std::pow(10.0, (g - cfg->grid_center) / 50.0);
      fg::PlanPack* pk = fg::plan_pack_create(xs.data() + (size_t)h * nn, nn, cfg->kind,
                                              c->grid[m][g], cfg->nugget, cfg->leaf, cfg->tol, s,
                                              st, err);
      if (!pk) { tp_free(c); return tfail(st, err); }
      c->packs[m].push_back(pk);
      c->caps.add(*pk);
    }
  }
  for (int h = 0; h < nf; ++h)
    for (int i = 0; i < 2; ++i)
      if ((st = fg::hodlr_alloc(c->H[h][i], c->caps, err)) != FG_OK ||
          (st = fg::factor_alloc(c->W[h][i], c->caps, err)) != FG_OK) {
        tp_free(c);
        return tfail(st, err);
      }
  if ((st = fg::factor_alloc(c->WP, c->caps, err)) != FG_OK) { tp_free(c); return tfail(st, err); }
  const size_t nb = sizeof(double) * (size_t)nn;
  if (fg::dev_alloc(reinterpret_cast<void**>(&c->perm), sizeof(int) * (size_t)d * nn) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->F), nb * nf) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->fs), nb * nf) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->Gc), nb * ncomp) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->R), nb) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->y), nb) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->vecs), nb * 8) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->dotwork), sizeof(double) * 2048) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->st), sizeof(fg::TpState)) != hipSuccess ||
      fg::host_alloc(reinterpret_cast<void**>(&c->st_host), sizeof(fg::TpState)) != hipSuccess) {
    tp_free(c);
    return tfail(FG_ENOMEM, "tensor chain allocation failed");
  }
  if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    tp_free(c);
    return tfail(FG_EDEVICE, "stream or event creation failed");
  }
  hipMemcpyAsync(c->perm, permh.data(), sizeof(int) * permh.size(), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(c->y, y, nb, hipMemcpyDeviceToDevice, s);
  std::vector<double> ones((size_t)nf * nn, 1.0);
  hipMemcpyAsync(c->F, ones.data(), nb * nf, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(c->fs, ones.data(), nb * nf, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(c->Gc, ones.data(), nb * ncomp, hipMemcpyHostToDevice, s);
  for (int m = 0; m < nf; ++m)
    for (int i = 0; i < 2; ++i)
      hipMemcpyAsync(c->H[m][i].x, xs.data() + (size_t)(m % d) * nn, nb, hipMemcpyHostToDevice, s);
  fg::TpState init{};
  init.tau = cfg->tau0;
  for (int cc = 0; cc < ncomp; ++cc) init.beta[cc] = cfg->beta0;
  for (int m = 0; m < nf; ++m) init.k[m] = cfg->grid_center;
  *c->st_host = init;
  hipMemcpyAsync(c->st, c->st_host, sizeof(fg::TpState), hipMemcpyHostToDevice, s);
  for (int h = 0; h < nf; ++h) {
    c->k[h] = cfg->grid_center;
    c->cur[h] = 0;
    c->H[h][0].pk = c->packs[h][c->k[h]];
    fg::launch_build(c->H[h][0], s);
    c->W[h][0].H = &c->H[h][0];
    c->W[h][0].alpha = 1.0;
    c->W[h][0].beta = 0.0;
    fg::launch_factor(c->W[h][0], nullptr, nullptr, nullptr, s);
    hipMemcpyAsync(&c->st->logdet[h], c->W[h][0].logdet, sizeof(double), hipMemcpyDeviceToDevice, s);
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
    tp_free(c);
    return tfail(FG_EDEVICE, "tensor chain set-up failed on the device");
  }
  *out = c;
  return FG_OK;
}

fg_status tp_step(fg_tp_chain c, int32_t iters, fg_stream stream) {
  if (!c || iters < 0) return tfail(FG_EINVAL, "bad arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n = c->n, d = c->d, C = c->C, nf = c->nf;
  const fg_tp_cfg& cf = c->cfg;
  double* D = c->vecs;
  double* Dinv = D + n;
  double* yt = Dinv + n;
  double* G = yt + n;
  double* v0 = G + n;
  double* v1 = v0 + n;
  double* v2 = v1 + n;  // v2, v3: the two right-hand sides [Z, y~]
  double* v3 = v2 + n;
  for (int it = 0; it < iters; ++it) {
    const uint64_t t = (uint64_t)c->iter;
    // Every factor's length-scale proposal is known on the host: build and factor the
    // proposals on the second stream while this one draws f_1..f_d, beta and tau.
    int kp[fg::TP_DMAX], ong[fg::TP_DMAX];
    hipEventRecord(c->ev_fork, s);
    hipStreamWaitEvent(c->aux, c->ev_fork, 0);
    for (int h = 0; h < nf; ++h) {
      uint64_t w[4];
      fg::philox4x64_10(0, fg::tp_factor_tag(5, h), t, cf.stream_id, cf.seed, 0, w);
      kp[h] = c->k[h] + (fg::to_unit(w[0]) < 0.5 ? 1 : -1);
      ong[h] = (kp[h] >= 0 && kp[h] < cf.grid_size) ? 1 : 0;
      if (!ong[h]) continue;
      const int oth = 1 - c->cur[h];
      fg::launch_zero_int(c->H[h][oth].status, 1, c->aux);
      fg::launch_zero_int(c->W[h][oth].status, 1, c->aux);
      c->H[h][oth].pk = c->packs[h][kp[h]];
      fg::launch_build(c->H[h][oth], c->aux);
      c->W[h][oth].H = &c->H[h][oth];
      c->W[h][oth].alpha = 1.0;
      c->W[h][oth].beta = 0.0;
      fg::launch_factor(c->W[h][oth], nullptr, nullptr, nullptr, c->aux);
      hipMemcpyAsync(&c->st->logdetp[h], c->W[h][oth].logdet, sizeof(double),
                     hipMemcpyDeviceToDevice, c->aux);
    }
    hipEventRecord(c->ev_join, c->aux);
    for (int cc = 0; cc < C; ++cc) {
      // component cc sees the partial residual (y itself when it is the only one)
      const double* rc = c->y;
      if (C > 1) {
        fg::launch_tp_partial(n, C, cc, c->y, c->Gc, c->st, c->R, s);
        rc = c->R;
      }
      // f_{cc,h} | -  for h = 1..d in turn (Algorithm 1.h)
      for (int hd = 0; hd < d; ++hd) {
        const int h = cc * d + hd;  // factor index
        fg::HodlrData& H = c->H[h][c->cur[h]];
        fg::FactorData& Wh = c->W[h][c->cur[h]];
        const int* ph = c->perm + (size_t)hd * n;
        fg::launch_tp_prepare(n, d, hd, ph, c->F + (size_t)cc * d * n, rc, c->st, &c->st->beta[cc],
                              D, Dinv, yt, s);
        c->WP.H = &H;
        c->WP.alpha = 1.0;
        c->WP.beta = 0.0;
        fg::launch_factor(c->WP, nullptr, nullptr, Dinv, s);
        fg::launch_normals(cf.seed, fg::tp_factor_tag(1, h), t, cf.stream_id, n, v0, s);
        fg::launch_scale_sqrt(n, D, v0, s);
        fg::launch_normals(cf.seed, fg::tp_factor_tag(2, h), t, cf.stream_id, n, v1, s);
        fg::launch_matvec(H, 1.0, 0.0, nullptr, nullptr, v0, v2, 1, n, H.work, s);
        fg::launch_apply_w(Wh, 0, v1, 1, n, Wh.work, s);
        fg::launch_axpby(n, v2, v1, v2, nullptr, 1.0, nullptr, 1.0, s);
        hipMemcpyAsync(v3, yt, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
        fg::launch_apply_w(c->WP, 2, v2, 2, n, c->WP.work, s);
        fg::launch_apply_w(c->WP, 3, v2, 2, n, c->WP.work, s);
        fg::launch_matvec(H, 1.0, 0.0, nullptr, nullptr, v3, v0, 1, n, H.work, s);
        fg::launch_hetero_finish(n, v0, v2, D, c->fs + (size_t)h * n, ph, c->F + (size_t)h * n, s);
      }
      // beta_cc | -  (on the partial residual)
      double* Gcc = c->Gc + (size_t)cc * n;
      fg::launch_tp_product(n, d, c->F + (size_t)cc * d * n, Gcc, s);
      fg::launch_dot(Gcc, Gcc, n, 0, &c->st->GG, c->dotwork, s);
      fg::launch_dot(Gcc, rc, n, 0, &c->st->Gy, c->dotwork + 1024, s);
      fg::launch_tp_beta_step(c->st, cc, cf.s_beta, cf.seed, t, cf.stream_id, s);
    }
    // tau | -  (full residual)
    fg::launch_tp_fit(n, C, c->Gc, c->st, G, s);
    fg::launch_dot(c->y, G, n, 1, &c->st->sse, c->dotwork, s);
    fg::launch_tp_tau_step(c->st, n, cf.a1, cf.b1, cf.seed, t, cf.stream_id, s);
    // ell_h | -  (grid Metropolis per factor)
    hipStreamWaitEvent(s, c->ev_join, 0);
    for (int h = 0; h < nf; ++h) {
      const int cur = c->cur[h], oth = 1 - cur;
      const double* fh = c->fs + (size_t)h * n;
      hipMemcpyAsync(v1, fh, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
      fg::launch_apply_w(c->W[h][cur], 2, v1, 1, n, c->W[h][cur].work, s);
      fg::launch_dot(v1, v1, n, 0, &c->st->q[h], c->dotwork, s);
      if (ong[h]) {
        hipMemcpyAsync(v1, fh, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
        fg::launch_apply_w(c->W[h][oth], 2, v1, 1, n, c->W[h][oth].work, s);
        fg::launch_dot(v1, v1, n, 0, &c->st->qp[h], c->dotwork, s);
      }
      fg::launch_tp_mh_step(c->st, h, kp[h], ong[h], cf.seed, t, cf.stream_id,
                            ong[h] ? c->H[h][oth].status : nullptr,
                            ong[h] ? c->W[h][oth].status : nullptr, s);
    }
    hipMemcpyAsync(c->st_host, c->st, sizeof(fg::TpState), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return tfail(FG_EDEVICE, "sweep failed on the device");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tfail(FG_EDEVICE, std::string("sweep launch: ") + hipGetErrorString(e));
    for (int h = 0; h < nf; ++h)
      if (c->st_host->accept[h]) {
        c->cur[h] = 1 - c->cur[h];
        c->k[h] = kp[h];
      }
    c->iter += 1;
  }
  return FG_OK;
}

fg_status tp_chain_state(fg_tp_chain c, fg_tp_snapshot* host_out, double* F_out,
                         fg_stream stream) {
  if (!c || !host_out) return tfail(FG_EINVAL, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (F_out)
    hipMemcpyAsync(F_out, c->F, sizeof(double) * (size_t)c->nf * c->n, hipMemcpyDeviceToDevice, s);
  hipMemcpyAsync(c->st_host, c->st, sizeof(fg::TpState), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return tfail(FG_EDEVICE, "state copy failed");
  int fst = c->st_host->status;
  for (int h = 0; h < c->nf; ++h) {
    int a = 0, b = 0;
    hipMemcpy(&a, c->H[h][c->cur[h]].status, sizeof(int), hipMemcpyDeviceToHost);
    hipMemcpy(&b, c->W[h][c->cur[h]].status, sizeof(int), hipMemcpyDeviceToHost);
    fst |= a | b;
  }
  int wp = 0;
  hipMemcpy(&wp, c->WP.status, sizeof(int), hipMemcpyDeviceToHost);
  fst |= wp;
  const fg::TpState& q = *c->st_host;
  *host_out = fg_tp_snapshot{};
  host_out->iteration = c->iter;
  host_out->tau = q.tau;
  host_out->beta = q.beta[0];
  host_out->sse = q.sse;
  host_out->beta_mean = q.beta_mean[0];
  host_out->beta_sd = q.beta_sd[0];
  host_out->ncomp = c->C;
  for (int cc = 0; cc < c->C; ++cc) {
    host_out->betas[cc] = q.beta[cc];
    host_out->beta_means[cc] = q.beta_mean[cc];
    host_out->beta_sds[cc] = q.beta_sd[cc];
  }
  for (int h = 0; h < c->nf; ++h) {
    host_out->k[h] = q.k[h];
    host_out->ell[h] = c->grid[h][q.k[h]];
    host_out->last_proposal[h] = q.kprop[h];
    host_out->last_accept[h] = q.accept[h];
    host_out->accepts[h] = q.accepts[h];
    host_out->logdet[h] = q.logdet[h];
    host_out->q[h] = q.q[h];
    host_out->mh_log_ratio[h] = q.mh[h];
  }
  host_out->status = (fst & fg::ST_NOTSPD) ? FG_ENOTSPD : (fst & fg::ST_NOTCONV) ? FG_ENOTCONV : FG_OK;
  return FG_OK;
}

void tp_chain_destroy(fg_tp_chain c) { tp_free(c); }

}  // extern "C"
