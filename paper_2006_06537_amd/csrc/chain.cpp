// One FIFA-GP Gibbs chain on the device (Section 4.1): f by Algorithm 1, tau and
// sigma_f^-2 by their conjugate Gamma conditionals, and the length-scale by a Metropolis
// step on a grid (the replacement for the discrete conditional that the paper
// suggests).  The chain keeps two slots of (K~_1, W_1) -- the current length-scale and
// the proposal -- and swaps them on acceptance; all plans of the grid are made and
// uploaded once, so a sweep only enqueues kernels and synchronises once at its end.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fg_chain.h"
#include "fg_group.h"
#include "fg_internal.h"
#include "fg_rng.h"
#include "fg_pcg.h"
#include "fg_timer.h"
#include "fg_tensor.h"

// a sweep's grid proposal: the proposed index and whether it lies on the grid
struct SweepProposal {
  int kp = 0, ongrid = 0;
};

struct fg_chain_s {
  fg_chain_cfg cfg{};
  SweepProposal pending;                      // the proposal of the sweep in flight
  int n = 0;
  std::vector<double> grid;
  std::vector<fg::PlanPack*> packs;
  fg::Caps caps;
  fg::HodlrData H[2];
  fg::FactorData W[2];
  fg::FactorData WM;
  int cur = 0;
  int k = 0;
  int64_t iter = 0;
  double *x = nullptr, *y = nullptr, *f = nullptr, *r = nullptr, *mu = nullptr;
  double* vecs = nullptr;     // 4 n workspace
  double* dotwork = nullptr;  // reduction partials
  fg::DevState* st = nullptr;
  fg::DevState* st_prev = nullptr;  // the state at the start of the last sweep
  fg::DevState* st_host = nullptr;  // pinned
  bool mixed = false;                         // FP32 leaf factor of M~ + PCG refinement
  bool fell_back = false;                     // M~ moved to FP64 after an FP32 failure
  fg::FactorData WM64;                        // FP64 factor of M~ used after the fallback
  fg::PcgWork pcg;
  int pcg_nit = 6;                            // PCG iterations enqueued per f-draw
  int pcg_iters = 0;
  double pcg_relres = 0.0;
  bool pcg_failed = false;
  hipStream_t aux = nullptr;                  // proposal build + factor, beside the f-draw
  hipStream_t zs = nullptr;                   // Z and tau y, beside the factorization of M~
  hipStream_t ls = nullptr;                   // the proposal's leaves, beside its build
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_z = nullptr, ev_f = nullptr,
             ev_leaf = nullptr;
  bool own_streams = true;                    // false: lent by the caller (serving slots)
  hipError_t enq_err = hipSuccess;            // first runtime error while enqueuing a sweep
  // exact discrete conditional of the length-scale: every grid point's K~_1 and W_1
  bool exact = false;
  std::vector<fg::HodlrData> Hg;
  std::vector<fg::FactorData> Wg;
  double* ldg = nullptr;                      // log det K~_1 per grid point
  double* qg = nullptr;                       // |W_h^-1 f|^2 per grid point
  double* qbuf = nullptr;                     // one work vector per q stream
  double* qdot = nullptr;                     // dot partials per q stream
  hipStream_t qs[4] = {};
  hipEvent_t qev[5] = {};
  std::vector<fg::Recorder> qrec;             // one per grid point (grouped q_h)
  fg::GroupExec qexec;
  // non-unique inputs: the chain runs on the unique inputs with the averages as y
  bool collapsed = false;
  double* cw = nullptr;                       // |Q_i| (n), then precisions and their inverses
  double within = 0.0;                        // within-group sum of squares
  int64_t n_obs = 0;                          // observations before collapsing
  double* xstar = nullptr;                    // new inputs of the predictive draws
  int nstar = 0;
  struct ZEntry {
    int k;                                    // grid index, -1 = empty
    double* z;                                // n x nstar: W_1^-1 k1(X, X*) at that grid point
    uint64_t used;                            // last use, for least-recently-used eviction
  };
  std::vector<ZEntry> zcache;                 // at most zcache_cap entries
  int zcache_cap = 0;
  uint64_t zclock = 0;
  int64_t zbuilds = 0;                        // Z computations so far (cache misses)
  double* pwork = nullptr;                    // W_1^-1 f (n), the draw's normals (nstar), partials
  std::map<uint64_t, hipGraphExec_t> graphs;  // captured sweeps by (cur, k, proposal)
  std::vector<uint64_t> graph_order;          // insertion order, for eviction
};

constexpr size_t GRAPH_CACHE = 48;  // captured sweeps kept per chain
constexpr double PCG_RTOL = 1e-10;  // relative residual of the mixed-precision solves
constexpr int PCG_MAXIT = 32;       // iteration budget beyond which M~ moves to FP64

using fg::set_error;

static fg_status cfail(fg_status st, const std::string& m) {
  set_error(m);
  return st;
}

// sync: wait for the whole device first (a public destroy: the caller may still have work
// queued that reads the chain); without it the caller guarantees that nothing queued
// touches the chain any more (the serving loop, after the chain's last event)
static void chain_free(fg_chain c, bool sync = true) {
  if (!c) return;
  if (sync) (void)hipDeviceSynchronize();
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->own_streams) {
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_z) (void)hipEventDestroy(c->ev_z);
    if (c->ev_f) (void)hipEventDestroy(c->ev_f);
    if (c->ev_leaf) (void)hipEventDestroy(c->ev_leaf);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->zs) (void)hipStreamDestroy(c->zs);
    if (c->ls) (void)hipStreamDestroy(c->ls);
  }
  fg::pcg_free(c->pcg);
  for (int i = 0; i < 2; ++i) { fg::hodlr_free(c->H[i]); fg::factor_free(c->W[i]); }
  for (auto& h : c->Hg) fg::hodlr_free(h);
  for (auto& w : c->Wg) fg::factor_free(w);
  for (auto q : c->qs)
    if (q) (void)hipStreamDestroy(q);
  for (auto e : c->qev)
    if (e) (void)hipEventDestroy(e);
  fg::factor_free(c->WM);
  fg::factor_free(c->WM64);
  for (auto* p : c->packs) fg::plan_pack_destroy(p);
  for (auto& e : c->zcache)
    if (e.z) fg::dev_free(e.z);
  double* bufs[] = {c->x, c->y, c->f, c->r, c->mu, c->vecs, c->dotwork, c->xstar, c->pwork,
                    c->cw, c->ldg, c->qg, c->qbuf, c->qdot};
  for (double* b : bufs)
    if (b) fg::dev_free(b);
  if (c->st) fg::dev_free(c->st);
  if (c->st_prev) fg::dev_free(c->st_prev);
  if (c->st_host) fg::host_free(c->st_host);
  delete c;
}

namespace {

using Proposal = SweepProposal;

// the current length-scale's K~_1 and W_1: a grid slot in exact mode, else the slot of the
// two-slot (current, proposal) pair
fg::HodlrData& Hcur(fg_chain c) { return c->exact ? c->Hg[c->k] : c->H[c->cur]; }
fg::FactorData& Wcur(fg_chain c) { return c->exact ? c->Wg[c->k] : c->W[c->cur]; }

// The grid proposal of the next sweep: its uniform is addressed by the iteration
// count, which the host knows, so the proposal needs no device round trip.
Proposal propose(fg_chain c) {
  if (c->exact) return Proposal{c->k, 0};  // no proposal: the whole grid is weighed
  uint64_t w[4];
  fg::philox4x64_10(0, 5, (uint64_t)c->iter, c->cfg.stream_id, c->cfg.seed, 0, w);
  Proposal p;
  p.kp = c->k + (fg::to_unit(w[0]) < 0.5 ? 1 : -1);
  p.ongrid = (p.kp >= 0 && p.kp < c->cfg.grid_size) ? 1 : 0;
  return p;
}

// Enqueues one sweep on s.  Every argument is fixed by (cur, k, proposal): the
// iteration word lives in device memory, so the sequence can be captured once and
// replayed.  Ends with the copy of the device state to pinned host memory.
// Host-side state of the sweep about to run: which plan and matrix each slot's
// launches refer to.  Runs before every sweep, captured or replayed, so that the host
// view always matches what the device holds.
void prepare_sweep(fg_chain c, const Proposal& pr) {
  const int cur = c->cur, oth = 1 - cur;
  fg::FactorData& WM = c->fell_back ? c->WM64 : c->WM;
  WM.H = &Hcur(c);
  if (c->collapsed) {  // K~_1 + D^-1, D^-1 passed as the diagonal
    WM.alpha = 1.0;
    WM.beta = 0.0;
  } else {
    WM.alpha = 0.0;  // taken from the device scalar
    WM.beta = 1.0;
  }
  if (pr.ongrid) {
    c->H[oth].pk = c->packs[pr.kp];
    c->W[oth].H = &c->H[oth];
    c->W[oth].alpha = 1.0;
    c->W[oth].beta = 0.0;
  }
}

// every runtime call that enqueues part of a sweep goes through here: the first failure
// is kept and reported once the sweep has been enqueued (or captured)
static inline void enq_check(fg_chain c, hipError_t e) {
  if (e != hipSuccess && c->enq_err == hipSuccess) c->enq_err = e;
}
// stream-order helpers of the sweep: while a recorder is open (grouped batches) the whole
// sweep is replayed on one stream in program order, so events are not needed and copies
// are recorded like launches
static void ev_record(fg_chain c, hipEvent_t e, hipStream_t s) {
  if (!fg::recording()) enq_check(c, hipEventRecord(e, s));
}
static void ev_wait(fg_chain c, hipStream_t s, hipEvent_t e) {
  if (!fg::recording()) enq_check(c, hipStreamWaitEvent(s, e, 0));
}
static void enq_copy(fg_chain c, void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                     hipStream_t s) {
  if (kind == hipMemcpyDeviceToDevice) {
    fg::launch_copy_d2d(dst, src, bytes, s);
    return;
  }
  FG_RUN(s, enq_check(c, hipMemcpyAsync(dst, src, bytes, kind, q_)));
}

// f | - and tau | - on collapsed data (Appendix, non-unique input points): Algorithm 1.h
// on g = f / sigma_f, whose prior is K~_1 and whose data ybar / sigma_f have precisions
// D = tau sigma_f^2 |Q_i|; then f = sigma_f g, and tau from the full-data residual.
static void enqueue_f_tau_collapsed(fg_chain c, hipStream_t s) {
  const int n = c->n;
  const fg_chain_cfg& cf = c->cfg;
  fg::HodlrData& H1 = Hcur(c);
  fg::FactorData& W1 = Wcur(c);
  double* v0 = c->vecs;
  double* v1 = v0 + n;
  double* v2 = v1 + n;  // v2, v3: the two right-hand sides [Z, ybar / sigma_f]
  double* v3 = v2 + n;
  double* dprec = c->cw + n;
  double* dinv = dprec + n;
  const uint64_t* itp = &c->st->iter;
  fg::launch_collapsed_weights(n, c->cw, &c->st->alphaM, dprec, dinv, s);
  fg::launch_factor(c->WM, nullptr, nullptr, dinv, s);
  enq_copy(c, &c->st->logdetM, c->WM.logdet, sizeof(double), hipMemcpyDeviceToDevice, s);
  fg::launch_normals(cf.seed, 1, 0, cf.stream_id, n, v0, s, itp);
  fg::launch_scale_sqrt(n, dprec, v0, s);  // a ~ N(0, D)
  fg::launch_normals(cf.seed, 2, 0, cf.stream_id, n, v1, s, itp);
  fg::launch_matvec(H1, 1.0, 0.0, nullptr, nullptr, v0, v2, 1, n, H1.work, s);
  fg::launch_apply_w(W1, 0, v1, 1, n, W1.work, s);
  fg::launch_axpby(n, v2, v1, v2, nullptr, 1.0, nullptr, 1.0, s);  // Z = K~_1 a + W_1 b
  fg::launch_div_scalar(n, c->y, &c->st->sigf, v3, s);
  fg::launch_apply_w(c->WM, 2, v2, 2, n, c->WM.work, s);
  fg::launch_apply_w(c->WM, 3, v2, 2, n, c->WM.work, s);
  fg::launch_matvec(H1, 1.0, 0.0, nullptr, nullptr, v3, v0, 1, n, H1.work, s);
  fg::launch_hetero_finish(n, v0, v2, dprec, c->f, nullptr, nullptr, s);  // g = R + Z* / D
  fg::launch_axpby(n, c->f, nullptr, c->f, &c->st->sigf, 0.0, nullptr, 0.0, s);
  fg::launch_axpby(n, v0, nullptr, c->mu, &c->st->sigf, 0.0, nullptr, 0.0, s);
  fg::launch_div_scalar(n, v3, &c->st->sigf, c->r, s);  // Sigma^-1 ybar
  fg::launch_dot(c->y, v3, n, 0, &c->st->yr, c->dotwork, s);
  fg::launch_wsse(c->y, c->f, c->cw, n, &c->st->sse, c->dotwork + 1024, s);
  fg::launch_tau_step_collapsed(c->st, n, c->n_obs, c->within, cf.a1, cf.b1, cf.seed,
                                cf.stream_id, s);
}

// q_h = |W_h^-1 f|^2 for every grid point, spread over the chain's q streams, then one
// draw from the discrete conditional (k_rho_exact).
static void enqueue_rho_exact(fg_chain c, hipStream_t s) {
  const int n = c->n, G = (int)c->Wg.size();
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  enq_check(c, hipStreamIsCapturing(s, &cap));
  if (!fg::recording() && cap == hipStreamCaptureStatusNone) {
    // Grouped: q_h = |W_h^-1 f|^2 of every grid point recorded separately (each on its
    // own work vector), then replayed as grouped launches: about 30 launches for the
    // whole grid instead of about 30 per grid point.  (Not under graph capture: the
    // grouped launches' argument upload is staged per call.)
    if (c->qrec.size() < (size_t)G) c->qrec.resize(G);
    std::vector<fg::Recorder*> rp(G);
    for (int h = 0; h < G; ++h) {
      fg::Recorder* r = &c->qrec[h];
      r->clear();
      fg::RecordScope scope(r);
      double* v = c->qbuf + (size_t)h * n;
      enq_copy(c, v, c->f, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
      fg::launch_apply_w(c->Wg[h], 2, v, 1, n, c->Wg[h].work, s);
      fg::launch_dot(v, v, n, 0, c->qg + h, c->qdot + (size_t)h * 2048, s);
      rp[h] = r;
    }
    std::string err;
    if (c->qexec.run(rp, s, err) != FG_OK) enq_check(c, hipErrorLaunchFailure);
    fg::launch_rho_exact(c->st, c->ldg, c->qg, G, c->cfg.seed, c->cfg.stream_id, s);
    return;
  }
  // inside a grouped batch (already recording): the grid in order, one work vector
  ev_record(c, c->qev[0], s);
  for (int q = 0; q < 4; ++q) ev_wait(c, c->qs[q], c->qev[0]);
  for (int h = 0; h < G; ++h) {
    const int q = h & 3;
    double* v = c->qbuf + (size_t)q * n;
    enq_copy(c, v, c->f, sizeof(double) * n, hipMemcpyDeviceToDevice, c->qs[q]);
    fg::launch_apply_w(c->Wg[h], 2, v, 1, n, c->Wg[h].work, c->qs[q]);
    fg::launch_dot(v, v, n, 0, c->qg + h, c->qdot + (size_t)q * 2048, c->qs[q]);
  }
  for (int q = 0; q < 4; ++q) {
    ev_record(c, c->qev[1 + q], c->qs[q]);
    ev_wait(c, s, c->qev[1 + q]);
  }
  fg::launch_rho_exact(c->st, c->ldg, c->qg, G, c->cfg.seed, c->cfg.stream_id, s);
}

// `side`: Z and tau y on the chain's third stream, the proposal's leaves on its fourth and
// the proposal's quadratic form on the second, which helps a chain that has the GPU to
// itself.  Without it (batches of chains, which fill the GPU by themselves, and captured
// sweeps) the sweep keeps the two-stream form: the proposal's build and whole
// factorization on the second stream, Z and both quadratic forms on this one.  (The
// serving loop, which captures from a worker thread, once ended in a host segmentation
// fault with the four-stream form; the cause was not found.)  The arithmetic is the same.
void enqueue_sweep(fg_chain c, const Proposal& pr, hipStream_t s, bool side) {
  const int n = c->n;
  const fg_chain_cfg& cf = c->cfg;
  double* v0 = c->vecs;
  double* v1 = v0 + n;
  double* v2 = v1 + n;  // v2, v3: the two right-hand sides [Z, tau y]
  double* v3 = v2 + n;
  const uint64_t* itp = &c->st->iter;
  const int oth = 1 - c->cur;
  fg::HodlrData& H1 = Hcur(c);
  fg::FactorData& W1 = Wcur(c);
  fg::launch_sweep_begin(c->st, c->st_prev, s);
  // The proposal's K~_1' and W_1' depend on the proposal only: build and factor them on
  // the chain's second stream while this stream factors M~ and draws f.
  ev_record(c, c->ev_fork, s);
  ev_wait(c, c->aux, c->ev_fork);
  if (pr.ongrid && !side) {
    fg::launch_zero_int(c->H[oth].status, 1, c->aux);
    fg::launch_zero_int(c->W[oth].status, 1, c->aux);
    fg::launch_build(c->H[oth], c->aux);
    fg::launch_factor(c->W[oth], nullptr, nullptr, nullptr, c->aux);
    enq_copy(c, &c->st->logdet1p, c->W[oth].logdet, sizeof(double), hipMemcpyDeviceToDevice,
             c->aux);
  } else if (pr.ongrid) {
    // its leaves need x and ell' only: a fourth stream factors them during the build
    ev_wait(c, c->ls, c->ev_fork);
    fg::launch_zero_int(c->W[oth].status, 1, c->ls);
    fg::launch_factor_leaves(c->W[oth], nullptr, nullptr, nullptr, c->ls);
    ev_record(c, c->ev_leaf, c->ls);
    fg::launch_zero_int(c->H[oth].status, 1, c->aux);
    fg::launch_build(c->H[oth], c->aux);
  }
  // the rest of the proposal's factorization, once its build and leaves are done; it is
  // enqueued after this stream's factorization of M~ and Z (one host thread enqueues every
  // stream, and those are needed first), but before them on collapsed data
  bool proposal_levels = side && pr.ongrid;
  auto enqueue_proposal_levels = [&]() {
    if (!proposal_levels) return;
    proposal_levels = false;
    ev_wait(c, c->aux, c->ev_leaf);
    fg::launch_factor_levels(c->W[oth], nullptr, c->aux);
    enq_copy(c, &c->st->logdet1p, c->W[oth].logdet, sizeof(double), hipMemcpyDeviceToDevice,
             c->aux);
  };
  if (c->collapsed) {
    enqueue_proposal_levels();
    enqueue_f_tau_collapsed(c, s);
  } else {
    // f | -  (Algorithm 1).  Z = sqrt(tau) sigma_f^2 K~_1 a + sigma_f W_1 b and tau y use
    // the previous sweep's scalars only: the chain's third stream forms them while this
    // stream factors M~.
    fg::FactorData& WM = c->fell_back ? c->WM64 : c->WM;
    fg::launch_factor(WM, &c->st->alphaM, nullptr, nullptr, s);
    enq_copy(c, &c->st->logdetM, WM.logdet, sizeof(double), hipMemcpyDeviceToDevice, s);
    hipStream_t zq = side ? c->zs : s;
    if (side) ev_wait(c, zq, c->ev_fork);
    fg::launch_normals(cf.seed, 1, 0, cf.stream_id, n, v0, zq, itp);
    fg::launch_normals(cf.seed, 2, 0, cf.stream_id, n, v1, zq, itp);
    fg::launch_matvec(H1, 1.0, 0.0, nullptr, nullptr, v0, v2, 1, n, H1.work, zq);
    fg::launch_apply_w(W1, 0, v1, 1, n, W1.work, zq);
    fg::launch_axpby(n, v2, v1, v2, &c->st->c_ka, 0.0, &c->st->sigf, 0.0, zq);
    fg::launch_axpby(n, c->y, nullptr, v3, &c->st->tau_draw, 0.0, nullptr, 0.0, zq);
    if (side) {
      ev_record(c, c->ev_z, zq);
      enqueue_proposal_levels();
      ev_wait(c, s, c->ev_z);
    }
    if (c->mixed && !c->fell_back) {
      // [w r] = M~^-1 [Z, tau y] by PCG on the FP64 HODLR M~, preconditioned with the
      // factor whose leaves are FP32: pcg_nit iterations with the convergence test on the
      // device (the host checks the record after the sweep and runs the sweep again with
      // a larger budget if it did not converge).  The solution goes to v0, v1 (free at
      // this point) and back into v2, v3.
      fg::pcg_enqueue(H1, 0.0, &c->st->alphaM, 1.0, c->WM, v2, v0, 2, n, PCG_RTOL, 0,
                      c->pcg_nit, c->pcg, s, true);
      fg::launch_pcg_record(c->pcg.sc, c->st, c->WM.status, s);
      enq_copy(c, v2, v0, 2 * sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    } else {
      fg::launch_apply_w(WM, 2, v2, 2, n, WM.work, s);
      fg::launch_apply_w(WM, 3, v2, 2, n, WM.work, s);
    }
    fg::launch_matvec(H1, 0.0, 0.0, &c->st->sigf2, nullptr, v3, c->mu, 1, n,
                      H1.work, s);
    fg::launch_axpby(n, v2, c->mu, c->f, nullptr, 1.0, nullptr, 1.0, s);
    enq_copy(c, c->r, v3, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    fg::launch_dot(c->y, c->r, n, 0, &c->st->yr, c->dotwork, s);
    fg::launch_dot(c->y, c->f, n, 1, &c->st->sse, c->dotwork + 1024, s);
    // tau | -
    fg::launch_tau_step(c->st, n, cf.a1, cf.b1, cf.seed, cf.stream_id, s);
  }
  // f is final: the proposal's quadratic form |W_1'^-1 f|^2 runs on the second stream,
  // beside this stream's |W_1^-1 f|^2 (v1 is free from here on).  This stream's part is
  // enqueued first: it is the longer one, and one host thread enqueues both.
  const bool qprop_side = side && !c->exact && pr.ongrid;
  if (qprop_side) ev_record(c, c->ev_f, s);
  // sigma_f^-2 | -
  enq_copy(c, v0, c->f, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
  fg::launch_apply_w(W1, 2, v0, 1, n, W1.work, s);
  fg::launch_dot(v0, v0, n, 0, &c->st->q, c->dotwork, s);
  fg::launch_sigf_step(c->st, n, cf.a2, cf.b2, cf.seed, cf.stream_id, s);
  if (qprop_side) {
    ev_wait(c, c->aux, c->ev_f);
    enq_copy(c, v1, c->f, sizeof(double) * n, hipMemcpyDeviceToDevice, c->aux);
    fg::launch_apply_w(c->W[oth], 2, v1, 1, n, c->W[oth].work, c->aux);
    fg::launch_dot(v1, v1, n, 0, &c->st->qprop, c->dotwork + 2048, c->aux);
  }
  ev_record(c, c->ev_join, c->aux);
  ev_wait(c, s, c->ev_join);
  if (c->exact) {  // length-scale | -  (exact, over the whole grid)
    enqueue_rho_exact(c, s);
    enq_copy(c, c->st_host, c->st, sizeof(fg::DevState), hipMemcpyDeviceToHost, s);
    return;
  }
  // length-scale | -  (Metropolis on the grid)
  if (!side && pr.ongrid) {
    enq_copy(c, v1, c->f, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    fg::launch_apply_w(c->W[oth], 2, v1, 1, n, c->W[oth].work, s);
    fg::launch_dot(v1, v1, n, 0, &c->st->qprop, c->dotwork, s);
  }
  fg::launch_mh_step(c->st, pr.kp, pr.ongrid, cf.seed, cf.stream_id,
                     pr.ongrid ? c->H[oth].status : nullptr, pr.ongrid ? c->W[oth].status : nullptr, s);
  enq_copy(c, c->st_host, c->st, sizeof(fg::DevState), hipMemcpyDeviceToHost, s);
}

// After the sweep's stream has been synchronised, before finish_sweep: whether the
// mixed-precision f-draw's PCG converged within its budget.  If it did, the budget of the
// next sweep becomes the iterations it needed plus one.  If not, the state is restored
// (enqueued on s) and the caller runs the same sweep again: with twice the budget, or,
// once the budget is at its cap, a residual was not finite or the FP32 leaf Cholesky met a
// non-positive pivot, with M~ factored in FP64 from then on (the FP32 leaf factor is then
// no preconditioner).  A sweep run again from
// the same state gives what it would have given with the larger budget at once.
bool sweep_retry(fg_chain c, hipStream_t s) {
  if (!c->mixed || c->fell_back || c->exact || c->collapsed) return false;
  const fg::DevState& d = *c->st_host;
  if (d.pcg_done == 1) {
    c->pcg_iters = d.pcg_iters;
    c->pcg_relres = d.pcg_relres;
    c->pcg_nit = std::min(std::max(d.pcg_iters + 1, 2), PCG_MAXIT);
    return false;
  }
  if (d.pcg_done == 0 && c->pcg_nit < PCG_MAXIT) {
    c->pcg_nit = std::min(2 * c->pcg_nit, PCG_MAXIT);
  } else {
    std::string err;
    if (fg::factor_alloc(c->WM64, c->caps, err) != FG_OK) {
      c->pcg_failed = true;  // reported as FG_ENOTCONV; the chain keeps the FP32 factor
      c->pcg_iters = d.pcg_iters;
      c->pcg_relres = d.pcg_relres;
      return false;
    }
    c->fell_back = true;
    c->pcg_iters = 0;
    c->pcg_relres = 0.0;
  }
  enq_copy(c, c->st, c->st_prev, sizeof(fg::DevState), hipMemcpyDeviceToDevice, s);
  return true;
}

// after the sweep's stream has been synchronised: the accepted proposal becomes current
void finish_sweep(fg_chain c, const Proposal& pr) {
  if (c->exact) {
    c->k = c->st_host->k;
  } else if (c->st_host->accept) {
    c->cur = 1 - c->cur;
    c->k = pr.kp;
  }
  c->iter += 1;
}

// A few default-priority streams shared by batched calls.  They are created once, and
// a batched call holds them (g_batch.mu) for its whole duration: two host threads that
// step batches at the same time take turns instead of interleaving on shared streams.
constexpr int BATCH_STREAMS = 4;
// the batch autotuner's candidates (mode, streams) and its record per batch signature
struct BatchCand {
  int mode, nstreams;
};
constexpr BatchCand TUNE_CANDS[] = {{FG_BATCH_GROUPED, 1},
                                    {FG_BATCH_EAGER, 4},
                                    {FG_BATCH_EAGER, 2},
                                    {FG_BATCH_GRAPHS, 4}};
constexpr int NTUNE = sizeof(TUNE_CANDS) / sizeof(TUNE_CANDS[0]);
struct BatchTune {
  int trial = 0;
  bool done = false;
  int mode = FG_BATCH_EAGER, nstreams = 4;
  double best_ms = -1.0;
};
struct BatchStreams {
  std::mutex mu;
  bool init = false;
  hipStream_t s[BATCH_STREAMS] = {};
  hipEvent_t ev_in = nullptr;
  std::vector<fg::Recorder> recs;       // one per chain of a grouped batch
  fg::GroupExec exec;
  std::map<uint64_t, BatchTune> tune;   // autotuner choices by batch signature
};
BatchStreams g_batch;

// with g_batch.mu held
fg_status batch_streams_init() {
  if (g_batch.init) return FG_OK;
  for (int q = 0; q < BATCH_STREAMS; ++q)
    if (!g_batch.s[q] && hipStreamCreateWithFlags(&g_batch.s[q], hipStreamNonBlocking) != hipSuccess)
      return cfail(FG_EDEVICE, "stream creation failed");
  if (!g_batch.ev_in && hipEventCreateWithFlags(&g_batch.ev_in, hipEventDisableTiming) != hipSuccess)
    return cfail(FG_EDEVICE, "event creation failed");
  g_batch.init = true;
  return FG_OK;
}

// The captured sweep for (cur, k, proposal), instantiated on first use.
fg_status sweep_graph(fg_chain c, const Proposal& pr, hipStream_t q, hipGraphExec_t& out) {
  // (slot, FP64 fallback, PCG budget, grid index, proposal): everything the enqueued
  // sequence depends on
  const uint64_t key = ((uint64_t)c->cur << 56) | ((uint64_t)c->fell_back << 55) |
                       ((uint64_t)(c->mixed ? c->pcg_nit : 0) << 44) |
                       ((uint64_t)(uint32_t)c->k << 22) | (uint64_t)(uint32_t)(pr.kp + 1);
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    out = it->second;
    return FG_OK;
  }
  if (c->graphs.size() >= GRAPH_CACHE) {  // drop the oldest entry
    const uint64_t old = c->graph_order.front();
    c->graph_order.erase(c->graph_order.begin());
    (void)hipGraphExecDestroy(c->graphs[old]);
    c->graphs.erase(old);
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return cfail(FG_EDEVICE, "stream capture failed to start");
  // captured sweeps always take the two-stream form (see DESIGN: a captured four-stream
  // sweep once ended in a host fault whose cause was not found)
  enqueue_sweep(c, pr, q, false);
  const hipError_t ce = hipStreamEndCapture(q, &g);
  if (c->enq_err != hipSuccess || ce != hipSuccess || !g) {
    const hipError_t e = c->enq_err != hipSuccess ? c->enq_err : ce;
    c->enq_err = hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    return cfail(FG_EDEVICE, std::string("stream capture failed: ") + hipGetErrorString(e));
  }
  hipGraphExec_t ge = nullptr;
  const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return cfail(FG_EDEVICE, "graph instantiation failed");
  c->graphs[key] = ge;
  c->graph_order.push_back(key);
  out = ge;
  return FG_OK;
}

// device bytes of a chain of capacity `caps` with `plan_bytes` of uploaded plans
size_t chain_bytes_from(const fg::Caps& caps, size_t plan_bytes, int n, bool mixed) {
  size_t b = plan_bytes + 2 * fg::hodlr_bytes(caps) + 2 * fg::factor_bytes(caps, false) +
             fg::factor_bytes(caps, mixed);
  b += sizeof(double) * ((size_t)9 * n + 3072) + 2 * sizeof(fg::DevState);
  // a mixed chain keeps room for the FP64 factor of M~ it falls back to, so that the
  // fallback allocates from the chain's own memory (a served job's block) and cannot fail
  if (mixed) b += sizeof(double) * ((size_t)4 * fg::NRHS_PCG * n + 4096) + fg::factor_bytes(caps, false);
  return b;
}

}  // namespace

namespace fg {

ChainPlans::~ChainPlans() {
  for (auto* p : packs) plan_pack_destroy(p);
}

fg_status chain_plan(const fg_chain_cfg& cfg, const double* xh, int n, ChainPlans& out,
                     std::string& err) {
  if (n < 1) { err = "n out of range"; return FG_EINVAL; }
  if (cfg.grid_size < 1 || cfg.grid_center < 0 || cfg.grid_center >= cfg.grid_size) {
    err = "bad grid";
    return FG_EINVAL;
  }
  if (!(cfg.tau0 > 0) || !(cfg.sigf2_0 > 0) || !(cfg.ell0 > 0)) {
    err = "tau0, sigf2_0 and ell0 must be > 0";
    return FG_EINVAL;
  }
  if (cfg.precision != FG_FP64 && cfg.precision != FG_MIXED) {
    err = "bad precision";
    return FG_EINVAL;
  }
  for (auto* p : out.packs) plan_pack_destroy(p);
  out.packs.clear();
  out.caps = Caps();
  out.plan_bytes = 0;
  for (int g = 0; g < cfg.grid_size; ++g) {
    fg_status st;
    const double ell = cfg.ell0 * std::pow(10.0, (g - cfg.grid_center) / 50.0);
    PlanPack* pk = plan_pack_make(xh, n, cfg.kind, ell, cfg.nugget, cfg.leaf, cfg.tol, st, err);
    if (!pk) return st;
    out.packs.push_back(pk);
    out.caps.add(*pk);
    out.plan_bytes += plan_device_bytes(*pk);
  }
  out.bytes = chain_bytes_from(out.caps, out.plan_bytes, n, cfg.precision == FG_MIXED);
  return FG_OK;
}

fg_status chain_create_planned(const fg_chain_cfg& cfg, ChainPlans& plans, const double* x,
                               const double* y, bool host_inputs, int n, hipStream_t s,
                               const ChainStreams* borrowed, bool sync, fg_chain* out,
                               std::string& err) {
  *out = nullptr;
  fg_chain c = new fg_chain_s();
  c->cfg = cfg;
  c->n = n;
  c->grid.resize(cfg.grid_size);
  for (int g = 0; g < cfg.grid_size; ++g)
    c->grid[g] = cfg.ell0 * std::pow(10.0, (g - cfg.grid_center) / 50.0);
  c->packs.swap(plans.packs);
  c->caps = plans.caps;
  fg_status st;
  auto fail = [&](fg_status code, const std::string& m) {
    err = m;
    (void)hipStreamSynchronize(s);  // uploads already enqueued may still read or write
    chain_free(c, sync);
    return code;
  };
  for (auto* pk : c->packs)
    if ((st = plan_pack_upload(pk, s, false, err)) != FG_OK) return fail(st, err);
  const bool async = !sync;
  for (int i = 0; i < 2; ++i) {
    if ((st = hodlr_alloc(c->H[i], c->caps, err, s, async)) != FG_OK ||
        (st = factor_alloc(c->W[i], c->caps, err, false, s, async)) != FG_OK)
      return fail(st, err);
  }
  c->mixed = cfg.precision == FG_MIXED;
  if ((st = factor_alloc(c->WM, c->caps, err, c->mixed, s, async)) != FG_OK) return fail(st, err);
  if (c->mixed && (st = pcg_alloc(c->pcg, n, err)) != FG_OK) return fail(st, err);
  const size_t nb = sizeof(double) * (size_t)n;
  if (dev_alloc(reinterpret_cast<void**>(&c->x), nb) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->y), nb) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->f), nb) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->r), nb) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->mu), nb) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->vecs), 4 * nb) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->dotwork), sizeof(double) * 3072) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->st), sizeof(DevState)) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&c->st_prev), sizeof(DevState)) != hipSuccess ||
      host_alloc(reinterpret_cast<void**>(&c->st_host), sizeof(DevState)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FG_ENOMEM, "chain allocation failed");
  }
  if (borrowed) {
    c->own_streams = false;
    c->aux = borrowed->aux;
    c->zs = borrowed->zs;
    c->ls = borrowed->ls;
    c->ev_fork = borrowed->ev[0];
    c->ev_join = borrowed->ev[1];
    c->ev_z = borrowed->ev[2];
    c->ev_f = borrowed->ev[3];
    c->ev_leaf = borrowed->ev[4];
  } else if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
             hipStreamCreateWithFlags(&c->zs, hipStreamNonBlocking) != hipSuccess ||
             hipStreamCreateWithFlags(&c->ls, hipStreamNonBlocking) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_z, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_f, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_leaf, hipEventDisableTiming) != hipSuccess) {
    return fail(FG_EDEVICE, "stream or event creation failed");
  }
  const hipMemcpyKind kind = host_inputs ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  hipMemcpyAsync(c->x, x, nb, kind, s);
  hipMemcpyAsync(c->y, y, nb, kind, s);
  hipMemsetAsync(c->f, 0, nb, s);
  for (int i = 0; i < 2; ++i) hipMemcpyAsync(c->H[i].x, c->x, nb, hipMemcpyDeviceToDevice, s);
  // initial state and the factor of K~_1 at the starting length-scale
  DevState init{};
  init.tau = cfg.tau0;
  init.sigf2 = cfg.sigf2_0;
  init.k = cfg.grid_center;
  *c->st_host = init;
  hipMemcpyAsync(c->st, c->st_host, sizeof(DevState), hipMemcpyHostToDevice, s);
  c->k = cfg.grid_center;
  c->cur = 0;
  c->H[0].pk = c->packs[c->k];
  launch_build(c->H[0], s);
  c->W[0].H = &c->H[0];
  c->W[0].alpha = 1.0;
  c->W[0].beta = 0.0;
  launch_factor(c->W[0], nullptr, nullptr, nullptr, s);
  hipMemcpyAsync(&c->st->logdet1, c->W[0].logdet, sizeof(double), hipMemcpyDeviceToDevice, s);
  if (sync && hipStreamSynchronize(s) != hipSuccess) return fail(FG_EDEVICE, "chain set-up failed on the device");
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FG_EDEVICE, std::string("chain set-up: ") + hipGetErrorString(e));
  *out = c;
  return FG_OK;
}

void chain_destroy_idle(fg_chain c) { chain_free(c, false); }

hipError_t chain_begin_sweep(fg_chain c, hipStream_t s, bool again) {
  if (!again) c->pending = propose(c);
  prepare_sweep(c, c->pending);
  enqueue_sweep(c, c->pending, s, false);
  const hipError_t e = c->enq_err;
  c->enq_err = hipSuccess;
  return e;
}

bool chain_end_sweep(fg_chain c, hipStream_t s) {
  if (sweep_retry(c, s)) return true;
  finish_sweep(c, c->pending);
  return false;
}

const double* chain_f(fg_chain c) { return c->f; }

// ten plan arrays per grid point; eleven per compressed matrix and eleven per factor,
// with three of each; the chain's ten vectors and state words; the PCG workspace
size_t chain_alloc_count(const fg_chain_cfg& cfg) {
  return 10 * (size_t)std::max(cfg.grid_size, 1) + 2 * 11 + 4 * 12 + 10 + 8;
}

size_t chain_device_bytes(fg_chain c) {
  size_t pb = 0;
  for (auto* p : c->packs) pb += plan_device_bytes(*p);
  return chain_bytes_from(c->caps, pb, c->n, c->mixed);  // (a fallback uses the room kept)
}
int64_t chain_iteration(fg_chain c) { return c->iter; }
}  // namespace fg

extern "C" {

fg_status fg_footprint_bytes(const fg_chain_cfg* cfg, const double* x_host, int64_t n,
                             uint64_t* bytes) {
  if (!cfg || !x_host || !bytes) return cfail(FG_EINVAL, "NULL argument");
  if (n < 1 || n >= (int64_t(1) << 31)) return cfail(FG_EINVAL, "n out of range");
  if (cfg->grid_size < 1 || cfg->grid_center < 0 || cfg->grid_center >= cfg->grid_size)
    return cfail(FG_EINVAL, "bad grid");
  // the capacity the chain takes is the largest over every plan of its grid
  fg::ChainPlans plans;
  std::string err;
  const fg_status st = fg::chain_plan(*cfg, x_host, int(n), plans, err);
  if (st != FG_OK) return cfail(st, err);
  *bytes = plans.bytes;
  return FG_OK;
}


fg_status gibbs_chain_create(const fg_chain_cfg* cfg, const double* x, const double* y, int64_t n,
                             fg_stream stream, fg_chain* out) {
  if (!out) return cfail(FG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || !x || !y) return cfail(FG_EINVAL, "NULL argument");
  if (n < 1 || n >= (int64_t(1) << 31)) return cfail(FG_EINVAL, "n out of range");
  // the configuration is checked before any device call
  if (cfg->grid_size < 1 || cfg->grid_center < 0 || cfg->grid_center >= cfg->grid_size)
    return cfail(FG_EINVAL, "bad grid");
  if (!(cfg->tau0 > 0) || !(cfg->sigf2_0 > 0) || !(cfg->ell0 > 0))
    return cfail(FG_EINVAL, "tau0, sigf2_0 and ell0 must be > 0");
  if (cfg->precision != FG_FP64 && cfg->precision != FG_MIXED)
    return cfail(FG_EINVAL, "bad precision");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<double> xh(n);
  if (hipMemcpyAsync(xh.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return cfail(FG_EDEVICE, "copy of x to the host failed");
  std::string err;
  fg::ChainPlans plans;
  fg_status st = fg::chain_plan(*cfg, xh.data(), int(n), plans, err);
  if (st != FG_OK) return cfail(st, err);
  st = fg::chain_create_planned(*cfg, plans, x, y, false, int(n), s, nullptr, true, out, err);
  return st == FG_OK ? FG_OK : cfail(st, err);
}

fg_status gibbs_chain_create_collapsed(const fg_chain_cfg* cfg, const double* x, const double* y,
                                       int64_t n, fg_stream stream, fg_chain* out) {
  if (!out) return cfail(FG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || !x || !y) return cfail(FG_EINVAL, "NULL argument");
  if (n < 1 || n >= (int64_t(1) << 31)) return cfail(FG_EINVAL, "n out of range");
  if (cfg->precision != FG_FP64) return cfail(FG_EINVAL, "collapsed chains run in FP64");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<double> xh(n), yh(n);
  if (hipMemcpyAsync(xh.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(yh.data(), y, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return cfail(FG_EDEVICE, "copy of x, y to the host failed");
  // group equal inputs (stable order inside a group), then average
  std::vector<int64_t> idx(n);
  for (int64_t i = 0; i < n; ++i) {
    if (!(xh[i] == xh[i])) return cfail(FG_EINVAL, "x holds a NaN");
    idx[i] = i;
  }
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return xh[a] < xh[b]; });
  std::vector<double> xu, ybar, w;
  std::vector<int64_t> start;
  for (int64_t k = 0; k < n; ++k) {
    if (k == 0 || xh[idx[k]] != xh[idx[k - 1]]) {
      xu.push_back(xh[idx[k]]);
      ybar.push_back(0.0);
      w.push_back(0.0);
      start.push_back(k);
    }
    ybar.back() += yh[idx[k]];
    w.back() += 1.0;
  }
  const int64_t u = (int64_t)xu.size();
  for (int64_t i = 0; i < u; ++i) ybar[i] /= w[i];
  double within = 0.0;
  for (int64_t i = 0; i < u; ++i) {
    const int64_t e = (i + 1 < u) ? start[i + 1] : n;
    for (int64_t k = start[i]; k < e; ++k) {
      const double d = yh[idx[k]] - ybar[i];
      within += d * d;
    }
  }
  double *dx = nullptr, *dy = nullptr;
  if (fg::dev_alloc(reinterpret_cast<void**>(&dx), sizeof(double) * u) != hipSuccess || fg::dev_alloc(reinterpret_cast<void**>(&dy), sizeof(double) * u) != hipSuccess) {
    if (dx) fg::dev_free(dx);
    (void)hipGetLastError();
    return cfail(FG_ENOMEM, "device allocation failed");
  }
  hipMemcpyAsync(dx, xu.data(), sizeof(double) * u, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(dy, ybar.data(), sizeof(double) * u, hipMemcpyHostToDevice, s);
  fg_chain c = nullptr;
  fg_status st = gibbs_chain_create(cfg, dx, dy, u, stream, &c);  // synchronises s
  fg::dev_free(dx);
  fg::dev_free(dy);
  if (st != FG_OK) return st;
  if (fg::dev_alloc(reinterpret_cast<void**>(&c->cw), sizeof(double) * 3 * (size_t)u) != hipSuccess) {
    chain_free(c);
    (void)hipGetLastError();
    return cfail(FG_ENOMEM, "device allocation failed");
  }
  hipMemcpyAsync(c->cw, w.data(), sizeof(double) * u, hipMemcpyHostToDevice, s);
  if (hipStreamSynchronize(s) != hipSuccess) {
    chain_free(c);
    return cfail(FG_EDEVICE, "copy of the counts failed");
  }
  c->collapsed = true;
  c->within = within;
  c->n_obs = n;
  *out = c;
  return FG_OK;
}

fg_status gibbs_chain_create_grid(const fg_chain_cfg* cfg, const double* x, const double* y,
                                  int64_t n, fg_stream stream, fg_chain* out) {
  if (!out) return cfail(FG_EINVAL, "out is NULL");
  *out = nullptr;
  if (cfg && cfg->precision != FG_FP64) return cfail(FG_EINVAL, "grid chains run in FP64");
  fg_chain c = nullptr;
  fg_status st = gibbs_chain_create(cfg, x, y, n, stream, &c);
  if (st != FG_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int G = cfg->grid_size;
  std::string err;
  c->Hg.resize(G);
  c->Wg.resize(G);
  for (int h = 0; h < G; ++h) {
    if ((st = fg::hodlr_alloc(c->Hg[h], c->caps, err)) != FG_OK ||
        (st = fg::factor_alloc(c->Wg[h], c->caps, err)) != FG_OK) {
      chain_free(c);
      return cfail(st, err + " (grid factorizations)");
    }
  }
  const size_t nb = sizeof(double) * (size_t)c->n;
  if (fg::dev_alloc(reinterpret_cast<void**>(&c->ldg), sizeof(double) * G) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->qg), sizeof(double) * G) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->qbuf), (size_t)std::max(G, 4) * nb) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->qdot), sizeof(double) * std::max(G, 4) * 2048) != hipSuccess) {
    chain_free(c);
    (void)hipGetLastError();
    return cfail(FG_ENOMEM, "grid chain allocation failed");
  }
  for (int q = 0; q < 4; ++q)
    if (hipStreamCreateWithFlags(&c->qs[q], hipStreamNonBlocking) != hipSuccess) {
      chain_free(c);
      return cfail(FG_EDEVICE, "stream creation failed");
    }
  for (auto& e : c->qev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      chain_free(c);
      return cfail(FG_EDEVICE, "event creation failed");
    }
  // every grid point's K~_1, W_1 and log-determinant, once
  for (int h = 0; h < G; ++h) {
    fg::HodlrData& H = c->Hg[h];
    fg::FactorData& W = c->Wg[h];
    hipMemcpyAsync(H.x, c->x, nb, hipMemcpyDeviceToDevice, s);
    H.pk = c->packs[h];
    fg::launch_build(H, s);
    W.H = &H;
    W.alpha = 1.0;
    W.beta = 0.0;
    fg::launch_factor(W, nullptr, nullptr, nullptr, s);
    hipMemcpyAsync(c->ldg + h, W.logdet, sizeof(double), hipMemcpyDeviceToDevice, s);
  }
  int bad = 0;
  for (int h = 0; h < G && hipStreamSynchronize(s) == hipSuccess; ++h) {
    int hs = 0, ws = 0;
    hipMemcpy(&hs, c->Hg[h].status, sizeof(int), hipMemcpyDeviceToHost);
    hipMemcpy(&ws, c->Wg[h].status, sizeof(int), hipMemcpyDeviceToHost);
    bad |= hs | ws;
  }
  if (hipGetLastError() != hipSuccess) {
    chain_free(c);
    return cfail(FG_EDEVICE, "grid factorizations failed on the device");
  }
  if (bad & fg::ST_NOTSPD) {
    chain_free(c);
    return cfail(FG_ENOTSPD, "a grid point's K~_1 is not positive definite");
  }
  c->exact = true;
  *out = c;
  return FG_OK;
}

fg_status gibbs_chain_inputs(fg_chain c, int64_t* n_points, int64_t* n_obs, double* x_out,
                             double* counts_out, fg_stream stream) {
  if (!c) return cfail(FG_EINVAL, "NULL chain");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t nb = sizeof(double) * (size_t)c->n;
  if (n_points) *n_points = c->n;
  if (n_obs) *n_obs = c->collapsed ? c->n_obs : c->n;
  if (x_out) hipMemcpyAsync(x_out, c->x, nb, hipMemcpyDeviceToDevice, s);
  if (counts_out) {
    if (c->collapsed)
      hipMemcpyAsync(counts_out, c->cw, nb, hipMemcpyDeviceToDevice, s);
    else {  // every input once
      const std::vector<double> ones((size_t)c->n, 1.0);
      hipMemcpyAsync(counts_out, ones.data(), nb, hipMemcpyHostToDevice, s);
      (void)hipStreamSynchronize(s);
    }
  }
  return hipGetLastError() == hipSuccess ? FG_OK : cfail(FG_EDEVICE, "copy failed");
}

fg_status gibbs_step(fg_chain c, int32_t iters, fg_stream stream) {
  if (!c || iters < 0) return cfail(FG_EINVAL, "bad arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int it = 0; it < iters; ++it) {
    const Proposal pr = propose(c);
    for (;;) {
      prepare_sweep(c, pr);
      enqueue_sweep(c, pr, s, true);
      if (c->enq_err != hipSuccess) {
        const hipError_t e = c->enq_err;
        c->enq_err = hipSuccess;
        return cfail(FG_EDEVICE, std::string("sweep enqueue: ") + hipGetErrorString(e));
      }
      if (hipStreamSynchronize(s) != hipSuccess) return cfail(FG_EDEVICE, "sweep failed on the device");
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return cfail(FG_EDEVICE, std::string("sweep launch: ") + hipGetErrorString(e));
      if (!sweep_retry(c, s)) break;
    }
    finish_sweep(c, pr);
  }
  return FG_OK;
}

// One batched sweep of `chains` in a fixed mode (the batch lock is held).
static fg_status batch_sweep(fg_chain* chains, int nchains, int mode, int nstreams) {
  fg_status st = FG_OK;
  std::vector<Proposal> pr(nchains);
  for (int i = 0; i < nchains; ++i) pr[i] = propose(chains[i]);
  std::vector<int> run(nchains), again;
  for (int i = 0; i < nchains; ++i) run[i] = i;
  auto enq_fail = [&](fg_chain c) -> fg_status {
    const hipError_t e = c->enq_err;
    c->enq_err = hipSuccess;
    return cfail(FG_EDEVICE, std::string("sweep enqueue: ") + hipGetErrorString(e));
  };
  // every chain's sweep, then again for the chains whose PCG budget was too small
  while (!run.empty()) {
    if (mode == FG_BATCH_GROUPED) {
      // each chain's sweep is recorded, then all are replayed as grouped launches on the
      // first batch stream
      if (g_batch.recs.size() < (size_t)nchains) g_batch.recs.resize(nchains);
      std::vector<fg::Recorder*> rp;
      for (int i : run) {
        fg_chain c = chains[i];
        fg::Recorder* r = &g_batch.recs[i];
        r->clear();
        {
          fg::RecordScope scope(r);
          prepare_sweep(c, pr[i]);
          enqueue_sweep(c, pr[i], g_batch.s[0], false);
        }
        if (c->enq_err != hipSuccess) return enq_fail(c);
        rp.push_back(r);
      }
      std::string err;
      if ((st = g_batch.exec.run(rp, g_batch.s[0], err)) != FG_OK) return cfail(st, err);
    } else {
      for (int i : run) {
        fg_chain c = chains[i];
        hipStream_t q = g_batch.s[i % nstreams];
        prepare_sweep(c, pr[i]);
        if (mode == FG_BATCH_EAGER) {
          enqueue_sweep(c, pr[i], q, false);
          if (c->enq_err != hipSuccess) return enq_fail(c);
          continue;
        }
        hipGraphExec_t ge = nullptr;
        if ((st = sweep_graph(c, pr[i], q, ge)) != FG_OK) return st;
        if (hipGraphLaunch(ge, q) != hipSuccess) return cfail(FG_EDEVICE, "graph launch failed");
      }
    }
    const int used = mode == FG_BATCH_GROUPED ? 1 : nstreams;
    for (int q = 0; q < used; ++q)
      if (hipStreamSynchronize(g_batch.s[q]) != hipSuccess)
        return cfail(FG_EDEVICE, "batched sweep failed on the device");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cfail(FG_EDEVICE, std::string("batched sweep: ") + hipGetErrorString(e));
    again.clear();
    for (int i : run)
      if (sweep_retry(chains[i], g_batch.s[mode == FG_BATCH_GROUPED ? 0 : i % nstreams]))
        again.push_back(i);
    run.swap(again);
  }
  for (int i = 0; i < nchains; ++i) finish_sweep(chains[i], pr[i]);
  return FG_OK;
}

// The batch autotuner's key: the chain count and the largest chain's size and precision.
static uint64_t tune_key(fg_chain* chains, int nchains) {
  int nmax = 0;
  bool mixed = false;
  for (int i = 0; i < nchains; ++i) {
    nmax = std::max(nmax, chains[i]->n);
    mixed |= chains[i]->mixed;
  }
  return ((uint64_t)nchains << 33) | ((uint64_t)nmax << 1) | (mixed ? 1u : 0u);
}

fg_status gibbs_step_batch(fg_chain* chains, int32_t nchains, int32_t iters, int32_t nstreams,
                           int32_t mode, fg_stream stream) {
  if (!chains || nchains < 0 || iters < 0 || nstreams < 1 || nstreams > BATCH_STREAMS ||
      mode < FG_BATCH_EAGER || mode > FG_BATCH_AUTO)
    return cfail(FG_EINVAL, "bad arguments");
  for (int i = 0; i < nchains; ++i) {
    if (!chains[i]) return cfail(FG_EINVAL, "NULL chain");
    for (int j = 0; j < i; ++j)
      if (chains[j] == chains[i]) return cfail(FG_EINVAL, "a chain appears twice");
  }
  hipStream_t caller = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> batch_lock(g_batch.mu);
  fg_status st = batch_streams_init();
  if (st != FG_OK) return st;
  // the batch starts after the work already queued on the caller's stream
  if (hipEventRecord(g_batch.ev_in, caller) != hipSuccess) return cfail(FG_EDEVICE, "event record failed");
  for (int q = 0; q < BATCH_STREAMS; ++q)
    if (hipStreamWaitEvent(g_batch.s[q], g_batch.ev_in, 0) != hipSuccess)
      return cfail(FG_EDEVICE, "stream wait failed");
  // live kernel timing records events at launch: no recorded or captured launches then
  const bool timing = fg::timer_active();
  const uint64_t key = tune_key(chains, nchains);
  for (int it = 0; it < iters; ++it) {
    int m = mode, ns = nstreams;
    if (mode == FG_BATCH_AUTO) {
      // The autotuner: while the batch's signature has no choice yet, each sweep runs in
      // the next candidate (mode, streams), two sweeps per candidate (the second one timed,
      // so that graph capture is not counted); then the fastest is kept.  Every mode gives
      // the same results bit for bit, so the trial sweeps are ordinary sweeps.
      BatchTune& t = g_batch.tune[key];
      if (t.done) {
        m = t.mode;
        ns = t.nstreams;
      } else {
        const BatchCand& cd = TUNE_CANDS[t.trial / 2];
        m = cd.mode;
        ns = cd.nstreams;
      }
    }
    if (timing && m != FG_BATCH_EAGER) m = FG_BATCH_EAGER;
    const auto t0 = std::chrono::steady_clock::now();
    if ((st = batch_sweep(chains, nchains, m, ns)) != FG_OK) return st;
    const double ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t0).count();
    if (mode == FG_BATCH_AUTO && !timing) {
      BatchTune& t = g_batch.tune[key];
      if (!t.done) {
        if (t.trial % 2 == 1 && (t.best_ms < 0 || ms < t.best_ms)) {
          t.best_ms = ms;
          t.mode = m;
          t.nstreams = ns;
        }
        if (++t.trial == 2 * NTUNE) t.done = true;
      }
    }
  }
  return FG_OK;
}

fg_status gibbs_batch_tuning(fg_chain* chains, int32_t nchains, int32_t* mode, int32_t* nstreams,
                             double* ms_per_sweep) {
  if (!chains || nchains < 1 || !mode || !nstreams) return cfail(FG_EINVAL, "bad arguments");
  for (int i = 0; i < nchains; ++i)
    if (!chains[i]) return cfail(FG_EINVAL, "NULL chain");
  std::lock_guard<std::mutex> batch_lock(g_batch.mu);
  auto itr = g_batch.tune.find(tune_key(chains, nchains));
  if (itr == g_batch.tune.end() || !itr->second.done) {
    *mode = -1;
    *nstreams = 0;
    if (ms_per_sweep) *ms_per_sweep = 0.0;
    return FG_OK;
  }
  *mode = itr->second.mode;
  *nstreams = itr->second.nstreams;
  if (ms_per_sweep) *ms_per_sweep = itr->second.best_ms;
  return FG_OK;
}

fg_status gibbs_chain_state(fg_chain c, fg_chain_snapshot* host_out, double* f_out, double* r_out,
                            double* mu_out, fg_stream stream) {
  if (!c || !host_out) return cfail(FG_EINVAL, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t nb = sizeof(double) * c->n;
  if (f_out) hipMemcpyAsync(f_out, c->f, nb, hipMemcpyDeviceToDevice, s);
  if (r_out) hipMemcpyAsync(r_out, c->r, nb, hipMemcpyDeviceToDevice, s);
  if (mu_out) hipMemcpyAsync(mu_out, c->mu, nb, hipMemcpyDeviceToDevice, s);
  hipMemcpyAsync(c->st_host, c->st, sizeof(fg::DevState), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return cfail(FG_EDEVICE, "state copy failed");
  int fst = 0;
  int hs = 0, ws = 0, ms = 0;
  hipMemcpy(&hs, Hcur(c).status, sizeof(int), hipMemcpyDeviceToHost);
  hipMemcpy(&ws, Wcur(c).status, sizeof(int), hipMemcpyDeviceToHost);
  hipMemcpy(&ms, (c->fell_back ? c->WM64 : c->WM).status, sizeof(int), hipMemcpyDeviceToHost);
  fst = c->st_host->status | hs | ws | ms;
  const fg::DevState& d = *c->st_host;
  host_out->iteration = c->iter;
  host_out->tau = d.tau;
  host_out->sigf2 = d.sigf2;
  host_out->k = d.k;
  host_out->ell = c->grid[d.k];
  host_out->last_proposal = d.kprop;
  host_out->last_accept = d.accept;
  host_out->accepts = d.accepts;
  host_out->logdet_sigma = d.logdet_sigma;
  host_out->yr = d.yr;
  host_out->loglik = d.loglik;
  host_out->sse = d.sse;
  host_out->q = d.q;
  host_out->logdet1 = d.logdet1;
  host_out->mh_log_ratio = d.mh;
  host_out->status = (fst & fg::ST_NOTSPD) ? FG_ENOTSPD : (fst & fg::ST_NOTCONV) ? FG_ENOTCONV : FG_OK;
  if (host_out->status == FG_OK && c->pcg_failed) host_out->status = FG_ENOTCONV;
  host_out->pcg_iters = c->pcg_iters;
  host_out->pcg_relres = c->pcg_relres;
  host_out->precision_used = (c->mixed && !c->fell_back) ? FG_MIXED : FG_FP64;
  return FG_OK;
}

static void predict_release(fg_chain c) {
  for (auto& e : c->zcache)
    if (e.z) fg::dev_free(e.z);
  c->zcache.clear();
  for (double** b : {&c->xstar, &c->pwork}) {
    if (*b) fg::dev_free(*b);
    *b = nullptr;
  }
  c->nstar = 0;
  c->zcache_cap = 0;
}

fg_status gibbs_predict_inputs(fg_chain c, const double* xstar, int64_t nstar,
                               int32_t max_grid_points, fg_stream stream) {
  if (!c || nstar < 0 || (nstar > 0 && (!xstar || max_grid_points < 1)))
    return cfail(FG_EINVAL, "bad arguments");
  if (nstar > (int64_t)fg::MAX_NSTAR) return cfail(FG_EINVAL, "too many new inputs");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // work already queued on the stream may still read the old buffers
  if (hipStreamSynchronize(s) != hipSuccess) return cfail(FG_EDEVICE, "stream failed");
  predict_release(c);
  if (nstar == 0) return FG_OK;
  const size_t n = (size_t)c->n, m = (size_t)nstar;
  double* z0 = nullptr;
  if (fg::dev_alloc(reinterpret_cast<void**>(&c->xstar), sizeof(double) * m) != hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&c->pwork), sizeof(double) * (n + m + fg::predict_part_doubles(c->n, (int)m))) !=
          hipSuccess ||
      fg::dev_alloc(reinterpret_cast<void**>(&z0), sizeof(double) * n * m) != hipSuccess) {
    if (z0) fg::dev_free(z0);
    predict_release(c);
    (void)hipGetLastError();
    return cfail(FG_ENOMEM, "device allocation for the new inputs failed");
  }
  c->zcache.push_back({-1, z0, 0});
  c->zcache_cap = max_grid_points;
  if (hipMemcpyAsync(c->xstar, xstar, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return cfail(FG_EDEVICE, "copy of the new inputs failed");
  c->nstar = (int)nstar;
  return FG_OK;
}

// The Z of the current grid point: a cached one, else an empty slot, a new slot while
// fewer than zcache_cap exist (and the allocation succeeds), or the least recently used.
static double* predict_z(fg_chain c, hipStream_t s) {
  const int n = c->n, N = c->nstar;
  ++c->zclock;
  for (auto& e : c->zcache)
    if (e.k == c->k) {
      e.used = c->zclock;
      return e.z;
    }
  fg_chain_s::ZEntry* slot = nullptr;
  for (auto& e : c->zcache)
    if (e.k < 0) { slot = &e; break; }
  if (!slot && (int)c->zcache.size() < c->zcache_cap) {
    double* z = nullptr;
    if (fg::dev_alloc(reinterpret_cast<void**>(&z), sizeof(double) * (size_t)n * (size_t)N) == hipSuccess) {
      c->zcache.push_back({-1, z, 0});
      slot = &c->zcache.back();
    } else {
      (void)hipGetLastError();
    }
  }
  if (!slot) {
    slot = &c->zcache[0];
    for (auto& e : c->zcache)
      if (e.used < slot->used) slot = &e;
  }
  fg::FactorData& W1 = Wcur(c);
  fg::launch_cross_cov(c->x, n, c->xstar, N, c->cfg.kind, c->grid[c->k], slot->z, n, s);
  for (int j = 0; j < N; j += 4)
    fg::launch_apply_w(W1, 2, slot->z + (size_t)j * n, std::min(4, N - j), n, W1.work, s);
  slot->k = c->k;
  slot->used = c->zclock;
  ++c->zbuilds;
  return slot->z;
}

fg_status gibbs_predict(fg_chain c, double* fstar, double* mu, double* s2, fg_stream stream) {
  if (!c || !fstar) return cfail(FG_EINVAL, "NULL argument");
  if (c->nstar == 0) return cfail(FG_EINVAL, "no new inputs set (gibbs_predict_inputs)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n = c->n, N = c->nstar;
  fg::FactorData& W1 = Wcur(c);
  const double* Z = predict_z(c, s);
  double* zf = c->pwork;
  double* xi = zf + n;
  hipMemcpyAsync(zf, c->f, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
  fg::launch_apply_w(W1, 2, zf, 1, n, W1.work, s);
  fg::launch_normals(c->cfg.seed, 8, (uint64_t)c->iter, c->cfg.stream_id, N, xi, s);
  fg::launch_predict_point(Z, n, n, zf, xi, &c->st->sigf2, c->cfg.nugget, N, xi + N, fstar, mu,
                           s2, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cfail(FG_EDEVICE, std::string("predict launch: ") + hipGetErrorString(e));
  return FG_OK;
}

fg_status gibbs_predict_stats(fg_chain c, int32_t* cached_grid_points, int64_t* builds) {
  if (!c) return cfail(FG_EINVAL, "NULL chain");
  int used = 0;
  for (auto& e : c->zcache) used += e.k >= 0;
  if (cached_grid_points) *cached_grid_points = used;
  if (builds) *builds = c->zbuilds;
  return FG_OK;
}

void gibbs_chain_destroy(fg_chain c) { chain_free(c); }

}  // extern "C"
