// Device resources of plans, compressed matrices and factors (host code).
#include <algorithm>
#include <cstring>

#include "fg_internal.h"
#include "fg_timer.h"

namespace fg {

template <class T>
static fg_status dalloc(T** p, size_t count, std::string& err) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (dev_alloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    err = "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed";
    return FG_ENOMEM;
  }
  return FG_OK;
}

template <class T>
static void dfree(T*& p) {
  if (p) dev_free(p);
  p = nullptr;
}

template <class T>
static fg_status upload(T** dst, const std::vector<T>& v, hipStream_t s, std::string& err) {
  fg_status st = dalloc(dst, v.size(), err);
  if (st != FG_OK) return st;
  if (!v.empty() &&
      hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess) {
    err = "plan upload failed";
    return FG_EDEVICE;
  }
  return FG_OK;
}

// buffer sizes of a plan (host only)
void plan_pack_sizes(PlanPack* pk) {
  HostPlan& P = pk->P;
  // per node offsets of (G_V, F1, F2) and factor scratch sizes
  pk->nodemat_off.resize(std::max(P.nint, 1));
  size_t off = 0;
  for (int h = 0; h < P.nint; ++h) {
    pk->nodemat_off[h] = int(off);
    const size_t kc = P.kcap[P.nodes[h].level];
    off += 3 * kc * kc;
  }
  pk->nodemat_size = std::max<size_t>(off, 1);
  for (int l = 0; l < P.L; ++l) {
    const size_t Wcap = P.coff[l + 1];
    const size_t per = (size_t)P.kcap[l] * Wcap;
    const size_t nt = P.ltask_off[l + 1] - P.ltask_off[l];
    pk->zpart_size = std::max(pk->zpart_size, nt * per);
    pk->zfin_size = std::max(pk->zfin_size, (size_t(1) << l) * 2 * per);
    pk->coef_size = std::max(pk->coef_size, (size_t(1) << l) * per);
  }
  pk->mpart_size = (size_t)std::max(P.nmt, 1) * P.mpart_stride;
  pk->mv_work = matvec_work_doubles(P, 4);
  pk->ap_work = apply_work_doubles(P, 4);
}

PlanPack* plan_pack_make(const double* xh, int n, int kind, double ell, double nugget, int leaf,
                         double tol, fg_status& st, std::string& err) {
  PlanPack* pk = new PlanPack();
  st = make_plan(xh, n, kind, ell, nugget, leaf, tol, pk->P, err);
  if (st != FG_OK) { delete pk; return nullptr; }
  plan_pack_sizes(pk);
  return pk;
}

fg_status plan_pack_upload(PlanPack* pk, hipStream_t s, bool sync, std::string& err) {
  fg_status st;
  HostPlan& P = pk->P;
  DevPlan& D = pk->D;
  pk->kc_host = P.kcap;
  pk->co_host = P.coff;
  if (pk->kc_host.empty()) pk->kc_host.push_back(0);
  if ((st = upload(&D.nodes, P.nodes, s, err)) != FG_OK ||
      (st = upload(&D.leaf_lo, P.leaf_lo, s, err)) != FG_OK ||
      (st = upload(&D.mtasks, P.mtasks, s, err)) != FG_OK ||
      (st = upload(&D.mtask_off, P.mtask_off, s, err)) != FG_OK ||
      (st = upload(&D.gtasks, P.gtasks, s, err)) != FG_OK ||
      (st = upload(&D.ltasks, P.ltasks, s, err)) != FG_OK ||
      (st = upload(&D.node_task_off, P.node_task_off, s, err)) != FG_OK ||
      (st = upload(&D.coff, pk->co_host, s, err)) != FG_OK ||
      (st = upload(&D.kcap, pk->kc_host, s, err)) != FG_OK ||
      (st = upload(&D.nodemat_off, pk->nodemat_off, s, err)) != FG_OK)
    return st;
  if (!sync) return FG_OK;  // the host vectors stay until the pack is destroyed
  // the uploads read host vectors: finish them before the vectors are released
  if (hipStreamSynchronize(s) != hipSuccess) {
    err = "stream synchronisation failed";
    return FG_EDEVICE;
  }
  std::vector<Task>().swap(P.mtasks);
  std::vector<Task>().swap(P.gtasks);
  std::vector<Task>().swap(P.ltasks);
  return FG_OK;
}

PlanPack* plan_pack_create(const double* xh, int n, int kind, double ell, double nugget, int leaf,
                           double tol, hipStream_t s, fg_status& st, std::string& err) {
  PlanPack* pk = plan_pack_make(xh, n, kind, ell, nugget, leaf, tol, st, err);
  if (!pk) return nullptr;
  if ((st = plan_pack_upload(pk, s, true, err)) != FG_OK) {
    plan_pack_destroy(pk);
    return nullptr;
  }
  return pk;
}

void plan_pack_destroy(PlanPack* pk) {
  if (!pk) return;
  DevPlan& D = pk->D;
  dfree(D.nodes); dfree(D.leaf_lo); dfree(D.mtasks); dfree(D.mtask_off); dfree(D.gtasks);
  dfree(D.ltasks); dfree(D.node_task_off); dfree(D.coff); dfree(D.kcap); dfree(D.nodemat_off);
  delete pk;
}

void Caps::add(const PlanPack& pk) {
  const HostPlan& P = pk.P;
  n = P.n; B = P.B; L = P.L; nint = P.nint; nleaf = P.nleaf;
  tbuf = std::max(tbuf, (size_t)P.tbuf_size);
  mpart = std::max(mpart, pk.mpart_size);
  Ktot = std::max(Ktot, (size_t)std::max(P.Ktot, 1));
  nodemat = std::max(nodemat, pk.nodemat_size);
  zpart = std::max(zpart, pk.zpart_size);
  zfin = std::max(zfin, pk.zfin_size);
  coef = std::max(coef, pk.coef_size);
  mv_work = std::max(mv_work, pk.mv_work);
  ap_work = std::max(ap_work, pk.ap_work);
}

static int round_ld(int n) { return (n + 63) / 64 * 64; }

size_t plan_device_bytes(const PlanPack& pk) {
  const HostPlan& P = pk.P;
  return sizeof(NodePlan) * std::max(P.nint, 1) + sizeof(int) * (P.nleaf + 1) +
         sizeof(Task) * ((size_t)P.nmt + P.ngt + P.nlt) + sizeof(int) * 2 * (2 * P.nint + 1) +
         sizeof(int) * 2 * std::max(P.L, 1) + sizeof(int) * std::max(P.nint, 1);
}

size_t hodlr_bytes(const Caps& c) {
  const size_t ld = round_ld(c.n), Lm = std::max(c.L, 1), ni = std::max(c.nint, 1);
  return 8 * ((size_t)c.n + c.tbuf + c.mpart + ni * PMAX + ld * c.Ktot + c.mv_work) +
         4 * (ni + 2 * Lm + Lm * c.Ktot + 1);
}

size_t factor_bytes(const Caps& c, bool fp32) {
  const size_t ld = round_ld(c.n), ni = std::max(c.nint, 1);
  const size_t leaves = 2 * (size_t)c.nleaf * c.B * c.B;  // L and its diagonal-block inverses
  return (fp32 ? 4 : 8) * leaves + 8 * ld * c.Ktot +
         8 * ((size_t)c.nleaf + c.nodemat + ni + c.zpart + c.zfin + c.coef + 1 + c.ap_work) + 4;
}

static void zero_bytes(void* p, size_t bytes, hipStream_t s, bool async) {
  if (async)
    (void)hipMemsetAsync(p, 0, bytes, s);
  else
    (void)hipMemset(p, 0, bytes);
}

fg_status hodlr_alloc(HodlrData& H, const Caps& c, std::string& err, hipStream_t s, bool async) {
  fg_status st;
  H.ld = round_ld(c.n);
  const int Lm = std::max(c.L, 1);
  if ((st = dalloc(&H.x, c.n, err)) != FG_OK || (st = dalloc(&H.tbuf, c.tbuf, err)) != FG_OK ||
      (st = dalloc(&H.mpart, c.mpart, err)) != FG_OK ||
      (st = dalloc(&H.sv, (size_t)std::max(c.nint, 1) * PMAX, err)) != FG_OK ||
      (st = dalloc(&H.rank, std::max(c.nint, 1), err)) != FG_OK ||
      (st = dalloc(&H.kmax, Lm, err)) != FG_OK ||
      (st = dalloc(&H.rcols, (size_t)Lm * c.Ktot, err)) != FG_OK ||
      (st = dalloc(&H.rcount, Lm, err)) != FG_OK ||
      (st = dalloc(&H.panel, (size_t)H.ld * c.Ktot, err)) != FG_OK ||
      (st = dalloc(&H.status, 1, err)) != FG_OK || (st = dalloc(&H.work, c.mv_work, err)) != FG_OK) {
    hodlr_free(H);
    return st;
  }
  zero_bytes(H.status, sizeof(int), s, async);
  zero_bytes(H.kmax, sizeof(int) * Lm, s, async);
  return FG_OK;
}

void hodlr_free(HodlrData& H) {
  timer_forget(H.kmax);
  dfree(H.x); dfree(H.tbuf); dfree(H.mpart); dfree(H.sv); dfree(H.rank); dfree(H.kmax);
  dfree(H.rcols); dfree(H.rcount); dfree(H.panel); dfree(H.status); dfree(H.work);
}

fg_status factor_alloc(FactorData& F, const Caps& c, std::string& err, bool fp32, hipStream_t s,
                       bool async) {
  fg_status st = FG_OK;
  const size_t ld = round_ld(c.n);
  const size_t bb = (size_t)c.nleaf * c.B * c.B;
  F.fp32 = fp32;
  const bool ok64 = fp32 || ((st = dalloc(&F.leafL, bb, err)) == FG_OK &&
                             (st = dalloc(&F.leafLinv, bb, err)) == FG_OK);
  const bool ok32 = !fp32 || ((st = dalloc(&F.leafLf, bb, err)) == FG_OK &&
                              (st = dalloc(&F.leafLinvf, bb, err)) == FG_OK);
  if (!ok64 || !ok32 || (st = dalloc(&F.panel, ld * c.Ktot, err)) != FG_OK) {
    factor_free(F);
    return st;
  }
  if ((st = dalloc(&F.leaf_ld, c.nleaf, err)) != FG_OK ||
      (st = dalloc(&F.nodemat, c.nodemat, err)) != FG_OK ||
      (st = dalloc(&F.node_ld, std::max(c.nint, 1), err)) != FG_OK ||
      (st = dalloc(&F.zpart, c.zpart, err)) != FG_OK ||
      (st = dalloc(&F.zfin, c.zfin, err)) != FG_OK || (st = dalloc(&F.coef, c.coef, err)) != FG_OK ||
      (st = dalloc(&F.logdet, 1, err)) != FG_OK || (st = dalloc(&F.status, 1, err)) != FG_OK ||
      (st = dalloc(&F.work, c.ap_work, err)) != FG_OK) {
    factor_free(F);
    return st;
  }
  zero_bytes(F.status, sizeof(int), s, async);
  zero_bytes(F.node_ld, sizeof(double) * std::max(c.nint, 1), s, async);
  return FG_OK;
}

void factor_free(FactorData& F) {
  dfree(F.leafL); dfree(F.leafLinv); dfree(F.leaf_ld); dfree(F.panel); dfree(F.nodemat);
  dfree(F.leafLf); dfree(F.leafLinvf);
  dfree(F.node_ld); dfree(F.zpart); dfree(F.zfin); dfree(F.coef); dfree(F.logdet);
  dfree(F.status); dfree(F.work);
}

}  // namespace fg
