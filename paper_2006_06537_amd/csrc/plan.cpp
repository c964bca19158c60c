// Host-side tree plan of a HODLR build: tree ranges, off-diagonal windows,
// interpolation sizes and the row tasks every device kernel iterates over.
//
// Section 3.2 of the paper fixes the format (recursive 2x2 partition of the sorted
// inputs, dense leaves no larger than the maximum block size B, low-rank off-diagonal
// blocks with a max-norm error bound by construction).  Readings taken here:
//   * a node of m rows splits into floor(m/2) + (m - floor(m/2)); all leaves share
//     the depth L = min{L : ceil(n / 2^L) <= B};
//   * window: left-child rows farther than R from the first right-child input, and
//     right-child rows farther than R from the last left-child input, carry kernel
//     values below tol/3 and are dropped (R = ell sqrt(2 ln(3/tol)) for SE,
//     ell ln(3/tol) for the exponential kernel);
//   * per side, p first-kind Chebyshev nodes on the window's input range, the
//     smallest p whose a-priori interpolation bound is within tol/6 (the right side
//     includes the left side's Lebesgue constant); a window with no more inputs
//     than p uses its inputs as nodes (exact side).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "fg_internal.h"

namespace fg {

// Error of p-node Chebyshev interpolation over half-width h: h^p / (2^(p-1) p!) times a
// bound on |d^p k_1| over the window.  Squared exponential: KAPPA_H ell^-p sqrt(p!)
// (Hermite functions); exponential on separated intervals: ell^-p; Matern on separated
// intervals (u = a t >= 0, a = sqrt(3)/ell or sqrt(5)/ell): the p-th u-derivative of
// (1+u)e^-u is e^-u (1 + u - p) up to sign, at most max(p-1, 1); that of (1+u+u^2/3)e^-u
// is e^-u (1 + u + u^2/3 - p(1 + 2u/3) + p(p-1)/3), at most p^2/3 + p + 1.
static double interp_bound(int kind, int p, double h, double ell) {
  if (h <= 0.0) return 0.0;
  if (kind == FG_KERNEL_MATERN32 || kind == FG_KERNEL_MATERN52) {
    const double a = (kind == FG_KERNEL_MATERN32 ? std::sqrt(3.0) : std::sqrt(5.0)) / ell;
    const double m = kind == FG_KERNEL_MATERN32 ? std::max(p - 1.0, 1.0) : p * p / 3.0 + p + 1.0;
    return std::exp(std::log(2.0 * m) + p * std::log(h * a / 2.0) - std::lgamma(p + 1.0));
  }
  const double r = std::log(h / (2.0 * ell));
  if (kind == FG_KERNEL_SE)
    return std::exp(std::log(2.0 * KAPPA_H) + p * r - 0.5 * std::lgamma(p + 1.0));
  return std::exp(std::log(2.0) + p * r - std::lgamma(p + 1.0));
}

static double lebesgue_bound(int p) { return 2.0 / M_PI * std::log(p + 1.0) + 1.0; }

// distance beyond which k_1 < tol/3; for Matern, P(u) e^-u = tol/3 with P increasing is
// solved by the increasing iteration u <- log(3 P(u) / tol)
static double window_radius(int kind, double ell, double tol) {
  if (kind == FG_KERNEL_SE) return ell * std::sqrt(2.0 * std::log(3.0 / tol));
  if (kind == FG_KERNEL_EXP) return ell * std::log(3.0 / tol);
  const bool m32 = kind == FG_KERNEL_MATERN32;
  double u = std::log(3.0 / tol);
  for (int it = 0; it < 200; ++it) {
    const double poly = m32 ? 1.0 + u : 1.0 + u + u * u / 3.0;
    const double un = std::log(3.0 * poly / tol);
    const bool done = std::fabs(un - u) <= 1e-14 * un;
    u = un;
    if (done) break;
  }
  return ell * u / (m32 ? std::sqrt(3.0) : std::sqrt(5.0));
}

static int choose_p(int kind, double h, double ell, double target, double factor) {
  for (int p = 1; p <= PMAX; ++p)
    if (factor * interp_bound(kind, p, h, ell) <= target) return p;
  return -1;
}

static void chunk(std::vector<Task>& out, int h, int side, int r0, int r1, int ch) {
  for (int r = r0; r < r1; r += ch) out.push_back(Task{h, side, r, std::min(r1, r + ch)});
}

fg_status make_plan(const double* xh, int n, int kind, double ell, double nugget, int leaf,
                    double tol, HostPlan& P, std::string& err) {
  if (n < 1) { err = "n must be >= 1"; return FG_EINVAL; }
  if (leaf < 2 || leaf > BMAX) { err = "leaf must be in [2, 128]"; return FG_EINVAL; }
  if (!(tol > 0.0) || !(ell > 0.0) || !(nugget >= 0.0)) {
    err = "tol and lengthscale must be > 0, nugget >= 0";
    return FG_EINVAL;
  }
  if (kind < FG_KERNEL_SE || kind > FG_KERNEL_MATERN52) { err = "unknown kernel"; return FG_EINVAL; }
  for (int i = 1; i < n; ++i)
    if (!(xh[i] >= xh[i - 1])) { err = "x must be sorted ascending"; return FG_EINVAL; }
  P = HostPlan();
  P.n = n; P.B = leaf; P.kind = kind; P.ell = ell; P.nugget = nugget; P.tol = tol;
  int L = 0;
  while ((n + (1 << L) - 1) / (1 << L) > leaf) ++L;
  P.L = L;
  P.nint = (1 << L) - 1;
  P.nleaf = 1 << L;
  // tree ranges, heap order
  std::vector<int> lo(2 * P.nleaf - 1), hi(2 * P.nleaf - 1);
  lo[0] = 0; hi[0] = n;
  for (int h = 0; h < P.nint; ++h) {
    const int m = hi[h] - lo[h], mid = lo[h] + m / 2;
    lo[2 * h + 1] = lo[h]; hi[2 * h + 1] = mid;
    lo[2 * h + 2] = mid;   hi[2 * h + 2] = hi[h];
  }
  P.leaf_lo.resize(P.nleaf + 1);
  for (int j = 0; j < P.nleaf; ++j) P.leaf_lo[j] = lo[P.nint + j];
  P.leaf_lo[P.nleaf] = n;
  const double R = window_radius(kind, ell, tol);
  P.nodes.resize(P.nint);
  P.kcap.assign(L, 0);
  P.lpmax.assign(std::max(L, 1), 0);
  P.coff.assign(L + 1, 0);
  for (int h = 0; h < P.nint; ++h) {
    NodePlan& q = P.nodes[h];
    std::memset(&q, 0, sizeof(q));
    int l = 0;
    while ((2 << l) - 1 <= h) ++l;
    q.level = l;
    q.lo = lo[h]; q.hi = hi[h]; q.mid = lo[h] + (hi[h] - lo[h]) / 2;
    q.i0 = int(std::lower_bound(xh + q.lo, xh + q.mid, xh[q.mid] - R) - xh);
    q.j1 = int(std::upper_bound(xh + q.mid, xh + q.hi, xh[q.mid - 1] + R) - xh);
    const int mI = q.mid - q.i0, mJ = q.j1 - q.mid;
    if (mI == 0 || mJ == 0) { q.pI = q.pJ = 0; continue; }
    const double hI = 0.5 * (xh[q.mid - 1] - xh[q.i0]);
    const double hJ = 0.5 * (xh[q.j1 - 1] - xh[q.mid]);
    const int pI = choose_p(kind, hI, ell, tol / 6.0, 1.0);
    if (pI < 0) { err = "tolerance needs more than 60 interpolation nodes"; return FG_ETOL; }
    q.exactI = mI <= pI;
    const double lam = q.exactI ? 1.0 : lebesgue_bound(pI);
    const int pJ = choose_p(kind, hJ, ell, tol / 6.0, lam);
    if (pJ < 0) { err = "tolerance needs more than 60 interpolation nodes"; return FG_ETOL; }
    q.exactJ = mJ <= pJ;
    q.pI = q.exactI ? mI : pI;
    q.pJ = q.exactJ ? mJ : pJ;
    q.aI = xh[q.i0]; q.bI = xh[q.mid - 1];
    q.aJ = xh[q.mid]; q.bJ = xh[q.j1 - 1];
    P.kcap[l] = std::max(P.kcap[l], std::min(q.pI, q.pJ));
    P.pmax = std::max(P.pmax, std::max(q.pI, q.pJ));
    P.lpmax[l] = std::max(P.lpmax[l], std::max(q.pI, q.pJ));
  }
  for (int l = 0; l < L; ++l) {
    P.kcap[l] = std::max(P.kcap[l], 1);
    P.coff[l + 1] = P.coff[l] + P.kcap[l];
    P.kcapmax = std::max(P.kcapmax, P.kcap[l]);
  }
  P.Ktot = P.coff[L];
  // T buffers and moments
  int toff = 0, moff = 0;
  for (int h = 0; h < P.nint; ++h) {
    NodePlan& q = P.nodes[h];
    const int kc = P.kcap[q.level];
    q.toff_u = toff; toff += q.pI * kc;
    q.toff_v = toff; toff += q.pJ * kc;
    q.mom_off_i = moff; moff += q.exactI ? 0 : 2 * q.pI - 1;
    q.mom_off_j = moff; moff += q.exactJ ? 0 : 2 * q.pJ - 1;
  }
  P.tbuf_size = std::max(toff, 1);
  P.mom_size = std::max(moff, 1);
  // moment tasks over window rows of interpolated sides
  P.mtask_off.assign(2 * P.nint + 1, 0);
  for (int h = 0; h < P.nint; ++h) {
    const NodePlan& q = P.nodes[h];
    P.mtask_off[2 * h] = int(P.mtasks.size());
    if (q.pI > 0 && !q.exactI) chunk(P.mtasks, h, 0, q.i0, q.mid, MCHM);
    P.mtask_off[2 * h + 1] = int(P.mtasks.size());
    if (q.pJ > 0 && !q.exactJ) chunk(P.mtasks, h, 1, q.mid, q.j1, MCHM);
  }
  P.mtask_off[2 * P.nint] = int(P.mtasks.size());
  P.mpart_stride = 2 * PMAX;
  // panel generation tasks: all rows of both sides of every node
  for (int h = 0; h < P.nint; ++h) {
    const NodePlan& q = P.nodes[h];
    chunk(P.gtasks, h, 0, q.lo, q.mid, MCH);
    chunk(P.gtasks, h, 1, q.mid, q.hi, MCH);
  }
  // level tasks (reduce / update), grouped by level in heap order
  P.ltask_off.assign(L + 1, 0);
  P.node_task_off.assign(2 * P.nint + 1, 0);
  for (int h = 0; h < P.nint; ++h) {
    const NodePlan& q = P.nodes[h];
    if (h == (1 << q.level) - 1) P.ltask_off[q.level] = int(P.ltasks.size());
    P.node_task_off[2 * h] = int(P.ltasks.size());
    chunk(P.ltasks, h, 0, q.lo, q.mid, RCH);
    P.node_task_off[2 * h + 1] = int(P.ltasks.size());
    chunk(P.ltasks, h, 1, q.mid, q.hi, RCH);
  }
  P.node_task_off[2 * P.nint] = int(P.ltasks.size());
  P.ltask_off[L] = int(P.ltasks.size());
  P.max_tps.assign(std::max(L, 1), 1);
  P.max_trows.assign(std::max(L, 1), 1);
  for (const Task& tk : P.ltasks)
    P.max_trows[P.nodes[tk.h].level] = std::max(P.max_trows[P.nodes[tk.h].level], tk.r1 - tk.r0);
  for (int l = 0; l < L; ++l)
    P.max_ltasks = std::max(P.max_ltasks, P.ltask_off[l + 1] - P.ltask_off[l]);
  for (int h = 0; h < P.nint; ++h)
    for (int sd = 0; sd < 2; ++sd)
      P.max_tps[P.nodes[h].level] = std::max(P.max_tps[P.nodes[h].level],
                                             P.node_task_off[2 * h + sd + 1] - P.node_task_off[2 * h + sd]);
  P.nmt = int(P.mtasks.size());
  P.ngt = int(P.gtasks.size());
  P.nlt = int(P.ltasks.size());
  return FG_OK;
}

}  // namespace fg
