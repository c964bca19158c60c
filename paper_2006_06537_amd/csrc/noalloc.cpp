// hodlr_solve_refined_noalloc: the refined solve with its PCG workspace in a fixed device
// array of this library instead of a per-call allocation, for callers that cannot
// allocate.  The array is one per GPU (each device holds its own copy, at its own address,
// until the process ends); its address on a device is taken once, with that device
// current, from the runtime's symbol table.  Calls on one GPU share the array: calls that
// overlap in time on the same GPU race.
#include <mutex>
#include <string>

#include "fg_internal.h"
#include "fg_pcg.h"

namespace {

constexpr int64_t NOALLOC_MAX = int64_t(1) << 20;  // n * nrhs of one call
constexpr size_t DOT_DOUBLES = 1024 * 4 * fg::NRHS_PCG;
constexpr size_t SC_DOUBLES = (sizeof(fg::PcgScalars) + 255) / 256 * 32;
constexpr size_t SCRATCH_DOUBLES = 4 * (size_t)NOALLOC_MAX + DOT_DOUBLES + SC_DOUBLES;

// r, z, p, q (nrhs columns of n each), the dot-product partials, the PCG scalars
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each device

// the array's address on the current device (looked up once per device)
fg_status scratch_ptr(double** out, std::string& err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    err = "no current device";
    return FG_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      err = "address of the scratch array not found";
      return FG_EDEVICE;
    }
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return FG_OK;
}

}  // namespace

// the two handles' internals (defined in abi.cpp)
namespace fg {
const HodlrData* hodlr_data(fg_hodlr A);
FactorData* factor_data(fg_factor F);
int factor_n(fg_factor F);
}  // namespace fg

extern "C" fg_status hodlr_solve_refined_noalloc(fg_hodlr A, fg_factor F, double alpha, double beta,
                                                 const double* b, double* x, int32_t nrhs,
                                                 int64_t ld, double rtol, int32_t maxit,
                                                 int32_t* iters, double* relres, fg_stream stream) {
  if (!A || !F || !b || !x) {
    fg::set_error("NULL argument");
    return FG_EINVAL;
  }
  const fg::HodlrData& H = *fg::hodlr_data(A);
  fg::FactorData& M = *fg::factor_data(F);
  const int n = H.pk->P.n;
  if (fg::factor_n(F) != n || M.H != &H) {
    fg::set_error("F is not a factor of A");
    return FG_EINVAL;
  }
  if (nrhs < 1 || nrhs > fg::NRHS_PCG || ld < n) {
    fg::set_error("bad nrhs or ld");
    return FG_EINVAL;
  }
  if ((int64_t)n * nrhs > NOALLOC_MAX) {
    fg::set_error("n * nrhs = " + std::to_string((int64_t)n * nrhs) + " exceeds the scratch "
                  "array of hodlr_solve_refined_noalloc (at most " + std::to_string(NOALLOC_MAX) +
                  "); use hodlr_solve_refined");
    return FG_EINVAL;
  }
  if (!(rtol > 0.0) || maxit < 1 || !(alpha > 0.0) || !(beta >= 0.0)) {
    fg::set_error("rtol and alpha must be > 0, beta >= 0, maxit >= 1");
    return FG_EINVAL;
  }
  std::string err;
  double* base = nullptr;
  fg_status st = scratch_ptr(&base, err);
  if (st != FG_OK) {
    fg::set_error(err);
    return st;
  }
  // the workspace, carved from the array: columns of n per right-hand side
  fg::PcgWork w;
  const size_t v = (size_t)nrhs * n;
  w.n = n;
  w.r = base;
  w.z = base + v;
  w.p = base + 2 * v;
  w.q = base + 3 * v;
  w.dotwork = base + 4 * (size_t)NOALLOC_MAX;
  w.sc = reinterpret_cast<fg::PcgScalars*>(w.dotwork + DOT_DOUBLES);
  fg::PcgScalars host_sc{};  // the convergence record read back (pageable, on the stack)
  w.sc_host = &host_sc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = fg::pcg_solve(H, alpha, nullptr, beta, M, b, x, nrhs, int(ld), rtol, maxit, w, s, iters,
                     relres, err);
  if (st != FG_OK) {
    fg::set_error(err);
    return st;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fg::set_error(std::string("hodlr_solve_refined_noalloc: ") + hipGetErrorString(e));
    return FG_EDEVICE;
  }
  return FG_OK;
}
