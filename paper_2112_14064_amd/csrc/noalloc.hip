// riga_solve_q without device allocation: the solve's workspace lives in a
// static device array of fixed size, one copy per GPU, instead of the
// handle's buffers.  The kernels and the order of the launches are those of
// riga_solve_q (solve_levels with an explicit workspace).
#include "problem.hpp"

#include <mutex>

namespace {

constexpr size_t kScratchDoubles = RIGA_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr int kMaxDevices = 64;

// Host code never uses this name as an address: the device address of each
// GPU's copy comes from hipGetSymbolAddress (scratch_on).
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of the array on `device` (which must be current), looked up
// on the first call there.
double* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) throw riga::detail::HipError{hipErrorInvalidDevice};
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device] == nullptr) {
    void* p = nullptr;
    riga::detail::ck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_ptr[device] = static_cast<double*>(p);
  }
  return g_ptr[device];
}

}  // namespace

extern "C" riga_status riga_solve_q_noalloc(riga_problem* h, int nrhs, const double* b, double* x) {
  if (!h || nrhs < 1 || nrhs > 4 || !b || !x) return RIGA_ERR_INVALID_ARG;
  const size_t N = (size_t)h->N(), U = (size_t)h->upd_len;
  // an FP64 factor needs tmp and upd; a mixed one also the refinement's three vectors
  const size_t need = (size_t)nrhs * ((h->mixed ? 4 * N : N) + U);
  if (need > kScratchDoubles) return RIGA_ERR_SCRATCH;
  if (!h->factored) return RIGA_ERR_STATE;
  return riga::detail::run([&]() -> riga_status {
    riga::detail::ck(hipSetDevice(h->device));
    double* base = scratch_on(h->device);
    riga::detail::SolveWork w{};
    w.tmp = base;
    w.upd = w.tmp + (size_t)nrhs * N;
    if (h->mixed) {
      w.irX = w.upd + (size_t)nrhs * U;
      w.irR = w.irX + (size_t)nrhs * N;
      w.irD = w.irR + (size_t)nrhs * N;
    }
    riga::detail::solve_levels(h, nrhs, b, h->N(), x, h->N(), nullptr, nullptr, 0, 0.0, &w);
    riga::detail::ck(hipGetLastError());
    return RIGA_OK;
  });
}
