// Assembly without allocation: gedmg_assemble_static runs the same kernels as
// gedmg_assemble, with the per-point scratch (network inputs, jets, phi at the
// points, history sensitivities) in a file-scope device array of fixed size
// instead of the context's buffers, R cleared by a kernel, and no profiling
// events.  For callers that cannot allocate while they run (graph capture,
// serving loops).
//
// Host code never passes the array's name to a kernel: in host code the name is
// a host-side stand-in.  gedmg_create looks up the array's device address once
// per device (hipGetSymbolAddress with that device current) and the entry
// point uses that address.
#include <mutex>

#include "gedmg_internal.h"

namespace gedmg {

// x [3], jet [10], phi [1] and sensitivities [2] per quadrature point.
constexpr long kStaticDoublesPerQp = 16;
constexpr long kStaticMaxQp = GEDMG_STATIC_MAX_QP;

static __device__ __align__(256) double scratch[kStaticMaxQp * kStaticDoublesPerQp];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch_init(int device, std::string& err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "device index out of range for the static scratch table";
    return GEDMG_E_ARG;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return GEDMG_OK;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess || cur != device) {
    err = "static scratch set-up needs its device current";
    return GEDMG_E_HIP;
  }
  double* p = nullptr;
  e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return GEDMG_E_HIP;
  }
  g_ptr[device] = p;
  return GEDMG_OK;
}

double* static_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace gedmg

using namespace gedmg;

extern "C" int gedmg_assemble_static(gedmg_ctx* c, const double* u, const double* phi, const double* kappa_n,
                                     int precision, double* R, double* K_vals, double* kappa_trial) {
  if (!c) return GEDMG_E_ARG;
  const long nq = (long)c->n_elems * c->nqp;
  if (nq > kStaticMaxQp) {
    c->err = "gedmg_assemble_static: " + std::to_string(nq) + " quadrature points exceed the static scratch limit of " +
             std::to_string(kStaticMaxQp);
    return GEDMG_E_ARG;
  }
  double* base = static_scratch_ptr(c->device);
  if (!base) {
    c->err = "gedmg_assemble_static: static scratch not set up on this device";
    return GEDMG_E_HIP;
  }
  // sub-arrays at fixed offsets of the maximum size (all multiples of 256 bytes)
  const AssembleScratch sc{base, base + 3 * kStaticMaxQp, base + 13 * kStaticMaxQp, base + 14 * kStaticMaxQp};
  return assemble_impl(c, u, phi, kappa_n, precision, R, K_vals, kappa_trial, sc, true, false);
}
