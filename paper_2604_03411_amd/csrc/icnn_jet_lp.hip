// Mixed-precision energy-network jets (placeholder until the matrix-core
// BF16 / FP16 kernels are in place): reports an unsupported precision.
#include "gedmg_internal.h"

namespace gedmg {

hipError_t launch_energy_jet_lp(int, int, const JetArgs&, hipStream_t, int) {
  return hipErrorInvalidValue;
}

}  // namespace gedmg
