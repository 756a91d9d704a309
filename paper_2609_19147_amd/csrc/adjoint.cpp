// Adjoint-method gradients (placeholder until the dual-state kernels land).
#include "runtime.h"

using namespace qs;

extern "C" qs_status qs_adjoint_grad(qs_state*, const qs_plan*, const qs_pauli*, size_t, double*, double*, size_t) {
  return QS_EUNSUPPORTED;
}
