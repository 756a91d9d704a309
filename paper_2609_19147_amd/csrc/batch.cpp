// Batched execution of many circuits (placeholder until the batched kernels land).
#include "runtime.h"

using namespace qs;

extern "C" qs_status qs_batch_create(size_t, const int*, const qs_plan* const*, int, qs_dtype, void*, qs_batch**) {
  return QS_EUNSUPPORTED;
}
extern "C" qs_status qs_batch_refresh(qs_batch*) { return QS_EUNSUPPORTED; }
extern "C" qs_status qs_batch_run(qs_batch*) { return QS_EUNSUPPORTED; }
extern "C" qs_status qs_batch_expect_diag(qs_batch*, const qs_pauli* const*, const size_t*, double*) {
  return QS_EUNSUPPORTED;
}
extern "C" qs_status qs_batch_state(qs_batch*, size_t, qs_state**) { return QS_EUNSUPPORTED; }
extern "C" qs_status qs_batch_free(qs_batch*) { return QS_OK; }
