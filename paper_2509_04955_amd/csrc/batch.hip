#include "internal.h"
extern "C" {
qs_status qs_batch_create(int, const int *, const qs_gate *const *, const size_t *, const uint64_t *const *,
                          const uint64_t *const *, const double *const *, const size_t *, const qs_contract_opts *,
                          void *, qs_batch *) { qs::set_error("batches not built yet"); return QS_EUNSUPPORTED; }
qs_status qs_batch_destroy(qs_batch) { return QS_OK; }
qs_status qs_batch_run(qs_batch, double *) { return QS_EUNSUPPORTED; }
qs_status qs_batch_state_copy_out(qs_batch, int, double *) { return QS_EUNSUPPORTED; }
}
