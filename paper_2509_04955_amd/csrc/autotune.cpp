#include "internal.h"
extern "C" qs_status qs_autotune(int, qs_dtype, const qs_gate *, size_t, const qs_contract_opts *, qs_contract_opts *) { return QS_EUNSUPPORTED; }
