#include "internal.h"
extern "C" {
int qs_costmodel_num_features(void) { return qs::kNumFeatures; }
int qs_costmodel_num_weights(void) { return qs::kNumWeights; }
qs_status qs_plan_pass_features(qs_plan, float *, uint64_t) { return QS_EUNSUPPORTED; }
qs_status qs_plan_time_passes(qs_plan, qs_dtype, int, double *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_train(const float *, const float *, int, int, int, float, uint64_t, const float *, float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_set_weights(const float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_get_weights(float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_predict(const float *, int, float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_grad(const float *, const float *, const float *, int, float *, float *) { return QS_EUNSUPPORTED; }
}
