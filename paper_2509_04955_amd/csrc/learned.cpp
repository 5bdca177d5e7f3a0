// placeholder: learned partition (filled in below)
#include "internal.h"
namespace qs {
bool costmodel_loaded() { return false; }
double costmodel_predict_host(const float *) { return 0.0; }
int pass_features(int, int, const std::vector<HBlock> &, int64_t, int64_t, float *) { return 0; }
}
