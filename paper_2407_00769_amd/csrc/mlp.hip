// Learned step-cost model (placeholder until the trainer lands).
#include "engine.h"

namespace tnc {
struct Mlp {
    int dummy;
};
void mlp_free(Mlp *m) { delete m; }
double mlp_path_cost(const Network &, const std::vector<int> &, const std::vector<int> &, const std::vector<int> &) {
    return -1.0;
}
}  // namespace tnc

extern "C" int tnc_mlp_train(tnc_ctx *, int64_t, const float *, const float *, int32_t, int32_t, float, uint64_t,
                             float *) {
    tnc::set_error("MLP not built yet");
    return TNC_EUNSUPPORTED;
}
extern "C" int tnc_mlp_predict(tnc_ctx *, int64_t, const float *, float *) {
    tnc::set_error("MLP not built yet");
    return TNC_EUNSUPPORTED;
}
extern "C" int tnc_mlp_grad(tnc_ctx *, int64_t, const float *, const float *, float *, float *) {
    tnc::set_error("MLP not built yet");
    return TNC_EUNSUPPORTED;
}
extern "C" int64_t tnc_mlp_param_count(void) {
    return (int64_t)TNC_MLP_HIDDEN * TNC_MLP_FEATURES + TNC_MLP_HIDDEN + TNC_MLP_HIDDEN * TNC_MLP_HIDDEN +
           TNC_MLP_HIDDEN + TNC_MLP_HIDDEN + 1;
}
extern "C" int tnc_mlp_get_params(tnc_ctx *, float *) {
    tnc::set_error("MLP not built yet");
    return TNC_EUNSUPPORTED;
}
extern "C" int tnc_mlp_set_params(tnc_ctx *, const float *) {
    tnc::set_error("MLP not built yet");
    return TNC_EUNSUPPORTED;
}
extern "C" int tnc_costmodel_use(tnc_ctx *) {
    tnc::set_error("MLP not built yet");
    return TNC_EUNSUPPORTED;
}
