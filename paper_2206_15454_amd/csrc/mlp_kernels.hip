// mlp_kernels.hip -- learned eddy-viscosity closure (placeholder until the
// fused MFMA inference kernel lands: every entry reports "not available").
#include "mlp_device.h"

namespace lbmx {

bool mlp_pack_blob(const void *, size_t, void *, std::string *why) {
    if (why) *why = "the learned closure kernel is not available in this build";
    return false;
}

hipError_t launch_step_mlp(int, const StepArgs &, int, int, hipStream_t) {
    return hipErrorNotSupported;
}

lbm_status mlp_fallback_count(const void *, int64_t *count, hipStream_t) {
    *count = 0;
    return LBM_OK;
}

}  // namespace lbmx
