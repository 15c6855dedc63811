// mlp.hip -- learned candidate proposer (placeholder until the MFMA kernels land).
#include "plan.h"

struct pchase_mlp {
    int unused;
};

namespace pc {
int infer_learned(Workspace*, const pchase_observation*, const pchase_model*, uint32_t, const std::vector<DevProbe>&,
                  const std::vector<uint64_t>&, const std::vector<uint64_t>&, const std::vector<uint64_t>&,
                  const uint32_t*, uint32_t, const pchase_mlp*, std::vector<uint8_t>*, hipStream_t) {
    return set_error(PCHASE_EINVAL, "learned proposer not available");
}
}  // namespace pc

extern "C" int pchase_mlp_create(uint32_t, uint64_t, pchase_mlp** net) {
    if (net) *net = nullptr;
    return pc::set_error(PCHASE_EINVAL, "learned proposer not available");
}
extern "C" void pchase_mlp_destroy(pchase_mlp*) {}
extern "C" int pchase_mlp_features(const pchase_model*, uint32_t, float*, hipStream_t) {
    return pc::set_error(PCHASE_EINVAL, "learned proposer not available");
}
extern "C" int pchase_mlp_train_step(pchase_mlp*, const float*, const int32_t*, uint32_t, float, float*, hipStream_t) {
    return pc::set_error(PCHASE_EINVAL, "learned proposer not available");
}
extern "C" int pchase_mlp_forward(const pchase_mlp*, const float*, uint32_t, float*, hipStream_t) {
    return pc::set_error(PCHASE_EINVAL, "learned proposer not available");
}
extern "C" int pchase_mlp_param(const pchase_mlp*, uint32_t, uint32_t, void*, uint64_t*, int) {
    return pc::set_error(PCHASE_EINVAL, "learned proposer not available");
}
extern "C" int pchase_mlp_step_count(const pchase_mlp*, uint64_t*, int) {
    return pc::set_error(PCHASE_EINVAL, "learned proposer not available");
}
