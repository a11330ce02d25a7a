// k_mlp.hip -- learned residual predictor kernels (under construction).
#include "mc_dev.h"
#include "mc_kernels.h"

namespace mck {
hipError_t mlp_pack(const float*, int, uint16_t*, uint16_t*, uint16_t*, uint16_t*, float*, float*, float*, float*,
                    hipStream_t) { return hipErrorNotSupported; }
hipError_t mlp_infer(const MlpDev&, const float*, long long, GridGeom, const int32_t*, const mc_result*,
                     const uint32_t*, int32_t*, hipStream_t) { return hipErrorNotSupported; }
hipError_t mlp_features(const MlpDev&, const float*, long long, GridGeom, const int32_t*, const mc_result*, long long,
                        long long, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t mlp_forward_z(const MlpDev&, const float*, long long, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t mlp_feature_sumsq(const float*, long long, GridGeom, const int32_t*, const mc_result*, int, double*, int,
                             hipStream_t) { return hipErrorNotSupported; }
hipError_t train_step_grad(const MlpDev&, const float*, long long, GridGeom, const int32_t*, const mc_result*,
                           const float*, const float*, const void*, int, long long, unsigned long long, long long,
                           float*, float*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t train_reduce_adam(int, int, const float*, const float*, float*, float*, float*, float*, float*, long long,
                             float, int, hipStream_t) { return hipErrorNotSupported; }
}  // namespace mck
