// model_kernels_f32_d2q5.hip -- the generic-model pass kernels in FP32 on
// D2Q5 (every compartment count and steps per pass).
#include "model_march.h"

namespace sslbm {

hipError_t launch_model_f32_d2q5(const void *in, void *out, const GridDesc &g,
                               const ModelCoefHost &h, const void *table, int K, hipStream_t s) {
    return model_detail::launch_t<float, 5>(in, out, g, h, table, K, s);
}

}  // namespace sslbm
