// model_kernels_inst.hip -- one instantiation of the generic-model pass
// kernels (every compartment count and steps per pass) for one arithmetic
// type and one lattice. The build compiles this file once per combination,
// in parallel, with MODEL_FP64 (0 or 1) and MODEL_Q (5 or 9) defined; each
// object exports the matching launch_model_f{32,64}_d2q{5,9}.
#include "model_march.h"

#if !defined(MODEL_FP64) || !defined(MODEL_Q)
#error "compile with -DMODEL_FP64=0|1 -DMODEL_Q=5|9"
#endif

#if MODEL_FP64
using model_real = double;
#else
using model_real = float;
#endif

#define MODEL_NAME3(t, q) launch_model_##t##_d2q##q
#define MODEL_NAME2(t, q) MODEL_NAME3(t, q)
#if MODEL_FP64
#define MODEL_LAUNCH MODEL_NAME2(f64, MODEL_Q)
#else
#define MODEL_LAUNCH MODEL_NAME2(f32, MODEL_Q)
#endif

static_assert(MODEL_Q == 5 || MODEL_Q == 9, "D2Q5 or D2Q9");

namespace sslbm {

hipError_t MODEL_LAUNCH(const void *in, void *out, const GridDesc &g, const ModelCoefHost &h,
                        const void *table, int K, hipStream_t s) {
    return model_detail::launch_t<model_real, MODEL_Q>(in, out, g, h, table, K, s);
}

}  // namespace sslbm
