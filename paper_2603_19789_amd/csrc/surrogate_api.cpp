// surrogate_api.cpp -- host side of surrogate.h: argument validation (before
// any HIP call) and dispatch to the surrogate kernels.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>

#include "sslbm.h"
#include "surrogate.h"
#include "surrogate_internal.h"

namespace {

constexpr int MAX_SIDE = 1 << 16;
constexpr int MAX_CHANNELS = 4096;

sslbm_status status(hipError_t e) { return e == hipSuccess ? SSLBM_OK : SSLBM_E_HIP; }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// A BF16 NHWC view of c channels with the given pitch.
bool view_ok(const void *p, int pitch, int c) {
    return p && aligned16(p) && c > 0 && c <= MAX_CHANNELS && c % 8 == 0 && pitch >= c &&
           pitch % 8 == 0;
}

bool dims_ok(int n, int h, int w) {
    return n > 0 && h > 0 && w > 0 && h <= MAX_SIDE && w <= MAX_SIDE &&
           (long long)n * h * w <= (1ll << 34);
}

// The convolution addresses its input view with 32-bit byte offsets: the
// view must span less than 2 GiB.
bool conv_input_fits(int pitch, int n, int h, int w, int c) {
    return (((long long)n * h * w - 1) * pitch + c) * 2 < (1ll << 31);
}

bool scales_ok(const float *s) {
    if (!s)
        return false;
    for (int c = 0; c < 5; ++c)
        if (!(std::isfinite(s[c]) && s[c] > 0.f))
            return false;
    return true;
}

sslbm::IoScales make_scales(const float *in, const float *out) {
    sslbm::IoScales sc{};
    for (int c = 0; c < 5; ++c) {
        sc.inv_in[c] = in ? 1.f / in[c] : 1.f;
        sc.out[c] = out ? out[c] : 1.f;
        sc.inv_out[c] = out ? 1.f / out[c] : 1.f;
    }
    return sc;
}

}  // namespace

extern "C" {

namespace {

sslbm_status conv_forward(const void *x, int x_pitch, int n, int h, int w, int cin,
                          const void *weight, const float *bias, void *y, int y_pitch, int cout,
                          int flags, float slope, void *pooled, int pooled_pitch,
                          void *hip_stream) {
    if (!view_ok(x, x_pitch, cin) || !dims_ok(n, h, w) || !weight || !aligned16(weight) || !y ||
        (flags & ~(SUR_LEAKY | SUR_OUT_F32)) || cout <= 0 || cout > MAX_CHANNELS ||
        y_pitch < cout || !std::isfinite(slope) || !conv_input_fits(x_pitch, n, h, w, cin))
        return SSLBM_E_ARG;
    if (!(flags & SUR_OUT_F32) && !view_ok(y, y_pitch, cout))
        return SSLBM_E_ARG;
    if ((flags & SUR_OUT_F32) && (cout % 4 != 0 || y_pitch % 4 != 0 || !aligned16(y)))
        return SSLBM_E_ARG;
    sslbm::ConvArgs a;
    a.x = x;
    a.x_pitch = x_pitch;
    a.n = n;
    a.h = h;
    a.w = w;
    a.cin = cin;
    a.wt = weight;
    a.bias = bias;
    a.y = y;
    a.y_pitch = y_pitch;
    a.cout = cout;
    a.slope = slope;
    a.pool = pooled;
    a.pool_pitch = pooled_pitch;
    a.xu = nullptr;
    a.xu_pitch = a.cu = 0;
    return status(sslbm::launch_conv_fwd(a, flags & SUR_LEAKY, flags & SUR_OUT_F32,
                                         (hipStream_t)hip_stream));
}

}  // namespace

sslbm_status sur_conv3x3_forward_up(const void *xu, int xu_pitch, int cu, const void *x,
                                    int x_pitch, int n, int h, int w, int cin, const void *weight,
                                    const float *bias, void *y, int y_pitch, int cout, int flags,
                                    float slope, void *hip_stream) {
    if (cu <= 0 || cu % 32 || cin <= cu || !view_ok(xu, xu_pitch, cu) ||
        !view_ok(x, x_pitch, cin - cu) || !dims_ok(n, h, w) || h % 2 || w % 2 || !weight ||
        !aligned16(weight) || (flags & ~SUR_LEAKY) || cout <= 0 || cout > MAX_CHANNELS ||
        cin > MAX_CHANNELS || !view_ok(y, y_pitch, cout) || !std::isfinite(slope) ||
        !conv_input_fits(x_pitch, n, h, w, cin - cu) ||
        !conv_input_fits(xu_pitch, n, h / 2, w / 2, cu))
        return SSLBM_E_ARG;
    if (h < 8 || w < 32)
        return SSLBM_E_UNSUPPORTED;  // needs the halo-tile kernel
    sslbm::ConvArgs a;
    a.x = x;
    a.x_pitch = x_pitch;
    a.n = n;
    a.h = h;
    a.w = w;
    a.cin = cin;
    a.wt = weight;
    a.bias = bias;
    a.y = y;
    a.y_pitch = y_pitch;
    a.cout = cout;
    a.slope = slope;
    a.pool = nullptr;
    a.pool_pitch = 0;
    a.xu = xu;
    a.xu_pitch = xu_pitch;
    a.cu = cu;
    return status(sslbm::launch_conv_fwd(a, flags & SUR_LEAKY, false, (hipStream_t)hip_stream));
}

sslbm_status sur_conv3x3_forward(const void *x, int x_pitch, int n, int h, int w, int cin,
                                 const void *weight, const float *bias, void *y, int y_pitch,
                                 int cout, int flags, float slope, void *hip_stream) {
    return conv_forward(x, x_pitch, n, h, w, cin, weight, bias, y, y_pitch, cout, flags, slope,
                        nullptr, 0, hip_stream);
}

sslbm_status sur_conv3x3_forward_pool(const void *x, int x_pitch, int n, int h, int w, int cin,
                                      const void *weight, const float *bias, void *y, int y_pitch,
                                      int cout, int flags, float slope, void *pooled,
                                      int pooled_pitch, void *hip_stream) {
    if ((flags & SUR_OUT_F32) || h % 2 || w % 2 || !view_ok(pooled, pooled_pitch, cout))
        return SSLBM_E_ARG;
    return conv_forward(x, x_pitch, n, h, w, cin, weight, bias, y, y_pitch, cout, flags, slope,
                        pooled, pooled_pitch, hip_stream);
}

namespace {

// The backward-data convolution with weights already flipped (after the
// arguments were checked), optionally through the activation adjoint.
sslbm_status backward_data(const void *dz, int dz_pitch, int n, int h, int w, int cout,
                           const void *flipped, int cin, void *dx, int dx_pitch, const void *act,
                           int act_pitch, float slope, hipStream_t s) {
    sslbm::ConvArgs a;
    a.x = dz;
    a.x_pitch = dz_pitch;
    a.n = n;
    a.h = h;
    a.w = w;
    a.cin = cout;
    a.wt = flipped;
    a.bias = nullptr;
    a.y = dx;
    a.y_pitch = dx_pitch;
    a.cout = cin;
    a.slope = slope;
    a.pool = nullptr;
    a.pool_pitch = 0;
    a.xu = nullptr;
    a.xu_pitch = a.cu = 0;
    a.mask = act;
    a.mask_pitch = act ? act_pitch : 0;
    return status(sslbm::launch_conv_fwd(a, false, false, s));
}

bool backward_data_args_ok(const void *dz, int dz_pitch, int n, int h, int w, int cout,
                           const void *weight, int cin, const void *dx, int dx_pitch) {
    return view_ok(dz, dz_pitch, cout) && view_ok(dx, dx_pitch, cin) && dims_ok(n, h, w) &&
           weight && conv_input_fits(dz_pitch, n, h, w, cout);
}

// An activation view for the adjoint: null (none), or a BF16 view of c
// channels with a finite slope.
bool act_ok(const void *act, int act_pitch, int c, float slope) {
    return !act || (view_ok(act, act_pitch, c) && std::isfinite(slope));
}

}  // namespace

sslbm_status sur_conv3x3_backward_data(const void *dz, int dz_pitch, int n, int h, int w, int cout,
                                       const void *weight, int cin, void *dx, int dx_pitch,
                                       void *flip_scratch, void *hip_stream) {
    if (!backward_data_args_ok(dz, dz_pitch, n, h, w, cout, weight, cin, dx, dx_pitch) ||
        !flip_scratch || !aligned16(flip_scratch))
        return SSLBM_E_ARG;
    const hipStream_t s = (hipStream_t)hip_stream;
    sslbm_status st = status(sslbm::launch_flip(weight, cout, cin, flip_scratch, s));
    if (st != SSLBM_OK)
        return st;
    return backward_data(dz, dz_pitch, n, h, w, cout, flip_scratch, cin, dx, dx_pitch, nullptr, 0,
                         0.f, s);
}

sslbm_status sur_flip_weights(int layers, const void *const *weight, const int *cout,
                              const int *cin, void *const *flipped, void *hip_stream) {
    if (layers < 1 || layers > sslbm::SUR_MAX_FLIP_LAYERS || !weight || !cout || !cin || !flipped)
        return SSLBM_E_ARG;
    sslbm::FlipTable t{};
    t.layers = layers;
    t.start[0] = 0;
    for (int l = 0; l < layers; ++l) {
        if (!weight[l] || !flipped[l] || !aligned16(flipped[l]) || cout[l] <= 0 ||
            cout[l] > MAX_CHANNELS || cin[l] <= 0 || cin[l] > MAX_CHANNELS)
            return SSLBM_E_ARG;
        t.w[l] = weight[l];
        t.wf[l] = flipped[l];
        t.cout[l] = cout[l];
        t.cin[l] = cin[l];
        t.start[l + 1] = t.start[l] + (long long)cout[l] * 9 * cin[l];
    }
    return status(sslbm::launch_flip_multi(t, (hipStream_t)hip_stream));
}

sslbm_status sur_conv3x3_backward_data_flipped(const void *dz, int dz_pitch, int n, int h, int w,
                                               int cout, const void *flipped, int cin, void *dx,
                                               int dx_pitch, const void *act, int act_pitch,
                                               float slope, void *hip_stream) {
    if (!backward_data_args_ok(dz, dz_pitch, n, h, w, cout, flipped, cin, dx, dx_pitch) ||
        !aligned16(flipped) || !act_ok(act, act_pitch, cin, slope) ||
        (act && !conv_input_fits(act_pitch, n, h, w, cin)))
        return SSLBM_E_ARG;
    return backward_data(dz, dz_pitch, n, h, w, cout, flipped, cin, dx, dx_pitch, act, act_pitch,
                         slope, (hipStream_t)hip_stream);
}

sslbm_status sur_conv3x3_backward_data_up(const void *dz, int dz_pitch, int n, int h, int w,
                                          int cout, const void *flipped, int cin, int cu,
                                          void *dx, int dx_pitch, void *du, int du_pitch,
                                          const void *du_act, int du_act_pitch, float slope,
                                          void *hip_stream) {
    if (!view_ok(dz, dz_pitch, cout) || !dims_ok(n, h, w) || !flipped || !aligned16(flipped) ||
        !conv_input_fits(dz_pitch, n, h, w, cout) || cin <= 0 || cin > MAX_CHANNELS ||
        cu <= 0 || cu % 16 || cu >= cin || h % 2 || w % 2 || !view_ok(dx, dx_pitch, cin - cu) ||
        !view_ok(du, du_pitch, cu) || !act_ok(du_act, du_act_pitch, cu, slope) ||
        (du_act && !conv_input_fits(du_act_pitch, n, h / 2, w / 2, cu)) ||
        !conv_input_fits(du_pitch, n, h / 2, w / 2, cu))
        return SSLBM_E_ARG;
    const hipStream_t s = (hipStream_t)hip_stream;
    sslbm::ConvArgs a;
    a.x = dz;
    a.x_pitch = dz_pitch;
    a.n = n;
    a.h = h;
    a.w = w;
    a.cin = cout;
    a.wt = flipped;
    a.bias = nullptr;
    a.y = dx;
    a.y_pitch = dx_pitch;
    a.cout = cin;
    a.slope = slope;
    a.pool = nullptr;
    a.pool_pitch = 0;
    a.xu = nullptr;
    a.xu_pitch = a.cu = 0;
    a.du = du;
    a.du_pitch = du_pitch;
    a.cd = cu;
    a.du_mask = du_act;
    a.du_mask_pitch = du_act ? du_act_pitch : 0;
    // images too small for halo tiles (or views too large for their 32-bit
    // offsets) are the caller's to run as the two separate passes
    const hipError_t e = sslbm::launch_conv_fwd(a, false, false, s);
    return e == hipErrorNotSupported ? SSLBM_E_UNSUPPORTED : status(e);
}

size_t sur_conv3x3_backward_weight_workspace(int n, int h, int w, int cin, int cout) {
    if (!dims_ok(n, h, w) || cin <= 0 || cin % 8 || cout <= 0 || cout % 8 ||
        cin > MAX_CHANNELS || cout > MAX_CHANNELS || w % 8)
        return 0;
    return sslbm::wgrad_plan(n, h, w, cin, cout).bytes();
}

sslbm_status sur_conv3x3_backward_weight(const void *x, int x_pitch, const void *dz, int dz_pitch,
                                         int n, int h, int w, int cin, int cout, float *dweight,
                                         float *dbias, void *workspace, size_t workspace_bytes,
                                         void *hip_stream) {
    if (!view_ok(x, x_pitch, cin) || !view_ok(dz, dz_pitch, cout) || !dims_ok(n, h, w) ||
        w % 8 || !dweight || !workspace || !aligned16(workspace) ||
        !conv_input_fits(x_pitch, n, h, w, cin) || !conv_input_fits(dz_pitch, n, h, w, cout))
        return SSLBM_E_ARG;
    if (workspace_bytes < sur_conv3x3_backward_weight_workspace(n, h, w, cin, cout))
        return SSLBM_E_ARG;
    return status(sslbm::launch_wgrad(x, x_pitch, nullptr, 0, 0, dz, dz_pitch, n, h, w, cin, cout,
                                      dweight, dbias, workspace, (hipStream_t)hip_stream,
                                      (hipStream_t)hip_stream, nullptr));
}

sslbm_status sur_conv3x3_backward_weight_overlap(const void *xu, int xu_pitch, int cu,
                                                 const void *x, int x_pitch, const void *dz,
                                                 int dz_pitch, int n, int h, int w, int cin,
                                                 int cout, float *dweight, float *dbias,
                                                 void *workspace, size_t workspace_bytes,
                                                 void *hip_stream, void *sum_stream, void *event) {
    const int cx = xu ? cin - cu : cin;  // channels read from x
    if (!view_ok(x, x_pitch, cx) || !view_ok(dz, dz_pitch, cout) || !dims_ok(n, h, w) ||
        w % 8 || !dweight || !workspace || !aligned16(workspace) || cin > MAX_CHANNELS ||
        !conv_input_fits(x_pitch, n, h, w, cx) || !conv_input_fits(dz_pitch, n, h, w, cout) ||
        (sum_stream != hip_stream && !event))
        return SSLBM_E_ARG;
    if (xu && (cu <= 0 || cu % 32 || cin <= cu || !view_ok(xu, xu_pitch, cu) || h % 2 ||
               !conv_input_fits(xu_pitch, n, h / 2, w / 2, cu)))
        return SSLBM_E_ARG;
    if (!xu && cu != 0)
        return SSLBM_E_ARG;
    if (workspace_bytes < sur_conv3x3_backward_weight_workspace(n, h, w, cin, cout))
        return SSLBM_E_ARG;
    if (xu && (h < 8 || w < 32))
        return SSLBM_E_UNSUPPORTED;  // needs the halo-tile kernel
    return status(sslbm::launch_wgrad(x, x_pitch, xu, xu_pitch, cu, dz, dz_pitch, n, h, w, cin,
                                      cout, dweight, dbias, workspace, (hipStream_t)hip_stream,
                                      (hipStream_t)sum_stream, (hipEvent_t)event));
}

sslbm_status sur_conv3x3_backward_weight_up(const void *xu, int xu_pitch, int cu, const void *x,
                                            int x_pitch, const void *dz, int dz_pitch, int n, int h,
                                            int w, int cin, int cout, float *dweight, float *dbias,
                                            void *workspace, size_t workspace_bytes,
                                            void *hip_stream) {
    if (cu <= 0 || cu % 32 || cin <= cu || cin > MAX_CHANNELS || !view_ok(xu, xu_pitch, cu) ||
        !view_ok(x, x_pitch, cin - cu) || !view_ok(dz, dz_pitch, cout) || !dims_ok(n, h, w) ||
        h % 2 || w % 8 || !dweight || !workspace || !aligned16(workspace) ||
        !conv_input_fits(x_pitch, n, h, w, cin - cu) ||
        !conv_input_fits(xu_pitch, n, h / 2, w / 2, cu) ||
        !conv_input_fits(dz_pitch, n, h, w, cout))
        return SSLBM_E_ARG;
    if (workspace_bytes < sur_conv3x3_backward_weight_workspace(n, h, w, cin, cout))
        return SSLBM_E_ARG;
    if (h < 8 || w < 32)
        return SSLBM_E_UNSUPPORTED;  // needs the halo-tile kernel
    return status(sslbm::launch_wgrad(x, x_pitch, xu, xu_pitch, cu, dz, dz_pitch, n, h, w, cin,
                                      cout, dweight, dbias, workspace, (hipStream_t)hip_stream,
                                      (hipStream_t)hip_stream, nullptr));
}

sslbm_status sur_leaky_backward(const void *dy, int dy_pitch, const void *y, int y_pitch, void *dz,
                                int dz_pitch, long long pixels, int c, float slope,
                                void *hip_stream) {
    if (!view_ok(dy, dy_pitch, c) || !view_ok(y, y_pitch, c) || !view_ok(dz, dz_pitch, c) ||
        pixels <= 0 || !std::isfinite(slope))
        return SSLBM_E_ARG;
    return status(sslbm::launch_leaky_bwd(dy, dy_pitch, y, y_pitch, dz, dz_pitch, pixels, c, slope,
                                          (hipStream_t)hip_stream));
}

sslbm_status sur_pool2(const void *x, int x_pitch, int n, int h, int w, int c, void *y, int y_pitch,
                       void *hip_stream) {
    if (!view_ok(x, x_pitch, c) || !view_ok(y, y_pitch, c) || !dims_ok(n, h, w) || h % 2 || w % 2)
        return SSLBM_E_ARG;
    return status(sslbm::launch_pool2(x, x_pitch, n, h, w, c, y, y_pitch, (hipStream_t)hip_stream));
}

sslbm_status sur_pool2_backward(const void *dy, int dy_pitch, int n, int h, int w, int c, void *dx,
                                int dx_pitch, int accumulate, void *hip_stream) {
    if (!view_ok(dy, dy_pitch, c) || !view_ok(dx, dx_pitch, c) || !dims_ok(n, h, w) || h % 2 ||
        w % 2)
        return SSLBM_E_ARG;
    return status(sslbm::launch_pool2_bwd(dy, dy_pitch, n, h, w, c, dx, dx_pitch, accumulate != 0,
                                          nullptr, 0, 0.f, (hipStream_t)hip_stream));
}

sslbm_status sur_pool2_backward_act(const void *dy, int dy_pitch, int n, int h, int w, int c,
                                    void *dx, int dx_pitch, int accumulate, const void *act,
                                    int act_pitch, float slope, void *hip_stream) {
    if (!view_ok(dy, dy_pitch, c) || !view_ok(dx, dx_pitch, c) || !dims_ok(n, h, w) || h % 2 ||
        w % 2 || !act || !act_ok(act, act_pitch, c, slope))
        return SSLBM_E_ARG;
    return status(sslbm::launch_pool2_bwd(dy, dy_pitch, n, h, w, c, dx, dx_pitch, accumulate != 0,
                                          act, act_pitch, slope, (hipStream_t)hip_stream));
}

sslbm_status sur_up2(const void *x, int x_pitch, int n, int h, int w, int c, void *y, int y_pitch,
                     void *hip_stream) {
    if (!view_ok(x, x_pitch, c) || !view_ok(y, y_pitch, c) || !dims_ok(n, 2 * h, 2 * w))
        return SSLBM_E_ARG;
    return status(sslbm::launch_up2(x, x_pitch, n, h, w, c, y, y_pitch, (hipStream_t)hip_stream));
}

sslbm_status sur_up2_backward(const void *dy, int dy_pitch, int n, int h, int w, int c, void *dx,
                              int dx_pitch, void *hip_stream) {
    if (!view_ok(dy, dy_pitch, c) || !view_ok(dx, dx_pitch, c) || !dims_ok(n, 2 * h, 2 * w))
        return SSLBM_E_ARG;
    return status(sslbm::launch_up2_bwd(dy, dy_pitch, n, h, w, c, dx, dx_pitch, nullptr, 0, 0.f,
                                        (hipStream_t)hip_stream));
}

sslbm_status sur_up2_backward_act(const void *dy, int dy_pitch, int n, int h, int w, int c,
                                  void *dx, int dx_pitch, const void *act, int act_pitch,
                                  float slope, void *hip_stream) {
    if (!view_ok(dy, dy_pitch, c) || !view_ok(dx, dx_pitch, c) || !dims_ok(n, 2 * h, 2 * w) ||
        !act || !act_ok(act, act_pitch, c, slope))
        return SSLBM_E_ARG;
    return status(sslbm::launch_up2_bwd(dy, dy_pitch, n, h, w, c, dx, dx_pitch, act, act_pitch,
                                        slope, (hipStream_t)hip_stream));
}

sslbm_status sur_pack_input(const float *rho, int batch, int h, int w, const float *planes,
                            const float *scale_in, void *x, void *hip_stream) {
    if (!rho || !planes || !x || !aligned16(x) || !dims_ok(batch, h, w) || !scales_ok(scale_in))
        return SSLBM_E_ARG;
    return status(sslbm::launch_pack_input(rho, batch, h, w, planes, make_scales(scale_in, nullptr),
                                           x, (hipStream_t)hip_stream));
}

sslbm_status sur_apply_output(const float *rho, const float *out, int batch, int h, int w,
                              const float *scale_out, float *rho_next, void *hip_stream) {
    if (!rho || !out || !rho_next || !dims_ok(batch, h, w) || !scales_ok(scale_out))
        return SSLBM_E_ARG;
    return status(sslbm::launch_apply_output(rho, out, batch, h, w, make_scales(nullptr, scale_out),
                                             rho_next, (hipStream_t)hip_stream));
}

sslbm_status sur_mse_loss(const float *out, const float *rho, const float *target, int batch, int h,
                          int w, const float *scale_out, void *dout, double *partials, double *loss,
                          void *hip_stream) {
    if (!out || !rho || !target || !dout || !aligned16(dout) || !partials || !loss ||
        !dims_ok(batch, h, w) || !scales_ok(scale_out))
        return SSLBM_E_ARG;
    return status(sslbm::launch_mse(out, rho, target, batch, h, w, make_scales(nullptr, scale_out),
                                    dout, partials, loss, (hipStream_t)hip_stream));
}

sslbm_status sur_adam(float *theta, void *theta_bf16, const float *grad, float *m, float *v,
                      long long count, int step, float lr, float beta1, float beta2, float eps,
                      void *hip_stream) {
    if (!theta || !grad || !m || !v || count <= 0 || step < 1 || !(lr >= 0.f) ||
        !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return SSLBM_E_ARG;
    sslbm::AdamArgs a;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    a.inv_bc2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    return status(sslbm::launch_adam(theta, theta_bf16, grad, m, v, count, a,
                                     (hipStream_t)hip_stream));
}

sslbm_status sur_crop_periodic(const float *rho, int h, int w, int y0, int x0, int ch, int cw,
                               float *dst, void *hip_stream) {
    if (!rho || !dst || !dims_ok(1, h, w) || !dims_ok(1, ch, cw))
        return SSLBM_E_ARG;
    return status(sslbm::launch_crop(rho, h, w, y0, x0, ch, cw, dst, (hipStream_t)hip_stream));
}

sslbm_status sur_to_bf16(const float *src, void *dst, long long count, void *hip_stream) {
    if (!src || !dst || count <= 0)
        return SSLBM_E_ARG;
    return status(sslbm::launch_to_bf16(src, dst, count, (hipStream_t)hip_stream));
}

}  // extern "C"
