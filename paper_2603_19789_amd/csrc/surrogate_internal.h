// surrogate_internal.h -- declarations shared by the surrogate's host entry
// points and its kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>

namespace sslbm {

constexpr int SUR_IN_CHANNELS = 16;   // 5 densities, 9 parameter planes, 2 zero
constexpr int SUR_OUT_CHANNELS = 16;  // 5 predicted increments, 11 unused
constexpr int SUR_LOSS_BLOCKS = 1024;

inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

struct ConvArgs {
    const void *x;      // BF16 NHWC view
    int x_pitch;
    int n, h, w, cin;
    const void *wt;     // BF16 [cout][9][cin]
    const float *bias;  // may be null
    void *y;            // BF16 or FP32 NHWC view
    int y_pitch;
    int cout;
    float slope;
    void *pool;  // BF16 NHWC view (n, h/2, w/2) of the 2 x 2 means of y, or null
    int pool_pitch;
    // Input channels [0, cu) from xu, a BF16 NHWC view (n, h/2, w/2) read
    // as its nearest 2x upsampling; channels [cu, cin) from x (its channel
    // cu is x's channel 0). xu null: all from x.
    const void *xu;
    int xu_pitch, cu;
    // Activation adjoint in the epilogue: each stored BF16 value v becomes
    // BF16(m > 0 ? v : slope v), m the element of this BF16 NHWC view (cout
    // channels, the pixels of y) at the same pixel and channel. Null: none.
    const void *mask = nullptr;
    int mask_pitch = 0;
    // Adjoint of a 2x nearest upsampling in the epilogue (backward-data of a
    // decoder's first convolution): y is a view of cout - cd channels that
    // receives output channels [cd, cout) (channel c at column c - cd).
    // Channels [0, cd) go elsewhere: the sum of each 2 x 2 window of their
    // BF16-rounded values, rounded to BF16 and passed through the activation
    // adjoint with du_mask (a BF16 NHWC view at du's pixels; null: none), to
    // du, a BF16 NHWC view (n, h/2, w/2) of cd channels. cd is a multiple of
    // 16; h and w are even. Null du: none.
    void *du = nullptr;
    int du_pitch = 0, cd = 0;
    const void *du_mask = nullptr;
    int du_mask_pitch = 0;
};

struct WgradArgs {
    const uint16_t *dz_t, *xs;
    float *part;
    int n, h, w, cin, cout;
    long long P, Pr, Pp, chunk;  // pixels; rounded to 128; plane length
    int splits;
};

struct WgradPlan {
    long long P, Pr, Pp, chunk, waves;
    int splits, ni;
    // halo-tile path (images of at least 8 x 32 pixels): channel blocks of
    // 32 x 32, gb workgroups per block
    bool halo;
    int nob, nib, gb, tiles, tiles_x, tiles_y;
    size_t dz_t_bytes, xs_bytes, part_bytes;
    size_t bytes() const { return align256(dz_t_bytes) + align256(xs_bytes) + align256(part_bytes); }
};

// Weights of several layers for one flip launch (the backward-data kernels
// of a whole network): layer l's [cout][9][cin] weights w[l] become
// [cin][9][cout] flipped in space at wf[l]; start[l] is the prefix sum of
// the layers' element counts.
constexpr int SUR_MAX_FLIP_LAYERS = 32;
struct FlipTable {
    int layers;
    const void *w[SUR_MAX_FLIP_LAYERS];
    void *wf[SUR_MAX_FLIP_LAYERS];
    int cout[SUR_MAX_FLIP_LAYERS], cin[SUR_MAX_FLIP_LAYERS];
    long long start[SUR_MAX_FLIP_LAYERS + 1];
};

struct IoScales {
    float inv_in[5];   // input density channel = rho / scale_in
    float out[5];      // increment = scale_out * network output
    float inv_out[5];  // 1 / scale_out
};

struct AdamArgs {
    float lr, beta1, beta2, eps, inv_bc1, inv_bc2;  // inv_bc = 1 / (1 - beta^step)
};

hipError_t launch_conv_fwd(const ConvArgs &a, bool leaky, bool f32out, hipStream_t s);
hipError_t launch_flip(const void *w, int cout, int cin, void *wf, hipStream_t s);
hipError_t launch_flip_multi(const FlipTable &t, hipStream_t s);
WgradPlan wgrad_plan(int n, int h, int w, int cin, int cout);
// xu: null, or the half-resolution view of input channels [0, cu) (images
// of at least 8 x 32 pixels; hipErrorNotSupported otherwise). The partial
// sums are computed on s; the sums over the splits run on sum_s, after s
// reaches them (ev recorded on s; unused when sum_s is s).
hipError_t launch_wgrad(const void *x, int xp, const void *xu, int xup, int cu, const void *dz,
                        int dzp, int n, int h, int w, int cin, int cout, float *dw, float *db,
                        void *ws, hipStream_t s, hipStream_t sum_s, hipEvent_t ev);
hipError_t launch_leaky_bwd(const void *dy, int dyp, const void *y, int yp, void *dz, int dzp,
                            long long pixels, int c, float slope, hipStream_t s);
hipError_t launch_pool2(const void *x, int xp, int n, int h, int w, int c, void *y, int yp,
                        hipStream_t s);
hipError_t launch_pool2_bwd(const void *dy, int dyp, int n, int h, int w, int c, void *dx,
                            int dxp, bool accumulate, const void *mask, int mp, float slope,
                            hipStream_t s);
hipError_t launch_up2(const void *x, int xp, int n, int h, int w, int c, void *y, int yp,
                      hipStream_t s);
hipError_t launch_up2_bwd(const void *dy, int dyp, int n, int h, int w, int c, void *dx, int dxp,
                          const void *mask, int mp, float slope, hipStream_t s);
hipError_t launch_pack_input(const float *rho, int batch, int h, int w, const float *planes,
                             const IoScales &sc, void *x, hipStream_t s);
hipError_t launch_apply_output(const float *rho, const float *out, int batch, int h, int w,
                               const IoScales &sc, float *next, hipStream_t s);
hipError_t launch_mse(const float *out, const float *rho, const float *target, int batch, int h,
                      int w, const IoScales &sc, void *dout, double *partials, double *loss,
                      hipStream_t s);
hipError_t launch_adam(float *theta, void *theta_bf16, const float *grad, float *m, float *v,
                       long long count, const AdamArgs &a, hipStream_t s);
hipError_t launch_to_bf16(const float *src, void *dst, long long count, hipStream_t s);
hipError_t launch_crop(const float *rho, int h, int w, int y0, int x0, int ch, int cw, float *dst,
                       hipStream_t s);

}  // namespace sslbm
