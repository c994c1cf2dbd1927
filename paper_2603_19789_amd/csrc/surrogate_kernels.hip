// surrogate_kernels.hip -- the operations of the learned surrogate on gfx950:
// periodic 3x3 convolutions on BF16 MFMA with FP32 accumulation (forward,
// and the two backward passes), pooling, upsampling, activation, the
// surrogate's input/output/loss maps and the Adam update.
//
// Activations are NHWC BF16 views: element (n, y, x, c) of a view lives at
// ptr[((n H + y) W + x) pitch + c]; a view's channels are a slice of a wider
// buffer when pitch > channels (that is how skip connections concatenate
// without copies). Channel counts, pitches and slice offsets are multiples of
// 8, so one lane moves 8 channels (16 bytes) per access. Weights are BF16
// [out][tap][in], tap = 3 (dy + 1) + (dx + 1), with FP32 master copies.
//
// Convolution as implicit GEMM on V_MFMA_F32_16X16X32_BF16. Lane l of a
// wavefront holds row l % 16 of A and column l % 16 of B, each with the 8
// consecutive k values 8 (l / 16) .. 8 (l / 16) + 7, and receives rows
// 4 (l / 16) + i, i = 0..3, of column l % 16 of the 16 x 16 FP32 result
// (layout checked on the device).
//   forward:  rows = output pixels, columns = output channels,
//             k = (tap, input channel): both fragments are 16-byte loads of
//             8 consecutive channels (NHWC activations, [out][tap][in] weights).
//   backward data: the forward kernel on dZ with the weights flipped in
//             space and transposed in channels (periodic padding makes the
//             adjoint of a correlation the correlation with the flipped kernel).
//   backward weights: rows = output channels, columns = input channels,
//             k = pixels. dZ and X are first transposed to channel-major
//             planes (X in three copies shifted by dx = -1, 0, +1), so a
//             fragment is again 8 consecutive values; dy moves whole rows.
//             Pixels are split across wavefronts; FP32 partial sums are added
//             in a fixed order by a second kernel, so results are deterministic.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "seird_device.h"  // xcd_tile
#include "surrogate_internal.h"

namespace sslbm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int THREADS = 256;

// FP32 -> BF16 with round-to-nearest-even (finite inputs; NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u)
        return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// Raw buffer access: the descriptor (base address, byte length) is
// wavefront-uniform; each lane gives a 32-bit byte offset. Descriptor word 3
// is the gfx9 raw-buffer format (32-bit data). Offsets at or past the length
// read zeros. The 16 loaded bytes are taken as one 128-bit integer (taking
// vector elements one by one lets this compiler narrow the load).
constexpr int BUF_FORMAT_WORD = 0x00020000;
__device__ __forceinline__ u32x4 load16(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(
        u32x4, __builtin_bit_cast(unsigned __int128, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0)));
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Eight BF16 values as one 16-byte vector (element 0 in the low half-word).
__device__ __forceinline__ uint4 pack8(const uint16_t *v) {
    return make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                      v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16));
}

// ------------------------------------------------------------- forward conv
// A workgroup computes (64 WM) consecutive output pixels x (16 NT WN) output
// channels, WN = 4 / WM, as a grid of WM x WN wavefronts that each own 64
// pixels x 16 NT channels (4 x NT MFMA tiles). The k loop runs over
// (32-channel chunk, tap). Each step's A tile (pixels x 32 channels of the
// tap-shifted input) and B tile (channels x 32 weights) go through LDS,
// double-buffered, with two steps in flight: while step k is multiplied,
// step k + 1 (loaded during step k - 1) moves from registers into the other
// buffer and the loads of step k + 2 are outstanding; one barrier per step.
// The per-step address work is a few masks and adds: the wrapped rows and
// columns of the three taps in each direction are computed once per thread.
// LDS rows are padded to 40 elements (80 bytes), so the 16 rows a fragment
// read touches fall into distinct banks.
constexpr int LDA = 40;

template <int WM, int NT, bool F32OUT, bool LEAKY>
__global__ __launch_bounds__(THREADS) void conv_fwd_kernel(ConvArgs a) {
    constexpr int WN = 4 / WM;
    constexpr int TP = 64 * WM;       // pixels per workgroup
    constexpr int TC = 16 * NT * WN;  // output channels per workgroup
    constexpr int APT = TP * 4 / THREADS;  // 16-byte A pieces per thread
    __shared__ __attribute__((aligned(16))) uint16_t As[2][TP * LDA];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][TC * LDA];

    const int groups = (a.cout + TC - 1) / TC;
    const long long P = (long long)a.n * a.h * a.w;
    const long long tile = blockIdx.x / groups;
    const int cg = (int)(blockIdx.x - tile * groups);
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int wm = wv % WM, wn = wv / WM;
    // Loads go through buffer descriptors over the input view and the
    // weights (byte offsets are 32-bit; the host checks the sizes). An offset
    // past the descriptor's range reads zeros: that is how channels past the
    // end of a layer (cin not a multiple of 32) are filled, with every load
    // issued unconditionally so that the memory counters stay exact.
    const long long P_last = P - 1;
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(a.x), (short)0, (int)((P_last * a.x_pitch + a.cin) * 2), BUF_FORMAT_WORD);
    const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(a.wt), (short)0, a.cout * 9 * a.cin * 2, BUF_FORMAT_WORD);

    // loader roles: A piece j of this thread is pixel row (tid + 256 j) / 4,
    // channel chunk (tid + 256 j) % 4; B piece (threads < 4 TC): output
    // channel row tid / 4, chunk tid % 4. The byte offset of A piece j at tap
    // (dy, dx) is the offset of the pixel's own row and column plus the
    // differences to the wrapped rows and columns of the neighbouring taps,
    // taken through wavefront-uniform bit masks (a select chain on the tap
    // becomes a lookup table in scratch memory with this compiler).
    int arow[APT], ach[APT];
    unsigned ry1[APT], rym[APT], ryp[APT], cx1[APT], cxm[APT], cxp[APT];
    const long long hw = (long long)a.h * a.w;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        const int i = tid + THREADS * j;
        arow[j] = i >> 2;
        ach[j] = i & 3;
        long long q = tile * TP + arow[j];
        if (q >= P)
            q = P_last;  // a clamped duplicate; its results are never stored
        const int n = (int)(q / hw);
        const int r = (int)(q - n * hw);
        const int y = r / a.w, xq = r - y * a.w;
        auto row_off = [&](int d) {
            return (unsigned)(((long long)n * a.h + wrap(y + d, a.h)) * a.w * a.x_pitch * 2);
        };
        auto col_off = [&](int d) {
            return (unsigned)(wrap(xq + d, a.w) * a.x_pitch * 2 + 16 * ach[j]);
        };
        ry1[j] = row_off(0);
        rym[j] = row_off(-1) - ry1[j];  // modulo 2^32
        ryp[j] = row_off(1) - ry1[j];
        cx1[j] = col_off(0);
        cxm[j] = col_off(-1) - cx1[j];
        cxp[j] = col_off(1) - cx1[j];
    }
    const bool bload = tid < 4 * TC;
    const int brow = tid >> 2, bch = tid & 3;
    const int bco = min(cg * TC + brow, a.cout - 1);
    const unsigned boff = (unsigned)((bco * 9 * a.cin + 8 * bch) * 2);
    constexpr unsigned OUT_OF_RANGE = 0x80000000u;

    const int nck = (a.cin + 31) / 32;
    const int steps = 9 * nck;
    // global loads of step st into registers (past the end: the last step again)
    struct Stage {
        u32x4 a[APT];
        u32x4 b;
    };
    auto gload = [&](int st) {
        Stage r;
        st = st < steps ? st : steps - 1;
        const int ck = st / 9;  // k order (chunk, tap), as in the halo kernel
        const int t = st - 9 * ck;
        const int c0 = 32 * ck;
        const int ty = t / 3, tx = t - 3 * ty;  // dy + 1, dx + 1
        const unsigned my = ty == 0 ? ~0u : 0u, py = ty == 2 ? ~0u : 0u;
        const unsigned mx = tx == 0 ? ~0u : 0u, px = tx == 2 ? ~0u : 0u;
        const int left = a.cin - c0;  // channels left in this chunk
#pragma unroll
        for (int j = 0; j < APT; ++j) {
            const unsigned rr = ry1[j] + (rym[j] & my) + (ryp[j] & py);
            const unsigned cc = cx1[j] + (cxm[j] & mx) + (cxp[j] & px);
            const unsigned off = 8 * ach[j] < left ? rr + cc + (unsigned)(2 * c0) : OUT_OF_RANGE;
            r.a[j] = load16(xr, off);
        }
        // every thread loads (rows past the tile are clamped duplicates); only
        // the B-loader threads store
        const unsigned off =
            8 * bch < left ? boff + (unsigned)((t * a.cin + c0) * 2) : OUT_OF_RANGE;
        r.b = load16(wr, off);
        return r;
    };
    auto lstore = [&](int buf, const Stage &r) {
#pragma unroll
        for (int j = 0; j < APT; ++j)
            *reinterpret_cast<u32x4 *>(&As[buf][arow[j] * LDA + 8 * ach[j]]) = r.a[j];
        if (bload)
            *reinterpret_cast<u32x4 *>(&Bs[buf][brow * LDA + 8 * bch]) = r.b;
    };

    f32x4 acc[4][NT];
#pragma unroll
    for (int ms = 0; ms < 4; ++ms)
#pragma unroll
        for (int ns = 0; ns < NT; ++ns)
            acc[ms][ns] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto compute = [&](int buf) {
        bf16x8 A[4], B[NT];
#pragma unroll
        for (int ms = 0; ms < 4; ++ms)
            A[ms] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&As[buf][(wm * 64 + 16 * ms + m) * LDA + 8 * g]));
#pragma unroll
        for (int ns = 0; ns < NT; ++ns)
            B[ns] = __builtin_bit_cast(
                bf16x8,
                *reinterpret_cast<const uint4 *>(&Bs[buf][(wn * 16 * NT + 16 * ns + m) * LDA + 8 * g]));
#pragma unroll
        for (int ms = 0; ms < 4; ++ms)
#pragma unroll
            for (int ns = 0; ns < NT; ++ns)
                acc[ms][ns] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ms], B[ns], acc[ms][ns], 0, 0, 0);
    };

    // Two steps in flight: while step st is multiplied out of LDS buffer
    // st % 2, step st + 1 (loaded during the previous step) goes from
    // registers into the other buffer and step st + 2 is being loaded. The
    // loop is unrolled by two so that both register sets are fixed.
    Stage s0 = gload(0);
    lstore(0, s0);
    Stage s1 = gload(1);
    __syncthreads();
    int st = 0;
    for (; st + 1 < steps; st += 2) {
        s0 = gload(st + 2);
        compute(0);
        lstore(1, s1);  // buffer 1 was last read before the previous barrier
        __syncthreads();
        s1 = gload(st + 3);
        compute(1);
        lstore(0, s0);
        __syncthreads();
    }
    if (st < steps)
        compute(0);

#pragma unroll
    for (int ns = 0; ns < NT; ++ns) {
        const int c = cg * TC + wn * 16 * NT + 16 * ns + m;
        if (c >= a.cout)
            continue;
        const float b = a.bias ? a.bias[c] : 0.f;
#pragma unroll
        for (int ms = 0; ms < 4; ++ms)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long q = tile * TP + wm * 64 + 16 * ms + 4 * g + i;
                if (q >= P)
                    continue;
                float v = acc[ms][ns][i] + b;
                if (LEAKY)
                    v = v > 0.f ? v : a.slope * v;
                if (F32OUT)
                    static_cast<float *>(a.y)[q * a.y_pitch + c] = v;
                else
                    static_cast<uint16_t *>(a.y)[q * a.y_pitch + c] = to_bf16(v);
            }
    }
}

// ------------------------------------------------ forward conv, halo tiles
// The tiled kernel above reloads the tap-shifted input tile at each of the
// nine taps: 16-32 KB from L2 per 8 MFMAs per wavefront. Here a workgroup
// owns an output tile of 8 rows x 32 columns of one image and 16 NT output
// channels (channel group cg; 4 wavefronts of 2 rows x 32 columns x 16 NT
// channels) and, per 32-channel chunk, loads the input tile with its
// one-pixel halo (10 x 34 pixels, periodic wrap) and the weights of all
// nine taps into LDS once; the nine taps then read shifted fragments of the
// same halo tile, at offsets known at compile time. The grid holds as many
// workgroups as are resident at once; workgroup b takes the units (tile,
// channel group) b, b + G, b + 2G, ... (G the grid size; the groups of a
// tile are consecutive units, so they run side by side and share the halo
// through L2), and the loads of its next (unit, chunk) item are in flight
// while the current one is multiplied. The k order is (chunk, tap), as in
// the tiled kernel, so both give the same bits. Needs h >= 8 and w >= 32
// (a halo wraps at most once).
constexpr int HALO_TH = 8, HALO_TW = 32;

// LDS use (50 KB for 32 channels, 73 KB for 64) allows 3 or 2 workgroups
// per CU; the register budget is held to the same occupancy. POOL: the
// epilogue also writes the 2 x 2 means of the BF16 output (a wavefront's two
// rows start at an even row and a lane's columns 4 g .. 4 g + 3 at an even
// column, so every window lies in one lane), with the sums of the separate
// pooling kernel in its order, hence its bits.
// UP: the first cu input channels are read from a half-resolution view
// as its nearest 2x upsampling (pixel (y, x) reads (y / 2, x / 2)), so a
// decoder's upsampled skip concatenation needs no upsampled copy in HBM.
// MASK (BF16 output, no pooling; the backward-data pass): the epilogue also
// applies the adjoint of the activation that produced the pass's output
// tensor, reading that activation from a.mask (see ConvArgs), with the
// roundings of a separate sur_leaky_backward over the stored values.
// UPB (BF16 output; the backward-data pass of a decoder's first convolution,
// whose first a.cd input channels were a 2x upsampling): output channels
// from a.cd on go to y, a view of a.cout - a.cd channels (channel c at
// column c - a.cd); those below a.cd are kept in registers; each 2 x 2 window of
// their BF16-rounded values (all in one lane, as for POOL) is summed in the
// order of the separate upsampling adjoint, rounded, passed through the
// activation adjoint with a.du_mask when given, and written to the
// half-resolution view a.du: the bits of the two separate passes.
template <int NT, bool F32OUT, bool LEAKY, bool POOL, bool UP, bool MASK, bool UPB>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(NT == 4 ? 2 : 3)))
void conv_halo_kernel(ConvArgs a, int tiles_x, int tiles_y, int units) {
    static_assert(!MASK || (!F32OUT && !POOL), "the mask applies to plain BF16 outputs");
    static_assert(!UPB || (!F32OUT && !LEAKY && !POOL && !UP && !MASK),
                  "the upsampling adjoint goes with plain BF16 outputs");
    constexpr int HW2 = HALO_TW + 2, HPIX = (HALO_TH + 2) * HW2;
    constexpr int HP = HPIX * 4, HPT = (HP + THREADS - 1) / THREADS;  // 16-byte pieces
    constexpr int TC = 16 * NT;
    constexpr int BP = 9 * TC * 4, BPT = (BP + THREADS - 1) / THREADS;
    constexpr unsigned OUT_OF_RANGE = 0x80000000u;
    __shared__ __attribute__((aligned(16))) uint16_t Hs[HPIX * LDA];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[9 * TC * LDA];
    __shared__ __attribute__((aligned(16))) float Cs[TC];  // bias of the group

    const int G = gridDim.x;
    if ((int)blockIdx.x >= units)
        return;  // whole workgroup, before any barrier
    // Workgroup b runs on XCD b % 8, each with its own L2: consecutive units
    // (the channel groups of a tile, then neighbouring tiles, which share
    // halo pixels) are given to the workgroups of one XCD.
    const int vb = G % 8 == 0 && G <= units ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8)
                                            : (int)blockIdx.x;
    const int groups = (a.cout + TC - 1) / TC;
    const int nck = (a.cin + 31) / 32;
    const int items = ((units - 1 - vb) / G + 1) * nck;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const long long P = (long long)a.n * a.h * a.w;
    const int cx = UP ? a.cin - a.cu : a.cin;  // channels read from x
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(a.x), (short)0, (int)(((P - 1) * a.x_pitch + cx) * 2), BUF_FORMAT_WORD);
    const int hu = a.h / 2, wu = a.w / 2;
    const __amdgpu_buffer_rsrc_t xur = __builtin_amdgcn_make_buffer_rsrc(
        UP ? const_cast<void *>(a.xu) : const_cast<void *>(a.x), (short)0,
        UP ? (int)((((long long)a.n * hu * wu - 1) * a.xu_pitch + a.cu) * 2) : 0, BUF_FORMAT_WORD);
    const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(a.wt), (short)0, a.cout * 9 * a.cin * 2, BUF_FORMAT_WORD);
    // the bias goes through LDS with the weights (no bias: a range of 0 bytes
    // reads zeros); channels past the layer's read zeros as well
    const __amdgpu_buffer_rsrc_t br = __builtin_amdgcn_make_buffer_rsrc(
        a.bias ? const_cast<float *>(a.bias) : const_cast<void *>(a.wt), (short)0,
        a.bias ? a.cout * 4 : 0, BUF_FORMAT_WORD);
    const bool cload = tid < TC / 4;

    // weight pieces: row (tap t, channel o of the group) of Bs, 8 channels k
    // of the chunk; channels past the layer's load its last one (their
    // results are never stored)
    unsigned boff[BPT], coff = 0;
    int bk[BPT], blds[BPT], bt[BPT], bo[BPT];
    bool bst[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int e = tid + THREADS * j;
        bst[j] = e < BP;
        const int row = min(e >> 2, 9 * TC - 1), k = e & 3;
        bt[j] = row / TC;
        bo[j] = row - bt[j] * TC;
        bk[j] = 8 * k;
        blds[j] = row * LDA + 8 * k;
    }
    // halo pieces: pixel hp of the halo tile, 8 channels k of the chunk
    // (hoffu: the same pixel in the half-resolution view)
    // (piece j of a thread: pixel (tid >> 2) + 64 j, the same 8 channels
    // hk for every j, LDS slot hlds + 64 j LDA; the pixel's row and column
    // are recomputed where needed rather than kept in registers)
    unsigned hoff[HPT], hoffu[HPT];
    const int hk = 8 * (tid & 3);
    const int hlds = (tid >> 2) * LDA + hk;
    auto hpix = [&](int j) { return min((tid >> 2) + 64 * j, HPIX - 1); };
    auto hst = [&](int j) { return tid + THREADS * j < HP; };
    auto unit_origin = [&](int unit, int &n, int &y0, int &x0, int &cg) {
        const int tile = unit / groups;
        cg = unit - tile * groups;
        const int per_image = tiles_x * tiles_y;
        n = tile / per_image;
        const int r = tile - n * per_image;
        const int ty = r / tiles_x;
        y0 = ty * HALO_TH;
        x0 = (r - ty * tiles_x) * HALO_TW;
    };
    auto unit_offsets = [&](int unit) {
        int n, y0, x0, cg;
        unit_origin(unit, n, y0, x0, cg);
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int hp = hpix(j), hy = hp / HW2, hx = hp - hy * HW2;
            const int y = wrap(y0 - 1 + hy, a.h), x = wrap(x0 - 1 + hx, a.w);
            hoff[j] = (unsigned)(((((long long)n * a.h + y) * a.w + x) * a.x_pitch + hk) * 2);
            if constexpr (UP)
                hoffu[j] = (unsigned)(
                    ((((long long)n * hu + (y >> 1)) * wu + (x >> 1)) * a.xu_pitch + hk) * 2);
        }
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int o = min(cg * TC + bo[j], a.cout - 1);
            boff[j] = (unsigned)(((o * 9 + bt[j]) * a.cin + bk[j]) * 2);
        }
        coff = cload ? (unsigned)((cg * TC + 4 * tid) * 4) : OUT_OF_RANGE;
    };

    struct Stage {
        u32x4 h[HPT];
        u32x4 b[BPT];
        u32x4 c;
    };
    // loads of one chunk (the weights and bias only when they change between
    // items)
    auto gload = [&](int chunk, bool weights) {
        Stage r;
        const int left = a.cin - 32 * chunk;
        if constexpr (UP) {
            // cu is a multiple of 32: a chunk comes from one view
            const bool from_up = 32 * chunk < a.cu;
            const __amdgpu_buffer_rsrc_t src = from_up ? xur : xr;
            const unsigned c2 = (unsigned)(64 * (from_up ? chunk : chunk - a.cu / 32));
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                r.h[j] = load16(src, hst(j) && hk < left ? (from_up ? hoffu[j] : hoff[j]) + c2
                                                         : OUT_OF_RANGE);
        } else {
            const unsigned c2 = (unsigned)(64 * chunk);
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                r.h[j] = load16(xr, hst(j) && hk < left ? hoff[j] + c2 : OUT_OF_RANGE);
        }
        const unsigned c2 = (unsigned)(64 * chunk);
        if (weights) {
#pragma unroll
            for (int j = 0; j < BPT; ++j)
                r.b[j] = load16(wr, bst[j] && bk[j] < left ? boff[j] + c2 : OUT_OF_RANGE);
            r.c = load16(br, coff);
        }
        return r;
    };
    auto lstore = [&](const Stage &r, bool weights) {
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (hst(j))
                *reinterpret_cast<u32x4 *>(&Hs[hlds + 64 * j * LDA]) = r.h[j];
        if (weights) {
#pragma unroll
            for (int j = 0; j < BPT; ++j)
                if (bst[j])
                    *reinterpret_cast<u32x4 *>(&Bs[blds[j]]) = r.b[j];
            if (cload)
                *reinterpret_cast<u32x4 *>(&Cs[4 * tid]) = r.c;
        }
    };
    f32x4 acc[4][NT];
    auto clear = [&]() {
#pragma unroll
        for (int ms = 0; ms < 4; ++ms)
#pragma unroll
            for (int ns = 0; ns < NT; ++ns)
                acc[ms][ns] = f32x4{0.f, 0.f, 0.f, 0.f};
    };
    // fragment ms of wavefront wv: tile row 2 wv + ms / 2, columns
    // 16 (ms % 2) .. + 15; at tap (dy, dx) it reads halo pixel
    // (row + 1 + dy, column + 1 + dx)
    const uint16_t *ha = &Hs[(2 * wv * HW2 + m) * LDA + 8 * g];
    const uint16_t *hb = &Bs[m * LDA + 8 * g];
    auto taps = [&]() {
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t % 3;  // shifted by one
            bf16x8 A[4], B[NT];
#pragma unroll
            for (int ms = 0; ms < 4; ++ms)
                A[ms] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(
                                ha + ((ms / 2 + dy) * HW2 + 16 * (ms % 2) + dx) * LDA));
#pragma unroll
            for (int ns = 0; ns < NT; ++ns)
                B[ns] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(hb + (t * TC + 16 * ns) * LDA));
#pragma unroll
            for (int ms = 0; ms < 4; ++ms)
#pragma unroll
                for (int ns = 0; ns < NT; ++ns)
                    acc[ms][ns] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ms], B[ns], acc[ms][ns], 0, 0, 0);
        }
    };
    // Output through a buffer descriptor: 32-bit offsets built from the
    // row's offset (wavefront-uniform) and the lane's column and channel;
    // pixels past the image's right edge and channels past the layer's get
    // an offset past the range, and the hardware drops those stores.
    constexpr int ESZ = F32OUT ? 4 : 2;
    // UPB: y holds only the channels from a.cd on (channel c at column c - cd)
    const int yc0 = UPB ? a.cd : 0;
    const __amdgpu_buffer_rsrc_t yr_ = __builtin_amdgcn_make_buffer_rsrc(
        a.y, (short)0, (int)(((P - 1) * a.y_pitch + a.cout - yc0) * ESZ), BUF_FORMAT_WORD);
    const unsigned ypb = (unsigned)(a.y_pitch * ESZ);  // bytes per pixel
    const int hp = a.h / 2, wp = a.w / 2;
    const __amdgpu_buffer_rsrc_t pr = __builtin_amdgcn_make_buffer_rsrc(
        POOL ? a.pool : a.y, (short)0,
        POOL ? (int)((((long long)a.n * hp * wp - 1) * a.pool_pitch + a.cout) * 2) : 0,
        BUF_FORMAT_WORD);
    const __amdgpu_buffer_rsrc_t mr = __builtin_amdgcn_make_buffer_rsrc(
        MASK ? const_cast<void *>(a.mask) : a.y, (short)0,
        MASK ? (int)(((P - 1) * a.mask_pitch + a.cout) * 2) : 0, BUF_FORMAT_WORD);
    const unsigned mpb = (unsigned)(a.mask_pitch * 2);
    const __amdgpu_buffer_rsrc_t ur = __builtin_amdgcn_make_buffer_rsrc(
        UPB ? a.du : a.y, (short)0,
        UPB ? (int)((((long long)a.n * hp * wp - 1) * a.du_pitch + a.cd) * 2) : 0,
        BUF_FORMAT_WORD);
    const bool umask = UPB && a.du_mask;
    const __amdgpu_buffer_rsrc_t umr = __builtin_amdgcn_make_buffer_rsrc(
        umask ? const_cast<void *>(a.du_mask) : a.y, (short)0,
        umask ? (int)((((long long)a.n * hp * wp - 1) * a.du_mask_pitch + a.cd) * 2) : 0,
        BUF_FORMAT_WORD);
    auto epilogue = [&](int unit) {
        int n, y0, x0, cg;
        unit_origin(unit, n, y0, x0, cg);
        const int yr = y0 + 2 * wv;  // the wavefront's first row (even)
#pragma unroll
        for (int ns = 0; ns < NT; ++ns) {
            const int c = cg * TC + 16 * ns + m;
            const bool c_ok = c < a.cout;
            const float b = Cs[16 * ns + m];
            // UPB: this 16-channel block belongs to the upsampled input
            // (wavefront-uniform; cd is a multiple of 16)
            const bool up_block = UPB && cg * TC + 16 * ns < a.cd;
            float fv[4][4];  // the stored BF16 values, as floats (POOL, UPB)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (yr + r >= a.h)
                    continue;  // wavefront-uniform
                // the activation's outputs at the row's 8 values of this lane
                // (MASK only), all requested before the first is used
                unsigned short mk[4][4];
                if constexpr (MASK) {
                    const unsigned mrow =
                        (unsigned)((((long long)n * a.h + yr + r) * a.w + x0) * mpb) +
                        (unsigned)(4 * g) * mpb + (unsigned)(c * 2);
#pragma unroll
                    for (int ms = 2 * r; ms < 2 * r + 2; ++ms)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int col = 16 * (ms % 2) + i;
                            const bool ok = c_ok && x0 + col + 4 * g < a.w;
                            mk[ms][i] = __builtin_amdgcn_raw_buffer_load_b16(
                                mr, ok ? mrow + (unsigned)col * mpb : OUT_OF_RANGE, 0, 0);
                        }
                }
                const unsigned lane_off =
                    (unsigned)((((long long)n * a.h + yr + r) * a.w + x0) * ypb) +
                    (unsigned)(4 * g) * ypb + (unsigned)((c - yc0) * ESZ);
#pragma unroll
                for (int ms = 2 * r; ms < 2 * r + 2; ++ms)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int col = 16 * (ms % 2) + i;  // plus 4 g
                        const bool ok = c_ok && x0 + col + 4 * g < a.w;
                        const unsigned off = ok ? lane_off + (unsigned)col * ypb : OUT_OF_RANGE;
                        float v = acc[ms][ns][i] + b;
                        if (LEAKY)
                            v = v > 0.f ? v : a.slope * v;
                        if (F32OUT) {
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v),
                                                                  yr_, off, 0, 0);
                        } else {
                            unsigned short hv = __builtin_bit_cast(unsigned short, (__bf16)v);
                            if constexpr (MASK) {
                                const float d = __builtin_bit_cast(float, (unsigned)hv << 16);
                                const float mv =
                                    __builtin_bit_cast(float, (unsigned)mk[ms][i] << 16);
                                hv = to_bf16(mv > 0.f ? d : a.slope * d);
                            }
                            if (!up_block)
                                __builtin_amdgcn_raw_buffer_store_b16(hv, yr_, off, 0, 0);
                            if (POOL || UPB)
                                fv[ms][i] = __builtin_bit_cast(float, (unsigned)hv << 16);
                        }
                    }
            }
            if constexpr (UPB) {
                if (up_block && yr + 1 < a.h) {  // wavefront-uniform; h is even
                    const long long lrow = ((long long)n * hp + yr / 2) * wp;
                    const unsigned urow = (unsigned)((lrow * a.du_pitch + c) * 2);
                    const unsigned mrow = (unsigned)((lrow * a.du_mask_pitch + c) * 2);
                    // window (rows yr, yr + 1; columns x, x + 1), x = x0 + 16 ms + 4 g + i
                    unsigned off[2][2];
                    unsigned short um[2][2];
#pragma unroll
                    for (int ms = 0; ms < 2; ++ms)
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            const int x = x0 + 16 * ms + 4 * g + 2 * j;
                            const bool ok = c_ok && x < a.w;
                            off[ms][j] = ok ? urow + (unsigned)(x / 2 * a.du_pitch * 2)
                                            : OUT_OF_RANGE;
                            if (umask)
                                um[ms][j] = __builtin_amdgcn_raw_buffer_load_b16(
                                    umr, ok ? mrow + (unsigned)(x / 2 * a.du_mask_pitch * 2)
                                            : OUT_OF_RANGE,
                                    0, 0);
                        }
#pragma unroll
                    for (int ms = 0; ms < 2; ++ms)
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            const int i = 2 * j;
                            const float sum =
                                ((fv[ms][i] + fv[ms][i + 1]) + fv[ms + 2][i]) + fv[ms + 2][i + 1];
                            unsigned short hs = to_bf16(sum);
                            if (umask) {
                                const float d = __builtin_bit_cast(float, (unsigned)hs << 16);
                                const float mv = __builtin_bit_cast(float, (unsigned)um[ms][j] << 16);
                                hs = to_bf16(mv > 0.f ? d : a.slope * d);
                            }
                            __builtin_amdgcn_raw_buffer_store_b16(hs, ur, off[ms][j], 0, 0);
                        }
                }
            }
            if constexpr (POOL && !F32OUT) {
                if (yr + 1 < a.h) {  // wavefront-uniform; h is even
                    const unsigned prow =
                        (unsigned)(((((long long)n * hp + yr / 2) * wp) * a.pool_pitch + c) * 2);
                    // window (rows yr, yr + 1; columns x, x + 1), x = x0 + 16 ms + 4 g + i
#pragma unroll
                    for (int ms = 0; ms < 2; ++ms)
#pragma unroll
                        for (int i = 0; i < 4; i += 2) {
                            const int x = x0 + 16 * ms + 4 * g + i;
                            const float sum =
                                ((fv[ms][i] + fv[ms][i + 1]) + fv[ms + 2][i]) + fv[ms + 2][i + 1];
                            const unsigned off =
                                c_ok && x < a.w ? prow + (unsigned)(x / 2 * a.pool_pitch * 2)
                                                : OUT_OF_RANGE;
                            __builtin_amdgcn_raw_buffer_store_b16(
                                __builtin_bit_cast(unsigned short, (__bf16)(0.25f * sum)), pr, off,
                                0, 0);
                        }
                }
            }
        }
    };

    int unit = vb, chunk = 0;
    unit_offsets(unit);
    Stage st = gload(0, true);
    lstore(st, true);
    __syncthreads();
    clear();
    // with one chunk and one channel group the weights stay in LDS
    const bool reload_b = nck > 1 || groups > 1;
    for (int it = 0; it < items; ++it) {
        int nunit = unit, nchunk = chunk + 1;
        if (nchunk == nck) {
            nchunk = 0;
            nunit += G;
        }
        const bool more = it + 1 < items;
        if (more) {
            if (nunit != unit)
                unit_offsets(nunit);
            st = gload(nchunk, reload_b);
        }
        taps();
        if (chunk == nck - 1) {
            epilogue(unit);
            clear();
        }
        __syncthreads();  // every wavefront is done with the LDS tiles
        if (more)
            lstore(st, reload_b);
        __syncthreads();
        unit = nunit;
        chunk = nchunk;
    }
}

// W'[i][t'][o] = W[o][8 - t][i]: the kernel of the backward-data pass.
__global__ __launch_bounds__(THREADS) void flip_kernel(const uint16_t *__restrict__ w, int cout,
                                                       int cin, uint16_t *__restrict__ wf) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    const long long total = (long long)cout * 9 * cin;
    if (e >= total)
        return;
    const int i = (int)(e % cin);
    const int t = (int)((e / cin) % 9);
    const int o = (int)(e / (9ll * cin));
    wf[((long long)i * 9 + (8 - t)) * cout + o] = w[e];
}

// The same for several layers in one launch: thread e flips element
// e - start[l] of layer l, start[l] <= e < start[l + 1].
__global__ __launch_bounds__(THREADS) void flip_multi_kernel(FlipTable t) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e >= t.start[t.layers])
        return;
    int l = 0;
    while (e >= t.start[l + 1])
        ++l;
    const long long k = e - t.start[l];
    const int cin = t.cin[l], cout = t.cout[l];
    const int i = (int)(k % cin);
    const int tap = (int)((k / cin) % 9);
    const int o = (int)(k / (9ll * cin));
    static_cast<uint16_t *>(t.wf[l])[((long long)i * 9 + (8 - tap)) * cout + o] =
        static_cast<const uint16_t *>(t.w[l])[k];
}

// ------------------------------------------------------- backward weights
// Channel-major copies through LDS tiles of 64 pixels x 64 channels:
// out[ch][q] = X[src(q)][ch], src(q) the pixel dx columns east of q in its
// row (wrapped), zero for the padding pixels q >= P. Loads read 8 channels
// of a pixel (16 bytes), stores write 8 pixels of a channel.
constexpr int TT = 64;

__global__ __launch_bounds__(THREADS) void transpose_kernel(const uint16_t *__restrict__ x,
                                                            int pitch, int c, long long P,
                                                            long long Pp, int w, int dx,
                                                            uint16_t *__restrict__ out) {
    __shared__ uint16_t tile[TT][TT + 8];
    const long long q0 = (long long)blockIdx.x * TT;
    const int c0 = blockIdx.y * TT;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int idx = threadIdx.x + THREADS * k;
        const int px = idx >> 3, chunk = idx & 7;
        const long long q = q0 + px;
        const int ch = c0 + 8 * chunk;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (q < P && ch < c) {
            const long long row = q / w;
            const int xx = wrap((int)(q - row * w) + dx, w);
            v = *reinterpret_cast<const uint4 *>(x + (row * w + xx) * pitch + ch);
        }
        const uint32_t words[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            tile[8 * chunk + 2 * j][px] = (uint16_t)(words[j] & 0xffffu);
            tile[8 * chunk + 2 * j + 1][px] = (uint16_t)(words[j] >> 16);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int idx = threadIdx.x + THREADS * k;
        const int row = idx >> 3, seg = idx & 7;
        const int ch = c0 + row;
        const long long q = q0 + 8 * seg;
        if (ch < c && q < Pp) {
            uint16_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = tile[row][8 * seg + j];
            *reinterpret_cast<uint4 *>(out + (long long)ch * Pp + q) = pack8(v);
        }
    }
}

// Bias gradient, deterministic: block (o, k) sums slice k of row o of dz_t,
// then one thread per channel adds the slices in order.
constexpr int BIAS_SLICES = 32;

__global__ __launch_bounds__(THREADS) void bias_partial_kernel(const uint16_t *__restrict__ dz_t,
                                                               long long Pp,
                                                               float *__restrict__ part) {
    __shared__ float red[THREADS];
    const int o = blockIdx.x, k = blockIdx.y;
    const long long len = (Pp + BIAS_SLICES - 1) / BIAS_SLICES;
    const long long a = k * len;
    const long long b = a + len < Pp ? a + len : Pp;
    const uint16_t *row = dz_t + (long long)o * Pp;
    float s = 0.f;
    for (long long q = a + threadIdx.x; q < b; q += THREADS)
        s += from_bf16(row[q]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = THREADS / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[(long long)o * BIAS_SLICES + k] = red[0];
}

__global__ __launch_bounds__(THREADS) void bias_sum_kernel(const float *__restrict__ part,
                                                           int cout, float *__restrict__ db) {
    const int o = blockIdx.x * THREADS + threadIdx.x;
    if (o >= cout)
        return;
    float s = 0.f;
    for (int k = 0; k < BIAS_SLICES; ++k)
        s += part[(long long)o * BIAS_SLICES + k];
    db[o] = s;
}

// One wavefront: 32 output channels x (16 NI) input channels of one tap,
// over the pixel range of its split; FP32 partial sums to part[split].
template <int NI>
__global__ __launch_bounds__(THREADS) void conv_wgrad_kernel(WgradArgs a) {
    // consecutive waves are the (tap, block) tiles of one pixel range: kept
    // on one XCD, they read that range from HBM once into its L2
    const int wave = xcd_tile(blockIdx.x, gridDim.x) * (THREADS / 64) + (threadIdx.x >> 6);
    const int ot = (a.cout + 31) / 32, it = (a.cin + 16 * NI - 1) / (16 * NI);
    const int per_split = ot * it * 9;
    const int split = wave / per_split;
    if (split >= a.splits)
        return;
    int r = wave - split * per_split;
    const int tap = r % 9;
    r /= 9;
    const int ib = r % it, ob = r / it;
    const int dy = tap / 3 - 1, s = tap % 3;
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, g = lane >> 4;

    int o[2], i[NI];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = ob * 32 + 16 * u + m;
        o[u] = c < a.cout ? c : a.cout - 1;
    }
#pragma unroll
    for (int u = 0; u < NI; ++u) {
        const int c = ib * 16 * NI + 16 * u + m;
        i[u] = c < a.cin ? c : a.cin - 1;
    }
    const uint16_t *dz = a.dz_t;
    const uint16_t *xs = a.xs + (long long)s * a.cin * a.Pp;

    f32x4 acc[2][NI];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < NI; ++v)
            acc[u][v] = f32x4{0.f, 0.f, 0.f, 0.f};

    const long long k0 = (long long)split * a.chunk;
    long long k1 = k0 + a.chunk;
    if (k1 > a.Pr)
        k1 = a.Pr;
    // The lane's 8 pixels q .. q + 7 lie in one row (w % 8 == 0). Its image,
    // row and column are found once and then advanced with the pixel index,
    // so the row shift dy (with its periodic wrap) costs no division per
    // step; padding pixels (q >= P, zero in both planes) are not shifted.
    const long long hw = (long long)a.h * a.w;
    long long q = k0 + 8 * g;
    int yy, xx;
    {
        const long long nn = q / hw;
        const int rr = (int)(q - nn * hw);
        yy = rr / a.w;
        xx = rr - yy * a.w;
    }
    auto shifted = [&]() {
        long long qs = q + (long long)dy * a.w;
        if (q >= a.P)
            qs = q;
        else if (yy + dy < 0)
            qs += hw;
        else if (yy + dy >= a.h)
            qs -= hw;
        return qs;
    };
    auto advance = [&]() {
        q += 32;
        xx += 32;
        while (xx >= a.w) {
            xx -= a.w;
            if (++yy == a.h)
                yy = 0;
        }
    };
    // four k steps of 32 pixels per trip (ranges are multiples of 128): their
    // loads are issued together, then their MFMAs
    constexpr int KB = 4;
    for (long long q0 = k0; q0 < k1; q0 += 32 * KB) {
        bf16x8 A[KB][2], B[KB][NI];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const long long qs = shifted();
#pragma unroll
            for (int u = 0; u < 2; ++u)
                A[kb][u] = load8(dz + (long long)o[u] * a.Pp + q);
#pragma unroll
            for (int v = 0; v < NI; ++v)
                B[kb][v] = load8(xs + (long long)i[v] * a.Pp + qs);
            advance();
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < NI; ++v)
                    acc[u][v] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[kb][u], B[kb][v], acc[u][v], 0, 0, 0);
    }
    // result rows (output channels) 4 g + j of subtile u, column m of subtile v
    float *part = a.part + (long long)split * a.cout * 9 * a.cin;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < NI; ++v) {
            const int ic = ib * 16 * NI + 16 * v + m;
            if (ic >= a.cin)
                continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int oc = ob * 32 + 16 * u + 4 * g + j;
                if (oc < a.cout)
                    part[((long long)oc * 9 + tap) * a.cin + ic] = acc[u][v][j];
            }
        }
}

// ------------------------------------------ weight gradient, halo tiles
// dW[o][t][i] = sum over pixels p of dZ[p][o] X[p + shift_t][i], on images of
// at least 8 x 32 pixels, straight from the NHWC activations. A workgroup
// owns a block of 32 output x 32 input channels and walks pixel tiles of 8
// rows x 32 columns. Per tile, LDS holds the dZ tile (256 pixels) and the
// input tile with its one-pixel halo (10 x 34 pixels, periodic wrap) in
// their natural pixel-major layout, one 16-byte store per 8 channels; pixels
// outside the image carry dZ = 0. The MFMA fragments need the opposite
// order (8 consecutive pixels of one channel per lane): they are read with
// the LDS transpose load, which hands lane i of each 16-lane group element
// j of the 8-byte piece addressed by lane 4 j + i / 4, at element i % 4.
// When lane 4 q + r of a group addresses pixel k0 + q, channels c0 + 4 r ..
// + 3, lane i receives channel c0 + i of pixels k0 .. k0 + 3; two such loads
// (k0 and k0 + 4) make a fragment. A tap's horizontal shift is a shift of
// the pixel rows, so one copy of the input tile serves all nine taps.
// Wavefront w takes tile rows 2w and 2w + 1 as its k steps (32 pixels
// each). For each horizontal shift it reads the four halo rows those steps
// touch once and uses each for every vertical shift it serves (12 MFMAs per
// pair of fragments); the next tile's loads are in flight meanwhile. The four
// wavefronts' sums are added in LDS and written as the workgroup's split of
// the fixed-order reduction below. The workgroups of input block 0 also sum
// the dZ tile per output channel (the bias gradient): thread (pixel group
// s, channels 8 j .. 8 j + 7) over pixels s, s + 64, s + 128, s + 192 of
// every tile; the 64 sums of a channel are then added in order.
constexpr int WH_TH = 8, WH_TW = 32;     // pixel tile
constexpr int WH_HW = WH_TW + 2;         // halo tile columns
constexpr int WH_HPIX = (WH_TH + 2) * WH_HW;
constexpr int WH_PZ = 40;  // LDS row pitch (elements) of a dZ pixel: 16-byte stores
constexpr int WH_PX = 40;  // and of an input pixel
constexpr int WH_ZP = WH_TH * WH_TW * 4 / THREADS;           // 16-byte pieces a thread loads
constexpr int WH_XP = (WH_HPIX * 4 + THREADS - 1) / THREADS;
constexpr int WH_RESIDENT = 512;         // two workgroups per CU on 256 CUs
constexpr int WH_LDS = WH_TH * WH_TW * WH_PZ + WH_HPIX * WH_PX;  // elements
static_assert(WH_LDS * 2 >= 9 * 2 * 2 * 4 * 64 * 4, "the cross-wavefront sums reuse the tiles");

typedef short v4s __attribute__((ext_vector_type(4)));

// One MFMA fragment from a pixel-major LDS tile: the element pointers p0 and
// p1 (8-byte aligned) are this lane's addresses for pixels k0 + q and
// k0 + 4 + q as described above.
__device__ __forceinline__ bf16x8 tr_fragment(const uint16_t *p0, const uint16_t *p1) {
    typedef __attribute__((address_space(3))) v4s *lds_v4s;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p0));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p1));
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

struct WgradHaloArgs {
    const uint16_t *x, *dz;
    int xp, dzp, n, h, w, cin, cout;
    // input channels [0, cu) from xu (n, h/2, w/2) as its nearest 2x
    // upsampling, [cu, cin) from x (x's channel 0 is input channel cu);
    // xu null: all from x (cu = 0). cu is a multiple of 32, so a block of
    // 32 input channels comes from one view.
    const uint16_t *xu;
    int xup, cu;
    int nob, nib, gb, tiles, tiles_x, tiles_y;
    float *part;    // [gb][cout][9][cin]
    float *part_b;  // [gb][cout]
};

__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void conv_wgrad_halo_kernel(WgradHaloArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[WH_LDS];
    uint16_t *const Zs = lds;
    uint16_t *const Xs = lds + WH_TH * WH_TW * WH_PZ;
    constexpr unsigned OUT_OF_RANGE = 0x80000000u;
    const int blocks = a.nob * a.nib;
    // Workgroup b runs on XCD b % 8, each with its own L2: the channel
    // blocks of one split (which read the same tiles) are given to the
    // workgroups of one XCD.
    const int nwg = gridDim.x;
    const int vb = nwg % 8 == 0 ? (int)(blockIdx.x % 8) * (nwg / 8) + (int)(blockIdx.x / 8)
                                : (int)blockIdx.x;
    const int blk = vb % blocks, kb = vb / blocks;
    const int ob = blk / a.nib, ib = blk - (blk / a.nib) * a.nib;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const long long P = (long long)a.n * a.h * a.w;
    const int oc0 = ob * 32, ic0 = ib * 32;
    const bool from_up = ic0 < a.cu;  // workgroup-uniform
    const int hu = a.h / 2, wu = a.w / 2;
    const __amdgpu_buffer_rsrc_t xr =
        from_up ? __builtin_amdgcn_make_buffer_rsrc(
                      const_cast<uint16_t *>(a.xu), (short)0,
                      (int)((((long long)a.n * hu * wu - 1) * a.xup + a.cu) * 2), BUF_FORMAT_WORD)
                : __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(a.x), (short)0,
                                                    (int)(((P - 1) * a.xp + a.cin - a.cu) * 2),
                                                    BUF_FORMAT_WORD);
    const __amdgpu_buffer_rsrc_t dr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t *>(a.dz), (short)0, (int)(((P - 1) * a.dzp + a.cout) * 2),
        BUF_FORMAT_WORD);

    // the 16-byte pieces of a tile: dZ piece e = tid + 256 r is pixel e / 4
    // (tile row e / 128, column (e / 4) % 32), channels 8 (e % 4) ..; input
    // piece e (e < 1360) is halo pixel e / 4, channels 8 (e % 4) ..
    const int j8 = 8 * (tid & 3);
    struct Stage {
        u32x4 z[WH_ZP], x[WH_XP];
    };
    auto gload = [&](int tile) {
        Stage st;
        const int per_image = a.tiles_x * a.tiles_y;
        const int n = tile / per_image;
        const int rt = tile - n * per_image;
        const int y0 = (rt / a.tiles_x) * WH_TH, x0 = (rt - (rt / a.tiles_x) * a.tiles_x) * WH_TW;
        const int oc = oc0 + j8;
#pragma unroll
        for (int r = 0; r < WH_ZP; ++r) {
            const int px = (tid >> 2) + 64 * r;
            const int y = y0 + (px >> 5), x = x0 + (px & 31);
            const bool ok = y < a.h && x < a.w && oc < a.cout;
            const long long q = ((long long)n * a.h + y) * a.w + x;
            st.z[r] = load16(dr, ok ? (unsigned)((q * a.dzp + oc) * 2) : OUT_OF_RANGE);
        }
        const int ic = ic0 + j8;
#pragma unroll
        for (int r = 0; r < WH_XP; ++r) {
            const int hp = min((tid >> 2) + 64 * r, WH_HPIX - 1);
            const int hr = hp / WH_HW, hc = hp - (hp / WH_HW) * WH_HW;
            const int y = wrap(y0 - 1 + hr, a.h), x = wrap(x0 - 1 + hc, a.w);
            unsigned off;
            if (from_up)
                off = (unsigned)(((((long long)n * hu + (y >> 1)) * wu + (x >> 1)) * a.xup + ic) * 2);
            else
                off = ic < a.cin ? (unsigned)(((((long long)n * a.h + y) * a.w + x) * a.xp + ic - a.cu) * 2)
                                 : OUT_OF_RANGE;
            st.x[r] = load16(xr, off);
        }
        return st;
    };
    auto lstore = [&](const Stage &st) {
#pragma unroll
        for (int r = 0; r < WH_ZP; ++r)
            *reinterpret_cast<u32x4 *>(&Zs[((tid >> 2) + 64 * r) * WH_PZ + j8]) = st.z[r];
#pragma unroll
        for (int r = 0; r < WH_XP; ++r)
            if ((tid >> 2) + 64 * r < WH_HPIX)
                *reinterpret_cast<u32x4 *>(&Xs[((tid >> 2) + 64 * r) * WH_PX + j8]) = st.x[r];
    };

    f32x4 acc[9][2][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
                acc[t][u][v] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool bias_block = ib == 0;
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // channels 8 (tid % 4) ..

    // this lane's transpose-load addresses (elements): pixel row offset q
    // within a group of four, channel offset 4 r
    const int tq = 8 * g + (m >> 2), tc = 4 * (m & 3);
    const uint16_t *za = Zs + (2 * wv * WH_TW + tq) * WH_PZ + tc;
    const uint16_t *xa = Xs + (2 * wv * WH_HW + tq) * WH_PX + tc;

    int tile = kb;
    if (tile < a.tiles)
        lstore(gload(tile));
    __syncthreads();
    for (; tile < a.tiles; tile += a.gb) {
        const bool more = tile + a.gb < a.tiles;
        Stage next;
        if (more)
            next = gload(tile + a.gb);
        if (bias_block) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const u32x4 v = *reinterpret_cast<const u32x4 *>(
                    &Zs[((tid >> 2) + 64 * r) * WH_PZ + j8]);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    bsum[2 * k] += __builtin_bit_cast(float, v[k] << 16);
                    bsum[2 * k + 1] += __builtin_bit_cast(float, v[k] & 0xffff0000u);
                }
            }
        }
        // dZ fragments of both k steps (rows 2 wv + kk), both 16-channel halves
        bf16x8 A[2][2];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint16_t *p = za + (kk * WH_TW) * WH_PZ + 16 * u;
                A[kk][u] = tr_fragment(p, p + 4 * WH_PZ);
            }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                // halo rows 2 wv + rr, rr = kk + dy
                bf16x8 B[4];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const uint16_t *p = xa + (rr * WH_HW + dx) * WH_PX + 16 * v;
                    B[rr] = tr_fragment(p, p + 4 * WH_PX);
                }
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                        for (int u = 0; u < 2; ++u)
                            acc[3 * dy + dx][u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                A[kk][u], B[kk + dy], acc[3 * dy + dx][u][v], 0, 0, 0);
            }
        __syncthreads();  // every wavefront is done with the tiles
        if (more)
            lstore(next);
        __syncthreads();
    }
    if (bias_block) {
        // channel 8 (t % 4) + k of thread t: the 64 sums of a channel (the
        // threads t with the same t % 4), added in thread order
        float *red = reinterpret_cast<float *>(lds);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            red[k * THREADS + tid] = bsum[k];
        __syncthreads();
        if (tid < 32) {
            const int k = tid & 7, c4 = tid >> 3;  // channel 8 c4 + k
            float b = 0.f;
            for (int s = 0; s < 64; ++s)
                b += red[k * THREADS + 4 * s + c4];
            if (oc0 + tid < a.cout)
                a.part_b[(long long)kb * a.cout + oc0 + tid] = b;
        }
        __syncthreads();
    }
    // The four wavefronts' sums, added in LDS in a fixed order,
    // (w0 + w2) + (w1 + w3), one wavefront's worth (144 values a lane) at a
    // time; the workgroup then writes its split.
    float *red = reinterpret_cast<float *>(lds);
    auto put = [&]() {
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        red[(((t * 2 + u) * 2 + v) * 4 + jj) * 64 + lane] = acc[t][u][v][jj];
    };
    auto add = [&]() {
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        acc[t][u][v][jj] += red[(((t * 2 + u) * 2 + v) * 4 + jj) * 64 + lane];
    };
    __syncthreads();  // the tile area is free
    if (wv == 2)
        put();
    __syncthreads();
    if (wv == 0)
        add();
    __syncthreads();
    if (wv == 3)
        put();
    __syncthreads();
    if (wv == 1)
        add();
    __syncthreads();
    if (wv == 1)
        put();
    __syncthreads();
    if (wv == 0) {
        add();
        // the block's sums in LDS as [o][t][i] (32 x 9 x 32), over the
        // values just read (a wavefront's LDS accesses stay in order)
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        red[((16 * u + 4 * g + jj) * 9 + t) * 32 + 16 * v + m] = acc[t][u][v][jj];
    }
    __syncthreads();
    // the workgroup's split, rows of 32 input channels per (output channel, tap)
    const long long count = (long long)a.cout * 9 * a.cin;
    float *part = a.part + (long long)kb * count;
    for (int e = tid; e < 32 * 9 * 32; e += THREADS) {
        const int o = e / 288, r = e - o * 288;
        const int t = r >> 5, i = r & 31;
        if (oc0 + o < a.cout && ic0 + i < a.cin)
            part[((long long)(oc0 + o) * 9 + t) * a.cin + ic0 + i] = red[e];
    }
}

// dW (and the bias gradient) = the sum of the splits' partials in a fixed
// order, in one launch. A workgroup owns C = 256 / R consecutive outputs
// (the dW values, then the bias values) and R groups of consecutive splits:
// thread (group r, output j) adds the splits of group r in order, and the
// R group sums of an output are then added in group order. Lanes of a
// wavefront read consecutive outputs of one split (coalesced rows).
__global__ __launch_bounds__(THREADS) void splits_sum_kernel(const float *__restrict__ part,
                                                             long long count, float *__restrict__ dw,
                                                             const float *__restrict__ part_b,
                                                             int nb, float *__restrict__ db,
                                                             int splits, int R) {
    __shared__ float red[THREADS];
    const int C = THREADS / R;
    const int tid = threadIdx.x, j = tid % C, r = tid / C;
    const long long e = (long long)blockIdx.x * C + j;
    const long long total = count + (db ? nb : 0);
    const float *src = nullptr;
    long long stride = 0;
    if (e < count) {
        src = part + e;
        stride = count;
    } else if (e < total) {
        src = part_b + (e - count);
        stride = nb;
    }
    const int per = (splits + R - 1) / R;
    const int k0 = r * per, k1 = min(k0 + per, splits);
    float sum = 0.f;
    if (src) {
#pragma unroll 8
        for (int k = k0; k < k1; ++k)
            sum += src[(long long)k * stride];
    }
    red[tid] = sum;
    __syncthreads();
    if (r == 0 && src) {
        float t = red[j];
        for (int q = 1; q < R; ++q)
            t += red[q * C + j];
        if (e < count)
            dw[e] = t;
        else
            db[e - count] = t;
    }
}


// --------------------------------------------------------- elementwise ops
// Each thread handles 8 channels of one pixel as one 16-byte access per
// operand (views are 16-byte aligned with pitches and channel counts that
// are multiples of 8).
__device__ __forceinline__ u32x4 ld8(const uint16_t *p) {
    return *reinterpret_cast<const u32x4 *>(p);
}
__device__ __forceinline__ void st8(uint16_t *p, u32x4 v) { *reinterpret_cast<u32x4 *>(p) = v; }
// the BF16 values 2k and 2k + 1 of an 8-value vector as floats
__device__ __forceinline__ float lo_of(unsigned w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float hi_of(unsigned w) {
    return __builtin_bit_cast(float, w & 0xffff0000u);
}
__device__ __forceinline__ unsigned pack2(float lo, float hi) {
    return (unsigned)to_bf16(lo) | ((unsigned)to_bf16(hi) << 16);
}
// The activation adjoint on eight stored BF16 gradients d: m > 0 ? d :
// slope d, m the activation's outputs at the same elements, rounded to BF16.
__device__ __forceinline__ u32x4 leaky_adjoint(u32x4 d, u32x4 m, float slope) {
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float d0 = lo_of(d[k]), d1 = hi_of(d[k]);
        o[k] = pack2(lo_of(m[k]) > 0.f ? d0 : slope * d0, hi_of(m[k]) > 0.f ? d1 : slope * d1);
    }
    return o;
}

__global__ __launch_bounds__(THREADS) void leaky_bwd_kernel(const uint16_t *__restrict__ dy,
                                                            int dyp, const uint16_t *__restrict__ y,
                                                            int yp, uint16_t *__restrict__ dz,
                                                            int dzp, long long pixels, int c,
                                                            float slope) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    const int c8 = c / 8;
    if (e >= pixels * c8)
        return;
    const long long q = e / c8;
    const int ch = (int)(e - q * c8) * 8;
    st8(dz + q * dzp + ch, leaky_adjoint(ld8(dy + q * dyp + ch), ld8(y + q * yp + ch), slope));
}

// y (n, h/2, w/2) = mean of 2x2 windows of x (n, h, w)
__global__ __launch_bounds__(THREADS) void pool2_kernel(const uint16_t *__restrict__ x, int xp,
                                                        int n, int h, int w, int c,
                                                        uint16_t *__restrict__ y, int yp) {
    const int ho = h / 2, wo = w / 2, c8 = c / 8;
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e >= (long long)n * ho * wo * c8)
        return;
    const long long q = e / c8;
    const int ch = (int)(e - q * c8) * 8;
    const int xo = (int)(q % wo);
    const long long r = q / wo;
    const int yo = (int)(r % ho);
    const int nn = (int)(r / ho);
    const uint16_t *p = x + (((long long)nn * h + 2 * yo) * w + 2 * xo) * xp + ch;
    const long long down = (long long)w * xp;
    const u32x4 v00 = ld8(p), v01 = ld8(p + xp), v10 = ld8(p + down), v11 = ld8(p + down + xp);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s0 = ((lo_of(v00[k]) + lo_of(v01[k])) + lo_of(v10[k])) + lo_of(v11[k]);
        const float s1 = ((hi_of(v00[k]) + hi_of(v01[k])) + hi_of(v10[k])) + hi_of(v11[k]);
        o[k] = pack2(0.25f * s0, 0.25f * s1);
    }
    st8(y + q * yp + ch, o);
}

// dx (n, h, w) (+)= dy (n, h/2, w/2) / 4 at the window's four inputs; with
// a mask (a BF16 view of the activation output at dx's pixels), the stored
// sum then goes through the activation's adjoint (leaky_adjoint).
__global__ __launch_bounds__(THREADS) void pool2_bwd_kernel(const uint16_t *__restrict__ dy,
                                                            int dyp, int n, int h, int w, int c,
                                                            uint16_t *__restrict__ dx, int dxp,
                                                            int accumulate,
                                                            const uint16_t *__restrict__ mask,
                                                            int mp, float slope) {
    const int c8 = c / 8;
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e >= (long long)n * h * w * c8)
        return;
    const long long q = e / c8;
    const int ch = (int)(e - q * c8) * 8;
    const int xx = (int)(q % w);
    const long long r = q / w;
    const int yy = (int)(r % h);
    const int nn = (int)(r / h);
    const long long qo = ((long long)nn * (h / 2) + yy / 2) * (w / 2) + xx / 2;
    const u32x4 d = ld8(dy + qo * dyp + ch);
    u32x4 o;
    if (accumulate) {
        const u32x4 v = ld8(dx + q * dxp + ch);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = pack2(0.25f * lo_of(d[k]) + lo_of(v[k]), 0.25f * hi_of(d[k]) + hi_of(v[k]));
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = pack2(0.25f * lo_of(d[k]), 0.25f * hi_of(d[k]));
    }
    if (mask)
        o = leaky_adjoint(o, ld8(mask + q * mp + ch), slope);
    st8(dx + q * dxp + ch, o);
}

// y (n, 2h, 2w) = x (n, h, w) repeated over 2x2 windows
__global__ __launch_bounds__(THREADS) void up2_kernel(const uint16_t *__restrict__ x, int xp,
                                                      int n, int h, int w, int c,
                                                      uint16_t *__restrict__ y, int yp) {
    const int c8 = c / 8, H = 2 * h, W = 2 * w;
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e >= (long long)n * H * W * c8)
        return;
    const long long q = e / c8;
    const int ch = (int)(e - q * c8) * 8;
    const int xx = (int)(q % W);
    const long long r = q / W;
    const int yy = (int)(r % H);
    const int nn = (int)(r / H);
    const long long qi = ((long long)nn * h + yy / 2) * w + xx / 2;
    st8(y + q * yp + ch, ld8(x + qi * xp + ch));
}

// dx (n, h, w) = sum of dy (n, 2h, 2w) over each 2x2 window; with a mask
// (a BF16 view of the activation output at dx's pixels), the stored sum
// then goes through the activation's adjoint (leaky_adjoint).
__global__ __launch_bounds__(THREADS) void up2_bwd_kernel(const uint16_t *__restrict__ dy,
                                                          int dyp, int n, int h, int w, int c,
                                                          uint16_t *__restrict__ dx, int dxp,
                                                          const uint16_t *__restrict__ mask,
                                                          int mp, float slope) {
    const int c8 = c / 8;
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e >= (long long)n * h * w * c8)
        return;
    const long long q = e / c8;
    const int ch = (int)(e - q * c8) * 8;
    const int xx = (int)(q % w);
    const long long r = q / w;
    const int yy = (int)(r % h);
    const int nn = (int)(r / h);
    const uint16_t *p = dy + (((long long)nn * 2 * h + 2 * yy) * 2 * w + 2 * xx) * dyp + ch;
    const long long down = 2LL * w * dyp;
    const u32x4 v00 = ld8(p), v01 = ld8(p + dyp), v10 = ld8(p + down), v11 = ld8(p + down + dyp);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s0 = ((lo_of(v00[k]) + lo_of(v01[k])) + lo_of(v10[k])) + lo_of(v11[k]);
        const float s1 = ((hi_of(v00[k]) + hi_of(v01[k])) + hi_of(v10[k])) + hi_of(v11[k]);
        o[k] = pack2(s0, s1);
    }
    if (mask)
        o = leaky_adjoint(o, ld8(mask + q * mp + ch), slope);
    st8(dx + q * dxp + ch, o);
}

// ------------------------------------------------- surrogate input / output
// x[b, y, x, :] = (rho_c / scale_c for c < 5, the 9 parameter values, 0, 0)
__global__ __launch_bounds__(THREADS) void pack_input_kernel(const float *__restrict__ rho,
                                                             int batch, int h, int w,
                                                             const float *__restrict__ planes,
                                                             IoScales s,
                                                             uint16_t *__restrict__ x) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    const long long hw = (long long)h * w;
    if (e >= batch * hw)
        return;
    const long long b = e / hw, p = e - b * hw;
    uint16_t v[SUR_IN_CHANNELS];
#pragma unroll
    for (int c = 0; c < 5; ++c)
        v[c] = to_bf16(rho[(b * 5 + c) * hw + p] * s.inv_in[c]);
#pragma unroll
    for (int k = 0; k < 9; ++k)
        v[5 + k] = to_bf16(planes[b * 9 + k]);
    v[14] = v[15] = 0;
    uint4 *dst = reinterpret_cast<uint4 *>(x + e * SUR_IN_CHANNELS);
    dst[0] = pack8(v);
    dst[1] = pack8(v + 8);
}

// rho_next[b, c] = rho[b, c] + scale_out_c * out[b, y, x, c] for c < 5
__global__ __launch_bounds__(THREADS) void apply_output_kernel(const float *__restrict__ rho,
                                                               const float *__restrict__ out,
                                                               int batch, int h, int w,
                                                               IoScales s,
                                                               float *__restrict__ next) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    const long long hw = (long long)h * w;
    if (e >= batch * hw * 5)
        return;
    const long long p = e % hw;
    const long long bc = e / hw;
    const int c = (int)(bc % 5);
    const long long b = bc / 5;
    next[e] = rho[e] + s.out[c] * out[(b * hw + p) * SUR_OUT_CHANNELS + c];
}

// Loss = mean over (b, y, x, c < 5) of (out - (target - rho) / scale_out)^2;
// dout = its gradient (BF16, channels >= 5 zero); per-block FP64 partials.
__global__ __launch_bounds__(THREADS) void mse_kernel(const float *__restrict__ out,
                                                      const float *__restrict__ rho,
                                                      const float *__restrict__ target, int batch,
                                                      int h, int w, IoScales s,
                                                      uint16_t *__restrict__ dout,
                                                      double *__restrict__ partials) {
    __shared__ double red[THREADS];
    const long long hw = (long long)h * w;
    const long long pixels = batch * hw;
    const double inv_count = 1.0 / (double)(pixels * 5);
    double acc = 0.0;
    for (long long q = (long long)blockIdx.x * THREADS + threadIdx.x; q < pixels;
         q += (long long)gridDim.x * THREADS) {
        const long long b = q / hw, p = q - b * hw;
        uint16_t gv[SUR_OUT_CHANNELS];
#pragma unroll
        for (int c = 0; c < SUR_OUT_CHANNELS; ++c)
            gv[c] = 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const long long k = (b * 5 + c) * hw + p;
            const float r = (target[k] - rho[k]) * s.inv_out[c];
            const float d = out[q * SUR_OUT_CHANNELS + c] - r;
            acc += (double)d * (double)d;
            gv[c] = to_bf16((float)(2.0 * inv_count) * d);
        }
        uint4 *dst = reinterpret_cast<uint4 *>(dout + q * SUR_OUT_CHANNELS);
        dst[0] = pack8(gv);
        dst[1] = pack8(gv + 8);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = THREADS / 2; k >= 1; k >>= 1) {
        if ((int)threadIdx.x < k)
            red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partials[blockIdx.x] = red[0] * inv_count;
}

__global__ __launch_bounds__(THREADS) void sum_partials_kernel(const double *__restrict__ p,
                                                               int count,
                                                               double *__restrict__ out) {
    __shared__ double red[THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += THREADS)
        s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = THREADS / 2; k >= 1; k >>= 1) {
        if ((int)threadIdx.x < k)
            red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = red[0];
}

// ------------------------------------------------------------------- Adam
__global__ __launch_bounds__(THREADS) void adam_kernel(float *__restrict__ theta,
                                                       uint16_t *__restrict__ theta_bf16,
                                                       const float *__restrict__ grad,
                                                       float *__restrict__ m,
                                                       float *__restrict__ v, long long count,
                                                       AdamArgs a) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e >= count)
        return;
    const float gr = grad[e];
    const float mm = a.beta1 * m[e] + (1.f - a.beta1) * gr;
    const float vv = a.beta2 * v[e] + (1.f - a.beta2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    const float t = theta[e] - a.lr * (mm * a.inv_bc1) / (sqrtf(vv * a.inv_bc2) + a.eps);
    theta[e] = t;
    if (theta_bf16)
        theta_bf16[e] = to_bf16(t);
}

__global__ __launch_bounds__(THREADS) void to_bf16_kernel(const float *__restrict__ src,
                                                          uint16_t *__restrict__ dst,
                                                          long long count) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (e < count)
        dst[e] = to_bf16(src[e]);
}

__global__ __launch_bounds__(THREADS) void crop_kernel(const float *__restrict__ rho, int h, int w,
                                                       int y0, int x0, int ch, int cw,
                                                       float *__restrict__ dst) {
    const long long e = (long long)blockIdx.x * THREADS + threadIdx.x;
    const long long area = (long long)ch * cw;
    if (e >= 5 * area)
        return;
    const int c = (int)(e / area);
    const long long r = e - c * area;
    const int j = (int)(r / cw), i = (int)(r - (long long)j * cw);
    int y = (y0 + j) % h, x = (x0 + i) % w;
    if (y < 0)
        y += h;
    if (x < 0)
        x += w;
    dst[e] = rho[((long long)c * h + y) * w + x];
}

unsigned blocks_for(long long work) { return (unsigned)((work + THREADS - 1) / THREADS); }

// The sums over `splits` partials of `count` dW values each (rows of
// `count`), and of `nb` bias values each when db is not null (rows of nb
// at part_b), in one launch: R groups of splits per output, R a power of
// two up to 16 with about four or more splits a group.
static void reduce_splits(const float *part, int splits, long long count, float *dw,
                          const float *part_b, int nb, float *db, hipStream_t s) {
    int R = 1;
    while (R < 16 && 4 * (2 * R) <= splits)
        R *= 2;
    const int C = THREADS / R;
    const long long total = count + (db ? nb : 0);
    hipLaunchKernelGGL(splits_sum_kernel, dim3((unsigned)((total + C - 1) / C)), dim3(THREADS), 0,
                       s, part, count, dw, part_b, nb, db, splits, R);
}

}  // namespace

template <int WM, int NT>
static void conv_fwd_cfg(const ConvArgs &a, bool leaky, bool f32out, hipStream_t s) {
    constexpr int TP = 64 * WM, TC = 16 * NT * (4 / WM);
    const long long P = (long long)a.n * a.h * a.w;
    const long long blocks = (P + TP - 1) / TP * ((a.cout + TC - 1) / TC);
    const dim3 grid((unsigned)blocks), block(THREADS);
    if (f32out && leaky)
        hipLaunchKernelGGL((conv_fwd_kernel<WM, NT, true, true>), grid, block, 0, s, a);
    else if (f32out)
        hipLaunchKernelGGL((conv_fwd_kernel<WM, NT, true, false>), grid, block, 0, s, a);
    else if (leaky)
        hipLaunchKernelGGL((conv_fwd_kernel<WM, NT, false, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((conv_fwd_kernel<WM, NT, false, false>), grid, block, 0, s, a);
}

// Workgroups of kernel f (256 threads) resident on the current device at
// once, from its register and LDS use; 0 if the runtime cannot say.
// (Queried once per kernel and device: `cache` holds one slot per device.)
constexpr int MAX_DEVICES = 64;
static int resident_workgroups(const void *f, std::atomic<int> *cache) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (dev >= 0 && dev < MAX_DEVICES) {
        const int known = cache[dev].load(std::memory_order_relaxed);
        if (known > 0)
            return known;
    }
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, THREADS, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (dev >= 0 && dev < MAX_DEVICES)
        cache[dev].store(cus * per_cu, std::memory_order_relaxed);
    return cus * per_cu;
}

template <int NT, bool F32OUT, bool LEAKY, bool POOL, bool UP = false, bool MASK = false,
          bool UPB = false>
static void conv_halo_go(const ConvArgs &a, hipStream_t s) {
    static std::atomic<int> cache[MAX_DEVICES];  // zero-initialised (static storage)
    const int tiles_x = (a.w + HALO_TW - 1) / HALO_TW, tiles_y = (a.h + HALO_TH - 1) / HALO_TH;
    const int units = a.n * tiles_x * tiles_y * ((a.cout + 16 * NT - 1) / (16 * NT));
    const void *f = (const void *)conv_halo_kernel<NT, F32OUT, LEAKY, POOL, UP, MASK, UPB>;
    const int resident = resident_workgroups(f, cache);
    const int blocks = resident > 0 && resident < units ? resident : units;
    hipLaunchKernelGGL((conv_halo_kernel<NT, F32OUT, LEAKY, POOL, UP, MASK, UPB>),
                       dim3((unsigned)blocks), dim3(THREADS), 0, s, a, tiles_x, tiles_y, units);
}

template <int NT>
static void conv_halo_cfg(const ConvArgs &a, bool leaky, bool f32out, hipStream_t s) {
    if (a.du) {  // backward-data with the upsampling adjoint: BF16, no bias
        conv_halo_go<NT, false, false, false, false, false, true>(a, s);
    } else if (a.mask) {  // the backward-data pass: BF16 output, no bias or activation
        conv_halo_go<NT, false, false, false, false, true>(a, s);
    } else if (a.xu) {  // BF16 output, no pooling (a decoder's first convolution)
        if (leaky)
            conv_halo_go<NT, false, true, false, true>(a, s);
        else
            conv_halo_go<NT, false, false, false, true>(a, s);
    } else if (a.pool) {  // BF16 output only
        if (leaky)
            conv_halo_go<NT, false, true, true>(a, s);
        else
            conv_halo_go<NT, false, false, true>(a, s);
    } else if (f32out && leaky) {
        conv_halo_go<NT, true, true, false>(a, s);
    } else if (f32out) {
        conv_halo_go<NT, true, false, false>(a, s);
    } else if (leaky) {
        conv_halo_go<NT, false, true, false>(a, s);
    } else {
        conv_halo_go<NT, false, false, false>(a, s);
    }
}

// Images of at least 8 x 32 pixels: halo tiles of 16, 32 or 64 output
// channels. Smaller images: workgroup tiles of 128 pixels x 64 channels for
// wide layers, 256 x 32 and 256 x 16 for narrow ones (no channel tile wider
// than the layer).
hipError_t launch_conv_fwd(const ConvArgs &a, bool leaky, bool f32out, hipStream_t s) {
    const long long units = (long long)a.n * ((a.h + HALO_TH - 1) / HALO_TH) *
                            ((a.w + HALO_TW - 1) / HALO_TW) * ((a.cout + 15) / 16);
    const long long out_bytes =
        (((long long)a.n * a.h * a.w - 1) * a.y_pitch + a.cout) * (f32out ? 4 : 2);
    const long long pool_bytes =
        a.pool ? (((long long)a.n * (a.h / 2) * (a.w / 2) - 1) * a.pool_pitch + a.cout) * 2 : 0;
    const long long mask_bytes =
        a.mask ? (((long long)a.n * a.h * a.w - 1) * a.mask_pitch + a.cout) * 2 : 0;
    if (a.mask && (leaky || f32out || a.pool || a.xu))
        return hipErrorInvalidValue;  // the mask goes with plain BF16 outputs only
    if (a.du && (leaky || f32out || a.pool || a.xu || a.mask || a.cd <= 0 || a.cd % 16 ||
                 a.cd > a.cout || a.h % 2 || a.w % 2))
        return hipErrorInvalidValue;  // the upsampling adjoint: plain BF16, even sizes
    const long long half = (long long)a.n * (a.h / 2) * (a.w / 2);
    const long long du_bytes = a.du ? ((half - 1) * a.du_pitch + a.cd) * 2 : 0;
    const long long du_mask_bytes = a.du_mask ? ((half - 1) * a.du_mask_pitch + a.cd) * 2 : 0;
    const bool halo = a.h >= HALO_TH && a.w >= HALO_TW && units < (1ll << 31) &&
                      out_bytes < (1ll << 31) && pool_bytes < (1ll << 31) &&
                      mask_bytes < (1ll << 31) && du_bytes < (1ll << 31) &&
                      du_mask_bytes < (1ll << 31);
    if ((a.xu || a.du) && !halo)
        return hipErrorNotSupported;  // the upsampled input and its adjoint need halo tiles
    if (halo) {
        if (a.cout > 32)
            conv_halo_cfg<4>(a, leaky, f32out, s);
        else if (a.cout > 16)
            conv_halo_cfg<2>(a, leaky, f32out, s);
        else
            conv_halo_cfg<1>(a, leaky, f32out, s);
        return hipGetLastError();
    }
    if (a.cout >= 64)
        conv_fwd_cfg<2, 2>(a, leaky, f32out, s);
    else if (a.cout > 16)
        conv_fwd_cfg<4, 2>(a, leaky, f32out, s);
    else
        conv_fwd_cfg<4, 1>(a, leaky, f32out, s);
    if (a.pool) {  // the tiled kernel has no pooling epilogue
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        return launch_pool2(a.y, a.y_pitch, a.n, a.h, a.w, a.cout, a.pool, a.pool_pitch, s);
    }
    if (a.mask) {  // nor a mask epilogue: the activation adjoint in place
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        return launch_leaky_bwd(a.y, a.y_pitch, a.mask, a.mask_pitch, a.y, a.y_pitch,
                                (long long)a.n * a.h * a.w, a.cout, a.slope, s);
    }
    return hipGetLastError();
}

hipError_t launch_flip(const void *w, int cout, int cin, void *wf, hipStream_t s) {
    hipLaunchKernelGGL(flip_kernel, dim3(blocks_for((long long)cout * 9 * cin)), dim3(THREADS), 0,
                       s, static_cast<const uint16_t *>(w), cout, cin,
                       static_cast<uint16_t *>(wf));
    return hipGetLastError();
}

hipError_t launch_flip_multi(const FlipTable &t, hipStream_t s) {
    hipLaunchKernelGGL(flip_multi_kernel, dim3(blocks_for(t.start[t.layers])), dim3(THREADS), 0, s,
                       t);
    return hipGetLastError();
}

WgradPlan wgrad_plan(int n, int h, int w, int cin, int cout) {
    WgradPlan p;
    p.P = (long long)n * h * w;
    p.tiles_x = (w + WH_TW - 1) / WH_TW;
    p.tiles_y = (h + WH_TH - 1) / WH_TH;
    const long long tiles = (long long)n * p.tiles_x * p.tiles_y;
    p.halo = h >= WH_TH && w >= WH_TW && tiles < (1ll << 31);
    if (p.halo) {
        p.tiles = (int)tiles;
        p.nob = (cout + 31) / 32;
        p.nib = (cin + 31) / 32;
        const int blocks = p.nob * p.nib;
        long long gb = WH_RESIDENT / blocks;
        gb = gb < 1 ? 1 : (gb > tiles ? tiles : gb);
        p.gb = (int)gb;
        p.splits = p.gb;  // one per workgroup
        p.Pr = p.Pp = p.chunk = p.waves = 0;
        p.ni = 0;
        p.dz_t_bytes = p.xs_bytes = 0;
        // dW partials, then the bias partials (one per workgroup of a block)
        p.part_bytes = ((size_t)p.splits * cout * 9 * cin + (size_t)p.gb * cout) * 4;
        return p;
    }
    p.nob = p.nib = p.gb = p.tiles = 0;
    // k runs over Pr = P rounded up to whole trips of four 32-pixel k steps.
    // The planes are 1152 pixels (2304 bytes) longer, so that they are not a
    // power of two apart: pixel counts here are powers of two, and the 16
    // planes a fragment load reads at one offset then fell on the same memory
    // channel and cache set (the weight-gradient GEMM ran 10% slower).
    p.Pr = (p.P + 127) / 128 * 128;
    p.Pp = p.Pr + 1152;
    p.ni = cin > 16 ? 2 : 1;
    const long long wtiles = (long long)((cout + 31) / 32) * ((cin + 16 * p.ni - 1) / (16 * p.ni)) * 9;
    long long splits = 4096 / wtiles;  // about 4096 wavefronts in all
    if (splits < 1)
        splits = 1;
    const long long max_splits = p.Pr / 256;  // at least 256 pixels each
    if (splits > max_splits)
        splits = max_splits > 0 ? max_splits : 1;
    long long chunk = (p.Pr + splits - 1) / splits;
    chunk = (chunk + 127) / 128 * 128;
    p.splits = (int)((p.Pr + chunk - 1) / chunk);
    p.chunk = chunk;
    p.waves = wtiles * p.splits;
    // workspace: dz_t (cout x Pp), xs (3 x cin x Pp) BF16, partials FP32
    p.dz_t_bytes = (size_t)cout * p.Pp * 2;
    p.xs_bytes = (size_t)3 * cin * p.Pp * 2;
    // FP32 partials of dW per split; afterwards the bias partials reuse them
    const size_t part_elems = (size_t)p.splits * cout * 9 * cin;
    const size_t bias_elems = (size_t)cout * BIAS_SLICES;
    p.part_bytes = (part_elems > bias_elems ? part_elems : bias_elems) * 4;
    return p;
}

hipError_t launch_wgrad(const void *x, int xp, const void *xu, int xup, int cu, const void *dz,
                        int dzp, int n, int h, int w, int cin, int cout, float *dw, float *db,
                        void *ws, hipStream_t s, hipStream_t sum_s, hipEvent_t ev) {
    const WgradPlan p = wgrad_plan(n, h, w, cin, cout);
    const long long count = (long long)cout * 9 * cin;
    // the sums of the splits go on sum_s once the partials on s are written
    auto hand_over = [&]() -> hipError_t {
        if (sum_s == s)
            return hipSuccess;
        hipError_t e = hipEventRecord(ev, s);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(sum_s, ev, 0);
        return e;
    };
    if (xu && !p.halo)
        return hipErrorNotSupported;  // the upsampled input needs halo tiles
    if (p.halo) {
        float *part = static_cast<float *>(ws);
        WgradHaloArgs a;
        a.x = static_cast<const uint16_t *>(x);
        a.dz = static_cast<const uint16_t *>(dz);
        a.xp = xp;
        a.dzp = dzp;
        a.n = n;
        a.h = h;
        a.w = w;
        a.cin = cin;
        a.cout = cout;
        a.nob = p.nob;
        a.nib = p.nib;
        a.gb = p.gb;
        a.tiles = p.tiles;
        a.tiles_x = p.tiles_x;
        a.tiles_y = p.tiles_y;
        a.part = part;
        a.part_b = part + (long long)p.splits * count;
        a.xu = static_cast<const uint16_t *>(xu);
        a.xup = xu ? xup : 0;
        a.cu = xu ? cu : 0;
        hipLaunchKernelGGL(conv_wgrad_halo_kernel, dim3((unsigned)(p.nob * p.nib * p.gb)),
                           dim3(THREADS), 0, s, a);
        const hipError_t e = hand_over();
        if (e != hipSuccess)
            return e;
        reduce_splits(part, p.splits, count, dw, a.part_b, cout, db, sum_s);
        return hipGetLastError();
    }
    uint16_t *dz_t = static_cast<uint16_t *>(ws);
    uint16_t *xs = reinterpret_cast<uint16_t *>(static_cast<char *>(ws) + align256(p.dz_t_bytes));
    float *part = reinterpret_cast<float *>(static_cast<char *>(ws) + align256(p.dz_t_bytes) +
                                            align256(p.xs_bytes));
    {
        const dim3 tb(THREADS);
        const unsigned qt = (unsigned)((p.Pp + TT - 1) / TT);
        hipLaunchKernelGGL(transpose_kernel, dim3(qt, (unsigned)((cout + TT - 1) / TT)), tb, 0, s,
                           static_cast<const uint16_t *>(dz), dzp, cout, p.P, p.Pp, w, 0, dz_t);
        for (int sh = 0; sh < 3; ++sh)
            hipLaunchKernelGGL(transpose_kernel, dim3(qt, (unsigned)((cin + TT - 1) / TT)), tb, 0,
                               s, static_cast<const uint16_t *>(x), xp, cin, p.P, p.Pp, w, sh - 1,
                               xs + (long long)sh * cin * p.Pp);
    }
    WgradArgs a;
    a.dz_t = dz_t;
    a.xs = xs;
    a.part = part;
    a.n = n;
    a.h = h;
    a.w = w;
    a.cin = cin;
    a.cout = cout;
    a.P = p.P;
    a.Pr = p.Pr;
    a.Pp = p.Pp;
    a.chunk = p.chunk;
    a.splits = p.splits;
    const dim3 grid((unsigned)((p.waves + 3) / 4));
    if (p.ni == 2)
        hipLaunchKernelGGL(conv_wgrad_kernel<2>, grid, dim3(THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(conv_wgrad_kernel<1>, grid, dim3(THREADS), 0, s, a);
    const hipError_t e = hand_over();
    if (e != hipSuccess)
        return e;
    reduce_splits(part, p.splits, count, dw, nullptr, 0, nullptr, sum_s);
    if (db) {
        // the bias partials reuse the start of the (already reduced) partials buffer
        hipLaunchKernelGGL(bias_partial_kernel, dim3((unsigned)cout, BIAS_SLICES), dim3(THREADS), 0,
                           sum_s, dz_t, p.Pp, part);
        hipLaunchKernelGGL(bias_sum_kernel, dim3((unsigned)((cout + THREADS - 1) / THREADS)),
                           dim3(THREADS), 0, sum_s, part, cout, db);
    }
    return hipGetLastError();
}

hipError_t launch_leaky_bwd(const void *dy, int dyp, const void *y, int yp, void *dz, int dzp,
                            long long pixels, int c, float slope, hipStream_t s) {
    hipLaunchKernelGGL(leaky_bwd_kernel, dim3(blocks_for(pixels * (c / 8))), dim3(THREADS), 0, s,
                       static_cast<const uint16_t *>(dy), dyp, static_cast<const uint16_t *>(y),
                       yp, static_cast<uint16_t *>(dz), dzp, pixels, c, slope);
    return hipGetLastError();
}

hipError_t launch_pool2(const void *x, int xp, int n, int h, int w, int c, void *y, int yp,
                        hipStream_t s) {
    hipLaunchKernelGGL(pool2_kernel, dim3(blocks_for((long long)n * (h / 2) * (w / 2) * (c / 8))),
                       dim3(THREADS), 0, s, static_cast<const uint16_t *>(x), xp, n, h, w, c,
                       static_cast<uint16_t *>(y), yp);
    return hipGetLastError();
}

hipError_t launch_pool2_bwd(const void *dy, int dyp, int n, int h, int w, int c, void *dx,
                            int dxp, bool accumulate, const void *mask, int mp, float slope,
                            hipStream_t s) {
    hipLaunchKernelGGL(pool2_bwd_kernel, dim3(blocks_for((long long)n * h * w * (c / 8))),
                       dim3(THREADS), 0, s, static_cast<const uint16_t *>(dy), dyp, n, h, w, c,
                       static_cast<uint16_t *>(dx), dxp, accumulate ? 1 : 0,
                       static_cast<const uint16_t *>(mask), mp, slope);
    return hipGetLastError();
}

hipError_t launch_up2(const void *x, int xp, int n, int h, int w, int c, void *y, int yp,
                      hipStream_t s) {
    hipLaunchKernelGGL(up2_kernel, dim3(blocks_for((long long)n * 4 * h * w * (c / 8))),
                       dim3(THREADS), 0, s, static_cast<const uint16_t *>(x), xp, n, h, w, c,
                       static_cast<uint16_t *>(y), yp);
    return hipGetLastError();
}

hipError_t launch_up2_bwd(const void *dy, int dyp, int n, int h, int w, int c, void *dx, int dxp,
                          const void *mask, int mp, float slope, hipStream_t s) {
    hipLaunchKernelGGL(up2_bwd_kernel, dim3(blocks_for((long long)n * h * w * (c / 8))),
                       dim3(THREADS), 0, s, static_cast<const uint16_t *>(dy), dyp, n, h, w, c,
                       static_cast<uint16_t *>(dx), dxp, static_cast<const uint16_t *>(mask), mp,
                       slope);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float *rho, int batch, int h, int w, const float *planes,
                             const IoScales &sc, void *x, hipStream_t s) {
    hipLaunchKernelGGL(pack_input_kernel, dim3(blocks_for((long long)batch * h * w)),
                       dim3(THREADS), 0, s, rho, batch, h, w, planes, sc,
                       static_cast<uint16_t *>(x));
    return hipGetLastError();
}

hipError_t launch_apply_output(const float *rho, const float *out, int batch, int h, int w,
                               const IoScales &sc, float *next, hipStream_t s) {
    hipLaunchKernelGGL(apply_output_kernel, dim3(blocks_for((long long)batch * h * w * 5)),
                       dim3(THREADS), 0, s, rho, out, batch, h, w, sc, next);
    return hipGetLastError();
}

hipError_t launch_mse(const float *out, const float *rho, const float *target, int batch, int h,
                      int w, const IoScales &sc, void *dout, double *partials, double *loss,
                      hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(SUR_LOSS_BLOCKS), dim3(THREADS), 0, s, out, rho, target,
                       batch, h, w, sc, static_cast<uint16_t *>(dout), partials);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(THREADS), 0, s, partials,
                       SUR_LOSS_BLOCKS, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, void *theta_bf16, const float *grad, float *m, float *v,
                       long long count, const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count)), dim3(THREADS), 0, s, theta,
                       static_cast<uint16_t *>(theta_bf16), grad, m, v, count, a);
    return hipGetLastError();
}

hipError_t launch_crop(const float *rho, int h, int w, int y0, int x0, int ch, int cw, float *dst,
                       hipStream_t s) {
    hipLaunchKernelGGL(crop_kernel, dim3(blocks_for(5ll * ch * cw)), dim3(THREADS), 0, s, rho, h,
                       w, y0 % h, x0 % w, ch, cw, dst);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, void *dst, long long count, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(count)), dim3(THREADS), 0, s, src,
                       static_cast<uint16_t *>(dst), count);
    return hipGetLastError();
}

}  // namespace sslbm
