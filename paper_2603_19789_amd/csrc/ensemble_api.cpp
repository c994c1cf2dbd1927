// ensemble_api.cpp -- host side of the ensemble entry points in sslbm.h:
// validation, the state layout, tile tables, the pass-shape tuner and HIP
// graph capture. Validation and layout queries need no GPU; device tables
// are built on first use.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "ensemble_internal.h"
#include "sslbm.h"
#include "sslbm_internal.h"

namespace {

constexpr int MAX_ENS_SIDE = 1 << 16;
constexpr int MAX_INSTANCES = 1 << 20;
constexpr long long ALIGN_ELEMS = 4;

struct TileTable {
    sslbm::EnsTile *dev = nullptr;
    int count = 0;
};

struct GraphKey {
    long long nsteps;
    void *rho, *scratch;
    int K, H, V;
    bool operator<(const GraphKey &o) const {
        return std::tie(nsteps, rho, scratch, K, H, V) <
               std::tie(o.nsteps, o.rho, o.scratch, o.K, o.H, o.V);
    }
};

}  // namespace

struct sslbm_ensemble {
    int count = 0, dtype = 0, bc = 0;
    std::vector<int> nx, ny;
    std::vector<long long> offset;
    long long elements = 0;
    std::vector<sslbm::StepCoef> coef;
    bool diffuse_d = false;
    bool even_rows = true;  // every nx even (two columns per lane possible)
    sslbm_launch launch{};
    int last_hip = 0;
    int device = -1;
    void *insts = nullptr;                           // device instance table
    std::map<std::tuple<int, int, int>, TileTable> tiles;  // (k, H, V) -> table
    hipStream_t stream = nullptr;                    // graph and tuning stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

namespace {

int hip_status(sslbm_ensemble *e, hipError_t err) {
    if (err == hipSuccess)
        return SSLBM_OK;
    e->last_hip = (int)err;
    return SSLBM_E_HIP;
}

size_t elem_bytes(const sslbm_ensemble *e) { return e->dtype == SSLBM_F32 ? 4 : 8; }

// Tiles of one pass of k steps: every instance cut into strips of
// strip_width(k, V) output columns and chunks of H output rows.
std::vector<sslbm::EnsTile> make_tiles(const sslbm_ensemble *e, int k, int H, int V) {
    std::vector<sslbm::EnsTile> t;
    const int w = sslbm::strip_width(k, V);
    for (int i = 0; i < e->count; ++i)
        for (int y0 = 0; y0 < e->ny[i]; y0 += H)
            for (int x0 = 0; x0 < e->nx[i]; x0 += w)
                t.push_back({i, x0, y0, std::min(y0 + H, e->ny[i]), (y0 / H) & 1});
    return t;
}

long long count_tiles(const sslbm_ensemble *e, int k, int H, int V) {
    const int w = sslbm::strip_width(k, V);
    long long n = 0;
    for (int i = 0; i < e->count; ++i)
        n += (long long)((e->nx[i] + w - 1) / w) * ((e->ny[i] + H - 1) / H);
    return n;
}

int max_rows(const sslbm_ensemble *e) {
    return *std::max_element(e->ny.begin(), e->ny.end());
}

// Columns per lane actually usable: two need every row length even.
int usable_cols(const sslbm_ensemble *e, int V, int k) {
    if (V == 2 && (!e->even_rows || k > sslbm::march_max_depth(e->dtype, 2)))
        return 1;
    return V;
}

// Automatic shape: the single-grid defaults; rows per wavefront the
// smallest for which all tiles of a pass are resident at once.
sslbm_launch resolve(const sslbm_ensemble *e) {
    sslbm_launch r = e->launch;
    if (r.steps_per_pass == 0)
        r.steps_per_pass = e->dtype == SSLBM_F32 ? 6 : 5;
    if (r.cols_per_lane == 0)
        r.cols_per_lane = e->dtype == SSLBM_F32 ? 2 : 1;
    r.cols_per_lane = usable_cols(e, r.cols_per_lane, r.steps_per_pass);
    if (r.rows_per_wave == 0) {
        long long resident =
            sslbm::march_resident_waves(e->dtype, r.steps_per_pass, r.cols_per_lane, e->diffuse_d);
        if (resident <= 0)
            resident = 2 * 4 * 256;
        int lo = 2 * r.steps_per_pass, hi = std::max(lo, max_rows(e));
        while (lo < hi) {  // smallest H with count_tiles(H) <= resident
            const int mid = lo + (hi - lo) / 2;
            if (count_tiles(e, r.steps_per_pass, mid, r.cols_per_lane) <= resident)
                hi = mid;
            else
                lo = mid + 1;
        }
        r.rows_per_wave = lo;
    }
    return r;
}

int ensure_device_tables(sslbm_ensemble *e) {
    int dev = 0;
    int st = hip_status(e, hipGetDevice(&dev));
    if (st != SSLBM_OK)
        return st;
    if (e->insts && e->device == dev)
        return SSLBM_OK;
    if (e->insts)
        return SSLBM_E_UNSUPPORTED;  // an ensemble stays on the device it first ran on
    const size_t rec = sslbm::ensemble_instance_bytes(e->dtype);
    std::vector<unsigned char> host(rec * e->count);
    for (int i = 0; i < e->count; ++i)
        sslbm::ensemble_pack_instance(e->dtype, host.data() + rec * i, e->offset[i], e->nx[i],
                                      e->ny[i], e->coef[i]);
    st = hip_status(e, hipMalloc(&e->insts, host.size()));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(e, hipMemcpy(e->insts, host.data(), host.size(), hipMemcpyHostToDevice));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(e, hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(e, hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(e, hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming));
    if (st != SSLBM_OK)
        return st;
    e->device = dev;
    return SSLBM_OK;
}

int tile_table(sslbm_ensemble *e, int k, int H, int V, TileTable **out) {
    auto key = std::make_tuple(k, H, V);
    auto it = e->tiles.find(key);
    if (it == e->tiles.end()) {
        const std::vector<sslbm::EnsTile> t = make_tiles(e, k, H, V);
        TileTable tab;
        tab.count = (int)t.size();
        int st = hip_status(e, hipMalloc((void **)&tab.dev, sizeof(sslbm::EnsTile) * t.size()));
        if (st != SSLBM_OK)
            return st;
        st = hip_status(e, hipMemcpy(tab.dev, t.data(), sizeof(sslbm::EnsTile) * t.size(),
                                     hipMemcpyHostToDevice));
        if (st != SSLBM_OK) {
            (void)hipFree(tab.dev);
            return st;
        }
        it = e->tiles.emplace(key, tab).first;
    }
    *out = &it->second;
    return SSLBM_OK;
}

// Enqueue the passes of nsteps steps on stream s (tables must exist).
int enqueue_run(sslbm_ensemble *e, const sslbm_launch &r, void *rho, void *scratch,
                long long nsteps, hipStream_t s) {
    void *src = rho, *dst = scratch;
    const sslbm::PassPlan plan = sslbm::plan_passes(nsteps, r.steps_per_pass);
    for (long long i = 0; i < plan.count; ++i) {
        const int k = plan.steps(i);
        const int V = usable_cols(e, r.cols_per_lane, k);
        TileTable *tab = nullptr;
        int st = tile_table(e, k, r.rows_per_wave, V, &tab);
        if (st != SSLBM_OK)
            return st;
        st = hip_status(e, sslbm::launch_ensemble(e->dtype, src, dst, tab->dev, tab->count,
                                                  e->insts, e->bc, k, V, e->diffuse_d, s));
        if (st != SSLBM_OK)
            return st;
        std::swap(src, dst);
    }
    if (src != rho)
        return hip_status(e, hipMemcpyAsync(rho, src, elem_bytes(e) * e->elements,
                                            hipMemcpyDeviceToDevice, s));
    return SSLBM_OK;
}

// Build every tile table a run of nsteps will use (before any capture).
int prepare_run(sslbm_ensemble *e, const sslbm_launch &r, long long nsteps) {
    const sslbm::PassPlan plan = sslbm::plan_passes(nsteps, r.steps_per_pass);
    // a run uses at most two depths: the longer and the shorter passes
    for (long long i : {0ll, plan.count - 1}) {
        if (i < 0)
            continue;
        const int k = plan.steps(i);
        TileTable *tab = nullptr;
        const int st = tile_table(e, k, r.rows_per_wave, usable_cols(e, r.cols_per_lane, k), &tab);
        if (st != SSLBM_OK)
            return st;
    }
    return SSLBM_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

int sslbm_ensemble_create(sslbm_ensemble **out, int count, const int *nx, const int *ny,
                          int dtype, int bc, const sslbm_params *params, int *bad_instance) {
    if (bad_instance)
        *bad_instance = -1;
    if (!out || !nx || !ny || !params || count < 1 || count > MAX_INSTANCES)
        return SSLBM_E_ARG;
    *out = nullptr;
    if (dtype != SSLBM_F32 && dtype != SSLBM_F64)
        return SSLBM_E_ARG;
    if (bc != SSLBM_PERIODIC && bc != SSLBM_NOFLUX)
        return SSLBM_E_ARG;
    sslbm_ensemble *e = new (std::nothrow) sslbm_ensemble();
    if (!e)
        return SSLBM_E_NOMEM;
    e->count = count;
    e->dtype = dtype;
    e->bc = bc;
    long long off = 0;
    for (int i = 0; i < count; ++i) {
        sslbm::StepCoef k;
        int st = SSLBM_OK;
        if (nx[i] < 1 || ny[i] < 1 || nx[i] > MAX_ENS_SIDE || ny[i] > MAX_ENS_SIDE)
            st = SSLBM_E_ARG;
        else
            st = sslbm::derive_coef(&params[i], &k);
        if (st != SSLBM_OK) {
            if (bad_instance)
                *bad_instance = i;
            delete e;
            return st;
        }
        e->nx.push_back(nx[i]);
        e->ny.push_back(ny[i]);
        e->coef.push_back(k);
        e->offset.push_back(off);
        e->diffuse_d = e->diffuse_d || k.diffuse_d;
        e->even_rows = e->even_rows && nx[i] % 2 == 0;
        off += (5ll * nx[i] * ny[i] + ALIGN_ELEMS - 1) / ALIGN_ELEMS * ALIGN_ELEMS;
    }
    e->elements = off;
    *out = e;
    return SSLBM_OK;
}

long long sslbm_ensemble_offset(const sslbm_ensemble *e, int instance) {
    if (!e || instance < 0 || instance >= e->count)
        return -1;
    return e->offset[instance];
}

long long sslbm_ensemble_elements(const sslbm_ensemble *e) { return e ? e->elements : -1; }

int sslbm_ensemble_set_launch(sslbm_ensemble *e, const sslbm_launch *shape) {
    if (!e || !shape)
        return SSLBM_E_ARG;
    const sslbm_launch &r = *shape;
    if (r.steps_per_pass < 0 || r.steps_per_pass > SSLBM_MAX_BLOCKING || r.rows_per_wave < 0 ||
        r.rows_per_wave > 65536 || r.cols_per_lane < 0 || r.cols_per_lane > 2)
        return SSLBM_E_ARG;
    const int K = r.steps_per_pass ? r.steps_per_pass : (e->dtype == SSLBM_F32 ? 6 : 5);
    if (K > sslbm::march_max_depth(e->dtype, 1) ||
        (r.cols_per_lane == 2 && K > sslbm::march_max_depth(e->dtype, 2)))
        return SSLBM_E_UNSUPPORTED;
    e->launch = r;
    return SSLBM_OK;
}

int sslbm_ensemble_get_launch(const sslbm_ensemble *e, sslbm_launch *shape) {
    if (!e || !shape)
        return SSLBM_E_ARG;
    *shape = resolve(e);
    return SSLBM_OK;
}

int sslbm_ensemble_run(sslbm_ensemble *e, void *rho, void *scratch, long long nsteps, int flags,
                       void *hip_stream) {
    if (!e || !rho || !scratch || nsteps < 0 || (flags & ~SSLBM_RUN_GRAPH))
        return SSLBM_E_ARG;
    const size_t bytes = elem_bytes(e) * e->elements;
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    if (nsteps == 0)
        return SSLBM_OK;
    // two columns per lane read aligned element pairs
    sslbm_launch r = resolve(e);
    const uintptr_t pair = 2 * elem_bytes(e);
    if ((uintptr_t)rho % pair || (uintptr_t)scratch % pair)
        r.cols_per_lane = 1;
    int st = ensure_device_tables(e);
    if (st != SSLBM_OK)
        return st;
    st = prepare_run(e, r, nsteps);
    if (st != SSLBM_OK)
        return st;
    const hipStream_t user = (hipStream_t)hip_stream;
    if (!(flags & SSLBM_RUN_GRAPH))
        return enqueue_run(e, r, rho, scratch, nsteps, user);

    const GraphKey key{nsteps, rho, scratch, r.steps_per_pass, r.rows_per_wave, r.cols_per_lane};
    auto it = e->graphs.find(key);
    if (it == e->graphs.end()) {
        st = hip_status(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        if (st != SSLBM_OK)
            return st;
        const int run_st = enqueue_run(e, r, rho, scratch, nsteps, e->stream);
        hipGraph_t graph = nullptr;
        const hipError_t end = hipStreamEndCapture(e->stream, &graph);
        if (run_st != SSLBM_OK) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return run_st;
        }
        st = hip_status(e, end);
        if (st != SSLBM_OK)
            return st;
        hipGraphExec_t exec = nullptr;
        st = hip_status(e, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        if (st != SSLBM_OK)
            return st;
        it = e->graphs.emplace(key, exec).first;
    }
    // order the graph after the caller's prior work and the caller's later
    // work after the graph
    st = hip_status(e, hipEventRecord(e->ev_in, user));
    if (st == SSLBM_OK)
        st = hip_status(e, hipStreamWaitEvent(e->stream, e->ev_in, 0));
    if (st == SSLBM_OK)
        st = hip_status(e, hipGraphLaunch(it->second, e->stream));
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventRecord(e->ev_out, e->stream));
    if (st == SSLBM_OK)
        st = hip_status(e, hipStreamWaitEvent(user, e->ev_out, 0));
    return st;
}

int sslbm_ensemble_tune(sslbm_ensemble *e, const void *rho, void *scratch, void *hip_stream,
                        sslbm_launch *best) {
    if (!e || !rho || !scratch)
        return SSLBM_E_ARG;
    const size_t bytes = elem_bytes(e) * e->elements;
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    int st = ensure_device_tables(e);
    if (st != SSLBM_OK)
        return st;
    const hipStream_t user = (hipStream_t)hip_stream;
    st = hip_status(e, hipStreamSynchronize(user));
    if (st != SSLBM_OK)
        return st;
    hipEvent_t t0, t1;
    st = hip_status(e, hipEventCreate(&t0));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(e, hipEventCreate(&t1));
    if (st != SSLBM_OK) {
        (void)hipEventDestroy(t0);
        return st;
    }
    const uintptr_t pair = 2 * elem_bytes(e);
    const bool pairs_ok = e->even_rows && !((uintptr_t)rho % pair) && !((uintptr_t)scratch % pair);
    long long cells = 0;
    for (int i = 0; i < e->count; ++i)
        cells += (long long)e->nx[i] * e->ny[i];

    double best_ns = 1e300;
    sslbm_launch best_shape = resolve(e);
    const sslbm_launch saved = e->launch;
    for (int V = 1; V <= (pairs_ok ? 2 : 1) && st == SSLBM_OK; ++V) {
        for (int K = 2; K <= sslbm::march_max_depth(e->dtype, V) && st == SSLBM_OK; ++K) {
            // candidate heights: one round of resident wavefronts, and fixed ones
            e->launch = sslbm_launch{K, 0, V};
            const int h_round = resolve(e).rows_per_wave;
            const int cands[] = {h_round, 16, 32, 64, 128};
            for (int H : cands) {
                if (H < 2 * K && H != h_round)
                    continue;
                TileTable *tab = nullptr;
                st = tile_table(e, K, H, V, &tab);
                if (st != SSLBM_OK)
                    break;
                // one untimed pass, then three timed ones, all rho -> scratch
                for (int rep = 0; rep < 4 && st == SSLBM_OK; ++rep) {
                    if (rep == 1)
                        st = hip_status(e, hipEventRecord(t0, e->stream));
                    if (st == SSLBM_OK)
                        st = hip_status(e, sslbm::launch_ensemble(e->dtype, rho, scratch, tab->dev,
                                                                  tab->count, e->insts, e->bc, K,
                                                                  V, e->diffuse_d, e->stream));
                }
                if (st == SSLBM_OK)
                    st = hip_status(e, hipEventRecord(t1, e->stream));
                if (st == SSLBM_OK)
                    st = hip_status(e, hipEventSynchronize(t1));
                float ms = 0.f;
                if (st == SSLBM_OK)
                    st = hip_status(e, hipEventElapsedTime(&ms, t0, t1));
                if (st != SSLBM_OK)
                    break;
                const double ns_per_update = ms * 1e6 / (3.0 * K * (double)cells);
                if (ns_per_update < best_ns) {
                    best_ns = ns_per_update;
                    best_shape = sslbm_launch{K, H, V};
                }
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    e->launch = st == SSLBM_OK ? best_shape : saved;
    if (st == SSLBM_OK && best)
        *best = best_shape;
    return st;
}

int sslbm_ensemble_last_hip_error(const sslbm_ensemble *e) { return e ? e->last_hip : 0; }

void sslbm_ensemble_destroy(sslbm_ensemble *e) {
    if (!e)
        return;
    for (auto &g : e->graphs)
        (void)hipGraphExecDestroy(g.second);
    for (auto &t : e->tiles)
        (void)hipFree(t.second.dev);
    if (e->insts)
        (void)hipFree(e->insts);
    if (e->ev_in)
        (void)hipEventDestroy(e->ev_in);
    if (e->ev_out)
        (void)hipEventDestroy(e->ev_out);
    if (e->stream)
        (void)hipStreamDestroy(e->stream);
    delete e;
}

}  // extern "C"
