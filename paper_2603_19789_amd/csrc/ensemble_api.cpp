// ensemble_api.cpp -- host side of the ensemble entry points in sslbm.h:
// validation, the state layout, size classes, tile tables, the per-class
// pass-shape tuner and HIP graph capture. Validation and layout queries need
// no GPU; device tables are built on first use.
//
// Size classes. Instances are grouped at creation:
//  * on chip: the five fields fit ENS_LDS_BYTES of LDS (64 x 64 in FP32).
//    One launch of the LDS-resident kernel advances all of them by every
//    step of a run (one workgroup per instance, read and written once).
//  * march classes, one per power-of-two bucket of the longest side (up to
//    2, 4, ..., 512, 1024, ...): passes of the tile-table kernel with a pass
//    shape (steps per pass, rows per wavefront, columns per lane) of their
//    own, automatic or tuned per class.
// A run gives every class its own chain of launches on its own stream,
// forked from and joined back to the caller's stream (or captured as
// parallel branches of one HIP graph): classes never wait for each other,
// only for their own previous pass.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
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
    bool operator<(const GraphKey &o) const {
        return std::tie(nsteps, rho, scratch) < std::tie(o.nsteps, o.rho, o.scratch);
    }
};

struct EnsClass {
    bool on_chip = false;
    int bucket = 0;  // march classes: longest side in (2^(bucket-1), 2^bucket]
    std::vector<int> insts;
    long long cells = 0;
    int max_side = 0;
    bool even_rows = true;  // every row length even (two columns per lane possible)
    sslbm_launch launch{};  // requested pass shape, zero fields automatic
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace

struct sslbm_ensemble {
    int count = 0, dtype = 0, bc = 0;
    std::vector<int> nx, ny;
    std::vector<long long> offset;
    long long elements = 0;
    std::vector<sslbm::StepCoef> coef;
    bool diffuse_d = false;
    std::vector<EnsClass> classes;  // march classes by bucket, then the on-chip class
    std::vector<int> class_of;      // class of every instance
    long long march_cells = 0;
    size_t lds_bytes = 0;  // the largest on-chip instance
    int last_hip = 0;
    int device = -1;
    void *insts = nullptr;    // device instance table
    int *lds_list = nullptr;  // device list of the on-chip instances
    std::map<std::tuple<int, int, int, int>, TileTable> tiles;  // (class, k, H, V) -> table
    hipStream_t stream = nullptr;  // graph and tuning stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

namespace {

sslbm_status hip_status(sslbm_ensemble *e, hipError_t err) {
    if (err == hipSuccess)
        return SSLBM_OK;
    e->last_hip = (int)err;
    return SSLBM_E_HIP;
}

size_t elem_bytes(const sslbm_ensemble *e) { return e->dtype == SSLBM_F32 ? 4 : 8; }

bool valid_class(const sslbm_ensemble *e, int c) {
    return c >= 0 && c < (int)e->classes.size();
}

// Tiles of one pass of k steps of class c: every instance of the class cut
// into strips of strip_width(k, V) output columns and chunks of H output rows.
std::vector<sslbm::EnsTile> make_tiles(const sslbm_ensemble *e, int c, int k, int H, int V) {
    std::vector<sslbm::EnsTile> t;
    const int w = sslbm::strip_width(k, V);
    for (int i : e->classes[c].insts)
        for (int y0 = 0; y0 < e->ny[i]; y0 += H)
            for (int x0 = 0; x0 < e->nx[i]; x0 += w)
                t.push_back({i, x0, y0, std::min(y0 + H, e->ny[i]), (y0 / H) & 1});
    return t;
}

long long count_tiles(const sslbm_ensemble *e, int c, int k, int H, int V) {
    const int w = sslbm::strip_width(k, V);
    long long n = 0;
    for (int i : e->classes[c].insts)
        n += (long long)((e->nx[i] + w - 1) / w) * ((e->ny[i] + H - 1) / H);
    return n;
}

// Columns per lane actually usable: two need every row length of the class
// even, pair-aligned buffers and a depth within the two-column register budget.
int usable_cols(const sslbm_ensemble *e, int c, int V, int k, bool pairs_ok) {
    if (V == 2 && (!pairs_ok || !e->classes[c].even_rows ||
                   k > sslbm::march_max_depth(e->dtype, 2)))
        return 1;
    return V;
}

// Pass shape of march class c: requested fields, automatic ones filled in.
// Automatic: the single-grid depth; two columns per lane where the longest
// side exceeds one two-column strip (narrower grids waste most of it); rows
// per wavefront the fewest for which the class's tiles fit its share of the
// resident wavefronts (its share of the march cells, since the classes run
// side by side).
sslbm_launch resolve(const sslbm_ensemble *e, int c, bool pairs_ok = true) {
    const EnsClass &cl = e->classes[c];
    sslbm_launch r = cl.launch;
    if (r.steps_per_pass == 0)
        r.steps_per_pass = e->dtype == SSLBM_F32 ? 6 : 5;
    if (r.cols_per_lane == 0)
        r.cols_per_lane =
            e->dtype == SSLBM_F32 && cl.max_side > sslbm::strip_width(r.steps_per_pass, 2) ? 2
                                                                                           : 1;
    r.cols_per_lane = usable_cols(e, c, r.cols_per_lane, r.steps_per_pass, pairs_ok);
    if (r.rows_per_wave == 0) {
        long long resident =
            sslbm::march_resident_waves(e->dtype, r.steps_per_pass, r.cols_per_lane, e->diffuse_d);
        if (resident <= 0)
            resident = 2 * 4 * 256;
        const double share = e->march_cells > 0 ? (double)cl.cells / (double)e->march_cells : 1.0;
        const long long target = std::max(64ll, (long long)(share * (double)resident));
        int lo = 2 * r.steps_per_pass, hi = std::max(lo, cl.max_side);
        while (lo < hi) {  // smallest H with count_tiles(H) <= target
            const int mid = lo + (hi - lo) / 2;
            if (count_tiles(e, c, r.steps_per_pass, mid, r.cols_per_lane) <= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        r.rows_per_wave = lo;
    }
    return r;
}

// The march class with the most cells (-1 if none).
int main_class(const sslbm_ensemble *e) {
    int best = -1;
    for (int c = 0; c < (int)e->classes.size(); ++c)
        if (!e->classes[c].on_chip && (best < 0 || e->classes[c].cells > e->classes[best].cells))
            best = c;
    return best;
}

void drop_graphs(sslbm_ensemble *e) {
    for (auto &g : e->graphs)
        (void)hipGraphExecDestroy(g.second);
    e->graphs.clear();
}

sslbm_status ensure_device_tables(sslbm_ensemble *e) {
    int dev = 0;
    sslbm_status st = hip_status(e, hipGetDevice(&dev));
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
    for (const EnsClass &cl : e->classes) {
        if (!cl.on_chip)
            continue;
        st = hip_status(e, hipMalloc((void **)&e->lds_list, sizeof(int) * cl.insts.size()));
        if (st != SSLBM_OK)
            return st;
        st = hip_status(e, hipMemcpy(e->lds_list, cl.insts.data(), sizeof(int) * cl.insts.size(),
                                     hipMemcpyHostToDevice));
        if (st != SSLBM_OK)
            return st;
    }
    st = hip_status(e, hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming));
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming));
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventCreateWithFlags(&e->ev_fork, hipEventDisableTiming));
    for (EnsClass &cl : e->classes) {
        if (st == SSLBM_OK)
            st = hip_status(e, hipStreamCreateWithFlags(&cl.stream, hipStreamNonBlocking));
        if (st == SSLBM_OK)
            st = hip_status(e, hipEventCreateWithFlags(&cl.done, hipEventDisableTiming));
    }
    if (st != SSLBM_OK)
        return st;
    e->device = dev;
    return SSLBM_OK;
}

sslbm_status tile_table(sslbm_ensemble *e, int c, int k, int H, int V, TileTable **out) {
    auto key = std::make_tuple(c, k, H, V);
    auto it = e->tiles.find(key);
    if (it == e->tiles.end()) {
        const std::vector<sslbm::EnsTile> t = make_tiles(e, c, k, H, V);
        TileTable tab;
        tab.count = (int)t.size();
        sslbm_status st =
            hip_status(e, hipMalloc((void **)&tab.dev, sizeof(sslbm::EnsTile) * t.size()));
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

// Enqueue nsteps steps of class c on stream s (tables must exist).
sslbm_status enqueue_class(sslbm_ensemble *e, int c, void *rho, void *scratch, long long nsteps,
                           bool pairs_ok, hipStream_t s) {
    const EnsClass &cl = e->classes[c];
    if (cl.on_chip)
        return hip_status(e, sslbm::launch_ensemble_lds(
                                 e->dtype, rho, e->lds_list, (int)cl.insts.size(), e->insts,
                                 e->bc, nsteps, e->diffuse_d, e->lds_bytes, s));
    const sslbm_launch r = resolve(e, c, pairs_ok);
    void *src = rho, *dst = scratch;
    const sslbm::PassPlan plan = sslbm::plan_passes(nsteps, r.steps_per_pass);
    for (long long i = 0; i < plan.count; ++i) {
        const int k = plan.steps(i);
        const int V = usable_cols(e, c, r.cols_per_lane, k, pairs_ok);
        TileTable *tab = nullptr;
        sslbm_status st = tile_table(e, c, k, r.rows_per_wave, V, &tab);
        if (st != SSLBM_OK)
            return st;
        st = hip_status(e, sslbm::launch_ensemble(e->dtype, src, dst, tab->dev, tab->count,
                                                  e->insts, e->bc, k, V, e->diffuse_d, s));
        if (st != SSLBM_OK)
            return st;
        std::swap(src, dst);
    }
    if (src != rho) {  // an odd number of passes: copy the class's instances back
        const size_t eb = elem_bytes(e);
        for (int i : cl.insts) {
            const size_t off = (size_t)e->offset[i] * eb;
            const sslbm_status st = hip_status(
                e, hipMemcpyAsync(static_cast<char *>(rho) + off, static_cast<char *>(src) + off,
                                  5 * (size_t)e->nx[i] * e->ny[i] * eb, hipMemcpyDeviceToDevice,
                                  s));
            if (st != SSLBM_OK)
                return st;
        }
    }
    return SSLBM_OK;
}

// Every class on its own stream, forked from and joined back to s.
sslbm_status enqueue_run(sslbm_ensemble *e, void *rho, void *scratch, long long nsteps,
                         bool pairs_ok, hipStream_t s) {
    if (e->classes.size() == 1)
        return enqueue_class(e, 0, rho, scratch, nsteps, pairs_ok, s);
    sslbm_status st = hip_status(e, hipEventRecord(e->ev_fork, s));
    for (size_t c = 0; c < e->classes.size() && st == SSLBM_OK; ++c) {
        EnsClass &cl = e->classes[c];
        st = hip_status(e, hipStreamWaitEvent(cl.stream, e->ev_fork, 0));
        if (st == SSLBM_OK)
            st = enqueue_class(e, (int)c, rho, scratch, nsteps, pairs_ok, cl.stream);
        if (st == SSLBM_OK)
            st = hip_status(e, hipEventRecord(cl.done, cl.stream));
        if (st == SSLBM_OK)
            st = hip_status(e, hipStreamWaitEvent(s, cl.done, 0));
    }
    return st;
}

// Build every tile table a run of nsteps will use (before any capture): a
// class's run uses at most two depths, the longer and the shorter passes.
sslbm_status prepare_run(sslbm_ensemble *e, long long nsteps, bool pairs_ok) {
    for (int c = 0; c < (int)e->classes.size(); ++c) {
        if (e->classes[c].on_chip)
            continue;
        const sslbm_launch r = resolve(e, c, pairs_ok);
        const sslbm::PassPlan plan = sslbm::plan_passes(nsteps, r.steps_per_pass);
        for (long long i : {0ll, plan.count - 1}) {
            if (i < 0)
                continue;
            const int k = plan.steps(i);
            TileTable *tab = nullptr;
            const sslbm_status st = tile_table(e, c, k, r.rows_per_wave,
                                      usable_cols(e, c, r.cols_per_lane, k, pairs_ok), &tab);
            if (st != SSLBM_OK)
                return st;
        }
    }
    return SSLBM_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

bool pairs_aligned(const sslbm_ensemble *e, const void *rho, const void *scratch) {
    const uintptr_t pair = 2 * elem_bytes(e);
    return !((uintptr_t)rho % pair) && !((uintptr_t)scratch % pair);
}

sslbm_status check_shape(const sslbm_ensemble *e, const sslbm_launch &r) {
    if (r.steps_per_pass < 0 || r.steps_per_pass > SSLBM_MAX_BLOCKING || r.rows_per_wave < 0 ||
        r.rows_per_wave > 65536 || r.cols_per_lane < 0 || r.cols_per_lane > 2)
        return SSLBM_E_ARG;
    const int K = r.steps_per_pass ? r.steps_per_pass : (e->dtype == SSLBM_F32 ? 6 : 5);
    if (K > sslbm::march_max_depth(e->dtype, 1) ||
        (r.cols_per_lane == 2 && K > sslbm::march_max_depth(e->dtype, 2)))
        return SSLBM_E_UNSUPPORTED;
    return SSLBM_OK;
}

// One pass of every march class side by side (each on its own stream,
// forked from and joined back to the ensemble's stream), rho -> scratch, with
// the classes' current shapes: one untimed round, then three timed ones.
// Returns the joint rate in cell-updates per nanosecond (0 on error).
double joint_rate(sslbm_ensemble *e, const void *rho, void *scratch, bool pairs_ok,
                  hipEvent_t t0, hipEvent_t t1, sslbm_status *status) {
    sslbm_status st = SSLBM_OK;
    double work = 0.0;  // cell-updates of one round
    for (int rep = 0; rep < 4 && st == SSLBM_OK; ++rep) {
        if (rep == 1)
            st = hip_status(e, hipEventRecord(t0, e->stream));
        if (st == SSLBM_OK)
            st = hip_status(e, hipEventRecord(e->ev_fork, e->stream));
        for (int c = 0; c < (int)e->classes.size() && st == SSLBM_OK; ++c) {
            EnsClass &cl = e->classes[c];
            if (cl.on_chip)
                continue;
            const sslbm_launch r = resolve(e, c, pairs_ok);
            TileTable *tab = nullptr;
            st = tile_table(e, c, r.steps_per_pass, r.rows_per_wave, r.cols_per_lane, &tab);
            if (st == SSLBM_OK)
                st = hip_status(e, hipStreamWaitEvent(cl.stream, e->ev_fork, 0));
            if (st == SSLBM_OK)
                st = hip_status(e, sslbm::launch_ensemble(e->dtype, rho, scratch, tab->dev,
                                                          tab->count, e->insts, e->bc,
                                                          r.steps_per_pass, r.cols_per_lane,
                                                          e->diffuse_d, cl.stream));
            if (st == SSLBM_OK)
                st = hip_status(e, hipEventRecord(cl.done, cl.stream));
            if (st == SSLBM_OK)
                st = hip_status(e, hipStreamWaitEvent(e->stream, cl.done, 0));
            if (rep == 0)
                work += (double)cl.cells * r.steps_per_pass;
        }
    }
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventRecord(t1, e->stream));
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventSynchronize(t1));
    float ms = 0.f;
    if (st == SSLBM_OK)
        st = hip_status(e, hipEventElapsedTime(&ms, t0, t1));
    *status = st;
    return st == SSLBM_OK && ms > 0.f ? 3.0 * work / (ms * 1e6) : 0.0;
}

// Candidate shapes of a march class: every depth and column count within
// the register budget, rows per wavefront automatic or 8 .. 128.
std::vector<sslbm_launch> candidates(const sslbm_ensemble *e, int c, bool pairs_ok) {
    std::vector<sslbm_launch> out;
    const EnsClass &cl = e->classes[c];
    for (int V = 1; V <= (pairs_ok && cl.even_rows ? 2 : 1); ++V)
        for (int K = 1; K <= sslbm::march_max_depth(e->dtype, V); ++K)
            for (int H : {0, 8, 16, 32, 64, 128})
                if (H == 0 || (H >= 2 * K && H <= cl.max_side))
                    out.push_back(sslbm_launch{K, H, V});
    return out;
}

// The tuner: first one shape for every march class (the best joint rate),
// then each class in turn, largest first, tries its candidates while the
// others keep theirs, and keeps whichever raises the joint rate.
sslbm_status tune_classes(sslbm_ensemble *e, const void *rho, void *scratch, bool pairs_ok,
                          hipEvent_t t0, hipEvent_t t1) {
    std::vector<int> march;
    for (int c = 0; c < (int)e->classes.size(); ++c)
        if (!e->classes[c].on_chip)
            march.push_back(c);
    if (march.empty())
        return SSLBM_OK;
    std::sort(march.begin(), march.end(),
              [&](int a, int b) { return e->classes[a].cells > e->classes[b].cells; });
    sslbm_status st = SSLBM_OK;
    double best = -1.0;
    sslbm_launch common{};
    for (const sslbm_launch &cand : candidates(e, march[0], pairs_ok)) {
        for (int c : march)
            e->classes[c].launch = cand;
        const double rate = joint_rate(e, rho, scratch, pairs_ok, t0, t1, &st);
        if (st != SSLBM_OK)
            return st;
        if (rate > best) {
            best = rate;
            common = cand;
        }
    }
    for (int c : march)
        e->classes[c].launch = common;
    if (march.size() == 1)
        return SSLBM_OK;
    for (int c : march) {
        sslbm_launch keep = e->classes[c].launch;
        for (const sslbm_launch &cand : candidates(e, c, pairs_ok)) {
            e->classes[c].launch = cand;
            const double rate = joint_rate(e, rho, scratch, pairs_ok, t0, t1, &st);
            if (st != SSLBM_OK)
                return st;
            if (rate > best) {
                best = rate;
                keep = cand;
            }
        }
        e->classes[c].launch = keep;
    }
    return SSLBM_OK;
}

}  // namespace

extern "C" {

sslbm_status sslbm_ensemble_create(sslbm_ensemble **out, int count, const int *nx, const int *ny,
                                   int dtype, int bc, const sslbm_params *params,
                                   int *bad_instance) {
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
        sslbm_status st = SSLBM_OK;
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
        off += (5ll * nx[i] * ny[i] + ALIGN_ELEMS - 1) / ALIGN_ELEMS * ALIGN_ELEMS;
    }
    e->elements = off;

    // size classes: on chip, else by the power-of-two bucket of the longest side
    const size_t eb = elem_bytes(e);
    std::map<int, int> bucket_class;
    std::vector<int> on_chip;
    for (int i = 0; i < count; ++i) {
        const size_t bytes = 5 * (size_t)nx[i] * ny[i] * eb;
        if (bytes <= (size_t)sslbm::ENS_LDS_BYTES) {
            on_chip.push_back(i);
            e->lds_bytes = std::max(e->lds_bytes, bytes);
            continue;
        }
        const int side = std::max(nx[i], ny[i]);
        int b = 0;
        while ((1 << b) < side)
            ++b;
        bucket_class[b] = 0;
    }
    for (auto &bc_pair : bucket_class) {
        bc_pair.second = (int)e->classes.size();
        EnsClass cl;
        cl.bucket = bc_pair.first;
        e->classes.push_back(cl);
    }
    if (!on_chip.empty()) {
        EnsClass cl;
        cl.on_chip = true;
        e->classes.push_back(cl);
    }
    e->class_of.assign(count, -1);
    for (int i = 0; i < count; ++i) {
        int c;
        if (5 * (size_t)nx[i] * ny[i] * eb <= (size_t)sslbm::ENS_LDS_BYTES) {
            c = (int)e->classes.size() - 1;
        } else {
            const int side = std::max(nx[i], ny[i]);
            int b = 0;
            while ((1 << b) < side)
                ++b;
            c = bucket_class[b];
        }
        EnsClass &cl = e->classes[c];
        e->class_of[i] = c;
        cl.insts.push_back(i);
        cl.cells += (long long)nx[i] * ny[i];
        cl.max_side = std::max(cl.max_side, std::max(nx[i], ny[i]));
        cl.even_rows = cl.even_rows && nx[i] % 2 == 0;
        if (!cl.on_chip)
            e->march_cells += (long long)nx[i] * ny[i];
    }
    *out = e;
    return SSLBM_OK;
}

long long sslbm_ensemble_offset(const sslbm_ensemble *e, int instance) {
    if (!e || instance < 0 || instance >= e->count)
        return -1;
    return e->offset[instance];
}

long long sslbm_ensemble_elements(const sslbm_ensemble *e) { return e ? e->elements : -1; }

int sslbm_ensemble_class_count(const sslbm_ensemble *e) {
    return e ? (int)e->classes.size() : SSLBM_E_ARG;
}

int sslbm_ensemble_instance_class(const sslbm_ensemble *e, int instance) {
    if (!e || instance < 0 || instance >= e->count)
        return SSLBM_E_ARG;
    return e->class_of[instance];
}

sslbm_status sslbm_ensemble_class_info(const sslbm_ensemble *e, int cls,
                                       sslbm_ensemble_class *info) {
    if (!e || !info || !valid_class(e, cls))
        return SSLBM_E_ARG;
    const EnsClass &cl = e->classes[cls];
    info->on_chip = cl.on_chip ? 1 : 0;
    info->instances = (int)cl.insts.size();
    info->cells = cl.cells;
    info->max_side = cl.max_side;
    info->launch = cl.on_chip ? sslbm_launch{0, 0, 0} : resolve(e, cls);
    return SSLBM_OK;
}

sslbm_status sslbm_ensemble_set_class_launch(sslbm_ensemble *e, int cls,
                                             const sslbm_launch *shape) {
    if (!e || !shape || !valid_class(e, cls))
        return SSLBM_E_ARG;
    const sslbm_status st = check_shape(e, *shape);
    if (st != SSLBM_OK)
        return st;
    if (e->classes[cls].on_chip)
        return SSLBM_E_UNSUPPORTED;
    e->classes[cls].launch = *shape;
    drop_graphs(e);
    return SSLBM_OK;
}

sslbm_status sslbm_ensemble_set_launch(sslbm_ensemble *e, const sslbm_launch *shape) {
    if (!e || !shape)
        return SSLBM_E_ARG;
    const sslbm_status st = check_shape(e, *shape);
    if (st != SSLBM_OK)
        return st;
    for (EnsClass &cl : e->classes)
        if (!cl.on_chip)
            cl.launch = *shape;
    drop_graphs(e);
    return SSLBM_OK;
}

sslbm_status sslbm_ensemble_get_launch(const sslbm_ensemble *e, sslbm_launch *shape) {
    if (!e || !shape)
        return SSLBM_E_ARG;
    const int c = main_class(e);
    *shape = c < 0 ? sslbm_launch{0, 0, 0} : resolve(e, c);
    return SSLBM_OK;
}

static sslbm_status run_checks(sslbm_ensemble *e, void *rho, void *scratch, long long nsteps) {
    if (!e || !rho || !scratch || nsteps < 0)
        return SSLBM_E_ARG;
    const size_t bytes = elem_bytes(e) * e->elements;
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    return SSLBM_OK;
}

sslbm_status sslbm_ensemble_run_class(sslbm_ensemble *e, int cls, void *rho, void *scratch,
                                      long long nsteps, void *hip_stream) {
    sslbm_status st = run_checks(e, rho, scratch, nsteps);
    if (st != SSLBM_OK)
        return st;
    if (!valid_class(e, cls))
        return SSLBM_E_ARG;
    if (nsteps == 0)
        return SSLBM_OK;
    const bool pairs_ok = pairs_aligned(e, rho, scratch);
    st = ensure_device_tables(e);
    if (st == SSLBM_OK)
        st = prepare_run(e, nsteps, pairs_ok);
    if (st != SSLBM_OK)
        return st;
    return enqueue_class(e, cls, rho, scratch, nsteps, pairs_ok, (hipStream_t)hip_stream);
}

sslbm_status sslbm_ensemble_run(sslbm_ensemble *e, void *rho, void *scratch, long long nsteps,
                                int flags, void *hip_stream) {
    sslbm_status st = run_checks(e, rho, scratch, nsteps);
    if (st != SSLBM_OK)
        return st;
    if (flags & ~SSLBM_RUN_GRAPH)
        return SSLBM_E_ARG;
    if (nsteps == 0)
        return SSLBM_OK;
    const bool pairs_ok = pairs_aligned(e, rho, scratch);
    st = ensure_device_tables(e);
    if (st != SSLBM_OK)
        return st;
    st = prepare_run(e, nsteps, pairs_ok);
    if (st != SSLBM_OK)
        return st;
    const hipStream_t user = (hipStream_t)hip_stream;
    if (!(flags & SSLBM_RUN_GRAPH))
        return enqueue_run(e, rho, scratch, nsteps, pairs_ok, user);

    const GraphKey key{nsteps, rho, scratch};
    auto it = e->graphs.find(key);
    if (it == e->graphs.end()) {
        st = hip_status(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        if (st != SSLBM_OK)
            return st;
        const sslbm_status run_st = enqueue_run(e, rho, scratch, nsteps, pairs_ok, e->stream);
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

sslbm_status sslbm_ensemble_tune(sslbm_ensemble *e, const void *rho, void *scratch,
                                 void *hip_stream, sslbm_launch *best) {
    if (!e || !rho || !scratch)
        return SSLBM_E_ARG;
    const size_t bytes = elem_bytes(e) * e->elements;
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    sslbm_status st = ensure_device_tables(e);
    if (st != SSLBM_OK)
        return st;
    st = hip_status(e, hipStreamSynchronize((hipStream_t)hip_stream));
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
    const bool pairs_ok = pairs_aligned(e, rho, scratch);
    std::vector<sslbm_launch> saved;
    for (const EnsClass &cl : e->classes)
        saved.push_back(cl.launch);
    st = tune_classes(e, rho, scratch, pairs_ok, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != SSLBM_OK) {
        for (size_t c = 0; c < e->classes.size(); ++c)
            e->classes[c].launch = saved[c];
        return st;
    }
    drop_graphs(e);
    if (best)
        sslbm_ensemble_get_launch(e, best);
    return SSLBM_OK;
}

int sslbm_ensemble_last_hip_error(const sslbm_ensemble *e) { return e ? e->last_hip : 0; }

void sslbm_ensemble_destroy(sslbm_ensemble *e) {
    if (!e)
        return;
    drop_graphs(e);
    for (auto &t : e->tiles)
        (void)hipFree(t.second.dev);
    if (e->insts)
        (void)hipFree(e->insts);
    if (e->lds_list)
        (void)hipFree(e->lds_list);
    for (EnsClass &cl : e->classes) {
        if (cl.done)
            (void)hipEventDestroy(cl.done);
        if (cl.stream)
            (void)hipStreamDestroy(cl.stream);
    }
    for (hipEvent_t ev : {e->ev_in, e->ev_out, e->ev_fork})
        if (ev)
            (void)hipEventDestroy(ev);
    if (e->stream)
        (void)hipStreamDestroy(e->stream);
    delete e;
}

}  // extern "C"
