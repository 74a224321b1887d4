// Batched sieve as one HIP graph launch.
//
// A batch over resident rows is the fixed sequence: upload of the request
// block, one clear of the counter replicas and survivor count, regrouping of
// rows by factor count (when some request is regrouped), the sweep, one
// finishing kernel (replica sums, counts in the caller's prime order, the
// survivor count, and for results in host memory up to kSmallSort survivors
// sorted) and one download of its output block, so that a call with few
// survivors needs no second round trip.  The sizes that vary from batch to batch
// (unit count, regrouping chunks) travel in the request block's header and the
// kernels read them from there, so one captured graph serves every batch with
// the same request count, tables, tuning and buffers.  Graphs are cached per
// context (least recently used out) and keyed by every pointer and size they
// bake in.
//
// The graph is one flat capture (a parent of captured parts costs more to
// launch); with per-call timing on, event-record nodes are then added on
// both sides of the sweep node.
// Clears are fill kernels: no memset nodes.
#include <string.h>

#include <algorithm>

#include "runtime.h"

namespace cuboid {

namespace {

constexpr size_t kHdrBytes = 32;         // unit count, chunk count, two unused words
constexpr uint32_t kBucketGrid = 4096;   // blocks of the regrouping node (grid-stride)
constexpr size_t kMaxGraphs = 8;         // cached graphs per context
constexpr uint64_t kMinOrderRows = 1u << 20;

struct Layout {
    size_t o_desc, o_cpre, o_rpre, o_col, bytes;
};

// Request block, identical in pinned staging and on the device:
// header | descriptors [n] | chunk prefix [n + 1] | row prefix [n + 1] |
// counter column of each caller prime [np] (int32, padded to 8 bytes)
Layout layout_of(uint32_t n, uint32_t np) {
    Layout L;
    L.o_desc = kHdrBytes;
    L.o_cpre = L.o_desc + (size_t)n * sizeof(ReqDesc);
    L.o_rpre = L.o_cpre + (size_t)(n + 1) * 8;
    L.o_col = L.o_rpre + (size_t)(n + 1) * 8;
    L.bytes = L.o_col + ((size_t)np * 4 + 7) / 8 * 8;
    return L;
}

template <typename T>
void put(std::vector<unsigned char> *k, const T &v) {
    const unsigned char *b = (const unsigned char *)&v;
    k->insert(k->end(), b, b + sizeof(T));
}

template <typename F>
hipError_t capture_part(hipStream_t s, hipGraph_t *g, F record) {
    *g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t e1 = record();
    const hipError_t e2 = hipStreamEndCapture(s, g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (*g) (void)hipGraphDestroy(*g);
        *g = nullptr;
        return e1 != hipSuccess ? e1 : e2;
    }
    return hipSuccess;
}

// With per-call timing: the captured graph is a chain (upload, clear, the
// regrouping when present, sweep, finishing kernel, download); put an
// event-record node on each side of the sweep, its node number `at` from 0.
hipError_t bracket_sweep(cuboid_ctx *ctx, hipGraph_t g, size_t at) {
    std::vector<hipGraphNode_t> chain;
    size_t n = 1;
    hipGraphNode_t node = nullptr;
    hipError_t e = hipGraphGetRootNodes(g, &node, &n);
    if (e != hipSuccess) return e;
    if (n != 1) return hipErrorInvalidValue;
    while (node) {
        chain.push_back(node);
        size_t nd = 0;
        e = hipGraphNodeGetDependentNodes(node, nullptr, &nd);
        if (e != hipSuccess) return e;
        if (nd > 1) return hipErrorInvalidValue;
        hipGraphNode_t next = nullptr;
        if (nd == 1) {
            e = hipGraphNodeGetDependentNodes(node, &next, &nd);
            if (e != hipSuccess) return e;
        }
        node = next;
    }
    if (at == 0 || at + 1 >= chain.size()) return hipErrorInvalidValue;
    hipGraphNodeType type;
    e = hipGraphNodeGetType(chain[at], &type);
    if (e != hipSuccess) return e;
    if (type != hipGraphNodeTypeKernel) return hipErrorInvalidValue;
    hipGraphNode_t before = chain[at - 1], sweep = chain[at], after = chain[at + 1];
    hipGraphNode_t ev0 = nullptr, ev1 = nullptr;
    e = hipGraphRemoveDependencies(g, &before, &sweep, 1);
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&ev0, g, &before, 1, ctx->ev_sweep0);
    if (e == hipSuccess) e = hipGraphAddDependencies(g, &ev0, &sweep, 1);
    if (e == hipSuccess) e = hipGraphRemoveDependencies(g, &sweep, &after, 1);
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&ev1, g, &sweep, 1, ctx->ev_sweep1);
    if (e == hipSuccess) e = hipGraphAddDependencies(g, &ev1, &after, 1);
    return e;
}

struct GraphArgs {
    SweepParams P;
    unsigned char *block;
    const unsigned char *stage;
    uint64_t *result;
    uint32_t *order;
    Layout L;
    uint32_t n, n_slots, nc, np, grid;
    bool gather;                  // counts come back in the caller's prime order
    bool bucket;                  // some request's rows are regrouped
    uint64_t *dcounts;            // device destinations (cuboid_sieve_batch_dev), else null:
    uint64_t *dpairs;             //   results go to the pinned result staging
    uint64_t small_sort;          // survivors sorted and downloaded in the graph (0: none)
    size_t lds;
    uint32_t max_p;
    bool timing;
};

hipError_t build_graph(cuboid_ctx *ctx, const GraphArgs &a, hipStream_t s, BatchGraph *out) {
    const uint32_t n = a.n, ns = a.n_slots, nc = a.nc;
    const uint64_t ncount = (uint64_t)ns * nc;
    const uint64_t nout = (uint64_t)ns * (a.gather ? a.np : nc);
    hipGraph_t parent = nullptr;
    hipGraphExec_t exec = nullptr;
    auto record_pre = [&]() -> hipError_t {
        hipError_t r = hipMemcpyAsync(a.block, a.stage, a.L.bytes, hipMemcpyHostToDevice, s);
        if (r == hipSuccess)
            r = launch_clear3((uint64_t *)ctx->counts.p, (uint64_t)ctx->n_rep * ncount,
                              (uint64_t *)ctx->pairs.p, (uint64_t)ctx->n_rep * ns,
                              (uint64_t *)ctx->surv_n.p, 2, s);
        if (r == hipSuccess && a.bucket)
            r = launch_bucket_rows((const ReqDesc *)(a.block + a.L.o_desc), n,
                                   (const uint64_t *)(a.block + a.L.o_cpre), 0,
                                   (const uint64_t *)(a.block + a.L.o_rpre), a.order, s,
                                   (const uint64_t *)a.block + 1, kBucketGrid);
        return r;
    };
    auto record_sweep = [&]() { return launch_sweep(a.P, (int)a.grid, a.lds, a.max_p, s); };
    auto record_post = [&]() -> hipError_t {
        // output block (device, downloaded whole into the result staging):
        // [nout counts | ns pairs | survivor count | small_sort survivors];
        // with device destinations only the survivor count is in it
        unsigned long long *ob = (unsigned long long *)ctx->gathered.p;
        unsigned long long *oc = a.dcounts ? (unsigned long long *)a.dcounts : ob;
        unsigned long long *op = a.dpairs ? (unsigned long long *)a.dpairs : ob + nout;
        unsigned long long *on = a.dcounts ? ob : ob + nout + ns;
        hipError_t r = launch_finish((const unsigned long long *)ctx->counts.p,
                                     (const unsigned long long *)ctx->pairs.p, ctx->n_rep,
                                     ctx->rep_stride_counts, ctx->rep_stride_pairs,
                                     a.gather ? (const int32_t *)(a.block + a.L.o_col) : nullptr,
                                     ns, nc, a.gather ? a.np : nc, oc, op,
                                     (const unsigned long long *)ctx->surv_n.p, on,
                                     (const SurvEntry *)ctx->surv.p, a.small_sort,
                                     (SurvEntry *)(on + 1), s);
        if (r == hipSuccess && a.dcounts)
            r = hipMemcpyAsync(a.result + nout + ns, on, 8, hipMemcpyDeviceToHost, s);
        else if (r == hipSuccess)
            r = hipMemcpyAsync(a.result, ob, (nout + ns + 1 + 2 * a.small_sort) * 8,
                               hipMemcpyDeviceToHost, s);
        return r;
    };
    // one flat capture (a nested graph costs more to launch)
    hipError_t e = capture_part(s, &parent, [&]() -> hipError_t {
        hipError_t r = record_pre();
        if (r == hipSuccess) r = record_sweep();
        if (r == hipSuccess) r = record_post();
        return r;
    });
    if (e == hipSuccess && a.timing) {
        // the sweep's place in the chain: the node count of the part before it
        hipGraph_t pre = nullptr;
        size_t n_pre = 0;
        e = capture_part(s, &pre, record_pre);
        if (e == hipSuccess) e = hipGraphGetNodes(pre, nullptr, &n_pre);
        if (pre) (void)hipGraphDestroy(pre);
        if (e == hipSuccess) e = bracket_sweep(ctx, parent, n_pre);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, parent, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (parent) (void)hipGraphDestroy(parent);
        return e;
    }
    out->graph = parent;
    out->exec = exec;
    return hipSuccess;
}

}  // namespace

void destroy_graph(BatchGraph *g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
}

void drop_graphs(cuboid_ctx *ctx) {
    for (auto &g : ctx->graphs) destroy_graph(&g);
    ctx->graphs.clear();
}

// Resident-row batch as one graph launch on `s`; the caller synchronizes `s`
// before reading counts, pair counts and the survivor count from the result
// staging ([n_slots * width] counts | [n_slots] pairs | survivor count), width
// being nc, or the caller's prime count when `col` maps them.  With `dev`
// (and `col`), counts and pair counts go to the caller's device buffers and
// only the survivor count to the staging.
int run_batch_graph(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const cuboid_tuning &tun,
                    std::vector<ReqDesc> &reqs, uint32_t n_slots,
                    const std::vector<int32_t> *col, uint64_t surv_cap, hipStream_t s,
                    uint64_t *units_out, const DevOut *dev) {
    const uint32_t n = (uint32_t)reqs.size();
    const uint32_t nc = ds.K + ds.n_deep;
    LaunchShape &sh = ctx->h_shape;
    shape_reqs(ctx, reqs, &sh);
    if (sh.n_order) {
        // room to spare so later batches keep the same buffer (and graph)
        uint64_t want = kMinOrderRows;
        while (want < sh.n_order) want <<= 1;
        if (ctx->order.ensure(want * 4) != hipSuccess) return CUBOID_E_DEVICE;
    }
    for (size_t i = 0; i < reqs.size(); ++i)
        reqs[i].order = sh.row_prefix[i + 1] > sh.row_prefix[i]
                            ? (const uint32_t *)ctx->order.p + sh.row_prefix[i] : nullptr;
    const size_t lds = (size_t)ds.words * 8 + kSweepFixedLds;
    if (lds > ctx->max_lds) return CUBOID_E_LIMIT;
    const uint32_t np = col ? (uint32_t)col->size() : 0;
    const Layout L = layout_of(n, np);
    const uint64_t nout = (uint64_t)n_slots * (col ? np : nc);
    // the previous reader of the staging buffers on this stream is done once
    // the stream is idle
    if (hipStreamSynchronize(s) != hipSuccess) return CUBOID_E_DEVICE;
    // survivors sorted inside the graph for results in host memory: at most
    // kSmallSort, and no more than the survivor scratch holds
    const uint64_t small_sort = dev ? 0 : std::min<uint64_t>(kSmallSort, surv_cap);
    const size_t out_bytes = (nout + n_slots + 1 + 2 * small_sort) * 8;
    if (ctx->gstage.ensure(L.bytes) != hipSuccess || ctx->gblock.ensure(L.bytes) != hipSuccess ||
        ctx->result_stage.ensure(out_bytes) != hipSuccess ||
        ctx->gathered.ensure(out_bytes) != hipSuccess)
        return CUBOID_E_DEVICE;
    unsigned char *st = (unsigned char *)ctx->gstage.p;
    const uint64_t hdr[4] = {sh.units, sh.n_chunks, 0, 0};
    memcpy(st, hdr, sizeof(hdr));
    memcpy(st + L.o_desc, reqs.data(), (size_t)n * sizeof(ReqDesc));
    memcpy(st + L.o_cpre, sh.chunk_prefix.data(), (size_t)(n + 1) * 8);
    memcpy(st + L.o_rpre, sh.row_prefix.data(), (size_t)(n + 1) * 8);
    if (np) memcpy(st + L.o_col, col->data(), (size_t)np * 4);

    GraphArgs a;
    a.block = (unsigned char *)ctx->gblock.p;
    a.stage = st;
    a.result = (uint64_t *)ctx->result_stage.p;
    a.order = (uint32_t *)ctx->order.p;
    a.L = L;
    a.n = n;
    a.n_slots = n_slots;
    a.nc = nc;
    a.np = np;
    a.gather = col != nullptr;
    a.bucket = sh.n_order > 0;
    a.dcounts = dev ? dev->counts : nullptr;
    a.dpairs = dev ? dev->pairs : nullptr;
    a.small_sort = small_sort;
    a.grid = tun.workgroups;
    a.lds = lds;
    a.max_p = sh.max_p;
    a.timing = ctx->timing;
    a.P = sweep_params(ctx, pl, ds, (const ReqDesc *)(a.block + L.o_desc), n, 0, surv_cap);
    a.P.schedule = tun.schedule;
    a.P.piece = tun.piece_units;
    for (const ReqDesc &d : reqs) a.P.band_split |= (d.flags & kReqBandSplit) ? 1u : 0u;
    a.P.units_dev = (const unsigned long long *)a.block;

    std::vector<unsigned char> key;
    put(&key, a.P);
    put(&key, (const void *)a.block);
    put(&key, (const void *)a.stage);
    put(&key, (const void *)a.result);
    put(&key, (const void *)a.order);
    put(&key, (uint64_t)L.bytes);
    put(&key, (uint64_t)a.lds);
    put(&key, ctx->n_rep);
    put(&key, n_slots);
    put(&key, np);
    put(&key, (uint32_t)a.gather);
    put(&key, (uint32_t)a.bucket);
    put(&key, a.small_sort);
    put(&key, (const void *)ctx->surv.p);
    put(&key, (const void *)ctx->gathered.p);
    put(&key, (const void *)a.dcounts);
    put(&key, (const void *)a.dpairs);
    put(&key, a.grid);
    put(&key, (uint32_t)sweep_factor_slots(sh.max_p));
    put(&key, (uint32_t)a.timing);
    put(&key, (const void *)ctx->ev_sweep0);
    put(&key, (const void *)ctx->ev_sweep1);

    BatchGraph *g = nullptr;
    for (auto &c : ctx->graphs)
        if (c.key == key) g = &c;
    ctx->last_graph = 1;
    if (!g) {
        if (ctx->graphs.size() >= kMaxGraphs) {
            auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                        [](const BatchGraph &x, const BatchGraph &y) {
                                            return x.last_use < y.last_use;
                                        });
            destroy_graph(&*lru);
            ctx->graphs.erase(lru);
        }
        BatchGraph fresh;
        if (build_graph(ctx, a, s, &fresh) != hipSuccess) {
            (void)hipGetLastError();
            return CUBOID_E_DEVICE;
        }
        fresh.key = std::move(key);
        ctx->graphs.push_back(std::move(fresh));
        g = &ctx->graphs.back();
        ctx->last_graph = 2;
    }
    g->last_use = ++ctx->graph_clock;
    if (hipGraphLaunch(g->exec, s) != hipSuccess) return CUBOID_E_DEVICE;
    *units_out = sh.units;
    return CUBOID_OK;
}

}  // namespace cuboid
