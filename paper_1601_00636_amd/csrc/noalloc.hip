// The allocation-free form of the batched sieve with device results
// (cuboid_sieve_batch_dev_noalloc, include/cuboid.h), for callers that cannot
// allocate device memory.  Every device buffer the call needs besides the
// caller's outputs -- request descriptors, row order, counter replicas,
// survivor list and its sort buffer, the survivor count and claim counter --
// is carved out of one file-scope device array per GPU, `scratch`, whose
// address is looked up once per device when a context is created there.
// Tables and the resident row table must already exist (built by an earlier
// call with the same prime list); the call then allocates no device or
// pinned memory.  The kernels are those of the regular path.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "runtime.h"

using namespace cuboid;

namespace {

constexpr size_t kNoAllocScratchBytes = 64ull << 20;     // the array, per GPU
constexpr uint64_t kNoAllocOrderBytes = 24ull << 20;     // regrouped rows, at most
constexpr uint64_t kNoAllocReplicaBytes = 16ull << 20;   // counter replicas, at most
constexpr uint64_t kNoAllocSurvMax = 1ull << 19;         // survivor entries, at most
constexpr uint64_t kNoAllocSurvMin = 1024;               // survivor entries, at least
constexpr int kMaxDevices = 64;

// In host code `scratch` is a host-side stand-in, not a device address: only
// the address hipGetSymbolAddress returns on a device is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_setup_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {nullptr};
// calls on one GPU share its array: they take turns, each holding the lock
// until its work on the device has completed
std::mutex g_dev_mu[kMaxDevices];

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace cuboid {

hipError_t noalloc_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_setup_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    // context creation has made `device` current
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (unsigned char *)ptr;
    return hipSuccess;
}

}  // namespace cuboid

#define HIPCHK(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return CUBOID_E_DEVICE; \
    } while (0)

extern "C" int cuboid_sieve_batch_dev_noalloc(cuboid_ctx *ctx, const cuboid_request *req,
                                              uint32_t n_req, const uint32_t *primes,
                                              uint32_t n_primes, uint64_t *counts_dev,
                                              uint64_t *pairs_dev, void *survivors_dev,
                                              uint64_t surv_cap, uint64_t *n_survivors,
                                              void *hip_stream) {
    CTX_ENTER(ctx);
    if (!req || n_req == 0 || n_req == 0xffffffffu || !counts_dev || !pairs_dev || !n_survivors ||
        (surv_cap && !survivors_dev))
        return CUBOID_E_ARG;
    *n_survivors = 0;
    for (uint32_t i = 0; i < n_req; ++i)
        if (rect_valid(req[i].p0, req[i].p1, req[i].q0, req[i].q1)) return CUBOID_E_RANGE;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    const uint64_t n = n_req;
    // the fixed part of the layout: control words, descriptors, the two
    // prefix arrays of the row regrouping, the caller's count columns
    const size_t fixed = align256(16) + align256(n * sizeof(ReqDesc)) + 2 * align256((n + 1) * 8) +
                         align256((size_t)n_primes * 4);
    if (fixed >= kNoAllocScratchBytes) return CUBOID_E_LIMIT;

    CtxLock g(ctx);
    if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
    // the tables must be resident: nothing is built here
    auto pit = ctx->plans.find(sorted);
    if (pit == ctx->plans.end()) return CUBOID_E_NOT_LOADED;
    const Plan &pl = *pit->second;
    const cuboid_tuning tun = tuning_for(ctx, sorted, pl);
    auto dit = pl.dense.find(tun.dense_primes);
    if (dit == pl.dense.end()) return CUBOID_E_NOT_LOADED;
    const DenseSet &ds = *dit->second;
    const uint32_t nc = ds.K + ds.n_deep;
    uint32_t pmax = 0;
    for (uint32_t i = 0; i < n_req; ++i) pmax = std::max(pmax, req[i].p1);
    if (pmax > ctx->rows_R) return pmax > kResidentRowsMax ? CUBOID_E_LIMIT : CUBOID_E_NOT_LOADED;
    const size_t lds = (size_t)ds.words * 8 + kSweepFixedLds;
    if (lds > ctx->max_lds) return CUBOID_E_LIMIT;
    const int dev = ctx->device;
    if (dev < 0 || dev >= kMaxDevices || !g_scratch_ptr[dev]) return CUBOID_E_DEVICE;
    std::lock_guard<std::mutex> dg(g_dev_mu[dev]);
    unsigned char *const base = g_scratch_ptr[dev];
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;

    // descriptors, rows from the resident table
    std::vector<ReqDesc> &reqs = ctx->h_reqs;
    reqs.resize(n_req);
    for (uint32_t i = 0; i < n_req; ++i) {
        ReqDesc &d = reqs[i];
        memset(&d, 0, sizeof(d));
        d.p0 = req[i].p0; d.p1 = req[i].p1; d.q0 = req[i].q0; d.q1 = req[i].q1;
        d.ip0 = req[i].p0;
        d.slot = i;
        d.rows = (const RowInfo *)ctx->rows.p;
        d.nfac = (const uint8_t *)ctx->nfac.p;
        d.rows_p0 = 1;
    }

    // layout: the fixed part, the row order, the counter replicas, then the
    // survivor list and its sort buffer in what is left
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += align256(bytes);
        return p;
    };
    unsigned long long *ctl = (unsigned long long *)take(16);   // survivor count, claim
    ReqDesc *dreq = (ReqDesc *)take(n * sizeof(ReqDesc));
    uint64_t *dchunk = (uint64_t *)take((n + 1) * 8);
    uint64_t *drowp = (uint64_t *)take((n + 1) * 8);
    int32_t *dcol = (int32_t *)take((size_t)n_primes * 4);
    const size_t one_rep = align256(n * nc * 8 + 8) + align256(n * 8 + 8);
    const size_t surv_min = 2 * align256(kNoAllocSurvMin * sizeof(SurvEntry));
    if (off + one_rep + surv_min > kNoAllocScratchBytes) return CUBOID_E_LIMIT;
    const uint64_t order_room = std::min<uint64_t>(
        kNoAllocOrderBytes, kNoAllocScratchBytes - off - one_rep - surv_min - 256);
    LaunchShape &sh = ctx->h_shape;
    shape_reqs(ctx, reqs, &sh, std::min<uint64_t>(kMaxOrderRows, order_room / 4));
    uint32_t *order = (uint32_t *)take(sh.n_order * 4);
    for (uint32_t i = 0; i < n_req; ++i)
        reqs[i].order = sh.row_prefix[i + 1] > sh.row_prefix[i] ? order + sh.row_prefix[i] : nullptr;
    const size_t rep_room =
        std::min<size_t>(kNoAllocReplicaBytes, kNoAllocScratchBytes - off - surv_min);
    uint32_t rep = 64;
    while (rep > 1 && align256(rep * n * nc * 8 + 8) + align256(rep * n * 8 + 8) > rep_room)
        rep >>= 1;
    if (one_rep > kNoAllocScratchBytes - off - surv_min) return CUBOID_E_LIMIT;
    unsigned long long *counts = (unsigned long long *)take(rep * n * nc * 8 + 8);
    unsigned long long *pairs = (unsigned long long *)take(rep * n * 8 + 8);
    const uint64_t surv_room = (kNoAllocScratchBytes - off) / (2 * sizeof(SurvEntry));
    const uint64_t S = std::min<uint64_t>(kNoAllocSurvMax, surv_room / 1024 * 1024);
    if (S < kNoAllocSurvMin) return CUBOID_E_LIMIT;
    SurvEntry *surv = (SurvEntry *)take(S * sizeof(SurvEntry));
    SurvEntry *surv_tmp = (SurvEntry *)take(S * sizeof(SurvEntry));
    if (off > kNoAllocScratchBytes) return CUBOID_E_LIMIT;

    // inputs in, counters cleared (fill kernels, no memset nodes)
    HIPCHK(hipMemcpyAsync(dreq, reqs.data(), n * sizeof(ReqDesc), hipMemcpyHostToDevice, s));
    const std::vector<int32_t> col = count_columns(pl, std::vector<uint32_t>(primes, primes + n_primes));
    HIPCHK(hipMemcpyAsync(dcol, col.data(), (size_t)n_primes * 4, hipMemcpyHostToDevice, s));
    HIPCHK(launch_fill_u64((uint64_t *)counts, rep * n * nc, 0, s));
    HIPCHK(launch_fill_u64((uint64_t *)pairs, rep * n, 0, s));
    HIPCHK(launch_fill_u64((uint64_t *)ctl, 2, 0, s));
    if (sh.n_order) {
        HIPCHK(hipMemcpyAsync(dchunk, sh.chunk_prefix.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(drowp, sh.row_prefix.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
        HIPCHK(launch_bucket_rows(dreq, n_req, dchunk, sh.n_chunks, drowp, order, s));
    }
    // the sweep, with every scratch pointer in the array
    SweepParams P = sweep_params(ctx, pl, ds, dreq, n_req, sh.units, S);
    P.counts = counts;
    P.pairs = pairs;
    P.n_rep = rep;
    P.rep_stride_counts = n * nc;
    P.rep_stride_pairs = n;
    P.surv = surv;
    P.surv_n = ctl;
    P.claim = ctl + 1;
    P.schedule = tun.schedule;
    P.piece = tun.piece_units;
    P.band_split = 0;
    HIPCHK(launch_sweep(P, (int)tun.workgroups, lds, sh.max_p, s));
    HIPCHK(launch_reduce_replicas(counts, n * nc, rep, n * nc, s));
    HIPCHK(launch_reduce_replicas(pairs, n, rep, n, s));
    // results into the caller's buffers: counts in the caller's prime order
    HIPCHK(launch_gather_counts(counts, dcol, n_req, nc, n_primes,
                                (unsigned long long *)counts_dev, s));
    HIPCHK(launch_copy_u64(pairs_dev, (const uint64_t *)pairs, n, s));
    uint64_t ns = 0;
    HIPCHK(hipMemcpyAsync(&ns, ctl, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ns && ns <= S) {
        SurvEntry *sorted_surv = nullptr;
        HIPCHK(launch_sort_surv(surv, surv_tmp, ctl, ns, &sorted_surv, s));
        const uint64_t k = std::min<uint64_t>(ns, surv_cap);
        if (k) HIPCHK(launch_copy_u64((uint64_t *)survivors_dev, (const uint64_t *)sorted_surv,
                                      2 * k, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    *n_survivors = ns;
    if (ns > S) return CUBOID_E_LIMIT;
    return ns > surv_cap ? CUBOID_E_CAPACITY : CUBOID_OK;
}
