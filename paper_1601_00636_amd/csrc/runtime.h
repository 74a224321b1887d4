// Host-side state of libcuboid (context, plans, device buffers).
#pragma once

#include <stdint.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "cuboid.h"
#include "internal.h"

namespace cuboid {

constexpr uint32_t kMaxPrimes = 6542;                 // primes below 2^16
constexpr uint32_t kResidentRowsMax = 1u << 24;       // rows with resident factor lists
constexpr uint64_t kBandRows = 1u << 22;              // rows per band beyond that
constexpr uint64_t kMaxSurvScratch = 1ull << 26;      // survivors held on the device per call
constexpr uint64_t kMaxOrderRows = 1ull << 27;        // rows regrouped per call
constexpr uint64_t kBucketMinRows = 128;              // smaller requests keep their row order
constexpr uint64_t kReplicaBytes = 32ull << 20;       // budget for counter replicas

// Grow-only device allocation.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n);
    void release();
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

// Pinned host staging, grow-only.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n);
    void release();
    ~HostBuf() { release(); }
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
};

// Dense window tables for the first K non-trivial primes of a plan, and the
// list of the remaining ("deep") primes.
struct DenseSet {
    uint32_t K = 0;
    uint32_t dr[kKMax] = {0}, dm[kKMax] = {0}, dinv[kKMax] = {0}, doff[kKMax] = {0};
    uint32_t dext[kKMax] = {0};
    uint32_t words = 0;
    DevBuf tab;
    uint32_t n_deep = 0;
    DevBuf deep;
};

// Everything the GPU needs for one canonical (sorted) prime list.
struct Plan {
    std::vector<uint32_t> primes;                 // ascending
    std::vector<uint8_t> trivial;                 // table identically zero
    std::vector<uint32_t> unsolvable_classes;     // per prime, from the ratio vector
    std::vector<uint32_t> nontriv_idx;            // indices of non-trivial primes, ascending
    std::vector<uint32_t> voff, ioff;             // per prime offsets into the pools
    DevBuf vpool;                                 // ratio vectors, one byte per class
    DevBuf ipool;                                 // inverse tables, uint16
    std::map<uint32_t, std::unique_ptr<DenseSet>> dense;
};

// Unit space and row regrouping of one sweep launch.
struct LaunchShape {
    uint64_t units = 0, n_order = 0, n_chunks = 0;
    uint32_t max_p = 0;
    std::vector<uint64_t> row_prefix, chunk_prefix;   // [n + 1]
};

// A captured batch launch with the bytes of every pointer and size it bakes in.
struct BatchGraph {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

// Results of one sweep over descriptors grouped into counter slots.
struct CoreOut {
    uint32_t nc = 0, n_slots = 0;
    uint32_t width = 0;             // counters per slot: nc, or the caller's primes
    // in the pinned result staging, valid until the next call on the context:
    const uint64_t *counts = nullptr;   // [n_slots][width]: non-trivial primes
                                        // ascending, or the caller's order
    const uint64_t *pairs = nullptr;    // [n_slots]
    std::vector<SurvEntry> surv;    // sorted by (slot, idx), when all fit the scratch
    uint64_t n_surv = 0;
    uint64_t units = 0;
    double sweep_ms = 0;
};
// Device destinations of a call's results (cuboid_sieve_batch_dev): counts
// (in the caller's prime order) and pair counts written by kernels into the
// caller's device buffers, the sorted survivor list copied there too; only
// the survivor count comes back to the host.
struct DevOut {
    uint64_t *counts = nullptr;   // [n_slots][caller primes]
    uint64_t *pairs = nullptr;    // [n_slots]
    SurvEntry *surv = nullptr;    // first surv_cap entries, sorted by (slot, idx)
    uint64_t surv_cap = 0;
};
// Results of one sieve call over several rectangles.
struct SieveOut {
    uint32_t n_req = 0, n_primes = 0;
    const uint64_t *counts = nullptr;   // [n_req][n_primes], caller's prime order
    const uint64_t *pairs = nullptr;    // [n_req] (both in the result staging)
    std::vector<SurvEntry> surv;    // all survivors sorted by (request, index), if fetched
    uint64_t n_surv = 0;            // survivors of the whole call
};

}  // namespace cuboid

struct cuboid_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::recursive_mutex mu;
    std::atomic<int> servers{0};
    std::atomic<int> searches{0};
    std::atomic<int> waiting{0};        // callers blocked on mu (see CtxLock)
    int cu_count = 0;
    size_t max_lds = 0;
    char arch[64] = {0};

    // constant tables
    cuboid::DevBuf primes16, magic16;   // primes below 2^16 and floor(2^32 / p)
    uint32_t n16 = 0;
    cuboid::DevBuf wheel;               // 9 x 30 coprimality windows
    cuboid::DevBuf patterns;            // multiple patterns of the factors >= 7

    // resident factor lists of rows 1..rows_R
    cuboid::DevBuf rows, nfac;
    uint32_t rows_R = 0;
    cuboid::DevBuf band_rows, band_nfac;

    std::map<std::vector<uint32_t>, std::unique_ptr<cuboid::Plan>> plans;
    std::map<std::vector<uint32_t>, cuboid_tuning> tunings;

    // per-call scratch
    cuboid::DevBuf reqbuf, counts, pairs, surv, surv_tmp, surv_n;
    cuboid::DevBuf order, chunk_prefix, row_prefix;   // row regrouping
    cuboid::DevBuf colbuf, gathered;    // counter columns of the caller's primes
    uint32_t n_rep = 1;                 // counter replicas of the current call
    uint64_t rep_stride_counts = 0, rep_stride_pairs = 0;
    bool bucketing = true;
    cuboid::HostBuf req_stage, result_stage;

    // host scratch reused from call to call (no per-call allocation, so no
    // page faults on fresh heap memory inside the timed path)
    std::vector<cuboid::ReqDesc> h_reqs;
    cuboid::LaunchShape h_shape;
    cuboid::CoreOut h_core;
    cuboid::SieveOut h_out;

    // captured batch launches
    bool use_graphs = true;
    std::vector<cuboid::BatchGraph> graphs;
    uint64_t graph_clock = 0;
    uint32_t last_graph = 0;            // 0 eager, 1 replayed, 2 captured for this call
    cuboid::DevBuf gblock;              // request block read by the graph
    cuboid::HostBuf gstage;             // its pinned staging

    // timing
    bool timing = false;
    hipEvent_t ev_sweep0 = nullptr, ev_sweep1 = nullptr, ev_total0 = nullptr, ev_total1 = nullptr;
    cuboid_timing last = {0, 0, 0, 0, 0, 0, 0};
};

namespace cuboid {

// A caller's hold on a context.  The wait is announced so that background
// loops that take the context step after step (the search thread) let
// callers in between their steps instead of re-taking it at once.
struct CtxLock {
    cuboid_ctx *c;
    explicit CtxLock(cuboid_ctx *x) : c(x) {
        c->waiting.fetch_add(1);
        c->mu.lock();
        c->waiting.fetch_sub(1);
    }
    ~CtxLock() { c->mu.unlock(); }
    CtxLock(const CtxLock &) = delete;
    CtxLock &operator=(const CtxLock &) = delete;
};

// A call's reference on a context, taken from the caller's handle (an opaque
// token, see api.cpp).  While it is held, cuboid_destroy returns E_BUSY, so
// the context outlives the call.  Empty if the handle names no live context.
class CtxRef {
   public:
    explicit CtxRef(cuboid_ctx *handle);
    ~CtxRef();
    cuboid_ctx *get() const { return ctx_; }
    explicit operator bool() const { return ctx_ != nullptr; }
    CtxRef(const CtxRef &) = delete;
    CtxRef &operator=(const CtxRef &) = delete;

   private:
    cuboid_ctx *ctx_ = nullptr;
    uint32_t slot_ = 0;
};

// First statement of an entry point taking a context handle `h`: holds a
// reference for the rest of the call and turns `h` into the context itself.
#define CTX_ENTER(h)                                \
    cuboid::CtxRef ctx_ref_(h);                     \
    if (!ctx_ref_) return CUBOID_E_NOT_LOADED;      \
    h = ctx_ref_.get()

const char *status_text(int s);
bool is_prime_u32(uint32_t x);
int canonical_primes(const uint32_t *primes, uint32_t n, std::vector<uint32_t> *sorted);
int build_plan(cuboid_ctx *ctx, const std::vector<uint32_t> &primes, Plan **out);
uint32_t default_dense(const Plan &pl, uint32_t lds_budget);
int build_dense(cuboid_ctx *ctx, Plan *pl, uint32_t K, DenseSet **out);
int ensure_rows(cuboid_ctx *ctx, uint32_t p_max);
int ensure_rows_serving(cuboid_ctx *ctx, uint32_t p_max);   // by a drained server
std::vector<int32_t> count_columns(const Plan &pl, const std::vector<uint32_t> &caller);
cuboid_tuning tuning_for(cuboid_ctx *ctx, const std::vector<uint32_t> &primes, const Plan &pl);
int rect_valid(uint32_t p0, uint32_t p1, uint32_t q0, uint32_t q1);
// max_order_rows: most rows regrouped by factor count in the launch (requests
// past it keep their natural row order)
void shape_reqs(cuboid_ctx *ctx, std::vector<ReqDesc> &reqs, LaunchShape *sh,
                uint64_t max_order_rows = kMaxOrderRows);
int sieve_core(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const cuboid_tuning &tun,
               std::vector<ReqDesc> &reqs, uint32_t n_slots, const std::vector<int32_t> *col,
               uint64_t surv_cap, hipStream_t s, CoreOut *out, const DevOut *dev = nullptr);
int prepare_primes(cuboid_ctx *ctx, const std::vector<uint32_t> &caller_primes, Plan **pl,
                   cuboid_tuning *tun, DenseSet **ds);
void record_timing(cuboid_ctx *ctx, hipStream_t s, const CoreOut &co, const DenseSet &ds,
                   const cuboid_tuning &tun);
int region_sieve(cuboid_ctx *ctx, uint32_t p0, uint32_t p1, uint32_t band_rows,
                 const std::vector<uint32_t> &caller_primes, uint64_t *survivors, uint64_t cap,
                 uint64_t *n_survivors, uint64_t *counts, uint64_t *n_pairs, uint32_t *r_max,
                 hipStream_t s);
SweepParams sweep_params(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const ReqDesc *req,
                         uint32_t n_req, uint64_t units, uint64_t surv_cap);
int run_batch_graph(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const cuboid_tuning &tun,
                    std::vector<ReqDesc> &reqs, uint32_t n_slots,
                    const std::vector<int32_t> *col, uint64_t surv_cap, hipStream_t s,
                    uint64_t *units_out, const DevOut *dev = nullptr);
void drop_graphs(cuboid_ctx *ctx);
// the allocation-free path's device scratch (noalloc.hip): looked up once per
// device at context creation
hipError_t noalloc_scratch_setup(int device);
int sieve_rects(cuboid_ctx *ctx, const std::vector<uint32_t> &caller_primes,
                const cuboid_request *rects, uint32_t n_req, uint64_t surv_cap_total,
                hipStream_t s, SieveOut *out, const DevOut *dev = nullptr);

}  // namespace cuboid
