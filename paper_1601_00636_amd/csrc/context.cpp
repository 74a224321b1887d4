// Host runtime of libcuboid: context, resident tables, prime plans, the plain
// and batched sieve entry points and the root check.  Every arithmetic step of
// the sieve runs in the HIP kernels; this file validates arguments, plans the
// launch (unit space, rows, tables) and moves results.
#include "runtime.h"

#include <string.h>

#include <algorithm>
#include <chrono>
#include <numeric>

#include "bigint.h"

using namespace cuboid;

namespace cuboid {

const char *status_text(int s) {
    switch (s) {
        case CUBOID_OK: return "ok";
        case CUBOID_E_BUSY: return "busy: work in flight";
        case CUBOID_E_RANGE: return "invalid range";
        case CUBOID_E_LIMIT: return "size limit exceeded";
        case CUBOID_E_PRIMES: return "invalid prime list";
        case CUBOID_E_CAPACITY: return "output capacity too small";
        case CUBOID_E_NOT_LOADED: return "context not loaded";
        case CUBOID_E_DEVICE: return "device or HIP runtime error";
        case CUBOID_E_ARG: return "invalid argument";
        case CUBOID_E_IO: return "file input/output error";
        case CUBOID_E_DATA: return "file contents differ from the tables";
        default: return "unknown status";
    }
}

bool is_prime_u32(uint32_t x) {
    if (x < 2) return false;
    for (uint32_t d = 2; (uint64_t)d * d <= x; ++d)
        if (x % d == 0) return false;
    return true;
}

int canonical_primes(const uint32_t *primes, uint32_t n, std::vector<uint32_t> *sorted) {
    if (!primes || n == 0) return CUBOID_E_PRIMES;
    if (n > kMaxPrimes) return CUBOID_E_PRIMES;
    sorted->assign(primes, primes + n);
    std::sort(sorted->begin(), sorted->end());
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t r = (*sorted)[i];
        if (r >= 65536 || !is_prime_u32(r)) return CUBOID_E_PRIMES;
        if (i && (*sorted)[i - 1] == r) return CUBOID_E_PRIMES;
    }
    return CUBOID_OK;
}

hipError_t DevBuf::ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    size_t want = n ? n : 1;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) { p = nullptr; bytes = 0; return e; }
    bytes = want;
    return hipSuccess;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

hipError_t HostBuf::ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    size_t want = n ? n : 1;
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) { p = nullptr; bytes = 0; return e; }
    bytes = want;
    return hipSuccess;
}

void HostBuf::release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

}  // namespace cuboid

#define HIPCHK(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return CUBOID_E_DEVICE; \
    } while (0)

namespace {

uint32_t magic_of(uint32_t r) { return (uint32_t)(0x100000000ull / r); }

hipStream_t pick_stream(cuboid_ctx *ctx, void *s) {
    return s ? (hipStream_t)s : ctx->stream;
}

template <typename T>
hipError_t upload(DevBuf &b, const std::vector<T> &v, hipStream_t s) {
    hipError_t e = b.ensure(v.size() * sizeof(T));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

std::vector<uint64_t> prefix_of(const std::vector<uint64_t> &w) {
    std::vector<uint64_t> pre(w.size() + 1, 0);
    for (size_t i = 0; i < w.size(); ++i) pre[i + 1] = pre[i] + w[i];
    return pre;
}

}  // namespace

namespace cuboid {

// Ratio vectors and inverse tables for every prime of the set, built on the
// GPU; the per-prime count of unsolvable ratio classes tells which tables are
// identically zero.
int build_plan(cuboid_ctx *ctx, const std::vector<uint32_t> &primes, Plan **out) {
    auto it = ctx->plans.find(primes);
    if (it != ctx->plans.end()) { *out = it->second.get(); return CUBOID_OK; }
    std::unique_ptr<Plan> pl(new Plan());
    pl->primes = primes;
    const uint32_t n = (uint32_t)primes.size();
    hipStream_t s = ctx->stream;
    std::vector<uint32_t> voff(n), ioff(n);
    std::vector<uint64_t> wv(n), wi(n);
    uint64_t tot = 0;
    for (uint32_t i = 0; i < n; ++i) {
        voff[i] = (uint32_t)tot;
        ioff[i] = (uint32_t)tot;
        tot += primes[i];
        wv[i] = primes[i] == 2 ? 1 : (primes[i] - 1) / 2;
        wi[i] = primes[i] - 1;
    }
    pl->voff = voff;
    pl->ioff = ioff;
    const std::vector<uint64_t> pv = prefix_of(wv), pi = prefix_of(wi);
    DevBuf d_pr, d_voff, d_ioff, d_pv, d_pi, d_pop;
    HIPCHK(upload(d_pr, primes, s));
    HIPCHK(upload(d_voff, voff, s));
    HIPCHK(upload(d_ioff, ioff, s));
    HIPCHK(upload(d_pv, pv, s));
    HIPCHK(upload(d_pi, pi, s));
    HIPCHK(pl->vpool.ensure(tot));
    HIPCHK(pl->ipool.ensure(tot * 2));
    HIPCHK(launch_fill_u8((uint8_t *)pl->vpool.p, tot, 0, s));
    HIPCHK(launch_fill_u8((uint8_t *)pl->ipool.p, tot * 2, 0, s));
    HIPCHK(launch_ratio_vectors((const uint32_t *)d_pr.p, (const uint32_t *)d_voff.p, n,
                                (const uint64_t *)d_pv.p, pv[n], (uint8_t *)pl->vpool.p, s));
    HIPCHK(launch_inverse_tables((const uint32_t *)d_pr.p, (const uint32_t *)d_ioff.p, n,
                                 (const uint64_t *)d_pi.p, pi[n], (uint16_t *)pl->ipool.p, s));
    HIPCHK(d_pop.ensure(n * 4));
    HIPCHK(launch_vector_popcount((const uint32_t *)d_pr.p, (const uint32_t *)d_voff.p, n,
                                  (const uint8_t *)pl->vpool.p, (uint32_t *)d_pop.p, s));
    std::vector<uint32_t> pop(n);
    HIPCHK(hipMemcpyAsync(pop.data(), d_pop.p, n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    pl->unsolvable_classes = pop;
    pl->trivial.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        pl->trivial[i] = pop[i] == 0;
        if (!pl->trivial[i]) pl->nontriv_idx.push_back(i);
    }
    *out = pl.get();
    ctx->plans[primes] = std::move(pl);
    return CUBOID_OK;
}

// LDS bytes of the dense window table of prime r: r rows of r + kDenseExt words
uint64_t dense_table_bytes(uint64_t r) { return 8 * r * (r + kDenseExt); }

uint32_t default_dense(const Plan &pl, uint32_t lds_budget) {
    uint64_t bytes = 0;
    uint32_t k = 0;
    while (k < pl.nontriv_idx.size() && k < (uint32_t)kKMax) {
        const uint64_t r = pl.primes[pl.nontriv_idx[k]];
        if (bytes + dense_table_bytes(r) > lds_budget) break;
        bytes += dense_table_bytes(r);
        ++k;
    }
    return k;
}

// Window tables for the first K non-trivial primes and the deep-prime list.
int build_dense(cuboid_ctx *ctx, Plan *pl, uint32_t K, DenseSet **out) {
    auto it = pl->dense.find(K);
    if (it != pl->dense.end()) { *out = it->second.get(); return CUBOID_OK; }
    if (K > pl->nontriv_idx.size() || K > (uint32_t)kKMax) return CUBOID_E_ARG;
    std::unique_ptr<DenseSet> ds(new DenseSet());
    hipStream_t s = ctx->stream;
    ds->K = K;
    std::vector<uint32_t> pr(K), vo(K), io(K), wo(K);
    std::vector<uint64_t> work(K);
    uint64_t words = 0;
    for (uint32_t k = 0; k < K; ++k) {
        const uint32_t i = pl->nontriv_idx[k];
        const uint32_t r = pl->primes[i];
        pr[k] = r; vo[k] = pl->voff[i]; io[k] = pl->ioff[i]; wo[k] = (uint32_t)words;
        work[k] = (uint64_t)r * (r + kDenseExt);
        ds->dr[k] = r;
        ds->dm[k] = magic_of(r);
        // 64^(r-2) = 64^-1 mod r
        uint64_t inv = 1, b = 64 % r;
        for (uint64_t e = r - 2; e; e >>= 1, b = b * b % r)
            if (e & 1) inv = inv * b % r;
        ds->dinv[k] = (uint32_t)inv;
        ds->dext[k] = kDenseExt % r;
        ds->doff[k] = (uint32_t)(words * 8);
        words += (uint64_t)r * (r + kDenseExt);
    }
    ds->words = (uint32_t)words;
    HIPCHK(ds->tab.ensure(words * 8));
    if (K) {
        const std::vector<uint64_t> pre = prefix_of(work);
        DevBuf d_pr, d_vo, d_io, d_wo, d_pre;
        HIPCHK(upload(d_pr, pr, s));
        HIPCHK(upload(d_vo, vo, s));
        HIPCHK(upload(d_io, io, s));
        HIPCHK(upload(d_wo, wo, s));
        HIPCHK(upload(d_pre, pre, s));
        HIPCHK(launch_dense_windows((const uint32_t *)d_pr.p, (const uint32_t *)d_vo.p,
                                    (const uint32_t *)d_io.p, (const uint32_t *)d_wo.p, K,
                                    (const uint64_t *)d_pre.p, pre[K], (const uint8_t *)pl->vpool.p,
                                    (const uint16_t *)pl->ipool.p, (uint64_t *)ds->tab.p, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    std::vector<DeepPrime> deep;
    for (size_t k = K; k < pl->nontriv_idx.size(); ++k) {
        const uint32_t i = pl->nontriv_idx[k];
        DeepPrime d;
        d.r = pl->primes[i];
        d.m = magic_of(d.r);
        d.voff = pl->voff[i];
        d.ioff = pl->ioff[i];
        deep.push_back(d);
    }
    ds->n_deep = (uint32_t)deep.size();
    HIPCHK(upload(ds->deep, deep, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = ds.get();
    pl->dense[K] = std::move(ds);
    return CUBOID_OK;
}

// Resident row table for 1 <= p <= R, grown to cover p_max when p_max <= 2^24.
// Growing reallocates the table, so it is refused (E_BUSY) while a server may
// have launches reading it, except from the one server when it is drained.
static int ensure_rows_impl(cuboid_ctx *ctx, uint32_t p_max, bool from_server) {
    if (p_max <= ctx->rows_R) return CUBOID_OK;
    if (p_max > kResidentRowsMax) return CUBOID_E_LIMIT;
    const int servers = ctx->servers.load();
    if (servers > (from_server ? 1 : 0)) return CUBOID_E_BUSY;
    uint64_t R = 1u << 16;
    while (R < p_max) R <<= 1;
    if (R > kResidentRowsMax) R = kResidentRowsMax;
    HIPCHK(ctx->rows.ensure(R * sizeof(RowInfo)));
    HIPCHK(ctx->nfac.ensure(R));
    HIPCHK(launch_row_info((const uint32_t *)ctx->primes16.p, (const uint32_t *)ctx->magic16.p,
                           ctx->n16, 1, R, (RowInfo *)ctx->rows.p, (uint8_t *)ctx->nfac.p,
                           ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->rows_R = (uint32_t)R;
    return CUBOID_OK;
}

int ensure_rows(cuboid_ctx *ctx, uint32_t p_max) { return ensure_rows_impl(ctx, p_max, false); }

int ensure_rows_serving(cuboid_ctx *ctx, uint32_t p_max) {
    return ensure_rows_impl(ctx, p_max, true);
}

cuboid_tuning tuning_for(cuboid_ctx *ctx, const std::vector<uint32_t> &primes, const Plan &pl) {
    cuboid_tuning t;
    auto it = ctx->tunings.find(primes);
    if (it != ctx->tunings.end()) t = it->second;
    else {
        t.dense_primes = 0xffffffffu; t.workgroups = 0; t.lds_budget = 0; t.schedule = 0;
        t.piece_units = 0;
    }
    // the dense tables and the sweep's fixed LDS must fit one workgroup; by
    // default the tables take all of the LDS left
    const uint32_t room = ctx->max_lds > kSweepFixedLds ? (uint32_t)(ctx->max_lds - kSweepFixedLds) : 0;
    if (t.lds_budget == 0 || t.lds_budget > room) t.lds_budget = room;
    const uint32_t kmax = default_dense(pl, t.lds_budget);
    if (t.dense_primes > kmax) t.dense_primes = kmax;
    // one workgroup per compute unit: waves take their units from a shared
    // counter, so more workgroups would only load the tables again
    if (t.workgroups == 0) t.workgroups = ctx->cu_count;
    return t;
}

// Unit space of one launch: each request's first unit and unit count, and
// which requests get their rows regrouped by factor count (prefix sums of
// regrouped rows and of 8192-row chunks).  Counter slots are the caller's.
void shape_reqs(cuboid_ctx *ctx, std::vector<ReqDesc> &reqs, LaunchShape *sh,
                uint64_t max_order_rows) {
    const uint32_t n = (uint32_t)reqs.size();
    sh->row_prefix.assign(n + 1, 0);
    sh->chunk_prefix.assign(n + 1, 0);
    uint64_t units = 0;
    uint32_t max_p = 0;
    for (uint32_t i = 0; i < n; ++i) {
        ReqDesc &r = reqs[i];
        const uint64_t rows = (uint64_t)r.p1 - r.p0 + 1;
        r.nrb = (uint32_t)((rows + 63) / 64);
        r.nwin = (uint32_t)(((uint64_t)r.q1 - r.q0 + 64) / 64);
        r.unit0 = units;
        r.ulo = 0;
        r.ucount = (uint64_t)r.nrb * r.nwin;
        units += r.ucount;
        max_p = std::max(max_p, r.p1);
        // band-split region requests keep their rows in natural order
        const bool group = ctx->bucketing && !(r.flags & kReqBandSplit) &&
                           rows >= kBucketMinRows && sh->row_prefix[i] + rows <= max_order_rows;
        sh->row_prefix[i + 1] = sh->row_prefix[i] + (group ? rows : 0);
        sh->chunk_prefix[i + 1] =
            sh->chunk_prefix[i] + (group ? (rows + kBucketChunk - 1) / kBucketChunk : 0);
    }
    sh->units = units;
    sh->max_p = max_p;
    sh->n_order = sh->row_prefix[n];
    sh->n_chunks = sh->chunk_prefix[n];
}

// Point each regrouped request at its segment of the row-order buffer.
static void set_order(std::vector<ReqDesc> &reqs, const LaunchShape &sh, uint32_t *order) {
    for (size_t i = 0; i < reqs.size(); ++i)
        reqs[i].order = sh.row_prefix[i + 1] > sh.row_prefix[i] ? order + sh.row_prefix[i] : nullptr;
}

SweepParams sweep_params(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const ReqDesc *req,
                         uint32_t n_req, uint64_t units, uint64_t surv_cap) {
    SweepParams P;
    memset(&P, 0, sizeof(P));
    P.K = ds.K;
    for (uint32_t k = 0; k < ds.K; ++k) {
        P.dr[k] = ds.dr[k]; P.dm[k] = ds.dm[k]; P.dinv[k] = ds.dinv[k]; P.doff[k] = ds.doff[k];
        P.dext[k] = ds.dext[k];
    }
    P.dense_words = ds.words;
    P.dense_tab = (const uint64_t *)ds.tab.p;
    P.wheel = (const uint64_t *)ctx->wheel.p;
    P.patterns = (const uint64_t *)ctx->patterns.p;
    P.n_deep = ds.n_deep;
    P.nc = ds.K + ds.n_deep;
    P.deep = (const DeepPrime *)ds.deep.p;
    P.vpool = (const uint8_t *)pl.vpool.p;
    P.ipool = (const uint16_t *)pl.ipool.p;
    P.req = req;
    P.n_req = n_req;
    P.n_units = units;
    P.counts = (unsigned long long *)ctx->counts.p;
    P.pairs = (unsigned long long *)ctx->pairs.p;
    P.n_rep = ctx->n_rep;
    P.rep_stride_counts = ctx->rep_stride_counts;
    P.rep_stride_pairs = ctx->rep_stride_pairs;
    P.surv = (SurvEntry *)ctx->surv.p;
    P.surv_cap = surv_cap;
    P.surv_n = (unsigned long long *)ctx->surv_n.p;
    P.claim = (unsigned long long *)ctx->surv_n.p + 1;
    return P;
}

// One sweep launch over `reqs` (already holding row pointers and counter
// slots), accumulating into the context's count / pair / survivor buffers
// (zeroed by the caller).
int launch_reqs(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const cuboid_tuning &tun,
                std::vector<ReqDesc> &reqs, uint64_t surv_cap, hipStream_t s,
                uint64_t *units_out) {
    const uint32_t n = (uint32_t)reqs.size();
    LaunchShape &sh = ctx->h_shape;
    shape_reqs(ctx, reqs, &sh);
    if (sh.n_order) HIPCHK(ctx->order.ensure(sh.n_order * 4));
    set_order(reqs, sh, (uint32_t *)ctx->order.p);
    // staged through pinned memory; the previous user of the staging buffer
    // on this stream has completed once the stream is idle
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(ctx->req_stage.ensure(n * sizeof(ReqDesc) + 2 * (n + 1) * 8));
    unsigned char *stage = (unsigned char *)ctx->req_stage.p;
    memcpy(stage, reqs.data(), n * sizeof(ReqDesc));
    HIPCHK(ctx->reqbuf.ensure(n * sizeof(ReqDesc)));
    HIPCHK(hipMemcpyAsync(ctx->reqbuf.p, stage, n * sizeof(ReqDesc), hipMemcpyHostToDevice, s));
    if (sh.n_order) {
        uint64_t *pre = (uint64_t *)(stage + n * sizeof(ReqDesc));
        memcpy(pre, sh.chunk_prefix.data(), (n + 1) * 8);
        memcpy(pre + n + 1, sh.row_prefix.data(), (n + 1) * 8);
        HIPCHK(ctx->chunk_prefix.ensure((n + 1) * 8));
        HIPCHK(ctx->row_prefix.ensure((n + 1) * 8));
        HIPCHK(hipMemcpyAsync(ctx->chunk_prefix.p, pre, (n + 1) * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(ctx->row_prefix.p, pre + n + 1, (n + 1) * 8, hipMemcpyHostToDevice, s));
        HIPCHK(launch_bucket_rows((const ReqDesc *)ctx->reqbuf.p, n,
                                  (const uint64_t *)ctx->chunk_prefix.p, sh.n_chunks,
                                  (const uint64_t *)ctx->row_prefix.p, (uint32_t *)ctx->order.p, s));
    }
    SweepParams P =
        sweep_params(ctx, pl, ds, (const ReqDesc *)ctx->reqbuf.p, n, sh.units, surv_cap);
    P.schedule = tun.schedule;
    P.piece = tun.piece_units;
    for (const ReqDesc &d : reqs) P.band_split |= (d.flags & kReqBandSplit) ? 1u : 0u;
    const size_t lds = (size_t)ds.words * 8 + kSweepFixedLds;
    if (lds > ctx->max_lds) return CUBOID_E_LIMIT;
    // a call may launch once per row window: each launch hands out its units
    // from a fresh claim counter
    HIPCHK(launch_fill_u64((uint64_t *)P.claim, 1, 0, s));
    if (ctx->timing) HIPCHK(hipEventRecord(ctx->ev_sweep0, s));
    HIPCHK(launch_sweep(P, (int)tun.workgroups, lds, sh.max_p, s));
    if (ctx->timing) HIPCHK(hipEventRecord(ctx->ev_sweep1, s));
    *units_out = sh.units;
    return CUBOID_OK;
}

int ensure_scratch(cuboid_ctx *ctx, uint32_t n_req, uint32_t nc, uint64_t surv_cap,
                   uint64_t units) {
    // counter replicas spread the end-of-wave atomics of one request over
    // several addresses: about one per 64 units of the launch (a small launch
    // has few waves to flush and its replicas would only cost summing), at
    // most 64 and as many as fit the budget
    uint32_t rep = 64;
    while (rep > 1 && (uint64_t)rep * 64 > units) rep >>= 1;
    while (rep > 1 && (uint64_t)rep * n_req * (nc + 1) * 8 > kReplicaBytes) rep >>= 1;
    ctx->n_rep = rep;
    ctx->rep_stride_counts = (uint64_t)n_req * nc;
    ctx->rep_stride_pairs = n_req;
    HIPCHK(ctx->counts.ensure((size_t)rep * n_req * nc * 8 + 8));
    HIPCHK(ctx->pairs.ensure((size_t)rep * n_req * 8 + 8));
    HIPCHK(ctx->surv_n.ensure(16));   // survivor count, claim counter
    const uint64_t rounded = (surv_cap + 1023) / 1024 * 1024;
    HIPCHK(ctx->surv.ensure(rounded * sizeof(SurvEntry) + sizeof(SurvEntry)));
    HIPCHK(ctx->surv_tmp.ensure(rounded * sizeof(SurvEntry) + sizeof(SurvEntry)));
    return CUBOID_OK;
}

int zero_scratch(cuboid_ctx *ctx, uint32_t n_req, uint32_t nc, hipStream_t s) {
    HIPCHK(launch_clear3((uint64_t *)ctx->counts.p, (uint64_t)ctx->n_rep * n_req * nc,
                         (uint64_t *)ctx->pairs.p, (uint64_t)ctx->n_rep * n_req,
                         (uint64_t *)ctx->surv_n.p, 1, s));
    return CUBOID_OK;
}

// Sorted survivor entries (n of them, n <= scratch) to host.
int fetch_survivors(cuboid_ctx *ctx, uint64_t n, std::vector<SurvEntry> *out, hipStream_t s) {
    out->resize(n);
    if (!n) return CUBOID_OK;
    SurvEntry *sorted = nullptr;
    HIPCHK(launch_sort_surv((SurvEntry *)ctx->surv.p, (SurvEntry *)ctx->surv_tmp.p,
                            (const unsigned long long *)ctx->surv_n.p, n, &sorted, s));
    HIPCHK(hipMemcpyAsync(out->data(), sorted, n * sizeof(SurvEntry), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return CUBOID_OK;
}

// Sorted survivors into the caller's device buffer (the first dev.surv_cap).
int place_survivors(cuboid_ctx *ctx, uint64_t n, const DevOut &dev, hipStream_t s) {
    SurvEntry *sorted = nullptr;
    HIPCHK(launch_sort_surv((SurvEntry *)ctx->surv.p, (SurvEntry *)ctx->surv_tmp.p,
                            (const unsigned long long *)ctx->surv_n.p, n, &sorted, s));
    const uint64_t k = std::min<uint64_t>(n, dev.surv_cap);
    static_assert(sizeof(SurvEntry) == 16, "survivor entry is two words");
    if (k) HIPCHK(launch_copy_u64((uint64_t *)dev.surv, (const uint64_t *)sorted, 2 * k, s));
    HIPCHK(hipStreamSynchronize(s));
    return CUBOID_OK;
}

// For each prime of the caller's list, its index among the plan's
// non-trivial primes (canonical counter slot), or -1 for a trivial prime.
std::vector<int32_t> count_columns(const Plan &pl, const std::vector<uint32_t> &caller) {
    std::vector<int32_t> col(caller.size(), -1);
    for (size_t i = 0; i < caller.size(); ++i) {
        const size_t pos =
            std::lower_bound(pl.primes.begin(), pl.primes.end(), caller[i]) - pl.primes.begin();
        if (pl.trivial[pos]) continue;
        col[i] = (int32_t)(std::lower_bound(pl.nontriv_idx.begin(), pl.nontriv_idx.end(),
                                            (uint32_t)pos) - pl.nontriv_idx.begin());
    }
    return col;
}

int rect_valid(uint32_t p0, uint32_t p1, uint32_t q0, uint32_t q1) {
    if (p0 == 0 || q0 == 0 || p0 > p1 || q0 > q1) return CUBOID_E_RANGE;
    return CUBOID_OK;
}

// The sweep over descriptors whose p0, p1, q0, q1, ip0, slot and flags are
// set; several descriptors may share a counter slot.  Rows come from the
// resident table when every p fits it (one graph replay when graphs are on),
// else from row windows of kBandRows rows computed on the fly, each
// descriptor split at window edges.
int sieve_core(cuboid_ctx *ctx, const Plan &pl, const DenseSet &ds, const cuboid_tuning &tun,
               std::vector<ReqDesc> &reqs, uint32_t n_slots, const std::vector<int32_t> *col,
               uint64_t surv_cap, hipStream_t s, CoreOut *out, const DevOut *dev) {
    const uint32_t nc = ds.K + ds.n_deep;
    if (dev && !col) return CUBOID_E_ARG;   // device results are in the caller's prime order
    // counters come back per slot either canonical (nc) or already in the
    // caller's prime order (col: the counter of each caller prime, -1 for a
    // trivial one), gathered on the device
    const uint32_t width = col ? (uint32_t)col->size() : nc;
    uint64_t units = 0;
    for (const ReqDesc &r : reqs)
        units += (((uint64_t)r.p1 - r.p0 + 64) / 64) * (((uint64_t)r.q1 - r.q0 + 64) / 64);
    int st = ensure_scratch(ctx, n_slots, nc, surv_cap, units);
    if (st) return st;
    uint32_t pmax = 0;
    for (auto &r : reqs) pmax = std::max(pmax, r.p1);
    const bool resident = pmax <= kResidentRowsMax;
    if (resident) {
        st = ensure_rows(ctx, pmax);
        if (st) return st;
    }
    out->units = 0;
    out->sweep_ms = 0;
    const size_t ncount = (size_t)n_slots * width;
    ctx->last_graph = 0;
    auto sweep_time = [&]() -> int {
        if (!ctx->timing) return CUBOID_OK;
        HIPCHK(hipEventSynchronize(ctx->ev_sweep1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_sweep0, ctx->ev_sweep1));
        out->sweep_ms += ms;
        return CUBOID_OK;
    };
    if (resident) {
        for (auto &d : reqs) {
            d.rows = (const RowInfo *)ctx->rows.p;
            d.nfac = (const uint8_t *)ctx->nfac.p;
            d.rows_p0 = 1;
        }
    }
    if (resident && ctx->use_graphs) {
        // clears, sweep, replica sums and downloads all inside the graph
        st = run_batch_graph(ctx, pl, ds, tun, reqs, n_slots, col, surv_cap, s, &out->units, dev);
        if (st) return st;
        HIPCHK(hipStreamSynchronize(s));
        st = sweep_time();
        if (st) return st;
    } else {
        st = zero_scratch(ctx, n_slots, nc, s);
        if (st) return st;
        if (resident) {
            st = launch_reqs(ctx, pl, ds, tun, reqs, surv_cap, s, &out->units);
            if (st) return st;
            st = sweep_time();
            if (st) return st;
        } else {
            // pieces of each descriptor per row window, windows in ascending p
            std::map<uint64_t, std::vector<ReqDesc>> win;
            for (const ReqDesc &d : reqs) {
                for (uint64_t a = d.p0; a <= d.p1;) {
                    const uint64_t w = (a - 1) / kBandRows;
                    const uint64_t b = std::min<uint64_t>(d.p1, (w + 1) * kBandRows);
                    ReqDesc piece = d;
                    piece.p0 = (uint32_t)a;
                    piece.p1 = (uint32_t)b;
                    win[w].push_back(piece);
                    a = b + 1;
                }
            }
            for (auto &kv : win) {
                std::vector<ReqDesc> &pieces = kv.second;
                uint32_t lo = 0xffffffffu, hi = 0;
                for (auto &d : pieces) { lo = std::min(lo, d.p0); hi = std::max(hi, d.p1); }
                const uint64_t nrows = (uint64_t)hi - lo + 1;
                HIPCHK(ctx->band_rows.ensure(nrows * sizeof(RowInfo)));
                HIPCHK(ctx->band_nfac.ensure(nrows));
                HIPCHK(launch_row_info((const uint32_t *)ctx->primes16.p,
                                       (const uint32_t *)ctx->magic16.p, ctx->n16, lo, nrows,
                                       (RowInfo *)ctx->band_rows.p, (uint8_t *)ctx->band_nfac.p, s));
                for (auto &d : pieces) {
                    d.rows = (const RowInfo *)ctx->band_rows.p;
                    d.nfac = (const uint8_t *)ctx->band_nfac.p;
                    d.rows_p0 = lo;
                }
                uint64_t units = 0;
                st = launch_reqs(ctx, pl, ds, tun, pieces, surv_cap, s, &units);
                if (st) return st;
                out->units += units;
                st = sweep_time();
                if (st) return st;
            }
        }
        // replica sums, the caller's prime order and the survivor count in
        // one kernel, into an output block [counts | pairs | survivor count]
        // that comes back in one copy (or counts and pairs into the caller's
        // device buffers, only the survivor count staged)
        if (col && width) {
            HIPCHK(ctx->colbuf.ensure(width * 4));
            HIPCHK(hipMemcpyAsync(ctx->colbuf.p, col->data(), width * 4, hipMemcpyHostToDevice, s));
        }
        const uint64_t small_sort = dev ? 0 : std::min<uint64_t>(kSmallSort, surv_cap);
        const size_t out_bytes = (ncount + n_slots + 1 + 2 * small_sort) * 8;
        HIPCHK(ctx->gathered.ensure(out_bytes));
        HIPCHK(ctx->result_stage.ensure(out_bytes));
        unsigned long long *ob = (unsigned long long *)ctx->gathered.p;
        unsigned long long *on = dev ? ob : ob + ncount + n_slots;
        HIPCHK(launch_finish((const unsigned long long *)ctx->counts.p,
                             (const unsigned long long *)ctx->pairs.p, ctx->n_rep,
                             ctx->rep_stride_counts, ctx->rep_stride_pairs,
                             col ? (const int32_t *)ctx->colbuf.p : nullptr, n_slots, nc, width,
                             dev ? (unsigned long long *)dev->counts : ob,
                             dev ? (unsigned long long *)dev->pairs : ob + ncount,
                             (const unsigned long long *)ctx->surv_n.p, on,
                             (const SurvEntry *)ctx->surv.p, small_sort, (SurvEntry *)(on + 1), s));
        uint64_t *rs = (uint64_t *)ctx->result_stage.p;
        if (dev)
            HIPCHK(hipMemcpyAsync(rs + ncount + n_slots, on, 8, hipMemcpyDeviceToHost, s));
        else
            HIPCHK(hipMemcpyAsync(rs, ob, out_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const uint64_t *stage = (const uint64_t *)ctx->result_stage.p;
    out->nc = nc;
    out->n_slots = n_slots;
    out->width = width;
    out->counts = dev ? nullptr : stage;
    out->pairs = dev ? nullptr : stage + ncount;
    out->n_surv = stage[ncount + n_slots];
    out->surv.clear();
    // with host results the finishing kernel has sorted and downloaded up to
    // kSmallSort survivors already, behind the survivor count
    const uint64_t sorted_small = dev ? 0 : std::min<uint64_t>(kSmallSort, surv_cap);
    if (out->n_surv > 0 && out->n_surv <= sorted_small) {
        const SurvEntry *e = (const SurvEntry *)(stage + ncount + n_slots + 1);
        out->surv.assign(e, e + out->n_surv);
    } else if (out->n_surv > 0 && out->n_surv <= surv_cap) {
        st = dev ? place_survivors(ctx, out->n_surv, *dev, s)
                 : fetch_survivors(ctx, out->n_surv, &out->surv, s);
        if (st) return st;
    }
    return CUBOID_OK;
}

// Canonical plan, tuning and dense tables of a caller's prime list.
int prepare_primes(cuboid_ctx *ctx, const std::vector<uint32_t> &caller_primes, Plan **pl,
                   cuboid_tuning *tun, DenseSet **ds) {
    std::vector<uint32_t> primes;
    int st = canonical_primes(caller_primes.data(), (uint32_t)caller_primes.size(), &primes);
    if (st) return st;
    st = build_plan(ctx, primes, pl);
    if (st) return st;
    *tun = tuning_for(ctx, primes, **pl);
    return build_dense(ctx, *pl, tun->dense_primes, ds);
}

void record_timing(cuboid_ctx *ctx, hipStream_t s, const CoreOut &co, const DenseSet &ds,
                   const cuboid_tuning &tun) {
    if (!ctx->timing) return;
    if (hipEventRecord(ctx->ev_total1, s) != hipSuccess) return;
    if (hipEventSynchronize(ctx->ev_total1) != hipSuccess) return;
    float ms = 0;
    if (hipEventElapsedTime(&ms, ctx->ev_total0, ctx->ev_total1) != hipSuccess) return;
    ctx->last.sweep_ms = co.sweep_ms;
    ctx->last.total_gpu_ms = ms;
    ctx->last.units = co.units;
    ctx->last.dense_primes = ds.K;
    ctx->last.workgroups = tun.workgroups;
    ctx->last.graph = ctx->last_graph;
}

// The plain and batched sieve share this path.  `rects` are validated.
int sieve_rects(cuboid_ctx *ctx, const std::vector<uint32_t> &caller_primes,
                const cuboid_request *rects, uint32_t n_req, uint64_t surv_cap_total,
                hipStream_t s, SieveOut *out, const DevOut *dev) {
    Plan *pl = nullptr;
    DenseSet *ds = nullptr;
    cuboid_tuning tun;
    int st = prepare_primes(ctx, caller_primes, &pl, &tun, &ds);
    if (st) return st;
    const uint64_t surv_cap = std::min<uint64_t>(surv_cap_total, kMaxSurvScratch);
    std::vector<ReqDesc> &reqs = ctx->h_reqs;
    reqs.resize(n_req);
    for (uint32_t i = 0; i < n_req; ++i) {
        ReqDesc &d = reqs[i];
        memset(&d, 0, sizeof(d));
        d.p0 = rects[i].p0; d.p1 = rects[i].p1; d.q0 = rects[i].q0; d.q1 = rects[i].q1;
        d.ip0 = rects[i].p0;
        d.slot = i;
    }
    if (ctx->timing) HIPCHK(hipEventRecord(ctx->ev_total0, s));
    const std::vector<int32_t> col = count_columns(*pl, caller_primes);
    CoreOut &co = ctx->h_core;
    st = sieve_core(ctx, *pl, *ds, tun, reqs, n_req, &col, surv_cap, s, &co, dev);
    if (st) return st;
    out->n_req = n_req;
    out->n_primes = (uint32_t)caller_primes.size();
    out->n_surv = co.n_surv;
    out->counts = co.counts;
    out->pairs = co.pairs;
    out->surv.assign(co.surv.begin(), co.surv.end());
    record_timing(ctx, s, co, *ds, tun);
    if (co.n_surv > surv_cap && surv_cap < surv_cap_total) return CUBOID_E_LIMIT;
    return CUBOID_OK;
}

}  // namespace cuboid
