// extern "C" entry points of libcuboid (declared in include/cuboid.h).
#include <string.h>

#include <algorithm>
#include <string>

#include "bigint.h"
#include "runtime.h"

using namespace cuboid;

#define HIPCHK(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return CUBOID_E_DEVICE; \
    } while (0)

namespace {

// Handles given to callers are opaque tokens, not addresses: a slot of the
// table below and the generation the slot had when the context was created
// there.  A handle of a destroyed context never matches again (its slot's
// generation has moved on), so stale handles are refused even when a new
// context reuses the slot or the old context's memory.  Every entry point
// holds a reference on the context for the length of the call (CtxRef); it
// is taken under g_ctx_mu while the context is in the table, and
// cuboid_destroy removes the context under the same lock only when no
// reference is held, so a call can never see its context freed under it.
constexpr uint32_t kSlots = 4096;
struct Slot {
    cuboid_ctx *ctx = nullptr;
    uint32_t gen = 0;
    uint32_t refs = 0;
};
std::mutex g_ctx_mu;
Slot g_slots[kSlots];

uintptr_t make_handle(uint32_t slot, uint32_t gen) {
    return ((uintptr_t)gen << 16 | (slot + 1)) << 4;
}

Slot *find_slot(cuboid_ctx *handle) {   // under g_ctx_mu
    const uintptr_t h = (uintptr_t)handle;
    if (!h || (h & 15)) return nullptr;
    const uint32_t slot = (uint32_t)((h >> 4) & 0xffff);
    if (slot == 0 || slot > kSlots) return nullptr;
    Slot &s = g_slots[slot - 1];
    if (!s.ctx || make_handle(slot - 1, s.gen) != h) return nullptr;
    return &s;
}

}  // namespace

namespace cuboid {

CtxRef::CtxRef(cuboid_ctx *handle) {
    std::lock_guard<std::mutex> g(g_ctx_mu);
    Slot *s = find_slot(handle);
    if (!s) return;
    ++s->refs;
    ctx_ = s->ctx;
    slot_ = (uint32_t)(s - g_slots);
}

CtxRef::~CtxRef() {
    if (!ctx_) return;
    std::lock_guard<std::mutex> g(g_ctx_mu);
    --g_slots[slot_].refs;
}

}  // namespace cuboid

namespace {

int set_device(cuboid_ctx *ctx) {
    return hipSetDevice(ctx->device) == hipSuccess ? CUBOID_OK : CUBOID_E_DEVICE;
}

std::vector<uint32_t> small_primes_below_2_16() {
    std::vector<uint8_t> comp(65536, 0);
    std::vector<uint32_t> out;
    for (uint32_t i = 2; i < 65536; ++i) {
        if (comp[i]) continue;
        out.push_back(i);
        for (uint64_t j = (uint64_t)i * i; j < 65536; j += i) comp[j] = 1;
    }
    return out;
}

int init_ctx(cuboid_ctx *ctx, int dev) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return CUBOID_E_DEVICE;
    if (dev < 0 || dev >= ndev) return CUBOID_E_DEVICE;
    ctx->device = dev;
    HIPCHK(hipSetDevice(dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    strncpy(ctx->arch, prop.gcnArchName, sizeof(ctx->arch) - 1);
    if (strncmp(ctx->arch, "gfx950", 6) != 0) return CUBOID_E_DEVICE;
    ctx->cu_count = prop.multiProcessorCount;
    int lds = 0;
    HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    ctx->max_lds = (size_t)lds;
    HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&ctx->ev_sweep0));
    HIPCHK(hipEventCreate(&ctx->ev_sweep1));
    HIPCHK(hipEventCreate(&ctx->ev_total0));
    HIPCHK(hipEventCreate(&ctx->ev_total1));
    const std::vector<uint32_t> pr = small_primes_below_2_16();
    std::vector<uint32_t> mg(pr.size());
    for (size_t i = 0; i < pr.size(); ++i) mg[i] = (uint32_t)(0x100000000ull / pr[i]);
    ctx->n16 = (uint32_t)pr.size();
    HIPCHK(ctx->primes16.ensure(pr.size() * 4));
    HIPCHK(ctx->magic16.ensure(mg.size() * 4));
    HIPCHK(hipMemcpy(ctx->primes16.p, pr.data(), pr.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->magic16.p, mg.data(), mg.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(ctx->wheel.ensure(kWheelBytes));
    HIPCHK(launch_wheel((uint64_t *)ctx->wheel.p, ctx->stream));
    HIPCHK(ctx->patterns.ensure(kPatBytes));
    HIPCHK(launch_patterns((uint64_t *)ctx->patterns.p, ctx->stream));
    HIPCHK(noalloc_scratch_setup(dev));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CUBOID_OK;
}

void free_ctx(cuboid_ctx *ctx) {
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx);
    if (ctx->ev_sweep0) (void)hipEventDestroy(ctx->ev_sweep0);
    if (ctx->ev_sweep1) (void)hipEventDestroy(ctx->ev_sweep1);
    if (ctx->ev_total0) (void)hipEventDestroy(ctx->ev_total0);
    if (ctx->ev_total1) (void)hipEventDestroy(ctx->ev_total1);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // namespace

extern "C" {

const char *cuboid_status_string(int status) { return status_text(status); }

const char *cuboid_version(void) { return "0.1.0 gfx950"; }

int cuboid_create(cuboid_ctx **out, int hip_device) {
    if (!out) return CUBOID_E_ARG;
    *out = nullptr;
    cuboid_ctx *ctx = new cuboid_ctx();
    const int st = init_ctx(ctx, hip_device);
    if (st != CUBOID_OK) {
        free_ctx(ctx);
        return st;
    }
    std::lock_guard<std::mutex> g(g_ctx_mu);
    for (uint32_t i = 0; i < kSlots; ++i) {
        Slot &s = g_slots[i];
        if (s.ctx) continue;
        s.gen = (s.gen + 1) & 0xffffffu;   // 24 bits of generation per slot
        s.ctx = ctx;
        s.refs = 0;
        *out = (cuboid_ctx *)make_handle(i, s.gen);
        return CUBOID_OK;
    }
    free_ctx(ctx);
    return CUBOID_E_LIMIT;
}

int cuboid_destroy(cuboid_ctx *handle) {
    cuboid_ctx *ctx = nullptr;
    {
        std::lock_guard<std::mutex> g(g_ctx_mu);
        Slot *s = find_slot(handle);
        if (!s) return CUBOID_E_NOT_LOADED;
        ctx = s->ctx;
        // a call in progress (or waiting for the context), a server or a search
        if (s->refs > 0 || ctx->servers.load() > 0 || ctx->searches.load() > 0)
            return CUBOID_E_BUSY;
        s->ctx = nullptr;   // no new reference can be taken from here on
    }
    free_ctx(ctx);
    return CUBOID_OK;
}

int cuboid_q_mod_prime(cuboid_ctx *ctx, const uint32_t *p, const uint32_t *q, const uint32_t *t,
                       const uint32_t *r, uint64_t n, uint32_t *out) {
    CTX_ENTER(ctx);
    if (n == 0) return CUBOID_OK;
    if (!p || !q || !t || !r || !out) return CUBOID_E_ARG;
    for (uint64_t i = 0; i < n; ++i)
        if (r[i] < 2 || r[i] >= 65536) return CUBOID_E_ARG;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    DevBuf d;
    HIPCHK(d.ensure(n * 4 * 5));
    uint32_t *dp = (uint32_t *)d.p, *dq = dp + n, *dt = dq + n, *dr = dt + n, *dout = dr + n;
    hipStream_t s = ctx->stream;
    HIPCHK(hipMemcpyAsync(dp, p, n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dq, q, n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dt, t, n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dr, r, n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(launch_q_eval(dp, dq, dt, dr, n, dout, s));
    HIPCHK(hipMemcpyAsync(out, dout, n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return CUBOID_OK;
}

int cuboid_table_bytes(cuboid_ctx *ctx, uint32_t r, uint8_t *out, size_t cap, size_t *written) {
    CTX_ENTER(ctx);
    if (!written) return CUBOID_E_ARG;
    if (r >= 65536 || !is_prime_u32(r)) return CUBOID_E_PRIMES;
    const size_t nbytes = ((size_t)r * r + 7) / 8;
    *written = nbytes;
    if (cap < nbytes) return CUBOID_E_CAPACITY;
    if (!out) return CUBOID_E_ARG;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    Plan *pl = nullptr;
    const std::vector<uint32_t> one(1, r);
    int st = build_plan(ctx, one, &pl);
    if (st) return st;
    DevBuf d;
    HIPCHK(d.ensure(nbytes));
    HIPCHK(launch_pack_table(r, (const uint8_t *)pl->vpool.p, (const uint16_t *)pl->ipool.p,
                             (uint8_t *)d.p, ctx->stream));
    HIPCHK(hipMemcpyAsync(out, d.p, nbytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CUBOID_OK;
}

int cuboid_sieve_range(cuboid_ctx *ctx, uint32_t p0, uint32_t p1, uint32_t q0, uint32_t q1,
                       const uint32_t *primes, uint32_t n_primes, uint64_t *survivors,
                       uint64_t cap, uint64_t *n_survivors, uint64_t *counts, uint64_t *n_pairs,
                       void *hip_stream) {
    CTX_ENTER(ctx);
    if (!n_survivors || !counts || !n_pairs || (cap && !survivors)) return CUBOID_E_ARG;
    int st = rect_valid(p0, p1, q0, q1);
    if (st) return st;
    std::vector<uint32_t> sorted;
    st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    const std::vector<uint32_t> caller(primes, primes + n_primes);
    cuboid_request rect;
    rect.p0 = p0; rect.p1 = p1; rect.q0 = q0; rect.q1 = q1;
    SieveOut &so = ctx->h_out;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    st = sieve_rects(ctx, caller, &rect, 1, cap, s, &so);
    if (st) return st;
    memcpy(counts, so.counts, n_primes * 8);
    *n_pairs = so.pairs[0];
    *n_survivors = so.n_surv;
    if (so.n_surv > cap) return CUBOID_E_CAPACITY;
    for (uint64_t i = 0; i < so.n_surv; ++i) survivors[i] = so.surv[i].idx;
    return CUBOID_OK;
}

int cuboid_sieve_region(cuboid_ctx *ctx, uint32_t p0, uint32_t p1, uint32_t band_rows,
                        const uint32_t *primes, uint32_t n_primes, uint64_t *survivors,
                        uint64_t cap, uint64_t *n_survivors, uint64_t *counts, uint64_t *n_pairs,
                        uint32_t *r_max, void *hip_stream) {
    CTX_ENTER(ctx);
    if (!n_survivors || !counts || !n_pairs || (cap && !survivors) || band_rows == 0)
        return CUBOID_E_ARG;
    if (p0 == 0 || p0 > p1) return CUBOID_E_RANGE;
    if (p1 > kRegionMaxP) return CUBOID_E_LIMIT;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    const std::vector<uint32_t> caller(primes, primes + n_primes);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    return region_sieve(ctx, p0, p1, band_rows, caller, survivors, cap, n_survivors, counts,
                        n_pairs, r_max, s);
}

int cuboid_sieve_batch(cuboid_ctx *ctx, const cuboid_request *req, uint32_t n_req,
                       const uint32_t *primes, uint32_t n_primes, cuboid_result *res,
                       void *hip_stream) {
    CTX_ENTER(ctx);
    if (!req || !res || n_req == 0 || n_req == 0xffffffffu) return CUBOID_E_ARG;
    int bad = 0;
    uint64_t cap_total = 0;
    for (uint32_t i = 0; i < n_req; ++i) {
        if (!res[i].counts || (res[i].cap && !res[i].survivors)) return CUBOID_E_ARG;
        res[i].status = rect_valid(req[i].p0, req[i].p1, req[i].q0, req[i].q1);
        if (res[i].status) bad = 1;
        cap_total += res[i].cap;
    }
    if (bad) return CUBOID_E_RANGE;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    const std::vector<uint32_t> caller(primes, primes + n_primes);
    SieveOut &so = ctx->h_out;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    // a request may hold more survivors than its own cap while the total fits;
    // the device list holds up to the sum of the caps
    st = sieve_rects(ctx, caller, req, n_req, cap_total, s, &so);
    if (st && st != CUBOID_E_LIMIT) return st;
    if (st == CUBOID_OK && so.n_surv > cap_total && so.n_surv <= kMaxSurvScratch) {
        // some request holds more survivors than its cap: run again with room
        // for all of them so every other request still gets its full list
        st = sieve_rects(ctx, caller, req, n_req, so.n_surv, s, &so);
        if (st && st != CUBOID_E_LIMIT) return st;
    }
    for (uint32_t i = 0; i < n_req; ++i) {
        memcpy(res[i].counts, so.counts + (size_t)i * n_primes, n_primes * 8);
        res[i].n_pairs = so.pairs[i];
    }
    if (st == CUBOID_E_LIMIT || so.surv.size() != so.n_surv) {
        // survivors beyond what the device list holds: numbers only, from the
        // conservation law sum(counts) + survivors = pairs
        for (uint32_t i = 0; i < n_req; ++i) {
            uint64_t sc = 0;
            for (uint32_t k = 0; k < n_primes; ++k) sc += so.counts[(size_t)i * n_primes + k];
            res[i].n_survivors = so.pairs[i] - sc;
            res[i].status = res[i].n_survivors > res[i].cap ? CUBOID_E_CAPACITY : CUBOID_E_LIMIT;
        }
        return CUBOID_E_LIMIT;
    }
    std::vector<uint64_t> per(n_req, 0);
    for (const SurvEntry &e : so.surv) per[e.req]++;
    int any_cap = 0;
    size_t k = 0;
    for (uint32_t i = 0; i < n_req; ++i) {
        res[i].n_survivors = per[i];
        if (per[i] > res[i].cap) {
            res[i].status = CUBOID_E_CAPACITY;
            any_cap = 1;
            k += per[i];
            continue;
        }
        res[i].status = CUBOID_OK;
        for (uint64_t j = 0; j < per[i]; ++j) res[i].survivors[j] = so.surv[k++].idx;
    }
    return any_cap ? CUBOID_E_CAPACITY : CUBOID_OK;
}

int cuboid_sieve_batch_dev(cuboid_ctx *ctx, const cuboid_request *req, uint32_t n_req,
                           const uint32_t *primes, uint32_t n_primes, uint64_t *counts_dev,
                           uint64_t *pairs_dev, void *survivors_dev, uint64_t surv_cap,
                           uint64_t *n_survivors, void *hip_stream) {
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
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    const std::vector<uint32_t> caller(primes, primes + n_primes);
    SieveOut &so = ctx->h_out;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    DevOut dev;
    dev.counts = counts_dev;
    dev.pairs = pairs_dev;
    dev.surv = (SurvEntry *)survivors_dev;
    dev.surv_cap = surv_cap;
    // the survivor scratch holds the caller's capacity; when more survive
    // (within the device scratch) the call runs again with room for all, so
    // that the first surv_cap in (request, index) order are the right ones
    st = sieve_rects(ctx, caller, req, n_req, std::max<uint64_t>(surv_cap, 1), s, &so, &dev);
    if (st && st != CUBOID_E_LIMIT) return st;
    if (so.n_surv > std::max<uint64_t>(surv_cap, 1) && so.n_surv <= kMaxSurvScratch) {
        st = sieve_rects(ctx, caller, req, n_req, so.n_surv, s, &so, &dev);
        if (st && st != CUBOID_E_LIMIT) return st;
    }
    *n_survivors = so.n_surv;
    if (st == CUBOID_E_LIMIT || so.n_surv > kMaxSurvScratch) return CUBOID_E_LIMIT;
    return so.n_surv > surv_cap ? CUBOID_E_CAPACITY : CUBOID_OK;
}

int cuboid_device_alloc(cuboid_ctx *ctx, size_t bytes, void **out) {
    if (!out) return CUBOID_E_ARG;
    *out = nullptr;
    CTX_ENTER(ctx);
    if (bytes == 0) return CUBOID_E_ARG;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    return hipMalloc(out, bytes) == hipSuccess ? CUBOID_OK : CUBOID_E_DEVICE;
}

int cuboid_device_free(cuboid_ctx *ctx, void *p) {
    CTX_ENTER(ctx);
    if (!p) return CUBOID_OK;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    // work of this context that may still read the buffer ends first
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return CUBOID_E_DEVICE;
    return hipFree(p) == hipSuccess ? CUBOID_OK : CUBOID_E_DEVICE;
}

int cuboid_device_read(cuboid_ctx *ctx, void *dst, const void *src_dev, size_t bytes,
                       void *hip_stream) {
    CTX_ENTER(ctx);
    if (bytes && (!dst || !src_dev)) return CUBOID_E_ARG;
    if (!bytes) return CUBOID_OK;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    if (hipMemcpyAsync(dst, src_dev, bytes, hipMemcpyDeviceToHost, s) != hipSuccess)
        return CUBOID_E_DEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? CUBOID_OK : CUBOID_E_DEVICE;
}

int cuboid_probe_peaks(cuboid_ctx *ctx, double *valu_lane_ops_per_s, double *lds_bytes_per_s) {
    if (!valu_lane_ops_per_s || !lds_bytes_per_s) return CUBOID_E_ARG;
    CTX_ENTER(ctx);
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    return run_peak_probes(ctx->cu_count, ctx->stream, valu_lane_ops_per_s, lds_bytes_per_s) ==
                   hipSuccess
               ? CUBOID_OK
               : CUBOID_E_DEVICE;
}

int cuboid_canonical_primes(const uint32_t *primes, uint32_t n, uint32_t *sorted_out,
                            uint8_t *trivial_out) {
    if (!sorted_out) return CUBOID_E_ARG;
    std::vector<uint32_t> s;
    const int st = canonical_primes(primes, n, &s);
    if (st) return st;
    for (uint32_t i = 0; i < n; ++i) {
        sorted_out[i] = s[i];
        if (trivial_out) trivial_out[i] = (s[i] == 2 || s[i] == 3 || s[i] == 5 || s[i] == 7);
    }
    return CUBOID_OK;
}

int cuboid_exact_check(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, int *is_root,
                       uint32_t *flags) {
    if (!is_root || !flags) return CUBOID_E_ARG;
    bool ok = true;
    const bool z = exact_is_root(p, q, t_lo, t_hi, &ok);
    if (!ok) return CUBOID_E_LIMIT;
    *is_root = z ? 1 : 0;
    *flags = theorem_flags(p, q, t_lo, t_hi);
    return CUBOID_OK;
}

int cuboid_exact_value(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, char *out,
                       size_t cap) {
    if (!out) return CUBOID_E_ARG;
    std::string v;
    if (!exact_value_decimal(p, q, t_lo, t_hi, &v)) return CUBOID_E_LIMIT;
    if (v.size() + 1 > cap) return CUBOID_E_CAPACITY;
    memcpy(out, v.c_str(), v.size() + 1);
    return CUBOID_OK;
}

int cuboid_root_check(cuboid_ctx *ctx, const uint32_t *p, const uint32_t *q, uint64_t n,
                      cuboid_root *roots, uint64_t cap, uint64_t *n_roots) {
    CTX_ENTER(ctx);
    if (!n_roots || (n && (!p || !q)) || (cap && !roots)) return CUBOID_E_ARG;
    *n_roots = 0;
    if (n == 0) return CUBOID_OK;
    if (n >= (1ull << 32)) return CUBOID_E_LIMIT;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    hipStream_t s = ctx->stream;
    DevBuf dpq, dcand, dpre, dhits, dnh;
    HIPCHK(dpq.ensure(n * 8));
    HIPCHK(dcand.ensure(n * sizeof(RootCand)));
    uint32_t *dp = (uint32_t *)dpq.p, *dq = dp + n;
    HIPCHK(hipMemcpyAsync(dp, p, n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dq, q, n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(launch_root_factor(dp, dq, n, (const uint32_t *)ctx->primes16.p,
                              (const uint32_t *)ctx->magic16.p, ctx->n16, (RootCand *)dcand.p, s));
    std::vector<RootCand> cand(n);
    HIPCHK(hipMemcpyAsync(cand.data(), dcand.p, n * sizeof(RootCand), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<uint64_t> pre(n + 1, 0);
    for (uint64_t i = 0; i < n; ++i) {
        if (cand[i].ndiv > (1ull << 40)) return CUBOID_E_LIMIT;
        pre[i + 1] = pre[i] + cand[i].ndiv;
    }
    HIPCHK(dpre.ensure((n + 1) * 8));
    HIPCHK(hipMemcpyAsync(dpre.p, pre.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
    uint64_t hit_cap = 1 << 16;
    std::vector<RootHit> hits;
    for (int attempt = 0; attempt < 2; ++attempt) {
        HIPCHK(dhits.ensure(hit_cap * sizeof(RootHit)));
        HIPCHK(dnh.ensure(8));
        HIPCHK(launch_fill_u64((uint64_t *)dnh.p, 1, 0, s));
        const uint64_t chunk = 1ull << 30;
        for (uint64_t w0 = 0; w0 < pre[n]; w0 += chunk) {
            const uint64_t nw = std::min(chunk, pre[n] - w0);
            HIPCHK(launch_root_eval((const RootCand *)dcand.p, n, (const uint64_t *)dpre.p, w0, nw,
                                    (RootHit *)dhits.p, hit_cap, (unsigned long long *)dnh.p, s));
        }
        uint64_t nh = 0;
        HIPCHK(hipMemcpyAsync(&nh, dnh.p, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (nh > hit_cap) { hit_cap = nh; continue; }
        hits.resize(nh);
        if (nh) {
            HIPCHK(hipMemcpyAsync(hits.data(), dhits.p, nh * sizeof(RootHit), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        break;
    }
    // exact confirmation on the CPU
    std::vector<cuboid_root> found;
    for (const RootHit &h : hits) {
        const RootCand &c = cand[h.cand];
        bool ok = true;
        if (!exact_is_root(c.p, c.q, h.t_lo, h.t_hi, &ok)) {
            if (!ok) return CUBOID_E_LIMIT;
            continue;
        }
        cuboid_root r;
        r.p = c.p; r.q = c.q; r.t = h.t_lo; r.t_hi = h.t_hi;
        r.flags = theorem_flags(c.p, c.q, h.t_lo, h.t_hi);
        r.input_index = h.cand;
        found.push_back(r);
    }
    std::sort(found.begin(), found.end(), [](const cuboid_root &a, const cuboid_root &b) {
        if (a.input_index != b.input_index) return a.input_index < b.input_index;
        return a.t_hi < b.t_hi || (a.t_hi == b.t_hi && a.t < b.t);
    });
    *n_roots = found.size();
    if (found.size() > cap) return CUBOID_E_CAPACITY;
    for (size_t i = 0; i < found.size(); ++i) roots[i] = found[i];
    return CUBOID_OK;
}

int cuboid_enable_timing(cuboid_ctx *ctx, int on) {
    CTX_ENTER(ctx);
    CtxLock g(ctx);
    ctx->timing = on != 0;
    return CUBOID_OK;
}

int cuboid_enable_graphs(cuboid_ctx *ctx, int on) {
    CTX_ENTER(ctx);
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    ctx->use_graphs = on != 0;
    if (!ctx->use_graphs) drop_graphs(ctx);
    return CUBOID_OK;
}

int cuboid_last_timing(cuboid_ctx *ctx, cuboid_timing *out) {
    CTX_ENTER(ctx);
    if (!out) return CUBOID_E_ARG;
    CtxLock g(ctx);
    *out = ctx->last;
    return CUBOID_OK;
}

int cuboid_set_tuning(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                      const cuboid_tuning *tuning) {
    CTX_ENTER(ctx);
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (!tuning) { ctx->tunings.erase(sorted); return CUBOID_OK; }
    if (tuning->dense_primes > (uint32_t)kKMax && tuning->dense_primes != 0xffffffffu)
        return CUBOID_E_ARG;
    if (tuning->schedule > 3) return CUBOID_E_ARG;
    if (tuning->piece_units > (1u << 20)) return CUBOID_E_ARG;
    ctx->tunings[sorted] = *tuning;
    return CUBOID_OK;
}

int cuboid_get_tuning(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                      cuboid_tuning *out) {
    CTX_ENTER(ctx);
    if (!out) return CUBOID_E_ARG;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (set_device(ctx)) return CUBOID_E_DEVICE;
    Plan *pl = nullptr;
    st = build_plan(ctx, sorted, &pl);
    if (st) return st;
    *out = tuning_for(ctx, sorted, *pl);
    return CUBOID_OK;
}

}  // extern "C"
