// Served form: a worker thread running continuous batching over the sieve
// sweep (see cuboid_server_* in include/cuboid.h).
//
// Each admitted request owns a counter slot (all replicas) and, when it has
// enough rows, a row-order buffer in a device arena, and is pinned to one of
// S streams so that all its launches are ordered.  A launch on a stream takes
// up to max_launch_units units from that stream's admitted requests in FIFO
// order; it first zeroes the slots of requests starting in it and regroups
// their rows, then sweeps, then sums the replicas of the requests finishing in
// it and copies their counters and the launch's survivors to pinned memory,
// and records an event.  The worker polls events, hands results to tickets,
// admits pending requests as slots and arena space free up, and refills idle
// streams, so requests arriving while others run join the next launch.
// A launch whose survivors overflow its stream's survivor pool is swept again
// (same units, counters into a discarded buffer) with the pool grown to hold
// them all, so every request still gets its complete list.  Requests with
// rows beyond the resident row table (p above 2^24) get their rows' factor
// lists computed into the arena at their first launch.
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "runtime.h"

using namespace cuboid;

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator of byte ranges in one device buffer.
struct Arena {
    std::map<uint64_t, uint64_t> free_;   // offset -> size
    void init(uint64_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(uint64_t size, uint64_t *off) {
        size = (size + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= size) {
                *off = it->first;
                const uint64_t rest = it->second - size, roff = it->first + size;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t size) {
        size = (size + 255) & ~255ull;
        auto it = free_.emplace(off, size).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct SrvReq {
    cuboid_request rect;
    uint64_t units_total = 0, units_issued = 0;
    uint32_t nrb = 0, nwin = 0;
    uint32_t slot = 0;
    int stream = -1;
    bool has_order = false;
    uint64_t order_off = 0, order_bytes = 0;
    bool own_rows = false;            // rows beyond the resident table:
    uint64_t rows_off = 0, rows_bytes = 0;   // RowInfo[rows] then nfac[rows] in the arena
    std::vector<SurvEntry> surv;
    std::vector<uint64_t> counts;     // caller order, when done
    uint64_t n_pairs = 0;
    int status = CUBOID_OK;
    bool done = false;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
};

constexpr uint64_t kSurvPool = 1u << 16;      // survivors per launch held on the device, at first
constexpr uint64_t kSurvCopy = 1024;          // copied back with every launch

struct StreamState {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::deque<uint64_t> queue;               // admitted tickets with units left, FIFO
    uint64_t queued_units = 0;
    std::vector<uint64_t> launch_tickets, final_tickets;
    DevBuf reqbuf, aux, out_dev, surv, surv_n;
    HostBuf stage, out_host;
    uint64_t surv_cap = kSurvPool;            // entries of surv (grows on overflow)
    // the last launch's descriptors (in reqbuf), for a survivor re-sweep
    uint32_t last_n = 0;
    uint64_t last_units = 0;
    size_t last_desc_off = 0;
    uint32_t last_max_p = 0;
};

// bytes of a request's own row table: RowInfo per row, then one factor count
// byte per row
uint64_t own_rows_bytes(uint64_t rows) {
    return ((rows * sizeof(RowInfo) + 255) & ~255ull) + rows;
}

}  // namespace

struct cuboid_server {
    cuboid_ctx *ctx = nullptr;
    std::vector<uint32_t> caller, sorted;
    Plan *pl = nullptr;
    DenseSet *ds = nullptr;
    cuboid_tuning tun;
    uint32_t nc = 0;
    std::vector<int32_t> col;
    cuboid_server_config cfg;
    uint32_t n_rep = 1;
    DevBuf counts, pairs, arena_buf;
    Arena arena;
    std::vector<uint32_t> free_slots;
    std::vector<uint64_t> slot_owner;
    std::vector<std::unique_ptr<StreamState>> streams;
    DevBuf discard_counts, discard_pairs;     // counters of survivor re-sweeps
    std::mutex mu;
    std::condition_variable cv_done, cv_work;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, SrvReq> reqs;
    uint64_t next_ticket = 1;
    uint32_t admitted = 0;
    bool stopping = false;
    int fatal = CUBOID_OK;
    cuboid_server_stats stats;
    std::thread worker;
};

namespace {

#define SRVCHK(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return CUBOID_E_DEVICE;  \
    } while (0)

bool all_idle(cuboid_server *S) {
    for (auto &st : S->streams)
        if (st->busy) return false;
    return true;
}

// Pending requests become admitted while slots, arena space and resident
// rows allow; each goes to the stream with the least queued work.
void admit(cuboid_server *S) {
    cuboid_ctx *ctx = S->ctx;
    while (!S->pending.empty()) {
        const uint64_t t = S->pending.front();
        SrvReq &r = S->reqs[t];
        if (S->free_slots.empty()) return;
        const uint64_t rows = (uint64_t)r.rect.p1 - r.rect.p0 + 1;
        r.own_rows = r.rect.p1 > kResidentRowsMax;
        if (r.own_rows) {
            r.rows_bytes = own_rows_bytes(rows);
            if (r.rows_bytes > S->cfg.hbm_budget_bytes) {
                // its row table alone is larger than the whole arena
                r.status = CUBOID_E_LIMIT; r.done = true; r.t_done = now_ns();
                r.counts.assign(S->caller.size(), 0);
                S->pending.pop_front();
                S->cv_done.notify_all();
                continue;
            }
        } else if (r.rect.p1 > ctx->rows_R) {
            // grow the resident row table only while nothing is in flight
            if (!all_idle(S)) return;
            int st;
            {
                CtxLock g(ctx);
                st = ensure_rows_serving(ctx, r.rect.p1);
            }
            if (st) {
                r.status = st; r.done = true; r.t_done = now_ns();
                r.counts.assign(S->caller.size(), 0);
                S->pending.pop_front();
                S->cv_done.notify_all();
                continue;
            }
        }
        if (r.own_rows && !S->arena.alloc(r.rows_bytes, &r.rows_off)) return;
        r.has_order = rows >= kBucketMinRows;
        if (r.has_order) {
            r.order_bytes = rows * 4;
            if (!S->arena.alloc(r.order_bytes, &r.order_off)) {
                if (S->admitted == 0 && all_idle(S)) {
                    // larger than the whole arena: run it in row order
                    r.has_order = false;
                } else {
                    if (r.own_rows) S->arena.release(r.rows_off, r.rows_bytes);
                    return;
                }
            }
        }
        r.slot = S->free_slots.back();
        S->free_slots.pop_back();
        S->slot_owner[r.slot] = t;
        int best = 0;
        for (int i = 1; i < (int)S->streams.size(); ++i)
            if (S->streams[i]->queued_units < S->streams[best]->queued_units) best = i;
        r.stream = best;
        S->streams[best]->queue.push_back(t);
        S->streams[best]->queued_units += r.units_total;
        r.t_admit = now_ns();
        S->pending.pop_front();
        ++S->admitted;
        S->stats.max_admitted = std::max(S->stats.max_admitted, S->admitted);
    }
}

// The sweep of the stream's last launch (its descriptors in st.reqbuf) with
// counters into cnt/prs (n_rep replicas) and survivors into st.surv.
hipError_t sweep_last(cuboid_server *S, StreamState &st, unsigned long long *cnt,
                      unsigned long long *prs, uint32_t n_rep) {
    cuboid_ctx *ctx = S->ctx;
    SweepParams P;
    memset(&P, 0, sizeof(P));
    const DenseSet &ds = *S->ds;
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
    P.nc = S->nc;
    P.deep = (const DeepPrime *)ds.deep.p;
    P.vpool = (const uint8_t *)S->pl->vpool.p;
    P.ipool = (const uint16_t *)S->pl->ipool.p;
    P.req = (const ReqDesc *)((unsigned char *)st.reqbuf.p + st.last_desc_off);
    P.n_req = st.last_n;
    P.n_units = st.last_units;
    P.counts = cnt;
    P.pairs = prs;
    P.n_rep = n_rep;
    P.rep_stride_counts = (uint64_t)S->cfg.max_slots * S->nc;
    P.rep_stride_pairs = S->cfg.max_slots;
    P.surv = (SurvEntry *)st.surv.p;
    P.surv_cap = st.surv_cap;
    P.surv_n = (unsigned long long *)st.surv_n.p;
    P.claim = (unsigned long long *)st.surv_n.p + 1;
    P.schedule = S->tun.schedule;
    P.piece = S->tun.piece_units;
    const size_t lds = (size_t)ds.words * 8 + kSweepFixedLds;
    return launch_sweep(P, (int)S->tun.workgroups, lds, st.last_max_p, st.s);
}

// Builds and enqueues one launch on an idle stream.
int launch(cuboid_server *S, StreamState &st) {
    cuboid_ctx *ctx = S->ctx;
    std::vector<ReqDesc> descs, bdescs;
    std::vector<uint32_t> new_slots, final_slots;
    // chunk_pre: prefix of bucketing chunks over the requests starting in this
    // launch; row_pre[i]: start of request i's row order, in uint32 elements
    // from the arena base (the kernel reads entry i for request i)
    std::vector<uint64_t> chunk_pre(1, 0), row_pre;
    st.launch_tickets.clear();
    st.final_tickets.clear();
    uint64_t budget = S->cfg.max_launch_units, unit0 = 0;
    while (budget && !st.queue.empty()) {
        const uint64_t t = st.queue.front();
        SrvReq &r = S->reqs[t];
        const uint64_t take = std::min(r.units_total - r.units_issued, budget);
        ReqDesc d;
        memset(&d, 0, sizeof(d));
        d.p0 = r.rect.p0; d.p1 = r.rect.p1; d.q0 = r.rect.q0; d.q1 = r.rect.q1;
        d.nrb = r.nrb; d.nwin = r.nwin;
        d.unit0 = unit0;
        d.ulo = r.units_issued;
        d.ucount = take;
        d.slot = r.slot;
        if (r.own_rows) {
            uint8_t *base = (uint8_t *)S->arena_buf.p + r.rows_off;
            const uint64_t rows = (uint64_t)r.rect.p1 - r.rect.p0 + 1;
            d.rows = (const RowInfo *)base;
            d.nfac = base + ((rows * sizeof(RowInfo) + 255) & ~255ull);
            d.rows_p0 = r.rect.p0;
        } else {
            d.rows = (const RowInfo *)ctx->rows.p;
            d.nfac = (const uint8_t *)ctx->nfac.p;
            d.rows_p0 = 1;
        }
        d.ip0 = r.rect.p0;
        d.order = r.has_order ? (const uint32_t *)((uint8_t *)S->arena_buf.p + r.order_off) : nullptr;
        if (r.units_issued == 0) {
            if (r.own_rows) {
                // the request's row factor lists, before its rows are regrouped
                SRVCHK(launch_row_info((const uint32_t *)ctx->primes16.p,
                                       (const uint32_t *)ctx->magic16.p, ctx->n16, r.rect.p0,
                                       (uint64_t)r.rect.p1 - r.rect.p0 + 1, (RowInfo *)d.rows,
                                       (uint8_t *)d.nfac, st.s));
            }
            new_slots.push_back(r.slot);
            if (r.has_order) {
                bdescs.push_back(d);
                const uint64_t rows = (uint64_t)r.rect.p1 - r.rect.p0 + 1;
                chunk_pre.push_back(chunk_pre.back() + (rows + kBucketChunk - 1) / kBucketChunk);
                row_pre.push_back(r.order_off / 4);
            }
        }
        descs.push_back(d);
        st.launch_tickets.push_back(t);
        r.units_issued += take;
        unit0 += take;
        budget -= take;
        st.queued_units -= take;
        if (r.units_issued == r.units_total) {
            final_slots.push_back(r.slot);
            st.final_tickets.push_back(t);
            st.queue.pop_front();
        }
    }
    if (descs.empty()) return CUBOID_OK;
    const uint32_t n = (uint32_t)descs.size(), nb = (uint32_t)bdescs.size();
    row_pre.push_back(0);   // (nb + 1 entries, like chunk_pre; the last is unused)
    // staging layout: descs | bucket descs | chunk prefix | row prefix | new slots | final slots
    const size_t bytes = (n + nb) * sizeof(ReqDesc) + 2 * (nb + 1) * 8 +
                         (new_slots.size() + final_slots.size()) * 4 + 64;
    SRVCHK(st.stage.ensure(bytes));
    SRVCHK(st.reqbuf.ensure(bytes));
    unsigned char *h = (unsigned char *)st.stage.p;
    size_t off = 0;
    auto put = [&](const void *src, size_t sz) {
        memcpy(h + off, src, sz);
        const size_t at = off;
        off += (sz + 7) & ~(size_t)7;
        return at;
    };
    const size_t o_desc = put(descs.data(), n * sizeof(ReqDesc));
    const size_t o_bdesc = nb ? put(bdescs.data(), nb * sizeof(ReqDesc)) : 0;
    const size_t o_cpre = nb ? put(chunk_pre.data(), (nb + 1) * 8) : 0;
    const size_t o_rpre = nb ? put(row_pre.data(), (nb + 1) * 8) : 0;
    const size_t o_new = new_slots.empty() ? 0 : put(new_slots.data(), new_slots.size() * 4);
    const size_t o_fin = final_slots.empty() ? 0 : put(final_slots.data(), final_slots.size() * 4);
    unsigned char *dv = (unsigned char *)st.reqbuf.p;
    SRVCHK(hipMemcpyAsync(dv, h, off, hipMemcpyHostToDevice, st.s));
    unsigned long long *cnt = (unsigned long long *)S->counts.p;
    unsigned long long *prs = (unsigned long long *)S->pairs.p;
    const uint64_t stride_c = (uint64_t)S->cfg.max_slots * S->nc, stride_p = S->cfg.max_slots;
    if (!new_slots.empty())
        SRVCHK(launch_zero_slots(cnt, prs, (const uint32_t *)(dv + o_new), (uint32_t)new_slots.size(),
                                 S->nc, S->n_rep, stride_c, stride_p, st.s));
    if (nb)
        SRVCHK(launch_bucket_rows((const ReqDesc *)(dv + o_bdesc), nb, (const uint64_t *)(dv + o_cpre),
                                  chunk_pre.back(), (const uint64_t *)(dv + o_rpre),
                                  (uint32_t *)S->arena_buf.p, st.s));
    SRVCHK(launch_fill_u64((uint64_t *)st.surv_n.p, 2, 0, st.s));
    uint32_t max_p = 0;
    for (const auto &d : descs) max_p = std::max(max_p, d.p1);
    st.last_n = n;
    st.last_units = unit0;
    st.last_desc_off = o_desc;
    st.last_max_p = max_p;
    SRVCHK(sweep_last(S, st, cnt, prs, S->n_rep));
    // outputs: [final][nc + 1] sums, survivor count, first survivors
    const size_t fout = final_slots.size() * (S->nc + 1) * 8;
    SRVCHK(st.out_dev.ensure(fout + 8));
    SRVCHK(st.out_host.ensure(fout + 8 + kSurvCopy * sizeof(SurvEntry)));
    if (!final_slots.empty())
        SRVCHK(launch_reduce_slots(cnt, prs, (const uint32_t *)(dv + o_fin), (uint32_t)final_slots.size(),
                                   S->nc, S->n_rep, stride_c, stride_p,
                                   (unsigned long long *)st.out_dev.p, st.s));
    unsigned char *oh = (unsigned char *)st.out_host.p;
    if (fout) SRVCHK(hipMemcpyAsync(oh, st.out_dev.p, fout, hipMemcpyDeviceToHost, st.s));
    SRVCHK(hipMemcpyAsync(oh + fout, st.surv_n.p, 8, hipMemcpyDeviceToHost, st.s));
    SRVCHK(hipMemcpyAsync(oh + fout + 8, st.surv.p, kSurvCopy * sizeof(SurvEntry), hipMemcpyDeviceToHost,
                          st.s));
    SRVCHK(hipEventRecord(st.ev, st.s));
    st.busy = true;
    S->stats.launches++;
    S->stats.units += unit0;
    return CUBOID_OK;
}

int sort_on_device(std::vector<SurvEntry> &v, hipStream_t s) {
    const uint64_t n = v.size();
    if (n < 2) return CUBOID_OK;
    const uint64_t rounded = (n + 1023) / 1024 * 1024;
    DevBuf a, b, nd;
    SRVCHK(a.ensure(rounded * sizeof(SurvEntry)));
    SRVCHK(b.ensure(rounded * sizeof(SurvEntry)));
    SRVCHK(nd.ensure(8));
    SRVCHK(hipMemcpyAsync(a.p, v.data(), n * sizeof(SurvEntry), hipMemcpyHostToDevice, s));
    SRVCHK(hipMemcpyAsync(nd.p, &n, 8, hipMemcpyHostToDevice, s));
    SurvEntry *out = nullptr;
    SRVCHK(launch_sort_surv((SurvEntry *)a.p, (SurvEntry *)b.p, (const unsigned long long *)nd.p, n,
                            &out, s));
    SRVCHK(hipMemcpyAsync(v.data(), out, n * sizeof(SurvEntry), hipMemcpyDeviceToHost, s));
    SRVCHK(hipStreamSynchronize(s));
    return CUBOID_OK;
}

// The launch on `st` has completed: hand out survivors and finished requests.
int complete(cuboid_server *S, StreamState &st) {
    const size_t fout = st.final_tickets.size() * (S->nc + 1) * 8;
    const unsigned char *oh = (const unsigned char *)st.out_host.p;
    uint64_t nsurv = 0;
    memcpy(&nsurv, oh + fout, 8);
    st.busy = false;
    if (nsurv > st.surv_cap && nsurv <= kMaxSurvScratch) {
        // the pool overflowed: sweep the same units again into a pool that
        // holds them all; the counters of the repeat go to a buffer that is
        // never read (the launch's own counts are complete already)
        uint64_t cap = st.surv_cap;
        while (cap < nsurv) cap *= 2;
        SRVCHK(st.surv.ensure(cap * sizeof(SurvEntry)));
        st.surv_cap = cap;
        SRVCHK(S->discard_counts.ensure((size_t)S->cfg.max_slots * S->nc * 8 + 8));
        SRVCHK(S->discard_pairs.ensure((size_t)S->cfg.max_slots * 8 + 8));
        SRVCHK(launch_fill_u64((uint64_t *)st.surv_n.p, 2, 0, st.s));
        SRVCHK(sweep_last(S, st, (unsigned long long *)S->discard_counts.p,
                          (unsigned long long *)S->discard_pairs.p, 1));
        uint64_t again = 0;
        SRVCHK(hipMemcpyAsync(&again, st.surv_n.p, 8, hipMemcpyDeviceToHost, st.s));
        SRVCHK(hipStreamSynchronize(st.s));
        if (again != nsurv) return CUBOID_E_DEVICE;
        S->stats.resweeps++;
    }
    if (nsurv) {
        std::vector<SurvEntry> e(std::min<uint64_t>(nsurv, st.surv_cap));
        if (e.size() <= kSurvCopy && nsurv <= kSurvPool) {
            memcpy(e.data(), oh + fout + 8, e.size() * sizeof(SurvEntry));
        } else {
            SRVCHK(hipMemcpyAsync(e.data(), st.surv.p, e.size() * sizeof(SurvEntry),
                                  hipMemcpyDeviceToHost, st.s));
            SRVCHK(hipStreamSynchronize(st.s));
        }
        if (nsurv > st.surv_cap) {
            // more than the largest pool: this launch's requests cannot be listed
            for (uint64_t t : st.launch_tickets) S->reqs[t].status = CUBOID_E_LIMIT;
        }
        for (const SurvEntry &x : e) S->reqs[S->slot_owner[x.req]].surv.push_back(x);
    }
    const uint32_t np = (uint32_t)S->caller.size();
    for (size_t i = 0; i < st.final_tickets.size(); ++i) {
        const uint64_t t = st.final_tickets[i];
        SrvReq &r = S->reqs[t];
        const uint64_t *c = (const uint64_t *)(oh + i * (S->nc + 1) * 8);
        r.counts.assign(np, 0);
        for (uint32_t j = 0; j < np; ++j) r.counts[j] = S->col[j] < 0 ? 0 : c[S->col[j]];
        r.n_pairs = c[S->nc];
        int st_sort = sort_on_device(r.surv, st.s);
        if (st_sort) r.status = st_sort;
        r.done = true;
        r.t_done = now_ns();
        S->free_slots.push_back(r.slot);
        if (r.has_order) S->arena.release(r.order_off, r.order_bytes);
        if (r.own_rows) S->arena.release(r.rows_off, r.rows_bytes);
        --S->admitted;
        S->stats.completed++;
    }
    S->cv_done.notify_all();
    return CUBOID_OK;
}

void worker_main(cuboid_server *S) {
    (void)hipSetDevice(S->ctx->device);
    // while launches are in flight the loop below checks their events every
    // 2 us; the default 50 us timer slack would stretch each of those sleeps
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        for (auto &stp : S->streams) {
            StreamState &st = *stp;
            if (!st.busy) continue;
            const hipError_t q = hipEventQuery(st.ev);
            if (q == hipSuccess) {
                const int e = complete(S, st);
                if (e) S->fatal = e;
                progress = true;
            } else if (q != hipErrorNotReady) {
                S->fatal = CUBOID_E_DEVICE;
                progress = true;
            }
        }
        if (S->fatal == CUBOID_OK) {
            admit(S);
            for (auto &stp : S->streams) {
                StreamState &st = *stp;
                if (!st.busy && !st.queue.empty()) {
                    const int e = launch(S, st);
                    if (e) S->fatal = e;
                    progress = true;
                }
            }
        }
        if (S->fatal != CUBOID_OK) {
            // a device error ends every unfinished request
            for (auto &kv : S->reqs) {
                if (!kv.second.done) {
                    kv.second.done = true;
                    kv.second.status = S->fatal;
                    kv.second.counts.assign(S->caller.size(), 0);
                    kv.second.t_done = now_ns();
                }
            }
            S->pending.clear();
            for (auto &st : S->streams) { st->queue.clear(); st->busy = false; }
            S->cv_done.notify_all();
        }
        bool busy = !S->pending.empty();
        for (auto &st : S->streams) busy = busy || st->busy || !st->queue.empty();
        if (S->stopping && !busy) break;
        if (!progress) {
            if (busy) S->cv_work.wait_for(lk, std::chrono::microseconds(2));
            else S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace

extern "C" {

int cuboid_server_start(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                        const cuboid_server_config *cfg, cuboid_server **out) {
    CTX_ENTER(ctx);
    if (!out) return CUBOID_E_ARG;
    *out = nullptr;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    std::unique_ptr<cuboid_server> S(new cuboid_server());
    S->ctx = ctx;
    S->caller.assign(primes, primes + n_primes);
    S->sorted = sorted;
    cuboid_server_config c = {0, 0, 0, 0};
    if (cfg) c = *cfg;
    if (c.streams == 0) c.streams = 2;
    if (c.streams > 8) return CUBOID_E_ARG;
    if (c.max_slots == 0) c.max_slots = 4096;
    if (c.max_launch_units == 0) c.max_launch_units = 1u << 22;
    CtxLock g(ctx);
    if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
    if (c.hbm_budget_bytes == 0) {
        // a quarter of the device memory free now, between 64 MiB and 4 GiB
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return CUBOID_E_DEVICE;
        c.hbm_budget_bytes = std::min<uint64_t>(4ull << 30, std::max<uint64_t>(64ull << 20, free_b / 4));
    }
    S->cfg = c;
    memset(&S->stats, 0, sizeof(S->stats));
    st = build_plan(ctx, sorted, &S->pl);
    if (st) return st;
    S->tun = tuning_for(ctx, sorted, *S->pl);
    st = build_dense(ctx, S->pl, S->tun.dense_primes, &S->ds);
    if (st) return st;
    S->nc = S->ds->K + S->ds->n_deep;
    S->col = count_columns(*S->pl, S->caller);
    st = ensure_rows(ctx, 1u << 21);
    if (st) return st;
    uint32_t rep = 16;
    while (rep > 1 && (uint64_t)rep * c.max_slots * (S->nc + 1) * 8 > kReplicaBytes) rep >>= 1;
    S->n_rep = rep;
    SRVCHK(S->counts.ensure((size_t)rep * c.max_slots * S->nc * 8 + 8));
    SRVCHK(S->pairs.ensure((size_t)rep * c.max_slots * 8 + 8));
    SRVCHK(S->arena_buf.ensure(c.hbm_budget_bytes));
    S->arena.init(c.hbm_budget_bytes);
    S->free_slots.resize(c.max_slots);
    for (uint32_t i = 0; i < c.max_slots; ++i) S->free_slots[i] = c.max_slots - 1 - i;
    S->slot_owner.assign(c.max_slots, 0);
    for (uint32_t i = 0; i < c.streams; ++i) {
        S->streams.emplace_back(new StreamState());
        StreamState &sst = *S->streams.back();
        SRVCHK(hipStreamCreateWithFlags(&sst.s, hipStreamNonBlocking));
        SRVCHK(hipEventCreateWithFlags(&sst.ev, hipEventDisableTiming));
        SRVCHK(sst.surv.ensure(kSurvPool * sizeof(SurvEntry)));
        SRVCHK(sst.surv_n.ensure(16));   // survivor count, claim counter
        // a launch covers at most max_slots requests: its staging and output
        // buffers are sized for that now, so that no launch grows them (a
        // device free synchronises the device, a pinned allocation takes
        // milliseconds)
        const size_t m = c.max_slots;
        const size_t stage = 2 * m * sizeof(ReqDesc) + 2 * (m + 1) * 8 + 2 * m * 4 + 64;
        const size_t fout = m * (S->nc + 1) * 8;
        SRVCHK(sst.stage.ensure(stage));
        SRVCHK(sst.reqbuf.ensure(stage));
        SRVCHK(sst.out_dev.ensure(fout + 8));
        SRVCHK(sst.out_host.ensure(fout + 8 + kSurvCopy * sizeof(SurvEntry)));
    }
    ctx->servers.fetch_add(1);
    cuboid_server *raw = S.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return CUBOID_OK;
}

int cuboid_server_submit(cuboid_server *S, const cuboid_request *req, uint64_t *ticket) {
    if (!S || !req || !ticket) return CUBOID_E_ARG;
    const int st = rect_valid(req->p0, req->p1, req->q0, req->q1);
    if (st) return st;
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopping) return CUBOID_E_BUSY;
    const uint64_t t = S->next_ticket++;
    SrvReq &r = S->reqs[t];
    r.rect = *req;
    const uint64_t rows = (uint64_t)req->p1 - req->p0 + 1;
    r.nrb = (uint32_t)((rows + 63) / 64);
    r.nwin = (uint32_t)(((uint64_t)req->q1 - req->q0 + 64) / 64);
    r.units_total = (uint64_t)r.nrb * r.nwin;
    r.t_submit = now_ns();
    S->pending.push_back(t);
    S->stats.submitted++;
    *ticket = t;
    S->cv_work.notify_one();
    return CUBOID_OK;
}

int cuboid_server_submit_many(cuboid_server *S, const cuboid_request *req, uint32_t n,
                              uint64_t *tickets, uint32_t *bad) {
    if (!S || !req || !tickets || n == 0) return CUBOID_E_ARG;
    for (uint32_t i = 0; i < n; ++i) {
        const int st = rect_valid(req[i].p0, req[i].p1, req[i].q0, req[i].q1);
        if (st) {
            if (bad) *bad = i;
            return st;
        }
    }
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopping) return CUBOID_E_BUSY;
    const uint64_t t_now = now_ns();
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t t = S->next_ticket++;
        SrvReq &r = S->reqs[t];
        r.rect = req[i];
        const uint64_t rows = (uint64_t)req[i].p1 - req[i].p0 + 1;
        r.nrb = (uint32_t)((rows + 63) / 64);
        r.nwin = (uint32_t)(((uint64_t)req[i].q1 - req[i].q0 + 64) / 64);
        r.units_total = (uint64_t)r.nrb * r.nwin;
        r.t_submit = t_now;
        S->pending.push_back(t);
        tickets[i] = t;
    }
    S->stats.submitted += n;
    S->cv_work.notify_one();
    return CUBOID_OK;
}

int cuboid_server_poll(cuboid_server *S, uint64_t ticket, cuboid_result *res, int wait,
                       cuboid_request_timing *timing) {
    if (!S || !res) return CUBOID_E_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return CUBOID_E_ARG;
    if (!it->second.done) {
        if (!wait) return CUBOID_E_BUSY;
        S->cv_done.wait(lk, [&] {
            auto jt = S->reqs.find(ticket);
            return jt == S->reqs.end() || jt->second.done;
        });
        it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return CUBOID_E_ARG;
    }
    SrvReq &r = it->second;
    if (timing) {
        timing->submit_ns = r.t_submit;
        timing->admit_ns = r.t_admit;
        timing->done_ns = r.t_done;
    }
    res->n_pairs = r.n_pairs;
    res->n_survivors = r.surv.size();
    if (res->counts) memcpy(res->counts, r.counts.data(), r.counts.size() * 8);
    if (r.status != CUBOID_OK) {
        res->status = r.status;
        S->reqs.erase(it);
        return res->status;
    }
    if (r.surv.size() > res->cap) {
        res->status = CUBOID_E_CAPACITY;
        return CUBOID_E_CAPACITY;
    }
    for (size_t i = 0; i < r.surv.size(); ++i) res->survivors[i] = r.surv[i].idx;
    res->status = CUBOID_OK;
    S->reqs.erase(it);
    return CUBOID_OK;
}

int cuboid_server_stats_get(cuboid_server *S, cuboid_server_stats *out) {
    if (!S || !out) return CUBOID_E_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    *out = S->stats;
    return CUBOID_OK;
}

int cuboid_server_stop(cuboid_server *S) {
    if (!S) return CUBOID_E_ARG;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stopping = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->ctx->device);
    for (auto &st : S->streams) {
        if (st->s) (void)hipStreamSynchronize(st->s);
        if (st->ev) (void)hipEventDestroy(st->ev);
        if (st->s) (void)hipStreamDestroy(st->s);
    }
    cuboid_ctx *ctx = S->ctx;
    delete S;
    ctx->servers.fetch_sub(1);
    return CUBOID_OK;
}

}  // extern "C"
