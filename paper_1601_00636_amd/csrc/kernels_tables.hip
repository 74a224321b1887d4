// Table construction on the GPU: Q_pq(t) mod r evaluation, the unsolvability
// tables of Definition 1.1 / eq. (2.3) of arXiv:1601.00636 in ratio form, the
// paper's packed layout (eq. 2.6), the 64-bit window tables the sweep stages in
// LDS, the coprimality wheel and per-row prime factors.
#include "devmath.h"
#include "internal.h"

namespace cuboid {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(uint64_t n, unsigned block = kBlock) {
    uint64_t g = (n + block - 1) / block;
    if (g > 1u << 20) g = 1u << 20;   // grid-stride beyond this
    return (unsigned)(g ? g : 1);
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Device-to-device copy as a kernel (also valid inside a captured graph and
// for buffers of any HIP allocator of this process).
__global__ void copy_u64_kernel(uint64_t *dst, const uint64_t *src, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void fill_u8_kernel(uint8_t *p, uint64_t n, uint8_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// out[i] = Q_{p q}(t) mod r for arbitrary 2 <= r < 2^16
__global__ void q_eval_kernel(const uint32_t *p, const uint32_t *q, const uint32_t *t,
                              const uint32_t *rr, uint64_t n, uint32_t *out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = rr[i];
        const uint32_t m = (uint32_t)(0x100000000ull / r);
        const QCoef c = q_coeffs(modr(p[i], r, m), modr(q[i], r, m), r, m);
        const uint32_t tr = modr(t[i], r, m);
        out[i] = q_eval_s(c, mulr(tr, tr, r, m), r, m);
    }
}

// Ratio vector of a prime r: v[x] = u_r(x, 1).  For a, b != 0 the weight-20
// homogeneity Q_{la,lb}(l^2 t) = l^20 Q_ab(t) gives u_r(a, b) = v[a / b]; the
// row and column of 0 are solvable (t = 0).  Q depends on x only through x^2
// and is even in t, so x and t run over half the residues.
// Work item g: prime i = segment of g, x = 1 + (g - prefix[i]).
__global__ void ratio_vector_kernel(const uint32_t *pr, const uint32_t *voff, uint32_t n,
                                    const uint64_t *prefix, uint64_t total, uint8_t *vpool) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = find_segment(prefix, n, g);
        const uint32_t r = pr[i];
        const uint32_t m = (uint32_t)(0x100000000ull / r);
        const uint32_t x = 1 + (uint32_t)(g - prefix[i]);
        const QCoef c = q_coeffs(x, 1, r, m);
        const uint32_t tmax = (r == 2) ? 1 : (r - 1) / 2;
        bool solvable = false;
        uint32_t s = 0;                        // t^2 mod r, advanced by 2t + 1
        for (uint32_t t = 0; t <= tmax; ++t) {
            if (q_eval_s(c, s, r, m) == 0) { solvable = true; break; }
            s = modr(s + 2 * t + 1, r, m);
        }
        const uint8_t u = solvable ? 0 : 1;
        vpool[voff[i] + x] = u;
        vpool[voff[i] + (r - x) % r] = u;
    }
}

// Modular inverses b^(r-2) mod r for b in [1, r); entry 0 stays 0.
__global__ void inverse_kernel(const uint32_t *pr, const uint32_t *ioff, uint32_t n,
                               const uint64_t *prefix, uint64_t total, uint16_t *ipool) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = find_segment(prefix, n, g);
        const uint32_t r = pr[i];
        const uint32_t m = (uint32_t)(0x100000000ull / r);
        const uint32_t b = 1 + (uint32_t)(g - prefix[i]);
        uint32_t e = r - 2, base = b, acc = 1 % r;
        while (e) {
            if (e & 1) acc = mulr(acc, base, r, m);
            base = mulr(base, base, r, m);
            e >>= 1;
        }
        ipool[ioff[i] + b] = (uint16_t)acc;
    }
}

// Number of unsolvable ratio classes per prime (0 => table identically zero).
__global__ void vector_popcount_kernel(const uint32_t *pr, const uint32_t *voff,
                                       const uint8_t *vpool, uint32_t *out) {
    __shared__ uint32_t part[kBlock];
    const uint32_t i = blockIdx.x, r = pr[i];
    uint32_t c = 0;
    for (uint32_t x = threadIdx.x; x < r; x += blockDim.x) c += vpool[voff[i] + x];
    part[threadIdx.x] = c;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = part[0];
}

__device__ __forceinline__ uint32_t unsolv_bit(uint32_t a, uint32_t b, uint32_t r, uint32_t m,
                                               const uint8_t *v, const uint16_t *inv) {
    if (a == 0 || b == 0) return 0;
    return v[mulr(a, inv[b], r, m)];
}

// eq. (2.6) layout: bit a*r + b of the byte string, least significant first
__global__ void pack_table_kernel(uint32_t r, const uint8_t *v, const uint16_t *inv,
                                  uint8_t *out) {
    const uint32_t m = (uint32_t)(0x100000000ull / r);
    const uint64_t nbits = (uint64_t)r * r, nbytes = (nbits + 7) / 8;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < nbytes;
         k += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t byte = 0;
        for (uint32_t j = 0; j < 8; ++j) {
            const uint64_t idx = 8 * k + j;
            if (idx >= nbits) break;
            uint32_t b;
            const uint32_t a = divr((uint32_t)idx, r, m, &b);
            byte |= unsolv_bit(a, b, r, m, v, inv) << j;
        }
        out[k] = (uint8_t)byte;
    }
}

// Window table of a dense prime r: entry a*(r + kDenseExt) + k holds the 64
// bits u_r(a, (o + j) mod r), j = 0..63, with o = 64 k mod r, so that one
// 64-bit read answers a whole run of 64 consecutive columns q with q mod r = o
// for row residue a, and the next 64 columns are at entry k + 1.
__global__ void dense_windows_kernel(const uint32_t *pr, const uint32_t *voff,
                                     const uint32_t *ioff, const uint32_t *woff, uint32_t n,
                                     const uint64_t *prefix, uint64_t total, const uint8_t *vpool,
                                     const uint16_t *ipool, uint64_t *out) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = find_segment(prefix, n, g);
        const uint32_t r = pr[i];
        const uint32_t m = (uint32_t)(0x100000000ull / r);
        // row a holds r + kDenseExt entries; entry k is the window that
        // starts at column offset 64 k mod r, so consecutive windows of a row
        // are consecutive entries
        const uint32_t e = (uint32_t)(g - prefix[i]);
        const uint32_t a = e / (r + kDenseExt), k = e % (r + kDenseExt);
        const uint32_t o = (uint32_t)(((uint64_t)k * 64) % r);
        const uint8_t *v = vpool + voff[i];
        const uint16_t *inv = ipool + ioff[i];
        uint64_t w = 0;
        uint32_t b = o;
        for (uint32_t j = 0; j < 64; ++j) {
            w |= (uint64_t)unsolv_bit(a, b, r, m, v, inv) << j;
            b = (b + 1 == r) ? 0 : b + 1;
        }
        out[woff[i] + e] = w;
    }
}

// Coprimality wheel: entry s*30 + o has bit j set when o + j is divisible by
// none of the primes of subset s of {2, 3, 5} (bit 0 = 2, bit 1 = 3, bit 2 =
// 5), i.e. the columns such a row keeps; row 8 is all zero (a lane without a
// row keeps no pairs).
__global__ void wheel_kernel(uint64_t *out) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kWheelSubsets * kWheel) return;
    const uint32_t s = e / kWheel, o = e % kWheel;
    if (s == kIdleSubset) { out[e] = 0; return; }
    const uint32_t sp[3] = {2, 3, 5};
    uint64_t w = 0;
    for (uint32_t j = 0; j < 64; ++j) {
        bool hit = false;
        for (int k = 0; k < 3; ++k)
            if (((s >> k) & 1) && (o + j) % sp[k] == 0) hit = true;
        if (hit) w |= 1ull << j;
    }
    out[e] = ~w;
}

__constant__ uint32_t kPatPrimes[15] = {7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61};

// Multiple patterns (see kPatSmall): prime l's entry d (the distance from a
// window's first column to the next multiple of l) has bit j for j = d mod l.
__global__ void patterns_kernel(uint64_t *out) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)kPatEntries) return;
    if (e >= (uint32_t)kPatSmall) {
        const uint32_t j = e - kPatSmall;
        out[e] = j < 64 ? (1ull << j) : 0ull;
        return;
    }
    uint32_t base = 0, i = 0;
    while (base + kPatPrimes[i] <= e) { base += kPatPrimes[i]; ++i; }
    const uint32_t l = kPatPrimes[i], d = e - base;
    uint64_t w = 0;
    for (uint32_t j = 0; j < 64; ++j)
        if (j % l == d) w |= 1ull << j;
    out[e] = w;
}

// Distinct prime factors of p = pstart + g by trial division with the primes
// below 2^16 (enough for any uint32).  primes16 starts 2, 3, 5, 7, 11, ...
__global__ void row_info_kernel(const uint32_t *primes16, const uint32_t *magic16, uint32_t n16,
                                uint32_t pstart, uint64_t count, RowInfo *out, uint8_t *nfac) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < count;
         g += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t x = pstart + (uint32_t)g;
        RowInfo ri;
        ri.meta = 0;
        uint32_t nf = 0;
        for (int k = 0; k < kMaxBigFactors; ++k) ri.f[k] = 0;
        for (uint32_t i = 0; i < n16; ++i) {
            const uint32_t l = primes16[i];
            if ((uint64_t)l * l > x) break;
            const uint32_t m = magic16[i];
            uint32_t rem;
            uint32_t qt = divr(x, l, m, &rem);
            if (rem) continue;
            if (i < 3) ri.meta |= 1u << i; else ri.f[nf++] = l;
            do { x = qt; qt = divr(x, l, m, &rem); } while (rem == 0);
        }
        if (x > 1) {
            // remaining cofactor is prime
            if (x == 2) ri.meta |= 1; else if (x == 3) ri.meta |= 2;
            else if (x == 5) ri.meta |= 4;
            else ri.f[nf++] = x;
        }
        ri.meta |= nf << 4;
        out[g] = ri;
        nfac[g] = (uint8_t)nf;
    }
}

// One block per chunk of kBucketChunk rows of a request: the chunk's rows are
// written to `order` grouped by their number of factors >= 7, so that the 64
// rows of a wavefront tend to share that number.
// Rows of each 8192-row chunk of a request regrouped by their number of prime
// factors >= 7, stably (ascending p inside each group).  The block first
// copies the chunk's factor counts into LDS with wide loads (one memory
// latency instead of one per 64 rows); each of the 4 waves then takes a
// quarter of the chunk: it counts its rows per group with ballots, the block
// turns the (group, wave) counts into start positions, and each wave places
// its rows 64 at a time at its running positions.
__global__ void __launch_bounds__(256) bucket_rows_kernel(const ReqDesc *req, uint32_t n_req,
                                                          const uint64_t *chunk_prefix,
                                                          const uint64_t *row_prefix,
                                                          uint32_t *order, uint64_t n_chunks,
                                                          const uint64_t *n_chunks_dev) {
    constexpr int kGroups = kMaxBigFactors + 1;
    constexpr uint32_t kPerWave = kBucketChunk / 4;
    __shared__ uint32_t cnt[kGroups][4];
    __shared__ uint8_t snf[kBucketChunk];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t nch = n_chunks_dev ? *n_chunks_dev : n_chunks;
    for (uint64_t b = blockIdx.x; b < nch; b += gridDim.x) {
        const uint32_t i = find_segment(chunk_prefix, n_req, b);
        const ReqDesc R = req[i];
        const uint64_t rows = (uint64_t)R.p1 - R.p0 + 1;
        const uint64_t r0 = (b - chunk_prefix[i]) * kBucketChunk;
        const uint32_t n = (uint32_t)((r0 + kBucketChunk < rows ? r0 + kBucketChunk : rows) - r0);
        const uint8_t *nf = R.nfac + (R.p0 + (uint32_t)r0 - R.rows_p0);
        // stage nf[0, n) in LDS: 4-byte loads where the source is aligned,
        // bytes for the unaligned head and the tail
        const uint32_t head = (uint32_t)((4 - ((uintptr_t)nf & 3)) & 3);
        const uint32_t h = head < n ? head : n;
        for (uint32_t r = tid; r < h; r += blockDim.x) snf[r] = nf[r];
        const uint32_t nw4 = (n - h) / 4;
        const uint32_t *nf4 = (const uint32_t *)(nf + h);
        for (uint32_t j = tid; j < nw4; j += blockDim.x) {
            const uint32_t v = nf4[j];
            const uint32_t o = h + 4 * j;
            snf[o] = (uint8_t)v;
            snf[o + 1] = (uint8_t)(v >> 8);
            snf[o + 2] = (uint8_t)(v >> 16);
            snf[o + 3] = (uint8_t)(v >> 24);
        }
        for (uint32_t r = h + 4 * nw4 + tid; r < n; r += blockDim.x) snf[r] = nf[r];
        __syncthreads();
        const uint32_t a = w * kPerWave;
        const uint32_t e = a + kPerWave < n ? a + kPerWave : n;   // this wave's rows [a, e)
        uint32_t run[kGroups];
        for (int k = 0; k < kGroups; ++k) run[k] = 0;
        for (uint32_t g = a; g < e; g += 64) {
            const uint32_t r = g + lane;
            const uint32_t k = r < e ? snf[r] : (uint32_t)kGroups;
            for (int kk = 0; kk < kGroups; ++kk) run[kk] += (uint32_t)__popcll(__ballot(k == (uint32_t)kk));
        }
        if (lane == 0)
            for (int kk = 0; kk < kGroups; ++kk) cnt[kk][w] = run[kk];
        __syncthreads();
        // start of (group kk, wave w): every row of lower groups, then of this
        // group in lower waves
        uint32_t acc = 0;
        for (int kk = 0; kk < kGroups; ++kk) {
            uint32_t below = 0;
            for (uint32_t v = 0; v < 4; ++v)
                if (v < w) below += cnt[kk][v];
            run[kk] = acc + below;
            acc += cnt[kk][0] + cnt[kk][1] + cnt[kk][2] + cnt[kk][3];
        }
        uint32_t *dst = order + row_prefix[i] + r0;
        for (uint32_t g = a; g < e; g += 64) {
            const uint32_t r = g + lane;
            const uint32_t k = r < e ? snf[r] : (uint32_t)kGroups;
            uint32_t pos = 0;
            for (int kk = 0; kk < kGroups; ++kk) {
                const uint64_t m = __ballot(k == (uint32_t)kk);
                if (k == (uint32_t)kk)
                    pos = run[kk] + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                run[kk] += (uint32_t)__popcll(m);
            }
            if (k < (uint32_t)kGroups) dst[pos] = R.p0 + (uint32_t)(r0 + r);
        }
        __syncthreads();   // cnt and snf are rewritten by the next chunk
    }
}

// Counter slots of a request: zero every replica of each listed slot.
__global__ void zero_slots_kernel(unsigned long long *counts, unsigned long long *pairs,
                                  const uint32_t *slots, uint32_t n, uint32_t nc, uint32_t n_rep,
                                  uint64_t stride_c, uint64_t stride_p) {
    const uint64_t per = (uint64_t)(nc + 1) * n_rep;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < per * n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(g / per), e = (uint32_t)(g % per);
        const uint32_t r = e / (nc + 1), k = e % (nc + 1);
        if (k < nc) counts[r * stride_c + (uint64_t)slots[i] * nc + k] = 0;
        else pairs[r * stride_p + slots[i]] = 0;
    }
}

// Sum the replicas of each listed slot into out[i * (nc + 1) + k] (k = nc: pairs).
__global__ void reduce_slots_kernel(const unsigned long long *counts,
                                    const unsigned long long *pairs, const uint32_t *slots,
                                    uint32_t n, uint32_t nc, uint32_t n_rep, uint64_t stride_c,
                                    uint64_t stride_p, unsigned long long *out) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < (uint64_t)n * (nc + 1);
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(g / (nc + 1)), k = (uint32_t)(g % (nc + 1));
        unsigned long long acc = 0;
        for (uint32_t r = 0; r < n_rep; ++r)
            acc += k < nc ? counts[r * stride_c + (uint64_t)slots[i] * nc + k]
                          : pairs[r * stride_p + slots[i]];
        out[g] = acc;
    }
}

// Per-slot counters (canonical order, nc per slot) into the caller's prime
// order (np per slot): out[i][j] = counts[i][col[j]], 0 where col[j] < 0.
__global__ void gather_counts_kernel(const unsigned long long *counts, const int32_t *col,
                                     uint32_t n_slots, uint32_t nc, uint32_t np,
                                     unsigned long long *out) {
    const uint64_t n = (uint64_t)n_slots * np;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = g / np;
        const int32_t c = col[g - i * np];
        out[g] = c < 0 ? 0ull : counts[i * nc + (uint32_t)c];
    }
}

// Zeroes three buffers in one launch (counter replicas, pair-count replicas,
// survivor count and claim counter).
__global__ void clear3_kernel(uint64_t *a, uint64_t na, uint64_t *b, uint64_t nb, uint64_t *c,
                              uint64_t nc) {
    const uint64_t n = na + nb + nc;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i < na) a[i] = 0;
        else if (i < na + nb) b[i - na] = 0;
        else c[i - na - nb] = 0;
    }
}

__global__ void reduce_replicas_kernel(unsigned long long *buf, uint64_t n, uint32_t n_rep,
                                       uint64_t stride) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        unsigned long long acc = buf[i];
        for (uint32_t r = 1; r < n_rep; ++r) acc += buf[r * stride + i];
        buf[i] = acc;
    }
}

}  // namespace

hipError_t launch_clear3(uint64_t *a, uint64_t na, uint64_t *b, uint64_t nb, uint64_t *c,
                         uint64_t nc, hipStream_t s) {
    const uint64_t n = na + nb + nc;
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(clear3_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, a, na, b, nb, c, nc);
    return hipGetLastError();
}

hipError_t launch_copy_u64(uint64_t *dst, const uint64_t *src, uint64_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    if (!dst || !src) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_u64_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    if (!p) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_q_eval(const uint32_t *p, const uint32_t *q, const uint32_t *t,
                         const uint32_t *r, uint64_t n, uint32_t *out, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(q_eval_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, q, t, r, n, out);
    return hipGetLastError();
}

hipError_t launch_ratio_vectors(const uint32_t *pr, const uint32_t *voff, uint32_t n,
                                const uint64_t *prefix, uint64_t total, uint8_t *vpool,
                                hipStream_t s) {
    if (!total) return hipSuccess;
    hipLaunchKernelGGL(ratio_vector_kernel, dim3(grid_for(total)), dim3(kBlock), 0, s, pr, voff,
                       n, prefix, total, vpool);
    return hipGetLastError();
}

hipError_t launch_inverse_tables(const uint32_t *pr, const uint32_t *ioff, uint32_t n,
                                 const uint64_t *prefix, uint64_t total, uint16_t *ipool,
                                 hipStream_t s) {
    if (!total) return hipSuccess;
    hipLaunchKernelGGL(inverse_kernel, dim3(grid_for(total)), dim3(kBlock), 0, s, pr, ioff, n,
                       prefix, total, ipool);
    return hipGetLastError();
}

hipError_t launch_vector_popcount(const uint32_t *pr, const uint32_t *voff, uint32_t n,
                                  const uint8_t *vpool, uint32_t *out, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(vector_popcount_kernel, dim3(n), dim3(kBlock), 0, s, pr, voff, vpool, out);
    return hipGetLastError();
}

hipError_t launch_pack_table(uint32_t r, const uint8_t *v, const uint16_t *inv, uint8_t *out,
                             hipStream_t s) {
    const uint64_t nbytes = ((uint64_t)r * r + 7) / 8;
    hipLaunchKernelGGL(pack_table_kernel, dim3(grid_for(nbytes)), dim3(kBlock), 0, s, r, v, inv,
                       out);
    return hipGetLastError();
}

hipError_t launch_dense_windows(const uint32_t *pr, const uint32_t *voff, const uint32_t *ioff,
                                const uint32_t *woff, uint32_t n, const uint64_t *prefix,
                                uint64_t total, const uint8_t *vpool, const uint16_t *ipool,
                                uint64_t *out, hipStream_t s) {
    if (!total) return hipSuccess;
    hipLaunchKernelGGL(dense_windows_kernel, dim3(grid_for(total)), dim3(kBlock), 0, s, pr, voff,
                       ioff, woff, n, prefix, total, vpool, ipool, out);
    return hipGetLastError();
}

hipError_t launch_wheel(uint64_t *out, hipStream_t s) {
    const uint32_t n = kWheelSubsets * kWheel;
    hipLaunchKernelGGL(wheel_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, out);
    return hipGetLastError();
}

hipError_t launch_row_info(const uint32_t *primes16, const uint32_t *magic16, uint32_t n16,
                           uint32_t pstart, uint64_t count, RowInfo *out, uint8_t *nfac,
                           hipStream_t s) {
    if (!count) return hipSuccess;
    hipLaunchKernelGGL(row_info_kernel, dim3(grid_for(count)), dim3(kBlock), 0, s, primes16,
                       magic16, n16, pstart, count, out, nfac);
    return hipGetLastError();
}

hipError_t launch_patterns(uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(patterns_kernel, dim3((kPatEntries + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       s, out);
    return hipGetLastError();
}

uint32_t pattern_offset(uint32_t l) {
    static const uint32_t pr[15] = {7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61};
    uint32_t base = 0;
    for (uint32_t i = 0; i < 15; ++i) {
        if (pr[i] == l) return base;
        base += pr[i];
    }
    return kPatSmall;   // the single-bit entries
}

hipError_t launch_bucket_rows(const ReqDesc *req, uint32_t n_req, const uint64_t *chunk_prefix,
                              uint64_t n_chunks, const uint64_t *row_prefix, uint32_t *order,
                              hipStream_t s, const uint64_t *n_chunks_dev, uint32_t grid) {
    if (!n_chunks_dev && !n_chunks) return hipSuccess;
    const uint32_t g = n_chunks_dev ? grid : (uint32_t)n_chunks;
    if (g == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bucket_rows_kernel, dim3(g), dim3(256), 0, s, req, n_req, chunk_prefix,
                       row_prefix, order, n_chunks, n_chunks_dev);
    return hipGetLastError();
}

hipError_t launch_zero_slots(unsigned long long *counts, unsigned long long *pairs,
                             const uint32_t *slots, uint32_t n, uint32_t nc, uint32_t n_rep,
                             uint64_t stride_c, uint64_t stride_p, hipStream_t s) {
    if (!n) return hipSuccess;
    const uint64_t work = (uint64_t)n * (nc + 1) * n_rep;
    hipLaunchKernelGGL(zero_slots_kernel, dim3(grid_for(work)), dim3(kBlock), 0, s, counts, pairs,
                       slots, n, nc, n_rep, stride_c, stride_p);
    return hipGetLastError();
}

hipError_t launch_reduce_slots(const unsigned long long *counts, const unsigned long long *pairs,
                               const uint32_t *slots, uint32_t n, uint32_t nc, uint32_t n_rep,
                               uint64_t stride_c, uint64_t stride_p, unsigned long long *out,
                               hipStream_t s) {
    if (!n) return hipSuccess;
    const uint64_t work = (uint64_t)n * (nc + 1);
    hipLaunchKernelGGL(reduce_slots_kernel, dim3(grid_for(work)), dim3(kBlock), 0, s, counts, pairs,
                       slots, n, nc, n_rep, stride_c, stride_p, out);
    return hipGetLastError();
}

hipError_t launch_gather_counts(const unsigned long long *counts, const int32_t *col,
                                uint32_t n_slots, uint32_t nc, uint32_t np,
                                unsigned long long *out, hipStream_t s) {
    const uint64_t n = (uint64_t)n_slots * np;
    if (!n) return hipSuccess;
    if (!counts || !col || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_counts_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, counts, col,
                       n_slots, nc, np, out);
    return hipGetLastError();
}

hipError_t launch_reduce_replicas(unsigned long long *buf, uint64_t n, uint32_t n_rep,
                                  uint64_t stride, hipStream_t s) {
    if (!n || n_rep <= 1) return hipSuccess;
    hipLaunchKernelGGL(reduce_replicas_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, buf, n, n_rep,
                       stride);
    return hipGetLastError();
}

}  // namespace cuboid
