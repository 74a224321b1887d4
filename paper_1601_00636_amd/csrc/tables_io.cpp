// The paper's binary table files: the concatenated packed tables of eq. (2.6)
// and the index of {int16 prime, uint32 byte offset} items (section 2, eq.
// 2.7), written from the tables built on the device, and read back with every
// table checked bit for bit against the device's.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "runtime.h"

using namespace cuboid;

namespace {

constexpr size_t kItemBytes = 8;   // int16 prime, 2 bytes padding, uint32 offset

struct File {
    FILE *f = nullptr;
    File(const char *path, const char *mode) { f = fopen(path, mode); }
    ~File() { if (f) fclose(f); }
};

// Packed tables (eq. 2.6) of the canonical list, concatenated in its order.
int pack_all(cuboid_ctx *ctx, const std::vector<uint32_t> &sorted, std::vector<uint8_t> *bytes,
             std::vector<uint64_t> *offsets) {
    Plan *pl = nullptr;
    int st = build_plan(ctx, sorted, &pl);
    if (st) return st;
    uint64_t total = 0;
    offsets->clear();
    for (uint32_t r : sorted) {
        offsets->push_back(total);
        total += ((uint64_t)r * r + 7) / 8;
    }
    if (total >= (1ull << 32)) return CUBOID_E_LIMIT;
    DevBuf d;
    if (d.ensure(total) != hipSuccess) return CUBOID_E_DEVICE;
    for (size_t i = 0; i < sorted.size(); ++i) {
        if (launch_pack_table(sorted[i], (const uint8_t *)pl->vpool.p + pl->voff[i],
                              (const uint16_t *)pl->ipool.p + pl->ioff[i],
                              (uint8_t *)d.p + (*offsets)[i], ctx->stream) != hipSuccess)
            return CUBOID_E_DEVICE;
    }
    bytes->resize(total);
    if (hipMemcpyAsync(bytes->data(), d.p, total, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return CUBOID_E_DEVICE;
    return CUBOID_OK;
}

void put_le(uint8_t *b, uint64_t v, int n) {
    for (int i = 0; i < n; ++i) b[i] = (uint8_t)(v >> (8 * i));
}

uint64_t get_le(const uint8_t *b, int n) {
    uint64_t v = 0;
    for (int i = 0; i < n; ++i) v |= (uint64_t)b[i] << (8 * i);
    return v;
}

}  // namespace

extern "C" {

int cuboid_write_table_files(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                             const char *tables_path, const char *primes_path,
                             const char *text_path) {
    CTX_ENTER(ctx);
    if (!tables_path || !primes_path) return CUBOID_E_ARG;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    if (sorted.back() >= 32768) return CUBOID_E_LIMIT;
    std::vector<uint8_t> bytes;
    std::vector<uint64_t> off;
    {
        CtxLock g(ctx);
        if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
        st = pack_all(ctx, sorted, &bytes, &off);
        if (st) return st;
    }
    {
        File t(tables_path, "wb");
        if (!t.f || fwrite(bytes.data(), 1, bytes.size(), t.f) != bytes.size()) return CUBOID_E_IO;
    }
    {
        std::vector<uint8_t> items(sorted.size() * kItemBytes, 0);
        for (size_t i = 0; i < sorted.size(); ++i) {
            put_le(&items[i * kItemBytes], sorted[i], 2);
            put_le(&items[i * kItemBytes + 4], off[i], 4);
        }
        File pf(primes_path, "wb");
        if (!pf.f || fwrite(items.data(), 1, items.size(), pf.f) != items.size()) return CUBOID_E_IO;
    }
    if (text_path) {
        File tf(text_path, "w");
        if (!tf.f) return CUBOID_E_IO;
        std::vector<char> line;
        for (size_t i = 0; i < sorted.size(); ++i) {
            const uint32_t r = sorted[i];
            const uint8_t *tab = bytes.data() + off[i];
            fprintf(tf.f, "r = %u\n", r);
            line.assign((size_t)2 * r, ' ');
            line[2 * r - 1] = '\n';
            for (uint32_t a = 0; a < r; ++a) {
                for (uint32_t b = 0; b < r; ++b) {
                    const uint64_t k = (uint64_t)a * r + b;
                    line[2 * b] = (tab[k >> 3] >> (k & 7)) & 1 ? '1' : '0';
                }
                if (fwrite(line.data(), 1, line.size(), tf.f) != line.size()) return CUBOID_E_IO;
            }
            fputc('\n', tf.f);
        }
        if (ferror(tf.f)) return CUBOID_E_IO;
    }
    return CUBOID_OK;
}

int cuboid_check_table_files(cuboid_ctx *ctx, const char *tables_path, const char *primes_path,
                             uint32_t *primes_out, uint32_t cap, uint32_t *n_primes) {
    CTX_ENTER(ctx);
    if (!tables_path || !primes_path || !n_primes || (cap && !primes_out)) return CUBOID_E_ARG;
    *n_primes = 0;
    std::vector<uint8_t> items, tables;
    auto slurp = [](const char *path, std::vector<uint8_t> *out) -> bool {
        File f(path, "rb");
        if (!f.f) return false;
        if (fseek(f.f, 0, SEEK_END) != 0) return false;
        const long n = ftell(f.f);
        if (n < 0 || fseek(f.f, 0, SEEK_SET) != 0) return false;
        out->resize((size_t)n);
        return fread(out->data(), 1, out->size(), f.f) == out->size();
    };
    if (!slurp(primes_path, &items) || !slurp(tables_path, &tables)) return CUBOID_E_IO;
    if (items.empty() || items.size() % kItemBytes) return CUBOID_E_IO;
    const size_t n = items.size() / kItemBytes;
    std::vector<uint32_t> list(n);
    uint64_t expect = 0;
    for (size_t i = 0; i < n; ++i) {
        const uint8_t *it = &items[i * kItemBytes];
        list[i] = (uint32_t)get_le(it, 2);
        if (get_le(it + 2, 2) != 0) return CUBOID_E_DATA;
        if (get_le(it + 4, 4) != expect) return CUBOID_E_DATA;
        expect += ((uint64_t)list[i] * list[i] + 7) / 8;
    }
    std::vector<uint32_t> sorted;
    int st = canonical_primes(list.data(), (uint32_t)n, &sorted);
    if (st) return st;
    if (sorted != list) return CUBOID_E_DATA;   // written in ascending order
    if (tables.size() < expect) return CUBOID_E_IO;
    if (tables.size() != expect) return CUBOID_E_DATA;
    *n_primes = (uint32_t)n;
    if (cap < n) return CUBOID_E_CAPACITY;
    std::vector<uint8_t> mine;
    std::vector<uint64_t> off;
    {
        CtxLock g(ctx);
        if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
        st = pack_all(ctx, sorted, &mine, &off);
        if (st) return st;
    }
    if (mine != tables) return CUBOID_E_DATA;
    std::copy(list.begin(), list.end(), primes_out);
    return CUBOID_OK;
}

}  // extern "C"
