// Micro-model storage, host cache and staging to the GPU (Eq. 2; Alg. 2).
//
// File: "FAM1" magic, int32 version, int32 nblocks, int32 reserved, then an
// index of (int64 offset, int64 size) per block, then the records.  A
// record is exactly the micro-model of Eq. 2: one header byte (the
// degree), the knot vectors of the three axes without their last knot
// (NCP + degree FP32 values each; a clamped vector on [0, 1] always ends in
// 1), and the NCP^3 FP32 control points [x][y][z], so its size is
// 1 + ((NCP + degree) * 3 + NCP^3) * 4 bytes and NCP follows from it.
//
// Cache: a fixed number of host slots (page-locked and mapped into the GPU's
// address space when asked for), least-recently-used replacement, a hit
// refreshing the block's recency.  Staging builds a table of (slot, knot and
// lattice destinations, descriptor) entries in mapped host memory and
// launches one gather kernel that reads the slots directly over the host
// link and writes the packed device batch (descriptors, knots, lattices at
// 64-element offsets): one launch per call instead of two copies per block.
// A slot is never refilled while a gather that reads it may still run: a
// call waits for the previous call's gather before touching the cache, and
// within a call the gather is launched (and waited for) before a batch
// reaches the cache's size, since only then could a refill hit one of its
// slots.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <vector>

#include "../../include/fa.h"
#include "fa_internal.hpp"

namespace {

constexpr char kMagic[4] = {'F', 'A', 'M', '1'};
constexpr int32_t kVersion = 1;
constexpr int64_t kHeader = 16;

int64_t record_bytes(int n, int p) { return 1 + ((int64_t)(n + p) * 3 + (int64_t)n * n * n) * 4; }

// NCP from a record size and degree (the inverse of Eq. 2); -1 if none fits
int ncp_from_size(int64_t size, int p) {
    for (int n = p + 1; n <= FA_MAX_NCP; ++n)
        if (record_bytes(n, p) == size) return n;
    return -1;
}

bool write_all(FILE *f, const void *p, size_t n) { return fwrite(p, 1, n, f) == n; }

bool read_at(int fd, void *dst, int64_t n, int64_t off) {
    char *d = static_cast<char *>(dst);
    while (n > 0) {
        const ssize_t r = pread(fd, d, (size_t)n, (off_t)off);
        if (r <= 0) return false;
        d += r;
        n -= r;
        off += r;
    }
    return true;
}

// A clamped knot vector of a record (n + p stored values, the last knot 1
// implicit): p + 1 leading zeros, p trailing stored ones, finite and
// non-decreasing -- the rules fa_validate_blocks applies to a batch.
bool knots_ok(const float *t, int n, int p) {
    for (int j = 0; j <= p; ++j)
        if (t[j] != 0.0f) return false;
    for (int j = n; j < n + p; ++j)
        if (t[j] != 1.0f) return false;
    for (int j = 1; j < n + p; ++j)
        if (!(t[j] >= t[j - 1]) || !(t[j] <= 1.0f)) return false;
    return true;
}

int64_t align64(int64_t v) { return (v + 63) / 64 * 64; }
int64_t knot_span(int n, int p) { return (3 * (int64_t)(n + p + 1) + 3) / 4 * 4; }

}  // namespace

struct fa_store {
    int fd = -1;
    int32_t nblocks = 0;
    std::vector<int64_t> off, size;
    std::vector<int32_t> ncp, deg;
    int32_t capacity = 0;
    bool pinned = false;
    int64_t slot_floats = 0;  // knots (padded to 4) + n^3 of the largest record
    float *slots = nullptr;
    const float *slots_dev = nullptr;  // device view of the mapped slots
    std::vector<char> raw;  // one record as read
    std::vector<int32_t> slot_of_block, block_of_slot;
    std::list<int32_t> lru;  // slots, most recently used first
    std::vector<std::list<int32_t>::iterator> where;
    fa::StageEntry *table = nullptr;  // mapped host table of one gather
    const fa::StageEntry *table_dev = nullptr;
    hipEvent_t stage_ev = nullptr;
    bool stage_live = false;
    fa_store_stats stats{};
};

namespace {

// Ensure block b is cached; returns its slot, kReadError on an I/O error or
// kFormatError for a record whose knots are not clamped and non-decreasing.
// The record is read and checked before the cache is touched, so a failure
// leaves the cache (slots, recency, counters) as it was.
constexpr int32_t kReadError = -1, kFormatError = -2;

int32_t fetch_one(fa_store *s, int32_t b) {
    int32_t slot = s->slot_of_block[b];
    if (slot >= 0) {
        s->stats.hits++;
        s->lru.splice(s->lru.begin(), s->lru, s->where[slot]);
        return slot;
    }
    const int n = s->ncp[b], p = s->deg[b];
    if (!read_at(s->fd, s->raw.data(), s->size[b], s->off[b])) return kReadError;
    for (int a = 0; a < 3; ++a) {
        float t[FA_MAX_NCP + FA_MAX_DEGREE];
        std::memcpy(t, s->raw.data() + 1 + (size_t)a * (n + p) * 4, (size_t)(n + p) * 4);
        if (!knots_ok(t, n, p)) return kFormatError;
    }
    s->stats.misses++;
    if ((int32_t)s->lru.size() < s->capacity) {
        slot = (int32_t)s->lru.size();
        s->lru.push_front(slot);
        s->where[slot] = s->lru.begin();
    } else {
        slot = s->lru.back();  // least recently used
        s->lru.splice(s->lru.begin(), s->lru, s->where[slot]);
        if (s->block_of_slot[slot] >= 0) s->slot_of_block[s->block_of_slot[slot]] = -1;
        s->stats.evictions++;
    }
    s->stats.bytes_read += s->size[b];
    float *dst = s->slots + (int64_t)slot * s->slot_floats;
    const char *src = s->raw.data() + 1;
    float *base = dst;
    for (int a = 0; a < 3; ++a) {
        std::memcpy(dst, src, (size_t)(n + p) * 4);
        dst[n + p] = 1.0f;  // the implicit last knot
        dst += n + p + 1;
        src += (size_t)(n + p) * 4;
    }
    std::memcpy(base + knot_span(n, p), src, (size_t)n * n * n * 4);
    s->slot_of_block[b] = slot;
    s->block_of_slot[slot] = b;
    return slot;
}

fa_status fetch_status(int32_t code) {
    return code == kFormatError ? FA_ERR_INVALID_ARG : FA_ERR_DEVICE;
}

// Wait for the gather of the previous fa_store_stage (it reads cache slots
// that a refill would overwrite).
bool wait_stage(fa_store *s) {
    if (!s->stage_live) return true;
    if (hipEventSynchronize(s->stage_ev) != hipSuccess) return false;
    s->stage_live = false;
    return true;
}

}  // namespace

extern "C" {

fa_status fa_store_write(const char *path, int32_t nblocks, const fa_block *blocks,
                         const float *knots, const float *ctrl) {
    if (!path || nblocks <= 0 || !blocks || !knots || !ctrl) return FA_ERR_INVALID_ARG;
    for (int32_t b = 0; b < nblocks; ++b) {
        const fa_block &B = blocks[b];
        const int n = B.ncp[0], p = B.degree[0];
        if (B.ncp[1] != n || B.ncp[2] != n || B.degree[1] != p || B.degree[2] != p || p < 1 ||
            n < p + 1)
            return FA_ERR_INVALID_ARG;  // Eq. 2 stores one NCP and one degree per block
        if (n > FA_MAX_NCP || p > FA_MAX_DEGREE) return FA_ERR_UNSUPPORTED;
        const float *t = knots + B.knot_off;
        for (int a = 0; a < 3; ++a)
            if (t[a * (n + p + 1) + n + p] != 1.0f || !knots_ok(t + a * (n + p + 1), n, p))
                return FA_ERR_INVALID_ARG;
    }
    FILE *f = fopen(path, "wb");
    if (!f) return FA_ERR_INVALID_ARG;
    bool ok = write_all(f, kMagic, 4) && write_all(f, &kVersion, 4) &&
              write_all(f, &nblocks, 4);
    const int32_t zero = 0;
    ok = ok && write_all(f, &zero, 4);
    int64_t off = kHeader + (int64_t)nblocks * 16;
    for (int32_t b = 0; b < nblocks && ok; ++b) {
        const int64_t sz = record_bytes(blocks[b].ncp[0], blocks[b].degree[0]);
        ok = write_all(f, &off, 8) && write_all(f, &sz, 8);
        off += sz;
    }
    for (int32_t b = 0; b < nblocks && ok; ++b) {
        const fa_block &B = blocks[b];
        const int n = B.ncp[0], p = B.degree[0];
        const uint8_t h = (uint8_t)p;
        ok = write_all(f, &h, 1);
        const float *t = knots + B.knot_off;
        for (int a = 0; a < 3 && ok; ++a) ok = write_all(f, t + a * (n + p + 1), (size_t)(n + p) * 4);
        ok = ok && write_all(f, ctrl + B.ctrl_off, (size_t)n * n * n * 4);
    }
    ok = (fclose(f) == 0) && ok;
    return ok ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_store_open(const char *path, int32_t cache_blocks, uint32_t flags, fa_store **out) {
    if (!path || cache_blocks <= 0 || !out || (flags & ~FA_STORE_PINNED) != 0)
        return FA_ERR_INVALID_ARG;
    *out = nullptr;
    const int fd = open(path, O_RDONLY);
    if (fd < 0) return FA_ERR_INVALID_ARG;
    fa_store *s = new fa_store();
    s->fd = fd;
    char magic[4];
    int32_t hdr[3];
    auto fail = [&](fa_status st) {
        fa_store_close(s);
        return st;
    };
    struct stat st;
    if (fstat(fd, &st) != 0) return fail(FA_ERR_INVALID_ARG);
    const int64_t fsize = (int64_t)st.st_size;
    if (!read_at(fd, magic, 4, 0) || std::memcmp(magic, kMagic, 4) != 0 ||
        !read_at(fd, hdr, 12, 4) || hdr[0] != kVersion || hdr[1] <= 0 ||
        kHeader + (int64_t)hdr[1] * 16 > fsize)
        return fail(FA_ERR_INVALID_ARG);
    s->nblocks = hdr[1];
    const int64_t first_record = kHeader + (int64_t)s->nblocks * 16;
    std::vector<int64_t> idx((size_t)s->nblocks * 2);
    if (!read_at(fd, idx.data(), (int64_t)idx.size() * 8, kHeader)) return fail(FA_ERR_INVALID_ARG);
    s->off.resize(s->nblocks);
    s->size.resize(s->nblocks);
    s->ncp.resize(s->nblocks);
    s->deg.resize(s->nblocks);
    int64_t maxsz = 0;
    for (int32_t b = 0; b < s->nblocks; ++b) {
        s->off[b] = idx[2 * b];
        s->size[b] = idx[2 * b + 1];
        // every record lies inside the file, after the index
        if (s->off[b] < first_record || s->size[b] < 1 || s->size[b] > fsize - s->off[b])
            return fail(FA_ERR_INVALID_ARG);
        uint8_t p = 0;
        if (!read_at(fd, &p, 1, s->off[b])) return fail(FA_ERR_INVALID_ARG);
        if (p < 1) return fail(FA_ERR_INVALID_ARG);
        if (p > FA_MAX_DEGREE) return fail(FA_ERR_UNSUPPORTED);
        const int n = ncp_from_size(s->size[b], p);
        if (n < 0) return fail(FA_ERR_INVALID_ARG);
        s->ncp[b] = n;
        s->deg[b] = p;
        s->slot_floats = std::max<int64_t>(s->slot_floats, knot_span(n, p) + (int64_t)n * n * n);
        maxsz = std::max(maxsz, s->size[b]);
    }
    s->capacity = cache_blocks;
    s->raw.resize((size_t)maxsz);
    s->slot_floats = (s->slot_floats + 3) / 4 * 4;  // 16-byte aligned slots
    const size_t bytes = (size_t)s->capacity * (size_t)s->slot_floats * 4;
    s->pinned = (flags & FA_STORE_PINNED) != 0;
    if (s->pinned) {
        void *p = nullptr, *d = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocMapped) != hipSuccess) return fail(FA_ERR_DEVICE);
        s->slots = static_cast<float *>(p);
        if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) return fail(FA_ERR_DEVICE);
        s->slots_dev = static_cast<const float *>(d);
        if (hipHostMalloc(&p, (size_t)s->capacity * sizeof(fa::StageEntry), hipHostMallocMapped) !=
            hipSuccess)
            return fail(FA_ERR_DEVICE);
        s->table = static_cast<fa::StageEntry *>(p);
        if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) return fail(FA_ERR_DEVICE);
        s->table_dev = static_cast<const fa::StageEntry *>(d);
        if (hipEventCreateWithFlags(&s->stage_ev, hipEventDisableTiming) != hipSuccess)
            return fail(FA_ERR_DEVICE);
    } else {
        s->slots = static_cast<float *>(std::malloc(bytes));
        if (!s->slots) return fail(FA_ERR_DEVICE);
    }
    s->slot_of_block.assign(s->nblocks, -1);
    s->block_of_slot.assign(s->capacity, -1);
    s->where.resize(s->capacity);
    *out = s;
    return FA_OK;
}

fa_status fa_store_close(fa_store *s) {
    if (!s) return FA_ERR_INVALID_ARG;
    if (s->pinned) {
        if (s->stage_ev) {
            if (s->stage_live) hipEventSynchronize(s->stage_ev);
            hipEventDestroy(s->stage_ev);
        }
        if (s->slots) hipHostFree(s->slots);
        if (s->table) hipHostFree(s->table);
    } else {
        std::free(s->slots);
    }
    if (s->fd >= 0) close(s->fd);
    delete s;
    return FA_OK;
}

fa_status fa_store_info(const fa_store *s, int32_t *nblocks, int32_t *ncp, int32_t *degree) {
    if (!s) return FA_ERR_INVALID_ARG;
    if (nblocks) *nblocks = s->nblocks;
    for (int32_t b = 0; b < s->nblocks; ++b) {
        if (ncp) ncp[b] = s->ncp[b];
        if (degree) degree[b] = s->deg[b];
    }
    return FA_OK;
}

fa_status fa_store_fetch(fa_store *s, const int32_t *ids, int32_t n, int32_t *slots,
                         fa_store_stats *stats) {
    if (!s || (n > 0 && !ids) || n < 0) return FA_ERR_INVALID_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (ids[i] < 0 || ids[i] >= s->nblocks) return FA_ERR_INVALID_ARG;
    // a gather of fa_store_stage may still read the slots this call refills
    if (s->pinned && !wait_stage(s)) return FA_ERR_DEVICE;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t slot = fetch_one(s, ids[i]);
        if (slot < 0) return fetch_status(slot);
        if (slots) slots[i] = slot;
    }
    if (stats) *stats = s->stats;
    return FA_OK;
}

fa_status fa_store_slot(const fa_store *s, int32_t slot, int32_t *block, const float **knots,
                        const float **ctrl) {
    if (!s || slot < 0 || slot >= s->capacity || s->block_of_slot[slot] < 0)
        return FA_ERR_INVALID_ARG;
    const int32_t b = s->block_of_slot[slot];
    const float *base = s->slots + (int64_t)slot * s->slot_floats;
    if (block) *block = b;
    if (knots) *knots = base;
    if (ctrl) *ctrl = base + knot_span(s->ncp[b], s->deg[b]);
    return FA_OK;
}

fa_status fa_store_stage(fa_store *s, const int32_t *ids, int32_t n, fa_block *dev_blocks,
                         float *dev_knots, int64_t knot_capacity, float *dev_ctrl,
                         int64_t ctrl_capacity, fa_store_stats *stats, void *stream) {
    if (!s || !s->pinned || n <= 0 || !ids || !dev_blocks || !dev_knots || !dev_ctrl ||
        n > s->nblocks)
        return FA_ERR_INVALID_ARG;
    int64_t kneed = 0, cneed = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (ids[i] < 0 || ids[i] >= s->nblocks) return FA_ERR_INVALID_ARG;
        const int nn = s->ncp[ids[i]], p = s->deg[ids[i]];
        kneed += 3 * (nn + p + 1);
        cneed = align64(cneed) + (int64_t)nn * nn * nn;
    }
    if (kneed > knot_capacity || align64(cneed) > ctrl_capacity) return FA_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    // the previous gather reads the table and its slots
    if (!wait_stage(s)) return FA_ERR_DEVICE;
    int32_t batch = 0;
    auto flush = [&](bool wait) -> bool {
        if (batch == 0) return true;
        if (fa::launch_stage_gather(s->table_dev, batch, s->slots_dev, dev_blocks, dev_knots,
                                    dev_ctrl, st) != hipSuccess ||
            hipEventRecord(s->stage_ev, st) != hipSuccess)
            return false;
        batch = 0;
        if (wait) return hipEventSynchronize(s->stage_ev) == hipSuccess;
        s->stage_live = true;
        return true;
    };
    int64_t ko = 0, co = 0;
    for (int32_t i = 0; i < n; ++i) {
        // a batch as large as the cache could see its own slots refilled
        if (batch == s->capacity && !flush(true)) return FA_ERR_DEVICE;
        const int32_t slot = fetch_one(s, ids[i]);
        if (slot < 0) {
            // entries already gathered into the table still go out
            if (!flush(false)) return FA_ERR_DEVICE;
            return fetch_status(slot);
        }
        const int nn = s->ncp[ids[i]], p = s->deg[ids[i]];
        const int64_t kl = 3 * (nn + p + 1), cl = (int64_t)nn * nn * nn;
        co = align64(co);
        const float *src = s->slots + (int64_t)slot * s->slot_floats;
        fa_block d{};
        for (int a = 0; a < 3; ++a) {
            d.ncp[a] = nn;
            d.degree[a] = p;
        }
        d.knot_off = ko;
        d.ctrl_off = co;
        d.scale = 1.0f;
        uint32_t fl = 0;
        for (int a = 0; a < 3; ++a) {  // uniform-knot flags, as fa_validate_blocks sets them
            const float *t = src + a * (nn + p + 1);
            bool uni = true;
            for (int j = 0; j <= nn - p && uni; ++j) uni = t[p + j] == (float)j / (float)(nn - p);
            if (uni) fl |= 1u << a;
        }
        d.flags = fl;
        fa::StageEntry &e = s->table[batch++];
        e.slot_off = (int64_t)slot * s->slot_floats;
        e.kdst = ko;
        e.cdst = co;
        e.kl = (int32_t)kl;
        e.koff = (int32_t)knot_span(nn, p);
        e.cl = cl;
        e.dst = i;
        e.desc = d;
        s->stats.bytes_h2d += (kl + cl) * 4 + (int64_t)sizeof(fa_block);
        ko += kl;
        co += cl;
    }
    if (!flush(false)) return FA_ERR_DEVICE;
    if (stats) *stats = s->stats;
    return FA_OK;
}

}  // extern "C"
