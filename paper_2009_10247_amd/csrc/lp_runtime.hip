// lp_runtime.hip -- device memory, matrix upload, fixpoint drivers and the C-ABI
// entry points. The kernels are in lp_step.hip (least models) and
// lp_spmm.hip (stable models); this file only launches them.
//
// Drivers of the Algorithm 1 loop:
//   PLAIN       one step launch per product, then the host reads the count;
//   BATCHED     steps_per_sync launches between host reads: a step whose
//               previous product changed nothing returns at once, so steps
//               issued past the fixpoint cost only a launch;
//   PERSISTENT  one cooperative launch runs every product on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <cstdlib>
#include <map>
#include <tuple>
#include <queue>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "lp_kernels.h"

namespace lp {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// ------------------------------------------------------------------ memory

static void *(*g_alloc)(size_t, void *, void *) = nullptr;
static void (*g_release)(void *, void *, void *) = nullptr;
static void *g_alloc_ctx = nullptr;
static std::atomic<int64_t> g_hook_live{0};  // blocks allocated through the hook and not yet released

static lp_status hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return LP_E_DEVICE;
}

#define LP_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// Caching pool behind the default allocation path. hipFree waits for the
// whole device, which would serialize solves running concurrently on other
// streams, so released blocks are kept for reuse. A block is handed back only
// once its last use has completed (Scratch synchronizes its stream first; a
// matrix or batch plan is released after its work is done), so a cached block
// may go to any stream. Sizes are rounded up to one of eight classes per
// power of two (at most 12.5% slack).
struct DevicePool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_blocks;  // (device, class) -> blocks
    std::unordered_map<void *, std::pair<int, size_t>> live;            // block -> (device, class)
    int64_t in_use = 0;
    int64_t cached = 0;
};

static DevicePool &pool() {
    static DevicePool *p = new DevicePool();  // never destroyed: blocks may be released at exit
    return *p;
}

static size_t size_class(size_t b) {
    if (b <= 4096) return (b + 255) & ~(size_t)255;
    int k = 63 - __builtin_clzll((unsigned long long)b);
    const size_t step = (size_t)1 << (k - 3);
    return (b + step - 1) & ~(step - 1);
}

// Frees every cached block of `device` (-1: all devices).
static void pool_trim(int device) {
    DevicePool &P = pool();
    std::vector<std::pair<int, void *>> victims;
    {
        std::lock_guard<std::mutex> lock(P.mu);
        for (auto it = P.free_blocks.begin(); it != P.free_blocks.end();) {
            if (device < 0 || it->first.first == device) {
                for (void *q : it->second) {
                    victims.emplace_back(it->first.first, q);
                    P.cached -= (int64_t)it->first.second;
                }
                it = P.free_blocks.erase(it);
            } else {
                ++it;
            }
        }
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    for (auto &v : victims) {
        (void)hipSetDevice(v.first);
        (void)hipFree(v.second);
    }
    if (prev >= 0) (void)hipSetDevice(prev);
}

static lp_status dev_alloc(void **p, size_t bytes, hipStream_t st) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (g_alloc) {
        *p = g_alloc(bytes, (void *)st, g_alloc_ctx);
        if (!*p) {
            set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
            return LP_E_NOMEM;
        }
        g_hook_live.fetch_add(1);
        return LP_OK;
    }
    int dev = 0;
    LP_HIP(hipGetDevice(&dev));
    const size_t cls = size_class(bytes);
    DevicePool &P = pool();
    {
        std::lock_guard<std::mutex> lock(P.mu);
        auto it = P.free_blocks.find({dev, cls});
        if (it != P.free_blocks.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            P.cached -= (int64_t)cls;
            P.in_use += (int64_t)cls;
            P.live[*p] = {dev, cls};
            return LP_OK;
        }
    }
    hipError_t e = hipMalloc(p, cls);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        pool_trim(dev);
        e = hipMalloc(p, cls);
    }
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc of " + std::to_string(bytes) + " bytes: out of memory");
        return LP_E_NOMEM;
    }
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    std::lock_guard<std::mutex> lock(P.mu);
    P.in_use += (int64_t)cls;
    P.live[*p] = {dev, cls};
    return LP_OK;
}

static void dev_free(void *p, hipStream_t st) {
    if (!p) return;
    if (g_release) {
        g_release(p, (void *)st, g_alloc_ctx);
        g_hook_live.fetch_sub(1);
        return;
    }
    DevicePool &P = pool();
    std::lock_guard<std::mutex> lock(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;  // not a pool block: nothing to do
    P.free_blocks[it->second].push_back(p);
    P.in_use -= (int64_t)it->second.second;
    P.cached += (int64_t)it->second.second;
    P.live.erase(it);
}

// LP_E_NOMEM unless `need` bytes fit in the device's free memory plus the
// pool's cached blocks (which are reused or trimmed before an allocation fails).
static lp_status check_device_memory(double need, const char *what) {
    size_t free_b = 0, total_b = 0;
    LP_HIP(hipMemGetInfo(&free_b, &total_b));
    double avail = (double)free_b;
    {
        DevicePool &P = pool();
        std::lock_guard<std::mutex> lock(P.mu);
        avail += (double)P.cached;
    }
    if (need > avail) {
        set_error(std::string(what) + " need " + std::to_string((long long)need) + " bytes of device memory, " +
                  std::to_string((long long)avail) + " available");
        return LP_E_NOMEM;
    }
    return LP_OK;
}

// Device buffers of one call: allocated from the pool (released, after the
// stream has synchronized, when the call ends), or carved in 256-byte steps
// from a fixed device region the caller owns (the no-allocation entry point).
struct Scratch {
    hipStream_t st;
    std::vector<void *> ptrs;
    uint8_t *region = nullptr;
    size_t region_size = 0, region_used = 0;
    explicit Scratch(hipStream_t s) : st(s) {}
    Scratch(hipStream_t s, void *fixed, size_t size) : st(s), region((uint8_t *)fixed), region_size(size) {}
    bool may_alloc() const { return region == nullptr; }
    template <class T>
    lp_status get(T **p, size_t count) {
        if (region) {
            const size_t b = std::max<size_t>(256, (count * sizeof(T) + 255) & ~(size_t)255);
            if (region_used + b > region_size) {
                set_error("the solve needs more than the " + std::to_string(region_size) +
                          " bytes of the fixed scratch region");
                return LP_E_INVAL;
            }
            *p = (T *)(region + region_used);
            region_used += b;
            return LP_OK;
        }
        void *q;
        lp_status rc = dev_alloc(&q, count * sizeof(T), st);
        if (rc) return rc;
        ptrs.push_back(q);
        *p = (T *)q;
        return LP_OK;
    }
    ~Scratch() {
        if (!ptrs.empty()) (void)hipStreamSynchronize(st);
        for (void *p : ptrs) dev_free(p, st);
    }
};

// Small pinned host buffer per thread for change counters.
static unsigned long long *pinned_ring() {
    static thread_local unsigned long long *p = nullptr;
    if (!p) {
        if (hipHostMalloc((void **)&p, sizeof(unsigned long long) * kRing, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
        }
    }
    return p;
}

// Pinned host staging of at least `bytes` per thread (grown on demand), for
// device-to-host copies that end a solve; nullptr if it cannot be allocated.
// Like the change-count ring, it is never freed at thread exit (the HIP
// runtime may already be gone by then).
static void *pinned_stage(size_t bytes) {
    struct Stage {
        void *p = nullptr;
        size_t size = 0;
    };
    static thread_local Stage s;
    if (s.size < bytes) {
        if (s.p) (void)hipHostFree(s.p);
        s.p = nullptr;
        s.size = 0;
        const size_t want = std::max<size_t>(bytes, 64 << 10);
        if (hipHostMalloc(&s.p, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s.p = nullptr;
            return nullptr;
        }
        s.size = want;
    }
    return s.p;
}

// ------------------------------------------------------------------ upload

static int64_t n_words_of(int64_t rows) { return (rows + 63) / 64; }

static std::vector<uint64_t> pack_bits(const std::vector<uint8_t> &x, int64_t words) {
    std::vector<uint64_t> w(words ? words : 1, 0);
    for (size_t i = 0; i < x.size(); ++i)
        if (x[i]) w[i >> 6] |= 1ull << (i & 63);
    return w;
}

template <class T>
static lp_status upload(T **d, const T *h, size_t count, hipStream_t st, int64_t *bytes) {
    lp_status rc = dev_alloc((void **)d, count * sizeof(T), st);
    if (rc) return rc;
    *bytes += (int64_t)(count * sizeof(T));
    if (count) LP_HIP(hipMemcpyAsync(*d, h, count * sizeof(T), hipMemcpyHostToDevice, st));
    return LP_OK;
}

struct DirtyState;  // below

// Stable-model solves by dirty rows of one matrix, kept between solves: the
// buffers (two interpretation matrices, the row bitmaps and their history)
// and a captured graph of the seed, the first kFirstBatch products and
// Algorithm 3's test. A solve leaves both interpretation buffers holding the
// initial matrix again (the rows it changed are set back to 0) and the
// bitmaps clear, so the next solve starts with the graph at once. One solve at a time uses it (try-lock);
// concurrent solves of the matrix take the allocating path.
struct StablePlan {
    std::mutex mu;
    bool ready = false;
    uint64_t *buf[2] = {nullptr, nullptr};
    uint32_t *sets = nullptr;  // row sets and history of the dirty-row products
    uint64_t *acc_d = nullptr;
    unsigned long long *cnt_d = nullptr;
    uint8_t *host = nullptr;  // pinned: |C_t| history (kDirtyHist int32), model count, accepted mask
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t bytes = 0;
};

static void release_plan(StablePlan *pl, hipStream_t st) {
    if (!pl) return;
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    for (void *p : {(void *)pl->buf[0], (void *)pl->buf[1], (void *)pl->sets, (void *)pl->acc_d, (void *)pl->cnt_d})
        dev_free(p, st);
    if (pl->host) (void)hipHostFree(pl->host);
    delete pl;
}

static void free_device(Matrix &m, hipStream_t st) {
    release_plan(m.dev.splan, st);
    m.dev.splan = nullptr;
    DeviceMatrix &d = m.dev;
    void *ps[] = {d.words,        d.and_len,       d.lens4,  d.col,      d.or_c0,  d.or_row,    d.fact_bits, d.segs, d.long_col,
                  d.full_row_ptr, d.full_col,      d.full_and_bits, d.q_rows, d.guess_pos};
    for (void *p : ps) dev_free(p, st);
    for (auto &wp : d.wave_parts) dev_free(wp.second, st);
    for (auto &sp : d.slice_parts) dev_free(sp.second, st);
    for (const SliceLayout &L : d.slices)
        for (void *p : {(void *)L.words, (void *)L.and_len, (void *)L.lens4, (void *)L.col}) dev_free(p, st);
    dev_free(d.and_all, st);
    for (void *p : {(void *)d.fr_ptr, (void *)d.fr_occ, (void *)d.fr_cnt0, (void *)d.fr_facts}) dev_free(p, st);
    d = DeviceMatrix{};
}

// AND entries as the kernels read them: the byte address of the 32-bit word
// of v holding atom c, shifted left by 5, and c's bit offset in that word in
// the low five bits.
static inline int32_t encode_entry(int32_t c) { return ((c >> 5) << 7) | (c & 31); }

// Least-model layout (see WordMeta and LongSeg): rows by kind, AND entries of
// block rows in col, OR rows as child ranges, long rows as segments.
// Words of v per column slice: what a workgroup's LDS stages in the step
// with the most chunks in flight (even: slices are staged with 16-byte loads),
// or 16 words (1,024 atoms) with LP_STEP_SLICES_SMALL.
static int32_t slice_words(const Matrix &m) {
    if (m.flags & LP_STEP_SLICES_SMALL) return 16;
    return step_lds_v_words(16) & ~1;
}

// Column-sliced layout of the block AND rows, when their columns span more
// than one slice: slice k holds, for every block AND row, its entries with
// columns in [64 k S, 64 (k + 1) S) (S = slice_words; entries are ascending
// within a row, so they are a contiguous part of it), relative to the slice,
// in the same form as the whole layout (words, lengths, lens4, entries).
static lp_status build_slices(Matrix &m, const std::vector<uint64_t> &and_all, hipStream_t st) {
    DeviceMatrix &d = m.dev;
    if (m.K != 0 || d.and_max_col < 0) return LP_OK;
    const int64_t S = slice_words(m), cols = 64 * S;
    const int64_t n_slices = (int64_t)d.and_max_col / cols + 1;
    if (n_slices < 2) return LP_OK;
    if (n_slices > kMaxSlices) {
        set_error("the least-model layout would need " + std::to_string(n_slices) + " column slices (at most " +
                  std::to_string(kMaxSlices) + ")");
        return LP_E_INVAL;
    }
    const int32_t n = m.n_rows;
    const int64_t W = n_words_of(n);
    lp_status rc;
    int64_t extra = 0;
    for (int64_t k = 0; k < n_slices; ++k) {
        const int32_t c_lo = (int32_t)(k * cols), c_hi = (int32_t)std::min<int64_t>((k + 1) * cols, INT32_MAX);
        std::vector<WordMeta> words(W + kWordPad);
        std::vector<uint8_t> and_len((size_t)(W + kWordPad) * 64, 0);
        std::vector<int32_t> col;
        int32_t max_col = -1;
        for (int32_t i = 0; i < n; ++i) {
            const int64_t w = i >> 6;
            if ((i & 63) == 0) {
                words[w] = WordMeta{};
                words[w].and_base = (int32_t)col.size();
            }
            if (!((and_all[w] >> (i & 63)) & 1ull)) continue;  // block AND rows only
            const int32_t *b = m.col.data() + m.row_ptr[i], *e = m.col.data() + m.row_ptr[i + 1];
            const int32_t *lo = std::lower_bound(b, e, c_lo), *hi = std::lower_bound(lo, e, c_hi);
            if (lo == hi) continue;
            words[w].and_bits |= 1ull << (i & 63);
            and_len[i] = (uint8_t)(hi - lo);
            for (const int32_t *c = lo; c < hi; ++c) {
                col.push_back(encode_entry(*c - c_lo));
                max_col = std::max(max_col, *c - c_lo);
            }
        }
        for (int64_t w = W; w < W + kWordPad; ++w) {
            words[w] = WordMeta{};
            words[w].and_base = (int32_t)col.size();
        }
        std::vector<int32_t> base((size_t)W + 1);
        for (int64_t w = 0; w < W; ++w) base[w] = words[w].and_base;
        base[W] = (int32_t)col.size();
        const int32_t n_entries = (int32_t)col.size();
        col.insert(col.end(), kColPad, 0);
        const int64_t n_quads = (W + kWordPad + 3) / 4;
        std::vector<uint32_t> lens4((size_t)n_quads * 64, 0);
        for (int64_t q = 0; q < n_quads; ++q)
            for (int j = 0; j < 4; ++j) {
                const int64_t w = 4 * q + j;
                if (w >= W + kWordPad) break;
                for (int l = 0; l < 64; ++l) lens4[q * 64 + l] |= (uint32_t)and_len[w * 64 + l] << (8 * j);
            }
        WordMeta *dw;
        uint8_t *dl;
        uint32_t *d4;
        int32_t *dc;
        if ((rc = upload(&dw, words.data(), words.size(), st, &d.bytes)) ||
            (rc = upload(&dl, and_len.data(), and_len.size(), st, &d.bytes)) ||
            (rc = upload(&d4, lens4.data(), lens4.size(), st, &d.bytes)) ||
            (rc = upload(&dc, col.data(), col.size(), st, &d.bytes)))
            return rc;
        SliceLayout L{};
        L.words = dw;
        L.and_len = dl;
        L.lens4 = d4;
        L.col = dc;
        L.and_end = n_entries;
        L.and_max_col = max_col;
        L.first_word = (int32_t)(k * S);
        L.lds_words = (int32_t)std::max<int64_t>(0, std::min<int64_t>(S, W - k * S));
        d.slices.push_back(L);
        d.slice_base.push_back(std::move(base));
        LP_HIP(hipStreamSynchronize(st));  // the host vectors end here
        extra += n + 4 * ((W + 3) / 4) + 4 * (int64_t)n_entries;
    }
    if ((rc = upload(&d.and_all, and_all.data(), and_all.size(), st, &d.bytes))) return rc;
    // what a sliced step streams: every slice's lengths, word offsets and
    // entries, the long rows, OR tables and segments, and the partial AND
    // words (written by the first pass, read and written by the others)
    d.stream_bytes += extra - (n + 4 * ((W + 3) / 4) + 4 * d.and_nnz) + 2 * n_slices * W * 8;
    return LP_OK;
}

static lp_status upload_least_layout(Matrix &m, hipStream_t st) {
    DeviceMatrix &d = m.dev;
    const int32_t n = m.n_rows;
    const int64_t W = n_words_of(n);
    // kWordPad words (and their rows) past the end: the step kernels load the
    // row data of a super-block without bounds checks
    std::vector<WordMeta> words(W + kWordPad);
    std::vector<uint8_t> and_len((size_t)(W + kWordPad) * 64, 0);
    std::vector<int32_t> col, lcol, or_c0, or_row;
    std::vector<LongSeg> segs;
    col.reserve(m.col.size());
    int32_t n_long_and = 0, max_col = -1, n_or = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t w = i >> 6;
        const uint64_t bit = 1ull << (i & 63);
        if ((i & 63) == 0) {
            words[w] = WordMeta{};
            words[w].and_base = (int32_t)col.size();
            words[w].or_idx = n_or;  // OR rows before this word
        }
        const int32_t s = m.row_ptr[i], e = m.row_ptr[i + 1], len = e - s;
        if (m.fact[i] || len == 0) continue;  // facts: true from v0 on; empty rows: never true
        if (m.kind[i]) {
            if (len > kLongAnd) {
                words[w].long_bits |= bit;
                const int32_t nseg = (len + kSegAnd - 1) / kSegAnd;
                const int32_t slot = nseg > 1 ? n_long_and++ : -1;
                for (int32_t q = 0; q < nseg; ++q) {
                    LongSeg sg{};
                    sg.row = i;
                    sg.is_and = 1;
                    sg.begin = (int64_t)lcol.size() + (int64_t)q * kSegAnd;
                    sg.len = std::min(kSegAnd, len - q * kSegAnd);
                    sg.nseg = nseg;
                    sg.and_slot = slot;
                    sg.seg = q;
                    segs.push_back(sg);
                }
                for (int32_t j = s; j < e; ++j) lcol.push_back(encode_entry(m.col[j]));
            } else {
                words[w].and_bits |= bit;
                and_len[i] = (uint8_t)len;
                for (int32_t j = s; j < e; ++j) col.push_back(encode_entry(m.col[j]));
            }
            for (int32_t j = s; j < e; ++j) max_col = std::max(max_col, m.col[j]);
        } else {
            // OR row: children are consecutive ids and follow the previous OR row's children
            const int32_t c0 = m.col[s];
            for (int32_t j = s; j < e; ++j)
                if (m.col[j] != c0 + (j - s)) {
                    set_error("OR row children are not consecutive");
                    return LP_E_INTERNAL;
                }
            if (!or_c0.empty() && or_c0.back() != c0) {
                set_error("OR rows' child ranges are not contiguous");
                return LP_E_INTERNAL;
            }
            if (or_c0.empty()) or_c0.push_back(c0);
            or_c0.push_back(c0 + len);  // or_c0[j] is the start of OR row j, or_c0[j+1] its end
            or_row.push_back(len > kLongOrBits ? -1 : i);
            ++n_or;
            words[w].or_bits |= bit;
            if (len > kLongOrBits) {
                words[w].long_bits |= bit;
                const int32_t nseg = (len + kSegOrBits - 1) / kSegOrBits;
                for (int32_t q = 0; q < nseg; ++q) {
                    LongSeg sg{};
                    sg.row = i;
                    sg.is_and = 0;
                    sg.begin = (int64_t)c0 + (int64_t)q * kSegOrBits;
                    sg.len = std::min(kSegOrBits, len - q * kSegOrBits);
                    sg.nseg = nseg;
                    sg.and_slot = -1;
                    sg.seg = q;
                    segs.push_back(sg);
                }
            }
        }
    }
    d.n_or = n_or;
    for (int64_t w = W; w < W + kWordPad; ++w) {
        words[w] = WordMeta{};
        words[w].and_base = (int32_t)col.size();
        words[w].or_idx = n_or;
    }
    if (max_col >= (1 << 26)) {
        set_error("least-model layout supports at most 2^26 rows");
        return LP_E_INVAL;
    }
    d.and_nnz = (int64_t)col.size();
    d.word_base.resize((size_t)W + 1);
    for (int64_t w = 0; w < W; ++w) d.word_base[w] = words[w].and_base;
    d.word_base[W] = (int32_t)d.and_nnz;
    d.long_nnz = (int64_t)lcol.size();
    d.n_segs = (int32_t)segs.size();
    d.n_long_and = n_long_and;
    d.and_max_col = max_col;
    if (or_c0.empty()) or_c0.push_back(0);
    if (or_row.empty()) or_row.push_back(-1);
    col.insert(col.end(), kColPad, 0);  // chunk loads of the last rounds read up to 64*U past the end
    lp_status rc;
    if ((rc = upload(&d.words, words.data(), words.size(), st, &d.bytes))) return rc;
    if ((rc = upload(&d.and_len, and_len.data(), and_len.size(), st, &d.bytes))) return rc;
    {
        const int64_t n_quads = (W + kWordPad + 3) / 4;
        std::vector<uint32_t> lens4((size_t)n_quads * 64, 0);
        for (int64_t q = 0; q < n_quads; ++q)
            for (int k = 0; k < 4; ++k) {
                const int64_t w = 4 * q + k;
                if (w >= W + kWordPad) break;
                for (int l = 0; l < 64; ++l) lens4[q * 64 + l] |= (uint32_t)and_len[w * 64 + l] << (8 * k);
            }
        if ((rc = upload(&d.lens4, lens4.data(), lens4.size(), st, &d.bytes))) return rc;
    }
    if ((rc = upload(&d.col, col.data(), col.size(), st, &d.bytes))) return rc;
    if ((rc = upload(&d.or_c0, or_c0.data(), or_c0.size(), st, &d.bytes))) return rc;
    if ((rc = upload(&d.or_row, or_row.data(), or_row.size(), st, &d.bytes))) return rc;
    if ((rc = upload(&d.segs, segs.data(), segs.size(), st, &d.bytes))) return rc;
    if ((rc = upload(&d.long_col, lcol.data(), lcol.size(), st, &d.bytes))) return rc;
    // what one step reads of the layout: the 8-bit AND lengths, the first AND
    // entry of every super-block (at most one per four words), the AND entries,
    // the OR range table and the long-row segments
    d.stream_bytes = n + 4 * ((W + 3) / 4) + 4 * (d.and_nnz + d.long_nnz) +
                     4 * (int64_t)(or_c0.size() + or_row.size()) + (int64_t)sizeof(LongSeg) * d.n_segs;
    // the block AND rows of every word, for a sliced step
    std::vector<uint64_t> and_all(W ? W : 1, 0);
    for (int64_t w = 0; w < W; ++w) and_all[w] = words[w].and_bits;
    return build_slices(m, and_all, st);
}

static lp_status ensure_frontier(const Matrix &m, hipStream_t st);
static bool dirty_products(const Matrix &m, int32_t log2W);
static int ilog2(int64_t x);
static bool lds_loop_fits(const Matrix &m);
static StepParams step_params(const Matrix &m);
static lp_status plan_step(const Matrix &m, const lp_schedule *sched, StepParams &p, StepShape *S, hipStream_t st,
                           bool may_alloc = true, bool slices = true);

static lp_status upload_matrix(Matrix &m, hipStream_t st) {
    DeviceMatrix &d = m.dev;
    LP_HIP(hipGetDevice(&d.device));
    const int64_t W = n_words_of(m.n_rows);
    std::vector<uint64_t> fact = pack_bits(m.fact, W);
    lp_status rc;
    if ((rc = upload(&d.fact_bits, fact.data(), fact.size(), st, &d.bytes))) return rc;
    if (m.K == 0) {
        if ((rc = upload_least_layout(m, st))) return rc;
    } else {
        std::vector<uint64_t> andb = pack_bits(m.kind, W);
        std::vector<int32_t> qrows(m.neg_atoms);
        if ((rc = upload(&d.full_row_ptr, m.row_ptr.data(), m.row_ptr.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.full_col, m.col.data(), m.col.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.full_and_bits, andb.data(), andb.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.q_rows, qrows.data(), qrows.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.guess_pos, m.guess_pos.data(), m.guess_pos.size(), st, &d.bytes))) return rc;
    }
    LP_HIP(hipStreamSynchronize(st));
    m.info.device_bytes = d.bytes;
    // stable solves by dirty rows read the transposed matrix: build it now,
    // so the device bytes reported from here on include it
    if (m.K > 0 && m.K_eff <= LP_MAX_NEG_ATOMS &&
        dirty_products(m, ilog2((((int64_t)1 << m.K_eff) + 63) / 64)) && (rc = ensure_frontier(m, st)))
        return rc;
    // the default driver's step split, so a solve with the default schedule
    // (lp_least_model_noalloc in particular) attaches nothing
    if (m.K == 0 && m.n_rows > 0 && !lds_loop_fits(m)) {
        StepParams p = step_params(m);
        StepShape S;
        if ((rc = plan_step(m, nullptr, p, &S, st))) return rc;
    }
    const int64_t vbytes = (m.n_rows + 7) / 8;
    if (m.K == 0) {
        m.info.step_bytes = d.stream_bytes + 2 * vbytes;
    } else if (m.K_eff <= LP_MAX_NEG_ATOMS) {
        const int keff = m.K_eff;
        const int64_t wbytes = ((((int64_t)1 << keff) + 63) / 64) * 8;
        m.info.step_bytes = 4 * ((int64_t)m.n_rows + 1) + 4 * m.nnz + vbytes + 2 * (int64_t)m.n_rows * wbytes;
    } else {
        m.info.step_bytes = 0;  // the guesses cannot be enumerated: the width depends on the guesses given
    }
    return LP_OK;
}

// ------------------------------------------------------------------ drivers

// Guards the structures attached to a matrix on first use (wave splits,
// transposed matrix) and their byte count.
static std::mutex g_lazy_mu;

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (dev >= 0 && hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

struct DevProps {
    int n_cu = 0;
    int max_lds = 0;
};

static lp_status dev_props(int dev, DevProps *out) {
    static std::mutex mu;
    static DevProps cache[64];
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) {
        set_error("device id out of range");
        return LP_E_DEVICE;
    }
    if (cache[dev].n_cu == 0) {
        DevProps d;
        LP_HIP(hipDeviceGetAttribute(&d.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        LP_HIP(hipDeviceGetAttribute(&d.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        if (d.max_lds > 4096) {
            batch_kernels_allow_lds(d.max_lds - 4096);
            frontier_kernels_allow_lds(d.max_lds - 4096);
        }
        cache[dev] = d;
    }
    *out = cache[dev];
    return LP_OK;
}

static StepParams step_params(const Matrix &m) {
    const DeviceMatrix &d = m.dev;
    StepParams p{};
    p.words = d.words;
    p.and_len = d.and_len;
    p.lens4 = d.lens4;
    p.col = d.col;
    p.or_c0 = d.or_c0;
    p.or_row = d.or_row;
    p.n_or = d.n_or;
    p.segs = d.segs;
    p.long_col = d.long_col;
    p.n_rows = m.n_rows;
    p.and_end = (int32_t)d.and_nnz;
    p.and_max_col = d.and_max_col;
    p.n_long_and = d.n_long_and;
    p.n_segs = d.n_segs;
    p.early_exit = 1;
    p.and_all = d.and_all;
    return p;
}

// Per-word cost of the block pass split, in AND entries. A word's row data
// (lengths, scans, the result) is cheap in dense stretches, but where words
// have few entries a round ends several super-blocks and each further one
// waits for its row data; measured on MI355X, the split balances best with a
// word counted as about 600 entries (the benchmark program has ~245 AND
// entries per word on average, with a stretch of sparse words).
constexpr int64_t kWordCost = 600;
// Cost of an OR tile and of a long-row segment in the same units: a wave that
// evaluates them gets that much less of the block pass.
constexpr int64_t kOrTileCost = 1600;
constexpr int64_t kSegCost = 1600;

// Split of the block pass between `waves` waves: wave k takes the words
// [t[2k], t[2k + 2]) and t[2k + 1] is the first AND entry of word t[2k]. Each
// wave gets about the same cost (AND entries + kWordCost per word of its
// block pass, plus its OR tiles and segments), so the waves end together.
// b: the layout's first AND entry of every word, then the entry count.
static lp_status split_waves(const std::vector<int32_t> &b, int64_t n_tiles, int64_t n_segs, int32_t waves,
                             hipStream_t st, int32_t **out, int64_t *bytes) {
    const int64_t W = (int64_t)b.size() - 1;
    // wave k also evaluates OR tiles k, k + waves, ... and segments k, k + waves, ...
    auto extra = [&](int64_t k) -> int64_t {
        const int64_t tiles = k < n_tiles ? (n_tiles - 1 - k) / waves + 1 : 0;
        const int64_t segs = k < n_segs ? (n_segs - 1 - k) / waves + 1 : 0;
        return kOrTileCost * tiles + kSegCost * segs;
    };
    int64_t total = (int64_t)b[W] + kWordCost * W;
    for (int64_t k = 0; k < waves; ++k) total += extra(k);
    std::vector<int32_t> t(2 * ((size_t)waves + 1));
    int64_t w = 0, cut = 0;  // cut: block-pass cost before wave k's first word
    for (int32_t k = 0; k < waves; ++k) {
        while (w < W && (int64_t)b[w] + kWordCost * w < cut) ++w;
        t[2 * (size_t)k] = (int32_t)w;
        t[2 * (size_t)k + 1] = b[w];
        cut += std::max<int64_t>(0, total / waves - extra(k));
    }
    t[2 * (size_t)waves] = (int32_t)W;
    t[2 * (size_t)waves + 1] = b[W];
    lp_status rc = upload(out, t.data(), t.size(), st, bytes);
    if (rc) return rc;
    LP_HIP(hipStreamSynchronize(st));  // t is a local
    return LP_OK;
}

// The split of the whole layout (slice < 0) or of column slice `slice` for
// `waves` waves, created once and kept with the matrix's device arrays. OR
// tiles and segments count in the whole layout's split and in the last
// slice's (a sliced step evaluates them in its last pass).
static lp_status wave_partition(const Matrix &m, int32_t waves, hipStream_t st, const int32_t **out,
                                bool may_alloc = true, int32_t slice = -1) {
    std::lock_guard<std::mutex> lock(g_lazy_mu);
    const DeviceMatrix &d = m.dev;
    const int64_t key = slice < 0 ? (int64_t)waves : ((int64_t)slice << 32) | (uint32_t)waves;
    if (slice < 0) {
        for (const auto &wp : d.wave_parts)
            if (wp.first == waves) {
                *out = wp.second;
                return LP_OK;
            }
    } else {
        for (const auto &sp : d.slice_parts)
            if (sp.first == key) {
                *out = sp.second;
                return LP_OK;
            }
    }
    if (!may_alloc) {
        set_error("no step split for " + std::to_string(waves) + " waves was made at upload");
        return LP_E_INTERNAL;
    }
    const std::vector<int32_t> &b = slice < 0 ? d.word_base : d.slice_base[slice];
    if (b.empty() || waves < 1) {
        set_error("no least-model layout to split");
        return LP_E_INTERNAL;
    }
    const bool with_or = slice < 0 || slice == (int32_t)d.slices.size() - 1;
    int32_t *dp = nullptr;
    int64_t bytes = 0;
    lp_status rc = split_waves(b, with_or ? ((int64_t)d.n_or + 63) / 64 : 0, with_or ? d.n_segs : 0, waves, st,
                               &dp, &bytes);
    if (rc) return rc;
    if (slice < 0) d.wave_parts.emplace_back(waves, dp);
    else d.slice_parts.emplace_back(key, dp);
    d.lazy_bytes += bytes;
    *out = dp;
    return LP_OK;
}

// Launch shape of the step for a whole solve. LDS shapes use one 1024-thread
// workgroup per CU (the staged v takes most of the CU's LDS); global shapes
// use 256-thread workgroups, eight per CU. A matrix with a column-sliced
// layout takes the sliced LDS step (one pass per slice) unless slices is
// false (then the mixed form).
static lp_status plan_step(const Matrix &m, const lp_schedule *sched, StepParams &p, StepShape *S, hipStream_t st,
                           bool may_alloc, bool slices) {
    int variant = sched ? sched->variant : LP_STEP_AUTO;
    if (variant == LP_STEP_AUTO) variant = LP_STEP_LDS;
    if (variant != LP_STEP_LDS && variant != LP_STEP_GLOBAL) {
        set_error("unknown step variant");
        return LP_E_INVAL;
    }
    DevProps d;
    lp_status rc = dev_props(m.dev.device, &d);
    if (rc) return rc;
    StepShape s;
    const bool staged = variant == LP_STEP_LDS;
    s.wpw = sched && sched->wpw > 0 ? sched->wpw : 8;
    s.unroll = sched && sched->unroll > 0 ? sched->unroll : (staged ? 16 : 8);
    if (!step_shape_supported(s)) {
        set_error("unsupported step shape (words per super-block 4 or 8, chunks in flight 4, 8 or 16)");
        return LP_E_INVAL;
    }
    const int64_t n_words = n_words_of(m.n_rows);
    if (staged) {
        if (d.max_lds < kStepLdsBytes) {
            set_error("the LDS-staged step needs 160 KB of LDS per workgroup");
            return LP_E_DEVICE;
        }
        p.lds_words = (int32_t)std::min<int64_t>({(int64_t)step_lds_v_words(s.unroll), n_words_of(m.n_atoms), n_words});
        s.mode = (int64_t)m.dev.and_max_col < (int64_t)p.lds_words * 64 ? kStepLds : kStepMixed;
        if (slices && !m.dev.slices.empty()) {
            s.mode = kStepSlice;
            s.n_slices = (int)m.dev.slices.size();
            s.slice = m.dev.slices.data();
        }
        s.block = 1024;
    } else {
        p.lds_words = 0;
        s.mode = kStepGlobal;
        s.block = 256;
    }
    const int waves = s.block / 64;
    const int64_t items = std::max<int64_t>({(n_words + s.wpw - 1) / s.wpw, (int64_t)p.n_segs,
                                             ((int64_t)p.n_or + 63) / 64});
    const int64_t want = std::max<int64_t>(1, (items + waves - 1) / waves);
    const int64_t dflt = staged ? d.n_cu : (int64_t)d.n_cu * 8;
    const int64_t grid = sched && sched->grid > 0 ? sched->grid : dflt;
    s.grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, want));
    for (int k = 0; k < s.n_slices; ++k)
        if ((rc = wave_partition(m, s.grid * waves, st, &s.slice_part[k], may_alloc, k))) return rc;
    *S = s;
    return wave_partition(m, s.grid * waves, st, &p.wave_part, may_alloc);
}

// Shape of the persistent fixpoint: the LDS step with at most as many
// workgroups as can be resident at once (the grid barrier needs all of them
// running). S->grid = 0 if not even one fits.
static lp_status plan_persistent(const Matrix &m, const lp_schedule *sched, StepParams &p, StepShape *S,
                                 hipStream_t st) {
    lp_schedule s2 = sched ? *sched : lp_schedule{};
    s2.variant = LP_STEP_LDS;
    lp_status rc = plan_step(m, &s2, p, S, st, true, false);  // the persistent kernel has no sliced form
    if (rc) return rc;
    int per_cu = 0;
    LP_HIP(persistent_occupancy(*S, &per_cu));
    DevProps d;
    if ((rc = dev_props(m.dev.device, &d))) return rc;
    const int64_t resident = (int64_t)per_cu * d.n_cu;
    S->grid = (int)std::min<int64_t>(S->grid, resident);
    if (S->grid < 1) return LP_OK;
    return wave_partition(m, S->grid * (S->block / 64), st, &p.wave_part);
}

// res: int32[4] device scratch (result, barrier count, abort flag).
static lp_status run_persistent(const Matrix &m, const StepParams &p, const StepShape &S, uint64_t *const buf[2],
                                int32_t *res, hipStream_t st) {
    PersistParams q{};
    q.p = p;
    q.buf0 = buf[0];
    q.buf1 = buf[1];
    q.max_steps = (int32_t)std::min<int64_t>((int64_t)m.n_rows + 1, INT32_MAX - 1);
    q.result = res;
    q.bar = reinterpret_cast<uint32_t *>(res + 1);
    q.abort = res + 2;
    LP_HIP(hipMemsetAsync(res, 0, 4 * sizeof(int32_t), st));
    LP_HIP(launch_persistent(S, q, st));
    return LP_OK;
}

// Least-model fixpoint. On success *out points at the device buffer holding
// the fixpoint (one of bufs[0..1]).
static lp_status frontier_fixpoint(const Matrix &m, hipStream_t st, Scratch &S, uint64_t **out, int32_t *products);

// Small programs under the automatic driver: the whole Algorithm 1 loop in
// one workgroup with both interpretations in LDS (tp_batch_kernel on a
// one-program queue): one launch and no grid-wide synchronization, where the
// other drivers pay a launch or a grid barrier per product. Everything the
// kernel reads or writes is allocated per call, so concurrent solves of one
// matrix on several streams stay independent.
constexpr int64_t kLdsLoopMaxWork = 1 << 17;  // stored entries + rows

static bool lds_loop_fits(const Matrix &m) {
    return m.dev.and_nnz + m.dev.long_nnz + m.n_rows <= kLdsLoopMaxWork && n_words_of(m.n_rows) * 16 <= 48 * 1024;
}

// *out holds the fixpoint's first ceil(n_atoms / 64) words only (the model),
// not a whole interpretation of n_rows bits. With host_bits (nullable) those
// words are also copied to the host, in the same copy as the product count.
// Device memory of a one-workgroup solve: the product count, then the
// model's words (the descriptor travels in the kernel arguments).
constexpr size_t kLdsLoopHead = 256;

// Descriptor of m for the batch kernel (outputs not set).
static ProgDesc prog_desc(const Matrix &m) {
    const DeviceMatrix &dm = m.dev;
    ProgDesc g{};
    g.words = dm.words;
    g.and_len = dm.and_len;
    g.lens4 = dm.lens4;
    g.col = dm.col;
    g.or_c0 = dm.or_c0;
    g.or_row = dm.or_row;
    g.segs = dm.segs;
    g.long_col = dm.long_col;
    g.fact_bits = dm.fact_bits;
    g.n_rows = m.n_rows;
    g.n_atoms = m.n_atoms;
    g.n_or = dm.n_or;
    g.n_segs = dm.n_segs;
    g.and_end = (int32_t)dm.and_nnz;
    g.team_size = 1;
    g.long_nnz = (int32_t)dm.long_nnz;
    return g;
}

// LDS bytes of m's layout in the batch kernel's LDS form.
static int64_t layout_lds_bytes(const Matrix &m) {
    return lds_layout(m.n_rows, m.dev.and_nnz, m.dev.n_or, m.dev.n_segs, m.dev.long_nnz).end;
}

static lp_status lds_loop_fixpoint(const Matrix &m, hipStream_t st, Scratch &S, uint64_t **out, int32_t *products,
                                  uint64_t *host_bits = nullptr) {
    const size_t head = kLdsLoopHead;
    const int64_t Wa = std::max<int64_t>(1, n_words_of(m.n_atoms));
    uint8_t *blk;
    lp_status rc;
    if ((rc = S.get(&blk, head + (size_t)Wa * 8))) return rc;
    int32_t *d_prods = reinterpret_cast<int32_t *>(blk);
    uint64_t *bits = reinterpret_cast<uint64_t *>(blk + head);
    DevProps dp;
    if ((rc = dev_props(m.dev.device, &dp))) return rc;
    BatchParams q{};
    q.single = 1;
    q.one = prog_desc(m);
    q.one.out_bits = bits;
    q.one.out_products = d_prods;
    q.n_items = 1;
    q.lds_words = (int32_t)n_words_of(m.n_rows);
    // the layout goes into LDS beside the two buffers when both fit
    const int64_t v_bytes = (int64_t)q.lds_words * 16, lay = layout_lds_bytes(m);
    if (v_bytes + lay <= (int64_t)dp.max_lds - 4096) q.lds_layout_bytes = (int32_t)lay;
    if (q.lds_layout_bytes > 0 && tiny_fits(m.n_rows, m.dev.n_or, m.dev.n_segs))
        LP_HIP(launch_tiny(q.one, q.lds_words, (size_t)(v_bytes + lay), st));  // rows kept in registers
    else
        LP_HIP(launch_batch(kBatchWpw, kBatchUnroll, 1, 1024, (size_t)(v_bytes + q.lds_layout_bytes), q, st));
    int32_t prods = 0;
    if (host_bits) {
        // the product count and the model bits in one copy: [products, pad .. last word of bits]
        const size_t n = head + (size_t)n_words_of(m.n_atoms) * 8;
        uint8_t *stage = reinterpret_cast<uint8_t *>(S.may_alloc() ? pinned_stage(n) : nullptr);
        std::vector<uint8_t> local;
        if (!stage) {
            local.resize(n);
            stage = local.data();
        }
        LP_HIP(hipMemcpyAsync(stage, blk, n, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        std::memcpy(&prods, stage, sizeof(int32_t));
        std::memcpy(host_bits, stage + head, (size_t)n_words_of(m.n_atoms) * 8);
    } else {
        LP_HIP(hipMemcpyAsync(&prods, d_prods, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
    }
    if (prods < 1) {
        set_error("fixpoint not reached within n_rows+1 products");
        return LP_E_INTERNAL;
    }
    *products = prods;
    *out = bits;
    return LP_OK;
}

// With host_bits (nullable), *on_host tells whether the first ceil(n_atoms / 64)
// words of the fixpoint were already copied there.
// ------------------------------------------------------------------ schedule cache
//
// Schedules found by lp_tune_schedule, kept per size bucket of the matrix:
// whether v fits a workgroup's LDS (the step's gather form), the rows'
// ceil log2, the mean AND row length in half entries, and whether long rows
// exist. The default driver solves a matrix whose bucket holds a schedule
// with that schedule. The cache lives in the process; lp_schedule_cache_save
// and _load keep it in a text file, and with LP_SCHEDULE_CACHE naming a file
// the library loads it on first use and saves it after every tune.

struct SchedKey {
    int32_t lds = 0, log2_rows = 0, len_q = 0, long_rows = 0;
    bool operator<(const SchedKey &o) const {
        return std::tie(lds, log2_rows, len_q, long_rows) < std::tie(o.lds, o.log2_rows, o.len_q, o.long_rows);
    }
};

static std::mutex g_sched_mu;
static std::map<SchedKey, lp_schedule> g_sched;
static bool g_sched_env_done = false;

static int ceil_log2(int64_t x) {
    int l = 0;
    while ((1ll << l) < x) ++l;
    return l;
}

static SchedKey sched_key(const Matrix &m) {
    SchedKey k;
    k.lds = n_words_of(m.n_atoms) <= step_lds_v_words(16) ? 1 : 0;
    k.log2_rows = ceil_log2(std::max(1, m.n_rows));
    const int64_t and_rows = std::max<int64_t>(1, m.info.n_and_rows);
    k.len_q = (int32_t)std::min<int64_t>(64, (2 * (m.dev.and_nnz + m.dev.long_nnz) + and_rows / 2) / and_rows);
    k.long_rows = m.info.n_long_rows > 0 ? 1 : 0;
    return k;
}

static const char kSchedMagic[] = "lp-sched-v1";

static bool sched_valid(const lp_schedule &s) {
    auto in = [](int32_t v, std::initializer_list<int32_t> ok) {
        for (int32_t x : ok)
            if (v == x) return true;
        return false;
    };
    return s.driver >= LP_DRIVER_AUTO && s.driver <= LP_DRIVER_FRONTIER && s.steps_per_sync >= 0 &&
           s.steps_per_sync <= 4096 && in(s.variant, {LP_STEP_AUTO, LP_STEP_GLOBAL, LP_STEP_LDS}) && s.grid >= 0 &&
           s.grid <= (1 << 20) && in(s.wpw, {0, 1, 2, 4, 8}) && in(s.unroll, {0, 4, 8, 16}) &&
           in(s.block, {0, 256, 512, 1024}) && s.team == 0 && s.team_polls == 0;
}

// Parses a cache file; all or nothing (lock held by the caller).
static lp_status sched_load_locked(const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) {
        set_error(std::string("cannot open schedule cache ") + path);
        return LP_E_INVAL;
    }
    std::map<SchedKey, lp_schedule> add;
    char line[512];
    int ln = 0;
    lp_status rc = LP_OK;
    while (std::fgets(line, sizeof line, f)) {
        ++ln;
        if (line[0] == '#' || line[0] == '\n') continue;
        char magic[32] = {0};
        SchedKey k;
        lp_schedule s{};
        char tail = 0;
        const int n = std::sscanf(line, "%31s %d %d %d %d %d %d %d %d %d %d %d %c", magic, &k.lds, &k.log2_rows,
                                  &k.len_q, &k.long_rows, &s.driver, &s.steps_per_sync, &s.variant, &s.grid,
                                  &s.wpw, &s.unroll, &s.block, &tail);
        if (n != 12 || std::strcmp(magic, kSchedMagic) != 0 || k.lds < 0 || k.lds > 1 || k.log2_rows < 0 ||
            k.log2_rows > 40 || k.len_q < 0 || k.len_q > 64 || k.long_rows < 0 || k.long_rows > 1 ||
            !sched_valid(s)) {
            set_error(std::string("malformed schedule cache line ") + std::to_string(ln) + " in " + path);
            rc = LP_E_INVAL;
            break;
        }
        add[k] = s;
    }
    std::fclose(f);
    if (rc) return rc;
    for (auto &e : add) g_sched[e.first] = e.second;
    return LP_OK;
}

static lp_status sched_save_locked(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) {
        set_error(std::string("cannot write schedule cache ") + path);
        return LP_E_INVAL;
    }
    std::fprintf(f, "# %s: lds log2_rows len_q long_rows | driver steps_per_sync variant grid wpw unroll block\n",
                 kSchedMagic);
    for (auto &e : g_sched) {
        const SchedKey &k = e.first;
        const lp_schedule &s = e.second;
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d\n", kSchedMagic, k.lds, k.log2_rows, k.len_q,
                     k.long_rows, s.driver, s.steps_per_sync, s.variant, s.grid, s.wpw, s.unroll, s.block);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        set_error(std::string("cannot write schedule cache ") + path);
        return LP_E_INVAL;
    }
    return LP_OK;
}

// Loads LP_SCHEDULE_CACHE once, if it is set and the file exists (lock held).
static void sched_env_locked() {
    if (g_sched_env_done) return;
    g_sched_env_done = true;
    const char *p = std::getenv("LP_SCHEDULE_CACHE");
    if (!p || !*p) return;
    FILE *f = std::fopen(p, "r");
    if (!f) return;  // created by the first tune
    std::fclose(f);
    (void)sched_load_locked(p);
}

static bool sched_lookup(const Matrix &m, lp_schedule *out) {
    std::lock_guard<std::mutex> lock(g_sched_mu);
    sched_env_locked();
    auto it = g_sched.find(sched_key(m));
    if (it == g_sched.end()) return false;
    *out = it->second;
    return true;
}

static void sched_store(const Matrix &m, const lp_schedule &s) {
    std::lock_guard<std::mutex> lock(g_sched_mu);
    sched_env_locked();
    g_sched[sched_key(m)] = s;
    const char *p = std::getenv("LP_SCHEDULE_CACHE");
    if (p && *p) (void)sched_save_locked(p);
}

static lp_status least_fixpoint(const Matrix &m, const lp_schedule *sched, hipStream_t st, Scratch &S,
                                uint64_t **out, int32_t *products, uint64_t *host_bits = nullptr,
                                bool *on_host = nullptr) {
    if (on_host) *on_host = false;
    if (sched && (sched->driver < LP_DRIVER_AUTO || sched->driver > LP_DRIVER_FRONTIER)) {
        set_error("unknown driver " + std::to_string(sched->driver));
        return LP_E_INVAL;
    }
    if (sched && sched->driver == LP_DRIVER_FRONTIER) return frontier_fixpoint(m, st, S, out, products);
    // the library's own choice only: a schedule that names a step shape gets the step kernel
    const bool all_default = !sched || (sched->driver == LP_DRIVER_AUTO && sched->steps_per_sync == 0 &&
                                        sched->variant == 0 && sched->grid == 0 && sched->wpw == 0 &&
                                        sched->unroll == 0 && sched->block == 0);
    if (all_default && m.n_rows > 0 && lds_loop_fits(m)) {
        lp_status rc = lds_loop_fixpoint(m, st, S, out, products, host_bits);
        if (rc == LP_OK && on_host) *on_host = host_bits != nullptr;
        return rc;
    }
    // a tuned schedule for matrices of this size bucket (not in a fixed scratch
    // region, whose size is that of the default schedule's buffers)
    lp_schedule cached;
    if (all_default && S.may_alloc() && sched_lookup(m, &cached)) sched = &cached;
    const int64_t W = n_words_of(m.n_rows);
    uint64_t *buf[2];
    unsigned long long *counters;
    uint32_t *and_cnt;
    uint64_t *pacc = nullptr;  // a sliced step's partial AND words (written before they are read)
    lp_status rc;
    if ((rc = S.get(&buf[0], W)) || (rc = S.get(&buf[1], W)) || (rc = S.get(&counters, kRing)) ||
        (rc = S.get(&and_cnt, 2 * (size_t)m.dev.n_long_and)) ||
        (!m.dev.slices.empty() && (rc = S.get(&pacc, W))))
        return rc;
    if (S.may_alloc()) {
        LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
        if (m.dev.n_long_and) LP_HIP(hipMemsetAsync(and_cnt, 0, sizeof(uint32_t) * 2 * m.dev.n_long_and, st));
    } else {  // a fixed region keeps the last call's contents: clear with a kernel
        LP_HIP(launch_zero_words(counters, 2 * (int64_t)kRing, st));
        if (m.dev.n_long_and) LP_HIP(launch_zero_words(and_cnt, 2 * (int64_t)m.dev.n_long_and, st));
    }
    LP_HIP(hipMemcpyAsync(buf[0], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
    LP_HIP(hipMemcpyAsync(buf[1], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
    if (m.n_rows == 0) {
        *out = buf[0];
        *products = 1;
        return LP_OK;
    }
    int driver = sched ? sched->driver : LP_DRIVER_AUTO;
    StepParams p = step_params(m);
    p.counters = counters;
    p.and_cnt = and_cnt;
    p.pacc = pacc;
    StepShape L;
    if (driver == LP_DRIVER_PERSISTENT) {
        if ((rc = plan_persistent(m, sched, p, &L, st))) return rc;
        if (L.grid >= 1) {
            int32_t *res;
            if ((rc = S.get(&res, 4))) return rc;
            if ((rc = run_persistent(m, p, L, buf, res, st))) return rc;
            int32_t prods = 0;
            LP_HIP(hipMemcpyAsync(&prods, res, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            LP_HIP(hipStreamSynchronize(st));
            if (prods == -2) {
                set_error("persistent step: a workgroup gave up waiting at the grid barrier");
                return LP_E_INTERNAL;
            }
            if (prods < 1) {
                set_error("fixpoint not reached within n_rows+1 products");
                return LP_E_INTERNAL;
            }
            *products = prods;
            *out = buf[prods & 1];
            return LP_OK;
        }
        set_error("the persistent step does not fit on this device");
        return LP_E_DEVICE;
    }
    int batch = 1;
    if (driver == LP_DRIVER_BATCHED || driver == LP_DRIVER_AUTO) {
        batch = (sched && sched->steps_per_sync > 0) ? sched->steps_per_sync : 32;
    }
    batch = std::max(1, std::min(batch, kRing / 2 - 1));
    if ((rc = plan_step(m, sched, p, &L, st, S.may_alloc()))) return rc;
    unsigned long long h_local[kRing];  // no pinned host allocation in a fixed-region call
    unsigned long long *h = S.may_alloc() ? pinned_ring() : h_local;
    if (!h) {
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    const int64_t limit = (int64_t)m.n_rows + 1;
    for (int64_t t = 0;; t += batch) {
        for (int i = 1; i <= batch; ++i) {
            p.step = (int32_t)(t + i);
            p.v = buf[(p.step - 1) & 1];
            p.u = buf[p.step & 1];
            LP_HIP(launch_step(L, p, st));
        }
        LP_HIP(hipMemcpyAsync(h, counters, sizeof(unsigned long long) * kRing, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        for (int i = 1; i <= batch; ++i) {
            const int64_t s = t + i;
            if (h[s & (kRing - 1)] == 0) {
                *products = (int32_t)s;
                *out = buf[s & 1];
                return LP_OK;
            }
        }
        if (t + batch > limit) {
            set_error("fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
}

// Transposed matrix of the frontier driver, built on first use from the host
// CSR and kept with the matrix: for each row c, the rows whose entries name c
// (fact rows and empty rows have no entries and are never counted down);
// each row's count of entries still false at the start (AND rows: their
// length; OR rows: 1, so the first true child fires them); the fact rows.
static lp_status ensure_frontier(const Matrix &m, hipStream_t st) {
    std::lock_guard<std::mutex> lock(g_lazy_mu);
    const DeviceMatrix &d = m.dev;
    if (d.fr_ptr) return LP_OK;
    const int32_t n = m.n_rows;
    std::vector<int32_t> ptr((size_t)n + 1, 0), cnt0((size_t)std::max(n, 1), 0), facts;
    for (int32_t r = 0; r < n; ++r) {
        if (m.fact[r]) {
            facts.push_back(r);
            continue;
        }
        for (int32_t j = m.row_ptr[r]; j < m.row_ptr[r + 1]; ++j) ++ptr[(size_t)m.col[j] + 1];
        const int32_t len = m.row_ptr[r + 1] - m.row_ptr[r];
        cnt0[r] = len == 0 ? 0 : (m.kind[r] ? len : 1);
    }
    for (int32_t c = 0; c < n; ++c) ptr[(size_t)c + 1] += ptr[c];
    std::vector<int32_t> occ((size_t)std::max<int32_t>(ptr[n], 1)), fill(ptr.begin(), ptr.end() - 1);
    for (int32_t r = 0; r < n; ++r) {
        if (m.fact[r]) continue;
        for (int32_t j = m.row_ptr[r]; j < m.row_ptr[r + 1]; ++j) occ[(size_t)fill[m.col[j]]++] = r;
    }
    if (facts.empty()) facts.push_back(0);  // not read: the fact count is 0
    int64_t bytes = 0;
    int32_t *dp = nullptr, *dq = nullptr, *dc = nullptr, *df = nullptr;
    lp_status rc;
    if ((rc = upload(&dp, ptr.data(), ptr.size(), st, &bytes)) || (rc = upload(&dq, occ.data(), occ.size(), st, &bytes)) ||
        (rc = upload(&dc, cnt0.data(), cnt0.size(), st, &bytes)) ||
        (rc = upload(&df, facts.data(), facts.size(), st, &bytes))) {
        for (void *x : {(void *)dp, (void *)dq, (void *)dc, (void *)df}) dev_free(x, st);
        return rc;
    }
    LP_HIP(hipStreamSynchronize(st));  // the host vectors are locals
    d.fr_ptr = dp;
    d.fr_occ = dq;
    d.fr_cnt0 = dc;
    d.fr_facts = df;
    d.fr_n_facts = (int32_t)std::count(m.fact.begin(), m.fact.end(), (uint8_t)1);
    d.lazy_bytes += bytes;
    return LP_OK;
}

// Least-model fixpoint by levels (lp_frontier.hip): level t pushes F_t and
// collects F_{t+1}; levels are issued in batches between host reads of
// their |F_t| history; the first empty F_t (t >= 1) ends the solve
// with t products, like the full sweep.
static lp_status frontier_fixpoint(const Matrix &m, hipStream_t st, Scratch &S, uint64_t **out, int32_t *products) {
    lp_status rc;
    if ((rc = ensure_frontier(m, st))) return rc;
    const DeviceMatrix &d = m.dev;
    const int32_t n = m.n_rows;
    const int64_t W = n_words_of(n);
    uint64_t *v;
    int32_t *cnt, *q[2], *hist;
    uint32_t *sizes;
    // hist holds the |F_t| history and, after it, the looped kernel's stop level
    if ((rc = S.get(&v, W)) || (rc = S.get(&cnt, std::max(n, 1))) || (rc = S.get(&q[0], std::max(n, 1))) ||
        (rc = S.get(&q[1], std::max(n, 1))) || (rc = S.get(&sizes, kFrontierRing)) ||
        (rc = S.get(&hist, kFrontierHist + 2)))
        return rc;
    LP_HIP(hipMemcpyAsync(v, d.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
    *out = v;
    if (n == 0) {
        *products = 1;
        return LP_OK;
    }
    LP_HIP(hipMemcpyAsync(cnt, d.fr_cnt0, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    DevProps dp;
    if ((rc = dev_props(d.device, &dp))) return rc;
    // Two launch shapes (every shape gives the same result): a launch per
    // level over the full grid, kLevelBatch levels per host read; or one
    // workgroup running up to kLoopBatch levels in a loop, with no launch per
    // level (a long derivation chain), until a frontier above kFrontierSmall
    // rows stops it and the full grid takes over from that level. The loop
    // follows a batch of launches whose last frontier was at most
    // kFrontierSmall rows, and a loop that was not stopped.
    constexpr int32_t kFrontierSmall = kFrontierLoopCap;
    const int grid_full = 4 * std::max(dp.n_cu, 1);
    bool looped = false;
    unsigned long long *h = pinned_ring();
    if (!h) {
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    static_assert((kFrontierHist + 2) * sizeof(int32_t) <= kRing * sizeof(unsigned long long), "pinned ring");
    int32_t *hh = reinterpret_cast<int32_t *>(h);
    // sizes = {|F_0|, 0, ...}, copied from the pinned buffer (written again only by a later copy on st)
    for (int i = 0; i < kFrontierRing; ++i) hh[i] = i == 0 ? d.fr_n_facts : 0;
    LP_HIP(hipMemcpyAsync(sizes, hh, sizeof(uint32_t) * kFrontierRing, hipMemcpyHostToDevice, st));
    // levels per host read: 64 launches, or one loop launch over up to
    // kFrontierHist levels (a batch's levels take distinct history slots)
    constexpr int kLevelBatch = 16, kLoopBatch = kFrontierHist;
    const int64_t limit = (int64_t)n + 1;
    FrontierParams f{};
    f.occ_ptr = d.fr_ptr;
    f.occ = d.fr_occ;
    f.cnt = cnt;
    f.v = v;
    f.sizes = sizes;
    f.hist = hist;
    for (int64_t t0 = 0;;) {
        const int64_t batch = looped ? kLoopBatch : kLevelBatch;
        if (looped) {
            f.level = (int32_t)t0;
            LP_HIP(launch_frontier_levels(f, d.fr_facts, q[0], q[1], (int32_t)batch, hist + kFrontierHist, st));
        } else {
            for (int64_t t = t0; t < t0 + batch; ++t) {
                f.level = (int32_t)t;
                f.in = t == 0 ? d.fr_facts : q[t & 1];
                f.out = q[(t + 1) & 1];
                LP_HIP(launch_frontier_level(f, grid_full, st));
            }
        }
        LP_HIP(hipMemcpyAsync(hh, hist, sizeof(int32_t) * (kFrontierHist + 1), hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        const int64_t t_end = looped ? (int64_t)hh[kFrontierHist] : t0 + batch;
        if (t_end < t0 || t_end > t0 + batch) {
            set_error("frontier loop reported an impossible level");
            return LP_E_INTERNAL;
        }
        for (int64_t t = t0; t < t_end; ++t) {
            if (hh[t % kFrontierHist] == 0) {
                *products = (int32_t)std::max<int64_t>(t, 1);
                return LP_OK;
            }
        }
        // a loop that stopped early stopped before a large frontier
        looped = looped ? t_end == t0 + batch : hh[(t_end - 1) % kFrontierHist] <= kFrontierSmall;
        t0 = t_end;
        if (t0 > limit) {
            set_error("fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
}

// Bit-packed interpretation -> one byte per atom. Eight atoms at a time: byte
// j of the packed words (bits 8j..8j+7, little-endian) expands through a
// 256-entry table to eight 0/1 bytes.
static const uint64_t *byte_expand_table() {
    static const std::vector<uint64_t> t = [] {
        std::vector<uint64_t> v(256);
        for (int b = 0; b < 256; ++b)
            for (int k = 0; k < 8; ++k)
                if ((b >> k) & 1) v[b] |= 1ull << (8 * k);
        return v;
    }();
    return t.data();
}

static void unpack_model(const uint64_t *bits, int32_t n, uint8_t *model) {
    const uint64_t *T = byte_expand_table();
    const uint8_t *by = reinterpret_cast<const uint8_t *>(bits);
    int32_t a = 0;
    for (; a + 8 <= n; a += 8) std::memcpy(model + a, &T[by[a >> 3]], 8);
    for (; a < n; ++a) model[a] = (uint8_t)((bits[a >> 6] >> (a & 63)) & 1ull);
}

static lp_status least_model_impl(const Matrix &m, uint8_t *model, int32_t *products, const lp_schedule *sched,
                                  hipStream_t st, Scratch &S) {
    uint64_t *fix = nullptr;
    int32_t prods = 0;
    const int64_t Wn = n_words_of(m.n_atoms);
    std::vector<uint64_t> hb(Wn ? Wn : 1);
    bool on_host = false;
    lp_status rc = least_fixpoint(m, sched, st, S, &fix, &prods, hb.data(), &on_host);
    if (rc) return rc;
    if (!on_host) {
        if (Wn) LP_HIP(hipMemcpyAsync(hb.data(), fix, Wn * 8, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
    }
    unpack_model(hb.data(), m.n_atoms, model);
    if (products) *products = prods;
    return LP_OK;
}

static lp_status least_model_impl(const Matrix &m, uint8_t *model, int32_t *products, const lp_schedule *sched,
                                  hipStream_t st) {
    Scratch S(st);
    return least_model_impl(m, model, products, sched, st, S);
}

// ------------------------------------------------------------------ fixed scratch region

// Device memory of lp_least_model_noalloc: every solve buffer of a call is
// carved from this array, one copy per device, held until the process ends.
// Host code uses the per-device address from hipGetSymbolAddress, never the
// array's name (a host-side stand-in).
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

static lp_status scratch_region(int dev, void **out) {
    static std::mutex mu;
    static void *addr[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) {
        set_error("device id out of range");
        return LP_E_DEVICE;
    }
    if (!addr[dev]) {
        void *p = nullptr;
        LP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));  // the current device is dev
        if (!p) {
            set_error("hipGetSymbolAddress gave no address for the scratch region");
            return LP_E_DEVICE;
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return LP_OK;
}

static size_t region_bytes(size_t b) { return std::max<size_t>(256, (b + 255) & ~(size_t)255); }

// Bytes of the fixed region a default-driver solve of m takes (the same
// buffers least_fixpoint and lds_loop_fixpoint carve, in 256-byte steps).
static size_t noalloc_need(const Matrix &m) {
    if (m.n_rows > 0 && lds_loop_fits(m))
        return region_bytes(kLdsLoopHead + (size_t)std::max<int64_t>(1, n_words_of(m.n_atoms)) * 8);
    const size_t W = (size_t)n_words_of(m.n_rows);
    return 2 * region_bytes(W * 8) + region_bytes(sizeof(unsigned long long) * kRing) +
           region_bytes(sizeof(uint32_t) * 2 * (size_t)m.dev.n_long_and) +
           (m.dev.slices.empty() ? 0 : region_bytes(W * 8));
}

static int ilog2(int64_t x) {
    int l = 0;
    while ((1ll << l) < x) ++l;
    return l;
}

// Workgroups of the stable-model step: eight per CU.
static int spmm_grid(const Matrix &m) {
    DevProps d;
    if (dev_props(m.dev.device, &d) || d.n_cu <= 0) return 2048;
    return 8 * d.n_cu;
}

// log2W < 0: the width of the enumerated guess space (K_eff <= LP_MAX_NEG_ATOMS).
static SpmmParams spmm_params(const Matrix &m, unsigned long long *counters, int log2W = -1) {
    const int64_t W = log2W >= 0 ? (1ll << log2W) : ((1ll << m.K_eff) + 63) / 64;
    SpmmParams p{};
    p.row_ptr = m.dev.full_row_ptr;
    p.col = m.dev.full_col;
    p.and_bits = m.dev.full_and_bits;
    p.counters = counters;
    p.log2W = ilog2(W);
    p.total = (int64_t)m.n_rows * W;
    p.early_exit = 1;
    return p;
}

// Stable-model products by dirty rows or full sweeps. Measured on MI355X
// (HIP events per solve, dirty rows against full sweeps): 17.6k row-words
// 0.14 vs 0.20 ms, 168k (4-word rows, product 1 nearly dense) 0.37 vs 0.34 ms,
// 436k 0.15 vs 0.37 ms, 1.75M 0.16 vs 0.46 ms, 28M 0.32 vs 2.0 ms. Below 16k
// row-words a solve is a few launches either way, and full sweeps spare the
// transposed matrix and the solve plan's capture.
constexpr int64_t kDirtyMinWords = 1 << 14;

static bool dirty_products(const Matrix &m, int32_t log2W) {
    if ((m.flags & LP_STABLE_FULL_SWEEP) || m.n_rows == 0) return false;
    return (m.flags & LP_STABLE_DIRTY_ROWS) || ((int64_t)m.n_rows << log2W) >= kDirtyMinWords;
}

// Algorithm 2's loop from the initial matrix (Definition 8) until no column
// changes; *fix is the buffer holding the fixpoint. The counters hold the bit
// count of each product's result (slot 0: the initial matrix); product s
// changed nothing iff its count equals that of product s - 1.
static lp_status stable_loop(const Matrix &m, SpmmParams p, hipStream_t st, uint64_t *const buf[2],
                             unsigned long long *counters, int32_t *products, uint64_t **fix);

static lp_status stable_fixpoint(const Matrix &m, hipStream_t st, uint64_t *const buf[2],
                                 unsigned long long *counters, int32_t *products, uint64_t **fix) {
    SpmmParams p = spmm_params(m, counters);
    LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
    // |M0|: every fact row holds all 2^K_eff guesses, every guessed qbar row half of them
    const unsigned long long H = 1ull << m.K_eff;
    const unsigned long long m0_bits = (unsigned long long)m.info.n_fact_rows * H + (unsigned long long)m.K_eff * (H / 2);
    LP_HIP(launch_init_m0(buf[0], buf[1], p.total, p.log2W, m.n_std, m.dev.fact_bits, m.dev.guess_pos, m.K_eff,
                          &counters[0], m0_bits, st));
    return stable_loop(m, p, st, buf, counters, products, fix);
}

static lp_status ensure_frontier(const Matrix &m, hipStream_t st);


// Products of Algorithm 2 by dirty rows (spmm_dirty_product_kernel, one
// launch per product): product t evaluates only the rows naming a row that
// changed in product t-1 (product 1: a fact or qbar row, the rows the initial
// matrix in both buffers does not hold at 0); the same products and fixpoint
// as the full sweep. Products are issued kFirstBatch, then kLaterBatch, at a
// time between host reads of |C_t|; products issued past the fixpoint return
// at once. (Later batches of 16 rather than 8: the serving pool's stable
// solves take 50-66 products, and fewer host reads cut the mean service time
// by 3% with the same throughput.)
constexpr int kFirstBatch = 16, kLaterBatch = 16;
static_assert(kFirstBatch < kDirtyHist / 2 && kLaterBatch < kDirtyHist / 2, "history slots");
static_assert(kDirtyHist * sizeof(int32_t) <= kRing * sizeof(unsigned long long), "pinned ring");

// Device state of the dirty-row products of one solve: the two interpretation
// buffers and the row sets, laid out as [D0 | D1 | D2 | C0 | C1 | C2 |
// changed] (bitmaps of nb words) followed by the history, so one clear
// covers them.
struct DirtyState {
    DirtyParams p{};
    uint64_t *buf[2] = {nullptr, nullptr};
    uint32_t *sets = nullptr;
    int32_t *hist = nullptr;
    int64_t nb = 0;
    int grid = 0, grid_small = 0;
};

static int64_t dirty_bitmap_words(const Matrix &m) { return ((int64_t)std::max(m.n_rows, 1) + 31) / 32; }

static size_t dirty_sets_words(const Matrix &m) { return 7 * (size_t)dirty_bitmap_words(m) + kDirtyHist; }

// Fills s.p from the matrix, the buffers s.buf and the sets s.sets.
static void dirty_setup(const Matrix &m, const SpmmParams &sp, DirtyState &s) {
    s.nb = dirty_bitmap_words(m);
    s.hist = reinterpret_cast<int32_t *>(s.sets + 7 * s.nb);
    DirtyParams &p = s.p;
    p.row_ptr = sp.row_ptr;
    p.col = sp.col;
    p.and_bits = sp.and_bits;
    p.occ_ptr = m.dev.fr_ptr;
    p.occ = m.dev.fr_occ;
    p.call = s.sets + 6 * s.nb;
    p.hist = s.hist;
    p.fact_bits = m.dev.fact_bits;
    p.nb = s.nb;
    p.n_rows = m.n_rows;
    p.n_std = m.n_std;
    p.log2W = sp.log2W;
    // product 1's dirty set (rows naming a fact or qbar row) can be large;
    // later ones are small on small matrices, where a launch of eight
    // workgroups per CU that mostly exit costs dispatch time; matrices of many
    // rows, or rows of 64 words or more (each row a wave's work), keep the
    // full grid for every product
    s.grid = spmm_grid(m);
    s.grid_small = (m.n_rows >= (1 << 18) || sp.log2W >= 6) ? s.grid : std::max(1, s.grid / 4);
}

static uint32_t *dirty_d(DirtyState &s, int64_t t) { return s.sets + (t % 3) * s.nb; }
static uint32_t *dirty_c(DirtyState &s, int64_t t) { return s.sets + (3 + t % 3) * s.nb; }

// D_1 (rows naming a fact or qbar row); the sets must be clear.
static hipError_t dirty_seed(const Matrix &m, DirtyState &s, hipStream_t st) {
    s.p.dnext = dirty_d(s, 1);
    return launch_dirty_seed(s.p, m.dev.fr_facts, m.dev.fr_n_facts, s.grid_small, st);
}

// Launches products t0 .. t1-1.
static hipError_t dirty_products_launch(DirtyState &s, int64_t t0, int64_t t1, hipStream_t st) {
    DirtyParams &p = s.p;
    for (int64_t t = t0; t < t1; ++t) {
        p.step = (int32_t)t;
        p.V = s.buf[(t - 1) & 1];
        p.U = s.buf[t & 1];
        p.dcur = dirty_d(s, t);
        p.dnext = dirty_d(s, t + 1);
        p.dclear = dirty_d(s, t + 2);
        p.cprev = dirty_c(s, t + 2);  // C_{t-1}
        p.ccur = dirty_c(s, t);
        p.cclear = dirty_c(s, t + 1);
        const int grid = t == 1 ? s.grid : s.grid_small;
        // narrow rows: enough bitmap words per wave to cover the bitmap in
        // about two rounds of the grid's waves, so dense sets spread over all waves
        p.wpi = (int32_t)std::max<int64_t>(1, std::min<int64_t>(8, s.nb / (2 * (int64_t)grid * 4)));
        hipError_t e = launch_dirty_product(p, grid, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// First product in [t0, t1) that changed nothing according to the host copy
// hh of the |C_t| history, or -1.
static int64_t dirty_first_fixpoint(const int32_t *hh, int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t)
        if (hh[t & (kDirtyHist - 1)] == 0) return t;
    return -1;
}

// Products from t0 on, in batches of kLaterBatch between host reads of the
// history (hh: kDirtyHist pinned int32), until one changes nothing.
static lp_status dirty_finish(const Matrix &m, DirtyState &s, int64_t t0, int32_t *hh, hipStream_t st,
                              int32_t *products, uint64_t **fix) {
    const int64_t limit = (int64_t)m.n_rows + 1;
    for (int64_t batch = t0 == 1 ? kFirstBatch : kLaterBatch;; batch = kLaterBatch) {
        LP_HIP(dirty_products_launch(s, t0, t0 + batch, st));
        LP_HIP(hipMemcpyAsync(hh, s.hist, sizeof(int32_t) * kDirtyHist, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        const int64_t t = dirty_first_fixpoint(hh, t0, t0 + batch);
        if (t > 0) {
            *products = (int32_t)t;
            *fix = s.buf[t & 1];
            return LP_OK;
        }
        t0 += batch;
        if (t0 > limit) {
            set_error("fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
}

static lp_status stable_dirty_loop(const Matrix &m, const SpmmParams &sp, hipStream_t st, uint64_t *const buf[2],
                                   int32_t *products, uint64_t **fix) {
    lp_status rc;
    if ((rc = ensure_frontier(m, st))) return rc;
    Scratch S(st);
    DirtyState s;
    s.buf[0] = buf[0];
    s.buf[1] = buf[1];
    if ((rc = S.get(&s.sets, dirty_sets_words(m)))) return rc;
    LP_HIP(hipMemsetAsync(s.sets, 0, sizeof(uint32_t) * dirty_sets_words(m), st));
    int32_t *hh = reinterpret_cast<int32_t *>(pinned_ring());
    if (!hh) {
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    dirty_setup(m, sp, s);
    LP_HIP(dirty_seed(m, s, st));
    return dirty_finish(m, s, 1, hh, st, products, fix);
}

// Products of Algorithm 2 from the initial matrix in buf[0] (and buf[1]),
// whose bit count is in counters[0], until a product changes no column.
static lp_status stable_loop(const Matrix &m, SpmmParams p, hipStream_t st, uint64_t *const buf[2],
                             unsigned long long *counters, int32_t *products, uint64_t **fix) {
    if (dirty_products(m, p.log2W)) return stable_dirty_loop(m, p, st, buf, products, fix);
    unsigned long long *h = pinned_ring();
    if (!h) {
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    const int batch = 8;
    const int64_t limit = (int64_t)m.n_rows + 1;
    for (int64_t t = 0;; t += batch) {
        for (int i = 1; i <= batch; ++i) {
            p.step = (int32_t)(t + i);
            p.V = buf[(p.step - 1) & 1];
            p.U = buf[p.step & 1];
            LP_HIP(launch_spmm_step(p, spmm_grid(m), st));
        }
        LP_HIP(hipMemcpyAsync(h, counters, sizeof(unsigned long long) * kRing, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        for (int i = 1; i <= batch; ++i) {
            const int64_t s = t + i;
            if (h[s & (kRing - 1)] == h[(s - 1) & (kRing - 1)]) {
                *products = (int32_t)s;
                *fix = buf[s & 1];
                return LP_OK;
            }
        }
        if (t + batch > limit) {
            set_error("fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
}

// Algorithm 3's results from the accepted mask of the compressed guess space
// (host acc_h, W words) and the fixpoint on the device: the mask in the full
// guess space, the model count, the first max_models models (extract_kernel)
// and, if asked, the interpretation matrix. The copies to the host are
// complete once the stream has synchronized: here, unless sync is false.
static lp_status stable_outputs(const Matrix &m, const uint64_t *fix, int log2W, int64_t W, const uint64_t *acc_h,
                                unsigned long long nm, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                                int64_t max_models, uint64_t *interp, Scratch &S, hipStream_t st, bool sync = true) {
    const int K = m.K;
    const int64_t W_full = (((int64_t)1 << K) + 63) / 64;
    // accepted guesses in the full guess space (deposit compressed bits)
    std::memset(accepted, 0, sizeof(uint64_t) * W_full);
    std::vector<int64_t> cols;
    for (int64_t w = 0; w < W; ++w) {
        uint64_t x = acc_h[w];
        while (x) {
            const int b = __builtin_ctzll(x);
            x &= x - 1;
            const int64_t jc = w * 64 + b;
            int64_t jf = 0;
            for (int t = 0; t < K; ++t)
                if (m.guess_pos[t] >= 0 && ((jc >> m.guess_pos[t]) & 1)) jf |= 1ll << t;
            accepted[jf >> 6] |= 1ull << (jf & 63);
            if (models && (int64_t)cols.size() < max_models) cols.push_back(jc);
        }
    }
    *n_models = (int64_t)nm;
    if (interp && m.n_atoms) {
        LP_HIP(hipMemcpyAsync(interp, fix, sizeof(uint64_t) * (size_t)m.n_atoms * W, hipMemcpyDeviceToHost, st));
    }
    if (models && !cols.empty() && m.n_atoms) {
        int64_t *cols_d;
        uint8_t *out_d;
        const int64_t nb = (int64_t)cols.size() * m.n_atoms;
        lp_status rc;
        if ((rc = S.get(&cols_d, cols.size())) || (rc = S.get(&out_d, nb))) return rc;
        LP_HIP(hipMemcpyAsync(cols_d, cols.data(), cols.size() * 8, hipMemcpyHostToDevice, st));
        LP_HIP(launch_extract(fix, log2W, cols_d, (int64_t)cols.size(), m.n_atoms, out_d, st));
        LP_HIP(hipMemcpyAsync(models, out_d, nb, hipMemcpyDeviceToHost, st));
    }
    if (sync) LP_HIP(hipStreamSynchronize(st));
    return LP_OK;
}

// Interpretation matrices of at most this many words get a stable-solve plan
// (two buffers of 2 GiB at most, kept with the matrix). At 2^25 the serving
// pool's largest stable programs (up to 4M rows x 64 words) wrote their whole
// initial matrix per solve (357 us of a 3.3 ms solve at 3.3M rows x 32 words);
// with plans for them the pool's mean service time fell from 0.580 to 0.561 ms
// and its device memory grew from 20 to 42 GB.
constexpr int64_t kPlanMaxWords = (int64_t)1 << 28;

// Layout of a plan's pinned host block: the |C_t| history, the model count,
// the accepted mask.
static size_t plan_host_bytes(int64_t W) { return sizeof(int32_t) * kDirtyHist + 8 + 8 * (size_t)W; }

// Allocates the plan's buffers and captures its graph: the seed of D_1, products
// 1..kFirstBatch, the model count cleared, Algorithm 3's test on buffer 0 (both
// buffers hold the fixpoint when it is reached within the batch), and the
// history, count and mask copied to the pinned block.
static lp_status plan_create(const Matrix &m, StablePlan *pl, DirtyState &s, int keff, int log2W, hipStream_t st) {
    const int64_t W = (int64_t)1 << log2W;
    const int64_t total = (int64_t)m.n_rows * W;
    lp_status rc;
    auto get = [&](void **p, size_t bytes) -> lp_status {
        lp_status r = dev_alloc(p, bytes, st);
        if (!r) pl->bytes += (int64_t)bytes;
        return r;
    };
    if ((rc = get((void **)&pl->buf[0], 8 * (size_t)total)) || (rc = get((void **)&pl->buf[1], 8 * (size_t)total)) ||
        (rc = get((void **)&pl->sets, 4 * dirty_sets_words(m))) || (rc = get((void **)&pl->acc_d, 8 * (size_t)W)) ||
        (rc = get((void **)&pl->cnt_d, 256)))
        return rc;
    if (hipHostMalloc((void **)&pl->host, plan_host_bytes(W), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        pl->host = nullptr;
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    s.buf[0] = pl->buf[0];
    s.buf[1] = pl->buf[1];
    s.sets = pl->sets;
    dirty_setup(m, spmm_params(m, nullptr, log2W), s);
    hipStream_t cs;
    LP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t el = dirty_seed(m, s, cs);
        if (el == hipSuccess) el = dirty_products_launch(s, 1, kFirstBatch + 1, cs);
        if (el == hipSuccess) el = launch_zero_words(pl->cnt_d, 2, cs);
        if (el == hipSuccess)
            el = launch_stable_check(pl->buf[0], log2W, W, m.dev.q_rows, m.n_std, m.K, keff, pl->acc_d, pl->cnt_d, cs);
        if (el == hipSuccess)
            el = hipMemcpyAsync(pl->host, s.hist, sizeof(int32_t) * kDirtyHist, hipMemcpyDeviceToHost, cs);
        if (el == hipSuccess)
            el = hipMemcpyAsync(pl->host + sizeof(int32_t) * kDirtyHist, pl->cnt_d, 8, hipMemcpyDeviceToHost, cs);
        if (el == hipSuccess)
            el = hipMemcpyAsync(pl->host + sizeof(int32_t) * kDirtyHist + 8, pl->acc_d, 8 * (size_t)W,
                                hipMemcpyDeviceToHost, cs);
        e = hipStreamEndCapture(cs, &pl->graph);
        if (e == hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "stable-solve graph capture");
    (void)st;
    (void)total;
    return LP_OK;
}

// stable_impl through the matrix's plan. *used is false when another solve
// holds the plan (the caller then takes the allocating path).
static lp_status stable_plan_solve(const Matrix &m, int keff, int log2W, uint64_t *accepted, int64_t *n_models,
                                   uint8_t *models, int64_t max_models, uint64_t *interp, int32_t *products,
                                   hipStream_t st, bool *used) {
    *used = false;
    StablePlan *pl;
    {
        std::lock_guard<std::mutex> lock(g_lazy_mu);
        if (!m.dev.splan) m.dev.splan = new StablePlan();
        pl = m.dev.splan;
    }
    std::unique_lock<std::mutex> hold(pl->mu, std::try_to_lock);
    if (!hold.owns_lock()) return LP_OK;
    *used = true;
    lp_status rc;
    if ((rc = ensure_frontier(m, st))) return rc;
    const int64_t W = (int64_t)1 << log2W;
    DirtyState s;
    if (!pl->exec) {
        const int64_t before = pl->bytes;
        rc = plan_create(m, pl, s, keff, log2W, st);
        {
            std::lock_guard<std::mutex> lock(g_lazy_mu);
            m.dev.lazy_bytes += pl->bytes - before;
        }
        if (rc) return rc;
    } else {
        s.buf[0] = pl->buf[0];
        s.buf[1] = pl->buf[1];
        s.sets = pl->sets;
        dirty_setup(m, spmm_params(m, nullptr, log2W), s);
    }
    if (!pl->ready) {  // first solve, or a solve that failed part way: the initial matrix afresh
        LP_HIP(launch_init_m0(pl->buf[0], pl->buf[1], (int64_t)m.n_rows * W, log2W, m.n_std, m.dev.fact_bits,
                              m.dev.guess_pos, keff, pl->cnt_d, 0, st));
        LP_HIP(launch_zero_words(pl->sets, (int64_t)dirty_sets_words(m), st));
    }
    pl->ready = false;  // until the buffers are back to the initial matrix
    LP_HIP(hipGraphLaunch(pl->exec, st));
    LP_HIP(hipStreamSynchronize(st));
    int32_t *hh = reinterpret_cast<int32_t *>(pl->host);
    unsigned long long nm = 0;
    std::memcpy(&nm, pl->host + sizeof(int32_t) * kDirtyHist, 8);
    std::vector<uint64_t> acc_h(W);
    std::memcpy(acc_h.data(), pl->host + sizeof(int32_t) * kDirtyHist + 8, 8 * (size_t)W);
    const int64_t T = dirty_first_fixpoint(hh, 1, kFirstBatch + 1);
    int32_t prods = (int32_t)T;
    uint64_t *fix = pl->buf[0];
    if (T < 0) {  // more products than the graph holds
        if ((rc = dirty_finish(m, s, kFirstBatch + 1, hh, st, &prods, &fix))) return rc;
        LP_HIP(launch_zero_words(pl->cnt_d, 2, st));
        LP_HIP(launch_stable_check(fix, log2W, W, m.dev.q_rows, m.n_std, m.K, keff, pl->acc_d, pl->cnt_d, st));
        LP_HIP(hipMemcpyAsync(acc_h.data(), pl->acc_d, 8 * (size_t)W, hipMemcpyDeviceToHost, st));
        LP_HIP(hipMemcpyAsync(&nm, pl->cnt_d, 8, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
    }
    Scratch S(st);
    // the reset follows the copies out of the fixpoint on the stream; one synchronization ends both
    if ((rc = stable_outputs(m, fix, log2W, W, acc_h.data(), nm, accepted, n_models, models, max_models, interp, S,
                             st, false)))
        return rc;
    LP_HIP(launch_dirty_reset(pl->buf[0], pl->buf[1], log2W, pl->sets, s.nb, s.grid, st));
    LP_HIP(hipStreamSynchronize(st));
    pl->ready = true;
    if (products) *products = prods;
    if (models && (int64_t)nm > max_models) return LP_E_TRUNCATED;
    return LP_OK;
}

static lp_status stable_impl(const Matrix &m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                             int64_t max_models, uint64_t *interp, int32_t *products, hipStream_t st) {
    const int K = m.K;
    if (K == 0) {
        // definite program: exactly one stable model, the least model
        std::vector<uint8_t> lm(m.n_atoms ? m.n_atoms : 1);
        lp_status rc = least_model_impl(m, lm.data(), products, nullptr, st);
        if (rc) return rc;
        accepted[0] = 1;
        *n_models = 1;
        if (models && max_models >= 1) std::memcpy(models, lm.data(), m.n_atoms);
        if (interp)
            for (int32_t a = 0; a < m.n_atoms; ++a) interp[a] = lm[a];
        if (models && max_models < 1) return LP_E_TRUNCATED;
        return LP_OK;
    }
    if (interp && m.K_eff != K) {
        set_error("interp output needs a matrix built without LP_PRUNE_FACT_GUESSES");
        return LP_E_INVAL;
    }
    const int keff = m.K_eff;
    const int64_t H = 1ll << keff;
    const int64_t W = (H + 63) / 64;
    const int log2W = ilog2(W);
    const int64_t total = (int64_t)m.n_rows * W;
    if (dirty_products(m, log2W) && total <= kPlanMaxWords) {
        bool used = false;
        lp_status rc = stable_plan_solve(m, keff, log2W, accepted, n_models, models, max_models, interp, products, st,
                                         &used);
        if (used) return rc;
    }
    lp_status rc = check_device_memory(2.0 * (double)total * 8.0 + (double)W * 8.0 + 4096.0, "stable models");
    if (rc) return rc;
    Scratch S(st);
    uint64_t *buf[2];
    uint64_t *acc_d;
    unsigned long long *counters;
    if ((rc = S.get(&buf[0], total)) || (rc = S.get(&buf[1], total)) || (rc = S.get(&acc_d, W)) ||
        (rc = S.get(&counters, kRing)))
        return rc;
    int32_t prods = -1;
    uint64_t *fix = nullptr;
    if ((rc = stable_fixpoint(m, st, buf, counters, &prods, &fix))) return rc;
    // Algorithm 3
    unsigned long long *cnt_d = counters;  // slot 0 is free once the loop is done
    LP_HIP(hipMemsetAsync(cnt_d, 0, sizeof(unsigned long long), st));
    LP_HIP(launch_stable_check(fix, log2W, W, m.dev.q_rows, m.n_std, K, keff, acc_d, cnt_d, st));
    std::vector<uint64_t> acc_h(W);
    unsigned long long nm = 0;
    LP_HIP(hipMemcpyAsync(acc_h.data(), acc_d, W * 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(&nm, cnt_d, 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    if ((rc = stable_outputs(m, fix, log2W, W, acc_h.data(), nm, accepted, n_models, models, max_models, interp, S,
                             st)))
        return rc;
    if (products) *products = prods;
    if (models && (int64_t)nm > max_models) return LP_E_TRUNCATED;
    return LP_OK;
}

// Algorithms 2 and 3 on caller-given guesses (K <= 64): column j of the
// initial matrix is guesses[j]. The columns are padded to a power of two of
// words with copies of guesses[0]; padded columns are ignored.
// accepted: bits of the n guesses; next (nullable): for each guess, the guess
// its fixpoint points to (qbar_t = not q_t); models (nullable): the first
// max_models accepted columns restricted to the original atoms.
static lp_status guesses_impl(const Matrix &m, const uint64_t *guesses, int64_t n, uint64_t *accepted,
                              int64_t *n_accepted, uint64_t *next, uint8_t *models, int64_t max_models,
                              int32_t *products, hipStream_t st) {
    const int K = m.K;
    const int64_t W = std::max<int64_t>(1, (int64_t)1 << ilog2((n + 63) / 64));
    const int64_t cols = W * 64;
    const int log2W = ilog2(W);
    const int64_t total = (int64_t)m.n_rows * W;
    size_t free_b = 0, total_b = 0;
    LP_HIP(hipMemGetInfo(&free_b, &total_b));
    double avail = (double)free_b;
    {
        DevicePool &P = pool();
        std::lock_guard<std::mutex> lock(P.mu);
        avail += (double)P.cached;
    }
    const double need = 2.0 * (double)total * 8.0 + 2.0 * (double)cols * 8.0 + (double)W * 8.0 + 4096.0;
    if (need > avail) {
        set_error("guess evaluation needs " + std::to_string((long long)need) + " bytes of device memory, " +
                  std::to_string((long long)avail) + " available");
        return LP_E_NOMEM;
    }
    const uint64_t kmask = K == 64 ? ~0ull : ((1ull << K) - 1ull);
    std::vector<uint64_t> g((size_t)cols);
    unsigned long long m0_bits = (unsigned long long)m.info.n_fact_rows * (unsigned long long)cols;
    for (int64_t j = 0; j < cols; ++j) {
        g[j] = (j < n ? guesses[j] : guesses[0]) & kmask;
        m0_bits += (unsigned long long)__builtin_popcountll(g[j]);
    }
    Scratch S(st);
    uint64_t *buf[2], *acc_d, *g_d, *next_d;
    unsigned long long *counters;
    lp_status rc;
    if ((rc = S.get(&buf[0], total)) || (rc = S.get(&buf[1], total)) || (rc = S.get(&acc_d, W)) ||
        (rc = S.get(&g_d, cols)) || (rc = S.get(&next_d, cols)) || (rc = S.get(&counters, kRing)))
        return rc;
    LP_HIP(hipMemcpyAsync(g_d, g.data(), cols * 8, hipMemcpyHostToDevice, st));
    LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
    LP_HIP(launch_init_guess(buf[0], buf[1], total, log2W, m.n_std, K, m.dev.fact_bits, g_d, st));
    LP_HIP(hipMemcpyAsync(counters, &m0_bits, 8, hipMemcpyHostToDevice, st));
    SpmmParams p = spmm_params(m, counters, log2W);
    int32_t prods = -1;
    uint64_t *fix = nullptr;
    if ((rc = stable_loop(m, p, st, buf, counters, &prods, &fix))) return rc;
    unsigned long long *cnt_d = counters;
    LP_HIP(hipMemsetAsync(cnt_d, 0, sizeof(unsigned long long), st));
    LP_HIP(launch_stable_check(fix, log2W, W, m.dev.q_rows, m.n_std, K, 6, acc_d, cnt_d, st));
    if (next) LP_HIP(launch_next_guess(fix, log2W, cols, m.dev.q_rows, K, next_d, st));
    std::vector<uint64_t> acc_h(W);
    LP_HIP(hipMemcpyAsync(acc_h.data(), acc_d, W * 8, hipMemcpyDeviceToHost, st));
    if (next) LP_HIP(hipMemcpyAsync(next, next_d, n * 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    std::memset(accepted, 0, sizeof(uint64_t) * (size_t)((n + 63) / 64));
    std::vector<int64_t> acc_cols;
    int64_t na = 0;
    for (int64_t j = 0; j < n; ++j)
        if ((acc_h[j >> 6] >> (j & 63)) & 1ull) {
            accepted[j >> 6] |= 1ull << (j & 63);
            ++na;
            if (models && (int64_t)acc_cols.size() < max_models) acc_cols.push_back(j);
        }
    *n_accepted = na;
    if (models && !acc_cols.empty() && m.n_atoms) {
        int64_t *cols_d;
        uint8_t *out_d;
        const int64_t nb = (int64_t)acc_cols.size() * m.n_atoms;
        if ((rc = S.get(&cols_d, acc_cols.size())) || (rc = S.get(&out_d, nb))) return rc;
        LP_HIP(hipMemcpyAsync(cols_d, acc_cols.data(), acc_cols.size() * 8, hipMemcpyHostToDevice, st));
        LP_HIP(launch_extract(fix, log2W, cols_d, (int64_t)acc_cols.size(), m.n_atoms, out_d, st));
        LP_HIP(hipMemcpyAsync(models, out_d, nb, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
    }
    if (products) *products = prods;
    if (models && na > max_models) return LP_E_TRUNCATED;
    return LP_OK;
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output number i of the stream with the given seed.
static inline uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Guess sampling with local search (for K too large to enumerate): rounds of
// n_samples guesses. Round 0 draws them from splitmix64(seed, j). Afterwards a
// column that was not accepted continues with its guess where each bit that
// disagrees with the guess its fixpoint points to (qbar_t = not q_t) is
// flipped with probability 1/2 (a random mask from the same stream; at least
// one bit flips): flipping all of them can oscillate, as in an even loop
// a <- not b, b <- not a, where assuming both or neither maps to the other.
// An accepted column continues with a fresh draw. Every accepted guess is a
// stable model (Algorithm 3's test); the search is not complete. found: the
// distinct accepted guesses, ascending, the first max_found of them.
static lp_status search_impl(const Matrix &m, int64_t n_samples, int32_t rounds, uint64_t seed, uint64_t *found,
                             int64_t max_found, int64_t *n_found, uint8_t *models, hipStream_t st) {
    const int K = m.K;
    const uint64_t kmask = K == 64 ? ~0ull : ((1ull << K) - 1ull);
    std::vector<uint64_t> g((size_t)n_samples), nx((size_t)n_samples), acc((size_t)(n_samples + 63) / 64);
    uint64_t draws = 0;
    for (int64_t j = 0; j < n_samples; ++j) g[j] = splitmix64(seed, draws++) & kmask;
    std::vector<uint64_t> hits;
    for (int32_t r = 0; r < rounds; ++r) {
        int64_t na = 0;
        lp_status rc = guesses_impl(m, g.data(), n_samples, acc.data(), &na, nx.data(), nullptr, 0, nullptr, st);
        if (rc) return rc;
        for (int64_t j = 0; j < n_samples; ++j) {
            const bool ok = (acc[j >> 6] >> (j & 63)) & 1ull;
            if (ok) hits.push_back(g[j]);
            const uint64_t diff = g[j] ^ nx[j];  // 0 iff accepted
            if (ok || diff == 0) {
                g[j] = splitmix64(seed, draws++) & kmask;
            } else {
                uint64_t flip = diff & splitmix64(seed, draws++);
                if (flip == 0) flip = diff & (~diff + 1);  // the lowest disagreeing bit
                g[j] ^= flip;
            }
        }
    }
    std::sort(hits.begin(), hits.end());
    hits.erase(std::unique(hits.begin(), hits.end()), hits.end());
    *n_found = (int64_t)hits.size();
    const int64_t keep = std::min<int64_t>((int64_t)hits.size(), max_found);
    if (keep > 0) std::memcpy(found, hits.data(), sizeof(uint64_t) * (size_t)keep);
    if (models && keep > 0) {
        std::vector<uint64_t> acc2((size_t)(keep + 63) / 64);
        int64_t na = 0;
        lp_status rc = guesses_impl(m, hits.data(), keep, acc2.data(), &na, nullptr, models, keep, nullptr, st);
        if (rc && rc != LP_E_TRUNCATED) return rc;
        if (na != keep) {
            set_error("a found guess was not accepted again");
            return LP_E_INTERNAL;
        }
    }
    return (int64_t)hits.size() > max_found ? LP_E_TRUNCATED : LP_OK;
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    lp_status init() {
        LP_HIP(hipEventCreate(&a));
        LP_HIP(hipEventCreate(&b));
        return LP_OK;
    }
    lp_status elapsed(float *ms) {
        LP_HIP(hipEventSynchronize(b));
        LP_HIP(hipEventElapsedTime(ms, a, b));
        return LP_OK;
    }
};

// Buffers for timing steps on a fixed v: the fixpoint (so every launch does
// the same work) and a destination pre-loaded with it.
struct StepBench {
    uint64_t *fix = nullptr, *dst = nullptr, *pacc = nullptr;
    unsigned long long *counters = nullptr;
    uint32_t *and_cnt = nullptr;
    int32_t products = 0;
};

static lp_status step_bench_init(const Matrix &m, const lp_schedule *sched, hipStream_t st, Scratch &S,
                                 StepBench *B) {
    // the timed steps read and write whole interpretations (n_rows bits); the
    // automatic driver's one-workgroup loop returns only the original atoms'
    // bits, so the fixpoint comes from the batched step driver instead
    lp_schedule fs = sched ? *sched : lp_schedule{};
    if (fs.driver == LP_DRIVER_AUTO) fs.driver = LP_DRIVER_BATCHED;
    lp_status rc = least_fixpoint(m, &fs, st, S, &B->fix, &B->products);
    if (rc) return rc;
    const int64_t W = n_words_of(m.n_rows);
    if ((rc = S.get(&B->dst, W)) || (rc = S.get(&B->counters, kRing)) ||
        (rc = S.get(&B->and_cnt, 2 * (size_t)m.dev.n_long_and)) ||
        (!m.dev.slices.empty() && (rc = S.get(&B->pacc, W))))
        return rc;
    LP_HIP(hipMemcpyAsync(B->dst, B->fix, W * 8, hipMemcpyDeviceToDevice, st));
    LP_HIP(hipMemsetAsync(B->counters, 0, sizeof(unsigned long long) * kRing, st));
    if (m.dev.n_long_and) LP_HIP(hipMemsetAsync(B->and_cnt, 0, sizeof(uint32_t) * 2 * m.dev.n_long_and, st));
    return LP_OK;
}

// Average ms of reps back-to-back full-sweep steps of shape L.
static lp_status time_steps(const Matrix &m, const StepBench &B, const StepShape &L, StepParams p, int reps,
                            hipStream_t st, float *avg_ms) {
    p.counters = B.counters;
    p.and_cnt = B.and_cnt;
    p.pacc = B.pacc;
    p.early_exit = 0;
    p.v = B.fix;
    p.u = B.dst;
    Events ev;
    lp_status rc = ev.init();
    if (rc) return rc;
    LP_HIP(hipEventRecord(ev.a, st));
    for (int i = 0; i < reps; ++i) {
        p.step = 2 + (i & 127);
        LP_HIP(launch_step(L, p, st));
    }
    LP_HIP(hipEventRecord(ev.b, st));
    float total = 0.f;
    if ((rc = ev.elapsed(&total))) return rc;
    *avg_ms = reps > 0 ? total / reps : 0.f;
    return LP_OK;
}

// Average ms per launch of the persistent kernel, each launch a whole fixpoint.
static lp_status time_persistent(const Matrix &m, const StepBench &B, const StepShape &L, StepParams p, int reps,
                                 hipStream_t st, Scratch &S, float *avg_ms) {
    const int64_t W = n_words_of(m.n_rows);
    uint64_t *buf[2] = {B.fix, B.dst};
    int32_t *res;
    lp_status rc;
    if ((rc = S.get(&res, 4))) return rc;
    p.counters = B.counters;
    p.and_cnt = B.and_cnt;
    Events ev;
    if ((rc = ev.init())) return rc;
    float total = 0.f;
    for (int i = 0; i < reps; ++i) {
        LP_HIP(hipMemcpyAsync(buf[0], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemcpyAsync(buf[1], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemsetAsync(B.counters, 0, sizeof(unsigned long long) * kRing, st));
        if (m.dev.n_long_and) LP_HIP(hipMemsetAsync(B.and_cnt, 0, sizeof(uint32_t) * 2 * m.dev.n_long_and, st));
        LP_HIP(hipEventRecord(ev.a, st));
        if ((rc = run_persistent(m, p, L, buf, res, st))) return rc;
        LP_HIP(hipEventRecord(ev.b, st));
        float ms = 0;
        if ((rc = ev.elapsed(&ms))) return rc;
        total += ms;
        int32_t prods = 0;
        LP_HIP(hipMemcpy(&prods, res, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (prods < 1) {
            set_error(prods == -2 ? "persistent step: a workgroup gave up waiting at the grid barrier"
                                  : "fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
    *avg_ms = reps > 0 ? total / reps : 0.f;
    return LP_OK;
}

// Average ms of the stable-model step on m's fixpoint interpretation matrix
// (every launch reads the same V and writes the same U), over reps launches.
static lp_status bench_spmm_impl(const Matrix &m, int32_t reps, float *avg_ms, int32_t *products, hipStream_t st) {
    const int64_t W = ((1ll << m.K_eff) + 63) / 64;
    const int64_t total = (int64_t)m.n_rows * W;
    Scratch S(st);
    uint64_t *buf[2];
    unsigned long long *counters;
    lp_status rc;
    if ((rc = S.get(&buf[0], total)) || (rc = S.get(&buf[1], total)) || (rc = S.get(&counters, kRing))) return rc;
    int32_t prods = 0;
    uint64_t *fix = nullptr;
    if ((rc = stable_fixpoint(m, st, buf, counters, &prods, &fix))) return rc;
    SpmmParams p = spmm_params(m, counters);
    p.early_exit = 0;
    p.V = fix;
    p.U = fix == buf[0] ? buf[1] : buf[0];
    p.step = 1;
    LP_HIP(launch_spmm_step(p, spmm_grid(m), st));  // warm-up
    Events ev;
    if ((rc = ev.init())) return rc;
    LP_HIP(hipEventRecord(ev.a, st));
    for (int i = 0; i < reps; ++i) LP_HIP(launch_spmm_step(p, spmm_grid(m), st));
    LP_HIP(hipEventRecord(ev.b, st));
    float ms = 0.f;
    if ((rc = ev.elapsed(&ms))) return rc;
    *avg_ms = ms / (float)reps;
    if (products) *products = prods;
    return LP_OK;
}

static lp_status bench_step_impl(const Matrix &m, const lp_schedule *sched, int32_t reps, float *avg_ms,
                                 hipStream_t st) {
    Scratch S(st);
    StepBench B;
    lp_status rc = step_bench_init(m, sched, st, S, &B);
    if (rc) return rc;
    StepParams p = step_params(m);
    StepShape L;
    if (sched && sched->driver == LP_DRIVER_PERSISTENT) {
        if ((rc = plan_persistent(m, sched, p, &L, st))) return rc;
        if (L.grid < 1) {
            set_error("the persistent step does not fit on this device");
            return LP_E_DEVICE;
        }
        return time_persistent(m, B, L, p, reps, st, S, avg_ms);
    }
    if ((rc = plan_step(m, sched, p, &L, st))) return rc;
    return time_steps(m, B, L, p, reps, st, avg_ms);
}

// Autotuner: time every supported step shape (LDS-staged and global
// gathers; 4 or 8 words per super-block; 4/8/16 chunks in flight) on the matrix's
// own fixpoint, then compare whole solves with the batched and persistent
// drivers at the fastest shape.
static lp_status tune_impl(const Matrix &m, int32_t reps, lp_schedule *best, float *best_step_ms,
                           float *best_solve_ms, hipStream_t st) {
    Scratch S(st);
    StepBench B;
    lp_status rc = step_bench_init(m, nullptr, st, S, &B);
    if (rc) return rc;
    lp_schedule cand{};
    lp_schedule win{};
    float win_ms = 0.f;
    bool have = false;
    const int variants[2] = {LP_STEP_LDS, LP_STEP_GLOBAL};
    const int wpws[2] = {4, 8};
    const int unrolls[3] = {4, 8, 16};
    for (int v : variants)
        for (int w : wpws)
            for (int u : unrolls) {
                cand = lp_schedule{};
                cand.variant = v;
                cand.wpw = w;
                cand.unroll = u;
                StepShape probe;
                probe.wpw = w;
                probe.unroll = u;
                if (!step_shape_supported(probe)) continue;
                StepParams p = step_params(m);
                StepShape L;
                if ((rc = plan_step(m, &cand, p, &L, st))) return rc;
                float ms = 0.f;
                if ((rc = time_steps(m, B, L, p, 2, st, &ms))) return rc;  // warm-up
                if ((rc = time_steps(m, B, L, p, reps, st, &ms))) return rc;
                if (!have || ms < win_ms) {
                    win = cand;
                    win_ms = ms;
                    have = true;
                }
            }
    // drivers at the winning shape: whole solves
    lp_schedule batched = win;
    batched.driver = LP_DRIVER_BATCHED;
    batched.steps_per_sync = 64;
    lp_schedule persistent = win;
    persistent.driver = LP_DRIVER_PERSISTENT;
    persistent.variant = LP_STEP_LDS;
    float t_b = 0.f, t_p = 1e30f;
    {
        Events ev;
        if ((rc = ev.init())) return rc;
        for (int i = 0; i < 2; ++i) {
            Scratch S2(st);
            uint64_t *fx;
            int32_t pr;
            LP_HIP(hipEventRecord(ev.a, st));
            if ((rc = least_fixpoint(m, &batched, st, S2, &fx, &pr))) return rc;
            LP_HIP(hipEventRecord(ev.b, st));
            if ((rc = ev.elapsed(&t_b))) return rc;
        }
    }
    // The persistent form only pays when a product is short enough for launch
    // overhead to matter; above ~20 us a back-to-back launch is cheaper than
    // the grid-wide barrier, so larger matrices skip the trial.
    if (win_ms < 0.020f) {
        StepParams p = step_params(m);
        StepShape L;
        if ((rc = plan_persistent(m, &persistent, p, &L, st))) return rc;
        if (L.grid >= 1) {
            float ms = 0.f;
            if ((rc = time_persistent(m, B, L, p, 1, st, S, &ms))) return rc;
            if ((rc = time_persistent(m, B, L, p, 2, st, S, &ms))) return rc;
            t_p = ms;
        }
    }
    *best = t_p < t_b ? persistent : batched;
    if (best_step_ms) *best_step_ms = win_ms;
    if (best_solve_ms) *best_solve_ms = t_p < t_b ? t_p : t_b;
    sched_store(m, *best);  // the default driver takes it for matrices of this size bucket
    return LP_OK;
}

// ------------------------------------------------------------------ batches
//
// A batch plan holds, for many definite programs, one descriptor per program
// (pointers into the programs' own device layouts), the queue order (largest
// first), the output words of every program and one hipGraph with the batch
// kernel. A run is one graph launch; results are read afterwards. Programs
// whose two LDS buffers exceed the workgroup's LDS are solved by the
// single-program drivers when the results are read.

struct BatchShape {
    int wpw = kBatchWpw;
    int unroll = kBatchUnroll;
    int block = 1024;  // the autotuner's usual winner (one workgroup of 16 waves per CU)
    int grid = 0;
    size_t lds_bytes = 0;
};

// Smallest program work (stored entries + rows) that a team is formed for: below
// it a product takes a workgroup a few microseconds, about a team barrier.
constexpr int64_t kTeamMinWork = 1 << 16;
// Cost model of the team layout, in units of work (stored entries + rows) per
// product, fitted to per-program times of the 512-program batch on MI355X: a
// team member is 1/8 slower per unit of work than a workgroup alone (barrier,
// exchange), and a product costs about 4,500 units more than its work.
constexpr double kTeamCost = 1.125;
constexpr double kProductCost = 4500.0;
// Polls after which a team barrier gives up (a few seconds: far beyond any
// wait of members that run at once).
constexpr uint32_t kTeamPolls = 1u << 22;
// Dynamic LDS of the frontier batch kernel for the counts and v of programs
// small enough to keep them there.
constexpr size_t kFBatchLdsBytes = 128 << 10;

struct BatchPlan {
    int device = -1;
    std::vector<const Matrix *> ms;
    std::vector<int32_t> order;      // resident programs: team programs first, then largest first
    std::vector<int32_t> large;      // programs solved by the single-program drivers
    std::vector<int32_t> team;       // workgroups per resident program (1: alone), by program index
    std::vector<int32_t> item_prog;  // queue position -> program
    std::vector<int32_t> item_member;// queue position -> member of the program's team
    int32_t n_teams = 0;
    mutable int32_t team_fallbacks = 0;  // team programs re-solved alone after a team gave up (counted by results)
    uint64_t *d_xch = nullptr;
    uint32_t *d_teams = nullptr;
    int32_t *d_member = nullptr;
    std::vector<int64_t> out_off;    // first output word of each resident program, -1 otherwise
    int64_t out_words = 0;
    int32_t lds_words = 0;
    ProgDesc *d_progs = nullptr;
    int32_t *d_order = nullptr;
    unsigned int *d_queue = nullptr;
    uint64_t *d_out = nullptr;
    int32_t *d_prod = nullptr;
    BatchShape shape;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    lp_schedule sched{};             // schedule of the single-program solves
    float tuned_ms = 0.f;
    bool use_graph = true;           // runs replay a captured graph (else a direct launch)
    bool weighted = false;           // order and teams weighted by the product counts of a run
    // frontier plans (sched->driver == LP_DRIVER_FRONTIER): every program by
    // frontier levels (frontier_batch_kernel); d_out holds whole interpretations
    bool frontier = false;
    FBatchProg *d_fprogs = nullptr;
    int32_t *d_cnt = nullptr;
    int32_t *d_fq = nullptr;
    int64_t fq_cap = 0;
    int32_t f_lds_rows = 0;          // frontier plans: programs of at most this many rows keep counts and v in LDS
};

static void batch_release(BatchPlan &b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    void *ps[] = {b.d_progs, b.d_order, b.d_queue, b.d_out, b.d_prod, b.d_xch, b.d_teams, b.d_member,
                  b.d_fprogs, b.d_cnt, b.d_fq};
    for (void *p : ps) dev_free(p, nullptr);
    b.d_fprogs = nullptr;
    b.d_cnt = nullptr;
    b.d_fq = nullptr;
    b.d_xch = nullptr;
    b.d_teams = nullptr;
    b.d_member = nullptr;
    b.d_progs = nullptr;
    b.d_order = nullptr;
    b.d_queue = nullptr;
    b.d_out = nullptr;
    b.d_prod = nullptr;
}

static BatchParams batch_params(const BatchPlan &b, const BatchShape &s) {
    BatchParams q{};
    q.lds_layout_bytes = (int32_t)std::max<int64_t>(0, (int64_t)s.lds_bytes - (int64_t)b.lds_words * 16);
    q.progs = b.d_progs;
    q.order = b.d_order;
    q.member = b.d_member;
    q.queue = b.d_queue;
    q.teams = b.d_teams;
    q.n_items = (int32_t)b.item_prog.size();
    q.n_teams = b.n_teams;
    q.lds_words = b.lds_words;
    q.team_polls = b.sched.team_polls > 0 ? (uint32_t)b.sched.team_polls : kTeamPolls;
    return q;
}

// Fills in lds_bytes and grid: as many workgroups as fit on the device at
// once, but no more than there are queue positions.
static lp_status batch_fit_shape(const BatchPlan &b, BatchShape *s) {
    if (!batch_shape_supported(s->wpw, s->unroll) || (s->block != 256 && s->block != 512 && s->block != 1024)) {
        set_error("unsupported batch shape (wpw/unroll 4/4, 4/8, 4/16, 8/8, 8/16; block 256, 512 or 1024)");
        return LP_E_INVAL;
    }
    DevProps d;
    lp_status rc = dev_props(b.device, &d);
    if (rc) return rc;
    s->lds_bytes = (size_t)b.lds_words * 16;
    int per_cu = 0;
    LP_HIP(batch_occupancy(s->wpw, s->unroll, s->block, s->lds_bytes, &per_cu));
    if (per_cu < 1) {
        set_error("the batch kernel does not fit on this device");
        return LP_E_DEVICE;
    }
    // LDS the resident workgroups leave unused holds the layouts of programs
    // small enough to be copied in: the largest extension that keeps as many
    // workgroups per CU
    for (size_t extra : {(size_t)128 << 10, (size_t)96 << 10, (size_t)64 << 10, (size_t)48 << 10,
                         (size_t)32 << 10, (size_t)16 << 10}) {
        const size_t want = s->lds_bytes + extra;
        if (want > (size_t)d.max_lds - 4096) continue;
        int pc = 0;
        if (batch_occupancy(s->wpw, s->unroll, s->block, want, &pc) == hipSuccess && pc >= per_cu) {
            s->lds_bytes = want;
            break;
        }
        (void)hipGetLastError();
    }
    const int64_t resident = (int64_t)per_cu * d.n_cu;
    const int64_t want = s->grid > 0 ? s->grid : resident;
    s->grid = (int)std::max<int64_t>(1, std::min<int64_t>({want, resident, (int64_t)b.item_prog.size()}));
    int32_t max_team = 1;
    for (int32_t i : b.order) max_team = std::max(max_team, b.team[i]);
    if (s->grid < max_team) {
        // a team waits for all of its members: they must be able to run at once
        set_error("batch grid of " + std::to_string(s->grid) + " workgroups is smaller than a team of " +
                  std::to_string(max_team));
        return LP_E_INVAL;
    }
    return LP_OK;
}

// Captures the batch kernel into b.exec (on a stream of its own: the legacy
// default stream cannot be captured).
static FBatchParams fbatch_params(const BatchPlan &b);

static lp_status batch_capture(BatchPlan &b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    if (b.order.empty()) return LP_OK;
    hipStream_t cs;
    LP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const BatchShape &s = b.shape;
        hipError_t el = b.frontier ? launch_frontier_batch(fbatch_params(b), s.grid, cs)
                                   : launch_batch(s.wpw, s.unroll, s.grid, s.block, s.lds_bytes, batch_params(b, s), cs);
        e = hipStreamEndCapture(cs, &b.graph);
        if (e == hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "batch graph capture");
    return LP_OK;
}

static lp_status batch_layout(BatchPlan &b, const lp_schedule *sched, hipStream_t st,
                              const std::vector<int32_t> *weights);
static lp_status frontier_batch_layout(BatchPlan &b, const lp_schedule *sched, hipStream_t st);

static lp_status batch_create(const lp_matrix *const *ms, int32_t count, const lp_schedule *sched, hipStream_t st,
                              bool use_graph, BatchPlan &b) {
    b.use_graph = use_graph;
    b.ms.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        if (!ms[i]) {
            set_error("NULL matrix at batch position " + std::to_string(i));
            return LP_E_INVAL;
        }
        const Matrix &m = ms[i]->m;
        if (m.flags & LP_BUILD_HOST_ONLY) {
            set_error("matrix " + std::to_string(i) + " was built with LP_BUILD_HOST_ONLY");
            return LP_E_HOST_ONLY;
        }
        if (m.K) {
            set_error("program " + std::to_string(i) + " has negative literals");
            return LP_E_NEGATION;
        }
        if (i == 0) b.device = m.dev.device;
        else if (m.dev.device != b.device) {
            set_error("the matrices of a batch must live on one device");
            return LP_E_INVAL;
        }
        b.ms[i] = &m;
    }
    if (count == 0) {
        LP_HIP(hipGetDevice(&b.device));
    }
    if (sched && sched->driver == LP_DRIVER_FRONTIER) return frontier_batch_layout(b, sched, st);
    return batch_layout(b, sched, st, nullptr);
}

// A frontier plan: every program's transposed matrix (built on first use and
// kept with the matrix), working counts and interpretation; the queue, largest
// program first; one 1,024-thread workgroup per CU, each with two frontier
// buffers as long as the largest program's rows.
static lp_status frontier_batch_layout(BatchPlan &b, const lp_schedule *sched, hipStream_t st) {
    const int32_t count = (int32_t)b.ms.size();
    b.frontier = true;
    if (sched) b.sched = *sched;
    b.order.clear();
    b.large.clear();
    b.team.assign(count, 1);
    DevProps d;
    lp_status rc = dev_props(b.device, &d);
    if (rc) return rc;
    std::vector<int32_t> idx(count);
    for (int32_t i = 0; i < count; ++i) {
        idx[i] = i;
        if ((rc = ensure_frontier(*b.ms[i], st))) return rc;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return b.ms[x]->nnz > b.ms[y]->nnz; });
    b.order = idx;
    b.out_off.assign(count, -1);
    std::vector<int64_t> cnt_off(count);
    int64_t words = 0, cnts = 0;
    int32_t max_rows = 1;
    for (int32_t i : idx) {
        b.out_off[i] = words;
        words += std::max<int64_t>(1, n_words_of(b.ms[i]->n_rows));
        cnt_off[i] = cnts;
        cnts += std::max(1, b.ms[i]->n_rows);
        max_rows = std::max(max_rows, b.ms[i]->n_rows);
    }
    b.out_words = words;
    b.lds_words = 0;
    BatchShape s;
    s.block = kFBatchBlock;
    s.grid = (int)std::max<int64_t>(1, std::min<int64_t>(d.n_cu, count));
    s.wpw = 0;
    s.unroll = 0;
    s.lds_bytes = 0;
    b.shape = s;
    b.fq_cap = max_rows;
    // programs of up to f_lds_rows rows keep their counts and v in LDS: as many
    // rows as kFBatchLdsBytes holds (beside the kernel's 8 KB of static LDS),
    // but no more than the largest program needs
    {
        int32_t r = (int32_t)std::min<int64_t>(max_rows, (int64_t)kFBatchLdsBytes / 4);
        const size_t cap = std::min<size_t>(kFBatchLdsBytes, (size_t)std::max(0, d.max_lds - 4096 - 8192));
        while (r > 0 && fbatch_lds_bytes(r) > cap) r -= 64;
        b.f_lds_rows = std::max(0, r);
    }
    if ((rc = dev_alloc((void **)&b.d_out, (size_t)std::max<int64_t>(1, words) * 8, st)) ||
        (rc = dev_alloc((void **)&b.d_prod, sizeof(int32_t) * std::max(1, count), st)) ||
        (rc = dev_alloc((void **)&b.d_cnt, sizeof(int32_t) * (size_t)std::max<int64_t>(1, cnts), st)) ||
        (rc = dev_alloc((void **)&b.d_fq, sizeof(int32_t) * 2 * (size_t)s.grid * (size_t)b.fq_cap, st)))
        return rc;
    std::vector<FBatchProg> desc(std::max(1, count));
    for (int32_t i : idx) {
        const Matrix &m = *b.ms[i];
        FBatchProg &g = desc[i];
        g = FBatchProg{};
        g.occ_ptr = m.dev.fr_ptr;
        g.occ = m.dev.fr_occ;
        g.cnt0 = m.dev.fr_cnt0;
        g.facts = m.dev.fr_facts;
        g.cnt = b.d_cnt + cnt_off[i];
        g.v = b.d_out + b.out_off[i];
        g.out_products = b.d_prod + i;
        g.n_rows = m.n_rows;
        g.n_facts = m.dev.fr_n_facts;
        g.n_words = (int32_t)n_words_of(m.n_rows);
    }
    int64_t dummy = 0;
    if ((rc = upload(&b.d_fprogs, desc.data(), desc.size(), st, &dummy))) return rc;
    std::vector<int32_t> ord(idx);
    if (ord.empty()) ord.push_back(0);
    if ((rc = upload(&b.d_order, ord.data(), ord.size(), st, &dummy))) return rc;
    if ((rc = dev_alloc((void **)&b.d_queue, sizeof(unsigned int) * 2, st))) return rc;
    LP_HIP(hipMemsetAsync(b.d_queue, 0, sizeof(unsigned int) * 2, st));
    LP_HIP(hipStreamSynchronize(st));
    return b.use_graph ? batch_capture(b) : LP_OK;
}

// Queue order, teams, descriptors and buffers of the plan's programs (b.ms),
// its shape and graph. weights: each program's product count from an earlier
// run (the time of a program is about its products times its work per
// product), or null before any run (all 1).
static lp_status batch_layout(BatchPlan &b, const lp_schedule *sched, hipStream_t st,
                              const std::vector<int32_t> *weights) {
    const int32_t count = (int32_t)b.ms.size();
    b.order.clear();
    b.large.clear();
    DevProps d;
    lp_status rc = dev_props(b.device, &d);
    if (rc) return rc;
    // programs whose two buffers fit in the dynamic LDS (the kernel's static
    // LDS takes at most 4 KiB); largest first by weighted work
    const int64_t cap_words = std::max<int64_t>(0, (d.max_lds - 4096) / 16);
    std::vector<int32_t> idx;
    for (int32_t i = 0; i < count; ++i) {
        if (n_words_of(b.ms[i]->n_rows) <= cap_words) idx.push_back(i);
        else b.large.push_back(i);
    }
    // work of one product (stored entries + rows), and of the whole solve
    auto step_work = [&](int32_t i) {
        const Matrix &a = *b.ms[i];
        return a.dev.and_nnz + a.dev.long_nnz + a.n_rows;
    };
    // Teams. sched->team: 0 automatic, 1 no teams, k >= 2 every program in
    // teams of k. Automatic: the layout that a simulation of the queue finds
    // fastest. The simulation prices program i on k workgroups at its product
    // count (weights; 1 before any run) times (work per product, / k and x
    // kTeamCost for a team, + kProductCost); team positions come first (every
    // team starts at once), then the other programs longest first, and each
    // workgroup takes the next position when it is free. Candidates: for a
    // threshold T, every program whose time alone exceeds T gets the fewest
    // members (at most kMaxTeam and half the grid; work per product at least
    // kTeamMinWork) that bring it to T or below; T runs over the longest
    // programs' times alone, and the fastest layout whose members fit in one
    // grid's worth of workgroups is kept.
    b.team.assign(count, 1);
    const int32_t opt = sched ? sched->team : 0;
    const int64_t grid_cap = (sched && sched->grid > 0) ? sched->grid : (int64_t)d.n_cu;
    const int32_t gmax = (int32_t)std::min<int64_t>(kMaxTeam, grid_cap / 2);
    auto est = [&](int32_t i, int32_t k) {
        const double w = (double)step_work(i);
        const double per = (k > 1 ? kTeamCost * w / k : w) + kProductCost;
        return (weights ? (double)std::max<int32_t>(1, (*weights)[i]) : 1.0) * per;
    };
    if (opt >= 2 && gmax >= 2) {
        for (int32_t i : idx) b.team[i] = std::min(opt, gmax);
    } else if (opt == 0 && gmax >= 2 && !idx.empty()) {
        std::vector<int32_t> team(count, 1), ord;
        auto order_by_time = [&]() {
            ord = idx;
            std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
                if ((team[x] > 1) != (team[y] > 1)) return team[x] > 1;
                return est(x, team[x]) > est(y, team[y]);
            });
        };
        auto makespan = [&]() {
            std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
            for (int64_t g = 0; g < grid_cap; ++g) free_at.push(0.0);
            double end = 0.0;
            for (int32_t i : ord) {
                double s = 0.0;
                for (int32_t k = 0; k < team[i]; ++k) {
                    s = std::max(s, free_at.top());
                    free_at.pop();
                }
                const double e = s + est(i, team[i]);
                for (int32_t k = 0; k < team[i]; ++k) free_at.push(e);
                end = std::max(end, e);
            }
            return end;
        };
        std::vector<int32_t> by_alone(idx);
        std::stable_sort(by_alone.begin(), by_alone.end(),
                         [&](int32_t x, int32_t y) { return est(x, 1) > est(y, 1); });
        order_by_time();
        double best = makespan();  // no teams
        std::vector<int32_t> best_team(team);
        const size_t n_cand = std::min<size_t>(by_alone.size(), (size_t)grid_cap);
        for (size_t c = 1; c <= n_cand; ++c) {
            // threshold: the time alone of the c-th longest program; the c-1 longer ones get teams
            const double T = est(by_alone[c - 1], 1);
            std::fill(team.begin(), team.end(), 1);
            int64_t members = 0;
            for (size_t j = 0; j + 1 < c; ++j) {
                const int32_t i = by_alone[j];
                if (step_work(i) < kTeamMinWork) continue;
                int32_t k = 2;
                while (k < gmax && est(i, k) > T) ++k;
                team[i] = k;
                members += k;
            }
            if (members > grid_cap) break;  // later thresholds only add members
            order_by_time();
            const double m = makespan();
            if (m < best) {
                best = m;
                best_team = team;
            }
        }
        for (int32_t i : idx) b.team[i] = best_team[i];
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
        if ((b.team[x] > 1) != (b.team[y] > 1)) return b.team[x] > 1;
        return est(x, b.team[x]) > est(y, b.team[y]);
    });
    b.order = idx;
    b.item_prog.clear();
    b.item_member.clear();
    b.n_teams = 0;
    for (int32_t i : idx)
        for (int32_t k = 0; k < b.team[i]; ++k) {
            b.item_prog.push_back(i);
            b.item_member.push_back(k);
        }
    b.out_off.assign(count, -1);
    std::vector<ProgDesc> desc(count ? count : 1);
    int64_t off = 0;
    int32_t maxw = 0;
    for (int32_t i : idx) {
        b.out_off[i] = off;
        off += n_words_of(b.ms[i]->n_atoms);
        maxw = std::max<int32_t>(maxw, (int32_t)n_words_of(b.ms[i]->n_rows));
    }
    b.out_words = off;
    b.lds_words = maxw;
    if ((rc = dev_alloc((void **)&b.d_out, (size_t)std::max<int64_t>(1, off) * 8, st))) return rc;
    if ((rc = dev_alloc((void **)&b.d_prod, sizeof(int32_t) * std::max(1, count), st))) return rc;
    // exchange buffers and states of the teams
    std::vector<int64_t> xoff(count, -1);
    int64_t xwords = 0;
    for (int32_t i : idx)
        if (b.team[i] > 1) {
            xoff[i] = xwords;
            xwords += 3 * n_words_of(b.ms[i]->n_rows);
            ++b.n_teams;
        }
    if ((rc = dev_alloc((void **)&b.d_xch, (size_t)std::max<int64_t>(1, xwords) * 8, st))) return rc;
    if ((rc = dev_alloc((void **)&b.d_teams, sizeof(uint32_t) * kTeamStateWords * std::max(1, b.n_teams), st)))
        return rc;
    LP_HIP(hipMemsetAsync(b.d_teams, 0, sizeof(uint32_t) * kTeamStateWords * std::max(1, b.n_teams), st));
    int32_t team_no = 0;
    for (int32_t i : idx) {
        const Matrix &m = *b.ms[i];
        ProgDesc &g = desc[i];
        g = prog_desc(m);
        g.out_bits = b.d_out + b.out_off[i];
        g.out_products = b.d_prod + i;
        g.team_size = b.team[i];
        g.xch = b.team[i] > 1 ? b.d_xch + xoff[i] : nullptr;
        g.team = b.team[i] > 1 ? b.d_teams + (int64_t)kTeamStateWords * team_no++ : nullptr;
    }
    int64_t dummy = 0;
    if ((rc = upload(&b.d_progs, desc.data(), desc.size(), st, &dummy))) return rc;
    std::vector<int32_t> ord(b.item_prog), mem(b.item_member);
    if (ord.empty()) ord.push_back(0);
    if (mem.empty()) mem.push_back(0);
    if ((rc = upload(&b.d_order, ord.data(), ord.size(), st, &dummy))) return rc;
    if ((rc = upload(&b.d_member, mem.data(), mem.size(), st, &dummy))) return rc;
    if ((rc = dev_alloc((void **)&b.d_queue, sizeof(unsigned int) * 2, st))) return rc;
    LP_HIP(hipMemsetAsync(b.d_queue, 0, sizeof(unsigned int) * 2, st));
    LP_HIP(hipStreamSynchronize(st));
    if (sched) b.sched = *sched;
    BatchShape s;
    if (sched && sched->wpw > 0) s.wpw = sched->wpw;
    if (sched && sched->unroll > 0) s.unroll = sched->unroll;
    if (sched && sched->block > 0) s.block = sched->block;
    if (sched && sched->grid > 0) s.grid = sched->grid;
    if (!b.order.empty()) {
        if ((rc = batch_fit_shape(b, &s))) return rc;
    }
    b.shape = s;
    return b.use_graph ? batch_capture(b) : LP_OK;
}

static FBatchParams fbatch_params(const BatchPlan &b) {
    FBatchParams q{};
    q.progs = b.d_fprogs;
    q.order = b.d_order;
    q.queue = b.d_queue;
    q.qbuf = b.d_fq;
    q.qcap = b.fq_cap;
    q.n_items = (int32_t)b.order.size();
    q.lds_rows = b.f_lds_rows;
    return q;
}

static lp_status batch_run(const BatchPlan &b, hipStream_t st) {
    if (b.order.empty()) return LP_OK;
    if (b.exec) {
        LP_HIP(hipGraphLaunch(b.exec, st));
    } else if (b.frontier) {
        LP_HIP(launch_frontier_batch(fbatch_params(b), b.shape.grid, st));
    } else {
        const BatchShape &s = b.shape;
        LP_HIP(launch_batch(s.wpw, s.unroll, s.grid, s.block, s.lds_bytes, batch_params(b, s), st));
    }
    return LP_OK;
}

int64_t batch_max_rows(int device) {
    DevProps d;
    if (dev_props(device, &d)) return 0;
    return std::max<int64_t>(0, (d.max_lds - 4096) / 16) * 64;
}

static lp_status batch_results(const BatchPlan &b, uint8_t *const *models, int32_t *products, hipStream_t st) {
    const int32_t count = (int32_t)b.ms.size();
    std::vector<uint64_t> hb(std::max<int64_t>(1, b.out_words));
    std::vector<int32_t> hp(std::max(1, count));
    if (b.out_words) LP_HIP(hipMemcpyAsync(hb.data(), b.d_out, b.out_words * 8, hipMemcpyDeviceToHost, st));
    if (count) LP_HIP(hipMemcpyAsync(hp.data(), b.d_prod, sizeof(int32_t) * count, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> alone(b.large);
    for (int32_t i : b.order) {
        if (hp[i] == -2) {
            // a team gave up waiting for a member (bounded barrier): solve it alone
            alone.push_back(i);
            ++b.team_fallbacks;
            continue;
        }
        if (hp[i] < 1) {
            set_error("fixpoint of batch program " + std::to_string(i) + " not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
        if (models && models[i]) unpack_model(hb.data() + b.out_off[i], b.ms[i]->n_atoms, models[i]);
        if (products) products[i] = hp[i];
    }
    for (int32_t i : alone) {
        int32_t pr = 0;
        std::vector<uint8_t> tmp;
        uint8_t *dst = models ? models[i] : nullptr;
        if (!dst) {
            tmp.resize(std::max(1, b.ms[i]->n_atoms));
            dst = tmp.data();
        }
        lp_status rc = least_model_impl(*b.ms[i], dst, &pr, &b.sched, st);
        if (rc) return rc;
        if (products) products[i] = pr;
    }
    return LP_OK;
}

// Autotuner of the batch kernel. First, once per plan, one run gives every
// program's product count and the queue order and teams are laid out again
// by products times work per product (the first layout knows only the work
// per product). Then it times every supported shape (words per wave and
// chunks in flight, 256/512/1024-thread workgroups) over reps launches of the
// whole batch and keeps the fastest.
static lp_status batch_tune(BatchPlan &b, int32_t reps, float *best_ms, hipStream_t st) {
    if (b.order.empty()) {
        if (best_ms) *best_ms = 0.f;
        return LP_OK;
    }
    if (b.frontier) {  // no shape to choose: the time of reps runs
        Events ev;
        lp_status rc = ev.init();
        if (rc) return rc;
        if ((rc = batch_run(b, st))) return rc;
        LP_HIP(hipEventRecord(ev.a, st));
        for (int r = 0; r < std::max(1, reps); ++r)
            if ((rc = batch_run(b, st))) return rc;
        LP_HIP(hipEventRecord(ev.b, st));
        float ms = 0.f;
        if ((rc = ev.elapsed(&ms))) return rc;
        b.tuned_ms = ms / (float)std::max(1, reps);
        if (best_ms) *best_ms = b.tuned_ms;
        return LP_OK;
    }
    lp_status rc;
    if (!b.weighted) {
        if ((rc = batch_run(b, st))) return rc;
        std::vector<int32_t> prods(b.ms.size(), 1);
        LP_HIP(hipMemcpyAsync(prods.data(), b.d_prod, sizeof(int32_t) * prods.size(), hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        for (int32_t &p : prods) p = std::max(1, p);  // large programs, and teams that gave up: 1
        for (int32_t i : b.large) prods[i] = 1;
        const lp_schedule keep = b.sched;
        batch_release(b);
        if ((rc = batch_layout(b, &keep, st, &prods))) return rc;
        b.weighted = true;
    }
    if (reps == 0) {  // the layout step only, at the plan's shape; one run, so results hold a run
        if (best_ms) *best_ms = 0.f;
        return batch_run(b, st);
    }
    static const int shapes[][2] = {{4, 4}, {4, 8}, {4, 16}, {8, 8}, {8, 16}};
    static const int blocks[] = {256, 512, 1024};
    Events ev;
    if ((rc = ev.init())) return rc;
    BatchShape win;
    float win_ms = 0.f;
    bool have = false;
    for (const auto &sh : shapes)
        for (int blk : blocks) {
            BatchShape s;
            s.wpw = sh[0];
            s.unroll = sh[1];
            s.block = blk;
            s.grid = 0;
            if (batch_fit_shape(b, &s)) continue;  // shapes that do not fit are skipped
            const BatchParams q = batch_params(b, s);
            LP_HIP(launch_batch(s.wpw, s.unroll, s.grid, s.block, s.lds_bytes, q, st));  // warm-up
            LP_HIP(hipEventRecord(ev.a, st));
            for (int r = 0; r < reps; ++r) LP_HIP(launch_batch(s.wpw, s.unroll, s.grid, s.block, s.lds_bytes, q, st));
            LP_HIP(hipEventRecord(ev.b, st));
            float ms = 0.f;
            if ((rc = ev.elapsed(&ms))) return rc;
            ms /= (float)reps;
            if (!have || ms < win_ms) {
                win = s;
                win_ms = ms;
                have = true;
            }
        }
    if (!have) {
        set_error("no batch shape fits on this device");
        return LP_E_DEVICE;
    }
    b.shape = win;
    b.tuned_ms = win_ms;
    if (best_ms) *best_ms = win_ms;
    return b.use_graph ? batch_capture(b) : LP_OK;
}

// ------------------------------------------------------------------ stable batches
//
// Stable models (Algorithms 2 and 3) of several normal programs together:
// each launch takes one product for every program still changing (the union
// of their interpretation matrices, lp_spmm.hip), so a batch of small
// programs costs about the launches of its longest solve instead of the sum
// of them. Programs whose enumerated guesses need more than 64 words per row,
// and definite programs, are solved one after another by stable_impl.

constexpr int kSBatchMaxKeff = 12;  // 2^12 guesses: 64 words per row

static bool sbatch_fits(const Matrix &m) { return m.K >= 1 && m.K_eff <= kSBatchMaxKeff; }

static lp_status sbatch_impl(const std::vector<const Matrix *> &ms, const std::vector<int32_t> &in,
                             uint64_t *const *accepted, int64_t *n_models, uint8_t *const *models, int32_t *products,
                             hipStream_t st) {
    const int32_t n = (int32_t)in.size();
    Scratch S(st);
    std::vector<SBatchProg> desc(n);
    std::vector<int64_t> acc_off(n), model_off(n);
    int64_t chunks = 0, words = 0, acc_words = 0, model_bytes = 0, limit = 0;
    for (int32_t k = 0; k < n; ++k) {
        const Matrix &m = *ms[in[k]];
        const int64_t W = (((int64_t)1 << m.K_eff) + 63) / 64;
        SBatchProg &d = desc[k];
        d = SBatchProg{};
        d.row_ptr = m.dev.full_row_ptr;
        d.col = m.dev.full_col;
        d.and_bits = m.dev.full_and_bits;
        d.fact_bits = m.dev.fact_bits;
        d.guess_pos = m.dev.guess_pos;
        d.q_rows = m.dev.q_rows;
        const unsigned long long H = 1ull << m.K_eff;
        d.m0_bits = (unsigned long long)m.info.n_fact_rows * H + (unsigned long long)m.K_eff * (H / 2);
        d.log2W = ilog2(W);
        d.total = (int64_t)m.n_rows * W;
        d.n_rows = m.n_rows;
        d.n_std = m.n_std;
        d.K = m.K;
        d.k_eff = m.K_eff;
        d.n_atoms = m.n_atoms;
        d.chunk0 = chunks;
        chunks += std::max<int64_t>(1, (d.total + kSBatchChunk - 1) / kSBatchChunk);
        words += 2 * d.total;
        acc_off[k] = acc_words;
        acc_words += W;
        model_off[k] = model_bytes;
        model_bytes += std::max(1, m.n_atoms);
        limit = std::max<int64_t>(limit, (int64_t)m.n_rows + 1);
    }
    uint64_t *bufs, *acc;
    unsigned long long *counts, *nm;
    uint8_t *mod;
    SBatchProg *d_desc;
    lp_status rc;
    if ((rc = S.get(&bufs, (size_t)std::max<int64_t>(1, words))) || (rc = S.get(&acc, (size_t)acc_words)) ||
        (rc = S.get(&counts, (size_t)n * kRing)) || (rc = S.get(&nm, (size_t)n)) ||
        (rc = S.get(&mod, (size_t)model_bytes)) || (rc = S.get(&d_desc, (size_t)n)))
        return rc;
    int64_t off = 0;
    for (int32_t k = 0; k < n; ++k) {
        SBatchProg &d = desc[k];
        d.buf[0] = bufs + off;
        d.buf[1] = bufs + off + d.total;
        off += 2 * d.total;
        d.count = counts + (int64_t)k * kRing;
        d.accepted = acc + acc_off[k];
        d.model = mod + model_off[k];
        d.n_models = nm + k;
    }
    LP_HIP(hipMemcpyAsync(d_desc, desc.data(), sizeof(SBatchProg) * n, hipMemcpyHostToDevice, st));
    DevProps dp;
    if ((rc = dev_props(ms[in[0]]->dev.device, &dp))) return rc;
    const int grid = 8 * std::max(1, dp.n_cu);
    SBatchParams b{d_desc, n, 0, chunks};
    LP_HIP(launch_sbatch_init(b, grid, st));
    // products in batches of 8 between host reads of the counts; a program's
    // product count is the first product whose count equals the one before
    std::vector<unsigned long long> h((size_t)n * kRing);
    std::vector<int32_t> prods(n, 0);
    int32_t left = n;
    const int batch = 8;
    int64_t t = 0;
    for (; left > 0; t += batch) {
        if (t + 1 > limit) {
            set_error("fixpoint of a batch program not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
        for (int i = 1; i <= batch; ++i) {
            b.step = (int32_t)(t + i);
            LP_HIP(launch_sbatch_step(b, grid, st));
        }
        LP_HIP(hipMemcpyAsync(h.data(), counts, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        for (int32_t k = 0; k < n; ++k) {
            if (prods[k]) continue;
            const unsigned long long *c = h.data() + (int64_t)k * kRing;
            for (int i = 1; i <= batch; ++i) {
                const int64_t s = t + i;
                if (c[s & (kRing - 1)] == c[(s - 1) & (kRing - 1)]) {
                    prods[k] = (int32_t)s;
                    --left;
                    break;
                }
            }
        }
    }
    b.step = (int32_t)t;
    LP_HIP(launch_sbatch_outputs(b, st));
    std::vector<uint64_t> acc_h((size_t)acc_words);
    std::vector<unsigned long long> nm_h(n);
    std::vector<uint8_t> mod_h((size_t)model_bytes);
    LP_HIP(hipMemcpyAsync(acc_h.data(), acc, sizeof(uint64_t) * acc_h.size(), hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(nm_h.data(), nm, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(mod_h.data(), mod, mod_h.size(), hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    for (int32_t k = 0; k < n; ++k) {
        const int32_t i = in[k];
        const Matrix &m = *ms[i];
        const int64_t W = (int64_t)1 << desc[k].log2W;
        const int64_t W_full = (((int64_t)1 << m.K) + 63) / 64;
        // accepted guesses in the full guess space (deposit compressed bits)
        std::memset(accepted[i], 0, sizeof(uint64_t) * W_full);
        for (int64_t w = 0; w < W; ++w) {
            uint64_t x = acc_h[acc_off[k] + w];
            while (x) {
                const int bit = __builtin_ctzll(x);
                x &= x - 1;
                const int64_t jc = w * 64 + bit;
                int64_t jf = 0;
                for (int q = 0; q < m.K; ++q)
                    if (m.guess_pos[q] >= 0 && ((jc >> m.guess_pos[q]) & 1)) jf |= 1ll << q;
                accepted[i][jf >> 6] |= 1ull << (jf & 63);
            }
        }
        n_models[i] = (int64_t)nm_h[k];
        if (models && models[i] && m.n_atoms) std::memcpy(models[i], mod_h.data() + model_off[k], m.n_atoms);
        if (products) products[i] = prods[k];
    }
    return LP_OK;
}

static lp_status stable_batch_impl(const std::vector<const Matrix *> &ms, uint64_t *const *accepted,
                                   int64_t *n_models, uint8_t *const *models, int32_t *products, hipStream_t st) {
    std::vector<int32_t> in, alone;
    for (int32_t i = 0; i < (int32_t)ms.size(); ++i) (sbatch_fits(*ms[i]) ? in : alone).push_back(i);
    lp_status rc;
    if (!in.empty() && (rc = sbatch_impl(ms, in, accepted, n_models, models, products, st))) return rc;
    for (int32_t i : alone) {
        int32_t pr = 0;
        rc = stable_impl(*ms[i], accepted[i], &n_models[i], models ? models[i] : nullptr, 1, nullptr, &pr, st);
        if (rc == LP_E_TRUNCATED) rc = LP_OK;  // the first model only
        if (rc) return rc;
        if (products) products[i] = pr;
    }
    return LP_OK;
}

// ------------------------------------------------------------------ dense contrast
//
// The dense-matrix method of the paper's experiments (Section 4): the same
// Algorithms 1 and 2 with M_P expanded to an ld x ld byte matrix (kernels in
// lp_dense.hip). Built per call, released at its end.

struct DenseMatrix {
    uint8_t *M = nullptr;   // [ld][ld]
    int32_t *thr = nullptr; // [ld] count a row needs to fire: AND length, OR 1, padding 1
    uint8_t *fact = nullptr;// [ld] fact rows (the initial vector of Definition 4)
    int64_t ld = 0;
};

static int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

static int64_t dense_ld(const Matrix &m) { return round_up(std::max<int64_t>(m.n_rows, 1), kDenseAlign); }

// Checks that the dense matrix plus extra_bytes fit, then builds it on st.
static lp_status dense_build(const Matrix &m, Scratch &S, hipStream_t st, double extra_bytes, DenseMatrix *D) {
    const int64_t ld = dense_ld(m);
    const double need = (double)ld * (double)ld + 5.0 * (double)ld + 4.0 * (double)(m.nnz + m.n_rows + 1) +
                        extra_bytes + 65536.0;
    lp_status rc = check_device_memory(need, "the dense matrix and its interpretations");
    if (rc) return rc;
    std::vector<int32_t> thr(ld, 1);
    std::vector<uint8_t> fact(ld, 0);
    for (int32_t i = 0; i < m.n_rows; ++i) {
        const int32_t len = m.row_ptr[i + 1] - m.row_ptr[i];
        if (m.kind[i]) {
            if (len == 0) {
                set_error("AND row without entries in the program matrix");
                return LP_E_INTERNAL;
            }
            thr[i] = len;
        }
        fact[i] = m.fact[i] ? 1 : 0;
    }
    int32_t *row_ptr_d, *col_d;
    if ((rc = S.get(&D->M, (size_t)(ld * ld))) || (rc = S.get(&D->thr, ld)) || (rc = S.get(&D->fact, ld)) ||
        (rc = S.get(&row_ptr_d, m.n_rows + 1)) || (rc = S.get(&col_d, std::max<int64_t>(m.nnz, 1))))
        return rc;
    D->ld = ld;
    LP_HIP(hipMemsetAsync(D->M, 0, (size_t)(ld * ld), st));
    LP_HIP(hipMemcpyAsync(D->thr, thr.data(), ld * sizeof(int32_t), hipMemcpyHostToDevice, st));
    LP_HIP(hipMemcpyAsync(D->fact, fact.data(), ld, hipMemcpyHostToDevice, st));
    LP_HIP(hipMemcpyAsync(row_ptr_d, m.row_ptr.data(), (m.n_rows + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (m.nnz) LP_HIP(hipMemcpyAsync(col_d, m.col.data(), m.nnz * sizeof(int32_t), hipMemcpyHostToDevice, st));
    LP_HIP(launch_dense_scatter(D->M, ld, row_ptr_d, col_d, m.n_rows, st));
    LP_HIP(hipStreamSynchronize(st));  // the host vectors above end here
    return LP_OK;
}

// Jacobi loop shared by both algorithms: product(in, out, counter) until a
// product changes nothing. *cur ends as the index of the fixpoint buffer;
// *kernel_ms gets the mean product time (HIP events around each launch).
template <class Product>
static lp_status dense_loop(const Matrix &m, hipStream_t st, Scratch &S, Product product, int *cur, int32_t *products,
                            float *kernel_ms) {
    constexpr size_t n_cnt = (size_t)kDenseCounters * kDenseCounterStride;
    unsigned long long *cnt_d;
    lp_status rc;
    if ((rc = S.get(&cnt_d, n_cnt))) return rc;
    std::vector<unsigned long long> h(n_cnt);
    Events ev;
    if ((rc = ev.init())) return rc;
    double total_ms = 0.0;
    int32_t p = 0;
    int c = 0;
    for (;;) {
        if (p > m.n_rows + 1) {
            set_error("dense fixpoint exceeded n_rows + 1 products");
            return LP_E_INTERNAL;
        }
        LP_HIP(hipMemsetAsync(cnt_d, 0, n_cnt * sizeof(unsigned long long), st));
        LP_HIP(hipEventRecord(ev.a, st));
        LP_HIP(product(c, cnt_d));
        LP_HIP(hipEventRecord(ev.b, st));
        LP_HIP(hipMemcpyAsync(h.data(), cnt_d, n_cnt * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        float ms = 0.f;
        if ((rc = ev.elapsed(&ms))) return rc;
        total_ms += ms;
        ++p;
        c ^= 1;
        unsigned long long changed = 0;
        for (int i = 0; i < kDenseCounters; ++i) changed += h[(size_t)i * kDenseCounterStride];
        if (changed == 0) break;
    }
    *cur = c;
    if (products) *products = p;
    if (kernel_ms) *kernel_ms = (float)(total_ms / p);
    return LP_OK;
}

static lp_status dense_least_impl(const Matrix &m, uint8_t *model, int32_t *products, float *kernel_ms,
                                  hipStream_t st) {
    Scratch S(st);
    DenseMatrix D;
    const int64_t ld = dense_ld(m);
    lp_status rc = dense_build(m, S, st, 2.0 * (double)ld, &D);
    if (rc) return rc;
    uint8_t *v[2];
    if ((rc = S.get(&v[0], ld)) || (rc = S.get(&v[1], ld))) return rc;
    LP_HIP(hipMemcpyAsync(v[0], D.fact, ld, hipMemcpyDeviceToDevice, st));
    int cur = 0;
    auto product = [&](int c, unsigned long long *cnt) {
        return launch_dense_gemv(D.M, ld, v[c], v[c ^ 1], D.thr, cnt, st);
    };
    if ((rc = dense_loop(m, st, S, product, &cur, products, kernel_ms))) return rc;
    if (m.n_atoms) LP_HIP(hipMemcpyAsync(model, v[cur], m.n_atoms, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    return LP_OK;
}

static lp_status dense_stable_impl(const Matrix &m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                                   int64_t max_models, int32_t *products, float *kernel_ms, hipStream_t st) {
    const int K = m.K;
    if (K == 0) {
        // definite program: exactly one stable model, the least model
        std::vector<uint8_t> lm(m.n_atoms ? m.n_atoms : 1);
        lp_status rc = dense_least_impl(m, lm.data(), products, kernel_ms, st);
        if (rc) return rc;
        accepted[0] = 1;
        *n_models = 1;
        if (models && max_models >= 1) std::memcpy(models, lm.data(), m.n_atoms);
        return models && max_models < 1 ? LP_E_TRUNCATED : LP_OK;
    }
    const int64_t h = 1ll << K;
    const int64_t hp = round_up(h, kDenseColAlign);
    const int64_t W = (h + 63) / 64;
    const int64_t ld = dense_ld(m);
    const int splits = dense_gemm_splits(ld, hp);
    const int64_t n_partial = splits > 1 ? splits * hp * ld : 0;
    Scratch S(st);
    DenseMatrix D;
    lp_status rc = dense_build(m, S, st, 2.0 * (double)hp * (double)ld + 4.0 * (double)n_partial + 8.0 * (double)W +
                                             4.0 * K, &D);
    if (rc) return rc;
    uint8_t *V[2];
    uint64_t *acc_d;
    int32_t *q_d, *partial = nullptr;
    unsigned long long *cnt_d;
    if ((rc = S.get(&V[0], (size_t)(hp * ld))) || (rc = S.get(&V[1], (size_t)(hp * ld))) || (rc = S.get(&acc_d, W)) ||
        (rc = S.get(&q_d, K)) || (rc = S.get(&cnt_d, 1)) || (n_partial && (rc = S.get(&partial, n_partial))))
        return rc;
    LP_HIP(hipMemcpyAsync(q_d, m.neg_atoms.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, st));
    LP_HIP(launch_dense_init(V[0], ld, h, hp, D.fact, m.n_std, K, st));
    int cur = 0;
    auto product = [&](int c, unsigned long long *cnt) {
        return launch_dense_gemm(D.M, V[c], V[c ^ 1], ld, hp, partial, D.thr, cnt, st);
    };
    if ((rc = dense_loop(m, st, S, product, &cur, products, kernel_ms))) return rc;
    // Algorithm 3
    LP_HIP(hipMemsetAsync(cnt_d, 0, sizeof(unsigned long long), st));
    LP_HIP(launch_dense_check(V[cur], ld, h, q_d, m.n_std, K, acc_d, cnt_d, st));
    unsigned long long nm = 0;
    LP_HIP(hipMemcpyAsync(accepted, acc_d, W * 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(&nm, cnt_d, 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    *n_models = (int64_t)nm;
    if (models && max_models > 0 && nm && m.n_atoms) {
        std::vector<int64_t> cols;
        for (int64_t w = 0; w < W && (int64_t)cols.size() < max_models; ++w)
            for (uint64_t x = accepted[w]; x && (int64_t)cols.size() < max_models; x &= x - 1)
                cols.push_back(w * 64 + __builtin_ctzll(x));
        int64_t *cols_d;
        uint8_t *out_d;
        const int64_t nb = (int64_t)cols.size() * m.n_atoms;
        if ((rc = S.get(&cols_d, cols.size())) || (rc = S.get(&out_d, nb))) return rc;
        LP_HIP(hipMemcpyAsync(cols_d, cols.data(), cols.size() * 8, hipMemcpyHostToDevice, st));
        LP_HIP(launch_dense_gather(V[cur], ld, cols_d, (int64_t)cols.size(), m.n_atoms, out_d, st));
        LP_HIP(hipMemcpyAsync(models, out_d, nb, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
    }
    if (models && (int64_t)nm > max_models) return LP_E_TRUNCATED;
    return LP_OK;
}

}  // namespace lp

// ------------------------------------------------------------------ C ABI

struct lp_batch {
    lp::BatchPlan b;
};

using namespace lp;

#define LP_GUARD_BEGIN try {
#define LP_GUARD_END                                              \
    }                                                             \
    catch (const std::bad_alloc &) {                              \
        set_error("host allocation failed");                      \
        return LP_E_NOMEM;                                        \
    }                                                             \
    catch (...) {                                                 \
        set_error("unexpected exception");                        \
        return LP_E_INTERNAL;                                     \
    }

extern "C" {

lp_status lp_build_matrix(int32_t n_atoms, int32_t n_rules, const int32_t *head, const int64_t *body_ptr,
                          const int32_t *body_lit, uint32_t flags, void *hip_stream, lp_matrix **out) {
    LP_GUARD_BEGIN
    if (!out) {
        set_error("out must be non-NULL");
        return LP_E_INVAL;
    }
    *out = nullptr;
    lp_matrix *mx = new lp_matrix();
    lp_status rc = build_host(n_atoms, n_rules, head, body_ptr, body_lit, flags, &mx->m);
    if (rc == LP_OK && !(flags & LP_BUILD_HOST_ONLY)) {
        rc = upload_matrix(mx->m, (hipStream_t)hip_stream);
        if (rc) free_device(mx->m, (hipStream_t)hip_stream);
    }
    if (rc) {
        delete mx;
        return rc;
    }
    *out = mx;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_free_matrix(lp_matrix *m) {
    LP_GUARD_BEGIN
    if (!m) return LP_OK;
    if (!(m->m.flags & LP_BUILD_HOST_ONLY)) {
        DeviceGuard g(m->m.dev.device);
        (void)hipDeviceSynchronize();
        free_device(m->m, nullptr);
    }
    delete m;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_matrix_upload(lp_matrix *m, void *hip_stream) {
    LP_GUARD_BEGIN
    if (!m) {
        set_error("NULL matrix");
        return LP_E_INVAL;
    }
    if (!(m->m.flags & LP_BUILD_HOST_ONLY)) return LP_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    lp_status rc = upload_matrix(m->m, st);
    if (rc) {
        (void)hipStreamSynchronize(st);
        free_device(m->m, st);
        return rc;
    }
    m->m.flags &= ~(uint32_t)LP_BUILD_HOST_ONLY;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_matrix_evict(lp_matrix *m) {
    LP_GUARD_BEGIN
    if (!m) {
        set_error("NULL matrix");
        return LP_E_INVAL;
    }
    if (m->m.flags & LP_BUILD_HOST_ONLY) return LP_OK;
    {
        DeviceGuard g(m->m.dev.device);
        free_device(m->m, nullptr);
    }
    m->m.flags |= LP_BUILD_HOST_ONLY;
    m->m.info.device_bytes = 0;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_memory_stats(int64_t *in_use, int64_t *cached) {
    DevicePool &P = pool();
    std::lock_guard<std::mutex> lock(P.mu);
    if (in_use) *in_use = P.in_use;
    if (cached) *cached = P.cached;
    return LP_OK;
}

lp_status lp_release_cached_memory(void) {
    LP_GUARD_BEGIN
    pool_trim(-1);
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_matrix_info(const lp_matrix *m, lp_info *out) {
    if (!m || !out) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    *out = m->m.info;
    if (!(m->m.flags & LP_BUILD_HOST_ONLY)) {
        std::lock_guard<std::mutex> lock(g_lazy_mu);
        out->device_bytes += m->m.dev.lazy_bytes;
        out->n_slices = (int32_t)m->m.dev.slices.size();
    }
    return LP_OK;
}

lp_status lp_matrix_neg_atoms(const lp_matrix *m, int32_t *out) {
    if (!m || (!out && m->m.K)) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    if (m->m.K) std::memcpy(out, m->m.neg_atoms.data(), sizeof(int32_t) * m->m.K);
    return LP_OK;
}

lp_status lp_matrix_csr(const lp_matrix *m, int32_t *row_ptr, int32_t *col, uint8_t *kind, uint8_t *fact) {
    if (!m) {
        set_error("NULL matrix");
        return LP_E_INVAL;
    }
    const Matrix &M = m->m;
    if (row_ptr) std::memcpy(row_ptr, M.row_ptr.data(), sizeof(int32_t) * M.row_ptr.size());
    if (col && M.nnz) std::memcpy(col, M.col.data(), sizeof(int32_t) * M.nnz);
    if (kind && M.n_rows) std::memcpy(kind, M.kind.data(), M.n_rows);
    if (fact && M.n_rows) std::memcpy(fact, M.fact.data(), M.n_rows);
    return LP_OK;
}

static lp_status check_solvable(const lp_matrix *m) {
    if (!m) {
        set_error("NULL matrix");
        return LP_E_INVAL;
    }
    if (m->m.flags & LP_BUILD_HOST_ONLY) {
        set_error("matrix was built with LP_BUILD_HOST_ONLY");
        return LP_E_HOST_ONLY;
    }
    return LP_OK;
}

lp_status lp_least_model(const lp_matrix *m, uint8_t *model, int32_t *products, const lp_schedule *sched,
                         void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K) {
        set_error("the program has negative literals; the least model is defined for definite programs");
        return LP_E_NEGATION;
    }
    if (!model && m->m.n_atoms) {
        set_error("model must be non-NULL");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return least_model_impl(m->m, model, products, sched, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_least_model_noalloc(const lp_matrix *m, uint8_t *model, int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K) {
        set_error("the program has negative literals; the least model is defined for definite programs");
        return LP_E_NEGATION;
    }
    if (!model && m->m.n_atoms) {
        set_error("model must be non-NULL");
        return LP_E_INVAL;
    }
    const size_t need = noalloc_need(m->m);
    if (need > kNoAllocScratchBytes) {
        set_error("the solve needs " + std::to_string(need) + " bytes of scratch; the no-allocation entry point "
                  "holds " + std::to_string(kNoAllocScratchBytes) + " per device");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    void *region = nullptr;
    if ((rc = scratch_region(m->m.dev.device, &region))) return rc;
    Scratch S((hipStream_t)hip_stream, region, kNoAllocScratchBytes);
    return least_model_impl(m->m, model, products, nullptr, (hipStream_t)hip_stream, S);
    LP_GUARD_END
}

lp_status lp_stable_models(const lp_matrix *m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                           int64_t max_models, uint64_t *interp, int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K > LP_MAX_NEG_ATOMS) {
        set_error("too many negated atoms: " + std::to_string(m->m.K));
        return LP_E_TOO_MANY_GUESSES;
    }
    if (!accepted || !n_models || max_models < 0) {
        set_error("accepted and n_models must be non-NULL, max_models >= 0");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return stable_impl(m->m, accepted, n_models, models, max_models, interp, products, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_stable_models_batch(const lp_matrix *const *ms, int32_t count, uint64_t *const *accepted,
                                 int64_t *n_models, uint8_t *const *models, int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    if (count < 0 || (count > 0 && (!ms || !accepted || !n_models))) {
        set_error("bad stable batch arguments (ms, accepted and n_models must be non-NULL)");
        return LP_E_INVAL;
    }
    if (count == 0) return LP_OK;
    std::vector<const Matrix *> v(count);
    for (int32_t i = 0; i < count; ++i) {
        lp_status rc = check_solvable(ms[i]);
        if (rc) return rc;
        if (ms[i]->m.K > LP_MAX_NEG_ATOMS) {
            set_error("program " + std::to_string(i) + " has too many negated atoms: " + std::to_string(ms[i]->m.K));
            return LP_E_TOO_MANY_GUESSES;
        }
        if (!accepted[i]) {
            set_error("accepted[" + std::to_string(i) + "] is NULL");
            return LP_E_INVAL;
        }
        if (ms[i]->m.dev.device != ms[0]->m.dev.device) {
            set_error("the matrices of a batch must live on one device");
            return LP_E_INVAL;
        }
        v[i] = &ms[i]->m;
    }
    DeviceGuard g(ms[0]->m.dev.device);
    return stable_batch_impl(v, accepted, n_models, models, products, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_stable_models_guesses(const lp_matrix *m, const uint64_t *guesses, int64_t n, uint64_t *accepted,
                                   int64_t *n_accepted, uint64_t *next, uint8_t *models, int64_t max_models,
                                   int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K == 0 || m->m.K > 64) {
        set_error("guess evaluation needs 1 to 64 negated atoms, the program has " + std::to_string(m->m.K));
        return m->m.K > 64 ? LP_E_TOO_MANY_GUESSES : LP_E_INVAL;
    }
    if (!guesses || n < 1 || n > (1ll << 30) || !accepted || !n_accepted || max_models < 0) {
        set_error("guesses and accepted must be non-NULL, 1 <= n <= 2^30, max_models >= 0");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return guesses_impl(m->m, guesses, n, accepted, n_accepted, next, models, max_models, products,
                        (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_stable_models_search(const lp_matrix *m, int64_t n_samples, int32_t rounds, uint64_t seed,
                                  uint64_t *found, int64_t max_found, int64_t *n_found, uint8_t *models,
                                  void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K == 0 || m->m.K > 64) {
        set_error("guess search needs 1 to 64 negated atoms, the program has " + std::to_string(m->m.K));
        return m->m.K > 64 ? LP_E_TOO_MANY_GUESSES : LP_E_INVAL;
    }
    if (n_samples < 1 || n_samples > (1ll << 30) || rounds < 1 || !n_found || max_found < 0 ||
        (max_found > 0 && !found)) {
        set_error("1 <= n_samples <= 2^30, rounds >= 1, n_found non-NULL, found non-NULL if max_found > 0");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return search_impl(m->m, n_samples, rounds, seed, found, max_found, n_found, models, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_least_model_batch(const lp_matrix *const *ms, int32_t count, uint8_t *const *models,
                               int32_t *products, const lp_schedule *sched, void *hip_stream) {
    LP_GUARD_BEGIN
    if (count < 0 || (count > 0 && (!ms || !models))) {
        set_error("bad batch arguments");
        return LP_E_INVAL;
    }
    for (int32_t i = 0; i < count; ++i)
        if (!models[i]) {
            set_error("models[" + std::to_string(i) + "] is NULL");
            return LP_E_INVAL;
        }
    if (count == 0) return LP_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    BatchPlan b;
    lp_status rc = LP_OK;
    {
        DeviceGuard g(ms[0] ? ms[0]->m.dev.device : -1);
        rc = batch_create(ms, count, sched, st, false, b);
        if (!rc) rc = batch_run(b, st);
        if (!rc) rc = batch_results(b, models, products, st);
        (void)hipStreamSynchronize(st);
        batch_release(b);
    }
    return rc;
    LP_GUARD_END
}

lp_status lp_batch_create(const lp_matrix *const *ms, int32_t count, const lp_schedule *sched, void *hip_stream,
                          lp_batch **out) {
    LP_GUARD_BEGIN
    if (!out || count < 0 || (count > 0 && !ms)) {
        set_error("bad batch arguments");
        return LP_E_INVAL;
    }
    *out = nullptr;
    lp_batch *b = new lp_batch();
    lp_status rc;
    {
        DeviceGuard g(count > 0 && ms[0] ? ms[0]->m.dev.device : -1);
        rc = batch_create(ms, count, sched, (hipStream_t)hip_stream, true, b->b);
        if (rc) {
            (void)hipStreamSynchronize((hipStream_t)hip_stream);
            batch_release(b->b);
        }
    }
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_batch_run(lp_batch *b, void *hip_stream) {
    LP_GUARD_BEGIN
    if (!b) {
        set_error("NULL batch");
        return LP_E_INVAL;
    }
    DeviceGuard g(b->b.device);
    return batch_run(b->b, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_batch_results(const lp_batch *b, uint8_t *const *models, int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    if (!b) {
        set_error("NULL batch");
        return LP_E_INVAL;
    }
    DeviceGuard g(b->b.device);
    return batch_results(b->b, models, products, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_batch_tune(lp_batch *b, int32_t reps, float *best_ms, void *hip_stream) {
    LP_GUARD_BEGIN
    if (!b || reps < 0) {
        set_error("lp_batch_tune needs a batch and reps >= 0");
        return LP_E_INVAL;
    }
    DeviceGuard g(b->b.device);
    return batch_tune(b->b, reps, best_ms, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_batch_get_info(const lp_batch *b, lp_batch_info *out) {
    LP_GUARD_BEGIN
    if (!b || !out) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    const BatchPlan &p = b->b;
    lp_batch_info I{};
    I.count = (int32_t)p.ms.size();
    I.n_resident = (int32_t)p.order.size();
    I.wpw = p.shape.wpw;
    I.unroll = p.shape.unroll;
    I.block = p.shape.block;
    I.grid = p.order.empty() ? 0 : p.shape.grid;
    I.lds_bytes = (int64_t)p.shape.lds_bytes;
    for (const Matrix *m : p.ms) {
        I.nnz += m->nnz;
        I.step_bytes += m->info.step_bytes;
    }
    I.tuned_ms = p.tuned_ms;
    I.n_teams = p.n_teams;
    for (int32_t i : p.order)
        if (p.team[i] > 1) I.team_members += p.team[i];
    I.team_fallbacks = p.team_fallbacks;
    *out = I;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_batch_free(lp_batch *b) {
    LP_GUARD_BEGIN
    if (!b) return LP_OK;
    {
        DeviceGuard g(b->b.device);
        (void)hipDeviceSynchronize();
        batch_release(b->b);
    }
    delete b;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_bench_step(const lp_matrix *m, const lp_schedule *sched, int32_t reps, float *avg_ms,
                        void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K || !avg_ms || reps < 1) {
        set_error("lp_bench_step needs a definite program, avg_ms and reps >= 1");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return bench_step_impl(m->m, sched, reps, avg_ms, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_dense_least_model(const lp_matrix *m, uint8_t *model, int32_t *products, float *kernel_ms,
                               void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K) {
        set_error("the program has negative literals; the least model is defined for definite programs");
        return LP_E_NEGATION;
    }
    if (!model && m->m.n_atoms) {
        set_error("model must be non-NULL");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return dense_least_impl(m->m, model, products, kernel_ms, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_dense_stable_models(const lp_matrix *m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                                 int64_t max_models, int32_t *products, float *kernel_ms, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K > LP_MAX_NEG_ATOMS) {
        set_error("too many negated atoms: " + std::to_string(m->m.K));
        return LP_E_TOO_MANY_GUESSES;
    }
    if (!accepted || !n_models || max_models < 0) {
        set_error("accepted and n_models must be non-NULL, max_models >= 0");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return dense_stable_impl(m->m, accepted, n_models, models, max_models, products, kernel_ms,
                             (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_bench_spmm(const lp_matrix *m, int32_t reps, float *avg_ms, int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K == 0 || m->m.K > LP_MAX_NEG_ATOMS || !avg_ms || reps < 1) {
        set_error("lp_bench_spmm needs a normal program (1 <= K <= 24), avg_ms and reps >= 1");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return bench_spmm_impl(m->m, reps, avg_ms, products, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_tune_schedule(const lp_matrix *m, int32_t reps, lp_schedule *best, float *best_step_ms,
                           float *best_solve_ms, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K || !best || reps < 1) {
        set_error("lp_tune_schedule needs a definite program, best and reps >= 1");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return tune_impl(m->m, reps, best, best_step_ms, best_solve_ms, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_schedule_cache_save(const char *path) {
    LP_GUARD_BEGIN
    if (!path || !*path) {
        set_error("NULL or empty path");
        return LP_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(g_sched_mu);
    sched_env_locked();
    return sched_save_locked(path);
    LP_GUARD_END
}

lp_status lp_schedule_cache_load(const char *path) {
    LP_GUARD_BEGIN
    if (!path || !*path) {
        set_error("NULL or empty path");
        return LP_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(g_sched_mu);
    sched_env_locked();
    return sched_load_locked(path);
    LP_GUARD_END
}

lp_status lp_schedule_cache_clear(void) {
    LP_GUARD_BEGIN
    std::lock_guard<std::mutex> lock(g_sched_mu);
    g_sched_env_done = true;  // a cleared cache stays empty until loaded or tuned
    g_sched.clear();
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_schedule_cache_lookup(const lp_matrix *m, lp_schedule *out, int32_t *found) {
    LP_GUARD_BEGIN
    if (!m || !out || !found) {
        set_error("m, out and found must be non-NULL");
        return LP_E_INVAL;
    }
    *found = 0;
    lp_status rc = check_solvable(m);  // the bucket reads the device layout's sizes
    if (rc) return rc;
    if (m->m.K) return LP_OK;  // schedules are for least models
    if (m->m.n_rows > 0 && lds_loop_fits(m->m)) {
        *found = 2;  // solved in one workgroup by the default driver: no schedule
        return LP_OK;
    }
    if (sched_lookup(m->m, out)) *found = 1;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_set_allocator(void *(*alloc)(size_t, void *, void *), void (*release)(void *, void *, void *),
                           void *ctx) {
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("alloc and release must both be set or both be NULL");
        return LP_E_INVAL;
    }
    {
        DevicePool &P = pool();
        std::lock_guard<std::mutex> lock(P.mu);
        if (P.in_use > 0 && alloc) {
            set_error("blocks of the library's own pool are live (free every matrix and plan first)");
            return LP_E_INVAL;
        }
    }
    if (g_hook_live.load() > 0 && (alloc != g_alloc || release != g_release || ctx != g_alloc_ctx)) {
        set_error(std::to_string(g_hook_live.load()) +
                  " blocks of the installed allocator are live (free every matrix and plan first)");
        return LP_E_INVAL;
    }
    g_alloc = alloc;
    g_release = release;
    g_alloc_ctx = ctx;
    return LP_OK;
}

const char *lp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
