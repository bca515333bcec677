// bwtset.cpp -- host runtime of libbwtset: handle state, device memory, the
// per-block driver of set-bwte (Algorithm 1) and the C ABI of bwtset.h.
//
// One handle owns three index buffers: the current index is only ever read
// during an append, and the blocks of the append alternate between the two
// others, so a failed append leaves the index untouched.  A workspace sized
// for the largest block holds the suffix sort, the ranks and the merge inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <thread>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <new>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/bwtset.h"
#include "bwt_internal.hpp"

using namespace bwt;

namespace {

thread_local int g_create_error = BWT_OK;
std::atomic<uint32_t> g_epoch{1};

// Every look-back launch gets a fresh epoch (30 bits, never 0).
uint32_t next_epoch() {
    uint32_t e = g_epoch.fetch_add(1) & 0x3fffffffu;
    if (e == 0) e = g_epoch.fetch_add(1) & 0x3fffffffu;
    return e;
}

// Staging of host reads streamed block by block (append_streamed): two pinned
// host slots, a copy stream and the events that order it with the compute
// stream.
struct Pipe {
    uint8_t *pinned = nullptr;       // 2 slots of slot_bytes
    uint64_t slot_bytes = 0;
    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, consumed[2] = {nullptr, nullptr};
};

void pipe_free(Pipe &p) {
    if (p.pinned) (void)hipHostFree(p.pinned);
    p.pinned = nullptr;
    p.slot_bytes = 0;
    for (auto &e : p.copied)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    for (auto &e : p.consumed)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    if (p.copy) (void)hipStreamDestroy(p.copy);
    p.copy = nullptr;
}

struct IndexBuf {
    Rec *recs = nullptr;
    uint64_t rec_cap = 0;
    uint64_t *sbc = nullptr;
    uint64_t sbc_cap = 0;
    uint64_t *meta = nullptr;
    bool host = false;   // recs and sbc in pinned host memory (the host-memory tier)
};

// Device scratch for one block of at most `cap` suffixes.
struct Workspace {
    uint64_t cap = 0;
    uint64_t *kA = nullptr, *kB = nullptr;   // sort keys (ping-pong)
    uint32_t *v[3] = {nullptr, nullptr, nullptr};  // sort values / suffix array
    uint32_t *U[2] = {nullptr, nullptr};     // unresolved SA slots
    uint32_t *rank = nullptr;                // group rank per block position
    uint64_t *g = nullptr;                   // ranks in text order
    uint64_t *gsa = nullptr;                 // second spare key buffer of the bucket finish
    uint8_t *tflag = nullptr;                // tie flag per position (bucket finish)
    uint32_t *bcnt = nullptr;                // B_int counts per 64 symbols, inside segments
    uint32_t *bseg = nullptr;                // counts before each segment, segment totals
    uint32_t *soff = nullptr;                // block position of each read
    uint32_t *tile_first = nullptr;
    uint64_t *status_radix = nullptr;        // radix look-back words
    uint64_t *status_scan = nullptr;         // scan look-back words
    uint32_t *misc = nullptr;                // counters, histograms, flags
    uint64_t *seg_list = nullptr;            // long-read segments of ComputeRanks
    uint32_t seg_cap = 0;
    uint32_t *fb_flag = nullptr, *fb_list = nullptr;
    uint32_t *bk = nullptr;                  // BK_TABLES bucket tables of bk_words each
    uint32_t bk_words = 0;
    uint8_t *region = nullptr;               // one allocation holding every array above
    uint64_t bytes = 0;                      // its size
};

// layout of Workspace::misc (uint32 words)
constexpr int MISC_CNT_RADIX = 0;
constexpr int MISC_CNT_HEADS = 1;
constexpr int MISC_NU = 4;       // followed by MISC_LARGE (read together)
constexpr int MISC_LARGE = 5;
constexpr int MISC_BAD = 6;
constexpr int MISC_ERR = 7;
constexpr int MISC_SEG = 8;      // 2 words: queued segments, fallback reads
constexpr int MISC_BK = 10;      // 3 words: tied suffixes, oversized buckets, their suffixes
constexpr int MISC_NU2 = 13;     // tied suffixes among the oversized buckets
constexpr int MISC_PILE = 14;    // 2 words: oversized buckets still to sort, their suffixes
constexpr int MISC_STATS = 16;   // running totals of ComputeRanks: segment retries, fallback
                                 // reads, then (words 18-19, 64-bit) symbols of queued reads
constexpr int BK_TABLES = 6;     // bucket starts, ends, tie counts, sizes; oversized list, offsets
constexpr uint32_t BK_PART = 3 * 4096 + 16;  // tile partials of the bucket scans
constexpr uint32_t MIN_SEG_LEN = 32;   // shortest ComputeRanks segment
constexpr int MAX_LANES = 4;
constexpr uint32_t BUCKET_TARGET = 32;  // suffixes per bucket the bucket count aims at
constexpr uint32_t BUCKET_MIN_BLOCK = 1u << 20;  // smallest block that takes the bucket finish
constexpr int MISC_HIST = 64;                 // HIST_WORDS digit counts
constexpr int MISC_WORDS = MISC_HIST + HIST_WORDS + 64;

struct Timer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Span {
        int stage;      // BWT_STAGE_* or 100+ for kernel-level spans
        hipEvent_t a, b;
        uint64_t units;
    };
    std::vector<Span> open;
    bwt_stats_t acc;
    Timer() { memset(&acc, 0, sizeof acc); }
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

enum {
    SPAN_RANKS_K = 100,
    SPAN_INSERT_K = 101,
    SPAN_RADIX_PASS = 102,
    SPAN_KEYS = 103,
    SPAN_HEADS = 104,
    SPAN_REFINE = 105,
    SPAN_BUCKET = 106,
    SPAN_RANKS_SEG = 107,
    SPAN_RANKS_FB = 108,
    SPAN_TILE_SORT = 109
};

}  // namespace

struct bwt_set {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t n = 0, m = 0;
    IndexBuf buf[3];
    int cur = 0;
    Workspace ws;
    uint64_t M = 1ull << 26;
    int key_bits = 64;               // width of the first suffix-sort key
    int radix_cfg = 3;               // radix pass tile shape (512 threads x 12 keys)
    uint32_t seg_len = 768;          // ComputeRanks segment length for long reads
    uint32_t seg_overlap = 64;       // symbols a segment walk starts past its end
    bool sort_buckets = true;        // first sort: top digits + LDS bucket finish
    bool host_index = false;         // index records and counters in pinned host memory
    bool pipeline = true;            // host reads streamed block by block (pipelined)
    Pipe *pipe = nullptr;
    uint64_t *first_new = nullptr;
    uint64_t first_new_cap = 0;
    // staging for host inputs / outputs
    uint8_t *stage_reads = nullptr;
    uint64_t stage_reads_cap = 0;
    uint64_t *stage_off = nullptr;
    uint64_t stage_off_cap = 0;
    uint64_t *cuts = nullptr;
    uint64_t cuts_cap = 0;
    uint8_t *stage_out = nullptr;
    uint64_t stage_out_cap = 0;
    // strand variants: the repacked reads and their offsets
    uint8_t *strand_reads = nullptr;
    uint64_t strand_reads_cap = 0;
    uint64_t *strand_off = nullptr;
    uint64_t strand_off_cap = 0;
    // batched form (when this handle drives a batch): device tables, staged
    // host inputs
    uint8_t *btab = nullptr;
    uint64_t btab_cap = 0;
    uint8_t *bstage = nullptr;
    uint64_t bstage_cap = 0;
    // extra lanes of a batch: internal handles used only for their stream and
    // workspace, so that independent blocks of a batch run side by side
    int batch_lanes = 2;
    std::vector<bwt_set *> lanes;
    uint64_t *res = nullptr;       // 4 words of device results
    uint64_t *pinned = nullptr;    // small pinned host area (512 words)
    int last_error = BWT_OK;
    bool broken = false;
    Timer timer;
    // captured appends (BWT_PARAM_GRAPH): executable graphs keyed by
    // everything the enqueued work depends on; `capturing` makes the block
    // path take its data-dependent decisions on the device
    bool graph = false;
    bool capturing = false;
    hipStream_t cap_stream = nullptr;
    struct GraphEntry {
        std::vector<uint64_t> key;
        hipGraphExec_t exec = nullptr;
        int src = 0;        // index buffer holding the result
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_replays = 0, graph_captures = 0, graph_redos = 0;
};

namespace {

constexpr size_t MAX_GRAPHS = 4;   // executable graphs kept per handle

void drop_graphs(bwt_set *h) {
    for (auto &g : h->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

int fail(bwt_set *h, int code) {
    if (h) {
        h->last_error = code;
        if (code == BWT_EHIP) h->broken = true;
    }
    return code;
}

#define HIPCHK(h, expr)                                                     \
    do {                                                                    \
        hipError_t _e = (expr);                                             \
        if (_e != hipSuccess) {                                             \
            if (getenv("BWTSET_DEBUG"))                                     \
                fprintf(stderr, "bwtset: %s failed: %s (%s:%d)\n", #expr,  \
                        hipGetErrorString(_e), __FILE__, __LINE__);         \
            return fail((h), BWT_EHIP);                                     \
        }                                                                   \
    } while (0)

// Bumped by every device allocation and free of the library: a captured
// append is replayed only while no buffer it names can have moved.
std::atomic<uint64_t> g_alloc_gen{1};

template <class T>
hipError_t dalloc(T **p, uint64_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    g_alloc_gen.fetch_add(1);
    return hipMalloc((void **)p, count * sizeof(T));
}

template <class T>
void dfree(T *&p) {
    if (p) {
        g_alloc_gen.fetch_add(1);
        (void)hipFree(p);
    }
    p = nullptr;
}

// Pinned host memory the GPU reads and writes directly (coherent, mapped
// into the device's address space): the host-memory tier of the index.
template <class T>
hipError_t halloc(T **p, uint64_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    g_alloc_gen.fetch_add(1);
    return hipHostMalloc((void **)p, count * sizeof(T), hipHostMallocDefault);
}

template <class T>
void hfree(T *&p) {
    if (p) {
        g_alloc_gen.fetch_add(1);
        (void)hipHostFree(p);
    }
    p = nullptr;
}

// Frees an index buffer's records and counters wherever they live.
void free_index_data(IndexBuf &b) {
    if (b.host) {
        hfree(b.recs);
        hfree(b.sbc);
    } else {
        dfree(b.recs);
        dfree(b.sbc);
    }
    b.rec_cap = b.sbc_cap = 0;
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// ---- timing ---------------------------------------------------------------
struct Scope {
    bwt_set *h;
    hipStream_t s;
    int stage;
    uint64_t units;
    hipEvent_t a = nullptr;
    Scope(bwt_set *h_, hipStream_t s_, int stage_, uint64_t units_ = 0)
        : h(h_), s(s_), stage(stage_), units(units_) {
        if (h->timer.on) {
            a = h->timer.get();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Scope() {
        if (h->timer.on && a) {
            hipEvent_t b = h->timer.get();
            if (b) {
                (void)hipEventRecord(b, s);
                h->timer.open.push_back({stage, a, b, units});
            }
        }
    }
};

// Events for the spans of a launcher that takes Marks (timing on only);
// add() turns the recorded pairs into spans once the launcher has returned.
struct MarkSet {
    bwt_set *h;
    Marks m;
    explicit MarkSet(bwt_set *h_, int spans) : h(h_) {
        if (!h->timer.on) return;
        for (int k = 0; k < spans; ++k) {
            m.a[k] = h->timer.get();
            m.b[k] = m.a[k] ? h->timer.get() : nullptr;
            if (m.a[k] && !m.b[k]) {
                h->timer.pool.push_back(m.a[k]);
                m.a[k] = nullptr;
            }
        }
    }
    const Marks *get() const { return h->timer.on ? &m : nullptr; }
    void add(int k, int stage, uint64_t units) {
        if (m.a[k] && m.b[k]) h->timer.open.push_back({stage, m.a[k], m.b[k], units});
        m.a[k] = m.b[k] = nullptr;
    }
    ~MarkSet() {  // events of spans never added go back to the pool
        for (int k = 0; k < 3; ++k) {
            if (m.a[k]) h->timer.pool.push_back(m.a[k]);
            if (m.b[k]) h->timer.pool.push_back(m.b[k]);
        }
    }
};

// Called after the stream has been synchronized.
void timer_collect(bwt_set *h) {
    Timer &T = h->timer;
    if (h->ws.misc) {
        // the device's running totals, taken and cleared
        uint32_t *pw = reinterpret_cast<uint32_t *>(h->pinned);
        if (hipMemcpyAsync(pw, h->ws.misc + MISC_STATS, 16, hipMemcpyDeviceToHost, h->stream) ==
                hipSuccess &&
            hipMemsetAsync(h->ws.misc + MISC_STATS, 0, 16, h->stream) == hipSuccess &&
            hipStreamSynchronize(h->stream) == hipSuccess) {
            T.acc.ranks_retries += pw[0];
            T.acc.ranks_fallback_reads += pw[1];
            T.acc.ranks_seg_symbols += (uint64_t)pw[2] | (uint64_t)pw[3] << 32;
        } else {
            (void)hipGetLastError();
        }
    }
    for (auto &sp : T.open) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) {
            (void)hipGetLastError();
            ms = 0.f;
        }
        if (sp.stage < BWT_NSTAGES) {
            T.acc.ms[sp.stage] += ms;
            T.acc.launches[sp.stage] += 1;
        } else if (sp.stage == SPAN_RANKS_K) {
            T.acc.ranks_kernel_ms += ms;
            T.acc.ranks_launches += 1;
            T.acc.ranks_steps += sp.units;
        } else if (sp.stage == SPAN_INSERT_K) {
            T.acc.insert_kernel_ms += ms;
            T.acc.insert_launches += 1;
        } else if (sp.stage == SPAN_RADIX_PASS) {
            T.acc.sort_pass_ms += ms;
            T.acc.sort_pass_launches += 1;
            T.acc.sort_pass_keys += sp.units;
        } else if (sp.stage == SPAN_KEYS) {
            T.acc.keys_ms += ms;
        } else if (sp.stage == SPAN_HEADS) {
            T.acc.heads_ms += ms;
        } else if (sp.stage == SPAN_REFINE) {
            T.acc.refine_ms += ms;
        } else if (sp.stage == SPAN_BUCKET) {
            T.acc.bucket_ms += ms;
        } else if (sp.stage == SPAN_RANKS_SEG) {
            T.acc.ranks_seg_ms += ms;
            T.acc.ranks_seg_launches += 1;
        } else if (sp.stage == SPAN_RANKS_FB) {
            T.acc.ranks_fb_ms += ms;
        } else if (sp.stage == SPAN_TILE_SORT) {
            T.acc.tile_sort_ms += ms;
            T.acc.tile_sort_launches += 1;
            T.acc.tile_sort_keys += sp.units;
        }
        T.pool.push_back(sp.a);
        T.pool.push_back(sp.b);
    }
    T.open.clear();
}

// ---- memory ---------------------------------------------------------------
int ensure_index(bwt_set *h, IndexBuf &b, uint64_t n) {
    uint64_t nr = records_for(n), ns = superblocks_for(n);
    if (b.host != h->host_index) {
        // the buffer moves to the tier the handle now uses
        free_index_data(b);
        b.host = h->host_index;
    }
    if (b.rec_cap < nr) {
        uint64_t cap = std::max<uint64_t>(nr, b.rec_cap + b.rec_cap / 2);
        if (b.host) hfree(b.recs);
        else dfree(b.recs);
        b.rec_cap = 0;
        if ((b.host ? halloc(&b.recs, cap) : dalloc(&b.recs, cap)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, BWT_ENOMEM);
        }
        b.rec_cap = cap;
    }
    if (b.sbc_cap < ns) {
        uint64_t cap = std::max<uint64_t>(ns, 4);
        if (b.host) hfree(b.sbc);
        else dfree(b.sbc);
        b.sbc_cap = 0;
        if ((b.host ? halloc(&b.sbc, cap * 4) : dalloc(&b.sbc, cap * 4)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, BWT_ENOMEM);
        }
        b.sbc_cap = cap;
    }
    if (!b.meta) {
        if (dalloc(&b.meta, META_WORDS) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, BWT_ENOMEM);
        }
    }
    return BWT_OK;
}

// Lays out a workspace for blocks of up to `cap` suffixes in one region at
// `base` (nullptr: sizes only) and returns the region's size.  Every array
// starts 256-byte aligned and is followed by a 4 KiB gap.
uint64_t carve_ws(Workspace &w, uint64_t cap, uint8_t *base) {
    uint64_t at = 0;
    auto take = [&](auto *&p, uint64_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
        at = (at + 255) & ~255ull;
        p = base ? reinterpret_cast<T *>(base + at) : nullptr;
        at += std::max<uint64_t>(count, 1) * sizeof(T) + 4096;
    };
    const uint64_t tiles = div_up(cap, RADIX_MIN_TILE) + 1;
    const uint64_t segs = 2 * div_up(cap, MIN_SEG_LEN) + 2;
    uint32_t nb = 256;
    while ((uint64_t)nb * BUCKET_TARGET < cap && nb < (1u << BUCKET_MAX_BITS)) nb <<= 1;
    w.bk_words = nb + 16;
    take(w.kA, cap);
    take(w.kB, cap);
    for (auto &p : w.v) take(p, cap);
    for (auto &p : w.U) take(p, cap);
    take(w.rank, cap);
    take(w.g, cap);
    take(w.gsa, cap);
    take(w.tflag, cap);
    take(w.bcnt, (div_up(cap, 64) + 2) * 4);
    take(w.bseg, (2 * (div_up(cap, 64 << BINT_SEG_SHIFT) + 2) + 1) * 4);
    take(w.soff, cap + 2);
    take(w.tile_first, div_up(cap, 1u << PREP_TILE_SHIFT) + 2);
    take(w.status_radix, tiles * 256);
    take(w.status_scan, tiles * 8);
    take(w.misc, MISC_WORDS);
    take(w.seg_list, segs);
    take(w.fb_flag, cap + 1);
    take(w.fb_list, cap + 1);
    // bucket tables, scan partials, and three words per 2048-position tile
    take(w.bk, (uint64_t)BK_TABLES * w.bk_words + BK_PART + 3 * (cap / 2048 + 2));
    w.seg_cap = (uint32_t)segs;
    w.cap = cap;
    w.region = base;
    w.bytes = at;
    return at;
}

void free_ws(Workspace &w) {
    dfree(w.region);
    w = Workspace();
}

int ensure_ws(bwt_set *h, uint64_t need) {
    Workspace &w = h->ws;
    if (w.cap >= need && w.misc) return BWT_OK;
    uint64_t cap = std::max<uint64_t>(need, w.cap + w.cap / 4);
    cap = std::min<uint64_t>(std::max<uint64_t>(cap, 4096), MAX_BLOCK + 1);
    free_ws(w);
    Workspace t;
    uint8_t *base = nullptr;
    if (dalloc(&base, carve_ws(t, cap, nullptr)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, BWT_ENOMEM);
    }
    carve_ws(w, cap, base);
    // counters start at zero; status words never need clearing (epoch tags),
    // zeroing them once makes the first launches read "not ready" cleanly
    HIPCHK(h, hipMemsetAsync(w.misc, 0, MISC_WORDS * 4, h->stream));
    const uint64_t tiles = div_up(cap, RADIX_MIN_TILE) + 1;
    HIPCHK(h, hipMemsetAsync(w.status_radix, 0, tiles * 256 * 8, h->stream));
    HIPCHK(h, hipMemsetAsync(w.status_scan, 0, tiles * 8 * 8, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return BWT_OK;
}

template <class T>
int ensure_buf(bwt_set *h, T *&p, uint64_t &cap, uint64_t need) {
    if (cap >= need && p) return BWT_OK;
    uint64_t c = std::max<uint64_t>(need, cap + cap / 2);
    dfree(p);
    cap = 0;
    if (dalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, BWT_ENOMEM);
    }
    cap = c;
    return BWT_OK;
}

int bits_for(uint64_t v) {  // bits needed to hold values < v (at least 1)
    int b = 1;
    while (b < 63 && (1ull << b) < v) ++b;
    return b;
}

// ---- radix sort -------------------------------------------------------------
// Sorts (kin, vin) by bits shift0 .. bits-1 of the keys, ping-ponging with
// (kalt, valt); returns via *ko / *vo where the sorted data ended up.  When
// counted0 is set, the producer of the keys already left the counts of their
// low digit in the first 256 histogram words.
int radix_sort(bwt_set *h, hipStream_t s, uint64_t *kin, uint32_t *vin, uint64_t *kalt,
               uint32_t *valt, uint64_t n, int bits, bool counted0, uint64_t **ko,
               uint32_t **vo, int shift0 = 0) {
    Workspace &w = h->ws;
    const int npass = bits - shift0 < 1 ? 1 : (bits - shift0 + 7) / 8;
    *ko = kin;
    *vo = vin;
    if (n <= 1) return BWT_OK;
    uint32_t *hist = w.misc + MISC_HIST;
    const uint32_t per_pass = HIST_COPIES * 256;
    if (!counted0) HIPCHK(h, launch_radix_hist1(kin, n, shift0, hist, s));
    if (npass > 1) HIPCHK(h, launch_zero_u32(hist + per_pass, per_pass * (npass - 1), s));
    uint64_t *ka = kin, *kb = kalt;
    uint32_t *va = vin, *vb = valt;
    for (int p = 0; p < npass; ++p) {
        {
            Scope sc(h, s, SPAN_RADIX_PASS, n);
            HIPCHK(h, launch_radix_pass(ka, va, kb, vb, n, shift0 + 8 * p, hist + per_pass * p,
                                        p + 1 < npass ? hist + per_pass * (p + 1) : nullptr,
                                        shift0 + 8 * (p + 1), w.status_radix, w.misc + MISC_CNT_RADIX,
                                        next_epoch(), w.misc + MISC_ERR, h->radix_cfg, s));
        }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *ko = ka;
    *vo = va;
    return BWT_OK;
}

int read_u32(bwt_set *h, hipStream_t s, const uint32_t *dptr, uint32_t *out) {
    HIPCHK(h, hipMemcpyAsync(h->pinned, dptr, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    *out = *reinterpret_cast<uint32_t *>(h->pinned);
    return BWT_OK;
}

// Clears the device consistency word (before a call that launches kernels).
int clear_err(bwt_set *h, hipStream_t s) {
    HIPCHK(h, hipMemsetAsync(h->ws.misc + MISC_ERR, 0, 4, s));
    return BWT_OK;
}

// After the stream is synchronized: a nonzero consistency word means a kernel
// met an impossible state; the call fails and the tile counters are reset.
int check_err(bwt_set *h, hipStream_t s) {
    uint32_t e = 0;
    int rc = read_u32(h, s, h->ws.misc + MISC_ERR, &e);
    if (rc) return rc;
    if (e) {
        if (getenv("BWTSET_DEBUG")) fprintf(stderr, "bwtset: device check failed: 0x%x\n", e);
        HIPCHK(h, hipMemsetAsync(h->ws.misc, 0, MISC_HIST * 4, s));
        HIPCHK(h, hipStreamSynchronize(s));
        h->last_error = BWT_EHIP;
        return BWT_EHIP;
    }
    return BWT_OK;
}

// Long-read segments for ComputeRanks; none when no read of the input is
// longer than a segment (the segment kernels would find an empty queue).
RankSegments rank_segments(bwt_set *h, uint64_t maxlen) {
    RankSegments sg;
    Workspace &w = h->ws;
    sg.seg_len = maxlen > h->seg_len ? h->seg_len : 0;
    sg.overlap = h->seg_overlap;
    sg.seg_list = w.seg_list;
    sg.seg_cap = w.seg_cap;
    sg.fb_flag = w.fb_flag;
    sg.fb_list = w.fb_list;
    sg.counters = w.misc + MISC_SEG;
    sg.stats = w.misc + MISC_STATS;
    return sg;
}

// ---- ConstructSA of one block --------------------------------------------
// soff (block position of each read) and the read-lookup tiles of a block.
int block_prep(bwt_set *h, hipStream_t s, const uint64_t *off, uint32_t m_blk, uint32_t n_blk) {
    Workspace &w = h->ws;
    HIPCHK(h, launch_block_soff(off, m_blk, w.soff, s));
    HIPCHK(h, launch_block_tile_first(w.soff, m_blk, n_blk, w.tile_first, s));
    return BWT_OK;
}

// Finishes a first sort whose radix passes covered only the top digits:
// buckets of up to BUCKET_CAP suffixes are sorted by one wave each, larger
// ones are gathered and radix-sorted on the whole key, all of them into the
// other key / value pair, where ks / vs point on return; the tied suffixes of
// both end up in U[0] (count in *nU, *large for a group above REFINE_LIMIT).
int bucket_finish(bwt_set *h, hipStream_t s, uint64_t *&ks, uint32_t *&vs, uint32_t n,
                  int sort_bits, int B, int kfirst, uint32_t *nU, bool *large) {
    Workspace &w = h->ws;
    const uint32_t nb = 1u << B;
    const int bshift = sort_bits - B;
    const uint32_t W = w.bk_words;
    uint32_t *bstart = w.bk, *obad = w.bk + W, *tcnt = w.bk + 2 * W, *osz = w.bk + 3 * W,
             *olist = w.bk + 4 * W, *ooff = w.bk + 5 * W, *part = w.bk + 6 * W,
             *trange = part + BK_PART;
    uint32_t *err = w.misc + MISC_ERR, *res = w.misc + MISC_BK;
    uint32_t *const olist2 = tcnt, *const ooff2 = osz;
    // the radix passes left (ks, vs) in one of the (kA, v[0]) / (kB, v[1])
    // pairs; the sorted buckets go to the other pair
    if ((ks != w.kA && ks != w.kB) || (vs != w.v[0] && vs != w.v[1])) return fail(h, BWT_EHIP);
    uint64_t *const kx = ks, *const ky = ks == w.kA ? w.kB : w.kA;
    uint32_t *const vx = vs, *const vy = vs == w.v[0] ? w.v[1] : w.v[0];
    ks = ky;
    vs = vy;
    HIPCHK(h, launch_zero_u32(w.misc + MISC_NU, 2, s));  // tied count, large flag
    {
        Scope sk(h, s, SPAN_BUCKET);
        MarkSet mk(h, 1);
        HIPCHK(h, launch_bucket_sort(kx, vx, ky, vy, n, bstart, trange, nb, bshift, kfirst,
                                     REFINE_LIMIT, w.misc + MISC_LARGE, tcnt, osz, w.tflag, part,
                                     res, olist, ooff, obad, err, s, mk.get()));
        mk.add(0, SPAN_TILE_SORT, n);
        // The tied suffixes go to U; beside that, every oversized bucket is
        // copied to the sorted pair, and those that hold copies of one
        // settled key (the short suffixes of the later blocks: every read's
        // "$", every "A$", ...) are already final there.  The tables of tie
        // counts and sizes are free by then and list the others.
        HIPCHK(h, launch_emit_and_check(w.tflag, n, trange, tcnt, nb, w.U[0], n, kx, vx, ky, vy,
                                        bstart, olist, ooff, res, kfirst, obad, olist2, ooff2,
                                        w.misc + MISC_PILE, err, s));
    }
    // one read of the counts: tied suffixes, large flag, oversized buckets
    // and those still to sort
    const uint32_t *pw = reinterpret_cast<const uint32_t *>(h->pinned);
    HIPCHK(h, hipMemcpyAsync(h->pinned, w.misc + MISC_NU, (MISC_PILE + 2 - MISC_NU) * 4,
                             hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    const uint32_t tied = pw[MISC_BK - MISC_NU];
    uint32_t nob = pw[MISC_BK + 1 - MISC_NU], no = pw[MISC_BK + 2 - MISC_NU];
    *nU = tied;
    *large = pw[MISC_LARGE - MISC_NU] != 0;
    if (no == 0) return BWT_OK;
    if (no > n || nob == 0 || nob > nb || tied > n) return fail(h, BWT_EHIP);
    nob = pw[MISC_PILE - MISC_NU];
    no = pw[MISC_PILE + 1 - MISC_NU];
    if (no == 0) return BWT_OK;
    if (no > n || nob == 0 || nob > nb) return fail(h, BWT_EHIP);
    olist = olist2;
    ooff = ooff2;
    // the oversized buckets are sorted in two key and two value buffers that
    // hold neither the sorted block nor g (the doubling fallback may build the
    // keys from g again): the spare pair and the radix output, which is free
    // once they are gathered
    uint64_t *kf[2] = {w.gsa, kx};
    uint32_t *vf[2] = {w.v[2], vx};
    HIPCHK(h, launch_oversize_gather(kx, vx, bstart, olist, ooff, nob, no, n, kf[0], vf[0], err, s));
    uint64_t *ck;
    uint32_t *cv;
    int rc = radix_sort(h, s, kf[0], vf[0], kf[1], vf[1], no, sort_bits, false, &ck, &cv);
    if (rc) return rc;
    {
        Scope sk(h, s, SPAN_BUCKET);
        HIPCHK(h, launch_oversize_scatter(ck, cv, no, bstart, olist, ooff, nob, n, ky, vy, err, s));
        HIPCHK(h, launch_group_heads(ck, cv, nullptr, no, kfirst, cv, nullptr, w.U[1],
                                     w.misc + MISC_NU2, REFINE_LIMIT, w.misc + MISC_LARGE,
                                     w.status_scan, w.misc + MISC_CNT_HEADS, next_epoch(), err, s));
        HIPCHK(h, launch_oversize_ties_map(w.U[1], w.misc + MISC_NU2, bstart, olist, ooff, nob, no,
                                           tied, n, w.U[0], w.misc + MISC_NU, err, s));
    }
    HIPCHK(h, hipMemcpyAsync(h->pinned, w.misc + MISC_NU, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    *nU = pw[0];
    *large = pw[1] != 0;
    return BWT_OK;
}

// Layout of a block's first sort key for gbits bits of g (see bwt_internal.hpp),
// and the digits its radix passes cover: with the bucket finish only the top
// digits, B bucket bits, enough for about BUCKET_TARGET suffixes per bucket
// (small blocks are latency-bound: fewer launches and host reads win there);
// shift0 is the first pass's digit.
struct KeyLayout {
    int key_bits, kfirst, gshift, sort_bits;
    bool buckets;
    int B, shift0;
};

KeyLayout key_layout(const bwt_set *h, int gbits, uint32_t n_blk) {
    KeyLayout L;
    L.key_bits = h->key_bits < gbits + 1 ? gbits + 1 : h->key_bits;
    if (L.key_bits > 64) L.key_bits = 64;
    L.kfirst = first_key_syms(gbits, L.key_bits);
    L.gshift = gbits ? L.key_bits - gbits : 64;
    L.sort_bits = gbits ? L.key_bits : 2 * L.kfirst + KEY_LEN_BITS;
    L.buckets = h->sort_buckets && !h->capturing && n_blk >= BUCKET_MIN_BLOCK;
    L.B = 0;
    L.shift0 = 0;
    if (L.buckets) {
        int B = 1;
        while (B < BUCKET_MAX_BITS && ((uint64_t)BUCKET_TARGET << B) < n_blk &&
               (2ull << B) + 16 <= h->ws.bk_words)
            ++B;
        if (B > L.sort_bits) B = L.sort_bits;
        L.B = B;
        L.shift0 = L.sort_bits - 8 * ((B + 7) / 8);
        if (L.shift0 < 0) L.shift0 = 0;
    }
    return L;
}

// The keys ComputeRanks writes for a block (g leading), with the counts of
// the first radix pass's digit.
RankKeys rank_keys(bwt_set *h, hipStream_t s, int gbits, uint32_t n_blk, int *rc) {
    Workspace &w = h->ws;
    const KeyLayout KL = key_layout(h, gbits, n_blk);
    uint32_t *hist = w.misc + MISC_HIST;
    *rc = launch_zero_u32(hist, HIST_COPIES * 256, s) == hipSuccess ? BWT_OK : BWT_EHIP;
    return RankKeys{w.kA, w.v[0], KL.gshift, KL.kfirst, hist, KL.shift0};
}

// Suffix array of one block (after block_prep).  reads/off: device; off
// points at the block's first read (m_blk + 1 entries).  g (text order, may
// be null when gbits == 0) leads the first sort key.  On return *sa_out holds
// the suffix array (values carry the preceding symbol in bits 29..31) and
// *gkeys_out / *gshift_out give g_sa per SA slot (g_sa = key >> gshift).
int block_sort(bwt_set *h, hipStream_t s, const uint8_t *reads, const uint64_t *off,
               uint32_t m_blk, uint32_t n_blk, uint64_t maxlen, uint64_t *g, int gbits,
               bool keys_ready, uint32_t **sa_out, const uint64_t **gkeys_out, int *gshift_out) {
    (void)m_blk;
    Workspace &w = h->ws;
    Scope sc(h, s, BWT_STAGE_SORT);
    const KeyLayout KL = key_layout(h, gbits, n_blk);
    int key_bits = KL.key_bits;
    int kfirst = KL.kfirst;
    int gshift = KL.gshift;
    const int sort_bits = KL.sort_bits;
    uint32_t *hist = w.misc + MISC_HIST;
    const bool buckets = KL.buckets;
    const int B = KL.B, shift0 = KL.shift0;
    if (!keys_ready) {
        HIPCHK(h, launch_zero_u32(hist, HIST_COPIES * 256, s));
        Scope sk(h, s, SPAN_KEYS);
        HIPCHK(h, launch_block_keys(reads, off, w.soff, w.tile_first, n_blk, gbits ? g : nullptr,
                                    gshift, kfirst, shift0, w.kA, w.v[0], hist, s));
    }
    uint64_t *ks;
    uint32_t *vs;
    // the key producer (ComputeRanks or the key build) counted the first digit
    int rc = radix_sort(h, s, w.kA, w.v[0], w.kB, w.v[1], n_blk, sort_bits, true, &ks, &vs,
                        shift0);
    if (rc) return rc;
    uint32_t *sa = vs;
    *sa_out = sa;
    *gkeys_out = ks;
    *gshift_out = gshift;
    uint32_t nU = 0;
    bool large = false;
    if (buckets) {
        if ((rc = bucket_finish(h, s, ks, vs, n_blk, sort_bits, B, kfirst, &nU, &large))) return rc;
        sa = vs;
        *sa_out = sa;
        *gkeys_out = ks;
    } else {
        HIPCHK(h, launch_zero_u32(w.misc + MISC_LARGE, 1, s));
        {
            Scope sk(h, s, SPAN_HEADS);
            HIPCHK(h, launch_group_heads(ks, vs, nullptr, n_blk, kfirst, sa, nullptr, w.U[0],
                                         w.misc + MISC_NU, REFINE_LIMIT, w.misc + MISC_LARGE,
                                         w.status_scan, w.misc + MISC_CNT_HEADS, next_epoch(),
                                         w.misc + MISC_ERR, s));
        }
        if (h->capturing) {
            // the tied count stays on the device: a persistent refinement
            // reads it there; a group too large for it flags the call for a
            // run that decides on the host (prefix doubling)
            const uint32_t max_iter = (uint32_t)(maxlen / KEY_K + 2);
            HIPCHK(h, launch_refine_dev(reads, off, w.soff, w.tile_first, ks, w.U[0],
                                        w.misc + MISC_NU, w.misc + MISC_LARGE, n_blk, sa, kfirst,
                                        max_iter, w.misc + MISC_ERR, s));
            return BWT_OK;
        }
        HIPCHK(h, hipMemcpyAsync(h->pinned, w.misc + MISC_NU, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        nU = reinterpret_cast<uint32_t *>(h->pinned)[0];
        large = reinterpret_cast<uint32_t *>(h->pinned)[1] != 0;
    }
    h->timer.acc.tied_suffixes += nU;
    if (nU == 0) return BWT_OK;
    if (!large) {
        // every tied group is small: finish them in LDS by chunk keys
        const uint32_t max_iter = (uint32_t)(maxlen / KEY_K + 2);
        Scope sk(h, s, SPAN_REFINE);
        HIPCHK(h, launch_refine(reads, off, w.soff, w.tile_first, ks, w.U[0], nU, sa, kfirst,
                                max_iter, w.misc + MISC_ERR, s));
        return BWT_OK;
    }
    // A tied group too large for LDS: prefix doubling over all tied
    // suffixes, from a first key with as many symbols as fit in 64 bits (a
    // doubling round needs the tied suffixes to share at least one symbol).
    // The doubling sorts reuse both key buffers, so g_sa moves to w.g first.
    h->timer.acc.fallback_blocks += 1;
    const int gshift_first = gshift;
    if (key_bits < 64 || kfirst < 1) {
        key_bits = 64;
        kfirst = first_key_syms(gbits, key_bits);
        gshift = gbits ? key_bits - gbits : 64;
        if (kfirst < 1) return fail(h, BWT_EHIP);
        // keys built by ComputeRanks left no g array: take g back from the keys
        if (keys_ready && gbits) HIPCHK(h, launch_scatter_g(ks, vs, n_blk, gshift_first, g, s));
        HIPCHK(h, launch_zero_u32(hist, HIST_COPIES * 256, s));
        HIPCHK(h, launch_block_keys(reads, off, w.soff, w.tile_first, n_blk, gbits ? g : nullptr,
                                    gshift, kfirst, 0, w.kA, w.v[0], hist, s));
        rc = radix_sort(h, s, w.kA, w.v[0], w.kB, w.v[1], n_blk, 64, true, &ks, &vs);
        if (rc) return rc;
        sa = vs;
        *sa_out = sa;
        *gshift_out = gshift;
    }
    HIPCHK(h, hipMemcpyAsync(w.g, ks, (uint64_t)n_blk * 8, hipMemcpyDeviceToDevice, s));
    *gkeys_out = w.g;
    uint32_t *spare[2];
    {
        int k = 0;
        for (auto *p : w.v)
            if (p != sa) spare[k++] = p;
    }
    int ui = 0;
    HIPCHK(h, launch_group_heads(ks, vs, nullptr, n_blk, kfirst, sa, w.rank, w.U[ui],
                                 w.misc + MISC_NU, 0xffffffffu, w.misc + MISC_LARGE,
                                 w.status_scan, w.misc + MISC_CNT_HEADS, next_epoch(),
                                 w.misc + MISC_ERR, s));
    if ((rc = read_u32(h, s, w.misc + MISC_NU, &nU))) return rc;
    const int rbits = bits_for(n_blk);
    uint32_t hlen = (uint32_t)kfirst;
    int rounds = 0;
    while (nU > 0) {
        // h doubles every round and no suffix is longer than a block
        if (++rounds > 40 || hlen > n_blk) return fail(h, BWT_EHIP);
        h->timer.acc.doubling_rounds += 1;
        HIPCHK(h, launch_doubling_keys(w.U[ui], nU, sa, w.rank, hlen, rbits, n_blk, w.kA,
                                       spare[0], w.misc + MISC_ERR, s));
        rc = radix_sort(h, s, w.kA, spare[0], w.kB, spare[1], nU, 2 * rbits, false, &ks, &vs);
        if (rc) return rc;
        HIPCHK(h, launch_group_heads(ks, vs, w.U[ui], nU, 0, sa, w.rank, w.U[ui ^ 1],
                                     w.misc + MISC_NU, 0xffffffffu, w.misc + MISC_LARGE,
                                     w.status_scan, w.misc + MISC_CNT_HEADS, next_epoch(),
                                     w.misc + MISC_ERR, s));
        ui ^= 1;
        if ((rc = read_u32(h, s, w.misc + MISC_NU, &nU))) return rc;
        hlen *= 2;
    }
    return BWT_OK;
}

// ---- Insert ------------------------------------------------------------------
// Merges the n_new sorted block symbols (gkeys/gbits give g_sa, vals the
// symbol codes; m_new of them terminators, when known, for the statistics)
// into src, writing dst.
int insert_block(bwt_set *h, hipStream_t s, const IndexBuf &src, IndexBuf &dst, uint64_t n_ext,
                 const uint64_t *gkeys, int gshift, const uint32_t *vals, uint64_t n_new,
                 uint64_t m_new) {
    Workspace &w = h->ws;
    const uint64_t n_out = n_ext + n_new;
    const uint64_t ntiles = div_up(records_for(n_out), INS_TILE_RECS);
    int rc = ensure_buf(h, h->first_new, h->first_new_cap, ntiles + 2);
    if (rc) return rc;
    Scope sc(h, s, BWT_STAGE_INSERT);
    const BintCounts bc{w.bcnt, w.bseg};
    HIPCHK(h, launch_count_bint(vals, (uint32_t)n_new, w.bcnt, w.bseg, s));
    HIPCHK(h, launch_ins_tile_first(gkeys, gshift, n_new, ntiles, h->first_new, s));
    HIPCHK(h, launch_ins_meta(src.recs, src.sbc, src.meta, gkeys, gshift, vals, bc, n_new,
                              dst.sbc, dst.meta, s));
    {
        Scope sk(h, s, SPAN_INSERT_K);
        HIPCHK(h, launch_insert(src.recs, src.sbc, n_ext, gkeys, gshift, vals, bc, n_new,
                                h->first_new, dst.recs, dst.sbc, w.misc + MISC_ERR, s));
    }
    if (h->timer.on) {
        h->timer.acc.insert_records_out += records_for(n_out);
        h->timer.acc.insert_records_in += records_for(n_ext);
        h->timer.acc.insert_new_symbols += n_new;
        h->timer.acc.insert_old_symbols += n_ext;
        h->timer.acc.insert_terminators += m_new;
    }
    return BWT_OK;
}

// ---- input planning -----------------------------------------------------------
struct Plan {
    const uint8_t *reads = nullptr;   // device (null: host reads left in place)
    const uint64_t *off = nullptr;    // device, m + 1 entries (null with host reads left)
    std::vector<uint64_t> cut_j;      // block boundaries (read indices), K + 1
    std::vector<uint64_t> cut_s;      // block-text position S(j) of each boundary
    uint64_t total_suffixes = 0;
    uint64_t maxlen = 0;              // longest read
    const uint8_t *host_reads = nullptr;  // host reads left in place (stream_host)
    std::vector<uint64_t> hoff;       // their offsets, on the host
};

// stream_host: host reads are not copied here (the caller streams them to
// the device block by block); the plan then keeps the host offsets.
int plan_input(bwt_set *h, hipStream_t s, const uint8_t *reads, const uint64_t *offsets,
               uint64_t m, uint64_t M, Plan &P, bool stream_host = false) {
    const bool off_dev = is_device_ptr(offsets);
    const bool reads_dev = is_device_ptr(reads);
    std::vector<uint64_t> hoff;
    if (!off_dev || !reads_dev) {
        // bring the offsets to the host and plan there
        hoff.resize(m + 1);
        if (off_dev) {
            HIPCHK(h, hipMemcpyAsync(hoff.data(), offsets, (m + 1) * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
        } else {
            memcpy(hoff.data(), offsets, (m + 1) * 8);
        }
        uint64_t maxlen = 0;
        for (uint64_t j = 0; j < m; ++j) {
            if (hoff[j + 1] < hoff[j]) return fail(h, BWT_EINVAL);
            maxlen = std::max(maxlen, hoff[j + 1] - hoff[j]);
        }
        if (maxlen > MAX_READ) return fail(h, BWT_EINVAL);
        P.maxlen = maxlen;
        const uint64_t o0 = hoff[0];
        P.cut_j.assign(1, 0);
        P.cut_s.assign(1, 0);
        uint64_t j = 0;
        while (j < m) {
            uint64_t Sj = hoff[j] - o0 + j, k = j + 1;
            // largest k with S(k) - S(j) <= M (at least j + 1)
            uint64_t lo = j + 1, hi = m;
            while (lo < hi) {
                uint64_t mid = lo + (hi - lo + 1) / 2;
                if (hoff[mid] - o0 + mid - Sj <= M) lo = mid;
                else hi = mid - 1;
            }
            k = lo;
            P.cut_j.push_back(k);
            P.cut_s.push_back(hoff[k] - o0 + k);
            j = k;
        }
        P.total_suffixes = hoff[m] - o0 + m;
        if (stream_host && !reads_dev) {
            P.host_reads = reads;
            P.hoff = std::move(hoff);
            return BWT_OK;
        }
        // device copies
        uint64_t base_sym = o0 & ~3ull;
        if (!reads_dev) {
            uint64_t nbytes = (hoff[m] + 3) / 4 - base_sym / 4;
            int rc = ensure_buf(h, h->stage_reads, h->stage_reads_cap, nbytes + 16);
            if (rc) return rc;
            HIPCHK(h, hipMemcpyAsync(h->stage_reads, reads + base_sym / 4, nbytes,
                                     hipMemcpyHostToDevice, s));
            for (auto &x : hoff) x -= base_sym;
            P.reads = h->stage_reads;
        } else {
            P.reads = reads;
        }
        int rc = ensure_buf(h, h->stage_off, h->stage_off_cap, m + 1);
        if (rc) return rc;
        HIPCHK(h, hipMemcpyAsync(h->stage_off, hoff.data(), (m + 1) * 8, hipMemcpyHostToDevice, s));
        // the host vector must outlive the copy
        HIPCHK(h, hipStreamSynchronize(s));
        P.off = h->stage_off;
        return BWT_OK;
    }
    // both on the device: check and split there, read back only the cuts
    HIPCHK(h, launch_check_offsets(offsets, m, h->res, s));
    int rc = ensure_buf(h, h->cuts, h->cuts_cap, 2 * (m + 1) + 2);
    if (rc) return rc;
    HIPCHK(h, launch_plan_blocks(offsets, m, M, h->cuts, h->res, s));
    HIPCHK(h, hipMemcpyAsync(h->pinned, h->res, 4 * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    uint64_t bad = h->pinned[0], maxlen = h->pinned[1], K = h->pinned[2];
    if (bad || maxlen > MAX_READ) return fail(h, BWT_EINVAL);
    P.maxlen = maxlen;
    std::vector<uint64_t> cuts(2 * (K + 1));
    HIPCHK(h, hipMemcpyAsync(cuts.data(), h->cuts, cuts.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    P.cut_j.resize(K + 1);
    P.cut_s.resize(K + 1);
    for (uint64_t k = 0; k <= K; ++k) {
        P.cut_j[k] = cuts[2 * k];
        P.cut_s[k] = cuts[2 * k + 1];
    }
    P.total_suffixes = P.cut_s[K];
    P.reads = reads;
    P.off = offsets;
    return BWT_OK;
}

uint64_t max_block(const Plan &P) {
    uint64_t mb = 0;
    for (size_t k = 0; k + 1 < P.cut_s.size(); ++k) mb = std::max(mb, P.cut_s[k + 1] - P.cut_s[k]);
    return mb;
}

int set_device(bwt_set *h) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, BWT_EHIP);
    }
    if (d != h->device) HIPCHK(h, hipSetDevice(h->device));
    return BWT_OK;
}

// ---- batched form ---------------------------------------------------------------
// One unit = one block of one set (Algorithm 1 blocks, cut per set).  Units
// are scheduled level by level (every set's first block, then every set's
// second block, ...) and packed greedily into device blocks of at most M
// suffixes; a new device block starts with each level, so a set's block k
// always runs after its block k-1 has been merged.
struct HostUnit {
    uint32_t set;        // position in the batch
    uint32_t level;      // block index within the set
    uint64_t j0, j1;     // reads of the set
    uint64_t nsuf, nsym;
    uint64_t dst_read0, dst_sym0;
    uint64_t n_ext;      // the set's index size before this unit
    int src, dst;        // index buffers of the set read and written
};

struct DevBlock {
    uint32_t u0, u1;     // units [u0, u1)
    uint64_t read0, m_blk, n_blk;
    uint64_t gtotal;     // sum of (n_ext + 1) over the units
    uint64_t ntiles;     // Insert tiles over all units
    size_t rank_off, ins_off;  // byte offsets of the unit tables in btab
};

// Read-only inputs shared by the blocks of a batch.
struct BatchInput {
    const uint8_t *reads;      // staged packed reads
    const uint64_t *off;       // staged offsets
    const uint8_t *tab;        // device unit tables
    uint64_t maxlen;
};

// One device block of a batch on lane L (its workspace) and stream s.
int run_block(bwt_set *L, hipStream_t s, const DevBlock &B, const std::vector<HostUnit> &units,
              const BatchInput &in) {
    Workspace &w = L->ws;
    const uint32_t nu = B.u1 - B.u0;
    const uint32_t m_blk = (uint32_t)B.m_blk, n_blk = (uint32_t)B.n_blk;
    const uint64_t *off = in.off + B.read0;
    const RankUnit *rdev = reinterpret_cast<const RankUnit *>(in.tab + B.rank_off);
    const InsertUnit *idev = reinterpret_cast<const InsertUnit *>(in.tab + B.ins_off);
    int rc;
    if ((rc = block_prep(L, s, off, m_blk, n_blk))) return rc;
    // one empty unit alone needs no ranks (all 0); otherwise the ranks
    // carry the unit offsets
    const int gbits = bits_for_value(B.gtotal - 1);
    if (gbits > 0) {
        Scope sc(L, s, BWT_STAGE_RANKS);
        const RankKeys kk = rank_keys(L, s, gbits, n_blk, &rc);
        if (rc) return fail(L, rc);
        MarkSet mk(L, 3);
        HIPCHK(L, launch_compute_ranks_units(in.reads, off, w.soff, m_blk, n_blk, rdev, nu, w.g,
                                             &kk, rank_segments(L, in.maxlen), w.misc + MISC_ERR, s,
                                             mk.get()));
        mk.add(0, SPAN_RANKS_K, n_blk - m_blk);
        mk.add(1, SPAN_RANKS_SEG, 0);
        mk.add(2, SPAN_RANKS_FB, 0);
    }
    uint32_t *sa = nullptr;
    const uint64_t *gkeys = nullptr;
    int gshift = 64;
    if ((rc = block_sort(L, s, in.reads, off, m_blk, n_blk, in.maxlen, w.g, gbits, gbits > 0, &sa,
                         &gkeys,
                         &gshift)))
        return rc;
    {
        Scope sc(L, s, BWT_STAGE_INSERT);
        const BintCounts bc{w.bcnt, w.bseg};
        HIPCHK(L, launch_count_bint(sa, n_blk, w.bcnt, w.bseg, s));
        HIPCHK(L, launch_ins_tile_first_units(idev, nu, gkeys, gshift, B.ntiles, L->first_new, s));
        HIPCHK(L, launch_ins_meta_units(idev, nu, gkeys, gshift, sa, bc, s));
        Scope sk(L, s, SPAN_INSERT_K);
        HIPCHK(L, launch_insert_units(idev, nu, gkeys, gshift, sa, bc, L->first_new, B.ntiles,
                                      w.misc + MISC_ERR, s));
    }
    if (L->timer.on) {
        for (uint32_t k = B.u0; k < B.u1; ++k) {
            L->timer.acc.insert_records_out += records_for(units[k].n_ext + units[k].nsuf);
            L->timer.acc.insert_records_in += records_for(units[k].n_ext);
            L->timer.acc.insert_old_symbols += units[k].n_ext;
        }
        L->timer.acc.insert_new_symbols += n_blk;
        L->timer.acc.insert_terminators += m_blk;
    }
    L->timer.acc.blocks += 1;
    return BWT_OK;
}

void stats_add(bwt_stats_t &a, const bwt_stats_t &b) {
    for (int k = 0; k < BWT_NSTAGES; ++k) {
        a.ms[k] += b.ms[k];
        a.launches[k] += b.launches[k];
    }
    a.ranks_kernel_ms += b.ranks_kernel_ms;
    a.ranks_launches += b.ranks_launches;
    a.ranks_steps += b.ranks_steps;
    a.insert_kernel_ms += b.insert_kernel_ms;
    a.insert_launches += b.insert_launches;
    a.insert_records_out += b.insert_records_out;
    a.insert_records_in += b.insert_records_in;
    a.insert_new_symbols += b.insert_new_symbols;
    a.sort_pass_ms += b.sort_pass_ms;
    a.sort_pass_launches += b.sort_pass_launches;
    a.sort_pass_keys += b.sort_pass_keys;
    a.blocks += b.blocks;
    a.doubling_rounds += b.doubling_rounds;
    a.keys_ms += b.keys_ms;
    a.heads_ms += b.heads_ms;
    a.refine_ms += b.refine_ms;
    a.bucket_ms += b.bucket_ms;
    a.tied_suffixes += b.tied_suffixes;
    a.fallback_blocks += b.fallback_blocks;
    a.ranks_seg_ms += b.ranks_seg_ms;
    a.ranks_seg_launches += b.ranks_seg_launches;
    a.ranks_fb_ms += b.ranks_fb_ms;
    a.tile_sort_ms += b.tile_sort_ms;
    a.tile_sort_launches += b.tile_sort_launches;
    a.tile_sort_keys += b.tile_sort_keys;
    a.insert_old_symbols += b.insert_old_symbols;
    a.insert_terminators += b.insert_terminators;
    a.ranks_retries += b.ranks_retries;
    a.ranks_fallback_reads += b.ranks_fallback_reads;
    a.ranks_seg_symbols += b.ranks_seg_symbols;
}

template <class T>
size_t put_table(std::vector<uint8_t> &tab, const std::vector<T> &v) {
    size_t at = (tab.size() + 255) & ~(size_t)255;
    tab.resize(at + v.size() * sizeof(T));
    if (!v.empty()) memcpy(tab.data() + at, v.data(), v.size() * sizeof(T));
    return at;
}

int append_many(bwt_set *d, bwt_set **hs, const uint8_t *const *reads,
                const uint64_t *const *offsets, const uint64_t *m, uint64_t count, hipStream_t s) {
    std::vector<uint32_t> act;
    for (uint64_t i = 0; i < count; ++i) {
        if (m[i] == 0) continue;
        if (!reads[i] || !offsets[i]) return fail(d, BWT_EINVAL);
        act.push_back((uint32_t)i);
    }
    if (act.empty()) return BWT_OK;
    const uint32_t na = (uint32_t)act.size();

    // 1. device copies of host inputs.  Host offsets are checked for order
    // here (their byte range depends on it); device offsets on the device.
    std::vector<const uint8_t *> dreads(na);
    std::vector<const uint64_t *> doff(na);
    std::vector<uint64_t> sym_base(na, 0);
    std::vector<uint64_t> stage_need(na, 0);
    std::vector<uint64_t> first_last(2 * na, 0);
    std::vector<bool> rdev(na), odev(na);
    uint64_t stage_total = 0;
    bool need_ends = false;
    for (uint32_t a = 0; a < na; ++a) {
        const uint32_t i = act[a];
        rdev[a] = is_device_ptr(reads[i]);
        odev[a] = is_device_ptr(offsets[i]);
        if (!odev[a]) {
            for (uint64_t j = 0; j < m[i]; ++j)
                if (offsets[i][j + 1] < offsets[i][j]) return fail(d, BWT_EINVAL);
            first_last[2 * a] = offsets[i][0];
            first_last[2 * a + 1] = offsets[i][m[i]];
            stage_total += ((m[i] + 1) * 8 + 255) & ~255ull;
        } else if (!rdev[a]) {
            need_ends = true;
        }
    }
    if (need_ends) {
        // host reads with device offsets: the byte range comes from the device
        for (uint32_t a = 0; a < na; ++a) {
            if (rdev[a] || !odev[a]) continue;
            const uint32_t i = act[a];
            HIPCHK(d, hipMemcpyAsync(&first_last[2 * a], offsets[i], 8, hipMemcpyDeviceToHost, s));
            HIPCHK(d, hipMemcpyAsync(&first_last[2 * a + 1], offsets[i] + m[i], 8,
                                     hipMemcpyDeviceToHost, s));
        }
        HIPCHK(d, hipStreamSynchronize(s));
    }
    for (uint32_t a = 0; a < na; ++a) {
        if (rdev[a]) continue;
        if (first_last[2 * a + 1] < first_last[2 * a]) return fail(d, BWT_EINVAL);
        const uint64_t b0 = first_last[2 * a] / 4, b1 = (first_last[2 * a + 1] + 3) / 4;
        stage_need[a] = b1 - b0;
        stage_total += ((b1 - b0) + 255) & ~255ull;
    }
    int rc;
    if (stage_total) {
        if ((rc = ensure_buf(d, d->bstage, d->bstage_cap, stage_total))) return rc;
        uint64_t at = 0;
        for (uint32_t a = 0; a < na; ++a) {
            const uint32_t i = act[a];
            if (!odev[a]) {
                HIPCHK(d, hipMemcpyAsync(d->bstage + at, offsets[i], (m[i] + 1) * 8,
                                         hipMemcpyHostToDevice, s));
                doff[a] = reinterpret_cast<const uint64_t *>(d->bstage + at);
                at += ((m[i] + 1) * 8 + 255) & ~255ull;
            } else {
                doff[a] = offsets[i];
            }
            if (!rdev[a]) {
                const uint64_t b0 = first_last[2 * a] / 4;
                if (stage_need[a])
                    HIPCHK(d, hipMemcpyAsync(d->bstage + at, reads[i] + b0, stage_need[a],
                                             hipMemcpyHostToDevice, s));
                dreads[a] = d->bstage + at;
                sym_base[a] = 4 * b0;
                at += (stage_need[a] + 255) & ~255ull;
            } else {
                dreads[a] = reads[i];
            }
        }
    } else {
        for (uint32_t a = 0; a < na; ++a) {
            dreads[a] = reads[act[a]];
            doff[a] = offsets[act[a]];
        }
    }

    // 2. plan: offsets check, suffix and block counts per set; cuts of the
    // sets with more than one block
    const uint64_t M = d->M;
    std::vector<PlanSet> ps(na);
    for (uint32_t a = 0; a < na; ++a) ps[a] = PlanSet{doff[a], m[act[a]], 0};
    std::vector<uint8_t> tab;
    size_t ps_at = put_table(tab, ps);
    size_t res_at = (tab.size() + 255) & ~(size_t)255;
    const uint64_t plan_bytes = res_at + (uint64_t)na * 32;
    if ((rc = ensure_buf(d, d->btab, d->btab_cap, plan_bytes))) return rc;
    HIPCHK(d, hipMemcpyAsync(d->btab + ps_at, tab.data() + ps_at, na * sizeof(PlanSet),
                             hipMemcpyHostToDevice, s));
    uint64_t *res_dev = reinterpret_cast<uint64_t *>(d->btab + res_at);
    HIPCHK(d, launch_plan_sets(reinterpret_cast<const PlanSet *>(d->btab + ps_at), na, M, res_dev,
                               nullptr, s));
    std::vector<uint64_t> res(4 * (size_t)na);
    HIPCHK(d, hipMemcpyAsync(res.data(), res_dev, res.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(d, hipStreamSynchronize(s));
    uint64_t maxlen = 0, cut_words = 0;
    bool multi = false;
    for (uint32_t a = 0; a < na; ++a) {
        if (res[4 * a] || res[4 * a + 1] > MAX_READ || res[4 * a + 3] == 0)
            return fail(d, BWT_EINVAL);
        maxlen = std::max(maxlen, res[4 * a + 1]);
        ps[a].cut_base = cut_words;
        cut_words += 2 * (res[4 * a + 3] + 1);
        multi |= res[4 * a + 3] > 1;
    }
    std::vector<uint64_t> cuts(cut_words);
    if (multi) {
        if ((rc = ensure_buf(d, d->cuts, d->cuts_cap, cut_words))) return rc;
        HIPCHK(d, hipMemcpyAsync(d->btab + ps_at, ps.data(), na * sizeof(PlanSet),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(d, launch_plan_sets(reinterpret_cast<const PlanSet *>(d->btab + ps_at), na, M,
                                   res_dev, d->cuts, s));
        HIPCHK(d, hipMemcpyAsync(cuts.data(), d->cuts, cut_words * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(d, hipStreamSynchronize(s));
    } else {
        for (uint32_t a = 0; a < na; ++a) {
            uint64_t *c = cuts.data() + ps[a].cut_base;
            c[0] = 0;
            c[1] = 0;
            c[2] = m[act[a]];
            c[3] = res[4 * a + 2];
        }
    }

    // 3. units, level by level, and device blocks
    std::vector<HostUnit> units;
    std::vector<uint64_t> n_run(na);
    std::vector<std::array<int, 2>> other(na);
    uint64_t maxK = 0;
    for (uint32_t a = 0; a < na; ++a) {
        bwt_set *h = hs[act[a]];
        n_run[a] = h->n;
        int k = 0;
        for (int b = 0; b < 3; ++b)
            if (b != h->cur) other[a][k++] = b;
        maxK = std::max(maxK, res[4 * a + 3]);
    }
    std::vector<DevBlock> blocks;
    uint64_t dst_read = 0, dst_sym = 0;
    for (uint64_t lv = 0; lv < maxK; ++lv) {
        bool open_block = false;
        for (uint32_t a = 0; a < na; ++a) {
            if (lv >= res[4 * a + 3]) continue;
            const uint64_t *c = cuts.data() + ps[a].cut_base;
            HostUnit u;
            u.set = a;
            u.level = (uint32_t)lv;
            u.j0 = c[2 * lv];
            u.j1 = c[2 * lv + 2];
            u.nsuf = c[2 * lv + 3] - c[2 * lv + 1];
            u.nsym = u.nsuf - (u.j1 - u.j0);
            u.dst_read0 = dst_read;
            u.dst_sym0 = dst_sym;
            u.n_ext = n_run[a];
            u.src = lv == 0 ? hs[act[a]]->cur : other[a][(lv - 1) & 1];
            u.dst = other[a][lv & 1];
            dst_read += u.j1 - u.j0;
            dst_sym += u.nsym;
            n_run[a] += u.nsuf;
            if (!open_block || blocks.back().n_blk + u.nsuf > M) {
                DevBlock B{};
                B.u0 = B.u1 = (uint32_t)units.size();
                B.read0 = u.dst_read0;
                blocks.push_back(B);
                open_block = true;
            }
            DevBlock &B = blocks.back();
            B.u1 += 1;
            B.m_blk += u.j1 - u.j0;
            B.n_blk += u.nsuf;
            B.gtotal += u.n_ext + 1;
            B.ntiles += div_up(records_for(u.n_ext + u.nsuf), INS_TILE_RECS);
            units.push_back(u);
        }
    }
    const uint64_t total_reads = dst_read, total_syms = dst_sym;
    uint64_t max_nblk = 0, max_fn = 0;
    for (auto &B : blocks) {
        if (B.n_blk > MAX_BLOCK) return fail(d, BWT_EINVAL);
        max_nblk = std::max(max_nblk, B.n_blk);
        max_fn = std::max(max_fn, B.ntiles + (B.u1 - B.u0));
    }

    // 4. memory: the sets' spare index buffers, the shared workspace, staging
    for (uint32_t a = 0; a < na; ++a) {
        bwt_set *h = hs[act[a]];
        for (int b : other[a])
            if ((rc = ensure_index(h, h->buf[b], n_run[a]))) return fail(d, rc);
    }
    if ((rc = ensure_ws(d, max_nblk))) return rc;
    if ((rc = ensure_buf(d, d->stage_reads, d->stage_reads_cap, div_up(total_syms, 16) * 4 + 16)))
        return rc;
    if ((rc = ensure_buf(d, d->stage_off, d->stage_off_cap, total_reads + 1))) return rc;
    if ((rc = ensure_buf(d, d->first_new, d->first_new_cap, max_fn + 2))) return rc;

    // 5. unit tables (one upload)
    tab.clear();
    std::vector<GatherUnit> gu(units.size());
    for (size_t k = 0; k < units.size(); ++k) {
        const HostUnit &u = units[k];
        // the staged copy of host reads starts at symbol sym_base of the set
        gu[k] = GatherUnit{dreads[u.set], doff[u.set], u.j0, u.j1, u.dst_read0, u.dst_sym0,
                           sym_base[u.set]};
    }
    const size_t gu_at = put_table(tab, gu);
    for (auto &B : blocks) {
        std::vector<RankUnit> ru;
        std::vector<InsertUnit> iu;
        uint64_t goff = 0, sa0 = 0, tile0 = 0;
        for (uint32_t k = B.u0; k < B.u1; ++k) {
            const HostUnit &u = units[k];
            bwt_set *h = hs[act[u.set]];
            const IndexBuf &S = h->buf[u.src];
            IndexBuf &D = h->buf[u.dst];
            ru.push_back(RankUnit{S.recs, S.sbc, S.meta, goff, (uint32_t)(u.dst_read0 - B.read0),
                                  u.n_ext >= (1ull << SB_SHIFT) ? 1u : 0u});
            iu.push_back(InsertUnit{S.recs, S.sbc, S.meta, D.recs, D.sbc, D.meta, u.n_ext, u.nsuf,
                                    sa0, goff, tile0});
            goff += u.n_ext + 1;
            sa0 += u.nsuf;
            tile0 += div_up(records_for(u.n_ext + u.nsuf), INS_TILE_RECS);
        }
        B.rank_off = put_table(tab, ru);
        B.ins_off = put_table(tab, iu);
    }
    if ((rc = ensure_buf(d, d->btab, d->btab_cap, tab.size()))) return rc;
    HIPCHK(d, hipMemcpyAsync(d->btab, tab.data(), tab.size(), hipMemcpyHostToDevice, s));
    HIPCHK(d, hipStreamSynchronize(s));  // tab is pageable host memory

    // 6-7 captured (BWT_PARAM_GRAPH on hs[0]): the staging and every device
    // block in one graph on one stream, replayed while the batch's plan and
    // the sets' index states stay the same
    if (d->graph && (max_nblk < BUCKET_MIN_BLOCK || !d->sort_buckets)) {
        std::vector<uint64_t> key = {0xba7c4ull, na, M, (uint64_t)d->key_bits,
                                     (uint64_t)d->radix_cfg, d->seg_len, d->seg_overlap,
                                     g_alloc_gen.load(), maxlen, total_reads, total_syms,
                                     blocks.size(), (uint64_t)(uintptr_t)d};
        for (uint32_t a = 0; a < na; ++a) {
            const bwt_set *h = hs[act[a]];
            key.insert(key.end(), {(uint64_t)(uintptr_t)h, (uint64_t)h->cur, h->n, h->m,
                                   (uint64_t)(uintptr_t)dreads[a], (uint64_t)(uintptr_t)doff[a],
                                   m[act[a]], sym_base[a]});
        }
        for (const HostUnit &u : units) key.insert(key.end(), {u.set, u.j0, u.j1, u.nsuf});
        bwt_set::GraphEntry *ge = nullptr;
        for (auto &g : d->graphs)
            if (g.key == key) ge = &g;
        if (!ge && (d->cap_stream || hipStreamCreateWithFlags(&d->cap_stream,
                                                              hipStreamNonBlocking) == hipSuccess)) {
            hipStream_t cs = d->cap_stream;
            const bool timing = d->timer.on;
            d->timer.on = false;
            d->capturing = true;
            bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                Workspace &w = d->ws;
                const uint64_t tiles = div_up(w.cap, RADIX_MIN_TILE) + 1;
                const GatherUnit *gdev = reinterpret_cast<const GatherUnit *>(d->btab + gu_at);
                ok = launch_zero_u32(reinterpret_cast<uint32_t *>(w.status_radix),
                                     (uint32_t)(tiles * 256 * 2), cs) == hipSuccess &&
                     launch_zero_u32(reinterpret_cast<uint32_t *>(w.status_scan),
                                     (uint32_t)(tiles * 8 * 2), cs) == hipSuccess &&
                     launch_zero_u32(w.misc, MISC_HIST, cs) == hipSuccess &&
                     launch_gather_offsets(gdev, (uint32_t)units.size(), total_reads, total_syms,
                                           d->stage_off, cs) == hipSuccess &&
                     launch_gather_reads(gdev, (uint32_t)units.size(), total_syms,
                                         d->stage_reads, cs) == hipSuccess;
                const BatchInput gin{d->stage_reads, d->stage_off, d->btab, maxlen};
                for (size_t b = 0; ok && b < blocks.size(); ++b)
                    ok = run_block(d, cs, blocks[b], units, gin) == BWT_OK;
                hipGraph_t g = nullptr;
                const bool ended = hipStreamEndCapture(cs, &g) == hipSuccess && g;
                ok = ok && ended;
                hipGraphExec_t exec = nullptr;
                if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
                if (g) (void)hipGraphDestroy(g);
                if (ok) {
                    if (d->graphs.size() >= MAX_GRAPHS) {
                        (void)hipGraphExecDestroy(d->graphs.front().exec);
                        d->graphs.erase(d->graphs.begin());
                    }
                    d->graphs.push_back({std::move(key), exec, 0});
                    d->graph_captures += 1;
                    ge = &d->graphs.back();
                }
            }
            if (!ok) (void)hipGetLastError();
            d->capturing = false;
            d->timer.on = timing;
            d->broken = false;
            d->last_error = BWT_OK;
        }
        if (ge) {
            HIPCHK(d, hipGraphLaunch(ge->exec, s));
            HIPCHK(d, hipStreamSynchronize(s));
            uint32_t e = 0;
            if ((rc = read_u32(d, s, d->ws.misc + MISC_ERR, &e))) return rc;
            d->graph_replays += 1;
            if (e == 0) {
                for (uint32_t a = 0; a < na; ++a) {
                    bwt_set *h = hs[act[a]];
                    const uint64_t K = res[4 * a + 3];
                    h->cur = other[a][(K - 1) & 1];
                    h->n = n_run[a];
                    h->m += m[act[a]];
                }
                return BWT_OK;
            }
            if (!(e & REFINE_REDO)) {
                rc = check_err(d, s);
                return fail(d, rc ? rc : BWT_EHIP);
            }
            d->graph_redos += 1;   // a tied group needs prefix doubling: run eagerly
        }
    }

    // 6. staging: every unit's reads, in schedule order, into one input
    {
        Scope sc(d, s, BWT_STAGE_PLAN);
        const GatherUnit *gdev = reinterpret_cast<const GatherUnit *>(d->btab + gu_at);
        HIPCHK(d, launch_gather_offsets(gdev, (uint32_t)units.size(), total_reads, total_syms,
                                        d->stage_off, s));
        HIPCHK(d, launch_gather_reads(gdev, (uint32_t)units.size(), total_syms, d->stage_reads, s));
    }

    // 7. the device blocks, level by level.  Blocks of one level touch
    // disjoint sets, so they are spread over lanes (streams with their own
    // workspace) that run side by side; the next level starts when all are done.
    HIPCHK(d, hipStreamSynchronize(s));
    const int nl = std::max(1, std::min<int>(d->batch_lanes, MAX_LANES));
    std::vector<bwt_set *> lane{d};
    for (int k = 1; k < nl; ++k) {
        if ((int)d->lanes.size() < k) {
            bwt_set *l = bwt_set_create("ACGT");
            if (!l) return fail(d, BWT_ENOMEM);
            d->lanes.push_back(l);
        }
        bwt_set *l = d->lanes[k - 1];
        l->key_bits = d->key_bits;
        l->radix_cfg = d->radix_cfg;
        l->seg_len = d->seg_len;
        l->seg_overlap = d->seg_overlap;
        l->sort_buckets = d->sort_buckets;
        l->timer.on = d->timer.on;
        lane.push_back(l);
    }
    for (int k = 1; k < nl; ++k) {
        if ((rc = ensure_ws(lane[k], max_nblk))) return fail(d, rc);
        if ((rc = ensure_buf(lane[k], lane[k]->first_new, lane[k]->first_new_cap, max_fn + 2)))
            return fail(d, rc);
    }
    std::vector<hipStream_t> ls{s};
    for (int k = 1; k < nl; ++k) ls.push_back(lane[k]->stream);
    for (int k = 0; k < nl; ++k)
        if ((rc = clear_err(lane[k], ls[k]))) return fail(d, rc);
    const BatchInput in{d->stage_reads, d->stage_off, d->btab, maxlen};
    size_t b0 = 0;
    while (b0 < blocks.size()) {
        size_t b1 = b0;
        while (b1 < blocks.size() && units[blocks[b1].u0].level == units[blocks[b0].u0].level) ++b1;
        const int used = (int)std::min<size_t>(nl, b1 - b0);
        // largest block first onto the least loaded lane
        std::vector<std::vector<size_t>> mine(used);
        {
            std::vector<size_t> ord;
            for (size_t b = b0; b < b1; ++b) ord.push_back(b);
            std::sort(ord.begin(), ord.end(),
                      [&](size_t x, size_t y) { return blocks[x].n_blk > blocks[y].n_blk; });
            std::vector<uint64_t> load(used, 0);
            for (size_t b : ord) {
                int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                mine[k].push_back(b);
                load[k] += blocks[b].n_blk;
            }
        }
        std::vector<int> lrc(used, BWT_OK);
        auto work = [&](int k) {
            if (k > 0 && hipSetDevice(d->device) != hipSuccess) {
                (void)hipGetLastError();
                lrc[k] = BWT_EHIP;
                return;
            }
            for (size_t b : mine[k]) {
                lrc[k] = run_block(lane[k], ls[k], blocks[b], units, in);
                if (lrc[k]) return;
            }
            if (hipStreamSynchronize(ls[k]) != hipSuccess) {
                (void)hipGetLastError();
                lrc[k] = BWT_EHIP;
            }
        };
        if (used == 1) {
            work(0);
        } else {
            std::vector<std::thread> th;
            for (int k = 1; k < used; ++k) th.emplace_back(work, k);
            work(0);
            for (auto &t : th) t.join();
        }
        for (int k = 0; k < used; ++k)
            if (lrc[k]) {
                for (int j = 0; j < nl; ++j) (void)hipStreamSynchronize(ls[j]);
                if (lrc[k] == BWT_EHIP) d->broken = true;
                return fail(d, lrc[k]);
            }
        b0 = b1;
    }
    for (int k = 0; k < nl; ++k) HIPCHK(d, hipStreamSynchronize(ls[k]));
    for (int k = 0; k < nl; ++k) {
        if (lane[k]->timer.on) timer_collect(lane[k]);
        if (k > 0) {
            stats_add(d->timer.acc, lane[k]->timer.acc);
            memset(&lane[k]->timer.acc, 0, sizeof lane[k]->timer.acc);
        }
    }
    for (int k = 0; k < nl; ++k)
        if ((rc = check_err(lane[k], ls[k]))) {
            if (k > 0) d->broken = lane[k]->broken;
            return fail(d, rc);
        }

    // 8. commit every set
    for (uint32_t a = 0; a < na; ++a) {
        bwt_set *h = hs[act[a]];
        const uint64_t K = res[4 * a + 3];
        h->cur = other[a][(K - 1) & 1];
        h->n = n_run[a];
        h->m += m[act[a]];
    }
    return BWT_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
// ---- ConstructSA without allocation ------------------------------------------
// bwt_set_block_sort_noalloc runs on a workspace carved from `scratch`, one
// array per GPU in the library's code object, instead of the handle's.  In
// host code the name `scratch` is only a stand-in: the array's device address
// on each GPU comes from hipGetSymbolAddress (taken once per device, with that
// device current, when the first handle on it is created) and only that
// address is passed to kernels.  Calls on one GPU share the array and keep the
// last call's contents; every call clears the counters it needs, and calls
// from threads of this process are serialized per device.
namespace {
constexpr uint64_t NOALLOC_MAX_SUFFIXES = 1ull << 18;
constexpr uint64_t NOALLOC_BYTES = 24ull << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu[NOALLOC_MAX_DEVICES];
uint8_t *g_scratch_ptr[NOALLOC_MAX_DEVICES];   // device address per device, or null
bool g_scratch_fresh[NOALLOC_MAX_DEVICES];     // status words not yet cleared
}  // namespace

static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

namespace {
// Takes the device address of `scratch` on device `dev` (current).  Failure
// is not fatal for the handle: the no-allocation entry point reports it.
void scratch_setup(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> g(g_scratch_mu[dev]);
    if (g_scratch_ptr[dev]) return;
    Workspace t;
    if (carve_ws(t, NOALLOC_MAX_SUFFIXES, nullptr) > NOALLOC_BYTES) return;
    uint8_t *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return;
    }
    g_scratch_ptr[dev] = ptr;
    g_scratch_fresh[dev] = true;
}

// Lends the handle the workspace view of the scratch array (timing off) for
// the length of one call.
struct ScratchWs {
    bwt_set *h;
    Workspace saved;
    bool timing;
    ScratchWs(bwt_set *h_, uint8_t *base) : h(h_), saved(h_->ws), timing(h_->timer.on) {
        Workspace w;
        carve_ws(w, NOALLOC_MAX_SUFFIXES, base);
        h->ws = w;
        h->timer.on = false;
    }
    ~ScratchWs() {
        h->ws = saved;
        h->timer.on = timing;
    }
};
}  // namespace

extern "C" {

bwt_set_t bwt_set_create(const char *alphabet) {
    if (!alphabet) {
        g_create_error = BWT_EINVAL;
        return nullptr;
    }
    if (strcmp(alphabet, "ACGT") != 0) {
        g_create_error = BWT_EALPHABET;
        return nullptr;
    }
    bwt_set *h = new (std::nothrow) bwt_set();
    if (!h) {
        g_create_error = BWT_ENOMEM;
        return nullptr;
    }
    bool ok = hipGetDevice(&h->device) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&h->pinned, 512 * 8, hipHostMallocDefault) == hipSuccess;
    ok = ok && dalloc(&h->res, 4) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        g_create_error = BWT_EHIP;
        bwt_set_destroy(h);
        return nullptr;
    }
    for (int b = 0; b < 3; ++b) {
        if (ensure_index(h, h->buf[b], 1024 * REC_SYMS) != BWT_OK) {
            g_create_error = BWT_ENOMEM;
            bwt_set_destroy(h);
            return nullptr;
        }
    }
    if (launch_index_init(h->buf[0].recs, h->buf[0].sbc, h->buf[0].meta, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        (void)hipGetLastError();
        g_create_error = BWT_EHIP;
        bwt_set_destroy(h);
        return nullptr;
    }
    scratch_setup(h->device);
    h->cur = 0;
    g_create_error = BWT_OK;
    return h;
}

void bwt_set_destroy(bwt_set_t h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto &b : h->buf) {
        free_index_data(b);
        dfree(b.meta);
    }
    free_ws(h->ws);
    dfree(h->first_new);
    dfree(h->stage_reads);
    dfree(h->stage_off);
    dfree(h->cuts);
    dfree(h->stage_out);
    dfree(h->strand_reads);
    dfree(h->strand_off);
    dfree(h->btab);
    dfree(h->bstage);
    for (auto *l : h->lanes) bwt_set_destroy(l);
    h->lanes.clear();
    drop_graphs(h);
    if (h->pipe) {
        pipe_free(*h->pipe);
        delete h->pipe;
        h->pipe = nullptr;
    }
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    dfree(h->res);
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (auto e : h->timer.pool) (void)hipEventDestroy(e);
    for (auto &sp : h->timer.open) {
        (void)hipEventDestroy(sp.a);
        (void)hipEventDestroy(sp.b);
    }
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // extern "C"

namespace {

// The blocks of one planned append, enqueued on s: block b reads the index
// written by block b-1 (the current one for b = 0) and writes other[b & 1].
// Nothing here waits for the device while h->capturing is set.  *src_out is
// the buffer that holds the result.
// One block of an append: reads/off (device; off points at the block's first
// read, m_blk + 1 entries) ranked against src, merged into dst.
int enqueue_block(bwt_set *h, hipStream_t s, const uint8_t *reads, const uint64_t *off,
                  uint32_t m_blk, uint32_t n_blk, uint64_t maxlen, int src, int dst,
                  uint64_t n_cur) {
    Workspace &w = h->ws;
    int rc;
    IndexBuf &S = h->buf[src];
    if ((rc = block_prep(h, s, off, m_blk, n_blk))) return rc;
    // ComputeRanks first: g leads the suffix sort key (an empty index ranks
    // every suffix 0, so the first block skips it)
    const int gbits = bits_for_value(n_cur);
    if (gbits > 0) {
        Scope sc(h, s, BWT_STAGE_RANKS);
        const RankKeys kk = rank_keys(h, s, gbits, n_blk, &rc);
        if (rc) return fail(h, rc);
        MarkSet mk(h, 3);
        HIPCHK(h, launch_compute_ranks(reads, off, w.soff, m_blk, n_blk, S.recs, S.sbc, S.meta,
                                       n_cur >= (1ull << SB_SHIFT) ? 1 : 0, w.g, &kk,
                                       rank_segments(h, maxlen), w.misc + MISC_ERR, s, mk.get()));
        mk.add(0, SPAN_RANKS_K, n_blk - m_blk);
        mk.add(1, SPAN_RANKS_SEG, 0);
        mk.add(2, SPAN_RANKS_FB, 0);
    }
    uint32_t *sa = nullptr;
    const uint64_t *gkeys = nullptr;
    int gshift = 64;
    if ((rc = block_sort(h, s, reads, off, m_blk, n_blk, maxlen, w.g, gbits, gbits > 0, &sa, &gkeys,
                         &gshift)))
        return rc;
    if ((rc = insert_block(h, s, S, h->buf[dst], n_cur, gkeys, gshift, sa, n_blk, m_blk)))
        return rc;
    h->timer.acc.blocks += 1;
    return BWT_OK;
}

// The blocks of one planned append, enqueued on s: block b reads the index
// written by block b-1 (the current one for b = 0) and writes other[b & 1].
// Nothing here waits for the device while h->capturing is set.  *src_out is
// the buffer that holds the result.
int enqueue_blocks(bwt_set *h, hipStream_t s, const Plan &P, const int other[2], int *src_out) {
    int src = h->cur, rc;
    uint64_t n_cur = h->n;
    const size_t K = P.cut_j.size() - 1;
    for (size_t b = 0; b < K; ++b) {
        const uint64_t j0 = P.cut_j[b], j1 = P.cut_j[b + 1];
        const uint32_t m_blk = (uint32_t)(j1 - j0);
        const uint32_t n_blk = (uint32_t)(P.cut_s[b + 1] - P.cut_s[b]);
        const int dst = other[b & 1];
        if ((rc = enqueue_block(h, s, P.reads, P.off + j0, m_blk, n_blk, P.maxlen, src, dst,
                                n_cur)))
            return rc;
        n_cur += n_blk;
        src = dst;
    }
    *src_out = src;
    return BWT_OK;
}

// ---- pipelined blocks: host reads streamed block by block -----------------------
// The paper's pipeline (Results, Figure 1) overlaps reading the input with
// the GPU and CPU stages, with multiple buffering.  Here a producer thread
// copies block k+1's reads (and its offsets, rebased) into one of two pinned
// slots and sends them to one of two device slots on a copy stream, while the
// blocks before it run on the compute stream; events order the two streams
// (a slot is refilled only after the block that used it is done).
int append_streamed(bwt_set *h, hipStream_t s, const Plan &P, const int other[2], int *src_out) {
    Pipe &pp = *h->pipe;
    const size_t K = P.cut_j.size() - 1;
    const uint64_t o0 = P.hoff[0];
    // per block: first byte of its reads, bytes, rebased offsets
    uint64_t max_bytes = 0, max_m = 0;
    for (size_t b = 0; b < K; ++b) {
        const uint64_t s0 = P.hoff[P.cut_j[b]], s1 = P.hoff[P.cut_j[b + 1]];
        max_bytes = std::max(max_bytes, (s1 + 3) / 4 - s0 / 4);
        max_m = std::max(max_m, P.cut_j[b + 1] - P.cut_j[b]);
    }
    (void)o0;
    const uint64_t rb = (max_bytes + 16 + 255) & ~255ull, ob = ((max_m + 1) * 8 + 255) & ~255ull;
    const uint64_t slot = rb + ob;
    int rc;
    if ((rc = ensure_buf(h, h->stage_reads, h->stage_reads_cap, 2 * slot))) return rc;
    if (pp.slot_bytes < slot) {
        if (pp.pinned) (void)hipHostFree(pp.pinned);
        pp.pinned = nullptr;
        pp.slot_bytes = 0;
        if (hipHostMalloc((void **)&pp.pinned, 2 * slot, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, BWT_ENOMEM);
        }
        pp.slot_bytes = slot;
    }
    if (!pp.copy && hipStreamCreateWithFlags(&pp.copy, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        pp.copy = nullptr;
        return fail(h, BWT_EHIP);
    }
    for (int q = 0; q < 2; ++q) {
        if (!pp.copied[q]) HIPCHK(h, hipEventCreateWithFlags(&pp.copied[q], hipEventDisableTiming));
        if (!pp.consumed[q])
            HIPCHK(h, hipEventCreateWithFlags(&pp.consumed[q], hipEventDisableTiming));
    }
    uint8_t *dev = h->stage_reads;
    // host side handshake: ready = blocks staged, enqueued = blocks whose
    // compute (and its consumed event) has been enqueued
    std::mutex mu;
    std::condition_variable cv;
    size_t ready = 0, enqueued = 0;
    bool stop = false;
    int prc = BWT_OK;
    std::thread producer([&] {
        int e = BWT_OK;
        if (hipSetDevice(h->device) != hipSuccess) e = BWT_EHIP;
        for (size_t b = 0; b < K && e == BWT_OK; ++b) {
            const int q = (int)(b & 1);
            if (b >= 2) {
                // the slot's previous block: its compute enqueued, its copy done
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || enqueued >= b - 1; });
                if (stop) break;
                lk.unlock();
                if (hipEventSynchronize(pp.copied[q]) != hipSuccess) {
                    e = BWT_EHIP;
                    break;
                }
            }
            const uint64_t j0 = P.cut_j[b], j1 = P.cut_j[b + 1];
            const uint64_t s0 = P.hoff[j0], s1 = P.hoff[j1];
            const uint64_t byte0 = s0 / 4, nbytes = (s1 + 3) / 4 - byte0;
            uint8_t *hp = pp.pinned + q * slot;
            if (nbytes) memcpy(hp, P.host_reads + byte0, nbytes);
            uint64_t *ho = reinterpret_cast<uint64_t *>(hp + rb);
            for (uint64_t j = j0; j <= j1; ++j) ho[j - j0] = P.hoff[j] - 4 * byte0;
            hipStream_t c = pp.copy;
            bool ok = true;
            if (b >= 2) ok = hipStreamWaitEvent(c, pp.consumed[q], 0) == hipSuccess;
            ok = ok && (!nbytes || hipMemcpyAsync(dev + q * slot, hp, nbytes, hipMemcpyHostToDevice,
                                                  c) == hipSuccess);
            ok = ok && hipMemcpyAsync(dev + q * slot + rb, ho, (j1 - j0 + 1) * 8,
                                      hipMemcpyHostToDevice, c) == hipSuccess;
            ok = ok && hipEventRecord(pp.copied[q], c) == hipSuccess;
            if (!ok) {
                e = BWT_EHIP;
                break;
            }
            std::lock_guard<std::mutex> lk(mu);
            ready = b + 1;
            cv.notify_all();
        }
        std::lock_guard<std::mutex> lk(mu);
        prc = e;
        stop = true;
        cv.notify_all();
    });
    int src = h->cur;
    uint64_t n_cur = h->n;
    for (size_t b = 0; b < K; ++b) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return ready > b || stop; });
            if (ready <= b) {
                rc = prc ? prc : BWT_EHIP;
                break;
            }
        }
        const int q = (int)(b & 1);
        const uint32_t m_blk = (uint32_t)(P.cut_j[b + 1] - P.cut_j[b]);
        const uint32_t n_blk = (uint32_t)(P.cut_s[b + 1] - P.cut_s[b]);
        const int dst = other[b & 1];
        rc = hipStreamWaitEvent(s, pp.copied[q], 0) == hipSuccess ? BWT_OK : BWT_EHIP;
        if (!rc)
            rc = enqueue_block(h, s, dev + q * slot,
                               reinterpret_cast<const uint64_t *>(dev + q * slot + rb), m_blk,
                               n_blk, P.maxlen, src, dst, n_cur);
        if (!rc && hipEventRecord(pp.consumed[q], s) != hipSuccess) rc = BWT_EHIP;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (rc) stop = true;
            else enqueued = b + 1;
            cv.notify_all();
        }
        if (rc) break;
        n_cur += n_blk;
        src = dst;
    }
    producer.join();
    if (rc) {
        (void)hipStreamSynchronize(pp.copy);
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        return fail(h, rc == BWT_EHIP ? BWT_EHIP : rc);
    }
    if (prc) return fail(h, prc);
    *src_out = src;
    return BWT_OK;
}

// Everything a captured append depends on besides the symbols themselves.
std::vector<uint64_t> graph_key(const bwt_set *h, const Plan &P) {
    std::vector<uint64_t> k = {(uint64_t)(uintptr_t)P.reads, (uint64_t)(uintptr_t)P.off,
                               P.maxlen, P.total_suffixes, h->n, h->m, (uint64_t)h->cur, h->M,
                               (uint64_t)h->key_bits, (uint64_t)h->radix_cfg, h->seg_len,
                               h->seg_overlap, g_alloc_gen.load()};
    k.insert(k.end(), P.cut_j.begin(), P.cut_j.end());
    k.insert(k.end(), P.cut_s.begin(), P.cut_s.end());
    return k;
}

// Captures the blocks of a planned append into an executable graph (or finds
// the one captured for the same key).  Returns the entry, or null when
// capture failed (the caller then runs the append eagerly).
bwt_set::GraphEntry *captured_append(bwt_set *h, const Plan &P, const int other[2]) {
    std::vector<uint64_t> key = graph_key(h, P);
    for (auto &g : h->graphs)
        if (g.key == key) return &g;
    if (!h->cap_stream &&
        hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        h->cap_stream = nullptr;
        return nullptr;
    }
    hipStream_t cs = h->cap_stream;
    const bool timing = h->timer.on;
    h->timer.on = false;
    h->capturing = true;
    int src = h->cur;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        Workspace &w = h->ws;
        // every replay starts from cleared look-back words and counters
        // (fill kernels: memset nodes are kept out of graphs), so the epochs
        // fixed at capture are fresh again
        const uint64_t tiles = div_up(w.cap, RADIX_MIN_TILE) + 1;
        ok = launch_zero_u32(reinterpret_cast<uint32_t *>(w.status_radix),
                             (uint32_t)(tiles * 256 * 2), cs) == hipSuccess &&
             launch_zero_u32(reinterpret_cast<uint32_t *>(w.status_scan), (uint32_t)(tiles * 8 * 2),
                             cs) == hipSuccess &&
             launch_zero_u32(w.misc, MISC_HIST, cs) == hipSuccess;
        ok = ok && enqueue_blocks(h, cs, P, other, &src) == BWT_OK;
        hipGraph_t g = nullptr;
        const bool ended = hipStreamEndCapture(cs, &g) == hipSuccess && g;
        ok = ok && ended;
        hipGraphExec_t exec = nullptr;
        if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (ok) {
            if (h->graphs.size() >= MAX_GRAPHS) {
                (void)hipGraphExecDestroy(h->graphs.front().exec);
                h->graphs.erase(h->graphs.begin());
            }
            h->graphs.push_back({std::move(key), exec, src});
            h->graph_captures += 1;
        }
    }
    if (!ok) (void)hipGetLastError();
    h->capturing = false;
    h->timer.on = timing;
    h->broken = false;   // a capture failure is not a device failure
    h->last_error = BWT_OK;
    return ok ? &h->graphs.back() : nullptr;
}

}  // namespace

extern "C" {

int bwt_set_append(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets, uint64_t m,
                   void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (m == 0) return BWT_OK;
    if (!reads || !offsets) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    Plan P;
    // host reads are streamed block by block (pipelined) unless captured
    const bool stream_in = h->pipeline && !h->graph && !is_device_ptr(reads);
    {
        Scope sc(h, s, BWT_STAGE_PLAN);
        rc = plan_input(h, s, reads, offsets, m, h->M, P, stream_in);
    }
    if (rc) {
        if (h->timer.on) {
            (void)hipStreamSynchronize(s);
            timer_collect(h);
        }
        return rc;
    }
    const uint64_t n_final = h->n + P.total_suffixes;
    // the two buffers other than the current one receive the blocks
    int other[2], k = 0;
    for (int b = 0; b < 3; ++b)
        if (b != h->cur) other[k++] = b;
    for (int b : other)
        if ((rc = ensure_index(h, h->buf[b], n_final))) return rc;
    if ((rc = ensure_ws(h, max_block(P)))) return rc;
    int src = h->cur;
    bool done = false;
    // capture is for launch-bound appends: blocks that take the bucket finish
    // (which decides on the host) run eagerly, where launches cost little
    if (h->graph && (max_block(P) < BUCKET_MIN_BLOCK || !h->sort_buckets)) {
        // a captured schedule: every buffer it names exists before capture
        const uint64_t nt = div_up(records_for(n_final), INS_TILE_RECS);
        if ((rc = ensure_buf(h, h->first_new, h->first_new_cap, nt + 2))) return rc;
        bwt_set::GraphEntry *ge = captured_append(h, P, other);
        if (ge) {
            HIPCHK(h, hipGraphLaunch(ge->exec, s));
            HIPCHK(h, hipStreamSynchronize(s));
            uint32_t e = 0;
            if ((rc = read_u32(h, s, h->ws.misc + MISC_ERR, &e))) return rc;
            h->graph_replays += 1;
            if (e == 0) {
                src = ge->src;
                done = true;
            } else if (e & REFINE_REDO) {
                h->graph_redos += 1;   // a tied group needs prefix doubling
            } else {
                if ((rc = check_err(h, s))) return rc;
            }
        }
    }
    if (!done) {
        if ((rc = clear_err(h, s))) return rc;
        if (P.host_reads) {
            if (!h->pipe) h->pipe = new (std::nothrow) Pipe();
            if (!h->pipe) return fail(h, BWT_ENOMEM);
            if ((rc = append_streamed(h, s, P, other, &src))) return rc;
        } else if ((rc = enqueue_blocks(h, s, P, other, &src))) {
            return rc;
        }
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->timer.on) timer_collect(h);
        if ((rc = check_err(h, s))) return rc;
    }
    h->cur = src;
    h->n = n_final;
    h->m += m;
    return BWT_OK;
}

int bwt_set_append_many(bwt_set_t *hs, const uint8_t *const *reads,
                        const uint64_t *const *offsets, const uint64_t *m, uint64_t count,
                        void *stream) {
    if (!hs || count == 0) return count == 0 ? BWT_OK : BWT_EINVAL;
    bwt_set *d = hs[0];
    if (!d) return BWT_EINVAL;
    if (!reads || !offsets || !m) return fail(d, BWT_EINVAL);
    std::vector<bwt_set *> seen;
    for (uint64_t i = 0; i < count; ++i) {
        if (!hs[i] || hs[i]->device != d->device) return fail(d, BWT_EINVAL);
        if (hs[i]->broken) return fail(d, BWT_ESTATE);
        seen.push_back(hs[i]);
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return fail(d, BWT_EINVAL);
    int rc = set_device(d);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : d->stream;
    rc = append_many(d, hs, reads, offsets, m, count, s);
    if (rc && d->timer.on) {
        (void)hipStreamSynchronize(s);
        timer_collect(d);
    }
    return rc;
}

uint64_t bwt_set_rank(bwt_set_t h, char c, uint64_t k) {
    if (!h) return UINT64_MAX;
    if (h->broken) {
        fail(h, BWT_ESTATE);
        return UINT64_MAX;
    }
    if (!(c == 'A' || c == 'C' || c == 'G' || c == 'T' || c == '$') || k > h->n) {
        fail(h, BWT_EINVAL);
        return UINT64_MAX;
    }
    if (set_device(h)) return UINT64_MAX;
    // device scratch: res[0] = query k, res[1] = result, byte query in res[2]
    uint64_t *hp = h->pinned;
    hp[0] = k;
    hp[2] = (uint64_t)(uint8_t)c;
    IndexBuf &B = h->buf[h->cur];
    if (hipMemcpyAsync(h->res, hp, 3 * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        launch_rank_many(B.recs, B.sbc, B.meta, reinterpret_cast<const uint8_t *>(h->res + 2),
                         h->res, h->res + 1, 1, h->stream) != hipSuccess ||
        hipMemcpyAsync(hp + 8, h->res + 1, 8, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        (void)hipGetLastError();
        fail(h, BWT_EHIP);
        return UINT64_MAX;
    }
    return hp[8];
}

int bwt_set_rank_many(bwt_set_t h, const uint8_t *cs, const uint64_t *ks, uint64_t *out,
                      uint64_t count, void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (count == 0) return BWT_OK;
    if (!cs || !ks || !out) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    IndexBuf &B = h->buf[h->cur];
    HIPCHK(h, launch_rank_many(B.recs, B.sbc, B.meta, cs, ks, out, count, s));
    return BWT_OK;
}

}  // extern "C"

// ---- autotuning -------------------------------------------------------------
// The tuning knobs never change a result, only the time: the tuner builds the
// caller's input from empty on a scratch handle with candidate settings and
// keeps the fastest, one knob at a time (first-key width, ComputeRanks
// segments, radix tile shape).  Results are cached per GPU architecture and
// shape class (block size, mean and longest read length) in the process and,
// when BWTSET_TUNE_CACHE names a file, in that file as lines of
// "<class> <radix tile> <key bits> <segment> <overlap>".
namespace {

struct TuneSet {
    int radix_cfg, key_bits;
    uint32_t seg_len, seg_overlap;
};
std::mutex g_tune_mu;
std::map<std::string, TuneSet> g_tune;
bool g_tune_loaded = false;

int log2_ceil(uint64_t v) {
    int b = 0;
    while (b < 63 && (1ull << b) < v) ++b;
    return b;
}

std::string tune_class(int dev, uint64_t M, const Plan &P, uint64_t m) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    } else {
        (void)hipGetLastError();
    }
    const uint64_t blk = std::min<uint64_t>(M, P.total_suffixes);
    const uint64_t mean = m ? (P.total_suffixes - m) / m : 0;
    std::ostringstream k;
    k << arch << "/b" << log2_ceil(blk) << "/r" << log2_ceil(mean + 1) << "/x"
      << log2_ceil(P.maxlen + 1);
    return k.str();
}

void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = getenv("BWTSET_TUNE_CACHE");
    if (!f || !*f) return;
    std::ifstream in(f);
    std::string cls;
    TuneSet t;
    while (in >> cls >> t.radix_cfg >> t.key_bits >> t.seg_len >> t.seg_overlap) g_tune[cls] = t;
}

void tune_store(const std::string &cls, const TuneSet &t) {
    g_tune[cls] = t;
    const char *f = getenv("BWTSET_TUNE_CACHE");
    if (!f || !*f) return;
    std::ofstream out(f, std::ios::app);
    out << cls << ' ' << t.radix_cfg << ' ' << t.key_bits << ' ' << t.seg_len << ' '
        << t.seg_overlap << '\n';
}

void tune_apply(bwt_set *h, const TuneSet &t) {
    h->radix_cfg = t.radix_cfg;
    h->key_bits = t.key_bits;
    h->seg_len = t.seg_len;
    h->seg_overlap = t.seg_overlap;
}

}  // namespace

extern "C" {

int bwt_set_autotune(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets, uint64_t m,
                     int force, bwt_tune_t *out) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (m == 0 || !reads || !offsets) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    Plan P;
    if ((rc = plan_input(h, h->stream, reads, offsets, m, h->M, P))) return rc;
    const std::string cls = tune_class(h->device, h->M, P, m);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    auto it = g_tune.find(cls);
    if (it != g_tune.end() && !force) {
        tune_apply(h, it->second);
        if (out) *out = bwt_tune_t{it->second.radix_cfg, it->second.key_bits,
                                   it->second.seg_len, it->second.seg_overlap, 1, 0.0, 0};
        return BWT_OK;
    }
    bwt_set *t = bwt_set_create("ACGT");
    if (!t) return fail(h, BWT_ENOMEM);
    t->M = h->M;
    t->sort_buckets = h->sort_buckets;
    int trials = 0;
    // median of three builds from empty (after one warm-up build)
    auto time_it = [&](const TuneSet &c, double *ms) -> int {
        tune_apply(t, c);
        double v[3];
        for (int r = -1; r < 3; ++r) {
            int e = bwt_set_reset(t);
            if (e) return e;
            auto t0 = std::chrono::steady_clock::now();
            if ((e = bwt_set_append(t, reads, offsets, m, nullptr))) return e;
            auto t1 = std::chrono::steady_clock::now();
            if (r >= 0) v[r] = std::chrono::duration<double, std::milli>(t1 - t0).count();
        }
        std::sort(v, v + 3);
        *ms = v[1];
        ++trials;
        return BWT_OK;
    };
    TuneSet best{h->radix_cfg, h->key_bits, h->seg_len, h->seg_overlap};
    double best_ms = 0;
    rc = time_it(best, &best_ms);
    auto consider = [&](TuneSet c) -> int {
        double ms;
        int e = time_it(c, &ms);
        if (e) return e;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        return BWT_OK;
    };
    const uint64_t mean = (P.total_suffixes - m) / m;
    for (int kb : {64, 48, 40, 32}) {
        if (rc) break;
        if (kb == best.key_bits) continue;
        TuneSet c = best;
        c.key_bits = kb;
        rc = consider(c);
    }
    {
        std::vector<std::pair<uint32_t, uint32_t>> segs = {{768, 64}, {1024, 128}, {0, 0}};
        if (mean <= 512) segs.insert(segs.end(), {{32, 16}, {64, 16}, {128, 32}});
        for (auto so : segs) {
            if (rc) break;
            if (so.first == best.seg_len && so.second == best.seg_overlap) continue;
            TuneSet c = best;
            c.seg_len = so.first;
            c.seg_overlap = so.second;
            rc = consider(c);
        }
    }
    for (int cfg : {3, 0, 1, 5}) {
        if (rc) break;
        if (cfg == best.radix_cfg) continue;
        TuneSet c = best;
        c.radix_cfg = cfg;
        rc = consider(c);
    }
    bwt_set_destroy(t);
    if (rc) return fail(h, rc);
    tune_store(cls, best);
    tune_apply(h, best);
    if (out) *out = bwt_tune_t{best.radix_cfg, best.key_bits, best.seg_len, best.seg_overlap, 0,
                               best_ms, trials};
    return BWT_OK;
}

int bwt_set_append_strands(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                           uint64_t m, int mode, void *stream) {
    if (!h) return BWT_EINVAL;
    if (mode == BWT_STRAND_FORWARD) return bwt_set_append(h, reads, offsets, m, stream);
    if (h->broken) return fail(h, BWT_ESTATE);
    if (mode != BWT_STRAND_REVERSE && mode != BWT_STRAND_BOTH) return fail(h, BWT_EINVAL);
    if (m == 0) return BWT_OK;
    if (!reads || !offsets) return fail(h, BWT_EINVAL);
    if (m > (1ull << 40)) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    // the input on the device, its offsets checked before anything reads
    // symbols through them
    const bool off_dev = is_device_ptr(offsets), reads_dev = is_device_ptr(reads);
    const uint64_t *doff = offsets;
    uint64_t first = 0, last = 0;
    if (!off_dev) {
        for (uint64_t j = 0; j < m; ++j)
            if (offsets[j + 1] < offsets[j]) return fail(h, BWT_EINVAL);
        first = offsets[0];
        last = offsets[m];
        if ((rc = ensure_buf(h, h->stage_off, h->stage_off_cap, m + 1))) return rc;
        HIPCHK(h, hipMemcpyAsync(h->stage_off, offsets, (m + 1) * 8, hipMemcpyHostToDevice, s));
        doff = h->stage_off;
    } else {
        HIPCHK(h, launch_check_offsets(offsets, m, h->res, s));
        HIPCHK(h, hipMemcpyAsync(h->pinned, h->res, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipMemcpyAsync(h->pinned + 1, offsets, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipMemcpyAsync(h->pinned + 2, offsets + m, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->pinned[0]) return fail(h, BWT_EINVAL);
        first = h->pinned[1];
        last = h->pinned[2];
    }
    const uint64_t syms = last - first;
    const uint8_t *din = reads;
    uint64_t in_base = 0;
    if (!reads_dev) {
        in_base = first & ~3ull;
        const uint64_t nbytes = (last + 3) / 4 - in_base / 4;
        if ((rc = ensure_buf(h, h->stage_reads, h->stage_reads_cap, nbytes + 16))) return rc;
        HIPCHK(h, hipMemcpyAsync(h->stage_reads, reads + in_base / 4, nbytes,
                                 hipMemcpyHostToDevice, s));
        din = h->stage_reads;
    }
    const uint64_t total = mode == BWT_STRAND_BOTH ? 2 * syms : syms;
    const uint64_t mo = mode == BWT_STRAND_BOTH ? 2 * m : m;
    if ((rc = ensure_buf(h, h->strand_reads, h->strand_reads_cap, div_up(total, 16) * 4 + 16)))
        return rc;
    if ((rc = ensure_buf(h, h->strand_off, h->strand_off_cap, mo + 1))) return rc;
    HIPCHK(h, launch_strands(din, in_base, doff, m, mode, h->strand_off, total, h->strand_reads, s));
    // the staged copies are complete before the append plans on its own
    HIPCHK(h, hipStreamSynchronize(s));
    return bwt_set_append(h, h->strand_reads, h->strand_off, mo, stream);
}

int bwt_set_count_many(bwt_set_t h, const uint8_t *pats, const uint64_t *offsets,
                       uint64_t count, uint64_t *lo_out, uint64_t *hi_out, void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (count == 0) return BWT_OK;
    if (!pats || !offsets || !lo_out || !hi_out) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    IndexBuf &B = h->buf[h->cur];
    HIPCHK(h, launch_count(B.recs, B.sbc, B.meta, pats, offsets, count, lo_out, hi_out, s));
    return BWT_OK;
}

int64_t bwt_set_export(bwt_set_t h, uint8_t *out) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (!out || h->n == 0) return (int64_t)h->n;
    int rc = set_device(h);
    if (rc) return rc;
    IndexBuf &B = h->buf[h->cur];
    if (is_device_ptr(out)) {
        HIPCHK(h, launch_export(B.recs, h->n, out, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return (int64_t)h->n;
    }
    if ((rc = ensure_buf(h, h->stage_out, h->stage_out_cap, h->n))) return rc;
    HIPCHK(h, launch_export(B.recs, h->n, h->stage_out, h->stream));
    HIPCHK(h, hipMemcpyAsync(out, h->stage_out, h->n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return (int64_t)h->n;
}

int bwt_set_import(bwt_set_t h, const uint8_t *B, uint64_t n, void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (!B && n) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    const bool dev = n ? is_device_ptr(B) : true;
    // Built into the two buffers other than the current one, chunk by chunk,
    // each chunk merged after every row so far (g_sa = current size); a bad
    // byte stops the build before the current index is replaced.
    int other[2], k = 0;
    for (int b = 0; b < 3; ++b)
        if (b != h->cur) other[k++] = b;
    for (int b : other)
        if ((rc = ensure_index(h, h->buf[b], n))) return rc;
    const uint64_t CH = std::min<uint64_t>(std::max<uint64_t>(n, 1), 1ull << 26);
    if ((rc = ensure_ws(h, CH))) return rc;
    Workspace &w = h->ws;
    if ((rc = clear_err(h, s))) return rc;
    int src = other[0], dst = other[1];
    HIPCHK(h, launch_index_init(h->buf[src].recs, h->buf[src].sbc, h->buf[src].meta, s));
    uint64_t n_cur = 0;
    for (uint64_t o = 0; o < n; o += CH) {
        const uint64_t cnt = std::min(CH, n - o);
        const uint8_t *chunk = B + o;
        if (!dev) {
            if ((rc = ensure_buf(h, h->stage_reads, h->stage_reads_cap, CH + 16))) return rc;
            HIPCHK(h, hipMemcpyAsync(h->stage_reads, chunk, cnt, hipMemcpyHostToDevice, s));
            chunk = h->stage_reads;
        }
        HIPCHK(h, hipMemsetAsync(w.misc + MISC_BAD, 0, 4, s));
        HIPCHK(h, launch_fill_u64(w.kA, cnt, n_cur, s));
        HIPCHK(h, launch_check_user_insert(chunk, w.kA, cnt, n_cur, w.misc + MISC_BAD, s));
        uint32_t bad = 0;
        if ((rc = read_u32(h, s, w.misc + MISC_BAD, &bad))) return rc;
        if (bad) return fail(h, BWT_EINVAL);
        HIPCHK(h, launch_pack_user_insert(chunk, w.kA, cnt, 0, w.kA, w.v[0], s));
        if ((rc = insert_block(h, s, h->buf[src], h->buf[dst], n_cur, w.kA, 0, w.v[0], cnt, 0)))
            return rc;
        if (!dev) HIPCHK(h, hipStreamSynchronize(s));  // the staging buffer is reused
        n_cur += cnt;
        std::swap(src, dst);
    }
    HIPCHK(h, hipMemcpyAsync(h->pinned, h->buf[src].meta, META_WORDS * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (h->timer.on) timer_collect(h);
    const uint64_t new_m = h->pinned[5];
    if ((rc = check_err(h, s))) return rc;
    h->cur = src;
    h->n = n;
    h->m = new_m;
    return BWT_OK;
}

int bwt_set_memory(bwt_set_t h, uint64_t *bytes) {
    if (!h || !bytes) return BWT_EINVAL;
    uint64_t b = 0;
    for (auto &x : h->buf) {
        if (x.recs && !x.host) b += x.rec_cap * sizeof(Rec);
        if (x.sbc && !x.host) b += x.sbc_cap * 4 * 8;
        if (x.meta) b += META_WORDS * 8;
    }
    const Workspace &w = h->ws;
    if (w.region) b += w.bytes;
    b += h->first_new_cap * 8 + h->stage_reads_cap + h->stage_off_cap * 8 + h->cuts_cap * 8 +
         h->stage_out_cap + h->btab_cap + h->bstage_cap + h->strand_reads_cap +
         h->strand_off_cap * 8;
    for (auto *l : h->lanes) {
        uint64_t lb = 0;
        if (bwt_set_memory(l, &lb) == BWT_OK) b += lb;
    }
    *bytes = b;
    return BWT_OK;
}

int bwt_set_trim(bwt_set_t h) {
    if (!h) return BWT_EINVAL;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->pipe) pipe_free(*h->pipe);
    for (int b = 0; b < 3; ++b) {
        if (b == h->cur) continue;
        IndexBuf &x = h->buf[b];
        free_index_data(x);
        dfree(x.meta);
    }
    free_ws(h->ws);
    dfree(h->first_new);
    h->first_new_cap = 0;
    dfree(h->stage_reads);
    h->stage_reads_cap = 0;
    dfree(h->stage_off);
    h->stage_off_cap = 0;
    dfree(h->cuts);
    h->cuts_cap = 0;
    dfree(h->stage_out);
    h->stage_out_cap = 0;
    dfree(h->strand_reads);
    h->strand_reads_cap = 0;
    dfree(h->strand_off);
    h->strand_off_cap = 0;
    dfree(h->btab);
    h->btab_cap = 0;
    dfree(h->bstage);
    h->bstage_cap = 0;
    for (auto *l : h->lanes) bwt_set_destroy(l);
    h->lanes.clear();
    return BWT_OK;
}

int bwt_set_size(bwt_set_t h, uint64_t *n, uint64_t *m) {
    if (!h) return BWT_EINVAL;
    if (n) *n = h->n;
    if (m) *m = h->m;
    return BWT_OK;
}

int bwt_set_reset(bwt_set_t h) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    int rc = set_device(h);
    if (rc) return rc;
    IndexBuf &B = h->buf[h->cur];
    HIPCHK(h, launch_index_init(B.recs, B.sbc, B.meta, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->n = 0;
    h->m = 0;
    return BWT_OK;
}

int bwt_set_set_block_size(bwt_set_t h, uint64_t M) {
    if (!h) return BWT_EINVAL;
    if (M < 1) return fail(h, BWT_EINVAL);
    h->M = std::min<uint64_t>(M, MAX_BLOCK);
    return BWT_OK;
}

int bwt_set_set_param(bwt_set_t h, int param, int64_t value) {
    if (!h) return BWT_EINVAL;
    switch (param) {
    case BWT_PARAM_KEY_BITS:
        if (value < 16 || value > 64) return fail(h, BWT_EINVAL);
        h->key_bits = (int)value;
        return BWT_OK;
    case BWT_PARAM_RADIX_TILE:
        if (value < 0 || value >= RADIX_CFGS) return fail(h, BWT_EINVAL);
        h->radix_cfg = (int)value;
        return BWT_OK;
    case BWT_PARAM_RANK_SEGMENT:
        if (value != 0 && (value < (int64_t)MIN_SEG_LEN || value > (1 << 24)))
            return fail(h, BWT_EINVAL);
        h->seg_len = (uint32_t)value;
        return BWT_OK;
    case BWT_PARAM_RANK_OVERLAP:
        if (value < 0 || value > (1 << 24)) return fail(h, BWT_EINVAL);
        h->seg_overlap = (uint32_t)value;
        return BWT_OK;
    case BWT_PARAM_PIPELINE:
        if (value != 0 && value != 1) return fail(h, BWT_EINVAL);
        h->pipeline = value != 0;
        return BWT_OK;
    case BWT_PARAM_HOST_INDEX:
        if (value != 0 && value != 1) return fail(h, BWT_EINVAL);
        h->host_index = value != 0;
        return BWT_OK;
    case BWT_PARAM_GRAPH:
        if (value != 0 && value != 1) return fail(h, BWT_EINVAL);
        h->graph = value != 0;
        if (!h->graph) drop_graphs(h);
        return BWT_OK;
    case BWT_PARAM_SORT_BUCKETS:
        if (value != 0 && value != 1) return fail(h, BWT_EINVAL);
        h->sort_buckets = value != 0;
        return BWT_OK;
    case BWT_PARAM_BATCH_LANES:
        if (value < 1 || value > MAX_LANES) return fail(h, BWT_EINVAL);
        h->batch_lanes = (int)value;
        return BWT_OK;
    default:
        return fail(h, BWT_EINVAL);
    }
}

int bwt_set_last_error(bwt_set_t h) { return h ? h->last_error : g_create_error; }

const char *bwt_set_strerror(int code) {
    switch (code) {
    case BWT_OK: return "ok";
    case BWT_EINVAL: return "invalid argument";
    case BWT_ENOMEM: return "out of device memory";
    case BWT_EHIP: return "HIP runtime error";
    case BWT_EALPHABET: return "unsupported alphabet (only \"ACGT\")";
    case BWT_ESTATE: return "handle unusable after an earlier HIP error";
    default: return "unknown error";
    }
}

int bwt_set_block_sort(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets, uint64_t m,
                       uint32_t *sa_out, uint8_t *bint_out, void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (m == 0) return BWT_OK;
    if (!reads || !offsets || !sa_out || !bint_out) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    Plan P;
    if ((rc = plan_input(h, s, reads, offsets, m, MAX_BLOCK, P))) return rc;
    if (P.total_suffixes > MAX_BLOCK) return fail(h, BWT_EINVAL);
    if ((rc = ensure_ws(h, P.total_suffixes))) return rc;
    if ((rc = clear_err(h, s))) return rc;
    uint32_t *sa = nullptr;
    const uint64_t *gkeys = nullptr;
    int gshift = 64;
    const uint32_t n_blk = (uint32_t)P.total_suffixes;
    if ((rc = block_prep(h, s, P.off, (uint32_t)m, n_blk))) return rc;
    if ((rc = block_sort(h, s, P.reads, P.off, (uint32_t)m, n_blk, P.maxlen, nullptr, 0, false, &sa,
                         &gkeys, &gshift)))
        return rc;
    HIPCHK(h, launch_vals_to_ascii(sa, n_blk, bint_out, s));
    HIPCHK(h, launch_sa_strip(sa, n_blk, sa_out, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (h->timer.on) timer_collect(h);
    return check_err(h, s);
}

int bwt_set_block_sort_noalloc(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                               uint64_t m, uint32_t *sa_out, uint8_t *bint_out, void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (m == 0) return BWT_OK;
    if (!reads || !offsets || !sa_out || !bint_out) return fail(h, BWT_EINVAL);
    if (m > NOALLOC_MAX_SUFFIXES) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    if (h->device < 0 || h->device >= NOALLOC_MAX_DEVICES) return fail(h, BWT_EHIP);
    if (!is_device_ptr(reads) || !is_device_ptr(offsets) || !is_device_ptr(sa_out) ||
        !is_device_ptr(bint_out))
        return fail(h, BWT_EINVAL);
    std::lock_guard<std::mutex> g(g_scratch_mu[h->device]);
    uint8_t *base = g_scratch_ptr[h->device];
    if (!base) return fail(h, BWT_EHIP);
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    // offsets in order, the longest read, and the block size from the ends
    HIPCHK(h, launch_check_offsets(offsets, m, h->res, s));
    HIPCHK(h, hipMemcpyAsync(h->pinned, h->res, 2 * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(h->pinned + 2, offsets, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(h->pinned + 3, offsets + m, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    const uint64_t bad = h->pinned[0], maxlen = h->pinned[1], o0 = h->pinned[2],
                   o1 = h->pinned[3];
    if (bad || o1 < o0 || maxlen > MAX_READ) return fail(h, BWT_EINVAL);
    const uint64_t n64 = o1 - o0 + m;
    if (n64 > NOALLOC_MAX_SUFFIXES) return fail(h, BWT_EINVAL);
    const uint32_t n_blk = (uint32_t)n64;
    ScratchWs view(h, base);
    Workspace &w = h->ws;
    // the counters must start at zero; the look-back status words only need
    // it once (each launch tags them with a fresh epoch)
    HIPCHK(h, launch_zero_u32(w.misc, MISC_WORDS, s));
    if (g_scratch_fresh[h->device]) {
        const uint64_t tiles = div_up(NOALLOC_MAX_SUFFIXES, RADIX_MIN_TILE) + 1;
        HIPCHK(h, launch_zero_u32(reinterpret_cast<uint32_t *>(w.status_radix),
                                  (uint32_t)(tiles * 256 * 2), s));
        HIPCHK(h, launch_zero_u32(reinterpret_cast<uint32_t *>(w.status_scan),
                                  (uint32_t)(tiles * 8 * 2), s));
        g_scratch_fresh[h->device] = false;
    }
    uint32_t *sa = nullptr;
    const uint64_t *gkeys = nullptr;
    int gshift = 64;
    if ((rc = block_prep(h, s, offsets, (uint32_t)m, n_blk))) return rc;
    if ((rc = block_sort(h, s, reads, offsets, (uint32_t)m, n_blk, maxlen, nullptr, 0, false, &sa,
                         &gkeys, &gshift)))
        return rc;
    HIPCHK(h, launch_vals_to_ascii(sa, n_blk, bint_out, s));
    HIPCHK(h, launch_sa_strip(sa, n_blk, sa_out, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return check_err(h, s);
}

int bwt_set_compute_ranks(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets, uint64_t m,
                          uint64_t *g_out, void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (m == 0) return BWT_OK;
    if (!reads || !offsets || !g_out) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    Plan P;
    if ((rc = plan_input(h, s, reads, offsets, m, MAX_BLOCK, P))) return rc;
    if (P.total_suffixes > MAX_BLOCK) return fail(h, BWT_EINVAL);
    if ((rc = ensure_ws(h, P.total_suffixes))) return rc;
    IndexBuf &B = h->buf[h->cur];
    if ((rc = clear_err(h, s))) return rc;
    HIPCHK(h, launch_block_soff(P.off, (uint32_t)m, h->ws.soff, s));
    {
        MarkSet mk(h, 3);
        HIPCHK(h, launch_compute_ranks(P.reads, P.off, h->ws.soff, (uint32_t)m,
                                       (uint32_t)P.total_suffixes, B.recs, B.sbc, B.meta,
                                       h->n >= (1ull << SB_SHIFT) ? 1 : 0, g_out, nullptr,
                                       rank_segments(h, P.maxlen), h->ws.misc + MISC_ERR, s,
                                       mk.get()));
        mk.add(0, SPAN_RANKS_K, P.total_suffixes - m);
        mk.add(1, SPAN_RANKS_SEG, 0);
        mk.add(2, SPAN_RANKS_FB, 0);
    }
    HIPCHK(h, hipStreamSynchronize(s));
    if (h->timer.on) timer_collect(h);
    return check_err(h, s);
}

int bwt_set_insert(bwt_set_t h, const uint8_t *bint, const uint64_t *gsa, uint64_t n_new,
                   void *stream) {
    if (!h) return BWT_EINVAL;
    if (h->broken) return fail(h, BWT_ESTATE);
    if (n_new == 0) return BWT_OK;
    if (!bint || !gsa || n_new > MAX_BLOCK) return fail(h, BWT_EINVAL);
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    const uint64_t n_final = h->n + n_new;
    int dst = (h->cur + 1) % 3;
    if ((rc = ensure_index(h, h->buf[dst], n_final))) return rc;
    if ((rc = ensure_ws(h, n_new))) return rc;
    if ((rc = clear_err(h, s))) return rc;
    Workspace &w = h->ws;
    HIPCHK(h, hipMemsetAsync(w.misc + MISC_BAD, 0, 4, s));
    HIPCHK(h, launch_check_user_insert(bint, gsa, n_new, h->n, w.misc + MISC_BAD, s));
    uint32_t bad = 0;
    if ((rc = read_u32(h, s, w.misc + MISC_BAD, &bad))) return rc;
    if (bad) return fail(h, BWT_EINVAL);
    const int gbits = bits_for_value(h->n);
    const int gshift = gbits ? 64 - gbits : 64;
    HIPCHK(h, launch_pack_user_insert(bint, gsa, n_new, gshift, w.kA, w.v[0], s));
    if ((rc = insert_block(h, s, h->buf[h->cur], h->buf[dst], h->n, w.kA, gshift, w.v[0], n_new,
                            0)))
        return rc;
    // the number of terminators merged in comes from the new counts
    HIPCHK(h, hipMemcpyAsync(h->pinned, h->buf[dst].meta, META_WORDS * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (h->timer.on) timer_collect(h);
    uint64_t new_n = h->pinned[4], new_m = h->pinned[5];
    if ((rc = check_err(h, s))) return rc;
    h->cur = dst;
    h->n = new_n;
    h->m = new_m;
    return BWT_OK;
}

int bwt_set_enable_timing(bwt_set_t h, int on) {
    if (!h) return BWT_EINVAL;
    if (on && !h->timer.on && h->ws.misc) {
        // the device's running totals restart with the timing
        int rc = set_device(h);
        if (rc) return rc;
        HIPCHK(h, hipMemsetAsync(h->ws.misc + MISC_STATS, 0, 16, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    h->timer.on = on != 0;
    return BWT_OK;
}

int bwt_set_get_stats(bwt_set_t h, bwt_stats_t *out, int reset) {
    if (!h || !out) return BWT_EINVAL;
    *out = h->timer.acc;
    out->graph_captures = h->graph_captures;
    out->graph_replays = h->graph_replays;
    out->graph_redos = h->graph_redos;
    if (reset) {
        memset(&h->timer.acc, 0, sizeof h->timer.acc);
        h->graph_captures = h->graph_replays = h->graph_redos = 0;
    }
    return BWT_OK;
}

}  // extern "C"
