// k_ranks.hip -- ComputeRanks (Section 4, Lemma 1 and Algorithm 2).
//
// For each read P_j of the block, a walk from the read's end gives the rank
// of every suffix among the old ones: the terminator suffix $_j is larger than
// exactly the m_ext terminators already in B_ext and smaller than every old
// suffix that starts with a base, so the walk starts at i = m_ext; then for
// k = |P_j|-1 .. 0, with c = P_j[k], i := C[c] + rank(c, i, B_ext) (Lemma 1),
// and g[off_j + k] = i, where off_j is the exclusive prefix sum of |P_j| + 1
// (the block text position of the read's first symbol).  Each step is one
// random 64-byte record read from the HBM-resident index.
//
// A read of more than `seg` symbols is cut into segments of `seg` symbols so
// that its walk does not serialize the block.  The walk of segment [a, b)
// starts `ov` symbols past b as an FM-index backward search: it keeps the
// interval [lo, hi) of old suffixes (rows) prefixed by the symbols read so
// far, starting from all rows.  Once no old suffix has that prefix (lo ==
// hi), lo is exactly the number of old suffixes smaller than the new suffix,
// and the walk continues as Lemma 1's single rank.  A segment whose interval
// has not closed by the time it reaches b (a repeat longer than ov) starts
// once more from further out; if that fails too, it hands its read to a last
// kernel that walks the whole read from its end, so the result is exact in
// every case.  When the queue has room, the short reads of a block with long
// ones are queued as one segment each, so that every walk of the block runs
// in the one launch (a walk takes as long as its dependent steps, so a lane
// walking a read alone while the segments wait would add its whole length).
#include "dev_util.hpp"

namespace bwt {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The values of one lane are written in descending order; they are kept in
// an N-entry shift register and written as one aligned chunk of 128 bytes
// when the register covers indices [Nq, Nq + N), so the writes are whole
// cache lines instead of single words spread over the cache (partial chunks
// at both ends of a walk are written word by word).  Plain stores: under the
// walks' random reads, non-temporal stores of the same chunks cut the rate
// of reads that the memory system sustains, and 128-byte chunks cost less
// than 64-byte ones (measured with dependent random reads beside streaming
// stores of each kind).
template <class T, int N>
struct OutBuf {
    static_assert(N * sizeof(T) == 128, "one cache line per chunk");
    static constexpr int SIZE = N;
    T r[N];  // r[0] = lowest index held
    uint32_t cnt;
    __device__ void push(T v) {
#pragma unroll
        for (int q = N - 1; q > 0; --q) r[q] = r[q - 1];
        r[0] = v;
        cnt = cnt < (uint32_t)N ? cnt + 1 : (uint32_t)N;
    }
    // write the held values to p[idx .. idx + cnt)
    __device__ void flush(T *__restrict__ p, uint64_t idx, bool vec) {
        if (cnt == (uint32_t)N && vec) {
            u32x4 *q = reinterpret_cast<u32x4 *>(p + idx);
            if constexpr (sizeof(T) == 8) {
#pragma unroll
                for (int c = 0; c < N / 2; ++c)
                    q[c] = u32x4{(uint32_t)r[2 * c], (uint32_t)(r[2 * c] >> 32),
                                 (uint32_t)r[2 * c + 1], (uint32_t)(r[2 * c + 1] >> 32)};
            } else {
#pragma unroll
                for (int c = 0; c < N / 4; ++c)
                    q[c] = u32x4{r[4 * c], r[4 * c + 1], r[4 * c + 2], r[4 * c + 3]};
            }
        } else {
#pragma unroll
            for (int q = 0; q < N; ++q)
                if ((uint32_t)q < cnt) p[idx + q] = r[q];
        }
        cnt = 0;
    }
};
using GBuf = OutBuf<uint64_t, 16>;  // g values or sort keys
using VBuf = OutBuf<uint32_t, 32>;  // sort values
constexpr uint64_t GMASK = GBuf::SIZE - 1, VMASK = VBuf::SIZE - 1;

// Where the walks write.  g mode (keys == nullptr): g[p] for every block
// position p.  Key mode: the first sort key of p, g << gshift | the next
// kfirst symbols << 5 | their count (the key launch_block_keys builds), and
// its sort value p | (previous symbol, 4 at a read start) << 29.
struct Out {
    uint64_t *g;
    uint64_t *keys;
    uint32_t *vals;
    int gshift, kfirst;
    bool vec, vvec;  // 128-byte aligned arrays: whole chunks may be written
    uint32_t *hist;  // key mode: counts of the key digit at bit hshift (or null)
    int hshift;
};

// The 8-byte word of packed input holding the current symbol, reloaded only
// when the walk crosses into the previous word.
struct SymReader {
    const uint8_t *base;
    uintptr_t wa;
    uint64_t word;
    __device__ int get(uint64_t s) {
        uintptr_t addr = (uintptr_t)base + (uintptr_t)(s >> 2);
        uintptr_t a0 = addr & ~(uintptr_t)7;
        if (a0 != wa) {
            word = *reinterpret_cast<const uint64_t *>(a0);
            wa = a0;
        }
        return (int)(word >> ((addr - a0) * 8 + 2 * (s & 3))) & 3;
    }
};

// C[c] and the size of B_ext, read from the index meta words
struct LF {
    uint64_t C0, C1, C2, C3, m_ext, n_ext;
    bool big;
    uint32_t *err;
    __device__ LF(const uint64_t *__restrict__ meta, int big_, uint32_t *err_) {
        m_ext = meta[5];
        n_ext = meta[4];
        C0 = m_ext;               // every terminator is smaller than A
        C1 = C0 + meta[0];
        C2 = C1 + meta[1];
        C3 = C2 + meta[2];
        big = big_ != 0;
        err = err_;
    }
    // Lemma 1: C[c] + rank(c, i, B_ext), at most n_ext in a consistent
    // index.  A larger value means counts and symbols disagree: the call is
    // failed through the err word (bit 1024), and the walk goes on clamped so
    // that it stays inside the index.  Against an empty index every rank is 0
    // (no record is read).
    __device__ uint64_t step(const Rec *__restrict__ recs, const uint64_t *__restrict__ sbc,
                             uint64_t i, int c) const {
        if (n_ext == 0) return 0;
        uint64_t Cc = c == 0 ? C0 : c == 1 ? C1 : c == 2 ? C2 : C3;
        uint64_t r = Cc + rank_base(recs, sbc, i, c, big);
        if (r > n_ext) {
            atomicOr(err, 1024u);
            r = n_ext;
        }
        return r;
    }
};

// The index a read is ranked against, and the offset added to its ranks.
struct Walker {
    const Rec *recs;
    const uint64_t *sbc;
    LF lf;
    uint64_t goff;
};

// Every read of the block against one index.
struct OneIndex {
    const Rec *recs;
    const uint64_t *sbc;
    const uint64_t *meta;
    int big;
    uint32_t *err;
    __device__ Walker at(uint32_t) const { return Walker{recs, sbc, LF(meta, big, err), 0}; }
};

// Read j against the index of its unit (the last unit with read0 <= j).
struct UnitIndex {
    const RankUnit *units;
    uint32_t n;
    uint32_t *err;
    __device__ Walker at(uint32_t j) const {
        uint32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (units[mid].read0 <= j) lo = mid;
            else hi = mid - 1;
        }
        const RankUnit &u = units[lo];
        return Walker{u.recs, u.sbc, LF(u.meta, (int)u.big, err), u.goff};
    }
};

// Whole-read walk from the terminator: writes the results of positions
// gb + len .. gb (terminator first).  In key mode the walk keeps the kfirst
// symbols after the current position in `win` (first symbol most
// significant), and writes each position's value one step late, once the
// symbol before it has been read.
// sh (key mode, may be null): LDS counts of the digit at bit o.hshift of
// every key written.
template <bool KEYS>
__device__ void walk_read(const Walker &W, SymReader &sym, uint64_t s0, uint32_t len, uint64_t gb,
                          const Out &o, uint32_t *sh) {
    GBuf buf;
    buf.cnt = 0;
    VBuf vb;
    vb.cnt = 0;
    uint64_t *dst = KEYS ? o.keys : o.g;
    uint64_t win = 0;
    const int top = 2 * (o.kfirst - 1);
    uint64_t i = W.lf.m_ext;
    uint32_t k = len;
    buf.push(KEYS ? (i + W.goff) << o.gshift : i + W.goff);  // terminator: no symbols
    if (KEYS && sh) atomicAdd(&sh[(uint32_t)(buf.r[0] >> o.hshift) & 255u], 1u);
    if (((gb + k) & GMASK) == 0) buf.flush(dst, gb + k, o.vec);
    while (k > 0) {
        --k;
        const int c = sym.get(s0 + k);
        i = W.lf.step(W.recs, W.sbc, i, c);
        if constexpr (KEYS) {
            vb.push((uint32_t)(gb + k + 1) | ((uint32_t)c << POS_BITS));
            if (((gb + k + 1) & VMASK) == 0) vb.flush(o.vals, gb + k + 1, o.vvec);
            if (o.kfirst > 0) win = (win >> 2) | ((uint64_t)c << top);
            const uint32_t t = len - k < (uint32_t)o.kfirst ? len - k : (uint32_t)o.kfirst;
            const uint64_t key = ((i + W.goff) << o.gshift) | (win << KEY_LEN_BITS) | t;
            buf.push(key);
            if (sh) atomicAdd(&sh[(uint32_t)(key >> o.hshift) & 255u], 1u);
        } else {
            buf.push(i + W.goff);
        }
        if (((gb + k) & GMASK) == 0) buf.flush(dst, gb + k, o.vec);
    }
    buf.flush(dst, gb, false);  // what is left below the last aligned index
    if constexpr (KEYS) {
        vb.push((uint32_t)gb | (4u << POS_BITS));  // the read's first position
        vb.flush(o.vals, gb, false);
    }
}

// One lane per read.  Reads longer than `seg` symbols (seg > 0) are cut into
// segments that are queued for rank_segments_kernel instead; with queue_all,
// every read is queued (a short read as one segment, which that kernel walks
// exactly from its terminator), so that no lane walks a read here while the
// segments wait for this launch to end.
// In key mode with o.hist set, the digit counts of the keys of the walked
// reads are gathered in LDS and added once per workgroup to one of the
// HIST_COPIES copies (the keys of queued reads are counted by the segment
// and whole-read kernels that write them).
template <class Src, bool KEYS>
__global__ __launch_bounds__(256) void compute_ranks_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, uint32_t m_blk, Src src, Out o, uint32_t seg,
    bool queue_all, uint64_t *__restrict__ seg_list, uint32_t *__restrict__ seg_count,
    uint32_t seg_cap, unsigned long long *__restrict__ seg_syms, uint32_t *__restrict__ err) {
    __shared__ uint32_t s_h[KEYS ? 256 : 1];
    const uint32_t tid = threadIdx.x;
    const bool count = KEYS && o.hist != nullptr;
    if (count) {
        s_h[tid] = 0;
        __syncthreads();
    }
    const uint32_t j = blockIdx.x * blockDim.x + tid;
    uint64_t s0 = 0;
    uint32_t len = 0, nseg = 0;
    if (j < m_blk) {
        s0 = off[j];
        len = (uint32_t)(off[j + 1] - s0);
        if (seg > 0 && (len > seg || queue_all)) nseg = len > seg ? (len + seg - 1) / seg : 1u;
    }
    // Queue places are reserved once per wave (one atomic on the shared
    // counter per 64 reads instead of one per read): every lane of the wave
    // takes part, queued or not.  The queued symbols are summed in two 16-bit
    // halves so that the wave's sums cannot overflow 32 bits.
    {
        const uint32_t lane = tid & (WAVE - 1);
        const uint32_t qlen = nseg ? len : 0u;
        const uint32_t incl = wave_incl_sum(nseg);
        const uint32_t sum_lo = wave_incl_sum(qlen & 0xffffu);
        const uint32_t sum_hi = wave_incl_sum(qlen >> 16);
        uint32_t base = 0;
        if (lane == WAVE - 1 && incl) {
            base = atomicAdd(seg_count, incl);
            atomicAdd(seg_syms, (unsigned long long)sum_lo + ((unsigned long long)sum_hi << 16));
        }
        base = __shfl(base, WAVE - 1, WAVE);
        if (nseg) {
            const uint32_t at = base + incl - nseg;
            if ((uint64_t)at + nseg > seg_cap) {
                atomicOr(err, 128u);
            } else {
                for (uint32_t s = 0; s < nseg; ++s) seg_list[at + s] = ((uint64_t)j << 32) | s;
            }
        }
    }
    if (j < m_blk && nseg == 0) {
        {
            SymReader sym{reads, 0, 0};
            walk_read<KEYS>(src.at(j), sym, s0, len, soff[j], o, count ? s_h : nullptr);
        }
    }
    if (count) {
        __syncthreads();
        if (s_h[tid]) atomicAdd(&o.hist[(blockIdx.x % HIST_COPIES) * 256 + tid], s_h[tid]);
    }
}

// Key mode: a key whose length field has every bit set never occurs (the
// field holds at most kfirst); a segment that hands its read to the
// whole-read walk fills its positions with it.
constexpr uint64_t NO_KEY = ~0ull;

// Queued segment t, (j, s) of a long read: symbols [a, b) with a = s * seg,
// b = min(len, a + seg); the walk starts at e = min(len, b + ov).  Its keys
// are written only once its interval has closed at its first own position,
// after which the walk is exact, so every key it writes is final (the
// whole-read walk of a read that falls back writes the same values there):
// sh (key mode, may be null) counts their digits at bit o.hshift.
template <class Src, bool KEYS>
__device__ void rank_segment(const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
                             const uint32_t *__restrict__ soff, uint32_t m_blk, Src src,
                             const Out &o, uint32_t seg, uint32_t ov,
                             const uint64_t *__restrict__ seg_list, uint32_t t,
                             uint32_t *__restrict__ fb_flag, uint32_t *__restrict__ fb_list,
                             uint32_t *__restrict__ fb_count, uint32_t *__restrict__ stats,
                             uint32_t *__restrict__ err, uint32_t *sh) {
    const uint64_t e_js = seg_list[t];
    const uint32_t j = (uint32_t)(e_js >> 32), s = (uint32_t)e_js;
    if (j >= m_blk) {  // only if the queue overflowed (already flagged)
        atomicOr(err, 128u);
        return;
    }
    const uint64_t s0 = off[j];
    const uint32_t len = (uint32_t)(off[j + 1] - s0);
    const uint64_t gb = soff[j];
    if (s > 0 && (uint64_t)s * seg >= len) {  // (an empty read is queued as segment 0)
        atomicOr(err, 128u);
        return;
    }
    const Walker W = src.at(j);
    const LF &lf = W.lf;
    const uint32_t a = s * seg;
    const uint32_t b = a + seg < len ? a + seg : len;
    uint64_t *dst = KEYS ? o.keys : o.g;
    SymReader sym{reads, 0, 0};
    GBuf buf;
    buf.cnt = 0;
    VBuf vb;
    vb.cnt = 0;
    const int top = 2 * (o.kfirst - 1);
    // First attempt with overlap ov; a segment whose interval is still open at
    // b (a repeat longer than ov) starts again RETRY_FACTOR1, then
    // RETRY_FACTOR2, times further out before its read is handed to the
    // whole-read walk.  Nothing of the
    // segment has been written when the interval is found open (that happens
    // at its first position), so a restart only resets the walk.
    uint32_t ovs = ov;
    for (int attempt = 0;; ++attempt) {
        const uint32_t e = len - b > ovs ? b + ovs : len;
        uint64_t win = 0;
        if (KEYS && o.kfirst > 0) {
            // the symbols a key of [a, b) needs beyond the walk's start
            const uint32_t need = b + (uint32_t)o.kfirst < len ? b + (uint32_t)o.kfirst : len;
            for (uint32_t q = need; q > e;) {
                --q;
                win = (win >> 2) | ((uint64_t)sym.get(s0 + q) << top);
            }
        }
        uint64_t lo, hi;
        if (e == len) {
            lo = hi = lf.m_ext;  // exact start at the terminator suffix
            if (b == len) {
                buf.push(KEYS ? (lo + W.goff) << o.gshift : lo + W.goff);
                if (KEYS && sh) atomicAdd(&sh[(uint32_t)(buf.r[0] >> o.hshift) & 255u], 1u);
                if (((gb + len) & GMASK) == 0) buf.flush(dst, gb + len, o.vec);
            }
        } else {
            lo = 0;             // the empty prefix: every row of B_ext
            hi = lf.n_ext;
        }
        bool open = false;
        uint32_t k = e;
        while (k > a) {
            --k;
            const int c = sym.get(s0 + k);
            const uint64_t nlo = lf.step(W.recs, W.sbc, lo, c);
            hi = (lo == hi) ? nlo : lf.step(W.recs, W.sbc, hi, c);
            lo = nlo;
            if (KEYS && o.kfirst > 0) win = (win >> 2) | ((uint64_t)c << top);
            if (k < b) {
                if (lo != hi) {
                    open = true;
                    break;
                }
                if constexpr (KEYS) {
                    if (k + 1 < b || k + 1 == len) {
                        vb.push((uint32_t)(gb + k + 1) | ((uint32_t)c << POS_BITS));
                        if (((gb + k + 1) & VMASK) == 0) vb.flush(o.vals, gb + k + 1, o.vvec);
                    }
                    const uint32_t tt = len - k < (uint32_t)o.kfirst ? len - k : (uint32_t)o.kfirst;
                    const uint64_t key = ((lo + W.goff) << o.gshift) | (win << KEY_LEN_BITS) | tt;
                    buf.push(key);
                    if (sh) atomicAdd(&sh[(uint32_t)(key >> o.hshift) & 255u], 1u);
                } else {
                    buf.push(lo + W.goff);
                }
                if (((gb + k) & GMASK) == 0) buf.flush(dst, gb + k, o.vec);
            }
        }
        if (!open) break;
        if (attempt > 1 || e == len) {
            // a repeat longer than the retry's overlap: the whole read is
            // walked exactly.  Nothing of this segment has been written or
            // counted; its positions get NO_KEY so that the whole-read walk
            // can tell the counted keys of the read's other segments.
            if constexpr (KEYS)
                for (uint32_t q = a; q < b; ++q) o.keys[gb + q] = NO_KEY;
            if (atomicExch(&fb_flag[j], 1u) == 0u) {
                fb_list[atomicAdd(fb_count, 1u)] = j;
                atomicAdd(stats + 1, 1u);
            }
            return;
        }
        const uint32_t f = attempt == 0 ? RETRY_FACTOR1 : RETRY_FACTOR2;
        const uint32_t mn = attempt == 0 ? RETRY_MIN1 : RETRY_MIN2;
        ovs = ov > (1u << 24) ? (1u << 28) : (ov * f > mn ? ov * f : mn);
        atomicAdd(stats, 1u);
    }
    buf.flush(dst, gb + a, false);
    if constexpr (KEYS) {
        const uint32_t prev = a > 0 ? (uint32_t)sym.get(s0 + a - 1) : 4u;
        vb.push((uint32_t)(gb + a) | (prev << POS_BITS));
        vb.flush(o.vals, gb + a, false);
    }
}

// One lane per queued segment.  In key mode with o.hist set, the digit
// counts of the keys written are gathered in LDS and added once per
// workgroup to one of the HIST_COPIES copies.
template <class Src, bool KEYS>
__global__ __launch_bounds__(256) void rank_segments_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, uint32_t m_blk, Src src, Out o, uint32_t seg, uint32_t ov,
    const uint64_t *__restrict__ seg_list, const uint32_t *__restrict__ seg_count,
    uint32_t *__restrict__ fb_flag, uint32_t *__restrict__ fb_list,
    uint32_t *__restrict__ fb_count, uint32_t *__restrict__ stats, uint32_t *__restrict__ err) {
    __shared__ uint32_t s_h[KEYS ? 256 : 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t nq = *seg_count;
    if (blockIdx.x * blockDim.x >= nq) return;  // the whole workgroup
    const bool count = KEYS && o.hist != nullptr;
    if (count) {
        s_h[tid] = 0;
        __syncthreads();
    }
    const uint32_t t = blockIdx.x * blockDim.x + tid;
    if (t < nq)
        rank_segment<Src, KEYS>(reads, off, soff, m_blk, src, o, seg, ov, seg_list, t, fb_flag,
                                fb_list, fb_count, stats, err, count ? s_h : nullptr);
    if (count) {
        __syncthreads();
        if (s_h[tid]) atomicAdd(&o.hist[(blockIdx.x % HIST_COPIES) * 256 + tid], s_h[tid]);
    }
}

// Whole-read walks for the reads whose segments could not close their
// interval within the overlap.  In key mode with o.hist set, the keys its
// other segments wrote (every position not NO_KEY) were counted already:
// their digits are taken off before the walk counts every key of the read.
template <class Src, bool KEYS>
__global__ __launch_bounds__(256) void rank_fallback_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, Src src, Out o, const uint32_t *__restrict__ fb_list,
    const uint32_t *__restrict__ fb_count) {
    __shared__ uint32_t s_h[KEYS ? 256 : 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t nf = *fb_count;
    if (blockIdx.x * blockDim.x >= nf) return;  // the whole workgroup
    const bool count = KEYS && o.hist != nullptr;
    if (count) {
        s_h[tid] = 0;
        __syncthreads();
    }
    const uint32_t t = blockIdx.x * blockDim.x + tid;
    if (t < nf) {
        const uint32_t j = fb_list[t];
        const uint64_t s0 = off[j];
        const uint32_t len = (uint32_t)(off[j + 1] - s0);
        const uint64_t gb = soff[j];
        if (count)
            for (uint32_t q = 0; q <= len; ++q) {
                const uint64_t key = o.keys[gb + q];
                if (key != NO_KEY) atomicSub(&s_h[(uint32_t)(key >> o.hshift) & 255u], 1u);
            }
        SymReader sym{reads, 0, 0};
        walk_read<KEYS>(src.at(j), sym, s0, len, gb, o, count ? s_h : nullptr);
    }
    if (count) {
        __syncthreads();
        if (s_h[tid]) atomicAdd(&o.hist[(blockIdx.x % HIST_COPIES) * 256 + tid], s_h[tid]);
    }
}

__global__ void zero_kernel(uint32_t *p, uint32_t n) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <class Src, bool KEYS>
hipError_t compute_ranks(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                         uint32_t m_blk, uint32_t n_blk, Src src, const Out &o,
                         const RankSegments &sg, uint32_t *err, hipStream_t s, const Marks *mk) {
    uint32_t seg = sg.seg_len;
    uint32_t cap = 0;
    bool queue_all = false;
    if (seg > 0) {
        cap = (uint32_t)(2 * div_up(n_blk, seg) + 2);
        // every read in the queue when it has room (a segment per short read)
        const uint64_t all = (uint64_t)m_blk + div_up(n_blk, seg) + 2;
        if (all <= sg.seg_cap) {
            queue_all = true;
            cap = (uint32_t)all;
        } else if (cap > sg.seg_cap) {
            seg = 0;  // no room to queue segments: whole-read walks
        }
    }
    if (seg > 0) {
        zero_kernel<<<1, 64, 0, s>>>(sg.counters, 2);
        zero_kernel<<<(unsigned)div_up(m_blk, 256), 256, 0, s>>>(sg.fb_flag, m_blk);
    }
    Marks::begin(mk, 0, s);
    compute_ranks_kernel<Src, KEYS><<<(unsigned)div_up(m_blk, 256), 256, 0, s>>>(
        reads, off, soff, m_blk, src, o, seg, queue_all, sg.seg_list, sg.counters, cap,
        reinterpret_cast<unsigned long long *>(sg.stats + 2), err);
    Marks::end(mk, 0, s);
    Marks::begin(mk, 1, s);
    if (seg > 0)
        rank_segments_kernel<Src, KEYS><<<(unsigned)div_up(cap, 256), 256, 0, s>>>(
            reads, off, soff, m_blk, src, o, seg, sg.overlap, sg.seg_list, sg.counters, sg.fb_flag,
            sg.fb_list, sg.counters + 1, sg.stats, err);
    Marks::end(mk, 1, s);
    Marks::begin(mk, 2, s);
    if (seg > 0) {
        rank_fallback_kernel<Src, KEYS><<<(unsigned)div_up(m_blk, 256), 256, 0, s>>>(
            reads, off, soff, src, o, sg.fb_list, sg.counters + 1);
    }
    Marks::end(mk, 2, s);
    return hipGetLastError();
}

template <class Src>
hipError_t compute_ranks_any(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                             uint32_t m_blk, uint32_t n_blk, Src src, uint64_t *g,
                             const RankKeys *kk, const RankSegments &sg, uint32_t *err,
                             hipStream_t s, const Marks *mk) {
    if (m_blk == 0) return hipSuccess;
    Out o{};
    if (kk) {
        o.keys = kk->keys;
        o.vals = kk->vals;
        o.gshift = kk->gshift;
        o.kfirst = kk->kfirst;
        o.vec = (reinterpret_cast<uintptr_t>(o.keys) & 127) == 0;
        o.vvec = (reinterpret_cast<uintptr_t>(o.vals) & 127) == 0;
        o.hist = kk->hist;
        o.hshift = kk->hshift;
        return compute_ranks<Src, true>(reads, off, soff, m_blk, n_blk, src, o, sg, err, s, mk);
    }
    o.g = g;
    o.vec = (reinterpret_cast<uintptr_t>(g) & 127) == 0;
    return compute_ranks<Src, false>(reads, off, soff, m_blk, n_blk, src, o, sg, err, s, mk);
}

}  // namespace

hipError_t launch_compute_ranks(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                                uint32_t m_blk, uint32_t n_blk, const Rec *recs,
                                const uint64_t *sbc, const uint64_t *meta, int big, uint64_t *g,
                                const RankKeys *kk, const RankSegments &sg, uint32_t *err,
                                hipStream_t s, const Marks *mk) {
    return compute_ranks_any(reads, off, soff, m_blk, n_blk, OneIndex{recs, sbc, meta, big, err},
                             g, kk, sg, err, s, mk);
}

hipError_t launch_compute_ranks_units(const uint8_t *reads, const uint64_t *off,
                                      const uint32_t *soff, uint32_t m_blk, uint32_t n_blk,
                                      const RankUnit *units, uint32_t nunits, uint64_t *g,
                                      const RankKeys *kk, const RankSegments &sg, uint32_t *err,
                                      hipStream_t s, const Marks *mk) {
    if (nunits == 0) return hipSuccess;
    return compute_ranks_any(reads, off, soff, m_blk, n_blk, UnitIndex{units, nunits, err}, g,
                             kk, sg, err, s, mk);
}

}  // namespace bwt
