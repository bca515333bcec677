// k_query.hip -- rank queries (Eq. 2), export of B, the device-side checks
// and block split of an append whose offsets live in device memory, and the
// staging of a batch of sets into one packed input.
#include "dev_util.hpp"

namespace bwt {

namespace {

__global__ void rank_many_kernel(const Rec *__restrict__ recs, const uint64_t *__restrict__ sbc,
                                 const uint64_t *__restrict__ meta, const uint8_t *__restrict__ cs,
                                 const uint64_t *__restrict__ ks, uint64_t *__restrict__ out,
                                 uint64_t count) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint64_t n = meta[4];
    const uint64_t k = ks[t];
    const uint8_t ch = cs[t];
    uint64_t r = ~0ull;
    if (k <= n) {
        int c = ch == 'A' ? 0 : ch == 'C' ? 1 : ch == 'G' ? 2 : ch == 'T' ? 3 : ch == '$' ? 4 : 5;
        if (c < 4) {
            r = rank_base(recs, sbc, k, c, true);
        } else if (c == 4) {
            // a row is either a base or a terminator
            r = k;
            for (int b = 0; b < 4; ++b) r -= rank_base(recs, sbc, k, b, true);
        }
    }
    out[t] = r;
}

// FM-index count by backward search: Lemma 1's step C[c] + rank(c, i) taken
// at both ends of the interval of rows whose suffixes start with the symbols
// read so far (Section 2: the BWT and its rank function, Eq. 2, form an
// FM-index).  Pattern t is symbols [poff[t], poff[t+1]) of the 2-bit packed
// pats, read from its last symbol; the interval starts as all n rows.  On
// return [lo, hi) are the rows whose suffix starts with the pattern: hi - lo
// occurrences, lo suffixes smaller than the pattern.  Once the interval is
// empty its ends move together, so one rank per step is enough.
__global__ void count_kernel(const Rec *__restrict__ recs, const uint64_t *__restrict__ sbc,
                             const uint64_t *__restrict__ meta, const uint8_t *__restrict__ pats,
                             const uint64_t *__restrict__ poff, uint64_t count,
                             uint64_t *__restrict__ lo_out, uint64_t *__restrict__ hi_out) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint64_t a = poff[t], b = poff[t + 1];
    if (b < a) {
        lo_out[t] = hi_out[t] = ~0ull;
        return;
    }
    const uint64_t C0 = meta[5];            // every terminator sorts before A
    const uint64_t C1 = C0 + meta[0], C2 = C1 + meta[1], C3 = C2 + meta[2];
    uint64_t lo = 0, hi = meta[4];
    for (uint64_t k = b; k > a;) {
        --k;
        const int c = load_sym(pats, k);
        const uint64_t Cc = c == 0 ? C0 : c == 1 ? C1 : c == 2 ? C2 : C3;
        const uint64_t nlo = Cc + rank_base(recs, sbc, lo, c, true);
        hi = lo == hi ? nlo : Cc + rank_base(recs, sbc, hi, c, true);
        lo = nlo;
    }
    lo_out[t] = lo;
    hi_out[t] = hi;
}

// A bounded grid strides over the rows, so indices of 2^32 symbols and more
// (beyond one launch's 32-bit work-item count) are covered.
__global__ void export_kernel(const Rec *__restrict__ recs, uint64_t n, uint8_t *__restrict__ out) {
    const char ascii[5] = {'A', 'C', 'G', 'T', '$'};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (uint8_t)ascii[rec_symbol(recs, i)];
}

__global__ void zero_words_kernel(uint64_t *p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

// res[0] |= 1 if offsets decrease somewhere; res[1] = longest read.  A fixed
// grid strides over the reads and each workgroup adds once, so the two
// result words see one atomic per workgroup.
__global__ __launch_bounds__(256) void check_offsets_kernel(const uint64_t *__restrict__ off,
                                                            uint64_t m,
                                                            uint64_t *__restrict__ res) {
    __shared__ uint64_t s_len[4];
    __shared__ uint32_t s_bad[4];
    uint64_t len = 0;
    bool bad = false;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
         j += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t a = off[j], b = off[j + 1];
        if (b < a) bad = true;
        else len = (b - a) > len ? (b - a) : len;
    }
    for (int d = 32; d > 0; d >>= 1) {
        uint64_t o = __shfl_xor(len, d, 64);
        len = o > len ? o : len;
    }
    const int w = threadIdx.x >> 6;
    const bool anybad = __ballot(bad) != 0;
    if (lane_id() == 0) {
        s_len[w] = len;
        s_bad[w] = anybad ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t L = 0;
        uint32_t B = 0;
        for (int k = 0; k < 4; ++k) {
            L = s_len[k] > L ? s_len[k] : L;
            B |= s_bad[k];
        }
        if (B) atomicOr((unsigned long long *)&res[0], 1ull);
        if (L) atomicMax((unsigned long long *)&res[1], (unsigned long long)L);
    }
}

// Greedy block split (Algorithm 1 blocks: whole reads, at most M suffixes,
// a read with more than M suffixes alone).  S(j) = off[j] - off[0] + j is the
// block-text position of read j.  With cuts, writes cuts[2k] = first read of
// block k, cuts[2k+1] = S(first read).  Returns the number of blocks.
__device__ uint64_t greedy_cuts(const uint64_t *__restrict__ off, uint64_t m, uint64_t M,
                                uint64_t *__restrict__ cuts) {
    const uint64_t o0 = off[0];
    uint64_t j = 0, K = 0;
    if (cuts) {
        cuts[0] = 0;
        cuts[1] = 0;
    }
    while (j < m) {
        const uint64_t Sj = off[j] - o0 + j;
        // largest k in [j+1, m] with S(k) - S(j) <= M, at least j+1
        uint64_t lo = j + 1, hi = m;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo + 1) / 2;
            uint64_t Sm = off[mid] - o0 + mid;
            if (Sm - Sj <= M) lo = mid;
            else hi = mid - 1;
        }
        j = lo;
        ++K;
        if (cuts) {
            cuts[2 * K] = j;
            cuts[2 * K + 1] = off[j] - o0 + j;
        }
    }
    return K;
}

// res[2] = number of blocks.  One thread.
__global__ void plan_blocks_kernel(const uint64_t *__restrict__ off, uint64_t m, uint64_t M,
                                   uint64_t *__restrict__ cuts, uint64_t *__restrict__ res) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    res[2] = greedy_cuts(off, m, M, cuts);
}

// One workgroup per set of a batch: the offsets check, the suffix count and
// the block count, and the cuts when a cut area is given.
__global__ __launch_bounds__(256) void plan_sets_kernel(const PlanSet *__restrict__ sets,
                                                        uint64_t M, uint64_t *__restrict__ res,
                                                        uint64_t *__restrict__ cuts) {
    __shared__ uint64_t s_len[4];
    __shared__ uint32_t s_bad[4];
    const PlanSet ps = sets[blockIdx.x];
    uint64_t len = 0;
    bool bad = false;
    for (uint64_t j = threadIdx.x; j < ps.m; j += blockDim.x) {
        uint64_t a = ps.off[j], b = ps.off[j + 1];
        if (b < a) bad = true;
        else len = (b - a) > len ? (b - a) : len;
    }
    for (int d = 32; d > 0; d >>= 1) {
        uint64_t o = __shfl_xor(len, d, 64);
        len = o > len ? o : len;
    }
    const int w = threadIdx.x >> 6;
    const bool anybad = __ballot(bad) != 0;
    if (lane_id() == 0) {
        s_len[w] = len;
        s_bad[w] = anybad ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t L = 0;
        uint32_t B = 0;
        for (int k = 0; k < 4; ++k) {
            L = s_len[k] > L ? s_len[k] : L;
            B |= s_bad[k];
        }
        uint64_t *r = res + 4ull * blockIdx.x;
        r[0] = B;
        r[1] = L;
        // a decreasing offsets array has no meaningful split
        r[2] = B ? 0 : ps.off[ps.m] - ps.off[0] + ps.m;
        r[3] = B ? 0 : greedy_cuts(ps.off, ps.m, M, cuts ? cuts + ps.cut_base : nullptr);
    }
}

// last unit with key(unit) <= x, for keys non-decreasing over units
template <class Key>
__device__ uint32_t last_unit_at_or_below(const GatherUnit *__restrict__ units, uint32_t n,
                                          uint64_t x, Key key) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (key(units[mid]) <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// staged offsets: entry r of unit u = dst_sym0 + off[j0 + r - dst_read0] - off[j0];
// the last entry is the total symbol count
__global__ void gather_offsets_kernel(const GatherUnit *__restrict__ units, uint32_t nunits,
                                      uint64_t total_reads, uint64_t total_syms,
                                      uint64_t *__restrict__ dst_off) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > total_reads) return;
    if (r == total_reads) {
        dst_off[r] = total_syms;
        return;
    }
    const uint32_t u = last_unit_at_or_below(units, nunits, r,
                                             [](const GatherUnit &g) { return g.dst_read0; });
    const GatherUnit &g = units[u];
    dst_off[r] = g.dst_sym0 + (g.off[g.j0 + (r - g.dst_read0)] - g.off[g.j0]);
}

// staged reads: one thread per 16 symbols (one 32-bit word) of the output
__global__ void gather_reads_kernel(const GatherUnit *__restrict__ units, uint32_t nunits,
                                    uint64_t total_syms, uint32_t *__restrict__ dst) {
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t q0 = w * 16;
    if (q0 >= total_syms) return;
    uint32_t u = last_unit_at_or_below(units, nunits, q0,
                                       [](const GatherUnit &g) { return g.dst_sym0; });
    uint64_t d0 = units[u].dst_sym0, s0 = units[u].off[units[u].j0] - units[u].sym_base;
    const uint8_t *src = units[u].reads;
    uint64_t next = u + 1 < nunits ? units[u + 1].dst_sym0 : ~0ull;
    uint32_t word = 0;
    for (int k = 0; k < 16; ++k) {
        const uint64_t q = q0 + k;
        if (q >= total_syms) break;
        while (q >= next) {  // later units (skipping units without symbols)
            ++u;
            d0 = units[u].dst_sym0;
            s0 = units[u].off[units[u].j0] - units[u].sym_base;
            src = units[u].reads;
            next = u + 1 < nunits ? units[u + 1].dst_sym0 : ~0ull;
        }
        const uint64_t p = s0 + (q - d0);
        word |= (uint32_t)((src[p >> 2] >> (2 * (p & 3))) & 3u) << (2 * k);
    }
    dst[w] = word;
}

// Strand variants of an input (Section 2 notes that the strings may also be
// indexed reversed).  mode 1: every read written backwards; mode 2: every
// read followed by its reverse complement (read backwards, code x -> 3 - x),
// so output string 2j is read j and 2j + 1 its reverse complement.  Output
// offsets start at 0; input symbol p is at p - in_base of `in`.
__global__ void strand_offsets_kernel(const uint64_t *__restrict__ off, uint64_t m, int mode,
                                      uint64_t *__restrict__ out_off) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > m) return;
    const uint64_t x = off[j] - off[0];
    if (mode == 2) {
        out_off[2 * j] = 2 * x;
        if (j < m) out_off[2 * j + 1] = 2 * x + (off[j + 1] - off[j]);
    } else {
        out_off[j] = x;
    }
}

// one thread per 16 output symbols (one 32-bit word of the packed output)
__global__ void strand_pack_kernel(const uint8_t *__restrict__ in, uint64_t in_base,
                                   const uint64_t *__restrict__ off, int mode,
                                   const uint64_t *__restrict__ out_off, uint64_t mo,
                                   uint64_t total, uint32_t *__restrict__ dst) {
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t q0 = w * 16;
    if (q0 >= total) return;
    // the last output string starting at or before q0
    uint64_t lo = 0, hi = mo - 1;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (out_off[mid] <= q0) lo = mid;
        else hi = mid - 1;
    }
    uint64_t r = lo;
    uint32_t word = 0;
    for (int k = 0; k < 16; ++k) {
        const uint64_t q = q0 + k;
        if (q >= total) break;
        while (q >= out_off[r + 1]) ++r;  // later strings (skipping empty ones)
        const uint64_t j = mode == 2 ? r >> 1 : r;
        const bool rc = mode == 2 && (r & 1);
        const bool rev = mode == 1 || rc;
        const uint64_t a = off[j], len = off[j + 1] - a, t = q - out_off[r];
        const uint64_t p = (rev ? a + len - 1 - t : a + t) - in_base;
        uint32_t c = (in[p >> 2] >> (2 * (p & 3))) & 3u;
        if (rc) c = 3u - c;
        word |= c << (2 * k);
    }
    dst[w] = word;
}

}  // namespace

hipError_t launch_strands(const uint8_t *in, uint64_t in_base, const uint64_t *off, uint64_t m,
                          int mode, uint64_t *out_off, uint64_t total, uint8_t *out,
                          hipStream_t s) {
    if (m == 0) return hipSuccess;
    strand_offsets_kernel<<<(unsigned)div_up(m + 1, 256), 256, 0, s>>>(off, m, mode, out_off);
    const uint64_t mo = mode == 2 ? 2 * m : m;
    if (total > 0) {
        const uint64_t words = div_up(total, 16);
        strand_pack_kernel<<<(unsigned)div_up(words, 256), 256, 0, s>>>(
            in, in_base, off, mode, out_off, mo, total, reinterpret_cast<uint32_t *>(out));
    }
    return hipGetLastError();
}

hipError_t launch_rank_many(const Rec *recs, const uint64_t *sbc, const uint64_t *meta,
                            const uint8_t *cs, const uint64_t *ks, uint64_t *out, uint64_t count,
                            hipStream_t s) {
    if (count == 0) return hipSuccess;
    rank_many_kernel<<<(unsigned)div_up(count, 256), 256, 0, s>>>(recs, sbc, meta, cs, ks, out,
                                                                  count);
    return hipGetLastError();
}

hipError_t launch_count(const Rec *recs, const uint64_t *sbc, const uint64_t *meta,
                        const uint8_t *pats, const uint64_t *poff, uint64_t count,
                        uint64_t *lo, uint64_t *hi, hipStream_t s) {
    if (count == 0) return hipSuccess;
    count_kernel<<<(unsigned)div_up(count, 256), 256, 0, s>>>(recs, sbc, meta, pats, poff, count,
                                                              lo, hi);
    return hipGetLastError();
}

hipError_t launch_export(const Rec *recs, uint64_t n, uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t want = div_up(n, 256);
    export_kernel<<<(unsigned)(want < (1u << 20) ? want : (1u << 20)), 256, 0, s>>>(recs, n, out);
    return hipGetLastError();
}

// res: 4 words, cleared here
hipError_t launch_check_offsets(const uint64_t *off, uint64_t m, uint64_t *res, hipStream_t s) {
    zero_words_kernel<<<1, 64, 0, s>>>(res, 4);
    if (m > 0) {
        uint64_t want = div_up(m, 256 * 8);
        unsigned grid = (unsigned)(want < 1024 ? (want > 0 ? want : 1) : 1024);
        check_offsets_kernel<<<grid, 256, 0, s>>>(off, m, res);
    }
    return hipGetLastError();
}

hipError_t launch_plan_blocks(const uint64_t *off, uint64_t m, uint64_t M, uint64_t *cuts,
                              uint64_t *res, hipStream_t s) {
    plan_blocks_kernel<<<1, 64, 0, s>>>(off, m, M, cuts, res);
    return hipGetLastError();
}

hipError_t launch_plan_sets(const PlanSet *sets, uint32_t nsets, uint64_t M, uint64_t *res,
                            uint64_t *cuts, hipStream_t s) {
    if (nsets == 0) return hipSuccess;
    plan_sets_kernel<<<nsets, 256, 0, s>>>(sets, M, res, cuts);
    return hipGetLastError();
}

hipError_t launch_gather_offsets(const GatherUnit *units, uint32_t nunits, uint64_t total_reads,
                                 uint64_t total_syms, uint64_t *dst_off, hipStream_t s) {
    if (nunits == 0) return hipSuccess;
    gather_offsets_kernel<<<(unsigned)div_up(total_reads + 1, 256), 256, 0, s>>>(
        units, nunits, total_reads, total_syms, dst_off);
    return hipGetLastError();
}

// dst must hold ceil(total_syms / 16) 32-bit words
hipError_t launch_gather_reads(const GatherUnit *units, uint32_t nunits, uint64_t total_syms,
                               uint8_t *dst, hipStream_t s) {
    if (nunits == 0 || total_syms == 0) return hipSuccess;
    const uint64_t words = div_up(total_syms, 16);
    gather_reads_kernel<<<(unsigned)div_up(words, 256), 256, 0, s>>>(
        units, nunits, total_syms, reinterpret_cast<uint32_t *>(dst));
    return hipGetLastError();
}

}  // namespace bwt
