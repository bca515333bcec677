// k_insert.hip -- Insert of Algorithm 1 / Section 5 and the rebuild of the
// occurrence counters, as one streaming merge from the old index into a new
// one in HBM.
//
// New symbol i (in suffix order) lands at output row g_sa[i] + i: g_sa is
// non-decreasing, so g_sa[i] + i is strictly increasing, and old row r lands at
// r + |{i : g_sa[i] <= r}|.  The output is cut into tiles of 16 records (2048
// rows); a tile finds by binary search how many new symbols precede it (a0),
// so it knows that old rows o0 = q0 - a0 ... follow, marks its new rows in an
// LDS bitmap, and fills every row from either B_int or the old records.  The
// counts stored in each record follow from the counts at the tile start,
//   count(c, q0) = rank(c, o0, B_ext) + rank(c, a0, B_int),
// plus popcounts inside the tile, so tiles never wait on each other.
// rank(c, a, B_int) comes from counts sampled every 64 symbols of B_int.
#include "dev_util.hpp"

namespace bwt {

namespace {

// ASCII symbol -> 0..3 for A,C,G,T, 4 for '$', 5 otherwise
__device__ __forceinline__ int code_of_ascii(uint8_t ch) {
    switch (ch) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    case '$': return 4;
    default: return 5;
    }
}

__global__ void index_init_kernel(Rec *recs, uint64_t *sbc, uint64_t *meta) {
    int t = threadIdx.x;
    if (t < 16) reinterpret_cast<uint32_t *>(recs)[t] = 0;
    if (t < 4) sbc[t] = 0;
    if (t < META_WORDS) meta[t] = 0;
}

// g_sa[i] sits in the key bits from gshift up (gshift = 64: no g, all zero);
// in a block of several units the key holds g_sa + goff (unit offset)
__device__ __forceinline__ uint64_t gsa_at(const uint64_t *__restrict__ gkeys, int gshift,
                                           uint64_t i, uint64_t goff = 0) {
    return gshift < 64 ? (gkeys[i] >> gshift) - goff : 0ull;
}

__device__ __forceinline__ int code_at(const uint32_t *__restrict__ vals, uint64_t i) {
    return (int)(vals[i] >> POS_BITS);
}

// count of base c among the first 64k sorted symbols of the block
__device__ __forceinline__ uint64_t bint_sample(const BintCounts &bc, uint64_t k, int c) {
    return (uint64_t)bc.chunk[k * 4 + c] + bc.seg[(k >> BINT_SEG_SHIFT) * 4 + c];
}

// occurrences of base c among the first a sorted symbols of the block
__device__ uint64_t rank_bint(const uint32_t *__restrict__ vals, const BintCounts &bcnt,
                              uint64_t a, int c) {
    uint64_t r = bint_sample(bcnt, a >> CHUNK_SHIFT, c);
    for (uint64_t x = a & ~63ull; x < a; ++x) r += (code_at(vals, x) == c);
    return r;
}

// One unit's share of an Insert: its n_new symbols are the sorted slots
// [sa0, sa0 + n_new) of the block (vals, bcnt and gkeys cover the block).
struct InsJob {
    const Rec *orecs;
    const uint64_t *osbc;
    Rec *nrecs;
    const uint64_t *nsbc;
    const uint64_t *gkeys;
    const uint32_t *vals;
    BintCounts bcnt;
    const uint64_t *first_new;   // the unit's tiles' entries
    uint64_t n_ext, n_new, sa0, goff;
    int gshift;
};

// first i in [0, n_new) of the unit with g_sa[i] + i >= Q (n_new if none)
__device__ uint64_t first_at_or_after(const uint64_t *__restrict__ gkeys, int gshift,
                                      uint64_t sa0, uint64_t goff, uint64_t n_new, uint64_t Q) {
    uint64_t lo = 0, hi = n_new;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (gsa_at(gkeys, gshift, sa0 + mid, goff) + mid >= Q) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Counts of each base per chunk of 64 sorted symbols, one workgroup of 16
// waves per segment of 1024 chunks (65,536 symbols): chunk[k] = counts in the
// segment before chunk k, and stot[seg] = the segment's totals.  Wave w counts
// the chunks w*64 .. w*64 + 63 of the segment, 16 rows of 64 symbols at a
// time, so every wave has 16 loads in flight and a short serial part.  The
// chunk after the last (k = ceil(n/64)) is written by the segment it falls in.
constexpr int BINT_WAVES = 16;
constexpr int BINT_WCH = (1 << BINT_SEG_SHIFT) / BINT_WAVES;  // chunks per wave

__global__ __launch_bounds__(BINT_WAVES * 64) void count_bint_kernel(
    const uint32_t *__restrict__ vals, uint32_t n, uint32_t nch, uint32_t *__restrict__ chunk,
    uint32_t *__restrict__ stot) {
    __shared__ uint32_t s_pre[1 << BINT_SEG_SHIFT][4];
    __shared__ uint32_t s_wt[BINT_WAVES][4];
    __shared__ uint32_t s_wb[BINT_WAVES][4];  // counts of the waves before
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t seg = blockIdx.x;
    const uint32_t k0 = seg << BINT_SEG_SHIFT;
    uint32_t run[4] = {0, 0, 0, 0};
    for (uint32_t r0 = 0; r0 < (uint32_t)BINT_WCH; r0 += 16) {
        int c[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t kl = (uint32_t)wave * BINT_WCH + r0 + e;  // chunk inside the segment
            const uint64_t x = (uint64_t)(k0 + kl) * 64 + lane;
            c[e] = x < n ? code_at(vals, x) : 6;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t kl = (uint32_t)wave * BINT_WCH + r0 + e;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (lane == q) s_pre[kl][q] = run[q];
                run[q] += (uint32_t)__popcll(__ballot(c[e] == q));
            }
        }
    }
    if (lane < 4) s_wt[wave][lane] = lane == 0 ? run[0] : lane == 1 ? run[1] : lane == 2 ? run[2] : run[3];
    __syncthreads();
    if (tid < 4 * BINT_WAVES) {
        const uint32_t w = tid >> 2, b = tid & 3;
        uint32_t off = 0;
        for (uint32_t v = 0; v < w; ++v) off += s_wt[v][b];
        s_wb[w][b] = off;
        if (w == BINT_WAVES - 1) stot[seg * 4 + b] = off + s_wt[w][b];
    }
    __syncthreads();
    // 1024 chunks x 4 bases = 4096 words, 4 per thread; a chunk adds the
    // counts of the waves before its own
    for (uint32_t i = tid; i < 4u << BINT_SEG_SHIFT; i += BINT_WAVES * 64) {
        const uint32_t kl = i >> 2, b = i & 3, w = kl / BINT_WCH;
        const uint32_t k = k0 + kl;
        if (k <= nch) chunk[(uint64_t)k * 4 + b] = s_wb[w][b] + s_pre[kl][b];
    }
}

// Exclusive scan of the segment totals (one workgroup of 1024 threads, at
// most 8 segments each): seg[s] = counts before segment s, seg[nseg] = all.
__global__ __launch_bounds__(1024) void bint_seg_scan_kernel(const uint32_t *__restrict__ stot,
                                                             uint32_t nseg,
                                                             uint32_t *__restrict__ seg) {
    __shared__ uint32_t s_w[16][4];
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t per = (nseg + 1023) / 1024;
    for (int b = 0; b < 4; ++b) {
        uint32_t sum = 0;
        for (uint32_t q = 0; q < per; ++q) {
            const uint32_t s_ = tid * per + q;
            if (s_ < nseg) sum += stot[s_ * 4 + b];
        }
        const uint32_t inc = wave_incl_sum(sum);
        if ((tid & 63) == 63) s_w[w][b] = inc;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (uint32_t k = 0; k < 16; ++k) {
            before += k < w ? s_w[k][b] : 0u;
            all += s_w[k][b];
        }
        uint32_t run = before + inc - sum;
        for (uint32_t q = 0; q < per; ++q) {
            const uint32_t s_ = tid * per + q;
            if (s_ < nseg) seg[s_ * 4 + b] = run;
            if (s_ < nseg) run += stot[s_ * 4 + b];
        }
        if (tid == 0) seg[nseg * 4 + b] = all;
        __syncthreads();
    }
}

// user-supplied Insert input: *bad |= 1 for a byte outside "ACGT$", 2 for a
// g_sa value that decreases or exceeds n_ext
__global__ void check_user_insert_kernel(const uint8_t *__restrict__ bint,
                                         const uint64_t *__restrict__ gsa, uint64_t n_new,
                                         uint64_t n_ext, uint32_t *__restrict__ bad) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_new) return;
    uint64_t v = gsa[i];
    if (v > n_ext || (i > 0 && gsa[i - 1] > v)) atomicOr(bad, 2u);
    if (code_of_ascii(bint[i]) > 4) atomicOr(bad, 1u);
}

__global__ void pack_user_insert_kernel(const uint8_t *__restrict__ bint,
                                        const uint64_t *__restrict__ gsa, uint64_t n_new, int gshift,
                                        uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_new) return;
    keys[i] = gshift < 64 ? gsa[i] << gshift : 0ull;
    vals[i] = (uint32_t)code_of_ascii(bint[i]) << POS_BITS;
}

// first_new[t] = number of new symbols whose output row is below t * 2048
__global__ void ins_tile_first_kernel(const uint64_t *__restrict__ gkeys, int gshift,
                                      uint64_t n_new, uint64_t ntiles,
                                      uint64_t *__restrict__ first_new) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    first_new[t] = first_at_or_after(gkeys, gshift, 0, 0, n_new, t * INS_TILE_SYMS);
}

// first_new of every unit of a block: entry e belongs to the last unit u with
// tile0[u] + u <= e, and is that unit's entry e - tile0[u] - u
__global__ void ins_tile_first_units_kernel(const InsertUnit *__restrict__ units,
                                            uint32_t nunits, const uint64_t *__restrict__ gkeys,
                                            int gshift, uint64_t nentries,
                                            uint64_t *__restrict__ first_new) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nentries) return;
    uint32_t lo = 0, hi = nunits - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (units[mid].tile0 + mid <= e) lo = mid;
        else hi = mid - 1;
    }
    const InsertUnit &u = units[lo];
    const uint64_t t = e - u.tile0 - lo;
    first_new[e] = first_at_or_after(gkeys, gshift, u.sa0, u.goff, u.n_new, t * INS_TILE_SYMS);
}


// New totals, n, m and superblock base counts of one merged index (one
// thread; the number of superblocks is n / 2^32 + 1).
__device__ void ins_meta_one(const Rec *__restrict__ orecs, const uint64_t *__restrict__ osbc,
                             const uint64_t *__restrict__ ometa, const uint64_t *__restrict__ gkeys,
                             int gshift, const uint32_t *__restrict__ vals,
                             const BintCounts bcnt, uint64_t sa0, uint64_t goff,
                             uint64_t n_new, uint64_t *__restrict__ nsbc,
                             uint64_t *__restrict__ nmeta) {
    uint64_t base[4];
    for (int c = 0; c < 4; ++c) base[c] = rank_bint(vals, bcnt, sa0, c);
    uint64_t add = 0;
    for (int c = 0; c < 4; ++c) {
        uint64_t t = rank_bint(vals, bcnt, sa0 + n_new, c) - base[c];
        nmeta[c] = ometa[c] + t;
        add += t;
    }
    const uint64_t n_out = ometa[4] + n_new;
    nmeta[4] = n_out;
    nmeta[5] = ometa[5] + (n_new - add);
    nmeta[6] = 0;
    nmeta[7] = 0;
    const uint64_t nsb = (n_out >> SB_SHIFT) + 1;
    for (int c = 0; c < 4; ++c) nsbc[c] = 0;
    for (uint64_t sb = 1; sb < nsb; ++sb) {
        const uint64_t Q = sb << SB_SHIFT;
        const uint64_t lo = first_at_or_after(gkeys, gshift, sa0, goff, n_new, Q);
        const uint64_t o = Q - lo;
        for (int c = 0; c < 4; ++c)
            nsbc[sb * 4 + c] = rank_base(orecs, osbc, o, c, true) +
                               (rank_bint(vals, bcnt, sa0 + lo, c) - base[c]);
    }
}

__global__ void ins_meta_kernel(const Rec *__restrict__ orecs, const uint64_t *__restrict__ osbc,
                                const uint64_t *__restrict__ ometa,
                                const uint64_t *__restrict__ gkeys, int gshift,
                                const uint32_t *__restrict__ vals,
                                const BintCounts bcnt, uint64_t n_new,
                                uint64_t *__restrict__ nsbc, uint64_t *__restrict__ nmeta) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ins_meta_one(orecs, osbc, ometa, gkeys, gshift, vals, bcnt, 0, 0, n_new, nsbc, nmeta);
}

// one thread per unit
__global__ void ins_meta_units_kernel(const InsertUnit *__restrict__ units, uint32_t nunits,
                                      const uint64_t *__restrict__ gkeys, int gshift,
                                      const uint32_t *__restrict__ vals,
                                      const BintCounts bcnt) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nunits) return;
    const InsertUnit &u = units[k];
    ins_meta_one(u.orecs, u.osbc, u.ometa, gkeys, gshift, vals, bcnt, u.sa0, u.goff, u.n_new,
                 u.nsbc, u.nmeta);
}

// LDS of one wave's tile.
struct InsLds {
    uint32_t bm[INS_TILE_SYMS / 32];           // bit per output row: a new symbol goes there
    uint8_t nsym[INS_TILE_SYMS];                // codes of the tile's new symbols, in order
    uint64_t old[(INS_TILE_RECS + 1) * 6];      // planes of the old records the tile reads
    uint64_t base[4];                           // counts of A, C, G, T before the tile
};

// Output tile t of one unit, by one wave: lane l builds rows 32l .. 32l + 31
// of the tile's 16 records (one 32-bit word of each bit plane) and writes
// 4 of the 256 words.
__device__ __forceinline__ void insert_tile(const InsJob &J, uint64_t t, InsLds &L,
                                            uint32_t *__restrict__ err) {
    const Rec *__restrict__ orecs = J.orecs;
    const uint64_t *__restrict__ osbc = J.osbc;
    const uint64_t *__restrict__ gkeys = J.gkeys;
    const uint32_t *__restrict__ vals = J.vals;
    const BintCounts bcnt = J.bcnt;
    const int gshift = J.gshift;
    const uint64_t sa0 = J.sa0, goff = J.goff;
    Rec *__restrict__ nrecs = J.nrecs;
    const uint64_t *__restrict__ nsbc = J.nsbc;
    const uint64_t n_out = J.n_ext + J.n_new;
    const uint64_t nrec_out = records_for(n_out);
    const uint64_t nrec_in = records_for(J.n_ext);
    const int lane = lane_id();

    const uint64_t R0 = t * INS_TILE_RECS;
    const uint64_t nrec = (nrec_out - R0) < (uint64_t)INS_TILE_RECS ? (nrec_out - R0) : INS_TILE_RECS;
    const uint64_t q0 = R0 * REC_SYMS;
    const uint64_t q1 = (q0 + INS_TILE_SYMS) < n_out ? (q0 + INS_TILE_SYMS) : n_out;
    const uint64_t a0 = J.first_new[t], a1 = J.first_new[t + 1];
    const uint64_t o0 = q0 - a0;                     // old rows before the tile
    const uint64_t nold = (q1 - q0) - (a1 - a0);     // old rows inside it
    const uint64_t r_lo = o0 >> REC_SHIFT;
    const uint32_t nr_old = nold ? (uint32_t)(((o0 + nold - 1) >> REC_SHIFT) - r_lo + 1) : 0u;
    // a consistent split never trips these; they keep a broken one in bounds
    if (a1 < a0 || a0 > q0 || o0 > J.n_ext || a1 - a0 > INS_TILE_SYMS ||
        nr_old > INS_TILE_RECS + 1 || (nr_old && r_lo + nr_old > nrec_in)) {
        if (lane == 0) atomicOr(err, 32u);
        return;
    }
    // Every load the tile needs depends only on a0 and a1, so all of them
    // go out here, before any result is used: the old records' planes, the
    // first eight rows of new symbols, the B_int samples and partial chunks
    // and the rank at o0 for the counts at the tile start, and the
    // superblock base of this lane's output record.
    const uint64_t A = sa0 + a0;
    const int cb = lane & 3;
    uint64_t ow[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        // at most (INS_TILE_RECS + 1) * 6 = 102 words: two per lane
        const uint32_t k = (uint32_t)lane + 64u * e;
        ow[e] = k < nr_old * 6
                    ? reinterpret_cast<const uint64_t *>(orecs + r_lo + k / 6)[2 + k % 6]
                    : 0ull;
    }
    constexpr int NB = 8;
    uint64_t gk[NB];
    uint32_t vv[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        const uint64_t i = a0 + (uint64_t)e * 64 + lane;
        gk[e] = i < a1 ? gkeys[sa0 + i] : 0ull;
        vv[e] = i < a1 ? vals[sa0 + i] : 0u;
    }
    const uint64_t x = (A & ~63ull) + lane;
    const uint64_t y = (sa0 & ~63ull) + lane;
    const uint32_t vx = x < A ? vals[x] : (6u << POS_BITS);
    const uint32_t vy = y < sa0 ? vals[y] : (6u << POS_BITS);
    const uint64_t sA = bint_sample(bcnt, A >> CHUNK_SHIFT, cb);
    const uint64_t s0 = bint_sample(bcnt, sa0 >> CHUNK_SHIFT, cb);
    const uint64_t rb = rank_base(orecs, osbc, o0, cb, true);
    const uint64_t r = (uint64_t)(lane >> 2);
    const uint64_t R = R0 + r;
    const uint64_t sbase = r < nrec ? nsbc[((R * REC_SYMS) >> SB_SHIFT) * 4 + cb] : 0ull;

    L.bm[lane] = 0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const uint32_t k = (uint32_t)lane + 64u * e;
        if (k < nr_old * 6) L.old[k] = ow[e];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // the tile's new symbols, eight rows of 64 at a time (the first rows are
    // already loaded; later ones, if any, have their loads issued together)
    for (uint64_t i0 = a0; i0 < a1; i0 += NB * 64) {
        if (i0 != a0) {
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                const uint64_t i = i0 + (uint64_t)e * 64 + lane;
                gk[e] = i < a1 ? gkeys[sa0 + i] : 0ull;
                vv[e] = i < a1 ? vals[sa0 + i] : 0u;
            }
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const uint64_t i = i0 + (uint64_t)e * 64 + lane;
            if (i < a1) {
                const uint64_t g = gshift < 64 ? (gk[e] >> gshift) - goff : 0ull;
                const uint64_t pos = g + i - q0;
                if (pos < INS_TILE_SYMS) atomicOr(&L.bm[pos >> 5], 1u << (pos & 31));
                else atomicOr(err, 32u);
                L.nsym[i - a0] = (uint8_t)(vv[e] >> POS_BITS);
            }
        }
    }
    {
        // counts at the tile start: old part by a rank on B_ext, new part from
        // the sampled B_int counts plus the < 64 symbols since the sample
        // (taken at the unit's first slot too, and subtracted)
        const int c = (int)(vx >> POS_BITS), d = (int)(vy >> POS_BITS);
        const uint32_t cA = __popcll(__ballot(c == 0)), cC = __popcll(__ballot(c == 1));
        const uint32_t cG = __popcll(__ballot(c == 2)), cT = __popcll(__ballot(c == 3));
        const uint32_t dA = __popcll(__ballot(d == 0)), dC = __popcll(__ballot(d == 1));
        const uint32_t dG = __popcll(__ballot(d == 2)), dT = __popcll(__ballot(d == 3));
        if (lane < 4) {
            const uint32_t part = lane == 0 ? cA : lane == 1 ? cC : lane == 2 ? cG : cT;
            const uint32_t part0 = lane == 0 ? dA : lane == 1 ? dC : lane == 2 ? dG : dT;
            L.base[lane] = (sA + part) - (s0 + part0) + rb;
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // this lane's 32 output rows: q0 + 32 * lane .. + 31
    const uint32_t word = L.bm[lane];
    const uint32_t nnew = (uint32_t)__popc(word);
    // (every lane of the wave is active from here: its exits are wave-uniform)
    uint32_t nb = wave_incl_sum_dpp(nnew) - nnew;          // new symbols before this lane
    uint64_t ob = o0 + 32ull * lane - nb - r_lo * REC_SYMS;  // old row, relative to record r_lo
    const uint64_t ql = q0 + 32ull * lane;
    const uint32_t nvalid = ql < q1 ? (q1 - ql < 32 ? (uint32_t)(q1 - ql) : 32u) : 0u;
    const uint32_t vmask0 = nvalid >= 32 ? 0xffffffffu : ((1u << nvalid) - 1u);
    // The lane's old rows come in order from bit ob of each plane of the
    // staged records: one 32-bit window per plane.  Every new row then opens
    // a gap at its place (lowest first) that takes the new symbol.
    uint32_t lo_w = 0, hi_w = 0, dl_w = 0;
    if ((uint32_t)__popc(word & vmask0) < nvalid) {
        constexpr uint32_t NW = (INS_TILE_RECS + 1) * 6;
        const uint32_t sh = (uint32_t)(ob & 63);
        const uint32_t r0 = (uint32_t)(ob >> 7), h0 = (uint32_t)(ob >> 6) & 1u;
        const uint32_t r1 = (uint32_t)((ob + 64) >> 7), h1 = (uint32_t)((ob + 64) >> 6) & 1u;
        uint32_t win[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
            uint32_t i0 = r0 * 6 + 2 * pl + h0, i1 = r1 * 6 + 2 * pl + h1;
            i0 = i0 < NW ? i0 : NW - 1;  // only rows past the tile's old rows get clamped
            i1 = i1 < NW ? i1 : NW - 1;
            const uint64_t w0 = L.old[i0], w1 = L.old[i1];
            win[pl] = (uint32_t)(sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0);
        }
        lo_w = win[0];
        hi_w = win[1];
        dl_w = win[2];
    }
    {
        uint32_t m = word & vmask0, k = nb;
        while (m) {
            const uint32_t u = (uint32_t)__builtin_ctz(m);
            m &= m - 1u;
            const uint32_t below = (1u << u) - 1u;
            lo_w = (lo_w & below) | ((lo_w & ~below) << 1);
            hi_w = (hi_w & below) | ((hi_w & ~below) << 1);
            dl_w = (dl_w & below) | ((dl_w & ~below) << 1);
            const int sym = L.nsym[k < INS_TILE_SYMS ? k : INS_TILE_SYMS - 1];
            ++k;
            if (sym == 4) dl_w |= 1u << u;
            else {
                lo_w |= (uint32_t)(sym & 1) << u;
                hi_w |= (uint32_t)(sym >> 1) << u;
            }
        }
    }
    lo_w &= vmask0;
    hi_w &= vmask0;
    dl_w &= vmask0;
    const uint32_t vmask = nvalid >= 32 ? 0xffffffffu : ((1u << nvalid) - 1u);
    // counts of each base before this lane's rows, then at each record start
    // (the record of lane l is l / 4; its first lane is l & ~3)
    uint64_t before[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t a = (c & 1) ? lo_w : ~lo_w, b = (c & 2) ? hi_w : ~hi_w;
        const uint32_t m = (uint32_t)__popc(a & b & ~dl_w & vmask);
        before[c] = L.base[c] + (wave_incl_sum_dpp(m) - m);
    }
    const int first = lane & ~3, k = lane & 3;
    uint64_t rec_before[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        rec_before[c] = (uint64_t)__shfl((long long)before[c], first, 64);
    if (r < nrec) {
        const uint64_t cabs = k == 0 ? rec_before[0] : k == 1 ? rec_before[1] : k == 2 ? rec_before[2] : rec_before[3];
        uint32_t *out = reinterpret_cast<uint32_t *>(nrecs) + R * 16;
        out[k] = (uint32_t)(cabs - sbase);
        out[4 + k] = lo_w;
        out[8 + k] = hi_w;
        out[12 + k] = dl_w;
    }
}

// four tiles per workgroup, one per wave
__global__ __launch_bounds__(256) void insert_kernel(InsJob J, uint64_t ntiles,
                                                     uint32_t *__restrict__ err) {
    __shared__ InsLds s_l[4];
    const int wave = threadIdx.x >> 6;
    const uint64_t t = (uint64_t)blockIdx.x * 4 + wave;
    if (t >= ntiles) return;
    insert_tile(J, t, s_l[wave], err);
}

// tiles of every unit, one per wave: tile T belongs to the last unit with
// tile0 <= T
__global__ __launch_bounds__(256) void insert_units_kernel(
    const InsertUnit *__restrict__ units, uint32_t nunits, const uint64_t *__restrict__ gkeys,
    int gshift, const uint32_t *__restrict__ vals, const BintCounts bcnt,
    const uint64_t *__restrict__ first_new, uint64_t ntiles_all, uint32_t *__restrict__ err) {
    __shared__ InsLds s_l[4];
    const int wave = threadIdx.x >> 6;
    const uint64_t T = (uint64_t)blockIdx.x * 4 + wave;
    if (T >= ntiles_all) return;
    uint32_t lo = 0, hi = nunits - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (units[mid].tile0 <= T) lo = mid;
        else hi = mid - 1;
    }
    const InsertUnit &u = units[lo];
    InsJob J;
    J.orecs = u.orecs;
    J.osbc = u.osbc;
    J.nrecs = u.nrecs;
    J.nsbc = u.nsbc;
    J.gkeys = gkeys;
    J.vals = vals;
    J.bcnt = bcnt;
    J.first_new = first_new + u.tile0 + lo;
    J.n_ext = u.n_ext;
    J.n_new = u.n_new;
    J.sa0 = u.sa0;
    J.goff = u.goff;
    J.gshift = gshift;
    insert_tile(J, T - u.tile0, s_l[wave], err);
}

__global__ void fill_u64_kernel(uint64_t *__restrict__ p, uint64_t n, uint64_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    fill_u64_kernel<<<(unsigned)div_up(n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_index_init(Rec *recs, uint64_t *sbc, uint64_t *meta, hipStream_t s) {
    index_init_kernel<<<1, 64, 0, s>>>(recs, sbc, meta);
    return hipGetLastError();
}

hipError_t launch_count_bint(const uint32_t *vals, uint32_t n, uint32_t *chunk, uint32_t *seg,
                             hipStream_t s) {
    const uint32_t nch = (uint32_t)div_up(n, 64);
    const uint32_t nseg = (nch >> BINT_SEG_SHIFT) + 1;  // the end chunk included
    // segment totals go after the scanned bases (nseg + 1 entries)
    uint32_t *stot = seg + 4 * (uint64_t)(nseg + 1);
    count_bint_kernel<<<nseg, BINT_WAVES * 64, 0, s>>>(vals, n, nch, chunk, stot);
    bint_seg_scan_kernel<<<1, 1024, 0, s>>>(stot, nseg, seg);
    return hipGetLastError();
}

hipError_t launch_check_user_insert(const uint8_t *bint, const uint64_t *gsa, uint64_t n_new,
                                   uint64_t n_ext, uint32_t *bad, hipStream_t s) {
    if (n_new == 0) return hipSuccess;
    check_user_insert_kernel<<<(unsigned)div_up(n_new, 256), 256, 0, s>>>(bint, gsa, n_new, n_ext,
                                                                          bad);
    return hipGetLastError();
}

hipError_t launch_pack_user_insert(const uint8_t *bint, const uint64_t *gsa, uint64_t n_new,
                                  int gshift, uint64_t *keys, uint32_t *vals, hipStream_t s) {
    if (n_new == 0) return hipSuccess;
    pack_user_insert_kernel<<<(unsigned)div_up(n_new, 256), 256, 0, s>>>(bint, gsa, n_new, gshift,
                                                                         keys, vals);
    return hipGetLastError();
}

hipError_t launch_ins_tile_first(const uint64_t *gkeys, int gshift, uint64_t n_new,
                                 uint64_t ntiles, uint64_t *first_new, hipStream_t s) {
    ins_tile_first_kernel<<<(unsigned)div_up(ntiles + 1, 256), 256, 0, s>>>(gkeys, gshift, n_new,
                                                                           ntiles, first_new);
    return hipGetLastError();
}

hipError_t launch_ins_meta(const Rec *orecs, const uint64_t *osbc, const uint64_t *ometa,
                           const uint64_t *gkeys, int gshift, const uint32_t *vals,
                           BintCounts bcnt, uint64_t n_new, uint64_t *nsbc, uint64_t *nmeta,
                           hipStream_t s) {
    ins_meta_kernel<<<1, 64, 0, s>>>(orecs, osbc, ometa, gkeys, gshift, vals, bcnt, n_new, nsbc,
                                     nmeta);
    return hipGetLastError();
}

hipError_t launch_insert(const Rec *orecs, const uint64_t *osbc, uint64_t n_ext,
                         const uint64_t *gkeys, int gshift, const uint32_t *vals,
                         BintCounts bcnt, uint64_t n_new, const uint64_t *first_new,
                         Rec *nrecs, const uint64_t *nsbc, uint32_t *err, hipStream_t s) {
    const uint64_t ntiles = div_up(records_for(n_ext + n_new), INS_TILE_RECS);
    InsJob J;
    J.orecs = orecs;
    J.osbc = osbc;
    J.nrecs = nrecs;
    J.nsbc = nsbc;
    J.gkeys = gkeys;
    J.vals = vals;
    J.bcnt = bcnt;
    J.first_new = first_new;
    J.n_ext = n_ext;
    J.n_new = n_new;
    J.sa0 = 0;
    J.goff = 0;
    J.gshift = gshift;
    insert_kernel<<<(unsigned)div_up(ntiles, 4), 256, 0, s>>>(J, ntiles, err);
    return hipGetLastError();
}

hipError_t launch_ins_tile_first_units(const InsertUnit *units, uint32_t nunits,
                                       const uint64_t *gkeys, int gshift, uint64_t ntiles_all,
                                       uint64_t *first_new, hipStream_t s) {
    if (nunits == 0) return hipSuccess;
    const uint64_t ne = ntiles_all + nunits;
    ins_tile_first_units_kernel<<<(unsigned)div_up(ne, 256), 256, 0, s>>>(units, nunits, gkeys,
                                                                          gshift, ne, first_new);
    return hipGetLastError();
}

hipError_t launch_ins_meta_units(const InsertUnit *units, uint32_t nunits, const uint64_t *gkeys,
                                 int gshift, const uint32_t *vals, BintCounts bcnt,
                                 hipStream_t s) {
    if (nunits == 0) return hipSuccess;
    ins_meta_units_kernel<<<(unsigned)div_up(nunits, 64), 64, 0, s>>>(units, nunits, gkeys,
                                                                      gshift, vals, bcnt);
    return hipGetLastError();
}

hipError_t launch_insert_units(const InsertUnit *units, uint32_t nunits, const uint64_t *gkeys,
                               int gshift, const uint32_t *vals, BintCounts bcnt,
                               const uint64_t *first_new, uint64_t ntiles_all, uint32_t *err,
                               hipStream_t s) {
    if (nunits == 0 || ntiles_all == 0) return hipSuccess;
    insert_units_kernel<<<(unsigned)div_up(ntiles_all, 4), 256, 0, s>>>(
        units, nunits, gkeys, gshift, vals, bcnt, first_new, ntiles_all, err);
    return hipGetLastError();
}

}  // namespace bwt
