// bwt_internal.hpp -- layouts and kernel launchers shared by the host runtime
// (bwtset.cpp) and the HIP kernel files.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bwt {

// ---------------------------------------------------------------------------
// Index layout in HBM (the partial BWT B_ext plus its occurrence counters).
//
// B_ext is cut into records of 128 symbols.  A record is one 64-byte line:
//   cnt[4]  occurrences of A, C, G, T in [superblock start, record start)
//   lo[2]   bit t = low bit of the code of symbol t   (A=0 C=1 G=2 T=3)
//   hi[2]   bit t = high bit of the code of symbol t
//   dl[2]   bit t = 1 where symbol t is a terminator ('$'; its lo/hi are 0)
// so rank(c, k) (Eq. 2) is one 64-byte record read plus two popcounts, the
// counterpart of the per-page counters sampled every 128 symbols that the
// paper keeps for DNA (Section 5).  Counts are 32-bit and relative to a
// superblock of 2^32 symbols; `sbc[sb*4 + c]` holds the 64-bit count of c
// before superblock sb.  An index of n symbols has n/128 + 1 records (the last
// one may be a sentinel holding only counts, so that rank(c, n) is a plain
// record lookup) and n/2^32 + 1 superblock entries.
//
// `meta` (device, uint64[8]): [0..3] total A, C, G, T; [4] n; [5] m (number of
// terminators); [6..7] unused.
// ---------------------------------------------------------------------------
struct alignas(64) Rec {
    uint32_t cnt[4];
    uint64_t lo[2];
    uint64_t hi[2];
    uint64_t dl[2];
};
static_assert(sizeof(Rec) == 64, "record must be one 64-byte line");

constexpr int REC_SHIFT = 7;
constexpr uint64_t REC_SYMS = 1ull << REC_SHIFT;
constexpr int SB_SHIFT = 32;
constexpr int META_WORDS = 8;

__host__ __device__ inline uint64_t records_for(uint64_t n) { return (n >> REC_SHIFT) + 1; }
__host__ __device__ inline uint64_t superblocks_for(uint64_t n) { return (n >> SB_SHIFT) + 1; }

// ---------------------------------------------------------------------------
// Block suffix sorting.
//
// Position p of a block's text (reads P_0 $ P_1 $ ..., local terminators in
// read order) is carried in sort values as p | prev << 29, where prev is the
// code of the symbol before p (0..3) or 4 when p starts a read, so that B_int
// falls out of the sorted values without a second gather.
//
// First sort key of p.  g[p] (ComputeRanks: old suffixes smaller than the
// block suffix at p) is non-decreasing in suffix order, so it can lead the
// key without changing the order, and g_sa comes out of the sort with it:
//   key = g[p] << gshift | sym << 5 | t,   gshift = key_bits - gbits,
// gbits = bits needed for values up to n_ext (0 for an empty index: no g),
// key_bits = width of the key (64 by default; fewer bits, fewer radix
// passes), K' = min(29, (key_bits - 5 - gbits) / 2) symbols, r = symbols of
// p's read before its terminator, t = min(r, K'), sym = the first t symbols,
// 2 bits each, first symbol most significant, zero-padded to K' symbols.  Equal keys with t < K'
// end in their terminators and are ordered by read index, i.e. by position,
// which the stable sort keeps.  Later chunks of 29 symbols at depth d use the
// same layout without g (chunk keys).
// ---------------------------------------------------------------------------
constexpr int KEY_K = 29;            // symbols in a chunk key
constexpr int KEY_LEN_BITS = 5;
constexpr int POS_BITS = 29;
constexpr uint32_t POS_MASK = (1u << POS_BITS) - 1u;
constexpr uint64_t MAX_BLOCK = (1ull << POS_BITS) - 1;  // suffixes per block
constexpr uint64_t MAX_READ = MAX_BLOCK - 1;            // symbols per read

// symbols that fit a first key of key_bits bits after gbits bits of g
__host__ __device__ inline int first_key_syms(int gbits, int key_bits) {
    int k = (key_bits - KEY_LEN_BITS - gbits) / 2;
    return k < 0 ? 0 : (k < KEY_K ? k : KEY_K);
}

// groups of tied suffixes up to this size are finished in LDS by comparing
// successive chunks; a block with a larger group uses prefix doubling
constexpr int REFINE_LIMIT = 256;
constexpr int REFINE_WINDOW = 512;

constexpr int PREP_TILE_SHIFT = 8;   // positions per read-lookup tile
constexpr int SCAN_TILE = 4096;      // elements per look-back scan tile
constexpr int INS_TILE_RECS = 16;    // output records per Insert tile
constexpr uint64_t INS_TILE_SYMS = INS_TILE_RECS * REC_SYMS;
constexpr int CHUNK_SHIFT = 6;       // B_int counts sampled every 64 symbols

// B_int counts sampled every 64 sorted symbols: the count of base c among the
// first 64k symbols is chunk[k*4 + c] + seg[(k >> BINT_SEG_SHIFT)*4 + c]
// (the count inside a segment of 1024 chunks, plus the count before the
// segment), for k = 0 .. ceil(n / 64).  chunk holds ceil(n/64) + 1 entries of
// 4 words, seg ceil(n / 65536) + 1.
constexpr int BINT_SEG_SHIFT = 10;
struct BintCounts {
    const uint32_t *chunk;
    const uint32_t *seg;
};

__host__ __device__ inline int bits_for_value(uint64_t v) {  // bits to hold 0..v
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Optional per-kernel timing.  A launcher that takes Marks records a[k] just
// before and b[k] just after the kernel(s) of its span k (documented at the
// launcher), on the stream it launches on; null events are skipped.
struct Marks {
    hipEvent_t a[3] = {nullptr, nullptr, nullptr};
    hipEvent_t b[3] = {nullptr, nullptr, nullptr};
    static void begin(const Marks *m, int k, hipStream_t s) {
        if (m && m->a[k]) (void)hipEventRecord(m->a[k], s);
    }
    static void end(const Marks *m, int k, hipStream_t s) {
        if (m && m->b[k]) (void)hipEventRecord(m->b[k], s);
    }
};

// ----------------------------------------------------------------- launchers
// Every launcher enqueues on `s` and returns hipGetLastError().  `err` is a
// device word into which kernels OR a bit when an internal consistency check
// fails (a bounded wait timed out, an index would leave its buffer); the host
// reads it after every append and treats a nonzero value as a failure.

// radix sort pieces (k_radix.hip).  Digit counts are spread over HIST_COPIES
// copies so that many workgroups adding to the same hot digit do not queue on
// one atomic word: hist[(pass * HIST_COPIES + copy) * 256 + digit].  Pass p
// sums the copies of its counts into digit starts (hist_cur = pass p's copies)
// and adds the next pass's counts.
constexpr int HIST_COPIES = 8;
constexpr uint32_t HIST_WORDS = 8 * HIST_COPIES * 256;
hipError_t launch_radix_hist1(const uint64_t *keys, uint64_t n, int shift, uint32_t *hist,
                              hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s);
// cfg selects the tile shape (see radix_tile_keys); the status array must
// hold 256 words per tile of the smallest shape
int radix_tile_keys(int cfg);
constexpr int RADIX_CFGS = 9;
constexpr int RADIX_MIN_TILE = 2048;
hipError_t launch_radix_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                             uint32_t *vout, uint64_t n, int shift, const uint32_t *hist_cur,
                             uint32_t *hist_next, int shift_next, uint64_t *status,
                             uint32_t *counter, uint32_t epoch, uint32_t *err, int cfg,
                             hipStream_t s);

// block preparation, suffix sorting and refinement (k_sa.hip)
hipError_t launch_block_soff(const uint64_t *off, uint32_t m_blk, uint32_t *soff, hipStream_t s);
hipError_t launch_block_tile_first(const uint32_t *soff, uint32_t m_blk, uint32_t n_blk,
                                   uint32_t *tile_first, hipStream_t s);
// key = g[p] << gshift | (kfirst symbols) << 5 | count (g may be null: no
// g); hist0 (the first pass's HIST_COPIES x 256 words, zeroed by the caller)
// receives the counts of the 8-bit digit at bit hshift
hipError_t launch_block_keys(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                             const uint32_t *tile_first, uint32_t n_blk, const uint64_t *g,
                             int gshift, int kfirst, int hshift, uint64_t *keys, uint32_t *vals,
                             uint32_t *hist0, hipStream_t s);

// Bucket finish of the first sort (k_bucket.hip).  After radix passes on the
// top digits, keys kin sit in nb = 2^B buckets of equal bits above bshift,
// each a contiguous run.  bucket_sort: every bucket of 1 .. BUCKET_CAP
// suffixes sorted by one wave into kout / vout at the same positions (*large
// set for a tied group above limit); per bucket tcnt = tied suffixes before it
// (exclusive prefix) and osz = its size if above BUCKET_CAP, with its start in
// bstart (oversized buckets only); the oversized buckets in bucket order in
// olist, their starts in the gathered array in ooff (ooff[count] = total); res
// = {tied suffixes, oversized buckets, oversized suffixes}; part holds 3 words
// per 4096 bucket ids; trange 3 words per 2048 positions; tflag one byte per
// position (1 = tied).  emit_and_check (below) lists the tied suffixes of the
// sorted buckets in U (slot order) from tflag.  oversize_gather copies the oversized
// buckets of kin to ck/cv; once sorted there on the whole key,
// oversize_scatter puts them into kout / vout and oversize_ties_map appends
// their tied suffixes (gathered indices U2[0 .. *nU2)) to U after the first
// `base`, setting *nU.
constexpr uint32_t BUCKET_CAP = 256;
constexpr int BUCKET_MAX_BITS = 24;
hipError_t launch_bucket_sort(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                              uint32_t *vout, uint32_t n, uint32_t *bstart, uint32_t *trange,
                              uint32_t nb, int bshift, int kshort, uint32_t limit, uint32_t *large,
                              uint32_t *tcnt, uint32_t *osz, uint8_t *tflag, uint32_t *part,
                              uint32_t *res, uint32_t *olist, uint32_t *ooff, uint32_t *obad,
                              uint32_t *err, hipStream_t s, const Marks *mk = nullptr);
// (marks: span 0 = the per-tile sort kernel)
// emit_and_check: the tied suffixes of the sorted buckets listed in U (slot
// order, from tflag) and, side by side in the same launch, the
// copy of every oversized bucket of (kx, vx) to (ky, vy); then the oversized
// buckets that still need sorting are listed in olist2 / ooff2 (res2 =
// {count, suffixes}): the others hold copies of one key that ends at its
// terminator.  The counts are read on the device from the bucket scans' res;
// obad is one word per oversized bucket, zeroed by bucket_sort.
hipError_t launch_emit_and_check(const uint8_t *tflag, uint32_t n, const uint32_t *trange,
                                 const uint32_t *tpre, uint32_t nb, uint32_t *U, uint32_t ucap,
                                 const uint64_t *kx, const uint32_t *vx, uint64_t *ky,
                                 uint32_t *vy, const uint32_t *bstart, const uint32_t *olist,
                                 const uint32_t *ooff, const uint32_t *res, int kshort,
                                 uint32_t *obad, uint32_t *olist2, uint32_t *ooff2,
                                 uint32_t *res2, uint32_t *err, hipStream_t s);
hipError_t launch_oversize_gather(const uint64_t *keys, const uint32_t *vals,
                                  const uint32_t *bstart, const uint32_t *olist,
                                  const uint32_t *ooff, uint32_t nob, uint32_t no, uint32_t n,
                                  uint64_t *ck, uint32_t *cv, uint32_t *err, hipStream_t s);
hipError_t launch_oversize_scatter(const uint64_t *ck, const uint32_t *cv, uint32_t no,
                                   const uint32_t *bstart, const uint32_t *olist,
                                   const uint32_t *ooff, uint32_t nob, uint32_t n, uint64_t *keys,
                                   uint32_t *vals, uint32_t *err, hipStream_t s);
hipError_t launch_oversize_ties_map(const uint32_t *U2, const uint32_t *nU2, const uint32_t *bstart,
                                    const uint32_t *olist, const uint32_t *ooff, uint32_t nob,
                                    uint32_t no, uint32_t base, uint32_t ucap, uint32_t *U,
                                    uint32_t *nU, uint32_t *err, hipStream_t s);
// Groups after a sort.  Round 0 (U == nullptr): element i is SA slot i, and a
// key whose length field is below kshort is a singleton.  Doubling round:
// element u is SA slot U[u] and its value is stored there.  rank == nullptr
// skips the rank scatter.  A group larger than `limit` sets *large.
hipError_t launch_group_heads(const uint64_t *keys, const uint32_t *vals, const uint32_t *U,
                              uint32_t n, int kshort, uint32_t *sa, uint32_t *rank,
                              uint32_t *Uout, uint32_t *nUout, uint32_t limit, uint32_t *large,
                              uint64_t *status, uint32_t *counter, uint32_t epoch, uint32_t *err,
                              hipStream_t s);
hipError_t launch_doubling_keys(const uint32_t *U, uint32_t nU, const uint32_t *sa,
                                const uint32_t *rank, uint32_t h, int rbits, uint32_t n_blk,
                                uint64_t *keys, uint32_t *vals, uint32_t *err, hipStream_t s);
// finishes every group of U (all of size <= REFINE_LIMIT) by chunk keys
hipError_t launch_refine(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                         const uint32_t *tile_first, const uint64_t *keys, const uint32_t *U,
                         uint32_t nU, uint32_t *sa, int kfirst, uint32_t max_iter, uint32_t *err,
                         hipStream_t s);
// The same with the count of tied suffixes on the device (*nUp, at most n_max)
// and a fixed grid of workgroups striding over the windows; with *largep set
// nothing is refined and REFINE_REDO is set in *err.
constexpr uint32_t REFINE_REDO = 1u << 20;
constexpr unsigned REFINE_MAX_GRID = 2048;
hipError_t launch_refine_dev(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                             const uint32_t *tile_first, const uint64_t *keys, const uint32_t *U,
                             const uint32_t *nUp, const uint32_t *largep, uint32_t n_max,
                             uint32_t *sa, int kfirst, uint32_t max_iter, uint32_t *err,
                             hipStream_t s);
// B_int as ASCII from sorted values, and the plain suffix array
hipError_t launch_vals_to_ascii(const uint32_t *sa, uint32_t n, uint8_t *bint, hipStream_t s);
// g in text order back from sorted first keys: g[vals[i] & POS_MASK] = keys[i] >> gshift
hipError_t launch_scatter_g(const uint64_t *keys, const uint32_t *vals, uint32_t n, int gshift,
                            uint64_t *g, hipStream_t s);
hipError_t launch_sa_strip(const uint32_t *sa, uint32_t n, uint32_t *out, hipStream_t s);

// ComputeRanks (k_ranks.hip).  Reads longer than seg_len symbols (0: never)
// are walked in segments of seg_len symbols, each starting overlap symbols
// past its end (see k_ranks.hip); seg_list holds seg_cap entries, fb_flag and
// fb_list one word per read of the block, counters two words.
struct RankSegments {
    uint32_t seg_len = 0;
    uint32_t overlap = 0;
    uint64_t *seg_list = nullptr;
    uint32_t seg_cap = 0;
    uint32_t *fb_flag = nullptr;
    uint32_t *fb_list = nullptr;
    uint32_t *counters = nullptr;
    uint32_t *stats = nullptr;   // running totals: segment retries, whole-read fallbacks,
                                 // and (64-bit, words 2-3) symbols ranked by segment walks
};
// A segment whose FM-index interval is still open at its end starts again
// with its overlap times RETRY_FACTOR1 (at least RETRY_MIN1), then times
// RETRY_FACTOR2 (at least RETRY_MIN2); after that its read is walked whole.
// The short first retry keeps the usual case (a chance agreement of noisy
// reads a little longer than the overlap) from stretching its launch.
constexpr uint32_t RETRY_FACTOR1 = 4, RETRY_MIN1 = 256;
constexpr uint32_t RETRY_FACTOR2 = 16, RETRY_MIN2 = 1024;
// Key mode (kk != null): instead of g, the walks write the first sort key of
// every block position, g << gshift | its next kfirst symbols << 5 | their
// count (what launch_block_keys builds), and its sort value (see below).
struct RankKeys {
    uint64_t *keys;
    uint32_t *vals;
    int gshift;
    int kfirst;
    uint32_t *hist;  // if set: counts of the key digit at bit hshift, added to
    int hshift;      // the HIST_COPIES copies (zeroed by the caller)
};
// Marks: span 0 = the one-lane-per-read walks, 1 = the long-read segment
// walks, 2 = the whole-read fallback walks and the key counts of long reads
// (spans 1 and 2 are empty when no read is cut into segments).
hipError_t launch_compute_ranks(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                                uint32_t m_blk, uint32_t n_blk, const Rec *recs,
                                const uint64_t *sbc, const uint64_t *meta, int big, uint64_t *g,
                                const RankKeys *kk, const RankSegments &sg, uint32_t *err,
                                hipStream_t s, const Marks *mk = nullptr);

// ---------------------------------------------------------------------------
// Batched form: one block holds reads of several independent sets (units).
// Unit u of a block is a run of consecutive reads of one set; its reads are
// ranked against that set's own index, and every rank is offset by
//   goff[u] = sum over the earlier units u' of (n_ext[u'] + 1),
// the number of values the earlier units' ranks can take, so that the ranks
// of different units never meet.  Leading the suffix-sort key with the offset
// rank sorts the block unit by unit, each unit in its own suffix order, so
// the units' sorted suffixes are consecutive runs of the sorted block and
// each run merges into its own set's index.
// ---------------------------------------------------------------------------
struct RankUnit {
    const Rec *recs;
    const uint64_t *sbc;
    const uint64_t *meta;
    uint64_t goff;
    uint32_t read0;   // first read of the unit in the block (ascending over units)
    uint32_t big;     // index of 2^32 symbols or more
};
hipError_t launch_compute_ranks_units(const uint8_t *reads, const uint64_t *off,
                                      const uint32_t *soff, uint32_t m_blk, uint32_t n_blk,
                                      const RankUnit *units, uint32_t nunits, uint64_t *g,
                                      const RankKeys *kk, const RankSegments &sg, uint32_t *err,
                                      hipStream_t s, const Marks *mk = nullptr);

struct InsertUnit {
    const Rec *orecs;
    const uint64_t *osbc;
    const uint64_t *ometa;
    Rec *nrecs;
    uint64_t *nsbc;
    uint64_t *nmeta;
    uint64_t n_ext, n_new;
    uint64_t sa0;    // first slot of the unit among the block's sorted suffixes
    uint64_t goff;   // subtracted from the key's g to give the unit's g_sa
    uint64_t tile0;  // first Insert tile of the unit; its first_new entries
                     // start at tile0 + (unit index)
};
// first_new for every unit; ntiles_all = sum of the units' tiles
hipError_t launch_ins_tile_first_units(const InsertUnit *units, uint32_t nunits,
                                       const uint64_t *gkeys, int gshift, uint64_t ntiles_all,
                                       uint64_t *first_new, hipStream_t s);
hipError_t launch_ins_meta_units(const InsertUnit *units, uint32_t nunits, const uint64_t *gkeys,
                                 int gshift, const uint32_t *vals, BintCounts bcnt,
                                 hipStream_t s);
hipError_t launch_insert_units(const InsertUnit *units, uint32_t nunits, const uint64_t *gkeys,
                               int gshift, const uint32_t *vals, BintCounts bcnt,
                               const uint64_t *first_new, uint64_t ntiles_all, uint32_t *err,
                               hipStream_t s);

// Staging of a batch: the reads of every unit, in schedule order, copied
// into one packed buffer with one offsets array, so that every block of the
// batch is a contiguous run of reads.  Unit u takes the reads [j0, j1) of its
// set and lands at staged read dst_read0 and staged symbol dst_sym0 (both
// non-decreasing over units, with no gaps).
struct GatherUnit {
    const uint8_t *reads;   // the set's packed reads (device), from symbol sym_base
    const uint64_t *off;    // the set's offsets (device)
    uint64_t j0, j1;
    uint64_t dst_read0, dst_sym0;
    uint64_t sym_base;      // multiple of 4: symbol p is at reads[(p - sym_base) / 4]
};
hipError_t launch_gather_offsets(const GatherUnit *units, uint32_t nunits, uint64_t total_reads,
                                 uint64_t total_syms, uint64_t *dst_off, hipStream_t s);
hipError_t launch_gather_reads(const GatherUnit *units, uint32_t nunits, uint64_t total_syms,
                               uint8_t *dst, hipStream_t s);
// Per set of a batch (device offsets, m reads): res[4s..4s+3] = {1 if the
// offsets decrease, longest read, suffixes, number of blocks of at most M
// suffixes}; with cuts (cut_base[s] words into it), the block cuts as
// launch_plan_blocks writes them.
struct PlanSet {
    const uint64_t *off;
    uint64_t m;
    uint64_t cut_base;
};
hipError_t launch_plan_sets(const PlanSet *sets, uint32_t nsets, uint64_t M, uint64_t *res,
                            uint64_t *cuts, hipStream_t s);

// Insert and index bookkeeping (k_insert.hip).  The new symbols come in
// suffix order as the sorted (key, value) pairs of ConstructSA: g_sa[i] is
// gkeys[i] >> gshift (0 for every i when gshift == 64) and the symbol code
// (0..3 for A..T, 4 for '$') is vals[i] >> 29.
hipError_t launch_index_init(Rec *recs, uint64_t *sbc, uint64_t *meta, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_count_bint(const uint32_t *vals, uint32_t n, uint32_t *chunk, uint32_t *seg,
                             hipStream_t s);
// user-supplied B_int (ASCII) and g_sa: *bad |= 1 for a byte outside "ACGT$",
// 2 for a g_sa that decreases or exceeds n_ext; then packed as keys/values
hipError_t launch_check_user_insert(const uint8_t *bint, const uint64_t *gsa, uint64_t n_new,
                                   uint64_t n_ext, uint32_t *bad, hipStream_t s);
hipError_t launch_pack_user_insert(const uint8_t *bint, const uint64_t *gsa, uint64_t n_new,
                                  int gshift, uint64_t *keys, uint32_t *vals, hipStream_t s);
hipError_t launch_ins_tile_first(const uint64_t *gkeys, int gshift, uint64_t n_new,
                                 uint64_t ntiles, uint64_t *first_new, hipStream_t s);
hipError_t launch_ins_meta(const Rec *orecs, const uint64_t *osbc, const uint64_t *ometa,
                           const uint64_t *gkeys, int gshift, const uint32_t *vals,
                           BintCounts bcnt, uint64_t n_new, uint64_t *nsbc, uint64_t *nmeta,
                           hipStream_t s);
hipError_t launch_insert(const Rec *orecs, const uint64_t *osbc, uint64_t n_ext,
                         const uint64_t *gkeys, int gshift, const uint32_t *vals,
                         BintCounts bcnt, uint64_t n_new, const uint64_t *first_new,
                         Rec *nrecs, const uint64_t *nsbc, uint32_t *err, hipStream_t s);

// queries and input checks (k_query.hip)
hipError_t launch_rank_many(const Rec *recs, const uint64_t *sbc, const uint64_t *meta,
                            const uint8_t *cs, const uint64_t *ks, uint64_t *out, uint64_t count,
                            hipStream_t s);
hipError_t launch_export(const Rec *recs, uint64_t n, uint8_t *out, hipStream_t s);
// strand variants: mode 1 every read reversed, mode 2 every read followed by
// its reverse complement; out_off gets m (mode 1) or 2m (mode 2) + 1 offsets
// from 0, out the packed symbols (total of them, 4-byte aligned buffer);
// input symbol p is at p - in_base of `in`; offsets must be non-decreasing
hipError_t launch_strands(const uint8_t *in, uint64_t in_base, const uint64_t *off, uint64_t m,
                          int mode, uint64_t *out_off, uint64_t total, uint8_t *out,
                          hipStream_t s);
// FM-index count: lo/hi per pattern (2-bit packed pats, count + 1 offsets)
hipError_t launch_count(const Rec *recs, const uint64_t *sbc, const uint64_t *meta,
                        const uint8_t *pats, const uint64_t *poff, uint64_t count,
                        uint64_t *lo, uint64_t *hi, hipStream_t s);
hipError_t launch_check_offsets(const uint64_t *off, uint64_t m, uint64_t *res, hipStream_t s);
hipError_t launch_plan_blocks(const uint64_t *off, uint64_t m, uint64_t M, uint64_t *cuts,
                              uint64_t *res, hipStream_t s);

}  // namespace bwt
