/*
 * bwtset.h -- C ABI of libbwtset: incremental BWT of a DNA string set on an
 * MI355X (gfx950) GPU, built block by block with set-bwte (Pantaleoni,
 * "A massively parallel algorithm for constructing the BWT of large string
 * sets", arXiv:1410.0562, Algorithm 1).
 *
 * What is computed (Section 2): for strings S_0..S_{m-1} over A<C<G<T, the BWT
 * B of T = S_0 $_0 S_1 $_1 ... S_{m-1} $_{m-1} with $_0 < ... < $_{m-1} < A,
 * B[i] = T[(SA[i]-1) mod n] (Eq. 1), n = sum(|S_j| + 1).  Every terminator is
 * reported as '$'.  Strings appended later are numbered after all earlier
 * ones, in array order, so an index built by several appends is the BWT of the
 * concatenation of all appended sets (new strings can be added at any time,
 * Section 2).
 *
 * Conventions shared by every entry point:
 *   - Input reads are 2-bit packed: code = index in the alphabet (A=0, C=1,
 *     G=2, T=3), symbol s at byte s>>2, bits 2*(s&3)..2*(s&3)+1 (LSB first).
 *   - offsets: m+1 non-decreasing uint64 symbol offsets into `reads`; read j
 *     is symbols [offsets[j], offsets[j+1]).  Empty reads are allowed and add
 *     one terminator.  A read may hold at most 2^29 - 2 symbols.
 *   - Pointers may be host or device memory (detected with
 *     hipPointerGetAttributes) unless an entry point says "device".  Device
 *     buffers must be readable by the GPU the handle was created on.
 *   - `stream` is a hipStream_t (NULL: the handle's own stream).  Unless an
 *     entry point says otherwise, it returns after the work is done and the
 *     result is visible to later work on any stream.
 *   - A handle is not thread-safe.  Distinct handles are independent.
 *   - Errors are negative return codes (BWT_E*); the last one is kept per
 *     handle (bwt_set_last_error).  An append that fails leaves the index as it
 *     was before the call.
 */
#ifndef BWTSET_H
#define BWTSET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bwt_set *bwt_set_t;

enum {
    BWT_OK = 0,
    BWT_EINVAL = -1,        /* invalid argument (NULL, bad offsets, bad k/c) */
    BWT_ENOMEM = -2,        /* device memory could not be allocated */
    BWT_EHIP = -3,          /* a HIP runtime call failed */
    BWT_EALPHABET = -4,     /* alphabet other than "ACGT" */
    BWT_ESTATE = -5         /* handle unusable after an earlier HIP failure */
};

/* Creates an empty index on the current HIP device.  alphabet: NUL-terminated
 * list of the sigma symbols in sort order, without '$'; only "ACGT" is
 * supported (2-bit symbols).  Returns NULL on error; bwt_set_last_error(NULL)
 * then gives the code. */
bwt_set_t bwt_set_create(const char *alphabet);

/* Frees the handle and all its device memory.  NULL is ignored. */
void bwt_set_destroy(bwt_set_t h);

/* Adds m strings to the index (Algorithm 1): the strings are split into
 * blocks of whole strings of at most M suffixes each (M from
 * bwt_set_set_block_size; a longer string is a block by itself), and each
 * block is suffix-sorted (ConstructSA, Section 3), ranked against the index by
 * LF steps (ComputeRanks, Section 4, Lemma 1 / Algorithm 2), reordered into
 * suffix order (g_sa) and merged into the index (Insert, Section 5), which
 * also rebuilds the occurrence counters used by rank.  reads/offsets: host or
 * device, layout above.  Host buffers are copied before the GPU work starts;
 * device buffers must stay valid until the call returns.  m == 0 is a no-op.
 * Returns BWT_OK or a negative code; on error the index is unchanged. */
int bwt_set_append(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                   uint64_t m, void *stream);

/* Strand variants of an append (Section 2 notes that the strings may also be
 * indexed reversed):
 *   BWT_STRAND_FORWARD: the same as bwt_set_append;
 *   BWT_STRAND_REVERSE: every read is indexed written backwards (m strings,
 *     in input order);
 *   BWT_STRAND_BOTH: every read is followed by its reverse complement (read
 *     backwards with A<->T, C<->G), 2m strings: string 2j is read j and
 *     2j + 1 its reverse complement, so every pattern then occurs as often as
 *     its reverse complement.
 * reads/offsets as for bwt_set_append (host or device; offsets checked
 * before any symbol is read).  The repacked reads are staged on the device
 * (held by the handle until bwt_set_trim) and appended as one call, so the
 * index is the BWT of the concatenation of all strings appended so far with
 * these in the stated order.  Returns BWT_OK or a negative code (BWT_EINVAL
 * for another mode); on error the index is unchanged. */
enum { BWT_STRAND_FORWARD = 0, BWT_STRAND_REVERSE = 1, BWT_STRAND_BOTH = 2 };
int bwt_set_append_strands(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                           uint64_t m, int mode, void *stream);

/* Batched form: appends reads[i]/offsets[i] (m[i] strings) to hs[i] for every
 * i < count, with the same result on each handle as bwt_set_append.  The sets
 * are cut into blocks as bwt_set_append cuts them (Algorithm 1), and blocks of
 * different sets (units) share one device block: the block is suffix-sorted as
 * one text whose keys lead with each suffix's rank among its own set's old
 * suffixes plus a per-unit offset, so that the units sort apart; each unit is
 * ranked against its own set's index (Lemma 1) and merged into it, all units
 * of a block in one launch per step.  Many small sets then share the launches
 * and synchronizations of a few blocks.
 * hs: count distinct handles of one device, none unusable.  The batch runs on
 * hs[0]'s workspace, block size and tuning parameters and on `stream` (NULL:
 * hs[0]'s stream).  m[i] == 0 leaves hs[i] as it is.  reads[i]/offsets[i]:
 * host or device, as for bwt_set_append, and valid until the call returns.
 * Returns BWT_OK or a negative code (kept as hs[0]'s last error); on error
 * every index is unchanged. */
int bwt_set_append_many(bwt_set_t *hs, const uint8_t *const *reads,
                        const uint64_t *const *offsets, const uint64_t *m,
                        uint64_t count, void *stream);

/* rank(c, k, B) = |{ i < k : B[i] = c }| (Eq. 2).  c: 'A','C','G','T' or '$';
 * 0 <= k <= n.  Returns the count, or UINT64_MAX on error. */
uint64_t bwt_set_rank(bwt_set_t h, char c, uint64_t k);

/* Batched rank: out[t] = rank(cs[t], ks[t], B) for t < count.  cs, ks, out:
 * device pointers (cs as ASCII bytes).  An invalid pair yields UINT64_MAX in
 * its slot.  Enqueued on `stream`; returns without waiting. */
int bwt_set_rank_many(bwt_set_t h, const uint8_t *cs, const uint64_t *ks,
                      uint64_t *out, uint64_t count, void *stream);

/* FM-index count by backward search (the BWT with its rank function, Eq. 2,
 * is an FM-index; Lemma 1's step C[c] + rank(c, i, B) applied to both ends of
 * the interval of rows whose suffixes start with the symbols read so far,
 * from the pattern's last symbol to its first).  Pattern q < count is symbols
 * [offsets[q], offsets[q+1]) of pats, 2-bit packed as the reads are.  On
 * completion lo_out[q] is the number of suffixes smaller than the pattern
 * (terminators before A) and hi_out[q] - lo_out[q] the number of its
 * occurrences in the strings; the empty pattern gives [0, n).  pats, offsets,
 * lo_out, hi_out: device pointers.  A pattern whose offsets decrease yields
 * UINT64_MAX in both slots.  Enqueued on `stream`; returns without waiting;
 * the index must not change until the work has finished. */
int bwt_set_count_many(bwt_set_t h, const uint8_t *pats, const uint64_t *offsets,
                       uint64_t count, uint64_t *lo_out, uint64_t *hi_out, void *stream);

/* Writes B as n ASCII bytes ('A','C','G','T','$') to out (host or device).
 * out == NULL: returns n without writing (length query).  Returns n or a
 * negative code. */
int64_t bwt_set_export(bwt_set_t h, uint8_t *out);

/* Replaces the index by the one whose BWT is B (n ASCII bytes over
 * "ACGT$", host or device): the records and occurrence counters are rebuilt
 * from B, so an exported index can be stored and loaded again (checkpoint,
 * or FM-index queries on a BWT built elsewhere).  Every '$' counts as one
 * string.  Returns BWT_EINVAL for another byte; on error the index is
 * unchanged. */
int bwt_set_import(bwt_set_t h, const uint8_t *B, uint64_t n, void *stream);

/* Device memory held by the handle, in bytes (index buffers, workspace,
 * staging). */
int bwt_set_memory(bwt_set_t h, uint64_t *bytes);

/* Frees everything but the current index (workspace, staging, spare index
 * buffers); the next call that needs them allocates them again. */
int bwt_set_trim(bwt_set_t h);

/* Number of symbols n and strings m in the index. */
int bwt_set_size(bwt_set_t h, uint64_t *n, uint64_t *m);

/* Empties the index, keeping its device memory for reuse. */
int bwt_set_reset(bwt_set_t h);

/* Block size M of Algorithm 1, in suffixes (terminators included); default
 * 2^26.  Must be at least 1.  The result does not depend on M. */
int bwt_set_set_block_size(bwt_set_t h, uint64_t M);

/* Tuning knobs; none changes the result.
 *   BWT_PARAM_KEY_BITS: width in bits (16..64, default 64) of the first
 *     suffix-sort key, which holds g (the rank among the old suffixes, from
 *     ComputeRanks) above as many 2-bit symbols as fit.  Fewer bits mean fewer
 *     8-bit radix passes and more ties left to the LDS refinement. */
/*   BWT_PARAM_RADIX_TILE: tile shape of the radix passes (threads x keys per
 *     thread): 0 = 256x16, 1 = 512x8, 2 = 256x8, 3 = 512x12 (default),
 *     4 = 1024x4, 5 = 512x16, 6 = 1024x8, 7 = 1024x12, 8 = 768x12. */
/*   BWT_PARAM_RANK_SEGMENT: ComputeRanks walks a read longer than this many
 *     symbols in segments of this length, each one started by a backward
 *     search (FM-index interval) BWT_PARAM_RANK_OVERLAP symbols past its end
 *     and continued by Lemma 1 once the interval holds no old suffix; reads
 *     with a longer repeat fall back to one whole walk.  0 = never (32 ..
 *     2^24, default 768).  A segment whose interval is still open at its
 *     end starts again with 4 times the overlap (at least 256), then with
 *     16 times (at least 1024), before its read is walked whole.
 *   BWT_PARAM_RANK_OVERLAP: see above (0 .. 2^24, default 64).
 *   BWT_PARAM_BATCH_LANES: blocks of one level of a batch (bwt_set_append_many
 *     on this handle as hs[0]) that run side by side, each on its own stream
 *     and workspace (1 .. 4, default 2).
 *   BWT_PARAM_SORT_BUCKETS: 1 (default) = the first suffix sort runs radix
 *     passes on the top 8-24 bits of the key only (about 32 suffixes per
 *     bucket of equal top bits) and one wavefront finishes each bucket in
 *     registers (blocks of 2^20 suffixes or more); 0 = radix passes over the
 *     whole key. */
/*   BWT_PARAM_PIPELINE: 1 (default) = reads in host memory are streamed to
 *     the device block by block (the paper's stage pipeline with multiple
 *     buffering, Results and Figure 1): a second host thread copies block
 *     k+1's reads into one of two pinned slots and a copy stream sends them
 *     to one of two device slots while block k runs, events ordering the two
 *     streams.  0 = all host reads are copied to the device before the first
 *     block.  Not used by captured appends (BWT_PARAM_GRAPH). */
/*   BWT_PARAM_HOST_INDEX: 1 = the host-memory tier (Section 5 keeps the
 *     partial BWT in system memory; Section 6's bound is constant GPU memory):
 *     the index records and their occurrence counters are allocated in
 *     pinned host memory that the kernels read and write over the host link,
 *     so an index may exceed device memory while the device holds only the
 *     per-block workspace (bounded by the block size) and a few words per
 *     index buffer.  Buffers move to the chosen tier as they are next
 *     written (the next append moves the whole index).  bwt_set_memory
 *     counts device memory only.  0 (default) = index in device memory. */
/*   BWT_PARAM_GRAPH: 1 = bwt_set_append captures its blocks (every kernel of
 *     ConstructSA, ComputeRanks and Insert, with the tied-suffix count read on
 *     the device by a persistent refinement) into a HIP graph the first time
 *     it meets an input plan and index state, and replays the graph while
 *     they stay the same (same input buffers and block cut, same index size
 *     and buffers, no reallocation in between; the symbols may change).  Only
 *     appends whose blocks all hold fewer than 2^20 suffixes are captured
 *     (larger blocks take the bucket finish, which decides on the host, and
 *     launch costs do not matter there); the first sort of a captured block
 *     runs full-width radix passes.  The same holds for bwt_set_append_many
 *     with the parameter set on hs[0] (one stream, no lanes).  A
 *     block with a tied group too large for the refinement makes that call
 *     run again eagerly.  Up to 4 graphs are kept per handle.  0 (default) =
 *     no capture. */
enum {
    BWT_PARAM_KEY_BITS = 1,
    BWT_PARAM_RADIX_TILE = 2,
    BWT_PARAM_RANK_SEGMENT = 3,
    BWT_PARAM_RANK_OVERLAP = 4,
    BWT_PARAM_BATCH_LANES = 5,
    BWT_PARAM_SORT_BUCKETS = 6,
    BWT_PARAM_GRAPH = 7,
    BWT_PARAM_HOST_INDEX = 8,
    BWT_PARAM_PIPELINE = 9
};
int bwt_set_set_param(bwt_set_t h, int param, int64_t value);

/* Autotuner for the knobs above that never change a result: the first-key
 * width, the ComputeRanks segment length and overlap, and the radix tile
 * shape.  It builds this input (reads/offsets as for bwt_set_append) from
 * empty on a scratch handle with h's block size, median of three builds per
 * setting, changing one knob at a time from h's current settings, and applies
 * the fastest to h.  The choice is cached per GPU architecture and shape
 * class (block size, mean and longest read length, rounded to powers of
 * two) for the process and, when the environment variable BWTSET_TUNE_CACHE
 * names a file, in that file; a later call of the same class applies the
 * cached choice without timing unless `force` is set.  h's index is not
 * changed.  out (may be NULL) receives the choice. */
typedef struct {
    int radix_tile;
    int key_bits;
    uint32_t rank_segment;
    uint32_t rank_overlap;
    int from_cache;      /* 1: taken from the cache, nothing timed */
    double ms;           /* build time of the choice (median), when timed */
    int trials;          /* settings timed */
} bwt_tune_t;
int bwt_set_autotune(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets, uint64_t m,
                     int force, bwt_tune_t *out);

/* Last error code recorded on h (or, for h == NULL, by bwt_set_create). */
int bwt_set_last_error(bwt_set_t h);

/* Static description of an error code. */
const char *bwt_set_strerror(int code);

/* ---- Single steps of Algorithm 1, for checking each step on its own ----- */

/* ConstructSA and B_int of one block made of all m reads (block-local
 * terminators in read order, Section 3 and Algorithm 1): sa_out[i] (device,
 * uint32, n_blk = sum(|P_j|+1) entries) is the i-th smallest suffix of the
 * block text P_0 $ P_1 $ ...; bint_out[i] (device, n_blk bytes) is the symbol
 * before it as ASCII, '$' when the suffix starts a read.  reads/offsets: host
 * or device.  Does not change the index. */
int bwt_set_block_sort(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                       uint64_t m, uint32_t *sa_out, uint8_t *bint_out, void *stream);

/* bwt_set_block_sort for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same sa_out / bint_out, computed on a fixed workspace that
 * the library holds per GPU (about 24 MiB, a static device array, kept until
 * the process ends) instead of the handle's.  It calls no hipMalloc, hipFree
 * or other allocating routine.  Limits: reads, offsets, sa_out and bint_out
 * must be device pointers, and the block may hold at most 2^18 = 262,144
 * suffixes (sum of |P_j| + 1); larger inputs return BWT_EINVAL without
 * launching work.  Calls on one GPU share the workspace: calls from threads of
 * one process are serialized, and work the caller enqueues on the same GPU
 * that overlaps a call must not touch its buffers.  Synchronizes `stream`.
 * Returns BWT_EHIP if the workspace's device address could not be taken when
 * the first handle on this GPU was created. */
int bwt_set_block_sort_noalloc(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                               uint64_t m, uint32_t *sa_out, uint8_t *bint_out, void *stream);

/* ComputeRanks (Section 4, Lemma 1 / Algorithm 2) of one block made of all m
 * reads against the current index: g_out[p] (device, uint64, n_blk entries, in
 * block text order) = number of suffixes in the index smaller than the block
 * suffix at p.  Does not change the index. */
int bwt_set_compute_ranks(bwt_set_t h, const uint8_t *reads, const uint64_t *offsets,
                          uint64_t m, uint64_t *g_out, void *stream);

/* Insert (Section 5): merges n_new <= 2^29 - 1 symbols bint (device,
 * ASCII 'A','C','G','T','$') into the index, bint[i] going in front of old
 * row gsa[i] (device, uint64, non-decreasing, each <= n), and rebuilds the
 * occurrence counters; every '$' in bint counts as one more string.  Returns
 * BWT_EINVAL (index unchanged) if gsa decreases or exceeds n, or if bint
 * holds another byte. */
int bwt_set_insert(bwt_set_t h, const uint8_t *bint, const uint64_t *gsa,
                   uint64_t n_new, void *stream);

/* ---- Timing of the GPU steps ------------------------------------------- */

enum {
    BWT_STAGE_PLAN = 0,     /* offsets check and block split */
    BWT_STAGE_SORT = 1,     /* ConstructSA: keys, radix passes, doubling */
    BWT_STAGE_RANKS = 2,    /* ComputeRanks kernel */
    BWT_STAGE_GATHER = 3,   /* B_int and g_sa from the suffix array */
    BWT_STAGE_INSERT = 4,   /* Insert + occurrence counters */
    BWT_NSTAGES = 5
};

typedef struct {
    double ms[BWT_NSTAGES];         /* summed GPU time per stage (HIP events) */
    uint64_t launches[BWT_NSTAGES]; /* timed intervals per stage */
    double ranks_kernel_ms;         /* ComputeRanks: the one-lane-per-read walks alone */
    uint64_t ranks_launches;
    uint64_t ranks_steps;           /* LF steps performed (symbols walked) */
    double insert_kernel_ms;        /* Insert merge kernel alone */
    uint64_t insert_launches;
    uint64_t insert_records_out;    /* index records written by Insert */
    uint64_t insert_records_in;     /* index records read by Insert */
    uint64_t insert_new_symbols;    /* symbols merged in */
    double sort_pass_ms;            /* radix passes alone */
    uint64_t sort_pass_launches;
    uint64_t sort_pass_keys;        /* keys moved by radix passes */
    uint64_t blocks;                /* blocks processed */
    uint64_t doubling_rounds;       /* prefix-doubling rounds (large tied groups only) */
    double keys_ms;                 /* first-key build */
    double heads_ms;                /* tied-group detection after the first sort */
    double refine_ms;               /* LDS refinement of tied groups */
    uint64_t tied_suffixes;         /* suffixes left tied by the first sort */
    uint64_t fallback_blocks;       /* blocks sorted by prefix doubling */
    double bucket_ms;               /* LDS bucket finish of the first sort */
    double ranks_seg_ms;            /* ComputeRanks: segment walks of long reads alone */
    uint64_t ranks_seg_launches;
    double ranks_fb_ms;             /* ComputeRanks: whole-read fallback walks and long-read
                                       key counts */
    double tile_sort_ms;            /* bucket finish: the per-tile sort kernel alone */
    uint64_t tile_sort_launches;
    uint64_t tile_sort_keys;        /* suffixes passed through it */
    uint64_t insert_old_symbols;    /* sum over Insert launches of the index size before it */
    uint64_t insert_terminators;    /* terminators merged in */
    uint64_t ranks_retries;         /* ComputeRanks segments started again with a longer
                                       overlap (interval still open at their end) */
    uint64_t ranks_fallback_reads;  /* reads walked whole after a retry failed too */
    uint64_t ranks_seg_symbols;     /* symbols of the reads ranked by the segment kernel
                                       (the others by the one-lane-per-read walks) */
    uint64_t graph_captures;        /* appends captured into a HIP graph (BWT_PARAM_GRAPH) */
    uint64_t graph_replays;         /* captured appends launched */
    uint64_t graph_redos;           /* replays run again eagerly (a tied group needed
                                       prefix doubling) */
} bwt_stats_t;

/* Turns per-stage HIP-event timing on (1) or off (0).  Timing adds event
 * records around the stages; results are unchanged. */
int bwt_set_enable_timing(bwt_set_t h, int on);

/* Copies the accumulated timings; clears them when reset != 0. */
int bwt_set_get_stats(bwt_set_t h, bwt_stats_t *out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* BWTSET_H */
