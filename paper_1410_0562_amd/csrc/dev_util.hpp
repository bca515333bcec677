// dev_util.hpp -- device helpers shared by the HIP kernel files: the index
// rank primitive, 2-bit symbol windows, wave/block scans and the decoupled
// look-back used by single-pass scans and radix passes.  Written for gfx950:
// 64-lane wavefronts, 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bwt_internal.hpp"

namespace bwt {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// bits set for the lanes below this one
__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ------------------------------------------------------------ rank on B_ext
// rank(c, k) of Eq. 2 for a base c in 0..3 (A,C,G,T), 0 <= k <= n.
// One 64-byte record read (loads of the same line: the count of c, the two
// code planes, and the terminator plane for A only); `big` is uniform and
// says whether the index reaches 2^32 symbols (then the 64-bit superblock
// count is added).
__device__ __forceinline__ uint64_t match_bits(uint64_t lo, uint64_t hi, uint64_t dl, int c) {
    uint64_t a = (c & 1) ? lo : ~lo;
    uint64_t b = (c & 2) ? hi : ~hi;
    return a & b & ~dl;   // a terminator has lo = hi = 0 and matches nothing
}

__device__ __forceinline__ uint64_t rank_base(const Rec *__restrict__ recs,
                                              const uint64_t *__restrict__ sbc, uint64_t k,
                                              int c, bool big) {
    const uint4 *p = reinterpret_cast<const uint4 *>(recs + (k >> REC_SHIFT));
    const uint32_t cnt = reinterpret_cast<const uint32_t *>(p)[c];
    uint4 q1 = p[1], q2 = p[2];
    // a terminator's code bits are those of A, so only A needs the terminator
    // plane: the other bases skip its load
    uint4 q3 = make_uint4(0u, 0u, 0u, 0u);
    if (c == 0) q3 = p[3];
    uint64_t lo0 = q1.x | ((uint64_t)q1.y << 32), lo1 = q1.z | ((uint64_t)q1.w << 32);
    uint64_t hi0 = q2.x | ((uint64_t)q2.y << 32), hi1 = q2.z | ((uint64_t)q2.w << 32);
    uint64_t dl0 = q3.x | ((uint64_t)q3.y << 32), dl1 = q3.z | ((uint64_t)q3.w << 32);
    uint32_t o = (uint32_t)(k & (REC_SYMS - 1));
    uint64_t m0 = match_bits(lo0, hi0, dl0, c);
    uint64_t m1 = match_bits(lo1, hi1, dl1, c);
    uint64_t mask0 = o >= 64 ? ~0ull : ((1ull << o) - 1ull);
    uint64_t mask1 = o > 64 ? ((1ull << (o - 64)) - 1ull) : 0ull;
    uint64_t r = (uint64_t)cnt + __popcll(m0 & mask0) + __popcll(m1 & mask1);
    if (big) r += sbc[(k >> SB_SHIFT) * 4 + c];
    return r;
}

// symbol code (0..3), '$' (4), from one record at offset o (0..127)
__device__ __forceinline__ int rec_symbol(const Rec *__restrict__ recs, uint64_t i) {
    const Rec *r = recs + (i >> REC_SHIFT);
    uint32_t o = (uint32_t)(i & (REC_SYMS - 1));
    int w = o >> 6, b = o & 63;
    if ((r->dl[w] >> b) & 1) return 4;
    return (int)(((r->lo[w] >> b) & 1) | (((r->hi[w] >> b) & 1) << 1));
}

// ---------------------------------------------------------- 2-bit symbols
// Bits of symbols s, s+1, ..., s+nsym-1 of a 2-bit LSB-first packing, symbol
// s in bits 0..1 (higher bits hold whatever follows; callers mask).  Reads
// only 8-byte-aligned words that contain at least one byte of the requested
// symbols, so it never touches a page the buffer does not.  1 <= nsym <= 29.
__device__ __forceinline__ uint64_t load_sym_window(const uint8_t *base, uint64_t s, int nsym) {
    uintptr_t addr = (uintptr_t)base + (uintptr_t)(s >> 2);
    uintptr_t a0 = addr & ~(uintptr_t)7;
    int bit = (int)((addr - a0) * 8 + 2 * (s & 3));
    uint64_t v = *reinterpret_cast<const uint64_t *>(a0) >> bit;
    if (bit + 2 * nsym > 64) v |= *reinterpret_cast<const uint64_t *>(a0 + 8) << (64 - bit);
    return v;
}

__device__ __forceinline__ int load_sym(const uint8_t *base, uint64_t s) {
    return (base[s >> 2] >> (2 * (s & 3))) & 3;
}

// reverse the order of the 2-bit groups of a 64-bit word
__device__ __forceinline__ uint64_t reverse_pairs(uint64_t v) {
    uint64_t r = __builtin_bitreverse64(v);
    return ((r >> 1) & 0x5555555555555555ull) | ((r & 0x5555555555555555ull) << 1);
}

// ------------------------------------------------------------------- scans
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (l >= d) v += t;
    }
    return v;
}

// The same sum with DPP moves instead of LDS-crossbar shuffles: shifts by 1,
// 2, 4 and 8 lanes inside each row of 16 (lanes shifted in from outside the
// row read 0), then the last lane of rows 0 and 2 added to rows 1 and 3
// (row_bcast:15 on row mask 0xA), then lane 31 added to rows 2 and 3
// (row_bcast:31 on row mask 0xC).  All 64 lanes of the wave must be active.
__device__ __forceinline__ uint32_t wave_incl_sum_dpp(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (l >= d) v = v > t ? v : t;
    }
    return v;
}

// Block-wide (256 threads) exclusive sum; `tmp` is 4 words of LDS.  Returns
// the exclusive prefix, and the block total in *total.  Contains barriers.
__device__ __forceinline__ uint32_t block_excl_sum256(uint32_t v, uint32_t *tmp, uint32_t *total) {
    int tid = threadIdx.x, w = tid >> 6;
    uint32_t inc = wave_incl_sum(v);
    if ((tid & 63) == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t t0 = tmp[0], t1 = tmp[1], t2 = tmp[2], t3 = tmp[3];
    uint32_t before = (w > 0 ? t0 : 0) + (w > 1 ? t1 : 0) + (w > 2 ? t2 : 0);
    *total = t0 + t1 + t2 + t3;
    __syncthreads();
    return before + inc - v;
}

// Block-wide (256 threads) inclusive max; `tmp` is 4 words of LDS.
__device__ __forceinline__ uint32_t block_incl_max256(uint32_t v, uint32_t *tmp, uint32_t *total) {
    int tid = threadIdx.x, w = tid >> 6;
    uint32_t inc = wave_incl_max(v);
    if ((tid & 63) == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t t0 = tmp[0], t1 = tmp[1], t2 = tmp[2], t3 = tmp[3];
    uint32_t before = 0;
    if (w > 0) before = t0;
    if (w > 1) before = before > t1 ? before : t1;
    if (w > 2) before = before > t2 ? before : t2;
    uint32_t all = t0 > t1 ? t0 : t1;
    all = all > t2 ? all : t2;
    all = all > t3 ? all : t3;
    *total = all;
    __syncthreads();
    return inc > before ? inc : before;
}

// ------------------------------------------------------ decoupled look-back
// A chain of tiles publishes per-tile aggregates and inclusive prefixes in
// 64-bit status words: high half = epoch*4 + kind (1 aggregate, 2 inclusive
// prefix), low half = 32-bit payload.  Flag and payload share one word, so a
// relaxed agent-scope atomic load sees both or neither and no fence is
// needed.  A word written by an earlier launch carries another epoch and
// reads as "not ready", so status arrays are never cleared.  Tiles must be
// taken in launch order from an atomic counter (acquire_tile), which
// guarantees that every tile waited on is already running.
__device__ __forceinline__ uint64_t status_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct OpSum {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct OpMax {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

// Called by one lane per chain.  status points at this chain's word of tile
// 0; consecutive tiles are `stride` words apart.  Returns the exclusive
// prefix of `tile` (identity for tile 0) and publishes the inclusive one.
// The wait is bounded: after LOOKBACK_SPIN_LIMIT empty polls (far longer
// than any predecessor tile can take) the lane gives up, sets bit 0 of *err
// and returns what it has, so a broken launch ends instead of hanging.
constexpr uint32_t LOOKBACK_SPIN_LIMIT = 1u << 24;

template <class Op>
__device__ __forceinline__ uint32_t lookback(uint64_t *status, uint32_t stride, uint32_t tile,
                                             uint32_t epoch, uint32_t agg, Op op, uint32_t ident,
                                             uint32_t *err) {
    const uint32_t tag_a = epoch * 4u + 1u, tag_p = epoch * 4u + 2u;
    if (tile == 0) {
        status_store(status, ((uint64_t)tag_p << 32) | agg);
        return ident;
    }
    status_store(status + (size_t)tile * stride, ((uint64_t)tag_a << 32) | agg);
    uint32_t prefix = ident;
    int64_t t = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (t >= 0) {
        uint64_t w = status_load(status + (size_t)t * stride);
        uint32_t tag = (uint32_t)(w >> 32);
        if (tag == tag_p) {
            prefix = op(prefix, (uint32_t)w);
            break;
        }
        if (tag == tag_a) {
            prefix = op(prefix, (uint32_t)w);
            --t;
            continue;
        }
        if (++spins > LOOKBACK_SPIN_LIMIT) {
            atomicOr(err, 1u);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    status_store(status + (size_t)tile * stride, ((uint64_t)tag_p << 32) | op(prefix, agg));
    return prefix;
}

// Takes the next tile number; the last taker resets the counter so the next
// launch starts from zero (all takers of this launch have taken by then).
__device__ __forceinline__ uint32_t acquire_tile(uint32_t *counter, uint32_t ntiles,
                                                 uint32_t *s_slot) {
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(counter, 1u);
        if (t == ntiles - 1) atomicExch(counter, 0u);
        *s_slot = t;
    }
    __syncthreads();
    return *s_slot;
}

}  // namespace bwt
