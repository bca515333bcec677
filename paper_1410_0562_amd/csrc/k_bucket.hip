// k_bucket.hip -- the second half of a block's suffix sort (Section 3).
//
// Radix passes on the top digits of the first key (see bwt_internal.hpp)
// leave the suffixes in buckets of equal top B bits, each bucket a contiguous
// run in position order (the passes are stable); B is chosen for about 32
// suffixes per bucket.  A workgroup takes a tile of positions, finds the
// bucket starts in it from the keys it loads, and one wavefront finishes a
// bucket of at most BUCKET_CAP = 256 suffixes in registers (four buckets of
// at most 64 at once, one per register row, so that their shuffles overlap):
// a bitonic network over (key, index in the bucket) -- the index keeps equal
// keys in position order, which is terminator order -- with 64 x E elements
// per wave (element r * 64 + lane in register r of that lane), so the
// compare-exchanges at distance >= 64 stay inside a lane and the shorter ones
// are lane shuffles; no workgroup barrier is involved.  The wave flags the
// bucket's tied suffixes (equal keys that do not end at a terminator); after
// a scan of the per-bucket counts, the flags of each tile are listed in slot
// order, so every tied group stays contiguous in the list of unresolved
// suffixes.  Larger buckets are piles of identical short suffixes (every
// read's terminator suffix has the same g, as have all suffixes "A$", ...):
// they are gathered into one array, radix-sorted on the whole key with the
// ordinary passes, put back, and their ties found by the ordinary scan.
#include "dev_util.hpp"

namespace bwt {

namespace {

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t n, uint32_t v) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// (key, index) order
__device__ __forceinline__ bool pair_gt(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka > kb || (ka == kb && ia > ib);
}

// Sorts the P = 64 * E elements held by one wave: element i = r * 64 + lane
// in (k[r], x[r]).  Ascending bitonic network.
template <int E>
__device__ __forceinline__ void wave_bitonic(uint64_t (&k)[E], uint32_t (&x)[E], int lane) {
    constexpr int P = 64 * E;
#pragma unroll
    for (int kk = 2; kk <= P; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                // partners in the same lane: registers r and r ^ (j / 64)
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int rr = r ^ (j >> 6);
                    if (rr > r) {
                        const uint32_t i = (uint32_t)(r * 64 + lane);
                        const bool up = (i & (uint32_t)kk) == 0;
                        if (pair_gt(k[r], x[r], k[rr], x[rr]) == up) {
                            uint64_t tk = k[r];
                            k[r] = k[rr];
                            k[rr] = tk;
                            uint32_t tx = x[r];
                            x[r] = x[rr];
                            x[rr] = tx;
                        }
                    }
                }
            } else {
                // partners in lanes lane ^ j, same register
                const bool lower = (lane & j) == 0;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const uint32_t i = (uint32_t)(r * 64 + lane);
                    const bool up = (i & (uint32_t)kk) == 0;
                    const uint64_t pk = __shfl_xor(k[r], j, 64);
                    const uint32_t px = __shfl_xor(x[r], j, 64);
                    // the lower index keeps the smaller element when ascending
                    const bool keep_min = lower == up;
                    const bool mine_gt = pair_gt(k[r], x[r], pk, px);
                    if (keep_min == mine_gt) {
                        k[r] = pk;
                        x[r] = px;
                    }
                }
            }
        }
    }
}

// Value of lane (lane ^ J) of the wave.  Distances 1 and 2 stay inside a
// quad (DPP quad_perm); 4 is a mirror inside each half-row of 8 followed by a
// reversal inside each quad (two DPP moves); 8 is a rotation by 8 inside a
// row of 16 (DPP row_ror:8); 16 and 32 go through the LDS crossbar.
// Every lane reads a valid source lane in these patterns, so the DPP moves
// need no initial destination value (mov_dpp, all rows and banks written).
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);
    } else if constexpr (J == 4) {
        const int m = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);
        return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, true);
    } else {
        return (uint32_t)__shfl_xor((int)v, J, 64);
    }
}

// One compare-exchange stage (block size KK, distance J) on R independent
// rows of composite words cut into segments of S lanes (each segment is
// sorted ascending as a whole at KK = S), then the stages of the same block
// at J / 2, J / 4, ...
template <int KK, int J, int R, int S>
__device__ __forceinline__ void row_stage(uint64_t (&c)[R], int lane) {
    const bool lower = (lane & J) == 0;
    const bool up = KK == S || (lane & KK) == 0;
    const bool keep_min = lower == up;
    uint64_t p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t lo = lane_xor<J>((uint32_t)c[r], lane);
        const uint32_t hi = lane_xor<J>((uint32_t)(c[r] >> 32), lane);
        p[r] = (uint64_t)lo | ((uint64_t)hi << 32);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (keep_min == (c[r] > p[r])) c[r] = p[r];
    if constexpr (J > 1) row_stage<KK, J / 2, R, S>(c, lane);
}

template <int KK, int R, int S>
__device__ __forceinline__ void row_levels(uint64_t (&c)[R], int lane) {
    row_stage<KK, KK / 2, R, S>(c, lane);
    if constexpr (KK < S) row_levels<KK * 2, R, S>(c, lane);
}

// Sorts each segment of S lanes of each of R rows of distinct 64-bit words
// ascending (S = 64: whole rows; S = 32: two segments per row).
template <int R, int S>
__device__ __forceinline__ void wave_sort_rows(uint64_t (&c)[R], int lane) {
    row_levels<2, R, S>(c, lane);
}

// Bitonic network over the 64 * E distinct words of one wave (element
// r * 64 + lane in c[r]), ascending: compare-exchanges at distance >= 64 stay
// inside a lane (registers r and r ^ (J / 64)), shorter ones use lane_xor.
template <int E, int KK, int J>
__device__ __forceinline__ void reg_stage(uint64_t (&c)[E], int lane) {
    if constexpr (J >= 64) {
        constexpr int D = J / 64;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if ((r & D) == 0) {
                const int rr = r | D;
                const bool up = ((r * 64) & KK) == 0;  // KK >= 128: uniform per register
                const uint64_t a = c[r], b = c[rr];
                if ((a > b) == up) {
                    c[r] = b;
                    c[rr] = a;
                }
            }
        }
    } else {
        const bool lower = (lane & J) == 0;
        uint64_t p[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t lo = lane_xor<J>((uint32_t)c[r], lane);
            const uint32_t hi = lane_xor<J>((uint32_t)(c[r] >> 32), lane);
            p[r] = (uint64_t)lo | ((uint64_t)hi << 32);
        }
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const bool up = (((uint32_t)(r * 64 + lane)) & (uint32_t)KK) == 0;
            if ((lower == up) == (c[r] > p[r])) c[r] = p[r];
        }
    }
    if constexpr (J > 1) reg_stage<E, KK, J / 2>(c, lane);
}

template <int E, int KK>
__device__ __forceinline__ void reg_levels(uint64_t (&c)[E], int lane) {
    reg_stage<E, KK, KK / 2>(c, lane);
    if constexpr (KK < 64 * E) reg_levels<E, KK * 2>(c, lane);
}

// Value of lane - 1 / lane + 1 of the wave (DPP wave_shr:1 / wave_shl:1);
// lane 0 / lane 63 gets its own value.
__device__ __forceinline__ uint64_t lane_prev(uint64_t v) {
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xF, 0xF, false);
    const uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xF, 0xF, false);
    return (uint64_t)a | ((uint64_t)b << 32);
}
__device__ __forceinline__ uint64_t lane_next(uint64_t v) {
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xF, 0xF, false);
    const uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xF, 0xF, false);
    return (uint64_t)a | ((uint64_t)b << 32);
}

// a key whose length field is below kshort ends at its terminator: never tied
__device__ __forceinline__ bool short_key(uint64_t k, int kshort) {
    return (k & ((1u << KEY_LEN_BITS) - 1)) < (uint64_t)kshort;
}

// Tied elements of a sorted bucket of z keys held by one wave (element
// r * 64 + lane in k[r]): bit r of the result is this lane's element of row
// r; *count = tied elements of the bucket (wave-uniform).  A tied group above
// `limit` sets *large.
template <int E>
__device__ __forceinline__ uint32_t wave_ties(const uint64_t (&k)[E], uint32_t z, int kshort,
                                              uint32_t limit, uint32_t *__restrict__ large,
                                              uint32_t *count) {
    const int lane = lane_id();
    uint32_t rows = 0, run = 0, head_run = 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        const bool ok = i < z;
        uint64_t kp = lane_prev(k[r]);
        uint64_t kn = lane_next(k[r]);
        const uint64_t last_prev = r > 0 ? __shfl(k[r > 0 ? r - 1 : 0], 63, 64) : 0ull;
        const uint64_t first_next = r + 1 < E ? __shfl(k[r + 1 < E ? r + 1 : r], 0, 64) : 0ull;
        if (lane == 0) kp = last_prev;
        if (lane == 63) kn = first_next;
        const bool eq_prev = ok && i > 0 && kp == k[r];
        const bool eq_next = ok && i + 1 < z && kn == k[r];
        const bool t = ok && !short_key(k[r], kshort) && (eq_prev || eq_next);
        run += (uint32_t)__popcll(__ballot(t));
        rows |= (t ? 1u : 0u) << r;
        // size of a group, at its last element: index of its head by a
        // running maximum over the heads
        const uint32_t hv = (ok && !eq_prev) ? i : 0u;
        uint32_t hm = wave_incl_max(hv);
        hm = hm > head_run ? hm : head_run;
        head_run = __shfl(hm, 63, 64);
        if (t && !eq_next && i - hm + 1 > limit) atomicOr(large, 1u);
    }
    *count = run;
    return rows;
}

// One bucket of z (2 .. 64 * E) suffixes at window offset st (keys s_k,
// values s_v in LDS), sorted by one wave and written to position p0 of
// kout / vout; its tie flags go to s_f[st ..].  Returns its number of tied
// suffixes.
template <int E>
__device__ uint32_t wave_bucket(const uint64_t *__restrict__ s_k, const uint32_t *__restrict__ s_v,
                                uint32_t st, uint32_t z, uint64_t *__restrict__ kout,
                                uint32_t *__restrict__ vout, uint32_t p0, int bshift, int kshort,
                                uint32_t limit, uint32_t *__restrict__ large,
                                uint8_t *__restrict__ s_f) {
    const int lane = lane_id();
    uint64_t k[E];
    uint32_t x[E];
    if (bshift <= 56) {
        // one word per suffix: (key - bucket base) << 8 | index in the bucket
        const uint64_t base = (s_k[st] >> bshift) << bshift;
        uint64_t c[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t i = (uint32_t)(r * 64 + lane);
            c[r] = i < z ? ((s_k[st + i] - base) << 8) | (uint64_t)i : ~0ull;
        }
        reg_levels<E, 2>(c, lane);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t i = (uint32_t)(r * 64 + lane);
            k[r] = i < z ? base + (c[r] >> 8) : ~0ull;
            x[r] = (uint32_t)(c[r] & 255u);
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t i = (uint32_t)(r * 64 + lane);
            x[r] = i;
            k[r] = i < z ? s_k[st + i] : ~0ull;  // a real key never has all length bits set
        }
        wave_bitonic<E>(k, x, lane);
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        if (i < z) {
            kout[p0 + i] = k[r];
            vout[p0 + i] = s_v[st + x[r]];
        }
    }
    uint32_t cnt;
    const uint32_t rows = wave_ties<E>(k, z, kshort, limit, large, &cnt);
#pragma unroll
    for (int r = 0; r < E; ++r)
        if ((rows >> r) & 1u) s_f[st + r * 64 + lane] = 1;
    return cnt;
}

// ---- exclusive scans over the bucket table, three columns at once:
// tied suffixes, oversized buckets, oversized suffixes (tiles of 4096 ids)
constexpr uint32_t BT_TILE = 4096;

__global__ __launch_bounds__(256) void bucket_scan_up_kernel(const uint32_t *__restrict__ tcnt,
                                                             const uint32_t *__restrict__ osz,
                                                             uint32_t nb,
                                                             uint32_t *__restrict__ part) {
    __shared__ uint32_t s_tmp[4];
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    uint32_t a = 0, c = 0, e = 0;
    uint32_t ar[BT_TILE / 256], zr[BT_TILE / 256];
#pragma unroll
    for (uint32_t q = 0; q < BT_TILE / 256; ++q) {
        const uint32_t b = t * BT_TILE + q * 256 + tid;
        ar[q] = b < nb ? tcnt[b] : 0u;
        zr[q] = b < nb ? osz[b] : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < BT_TILE / 256; ++q) {
        a += ar[q];
        c += zr[q] ? 1u : 0u;
        e += zr[q];
    }
    uint32_t ta, tc, te;
    (void)block_excl_sum256(a, s_tmp, &ta);
    (void)block_excl_sum256(c, s_tmp, &tc);
    (void)block_excl_sum256(e, s_tmp, &te);
    if (tid == 0) {
        part[3 * t] = ta;
        part[3 * t + 1] = tc;
        part[3 * t + 2] = te;
    }
}

// One workgroup of 1024 threads over at most 4 * 1024 tiles: exclusive tile
// offsets in place; res = {tied, oversized buckets, oversized suffixes}.
__global__ __launch_bounds__(1024) void bucket_scan_top_kernel(uint32_t *__restrict__ part,
                                                               uint32_t ntiles,
                                                               uint32_t *__restrict__ res) {
    __shared__ uint32_t s_w[16];
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    for (int col = 0; col < 3; ++col) {
        uint32_t v[4], sum = 0;
        for (int q = 0; q < 4; ++q) {
            const uint32_t t = tid * 4 + q;
            v[q] = t < ntiles ? part[3 * t + col] : 0u;
            sum += v[q];
        }
        const uint32_t inc = wave_incl_sum(sum);
        if ((tid & 63) == 63) s_w[w] = inc;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int k = 0; k < 16; ++k) {
            before += (uint32_t)k < w ? s_w[k] : 0u;
            all += s_w[k];
        }
        uint32_t run = before + inc - sum;
        for (int q = 0; q < 4; ++q) {
            const uint32_t t = tid * 4 + q;
            if (t < ntiles) part[3 * t + col] = run;
            run += v[q];
        }
        if (tid == 0) res[col] = all;
        __syncthreads();
    }
}

// tpre[b] = tied suffixes before bucket b (in place over tcnt); oversized
// buckets listed in bucket order: olist[q] = b, ooff[q] = gathered start,
// obad[q] = 0; ooff[count] = total.
__global__ __launch_bounds__(256) void bucket_scan_down_kernel(
    uint32_t *__restrict__ tcnt, const uint32_t *__restrict__ osz, uint32_t nb,
    const uint32_t *__restrict__ part, const uint32_t *__restrict__ res,
    uint32_t *__restrict__ olist, uint32_t *__restrict__ ooff, uint32_t *__restrict__ obad) {
    __shared__ uint32_t s_tmp[4];
    constexpr uint32_t PER = BT_TILE / 256;  // consecutive bucket ids per thread
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    const uint32_t b0 = t * BT_TILE + tid * PER;
    uint32_t ar[PER], zr[PER];
    uint32_t sa = 0, sc = 0, se = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t b = b0 + q;
        ar[q] = b < nb ? tcnt[b] : 0u;
        zr[q] = b < nb ? osz[b] : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        sa += ar[q];
        sc += zr[q] ? 1u : 0u;
        se += zr[q];
    }
    uint32_t ta, tc, te;
    uint32_t ra = part[3 * t] + block_excl_sum256(sa, s_tmp, &ta);
    uint32_t rc = part[3 * t + 1] + block_excl_sum256(sc, s_tmp, &tc);
    uint32_t re = part[3 * t + 2] + block_excl_sum256(se, s_tmp, &te);
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t b = b0 + q;
        if (b < nb) {
            tcnt[b] = ra;
            if (zr[q]) {
                olist[rc] = b;
                ooff[rc] = re;
                obad[rc] = 0;
            }
        }
        ra += ar[q];
        rc += zr[q] ? 1u : 0u;
        re += zr[q];
    }
    if (t == 0 && tid == 0) ooff[res[1]] = res[2];
}

// ---- tile-wise finish: a workgroup owns the buckets that start in its tile
// of BT_T positions; they end at most BUCKET_CAP past it unless oversized.
constexpr uint32_t BT_T = 2048;
constexpr uint32_t BT_WIN = BT_T + BUCKET_CAP;

// Rows of packed buckets sorted together by one wave.  One: with more rows
// at once the compare masks of every row are live together and the scalar
// registers spill into vector lanes, which costs more VALU than the overlap
// of the rows' exchanges saves (1 row: 16.3 ms of bucket finish on the
// 250k long-read workload, 2: 16.9, 4: 17.7).
constexpr int PACK_ROWS = 1;

// Sorts up to PACK_ROWS rows of whole consecutive buckets held in LDS (row r:
// window offsets rst[r] .. rst[r] + rlen[r] - 1, first bucket rid[r]; rlen 0
// = no row), one row per register, into kout / vout at t0 + offset.  Tied
// suffixes get their flag in s_f, and the last lane of each bucket with ties
// writes the bucket's tie count.
__device__ __forceinline__ void sort_packed_rows(
    const uint64_t *__restrict__ s_k, const uint32_t *__restrict__ s_v, const uint32_t (&rst)[PACK_ROWS],
    const uint32_t (&rlen)[PACK_ROWS], const uint32_t (&rid)[PACK_ROWS], uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint32_t t0, int bshift, int kshort, uint8_t *__restrict__ s_f,
    uint32_t *__restrict__ tcnt) {
    const int lane = lane_id();
    const uint32_t l = (uint32_t)lane;
    uint64_t c[PACK_ROWS];
#pragma unroll
    for (int r = 0; r < PACK_ROWS; ++r) {
        const uint64_t base = (uint64_t)rid[r] << bshift;
        c[r] = l < rlen[r] ? ((s_k[rst[r] + l] - base) << 6) | (uint64_t)l
                           : ~0ull;  // a real key never has all length bits set
    }
    wave_sort_rows<PACK_ROWS, 64>(c, lane);
    const uint64_t le = lanemask_lt() | (1ull << lane);  // lanes up to this one
#pragma unroll
    for (int r = 0; r < PACK_ROWS; ++r) {
        const bool ok = l < rlen[r];
        const uint64_t k = ok ? ((uint64_t)rid[r] << bshift) + (c[r] >> 6) : ~0ull;
        if (ok) {
            kout[t0 + rst[r] + l] = k;
            vout[t0 + rst[r] + l] = s_v[rst[r] + (uint32_t)(c[r] & 63u)];
        }
        const uint64_t kp = lane_prev(k);
        const uint64_t kn = lane_next(k);
        const bool eq_prev = ok && l > 0 && kp == k;
        const bool eq_next = ok && l + 1 < rlen[r] && kn == k;
        const bool t = ok && !short_key(k, kshort) && (eq_prev || eq_next);
        if (t) s_f[rst[r] + l] = 1;
        const uint64_t tb = __ballot(t);
        if (tb) {
            const uint64_t id = k >> bshift;
            const bool head = ok && (l == 0 || (kp >> bshift) != id);
            const bool last = ok && (l + 1 == rlen[r] || (kn >> bshift) != id);
            const uint64_t hb = __ballot(head);
            if (last) {
                // lanes of this bucket: from its head (the highest head at or
                // below this lane) up to this lane
                const int first = 63 - __builtin_clzll(hb & le);
                const uint32_t cnt = (uint32_t)__popcll(tb & le & ~((1ull << first) - 1ull));
                if (cnt) tcnt[(uint32_t)id] = cnt;
            }
        }
    }
}

// First position in [lo, hi) whose bucket (key >> bshift) is not bkt, where
// the positions of bucket bkt form a prefix of [lo, hi); hi if there is none.
// One wave, 65-way steps: about five dependent loads for a whole block.
__device__ uint32_t bucket_end_search(const uint64_t *__restrict__ keys, int bshift, uint64_t bkt,
                                      uint32_t lo, uint32_t hi) {
    const int lane = lane_id();
    while (hi - lo > 64) {
        const uint64_t span = hi - lo;
        // strictly increasing probes inside (lo, hi)
        const uint32_t pr = lo + (uint32_t)((span * (uint64_t)(lane + 1)) / 65u);
        const bool eq = (keys[pr] >> bshift) == bkt;
        const int c = __popcll(__ballot(eq));  // the equal lanes are a prefix
        const uint32_t plo = __shfl(pr, c > 0 ? c - 1 : 0, 64);
        const uint32_t phi = __shfl(pr, c < 64 ? c : 63, 64);
        if (c > 0) lo = plo + 1;
        if (c < 64) hi = phi;
    }
    const uint32_t p = lo + (uint32_t)lane;
    const bool ne = p < hi && (keys[p] >> bshift) != bkt;
    const uint64_t m = __ballot(ne);
    return m ? lo + (uint32_t)__builtin_ctzll(m) : hi;
}

// One workgroup per tile of BT_T positions of the key array kin (sorted by
// the top digits, so each bucket is a contiguous run).  It loads the window
// [t0, t0 + BT_WIN) and finds the bucket starts in it; it owns the buckets
// that start in [t0, t0 + BT_T), which end inside the window unless they are
// oversized.  Those of at most BUCKET_CAP suffixes are sorted in registers:
// groups of four buckets of at most 64 (one per row, or eight of at most 32
// in half rows), larger ones one at a time, and written to kout / vout at the
// same positions (kin is only read, so the windows that overlap the next tile
// see unchanged keys).  Per owned bucket b it records tcnt[b] (tied suffixes)
// and, when oversized, osz[b] (its size) and bstart[b] (its start); both
// tables are zeroed beforehand.  trange[3t], trange[3t + 1] = the owned range
// [a, e), trange[3t + 2] = its first bucket, and tflag[p] for p in
// [a, min(e, t0 + BT_WIN)) = 1 if the suffix is tied, else 0.
__global__ __launch_bounds__(256) void bucket_tile_sort_kernel(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t n, int bshift, uint32_t nb,
    uint32_t *__restrict__ bstart, uint32_t *__restrict__ trange, int kshort, uint32_t limit,
    uint32_t *__restrict__ large, uint32_t *__restrict__ tcnt, uint32_t *__restrict__ osz,
    uint8_t *__restrict__ tflag, uint32_t *__restrict__ err) {
    __shared__ uint64_t s_k[BT_WIN];
    __shared__ uint32_t s_v[BT_WIN];
    __shared__ uint16_t s_bs[BT_WIN + 1];
    __shared__ uint32_t s_tmp[4];
    __shared__ uint8_t s_f[BT_WIN];
    __shared__ uint32_t s_end;
    const uint32_t tid = threadIdx.x;
    const int wave = (int)(tid >> 6), lane = lane_id();
    const uint32_t t0 = blockIdx.x * BT_T;
    const uint32_t wl = n - t0 < BT_WIN ? n - t0 : BT_WIN;
    const uint64_t bprev = t0 > 0 ? kin[t0 - 1] >> bshift : ~0ull;
    {
        // all of a thread's loads go out before the first LDS store
        constexpr uint32_t PER = (BT_WIN + 255) / 256;
        uint64_t kr[PER];
        uint32_t vr[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint32_t i = tid + 256 * q;
            kr[q] = i < wl ? kin[t0 + i] : 0ull;
            vr[q] = i < wl ? vin[t0 + i] : 0u;
        }
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint32_t i = tid + 256 * q;
            if (i < wl) {
                s_k[i] = kr[q];
                s_v[i] = vr[q];
                s_f[i] = 0;
            }
        }
    }
    __syncthreads();
    // bucket starts of the window, in order (each thread a contiguous run);
    // nbk of them lie in the tile
    uint32_t nbk;
    {
        constexpr uint32_t PER = (BT_WIN + 255) / 256;
        const uint32_t i0 = tid * PER;
        uint32_t flags = 0, cnt = 0, own = 0;
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint32_t i = i0 + q;
            if (i < wl) {
                const uint64_t bi = s_k[i] >> bshift;
                if (bi != (i ? s_k[i - 1] >> bshift : bprev)) {
                    flags |= 1u << q;
                    ++cnt;
                    own += i < BT_T ? 1u : 0u;
                }
                if (bi >= nb) atomicOr(err, 256u);
            }
        }
        uint32_t tot;
        uint32_t at = block_excl_sum256(cnt, s_tmp, &tot);
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q)
            if ((flags >> q) & 1u) s_bs[at++] = (uint16_t)(i0 + q);
        (void)block_excl_sum256(own, s_tmp, &nbk);
        if (tid == 0) s_bs[tot] = (uint16_t)wl;
    }
    __syncthreads();
    if (nbk == 0) {
        if (tid == 0) {
            trange[3 * blockIdx.x] = 0;
            trange[3 * blockIdx.x + 1] = 0;
            trange[3 * blockIdx.x + 2] = 0;
        }
        return;
    }
    // end of the last owned bucket: the next start in the window, else the
    // window reaches the end of the keys, else the bucket is oversized and
    // goes on past the window
    if (wave == 0) {
        const uint32_t e = s_bs[nbk];
        uint32_t end = t0 + e;
        if (e == wl && t0 + wl < n)
            end = bucket_end_search(kin, bshift, s_k[s_bs[nbk - 1]] >> bshift, t0 + wl, n);
        if (lane == 0) {
            s_end = end;
            trange[3 * blockIdx.x] = t0 + s_bs[0];
            trange[3 * blockIdx.x + 1] = end;
            trange[3 * blockIdx.x + 2] = (uint32_t)(s_k[s_bs[0]] >> bshift);
        }
    }
    __syncthreads();
    const uint32_t tend = s_end - t0;  // may exceed the window (oversized)
    // Each wave takes a quarter of the owned buckets in order and packs runs
    // of whole consecutive buckets of at most 64 suffixes into rows of at
    // most 64 lanes; PACK_ROWS rows are sorted at once.  A row's words are
    // (key - first bucket's base) << 6 | lane, so one sort orders its
    // buckets apart and each bucket inside (buckets id0 .. id0 + span - 1 fit
    // one word).  Larger buckets are sorted one at a time; oversized ones are
    // only recorded.
    const uint32_t span = bshift > 58 ? 0u : bshift >= 27 ? (1u << (58 - bshift)) : 0xffffffffu;
    {
        const uint32_t jb0 = nbk * (uint32_t)wave / 4, jb1 = nbk * (uint32_t)(wave + 1) / 4;
        uint32_t rst[PACK_ROWS] = {}, rlen[PACK_ROWS] = {}, rid[PACK_ROWS] = {};
        uint32_t nr = 0;
        uint32_t cst = 0, clen = 0, cid = 0;  // the open row (none while clen == 0)
        for (uint32_t jb = jb0; jb < jb1; jb += 64) {
            // lane q holds bucket jb + q of this batch
            const uint32_t jl = jb + (uint32_t)lane;
            uint32_t st_l = 0, z_l = 0, id_l = 0;
            if (jl < jb1) {
                st_l = s_bs[jl];
                z_l = (jl + 1 < nbk ? (uint32_t)s_bs[jl + 1] : tend) - st_l;
                id_l = (uint32_t)(s_k[st_l] >> bshift);
            }
            const uint32_t cnt = jb1 - jb < 64 ? jb1 - jb : 64;
            for (uint32_t q = 0; q < cnt; ++q) {
                const uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)st_l, (int)q);
                const uint32_t z = (uint32_t)__builtin_amdgcn_readlane((int)z_l, (int)q);
                const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)id_l, (int)q);
                const bool small = span != 0 && z <= 64;
                if (clen && (!small || clen + z > 64 || id - cid >= span)) {
                    // close the open row
#pragma unroll
                    for (int r = PACK_ROWS - 1; r > 0; --r) {
                        rst[r] = rst[r - 1];
                        rlen[r] = rlen[r - 1];
                        rid[r] = rid[r - 1];
                    }
                    rst[0] = cst;
                    rlen[0] = clen;
                    rid[0] = cid;
                    clen = 0;
                    if (++nr == PACK_ROWS) {
                        sort_packed_rows(s_k, s_v, rst, rlen, rid, kout, vout, t0, bshift, kshort,
                                         s_f, tcnt);
                        nr = 0;
#pragma unroll
                        for (int r = 0; r < PACK_ROWS; ++r) rlen[r] = 0;
                    }
                }
                if (small) {
                    if (!clen) {
                        cst = st;
                        cid = id;
                    }
                    clen += z;
                } else if (z <= BUCKET_CAP) {
                    uint32_t tt;
                    if (z <= 64) tt = wave_bucket<1>(s_k, s_v, st, z, kout, vout, t0 + st, bshift, kshort, limit, large, s_f);
                    else if (z <= 128) tt = wave_bucket<2>(s_k, s_v, st, z, kout, vout, t0 + st, bshift, kshort, limit, large, s_f);
                    else tt = wave_bucket<4>(s_k, s_v, st, z, kout, vout, t0 + st, bshift, kshort, limit, large, s_f);
                    if (lane == 0 && tt && id < nb) tcnt[id] = tt;
                } else if (lane == 0 && id < nb) {
                    osz[id] = z;
                    bstart[id] = t0 + st;
                }
            }
        }
        if (clen) {
#pragma unroll
            for (int r = PACK_ROWS - 1; r > 0; --r) {
                rst[r] = rst[r - 1];
                rlen[r] = rlen[r - 1];
                rid[r] = rid[r - 1];
            }
            rst[0] = cst;
            rlen[0] = clen;
            rid[0] = cid;
            ++nr;
        }
        if (nr)
            sort_packed_rows(s_k, s_v, rst, rlen, rid, kout, vout, t0, bshift, kshort, s_f, tcnt);
    }
    __syncthreads();
    const uint32_t fe = tend < wl ? tend : wl;
    for (uint32_t i = s_bs[0] + tid; i < fe; i += 256) tflag[t0 + i] = s_f[i];
}

// Lists the tied suffixes of the owned buckets of tile t in slot order, from
// U[tpre[b]] for the tile's first bucket b, using the flags the tile sort left
// for the owned part of the tile's window (one workgroup; s_f holds BT_WIN
// bytes, s_tmp 4 words).
__device__ void emit_tile(const uint8_t *__restrict__ tflag, const uint32_t *__restrict__ trange,
                          const uint32_t *__restrict__ tpre, uint32_t nb, uint32_t *__restrict__ U,
                          uint32_t ucap, uint32_t *__restrict__ err, uint32_t t,
                          uint8_t *__restrict__ s_f, uint32_t *__restrict__ s_tmp) {
    const uint32_t tid = threadIdx.x;
    const uint32_t a = trange[3 * t], b = trange[3 * t + 1];
    if (a >= b) return;
    const uint32_t id = trange[3 * t + 2];
    const uint32_t base0 = id < nb ? tpre[id] : 0u;
    const uint32_t t0 = t * BT_T;
    const uint32_t w = (b - t0 < BT_WIN ? b : t0 + BT_WIN) - a;
    {
        constexpr uint32_t PER = (BT_WIN + 255) / 256;
        uint8_t fr[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint32_t i = tid + 256 * q;
            fr[q] = i < w ? tflag[a + i] : (uint8_t)0;
        }
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint32_t i = tid + 256 * q;
            if (i < w) s_f[i] = fr[q];
        }
    }
    __syncthreads();
    // each thread a contiguous run of the window, so the list keeps order
    constexpr uint32_t PER = (BT_WIN + 255) / 256;
    const uint32_t i0 = tid * PER;
    uint32_t flags = 0, cnt = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t i = i0 + q;
        if (i < w && s_f[i]) {
            flags |= 1u << q;
            ++cnt;
        }
    }
    uint32_t tot;
    uint32_t at = block_excl_sum256(cnt, s_tmp, &tot);
    if (tot == 0) return;
    if (id >= nb) {
        if (tid == 0) atomicOr(err, 512u);
        return;
    }
    const uint32_t base = base0;
    if (base + tot > ucap) {
        if (tid == 0) atomicOr(err, 512u);
        return;
    }
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q)
        if ((flags >> q) & 1u) U[base + at++] = a + i0 + q;
}

// Gathered index j lies in the oversized bucket olist[q] with
// ooff[q] <= j < ooff[q + 1] (the list is in bucket order).
__global__ void oversize_gather_kernel(const uint64_t *__restrict__ keys,
                                       const uint32_t *__restrict__ vals,
                                       const uint32_t *__restrict__ bstart,
                                       const uint32_t *__restrict__ olist,
                                       const uint32_t *__restrict__ ooff, uint32_t nob, uint32_t no,
                                       uint32_t n, uint64_t *__restrict__ ck,
                                       uint32_t *__restrict__ cv, uint32_t *__restrict__ err) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= no) return;
    uint32_t lo = 0, hi = nob - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (ooff[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t src = bstart[olist[lo]] + (j - ooff[lo]);
    if (src >= n) {
        atomicOr(err, 256u);
        return;
    }
    ck[j] = keys[src];
    cv[j] = vals[src];
}

// The sorted gathered array keeps the bucket order, so bucket olist[q]
// occupies [ooff[q], ooff[q + 1]) of it again: element j goes back to
// bstart[b] + (j - ooff[q]).
__global__ void oversize_scatter_kernel(const uint64_t *__restrict__ ck,
                                        const uint32_t *__restrict__ cv, uint32_t no,
                                        const uint32_t *__restrict__ bstart,
                                        const uint32_t *__restrict__ olist,
                                        const uint32_t *__restrict__ ooff, uint32_t nob,
                                        uint32_t n, uint64_t *__restrict__ keys,
                                        uint32_t *__restrict__ vals, uint32_t *__restrict__ err) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= no) return;
    uint32_t lo = 0, hi = nob - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (ooff[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t dst = bstart[olist[lo]] + (j - ooff[lo]);
    if (dst >= n) {
        atomicOr(err, 256u);
        return;
    }
    keys[dst] = ck[j];
    vals[dst] = cv[j];
}

// Tied elements of the gathered array (listed by the group scan as gathered
// indices U2[t], t < *nU2) appended to U as block slots after the first
// base = res[0] entries; *nU = base + *nU2.
__global__ void oversize_ties_map_kernel(const uint32_t *__restrict__ U2,
                                         const uint32_t *__restrict__ nU2,
                                         const uint32_t *__restrict__ bstart,
                                         const uint32_t *__restrict__ olist,
                                         const uint32_t *__restrict__ ooff, uint32_t nob,
                                         uint32_t no, uint32_t base, uint32_t ucap,
                                         uint32_t *__restrict__ U, uint32_t *__restrict__ nU,
                                         uint32_t *__restrict__ err) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t m = *nU2;
    if (t == 0) *nU = base + m;
    if (t >= m) return;
    const uint32_t j = U2[t];
    if (j >= no || base + t >= ucap) {
        atomicOr(err, 512u);
        return;
    }
    uint32_t lo = 0, hi = nob - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (ooff[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    U[base + t] = bstart[olist[lo]] + (j - ooff[lo]);
}

// Oversized bucket q (gathered index j, as for the gather) copied from
// (kx, vx) to (ky, vy) at the same positions; obad[q] is set when one of its
// keys differs from its first key or does not end at a terminator.  A bucket
// with obad[q] == 0 holds copies of one settled key: it is already in its
// final order (position order, which the stable passes kept) and has no ties.
// The counts come from the bucket scans (res[1] buckets, res[2] suffixes).
__device__ void check_chunk(const uint64_t *__restrict__ kx, const uint32_t *__restrict__ vx,
                            uint64_t *__restrict__ ky, uint32_t *__restrict__ vy,
                            const uint32_t *__restrict__ bstart, const uint32_t *__restrict__ olist,
                            const uint32_t *__restrict__ ooff, const uint32_t *__restrict__ res,
                            uint32_t n, int kshort, uint32_t *__restrict__ obad,
                            uint32_t *__restrict__ err, uint32_t g, uint32_t G) {
    const uint32_t nob = res[1], no = res[2];
    if (no > n || (no > 0 && nob == 0)) {  // cannot happen; keeps the indexing in bounds
        if (g == 0 && threadIdx.x == 0) atomicOr(err, 256u);
        return;
    }
    const int lane = lane_id();
    // workgroup g of G takes the gathered indices [c0, c1), 256 at a time; each
    // wave finds its bucket once and then only steps forward (a bucket holds
    // more than 64 suffixes, so a step of 64 indices crosses at most one end)
    const uint32_t per = (no + G - 1) / G;
    const uint32_t c0 = g * per, c1 = c0 + per < no ? c0 + per : no;
    const uint32_t wave_off = threadIdx.x & ~63u;
    uint32_t qw = 0;
    if (c0 + wave_off < c1 && lane == 0) {
        const uint32_t jw = c0 + wave_off;
        uint32_t lo = 0, hi = nob - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (ooff[mid] <= jw) lo = mid;
            else hi = mid - 1;
        }
        qw = lo;
    }
    uint32_t q = __shfl(qw, 0, 64);
    for (uint32_t j0 = c0; j0 < c1; j0 += blockDim.x) {
        const uint32_t j = j0 + threadIdx.x;
        bool mis = false;
        if (j < c1) {
            while (q + 1 < nob && ooff[q + 1] <= j) ++q;
            const uint32_t p0 = bstart[olist[q]], pos = p0 + (j - ooff[q]);
            if (pos < n) {
                const uint64_t k = kx[pos];
                ky[pos] = k;
                vy[pos] = vx[pos];
                mis = k != kx[p0] || !short_key(k, kshort);
            } else {
                atomicOr(err, 256u);
            }
        }
        // one flag update per bucket per wave (q does not decrease along the lanes)
        const uint64_t m = __ballot(mis);
        const uint64_t below = m & lanemask_lt();
        const int prev = below ? 63 - __builtin_clzll(below) : lane;
        const uint32_t qprev = __shfl(q, prev, 64);
        if (mis && (below == 0 || qprev != q)) atomicOr(&obad[q], 1u);
        // every lane takes the bucket of the wave's last lane into the next step
        q = __shfl(q, 63, 64);
    }
}

// The emit of every tile and the copy and check of the oversized buckets in
// one launch: both need only the bucket scans, so they run side by side.
// Workgroups below ntiles emit tile blockIdx.x; the others take chunk
// blockIdx.x - ntiles of G.
__global__ __launch_bounds__(256) void emit_and_check_kernel(
    const uint8_t *__restrict__ tflag, const uint32_t *__restrict__ trange,
    const uint32_t *__restrict__ tpre, uint32_t nb, uint32_t *__restrict__ U, uint32_t ucap,
    uint32_t ntiles, const uint64_t *__restrict__ kx, const uint32_t *__restrict__ vx,
    uint64_t *__restrict__ ky, uint32_t *__restrict__ vy, const uint32_t *__restrict__ bstart,
    const uint32_t *__restrict__ olist, const uint32_t *__restrict__ ooff,
    const uint32_t *__restrict__ res, uint32_t n, int kshort, uint32_t *__restrict__ obad,
    uint32_t G, uint32_t *__restrict__ err) {
    __shared__ uint8_t s_f[BT_WIN];
    __shared__ uint32_t s_tmp[4];
    if (blockIdx.x < ntiles)
        emit_tile(tflag, trange, tpre, nb, U, ucap, err, blockIdx.x, s_f, s_tmp);
    else
        check_chunk(kx, vx, ky, vy, bstart, olist, ooff, res, n, kshort, obad, err,
                    blockIdx.x - ntiles, G);
}

// The oversized buckets with obad set, listed again in bucket order (one
// workgroup of 1024 threads, res[1] buckets): olist2[c] = olist[q], ooff2[c] =
// their gathered start; ooff2[count] = total; res2 = {count, total}.
__global__ __launch_bounds__(1024) void oversize_compact_kernel(
    const uint32_t *__restrict__ olist, const uint32_t *__restrict__ ooff,
    const uint32_t *__restrict__ obad, const uint32_t *__restrict__ res, uint32_t nbmax,
    uint32_t *__restrict__ olist2, uint32_t *__restrict__ ooff2, uint32_t *__restrict__ res2) {
    __shared__ uint32_t s_w[2][16];
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t nob = res[1] < nbmax ? res[1] : 0u;  // more cannot happen
    uint32_t rc = 0, re = 0;  // buckets and suffixes kept so far
    for (uint32_t base = 0; base < nob; base += 1024) {
        const uint32_t q = base + tid;
        const uint32_t keep = q < nob && obad[q] ? 1u : 0u;
        const uint32_t z = keep ? ooff[q + 1] - ooff[q] : 0u;
        const uint32_t ic = wave_incl_sum(keep), ie = wave_incl_sum(z);
        if ((tid & 63) == 63) {
            s_w[0][w] = ic;
            s_w[1][w] = ie;
        }
        __syncthreads();
        uint32_t bc = 0, be = 0, tc = 0, te = 0;
        for (uint32_t k = 0; k < 16; ++k) {
            bc += k < w ? s_w[0][k] : 0u;
            be += k < w ? s_w[1][k] : 0u;
            tc += s_w[0][k];
            te += s_w[1][k];
        }
        if (keep) {
            olist2[rc + bc + ic - 1] = olist[q];
            ooff2[rc + bc + ic - 1] = re + be + ie - z;
        }
        rc += tc;
        re += te;
        __syncthreads();
    }
    if (tid == 0) {
        ooff2[rc] = re;
        res2[0] = rc;
        res2[1] = re;
    }
}

}  // namespace

hipError_t launch_bucket_sort(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                              uint32_t *vout, uint32_t n, uint32_t *bstart, uint32_t *trange,
                              uint32_t nb, int bshift, int kshort, uint32_t limit, uint32_t *large,
                              uint32_t *tcnt, uint32_t *osz, uint8_t *tflag, uint32_t *part,
                              uint32_t *res, uint32_t *olist, uint32_t *ooff, uint32_t *obad,
                              uint32_t *err, hipStream_t s, const Marks *mk) {
    const uint32_t ntiles = (uint32_t)div_up(nb, BT_TILE);
    if (ntiles > 4 * 1024) return hipErrorInvalidValue;
    fill_u32_kernel<<<(unsigned)div_up(nb, 256), 256, 0, s>>>(tcnt, nb, 0u);
    fill_u32_kernel<<<(unsigned)div_up(nb, 256), 256, 0, s>>>(osz, nb, 0u);
    const uint32_t nt = (uint32_t)div_up(n, BT_T);
    Marks::begin(mk, 0, s);
    if (nt > 0)
        bucket_tile_sort_kernel<<<nt, 256, 0, s>>>(kin, vin, kout, vout, n, bshift, nb, bstart,
                                                   trange, kshort, limit, large, tcnt, osz, tflag,
                                                   err);
    Marks::end(mk, 0, s);
    bucket_scan_up_kernel<<<ntiles, 256, 0, s>>>(tcnt, osz, nb, part);
    bucket_scan_top_kernel<<<1, 1024, 0, s>>>(part, ntiles, res);
    bucket_scan_down_kernel<<<ntiles, 256, 0, s>>>(tcnt, osz, nb, part, res, olist, ooff, obad);
    return hipGetLastError();
}

hipError_t launch_emit_and_check(const uint8_t *tflag, uint32_t n, const uint32_t *trange,
                                 const uint32_t *tpre, uint32_t nb, uint32_t *U, uint32_t ucap,
                                 const uint64_t *kx, const uint32_t *vx, uint64_t *ky,
                                 uint32_t *vy, const uint32_t *bstart, const uint32_t *olist,
                                 const uint32_t *ooff, const uint32_t *res, int kshort,
                                 uint32_t *obad, uint32_t *olist2, uint32_t *ooff2,
                                 uint32_t *res2, uint32_t *err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t ntiles = (uint32_t)div_up(n, BT_T);
    const uint32_t want = (uint32_t)div_up(n, 256);
    const uint32_t G = want < 8192 ? want : 8192;
    emit_and_check_kernel<<<ntiles + G, 256, 0, s>>>(tflag, trange, tpre, nb, U, ucap, ntiles, kx,
                                                     vx, ky, vy, bstart, olist, ooff, res, n,
                                                     kshort, obad, G, err);
    oversize_compact_kernel<<<1, 1024, 0, s>>>(olist, ooff, obad, res, nb, olist2, ooff2, res2);
    return hipGetLastError();
}

hipError_t launch_oversize_gather(const uint64_t *keys, const uint32_t *vals,
                                  const uint32_t *bstart, const uint32_t *olist,
                                  const uint32_t *ooff, uint32_t nob, uint32_t no, uint32_t n,
                                  uint64_t *ck, uint32_t *cv, uint32_t *err, hipStream_t s) {
    if (no == 0 || nob == 0) return hipSuccess;
    oversize_gather_kernel<<<(unsigned)div_up(no, 256), 256, 0, s>>>(keys, vals, bstart, olist,
                                                                    ooff, nob, no, n, ck, cv, err);
    return hipGetLastError();
}

hipError_t launch_oversize_scatter(const uint64_t *ck, const uint32_t *cv, uint32_t no,
                                   const uint32_t *bstart, const uint32_t *olist,
                                   const uint32_t *ooff, uint32_t nob, uint32_t n, uint64_t *keys,
                                   uint32_t *vals, uint32_t *err, hipStream_t s) {
    if (no == 0 || nob == 0) return hipSuccess;
    oversize_scatter_kernel<<<(unsigned)div_up(no, 256), 256, 0, s>>>(ck, cv, no, bstart, olist,
                                                                     ooff, nob, n, keys, vals, err);
    return hipGetLastError();
}

hipError_t launch_oversize_ties_map(const uint32_t *U2, const uint32_t *nU2, const uint32_t *bstart,
                                    const uint32_t *olist, const uint32_t *ooff, uint32_t nob,
                                    uint32_t no, uint32_t base, uint32_t ucap, uint32_t *U,
                                    uint32_t *nU, uint32_t *err, hipStream_t s) {
    if (no == 0 || nob == 0) return hipSuccess;
    oversize_ties_map_kernel<<<(unsigned)div_up(no, 256), 256, 0, s>>>(
        U2, nU2, bstart, olist, ooff, nob, no, base, ucap, U, nU, err);
    return hipGetLastError();
}

}  // namespace bwt
