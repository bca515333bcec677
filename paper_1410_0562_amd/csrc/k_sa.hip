// k_sa.hip -- ConstructSA of one block (Section 3) by prefix doubling over
// radix-sorted keys, and the B_int / g_sa gather of Algorithm 1.
//
// Round 0 sorts every block suffix by a 63-bit key made of its first KEY_K
// symbols (terminator-aware, see bwt_internal.hpp).  After a sort, groups of
// equal keys get the SA index of their first member as rank; singletons and
// keys that reach their terminator are final.  Each later round sorts only
// the still-unresolved suffixes by (rank[p], rank[p + h]) -- the sort
// doubles the compared prefix from h to 2h, as in Larsson-Sadakane prefix
// doubling (the paper's GPU sorter also discards resolved suffixes between
// iterations) -- and writes them back into their group's SA slots.  Since an
// unresolved suffix has at least h symbols before its terminator, p + h never
// leaves its read.
#include "dev_util.hpp"

namespace bwt {

namespace {

__global__ void block_soff_kernel(const uint64_t *__restrict__ off, uint32_t m_blk,
                                  uint32_t *__restrict__ soff) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > m_blk) return;
    soff[j] = (uint32_t)(off[j] - off[0]) + j;
}

// tile_first[T] = read containing position T << PREP_TILE_SHIFT (last read if
// the position is past the end).  soff[m_blk] = n_blk.
__global__ void block_tile_first_kernel(const uint32_t *__restrict__ soff, uint32_t m_blk,
                                        uint32_t n_blk, uint32_t ntile,
                                        uint32_t *__restrict__ tile_first) {
    uint32_t T = blockIdx.x * blockDim.x + threadIdx.x;
    if (T > ntile) return;
    uint64_t P = (uint64_t)T << PREP_TILE_SHIFT;
    uint32_t lo = 0, hi = m_blk - 1;
    if (P >= n_blk) {
        tile_first[T] = hi;
        return;
    }
    while (lo < hi) {  // largest j with soff[j] <= P
        uint32_t mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= P) lo = mid;
        else hi = mid - 1;
    }
    tile_first[T] = lo;
}

__global__ __launch_bounds__(256) void block_keys_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, const uint32_t *__restrict__ tile_first, uint32_t n_blk,
    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_blk) return;
    uint32_t T = p >> PREP_TILE_SHIFT;
    uint32_t lo = tile_first[T], hi = tile_first[T + 1];
    while (lo < hi) {  // largest j in [lo, hi] with soff[j] <= p
        uint32_t mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t j = lo;
    const uint32_t sj = soff[j];
    const uint32_t len = soff[j + 1] - sj - 1;
    const uint32_t t = p - sj;
    const uint32_t r = len - t;  // symbols before the terminator
    const uint64_t s = off[j] + t;
    const int take = r < (uint32_t)KEY_K ? (int)r : KEY_K;
    uint64_t sym = 0;
    if (take > 0) {
        uint64_t v = load_sym_window(reads, s, take);
        v &= (1ull << (2 * take)) - 1ull;
        sym = reverse_pairs(v) >> (64 - 2 * KEY_K);
    }
    keys[p] = (sym << KEY_LEN_BITS) | (uint64_t)take;
    uint32_t prev = t == 0 ? 4u : (uint32_t)load_sym(reads, s - 1);
    vals[p] = p | (prev << POS_BITS);
}

constexpr int GH_ITEMS = SCAN_TILE / 256;  // 16 rows of 64 per wave... per thread

// Group heads after a sort, with one look-back chain for the last head index
// (max) and one for the number of unresolved elements (sum).
//
// Element x (sorted order) has slot = x in round 0, U[x] in a doubling round.
//   head(x)   : x == 0, or its key differs from x-1's, or (round 0) its key
//               ends at the terminator (length field < KEY_K)
//   unresolved: in a group of two or more
//   rank[p]   = slot of the first element of x's group
//   Uout[...] = slots of unresolved elements, in increasing order
// A doubling round also stores the sorted value into SA slot U[x].
__global__ __launch_bounds__(256) void group_heads_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
    const uint32_t *__restrict__ U, uint32_t n, uint32_t *__restrict__ sa,
    uint32_t *__restrict__ rank, uint32_t *__restrict__ Uout, uint32_t *__restrict__ nUout,
    uint64_t *__restrict__ status, uint32_t *__restrict__ counter, uint32_t ntiles,
    uint32_t epoch, uint32_t *__restrict__ err) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wmax[4], s_wsum[4];
    __shared__ uint32_t s_pmax, s_psum;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t tile = acquire_tile(counter, ntiles, &s_tile);
    if (tile >= ntiles) {
        if (tid == 0) atomicOr(err, 2u);
        return;
    }
    const uint64_t wbase = (uint64_t)tile * SCAN_TILE + (uint64_t)wave * (GH_ITEMS * 64);
    const bool round0 = (U == nullptr);

    uint32_t hx[GH_ITEMS], ui[GH_ITEMS];
    uint32_t unres_bits = 0;
    uint32_t carry_max = 0, carry_sum = 0;
#pragma unroll
    for (int e = 0; e < GH_ITEMS; ++e) {
        uint64_t x = wbase + (uint64_t)e * 64 + lane;
        bool ok = x < n;
        uint32_t hv = 0, uv = 0;
        if (ok) {
            uint64_t key = keys[x];
            bool is_short = round0 && (key & ((1u << KEY_LEN_BITS) - 1)) < (uint64_t)KEY_K;
            bool head = (x == 0) || keys[x - 1] != key || is_short;
            bool nhead = (x + 1 == n) || keys[x + 1] != key || is_short;
            bool unres = !(head && nhead);
            hv = head ? (uint32_t)x : 0u;
            uv = unres ? 1u : 0u;
            unres_bits |= (unres ? 1u : 0u) << e;
        }
        uint32_t im = wave_incl_max(hv);
        im = im > carry_max ? im : carry_max;
        uint32_t is = wave_incl_sum(uv) + carry_sum;
        hx[e] = im;
        ui[e] = is - uv;
        carry_max = __shfl(im, 63, 64);
        carry_sum = __shfl(is, 63, 64);
    }
    if (lane == 0) {
        s_wmax[wave] = carry_max;
        s_wsum[wave] = carry_sum;
    }
    __syncthreads();
    uint32_t wpmax = 0, wpsum = 0;
    for (int w = 0; w < wave; ++w) {
        wpmax = wpmax > s_wmax[w] ? wpmax : s_wmax[w];
        wpsum += s_wsum[w];
    }
    if (wave == 0 && lane < 2) {
        uint32_t tmax = 0, tsum = 0;
        for (int w = 0; w < 4; ++w) {
            tmax = tmax > s_wmax[w] ? tmax : s_wmax[w];
            tsum += s_wsum[w];
        }
        if (lane == 0) {
            s_pmax = lookback(status, 2u, tile, epoch, tmax, OpMax(), 0u, err);
        } else {
            uint32_t ps = lookback(status + 1, 2u, tile, epoch, tsum, OpSum(), 0u, err);
            s_psum = ps;
            if (tile == ntiles - 1) *nUout = ps + tsum;
        }
    }
    __syncthreads();
    const uint32_t pmax = s_pmax > wpmax ? s_pmax : wpmax;
    const uint32_t psum = s_psum + wpsum;
#pragma unroll
    for (int e = 0; e < GH_ITEMS; ++e) {
        uint64_t x = wbase + (uint64_t)e * 64 + lane;
        if (x >= n) continue;
        uint32_t head_x = hx[e] > pmax ? hx[e] : pmax;
        uint32_t v = vals[x];
        uint32_t slot, gs;
        if (head_x > (uint32_t)x) {  // cannot happen; guards the indexing below
            atomicOr(err, 8u);
            head_x = (uint32_t)x;
        }
        if (round0) {
            slot = (uint32_t)x;
            gs = head_x;
        } else {
            slot = U[x];
            gs = U[head_x];
            sa[slot] = v;
        }
        rank[v & POS_MASK] = gs;
        uint32_t dst = psum + ui[e];
        if ((unres_bits >> e) & 1u) {
            if (dst < n) Uout[dst] = slot;
            else atomicOr(err, 8u);
        }
    }
}

// keys of a doubling round: (rank[p] << rbits) | rank[p + h]
// (an unresolved suffix has at least h symbols before its terminator, so
// p + h stays inside its read; the clamp only keeps a broken state in bounds)
__global__ void doubling_keys_kernel(const uint32_t *__restrict__ U, uint32_t nU,
                                     const uint32_t *__restrict__ sa,
                                     const uint32_t *__restrict__ rank, uint32_t h, int rbits,
                                     uint32_t n_blk, uint64_t *__restrict__ keys,
                                     uint32_t *__restrict__ vals, uint32_t *__restrict__ err) {
    uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nU) return;
    uint32_t v = sa[U[u]];
    uint32_t p = v & POS_MASK;
    uint64_t q = (uint64_t)p + h;
    if (q >= n_blk) {
        atomicOr(err, 16u);
        q = n_blk - 1;
    }
    keys[u] = ((uint64_t)rank[p] << rbits) | (uint64_t)rank[q];
    vals[u] = v;
}

// Algorithm 1: B_int[i] = symbol before suffix SA_int[i] ('$' at a read
// start), g_sa[i] = g[SA_int[i]]
__global__ void gather_kernel(const uint32_t *__restrict__ sa, const uint64_t *__restrict__ g,
                              uint32_t n, uint8_t *__restrict__ bint, uint64_t *__restrict__ gsa) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t v = sa[i];
    const char ascii[5] = {'A', 'C', 'G', 'T', '$'};
    bint[i] = (uint8_t)ascii[v >> POS_BITS];
    gsa[i] = g[v & POS_MASK];
}

__global__ void sa_strip_kernel(const uint32_t *__restrict__ sa, uint32_t n,
                                uint32_t *__restrict__ out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = sa[i] & POS_MASK;
}

inline unsigned grid_for(uint64_t n, unsigned b) { return (unsigned)div_up(n, b); }

}  // namespace

hipError_t launch_block_soff(const uint64_t *off, uint32_t m_blk, uint32_t *soff, hipStream_t s) {
    block_soff_kernel<<<grid_for((uint64_t)m_blk + 1, 256), 256, 0, s>>>(off, m_blk, soff);
    return hipGetLastError();
}

hipError_t launch_block_tile_first(const uint32_t *soff, uint32_t m_blk, uint32_t n_blk,
                                   uint32_t *tile_first, hipStream_t s) {
    uint32_t ntile = (uint32_t)div_up(n_blk, 1u << PREP_TILE_SHIFT);
    block_tile_first_kernel<<<grid_for((uint64_t)ntile + 1, 256), 256, 0, s>>>(soff, m_blk, n_blk,
                                                                              ntile, tile_first);
    return hipGetLastError();
}

hipError_t launch_block_keys(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                             const uint32_t *tile_first, uint32_t m_blk, uint32_t n_blk,
                             uint64_t *keys, uint32_t *vals, hipStream_t s) {
    (void)m_blk;
    block_keys_kernel<<<grid_for(n_blk, 256), 256, 0, s>>>(reads, off, soff, tile_first, n_blk,
                                                          keys, vals);
    return hipGetLastError();
}

hipError_t launch_group_heads(const uint64_t *keys, const uint32_t *vals, const uint32_t *U,
                              uint32_t n, uint32_t *sa, uint32_t *rank, uint32_t *Uout,
                              uint32_t *nUout, uint64_t *status, uint32_t *counter,
                              uint32_t epoch, uint32_t *err, hipStream_t s) {
    uint32_t ntiles = (uint32_t)div_up(n, SCAN_TILE);
    if (ntiles == 0) return hipSuccess;
    group_heads_kernel<<<ntiles, 256, 0, s>>>(keys, vals, U, n, sa, rank, Uout, nUout, status,
                                              counter, ntiles, epoch, err);
    return hipGetLastError();
}

hipError_t launch_doubling_keys(const uint32_t *U, uint32_t nU, const uint32_t *sa,
                                const uint32_t *rank, uint32_t h, int rbits, uint32_t n_blk,
                                uint64_t *keys, uint32_t *vals, uint32_t *err, hipStream_t s) {
    doubling_keys_kernel<<<grid_for(nU, 256), 256, 0, s>>>(U, nU, sa, rank, h, rbits, n_blk, keys,
                                                          vals, err);
    return hipGetLastError();
}

hipError_t launch_gather(const uint32_t *sa, const uint64_t *g, uint32_t n, uint8_t *bint,
                         uint64_t *gsa, hipStream_t s) {
    gather_kernel<<<grid_for(n, 256), 256, 0, s>>>(sa, g, n, bint, gsa);
    return hipGetLastError();
}

hipError_t launch_sa_strip(const uint32_t *sa, uint32_t n, uint32_t *out, hipStream_t s) {
    sa_strip_kernel<<<grid_for(n, 256), 256, 0, s>>>(sa, n, out);
    return hipGetLastError();
}

}  // namespace bwt
