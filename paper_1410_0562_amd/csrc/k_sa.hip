// k_sa.hip -- ConstructSA of one block (Section 3) and the pieces of
// Algorithm 1 that come out of it (B_int, g_sa).
//
// Round 0 radix-sorts every block suffix by (g, first K' symbols), see
// bwt_internal.hpp: g is non-decreasing in suffix order, so it may lead the
// key, and it splits ties that symbols alone would leave.  Groups of equal
// keys that do not end at a terminator are still tied.  The usual case --
// every tied group has at most REFINE_LIMIT members -- is finished in LDS:
// one workgroup takes a window of groups and sorts each group by successive
// 29-symbol chunks of its suffixes, splitting it until every subgroup is a
// single suffix or ends at its terminator (the paper's GPU sorter likewise
// compares suffixes as strings of fixed-size words and drops settled ones
// between iterations).  A block with a larger group instead runs prefix
// doubling (Larsson-Sadakane) over all its tied suffixes: sort by
// (rank[p], rank[p + h]) so the compared prefix doubles from h to 2h; an
// unresolved suffix has at least h symbols before its terminator, so p + h
// never leaves its read.
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

// read containing block position p
__device__ __forceinline__ uint32_t find_read(const uint32_t *__restrict__ soff,
                                              const uint32_t *__restrict__ tile_first,
                                              uint32_t p) {
    uint32_t T = p >> PREP_TILE_SHIFT;
    uint32_t lo = tile_first[T], hi = tile_first[T + 1];
    while (lo < hi) {  // largest j in [lo, hi] with soff[j] <= p
        uint32_t mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Chunk key of the suffix whose first symbol is global symbol s and which
// has r symbols before its terminator: min(r, K) symbols, first one most
// significant, zero-padded to K symbols, then the count in the low 5 bits.
__device__ __forceinline__ uint64_t chunk_key(const uint8_t *__restrict__ reads, uint64_t s,
                                              uint32_t r, int K) {
    const int take = r < (uint32_t)K ? (int)r : K;
    uint64_t sym = 0;
    if (take > 0) {
        uint64_t v = load_sym_window(reads, s, take);
        v &= (1ull << (2 * take)) - 1ull;
        sym = reverse_pairs(v) >> (64 - 2 * K);
    }
    return (sym << KEY_LEN_BITS) | (uint64_t)take;
}

// A fixed grid strides over the block, one suffix per thread per step; a
// wave covers 64 consecutive positions, so lane 0 finds the read of the
// first one and every lane steps forward from there.  The counts of the
// first radix pass's digit (bits hshift .. hshift + 7 of the key) are
// gathered in LDS and added once per workgroup to one of the HIST_COPIES
// copies.
__global__ __launch_bounds__(256) void block_keys_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, const uint32_t *__restrict__ tile_first, uint32_t n_blk,
    const uint64_t *__restrict__ g, int gshift, int kfirst, int hshift,
    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, uint32_t *__restrict__ hist0) {
    __shared__ uint32_t s_h[256];
    const int tid = threadIdx.x;
    s_h[tid] = 0;
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n_blk;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p0 = (uint32_t)base + (tid & ~63);
        const uint32_t p = p0 + (tid & 63);
        if (p0 >= n_blk) continue;
        uint32_t j = 0;
        if ((tid & 63) == 0) j = find_read(soff, tile_first, p0);
        j = __shfl(j, 0, 64);
        if (p < n_blk) {
            while (soff[j + 1] <= p) ++j;
            const uint32_t sj = soff[j];
            const uint32_t t = p - sj;
            const uint32_t r = soff[j + 1] - 1 - p;  // symbols before the terminator
            const uint64_t s = off[j] + t;
            uint64_t key = kfirst > 0 ? chunk_key(reads, s, r, kfirst) : 0ull;
            if (g) key |= g[p] << gshift;
            keys[p] = key;
            uint32_t prev = t == 0 ? 4u : (uint32_t)load_sym(reads, s - 1);
            vals[p] = p | (prev << POS_BITS);
            atomicAdd(&s_h[(uint32_t)(key >> hshift) & 255u], 1u);
        }
    }
    __syncthreads();
    if (s_h[tid]) atomicAdd(&hist0[(blockIdx.x % HIST_COPIES) * 256 + tid], s_h[tid]);
}

constexpr int GH_ITEMS = SCAN_TILE / 256;  // 16 rows of 64 elements per wave

// Group heads after a sort, with one look-back chain for the last head index
// (max) and one for the number of unresolved elements (sum).
//
// Element x (sorted order) has slot = x in round 0, U[x] in a doubling round.
//   head(x)   : x == 0, or its key differs from x-1's, or (round 0) its key
//               ends at the terminator (length field < kshort)
//   unresolved: in a group of two or more
//   rank[p]   = slot of the first element of x's group (when rank != null)
//   Uout[...] = slots of unresolved elements, in increasing order
// A doubling round also stores the sorted value into SA slot U[x].
__global__ __launch_bounds__(256) void group_heads_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
    const uint32_t *__restrict__ U, uint32_t n, int kshort, uint32_t *__restrict__ sa,
    uint32_t *__restrict__ rank, uint32_t *__restrict__ Uout, uint32_t *__restrict__ nUout,
    uint32_t limit, uint32_t *__restrict__ large, uint64_t *__restrict__ status,
    uint32_t *__restrict__ counter, uint32_t ntiles, uint32_t epoch, uint32_t *__restrict__ err) {
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
    uint32_t unres_bits = 0, last_bits = 0;
    uint32_t carry_max = 0, carry_sum = 0;
#pragma unroll
    for (int e = 0; e < GH_ITEMS; ++e) {
        uint64_t x = wbase + (uint64_t)e * 64 + lane;
        bool ok = x < n;
        uint32_t hv = 0, uv = 0;
        uint64_t key = ok ? keys[x] : 0ull;
        // neighbours from the adjacent lanes; the row ends load their own
        uint64_t kprev = __shfl_up(key, 1, 64), knext = __shfl_down(key, 1, 64);
        if (ok && lane == 0 && x > 0) kprev = keys[x - 1];
        if (ok && lane == 63 && x + 1 < n) knext = keys[x + 1];
        if (ok) {
            bool is_short =
                round0 && (key & ((1u << KEY_LEN_BITS) - 1)) < (uint64_t)kshort;
            bool head = (x == 0) || kprev != key || is_short;
            bool nhead = (x + 1 == n) || knext != key || is_short;
            bool unres = !(head && nhead);
            hv = head ? (uint32_t)x : 0u;
            uv = unres ? 1u : 0u;
            unres_bits |= (unres ? 1u : 0u) << e;
            last_bits |= (unres && nhead ? 1u : 0u) << e;
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
        if (head_x > (uint32_t)x) {  // cannot happen; guards the indexing below
            atomicOr(err, 8u);
            head_x = (uint32_t)x;
        }
        if ((last_bits >> e) & 1u) {
            if ((uint32_t)x - head_x + 1 > limit) atomicOr(large, 1u);
        }
        uint32_t slot = round0 ? (uint32_t)x : U[x];
        if (!round0 || rank) {
            uint32_t v = vals[x];
            if (!round0) sa[slot] = v;
            if (rank) rank[v & POS_MASK] = round0 ? head_x : U[head_x];
        }
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

// ---------------------------------------------------------------- refinement
constexpr int RF_CAP = REFINE_WINDOW + REFINE_LIMIT;
constexpr int RF_PER_THREAD = (RF_CAP + 255) / 256;
constexpr int RF_K = 2 * KEY_K;   // symbols compared per pass
constexpr int RF_LEN_BITS = 6;    // holds a count up to RF_K
static_assert(RF_K < (1 << RF_LEN_BITS), "count field");

// U[x] starts a tied group: groups are runs of consecutive slots with equal
// round-0 keys
__device__ __forceinline__ bool group_start(const uint32_t *__restrict__ U,
                                            const uint64_t *__restrict__ keys, uint32_t x) {
    if (x == 0) return true;
    uint32_t a = U[x - 1], b = U[x];
    return a + 1 != b || keys[a] != keys[b];
}

// One workgroup per window of REFINE_WINDOW unresolved elements, extended to
// whole groups.  Every member of a group shares g and the first kfirst
// symbols.  Each pass takes, for every member of a still-tied subgroup, the
// chunk key of its suffix at depth d -- RF_K = 58 symbols as two words (the
// first 29 symbols; the next 29 symbols and the count of symbols before the
// terminator, at most RF_K), each zero-padded, first symbol most significant,
// so comparing (high word, low word) orders the chunks with the terminator
// below every base -- reorders the subgroup by (chunk key, current order) --
// stable, so members equal up to their terminators stay in position order,
// which is terminator order -- and splits it where the key changes.  A
// subgroup is settled when it has one member or its key reaches the
// terminator.  d grows by RF_K per pass, so a group settles within
// (longest read / RF_K) + 1 passes.
// One window (number `win`) of the tied suffixes U[0 .. nU).
__device__ __forceinline__ void refine_window(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, const uint32_t *__restrict__ tile_first,
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ U, uint32_t nU,
    uint32_t *__restrict__ sa, int kfirst, uint32_t max_iter, uint32_t *__restrict__ err,
    uint32_t win) {
    __shared__ uint32_t s_val[RF_CAP];
    __shared__ uint64_t s_pos[RF_CAP];   // global symbol index of the suffix start
    __shared__ uint32_t s_rem[RF_CAP];   // symbols before its terminator
    __shared__ uint64_t s_kh[RF_CAP], s_kl[RF_CAP];  // chunk key: symbols, then symbols + count
    __shared__ uint16_t s_gs[RF_CAP], s_ge[RF_CAP];  // subgroup [start, end)
    __shared__ uint32_t s_win[2];
    const int tid = threadIdx.x;
    if (tid < 128) {
        // wave 0 moves the window start, wave 1 its end, to the next group
        // start (at most REFINE_LIMIT places on, or the end of U), 64 places
        // per step
        const int wv = tid >> 6, ln = tid & 63;
        uint64_t x0 = (uint64_t)win * REFINE_WINDOW + (wv ? REFINE_WINDOW : 0);
        x0 = x0 < nU ? x0 : nU;
        uint64_t r = x0 + REFINE_LIMIT < nU ? x0 + REFINE_LIMIT : nU;
        for (uint64_t y0 = x0; y0 < r; y0 += 64) {
            const uint64_t y = y0 + ln;
            const bool st = y >= r || group_start(U, keys, (uint32_t)y);
            const uint64_t m = __ballot(st);
            if (m) {
                r = y0 + __builtin_ctzll(m);
                break;
            }
        }
        if (ln == 0) s_win[wv] = (uint32_t)r;
    }
    __syncthreads();
    const uint32_t a = s_win[0], b = s_win[1];
    if (a >= b) return;
    const uint32_t W = b - a;
    if (W > (uint32_t)RF_CAP) {
        if (tid == 0) atomicOr(err, 64u);
        return;
    }
    // load the members.  Each step issues the loads of all of a thread's
    // members before it uses any of them (a member past W works on a copy of
    // element a, so every address stays valid), which keeps the dependent
    // chain -- slot, value, read lookup, read start -- at one latency per step.
    uint32_t v_m[RF_PER_THREAD], p_m[RF_PER_THREAD], lo[RF_PER_THREAD], hi[RF_PER_THREAD];
    bool head_m[RF_PER_THREAD];
    {
        uint32_t u_m[RF_PER_THREAD], up_m[RF_PER_THREAD];
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            uint32_t ix = x < W ? a + x : a;
            u_m[t] = U[ix];
            up_m[t] = U[ix > 0 ? ix - 1 : 0];
        }
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            uint32_t ix = x < W ? a + x : a;
            v_m[t] = sa[u_m[t]];
            uint64_t ku = keys[u_m[t]], kp = keys[up_m[t]];
            head_m[t] = ix == 0 || up_m[t] + 1 != u_m[t] || kp != ku;
        }
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            p_m[t] = v_m[t] & POS_MASK;
            uint32_t T = p_m[t] >> PREP_TILE_SHIFT;
            lo[t] = tile_first[T];
            hi[t] = tile_first[T + 1];
        }
    }
    // read of each member: largest j in [lo, hi] with soff[j] <= p, all of a
    // thread's searches stepping together
    for (;;) {
        bool more = false;
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) more |= lo[t] < hi[t];
        if (!more) break;
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            const bool open = lo[t] < hi[t];
            const uint32_t mid = open ? (lo[t] + hi[t] + 1) >> 1 : lo[t];
            const uint32_t sm = soff[mid];
            if (open) {
                if (sm <= p_m[t]) lo[t] = mid;
                else hi[t] = mid - 1;
            }
        }
    }
    {
        // soff[j] = off[j] - off[0] + j, so the suffix at block position p of
        // read j starts at global symbol off[j] + p - soff[j] = off[0] + p - j
        const uint64_t off0 = off[0];
        uint32_t s1[RF_PER_THREAD];
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) s1[t] = soff[lo[t] + 1];
#pragma unroll
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            if (x < W) {
                s_val[x] = v_m[t];
                s_pos[x] = off0 + p_m[t] - lo[t];
                s_rem[x] = s1[t] - 1 - p_m[t];
                s_gs[x] = head_m[t] ? 1 : 0;  // head flag for now
            }
        }
    }
    __syncthreads();
    uint16_t gs_r[RF_PER_THREAD], ge_r[RF_PER_THREAD];
    for (int t = 0; t < RF_PER_THREAD; ++t) {
        uint32_t x = tid + 256 * t;
        if (x < W) {
            uint32_t y = x;
            while (y > 0 && !s_gs[y]) --y;
            uint32_t z = x + 1;
            while (z < W && !s_gs[z]) ++z;
            gs_r[t] = (uint16_t)y;
            ge_r[t] = (uint16_t)z;
        }
    }
    __syncthreads();
    for (int t = 0; t < RF_PER_THREAD; ++t) {
        uint32_t x = tid + 256 * t;
        if (x < W) {
            s_gs[x] = gs_r[t];
            s_ge[x] = ge_r[t];
        }
    }
    __syncthreads();

    uint64_t d = (uint64_t)kfirst;
    for (uint32_t iter = 0;; ++iter) {
        // chunk keys of the members of still-tied subgroups; the loads of all
        // of a thread's members go out before any is used (an inactive member
        // loads the word holding the first symbol of the reads, which exists)
        int any = 0;
        {
            bool act[RF_PER_THREAD];
            uint32_t take[RF_PER_THREAD], bit[RF_PER_THREAD];
            uint64_t w0[RF_PER_THREAD], w1[RF_PER_THREAD], w2[RF_PER_THREAD];
#pragma unroll
            for (int t = 0; t < RF_PER_THREAD; ++t) {
                uint32_t x = tid + 256 * t;
                act[t] = x < W && s_ge[x] - s_gs[x] >= 2;
                uint64_t sp = 0;
                take[t] = 0;
                if (act[t]) {
                    uint32_t rem = s_rem[x];
                    uint32_t rd = rem >= d ? (uint32_t)(rem - d) : 0u;
                    take[t] = rd < (uint32_t)RF_K ? rd : (uint32_t)RF_K;
                    sp = take[t] ? s_pos[x] + d : 0;
                }
                uintptr_t addr = (uintptr_t)reads + (uintptr_t)(sp >> 2);
                uintptr_t a0 = addr & ~(uintptr_t)7;
                bit[t] = (uint32_t)((addr - a0) * 8 + 2 * (sp & 3));
                const uint32_t end = bit[t] + 2 * take[t];  // bits used from a0 on
                w0[t] = *reinterpret_cast<const uint64_t *>(a0);
                w1[t] = *reinterpret_cast<const uint64_t *>(end > 64 ? a0 + 8 : a0);
                w2[t] = *reinterpret_cast<const uint64_t *>(end > 128 ? a0 + 16 : a0);
                if (end <= 64) w1[t] = 0;
                if (end <= 128) w2[t] = 0;
            }
#pragma unroll
            for (int t = 0; t < RF_PER_THREAD; ++t) {
                uint32_t x = tid + 256 * t;
                if (act[t]) {
                    const uint32_t tk = take[t], sh = bit[t];
                    // symbols 0..31 and 32..63 of the window, first in the low bits
                    uint64_t lo64 = w0[t] >> sh, hi64 = w1[t] >> sh;
                    if (sh) {
                        lo64 |= w1[t] << (64 - sh);
                        hi64 |= w2[t] << (64 - sh);
                    }
                    const uint32_t ta = tk < (uint32_t)KEY_K ? tk : (uint32_t)KEY_K;
                    const uint32_t tb = tk - ta;
                    uint64_t sa_ = ta ? lo64 & ((1ull << (2 * ta)) - 1ull) : 0ull;
                    uint64_t sb_ = ((lo64 >> (2 * KEY_K)) | (hi64 << (64 - 2 * KEY_K)));
                    sb_ = tb ? sb_ & ((1ull << (2 * tb)) - 1ull) : 0ull;
                    s_kh[x] = reverse_pairs(sa_) >> (64 - 2 * KEY_K);
                    s_kl[x] = ((reverse_pairs(sb_) >> (64 - 2 * KEY_K)) << RF_LEN_BITS) | tk;
                    any = 1;
                }
            }
        }
        any = __syncthreads_or(any);
        if (!any) break;
        if (iter >= max_iter) {
            if (tid == 0) atomicOr(err, 64u);
            break;
        }
        // new place of every member inside its subgroup
        uint32_t np[RF_PER_THREAD], v_r[RF_PER_THREAD], rem_r[RF_PER_THREAD];
        uint64_t pos_r[RF_PER_THREAD], kh_r[RF_PER_THREAD], kl_r[RF_PER_THREAD];
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            np[t] = x;
            if (x < W) {
                uint32_t gs = s_gs[x], ge = s_ge[x];
                if (ge - gs >= 2) {
                    const uint64_t hx = s_kh[x], lx = s_kl[x];
                    uint32_t c = 0;
                    for (uint32_t y = gs; y < ge; ++y) {
                        const uint64_t hy = s_kh[y], ly = s_kl[y];
                        c += hy < hx || (hy == hx && (ly < lx || (ly == lx && y < x)));
                    }
                    np[t] = gs + c;
                }
                v_r[t] = s_val[x];
                pos_r[t] = s_pos[x];
                rem_r[t] = s_rem[x];
                kh_r[t] = s_kh[x];
                kl_r[t] = s_kl[x];
            }
        }
        __syncthreads();
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            if (x < W) {
                uint32_t q = np[t];
                s_val[q] = v_r[t];
                s_pos[q] = pos_r[t];
                s_rem[q] = rem_r[t];
                s_kh[q] = kh_r[t];
                s_kl[q] = kl_r[t];
            }
        }
        __syncthreads();
        // split every reordered subgroup where the chunk key changes; a key
        // that reaches the terminator settles its members where they are
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            if (x < W) {
                uint32_t gs = s_gs[x], ge = s_ge[x];
                gs_r[t] = (uint16_t)gs;
                ge_r[t] = (uint16_t)ge;
                if (ge - gs >= 2) {
                    const uint64_t kh = s_kh[x], kl = s_kl[x];
                    if ((kl & ((1u << RF_LEN_BITS) - 1)) < (uint64_t)RF_K) {
                        gs_r[t] = (uint16_t)x;
                        ge_r[t] = (uint16_t)(x + 1);
                    } else {
                        uint32_t y = x;
                        while (y > gs && s_kh[y - 1] == kh && s_kl[y - 1] == kl) --y;
                        uint32_t z = x + 1;
                        while (z < ge && s_kh[z] == kh && s_kl[z] == kl) ++z;
                        gs_r[t] = (uint16_t)y;
                        ge_r[t] = (uint16_t)z;
                    }
                }
            }
        }
        __syncthreads();
        for (int t = 0; t < RF_PER_THREAD; ++t) {
            uint32_t x = tid + 256 * t;
            if (x < W) {
                s_gs[x] = gs_r[t];
                s_ge[x] = ge_r[t];
            }
        }
        __syncthreads();
        d += RF_K;
    }
    for (int t = 0; t < RF_PER_THREAD; ++t) {
        uint32_t x = tid + 256 * t;
        if (x < W) sa[U[a + x]] = s_val[x];
    }
}

// Workgroups stride over the windows of the tied suffixes.  nUp (when set)
// holds the count on the device, so a grid sized for the largest count can
// be launched before the count exists (a captured schedule); a set *largep
// (a tied group too large for the windows: prefix doubling needed) makes the
// launch do nothing and sets REFINE_REDO in *err, and the caller runs the
// block again on the path that decides on the host.
__global__ __launch_bounds__(256) void refine_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, const uint32_t *__restrict__ tile_first,
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ U, uint32_t nU_val,
    const uint32_t *__restrict__ nUp, const uint32_t *__restrict__ largep,
    uint32_t *__restrict__ sa, int kfirst, uint32_t max_iter, uint32_t *__restrict__ err) {
    const uint32_t nU = nUp ? *nUp : nU_val;
    if (largep && *largep) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, REFINE_REDO);
        return;
    }
    for (uint32_t win = blockIdx.x; (uint64_t)win * REFINE_WINDOW < nU; win += gridDim.x) {
        refine_window(reads, off, soff, tile_first, keys, U, nU, sa, kfirst, max_iter, err, win);
        __syncthreads();  // the next window reuses the LDS arrays
    }
}

__global__ void vals_to_ascii_kernel(const uint32_t *__restrict__ sa, uint32_t n,
                                     uint8_t *__restrict__ bint) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const char ascii[5] = {'A', 'C', 'G', 'T', '$'};
    bint[i] = (uint8_t)ascii[sa[i] >> POS_BITS];
}

__global__ void scatter_g_kernel(const uint64_t *__restrict__ keys,
                                 const uint32_t *__restrict__ vals, uint32_t n, int gshift,
                                 uint64_t *__restrict__ g) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[vals[i] & POS_MASK] = keys[i] >> gshift;
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
                             const uint32_t *tile_first, uint32_t n_blk, const uint64_t *g,
                             int gshift, int kfirst, int hshift, uint64_t *keys, uint32_t *vals,
                             uint32_t *hist0, hipStream_t s) {
    uint64_t want = div_up(n_blk, 256 * 8);
    unsigned grid = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    block_keys_kernel<<<grid, 256, 0, s>>>(reads, off, soff, tile_first, n_blk, g, gshift, kfirst,
                                           hshift, keys, vals, hist0);
    return hipGetLastError();
}

hipError_t launch_group_heads(const uint64_t *keys, const uint32_t *vals, const uint32_t *U,
                              uint32_t n, int kshort, uint32_t *sa, uint32_t *rank,
                              uint32_t *Uout, uint32_t *nUout, uint32_t limit, uint32_t *large,
                              uint64_t *status, uint32_t *counter, uint32_t epoch, uint32_t *err,
                              hipStream_t s) {
    uint32_t ntiles = (uint32_t)div_up(n, SCAN_TILE);
    if (ntiles == 0) return hipSuccess;
    group_heads_kernel<<<ntiles, 256, 0, s>>>(keys, vals, U, n, kshort, sa, rank, Uout, nUout,
                                              limit, large, status, counter, ntiles, epoch, err);
    return hipGetLastError();
}

hipError_t launch_doubling_keys(const uint32_t *U, uint32_t nU, const uint32_t *sa,
                                const uint32_t *rank, uint32_t h, int rbits, uint32_t n_blk,
                                uint64_t *keys, uint32_t *vals, uint32_t *err, hipStream_t s) {
    doubling_keys_kernel<<<grid_for(nU, 256), 256, 0, s>>>(U, nU, sa, rank, h, rbits, n_blk, keys,
                                                          vals, err);
    return hipGetLastError();
}

hipError_t launch_refine(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                         const uint32_t *tile_first, const uint64_t *keys, const uint32_t *U,
                         uint32_t nU, uint32_t *sa, int kfirst, uint32_t max_iter, uint32_t *err,
                         hipStream_t s) {
    if (nU == 0) return hipSuccess;
    refine_kernel<<<grid_for(nU, REFINE_WINDOW), 256, 0, s>>>(
        reads, off, soff, tile_first, keys, U, nU, nullptr, nullptr, sa, kfirst, max_iter, err);
    return hipGetLastError();
}

hipError_t launch_refine_dev(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                             const uint32_t *tile_first, const uint64_t *keys, const uint32_t *U,
                             const uint32_t *nUp, const uint32_t *largep, uint32_t n_max,
                             uint32_t *sa, int kfirst, uint32_t max_iter, uint32_t *err,
                             hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    const unsigned want = grid_for(n_max, REFINE_WINDOW);
    refine_kernel<<<want < REFINE_MAX_GRID ? want : REFINE_MAX_GRID, 256, 0, s>>>(
        reads, off, soff, tile_first, keys, U, 0u, nUp, largep, sa, kfirst, max_iter, err);
    return hipGetLastError();
}

hipError_t launch_vals_to_ascii(const uint32_t *sa, uint32_t n, uint8_t *bint, hipStream_t s) {
    vals_to_ascii_kernel<<<grid_for(n, 256), 256, 0, s>>>(sa, n, bint);
    return hipGetLastError();
}

hipError_t launch_scatter_g(const uint64_t *keys, const uint32_t *vals, uint32_t n, int gshift,
                            uint64_t *g, hipStream_t s) {
    if (n == 0) return hipSuccess;
    scatter_g_kernel<<<grid_for(n, 256), 256, 0, s>>>(keys, vals, n, gshift, g);
    return hipGetLastError();
}

hipError_t launch_sa_strip(const uint32_t *sa, uint32_t n, uint32_t *out, hipStream_t s) {
    sa_strip_kernel<<<grid_for(n, 256), 256, 0, s>>>(sa, n, out);
    return hipGetLastError();
}

}  // namespace bwt
