// k_radix.hip -- stable LSD radix sort of (uint64 key, uint32 value) pairs,
// 8-bit digits, one kernel per digit pass with decoupled look-back across
// tiles (onesweep style), for the block suffix sort of set-bwte (Section 3:
// any suffix sorting algorithm may build the block's suffix array).
//
// Per pass, a workgroup takes a tile of keys (in tile order from an atomic
// counter), ranks every key among equal digits of its tile with 8 wave
// ballots per key (stable: tile order is wave, item, lane), gets the count of
// each digit in all earlier tiles by look-back, stages the tile in LDS in
// sorted order and writes each digit run contiguously.  Keys are read once
// and written once per pass.  The digit totals a pass needs are counted by
// the previous pass while it holds the keys in registers (the first pass's by
// whoever built the keys), so no pass re-reads the keys; every tile sums the
// copies of those counts into digit starts itself.
#include "dev_util.hpp"

namespace bwt {

namespace {


__global__ void radix_zero_kernel(uint32_t *hist, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) hist[i] = 0;
}

// Counts of one digit of the keys (the first pass's digit for key producers
// that do not count it themselves), into the copies of one pass.  hist must be
// zero on entry.
__global__ __launch_bounds__(256) void radix_hist1_kernel(const uint64_t *__restrict__ keys,
                                                          uint64_t n, int shift,
                                                          uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + tid; i < n; i += (uint64_t)gridDim.x * 256)
        atomicAdd(&h[(keys[i] >> shift) & 255], 1u);
    __syncthreads();
    if (h[tid]) atomicAdd(&hist[(blockIdx.x % HIST_COPIES) * 256 + tid], h[tid]);
}

// Block-wide exclusive sums of two values at once over THREADS threads
// (every thread calls it, with all lanes active); tmp holds 2 * THREADS/64
// words.  One barrier: tmp must not be written again before the next one.
template <int THREADS>
__device__ __forceinline__ void block_excl_sum2(uint32_t a, uint32_t b, uint32_t *tmp,
                                                uint32_t &ea, uint32_t &eb) {
    constexpr int W = THREADS / WAVE;
    const int tid = threadIdx.x, w = tid >> 6;
    const uint32_t ia = wave_incl_sum_dpp(a), ib = wave_incl_sum_dpp(b);
    if ((tid & 63) == 63) {
        tmp[w] = ia;
        tmp[W + w] = ib;
    }
    __syncthreads();
    uint32_t ba = 0, bb = 0;
#pragma unroll
    for (int k = 0; k < W; ++k)
        if (k < w) {
            ba += tmp[k];
            bb += tmp[W + k];
        }
    ea = ba + ia - a;
    eb = bb + ib - b;
}

// One digit pass over tiles of THREADS * ITEMS keys.  Wave w of a tile owns
// the ITEMS * 64 consecutive keys starting at w * ITEMS * 64 and takes them
// row by row, so tile order = (wave, row, lane) and the ranking is stable.
// A key's rank among the equal digits of its wave is the count of that digit
// in the wave's earlier rows plus its lower lanes in its own row: the lowest
// lane of each group of equal digits in a row adds the group's size to the
// wave's count with one LDS add-with-return (the rows' adds are issued back
// to back and run in row order), and the other lanes take the earlier count
// from that lane.  Keys and then values go through the same LDS buffer; each
// thread keeps the destinations of its write-out slots in registers for the
// value phase.  Full tiles (all but possibly the last) take a path with no
// bounds tests.
template <int THREADS, int ITEMS, bool FULL>
__device__ __forceinline__ void radix_tile(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint64_t n, int shift, const uint32_t *__restrict__ hist_cur,
    uint32_t *__restrict__ hist_next, int shift_next, uint64_t *__restrict__ status,
    uint32_t tile, uint32_t epoch, uint32_t *__restrict__ err, uint32_t (*s_wh)[256],
    int32_t *s_gbase, uint32_t *s_next, uint32_t *s_tmp, uint64_t *s_buf) {
    constexpr int WAVES = THREADS / WAVE;
    constexpr int TILE = THREADS * ITEMS;
    constexpr int WKEYS = ITEMS * WAVE;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t base = (uint64_t)tile * TILE;
    const uint64_t wbase = base + (uint64_t)wave * WKEYS;
    const uint32_t cnt_tile = FULL ? (uint32_t)TILE : (uint32_t)(n - base);

    uint64_t k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) {
        const uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        const bool ok = FULL || idx < n;
        k[e] = ok ? kin[idx] : 0;
        v[e] = ok ? vin[idx] : 0;
    }
    // this pass's count of every digit: the sum of its HIST_COPIES copies
    uint32_t dcount = 0;
    if (tid < 256) {
        uint32_t hc[HIST_COPIES];
#pragma unroll
        for (int c = 0; c < HIST_COPIES; ++c) hc[c] = hist_cur[c * 256 + tid];
#pragma unroll
        for (int c = 0; c < HIST_COPIES; ++c) dcount += hc[c];
    }
    if (hist_next) {
        // histogram of the next pass's digit while the keys are in registers
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) {
            const uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
            if (FULL || idx < n) atomicAdd(&s_next[(uint32_t)(k[e] >> shift_next) & 255u], 1u);
        }
    }
    const uint64_t ltm = lanemask_lt();
    uint32_t rk[ITEMS], lead[ITEMS], prev[ITEMS];
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) {
        const uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        const bool ok = FULL || idx < n;
        const uint32_t d = (uint32_t)(k[e] >> shift) & 255u;
        uint64_t peers = FULL ? ~0ull : __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        rk[e] = __popcll(peers & ltm);
        lead[e] = (uint32_t)__builtin_ctzll(peers | (1ull << 63));
        prev[e] = 0;
        if (ok && rk[e] == 0) prev[e] = atomicAdd(&s_wh[wave][d], (uint32_t)__popcll(peers));
    }
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) rk[e] += (uint32_t)__shfl((int)prev[e], (int)lead[e], WAVE);
    __syncthreads();
    // digit totals of the tile; the wave offsets then hold the tile-local
    // digit start plus the counts of the earlier waves
    uint32_t total = 0;
    uint32_t wc[WAVES];
    if (tid < 256) {
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            wc[w] = s_wh[w][tid];
            total += wc[w];
        }
    }
    uint32_t lstart, dstart;
    block_excl_sum2<THREADS>(tid < 256 ? total : 0u, tid < 256 ? dcount : 0u, s_tmp, lstart, dstart);
    if (tid < 256) {
        uint32_t run = lstart;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            s_wh[w][tid] = run;
            run += wc[w];
        }
        const uint32_t excl = lookback(status + tid, 256u, tile, epoch, total, OpSum(), 0u, err);
        s_gbase[tid] = (int32_t)(dstart + excl) - (int32_t)lstart;
        if (hist_next && s_next[tid])
            atomicAdd(&hist_next[(tile % HIST_COPIES) * 256 + tid], s_next[tid]);
    }
    __syncthreads();
    // keys: stage in LDS in sorted order, then write each digit run out
    uint32_t pos[ITEMS];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) {
        const uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        const uint32_t d = (uint32_t)(k[e] >> shift) & 255u;
        uint32_t q = s_wh[wave][d] + rk[e];
        bad |= q >= (uint32_t)TILE;
        q = q < (uint32_t)TILE ? q : (uint32_t)TILE - 1;
        pos[e] = q;
        if (FULL || idx < n) s_buf[q] = k[e];
    }
    __syncthreads();
    uint32_t dst[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t i = (uint32_t)tid + (uint32_t)r * THREADS;
        dst[r] = 0xffffffffu;
        if (FULL || i < cnt_tile) {
            const uint64_t kk = s_buf[i];
            const uint32_t t = (uint32_t)(s_gbase[(uint32_t)(kk >> shift) & 255u] + (int32_t)i);
            if ((uint64_t)t < n) {
                dst[r] = t;
                kout[t] = kk;
            } else {
                bad = true;
            }
        }
    }
    __syncthreads();
    // values through the same buffer
    uint32_t *s_val = reinterpret_cast<uint32_t *>(s_buf);
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) {
        const uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        if (FULL || idx < n) s_val[pos[e]] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t i = (uint32_t)tid + (uint32_t)r * THREADS;
        if (dst[r] != 0xffffffffu) vout[dst[r]] = s_val[i];
    }
    if (bad) atomicOr(err, 4u);
}

// Destinations are 32-bit: a block sort runs on at most MAX_BLOCK keys.
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void radix_pass_kernel(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint64_t n, int shift, const uint32_t *__restrict__ hist_cur,
    uint32_t *__restrict__ hist_next, int shift_next, uint64_t *__restrict__ status,
    uint32_t *__restrict__ counter, uint32_t ntiles, uint32_t epoch, uint32_t *__restrict__ err) {
    constexpr int WAVES = THREADS / WAVE;
    constexpr int TILE = THREADS * ITEMS;
    static_assert(THREADS >= 256, "one thread per digit");
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wh[WAVES][256];  // per-wave digit counts, then offsets
    __shared__ int32_t s_gbase[256];       // global position minus tile position
    __shared__ uint32_t s_next[256];       // this tile's counts of the next pass's digit
    __shared__ uint32_t s_tmp[2 * WAVES];
    __shared__ uint64_t s_buf[TILE];       // keys, then values
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int d = lane; d < 256; d += WAVE) s_wh[wave][d] = 0;
    if (tid < 256) s_next[tid] = 0;
    const uint32_t tile = acquire_tile(counter, ntiles, &s_tile);
    if (tile >= ntiles) {  // only if the tile counter was not zero at launch
        if (tid == 0) atomicOr(err, 2u);
        return;
    }
    if ((uint64_t)(tile + 1) * TILE <= n)
        radix_tile<THREADS, ITEMS, true>(kin, vin, kout, vout, n, shift, hist_cur, hist_next,
                                         shift_next, status, tile, epoch, err, s_wh, s_gbase,
                                         s_next, s_tmp, s_buf);
    else
        radix_tile<THREADS, ITEMS, false>(kin, vin, kout, vout, n, shift, hist_cur, hist_next,
                                          shift_next, status, tile, epoch, err, s_wh, s_gbase,
                                          s_next, s_tmp, s_buf);
}

}  // namespace

// hist: the copies of one pass (HIST_COPIES x 256 words); zeroed here first
hipError_t launch_radix_hist1(const uint64_t *keys, uint64_t n, int shift, uint32_t *hist,
                              hipStream_t s) {
    radix_zero_kernel<<<HIST_COPIES, 256, 0, s>>>(hist, HIST_COPIES * 256);
    uint64_t want = div_up(n, 256 * 16);
    int grid = (int)(want < 2048 ? (want > 0 ? want : 1) : 2048);
    radix_hist1_kernel<<<grid, 256, 0, s>>>(keys, n, shift, hist);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s) {
    radix_zero_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, (int)n);
    return hipGetLastError();
}

// Tile shapes (threads x keys per thread) the pass can run with.
int radix_tile_keys(int cfg) {
    switch (cfg) {
    case 1: return 512 * 8;
    case 2: return 256 * 8;
    case 3: return 512 * 12;
    case 4: return 1024 * 4;
    case 5: return 512 * 16;
    case 6: return 1024 * 8;
    case 7: return 1024 * 12;
    case 8: return 768 * 12;
    default: return 256 * 16;
    }
}

hipError_t launch_radix_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                             uint32_t *vout, uint64_t n, int shift, const uint32_t *hist_cur,
                             uint32_t *hist_next, int shift_next, uint64_t *status,
                             uint32_t *counter, uint32_t epoch, uint32_t *err, int cfg,
                             hipStream_t s) {
    const uint32_t ntiles = (uint32_t)div_up(n, (uint64_t)radix_tile_keys(cfg));
    if (ntiles == 0) return hipSuccess;
#define BWT_PASS(T, I)                                                                      \
    radix_pass_kernel<T, I><<<ntiles, T, 0, s>>>(kin, vin, kout, vout, n, shift, hist_cur,  \
                                                 hist_next, shift_next, status, counter,    \
                                                 ntiles, epoch, err)
    switch (cfg) {
    case 1: BWT_PASS(512, 8); break;
    case 2: BWT_PASS(256, 8); break;
    case 3: BWT_PASS(512, 12); break;
    case 4: BWT_PASS(1024, 4); break;
    case 5: BWT_PASS(512, 16); break;
    case 6: BWT_PASS(1024, 8); break;
    case 7: BWT_PASS(1024, 12); break;
    case 8: BWT_PASS(768, 12); break;
    default: BWT_PASS(256, 16); break;
    }
#undef BWT_PASS
    return hipGetLastError();
}

}  // namespace bwt
