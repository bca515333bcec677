// k_radix.hip -- stable LSD radix sort of (uint64 key, uint32 value) pairs,
// 8-bit digits, one kernel per digit pass with decoupled look-back across
// tiles (onesweep style), for the block suffix sort of set-bwte (Section 3:
// any suffix sorting algorithm may build the block's suffix array).
//
// Per pass, a 256-thread workgroup takes a tile of 4096 keys (in tile order
// from an atomic counter), ranks every key among equal digits of its tile
// with 8 wave ballots per key (stable: tile order is wave, item, lane), gets
// the count of each digit in all earlier tiles by look-back, stages the tile
// in LDS in sorted order and writes each digit run contiguously.  Keys are
// read once and written once per pass.  The digit totals a pass needs are
// counted by the previous pass while it holds the keys in registers (the
// first pass's by whoever built the keys), so no pass re-reads the keys.
#include "dev_util.hpp"

namespace bwt {

namespace {

constexpr int RB_THREADS = 256;
constexpr int RB_ITEMS = RADIX_TILE / RB_THREADS;  // 16
constexpr int RB_WAVES = RB_THREADS / WAVE;          // 4
constexpr int RB_WAVE_KEYS = RB_ITEMS * WAVE;        // 1024 keys per wave

__global__ void radix_zero_kernel(uint32_t *hist, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) hist[i] = 0;
}

// Counts of one digit of the keys (the first pass's digit for key producers
// that do not count it themselves).  hist must be zero on entry.
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
    if (h[tid]) atomicAdd(&hist[tid], h[tid]);
}

__global__ __launch_bounds__(RB_THREADS) void radix_pass_kernel(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint64_t n, int shift, const uint32_t *__restrict__ hist,
    uint32_t *__restrict__ hist_next, int shift_next, uint64_t *__restrict__ status,
    uint32_t *__restrict__ counter, uint32_t ntiles, uint32_t epoch, uint32_t *__restrict__ err) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_dstart[256];        // global start of each digit
    __shared__ uint32_t s_next[256];          // this tile's counts of the next pass's digit
    __shared__ uint32_t s_wh[RB_WAVES][256];  // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_lstart[256];        // start of each digit inside the tile
    __shared__ int64_t s_gbase[256];          // global position minus tile position
    __shared__ uint32_t s_tmp[4];
    __shared__ uint64_t s_keys[RADIX_TILE];
    __shared__ uint32_t s_vals[RADIX_TILE];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int d = lane; d < 256; d += WAVE) s_wh[wave][d] = 0;
    s_next[tid] = 0;
    {
        // digit totals of this pass (counted by the previous pass or by the
        // key builder) -> exclusive starts
        uint32_t tot;
        s_dstart[tid] = block_excl_sum256(hist[tid], s_tmp, &tot);
    }
    const uint32_t tile = acquire_tile(counter, ntiles, &s_tile);
    if (tile >= ntiles) {  // only if the tile counter was not zero at launch
        if (tid == 0) atomicOr(err, 2u);
        return;
    }
    const uint64_t base = (uint64_t)tile * RADIX_TILE;
    const uint64_t wbase = base + (uint64_t)wave * RB_WAVE_KEYS;

    uint64_t k[RB_ITEMS];
    uint32_t v[RB_ITEMS];
    uint32_t rk[RB_ITEMS];
#pragma unroll
    for (int e = 0; e < RB_ITEMS; ++e) {
        uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        bool ok = idx < n;
        k[e] = ok ? kin[idx] : 0;
        v[e] = ok ? vin[idx] : 0;
    }
    if (hist_next) {
        // histogram of the next pass's digit while the keys are in registers
#pragma unroll
        for (int e = 0; e < RB_ITEMS; ++e) {
            uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
            if (idx < n) atomicAdd(&s_next[(uint32_t)(k[e] >> shift_next) & 255u], 1u);
        }
    }
    const uint64_t ltm = lanemask_lt();
#pragma unroll
    for (int e = 0; e < RB_ITEMS; ++e) {
        uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        bool ok = idx < n;
        uint32_t d = (uint32_t)(k[e] >> shift) & 255u;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t before = __popcll(peers & ltm);
        uint32_t cnt = __popcll(peers);
        uint32_t prev = ok ? s_wh[wave][d] : 0;
        rk[e] = prev + before;
        if (ok && before == 0) s_wh[wave][d] = prev + cnt;
    }
    __syncthreads();
    // digit totals of the tile, wave offsets, tile-local digit starts
    const int d = tid;
    uint32_t c0 = s_wh[0][d], c1 = s_wh[1][d], c2 = s_wh[2][d], c3 = s_wh[3][d];
    uint32_t total = c0 + c1 + c2 + c3;
    uint32_t tile_total;
    uint32_t lstart = block_excl_sum256(total, s_tmp, &tile_total);
    s_wh[0][d] = 0;
    s_wh[1][d] = c0;
    s_wh[2][d] = c0 + c1;
    s_wh[3][d] = c0 + c1 + c2;
    s_lstart[d] = lstart;
    uint32_t excl = lookback(status + d, 256u, tile, epoch, total, OpSum(), 0u, err);
    s_gbase[d] = (int64_t)s_dstart[d] + (int64_t)excl - (int64_t)lstart;
    if (hist_next && s_next[d]) atomicAdd(&hist_next[d], s_next[d]);
    __syncthreads();
    // stage in LDS in sorted order
#pragma unroll
    for (int e = 0; e < RB_ITEMS; ++e) {
        uint64_t idx = wbase + (uint64_t)e * WAVE + lane;
        if (idx < n) {
            uint32_t dd = (uint32_t)(k[e] >> shift) & 255u;
            uint32_t pos = s_lstart[dd] + s_wh[wave][dd] + rk[e];
            if (pos < RADIX_TILE) {
                s_keys[pos] = k[e];
                s_vals[pos] = v[e];
            } else {
                atomicOr(err, 4u);
            }
        }
    }
    __syncthreads();
    uint32_t cnt_tile = (uint32_t)((n - base) < (uint64_t)RADIX_TILE ? (n - base) : RADIX_TILE);
    for (uint32_t i = tid; i < cnt_tile; i += RB_THREADS) {
        uint64_t key = s_keys[i];
        uint32_t dd = (uint32_t)(key >> shift) & 255u;
        uint64_t dst = (uint64_t)(s_gbase[dd] + (int64_t)i);
        if (dst < n) {
            kout[dst] = key;
            vout[dst] = s_vals[i];
        } else {
            atomicOr(err, 4u);
        }
    }
}

}  // namespace

// hist: counts of the digit at `shift`; zeroed here first
hipError_t launch_radix_hist1(const uint64_t *keys, uint64_t n, int shift, uint32_t *hist,
                              hipStream_t s) {
    radix_zero_kernel<<<1, 256, 0, s>>>(hist, 256);
    uint64_t want = div_up(n, 256 * 16);
    int grid = (int)(want < 2048 ? (want > 0 ? want : 1) : 2048);
    radix_hist1_kernel<<<grid, 256, 0, s>>>(keys, n, shift, hist);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s) {
    radix_zero_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, (int)n);
    return hipGetLastError();
}

hipError_t launch_radix_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                             uint32_t *vout, uint64_t n, int shift, const uint32_t *hist,
                             uint32_t *hist_next, int shift_next, uint64_t *status,
                             uint32_t *counter, uint32_t epoch, uint32_t *err, hipStream_t s) {
    uint32_t ntiles = (uint32_t)div_up(n, RADIX_TILE);
    if (ntiles == 0) return hipSuccess;
    radix_pass_kernel<<<ntiles, RB_THREADS, 0, s>>>(kin, vin, kout, vout, n, shift, hist, hist_next,
                                                    shift_next, status, counter, ntiles, epoch,
                                                    err);
    return hipGetLastError();
}

}  // namespace bwt
