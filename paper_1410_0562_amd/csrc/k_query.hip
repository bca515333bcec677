// k_query.hip -- rank queries (Eq. 2), export of B, and the device-side
// checks and block split of an append whose offsets live in device memory.
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

__global__ void export_kernel(const Rec *__restrict__ recs, uint64_t n, uint8_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const char ascii[5] = {'A', 'C', 'G', 'T', '$'};
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
// block-text position of read j.  Writes cuts[2k] = first read of block k,
// cuts[2k+1] = S(first read); res[2] = number of blocks.  One thread.
__global__ void plan_blocks_kernel(const uint64_t *__restrict__ off, uint64_t m, uint64_t M,
                                   uint64_t *__restrict__ cuts, uint64_t *__restrict__ res) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint64_t o0 = off[0];
    uint64_t j = 0, K = 0;
    cuts[0] = 0;
    cuts[1] = 0;
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
        cuts[2 * K] = j;
        cuts[2 * K + 1] = off[j] - o0 + j;
    }
    res[2] = K;
}

}  // namespace

hipError_t launch_rank_many(const Rec *recs, const uint64_t *sbc, const uint64_t *meta,
                            const uint8_t *cs, const uint64_t *ks, uint64_t *out, uint64_t count,
                            hipStream_t s) {
    if (count == 0) return hipSuccess;
    rank_many_kernel<<<(unsigned)div_up(count, 256), 256, 0, s>>>(recs, sbc, meta, cs, ks, out,
                                                                  count);
    return hipGetLastError();
}

hipError_t launch_export(const Rec *recs, uint64_t n, uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    export_kernel<<<(unsigned)div_up(n, 256), 256, 0, s>>>(recs, n, out);
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

}  // namespace bwt
