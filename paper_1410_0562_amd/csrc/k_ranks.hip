// k_ranks.hip -- ComputeRanks (Section 4, Lemma 1 and Algorithm 2).
//
// For each read P_j of the block, one lane walks the read from its end:
// the terminator suffix $_j is larger than exactly the m_ext terminators
// already in B_ext and smaller than every old suffix that starts with a base,
// so it starts at i = m_ext; then for k = |P_j|-1 .. 0, with c = P_j[k],
// i := C[c] + rank(c, i, B_ext) (Lemma 1), and g[off_j + k] = i, where off_j
// is the exclusive prefix sum of |P_j| + 1 (the block text position of the
// read's first symbol).  Each step is one random 64-byte record read from
// the HBM-resident index; the reads of a block are independent, so a block
// keeps hundreds of thousands of walks in flight.
#include "dev_util.hpp"

namespace bwt {

namespace {

__global__ __launch_bounds__(256) void compute_ranks_kernel(
    const uint8_t *__restrict__ reads, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ soff, uint32_t m_blk, const Rec *__restrict__ recs,
    const uint64_t *__restrict__ sbc, const uint64_t *__restrict__ meta, int big,
    uint64_t *__restrict__ g) {
    // C[c]: symbols of B_ext smaller than c; every terminator is smaller than A
    const uint64_t m_ext = meta[5], n_ext = meta[4];
    const uint64_t C0 = m_ext, C1 = C0 + meta[0], C2 = C1 + meta[1], C3 = C2 + meta[2];
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_blk) return;
    const uint64_t s0 = off[j];
    uint32_t k = (uint32_t)(off[j + 1] - s0);
    uint64_t *gj = g + soff[j];
    uint64_t i = m_ext;
    gj[k] = i;
    // the 8-byte word of packed input holding the current symbol
    uintptr_t wa = 0;
    uint64_t word = 0;
    const bool isbig = big != 0;
    while (k > 0) {
        --k;
        uint64_t s = s0 + k;
        uintptr_t addr = (uintptr_t)reads + (uintptr_t)(s >> 2);
        uintptr_t a0 = addr & ~(uintptr_t)7;
        if (a0 != wa) {
            word = *reinterpret_cast<const uint64_t *>(a0);
            wa = a0;
        }
        int c = (int)(word >> ((addr - a0) * 8 + 2 * (s & 3))) & 3;
        uint64_t Cc = c == 0 ? C0 : c == 1 ? C1 : c == 2 ? C2 : C3;
        i = Cc + rank_base(recs, sbc, i, c, isbig);
        i = i < n_ext ? i : n_ext;  // a consistent index never needs the clamp
        gj[k] = i;
    }
}

}  // namespace

hipError_t launch_compute_ranks(const uint8_t *reads, const uint64_t *off, const uint32_t *soff,
                                uint32_t m_blk, const Rec *recs, const uint64_t *sbc,
                                const uint64_t *meta, int big, uint64_t *g, hipStream_t s) {
    if (m_blk == 0) return hipSuccess;
    compute_ranks_kernel<<<(unsigned)div_up(m_blk, 256), 256, 0, s>>>(reads, off, soff, m_blk, recs,
                                                                      sbc, meta, big, g);
    return hipGetLastError();
}

}  // namespace bwt
