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

// The values of one lane are written in descending order; they are kept in
// an 8-entry shift register and written as one aligned 64-byte chunk when the
// register covers indices [8q, 8q + 8), so the writes are whole half-lines
// instead of single words spread over the cache (partial chunks at both ends
// of a read are written word by word).
struct GBuf {
    uint64_t r0, r1, r2, r3, r4, r5, r6, r7;  // r0 = lowest index held
    uint32_t cnt;
    __device__ void push(uint64_t v) {
        r7 = r6; r6 = r5; r5 = r4; r4 = r3; r3 = r2; r2 = r1; r1 = r0; r0 = v;
        cnt = cnt < 8 ? cnt + 1 : 8;
    }
    // write the held values to g[idx .. idx + cnt)
    __device__ void flush(uint64_t *__restrict__ g, uint64_t idx, bool vec) {
        if (cnt == 8 && vec) {
            uint4 *q = reinterpret_cast<uint4 *>(g + idx);
            q[0] = make_uint4((uint32_t)r0, (uint32_t)(r0 >> 32), (uint32_t)r1, (uint32_t)(r1 >> 32));
            q[1] = make_uint4((uint32_t)r2, (uint32_t)(r2 >> 32), (uint32_t)r3, (uint32_t)(r3 >> 32));
            q[2] = make_uint4((uint32_t)r4, (uint32_t)(r4 >> 32), (uint32_t)r5, (uint32_t)(r5 >> 32));
            q[3] = make_uint4((uint32_t)r6, (uint32_t)(r6 >> 32), (uint32_t)r7, (uint32_t)(r7 >> 32));
        } else {
            if (cnt > 0) g[idx] = r0;
            if (cnt > 1) g[idx + 1] = r1;
            if (cnt > 2) g[idx + 2] = r2;
            if (cnt > 3) g[idx + 3] = r3;
            if (cnt > 4) g[idx + 4] = r4;
            if (cnt > 5) g[idx + 5] = r5;
            if (cnt > 6) g[idx + 6] = r6;
            if (cnt > 7) g[idx + 7] = r7;
        }
        cnt = 0;
    }
};

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
    const bool vec = (reinterpret_cast<uintptr_t>(g) & 63) == 0;  // uniform
    const uint64_t s0 = off[j];
    uint32_t k = (uint32_t)(off[j + 1] - s0);
    const uint64_t gb = soff[j];
    GBuf buf;
    buf.cnt = 0;
    uint64_t i = m_ext;
    buf.push(i);
    if (((gb + k) & 7) == 0) buf.flush(g, gb + k, vec);
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
        buf.push(i);
        if (((gb + k) & 7) == 0) buf.flush(g, gb + k, vec);
    }
    buf.flush(g, gb, false);  // what is left below the last aligned index
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
