// k_bucket.hip -- the second half of a block's suffix sort (Section 3).
//
// Radix passes on the top digits of the first key (see bwt_internal.hpp)
// leave the suffixes in buckets of equal top B bits, each bucket a contiguous
// run in position order (the passes are stable); B is chosen for about 64
// suffixes per bucket.  One wavefront finishes a bucket of at most
// BUCKET_CAP = 256 suffixes in registers: a bitonic network over
// (key, index in the bucket) -- the index keeps equal keys in position order,
// which is terminator order -- with 64 x E elements per wave (element
// r * 64 + lane in register r of that lane), so the compare-exchanges at
// distance >= 64 stay inside a lane and the shorter ones are lane shuffles;
// no workgroup barrier is involved.  The wave then appends the bucket's tied
// groups (equal keys that do not end at a terminator) to the list of
// unresolved suffixes with one reservation, so every group stays contiguous
// in the list.  Larger buckets are piles of identical short suffixes (every
// read's terminator suffix has the same g, as have all suffixes "A$", ...):
// they are gathered into one array, radix-sorted on the whole key with the
// ordinary passes, put back, and their ties found by the ordinary scan.
#include "dev_util.hpp"

namespace bwt {

namespace {

constexpr uint32_t ABSENT = 0xffffffffu;

__global__ void bucket_fill_kernel(uint32_t *__restrict__ bstart, uint32_t nb) {
    uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) bstart[b] = ABSENT;
}

// Keys sorted by their bits above bshift: bstart[b] / bend[b] = first / one
// past the last position of bucket b (only for buckets that occur).
__global__ void bucket_bounds_kernel(const uint64_t *__restrict__ keys, uint32_t n, int bshift,
                                     uint32_t nb, uint32_t *__restrict__ bstart,
                                     uint32_t *__restrict__ bend, uint32_t *__restrict__ err) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t b = keys[i] >> bshift;
    if (b >= nb) {
        atomicOr(err, 256u);
        return;
    }
    const uint64_t bp = i > 0 ? keys[i - 1] >> bshift : ~0ull;
    if (bp != b) {
        bstart[(uint32_t)b] = i;
        if (i > 0 && bp < nb) bend[(uint32_t)bp] = i;
    }
    if (i + 1 == n) bend[(uint32_t)b] = n;
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
        uint64_t kp = __shfl_up(k[r], 1, 64);
        uint64_t kn = __shfl_down(k[r], 1, 64);
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

// One bucket of z (2 .. 64 * E) suffixes at s0, sorted by one wave and
// written back; returns its number of tied suffixes.
template <int E>
__device__ uint32_t wave_bucket(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                uint32_t s0, uint32_t z, int kshort, uint32_t *__restrict__ s_v,
                                uint32_t limit, uint32_t *__restrict__ large) {
    const int lane = lane_id();
    uint64_t k[E];
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        x[r] = i;
        if (i < z) {
            k[r] = keys[s0 + i];
            s_v[i] = vals[s0 + i];
        } else {
            k[r] = ~0ull;  // a real key never has all length bits set
        }
    }
    wave_bitonic<E>(k, x, lane);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        if (i < z) {
            keys[s0 + i] = k[r];
            vals[s0 + i] = s_v[x[r]];
        }
    }
    uint32_t cnt;
    (void)wave_ties<E>(k, z, kshort, limit, large, &cnt);
    return cnt;
}

// Four waves per workgroup, one bucket id per wave.  Every bucket id gets
// tcnt[b] (its tied suffixes) and osz[b] (its size if above BUCKET_CAP, else
// 0); buckets of 2 .. BUCKET_CAP suffixes are sorted here.
__global__ __launch_bounds__(256) void bucket_sort_kernel(
    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, const uint32_t *__restrict__ bstart,
    const uint32_t *__restrict__ bend, uint32_t nb, int kshort, uint32_t limit,
    uint32_t *__restrict__ large, uint32_t *__restrict__ tcnt, uint32_t *__restrict__ osz,
    uint32_t *__restrict__ err) {
    __shared__ uint32_t s_v[4][BUCKET_CAP];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const uint32_t b = blockIdx.x * 4 + wave;
    if (b >= nb) return;
    const uint32_t s0 = bstart[b];
    uint32_t z = 0;
    if (s0 != ABSENT) {
        const uint32_t e = bend[b];
        if (e <= s0) {
            if (lane == 0) atomicOr(err, 256u);
        } else {
            z = e - s0;
        }
    }
    uint32_t ties = 0;
    if (z >= 2 && z <= BUCKET_CAP) {
        uint32_t *sv = s_v[wave];
        if (z <= 64) ties = wave_bucket<1>(keys, vals, s0, z, kshort, sv, limit, large);
        else if (z <= 128) ties = wave_bucket<2>(keys, vals, s0, z, kshort, sv, limit, large);
        else ties = wave_bucket<4>(keys, vals, s0, z, kshort, sv, limit, large);
    }
    static_assert(BUCKET_CAP == 256, "the size classes above cover 2 .. 256");
    if (lane == 0) {
        tcnt[b] = ties;
        osz[b] = z > BUCKET_CAP ? z : 0u;
    }
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
    for (uint32_t q = 0; q < BT_TILE / 256; ++q) {
        const uint32_t b = t * BT_TILE + q * 256 + tid;
        if (b < nb) {
            a += tcnt[b];
            const uint32_t z = osz[b];
            c += z ? 1u : 0u;
            e += z;
        }
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
// buckets listed in bucket order: olist[q] = b, ooff[q] = gathered start;
// ooff[count] = total.
__global__ __launch_bounds__(256) void bucket_scan_down_kernel(
    uint32_t *__restrict__ tcnt, const uint32_t *__restrict__ osz, uint32_t nb,
    const uint32_t *__restrict__ part, const uint32_t *__restrict__ res,
    uint32_t *__restrict__ olist, uint32_t *__restrict__ ooff) {
    __shared__ uint32_t s_tmp[4];
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    uint32_t ra = part[3 * t], rc = part[3 * t + 1], re = part[3 * t + 2];
    for (uint32_t q = 0; q < BT_TILE / 256; ++q) {
        const uint32_t b = t * BT_TILE + q * 256 + tid;
        uint32_t a = 0, z = 0;
        if (b < nb) {
            a = tcnt[b];
            z = osz[b];
        }
        uint32_t ta, tc, te;
        const uint32_t pa = block_excl_sum256(a, s_tmp, &ta);
        const uint32_t pc = block_excl_sum256(z ? 1u : 0u, s_tmp, &tc);
        const uint32_t pe = block_excl_sum256(z, s_tmp, &te);
        if (b < nb) {
            tcnt[b] = ra + pa;
            if (z) {
                olist[rc + pc] = b;
                ooff[rc + pc] = re + pe;
            }
        }
        ra += ta;
        rc += tc;
        re += te;
    }
    if (t == 0 && tid == 0) ooff[res[1]] = res[2];
}

// Tied suffixes of the buckets sorted in registers, listed from U[tpre[b]]
// in slot order (the keys are read again, sorted).
template <int E>
__device__ void wave_emit(const uint64_t *__restrict__ keys, uint32_t s0, uint32_t z, int kshort,
                          uint32_t at, uint32_t *__restrict__ U, uint32_t ucap,
                          uint32_t *__restrict__ err) {
    const int lane = lane_id();
    uint64_t k[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        k[r] = i < z ? keys[s0 + i] : ~0ull;
    }
    uint32_t cnt, dummy = 0;
    const uint32_t rows = wave_ties<E>(k, z, kshort, 0xffffffffu, &dummy, &cnt);
    if (at + cnt > ucap) {
        if (lane == 0) atomicOr(err, 512u);
        return;
    }
    const uint64_t ltm = lanemask_lt();
    uint32_t before = 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const bool t = (rows >> r) & 1u;
        const uint64_t tb = __ballot(t);
        if (t) U[at + before + (uint32_t)__popcll(tb & ltm)] = s0 + (uint32_t)(r * 64 + lane);
        before += (uint32_t)__popcll(tb);
    }
}

__global__ __launch_bounds__(256) void bucket_emit_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ bstart,
    const uint32_t *__restrict__ bend, const uint32_t *__restrict__ tpre, uint32_t nb,
    int kshort, uint32_t *__restrict__ U, uint32_t ucap, uint32_t *__restrict__ err) {
    const int wave = threadIdx.x >> 6;
    const uint32_t b = blockIdx.x * 4 + wave;
    if (b >= nb) return;
    const uint32_t at = tpre[b];
    const uint32_t next = b + 1 < nb ? tpre[b + 1] : ucap;
    if (next == at) return;  // no tied suffix in this bucket
    const uint32_t s0 = bstart[b];
    if (s0 == ABSENT) return;
    const uint32_t z = bend[b] - s0;
    if (z < 2 || z > BUCKET_CAP) return;
    if (z <= 64) wave_emit<1>(keys, s0, z, kshort, at, U, ucap, err);
    else if (z <= 128) wave_emit<2>(keys, s0, z, kshort, at, U, ucap, err);
    else wave_emit<4>(keys, s0, z, kshort, at, U, ucap, err);
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

}  // namespace

hipError_t launch_bucket_bounds(const uint64_t *keys, uint32_t n, int bshift, uint32_t nb,
                                uint32_t *bstart, uint32_t *bend, uint32_t *err, hipStream_t s) {
    bucket_fill_kernel<<<(unsigned)div_up(nb, 256), 256, 0, s>>>(bstart, nb);
    if (n > 0)
        bucket_bounds_kernel<<<(unsigned)div_up(n, 256), 256, 0, s>>>(keys, n, bshift, nb, bstart,
                                                                     bend, err);
    return hipGetLastError();
}

hipError_t launch_bucket_sort(uint64_t *keys, uint32_t *vals, const uint32_t *bstart,
                              const uint32_t *bend, uint32_t nb, int kshort, uint32_t limit,
                              uint32_t *large, uint32_t *tcnt, uint32_t *osz, uint32_t *part,
                              uint32_t *res, uint32_t *olist, uint32_t *ooff, uint32_t *err,
                              hipStream_t s) {
    const uint32_t ntiles = (uint32_t)div_up(nb, BT_TILE);
    if (ntiles > 4 * 1024) return hipErrorInvalidValue;
    bucket_sort_kernel<<<(unsigned)div_up(nb, 4), 256, 0, s>>>(keys, vals, bstart, bend, nb,
                                                               kshort, limit, large, tcnt, osz,
                                                               err);
    bucket_scan_up_kernel<<<ntiles, 256, 0, s>>>(tcnt, osz, nb, part);
    bucket_scan_top_kernel<<<1, 1024, 0, s>>>(part, ntiles, res);
    bucket_scan_down_kernel<<<ntiles, 256, 0, s>>>(tcnt, osz, nb, part, res, olist, ooff);
    return hipGetLastError();
}

hipError_t launch_bucket_emit(const uint64_t *keys, const uint32_t *bstart, const uint32_t *bend,
                              const uint32_t *tpre, uint32_t nb, int kshort, uint32_t *U,
                              uint32_t ucap, uint32_t *err, hipStream_t s) {
    bucket_emit_kernel<<<(unsigned)div_up(nb, 4), 256, 0, s>>>(keys, bstart, bend, tpre, nb,
                                                               kshort, U, ucap, err);
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
