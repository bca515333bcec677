// bench_random_reads.hip -- the rate of dependent random reads on one GPU:
// the ceiling for the LF walks of ComputeRanks, each step of which reads one
// 64-byte index record at a place that depends on the previous read.
//
// Every lane follows its own chain: it reads BYTES at a pseudo-random
// record-aligned place of a buffer of the given size, and the next place
// depends on the value read.  The table gives reads per second for read sizes
// of 16, 64 and 128 bytes, working sets of 200 MB (inside the 256 MB
// Infinity Cache), 625 MB (the long-read index at its last block) and 2.5 GB,
// and 1 to 8 waves per SIMD; the last line is a JSON summary.
//
// Built by paper_1410_0562_amd/build.py; run by `python bench.py
// --calibrate-random` (or directly).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CK(x)                                                                          \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), \
                         __LINE__);                                                    \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

template <int BYTES>
__global__ __launch_bounds__(256) void chase(const uint4 *__restrict__ buf, uint32_t nslots,
                                             int steps, uint64_t *__restrict__ sink) {
    constexpr int SLOT = BYTES >= 64 ? BYTES / 16 : 4;  // slot = max(BYTES, 64) bytes
    uint64_t x = (uint64_t)(blockIdx.x * blockDim.x + threadIdx.x) * 0x9E3779B97F4A7C15ull + 1;
    uint32_t acc = 0;
    for (int s = 0; s < steps; ++s) {
        x ^= x >> 31;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 29;
        const uint32_t r = __umulhi((uint32_t)x ^ (uint32_t)(x >> 32) ^ acc, nslots);
        const uint4 *p = buf + (uint64_t)r * SLOT;
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < BYTES / 16; ++q) {
            const uint4 w = p[q];
            v += w.x ^ w.y ^ w.z ^ w.w;
        }
        acc = (acc << 1) ^ (v & 1u);
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the reads live
}

__global__ void fill(uint4 *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4((uint32_t)i, (uint32_t)(i >> 7), 3u, 5u);
}

int main() {
    const uint64_t sizes_mb[3] = {200, 625, 2560};
    const int read_bytes[3] = {16, 64, 128};
    const int steps = 200;
    int dev = 0, ncu = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    uint4 *buf;
    uint64_t *sink;
    const uint64_t max_bytes = sizes_mb[2] << 20;
    CK(hipMalloc(&buf, max_bytes));
    CK(hipMalloc(&sink, 8));
    fill<<<4096, 256>>>(buf, max_bytes / 16);
    CK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    std::vector<double> rates64;
    std::printf("| working set | bytes per read | waves per SIMD | ms | G reads/s | TB/s read |\n");
    std::printf("|---:|---:|---:|---:|---:|---:|\n");
    for (uint64_t mb : sizes_mb) {
        for (int B : read_bytes) {
            const uint64_t slot = (uint64_t)std::max(B, 64);
            const uint32_t nslots = (uint32_t)((mb << 20) / slot);
            for (int wps = 1; wps <= 8; wps *= 2) {
                const int blocks = ncu * wps;  // 4 waves per block, 4 SIMDs per CU
                float best = 1e30f;
                for (int it = 0; it < 3; ++it) {
                    CK(hipEventRecord(e0));
                    if (B == 16) chase<16><<<blocks, 256>>>(buf, nslots, steps, sink);
                    else if (B == 64) chase<64><<<blocks, 256>>>(buf, nslots, steps, sink);
                    else chase<128><<<blocks, 256>>>(buf, nslots, steps, sink);
                    CK(hipGetLastError());
                    CK(hipEventRecord(e1));
                    CK(hipEventSynchronize(e1));
                    float ms;
                    CK(hipEventElapsedTime(&ms, e0, e1));
                    best = std::min(best, ms);
                }
                const double reads = (double)blocks * 256 * steps;
                const double rate = reads / best / 1e6;  // G reads/s
                if (B == 64 && mb == 625) rates64.push_back(rate);
                std::printf("| %llu MB | %d | %d | %.3f | %.1f | %.2f |\n", (unsigned long long)mb,
                            B, wps, best, rate, rate * B / 1e3);
                std::fflush(stdout);
            }
        }
    }
    std::sort(rates64.begin(), rates64.end());
    std::printf("{\"metric\": \"dependent random 64-byte reads per second, 625 MB working set\", "
                "\"value\": %.2f, \"unit\": \"G reads/s\", \"cus\": %d}\n",
                rates64[rates64.size() / 2], ncu);
    CK(hipFree(buf));
    CK(hipFree(sink));
    return 0;
}
