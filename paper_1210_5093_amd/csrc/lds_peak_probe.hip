// LDS table-lookup throughput probe for gfx950: the roofline denominator of
// the chunk matchers.  Every lane runs 8 independent chains of dependent
// ds_read_u16 lookups, as the matchers do; the table is 4 KiB so that 32
// wavefronts fit on a CU.  Three address patterns:
//   0: 64 lanes on 64 distinct dwords (no bank conflict, two bank passes),
//   1: all lanes on one address (broadcast),
//   2: pseudo-random addresses (bank conflicts).
// Prints lookups per second and per CU-clock (at 2.4 GHz).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                    \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

constexpr int kEntries = 2048;       // uint16 entries = 4 KiB
constexpr int kChains = 8;

__global__ __launch_bounds__(256) void probe(const uint16_t *g, int mode, int iters,
                                             uint32_t *out) {
    __shared__ __align__(16) uint16_t t[kEntries];
    for (int i = threadIdx.x; i < kEntries; i += blockDim.x) t[i] = g[i];
    __syncthreads();
    const uint8_t *tb = reinterpret_cast<const uint8_t *>(t);
    const uint32_t lane = threadIdx.x & 63;
    constexpr uint32_t kMask = kEntries * 2 - 2;   // byte offsets stay even and inside
    uint32_t st[kChains];
    for (int j = 0; j < kChains; ++j) {
        if (mode == 0) st[j] = (lane * 4 + j * 256) & kMask;
        else if (mode == 1) st[j] = (j * 256) & kMask;
        else st[j] = ((lane * 2654435761u + j * 40503u) & (kEntries - 1)) * 2;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            st[j] = *reinterpret_cast<const uint16_t *>(tb + (st[j] & kMask));
    }
    uint32_t acc = 0;
    for (int j = 0; j < kChains; ++j) acc ^= st[j];
    if (acc == 0xFFFFFFFFu) out[0] = acc;   // keeps the chains live
}

int main() {
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<uint16_t> h(kEntries);
    const char *names[3] = {"distinct dwords", "broadcast", "random"};
    for (int mode = 0; mode < 3; ++mode) {
        for (int i = 0; i < kEntries; ++i)
            h[i] = mode == 2 ? (uint16_t)((((uint32_t)i * 2246822519u) >> 7) & (kEntries - 1)) * 2
                             : (uint16_t)(i * 2);   // each entry points at itself
        uint16_t *g = nullptr;
        uint32_t *o = nullptr;
        CHECK(hipMalloc(&g, kEntries * 2));
        CHECK(hipMalloc(&o, 4));
        CHECK(hipMemcpy(g, h.data(), kEntries * 2, hipMemcpyHostToDevice));
        const int blocks = cus * 32, iters = 2000;
        hipEvent_t a, b;
        CHECK(hipEventCreate(&a));
        CHECK(hipEventCreate(&b));
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            CHECK(hipEventRecord(a));
            hipLaunchKernelGGL(probe, dim3(blocks), dim3(256), 0, 0, g, mode, iters, o);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(b));
            CHECK(hipEventSynchronize(b));
            CHECK(hipEventElapsedTime(&ms, a, b));
        }
        const double lookups = (double)blocks * 256 * kChains * iters;
        std::printf("%-16s %8.3f ms  %6.2f Tlookup/s  %5.2f lookups per CU-clock at 2.4 GHz\n",
                    names[mode], ms, lookups / ms / 1e9, lookups / (ms * 1e-3) / cus / 2.4e9);
        CHECK(hipFree(g));
        CHECK(hipFree(o));
        CHECK(hipEventDestroy(a));
        CHECK(hipEventDestroy(b));
    }
    return 0;
}
