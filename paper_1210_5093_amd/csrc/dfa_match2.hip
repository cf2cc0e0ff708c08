// Packed-pair chunk matcher (gfx950).
//
// The work of Algorithm 3 is a set of (chunk, start state) pairs: chunk 0
// with the start state, chunk i >= 1 with every state of I_sigma_i (Eq. 11).
// Every pair costs one walk over its chunk, so any packing of pairs onto
// lanes balances the load.  This path packs the pairs densely: lane L of slot
// row j of wave-tile w takes pair w*T + 64*j + L (T = 64 * KS pairs per
// tile), so no lane idles because a set is smaller than a wavefront.  Pairs
// of one chunk stay adjacent, which keeps their (quickly converging) lookups
// on the same LDS addresses.
//
// Because lanes of one wave may walk different chunks, each lane reads its own
// chunk: a translation pass first turns every input byte into a one- or
// two-byte stream code, so that a step is a single SDWA add (state offset +
// selected byte/word of the loaded codes) and a single ds_read_u16:
//   layout 1: LDS address = R * s + 2 * class  (state-major rows of R bytes)
//   layout 2: LDS address = class * colstride + 2 * s  (class-major columns)
// The table sits at LDS address 0 (the kernel has no static LDS), so stored
// table entries are LDS addresses themselves.
//
// Kernels: k_translate (bytes -> codes, invalid-byte flags), k_chunkinfo
// (lookahead class and |I| per chunk), k_scan (exclusive prefix of set
// sizes = first pair of each chunk), k_match2 (persistent tiles of pairs).
// The sparse maps it writes have the same form as the one-chunk-per-wave
// matcher's, so the combination kernels are shared.
#include <type_traits>

#include "dfa_internal.h"

namespace dfaspec {

constexpr int kWave2 = 64;
constexpr int kSlots2 = 4;                 // pairs per lane per tile
constexpr int kTile2 = kWave2 * kSlots2;   // pairs per wave-tile

typedef __attribute__((address_space(3))) const uint16_t lds_u16_t;
__device__ __forceinline__ uint32_t lds_ld(uint32_t addr) {
    return *(lds_u16_t *)(size_t)addr;
}

// state_offset + selected byte (layout 1) or 16-bit word (layout 2) of w.
template <int L, int K>
__device__ __forceinline__ uint32_t add_sel(uint32_t s, uint32_t w) {
    uint32_t r;
    if constexpr (L == 1) {
        if constexpr (K == 0)
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0" : "=v"(r) : "v"(s), "v"(w));
        else if constexpr (K == 1)
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1" : "=v"(r) : "v"(s), "v"(w));
        else if constexpr (K == 2)
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2" : "=v"(r) : "v"(s), "v"(w));
        else
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3" : "=v"(r) : "v"(s), "v"(w));
    } else {
        if constexpr (K == 0)
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0" : "=v"(r) : "v"(s), "v"(w));
        else
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1" : "=v"(r) : "v"(s), "v"(w));
    }
    return r;
}

// Apply the codes packed in one dword (4 one-byte or 2 two-byte codes).
template <int L>
__device__ __forceinline__ uint32_t step_dword(uint32_t s, uint32_t w) {
    if constexpr (L == 1) {
        s = lds_ld(add_sel<1, 0>(s, w));
        s = lds_ld(add_sel<1, 1>(s, w));
        s = lds_ld(add_sel<1, 2>(s, w));
        s = lds_ld(add_sel<1, 3>(s, w));
    } else {
        s = lds_ld(add_sel<2, 0>(s, w));
        s = lds_ld(add_sel<2, 1>(s, w));
    }
    return s;
}

// ---------------------------------------------------------------------------
// Translation: code[i] = code_lut[in[i]]; per-block flag if a byte is outside
// Sigma.  Threads take 16 input bytes at a time (grid-stride); the output is
// 16-byte aligned.
// ---------------------------------------------------------------------------
template <typename CodeT>
__global__ __launch_bounds__(256) void k_translate(const uint8_t *__restrict__ in, uint64_t n,
                                                   const uint16_t *__restrict__ code_lut,
                                                   CodeT *__restrict__ out,
                                                   uint32_t *__restrict__ block_bad) {
    __shared__ uint16_t lut[256];
    __shared__ uint32_t bad_any;
    lut[threadIdx.x] = code_lut[threadIdx.x];
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint64_t first = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16; first < n;
         first += (uint64_t)gridDim.x * blockDim.x * 16) {
        uint8_t b[16];
        const bool aligned = ((reinterpret_cast<uintptr_t>(in) & 15) == 0) && first + 16 <= n;
        if (aligned) {
            const uint4 v = *reinterpret_cast<const uint4 *>(in + first);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) b[k] = (uint8_t)(w[k >> 2] >> (8 * (k & 3)));
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) b[k] = first + k < n ? in[first + k] : 0;
        }
        uint16_t c[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            uint16_t v = lut[b[k]];
            const bool inside = first + k < n;
            bad |= (inside && v == kCodeInvalid) ? 1u : 0u;
            c[k] = (v == kCodeInvalid || !inside) ? (uint16_t)0 : v;
        }
        if constexpr (sizeof(CodeT) == 1) {
            uint4 o;
            uint32_t *ow = reinterpret_cast<uint32_t *>(&o);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ow[q] = (uint32_t)c[4 * q] | ((uint32_t)c[4 * q + 1] << 8) |
                        ((uint32_t)c[4 * q + 2] << 16) | ((uint32_t)c[4 * q + 3] << 24);
            *reinterpret_cast<uint4 *>(out + first) = o;
        } else {
            uint4 o[2];
            uint32_t *ow = reinterpret_cast<uint32_t *>(o);
#pragma unroll
            for (int q = 0; q < 8; ++q) ow[q] = (uint32_t)c[2 * q] | ((uint32_t)c[2 * q + 1] << 16);
            *reinterpret_cast<uint4 *>(out + first) = o[0];
            *reinterpret_cast<uint4 *>(out + first + 8) = o[1];
        }
    }
    if (bad) atomicOr(&bad_any, 1u);
    __syncthreads();
    if (threadIdx.x == 0) block_bad[blockIdx.x] = bad_any;
}

// Lookahead class and set size of every chunk (chunk 0: the start state).
__global__ void k_chunkinfo(DevDFA d, const uint8_t *__restrict__ in, uint64_t chunk,
                            uint32_t nch, uint32_t mode, uint16_t *__restrict__ msize,
                            uint16_t *__restrict__ ccls) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nch) return;
    uint32_t m = 1, cls = 0;
    if (i > 0) {
        const uint32_t e = d.lut[in[(uint64_t)i * chunk - 1]];
        if (e == kLutInvalid) {
            m = 0;
        } else {
            cls = e >> 24;
            m = d.set_off[mode][cls + 1] - d.set_off[mode][cls];
        }
    }
    msize[i] = (uint16_t)m;
    ccls[i] = (uint16_t)cls;
}

// Exclusive scan of the set sizes in three phases: first[i] = sum_{k<i} m_k,
// first[nch] = number of pairs, tile_first[w] = chunk holding pair w * kTile2.
// Phase 2 also folds the translation flags into the flag bit of chunk 0's
// size, from where the compose levels carry it up.
constexpr uint32_t kScanThreads = 1024;
constexpr uint32_t kScanItems = 4;
constexpr uint32_t kScanBlock = kScanThreads * kScanItems;   // chunks per scan block

// Inclusive scan of one value per thread across the workgroup (in place).
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t *part) {
    const uint32_t t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < blockDim.x; off <<= 1) {
        const uint32_t u = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += u;
        __syncthreads();
    }
    return part[t];
}

__global__ __launch_bounds__(1024) void k_scan_sums(const uint16_t *__restrict__ msize,
                                                    uint32_t nch, uint32_t *__restrict__ bsum) {
    __shared__ uint32_t part[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint32_t v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k)
        if (base + k < nch) v += msize[base + k] & 0x7FFFu;
    const uint32_t inc = block_inclusive_scan(v, part);
    if (threadIdx.x == blockDim.x - 1) bsum[blockIdx.x] = inc;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *__restrict__ bsum, uint32_t nb,
                                                   uint16_t *__restrict__ msize, uint32_t nch,
                                                   const uint32_t *__restrict__ block_bad,
                                                   uint32_t nbad, uint32_t *__restrict__ first) {
    __shared__ uint32_t part[kScanThreads];
    __shared__ uint32_t bad_any;
    const uint32_t t = threadIdx.x, T = blockDim.x;
    if (t == 0) bad_any = 0;
    uint32_t bad = 0;
    for (uint32_t b = t; b < nbad; b += T) bad |= block_bad[b];
    // sequential segments per thread, then one workgroup scan of the segment sums
    const uint32_t per = (nb + T - 1) / T;
    const uint32_t lo = min(nb, t * per), hi = min(nb, lo + per);
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i) sum += bsum[i];
    __syncthreads();
    if (bad) atomicOr(&bad_any, 1u);
    const uint32_t inc = block_inclusive_scan(sum, part);
    uint32_t run = inc - sum;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = bsum[i];
        bsum[i] = run;        // exclusive offset of scan block i
        run += v;
    }
    if (t == T - 1) first[nch] = inc;
    __syncthreads();
    if (t == 0 && bad_any) msize[0] = (uint16_t)(msize[0] | kFlagSymbol);
}

__global__ __launch_bounds__(1024) void k_scan_apply(const uint16_t *__restrict__ msize,
                                                     uint32_t nch,
                                                     const uint32_t *__restrict__ boff,
                                                     uint32_t *__restrict__ first,
                                                     uint32_t *__restrict__ tile_first) {
    __shared__ uint32_t part[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint32_t m[kScanItems], v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        m[k] = base + k < nch ? (msize[base + k] & 0x7FFFu) : 0u;
        v += m[k];
    }
    const uint32_t inc = block_inclusive_scan(v, part);
    uint32_t run = boff[blockIdx.x] + inc - v;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        if (base + k < nch) {
            first[base + k] = run;
            if (m[k]) {
                for (uint32_t w = (run + kTile2 - 1) / kTile2; w <= (run + m[k] - 1) / kTile2; ++w)
                    tile_first[w] = (uint32_t)(base + k);
            }
        }
        run += m[k];
    }
}

struct Match2Args {
    DevDFA d;
    const void *codes;       // translated stream (1- or 2-byte codes)
    uint64_t n;
    uint64_t chunk;
    uint32_t nch;
    uint32_t start;
    uint32_t mode;
    uint32_t stride;
    const uint32_t *first;   // [nch + 1]
    const uint32_t *tile_first;
    const uint16_t *ccls;    // [nch]
    uint16_t *maps;
};

// Walk KS pairs per lane.  Fast path: every pair of the tile has a full,
// 16-byte-aligned chunk (o16 = its first code's offset in 16-byte units),
// read as uint4 blocks with one block of prefetch.
template <int L>
__device__ __forceinline__ void walk_fast(const uint4 *__restrict__ codes16,
                                          const uint32_t (&o16)[kSlots2], uint32_t blocks,
                                          uint32_t (&st)[kSlots2]) {
    uint4 cur[kSlots2], nxt[kSlots2];
#pragma unroll
    for (int j = 0; j < kSlots2; ++j) cur[j] = codes16[o16[j]];
    for (uint32_t b = 1; ; ++b) {
        const bool more = b < blocks;
        if (more) {
#pragma unroll
            for (int j = 0; j < kSlots2; ++j) nxt[j] = codes16[(size_t)o16[j] + b];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int j = 0; j < kSlots2; ++j) {
                const uint32_t w = q == 0 ? cur[j].x : q == 1 ? cur[j].y : q == 2 ? cur[j].z : cur[j].w;
                st[j] = step_dword<L>(st[j], w);
            }
        }
        if (!more) break;
#pragma unroll
        for (int j = 0; j < kSlots2; ++j) cur[j] = nxt[j];
    }
}

template <int L>
__global__ __launch_bounds__(1024, 8) void k_match2(Match2Args a) {
    extern __shared__ __align__(16) uint8_t smem[];
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(L == 1 ? a.d.stab : a.d.table);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (uint32_t i = threadIdx.x; i < a.d.stab_bytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    using CodeT = typename std::conditional<L == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t kPer16 = 16 / sizeof(CodeT);   // codes per 16 bytes
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t waves = blockDim.x / kWave2;
    const uint32_t wave_id = blockIdx.x * waves + threadIdx.x / kWave2;
    const uint32_t total_waves = gridDim.x * waves;
    const uint32_t total = a.first[a.nch];
    const uint32_t ntiles = (total + kTile2 - 1) / kTile2;
    const uint32_t R = L == 1 ? a.d.rowbytes : 2u;
    const CodeT *codes = reinterpret_cast<const CodeT *>(a.codes);
    // full chunks start on 16-byte boundaries iff the chunk length does
    const bool aligned_chunks = (a.chunk % kPer16) == 0;

    for (uint32_t tile = wave_id; tile < ntiles; tile += total_waves) {
        const uint32_t lo0 = a.tile_first[tile];
        const uint32_t hi0 = tile + 1 < ntiles ? a.tile_first[tile + 1] + 1 : a.nch;
        uint32_t st[kSlots2], ci[kSlots2], o16[kSlots2];
        bool ok = aligned_chunks;
#pragma unroll
        for (int j = 0; j < kSlots2; ++j) {
            const uint32_t P = tile * kTile2 + j * kWave2 + lane;
            const bool valid = P < total;
            uint32_t lo = lo0, hi = hi0;   // first[lo] <= P < first[hi]
            while (valid && hi > lo + 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (a.first[mid] <= P) lo = mid; else hi = mid;
            }
            const uint32_t c = valid ? lo : 0u;
            uint32_t s = 0;
            if (valid) {
                s = (c == 0) ? a.start
                             : a.d.set_st[a.mode][a.d.set_off[a.mode][a.ccls[c]] + (P - a.first[c])];
            }
            st[j] = R * s;
            ci[j] = valid ? c : 0xFFFFFFFFu;
            o16[j] = aligned_chunks ? (uint32_t)((uint64_t)c * a.chunk / kPer16) : 0u;
            ok = ok && (!valid || c + 1 < a.nch || a.n - (uint64_t)c * a.chunk == a.chunk);
        }
        if (__all(ok)) {
            walk_fast<L>(reinterpret_cast<const uint4 *>(codes), o16,
                         (uint32_t)(a.chunk / kPer16), st);
        } else {
            // general path: per-lane code loads, chunks of any length and alignment
            for (uint64_t t = 0; t < a.chunk; ++t) {
#pragma unroll
                for (int j = 0; j < kSlots2; ++j) {
                    if (ci[j] != 0xFFFFFFFFu) {
                        const uint64_t pos = (uint64_t)ci[j] * a.chunk + t;
                        if (pos < a.n) st[j] = lds_ld(st[j] + (uint32_t)codes[pos]);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kSlots2; ++j) {
            if (ci[j] != 0xFFFFFFFFu) {
                const uint32_t e = st[j] / R;
                const uint32_t c = ci[j];
                const uint32_t p = tile * kTile2 + j * kWave2 + lane - a.first[c];
                uint16_t v;
                if (c + 1 == a.nch) {
                    v = (uint16_t)(kTerm | e);
                } else {
                    v = a.d.pos[a.mode][(size_t)a.ccls[c + 1] * a.d.nq + e];
                }
                a.maps[(size_t)c * a.stride + p] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
int launch_match2(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                  void *codes, uint32_t *block_bad, uint32_t *bsum, uint32_t *first,
                  uint32_t *tile_first, uint16_t *ccls, uint16_t *maps, uint16_t *msize,
                  hipStream_t s, hipEvent_t ev_before_matcher) {
    const uint32_t L = d->dev.layout;
    const uint32_t tblocks = p.tblocks;
    if (L == 1)
        hipLaunchKernelGGL(k_translate<uint8_t>, dim3(tblocks), dim3(256), 0, s, d_in, p.n,
                           d->dev.code, (uint8_t *)codes, block_bad);
    else
        hipLaunchKernelGGL(k_translate<uint16_t>, dim3(tblocks), dim3(256), 0, s, d_in, p.n,
                           d->dev.code, (uint16_t *)codes, block_bad);
    hipLaunchKernelGGL(k_chunkinfo, dim3((p.nch + 255) / 256), dim3(256), 0, s, d->dev, d_in,
                       p.chunk, p.nch, p.lookahead, msize, ccls);
    const uint32_t nsb = (p.nch + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_sums, dim3(nsb), dim3(kScanThreads), 0, s, msize, p.nch, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, bsum, nsb, msize, p.nch,
                       block_bad, tblocks, first);
    hipLaunchKernelGGL(k_scan_apply, dim3(nsb), dim3(kScanThreads), 0, s, msize, p.nch, bsum,
                       first, tile_first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "packed-matcher preparation launch");
    if (ev_before_matcher) {
        e = hipEventRecord(ev_before_matcher, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    Match2Args a;
    a.d = d->dev;
    a.codes = codes;
    a.n = p.n;
    a.chunk = p.chunk;
    a.nch = p.nch;
    a.start = start;
    a.mode = p.lookahead;
    a.stride = p.stride;
    a.first = first;
    a.tile_first = tile_first;
    a.ccls = ccls;
    a.maps = maps;
    const size_t lds = d->dev.stab_bytes;
    if (L == 1)
        hipLaunchKernelGGL(k_match2<1>, dim3(p.blocks2), dim3(p.threads2), lds, s, a);
    else
        hipLaunchKernelGGL(k_match2<2>, dim3(p.blocks2), dim3(p.threads2), lds, s, a);
    e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "k_match2 launch");
}

int set_match2_lds_limit(int lds) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_match2<1>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_match2<2>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e == hipSuccess ? DFA_OK : DFA_E_DEVICE;
}

uint32_t match2_tile_pairs() { return kTile2; }
uint32_t match2_scan_blocks(uint32_t nch) { return (nch + kScanBlock - 1) / kScanBlock; }

}  // namespace dfaspec
