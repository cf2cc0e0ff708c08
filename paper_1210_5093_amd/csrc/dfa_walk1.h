// Device code shared by the one-chunk-per-wavefront matcher and the batched
// matcher: one wavefront walks one chunk from every state of its
// initial-state set (lanes x slots), the class offset of each input byte
// broadcast with v_readlane (see dfa_kernels.hip).
#pragma once

#include "dfa_internal.h"

namespace dfaspec {

constexpr int kWave = 64;
constexpr int kMaxSlots = 8;    // states per lane per pass: up to 512 per wave (64 VGPRs, no spills)

struct MatchArgs {
    DevDFA d;
    const uint8_t *in;
    uint64_t n;
    uint64_t chunk;
    uint32_t nch;
    uint32_t start;
    uint32_t mode;      // 1 = initial-state sets, 0 = all non-absorbing states
    uint32_t stride;    // map entries per chunk
    uint16_t *maps;
    uint16_t *msize;
};

__device__ __forceinline__ uint16_t lds_u16(const uint8_t *base, uint32_t byte_off) {
    return *reinterpret_cast<const uint16_t *>(base + byte_off);
}

// One pass over the chunk [beg, end) for up to KS * 64 start states.  st[j]
// holds 2 * state (a byte offset inside a table column).  Returns true in
// every lane if some byte of the chunk is outside Sigma.
template <int KS>
__device__ __forceinline__ bool walk_pass(const uint8_t *tab, const uint32_t *lut,
                                          const uint8_t *__restrict__ in, uint64_t beg,
                                          uint64_t end, uint32_t (&st)[KS > 0 ? KS : 1],
                                          uint32_t lane) {
    bool bad = false;
    uint64_t blk = beg;
    uint32_t nb = (uint32_t)min<uint64_t>(kWave, end - blk);
    uint32_t byte = lane < nb ? in[blk + lane] : 0u;
    while (true) {
        uint32_t e = lut[byte];
        bool inval = (lane < nb) && (e == kLutInvalid);
        bad |= inval;
        uint32_t co = (e == kLutInvalid) ? 0u : (e & 0xFFFFFFu);
        // prefetch the next block's bytes while this block is walked
        uint64_t nblk = blk + kWave;
        uint32_t nnb = nblk < end ? (uint32_t)min<uint64_t>(kWave, end - nblk) : 0u;
        uint32_t nbyte = lane < nnb ? in[nblk + lane] : 0u;
        if (KS > 0) {
            if (nb == kWave) {
#pragma unroll 16
                for (int t = 0; t < kWave; ++t) {
                    uint32_t s = __builtin_amdgcn_readlane(co, t);
#pragma unroll
                    for (int j = 0; j < KS; ++j) st[j] = lds_u16(tab, s + st[j]);
                }
            } else {
                for (uint32_t t = 0; t < nb; ++t) {
                    uint32_t s = __builtin_amdgcn_readlane(co, t);
#pragma unroll
                    for (int j = 0; j < KS; ++j) st[j] = lds_u16(tab, s + st[j]);
                }
            }
        }
        if (nnb == 0) break;
        blk = nblk;
        nb = nnb;
        byte = nbyte;
    }
    return __builtin_amdgcn_read_exec() != 0 && __any(bad);
}

template <int KS>
__device__ __forceinline__ bool run_pass(const MatchArgs &a, const uint8_t *tab,
                                         const uint32_t *lut, uint32_t chunk_id, uint64_t beg,
                                         uint64_t end, const uint16_t *set, uint32_t base,
                                         uint32_t m, uint32_t next_class, uint32_t lane) {
    uint32_t st[KS > 0 ? KS : 1];
#pragma unroll
    for (int j = 0; j < (KS > 0 ? KS : 1); ++j) {
        uint32_t p = base + j * kWave + lane;
        uint32_t s = 0;
        if (p < m) s = set ? set[p] : a.start;
        st[j] = 2u * s;
    }
    bool bad = walk_pass<KS>(tab, lut, a.in, beg, end, st, lane);
    if (KS > 0) {
        const bool last = (chunk_id + 1 == a.nch);
        const uint16_t *pos = a.d.pos[a.mode] + (size_t)next_class * a.d.nq;
        uint16_t *out = a.maps + (size_t)chunk_id * a.stride;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            uint32_t p = base + j * kWave + lane;
            if (p < m) {
                uint32_t e = st[j] >> 1;
                out[p] = last ? (uint16_t)(kTerm | e) : pos[e];
            }
        }
    }
    return bad;
}

// Calls run_pass<ks> for a runtime ks in 1..K (a chain of uniform branches).
template <int K>
__device__ __forceinline__ bool dispatch_pass(uint32_t ks, const MatchArgs &a, const uint8_t *tab,
                                              const uint32_t *lut, uint32_t chunk_id,
                                              uint64_t beg, uint64_t end, const uint16_t *set,
                                              uint32_t base, uint32_t m, uint32_t next_class,
                                              uint32_t lane) {
    if constexpr (K == 0) {
        return false;
    } else {
        if (ks == K)
            return run_pass<K>(a, tab, lut, chunk_id, beg, end, set, base, m, next_class, lane);
        return dispatch_pass<K - 1>(ks, a, tab, lut, chunk_id, beg, end, set, base, m,
                                    next_class, lane);
    }
}


// Matches one chunk (all passes over its set, up to MaxSlots * 64 states per
// pass) and writes its map entries and size; `lane` is the lane index.
template <int MaxSlots = kMaxSlots>
__device__ __forceinline__ void match_one_chunk(const MatchArgs &a, const uint8_t *tab,
                                                const uint32_t *lut, uint32_t c, uint32_t lane) {
    const uint64_t beg = (uint64_t)c * a.chunk;
    const uint64_t end = min(beg + a.chunk, a.n);
    const uint16_t *set = nullptr;
    uint32_t m = 1;
    if (c > 0) {
        uint32_t e = lut[a.in[beg - 1]];
        if (e == kLutInvalid) {
            m = 0;   // the preceding chunk reports the byte
        } else {
            uint32_t cls = e >> 24;
            uint32_t o0 = a.d.set_off[a.mode][cls];
            m = a.d.set_off[a.mode][cls + 1] - o0;
            set = a.d.set_st[a.mode] + o0;
        }
    }
    uint32_t next_class = 0;
    if (c + 1 < a.nch) {
        uint32_t e = lut[a.in[end - 1]];
        next_class = (e == kLutInvalid) ? 0u : (e >> 24);
    }
    bool bad = false;
    if (m == 0) {
        bad = run_pass<0>(a, tab, lut, c, beg, end, set, 0, 0, next_class, lane);
    } else {
        for (uint32_t base = 0; base < m; base += MaxSlots * kWave) {
            const uint32_t ks = min<uint32_t>(MaxSlots, (m - base + kWave - 1) / kWave);
            bad |= dispatch_pass<MaxSlots>(ks, a, tab, lut, c, beg, end, set, base, m,
                                           next_class, lane);
        }
    }
    if (lane == 0) a.msize[c] = (uint16_t)(m | (bad ? kFlagSymbol : 0));
}

// Composes member maps t = 0 .. cnt-1 (staged in LDS at sm[t * stride]) for
// the domain entries p < m (Eq. 9).
__device__ __forceinline__ void compose_staged(const uint16_t *sm, uint32_t cnt, uint32_t stride,
                                               uint32_t m, uint16_t *out) {
    for (uint32_t p = threadIdx.x; p < m; p += blockDim.x) {
        uint32_t v = sm[p];
        for (uint32_t t = 1; t < cnt && !(v & kTerm); ++t) v = (v < stride) ? sm[t * stride + v] : kBadPos;
        out[p] = (uint16_t)v;
    }
}

}  // namespace dfaspec
