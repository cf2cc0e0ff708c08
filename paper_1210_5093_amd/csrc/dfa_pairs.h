// Device helpers of the packed-pair matchers (single string and batched).
// See dfa_match2.hip for the layouts: a step adds the selected code byte
// (layout 1) or word (layout 2) to the state's LDS offset and loads the next
// state's offset with one ds_read_u16 from a table staged at LDS address 0.
// L = 3 is layout 1 walked over the raw input of a direct table: each loaded
// word of bytes becomes four codes 2 * (byte & 0x7F) before the steps.
#pragma once

#include "dfa_internal.h"

namespace dfaspec {

constexpr int kWave2 = 64;
// A wave-tile holds 64 * S pairs: S slots (independent walks) per lane.  The
// matchers are compiled for S = 2 and S = 4; the plan picks one.

typedef __attribute__((address_space(3))) const uint16_t lds_u16_t;
__device__ __forceinline__ uint32_t lds_ld(uint32_t addr) {
    return *(lds_u16_t *)(size_t)addr;
}

// Code streams of 16-bit codes: layout 2 (one symbol per code); every other
// L reads one-byte codes.
template <int L>
constexpr bool kWideCodes = L == 2;

// state_offset + selected byte (one-byte codes) or 16-bit word of w.
template <int L, int K>
__device__ __forceinline__ uint32_t add_sel(uint32_t s, uint32_t w) {
    uint32_t r;
    if constexpr (!kWideCodes<L>) {
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

// Codes of one loaded word: the word itself, or for L = 3 (raw bytes of a
// direct table) 2 * (byte & 0x7F) per byte.  Bytes of Sigma are below 128, so
// the mask only keeps the codes of invalid bytes even and below 256.
template <int L>
__device__ __forceinline__ uint32_t word_codes(uint32_t w) {
    if constexpr (L == 3) return (w & 0x7F7F7F7Fu) << 1;
    else return w;
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

// Class-string id of the k bytes at in[pos ..] (first byte most significant);
// *bad is set if one of them is outside Sigma.
__device__ __forceinline__ uint32_t class_string_id(const DevDFA &d, const uint8_t *__restrict__ in,
                                                    uint64_t pos, uint32_t k, bool *bad) {
    uint32_t id = 0;
    for (uint32_t j = 0; j < k; ++j) {
        const uint32_t e = d.lut[in[pos + j]];
        if (e == kLutInvalid) { *bad = true; return 0; }
        id = id * d.nclass + (e >> 24);
    }
    return id;
}

__device__ __forceinline__ uint32_t mset_begin(const DevDFA &d, uint32_t k, uint32_t id) {
    return d.mset_off[d.moff[k] + id];
}
__device__ __forceinline__ uint32_t mset_end(const DevDFA &d, uint32_t k, uint32_t id) {
    return d.mset_off[d.moff[k] + id + 1];
}

// Position of state e in the sorted member list [lo, hi), or kBadPos.
__device__ __forceinline__ uint32_t member_rank(const uint16_t *__restrict__ members, uint32_t lo,
                                                uint32_t hi, uint32_t e) {
    uint32_t a = lo, b = hi;
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if (members[mid] < e) a = mid + 1; else b = mid;
    }
    return (a < hi && members[a] == e) ? a - lo : kBadPos;
}

// Walk KS pairs per lane.  Fast path: every pair of the tile has a full,
// 16-byte-aligned chunk (o16 = its first code's offset in 16-byte units),
// read as uint4 blocks with one block of prefetch; consecutive blocks of a
// chunk are `stride` units apart (1 in a linear code stream, 64 in the
// chunk-interleaved one).
// The 16 input bytes at in[pos ..] (zero at and past n), read as whole
// aligned words: one 16-byte load when in + pos is 16-byte aligned, two
// loads and a byte funnel shift when it is not (then only while the second
// word lies inside the input), single bytes at the very end.  pos is a
// multiple of 16, so the misalignment is the same for every block of a
// string.
__device__ __forceinline__ void load16(const uint8_t *__restrict__ in, uint64_t pos, uint64_t n,
                                       uint32_t (&o)[4]) {
    const uint8_t *p = in + pos;
    const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(p) & 15u);
    if (sh == 0 && pos + 16 <= n) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else if (pos + 32 <= n) {
        const uint4 v0 = *reinterpret_cast<const uint4 *>(p - sh);
        const uint4 v1 = *reinterpret_cast<const uint4 *>(p - sh + 16);
        const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        const uint32_t r = sh & 3u;
        switch (sh >> 2) {
#define DFA_SEL(D)                                                                   \
    case D:                                                                          \
        for (int q = 0; q < 4; ++q) o[q] = __builtin_amdgcn_alignbyte(w[q + D + 1], w[q + D], r); \
        break;
            DFA_SEL(0)
            DFA_SEL(1)
            DFA_SEL(2)
            default:
            DFA_SEL(3)
#undef DFA_SEL
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t v = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t i = pos + 4 * q + k;
                v |= (i < n ? (uint32_t)in[i] : 0u) << (8 * k);
            }
            o[q] = v;
        }
    }
}

typedef __attribute__((address_space(3))) const uint32_t lds_u32_t;
__device__ __forceinline__ uint32_t lds_ld32(uint32_t addr) {
    return *(lds_u32_t *)(size_t)addr;
}

// True in every lane when every live slot of the wavefront sits in an
// absorbing state (bit st >> shift of the LDS bitmap at byte `base`).
template <int S>
__device__ __forceinline__ bool wave_absorbed(const uint32_t (&st)[S], uint32_t live,
                                              uint32_t base, uint32_t shift) {
    bool dead = true;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if ((live >> j) & 1u) {
            const uint32_t idx = st[j] >> shift;
            const uint32_t w = lds_ld32(base + ((idx >> 5) << 2));
            dead = dead && ((w >> (idx & 31)) & 1u);
        }
    }
    return __all(dead);
}

// One step of every slot with code K of its dword.
template <int L, int K, int S>
__device__ __forceinline__ void step_slots(uint32_t (&st)[S], const uint32_t (&w)[S]) {
#pragma unroll
    for (int j = 0; j < S; ++j) st[j] = add_sel<L, K>(st[j], w[j]);
#pragma unroll
    for (int j = 0; j < S; ++j) st[j] = lds_ld(st[j]);
}

// With EXIT the walk stops early (every few blocks it checks) once every live
// slot of the wavefront is absorbing: the rest of the chunk cannot change
// those states.  exit_base = 0 (no absorbing state) skips the check.
//
// Code blocks are software-pipelined: A = PF + 1 blocks per slot sit in
// registers, and the register that held block b is reloaded with block
// b + A right after its last use, so each load has PF blocks of walking to
// arrive.  The steady-state loop is unrolled by A and issues every load
// without a branch (past the last block it reloads the last block, which is
// never walked again), so that the wait before a block's first step waits
// for that block's own load only; a load under a branch, or a register
// copied between ring slots, would make it wait for every load in flight.
template <int L, int S>
__device__ __forceinline__ void walk_block(const uint4 (&blk)[S], uint32_t (&st)[S]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t w[S];
#pragma unroll
        for (int j = 0; j < S; ++j)
            w[j] = word_codes<L>(q == 0 ? blk[j].x : q == 1 ? blk[j].y : q == 2 ? blk[j].z : blk[j].w);
        // round-robin over the slots, one code at a time, so that the
        // slots' independent chains keep several LDS loads in flight
        step_slots<L, 0, S>(st, w);
        step_slots<L, 1, S>(st, w);
        if constexpr (!kWideCodes<L>) {
            step_slots<L, 2, S>(st, w);
            step_slots<L, 3, S>(st, w);
        }
    }
}

template <int L, int S, bool EXIT = false, int PF = 1>
__device__ __forceinline__ void walk_fast(const uint4 *__restrict__ codes16,
                                          const uint32_t (&o16)[S], uint32_t blocks,
                                          uint32_t (&st)[S], uint32_t exit_base = 0,
                                          uint32_t exit_shift = 0, uint32_t live = 0,
                                          uint32_t stride = 1) {
    constexpr uint32_t A = PF + 1;
    if (blocks == 0) return;
    const uint32_t last = blocks - 1;
    uint4 buf[A][S];
#pragma unroll
    for (uint32_t k = 0; k < A; ++k)
#pragma unroll
        for (int j = 0; j < S; ++j)
            buf[k][j] = codes16[(size_t)o16[j] + (size_t)min(k, last) * stride];
    uint32_t b0 = 0;
    for (; b0 + A <= blocks; b0 += A) {
#pragma unroll
        for (uint32_t k = 0; k < A; ++k) {
            walk_block<L, S>(buf[k], st);
            const uint32_t nb = min(b0 + k + A, last);
#pragma unroll
            for (int j = 0; j < S; ++j)
                buf[k][j] = codes16[(size_t)o16[j] + (size_t)nb * stride];
        }
        if constexpr (EXIT)
            if (exit_base && ((b0 / A) & 1u) && wave_absorbed(st, live, exit_base, exit_shift))
                return;
    }
    // fewer than A blocks left: they are in buf[0 ..]
#pragma unroll
    for (uint32_t k = 0; k + 1 < A; ++k)
        if (b0 + k < blocks) walk_block<L, S>(buf[k], st);
}

// Walk pairs whose chunks may end inside a 16-byte block: slot j walks
// len_of(j) codes from 16-byte unit o16[j].  All slots first walk their
// common whole blocks on the fast path; then each slot finishes its own
// remaining blocks, stepping only over codes it owns (the last block of a
// translated stream is read whole, as code streams are padded to whole
// blocks; raw input (L = 3) is read byte by byte past its last whole block).
// len_of recomputes a slot's length, so no per-slot length stays live through
// the fast path.
template <int L, int S, bool EXIT = false, int PF = 1, typename LenFn>
__device__ __forceinline__ void walk_var(const uint4 *__restrict__ codes16,
                                         const uint32_t (&o16)[S], LenFn len_of,
                                         uint32_t (&st)[S], uint32_t exit_base = 0,
                                         uint32_t exit_shift = 0, uint32_t live = 0,
                                         uint32_t stride = 1) {
    constexpr uint32_t kPer16 = kWideCodes<L> ? 8u : 16u;
    uint32_t common = 0xFFFFFFFFu, most = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const uint32_t len = len_of(j);
        common = min(common, len / kPer16);
        most = max(most, (len + kPer16 - 1) / kPer16);
    }
    if (common > 0)
        walk_fast<L, S, EXIT, PF>(codes16, o16, common, st, exit_base, exit_shift, live, stride);
    for (uint32_t b = common; b < most; ++b) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const uint32_t len = len_of(j);
            if (b * kPer16 >= len) continue;
            const uint32_t cnt = min(kPer16, len - b * kPer16);
            uint32_t w[4];
            if (L == 3 && cnt < kPer16) {
                const uint8_t *p =
                    reinterpret_cast<const uint8_t *>(codes16 + o16[j] + (size_t)b * stride);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t v = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if ((uint32_t)(4 * q + k) < cnt) v |= (uint32_t)p[4 * q + k] << (8 * k);
                    w[q] = word_codes<L>(v);
                }
            } else {
                const uint4 v = codes16[(size_t)o16[j] + (size_t)b * stride];
                w[0] = word_codes<L>(v.x); w[1] = word_codes<L>(v.y);
                w[2] = word_codes<L>(v.z); w[3] = word_codes<L>(v.w);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (!kWideCodes<L>) {
                    if (4 * q + 0 < cnt) st[j] = lds_ld(add_sel<1, 0>(st[j], w[q]));
                    if (4 * q + 1 < cnt) st[j] = lds_ld(add_sel<1, 1>(st[j], w[q]));
                    if (4 * q + 2 < cnt) st[j] = lds_ld(add_sel<1, 2>(st[j], w[q]));
                    if (4 * q + 3 < cnt) st[j] = lds_ld(add_sel<1, 3>(st[j], w[q]));
                } else {
                    if (2 * q + 0 < cnt) st[j] = lds_ld(add_sel<2, 0>(st[j], w[q]));
                    if (2 * q + 1 < cnt) st[j] = lds_ld(add_sel<2, 1>(st[j], w[q]));
                }
            }
        }
    }
}

// Owner chunk of pair P: the last i with first[i] <= P, searched in the
// tile's window [lo, hi) (first[lo] <= P < first[hi]).
__device__ __forceinline__ uint32_t owner_chunk(const uint32_t *__restrict__ first, uint32_t lo,
                                                uint32_t hi, uint32_t P) {
    while (hi > lo + 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (first[mid] <= P) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace dfaspec
