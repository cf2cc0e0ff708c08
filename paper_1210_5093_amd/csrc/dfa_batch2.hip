// Batched membership tests on the packed-pair matcher.
//
// Many (DFA, string) pairs of uneven size run as one flat set of (chunk,
// start state) pairs, exactly as one long string does in dfa_match2.hip:
// every string is cut into chunks of one length C, chunk i >= 1 of a string
// is walked from each state of its reverse-lookahead set (Eq. 11, or the
// precomputed I_{c1..ck} of Eq. 13 when the DFA has them), and the pairs are
// packed 256 to a wave-tile, so lanes stay busy whatever the set sizes are.
// Strings that share a DFA form a group; a group's pairs start on a tile
// boundary, so every tile belongs to one DFA, and a workgroup stages that
// DFA's table in LDS once per task (a task is up to one tile per wave of the
// workgroup, from one group).  Per run, on the device only:
//   reset -> translate (bytes -> codes, per string) -> chunk info (set size
//   and id per chunk) -> size scan -> group layout (aligned pair bases, tile
//   and task counts) -> pair layout (first pair and tile owners per chunk) ->
//   matcher (persistent, tasks from a counter) -> composition (Eq. 9) per
//   string, level by level -> final record per string.
// The host plans everything that depends only on the lengths, so a run
// allocates nothing and can be captured in a HIP graph.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>

#include "dfa_pairs.h"
#include "dfa_walk1.h"

namespace dfaspec {

namespace {

constexpr uint32_t kB2Levels = 12;
constexpr uint64_t kB2Segment = 1u << 20;         // translation segment (bytes)

struct B2Str {            // one string
    const uint8_t *in;
    uint64_t code_off;    // byte offset of its code stream in the code arena (16-aligned)
    uint64_t n;
    uint32_t chunk0;      // global index of its chunk 0
    uint32_t nch;
    uint32_t r;           // lookahead symbols: 1 = I_sigma, >= 2 = precomputed sets
    uint32_t start;
    uint32_t dfa;
    uint32_t group;
};

struct B2Req {            // per-string composition plan (strided levels 1 .. levels)
    uint32_t stride;      // entries of a strided map (the DFA's I_max, padded)
    uint32_t G;           // fan-in
    uint32_t levels;
    uint32_t pad;
    uint32_t count[kB2Levels];
    uint64_t map_off[kB2Levels];
    uint64_t size_off[kB2Levels];
};

struct B2Group {          // strings sharing a DFA; their chunks are contiguous
    uint32_t dfa;
    uint32_t layout;
    uint32_t chunk_lo, chunk_hi;
};

struct B2Seg {            // translation segment [beg, beg + len) of one string
    uint32_t str;
    uint32_t pad;
    uint64_t beg, len;
};

struct B2Item {           // one output map of a composition level
    uint32_t str;
    uint32_t g;
};

struct B2Args {
    const DevDFA *dfas;
    const B2Str *strs;
    const B2Req *reqs;
    const B2Group *groups;
    uint32_t ngroups;
    uint32_t count;
    const uint32_t *chunk_str;   // [N] string of each global chunk
    uint32_t nchunks;
    uint64_t chunk;
    uint8_t *codes;
    uint32_t *str_bad;           // [count] a byte outside Sigma
    uint16_t *msize0;            // [N] start-set size per chunk
    uint32_t *cset;              // [N] class (r = 1) or set id (r >= 2) per chunk
    uint32_t *first_raw;         // [N + 1] exclusive scan of msize0
    uint32_t *first2;            // [N + 1] first pair of each chunk, groups tile-aligned
    uint32_t *tile_first2;       // [tiles] chunk holding the first pair of each tile
    uint32_t *gtile;             // [ngroups + 1] first tile of each group
    uint32_t *gtask;             // [ngroups + 1] first task of each group
    uint32_t *gend;              // [ngroups] end pair of each group
    uint32_t *counter;
    uint16_t *maps0;             // pair-indexed level-0 maps
    uint16_t *maps;              // strided levels
    uint16_t *msize;
    uint32_t task_slot;          // LDS byte offset of the task broadcast word
    uint32_t wpb;                // waves per matcher workgroup = tiles per task
    uint32_t early_exit;         // stop a tile once all its pairs are absorbing
    uint32_t slots;              // pairs per lane (2 or 4); a tile holds 64 * slots pairs
    uint32_t tile;
};

__global__ void k_b2_reset(B2Args a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.count) a.str_bad[i] = 0;
    if (i == 0) *a.counter = 0;
}

// Bytes -> codes with the segment's DFA (one-byte codes for layout 1,
// two-byte codes for layout 2); a byte outside Sigma flags its string.
__global__ __launch_bounds__(256) void k_b2_translate(B2Args a, const B2Seg *__restrict__ segs,
                                                      uint32_t nseg) {
    __shared__ uint16_t lut[256];
    for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const B2Seg seg = segs[sg];
        const B2Str st = a.strs[seg.str];
        const DevDFA &d = a.dfas[st.dfa];
        __syncthreads();
        lut[threadIdx.x] = d.code[threadIdx.x];
        __syncthreads();
        const bool wide = d.layout != 1;
        uint32_t bad = 0;
        auto convert = [&](const uint32_t (&w)[4], uint64_t off) {
            const uint64_t pos = seg.beg + off;
            const uint32_t cnt = (uint32_t)min<uint64_t>(16, seg.len - off);
            uint16_t c[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint16_t v = lut[(w[k >> 2] >> (8 * (k & 3))) & 0xFFu];
                const bool inside = (uint32_t)k < cnt;
                bad |= (inside && v == kCodeInvalid) ? 1u : 0u;
                c[k] = (v == kCodeInvalid || !inside) ? (uint16_t)0 : v;
            }
            // pos is a multiple of 16 and the code stream is 16-aligned
            if (!wide) {
                uint4 o;
                uint32_t *ow = reinterpret_cast<uint32_t *>(&o);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ow[q] = (uint32_t)c[4 * q] | ((uint32_t)c[4 * q + 1] << 8) |
                            ((uint32_t)c[4 * q + 2] << 16) | ((uint32_t)c[4 * q + 3] << 24);
                *reinterpret_cast<uint4 *>(a.codes + st.code_off + pos) = o;
            } else {
                uint4 o[2];
                uint32_t *ow = reinterpret_cast<uint32_t *>(o);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    ow[q] = (uint32_t)c[2 * q] | ((uint32_t)c[2 * q + 1] << 16);
                uint4 *dst = reinterpret_cast<uint4 *>(a.codes + st.code_off + 2 * pos);
                dst[0] = o[0];
                dst[1] = o[1];
            }
        };
        // Whole rounds first: U blocks of 16 bytes per thread, all loaded
        // before any is used (one load in flight per lane leaves the pass
        // latency bound).  The segment start and its misalignment are the
        // same for every lane, so these rounds take no per-lane branches.
        constexpr int U = 4;
        typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(1))) const u32x4_t gu4_t;
        const uint64_t round = (uint64_t)blockDim.x * 16 * U;
        const uintptr_t p0 = (uintptr_t)(st.in + seg.beg);
        const uint32_t sh = (uint32_t)(p0 & 15u);
        const uintptr_t a0 = p0 - sh;                    // aligned base
        // the aligned words read stay inside the string: whole rounds end at
        // or before seg.len, and a misaligned round also reads the 16 bytes
        // after its last block (up to byte seg.beg + end + sh + 15 < n)
        const uint64_t avail = st.n - seg.beg;
        uint64_t whole = seg.len / round * round;
        if (sh != 0)
            while (whole > 0 && whole + 16 > avail) whole -= round;
        uint64_t base = 0;
        for (; base < whole; base += round) {
            uint32_t w[U][4];
            if (sh == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t off = base + ((uint64_t)u * blockDim.x + threadIdx.x) * 16;
                    const u32x4_t v = *(gu4_t *)(a0 + off);
                    w[u][0] = v.x; w[u][1] = v.y; w[u][2] = v.z; w[u][3] = v.w;
                }
            } else {
                u32x4_t v0[U], v1[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t off = base + ((uint64_t)u * blockDim.x + threadIdx.x) * 16;
                    v0[u] = *(gu4_t *)(a0 + off);
                    v1[u] = *(gu4_t *)(a0 + off + 16);
                }
                const uint32_t r = sh & 3u, q0 = sh >> 2;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t x[8] = {v0[u].x, v0[u].y, v0[u].z, v0[u].w,
                                           v1[u].x, v1[u].y, v1[u].z, v1[u].w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // words q0 + q and q0 + q + 1 of x, selected without
                        // dynamic register indexing
                        uint32_t lo = x[q], hi = x[q + 1];
                        if (q0 == 1) { lo = x[q + 1]; hi = x[q + 2]; }
                        if (q0 == 2) { lo = x[q + 2]; hi = x[q + 3]; }
                        if (q0 == 3) { lo = x[q + 3]; hi = x[q + 4]; }
                        w[u][q] = __builtin_amdgcn_alignbyte(hi, lo, r);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                convert(w[u], base + ((uint64_t)u * blockDim.x + threadIdx.x) * 16);
        }
        // the rest: one block at a time
        for (uint64_t off = base + (uint64_t)threadIdx.x * 16; off < seg.len;
             off += (uint64_t)blockDim.x * 16) {
            uint32_t w[4];
            load16(st.in, seg.beg + off, st.n, w);   // seg.beg + off < n
            convert(w, off);
        }
        if (bad) atomicOr(&a.str_bad[seg.str], 1u);
    }
}

// Start-set size and id of every chunk (chunk 0 of a string: its start state).
__global__ void k_b2_chunkinfo(B2Args a) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.nchunks) return;
    const B2Str st = a.strs[a.chunk_str[g]];
    const DevDFA &d = a.dfas[st.dfa];
    const uint32_t i = g - st.chunk0;
    uint32_t m = 1, id = 0;
    if (i > 0) {
        const uint64_t p = (uint64_t)i * a.chunk;
        if (st.r <= 1) {
            const uint32_t e = d.lut[st.in[p - 1]];
            if (e == kLutInvalid) {
                m = 0;     // the translation flags the string
            } else {
                id = e >> 24;
                m = d.set_off[1][id + 1] - d.set_off[1][id];
            }
        } else {
            const uint32_t k = (uint32_t)min<uint64_t>(st.r, p);
            bool bad = false;
            id = class_string_id(d, st.in, p - k, k, &bad);
            m = bad ? 0u : mset_end(d, k, id) - mset_begin(d, k, id);
        }
    }
    a.msize0[g] = (uint16_t)m;
    a.cset[g] = id;
}

// One workgroup: per group, its pair count, tiles and tasks, and their
// exclusive prefixes (groups start on tile boundaries).
__global__ __launch_bounds__(1024) void k_b2_groups(B2Args a) {
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x, T = blockDim.x;
    const uint32_t per = (a.ngroups + T - 1) / T;
    const uint32_t lo = min(a.ngroups, t * per), hi = min(a.ngroups, lo + per);
    uint32_t tiles = 0, tasks = 0;
    for (uint32_t k = lo; k < hi; ++k) {
        const B2Group gr = a.groups[k];
        const uint32_t pairs = a.first_raw[gr.chunk_hi] - a.first_raw[gr.chunk_lo];
        const uint32_t tk = (pairs + a.tile - 1) / a.tile;
        tiles += tk;
        tasks += (tk + a.wpb - 1) / a.wpb;
    }
    // two inclusive scans (tiles, tasks) over the threads' segment sums
    part[t] = tiles;
    __syncthreads();
    for (uint32_t off = 1; off < T; off <<= 1) {
        const uint32_t u = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += u;
        __syncthreads();
    }
    uint32_t tile_run = part[t] - tiles;
    const uint32_t tile_total = part[T - 1];
    __syncthreads();
    part[t] = tasks;
    __syncthreads();
    for (uint32_t off = 1; off < T; off <<= 1) {
        const uint32_t u = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += u;
        __syncthreads();
    }
    uint32_t task_run = part[t] - tasks;
    const uint32_t task_total = part[T - 1];
    for (uint32_t k = lo; k < hi; ++k) {
        const B2Group gr = a.groups[k];
        const uint32_t pairs = a.first_raw[gr.chunk_hi] - a.first_raw[gr.chunk_lo];
        const uint32_t tk = (pairs + a.tile - 1) / a.tile;
        a.gtile[k] = tile_run;
        a.gtask[k] = task_run;
        a.gend[k] = tile_run * a.tile + pairs;
        tile_run += tk;
        task_run += (tk + a.wpb - 1) / a.wpb;
    }
    if (t == T - 1) {
        a.gtile[a.ngroups] = tile_total;
        a.gtask[a.ngroups] = task_total;
        a.first2[a.nchunks] = tile_total * a.tile;
    }
}

// Aligned first pair of every chunk and the owner chunk of every tile start.
__global__ void k_b2_pairs(B2Args a) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.nchunks) return;
    const uint32_t k = a.strs[a.chunk_str[g]].group;
    const B2Group gr = a.groups[k];
    const uint32_t A = a.gtile[k] * a.tile + (a.first_raw[g] - a.first_raw[gr.chunk_lo]);
    const uint32_t m = a.msize0[g] & 0x7FFFu;
    a.first2[g] = A;
    if (m)
        for (uint32_t w = (A + a.tile - 1) / a.tile; w <= (A + m - 1) / a.tile; ++w)
            a.tile_first2[w] = g;
}

// Group of task t: the last k with gtask[k] <= t (wave-uniform).
__device__ __forceinline__ uint32_t group_of(const uint32_t *__restrict__ gtask, uint32_t ng,
                                             uint32_t t) {
    uint32_t lo = 0, hi = ng;
    while (hi > lo + 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (gtask[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// One wave-tile of group k (all pairs of one DFA), layout L.
template <int L, int S>
__device__ __forceinline__ void b2_tile(const B2Args &a, const DevDFA &d, uint32_t k,
                                        uint32_t tile, uint32_t lane) {
    constexpr uint32_t kTile = kWave2 * S;
    using CodeT = typename std::conditional<L == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t kPer16 = 16 / sizeof(CodeT);
    const uint32_t pair_end = a.gend[k];
    const uint32_t tile_end = a.gtile[k + 1];
    const B2Group gr = a.groups[k];
    const uint32_t lo0 = a.tile_first2[tile];
    const uint32_t hi0 = tile + 1 < tile_end ? a.tile_first2[tile + 1] + 1 : gr.chunk_hi;
    const uint32_t R = L == 1 ? d.rowbytes : 2u;
    uint32_t st[S], ci[S], o16[S], len[S];   // len: codes per slot
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const uint32_t P = tile * kTile + j * kWave2 + lane;
        const bool valid = P < pair_end;
        // a pair beyond the group's end shadows the tile's first pair (a real
        // chunk of this DFA) from state 0, so its loads stay valid; its end
        // state is discarded
        const uint32_t c = valid ? owner_chunk(a.first2, lo0, hi0, P) : lo0;
        const B2Str s = a.strs[a.chunk_str[c]];
        const uint32_t i = c - s.chunk0;
        uint32_t q = 0;
        if (valid) {
            if (i == 0) {
                q = s.start;
            } else if (s.r <= 1) {
                q = d.set_st[1][d.set_off[1][a.cset[c]] + (P - a.first2[c])];
            } else {
                const uint32_t kk = (uint32_t)min<uint64_t>(s.r, (uint64_t)i * a.chunk);
                q = d.mset_st[d.mst[kk] + mset_begin(d, kk, a.cset[c]) + (P - a.first2[c])];
            }
        }
        st[j] = R * q;
        ci[j] = valid ? c : 0xFFFFFFFFu;
        // chunk starts are whole 16-byte units: the chunk length is a
        // multiple of 64 and every code stream starts 16-byte aligned
        o16[j] = (uint32_t)((s.code_off / sizeof(CodeT) + (uint64_t)i * a.chunk) / kPer16);
        len[j] = (uint32_t)min<uint64_t>(a.chunk, s.n - (uint64_t)i * a.chunk);
    }
    uint32_t live = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) live |= (ci[j] != 0xFFFFFFFFu ? 1u : 0u) << j;
    auto len_of = [&](int j) -> uint32_t { return len[j]; };
    if (a.early_exit && d.nabs > 0)
        walk_var<L, S, true>(reinterpret_cast<const uint4 *>(a.codes), o16, len_of, st, d.abs_off,
                             d.abs_shift, live);
    else
        walk_var<L, S, false>(reinterpret_cast<const uint4 *>(a.codes), o16, len_of, st);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (ci[j] == 0xFFFFFFFFu) continue;
        const uint32_t c = ci[j];
        const B2Str s = a.strs[a.chunk_str[c]];
        const uint32_t i = c - s.chunk0;
        const uint32_t e = st[j] / R;
        const uint32_t P = tile * kTile + j * kWave2 + lane;
        uint16_t v;
        if (i + 1 == s.nch) {
            v = (uint16_t)(kTerm | e);
        } else if (s.r <= 1) {
            v = d.pos[1][(size_t)a.cset[c + 1] * d.nq + e];
        } else {
            const uint16_t ab = d.pos[1][e];   // class-0 row: kTerm|e iff e is absorbing
            const uint32_t kk = (uint32_t)min<uint64_t>(s.r, (uint64_t)(i + 1) * a.chunk);
            const uint32_t id = a.cset[c + 1];
            v = ab == (uint16_t)(kTerm | e)
                    ? ab
                    : (uint16_t)member_rank(d.mset_st + d.mst[kk], mset_begin(d, kk, id),
                                            mset_end(d, kk, id), e);
        }
        a.maps0[P] = v;
    }
}

// Persistent matcher: a task is up to a.wpb tiles of one group.  The
// table sits at LDS address 0 (no static LDS in this kernel); the task word
// is broadcast through LDS at a.task_slot.  S: pairs per lane.
template <int S>
__global__ __launch_bounds__(1024) void k_b2_match(B2Args a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *s_task = reinterpret_cast<uint32_t *>(smem + a.task_slot);
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t wave = threadIdx.x / kWave2;
    const uint32_t ntasks = a.gtask[a.ngroups];
    uint32_t cur = 0xFFFFFFFFu;
    while (true) {
        if (threadIdx.x == 0) *s_task = atomicAdd(a.counter, 1u);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(*s_task);
        __syncthreads();
        if (t >= ntasks) break;
        const uint32_t k = group_of(a.gtask, a.ngroups, t);
        const B2Group gr = a.groups[k];
        const DevDFA &d = a.dfas[gr.dfa];
        if (gr.dfa != cur) {
            const uint4 *src = reinterpret_cast<const uint4 *>(d.stab);
            uint4 *dst = reinterpret_cast<uint4 *>(smem);
            for (uint32_t x = threadIdx.x; x < d.stab_bytes / 16; x += blockDim.x) dst[x] = src[x];
            __syncthreads();
            cur = gr.dfa;
        }
        const uint32_t tile = a.gtile[k] + (t - a.gtask[k]) * a.wpb + wave;
        if (tile < a.gtile[k + 1]) {
            if (gr.layout == 1)
                b2_tile<1, S>(a, d, k, tile, lane);
            else
                b2_tile<2, S>(a, d, k, tile, lane);
        }
        __syncthreads();   // the table may be restaged by the next task
    }
}

// Level 0 (pair-indexed) -> level 1 (strided): one workgroup per output map.
__global__ __launch_bounds__(256) void k_b2_compose0(B2Args a, const B2Item *__restrict__ items) {
    extern __shared__ __align__(16) uint8_t smem[];
    const B2Item it = items[blockIdx.x];
    const B2Str s = a.strs[it.str];
    const B2Req rq = a.reqs[it.str];
    const uint32_t G = rq.G;
    const uint32_t c0 = s.chunk0 + it.g * G;
    const uint32_t cnt = min(G, s.chunk0 + s.nch - c0);
    uint32_t *off = reinterpret_cast<uint32_t *>(smem);
    uint16_t *sm = reinterpret_cast<uint16_t *>(smem + 4 * (G + 1));
    const uint32_t base = a.first2[c0];
    for (uint32_t t = threadIdx.x; t <= cnt; t += blockDim.x) off[t] = a.first2[c0 + t] - base;
    __syncthreads();
    const uint32_t entries = off[cnt];
    for (uint32_t x = threadIdx.x; x < entries; x += blockDim.x) sm[x] = a.maps0[base + x];
    __syncthreads();
    const uint32_t m = a.msize0[c0] & 0x7FFFu;
    uint16_t *out = a.maps + rq.map_off[1] + (size_t)it.g * rq.stride;
    for (uint32_t p = threadIdx.x; p < m; p += blockDim.x) {
        uint32_t v = sm[p];
        for (uint32_t t = 1; t < cnt && !(v & kTerm); ++t)
            v = (v < off[t + 1] - off[t]) ? sm[off[t] + v] : kBadPos;
        out[p] = (uint16_t)v;
    }
    if (threadIdx.x == 0) a.msize[rq.size_off[1] + it.g] = (uint16_t)m;
}

// Strided level l -> l + 1: one workgroup per output map.
__global__ __launch_bounds__(256) void k_b2_compose(B2Args a, const B2Item *__restrict__ items,
                                                    uint32_t l) {
    extern __shared__ __align__(16) uint16_t sm2[];
    const B2Item it = items[blockIdx.x];
    const B2Req rq = a.reqs[it.str];
    const uint32_t G = rq.G, stride = rq.stride;
    const uint32_t first = it.g * G;
    const uint32_t cnt = min(G, rq.count[l] - first);
    const uint16_t *src = a.maps + rq.map_off[l] + (size_t)first * stride;
    for (uint32_t x = threadIdx.x; x < cnt * stride; x += blockDim.x) sm2[x] = src[x];
    __syncthreads();
    const uint32_t m = a.msize[rq.size_off[l] + first] & 0x7FFFu;
    compose_staged(sm2, cnt, stride, m, a.maps + rq.map_off[l + 1] + (size_t)it.g * stride);
    if (threadIdx.x == 0) a.msize[rq.size_off[l + 1] + it.g] = (uint16_t)m;
}

__global__ void k_b2_finalize(B2Args a, uint32_t *__restrict__ results) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const B2Str s = a.strs[i];
    const B2Req rq = a.reqs[i];
    const DevDFA &d = a.dfas[s.dfa];
    uint32_t fin = 0xFFFFFFFFu, acc = 0, flags = 0;
    if (a.str_bad[i]) {
        flags = DFA_FLAG_SYMBOL;
    } else if (s.nch == 0) {
        fin = s.start;
    } else {
        const uint32_t v = rq.levels == 0 ? a.maps0[a.first2[s.chunk0]] : a.maps[rq.map_off[rq.levels]];
        if (!(v & kTerm) || (v & 0x7FFFu) >= d.nq)
            flags = DFA_FLAG_SPECULATION;
        else
            fin = v & 0x7FFFu;
    }
    if (!flags) acc = (d.accept_bits[fin >> 5] >> (fin & 31)) & 1u;
    results[4 * i + 0] = fin;
    results[4 * i + 1] = acc;
    results[4 * i + 2] = flags;
    results[4 * i + 3] = s.nch;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }
bool g_b2_attr_set = false;

}  // namespace

// ---------------------------------------------------------------------------
// Host: planning (pure host work) and launching (device work only)
// ---------------------------------------------------------------------------
bool batch2_supported(const dfa_t *const *dfas, size_t count) {
    for (size_t i = 0; i < count; ++i)
        if (!dfas[i] || dfas[i]->dev.layout == 0) return false;
    return true;
}

int plan_batch2(const dfa_t *const *dfas, const uint8_t *const *d_inputs, const size_t *lens,
                size_t count, uint64_t chunk_req, uint32_t lookahead, Batch2Plan *out,
                uint32_t flags) {
    Batch2Plan &P = *out;
    P = Batch2Plan();
    P.early_exit = (flags & DFA_MATCH_EARLY_EXIT) ? 1u : 0u;
    // two pairs per lane (shorter tiles); DFA_SLOTS=4 forces four
    const char *fs = std::getenv("DFA_SLOTS");
    P.slots = fs && fs[0] == '4' ? 4u : 2u;
    const uint32_t kTile = match2_tile_pairs(P.slots);
    if (count && (!dfas || !d_inputs || !lens)) return fail(DFA_E_INVAL, "batch plan: NULL argument");
    if (count > 0x7FFFFFFFull) return fail(DFA_E_TOOBIG, "batch plan: too many strings");
    const int lds = device_lds_bytes();
    const int cus = std::max(device_cu_count(), 1);
    if (lds <= 0) return fail(DFA_E_DEVICE, "no HIP device");
    P.count = (uint32_t)count;

    // distinct DFAs, groups of strings per DFA (costlier DFAs first)
    std::map<const dfa_t *, uint32_t> index;
    std::vector<const dfa_t *> uniq;
    for (size_t i = 0; i < count; ++i) {
        if (!dfas[i]) return fail(DFA_E_INVAL, "batch plan: NULL dfa");
        if (dfas[i]->dev.layout == 0) return fail(DFA_E_INVAL, "batch plan: DFA without a packed layout");
        if (lens[i] && !d_inputs[i]) return fail(DFA_E_INVAL, "batch plan: NULL input");
        if (index.emplace(dfas[i], (uint32_t)uniq.size()).second) uniq.push_back(dfas[i]);
    }
    auto r_of = [&](const dfa_t *d) -> uint32_t {
        if (lookahead <= 1 || d->dev.r0 < 2) return 1u;
        return std::min<uint32_t>(lookahead, d->dev.r0);
    };
    auto mean_set = [&](const dfa_t *d) -> double {
        const uint32_t r = r_of(d);
        return r <= 1 ? std::max(d->info.mean_iset, 1.0) : std::max(d->mset_mean[r], 1.0);
    };
    std::vector<uint32_t> dorder(uniq.size());
    std::iota(dorder.begin(), dorder.end(), 0u);
    std::stable_sort(dorder.begin(), dorder.end(), [&](uint32_t x, uint32_t y) {
        return mean_set(uniq[x]) > mean_set(uniq[y]);
    });
    uint32_t max_stab = 16;
    for (auto *d : uniq) max_stab = std::max(max_stab, d->dev.stab_bytes);
    if ((size_t)max_stab + 16 > (size_t)lds) return fail(DFA_E_TOOBIG, "batch plan: table exceeds LDS");

    // chunk length: about 64 wave-tiles of pairs per resident wave slot, so
    // that chains stay short (the matcher is latency bound when they are
    // long) while the per-chunk work stays small
    uint64_t chunk = chunk_req;
    if (!chunk) {
        double work = 0.0;
        for (size_t i = 0; i < count; ++i) work += (double)lens[i] * mean_set(dfas[i]);
        const double target_pairs = 64.0 * cus * 16.0 * kTile;
        chunk = (uint64_t)std::max(1024.0, work / target_pairs);
        chunk = std::min<uint64_t>((chunk + 63) / 64 * 64, 1u << 20);
    }
    chunk = std::max<uint64_t>(64, (chunk + 63) / 64 * 64);   // 16-code aligned chunks
    P.chunk = chunk;

    // strings in group order
    std::vector<std::vector<uint32_t>> by_dfa(uniq.size());
    for (size_t i = 0; i < count; ++i) by_dfa[index[dfas[i]]].push_back((uint32_t)i);
    std::vector<B2Str> strs(count);
    std::vector<B2Req> reqs(count);
    std::vector<B2Group> groups;
    std::vector<uint32_t> chunk_str;
    std::vector<B2Seg> segs;
    uint64_t code_bytes = 0, pairs_ub = 0, map_entries = 0, size_entries = 0;
    size_t compose_stage = 0, compose0_stage = 0;
    for (uint32_t di : dorder) {
        const dfa_t *d = uniq[di];
        B2Group gr;
        gr.dfa = di;
        gr.layout = d->dev.layout;
        gr.chunk_lo = (uint32_t)chunk_str.size();
        const uint32_t cb = d->dev.layout == 1 ? 1u : 2u;
        const uint32_t r = r_of(d);
        const uint32_t setmax = std::max<uint32_t>(d->setmax_host[1], 1u);
        for (uint32_t i : by_dfa[di]) {
            B2Str &s = strs[i];
            std::memset(&s, 0, sizeof(s));
            s.in = d_inputs[i];
            s.n = lens[i];
            s.code_off = code_bytes;
            code_bytes += (lens[i] + 15) / 16 * 16 * cb;   // whole 16-code blocks
            const uint64_t nch = (lens[i] + chunk - 1) / chunk;
            if (chunk_str.size() + nch > 0x7FFFFFFFull) return fail(DFA_E_TOOBIG, "batch plan: too many chunks");
            s.chunk0 = (uint32_t)chunk_str.size();
            s.nch = (uint32_t)nch;
            s.r = r;
            s.start = d->dev.q0;
            s.dfa = di;
            s.group = (uint32_t)groups.size();
            for (uint64_t c = 0; c < nch; ++c) chunk_str.push_back(i);
            if (nch) pairs_ub += 1 + (nch - 1) * setmax;
            for (uint64_t b = 0; b < lens[i]; b += kB2Segment) {
                B2Seg sg;
                sg.str = i;
                sg.pad = 0;
                sg.beg = b;
                sg.len = std::min<uint64_t>(kB2Segment, lens[i] - b);
                segs.push_back(sg);
            }
            // composition plan: level 0 is pair-indexed; strided levels 1..L
            B2Req &q = reqs[i];
            std::memset(&q, 0, sizeof(q));
            q.stride = (setmax + 7u) & ~7u;
            q.G = (uint32_t)std::max<uint64_t>(2, std::min<uint64_t>(64, (96u * 1024u) / (2ull * q.stride)));
            uint64_t c = nch;
            uint32_t L = 0;
            q.count[0] = (uint32_t)nch;
            while (c > 1) {
                if (L + 1 >= kB2Levels) return fail(DFA_E_TOOBIG, "batch plan: too many levels");
                c = (c + q.G - 1) / q.G;
                ++L;
                q.count[L] = (uint32_t)c;
                q.map_off[L] = map_entries;
                q.size_off[L] = size_entries;
                map_entries += c * q.stride;
                size_entries += c;
            }
            q.levels = L;
            P.max_levels = std::max(P.max_levels, L);
            compose_stage = std::max(compose_stage, (size_t)q.G * q.stride * 2);
            compose0_stage = std::max(compose0_stage, 4 * ((size_t)q.G + 1) +
                                                          2 * ((size_t)q.G * setmax + kTile));
        }
        gr.chunk_hi = (uint32_t)chunk_str.size();
        groups.push_back(gr);
        pairs_ub += kTile;   // alignment of the group's first pair
    }
    if (pairs_ub > 0xFFFFFFFFull - 2 * kTile) return fail(DFA_E_TOOBIG, "batch plan: too many pairs");
    P.nchunks = (uint32_t)chunk_str.size();
    P.ngroups = (uint32_t)groups.size();
    P.nsegs = (uint32_t)segs.size();
    const uint64_t tiles_ub = pairs_ub / kTile + groups.size() + 2;

    // composition items per level (level l -> l + 1, l = 0 .. max_levels - 1)
    std::vector<B2Item> items;
    P.items_per_level.assign(P.max_levels, 0);
    P.item_base.assign(P.max_levels, 0);
    for (uint32_t l = 0; l < P.max_levels; ++l) {
        P.item_base[l] = items.size();
        for (size_t i = 0; i < count; ++i)
            if (reqs[i].levels > l)
                for (uint32_t g = 0; g < reqs[i].count[l + 1]; ++g) items.push_back({(uint32_t)i, g});
        P.items_per_level[l] = (uint32_t)(items.size() - P.item_base[l]);
    }

    // device layout: descriptors (uploaded) then per-run arenas
    std::vector<DevDFA> ddfas(uniq.size());
    for (size_t k = 0; k < uniq.size(); ++k) ddfas[k] = uniq[k]->dev;
    size_t at = 0;
    auto place = [&](size_t bytes) { size_t o = at; at = align256(at + std::max<size_t>(bytes, 1)); return o; };
    P.o_dfas = place(ddfas.size() * sizeof(DevDFA));
    P.o_strs = place(strs.size() * sizeof(B2Str));
    P.o_reqs = place(reqs.size() * sizeof(B2Req));
    P.o_groups = place(groups.size() * sizeof(B2Group));
    P.o_segs = place(segs.size() * sizeof(B2Seg));
    P.o_items = place(items.size() * sizeof(B2Item));
    P.o_chunk_str = place(chunk_str.size() * 4);
    P.desc_bytes = at;
    const uint32_t N = P.nchunks;
    P.o_counter = place(4);
    P.o_str_bad = place((size_t)count * 4);
    P.o_msize0 = place((size_t)N * 2);
    P.o_cset = place((size_t)N * 4);
    P.o_first_raw = place(((size_t)N + 1) * 4);
    P.o_first2 = place(((size_t)N + 1) * 4);
    P.o_bsum = place((size_t)match2_scan_blocks(N) * 4 + 4);
    P.o_tile_raw = place((size_t)tiles_ub * 4);
    P.o_tile_first2 = place((size_t)tiles_ub * 4);
    P.o_gtile = place(((size_t)groups.size() + 1) * 4);
    P.o_gtask = place(((size_t)groups.size() + 1) * 4);
    P.o_gend = place((size_t)groups.size() * 4);
    P.o_maps0 = place((size_t)(pairs_ub + kTile) * 2);
    P.o_maps = place((size_t)map_entries * 2);
    P.o_msize = place((size_t)size_entries * 2);
    P.o_codes = place((size_t)code_bytes + 2 * chunk + 16);
    P.total_bytes = at;
    P.desc.assign(P.desc_bytes, 0);
    auto put = [&](size_t o, const void *src, size_t bytes) {
        if (bytes) std::memcpy(P.desc.data() + o, src, bytes);
    };
    put(P.o_dfas, ddfas.data(), ddfas.size() * sizeof(DevDFA));
    put(P.o_strs, strs.data(), strs.size() * sizeof(B2Str));
    put(P.o_reqs, reqs.data(), reqs.size() * sizeof(B2Req));
    put(P.o_groups, groups.data(), groups.size() * sizeof(B2Group));
    put(P.o_segs, segs.data(), segs.size() * sizeof(B2Seg));
    put(P.o_items, items.data(), items.size() * sizeof(B2Item));
    put(P.o_chunk_str, chunk_str.data(), chunk_str.size() * 4);

    P.task_slot = (max_stab + 15) / 16 * 16;
    P.lds_match = P.task_slot + 16;
    P.lds_compose0 = std::max<size_t>(compose0_stage, 16);
    P.lds_compose = std::max<size_t>(compose_stage, 16);
    // persistent matcher grid: the workgroups the LDS allows per CU (up to 8),
    // each wide enough for about 32 resident waves per CU in total
    const uint32_t per_cu = std::max<uint32_t>(1u, std::min<uint32_t>(8u, (uint32_t)(lds / P.lds_match)));
    P.wpb = std::max<uint32_t>(4u, std::min<uint32_t>(16u, 32u / per_cu));
    P.blocks = (uint32_t)cus * per_cu;
    P.tblocks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(P.nsegs, 1), (uint64_t)cus * 8);
    if (!g_b2_attr_set) {
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&k_b2_match<2>), lds) != DFA_OK ||
            allow_dynamic_lds(reinterpret_cast<const void *>(&k_b2_match<4>), lds) != DFA_OK ||
            allow_dynamic_lds(reinterpret_cast<const void *>(&k_b2_compose0), lds) != DFA_OK ||
            allow_dynamic_lds(reinterpret_cast<const void *>(&k_b2_compose), lds) != DFA_OK)
            return fail(DFA_E_DEVICE, "batch plan: cannot enable the device's LDS size");
        g_b2_attr_set = true;
    }
    if (P.lds_compose0 > (size_t)lds || P.lds_compose > (size_t)lds)
        return fail(DFA_E_TOOBIG, "batch plan: composition stage exceeds LDS");
    return DFA_OK;
}

int launch_batch2(const Batch2Plan &P, void *dev_base, hipStream_t s, uint32_t *d_results,
                  hipEvent_t ev_before_match, hipEvent_t ev_after_match) {
    if (!P.count) return DFA_OK;
    uint8_t *base = (uint8_t *)dev_base;
    B2Args a;
    a.dfas = (const DevDFA *)(base + P.o_dfas);
    a.strs = (const B2Str *)(base + P.o_strs);
    a.reqs = (const B2Req *)(base + P.o_reqs);
    a.groups = (const B2Group *)(base + P.o_groups);
    a.ngroups = P.ngroups;
    a.count = P.count;
    a.chunk_str = (const uint32_t *)(base + P.o_chunk_str);
    a.nchunks = P.nchunks;
    a.chunk = P.chunk;
    a.codes = base + P.o_codes;
    a.str_bad = (uint32_t *)(base + P.o_str_bad);
    a.msize0 = (uint16_t *)(base + P.o_msize0);
    a.cset = (uint32_t *)(base + P.o_cset);
    a.first_raw = (uint32_t *)(base + P.o_first_raw);
    a.first2 = (uint32_t *)(base + P.o_first2);
    a.tile_first2 = (uint32_t *)(base + P.o_tile_first2);
    a.gtile = (uint32_t *)(base + P.o_gtile);
    a.gtask = (uint32_t *)(base + P.o_gtask);
    a.gend = (uint32_t *)(base + P.o_gend);
    a.counter = (uint32_t *)(base + P.o_counter);
    a.maps0 = (uint16_t *)(base + P.o_maps0);
    a.maps = (uint16_t *)(base + P.o_maps);
    a.msize = (uint16_t *)(base + P.o_msize);
    a.task_slot = P.task_slot;
    a.wpb = P.wpb;
    a.early_exit = P.early_exit;
    a.slots = P.slots;
    a.tile = match2_tile_pairs(P.slots);
    const B2Seg *segs = (const B2Seg *)(base + P.o_segs);
    const B2Item *items = (const B2Item *)(base + P.o_items);

    hipLaunchKernelGGL(k_b2_reset, dim3((P.count + 255) / 256), dim3(256), 0, s, a);
    if (P.nchunks) {
        if (P.nsegs)
            hipLaunchKernelGGL(k_b2_translate, dim3(P.tblocks), dim3(256), 0, s, a, segs, P.nsegs);
        hipLaunchKernelGGL(k_b2_chunkinfo, dim3((P.nchunks + 255) / 256), dim3(256), 0, s, a);
        int rc = launch_size_scan(P.nchunks, a.msize0, (uint32_t *)(base + P.o_bsum), a.first_raw,
                                  (uint32_t *)(base + P.o_tile_raw), a.tile, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_b2_groups, dim3(1), dim3(1024), 0, s, a);
        hipLaunchKernelGGL(k_b2_pairs, dim3((P.nchunks + 255) / 256), dim3(256), 0, s, a);
        if (ev_before_match) (void)hipEventRecord(ev_before_match, s);
        if (P.slots == 2)
            hipLaunchKernelGGL(k_b2_match<2>, dim3(P.blocks), dim3(P.wpb * kWave2), P.lds_match, s, a);
        else
            hipLaunchKernelGGL(k_b2_match<4>, dim3(P.blocks), dim3(P.wpb * kWave2), P.lds_match, s, a);
        if (ev_after_match) (void)hipEventRecord(ev_after_match, s);
        for (uint32_t l = 0; l < P.max_levels; ++l) {
            if (!P.items_per_level[l]) continue;
            if (l == 0)
                hipLaunchKernelGGL(k_b2_compose0, dim3(P.items_per_level[0]), dim3(256),
                                   P.lds_compose0, s, a, items + P.item_base[0]);
            else
                hipLaunchKernelGGL(k_b2_compose, dim3(P.items_per_level[l]), dim3(256),
                                   P.lds_compose, s, a, items + P.item_base[l], l);
        }
    }
    hipLaunchKernelGGL(k_b2_finalize, dim3((P.count + 255) / 256), dim3(256), 0, s, a, d_results);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "batch launch");
}

}  // namespace dfaspec
