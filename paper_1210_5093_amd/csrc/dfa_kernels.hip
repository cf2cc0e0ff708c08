// HIP kernels of the speculative DFA membership test for gfx950 (wave64).
//
// Chunk matcher (Algorithm 3's parallel loop; Section 4.2): one wavefront
// takes one chunk c_i = w[i*C, min((i+1)*C, n)).  Chunk 0 is walked from the
// start state only; chunk i >= 1 from every state of I_sigma, sigma being the
// class of the chunk's reverse-lookahead byte w[i*C - 1] (Eq. 11).  The
// states of the set are spread across the 64 lanes and KS "slots" per lane
// (state p of the set -> lane p % 64, slot p / 64), so one wave issues KS
// independent table lookups per input byte.  The class-major transition
// table T[c][s] (entries premultiplied to byte offsets) is staged in LDS, so a
// step is one add and one ds_read_u16.  The 64 lanes translate a 64-byte
// block of input through the byte->class LUT in one go (one byte per lane,
// coalesced); v_readlane then hands each byte's column offset to the whole
// wave as a scalar.
//
// Combination (Eqs. 8-9): the sparse state map of chunk i stores, for each
// state of its set, where the walk ends: the end state's position in the next
// chunk's set, or kTerm|state once the state is absorbing or the chunk is the
// last.  Composing G consecutive maps (Eq. 9) yields a map of the same form
// whose domain is the first chunk's set, so a tree of compose levels reduces
// all maps to one; chunk 0's domain is the single start state, so the top
// map has one entry: the final state.  A down-sweep over the same levels
// recovers the state at every chunk boundary (Eq. 8 applied left to right).
#include <cstdlib>

#include "dfa_walk1.h"

namespace dfaspec {

__global__ __launch_bounds__(1024, 8) void k_match(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint8_t *tab = smem;
    const uint32_t *lut = reinterpret_cast<const uint32_t *>(smem + a.d.table_bytes);
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.d.table);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (uint32_t i = threadIdx.x; i < a.d.table_bytes / 16; i += blockDim.x) dst[i] = src[i];
        const uint4 *lsrc = reinterpret_cast<const uint4 *>(a.d.lut);
        uint4 *ldst = reinterpret_cast<uint4 *>(smem + a.d.table_bytes);
        for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x) ldst[i] = lsrc[i];
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t waves = blockDim.x / kWave;
    for (uint32_t c = blockIdx.x * waves + wave; c < a.nch; c += gridDim.x * waves)
        match_one_chunk(a, tab, lut, c, lane);
}

// Compose G consecutive maps of one level into one map of the next (Eq. 9).
__global__ __launch_bounds__(256) void k_compose(const uint16_t *__restrict__ in_maps,
                                                 const uint16_t *__restrict__ in_msize,
                                                 uint32_t n_in, uint32_t stride, uint32_t G,
                                                 uint16_t *__restrict__ out_maps,
                                                 uint16_t *__restrict__ out_msize) {
    extern __shared__ __align__(16) uint16_t sm[];
    __shared__ uint32_t flag;
    const uint32_t g = blockIdx.x;
    const uint32_t first = g * G;
    const uint32_t cnt = min(G, n_in - first);
    if (threadIdx.x == 0) flag = 0;
    __syncthreads();
    if (threadIdx.x < cnt && (in_msize[first + threadIdx.x] & kFlagSymbol)) atomicOr(&flag, 1u);
    const uint16_t *src = in_maps + (size_t)first * stride;
    const uint32_t entries = cnt * stride;
    for (uint32_t i = threadIdx.x; i < entries; i += blockDim.x) sm[i] = src[i];
    __syncthreads();
    const uint32_t m = in_msize[first] & 0x7FFFu;
    compose_staged(sm, cnt, stride, m, out_maps + (size_t)g * stride);
    if (threadIdx.x == 0) out_msize[g] = (uint16_t)(m | (flag ? kFlagSymbol : 0));
}

// Compose groups of up to G consecutive maps (Eq. 9) by a log-depth tree in
// LDS: in round k, the map of every member t with t % 2^(k+1) == 0 (covering
// members t .. t + 2^k - 1) absorbs the map of member t + 2^k, entry by entry
// and in place.  Round k touches only the entries of its active maps, so the
// whole tree costs about one pass over the group's entries.  After
// ceil(log2 G) rounds member 0's map covers the whole group; its domain is
// the group's first set.  Input maps are pair-indexed (`first` != null: member
// t's entries start at first[t] - first[group start]) or strided (`stride_in`
// entries per map, domain sizes in in_msize); every domain holds at most
// stride_in entries.  Output maps are strided.
// The result record from the top map's single entry (chunk 0's domain is the
// start state): the final state, its accept bit, and the flags.
struct FinalArgs {
    const uint32_t *accept_bits;
    uint32_t nq;
    uint32_t nch;
    uint32_t *result;        // NULL: not the top level
    uint32_t *boundaries;    // optional: boundaries[nch] = final state
    const uint32_t *bad;     // translation blocks' flags (byte outside Sigma), or NULL
    uint32_t nbad;
};

__device__ __forceinline__ void write_result(const FinalArgs &fa, uint32_t v, bool symbol) {
    uint32_t flags = 0, fin = 0xFFFFFFFFu, acc = 0;
    if (symbol) {
        flags |= DFA_FLAG_SYMBOL;
    } else if (!(v & kTerm) || (v & 0x7FFFu) >= fa.nq) {
        flags |= DFA_FLAG_SPECULATION;
    } else {
        fin = v & 0x7FFFu;
        acc = (fa.accept_bits[fin >> 5] >> (fin & 31)) & 1u;
    }
    fa.result[0] = fin;
    fa.result[1] = acc;
    fa.result[2] = flags;
    fa.result[3] = fa.nch;
    if (fa.boundaries) fa.boundaries[fa.nch] = fin;
}

// Copies src[0 .. E) into LDS dst[0 .. E) (dst 4-byte aligned): 16-byte
// loads from src's first 16-byte boundary on, four per thread in flight
// before their LDS writes.
__device__ __forceinline__ void stage_u16(uint16_t *dst, const uint16_t *__restrict__ src,
                                          uint32_t E) {
    const uint32_t T = blockDim.x, t = threadIdx.x;
    const uint32_t mis = (uint32_t)((reinterpret_cast<uintptr_t>(src) >> 1) & 7u);
    const uint32_t head = min(E, (8u - mis) & 7u);
    if (t < head) dst[t] = src[t];
    const uint32_t n16 = (E - head) / 8u;
    const uint4 *v = reinterpret_cast<const uint4 *>(src + head);
    uint16_t *d = dst + head;
    constexpr uint32_t U = 4;
    for (uint32_t i0 = 0; i0 < n16; i0 += U * T) {
        uint4 x[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * T + t;
            if (i < n16) x[u] = v[i];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * T + t;
            if (i >= n16) continue;
            const uint32_t w[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
            if ((head & 1u) == 0) {
                uint32_t *d32 = reinterpret_cast<uint32_t *>(d) + 4u * i;
#pragma unroll
                for (int k = 0; k < 4; ++k) d32[k] = w[k];
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    d[8u * i + 2u * k] = (uint16_t)w[k];
                    d[8u * i + 2u * k + 1u] = (uint16_t)(w[k] >> 16);
                }
            }
        }
    }
    for (uint32_t e = head + 8u * n16 + t; e < E; e += T) dst[e] = src[e];
}

__global__ __launch_bounds__(1024) void k_compose_tree(const uint16_t *__restrict__ in_maps,
                                                       const uint32_t *__restrict__ first,
                                                       const uint16_t *__restrict__ in_msize,
                                                       uint32_t n_in, uint32_t stride_in,
                                                       uint32_t G, uint32_t emax,
                                                       uint16_t *__restrict__ out_maps,
                                                       uint32_t stride_out,
                                                       uint16_t *__restrict__ out_msize,
                                                       FinalArgs fa) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t flag;
    uint32_t *off = reinterpret_cast<uint32_t *>(smem);                      // [G + 1]
    uint16_t *dom = reinterpret_cast<uint16_t *>(smem + 4 * (G + 1));        // [G]
    uint16_t *sm = dom + ((G + 1) & ~1u);                                     // [emax]
    const uint32_t g = blockIdx.x, T = blockDim.x;
    const uint32_t c0 = g * G;
    const uint32_t cnt = min(G, n_in - c0);
    const uint32_t W = stride_in;
    const float invW = 1.0f / (float)W;
    if (threadIdx.x == 0) flag = 0;
    __syncthreads();
    // every global read of the group in one phase: offsets, domains, flags
    // and the maps themselves
    const uint64_t base = first ? (uint64_t)first[c0] : (uint64_t)c0 * stride_in;
    const uint32_t E = first ? first[c0 + cnt] - (uint32_t)base : cnt * stride_in;
    for (uint32_t t = threadIdx.x; t <= cnt; t += T)
        off[t] = first ? first[c0 + t] - (uint32_t)base : t * stride_in;
    for (uint32_t t = threadIdx.x; t < cnt; t += T) {
        const uint16_t ms = in_msize[c0 + t];
        if (ms & kFlagSymbol) atomicOr(&flag, 1u);
        dom[t] = first ? (uint16_t)(first[c0 + t + 1] - first[c0 + t]) : (uint16_t)(ms & 0x7FFFu);
    }
    if (fa.result && fa.bad) {
        // the top level also takes the translation pass's flags
        uint32_t any = 0;
        for (uint32_t b = threadIdx.x; b < fa.nbad; b += T) any |= fa.bad[b];
        if (any) atomicOr(&flag, 1u);
    }
    stage_u16(sm, in_maps + base, E);
    __syncthreads();
    for (uint32_t step = 1; step < cnt; step <<= 1) {
        const uint32_t na = (cnt - step + 2 * step - 1) / (2 * step);   // maps with t + step < cnt
        const uint32_t items = na * W;
        for (uint32_t x = threadIdx.x; x < items; x += T) {
            uint32_t i = (uint32_t)((float)x * invW);   // x / W, corrected below
            if (i * W > x) --i;
            else if ((i + 1) * W <= x) ++i;
            const uint32_t j = x - i * W;
            const uint32_t t = i * 2 * step;
            if (j >= dom[t]) continue;
            const uint32_t e = off[t] + j;
            uint32_t v = sm[e];
            if (!(v & kTerm)) {
                const uint32_t u = t + step;
                v = v < dom[u] ? sm[off[u] + v] : kBadPos;
                sm[e] = (uint16_t)v;
            }
        }
        __syncthreads();
    }
    const uint32_t m0 = dom[0];
    for (uint32_t p = threadIdx.x; p < m0; p += T) out_maps[(size_t)g * stride_out + p] = sm[p];
    if (threadIdx.x == 0) {
        out_msize[g] = (uint16_t)(m0 | (flag ? kFlagSymbol : 0));
        if (fa.result) write_result(fa, sm[0], flag != 0);
    }
}

// Down-sweep: the value at the start of group g (bv_up[g], or position 0 at
// the top) is pushed through the group's member maps; bv_l[i] receives the
// value at the start of member i.
__global__ void k_down(const uint16_t *__restrict__ maps_l, uint32_t n_l, uint32_t stride,
                       uint32_t G, const uint16_t *__restrict__ bv_up, uint32_t n_up,
                       uint16_t *__restrict__ bv_l) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_up) return;
    uint32_t v = bv_up ? bv_up[g] : 0u;
    const uint32_t first = g * G;
    const uint32_t cnt = min(G, n_l - first);
    for (uint32_t t = 0; t < cnt; ++t) {
        bv_l[first + t] = (uint16_t)v;
        if (!(v & kTerm)) v = (v < stride) ? maps_l[(size_t)(first + t) * stride + v] : kBadPos;
    }
}

// Level-0 boundary values -> states in the caller's numbering.
__global__ void k_bound_states(DevDFA d, const uint8_t *__restrict__ in, uint64_t chunk,
                               uint32_t nch, uint32_t start, uint32_t mode,
                               const uint16_t *__restrict__ bv0, const uint32_t *__restrict__ first,
                               const uint16_t *__restrict__ members,
                               const uint32_t *__restrict__ cset, uint32_t r,
                               uint32_t *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nch) return;
    const uint32_t v = bv0[i];
    uint32_t s;
    if (v & kTerm) {
        s = v & 0x7FFFu;
    } else if (i == 0) {
        s = start;
    } else if (mode == 2) {
        s = (v < first[i + 1] - first[i]) ? members[first[i] + v] : 0xFFFFFFFFu;
    } else if (mode == 3) {
        const uint32_t k = (uint32_t)min<uint64_t>(r, (uint64_t)i * chunk);
        const uint32_t lo = d.mset_off[d.moff[k] + cset[i]];
        const uint32_t hi = d.mset_off[d.moff[k] + cset[i] + 1];
        s = (v < hi - lo) ? d.mset_st[d.mst[k] + lo + v] : 0xFFFFFFFFu;
    } else {
        const uint32_t e = d.lut[in[(uint64_t)i * chunk - 1]];
        if (e == kLutInvalid) {
            s = 0xFFFFFFFFu;
        } else {
            const uint32_t cls = e >> 24;
            const uint32_t o0 = d.set_off[mode][cls];
            s = (v < d.set_off[mode][cls + 1] - o0) ? d.set_st[mode][o0 + v] : 0xFFFFFFFFu;
        }
    }
    out[i] = s;
}

__global__ void k_finalize(DevDFA d, const uint16_t *__restrict__ top_map,
                           const uint16_t *__restrict__ top_msize, uint32_t nch,
                           uint32_t *__restrict__ result, uint32_t *__restrict__ boundaries,
                           const uint32_t *__restrict__ bad, uint32_t nbad) {
    uint32_t any = 0;
    for (uint32_t b = threadIdx.x; b < nbad; b += blockDim.x) any |= bad[b];
    const bool symbol = __any(any != 0) || (top_msize[0] & kFlagSymbol) != 0;
    if (threadIdx.x != 0) return;
    write_result(FinalArgs{d.accept_bits, d.nq, nch, result, boundaries, nullptr, 0u}, top_map[0],
                 symbol);
}

__global__ void k_empty(DevDFA d, uint32_t start, uint32_t *__restrict__ result,
                        uint32_t *__restrict__ boundaries) {
    if (threadIdx.x != 0) return;
    result[0] = start;
    result[1] = (d.accept_bits[start >> 5] >> (start & 31)) & 1u;
    result[2] = 0;
    result[3] = 0;
    if (boundaries) boundaries[0] = start;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Let kernel f use dynamic LDS up to `lds` bytes minus its static LDS.  Asks
// only when the current limit is lower, and leaves no error pending on the
// thread (the launch paths check hipGetLastError after their launches).
int allow_dynamic_lds(const void *f, int lds) {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, f) != hipSuccess) {
        (void)hipGetLastError();
        return DFA_E_DEVICE;
    }
    const int need = lds - (int)fa.sharedSizeBytes;
    if (need <= fa.maxDynamicSharedSizeBytes) return DFA_OK;
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, need) != hipSuccess) {
        (void)hipGetLastError();
        return DFA_E_DEVICE;
    }
    return DFA_OK;
}

namespace {
struct DevProps {
    int lds = 0;
    int cus = 0;
    bool ok = false;
};
DevProps &props() {
    static std::mutex mu;
    static DevProps cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        static DevProps none;
        return none;
    }
    DevProps &p = cache[dev];
    std::lock_guard<std::mutex> lk(mu);
    if (!p.ok) {
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) {
            p.lds = (int)pr.maxSharedMemoryPerMultiProcessor;
            if (p.lds <= 0) p.lds = (int)pr.sharedMemPerBlock;
            if ((int)pr.sharedMemPerBlock < p.lds) {
                // dynamic LDS beyond the default per-block limit needs opting in
                if (allow_dynamic_lds(reinterpret_cast<const void *>(&k_match), p.lds) != DFA_OK)
                    p.lds = (int)pr.sharedMemPerBlock;
                (void)allow_dynamic_lds(reinterpret_cast<const void *>(&k_compose), p.lds);
                (void)allow_dynamic_lds(reinterpret_cast<const void *>(&k_compose_tree), p.lds);
                (void)set_match2_lds_limit(p.lds);
            }
            p.cus = pr.multiProcessorCount;
            p.ok = true;
        }
    }
    return p;
}
}  // namespace

size_t tree_lds_bytes(uint32_t G, uint32_t stride) {
    return 4u * ((size_t)G + 1) + 2u * (((size_t)G + 1) & ~(size_t)1) + 2u * (size_t)G * stride + 16u;
}

int device_lds_bytes() { return props().lds; }
int device_cu_count() { return props().cus; }

int plan_match(const dfa *d, uint64_t n, uint64_t chunk_req, uint32_t lookahead, MatchPlan *p,
               uint32_t flags, uint64_t before) {
    *p = MatchPlan();
    p->n = n;
    // r >= 2 needs the packed matcher (bitmaps); without a packed layout the
    // one-symbol sets are used, which give the same result.
    if (lookahead >= 2 && d->dev.layout == 0) lookahead = 1;
    // a block map takes precomputed sets only: a longer lookahead is lowered
    // to them (the set of fewer symbols contains the set of more, Section 4.3)
    if ((flags & kPlanBlock) && lookahead >= 2 && lookahead > d->dev.r0)
        lookahead = d->dev.r0 >= 2 ? d->dev.r0 : 1;
    if (lookahead > 64) return fail(DFA_E_INVAL, "lookahead must be at most 64 symbols");
    p->r = lookahead;
    p->lookahead = lookahead <= 1 ? lookahead : (lookahead <= d->dev.r0 ? 3u : 2u);
    p->bitmap_words = (d->dev.nq + 31) / 32;
    // sets with r >= 2 are subsets of the one-symbol sets (Lemma, Section 4.3),
    // and of the precomputed set of their last r' <= r0 symbols
    uint32_t setmax = std::max<uint32_t>(d->setmax_host[p->lookahead == 0 ? 0 : 1], 1u);
    if (p->lookahead >= 2) {
        const uint32_t k = std::min(p->r, d->dev.r0);
        if (k >= 1 && d->mset_max[k] > 0) setmax = std::max<uint32_t>(d->mset_max[k], 1u);
    }
    p->stride = (setmax + 7u) & ~7u;
    const int lds = device_lds_bytes();
    const int cus = std::max(device_cu_count(), 1);
    const uint32_t footprint = d->dev.table_bytes + 1024u;
    const uint32_t wg_per_cu = std::max<uint32_t>(1u, std::min<uint32_t>(8u, (uint32_t)lds / footprint));
    p->waves_per_block = std::min<uint32_t>(16u, std::max<uint32_t>(4u, (32u + wg_per_cu - 1) / wg_per_cu));
    if (n == 0) return DFA_OK;
    uint64_t chunk = chunk_req;
    if (chunk == 0) {
        const uint64_t conc = (uint64_t)cus * std::min<uint32_t>(32u, wg_per_cu * p->waves_per_block);
        const uint64_t target = 4 * conc;
        chunk = (n + target - 1) / target;
        chunk = (chunk + 63) / 64 * 64;
        chunk = std::max<uint64_t>(chunk, 256);
    }
    const char *force = std::getenv("DFA_KERNEL");
    // Packed pairs pay a translation pass and per-lane code loads; they win
    // when one chunk per wavefront would leave many lanes idle (sets far from
    // a multiple of 64).  Small inputs are launch-bound; the one-chunk-per-wave
    // path needs fewer launches.  DFA_KERNEL=1 / =2 force either kernel.
    const bool idle_lanes = p->lookahead == 0 ? false : d->wave_util < 0.85;
    p->packed = d->dev.layout != 0 &&
                (p->lookahead >= 2 || (flags & kPlanBlock) ||
                 (!(force && force[0] == '1') &&
                  ((n >= (4u << 20) && idle_lanes) || (force && force[0] == '2'))));
    // two-symbol steps halve the lookups; they need whole 32-byte chunk
    // multiples (16-byte blocks of pair codes) and per-byte codes for the
    // window pass.  DFA_PAIRS=0 keeps one symbol per step.
    const char *fpairs = std::getenv("DFA_PAIRS");
    p->pairs = p->packed && d->dev.pairs && p->lookahead != 2 && !(flags & DFA_MATCH_SINGLE_STEP) &&
               !(fpairs && fpairs[0] == '0') && (chunk_req == 0 || chunk_req % 32 == 0);
    if (p->packed) {
        // two pairs per lane when the start sets are tiny (many chunks per
        // tile: shorter tiles spread the chains over more wavefronts), four
        // otherwise (more independent walks per wavefront);
        // DFA_SLOTS=2 / =4 forces either
        const double mean_set = std::max(1.0, p->lookahead == 0 ? (double)d->setmax_host[0]
                                              : p->lookahead == 1 ? d->info.mean_iset
                                              : d->mset_mean[std::min(p->r, d->dev.r0)]);
        const char *fs = std::getenv("DFA_SLOTS");
        p->slots = fs && fs[0] == '2' ? 2u : fs && fs[0] == '4' ? 4u : (mean_set < 8.0 ? 2u : 4u);
        // workgroups per CU by LDS: the staged table plus, for merged rounds,
        // the round kernel's grouping tables at their largest (16 waves), so
        // that every workgroup of the persistent grid is resident
        const uint32_t staged = p->pairs ? d->dev.stab2_bytes : d->dev.stab_bytes;
        const uint32_t with_rounds = DFA_MATCH_ROUNDS_OF(flags) > 1
                                         ? staged + (uint32_t)round_lds_bytes(1024u) : staged;
        const uint32_t per_cu = std::max<uint32_t>(
            1u, std::min<uint32_t>(8u, (uint32_t)lds / std::max<uint32_t>(with_rounds, 1024u)));
        // 32 wavefronts per CU: blocks of up to 16 waves when few tables fit
        p->threads2 = 64u * std::min<uint32_t>(16u, std::max<uint32_t>(4u, (32u + per_cu - 1) / per_cu));
        p->blocks2 = (uint32_t)cus * per_cu;
        p->code_bytes = d->dev.layout == 1 ? 1u : 2u;
        // translation grid: 8 blocks per CU; 4 with the 33 KB pair-code table
        // of direct tables (each block stages it)
        const uint32_t tpc = p->pairs && d->dev.pcode2 ? 4u : 8u;
        p->tblocks = (uint32_t)std::min<uint64_t>((n + 4095) / 4096, (uint64_t)cus * tpc);
        if (chunk_req == 0) {
            // about six wave-tiles of pairs per resident wavefront
            const double mean = std::max(1.0, p->lookahead == 0 ? (double)d->setmax_host[0]
                                              : p->lookahead == 1 ? d->info.mean_iset
                                              : d->mset_mean[std::min(p->r, d->dev.r0)]);
            const double tiles = 6.0 * p->blocks2 * (p->threads2 / 64.0);
            const double nch_target = tiles * match2_tile_pairs(p->slots) / mean;
            chunk = (uint64_t)((double)n / std::max(1.0, nch_target));
            chunk = (chunk + 63) / 64 * 64;
            chunk = std::max<uint64_t>(chunk, 256);
        }
    }
    p->chunk = chunk;
    // a chunk whose lookahead reaches back fewer than r bytes (chunk 1 when
    // chunks are shorter than r; a block map's chunk 0 with fewer bytes
    // before it) starts from the set of that many symbols, which can be
    // larger than the r-symbol sets: size maps and tiles for the shortest
    // lookahead any chunk has
    if (p->lookahead >= 2) {
        const uint64_t lead = before ? before : chunk;
        const uint32_t kmin = (uint32_t)std::min<uint64_t>(std::min(p->r, d->dev.r0), lead);
        if (kmin >= 1 && d->mset_max[kmin] > setmax) {
            setmax = d->mset_max[kmin];
            p->stride = (setmax + 7u) & ~7u;
        }
    }
    const uint64_t nch = (n + chunk - 1) / chunk;
    if (nch > 0xFFFFFFFFull) return fail(DFA_E_TOOBIG, "too many chunks; raise chunk_len");
    p->nch = (uint32_t)nch;
    p->early_exit = p->packed && (flags & DFA_MATCH_EARLY_EXIT) && d->dev.nabs > 0;
    // chunk-interleaved codes: the packed matcher's chunks are whole blocks
    // of 64 consecutive chunks' code streams; the window pass reads codes
    // across chunk ends, so it keeps the linear stream
    // (one chunk per lane over a direct table's raw input keeps the input's
    // own order: each lane reads its chunk)
    const bool raw_lanes = (flags & DFA_MATCH_CHUNK_LANES) && !(flags & DFA_MATCH_INTERLEAVE) &&
                           d->dev.direct && !p->pairs;
    if (p->packed && (flags & (DFA_MATCH_INTERLEAVE | DFA_MATCH_CHUNK_LANES)) && !raw_lanes &&
        chunk % 32 == 0) {
        const uint64_t bytes_per_chunk = p->pairs ? chunk / 2 : chunk * p->code_bytes;
        p->ilv_nblk = (uint32_t)(bytes_per_chunk / 16);
    }
    // one chunk per lane (merged walks): interleaved codes and precomputed
    // sets; a lane walks every start state over the prefix, so sets are
    // bounded (128) to keep that serial part short
    {
        uint32_t set_bound = std::max<uint32_t>(d->setmax_host[p->lookahead == 0 ? 0 : 1], 1u);
        if (p->lookahead == 3) set_bound = d->mset_max[std::min(p->r, d->dev.r0)];
        p->chunk_lanes = (flags & DFA_MATCH_CHUNK_LANES) && (p->ilv_nblk || raw_lanes) &&
                         !p->early_exit && p->lookahead != 2 && chunk % 32 == 0 &&
                         set_bound <= 128;
    }
    // merged walks: two rounds unless asked otherwise; the last round must
    // start inside a chunk
    {
        const uint32_t req = DFA_MATCH_ROUNDS_OF(flags);
        uint32_t rounds = std::min<uint32_t>(req ? req : 1u, kMaxRounds);
        if (!p->packed || p->early_exit || chunk % 32 != 0 || p->chunk_lanes)
            rounds = 1;
        // the round kernel's grouping tables must fit beside the staged table
        const uint64_t staged = p->packed ? (p->pairs ? d->dev.stab2_bytes : d->dev.stab_bytes) : 0u;
        if (rounds > 1 && staged + round_lds_bytes(p->threads2) > (uint64_t)lds) rounds = 1;
        while (rounds > 1 && ((uint64_t)kRound1Bytes << (2 * (rounds - 2))) >= chunk) --rounds;
        p->rounds = rounds;
    }
    // merged walks over interleaved codes: four pairs per lane whatever the
    // set size (the later rounds' short chains need more walks per wavefront
    // in flight); DFA_SLOTS still forces either
    {
        const char *fs = std::getenv("DFA_SLOTS");
        if (p->packed && p->rounds > 1 && p->ilv_nblk && !(fs && (fs[0] == '2' || fs[0] == '4')))
            p->slots = 4;
    }
    // compose fan-in: G maps of `stride` entries staged in LDS for the tree
    // composition
    const uint64_t stage = std::min<uint64_t>(96u * 1024u, (uint64_t)lds - 1024u);
    p->group = (uint32_t)std::max<uint64_t>(2, std::min<uint64_t>(1024, stage / (2ull * p->stride + 8)));
    // The first level takes a smaller fan-in when that still gives every CU
    // a group without adding a level (131072 chunks: 256 groups of 512, then
    // one group of 256; a smaller top group shortens the one-workgroup level
    // more than the larger first groups lengthen theirs).
    auto count_levels = [&](uint64_t g0) {
        uint32_t lv = 0;
        for (uint64_t c = nch; c > 1; c = (c + (lv == 0 ? g0 : p->group) - 1) / (lv == 0 ? g0 : p->group))
            ++lv;
        return lv;
    };
    uint64_t g0 = p->group;
    const uint32_t lv_max = count_levels(g0);
    while (g0 > 64 && (nch + g0 - 1) / g0 < (uint64_t)cus && count_levels(g0 / 2) == lv_max)
        g0 /= 2;
    uint64_t cnt = nch, moff = 0, soff = 0;
    uint32_t L = 0;
    p->level_count[0] = (uint32_t)cnt;
    p->level_off[0] = 0;
    p->msize_off[0] = 0;
    moff += cnt * p->stride;
    soff += cnt;
    while (cnt > 1) {
        if (L + 1 >= kMaxLevels) return fail(DFA_E_TOOBIG, "too many compose levels");
        p->group_l[L] = (uint32_t)(L == 0 ? g0 : p->group);
        cnt = (cnt + p->group_l[L] - 1) / p->group_l[L];
        ++L;
        moff = (moff + 7u) & ~7ull;   // levels start on 16-byte boundaries
        p->level_count[L] = (uint32_t)cnt;
        p->level_off[L] = moff;
        p->msize_off[L] = soff;
        moff += cnt * p->stride;
        soff += cnt;
    }
    p->levels = L;
    p->map_entries = moff;
    p->msize_entries = soff;
    p->blocks = (uint32_t)std::min<uint64_t>((nch + p->waves_per_block - 1) / p->waves_per_block,
                                             0x7FFFFFFFull);
    p->max_tiles = (nch * (uint64_t)setmax + match2_tile_pairs(p->slots) - 1) /
                       match2_tile_pairs(p->slots) + 1;
    if (p->packed && nch * (uint64_t)setmax >= 0xFFFFFFFFull)
        return fail(DFA_E_TOOBIG, "too many (chunk, state) pairs; raise chunk_len");
    // merged walks number walks and list places below 2^30 (their outcomes
    // carry two flag bits above); beyond that a single round runs
    if (p->rounds > 1 && (uint64_t)p->max_tiles * match2_tile_pairs(p->slots) +
                                 (uint64_t)p->nch * kTailSlots >= (1ull << 30))
        p->rounds = 1;
    // first merged round chunk-major (one wavefront per chunk, its codes
    // loaded once, its walks grouped by end state alone) over interleaved
    // one-symbol codes, when start sets average at least 128 states (a
    // wavefront's 320 walks then mostly busy) and never exceed 320;
    // DFA_ROUND1=0 / =1 turns it off / on wherever it can run
    {
        const char *f1 = std::getenv("DFA_ROUND1");
        const double mean_set = p->lookahead == 0 ? (double)d->setmax_host[0]
                                : p->lookahead == 1 ? d->info.mean_iset
                                                    : d->mset_mean[std::min(p->r, d->dev.r0)];
        const bool can = p->packed && p->rounds > 1 && p->ilv_nblk && !p->pairs && p->stride <= 320 &&
                         (d->dev.layout == 1 || d->dev.layout == 2) && !d->dev.direct;
        p->round1c = can && (f1 && (f1[0] == '0' || f1[0] == '1') ? f1[0] == '1' : mean_set >= 128.0);
    }
    // merged walks over interleaved one-symbol codes: the last round takes
    // one chunk per lane and reads the raw input (bytes to codes through a
    // table in LDS), so only the first tail_t0 bytes of each chunk are
    // translated.  Needs a 16-byte aligned input and room for the 32 KiB byte
    // table; DFA_TAIL=0 keeps the wave-tile last round.
    {
        const char *ft = std::getenv("DFA_TAIL");
        const uint64_t tail_lds = (uint64_t)d->dev.stab_bytes + tail_lut_bytes() + round_lds_extra();
        p->tail = p->packed && p->rounds > 1 && p->ilv_nblk && !p->pairs && chunk < (1ull << 31) &&
                  !(flags & kPlanUnaligned) && !(ft && ft[0] == '0') && tail_lds <= (uint64_t)lds;
        if (p->tail) {
            p->tail_t0 = kRound1Bytes << (2 * (p->rounds - 2));
            p->ilv_nblk = p->tail_t0 * p->code_bytes / 16;
            // workgroups of whole wavefronts, sized so that every CU holds as
            // many as its LDS allows; each adds one wavefront for the
            // overflow list
            const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(8, (uint64_t)lds / tail_lds));
            // two chunks per lane when one per lane would not fit the chip at
            // once: a lane's steps form one dependent chain per chunk, so the
            // second chunk's steps fill the first's waits (DFA_TAIL_K=1 or 2
            // sets it)
            const char *fk = std::getenv("DFA_TAIL_K");
            const uint64_t once = (uint64_t)cus * per_cu * 960;
            p->tail_k = fk && (fk[0] == '1' || fk[0] == '2') ? (uint32_t)(fk[0] - '0')
                                                              : (nch > once ? 2u : 1u);
            const uint64_t lanes = (nch + p->tail_k - 1) / p->tail_k;
            const uint64_t want = (lanes + (uint64_t)cus * per_cu - 1) / ((uint64_t)cus * per_cu);
            p->tail_threads = (uint32_t)std::min<uint64_t>(960, std::max<uint64_t>(64, (want + 63) / 64 * 64));
            p->tail_blocks = (uint32_t)std::min<uint64_t>((lanes + p->tail_threads - 1) / p->tail_threads,
                                                          0x7FFFFFFFull);
        }
    }
    return DFA_OK;
}

int launch_match(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                 uint16_t *maps, uint16_t *msize, uint16_t *bvals, uint32_t *d_result,
                 uint32_t *d_boundaries, hipStream_t s, hipEvent_t ev_after_match) {
    if (p.n == 0) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, d->dev, start, d_result, d_boundaries);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && ev_after_match) e = hipEventRecord(ev_after_match, s);
        return e == hipSuccess ? DFA_OK : hip_fail(e, "k_empty launch");
    }
    if (p.packed) return fail(DFA_E_INVAL, "launch_match: plan is for the packed matcher");
    MatchArgs a;
    a.d = d->dev;
    a.in = d_in;
    a.n = p.n;
    a.chunk = p.chunk;
    a.nch = p.nch;
    a.start = start;
    a.mode = p.lookahead;
    a.stride = p.stride;
    a.maps = maps + p.level_off[0];
    a.msize = msize + p.msize_off[0];
    const size_t lds_match = d->dev.table_bytes + 1024u;
    hipLaunchKernelGGL(k_match, dim3(p.blocks), dim3(p.waves_per_block * kWave), lds_match, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_match launch");
    if (ev_after_match) {
        e = hipEventRecord(ev_after_match, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    return launch_combine(d, d_in, start, p, maps, msize, bvals, nullptr, d_result, d_boundaries,
                          s);
}

int launch_combine(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                   uint16_t *maps, uint16_t *msize, uint16_t *bvals, const PackedBufs *pb,
                   uint32_t *d_result, uint32_t *d_boundaries, hipStream_t s) {
    hipError_t e;
    // the packed path's translation flags (one word per translation block)
    // reach the result through the top level
    const uint32_t nbad = pb ? p.tblocks : 0u;
    for (uint32_t l = 0; l < p.levels; ++l) {
        // level 0 of the packed matcher is pair-indexed; every other level
        // strided.  The last level (one group) also writes the result.
        const uint32_t G = p.group_l[l];
        const uint32_t *first = (l == 0 && pb) ? pb->first : nullptr;
        const bool top = l + 1 == p.levels;
        FinalArgs fa{d->dev.accept_bits, d->dev.nq, p.nch, top ? d_result : nullptr,
                     top ? d_boundaries : nullptr, pb ? pb->block_bad : nullptr, nbad};
        hipLaunchKernelGGL(k_compose_tree, dim3(p.level_count[l + 1]), dim3(1024),
                           tree_lds_bytes(G, p.stride), s, maps + p.level_off[l], first,
                           msize + p.msize_off[l], p.level_count[l], p.stride, G, G * p.stride,
                           maps + p.level_off[l + 1], p.stride, msize + p.msize_off[l + 1], fa);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "k_compose_tree launch");
    }
    if (p.levels == 0) {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, d->dev, maps, msize, p.nch,
                           d_result, d_boundaries, pb ? pb->block_bad : nullptr, nbad);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "k_finalize launch");
    }
    if (d_boundaries) {
        // bvals reuses the msize offsets (one value per map at every level)
        for (int l = (int)p.levels; l >= 1; --l) {
            if (l == 1 && pb) {
                const uint16_t *up = (p.levels == 1) ? nullptr : bvals + p.msize_off[1];
                int rc = launch_down0(p, maps, pb->first, up, bvals, s);
                if (rc) return rc;
                continue;
            }
            const uint32_t n_up = p.level_count[l];
            const uint16_t *up = (l == (int)p.levels) ? nullptr : bvals + p.msize_off[l];
            hipLaunchKernelGGL(k_down, dim3((n_up + 255) / 256), dim3(256), 0, s,
                               maps + p.level_off[l - 1], p.level_count[l - 1], p.stride,
                               p.group_l[l - 1], up, n_up, bvals + p.msize_off[l - 1]);
        }
        if (p.levels == 0) {
            hipLaunchKernelGGL(k_down, dim3(1), dim3(256), 0, s, maps, 1u, p.stride, 1u,
                               (const uint16_t *)nullptr, 1u, bvals);
        }
        hipLaunchKernelGGL(k_bound_states, dim3((p.nch + 255) / 256), dim3(256), 0, s, d->dev,
                           d_in, p.chunk, p.nch, start, p.lookahead, bvals,
                           pb ? pb->first : nullptr, pb ? pb->members : nullptr,
                           pb ? pb->cset : nullptr, p.r, d_boundaries);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "boundary kernels launch");
    }
    return DFA_OK;
}

}  // namespace dfaspec
