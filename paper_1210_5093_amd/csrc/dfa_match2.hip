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
// A direct layout-1 table (alphabets of bytes below 128) has byte-indexed
// rows, LDS address = R * s + 2 * byte; the matcher (L = 3) then reads the
// raw input and forms the codes itself, and the translation pass shrinks to a
// validation pass (k_translate without output) that only flags bytes outside
// Sigma.
// The table sits at LDS address 0 (the kernel has no static LDS), so stored
// table entries are LDS addresses themselves.
//
// Kernels: k_translate (bytes -> codes, invalid-byte flags), k_chunkinfo
// (lookahead class and |I| per chunk), k_scan (exclusive prefix of set
// sizes = first pair of each chunk), k_match2 (persistent tiles of pairs).
// The sparse maps it writes have the same form as the one-chunk-per-wave
// matcher's, so the combination kernels are shared.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "dfa_pairs.h"

namespace dfaspec {

// ---------------------------------------------------------------------------
// Translation: code[i] = code_lut[in[i]]; per-block flag if a byte is outside
// Sigma.  WRITE = false only validates (direct tables).  The output is
// 16-byte aligned.
// ---------------------------------------------------------------------------
constexpr int kTrU = 4;

// The grid walk shared by the translation kernels: convert(tag, w, first)
// handles the 16 input bytes at `first` (tag: std::true_type when all lie
// before n).  Whole rounds of an aligned input load kTrU blocks per thread
// before converting any (block u of a round is u * threads + thread, so every
// load instruction is coalesced): with one 16-byte load in flight per lane a
// pass is bound by memory latency well below HBM bandwidth.  The last partial
// round and misaligned inputs go one block at a time.
template <typename Conv>
__device__ __forceinline__ void translate_grid(const uint8_t *__restrict__ in, uint64_t n,
                                               Conv &convert) {
    const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t base = 0;
    if ((reinterpret_cast<uintptr_t>(in) & 15u) == 0) {
        for (; base + T * 16 * kTrU <= n; base += T * 16 * kTrU) {
            uint4 v[kTrU];
#pragma unroll
            for (int u = 0; u < kTrU; ++u)
                v[u] = *reinterpret_cast<const uint4 *>(in + base + ((uint64_t)u * T + tid) * 16);
#pragma unroll
            for (int u = 0; u < kTrU; ++u) {
                const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
                convert(std::true_type{}, w, base + ((uint64_t)u * T + tid) * 16);
            }
        }
    }
    for (uint64_t first = base + tid * 16; first < n; first += T * 16) {
        uint32_t w[4];
        load16(in, first, n, w);
        if (first + 16 <= n) convert(std::true_type{}, w, first);
        else convert(std::false_type{}, w, first);
    }
}

// Bytes 0 of four words packed into one (v_perm_b32).
__device__ __forceinline__ uint32_t pack_low_bytes(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
    return __builtin_amdgcn_perm(c1, c0, 0x0C0C0400u) | __builtin_amdgcn_perm(c3, c2, 0x04000C0Cu);
}

template <typename CodeT, bool WRITE = true>
__global__ __launch_bounds__(256) void k_translate(const uint8_t *__restrict__ in, uint64_t n,
                                                   const uint16_t *__restrict__ code_lut,
                                                   CodeT *__restrict__ out,
                                                   uint32_t *__restrict__ block_bad) {
    // one-byte codes (< 256) are staged with bytes outside Sigma as 0xFF00:
    // the low byte (the code written) is 0 and an OR of the entries flags them
    constexpr bool kNarrow = sizeof(CodeT) == 1;
    __shared__ uint16_t lut[256];
    __shared__ uint32_t bad_any;
    {
        const uint16_t v = code_lut[threadIdx.x];
        lut[threadIdx.x] = kNarrow && v == kCodeInvalid ? (uint16_t)0xFF00u : v;
    }
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    uint32_t bad = 0;
    // WHOLE: all 16 bytes lie before n (no per-byte bounds)
    auto convert = [&](auto whole_tag, const uint32_t (&w)[4], uint64_t first) {
        constexpr bool WHOLE = decltype(whole_tag)::value;
        uint32_t c[16];
        if constexpr (WHOLE) {
            uint32_t acc = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = lut[(w[k >> 2] >> (8 * (k & 3))) & 0xFFu];
                if constexpr (kNarrow) {
                    acc |= v;
                    c[k] = v;
                } else {
                    const bool inv = v == kCodeInvalid;
                    bad |= inv ? 1u : 0u;
                    c[k] = inv ? 0u : v;
                }
            }
            if constexpr (kNarrow) bad |= acc >> 8;
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = lut[(w[k >> 2] >> (8 * (k & 3))) & 0xFFu];
                const bool inside = first + k < n;
                const bool inv = kNarrow ? (v >> 8) != 0 : v == kCodeInvalid;
                bad |= (inside && inv) ? 1u : 0u;
                c[k] = (inv || !inside) ? 0u : v;
            }
        }
        if constexpr (!WRITE) {
        } else if constexpr (kNarrow) {
            uint4 o;
            o.x = pack_low_bytes(c[0], c[1], c[2], c[3]);
            o.y = pack_low_bytes(c[4], c[5], c[6], c[7]);
            o.z = pack_low_bytes(c[8], c[9], c[10], c[11]);
            o.w = pack_low_bytes(c[12], c[13], c[14], c[15]);
            *reinterpret_cast<uint4 *>(out + first) = o;
        } else {
            uint4 o[2];
            uint32_t *ow = reinterpret_cast<uint32_t *>(o);
#pragma unroll
            for (int q = 0; q < 8; ++q) ow[q] = __builtin_amdgcn_perm(c[2 * q + 1], c[2 * q], 0x05040100u);
            *reinterpret_cast<uint4 *>(out + first) = o[0];
            *reinterpret_cast<uint4 *>(out + first + 8) = o[1];
        }
    };
    translate_grid(in, n, convert);
    if (bad) atomicOr(&bad_any, 1u);
    __syncthreads();
    if (threadIdx.x == 0) block_bad[blockIdx.x] = bad_any;
}


// Two-symbol translation: code i = the pair code of bytes 2i and 2i + 1 (the
// class alone when 2i + 1 = n); per-block flag if a byte is outside Sigma.
// pcode: byte -> class (256 bytes), then the codes of the K x (K + 1) pairs.
__global__ __launch_bounds__(256) void k_translate_pairs(const uint8_t *__restrict__ in, uint64_t n,
                                                         const uint8_t *__restrict__ pcode,
                                                         uint32_t K, uint8_t *__restrict__ out,
                                                         uint32_t *__restrict__ block_bad) {
    // pc covers every index c1 * (K + 1) + c2 with c1, c2 <= 255, so that a
    // class 0xFF (byte outside Sigma) reads a staged value: a pair code, or 0
    // past the K x (K + 1) codes; such blocks are flagged and their codes
    // only need to stay valid table offsets
    constexpr uint32_t kPc = 256u * 64u + 256u;
    __shared__ uint8_t cls[256];
    __shared__ __align__(16) uint8_t pc[kPc];
    __shared__ uint32_t bad_any;
    cls[threadIdx.x] = pcode[threadIdx.x];
    for (uint32_t i = threadIdx.x; i < kPc / 4; i += blockDim.x)
        reinterpret_cast<uint32_t *>(pc)[i] = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < K * (K + 1); i += blockDim.x) pc[i] = pcode[256 + i];
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    const uint32_t K1 = K + 1;
    uint32_t bad = 0;
    auto convert = [&](auto whole_tag, const uint32_t (&w)[4], uint64_t first) {
        constexpr bool WHOLE = decltype(whole_tag)::value;
        uint32_t c[8];
        if constexpr (WHOLE) {
            uint32_t acc = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t c1 = cls[(w[k >> 1] >> (16 * (k & 1))) & 0xFFu];
                const uint32_t c2 = cls[(w[k >> 1] >> (16 * (k & 1) + 8)) & 0xFFu];
                acc |= c1 | c2;
                c[k] = pc[__umul24(c1, K1) + c2];
            }
            bad |= (acc & 0x80u) ? 1u : 0u;   // classes are below 64; 0xFF marks a bad byte
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t b1 = (w[k >> 1] >> (16 * (k & 1))) & 0xFFu;
                const uint32_t b2 = (w[k >> 1] >> (16 * (k & 1) + 8)) & 0xFFu;
                const bool in1 = first + 2 * k < n, in2 = first + 2 * k + 1 < n;
                const uint32_t c1 = cls[b1];
                const uint32_t c2 = in2 ? (uint32_t)cls[b2] : K;
                const bool bad1 = in1 && c1 == 0xFFu, bad2 = in2 && c2 == 0xFFu;
                bad |= (bad1 || bad2) ? 1u : 0u;
                c[k] = (in1 && !bad1 && !bad2) ? (uint32_t)pc[c1 * K1 + c2] : 0u;
            }
        }
        *reinterpret_cast<uint2 *>(out + first / 2) =
            make_uint2(pack_low_bytes(c[0], c[1], c[2], c[3]), pack_low_bytes(c[4], c[5], c[6], c[7]));
    };
    translate_grid(in, n, convert);
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

// Multi-symbol reverse lookahead (Eq. 13).  The start set of chunk i >= 1 is
// the image of Q under the r' = min(r, p) bytes before it (p = i*C), minus the
// absorbing states; the true state at p lies in it, and so does the end state
// of every walk of chunk i-1 from its own start set.  Unlike the paper's
// precomputed I_{sigma_1..sigma_r} tables (|Sigma|^r of them), the image is
// computed for the actual lookahead string: the image of Q under its first
// byte is I_{sigma_1} (a precomputed class set), so every (chunk, state of
// I_{sigma_1}) "window pair" walks the remaining r'-1 bytes and sets its end
// state's bit in the chunk's bitmap.  A scan over the bitmaps' popcounts then
// lays out the start sets as sorted member lists.
//
// r <= r0: the start set of chunk i >= 1 is the precomputed I_{c_1..c_k} of
// its k = min(r, p) lookahead bytes (Eq. 13).
__global__ void k_chunkinfo_m(DevDFA d, const uint8_t *__restrict__ in, uint64_t chunk,
                              uint32_t nch, uint32_t r, uint16_t *__restrict__ msize,
                              uint32_t *__restrict__ cset) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nch) return;
    uint32_t m = 1, id = 0;
    if (i > 0) {
        const uint64_t p = (uint64_t)i * chunk;
        const uint32_t k = (uint32_t)min<uint64_t>(r, p);
        bool bad = false;
        id = class_string_id(d, in, p - k, k, &bad);
        m = bad ? 0u : mset_end(d, k, id) - mset_begin(d, k, id);
    }
    msize[i] = (uint16_t)m;
    cset[i] = id;
}

// r > r0: window pairs start from the precomputed set of the window's first
// k0 = min(r', r0) bytes; cset holds that set's id.  Clears the bitmaps.
__global__ void k_chunkinfo_w(DevDFA d, const uint8_t *__restrict__ in, uint64_t chunk,
                              uint32_t nch, uint32_t r, uint32_t W,
                              uint16_t *__restrict__ msize, uint32_t *__restrict__ cset,
                              uint32_t *__restrict__ bits) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nch) return;
    for (uint32_t k = 0; k < W; ++k) bits[(size_t)i * W + k] = 0;
    uint32_t m = 0, id = 0;
    if (i > 0) {
        const uint64_t p = (uint64_t)i * chunk;
        const uint32_t rr = (uint32_t)min<uint64_t>(r, p);
        const uint32_t k0 = min(rr, d.r0);
        bool bad = false;
        id = class_string_id(d, in, p - rr, k0, &bad);
        m = bad ? 0u : mset_end(d, k0, id) - mset_begin(d, k0, id);
    }
    msize[i] = (uint16_t)m;
    cset[i] = id;
}

// Exclusive scan of the set sizes in three phases: first[i] = sum_{k<i} m_k,
// first[nch] = number of pairs, tile_first[w] = chunk holding pair w * tile.
// Sizes come from msize (SRC 0) or from the popcounts of the start-set
// bitmaps (SRC 1: chunk 0 holds the start state; the sizes are also written to
// msize and the sorted member lists to members[first[i] ..]).  Phase 2 folds
// the translation flags into the flag bit of chunk 0's size, from where the
// compose levels carry it up.
constexpr uint32_t kScanThreads = 1024;
constexpr uint32_t kScanItems = 4;
constexpr uint32_t kScanBlock = kScanThreads * kScanItems;   // chunks per scan block

// Inclusive scan of one value per thread across the workgroup.
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

struct ScanSrc {
    uint16_t *msize;
    const uint32_t *bits;    // SRC 1
    uint32_t W;
    uint32_t nch;
    uint32_t tile;           // pairs per wave-tile
};

template <int SRC>
__device__ __forceinline__ uint32_t scan_size(const ScanSrc &q, uint64_t i) {
    if constexpr (SRC == 0) {
        return q.msize[i] & 0x7FFFu;
    } else {
        if (i == 0) return 1u;
        uint32_t m = 0;
        for (uint32_t k = 0; k < q.W; ++k) m += __popc(q.bits[i * q.W + k]);
        return m;
    }
}

template <int SRC>
__global__ __launch_bounds__(1024) void k_scan_sums(ScanSrc q, uint32_t *__restrict__ bsum) {
    __shared__ uint32_t part[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint32_t v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k)
        if (base + k < q.nch) v += scan_size<SRC>(q, base + k);
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
    if (t == 0 && bad_any && msize) msize[0] = (uint16_t)(msize[0] | kFlagSymbol);
}

template <int SRC>
__global__ __launch_bounds__(1024) void k_scan_apply(ScanSrc q, const uint32_t *__restrict__ boff,
                                                     uint32_t *__restrict__ first,
                                                     uint32_t *__restrict__ tile_first,
                                                     uint16_t *__restrict__ members,
                                                     uint32_t start) {
    __shared__ uint32_t part[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint32_t m[kScanItems], v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        m[k] = base + k < q.nch ? scan_size<SRC>(q, base + k) : 0u;
        v += m[k];
    }
    const uint32_t inc = block_inclusive_scan(v, part);
    uint32_t run = boff[blockIdx.x] + inc - v;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + k;
        if (i < q.nch) {
            first[i] = run;
            if (m[k]) {
                for (uint32_t w = (run + q.tile - 1) / q.tile; w <= (run + m[k] - 1) / q.tile; ++w)
                    tile_first[w] = (uint32_t)i;
            }
            if constexpr (SRC == 1) {
                if (i == 0) {
                    members[run] = (uint16_t)start;
                    q.msize[0] = (uint16_t)((q.msize[0] & kFlagSymbol) | 1u);
                } else {
                    uint32_t j = run;
                    for (uint32_t kk = 0; kk < q.W; ++kk) {
                        uint32_t w = q.bits[i * q.W + kk];
                        while (w) {
                            members[j++] = (uint16_t)(32u * kk + (uint32_t)__builtin_ctz(w));
                            w &= w - 1;
                        }
                    }
                    q.msize[i] = (uint16_t)m[k];
                }
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
    uint32_t mode;           // 0, 1, 2 (see MatchPlan::lookahead)
    uint32_t r;              // window passes: lookahead symbols
    const uint32_t *first;   // [nch + 1]
    const uint32_t *tile_first;
    const uint16_t *ccls;    // [nch] modes 0, 1: lookahead class
    const uint32_t *cset;    // [nch] modes 2, 3: precomputed set id
    const uint16_t *members; // mode 2: sorted start sets
    uint32_t *bits;          // window pass: start-set bitmaps
    uint32_t W;
    uint16_t *maps;          // level-0 maps, indexed by pair
    uint32_t exit_base;      // early exit: LDS byte offset of the absorbing bitmap (0 = off)
    uint32_t exit_shift;
    uint32_t c_lo, c_hi;     // this launch walks the pairs of chunks [c_lo, c_hi)
};

template <int L>
__device__ __forceinline__ void stage_table(const DevDFA &d, uint8_t *smem) {
    const uint4 *src = reinterpret_cast<const uint4 *>(d.stab);
    uint4 *dst = reinterpret_cast<uint4 *>(smem);
    for (uint32_t i = threadIdx.x; i < d.stab_bytes / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Window pass: pair P of chunk c starts at the (P - first[c])-th state of
// I_{sigma_1} and walks w[p - r' + 1, p); its end state joins chunk c's set.
template <int L, int S>
__global__ __launch_bounds__(1024, 8) void k_window2(Match2Args a) {
    constexpr uint32_t kTile = kWave2 * S;
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<L>(a.d, smem);
    using CodeT = typename std::conditional<L == 1, uint8_t, uint16_t>::type;
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t waves = blockDim.x / kWave2;
    const uint32_t wave_id = blockIdx.x * waves + threadIdx.x / kWave2;
    const uint32_t total = a.first[a.nch];
    const uint32_t ntiles = (total + kTile - 1) / kTile;
    const uint32_t R = L == 1 ? a.d.rowbytes : 2u;
    const CodeT *codes = reinterpret_cast<const CodeT *>(a.codes);
    for (uint32_t tile = wave_id; tile < ntiles; tile += gridDim.x * waves) {
        const uint32_t lo0 = a.tile_first[tile];
        const uint32_t hi0 = tile + 1 < ntiles ? a.tile_first[tile + 1] + 1 : a.nch;
        uint32_t st[S], ci[S], len[S];
        uint64_t beg[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const uint32_t P = tile * kTile + j * kWave2 + lane;
            const bool valid = P < total;
            const uint32_t c = valid ? owner_chunk(a.first, lo0, hi0, P) : 0u;
            uint32_t s = 0;
            const uint64_t p = (uint64_t)c * a.chunk;
            const uint32_t rr = (uint32_t)min<uint64_t>(a.r, p);
            const uint32_t k0 = min(rr, a.d.r0);
            if (valid)
                s = a.d.mset_st[a.d.mst[k0] + mset_begin(a.d, k0, a.cset[c]) + (P - a.first[c])];
            st[j] = R * s;
            ci[j] = valid ? c : 0xFFFFFFFFu;
            beg[j] = valid ? p - rr + k0 : 0;
            len[j] = valid ? rr - k0 : 0;
        }
        uint32_t maxlen = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) maxlen = max(maxlen, len[j]);
        for (uint32_t t = 0; t < maxlen; ++t) {
#pragma unroll
            for (int j = 0; j < S; ++j)
                if (t < len[j]) st[j] = lds_ld(st[j] + (uint32_t)codes[beg[j] + t]);
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            // walks of one chunk converge, and its pairs sit in adjacent lanes:
            // skip the atomic when the previous lane already set the same bit
            const uint32_t e = st[j] / R;
            const uint32_t prev_c = __shfl_up(ci[j], 1);
            const uint32_t prev_e = __shfl_up(e, 1);
            const bool dup = lane > 0 && prev_c == ci[j] && prev_e == e;
            if (ci[j] != 0xFFFFFFFFu && !dup && a.d.pos[1][e] != (uint16_t)(kTerm | e))
                atomicOr(&a.bits[(size_t)ci[j] * a.W + (e >> 5)], 1u << (e & 31));
        }
    }
}

// L: layout (3 = a direct layout-1 table walked over the raw input, 4 = the
// two-symbol table walked over pair codes);
// S: slots (pairs) per lane; EXIT: early exit at absorbing states.  The
// four-slot walk without exit is held to 64 VGPRs (8 waves per SIMD; a few
// values spill once per tile, outside the walk).
template <int L, int S, bool EXIT>
__global__ __launch_bounds__(1024, (S == 4 && !EXIT) ? 8 : 6) void k_match2(Match2Args a) {
    constexpr uint32_t kTile = kWave2 * S;
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<L>(a.d, smem);
    using CodeT = typename std::conditional<L != 2, uint8_t, uint16_t>::type;
    constexpr uint32_t kPer16 = 16 / sizeof(CodeT);   // codes per 16 bytes
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t waves = blockDim.x / kWave2;
    const uint32_t wave_id = blockIdx.x * waves + threadIdx.x / kWave2;
    const uint32_t total_waves = gridDim.x * waves;
    const uint32_t total = a.first[a.nch];
    const uint32_t ntiles = (total + kTile - 1) / kTile;
    // pairs of chunks [c_lo, c_hi): the tiles that overlap them
    const uint32_t p_lo = a.first[a.c_lo], p_hi = a.first[a.c_hi];
    const uint32_t t_lo = p_lo / kTile, t_hi = (p_hi + kTile - 1) / kTile;
    const uint32_t R = L != 2 ? a.d.rowbytes : 2u;
    const CodeT *codes = reinterpret_cast<const CodeT *>(a.codes);
    auto code_at = [&](uint64_t pos) -> uint32_t {
        return L == 3 ? 2u * (codes[pos] & 0x7Fu) : (uint32_t)codes[pos];
    };
    // L = 4 (two-symbol steps): one code per two input bytes, chunk lengths
    // are even (the host only picks it for multiples of 32)
    constexpr uint32_t kSym = L == 4 ? 2u : 1u;       // symbols per code
    // full chunks start on 16-byte boundaries iff the chunk length does
    const bool aligned_chunks = (a.chunk % (kPer16 * kSym)) == 0;

    for (uint32_t tile = t_lo + wave_id; tile < t_hi; tile += total_waves) {
        const uint32_t lo0 = a.tile_first[tile];
        const uint32_t hi0 = tile + 1 < ntiles ? a.tile_first[tile + 1] + 1 : a.nch;
        uint32_t st[S], ci[S], o16[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const uint32_t P = tile * kTile + j * kWave2 + lane;
            const bool valid = P >= p_lo && P < p_hi;
            const uint32_t c = valid ? owner_chunk(a.first, lo0, hi0, P) : 0u;
            uint32_t s = 0;
            if (valid) {
                if (c == 0) {
                    s = a.start;
                } else if (a.mode == 2) {
                    s = a.members[P];
                } else if (a.mode == 3) {
                    const uint32_t k = (uint32_t)min<uint64_t>(a.r, (uint64_t)c * a.chunk);
                    s = a.d.mset_st[a.d.mst[k] + mset_begin(a.d, k, a.cset[c]) + (P - a.first[c])];
                } else {
                    s = a.d.set_st[a.mode][a.d.set_off[a.mode][a.ccls[c]] + (P - a.first[c])];
                }
            }
            st[j] = R * s;
            ci[j] = valid ? c : 0xFFFFFFFFu;
            o16[j] = aligned_chunks ? (uint32_t)((uint64_t)c * a.chunk / (kPer16 * kSym)) : 0u;
        }
        if (aligned_chunks) {
            uint32_t live = 0;
#pragma unroll
            for (int j = 0; j < S; ++j) live |= (ci[j] != 0xFFFFFFFFu ? 1u : 0u) << j;
            // pairs past the end shadow chunk 0 from state 0 (loads stay in
            // bounds; their end states are discarded)
            auto len_of = [&](int j) -> uint32_t {
                const uint64_t c = ci[j] == 0xFFFFFFFFu ? 0u : ci[j];
                return (uint32_t)((min<uint64_t>(a.chunk, a.n - c * a.chunk) + kSym - 1) / kSym);
            };
            walk_var<L, S, EXIT>(reinterpret_cast<const uint4 *>(codes), o16, len_of, st,
                                  a.exit_base, a.exit_shift, live);
        } else {
            // general path: per-lane code loads, chunks of any length and alignment
            const uint64_t ncodes = (a.n + kSym - 1) / kSym;
            for (uint64_t t = 0; t < (a.chunk + kSym - 1) / kSym; ++t) {
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    if (ci[j] != 0xFFFFFFFFu) {
                        const uint64_t pos = (uint64_t)ci[j] * a.chunk / kSym + t;
                        if (pos < ncodes) st[j] = lds_ld(st[j] + code_at(pos));
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (ci[j] != 0xFFFFFFFFu) {
                const uint32_t e = st[j] / R;
                const uint32_t c = ci[j];
                const uint32_t P = tile * kTile + j * kWave2 + lane;
                uint16_t v;
                if (c + 1 == a.nch) {
                    v = (uint16_t)(kTerm | e);
                } else if (a.mode == 2) {
                    const uint16_t ab = a.d.pos[1][e];   // class-0 row: kTerm|e iff absorbing
                    v = ab == (uint16_t)(kTerm | e)
                            ? ab
                            : (uint16_t)member_rank(a.members, a.first[c + 1], a.first[c + 2], e);
                } else if (a.mode == 3) {
                    const uint16_t ab = a.d.pos[1][e];
                    const uint32_t k = (uint32_t)min<uint64_t>(a.r, (uint64_t)(c + 1) * a.chunk);
                    const uint32_t id = a.cset[c + 1];
                    v = ab == (uint16_t)(kTerm | e)
                            ? ab
                            : (uint16_t)member_rank(a.d.mset_st + a.d.mst[k], mset_begin(a.d, k, id),
                                                    mset_end(a.d, k, id), e);
                } else {
                    v = a.d.pos[a.mode][(size_t)a.ccls[c + 1] * a.d.nq + e];
                }
                a.maps[P] = v;
            }
        }
    }
}

// Translation flags of a segmented run -> the symbol flag of chunk 0's size
// (from where the composition carries it up).
__global__ void k_fold_bad(const uint32_t *__restrict__ block_bad, uint32_t nbad,
                           uint16_t *__restrict__ msize) {
    __shared__ uint32_t any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint32_t b = threadIdx.x; b < nbad; b += blockDim.x) bad |= block_bad[b];
    if (bad) atomicOr(&any, 1u);
    __syncthreads();
    if (threadIdx.x == 0 && any) msize[0] = (uint16_t)(msize[0] | kFlagSymbol);
}

// Down-sweep into pair-indexed level-0 maps: bv0[i] = value at chunk i's start.
__global__ void k_down0(const uint16_t *__restrict__ maps0, const uint32_t *__restrict__ first,
                        uint32_t nch, uint32_t G, const uint16_t *__restrict__ bv_up,
                        uint32_t n_up, uint16_t *__restrict__ bv0) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_up) return;
    uint32_t v = bv_up ? bv_up[g] : 0u;
    const uint32_t c0 = g * G;
    const uint32_t cnt = min(G, nch - c0);
    for (uint32_t t = 0; t < cnt; ++t) {
        const uint32_t c = c0 + t;
        bv0[c] = (uint16_t)v;
        if (!(v & kTerm)) v = (v < first[c + 1] - first[c]) ? maps0[first[c] + v] : kBadPos;
    }
}

// ---------------------------------------------------------------------------
namespace {
template <int SRC>
void launch_scan(const MatchPlan &p, const ScanSrc &q, const PackedBufs &b, uint16_t *flag_msize,
                 uint32_t start, hipStream_t s) {
    const uint32_t nsb = (p.nch + kScanBlock - 1) / kScanBlock;
    ScanSrc qq = q;
    qq.tile = kWave2 * p.slots;
    hipLaunchKernelGGL(k_scan_sums<SRC>, dim3(nsb), dim3(kScanThreads), 0, s, qq, b.bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, b.bsum, nsb, flag_msize,
                       p.nch, b.block_bad, flag_msize ? p.tblocks : 0u, b.first);
    hipLaunchKernelGGL(k_scan_apply<SRC>, dim3(nsb), dim3(kScanThreads), 0, s, qq, b.bsum, b.first,
                       b.tile_first, b.members, start);
}
}  // namespace

namespace {
const void *match2_kernel(uint32_t L, uint32_t slots, bool ex) {
    static const void *const tab[4][2][2] = {
        {{reinterpret_cast<const void *>(&k_match2<1, 2, false>),
          reinterpret_cast<const void *>(&k_match2<1, 2, true>)},
         {reinterpret_cast<const void *>(&k_match2<1, 4, false>),
          reinterpret_cast<const void *>(&k_match2<1, 4, true>)}},
        {{reinterpret_cast<const void *>(&k_match2<2, 2, false>),
          reinterpret_cast<const void *>(&k_match2<2, 2, true>)},
         {reinterpret_cast<const void *>(&k_match2<2, 4, false>),
          reinterpret_cast<const void *>(&k_match2<2, 4, true>)}},
        {{reinterpret_cast<const void *>(&k_match2<3, 2, false>),
          reinterpret_cast<const void *>(&k_match2<3, 2, true>)},
         {reinterpret_cast<const void *>(&k_match2<3, 4, false>),
          reinterpret_cast<const void *>(&k_match2<3, 4, true>)}},
        {{reinterpret_cast<const void *>(&k_match2<4, 2, false>),
          reinterpret_cast<const void *>(&k_match2<4, 2, true>)},
         {reinterpret_cast<const void *>(&k_match2<4, 4, false>),
          reinterpret_cast<const void *>(&k_match2<4, 4, true>)}}};
    return tab[L - 1][slots >= 4 ? 1 : 0][ex ? 1 : 0];
}
const void *window2_kernel(uint32_t L, uint32_t slots) {
    static const void *const tab[2][2] = {
        {reinterpret_cast<const void *>(&k_window2<1, 2>), reinterpret_cast<const void *>(&k_window2<1, 4>)},
        {reinterpret_cast<const void *>(&k_window2<2, 2>), reinterpret_cast<const void *>(&k_window2<2, 4>)}};
    return tab[L == 1 ? 0 : 1][slots >= 4 ? 1 : 0];
}
}  // namespace

int launch_match2(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                  const PackedBufs &b, uint16_t *maps, uint16_t *msize, hipStream_t s,
                  hipEvent_t ev_before_matcher) {
    // two-symbol steps (the plan checked the chunk length); else direct
    // tables: the matcher reads the (16-byte aligned) input itself
    const bool pairs = p.pairs && d->dev.pairs;
    const bool direct = !pairs && d->dev.direct && p.lookahead != 2 && p.segments <= 1 &&
                        (reinterpret_cast<uintptr_t>(d_in) & 15u) == 0;
    const uint32_t L = pairs ? 4u : direct ? 3u : d->dev.layout;
    if (pairs && (p.segments > 1 || p.chunk % 32 != 0 || p.lookahead == 2))
        return fail(DFA_E_INVAL, "two-symbol plan with segments, window pass or odd chunks");
    const uint32_t nseg = std::max<uint32_t>(1u, std::min(p.segments, kMaxSegments));
    uint32_t cb[kMaxSegments + 1];
    for (uint32_t k = 0; k <= nseg; ++k) cb[k] = (uint32_t)((uint64_t)p.nch * k / nseg);
    hipStream_t ts = s;
    if (nseg > 1) {
        if (!b.aux || !b.ev_fork) return fail(DFA_E_DEVICE, "segmented match without an aux stream");
        hipError_t fe = hipEventRecord(b.ev_fork, s);
        if (fe == hipSuccess) fe = hipStreamWaitEvent(b.aux, b.ev_fork, 0);
        if (fe != hipSuccess) return hip_fail(fe, "fork to the translation stream");
        ts = b.aux;
    }
    for (uint32_t k = 0; k < nseg; ++k) {
        const uint64_t off = (uint64_t)cb[k] * p.chunk;
        const uint64_t end = std::min<uint64_t>((uint64_t)cb[k + 1] * p.chunk, p.n);
        uint32_t *bad = b.block_bad + (size_t)k * p.tblocks;
        if (pairs)
            hipLaunchKernelGGL(k_translate_pairs, dim3(p.tblocks), dim3(256), 0, ts, d_in + off,
                               end - off, d->dev.pcode, d->dev.nclass, (uint8_t *)b.codes + off / 2,
                               bad);
        else if (direct)
            hipLaunchKernelGGL((k_translate<uint8_t, false>), dim3(p.tblocks), dim3(256), 0, ts,
                               d_in + off, end - off, d->dev.code, (uint8_t *)nullptr, bad);
        else if (L == 1)
            hipLaunchKernelGGL(k_translate<uint8_t>, dim3(p.tblocks), dim3(256), 0, ts, d_in + off,
                               end - off, d->dev.code, (uint8_t *)b.codes + off, bad);
        else
            hipLaunchKernelGGL(k_translate<uint16_t>, dim3(p.tblocks), dim3(256), 0, ts, d_in + off,
                               end - off, d->dev.code, (uint16_t *)b.codes + off, bad);
        if (nseg > 1) {
            hipError_t fe = hipEventRecord(b.ev_seg[k], ts);
            if (fe != hipSuccess) return hip_fail(fe, "hipEventRecord (segment)");
        }
    }
    Match2Args a;
    a.d = d->dev;
    if (pairs) {   // the matcher stages and indexes the pair table instead
        a.d.stab = d->dev.stab2;
        a.d.stab_bytes = d->dev.stab2_bytes;
        a.d.rowbytes = d->dev.rowbytes2;
        a.d.abs_off = d->dev.abs_off2;
        a.d.abs_shift = 2;
    }
    a.codes = direct ? static_cast<const void *>(d_in) : b.codes;
    a.n = p.n;
    a.chunk = p.chunk;
    a.nch = p.nch;
    a.start = start;
    a.mode = p.lookahead;
    a.r = p.r;
    a.first = b.first;
    a.tile_first = b.tile_first;
    a.ccls = b.ccls;
    a.cset = b.cset;
    a.members = b.members;
    a.bits = b.bits;
    a.W = p.bitmap_words;
    a.maps = maps;
    a.exit_base = p.early_exit ? a.d.abs_off : 0u;
    a.exit_shift = a.d.abs_shift;
    a.c_lo = 0;
    a.c_hi = p.nch;
    const size_t lds = a.d.stab_bytes;
    ScanSrc q{msize, b.bits, p.bitmap_words, p.nch, kWave2 * p.slots};
    if (p.lookahead == 2) {
        // window pairs (chunk, state of I_sigma_1) -> start-set bitmaps -> member lists
        hipLaunchKernelGGL(k_chunkinfo_w, dim3((p.nch + 255) / 256), dim3(256), 0, s, d->dev, d_in,
                           p.chunk, p.nch, p.r, p.bitmap_words, msize, b.cset, b.bits);
        launch_scan<0>(p, q, b, nullptr, start, s);
        const void *wf = window2_kernel(L, p.slots);
        void *wargs[] = {&a};
        hipError_t we = hipLaunchKernel(wf, dim3(p.blocks2), dim3(p.threads2), wargs, lds, s);
        if (we != hipSuccess) return hip_fail(we, "k_window2 launch");
        launch_scan<1>(p, q, b, msize, start, s);
    } else if (p.lookahead == 3) {
        hipLaunchKernelGGL(k_chunkinfo_m, dim3((p.nch + 255) / 256), dim3(256), 0, s, d->dev, d_in,
                           p.chunk, p.nch, p.r, msize, b.cset);
        launch_scan<0>(p, q, b, nseg > 1 ? nullptr : msize, start, s);
    } else {
        hipLaunchKernelGGL(k_chunkinfo, dim3((p.nch + 255) / 256), dim3(256), 0, s, d->dev, d_in,
                           p.chunk, p.nch, p.lookahead, msize, b.ccls);
        launch_scan<0>(p, q, b, nseg > 1 ? nullptr : msize, start, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "packed-matcher preparation launch");
    const void *fn = match2_kernel(L, p.slots, p.early_exit);
    for (uint32_t k = 0; k < nseg; ++k) {
        if (nseg > 1) {
            e = hipStreamWaitEvent(s, b.ev_seg[k], 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent (segment)");
        }
        if (k == 0 && ev_before_matcher) {
            e = hipEventRecord(ev_before_matcher, s);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        a.c_lo = cb[k];
        a.c_hi = cb[k + 1];
        void *args[] = {&a};
        e = hipLaunchKernel(fn, dim3(p.blocks2), dim3(p.threads2), args, lds, s);
        if (e != hipSuccess) return hip_fail(e, "k_match2 launch");
    }
    if (nseg > 1)
        hipLaunchKernelGGL(k_fold_bad, dim3(1), dim3(256), 0, s, b.block_bad, nseg * p.tblocks, msize);
    e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "k_match2 launch");
}

int launch_size_scan(uint32_t nch, uint16_t *msize, uint32_t *bsum, uint32_t *first,
                     uint32_t *tile_first, uint32_t tile, hipStream_t s) {
    if (nch == 0) return DFA_OK;
    const uint32_t nsb = (nch + kScanBlock - 1) / kScanBlock;
    ScanSrc q{msize, nullptr, 0, nch, tile};
    hipLaunchKernelGGL(k_scan_sums<0>, dim3(nsb), dim3(kScanThreads), 0, s, q, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, bsum, nsb,
                       (uint16_t *)nullptr, nch, (const uint32_t *)nullptr, 0u, first);
    hipLaunchKernelGGL(k_scan_apply<0>, dim3(nsb), dim3(kScanThreads), 0, s, q, bsum, first,
                       tile_first, (uint16_t *)nullptr, 0u);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "size scan launch");
}

int launch_down0(const MatchPlan &p, const uint16_t *maps0, const uint32_t *first,
                 const uint16_t *bv_up, uint16_t *bv0, hipStream_t s) {
    const uint32_t n_up = p.levels >= 1 ? p.level_count[1] : 1u;
    const uint32_t G = p.levels >= 1 ? p.group : 1u;
    hipLaunchKernelGGL(k_down0, dim3((n_up + 255) / 256), dim3(256), 0, s, maps0, first, p.nch, G,
                       bv_up, n_up, bv0);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "k_down0 launch");
}


int set_match2_lds_limit(int lds) {
    const void *fns[] = {match2_kernel(1, 2, false), match2_kernel(1, 2, true),
                         match2_kernel(1, 4, false), match2_kernel(1, 4, true),
                         match2_kernel(2, 2, false), match2_kernel(2, 2, true),
                         match2_kernel(2, 4, false), match2_kernel(2, 4, true),
                         match2_kernel(3, 2, false), match2_kernel(3, 2, true),
                         match2_kernel(3, 4, false), match2_kernel(3, 4, true),
                         match2_kernel(4, 2, false), match2_kernel(4, 2, true),
                         match2_kernel(4, 4, false), match2_kernel(4, 4, true),
                         window2_kernel(1, 2), window2_kernel(1, 4),
                         window2_kernel(2, 2), window2_kernel(2, 4)};
    int rc = DFA_OK;
    for (const void *f : fns)
        if (allow_dynamic_lds(f, lds) != DFA_OK) rc = DFA_E_DEVICE;
    return rc;
}

uint32_t match2_tile_pairs(uint32_t slots) { return kWave2 * slots; }
uint32_t match2_scan_blocks(uint32_t nch) { return (nch + kScanBlock - 1) / kScanBlock; }

}  // namespace dfaspec
