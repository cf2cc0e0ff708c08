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
// Kernels: k_translate (bytes -> codes, invalid-byte flags), k_scan
// (lookahead class or set and |I| per chunk, exclusive prefix of the set
// sizes = first pair of each chunk), k_match2 (persistent tiles of pairs).
// The sparse maps it writes have the same form as the one-chunk-per-wave
// matcher's, so the combination kernels are shared.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <map>
#include <type_traits>

#include "dfa_pairs.h"

namespace dfaspec {

// ---------------------------------------------------------------------------
// Translation: code[i] = code_lut[in[i]]; per-block flag if a byte is outside
// Sigma.  WRITE = false only validates (direct tables).  The output is
// 16-byte aligned.
// ---------------------------------------------------------------------------
constexpr int kTrU = 4;

// Chunk-interleaved code stream: with chunks of nblk 16-byte code blocks,
// block b of chunk c is unit ((c / 64) * nblk + b) * 64 + c % 64, so that the
// walks of 64 consecutive chunks read one contiguous KiB per block.  nblk = 0:
// the linear stream (unit c * nblk + b, i.e. the byte offset itself).
struct Ilv {
    uint32_t nblk;     // 16-byte code blocks per chunk; 0 = linear
    uint32_t nch;
    uint64_t chunk;    // input bytes per chunk
};

// Where byte `ob` of the linear code stream goes (a store never crosses a
// 16-byte unit): the linear stream itself, or its interleaved place for the
// chunk c the grid is converting.
struct LinearSink {
    uint8_t *out;
    __device__ __forceinline__ uint8_t *at(uint64_t ob) const { return out + ob; }
};
struct IlvSink {
    uint8_t *out;
    uint32_t nblk;
    uint32_t c;
    uint64_t base;           // linear offset of chunk c's first code byte
    __device__ __forceinline__ uint8_t *at(uint64_t ob) const {
        const uint32_t b = (uint32_t)((ob - base) >> 4);
        const uint64_t unit = ((uint64_t)(c >> 6) * nblk + b) * 64u + (c & 63u);
        return out + unit * 16u + (ob & 15u);
    }
};

// The grid walk shared by the translation kernels: convert(tag, w, first,
// sink) handles the 16 input bytes at `first` (tag: std::true_type when all
// lie before n) and stores its codes through the sink.  Whole rounds of an aligned input load kTrU blocks per thread
// before converting any (block u of a round is u * threads + thread, so every
// load instruction is coalesced): with one 16-byte load in flight per lane a
// pass is bound by memory latency well below HBM bandwidth.  The last partial
// round and misaligned inputs go one block at a time.
template <typename Conv>
__device__ __forceinline__ void translate_grid(const uint8_t *__restrict__ in, uint64_t n,
                                               uint8_t *out, Conv &convert) {
    const LinearSink sink{out};
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
                convert(std::true_type{}, w, base + ((uint64_t)u * T + tid) * 16, sink);
            }
        }
    }
    for (uint64_t first = base + tid * 16; first < n; first += T * 16) {
        uint32_t w[4];
        load16(in, first, n, w);
        if (first + 16 <= n) convert(std::true_type{}, w, first, sink);
        else convert(std::false_type{}, w, first, sink);
    }
}

// Grid walk of the interleaved translation.  A wave takes 64 / PIECES
// consecutive chunks (lane l: chunk l / PIECES, piece l % PIECES) and goes
// through their code blocks a quad (4 blocks, PIECES 16-byte input pieces per
// chunk) at a time, kTrU quads in flight, so that loads are contiguous per
// chunk and every block's stores of the wave are contiguous too.  The stream
// holds v.nblk blocks per chunk: the whole chunk, or its first bytes when
// the last round reads the raw input (bytes past them are not read here).
// code_bytes_per_chunk: a chunk's code bytes in the linear numbering.
template <int PIECES, typename Conv>
__device__ __forceinline__ void translate_ilv_grid(const uint8_t *__restrict__ in, uint64_t n,
                                                   uint8_t *out, const Ilv &v,
                                                   uint64_t code_bytes_per_chunk, Conv &convert) {
    constexpr uint32_t kCpw = 64 / PIECES;
    const uint32_t nquad = (v.nblk + 3) / 4;
    const uint32_t nsg = (v.nch + kCpw - 1) / kCpw;
    const uint64_t span = (uint64_t)PIECES * 16u;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t cc = lane / PIECES, k = lane % PIECES;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t sg = wave; sg < nsg; sg += nwaves) {
        const uint32_t c = sg * kCpw + cc;
        const bool live = c < v.nch;
        const uint64_t c0 = (uint64_t)c * v.chunk;
        const uint64_t coded = min<uint64_t>(v.chunk, (uint64_t)v.nblk * PIECES * 4u);
        const uint64_t end = live ? min<uint64_t>(c0 + coded, n) : 0u;
        const IlvSink sink{out, v.nblk, c, (uint64_t)c * code_bytes_per_chunk};
        for (uint32_t q0 = 0; q0 < nquad; q0 += kTrU) {
            uint32_t w[kTrU][4];
#pragma unroll
            for (int u = 0; u < kTrU; ++u) {
                const uint64_t first = c0 + (uint64_t)(q0 + u) * span + 16u * k;
                if (first < end) load16(in, first, n, w[u]);
            }
#pragma unroll
            for (int u = 0; u < kTrU; ++u) {
                const uint64_t first = c0 + (uint64_t)(q0 + u) * span + 16u * k;
                if (first >= end) continue;
                if (first + 16 <= n) convert(std::true_type{}, w[u], first, sink);
                else convert(std::false_type{}, w[u], first, sink);
            }
        }
    }
}

// Interleaved grid walk of the two-symbol translations: a thread item is 32
// input bytes (two pieces, 16 codes) stored as one 16-byte unit, so that
// every store instruction writes whole lines.  conv(tag, w, first) returns the
// 8 codes of the piece at `first` (tag: all 16 bytes before n).
template <typename Conv>
__device__ __forceinline__ uint2 pair_piece(Conv &conv, const uint32_t (&w)[4], uint64_t first,
                                            uint64_t n) {
    if (first >= n) return make_uint2(0u, 0u);
    if (first + 16 <= n) return conv(std::true_type{}, w, first);
    return conv(std::false_type{}, w, first);
}

// Interleaved: a wave takes 16 consecutive chunks, 4 lanes per chunk (32
// input bytes each: one code block), kTrU blocks per lane in flight.
template <typename Conv>
__device__ __forceinline__ void pairs_grid_ilv(const uint8_t *__restrict__ in, uint64_t n,
                                               uint8_t *out, const Ilv &v, Conv &conv) {
    const uint32_t nsg = (v.nch + 15) / 16;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t cc = lane >> 2, k = lane & 3u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t sg = wave; sg < nsg; sg += nwaves) {
        const uint32_t c = sg * 16 + cc;
        const uint64_t c0 = (uint64_t)c * v.chunk;
        const uint64_t end = c < v.nch ? min<uint64_t>(c0 + v.chunk, n) : 0u;
        for (uint32_t b0 = 0; b0 < v.nblk; b0 += 4 * kTrU) {
            uint32_t w[kTrU][2][4];
#pragma unroll
            for (int u = 0; u < kTrU; ++u) {
                const uint64_t first = c0 + (uint64_t)(b0 + 4 * u + k) * 32;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (first + 16 * h < end) load16(in, first + 16 * h, n, w[u][h]);
            }
#pragma unroll
            for (int u = 0; u < kTrU; ++u) {
                const uint32_t b = b0 + 4 * u + k;
                const uint64_t first = c0 + (uint64_t)b * 32;
                if (first >= end) continue;
                const uint2 lo = pair_piece(conv, w[u][0], first, n);
                const uint2 hi = first + 16 < end ? pair_piece(conv, w[u][1], first + 16, n)
                                                  : make_uint2(0u, 0u);
                const uint64_t unit = ((uint64_t)(c >> 6) * v.nblk + b) * 64u + (c & 63u);
                *reinterpret_cast<uint4 *>(out + unit * 16u) = make_uint4(lo.x, lo.y, hi.x, hi.y);
            }
        }
    }
}

// Bytes 0 of four words packed into one (v_perm_b32).
__device__ __forceinline__ uint32_t pack_low_bytes(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
    return __builtin_amdgcn_perm(c1, c0, 0x0C0C0400u) | __builtin_amdgcn_perm(c3, c2, 0x04000C0Cu);
}

// Exclusive scan of the set sizes in three phases: first[i] = sum_{k<i} m_k,
// first[nch] = number of pairs, tile_first[w] = chunk holding pair w * tile.
// Sizes come from msize (SRC 0) or from the popcounts of the start-set
// bitmaps (SRC 1: chunk 0 holds the start state; the sizes are also written to
// msize and the sorted member lists to members[first[i] ..]).  Phase 2 folds
// the translation flags into the flag bit of chunk 0's size, from where the
// compose levels carry it up.
constexpr uint32_t kScanThreads = 256;    // enough blocks to spread the first phase
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

// The first phase fused with the per-chunk lookahead information of modes
// 0, 1 (class sets: ccls) and 3 (precomputed multi-symbol sets: cset): the
// sizes it sums are computed here and written to msize for the later phases.
struct InfoSrc {
    DevDFA d;
    const uint8_t *in;
    uint64_t chunk;
    uint32_t mode;
    uint32_t r;
    uint16_t *ccls;
    uint32_t *cset;
    uint64_t before;         // bytes readable before `in` (a block map: chunk 0 then
                             // starts from its lookahead set, not the start state)
};

__device__ __forceinline__ uint32_t chunk_info(const InfoSrc &f, uint64_t i) {
    uint32_t m = 1, id = 0;
    if (i > 0 || f.before > 0) {
        // chunk i starts at in + p, with `avail` bytes of lookahead behind it
        const int64_t p = (int64_t)(i * f.chunk);
        const uint64_t avail = f.before + i * f.chunk;
        if (f.mode == 3) {
            const uint32_t k = (uint32_t)min<uint64_t>(f.r, avail);
            bool bad = false;
            if (k <= 8 && avail >= 8 && ((reinterpret_cast<uintptr_t>(f.in) + p) & 7u) == 0) {
                // the 8 bytes before p in one aligned load; the k class
                // lookups are independent
                const uint64_t wv = *reinterpret_cast<const uint64_t *>(f.in + p - 8);
                uint32_t cls[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) cls[j] = f.d.lut[(uint32_t)(wv >> (8 * j)) & 0xFFu];
                for (uint32_t j = 8 - k; j < 8; ++j) {
                    if (cls[j] == kLutInvalid) { bad = true; id = 0; break; }
                    id = id * f.d.nclass + (cls[j] >> 24);
                }
            } else {
                id = class_string_id(f.d, f.in + p - (int64_t)k, 0, k, &bad);
            }
            m = bad ? 0u : mset_end(f.d, k, id) - mset_begin(f.d, k, id);
        } else {
            const uint32_t e = f.d.lut[f.in[p - 1]];
            if (e == kLutInvalid) {
                m = 0;
            } else {
                id = e >> 24;
                m = f.d.set_off[f.mode][id + 1] - f.d.set_off[f.mode][id];
            }
        }
    }
    if (f.mode == 3) f.cset[i] = id;
    else f.ccls[i] = (uint16_t)id;
    return m;
}

// The first phase for scan block sb (kScanThreads threads).
__device__ __forceinline__ void scan_sums_block(const ScanSrc &q, const InfoSrc &f,
                                                uint32_t *__restrict__ bsum, uint32_t sb,
                                                uint32_t *part, uint16_t *ms) {
    // the block's chunks are computed strided over the threads (independent,
    // coalesced), then summed in consecutive runs for the scan
    const uint64_t b0 = (uint64_t)sb * kScanBlock;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint32_t t = k * kScanThreads + threadIdx.x;
        uint32_t m = 0;
        if (b0 + t < q.nch) {
            m = chunk_info(f, b0 + t);
            q.msize[b0 + t] = (uint16_t)m;
        }
        ms[t] = (uint16_t)m;
    }
    __syncthreads();
    uint32_t v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) v += ms[threadIdx.x * kScanItems + k];
    const uint32_t inc = block_inclusive_scan(v, part);
    if (threadIdx.x == kScanThreads - 1) bsum[sb] = inc;
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_scan_sums_info(ScanSrc q, InfoSrc f,
                                                         uint32_t *__restrict__ bsum) {
    __shared__ uint32_t part[kScanThreads];
    __shared__ uint16_t ms[kScanBlock];
    scan_sums_block(q, f, bsum, blockIdx.x, part, ms);
}

// The first phase run by the workgroups of a translation pass (256 threads)
// before they translate: scan blocks blockIdx.x, blockIdx.x + gridDim.x, ...
// (nsb = 0: none).
struct SumsArgs {
    ScanSrc q;
    InfoSrc f;
    uint32_t *bsum;
    uint32_t nsb;
};

__device__ __forceinline__ void scan_sums_in_pass(const SumsArgs &sa) {
    if (blockIdx.x >= sa.nsb) return;
    __shared__ uint32_t part[kScanThreads];
    __shared__ uint16_t ms[kScanBlock];
    for (uint32_t sb = blockIdx.x; sb < sa.nsb; sb += gridDim.x)
        scan_sums_block(sa.q, sa.f, sa.bsum, sb, part, ms);
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *__restrict__ bsum, uint32_t nb,
                                                   uint16_t *__restrict__ msize, uint32_t nch,
                                                   const uint32_t *__restrict__ block_bad,
                                                   uint32_t nbad, uint32_t *__restrict__ first,
                                                   uint32_t *__restrict__ zero, uint32_t nzero) {
    __shared__ uint32_t part[kScanThreads];
    __shared__ uint32_t bad_any;
    const uint32_t t = threadIdx.x, T = blockDim.x;
    for (uint32_t i = t; i < nzero; i += T) zero[i] = 0;   // counters of the merged-walk rounds
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


// The last two phases in one pass, for sizes from msize: workgroup b adds up
// the totals of scan blocks 0 .. b - 1 itself (a few thousand at most), then
// lays out its chunks as k_scan_apply does; the last workgroup writes
// first[nch], the first clears the merged-walk round counters, and every
// chunk's entry of chunk_zero (per-chunk counters, may be null) is cleared.
__global__ __launch_bounds__(1024) void k_scan_finish(ScanSrc q, const uint32_t *__restrict__ btot,
                                                      uint32_t *__restrict__ first,
                                                      uint32_t *__restrict__ tile_first,
                                                      uint32_t *__restrict__ zero, uint32_t nzero,
                                                      uint32_t *__restrict__ chunk_zero) {
    __shared__ uint32_t part[kScanThreads];
    const uint32_t t = threadIdx.x, T = blockDim.x;
    if (blockIdx.x == 0)
        for (uint32_t i = t; i < nzero; i += T) zero[i] = 0;
    uint32_t acc = 0;
    for (uint32_t j = t; j < blockIdx.x; j += T) acc += btot[j];
    block_inclusive_scan(acc, part);
    const uint32_t pre = part[T - 1];
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + t * kScanItems;
    uint32_t m[kScanItems], v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        m[k] = base + k < q.nch ? scan_size<0>(q, base + k) : 0u;
        v += m[k];
    }
    const uint32_t inc = block_inclusive_scan(v, part);
    uint32_t run = pre + inc - v;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + k;
        if (i < q.nch) {
            first[i] = run;
            if (chunk_zero) chunk_zero[i] = 0;
            if (m[k]) {
                for (uint32_t w = (run + q.tile - 1) / q.tile; w <= (run + m[k] - 1) / q.tile; ++w)
                    tile_first[w] = (uint32_t)i;
            }
        }
        run += m[k];
    }
    if (blockIdx.x + 1 == gridDim.x && t == T - 1) first[q.nch] = pre + inc;
}

template <typename CodeT, bool WRITE = true>
__global__ __launch_bounds__(256) void k_translate(const uint8_t *__restrict__ in, uint64_t n,
                                                   const uint16_t *__restrict__ code_lut,
                                                   CodeT *__restrict__ out,
                                                   uint32_t *__restrict__ block_bad, Ilv ilv,
                                                   SumsArgs sa) {
    scan_sums_in_pass(sa);
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
    auto convert = [&](auto whole_tag, const uint32_t (&w)[4], uint64_t first, const auto &sink) {
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
            *reinterpret_cast<uint4 *>(sink.at(first)) = o;
        } else {
            uint4 o[2];
            uint32_t *ow = reinterpret_cast<uint32_t *>(o);
#pragma unroll
            for (int q = 0; q < 8; ++q) ow[q] = __builtin_amdgcn_perm(c[2 * q + 1], c[2 * q], 0x05040100u);
            *reinterpret_cast<uint4 *>(sink.at(2 * first)) = o[0];
            *reinterpret_cast<uint4 *>(sink.at(2 * first + 16)) = o[1];
        }
    };
    uint8_t *ob = reinterpret_cast<uint8_t *>(out);
    if (WRITE && ilv.nblk)
        translate_ilv_grid<kNarrow ? 4 : 2>(in, n, ob, ilv, ilv.chunk * sizeof(CodeT), convert);
    else
        translate_grid(in, n, ob, convert);
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
                                                         uint32_t *__restrict__ block_bad, Ilv ilv,
                                                         SumsArgs sa) {
    scan_sums_in_pass(sa);
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
    auto convert = [&](auto whole_tag, const uint32_t (&w)[4], uint64_t first) -> uint2 {
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
        return make_uint2(pack_low_bytes(c[0], c[1], c[2], c[3]), pack_low_bytes(c[4], c[5], c[6], c[7]));
    };
    if (ilv.nblk) {
        pairs_grid_ilv(in, n, out, ilv, convert);
    } else {
        auto store8 = [&](auto tag, const uint32_t (&w)[4], uint64_t first, const auto &sink) {
            *reinterpret_cast<uint2 *>(sink.at(first / 2)) = convert(tag, w, first);
        };
        translate_grid(in, n, out, store8);
    }
    if (bad) atomicOr(&bad_any, 1u);
    __syncthreads();
    if (threadIdx.x == 0) block_bad[blockIdx.x] = bad_any;
}

// Two-symbol translation for direct tables (every byte of Sigma below 128):
// one LDS lookup per pair, pc2[b1 + 256 * b2] (a lone last byte: pc2[32768 +
// b]).  Entries of bytes outside Sigma are 0xFF (odd, unlike every code); a
// block whose OR of entries is odd or that holds a byte >= 128 is redone on
// the checked path, which writes 0 for such pairs.
__global__ __launch_bounds__(256) void k_translate_pairs_direct(const uint8_t *__restrict__ in,
                                                                uint64_t n,
                                                                const uint8_t *__restrict__ pcode2,
                                                                uint8_t *__restrict__ out,
                                                                uint32_t *__restrict__ block_bad,
                                                                Ilv ilv, SumsArgs sa) {
    scan_sums_in_pass(sa);
    constexpr uint32_t kPc2 = 32768u + 128u;
    __shared__ __align__(16) uint8_t pc2[kPc2];
    __shared__ uint32_t bad_any;
    for (uint32_t i = threadIdx.x; i < kPc2 / 16; i += blockDim.x)
        reinterpret_cast<uint4 *>(pc2)[i] = reinterpret_cast<const uint4 *>(pcode2)[i];
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    uint32_t bad = 0;
    auto checked = [&](const uint32_t (&w)[4], uint64_t first, uint32_t (&c)[8]) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t b1 = (w[k >> 1] >> (16 * (k & 1))) & 0xFFu;
            const uint32_t b2 = (w[k >> 1] >> (16 * (k & 1) + 8)) & 0xFFu;
            const bool in1 = first + 2 * k < n, in2 = first + 2 * k + 1 < n;
            uint32_t v = 0xFFu;
            if (in2) {
                if (b1 < 128u && b2 < 128u) v = pc2[b1 + 256u * b2];
            } else if (b1 < 128u) {
                v = pc2[32768u + b1];
            }
            const bool inv = in1 && (v & 1u);
            bad |= inv ? 1u : 0u;
            c[k] = (!in1 || inv) ? 0u : v;
        }
    };
    auto convert = [&](auto whole_tag, const uint32_t (&w)[4], uint64_t first) -> uint2 {
        constexpr bool WHOLE = decltype(whole_tag)::value;
        uint32_t c[8];
        if constexpr (WHOLE) {
            uint32_t acc = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                c[k] = pc2[(w[k >> 1] >> (16 * (k & 1))) & 0x7F7Fu];
                acc |= c[k];
            }
            const uint32_t high = (w[0] | w[1] | w[2] | w[3]) & 0x80808080u;
            if ((acc & 1u) || high) checked(w, first, c);
        } else {
            checked(w, first, c);
        }
        return make_uint2(pack_low_bytes(c[0], c[1], c[2], c[3]), pack_low_bytes(c[4], c[5], c[6], c[7]));
    };
    if (ilv.nblk) {
        pairs_grid_ilv(in, n, out, ilv, convert);
    } else {
        auto store8 = [&](auto tag, const uint32_t (&w)[4], uint64_t first, const auto &sink) {
            *reinterpret_cast<uint2 *>(sink.at(first / 2)) = convert(tag, w, first);
        };
        translate_grid(in, n, out, store8);
    }
    if (bad) atomicOr(&bad_any, 1u);
    __syncthreads();
    if (threadIdx.x == 0) block_bad[blockIdx.x] = bad_any;
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
// For r <= r0 the start set of chunk i >= 1 is the precomputed I_{c_1..c_k}
// of its k = min(r, p) lookahead bytes (chunk_info, in the scan's first
// phase).  r > r0: window pairs start from the precomputed set of the window's first
// k0 = min(r', r0) bytes; cset holds that set's id.  Clears the bitmaps.
__global__ void k_chunkinfo_w(DevDFA d, const uint8_t *__restrict__ in, uint64_t chunk,
                              uint32_t nch, uint32_t r, uint32_t W,
                              uint16_t *__restrict__ msize, uint32_t *__restrict__ cset,
                              uint32_t *__restrict__ bits, uint32_t *__restrict__ chunk_zero) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nch) return;
    for (uint32_t k = 0; k < W; ++k) bits[(size_t)i * W + k] = 0;
    if (chunk_zero) chunk_zero[i] = 0;   // per-chunk slot counters of the last round
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
    uint32_t tile;           // pairs per wave-tile (64 * slots)
    uint32_t ilv_nblk;       // chunk-interleaved codes: 16-byte blocks per chunk; 0 = linear
    uint32_t spread;         // tiles to waves: 1 = first wave of every workgroup first
                             // (few, large workgroups per CU), 0 = workgroup by workgroup
    uint64_t before;         // bytes of lookahead before the input (block maps; 0 = none)
    const uint8_t *raw;      // the input itself (the window pass reads it when the code
                             // stream is chunk-interleaved)
};

// First 16-byte unit of block b of chunk c in the code stream, and the
// distance between a chunk's consecutive blocks.
__device__ __forceinline__ uint32_t code_unit(const Match2Args &a, uint32_t c, uint32_t b,
                                              uint32_t per_chunk_linear) {
    if (a.ilv_nblk) return ((c >> 6) * a.ilv_nblk + b) * 64u + (c & 63u);
    return c * per_chunk_linear + b;
}

template <int L>
__device__ __forceinline__ void stage_table(const DevDFA &d, uint8_t *smem) {
    const uint4 *src = reinterpret_cast<const uint4 *>(d.stab);
    uint4 *dst = reinterpret_cast<uint4 *>(smem);
    for (uint32_t i = threadIdx.x; i < d.stab_bytes / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Map entry of a walk of chunk c that ended in state e: kTerm | e for the
// last chunk or an absorbing e, else e's position in chunk c + 1's start set.
__device__ __forceinline__ uint16_t map_entry(const Match2Args &a, uint32_t c, uint32_t e) {
    if (c + 1 == a.nch) return (uint16_t)(kTerm | e);
    if (a.mode == 2) {
        const uint16_t ab = a.d.pos[1][e];   // class-0 row: kTerm|e iff absorbing
        return ab == (uint16_t)(kTerm | e)
                   ? ab
                   : (uint16_t)member_rank(a.members, a.first[c + 1], a.first[c + 2], e);
    }
    if (a.mode == 3) {
        const uint16_t ab = a.d.pos[1][e];
        const uint32_t k = (uint32_t)min<uint64_t>(a.r, a.before + (uint64_t)(c + 1) * a.chunk);
        const uint32_t id = a.cset[c + 1];
        return ab == (uint16_t)(kTerm | e)
                   ? ab
                   : (uint16_t)member_rank(a.d.mset_st + a.d.mst[k], mset_begin(a.d, k, id),
                                           mset_end(a.d, k, id), e);
    }
    return a.d.pos[a.mode][(size_t)a.ccls[c + 1] * a.d.nq + e];
}

// Start state of pair P (chunk c >= 0 of the pair numbering).
__device__ __forceinline__ uint32_t pair_start(const Match2Args &a, uint32_t c, uint32_t P) {
    if (c == 0 && a.before == 0) return a.start;
    if (a.mode == 2) return a.members[P];
    if (a.mode == 3) {
        const uint32_t k = (uint32_t)min<uint64_t>(a.r, a.before + (uint64_t)c * a.chunk);
        return a.d.mset_st[a.d.mst[k] + mset_begin(a.d, k, a.cset[c]) + (P - a.first[c])];
    }
    return a.d.set_st[a.mode][a.d.set_off[a.mode][a.ccls[c]] + (P - a.first[c])];
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
    // spread: tiles go to the first wave of every workgroup, then the
    // second, ..., so that a launch with fewer tiles than waves still keeps
    // every CU busy when each CU holds only one or two workgroups; else
    // consecutive tiles stay in one workgroup
    const uint32_t wave_id = a.spread ? (threadIdx.x / kWave2) * gridDim.x + blockIdx.x
                                      : blockIdx.x * waves + threadIdx.x / kWave2;
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
        if (a.ilv_nblk) {
            // the code stream is chunk-interleaved (and may cover only each
            // chunk's first bytes): read the bytes before the chunk from the
            // input and turn them into codes here.  A byte outside Sigma
            // (flagged where its own chunk is walked) steps as code 0, so the
            // walk stays on table rows.
            for (uint32_t t = 0; t < maxlen; ++t) {
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    if (t < len[j]) {
                        const uint16_t c = a.d.code[a.raw[beg[j] + t]];
                        st[j] = lds_ld(st[j] + (c == kCodeInvalid ? 0u : (uint32_t)c));
                    }
                }
            }
        } else {
            for (uint32_t t = 0; t < maxlen; ++t) {
#pragma unroll
                for (int j = 0; j < S; ++j)
                    if (t < len[j]) st[j] = lds_ld(st[j] + (uint32_t)codes[beg[j] + t]);
            }
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
    using CodeT = typename std::conditional<kWideCodes<L>, uint16_t, uint8_t>::type;
    constexpr uint32_t kPer16 = 16 / sizeof(CodeT);   // codes per 16 bytes
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t waves = blockDim.x / kWave2;
    // spread: tiles go to the first wave of every workgroup, then the
    // second, ..., so that a launch with fewer tiles than waves still keeps
    // every CU busy when each CU holds only one or two workgroups; else
    // consecutive tiles stay in one workgroup
    const uint32_t wave_id = a.spread ? (threadIdx.x / kWave2) * gridDim.x + blockIdx.x
                                      : blockIdx.x * waves + threadIdx.x / kWave2;
    const uint32_t total_waves = gridDim.x * waves;
    const uint32_t total = a.first[a.nch];
    const uint32_t ntiles = (total + kTile - 1) / kTile;
    // pairs of chunks [c_lo, c_hi): the tiles that overlap them
    const uint32_t p_lo = a.first[a.c_lo], p_hi = a.first[a.c_hi];
    const uint32_t t_lo = p_lo / kTile, t_hi = (p_hi + kTile - 1) / kTile;
    // class-major tables (16-bit codes) hold 2 * state; row tables R * state
    const uint32_t R = kWideCodes<L> ? 2u : a.d.rowbytes;
    const CodeT *codes = reinterpret_cast<const CodeT *>(a.codes);
    auto code_at = [&](uint64_t pos) -> uint32_t {
        return L == 3 ? 2u * (codes[pos] & 0x7Fu) : (uint32_t)codes[pos];
    };
    // L = 4 (two-symbol steps): one code per two input bytes.  Chunk lengths
    // are multiples of the step (the host picks them for multiples of 32)
    constexpr uint32_t kSym = L == 4 ? 2u : 1u;   // symbols per code
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
            const uint32_t s = valid ? pair_start(a, c, P) : 0u;
            st[j] = R * s;
            ci[j] = valid ? c : 0xFFFFFFFFu;
            o16[j] = aligned_chunks ? code_unit(a, c, 0u, (uint32_t)(a.chunk / (kPer16 * kSym))) : 0u;
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
                                  a.exit_base, a.exit_shift, live, a.ilv_nblk ? 64u : 1u);
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
                const uint32_t P = tile * kTile + j * kWave2 + lane;
                a.maps[P] = map_entry(a, ci[j], st[j] / R);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Merged walks.  delta is a function, so two walks of one chunk that are in
// the same state at the same position stay together to the chunk's end.  The
// walk runs in rounds over byte ranges [t0, t1) of every chunk; after a round
// that is not the last, the walks of each wave-tile are grouped by (chunk,
// state), one walk per group (the leader) goes on into the next round's
// list, and every walk records its leader's index there.  A walk whose chunk
// ends within the round, or that reached an absorbing state, is done and
// records kDone | its end state.  Walks of one chunk split over two tiles may
// keep two leaders; the result is exact either way.
// ---------------------------------------------------------------------------
constexpr uint32_t kDone = 0x80000000u;     // outcome: the walk ended (low bits: state)
constexpr uint32_t kMapped = 0x40000000u;   // with kDone: low 16 bits are the map entry

// A round's list is split into kRegions regions of `cap` places, each with
// its own counter: tile t appends its leaders to region t % kRegions (one
// atomic add per tile, spread over kRegions addresses), and the next round
// numbers the walks densely across the regions.
struct RoundArgs {
    uint32_t t0, t1;           // chunk bytes of this round
    uint32_t first_round;      // walks are the pairs (start states from the sets)
    uint32_t last_round;       // walks run to the chunk end; no grouping
    uint32_t cap;              // places per region
    const uint32_t *in_cnt;    // later rounds: [kRegions] walks per region of in_list
    const uint2 *in_list;      // later rounds: {chunk, state} per place
    uint32_t *out_lo;          // per walk (pair, or place of in_list): kDone | end
                               //  state, or the place of its leader in out_list
    uint2 *out_list;           // the next round's walks
    uint32_t *out_cnt;         // [kRegions] its counters (zero before the first round)
    // the round before a one-chunk-per-lane last round: a leader takes a slot
    // of its chunk (tail_cnt[c] counts them; place c * kTailSlots + slot);
    // leaders beyond kTailSlots go to out_list, whose places then start at
    // next_off in the last round's outcomes
    uint32_t *tail_cnt;
    uint16_t *tail_st;
    uint32_t next_off;
};

template <int S>
constexpr int kRoundAhead = S >= 4 ? 1 : 2;

constexpr uint32_t kRoundPreBytes = (4u * (kRegions + 1) + 15u) / 16u * 16u;
// First-round grouping table per wavefront (LDS, after the region prefix):
// kRoundHash 32-bit entries, linear probing.  In the first round a tile's
// walks are pairs in chunk order, so a tile spans few chunks and an entry
// holds the chunk's offset from the tile's first chunk (8 bits), the end
// state (15 bits) and the leader's tile position (8 bits), exactly.
constexpr uint32_t kRoundHashBits = 7;
constexpr uint32_t kRoundHash = 1u << kRoundHashBits;
constexpr uint32_t kRoundProbes = 8;
constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;   // bit 31 is never set in an entry

// EXIT: the DFA has absorbing states; a wave stops once all its walks are in one.
template <int L, int S, bool EXIT>
__global__ __launch_bounds__(1024, S == 4 ? 5 : 6) void k_round(Match2Args a, RoundArgs m) {
    constexpr uint32_t kTile = kWave2 * S;
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<L>(a.d, smem);
    using CodeT = typename std::conditional<L != 2, uint8_t, uint16_t>::type;
    constexpr uint32_t kPer16 = 16 / sizeof(CodeT);
    constexpr uint32_t kSym = L == 4 ? 2u : 1u;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t waves = blockDim.x / kWave2;
    // spread: tiles go to the first wave of every workgroup, then the
    // second, ..., so that a launch with fewer tiles than waves still keeps
    // every CU busy when each CU holds only one or two workgroups; else
    // consecutive tiles stay in one workgroup
    const uint32_t wave_id = a.spread ? (threadIdx.x / kWave2) * gridDim.x + blockIdx.x
                                      : blockIdx.x * waves + threadIdx.x / kWave2;
    const uint32_t total_waves = gridDim.x * waves;
    // later rounds: exclusive prefix of the regions' counts, in LDS after the
    // staged table (the kernel has no static LDS: the table stays at address 0)
    uint32_t *region_pre = reinterpret_cast<uint32_t *>(smem + a.d.stab_bytes);
    uint32_t *round_table = reinterpret_cast<uint32_t *>(smem + a.d.stab_bytes + kRoundPreBytes);
    if (!m.first_round) {
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            for (uint32_t g = 0; g < kRegions; ++g) {
                region_pre[g] = acc;
                acc += m.in_cnt[g];
            }
            region_pre[kRegions] = acc;
        }
        __syncthreads();
    }
    const uint32_t total = m.first_round ? a.first[a.nch] : region_pre[kRegions];
    const uint32_t ntiles = (total + kTile - 1) / kTile;
    const uint32_t R = L != 2 ? a.d.rowbytes : 2u;
    const uint4 *codes16 = reinterpret_cast<const uint4 *>(a.codes);
    const uint64_t lanes_lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    // place of dense walk w of a later round: region by binary search
    auto place_of = [&](uint32_t w) -> uint32_t {
        uint32_t lo = 0, hi = kRegions;
        while (hi > lo + 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (region_pre[mid] <= w) lo = mid; else hi = mid;
        }
        return lo * m.cap + (w - region_pre[lo]);
    };

    for (uint32_t tile = wave_id; tile < ntiles; tile += total_waves) {
        uint32_t st[S], ci[S], o16[S];
        const uint32_t lo0 = m.first_round ? a.tile_first[tile] : 0u;
        const uint32_t hi0 = m.first_round ? (tile + 1 < ntiles ? a.tile_first[tile + 1] + 1 : a.nch) : 0u;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const uint32_t w = tile * kTile + j * kWave2 + lane;
            const bool valid = w < total;
            uint32_t c = 0, s0 = 0;
            if (valid) {
                if (m.first_round) {
                    c = owner_chunk(a.first, lo0, hi0, w);
                    s0 = pair_start(a, c, w);
                } else {
                    const uint2 rec = m.in_list[place_of(w)];
                    c = rec.x;
                    s0 = rec.y;
                }
            }
            st[j] = R * s0;
            ci[j] = valid ? c : kNone;
            o16[j] = code_unit(a, c, m.t0 / (kSym * kPer16), (uint32_t)(a.chunk / (kSym * kPer16)));
        }
        uint32_t live = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) live |= (ci[j] != kNone ? 1u : 0u) << j;
        // codes of [t0, min(t1, chunk length)); walks past the list's end
        // shadow chunk 0 (their loads stay in bounds; results discarded)
        auto len_of = [&](int j) -> uint32_t {
            const uint64_t c = ci[j] == kNone ? 0u : ci[j];
            const uint64_t len = min<uint64_t>(a.chunk, a.n - c * a.chunk);
            const uint64_t end = m.last_round ? len : min<uint64_t>(len, m.t1);
            return end > m.t0 ? (uint32_t)((end - m.t0 + kSym - 1) / kSym) : 0u;
        };
        // a wave stops walking once all its walks are absorbing (checked every
        // four blocks); their end states are then final
        // blocks of prefetch: the last round's walks run the rest of their
        // chunks (thousands of blocks) and each lane's S walks read S
        // unrelated code streams, so loads must be issued well ahead
        walk_var<L, S, EXIT, kRoundAhead<S>>(codes16, o16, len_of, st, EXIT ? a.d.abs_off : 0u, a.d.abs_shift,
                             live, a.ilv_nblk ? 64u : 1u);

        // end states; done = the chunk ended or the state is absorbing
        uint32_t e[S];
        bool act[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            e[j] = st[j] / R;
            bool done = true;
            if (ci[j] != kNone && !m.last_round) {
                const uint64_t len = min<uint64_t>(a.chunk, a.n - (uint64_t)ci[j] * a.chunk);
                const uint32_t idx = st[j] >> a.d.abs_shift;
                const bool absorbed = (lds_ld32(a.d.abs_off + ((idx >> 5) << 2)) >> (idx & 31)) & 1u;
                done = len <= m.t1 || absorbed;
            }
            act[j] = ci[j] != kNone && !done;
        }
        uint32_t lead[S];      // tile position of the walk's leader
        bool is_lead[S];
#pragma unroll
        for (int j = 0; j < S; ++j) { lead[j] = kNone; is_lead[j] = false; }
        // first round: the wave's hash table in LDS groups the walks (the
        // first walk to claim an empty entry for its key leads, walks that
        // find their key follow it; a walk whose probes all meet other keys
        // leads alone), unless the tile spans 256 chunks or more
        const uint32_t cbase = __builtin_amdgcn_readfirstlane(ci[0]);
        bool hashed = false;
        if (m.first_round) {
            bool wide = false;
#pragma unroll
            for (int j = 0; j < S; ++j) wide = wide || (act[j] && ci[j] - cbase >= 256u);
            hashed = !__any(wide);
        }
        if (hashed) {
            uint32_t *tab = round_table + (threadIdx.x / kWave2) * kRoundHash;
            for (uint32_t k = lane; k < kRoundHash; k += kWave2) tab[k] = kHashEmpty;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (!act[j]) continue;
                const uint32_t key = (ci[j] - cbase) << 23 | e[j] << 8;
                const uint32_t q = (uint32_t)j * kWave2 + lane;
                uint32_t h = ((ci[j] * 0x9E3779B1u) ^ (e[j] * 0x85EBCA77u)) >> (32 - kRoundHashBits);
                bool placed = false;
                for (int probe = 0; probe < (int)kRoundProbes && !placed; ++probe) {
                    const uint32_t old = atomicCAS(tab + h, kHashEmpty, key | q);
                    if (old == kHashEmpty) {
                        is_lead[j] = true;
                        lead[j] = q;
                        placed = true;
                    } else if ((old & ~0xFFu) == key) {
                        lead[j] = old & 0xFFu;
                        placed = true;
                    }
                    h = (h + 1) & (kRoundHash - 1);
                }
                if (!placed) {
                    is_lead[j] = true;
                    lead[j] = q;
                }
            }
        } else if (!m.last_round) {
            // group the active walks by (chunk, state): one pass per distinct
            // key, taking the first unresolved lane's key (at most 64 passes
            // per slot; each removes at least that lane)
#pragma unroll
            for (int j = 0; j < S; ++j) {
                uint64_t todo = __ballot(act[j]);
                while (todo) {
                    const uint32_t l0 = (uint32_t)__ffsll((unsigned long long)todo) - 1u;
                    const uint32_t kc = __builtin_amdgcn_readlane(ci[j], l0);
                    const uint32_t ke = __builtin_amdgcn_readlane(e[j], l0);
                    uint32_t q = (uint32_t)j * kWave2 + l0;
                    // a leader with this key in an earlier slot?
#pragma unroll
                    for (int jj = 0; jj < j; ++jj) {
                        const uint64_t mm = __ballot(is_lead[jj] && ci[jj] == kc && e[jj] == ke);
                        if (mm && q == (uint32_t)j * kWave2 + l0)
                            q = (uint32_t)jj * kWave2 + (uint32_t)__ffsll((unsigned long long)mm) - 1u;
                    }
                    const uint64_t mine = __ballot(act[j] && ci[j] == kc && e[j] == ke) & todo;
                    if ((mine >> lane) & 1ull) lead[j] = q;
                    if (lane == l0 && q == (uint32_t)j * kWave2 + l0) is_lead[j] = true;
                    todo &= ~mine;
                }
            }
        }
        // leaders take a slot of their chunk (before a one-chunk-per-lane
        // last round), else consecutive places in the next list
        uint32_t nlead = 0, myidx[S];
        bool listed[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            listed[j] = is_lead[j];
            myidx[j] = 0;
            if (m.tail_cnt && is_lead[j]) {
                const uint32_t k = atomicAdd(m.tail_cnt + ci[j], 1u);
                if (k < kTailSlots) {
                    myidx[j] = ci[j] * kTailSlots + k;
                    m.tail_st[myidx[j]] = (uint16_t)e[j];
                    listed[j] = false;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const uint64_t lm = __ballot(listed[j]);
            if (listed[j]) myidx[j] = nlead + (uint32_t)__popcll(lm & lanes_lt);
            nlead += (uint32_t)__popcll(lm);
        }
        uint32_t base = 0;
        if (nlead) {
            const uint32_t g = tile % kRegions;
            if (lane == 0) base = g * m.cap + atomicAdd(m.out_cnt + g, nlead);
            base = __shfl(base, 0);
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (listed[j]) {
                myidx[j] += base;
                m.out_list[myidx[j]] = make_uint2(ci[j], e[j]);
                myidx[j] += m.next_off;
            }
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            // the leader's list index, from its slot and lane
            uint32_t li = 0;
            const uint32_t ql = lead[j] == kNone ? 0u : lead[j];
#pragma unroll
            for (int jj = 0; jj < S; ++jj) {
                const uint32_t v = __shfl(myidx[jj], (int)(ql & (kWave2 - 1)));
                if ((ql >> 6) == (uint32_t)jj) li = v;
            }
            if (ci[j] != kNone) {
                const uint32_t w = tile * kTile + j * kWave2 + lane;
                // the last round stores the map entry itself (one per leader;
                // the walks that follow it take it as it is)
                const uint32_t done = m.last_round ? (kDone | kMapped | map_entry(a, ci[j], e[j]))
                                                   : (kDone | e[j]);
                m.out_lo[m.first_round ? w : place_of(w)] = act[j] ? li : done;
            }
        }
    }
}

// First merged round, chunk-major (interleaved codes, large start sets): a
// wavefront takes one chunk at a time and walks its whole start set, up to
// kR1Slots walks per lane, over the chunk's first t1 bytes.  The chunk's codes
// are the same for every walk of the wavefront, so they are loaded once (as
// wavefront-uniform values); the grouping key is the end state alone (a
// per-wavefront hash table as in k_round); the leaders' slots of a
// one-chunk-per-lane last round are numbered without atomics (the wavefront
// holds all of its chunk's leaders), and the rest of its leaders go to the
// next round's list, region c mod kRegions.  Outcomes as k_round's.
constexpr uint32_t kR1Slots = 5;   // 320 walks per wavefront >= any start set here

template <int L>
__global__ __launch_bounds__(1024, 5) void k_round1c(Match2Args a, RoundArgs m) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<L>(a.d, smem);
    constexpr uint32_t kCodeBytes = L == 2 ? 2u : 1u;
    const uint32_t lane = threadIdx.x & (kWave2 - 1);
    const uint32_t waves = blockDim.x / kWave2;
    const uint32_t wave_id = blockIdx.x * waves + threadIdx.x / kWave2;
    const uint32_t total_waves = gridDim.x * waves;
    uint32_t *round_table = reinterpret_cast<uint32_t *>(smem + a.d.stab_bytes + kRoundPreBytes);
    uint32_t *tab = round_table + (threadIdx.x / kWave2) * kRoundHash;
    const uint32_t R = L == 2 ? 2u : a.d.rowbytes;
    const uint4 *codes16 = reinterpret_cast<const uint4 *>(a.codes);
    const uint64_t lanes_lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    for (uint32_t c = wave_id; c < a.nch; c += total_waves) {
        const uint32_t f0 = a.first[c];
        const uint32_t mcnt = a.first[c + 1] - f0;
        const uint64_t len = min<uint64_t>(a.chunk, a.n - (uint64_t)c * a.chunk);
        const uint32_t steps = (uint32_t)min<uint64_t>(len, m.t1);
        uint32_t st[kR1Slots];
#pragma unroll
        for (uint32_t j = 0; j < kR1Slots; ++j) {
            const uint32_t q = j * kWave2 + lane;
            st[j] = q < mcnt ? R * pair_start(a, c, f0 + q) : 0u;
        }
        // the chunk's first 32 codes (16 B units of the interleaved stream)
        uint32_t cw[16];
#pragma unroll
        for (uint32_t b = 0; b < 32u * kCodeBytes / 16u; ++b) {
            const uint4 u = codes16[code_unit(a, c, b, (uint32_t)(a.chunk * kCodeBytes / 16))];
            cw[4 * b] = u.x;
            cw[4 * b + 1] = u.y;
            cw[4 * b + 2] = u.z;
            cw[4 * b + 3] = u.w;
        }
#pragma unroll
        for (uint32_t t = 0; t < 32; ++t) {
            if (t >= steps) break;
            const uint32_t code = L == 2 ? (cw[t >> 1] >> (16 * (t & 1))) & 0xFFFFu
                                         : (cw[t >> 2] >> (8 * (t & 3))) & 0xFFu;
#pragma unroll
            for (uint32_t j = 0; j < kR1Slots; ++j)
                if (j * kWave2 < mcnt) st[j] = lds_ld(st[j] + code);
        }
        // end states; done = the chunk ended or the state is absorbing
        uint32_t e[kR1Slots];
        bool act[kR1Slots], valid[kR1Slots];
#pragma unroll
        for (uint32_t j = 0; j < kR1Slots; ++j) {
            valid[j] = j * kWave2 + lane < mcnt;
            e[j] = st[j] / R;
            bool done = true;
            if (valid[j]) {
                const uint32_t idx = st[j] >> a.d.abs_shift;
                const bool absorbed = (lds_ld32(a.d.abs_off + ((idx >> 5) << 2)) >> (idx & 31)) & 1u;
                done = len <= m.t1 || absorbed;
            }
            act[j] = valid[j] && !done;
        }
        // group the active walks by end state: the first to claim a hash
        // entry leads, walks that find their state follow it; a walk whose
        // probes all meet other states leads alone
        for (uint32_t k = lane; k < kRoundHash; k += kWave2) tab[k] = kHashEmpty;
        uint32_t lead[kR1Slots];
        bool is_lead[kR1Slots];
#pragma unroll
        for (uint32_t j = 0; j < kR1Slots; ++j) {
            lead[j] = kNone;
            is_lead[j] = false;
            if (!act[j]) continue;
            const uint32_t key = e[j] << 9;
            const uint32_t q = j * kWave2 + lane;   // < 320: 9 bits
            uint32_t h = (e[j] * 0x85EBCA77u) >> (32 - kRoundHashBits);
            bool placed = false;
            for (int probe = 0; probe < (int)kRoundProbes && !placed; ++probe) {
                const uint32_t old = atomicCAS(tab + h, kHashEmpty, key | q);
                if (old == kHashEmpty) {
                    is_lead[j] = true;
                    lead[j] = q;
                    placed = true;
                } else if ((old & ~0x1FFu) == key) {
                    lead[j] = old & 0x1FFu;
                    placed = true;
                }
                h = (h + 1) & (kRoundHash - 1);
            }
            if (!placed) {
                is_lead[j] = true;
                lead[j] = q;
            }
        }
        // leaders numbered in (slot, lane) order: the first kTailSlots take
        // the chunk's slots of a one-chunk-per-lane last round, the others
        // (all of them without such a round) go to the next list
        uint32_t rank[kR1Slots], nlead = 0;
#pragma unroll
        for (uint32_t j = 0; j < kR1Slots; ++j) {
            const uint64_t lm = __ballot(is_lead[j]);
            rank[j] = nlead + (uint32_t)__popcll(lm & lanes_lt);
            nlead += (uint32_t)__popcll(lm);
        }
        const uint32_t nslot = m.tail_cnt ? min(nlead, kTailSlots) : 0u;
        const uint32_t nlist = nlead - nslot;
        uint32_t base = 0;
        const uint32_t g = c % kRegions;
        if (nlist) {
            if (lane == 0) base = g * m.cap + atomicAdd(m.out_cnt + g, nlist);
            base = __shfl(base, 0);
        }
        if (m.tail_cnt && lane == 0) m.tail_cnt[c] = nslot;
        uint32_t myidx[kR1Slots];
#pragma unroll
        for (uint32_t j = 0; j < kR1Slots; ++j) {
            myidx[j] = 0;
            if (!is_lead[j]) continue;
            if (rank[j] < nslot) {
                myidx[j] = c * kTailSlots + rank[j];
                m.tail_st[myidx[j]] = (uint16_t)e[j];
            } else {
                myidx[j] = base + (rank[j] - nslot);
                m.out_list[myidx[j]] = make_uint2(c, e[j]);
                myidx[j] += m.next_off;
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kR1Slots; ++j) {
            // the leader's index, from its slot and lane
            uint32_t li = 0;
            const uint32_t ql = lead[j] == kNone ? 0u : lead[j];
#pragma unroll
            for (uint32_t jj = 0; jj < kR1Slots; ++jj) {
                const uint32_t v = __shfl(myidx[jj], (int)(ql & (kWave2 - 1)));
                if ((ql >> 6) == jj) li = v;
            }
            if (valid[j]) m.out_lo[f0 + j * kWave2 + lane] = act[j] ? li : (kDone | e[j]);
        }
    }
}

// Map entries of merged walks: pair P follows its leaders round by round to
// the walk that ran to the end (which stored the map entry), or to its own
// end state if its walk stopped early.
struct MergeMapArgs {
    const uint32_t *lo[kMaxRounds];
    uint32_t rounds;
};

// Four pairs per thread (256 apart, so loads stay coalesced): their leader
// chains are followed side by side, four dependent gathers in flight.
constexpr uint32_t kMergePer = 4;

__global__ __launch_bounds__(256) void k_merge_maps(Match2Args a, MergeMapArgs mm) {
    const uint32_t total = a.first[a.nch];
    const uint32_t base = blockIdx.x * blockDim.x * kMergePer + threadIdx.x;
    uint32_t v[kMergePer];
#pragma unroll
    for (uint32_t j = 0; j < kMergePer; ++j) {
        const uint32_t P = base + j * blockDim.x;
        v[j] = P < total ? mm.lo[0][P] : (kDone | kMapped);
    }
    for (uint32_t k = 1; k < mm.rounds; ++k) {
#pragma unroll
        for (uint32_t j = 0; j < kMergePer; ++j)
            if (!(v[j] & kDone)) v[j] = mm.lo[k][v[j]];
    }
#pragma unroll
    for (uint32_t j = 0; j < kMergePer; ++j) {
        const uint32_t P = base + j * blockDim.x;
        if (P >= total) continue;
        if ((v[j] & (kDone | kMapped)) == (kDone | kMapped)) {
            a.maps[P] = (uint16_t)(v[j] & 0xFFFFu);
            continue;
        }
        // a walk that stopped before the last round: its end state
        const uint32_t e = (v[j] & kDone) ? (v[j] & 0x7FFFu) : 0xFFFFu;   // 0xFFFF: not reached
        const uint32_t tile = P / a.tile;
        const uint32_t ntiles = (total + a.tile - 1) / a.tile;
        const uint32_t lo0 = a.tile_first[tile];
        const uint32_t hi0 = tile + 1 < ntiles ? a.tile_first[tile + 1] + 1 : a.nch;
        const uint32_t c = owner_chunk(a.first, lo0, hi0, P);
        a.maps[P] = e < a.d.nq ? map_entry(a, c, e) : kBadPos;
    }
}

// ---------------------------------------------------------------------------
// One chunk per lane with merged walks (interleaved code streams).  The lane
// walks its chunk's start states four at a time over the first `prefix`
// codes and keeps the distinct states reached (at most kCwDistinct; each
// pair's map entry temporarily holds the index of its state); since the
// walks of one chunk converge, it then walks only those to the chunk's end,
// four chains (or fewer) in step, and rewrites every pair's map entry from
// its state's end.  A chunk whose
// states do not reduce that far is walked state by state to the end.  The
// 64 lanes of a wave hold 64 consecutive chunks, whose code blocks sit side
// by side in the interleaved stream, so each block load is one contiguous
// KiB.
// ---------------------------------------------------------------------------
constexpr uint32_t kCwDistinct = 4;

// Walk NS chains of one chunk over ncodes codes (whole 16-byte blocks from
// unit u0 on, `stride` units apart; the last block may be partial).  A lane
// walks one chunk, so one block lasts only 16 (or 8) steps: kCwAhead blocks
// are loaded ahead to cover the memory latency.  The raw input (L = 3) is
// read chunk by chunk, each lane from its own chunk: a lane's blocks are
// consecutive 16-byte pieces of its chunk.
constexpr uint32_t kCwAhead = 3;

template <int L, int NS>
__device__ __forceinline__ void walk_one_chunk(const uint4 *__restrict__ codes16, uint32_t u0,
                                               uint32_t stride, uint32_t ncodes,
                                               uint32_t (&st)[NS]) {
    constexpr uint32_t kPer16 = L == 2 ? 8u : 16u;
    constexpr uint32_t A = kCwAhead;
    const uint32_t whole = ncodes / kPer16;
    // ring slot k holds block b0 + k and is reloaded with block b0 + k + A
    // right after its last use; loads are issued without branches (see
    // walk_fast)
    auto walk_ring_block = [&](const uint4 &blk) {
        const uint32_t w4[4] = {blk.x, blk.y, blk.z, blk.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t w = word_codes<L>(w4[q]);
            if constexpr (L != 2) {
#pragma unroll
                for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<1, 0>(st[j], w));
#pragma unroll
                for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<1, 1>(st[j], w));
#pragma unroll
                for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<1, 2>(st[j], w));
#pragma unroll
                for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<1, 3>(st[j], w));
            } else {
#pragma unroll
                for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<2, 0>(st[j], w));
#pragma unroll
                for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<2, 1>(st[j], w));
            }
        }
    };
    if (whole) {
        const uint32_t lastb = whole - 1;
        uint4 ring[A];
#pragma unroll
        for (uint32_t k = 0; k < A; ++k) ring[k] = codes16[(size_t)u0 + (size_t)min(k, lastb) * stride];
        uint32_t b0 = 0;
        for (; b0 + A <= whole; b0 += A) {
#pragma unroll
            for (uint32_t k = 0; k < A; ++k) {
                walk_ring_block(ring[k]);
                ring[k] = codes16[(size_t)u0 + (size_t)min(b0 + k + A, lastb) * stride];
            }
        }
#pragma unroll
        for (uint32_t k = 0; k + 1 < A; ++k)
            if (b0 + k < whole) walk_ring_block(ring[k]);
    }
    const uint32_t rest = ncodes - whole * kPer16;
    if (rest) {
        // the last, partial block: a translated stream is padded to whole
        // blocks; raw input (L = 3) is read byte by byte up to its end
        uint32_t w4[4] = {0, 0, 0, 0};
        if constexpr (L == 3) {
            const uint8_t *p = reinterpret_cast<const uint8_t *>(codes16 + u0 + (size_t)whole * stride);
            for (uint32_t t = 0; t < rest; ++t) w4[t >> 2] |= (uint32_t)p[t] << (8 * (t & 3));
        } else {
            const uint4 v = codes16[(size_t)u0 + (size_t)whole * stride];
            w4[0] = v.x; w4[1] = v.y; w4[2] = v.z; w4[3] = v.w;
        }
        for (uint32_t t = 0; t < rest; ++t) {
            const uint32_t w = word_codes<L>(w4[t / (kPer16 / 4)]);
            const uint32_t code = L == 2 ? (w >> (16 * (t & 1))) & 0xFFFFu : (w >> (8 * (t & 3))) & 0xFFu;
#pragma unroll
            for (int j = 0; j < NS; ++j) st[j] = lds_ld(st[j] + code);
        }
    }
}

struct ChunkWalkArgs {
    uint32_t prefix;          // codes walked by every start state (multiple of 16)
};

// L = 3: the raw input (direct table) in its own order, 16-byte aligned,
// read by each lane from its chunk (stride 1); otherwise interleaved codes
// (stride 64).  Workgroups of up to 1024 threads: with a table of tens of
// KiB staged per workgroup, large workgroups keep 32 waves (32 x 64 walks)
// on each CU.
template <int L>
__global__ __launch_bounds__(1024, 8) void k_chunk_walk(Match2Args a, ChunkWalkArgs cw) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<L>(a.d, smem);
    constexpr uint32_t kPer16 = L == 2 ? 8u : 16u;
    constexpr uint32_t kSym = L == 4 ? 2u : 1u;
    const uint32_t R = L != 2 ? a.d.rowbytes : 2u;
    const uint4 *codes16 = reinterpret_cast<const uint4 *>(a.codes);
    const uint32_t stride = a.ilv_nblk ? 64u : 1u;
    const uint32_t per_chunk = (uint32_t)(a.chunk / (kPer16 * kSym));   // blocks per chunk
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < a.nch;
         c += gridDim.x * blockDim.x) {
        const uint32_t P0 = a.first[c];
        const uint32_t m = a.first[c + 1] - P0;
        if (m == 0) continue;
        const uint64_t len = min<uint64_t>(a.chunk, a.n - (uint64_t)c * a.chunk);
        const uint32_t ncodes = (uint32_t)((len + kSym - 1) / kSym);
        const uint32_t u0 = code_unit(a, c, 0u, per_chunk);
        const uint32_t pre = min(cw.prefix, ncodes);
        // phase 1: every start state over the prefix, four at a time
        uint32_t dst[kCwDistinct];
        uint32_t nd = 0;
        bool spill = false;
        for (uint32_t b0 = 0; b0 < m && !spill; b0 += 4) {
            uint32_t st[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                st[j] = R * (b0 + j < m ? pair_start(a, c, P0 + b0 + j) : pair_start(a, c, P0));
            walk_one_chunk<L, 4>(codes16, u0, stride, pre, st);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (b0 + j >= m) break;
                uint32_t idx = kCwDistinct;
                for (uint32_t t = 0; t < nd; ++t)
                    if (dst[t] == st[j]) idx = t;
                if (idx == kCwDistinct) {
                    if (nd == kCwDistinct) { spill = true; break; }
                    dst[nd] = st[j];
                    idx = nd++;
                }
                a.maps[P0 + b0 + j] = (uint16_t)idx;
            }
        }
        if (!spill) {
            // phase 2: the distinct states to the chunk's end
            const uint32_t rest = ncodes - pre;
            const uint32_t ur = u0 + (pre / kPer16) * stride;   // pre is whole blocks
            if (rest) {
                if (nd == 1) {
                    uint32_t st[1] = {dst[0]};
                    walk_one_chunk<L, 1>(codes16, ur, stride, rest, st);
                    dst[0] = st[0];
                } else if (nd == 2) {
                    uint32_t st[2] = {dst[0], dst[1]};
                    walk_one_chunk<L, 2>(codes16, ur, stride, rest, st);
                    dst[0] = st[0]; dst[1] = st[1];
                } else {
                    uint32_t st[4] = {dst[0], dst[1], nd > 2 ? dst[2] : dst[0], nd > 3 ? dst[3] : dst[0]};
                    walk_one_chunk<L, 4>(codes16, ur, stride, rest, st);
                    dst[0] = st[0]; dst[1] = st[1]; dst[2] = st[2]; dst[3] = st[3];
                }
            }
            uint16_t v[kCwDistinct];
            for (uint32_t t = 0; t < nd; ++t) v[t] = map_entry(a, c, dst[t] / R);
            for (uint32_t k = 0; k < m; ++k) a.maps[P0 + k] = v[a.maps[P0 + k] & 3u];
        } else {
            // the states did not reduce: every start state to the end
            for (uint32_t b0 = 0; b0 < m; b0 += 4) {
                uint32_t st[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    st[j] = R * (b0 + j < m ? pair_start(a, c, P0 + b0 + j) : pair_start(a, c, P0));
                walk_one_chunk<L, 4>(codes16, u0, stride, ncodes, st);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (b0 + j < m) a.maps[P0 + b0 + j] = map_entry(a, c, st[j] / R);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The last round of merged walks, one chunk per lane (MatchPlan::tail).  By
// the start of the last round the walks of a chunk have mostly met: the
// round before hands each chunk's remaining walks to this kernel (up to
// kTailSlots per chunk; more go to an overflow list).  Lane c walks chunk c's
// states from byte t0 to the chunk's end, reading the raw input: each byte
// becomes its code through a 256-entry table in LDS (an entry is the code,
// with kTailBad set for a byte outside Sigma).  The bytes a tail reads are
// validated here: the translation pass covered only every chunk's first t0
// bytes, so every lane whose chunk extends past t0 walks it, with no state
// if its walks all ended.  Walks of a lane that meet are merged at segment
// ends (2 t0, 4 t0, ...): a wavefront runs as many chains as its busiest
// lane (0, 1, 2, 4 or 8), mostly one.  A lane loads its chunk 64 bytes at a
// time (16 or 32 with four or eight chains), one group ahead.
// The byte table is held in kTailLutCopies copies, entry e of copy k at
// dword 32 e + k, and lane l reads copy l mod 32: the 32 lanes of a half
// wavefront then hit 32 distinct banks whatever bytes they read (random
// bytes on one copy would pile up on a few banks).
// The last wavefront of every workgroup walks the overflow list, one walk
// per lane, beside the chunk lanes (a lone overflow walk is as long as a
// chunk's tail; run after them it would add its whole length).
// ---------------------------------------------------------------------------
constexpr uint32_t kTailBad = 0x10000u;
constexpr uint32_t kTailChains = 8;     // chains a lane can run (= kTailSlots)
constexpr uint32_t kTailLutCopies = 32;
constexpr uint32_t kTailLutBytes = 256u * kTailLutCopies * 4u;   // 32 KiB
static_assert(kTailSlots == kTailChains, "a lane holds every slot of its chunk");

struct TailArgs {
    const uint8_t *in;         // the raw input (16-byte aligned)
    uint32_t t0;               // chunk bytes walked by the earlier rounds
    const uint32_t *cnt;       // [nch] walks handed over per chunk
    const uint16_t *st;        // [nch][kTailSlots] their states
    uint32_t *lo;              // the last round's outcomes: [nch][kTailSlots], then the
                               //  overflow list's places
    const uint32_t *ovf_cnt;   // [kRegions] overflow walks per region
    const uint2 *ovf_list;     // overflow walks {chunk, state} per place
    uint32_t cap;              // places per region
    uint32_t *bad;             // OR-ed with 1 when a byte outside Sigma is read
    uint32_t chunk_threads;    // threads per workgroup on chunks (the rest: overflow)
};

// 16 bytes: codes from the byte table (lut: this lane's copy), then 16
// steps of each of the NS chains (NS = 0: validation only).
template <int NS>
__device__ __forceinline__ void tail_piece(const uint4 &v, uint32_t lut,
                                           uint32_t (&st)[NS > 0 ? NS : 1], uint32_t &bad) {
    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            e[k] = lds_ld32(lut + (((w4[q] >> (8 * k)) & 0xFFu) << 7));
            bad |= e[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<2, 0>(st[j], e[k]));
    }
}

// Bytes [from, to) of the chunk at cb (from a multiple of 16; to = from
// when the lane has nothing to walk).
template <int NS>
__device__ __forceinline__ void tail_walk(const uint8_t *__restrict__ cb, uint32_t from, uint32_t to,
                                          uint32_t lut, uint32_t (&st)[NS > 0 ? NS : 1],
                                          uint32_t &bad) {
    const uint4 *p = reinterpret_cast<const uint4 *>(cb + from);
    // pieces per group: a lane's whole 64 bytes of a line half per load
    // group for one or two chains (parts of a line fetched by one group are
    // not evicted before the next group reads them), fewer for more chains
    constexpr uint32_t GP = NS >= 8 ? 1 : NS >= 4 ? 2 : 4;
    const uint32_t ng = (to - from) / (16 * GP);
    if (ng) {
        // ring of two groups: a group is reloaded right after its walk, so
        // the other group's walk covers the load
        const uint32_t lastg = ng - 1;
        uint4 ring[2][GP];
#pragma unroll
        for (uint32_t k = 0; k < 2; ++k)
#pragma unroll
            for (int h = 0; h < GP; ++h) ring[k][h] = p[min(k, lastg) * GP + h];
        uint32_t g0 = 0;
        for (; g0 + 2 <= ng; g0 += 2) {
#pragma unroll
            for (uint32_t k = 0; k < 2; ++k) {
#pragma unroll
                for (int h = 0; h < GP; ++h) tail_piece<NS>(ring[k][h], lut, st, bad);
                const uint32_t gn = min(g0 + k + 2, lastg);
#pragma unroll
                for (int h = 0; h < GP; ++h) ring[k][h] = p[gn * GP + h];
            }
        }
        if (g0 < ng) {
#pragma unroll
            for (int h = 0; h < GP; ++h) tail_piece<NS>(ring[0][h], lut, st, bad);
        }
    }
    uint32_t at = from + ng * 16 * GP;
    for (; at + 16 <= to; at += 16) tail_piece<NS>(*reinterpret_cast<const uint4 *>(cb + at), lut, st, bad);
    for (; at < to; ++at) {   // the input's last bytes
        const uint32_t e = lds_ld32(lut + ((uint32_t)cb[at] << 7));
        bad |= e;
#pragma unroll
        for (int j = 0; j < NS; ++j) st[j] = lds_ld(add_sel<2, 0>(st[j], e));
    }
}

// Two chunks side by side in one lane, one chain each: 16 bytes of each,
// their codes first, then the two chains' steps interleaved (two independent
// lookups in flight per step).
__device__ __forceinline__ void tail_piece2(const uint4 &va, const uint4 &vb, uint32_t lut,
                                            uint32_t &sa, uint32_t &sb, uint32_t &bad) {
    const uint32_t wa[4] = {va.x, va.y, va.z, va.w};
    const uint32_t wb[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t ea[4], eb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ea[k] = lds_ld32(lut + (((wa[q] >> (8 * k)) & 0xFFu) << 7));
            eb[k] = lds_ld32(lut + (((wb[q] >> (8 * k)) & 0xFFu) << 7));
            bad |= ea[k] | eb[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sa = lds_ld(add_sel<2, 0>(sa, ea[k]));
            sb = lds_ld(add_sel<2, 0>(sb, eb[k]));
        }
    }
}

// n16 16-byte pieces from pa and from pb (both 16-byte aligned), walked in
// lockstep; load groups of 64 bytes per chunk in a ring of two, as tail_walk.
__device__ __forceinline__ void tail_walk2(const uint8_t *__restrict__ pa, const uint8_t *__restrict__ pb,
                                           uint32_t n16, uint32_t lut, uint32_t &sa, uint32_t &sb,
                                           uint32_t &bad) {
    constexpr uint32_t GP = 4;
    const uint4 *qa = reinterpret_cast<const uint4 *>(pa);
    const uint4 *qb = reinterpret_cast<const uint4 *>(pb);
    const uint32_t ng = n16 / GP;
    if (ng) {
        const uint32_t lastg = ng - 1;
        uint4 ra[2][GP], rb[2][GP];
#pragma unroll
        for (uint32_t k = 0; k < 2; ++k)
#pragma unroll
            for (int h = 0; h < GP; ++h) {
                ra[k][h] = qa[min(k, lastg) * GP + h];
                rb[k][h] = qb[min(k, lastg) * GP + h];
            }
        uint32_t g0 = 0;
        for (; g0 + 2 <= ng; g0 += 2) {
#pragma unroll
            for (uint32_t k = 0; k < 2; ++k) {
#pragma unroll
                for (int h = 0; h < GP; ++h) tail_piece2(ra[k][h], rb[k][h], lut, sa, sb, bad);
                const uint32_t gn = min(g0 + k + 2, lastg);
#pragma unroll
                for (int h = 0; h < GP; ++h) {
                    ra[k][h] = qa[gn * GP + h];
                    rb[k][h] = qb[gn * GP + h];
                }
            }
        }
        if (g0 < ng) {
#pragma unroll
            for (int h = 0; h < GP; ++h) tail_piece2(ra[0][h], rb[0][h], lut, sa, sb, bad);
        }
    }
    for (uint32_t i = ng * GP; i < n16; ++i) tail_piece2(qa[i], qb[i], lut, sa, sb, bad);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

// Walk the lane's first `NS` chains of st over [from, to).
template <int NS>
__device__ __forceinline__ void tail_walk_first(const uint8_t *cb, uint32_t from, uint32_t to,
                                                uint32_t lut, uint32_t (&st)[kTailChains],
                                                uint32_t &bad) {
    uint32_t sn[NS > 0 ? NS : 1];
#pragma unroll
    for (int j = 0; j < (NS > 0 ? NS : 1); ++j) sn[j] = st[j];
    tail_walk<NS>(cb, from, to, lut, sn, bad);
#pragma unroll
    for (int j = 0; j < NS; ++j) st[j] = sn[j];
}

// The wave's chain count ns (wave-uniform; lanes with fewer chains repeat
// their first): 0, 1, 2, 4 or 8 chains.
__device__ __forceinline__ void tail_walk_n(uint32_t ns, const uint8_t *cb, uint32_t from,
                                            uint32_t to, uint32_t lut,
                                            uint32_t (&st)[kTailChains], uint32_t &bad) {
    if (ns == 0) tail_walk_first<0>(cb, from, to, lut, st, bad);
    else if (ns == 1) tail_walk_first<1>(cb, from, to, lut, st, bad);
    else if (ns == 2) tail_walk_first<2>(cb, from, to, lut, st, bad);
    else if (ns <= 4) tail_walk_first<4>(cb, from, to, lut, st, bad);
    else tail_walk_first<8>(cb, from, to, lut, st, bad);
}

// Chains that reached the same state become one: st[0 .. nl) keeps the
// distinct states in order (the rest repeat st[0]); map (4 bits per
// handed-over walk: the index of its chain) is updated.
__device__ __forceinline__ void tail_merge(uint32_t (&st)[kTailChains], uint32_t &nl,
                                           uint32_t &map) {
    constexpr int C = (int)kTailChains;
    uint32_t where[C], nst[C], k2 = 0;
#pragma unroll
    for (int q = 0; q < C; ++q) nst[q] = st[0];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        uint32_t f = 0xFFu;
#pragma unroll
        for (int i = 0; i < j; ++i)
            if (f == 0xFFu && (uint32_t)i < nl && st[i] == st[j]) f = where[i];
        if ((uint32_t)j < nl && f == 0xFFu) {
#pragma unroll
            for (int q = 0; q < C; ++q)
                if ((uint32_t)q == k2) nst[q] = st[j];
            f = k2++;
        }
        where[j] = f;
    }
    uint32_t m2 = 0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const uint32_t cur = (map >> (4 * k)) & 0xFu;
        uint32_t w = where[0];
#pragma unroll
        for (int j = 1; j < C; ++j)
            if (cur == (uint32_t)j) w = where[j];
        m2 |= (w & 0xFu) << (4 * k);
    }
#pragma unroll
    for (int q = 0; q < C; ++q) st[q] = nst[q];
    nl = k2;
    map = m2;
}

// A chunk's handed-over walks in the last round (two chunks per lane): chains
// st[0 .. nl) (the rest repeat st[0]), map (4 bits per walk: its chain), the
// position the chains stand at and the chunk's end.
__device__ __forceinline__ void tail_load(const Match2Args &a, const TailArgs &t, uint32_t c,
                                          uint32_t R, uint32_t (&st)[kTailChains], uint32_t &cnt,
                                          uint32_t &to) {
    const bool in = c < a.nch;
    const uint64_t len = in ? min<uint64_t>(a.chunk, a.n - (uint64_t)c * a.chunk) : 0u;
    to = len > t.t0 ? (uint32_t)len : t.t0;
    cnt = len > t.t0 ? min(t.cnt[c], kTailSlots) : 0u;
#pragma unroll
    for (int j = 0; j < (int)kTailChains; ++j) st[j] = 0;
    if (cnt) {
        const uint4 sv = reinterpret_cast<const uint4 *>(t.st)[c];   // kTailSlots == 8
        const uint32_t w4[4] = {sv.x, sv.y, sv.z, sv.w};
        const uint32_t s0 = w4[0] & 0xFFFFu;
#pragma unroll
        for (int j = 0; j < (int)kTailChains; ++j) {
            const uint32_t s = (w4[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
            st[j] = R * ((uint32_t)j < cnt ? s : s0);
        }
    }
}

// Segments [pos, 2 t0), [2 t0, 4 t0), ... while some lane of the wavefront
// has two chains or more; chains that meet become one at each segment's end.
// Returns with at most one chain in every lane that has bytes left.
__device__ __forceinline__ void tail_multi(const uint8_t *cb, uint32_t t0, uint32_t lut,
                                           uint32_t (&st)[kTailChains], uint32_t &nl, uint32_t &map,
                                           uint32_t &pos, uint32_t to, uint32_t &bad) {
    uint64_t seg = 2ull * t0;
    for (;;) {
        const uint32_t ns = wave_max(pos < to ? nl : 0u);
        if (ns <= 1) break;
        const uint32_t end = (uint32_t)min<uint64_t>(seg, to);
        const uint32_t lo = min(pos, to), hi = max(min(end, to), lo);
        if (ns == 2) tail_walk_first<2>(cb, lo, hi, lut, st, bad);
        else if (ns <= 4) tail_walk_first<4>(cb, lo, hi, lut, st, bad);
        else tail_walk_first<8>(cb, lo, hi, lut, st, bad);
        pos = max(pos, hi);
        tail_merge(st, nl, map);
        seg *= 2;
    }
}

// Outcomes of chunk c's walks whose chain has ended: those of chains other
// than the first once tail_multi returns, so that only the first chain's
// state stays live.  (The chain is picked by masks, not by index, which keeps
// st in registers.)
__device__ __forceinline__ void tail_store_others(const Match2Args &a, const TailArgs &t, uint32_t c,
                                                  uint32_t R, const uint32_t (&st)[kTailChains],
                                                  uint32_t cnt, uint32_t map) {
    for (uint32_t w = 0; w < cnt; ++w) {
        const uint32_t cur = (map >> (4 * w)) & 0xFu;
        if (cur == 0) continue;
        uint32_t s = 0;
#pragma unroll
        for (int j = 1; j < (int)kTailChains; ++j) s |= st[j] & (0u - (uint32_t)(cur == (uint32_t)j));
        t.lo[c * kTailSlots + w] = kDone | kMapped | map_entry(a, c, s / R);
    }
}

// ... and the first chain's walks, from its end state s0.  Nothing for a
// lane without walks: its chunk may lie past the last (c >= nch), where
// map_entry would read beyond the per-chunk arrays.
__device__ __forceinline__ void tail_store_first(const Match2Args &a, const TailArgs &t, uint32_t c,
                                                 uint32_t R, uint32_t cnt, uint32_t map, uint32_t s0) {
    if (cnt == 0) return;
    const uint32_t v = kDone | kMapped | map_entry(a, c, s0 / R);
    for (uint32_t w = 0; w < cnt; ++w)
        if (((map >> (4 * w)) & 0xFu) == 0) t.lo[c * kTailSlots + w] = v;
}

// K: chunks per lane (1 or 2; with 2, wavefront w takes chunks 128 w + lane
// and 128 w + 64 + lane, walked side by side once each has one chain left).
template <int L, int K>
__global__ __launch_bounds__(1024, K == 1 ? 5 : 4) void k_tail(Match2Args a, TailArgs t) {
    extern __shared__ __align__(16) uint8_t smem[];
    stage_table<L>(a.d, smem);
    uint32_t *lut_w = reinterpret_cast<uint32_t *>(smem + a.d.stab_bytes);
    uint32_t *region_pre = reinterpret_cast<uint32_t *>(smem + a.d.stab_bytes + kTailLutBytes);
    for (uint32_t i = threadIdx.x; i < 256u * kTailLutCopies; i += blockDim.x) {
        const uint16_t c = a.d.code[i / kTailLutCopies];
        lut_w[i] = c == kCodeInvalid ? kTailBad : (uint32_t)c;
    }
    // this lane's copy of the byte table
    const uint32_t lut = a.d.stab_bytes + 4u * (threadIdx.x % kTailLutCopies);
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t g = 0; g < kRegions; ++g) {
            region_pre[g] = acc;
            acc += t.ovf_cnt[g];
        }
        region_pre[kRegions] = acc;
    }
    __syncthreads();
    const uint32_t R = L == 1 ? a.d.rowbytes : 2u;
    const uint32_t CT = t.chunk_threads;
    uint32_t bad = 0;
    if (threadIdx.x < CT) {
        // lanes over chunks (the loop bound is uniform per wavefront: every
        // lane of a wavefront takes part in its shuffles)
        const uint32_t T = gridDim.x * CT * K;
        for (uint32_t c0 = (blockIdx.x * CT + (threadIdx.x & ~63u)) * K; c0 < a.nch; c0 += T) {
            const uint32_t c = c0 + (threadIdx.x & 63u);
            if (K == 1) {
                const bool in = c < a.nch;
                const uint64_t len = in ? min<uint64_t>(a.chunk, a.n - (uint64_t)c * a.chunk) : 0u;
                const uint32_t to = len > t.t0 ? (uint32_t)len : t.t0;
                const uint32_t cnt = len > t.t0 ? min(t.cnt[c], kTailSlots) : 0u;
                uint32_t st[kTailChains];
#pragma unroll
                for (int k = 0; k < (int)kTailChains; ++k) st[k] = 0;
                if (cnt) {
                    const uint4 sv = reinterpret_cast<const uint4 *>(t.st)[c];   // kTailSlots == 8
                    const uint32_t w4[4] = {sv.x, sv.y, sv.z, sv.w};
                    const uint32_t s0 = w4[0] & 0xFFFFu;
#pragma unroll
                    for (int k = 0; k < (int)kTailChains; ++k) {
                        const uint32_t s = (w4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
                        st[k] = R * ((uint32_t)k < cnt ? s : s0);
                    }
                }
                uint32_t nl = cnt, map = 0x76543210u;
                const uint8_t *cb = t.in + (uint64_t)c * a.chunk;
                uint32_t pos = t.t0;
                uint64_t seg = 2ull * t.t0;
                while (__any(pos < to)) {
                    const uint32_t ns = wave_max(pos < to ? nl : 0u);
                    const uint32_t end = ns <= 1 ? to : (uint32_t)min<uint64_t>(seg, to);
                    const uint32_t lo = min(pos, to), hi = max(min(end, to), lo);
                    tail_walk_n(ns, cb, lo, hi, lut, st, bad);
                    pos = max(pos, hi);
                    if (ns > 1) tail_merge(st, nl, map);
                    seg *= 2;
                }
                for (uint32_t k = 0; k < cnt; ++k) {
                    const uint32_t cur = (map >> (4 * k)) & 0xFu;
                    uint32_t s = st[0];
#pragma unroll
                    for (int j = 1; j < (int)kTailChains; ++j)
                        if (cur == (uint32_t)j) s = st[j];
                    t.lo[c * kTailSlots + k] = kDone | kMapped | map_entry(a, c, s / R);
                }
            } else {
                const uint8_t *cb = t.in + (uint64_t)c * a.chunk;
                const uint32_t c2 = c + 64u;
                const uint8_t *cb2 = t.in + (uint64_t)c2 * a.chunk;
                uint32_t sa, pa, ta, na, ma;
                {
                    uint32_t st[kTailChains], nl;
                    tail_load(a, t, c, R, st, na, ta);
                    nl = na;
                    ma = 0x76543210u;
                    pa = t.t0;
                    tail_multi(cb, t.t0, lut, st, nl, ma, pa, ta, bad);
                    tail_store_others(a, t, c, R, st, na, ma);
                    sa = st[0];
                    pa = min(pa, ta);
                }
                uint32_t sb, pb, tb, nb, mb;
                {
                    uint32_t st[kTailChains], nl;
                    tail_load(a, t, c2, R, st, nb, tb);
                    nl = nb;
                    mb = 0x76543210u;
                    pb = t.t0;
                    tail_multi(cb2, t.t0, lut, st, nl, mb, pb, tb, bad);
                    tail_store_others(a, t, c2, R, st, nb, mb);
                    sb = st[0];
                    pb = min(pb, tb);
                }
                // one chain each (a lane without walks keeps a dummy chain
                // that only validates bytes): both chunks side by side, then
                // what one has left alone
                const uint32_t n = min(ta - pa, tb - pb) / 16u * 16u;
                tail_walk2(cb + pa, cb2 + pb, n / 16u, lut, sa, sb, bad);
                uint32_t s1[1] = {sa}, s2[1] = {sb};
                if (pa + n < ta) tail_walk<1>(cb, pa + n, ta, lut, s1, bad);
                if (pb + n < tb) tail_walk<1>(cb2, pb + n, tb, lut, s2, bad);
                tail_store_first(a, t, c, R, na, ma, s1[0]);
                tail_store_first(a, t, c2, R, nb, mb, s2[0]);
            }
        }
    } else {
        // the overflow list, one walk per lane
        const uint32_t total = region_pre[kRegions];
        const uint32_t T = gridDim.x * 64u;
        for (uint32_t w = blockIdx.x * 64u + (threadIdx.x - CT); w < total; w += T) {
            uint32_t lo = 0, hi = kRegions;
            while (hi > lo + 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (region_pre[mid] <= w) lo = mid; else hi = mid;
            }
            const uint32_t place = lo * t.cap + (w - region_pre[lo]);
            const uint2 rec = t.ovf_list[place];
            const uint32_t c = rec.x;
            const uint32_t len = (uint32_t)min<uint64_t>(a.chunk, a.n - (uint64_t)c * a.chunk);
            uint32_t s1[1] = {R * rec.y};
            tail_walk<1>(t.in + (uint64_t)c * a.chunk, t.t0, len, lut, s1, bad);
            t.lo[a.nch * kTailSlots + place] = kDone | kMapped | map_entry(a, c, s1[0] / R);
        }
    }
    if (__any(bad & kTailBad) && (threadIdx.x & 63u) == 0) atomicOr(t.bad, 1u);
}

// Block map output (a shard matched from its lookahead set): entry p of the
// composed top-level map belongs to chunk 0's p-th start state; it holds
// kTerm | the state at the shard's end, or names no state (kBadPos: the walk
// from that start state met a chunk start outside the next chunk's set).
// rec: the combine's result record (its flags carry bytes outside Sigma).
struct BlockOut {
    uint32_t *info;          // [4]: entries, flags, chunks, 0
    uint16_t *start;         // [max]
    uint16_t *end;           // [max]; 0xFFFF = no state
    uint32_t max;
};

__global__ __launch_bounds__(256) void k_block_out(Match2Args a, const uint16_t *__restrict__ top,
                                                   const uint16_t *__restrict__ top_msize,
                                                   const uint32_t *__restrict__ rec, BlockOut bo) {
    const uint32_t m0 = top_msize ? (top_msize[0] & 0x7FFFu) : a.first[1];
    const uint32_t n = min(m0, bo.max);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        bo.start[p] = (uint16_t)pair_start(a, 0, p);
        const uint32_t v = top[p];
        bo.end[p] = (v & kTerm) && (v & 0x7FFFu) < a.d.nq ? (uint16_t)(v & 0x7FFFu) : (uint16_t)0xFFFFu;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bo.info[0] = m0;
        bo.info[1] = rec[2] & DFA_FLAG_SYMBOL;
        bo.info[2] = a.nch;
        bo.info[3] = 0;
    }
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

// Readout of the level-0 maps in the caller's numbering (test and
// diagnostic use): out_first[i] = first pair of chunk i (out_first[nch] =
// number of pairs); for pair P < cap: its start state and the end state its
// walk reached, delta*(start, chunk) (Section 4.1's L_i[j]).  An entry that
// names no state of the next chunk's set reads 0xFFFF.
struct MapOut {
    uint32_t *first;
    uint16_t *start;
    uint16_t *end;
    uint64_t cap;
};

__global__ __launch_bounds__(256) void k_decode_maps(Match2Args a, MapOut mo) {
    const uint32_t total = a.first[a.nch];
    const uint32_t P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P <= a.nch) mo.first[P] = a.first[P];
    if (P >= total || P >= mo.cap) return;
    const uint32_t tile = P / a.tile;
    const uint32_t ntiles = (total + a.tile - 1) / a.tile;
    const uint32_t lo0 = a.tile_first[tile];
    const uint32_t hi0 = tile + 1 < ntiles ? a.tile_first[tile + 1] + 1 : a.nch;
    const uint32_t c = owner_chunk(a.first, lo0, hi0, P);
    const uint32_t v = a.maps[P];
    uint32_t e = 0xFFFFu;
    if (v == kBadPos) {
        e = 0xFFFFu;
    } else if (v & kTerm) {
        e = v & 0x7FFFu;
    } else if (c + 1 < a.nch && v < a.first[c + 2] - a.first[c + 1]) {
        e = pair_start(a, c + 1, a.first[c + 1] + v);
    }
    mo.start[P] = (uint16_t)pair_start(a, c, P);
    mo.end[P] = (uint16_t)e;
}

// ---------------------------------------------------------------------------
namespace {
template <int SRC>
void launch_scan(const MatchPlan &p, const ScanSrc &q, const PackedBufs &b, uint16_t *flag_msize,
                 uint32_t start, hipStream_t s, const InfoSrc *info = nullptr) {
    const uint32_t nsb = (p.nch + kScanBlock - 1) / kScanBlock;
    ScanSrc qq = q;
    qq.tile = kWave2 * p.slots;
    if (info)
        hipLaunchKernelGGL(k_scan_sums_info, dim3(nsb), dim3(kScanThreads), 0, s, qq, *info, b.bsum);
    else
        hipLaunchKernelGGL(k_scan_sums<SRC>, dim3(nsb), dim3(kScanThreads), 0, s, qq, b.bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, b.bsum, nsb, flag_msize,
                       p.nch, b.block_bad, flag_msize ? p.tblocks : 0u, b.first, b.cnt,
                       b.cnt ? kMaxRounds * kRegions : 0u);
    hipLaunchKernelGGL(k_scan_apply<SRC>, dim3(nsb), dim3(kScanThreads), 0, s, qq, b.bsum, b.first,
                       b.tile_first, b.members, start);
}
}  // namespace

namespace {
const void *match2_kernel(uint32_t L, uint32_t slots, bool ex) {
#define DFA_MK(l) {{reinterpret_cast<const void *>(&k_match2<l, 2, false>),      \
                    reinterpret_cast<const void *>(&k_match2<l, 2, true>)},       \
                   {reinterpret_cast<const void *>(&k_match2<l, 4, false>),      \
                    reinterpret_cast<const void *>(&k_match2<l, 4, true>)}}
    static const void *const tab[4][2][2] = {DFA_MK(1), DFA_MK(2), DFA_MK(3), DFA_MK(4)};
#undef DFA_MK
    return tab[L - 1][slots >= 4 ? 1 : 0][ex ? 1 : 0];
}
const void *chunk_walk_kernel(uint32_t L) {
    static const void *const tab[4] = {
        reinterpret_cast<const void *>(&k_chunk_walk<1>), reinterpret_cast<const void *>(&k_chunk_walk<2>),
        reinterpret_cast<const void *>(&k_chunk_walk<3>), reinterpret_cast<const void *>(&k_chunk_walk<4>)};
    return tab[L - 1];
}
const void *tail_kernel(uint32_t L, uint32_t K) {
    static const void *const tab[2][2] = {
        {reinterpret_cast<const void *>(&k_tail<1, 1>), reinterpret_cast<const void *>(&k_tail<1, 2>)},
        {reinterpret_cast<const void *>(&k_tail<2, 1>), reinterpret_cast<const void *>(&k_tail<2, 2>)}};
    return tab[L == 1 ? 0 : 1][K >= 2 ? 1 : 0];
}
const void *round_kernel(uint32_t L, uint32_t slots, bool ex) {
#define DFA_RK(l) {{reinterpret_cast<const void *>(&k_round<l, 2, false>),      \
                    reinterpret_cast<const void *>(&k_round<l, 2, true>)},       \
                   {reinterpret_cast<const void *>(&k_round<l, 4, false>),      \
                    reinterpret_cast<const void *>(&k_round<l, 4, true>)}}
    static const void *const tab[4][2][2] = {DFA_RK(1), DFA_RK(2), DFA_RK(3), DFA_RK(4)};
#undef DFA_RK
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
                  hipEvent_t ev_before_matcher, hipEvent_t ev_kern_begin,
                  hipEvent_t ev_kern_end) {
    // events around the plan's longest single matcher launch (timing only)
    auto mark = [&](hipEvent_t ev) -> int {
        if (!ev) return DFA_OK;
        const hipError_t er = hipEventRecord(ev, s);
        return er == hipSuccess ? DFA_OK : hip_fail(er, "hipEventRecord");
    };
    // two-symbol steps (the plan checked the chunk length); else direct
    // tables: the matcher reads the (16-byte aligned) input itself
    const bool pairs = p.pairs && d->dev.pairs;
    const bool direct = !pairs && !p.ilv_nblk && d->dev.direct && p.lookahead != 2 &&
                        (reinterpret_cast<uintptr_t>(d_in) & 15u) == 0;
    const Ilv ilv{p.ilv_nblk, p.nch, p.chunk};
    if (p.ilv_nblk && p.chunk % 32 != 0)
        return fail(DFA_E_INVAL, "interleaved codes with odd chunks");
    const uint32_t L = pairs ? 4u : direct ? 3u : d->dev.layout;
    if (pairs && (p.chunk % 32 != 0 || p.lookahead == 2))
        return fail(DFA_E_INVAL, "two-symbol plan with a window pass or odd chunks");
    // Scan of the start-set sizes.  With precomputed sets the translation
    // pass's workgroups also run the scan's first phase (the lookahead sets
    // from the raw input) before they translate, and one pass finishes the
    // scan; the window pass needs the three-phase scan.
    ScanSrc q{msize, b.bits, p.bitmap_words, p.nch, kWave2 * p.slots};
    const InfoSrc info{d->dev, d_in, p.chunk, p.lookahead, p.r, b.ccls, b.cset, p.before};
    const bool fused_scan = p.lookahead != 2;
    const uint32_t nsb = match2_scan_blocks(p.nch);
    {
        const SumsArgs sa{q, info, b.bsum, fused_scan ? nsb : 0u};
        if (pairs && d->dev.pcode2)
            hipLaunchKernelGGL(k_translate_pairs_direct, dim3(p.tblocks), dim3(256), 0, s, d_in, p.n,
                               d->dev.pcode2, (uint8_t *)b.codes, b.block_bad, ilv, sa);
        else if (pairs)
            hipLaunchKernelGGL(k_translate_pairs, dim3(p.tblocks), dim3(256), 0, s, d_in, p.n,
                               d->dev.pcode, d->dev.nclass, (uint8_t *)b.codes, b.block_bad, ilv,
                               sa);
        else if (direct)
            hipLaunchKernelGGL((k_translate<uint8_t, false>), dim3(p.tblocks), dim3(256), 0, s, d_in,
                               p.n, d->dev.code, (uint8_t *)nullptr, b.block_bad, ilv, sa);
        else if (L == 1)
            hipLaunchKernelGGL(k_translate<uint8_t>, dim3(p.tblocks), dim3(256), 0, s, d_in, p.n,
                               d->dev.code, (uint8_t *)b.codes, b.block_bad, ilv, sa);
        else
            hipLaunchKernelGGL(k_translate<uint16_t>, dim3(p.tblocks), dim3(256), 0, s, d_in, p.n,
                               d->dev.code, (uint16_t *)b.codes, b.block_bad, ilv, sa);
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
    a.raw = d_in;
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
    a.tile = kWave2 * p.slots;
    a.ilv_nblk = p.ilv_nblk;
    a.spread = p.threads2 >= 1024 ? 1u : 0u;
    a.before = p.before;
    const size_t lds = a.d.stab_bytes;
    if (p.lookahead == 2) {
        // window pairs (chunk, state of I_sigma_1) -> start-set bitmaps -> member lists
        hipLaunchKernelGGL(k_chunkinfo_w, dim3((p.nch + 255) / 256), dim3(256), 0, s, d->dev, d_in,
                           p.chunk, p.nch, p.r, p.bitmap_words, msize, b.cset, b.bits, b.tail_cnt);
        launch_scan<0>(p, q, b, nullptr, start, s);
        const void *wf = window2_kernel(L, p.slots);
        void *wargs[] = {&a};
        hipError_t we = hipLaunchKernel(wf, dim3(p.blocks2), dim3(p.threads2), wargs, lds, s);
        if (we != hipSuccess) return hip_fail(we, "k_window2 launch");
        launch_scan<1>(p, q, b, nullptr, start, s);
    } else {
        hipLaunchKernelGGL(k_scan_finish, dim3(nsb), dim3(kScanThreads), 0, s, q, b.bsum, b.first,
                           b.tile_first, b.cnt, b.cnt ? kMaxRounds * kRegions : 0u, b.tail_cnt);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "packed-matcher preparation launch");
    if (ev_before_matcher) {
        e = hipEventRecord(ev_before_matcher, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (p.chunk_lanes) {
        // (interleaved codes, the raw input, or a linear code stream when a
        // direct table's input is not 16-byte aligned)
        if (p.lookahead == 2)
            return fail(DFA_E_INVAL, "chunk lanes need precomputed start sets");
        ChunkWalkArgs cw{kRound1Bytes};
        void *cargs[] = {&a, &cw};
        const uint32_t tpb = p.threads2;
        const uint32_t blocks =
            std::max<uint32_t>(1u, std::min<uint32_t>((p.nch + tpb - 1) / tpb, p.blocks2));
        if (int rc = mark(ev_kern_begin)) return rc;
        e = hipLaunchKernel(chunk_walk_kernel(L), dim3(blocks), dim3(tpb), cargs, lds, s);
        if (e != hipSuccess) return hip_fail(e, "k_chunk_walk launch");
        if (int rc = mark(ev_kern_end)) return rc;
    } else if (p.rounds > 1) {
        if (p.early_exit || p.chunk % 32 != 0 || !b.cnt)
            return fail(DFA_E_INVAL, "merged walks need no early exit and chunks of 32k");
        if (p.tail && (!b.tail_cnt || (L != 1 && L != 2) || p.tail_t0 % 32 != 0))
            return fail(DFA_E_INVAL, "one-chunk-per-lane last round: plan and buffers disagree");
        const void *rf = round_kernel(L, p.slots, a.d.nabs > 0);
        // with a one-chunk-per-lane last round the wave-tile rounds stop one
        // round early; the last of them hands its walks to k_tail
        const uint32_t tiled = p.tail ? p.rounds - 1 : p.rounds;
        for (uint32_t k = 0; k < tiled; ++k) {
            RoundArgs m;
            m.t0 = k == 0 ? 0u : kRound1Bytes << (2 * (k - 1));
            m.t1 = kRound1Bytes << (2 * k);
            m.first_round = k == 0;
            m.last_round = k + 1 == p.rounds;
            m.cap = round_region_cap(p);
            m.in_cnt = k ? b.cnt + (size_t)k * kRegions : nullptr;
            m.in_list = k ? b.list[k] : nullptr;
            m.out_lo = b.lo[k];
            m.out_list = m.last_round ? nullptr : b.list[k + 1];
            m.out_cnt = m.last_round ? nullptr : b.cnt + (size_t)(k + 1) * kRegions;
            const bool hand = p.tail && k + 1 == tiled;
            m.tail_cnt = hand ? b.tail_cnt : nullptr;
            m.tail_st = hand ? b.tail_st : nullptr;
            m.next_off = hand ? p.nch * kTailSlots : 0u;
            void *rargs[] = {&a, &m};
            const bool timed = !p.tail && k + 1 == tiled;
            if (timed)
                if (int rc = mark(ev_kern_begin)) return rc;
            const bool chunk_major = k == 0 && p.round1c && (L == 1 || L == 2) && m.t1 == 32u;
            const void *kf = chunk_major ? (L == 1 ? reinterpret_cast<const void *>(&k_round1c<1>)
                                                   : reinterpret_cast<const void *>(&k_round1c<2>))
                                         : rf;
            uint32_t kthreads = p.threads2, kblocks = p.blocks2;
            if (chunk_major) {
                // workgroups sized so that as many wavefronts as the kernel's
                // registers and the staged table allow are resident at once
                // (its waves loop over chunks, so a workgroup that cannot be
                // resident only waits); cached per kernel and table size
                static std::mutex mu;
                static std::map<std::pair<const void *, size_t>, std::pair<uint32_t, uint32_t>> cache;
                std::lock_guard<std::mutex> lk(mu);
                auto it = cache.find({kf, lds});
                if (it == cache.end()) {
                    int best_res = 0;
                    std::pair<uint32_t, uint32_t> pick{p.threads2, p.blocks2};
                    for (uint32_t t = 1024; t >= 256; t -= 64) {
                        int nb = 0;
                        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kf, (int)t,
                                                                         lds + round_lds_bytes(t)) != hipSuccess)
                            break;
                        if (nb > 0 && nb * (int)t > best_res) {
                            best_res = nb * (int)t;
                            pick = {t, (uint32_t)(nb * device_cu_count())};
                        }
                    }
                    it = cache.emplace(std::make_pair(kf, lds), pick).first;
                }
                kthreads = it->second.first;
                kblocks = it->second.second;
            }
            e = hipLaunchKernel(kf, dim3(kblocks), dim3(kthreads), rargs,
                                lds + round_lds_bytes(kthreads), s);
            if (e != hipSuccess) return hip_fail(e, "k_round launch");
            if (timed)
                if (int rc = mark(ev_kern_end)) return rc;
        }
        if (p.tail) {
            const uint32_t last = p.rounds - 1;
            TailArgs t{d_in, p.tail_t0, b.tail_cnt, b.tail_st, b.lo[last], b.cnt + (size_t)last * kRegions,
                       b.list[last], round_region_cap(p), b.block_bad, p.tail_threads};
            const size_t tl = lds + kTailLutBytes + round_lds_extra();
            void *targs[] = {&a, &t};
            if (int rc = mark(ev_kern_begin)) return rc;
            e = hipLaunchKernel(tail_kernel(L, p.tail_k), dim3(p.tail_blocks), dim3(p.tail_threads + 64u), targs,
                                tl, s);
            if (e != hipSuccess) return hip_fail(e, "k_tail launch");
            if (int rc = mark(ev_kern_end)) return rc;
        }
        MergeMapArgs mm{};
        for (uint32_t k = 0; k < p.rounds; ++k) mm.lo[k] = b.lo[k];
        mm.rounds = p.rounds;
        const uint64_t bound = (uint64_t)p.max_tiles * kWave2 * p.slots;
        hipLaunchKernelGGL(k_merge_maps, dim3((uint32_t)((bound + 256 * kMergePer - 1) / (256 * kMergePer))),
                           dim3(256), 0, s, a, mm);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "k_merge_maps launch");
    } else {
        void *args[] = {&a};
        if (int rc = mark(ev_kern_begin)) return rc;
        e = hipLaunchKernel(match2_kernel(L, p.slots, p.early_exit), dim3(p.blocks2),
                            dim3(p.threads2), args, lds, s);
        if (e != hipSuccess) return hip_fail(e, "k_match2 launch");
        if (int rc = mark(ev_kern_end)) return rc;
    }
    if (b.out_first) {
        // readout of the level-0 maps: one thread per chunk boundary and pair
        const uint64_t bound = std::max<uint64_t>((uint64_t)p.max_tiles * kWave2 * p.slots,
                                                  (uint64_t)p.nch + 1);
        const MapOut mo{b.out_first, b.out_start, b.out_end, b.out_cap};
        hipLaunchKernelGGL(k_decode_maps, dim3((uint32_t)((bound + 255) / 256)), dim3(256), 0, s,
                           a, mo);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "k_decode_maps launch");
    }
    return DFA_OK;
}

int launch_block_out(const dfa *d, uint32_t start, const MatchPlan &p, const PackedBufs &b,
                     const uint16_t *maps, const uint16_t *msize, const uint32_t *rec,
                     uint32_t *info, uint16_t *out_start, uint16_t *out_end, uint32_t max,
                     hipStream_t s) {
    Match2Args a{};
    a.d = d->dev;
    a.n = p.n;
    a.chunk = p.chunk;
    a.nch = p.nch;
    a.start = start;
    a.mode = p.lookahead;
    a.r = p.r;
    a.first = b.first;
    a.ccls = b.ccls;
    a.cset = b.cset;
    a.members = b.members;
    a.before = p.before;
    const uint16_t *top = maps + p.level_off[p.levels];
    const uint16_t *top_msize = p.levels ? msize + p.msize_off[p.levels] : nullptr;
    const BlockOut bo{info, out_start, out_end, max};
    hipLaunchKernelGGL(k_block_out, dim3((std::max<uint32_t>(max, 1u) + 255) / 256), dim3(256), 0, s,
                       a, top, top_msize, rec, bo);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "k_block_out launch");
}

// Ordered composition of block maps (Eq. 9 over shards): one wavefront
// follows the state from block to block, each lane searching a slice of the
// block's start states.
__global__ __launch_bounds__(64) void k_compose_blocks(DevDFA d, uint32_t count,
                                                       const uint32_t *__restrict__ infos,
                                                       const uint16_t *__restrict__ starts,
                                                       const uint16_t *__restrict__ ends,
                                                       uint32_t max, uint32_t start,
                                                       uint32_t *__restrict__ result,
                                                       uint32_t *__restrict__ states) {
    const uint32_t lane = threadIdx.x;
    uint32_t s = start, flags = 0, chunks = 0;
    if (states && lane == 0) states[0] = s;
    for (uint32_t g = 0; g < count; ++g) {
        const uint32_t *inf = infos + 4ull * g;
        flags |= inf[1] & DFA_FLAG_SYMBOL;
        chunks += inf[2];
        if (!flags) {
            const uint32_t m = min(inf[0], max);
            uint32_t hit = 0xFFFFFFFFu;
            for (uint32_t p = lane; p < m; p += 64)
                if (starts[(size_t)g * max + p] == s) hit = p;
            const uint64_t mask = __ballot(hit != 0xFFFFFFFFu);
            if (mask) {
                const uint32_t p = __shfl(hit, (int)(__ffsll((unsigned long long)mask) - 1));
                const uint32_t e = ends[(size_t)g * max + p];
                if (e < d.nq) s = e; else flags |= DFA_FLAG_SPECULATION;
            } else {
                flags |= DFA_FLAG_SPECULATION;
            }
        }
        if (states && lane == 0) states[g + 1] = flags ? 0xFFFFFFFFu : s;
    }
    if (lane == 0) {
        const bool ok = flags == 0;
        result[0] = ok ? s : 0xFFFFFFFFu;
        result[1] = ok ? (d.accept_bits[s >> 5] >> (s & 31)) & 1u : 0u;
        result[2] = flags;
        result[3] = chunks;
    }
}

int launch_compose_blocks(const dfa *d, uint32_t count, const uint32_t *infos,
                          const uint16_t *starts, const uint16_t *ends, uint32_t max,
                          uint32_t start, uint32_t *result, uint32_t *states, hipStream_t s) {
    hipLaunchKernelGGL(k_compose_blocks, dim3(1), dim3(64), 0, s, d->dev, count, infos, starts, ends,
                       max, start, result, states);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "k_compose_blocks launch");
}

int launch_size_scan(uint32_t nch, uint16_t *msize, uint32_t *bsum, uint32_t *first,
                     uint32_t *tile_first, uint32_t tile, hipStream_t s) {
    if (nch == 0) return DFA_OK;
    const uint32_t nsb = (nch + kScanBlock - 1) / kScanBlock;
    ScanSrc q{msize, nullptr, 0, nch, tile};
    hipLaunchKernelGGL(k_scan_sums<0>, dim3(nsb), dim3(kScanThreads), 0, s, q, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, bsum, nsb,
                       (uint16_t *)nullptr, nch, (const uint32_t *)nullptr, 0u, first,
                       (uint32_t *)nullptr, 0u);
    hipLaunchKernelGGL(k_scan_apply<0>, dim3(nsb), dim3(kScanThreads), 0, s, q, bsum, first,
                       tile_first, (uint16_t *)nullptr, 0u);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "size scan launch");
}

int launch_down0(const MatchPlan &p, const uint16_t *maps0, const uint32_t *first,
                 const uint16_t *bv_up, uint16_t *bv0, hipStream_t s) {
    const uint32_t n_up = p.levels >= 1 ? p.level_count[1] : 1u;
    const uint32_t G = p.levels >= 1 ? p.group_l[0] : 1u;
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
                         chunk_walk_kernel(1), chunk_walk_kernel(2), chunk_walk_kernel(3),
                         chunk_walk_kernel(4), reinterpret_cast<const void *>(&k_round1c<1>),
                         reinterpret_cast<const void *>(&k_round1c<2>), tail_kernel(1, 1), tail_kernel(2, 1),
                         tail_kernel(1, 2), tail_kernel(2, 2),
                         round_kernel(1, 2, false), round_kernel(1, 4, false),
                         round_kernel(2, 2, false), round_kernel(2, 4, false),
                         round_kernel(3, 2, false), round_kernel(3, 4, false),
                         round_kernel(4, 2, false), round_kernel(4, 4, false),
                         round_kernel(1, 2, true), round_kernel(1, 4, true),
                         round_kernel(2, 2, true), round_kernel(2, 4, true),
                         round_kernel(3, 2, true), round_kernel(3, 4, true),
                         round_kernel(4, 2, true), round_kernel(4, 4, true),
                         window2_kernel(1, 2), window2_kernel(1, 4),
                         window2_kernel(2, 2), window2_kernel(2, 4)};
    int rc = DFA_OK;
    for (const void *f : fns)
        if (allow_dynamic_lds(f, lds) != DFA_OK) rc = DFA_E_DEVICE;
    return rc;
}

uint32_t match2_tile_pairs(uint32_t slots) { return kWave2 * slots; }
size_t round_lds_extra() { return kRoundPreBytes; }
size_t round_lds_bytes(uint32_t threads) {
    return kRoundPreBytes + (size_t)(threads / kWave2) * kRoundHash * sizeof(uint32_t);
}
size_t tail_lut_bytes() { return kTailLutBytes; }
uint32_t round_region_cap(const MatchPlan &p) {
    // a region receives the leaders of every kRegions-th tile, at most a
    // tile's walks each (chunk-major first round: of every kRegions-th
    // chunk, at most a start set each)
    const uint64_t tiles = ((p.max_tiles + kRegions - 1) / kRegions) * kWave2 * p.slots;
    const uint64_t chunks = p.round1c ? ((uint64_t)p.nch + kRegions - 1) / kRegions * p.stride : 0u;
    return (uint32_t)std::max<uint64_t>(tiles, chunks);
}
uint32_t match2_scan_blocks(uint32_t nch) { return (nch + kScanBlock - 1) / kScanBlock; }

}  // namespace dfaspec
