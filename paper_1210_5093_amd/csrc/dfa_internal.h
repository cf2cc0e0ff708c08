// Internal declarations shared by the library's own translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "dfa_spec.h"

namespace dfaspec {

// Map-entry encoding (uint16).  A chunk's state map L_i (Section 4.1) is kept
// sparse: entry p belongs to the p-th state of the chunk's initial-state set.
// Its value is either the position of the end state in the next chunk's
// initial-state set (< 0x8000), or 0x8000 | state when the end state is
// absorbing or the chunk is the last one (the value then never changes).
constexpr uint16_t kTerm = 0x8000;
constexpr uint16_t kBadPos = 0xFFFF;      // "not in the next set": invariant violated
constexpr uint16_t kFlagSymbol = 0x8000;  // msize bit: chunk held a byte outside Sigma
constexpr uint32_t kLutInvalid = 0xFFFFFFFFu;
constexpr uint32_t kMaxStates = 32767;
constexpr uint32_t kMaxMsetLevel = 8;   // precomputed multi-symbol sets up to this r
constexpr uint16_t kCodeInvalid = 0xFFFF;
constexpr uint32_t kMaxRounds = 6;        // walk rounds with merging (DFA_MATCH_ROUNDS)
constexpr uint32_t kRound1Bytes = 32;     // bytes of the first round; x4 per later round
constexpr uint32_t kRegions = 64;         // regions (counters) of a round's walk list
constexpr uint32_t kTailSlots = 8;        // walks per chunk held for the one-chunk-per-lane
                                          // last round (more go to its overflow list)
// plan_match flags (not DFA_MATCH_* bits): the input is not 16-byte aligned;
// the plan is for a block map (the packed matcher, whatever the input size)
constexpr uint32_t kPlanUnaligned = 1u << 31;
constexpr uint32_t kPlanBlock = 1u << 30;

// Device-resident compiled DFA, passed by value to kernels.
struct DevDFA {
    const uint16_t *table;       // [K][Qp] class-major; entry = 2 * delta(s, c)
    const uint32_t *lut;         // [256]: (class << 24) | class * colstride; kLutInvalid
    const uint32_t *set_off[2];  // [K+1] per lookahead mode (0: all states, 1: I_c)
    const uint16_t *set_st[2];   // states of each class's set, ascending
    const uint16_t *pos[2];      // [K][Q]: position of s in the class's set,
                                 //  kTerm|s for absorbing s, kBadPos otherwise
    const uint32_t *accept_bits; // ceil(Q/32) words
    // Packed-pair matcher: per-byte stream codes and the table they index.
    //  layout 1 (state-major): code = 2 * class; stab[s][c] = R * delta(s, c),
    //           R = row bytes; an LDS address is R * s + code.
    //  layout 2 (class-major): code = class * colstride; the table is `table`
    //           (entries 2 * delta); an LDS address is code + 2 * s.
    //  direct (a layout-1 variant for alphabets of bytes below 128): rows are
    //           indexed by the byte itself, code = 2 * byte, so the matcher
    //           derives codes from the raw input ((w & 0x7F7F7F7F) << 1 per
    //           word) and needs no translation pass.  Row s starts at R * s;
    //           entry (s, b) sits at R * s + 2 * b (rows overlap outside the
    //           bytes of Sigma; every address R * s + c, c even <= 254, holds a
    //           valid state offset, so a walk over an invalid byte stays in the
    //           table while the validation pass reports the byte).
    // Multi-symbol initial-state sets I_{c_1..c_k} (Eq. 13) over class strings,
    // k = 1..r0; set id = c_1 K^(k-1) + ... + c_k; level k's offsets start at
    // mset_off[moff[k]], its states at mset_st[mst[k]] (sorted ascending).
    const uint32_t *mset_off;
    const uint16_t *mset_st;
    uint32_t moff[kMaxMsetLevel + 1];
    uint32_t mst[kMaxMsetLevel + 1];
    uint32_t r0;
    const uint16_t *code;        // [256]; kCodeInvalid for bytes outside Sigma
    const uint16_t *stab;        // layout 1 table (nq rows of R bytes)
    uint32_t layout;             // 0 = packed matcher unavailable, 1, 2
    uint32_t direct;             // layout 1 with byte-indexed rows (see above)
    uint32_t rowbytes;           // R (layout 1)
    uint32_t stab_bytes;         // bytes staged for the packed matcher, multiple of 16:
                                 //  the table (stab for layout 1, a copy of `table`
                                 //  for layout 2), then the absorbing-state bitmap
    uint32_t abs_off;            // LDS byte offset of that bitmap; bit (LDS state
    uint32_t abs_shift;          //  offset >> abs_shift) is set iff the state is absorbing
    uint32_t nabs;               // number of absorbing states
    // Two-symbol steps: a state-major table of delta2(s, c1 c2) =
    // delta(delta(s, c1), c2) over the distinct pair columns (c2 = K stands
    // for "no second symbol": a string's odd last byte), laid out as layout 1
    // (entry R2 * delta2, code = 2 * pair column, rows of R2 bytes), staged
    // with its own absorbing-state bitmap (index R2 * s / 4).  pcode holds
    // 256 bytes byte -> class (0xFF outside Sigma), then the one-byte codes
    // of the K x (K + 1) class pairs.
    uint32_t pairs;              // 1 if the pair table exists
    const uint16_t *stab2;
    uint32_t stab2_bytes;        // multiple of 16
    uint32_t rowbytes2;          // R2
    uint32_t abs_off2;           // LDS byte offset of its absorbing bitmap
    const uint8_t *pcode;
    const uint8_t *pcode2;       // direct tables only (else NULL): 32768 + 128 bytes, the
                                 // pair code of bytes b1, b2 < 128 at b1 + 256 * b2 and of a
                                 // lone last byte at 32768 + b; 0xFF for bytes outside Sigma
    uint32_t nq;
    uint32_t nclass;
    uint32_t colstride;          // bytes between class columns (2 * Qp)
    uint32_t table_bytes;        // staged bytes, multiple of 16
    uint32_t setmax[2];          // largest set per mode
    uint32_t q0;
};

}  // namespace dfaspec

struct dfa {
    dfaspec::DevDFA dev{};
    void *arena = nullptr;       // one device allocation holding all tables
    size_t arena_bytes = 0;
    int device = 0;
    dfa_info_t info{};
    uint32_t nsym = 0;
    uint32_t setmax_host[2] = {0, 0};
    double wave_util = 0.0;      // lane utilisation of one-chunk-per-wave matching (lookahead 1)
    double mset_mean[dfaspec::kMaxMsetLevel + 1] = {};   // mean precomputed set size per level
    uint32_t mset_max[dfaspec::kMaxMsetLevel + 1] = {};  // largest precomputed set per level
    // host copies for dfa_lookahead_set
    std::vector<uint32_t> h_mset_off;
    std::vector<uint16_t> h_mset_st;
    int16_t h_byte_class[256] = {};
};

namespace dfaspec {

// Thread-local last-error message helpers (dfa_api.cpp).
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// One membership test (dfa_match_ex's path) with every scratch buffer taken
// from `region` (region_bytes of device memory); allocates nothing and
// returns DFA_E_TOOBIG when the plan needs more (dfa_api.cpp).
int match_in_region(const dfa_t *d, const uint8_t *d_in, size_t len, uint32_t start,
                    const dfa_match_opts_t *opts, hipStream_t s, uint32_t *d_result,
                    uint8_t *region, size_t region_bytes);

// Kernel launchers (dfa_kernels.hip).
struct Workspace;
constexpr uint32_t kMaxLevels = 40;  // fan-in >= 2 and < 2^32 chunks need at most 32
struct MatchPlan {
    uint64_t n = 0;
    uint64_t chunk = 0;
    uint32_t nch = 0;
    uint32_t lookahead = 1;      // set mode: 0 all states, 1 I_sigma, 2 image of r > r0 bytes
                                 // (window pass), 3 precomputed I_{c_1..c_r} (r <= r0)
    uint32_t r = 1;              // reverse-lookahead symbols (mode 2: r >= 2)
    uint32_t bitmap_words = 0;   // mode 2: words per chunk bitmap
    uint32_t stride = 0;         // map entries per chunk (>= largest set)
    uint32_t group = 0;          // largest fan-in of a compose step (LDS bound)
    uint32_t group_l[kMaxLevels] = {};  // fan-in from level l to level l + 1
    uint32_t levels = 0;         // compose levels above level 0
    uint32_t level_count[kMaxLevels] = {};
    uint64_t level_off[kMaxLevels] = {};  // entry offsets of each level's maps
    uint64_t msize_off[kMaxLevels] = {};  // entry offsets of each level's sizes
    uint64_t map_entries = 0;    // total uint16 entries for maps
    uint64_t msize_entries = 0;
    uint32_t waves_per_block = 4;
    uint32_t blocks = 0;
    // packed-pair matcher
    bool packed = false;
    bool early_exit = false;     // DFA_MATCH_EARLY_EXIT honoured (packed, absorbing states)
    uint32_t slots = 4;          // pairs per lane of a wave-tile (2 or 4)
    bool pairs = false;          // two-symbol steps over the pair table (chunk % 32 == 0)
    uint32_t rounds = 1;         // walk rounds (> 1: merged walks, chunk % 32 == 0)
    bool tail = false;           // merged walks whose last round runs one chunk per lane
                                 // over the raw input (the code stream then holds only
                                 // each chunk's first tail_t0 bytes)
    uint32_t tail_t0 = 0;        // chunk bytes before the last round
    uint32_t tail_threads = 0;   // its grid: one lane per chunk (+ one wavefront per
                                 // workgroup for the overflow list)
    uint32_t tail_blocks = 0;
    uint32_t tail_k = 1;         // chunks per lane in that round (2: two chunks side by side
                                 // once each has one chain left)
    bool round1c = false;        // first merged round chunk-major (k_round1c): one wavefront
                                 // per chunk over its whole start set
    uint64_t before = 0;         // block map of a shard: bytes of lookahead readable before
                                 // the input; chunk 0 then starts from its lookahead set
    bool chunk_lanes = false;    // one chunk per lane with merged walks (interleaved codes)
    uint32_t ilv_nblk = 0;       // chunk-interleaved code stream: 16-byte code blocks per
                                 // chunk (0: linear stream, or the raw input)
    uint32_t blocks2 = 0;        // persistent grid
    uint32_t threads2 = 256;     // threads per block (more for large tables)
    uint32_t tblocks = 0;        // translation blocks (4 KiB of input each)
    uint32_t code_bytes = 1;     // 1 (layout 1) or 2 (layout 2)
    uint64_t max_tiles = 0;      // upper bound on wave-tiles of pairs
};

// flags: DFA_MATCH_* bits (early exit, walk rounds) and kPlan* bits.
// before: bytes of lookahead readable before the input (block maps; 0 = a
// whole string, whose chunk 0 starts from the start state).
int plan_match(const dfa *d, uint64_t n, uint64_t chunk_req, uint32_t lookahead, MatchPlan *p,
               uint32_t flags = 0, uint64_t before = 0);
// ev_after_match (may be null) is recorded right after the matcher kernel.
int launch_match(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                 uint16_t *maps, uint16_t *msize, uint16_t *bvals, uint32_t *d_result,
                 uint32_t *d_boundaries, hipStream_t s, hipEvent_t ev_after_match);
// Per-call buffers of the packed-pair matcher (workspace views).
struct PackedBufs {
    void *codes = nullptr;           // translated stream
    uint32_t *block_bad = nullptr;   // per translation block: byte outside Sigma
    uint32_t *bsum = nullptr;        // scan block sums
    uint32_t *first = nullptr;       // [nch + 1] first pair of each chunk
    uint32_t *tile_first = nullptr;  // owner chunk of each wave-tile's first pair
    uint16_t *ccls = nullptr;        // lookahead class per chunk (r = 0, 1)
    uint32_t *cset = nullptr;        // precomputed-set id per chunk (r >= 2)
    uint32_t *bits = nullptr;        // r >= 2: start-set bitmaps
    uint16_t *members = nullptr;     // r >= 2: sorted start sets, indexed by pair
    // merged walks (MatchPlan::rounds > 1): per round k the walks' outcomes
    // lo[k] (kDone | end state, or the walk's index in list[k + 1]), the
    // walk lists of rounds >= 1 ({chunk, state}) and their counters
    uint32_t *lo[kMaxRounds] = {};
    uint2 *list[kMaxRounds] = {};
    uint32_t *cnt = nullptr;         // [kMaxRounds][kRegions]
    // one-chunk-per-lane last round (MatchPlan::tail): per chunk the number
    // of walks that reach it and the states of the first kTailSlots
    uint32_t *tail_cnt = nullptr;    // [nch]
    uint16_t *tail_st = nullptr;     // [nch][kTailSlots]
    // optional readout of the level-0 maps (dfa_match_maps): the first pair
    // of every chunk, and per pair its start and end state, for pairs < out_cap
    uint32_t *out_first = nullptr;
    uint16_t *out_start = nullptr;
    uint16_t *out_end = nullptr;
    uint64_t out_cap = 0;
};
// The packed path stores level-0 maps indexed by pair (maps[first[i] + p]);
// pb is null for the one-chunk-per-wave path (maps[i * stride + p]).
// Block maps of shards (dfa_match_block / dfa_compose_blocks): the composed
// top-level map with chunk 0's start states, and the ordered composition of
// several blocks' maps from one start state.
int launch_block_out(const dfa *d, uint32_t start, const MatchPlan &p, const PackedBufs &b,
                     const uint16_t *maps, const uint16_t *msize, const uint32_t *rec,
                     uint32_t *info, uint16_t *out_start, uint16_t *out_end, uint32_t max,
                     hipStream_t s);
int launch_compose_blocks(const dfa *d, uint32_t count, const uint32_t *infos,
                          const uint16_t *starts, const uint16_t *ends, uint32_t max,
                          uint32_t start, uint32_t *result, uint32_t *states, hipStream_t s);
int launch_combine(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                   uint16_t *maps, uint16_t *msize, uint16_t *bvals, const PackedBufs *pb,
                   uint32_t *d_result, uint32_t *d_boundaries, hipStream_t s);
// ev_before_matcher (may be null) is recorded after the preparation kernels,
// right before the packed matcher kernel.
// ev_kern_begin / ev_kern_end (may be null): recorded around the plan's
// longest single matcher launch (the one-chunk-per-lane last round, else the
// last merged round, else the matcher).
int launch_match2(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                  const PackedBufs &b, uint16_t *maps, uint16_t *msize, hipStream_t s,
                  hipEvent_t ev_before_matcher, hipEvent_t ev_kern_begin = nullptr,
                  hipEvent_t ev_kern_end = nullptr);
int launch_down0(const MatchPlan &p, const uint16_t *maps0, const uint32_t *first,
                 const uint16_t *bv_up, uint16_t *bv0, hipStream_t s);
int set_match2_lds_limit(int lds);
int allow_dynamic_lds(const void *f, int lds);

// Batches (dfa_batch.hip): a host-side plan -- descriptor bytes to upload to
// the start of a device region of total_bytes -- and a launcher that only
// enqueues device work.
struct BatchPlan {
    std::vector<uint8_t> desc;   // first desc_bytes of the device region
    size_t o_dfas = 0, o_reqs = 0, o_tasks = 0, o_groups = 0;
    size_t desc_bytes = 0;
    size_t o_counter = 0, o_maps = 0, o_msize = 0;
    size_t total_bytes = 0;
    uint32_t count = 0, ntasks = 0, max_levels = 0;
    std::vector<uint32_t> groups_per_level;
    std::vector<size_t> group_base;
    uint32_t blocks = 0, threads = 0;
    size_t lds_match = 0, lds_compose = 0;
    uint64_t chunk = 0;
};
int plan_batch(const dfa_t *const *dfas, const uint8_t *const *d_inputs, const size_t *lens,
               size_t count, uint64_t chunk_req, BatchPlan *out);
int launch_batch(const BatchPlan &p, void *dev_base, hipStream_t s, uint32_t *d_results,
                 hipEvent_t ev_before_match = nullptr, hipEvent_t ev_after_match = nullptr);

// Batched packed-pair path (dfa_batch2.hip): all DFAs need a packed layout.
struct Batch2Plan {
    std::vector<uint8_t> desc;   // first desc_bytes of the device region
    size_t o_dfas = 0, o_strs = 0, o_reqs = 0, o_groups = 0, o_segs = 0, o_items = 0;
    size_t o_chunk_str = 0, desc_bytes = 0;
    size_t o_counter = 0, o_str_bad = 0, o_msize0 = 0, o_cset = 0, o_first_raw = 0;
    size_t o_first2 = 0, o_bsum = 0, o_tile_raw = 0, o_tile_first2 = 0, o_gtile = 0;
    size_t o_gtask = 0, o_gend = 0, o_maps0 = 0, o_maps = 0, o_msize = 0, o_codes = 0;
    size_t total_bytes = 0;
    uint32_t count = 0, nchunks = 0, ngroups = 0, nsegs = 0, max_levels = 0;
    std::vector<uint32_t> items_per_level;
    std::vector<size_t> item_base;
    uint64_t chunk = 0;
    uint32_t task_slot = 0, wpb = 4, blocks = 0, tblocks = 0, early_exit = 0, slots = 2;
    size_t lds_match = 0, lds_compose0 = 0, lds_compose = 0;
};
bool batch2_supported(const dfa_t *const *dfas, size_t count);
int plan_batch2(const dfa_t *const *dfas, const uint8_t *const *d_inputs, const size_t *lens,
                size_t count, uint64_t chunk_req, uint32_t lookahead, Batch2Plan *out,
                uint32_t flags = 0);
int launch_batch2(const Batch2Plan &p, void *dev_base, hipStream_t s, uint32_t *d_results,
                  hipEvent_t ev_before_match = nullptr, hipEvent_t ev_after_match = nullptr);

// Timing hooks of dfa_timing_enable for entry points outside the single-
// string path.  timing_begin returns false (and creates nothing) when timing
// is off for the stream; otherwise it creates ev[0..3] and records ev[0].
// timing_end records ev[3] and keeps the four events for dfa_timing_read.
bool timing_begin(hipStream_t s, hipEvent_t ev[4]);
int timing_end(hipStream_t s, hipEvent_t ev[4]);
// Exclusive scan of msize[0..nch) (low 15 bits): first[i], first[nch] = total,
// tile_first[w] = chunk holding pair w * tile.  bsum holds
// match2_scan_blocks(nch) words.
int launch_size_scan(uint32_t nch, uint16_t *msize, uint32_t *bsum, uint32_t *first,
                     uint32_t *tile_first, uint32_t tile, hipStream_t s);
uint32_t match2_tile_pairs(uint32_t slots);
uint32_t round_region_cap(const MatchPlan &p);   // places per region of a walk list
size_t round_lds_extra();                         // LDS of the region prefix after the table
size_t round_lds_bytes(uint32_t threads);         // all LDS k_round adds after the table
size_t tail_lut_bytes();                          // LDS of k_tail's byte table (all copies)
uint32_t match2_scan_blocks(uint32_t nch);
int device_lds_bytes();
size_t tree_lds_bytes(uint32_t G, uint32_t stride);   // LDS of k_compose_tree
int device_cu_count();

}  // namespace dfaspec
