// C ABI entry points: matching calls, workspaces, error reporting.
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <utility>

#include "dfa_internal.h"

using namespace dfaspec;

namespace dfaspec {

namespace {
thread_local std::string g_last_error;
}

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return DFA_E_DEVICE;
}

// Per-(device, stream) scratch memory for maps, sizes, boundary values and
// staged host input.  Calls on one stream are ordered by the stream, so they
// may share it; callers that use one stream from several host threads must
// serialise those calls themselves.
struct Workspace {
    void *buf = nullptr;
    size_t bytes = 0;
    uint8_t *in = nullptr;
    size_t in_bytes = 0;
    uint32_t *result = nullptr;   // 4 words for the synchronous path
    bool timing = false;
    // kern_begin / kern_end (may be null): around the call's longest single
    // matcher launch (see dfa_timing_read_ex)
    struct Stamp { hipEvent_t begin, before_match, after_match, end, kern_begin, kern_end; };
    std::vector<Stamp> stamps;    // one per timed call, read by dfa_timing_read
};

namespace {
std::mutex g_ws_mutex;
std::map<std::pair<int, void *>, std::unique_ptr<Workspace>> g_ws;

Workspace *workspace_for(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    auto &slot = g_ws[{dev, (void *)s}];
    if (!slot) slot.reset(new Workspace());
    return slot.get();
}

// Grows a per-stream buffer.  Only work on stream s uses it, so waiting for
// s (not the whole device) makes the old buffer free to release.
int ensure(void **ptr, size_t *have, size_t need, hipStream_t s) {
    if (*have >= need && *ptr) return DFA_OK;
    if (*ptr) {
        // the stream may still be reading the old buffer
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize (workspace)");
        (void)hipFree(*ptr);
        *ptr = nullptr;
        *have = 0;
    }
    size_t want = need + need / 4 + 4096;
    hipError_t e = hipMalloc(ptr, want);
    if (e != hipSuccess) return fail(DFA_E_NOMEM, "workspace hipMalloc failed");
    *have = want;
    return DFA_OK;
}

uint64_t env_chunk() {
    const char *v = std::getenv("DFA_CHUNK");
    return v ? std::strtoull(v, nullptr, 10) : 0;
}

// Autotuner cache: (DFA, length bucket) -> options.
std::mutex g_tune_mutex;
std::map<std::pair<const dfa_t *, int>, dfa_match_opts_t> g_tuned;

int length_bucket(size_t len) {
    int b = 0;
    while ((len >> b) > 1) ++b;
    return b;
}

dfa_match_opts_t resolve_opts(const dfa_t *d, size_t len, const dfa_match_opts_t *opts) {
    dfa_match_opts_t o{};
    o.lookahead = 1;
    if (opts) o = *opts;
    if (o.lookahead == DFA_LOOKAHEAD_AUTO) {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tuned.find({d, length_bucket(len)});
        if (it != g_tuned.end()) {
            const uint64_t user_chunk = o.chunk_len;
            o = it->second;
            if (user_chunk) o.chunk_len = user_chunk;
        } else {
            o.lookahead = 1;
        }
    }
    return o;
}

// A block map request (dfa_match_block): the shard's input starts `before`
// bytes into the caller's string, and the composed map goes to these buffers.
struct BlockReq {
    uint64_t before;
    uint32_t *info;
    uint16_t *start;
    uint16_t *end;
    uint32_t max;
};

// fixed: when not null, the call's scratch memory (fixed_bytes of device
// memory) instead of the stream's workspace; nothing is allocated and no
// timing events are made.
int run_match(const dfa_t *d, const uint8_t *d_in, size_t len, uint32_t start,
              const dfa_match_opts_t *opts_in, hipStream_t s, uint32_t *d_result,
              uint32_t *d_bound, const PackedBufs *readout = nullptr,
              uint8_t *fixed = nullptr, size_t fixed_bytes = 0,
              const BlockReq *block = nullptr) {
    if (!d || (!d_result && !block) || (len && !d_in)) return fail(DFA_E_INVAL, "match: NULL argument");
    if (start == DFA_Q0) start = d->dev.q0;
    if (start >= d->dev.nq) return fail(DFA_E_INVAL, "match: start state out of range");
    const dfa_match_opts_t resolved = resolve_opts(d, len, opts_in);
    const dfa_match_opts_t *opts = &resolved;
    uint64_t chunk = opts->chunk_len ? opts->chunk_len : env_chunk();
    uint32_t look = opts->lookahead;
    MatchPlan p;
    const bool unaligned = (reinterpret_cast<uintptr_t>(d_in) & 15u) != 0;
    int rc = plan_match(d, len, chunk, look, &p,
                        opts->flags | (unaligned ? kPlanUnaligned : 0u) | (block ? kPlanBlock : 0u),
                        block ? block->before : 0u);
    if (rc) return rc;
    if (block) {
        if (!p.packed)
            return fail(DFA_E_INVAL, "block maps need a DFA with a packed layout (dfa_info_t)");
        if (p.lookahead == 2)
            return fail(DFA_E_INVAL, "block maps need lookahead 0, 1 or a precomputed r (<= r0)");
        if (len == 0 || d_bound || readout)
            return fail(DFA_E_INVAL, "block maps: empty shard, or boundaries/readout requested");
        if (block->max < p.stride)
            return fail(DFA_E_TOOBIG, "block maps: max_entries below the largest start set (" +
                                          std::to_string(p.stride) + ")");
        p.before = block->before;
    }
    if (readout && (!p.packed || len == 0))
        return fail(DFA_E_INVAL, "map readout needs the packed-pair matcher and a non-empty input");
    Workspace *ws = fixed ? nullptr : workspace_for(s);
    if (!fixed && !ws) return fail(DFA_E_DEVICE, "no HIP device");
    const bool timing = ws && ws->timing;
    auto a256 = [](uint64_t b) { return (size_t)((b + 255) / 256 * 256); };
    const size_t map_bytes = a256(p.map_entries * 2);
    const size_t sz_bytes = a256(p.msize_entries * 2);
    size_t need = map_bytes + 2 * sz_bytes + (block ? 256u : 0u);   // + block: result record
    size_t code_off = need, bad_off = 0, bsum_off = 0, first_off = 0, tf_off = 0, ccls_off = 0,
           bits_off = 0, mem_off = 0, cset_off = 0, round_off = 0;
    if (p.packed && len) {
        // the translated stream: none when the matcher reads the raw input (a
        // direct table, 16-byte aligned input, linear layout), one byte per
        // two input bytes for pair codes (whole 16-byte units of 32 bytes),
        // else code_bytes per byte
        const bool raw = !p.pairs && !p.ilv_nblk && d->dev.direct && p.lookahead != 2 &&
                         (reinterpret_cast<uintptr_t>(d_in) & 15u) == 0;
        uint64_t code_stream =
            raw ? 64
                : p.pairs ? ((uint64_t)len + 32) / 32 * 16 + 64
                          : ((uint64_t)len + 16) / 16 * 16 * p.code_bytes + 64;
        if (p.ilv_nblk)   // whole groups of 64 chunks of ilv_nblk blocks each (with a
                          // one-chunk-per-lane last round, each chunk's first bytes only)
            code_stream = ((uint64_t)p.nch + 63) / 64 * 64 * p.ilv_nblk * 16 + 64;
        need += a256(code_stream);
        bad_off = need;
        need += a256((uint64_t)p.tblocks * 4);
        bsum_off = need;
        need += a256((uint64_t)match2_scan_blocks(p.nch) * 4 + 4);
        first_off = need;
        need += a256(((uint64_t)p.nch + 1) * 4);
        tf_off = need;
        need += a256((p.max_tiles + 1) * 4);
        ccls_off = need;
        need += a256((uint64_t)p.nch * 2);
        cset_off = need;
        need += a256((uint64_t)p.nch * 4);
        if (p.lookahead == 2) {
            bits_off = need;
            need += a256((uint64_t)p.nch * p.bitmap_words * 4);
            mem_off = need;
            need += a256(((uint64_t)p.nch * p.stride + 1) * 2);
        }
        if (p.rounds > 1) {
            // per round: outcomes (4 B per walk or place); rounds >= 1: walk
            // lists of kRegions regions (8 B per place); a one-chunk-per-lane
            // last round: per-chunk counts and states, and its outcomes
            // start with kTailSlots places per chunk
            const uint64_t walks = p.max_tiles * (uint64_t)match2_tile_pairs(p.slots);
            const uint64_t places = (uint64_t)kRegions * round_region_cap(p);
            const uint64_t tail_places = p.tail ? (uint64_t)p.nch * kTailSlots : 0u;
            round_off = need;
            need += a256((uint64_t)kMaxRounds * kRegions * 4);
            for (uint32_t k = 0; k < p.rounds; ++k)
                need += k ? a256((places + (k + 1 == p.rounds ? tail_places : 0u)) * 4) +
                                a256(places * 8)
                          : a256(walks * 4);
            if (p.tail) need += a256((uint64_t)p.nch * 4) + a256(tail_places * 2);
        }
    }
    uint8_t *base = fixed;
    if (fixed) {
        if (need > fixed_bytes)
            return fail(DFA_E_TOOBIG, "match: needs " + std::to_string(need) +
                                          " bytes of scratch, more than the " +
                                          std::to_string(fixed_bytes) + " the call may use");
    } else {
        rc = ensure(&ws->buf, &ws->bytes, need + 256, s);
        if (rc) return rc;
        base = (uint8_t *)ws->buf;
    }
    uint16_t *maps = (uint16_t *)base;
    uint16_t *msize = (uint16_t *)(base + map_bytes);
    uint16_t *bvals = (uint16_t *)(base + map_bytes + sz_bytes);
    // a block map's combine writes its result record into the workspace
    if (block) d_result = (uint32_t *)(base + map_bytes + 2 * sz_bytes);
    Workspace::Stamp st{};
    hipError_t e = hipSuccess;
    if (timing) {
        e = hipEventCreate(&st.begin);
        if (e == hipSuccess) e = hipEventCreate(&st.before_match);
        if (e == hipSuccess) e = hipEventCreate(&st.after_match);
        if (e == hipSuccess) e = hipEventCreate(&st.end);
        if (e == hipSuccess && p.packed && len) e = hipEventCreate(&st.kern_begin);
        if (e == hipSuccess && p.packed && len) e = hipEventCreate(&st.kern_end);
        if (e == hipSuccess) e = hipEventRecord(st.begin, s);
        if (e != hipSuccess) return hip_fail(e, "timing events");
    }
    if (p.packed && len) {
        PackedBufs pb;
        pb.codes = base + code_off;
        pb.block_bad = (uint32_t *)(base + bad_off);
        pb.bsum = (uint32_t *)(base + bsum_off);
        pb.first = (uint32_t *)(base + first_off);
        pb.tile_first = (uint32_t *)(base + tf_off);
        pb.ccls = (uint16_t *)(base + ccls_off);
        pb.cset = (uint32_t *)(base + cset_off);
        if (p.lookahead == 2) {
            pb.bits = (uint32_t *)(base + bits_off);
            pb.members = (uint16_t *)(base + mem_off);
        }
        if (p.rounds > 1) {
            const uint64_t walks = p.max_tiles * (uint64_t)match2_tile_pairs(p.slots);
            const uint64_t places = (uint64_t)kRegions * round_region_cap(p);
            size_t at = round_off;
            pb.cnt = (uint32_t *)(base + at);
            at += a256((uint64_t)kMaxRounds * kRegions * 4);
            const uint64_t tail_places = p.tail ? (uint64_t)p.nch * kTailSlots : 0u;
            for (uint32_t k = 0; k < p.rounds; ++k) {
                pb.lo[k] = (uint32_t *)(base + at);
                at += a256((k ? places + (k + 1 == p.rounds ? tail_places : 0u) : walks) * 4);
                if (k) {
                    pb.list[k] = (uint2 *)(base + at);
                    at += a256(places * 8);
                }
            }
            if (p.tail) {
                pb.tail_cnt = (uint32_t *)(base + at);
                at += a256((uint64_t)p.nch * 4);
                pb.tail_st = (uint16_t *)(base + at);
                at += a256(tail_places * 2);
            }
        }
        if (readout) {
            pb.out_first = readout->out_first;
            pb.out_start = readout->out_start;
            pb.out_end = readout->out_end;
            pb.out_cap = readout->out_cap;
        }
        rc = launch_match2(d, d_in, start, p, pb, maps, msize, s,
                           timing ? st.before_match : nullptr, st.kern_begin, st.kern_end);
        if (rc) return rc;
        if (timing) {
            e = hipEventRecord(st.after_match, s);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        rc = launch_combine(d, d_in, start, p, maps, msize, bvals, &pb, d_result, d_bound, s);
        if (!rc && block)
            rc = launch_block_out(d, start, p, pb, maps, msize, d_result, block->info, block->start,
                                  block->end, block->max, s);
    } else {
        if (timing) {
            e = hipEventRecord(st.before_match, s);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        rc = launch_match(d, d_in, start, p, maps, msize, bvals, d_result, d_bound, s,
                          timing ? st.after_match : nullptr);
    }
    if (rc) return rc;
    if (!timing) return DFA_OK;
    e = hipEventRecord(st.end, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ws->stamps.push_back(st);
    return DFA_OK;
}
}  // namespace

int match_in_region(const dfa_t *d, const uint8_t *d_in, size_t len, uint32_t start,
                    const dfa_match_opts_t *opts, hipStream_t s, uint32_t *d_result,
                    uint8_t *region, size_t region_bytes) {
    return run_match(d, d_in, len, start, opts, s, d_result, nullptr, nullptr, region,
                     region_bytes);
}

}  // namespace dfaspec

extern "C" int dfa_match_ex(const dfa_t *d, const uint8_t *d_input, size_t len,
                            uint32_t start_state, const dfa_match_opts_t *opts, void *stream,
                            uint32_t *d_result, uint32_t *d_boundaries) {
    return run_match(d, d_input, len, start_state, opts, (hipStream_t)stream, d_result,
                     d_boundaries);
}

namespace {
// dfa_match_noalloc's scratch: one fixed region per GPU.  A file-scope device
// array exists once on every device the code object is loaded on, for the
// life of the process.  Host code reaches it only through the address
// hipGetSymbolAddress returns with that device current (the array's name is
// not a device address in host code).
constexpr size_t kScratchBytes = (size_t)DFA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, uint8_t *> g_scratch;   // device -> address of its region

int scratch_region(uint8_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress (scratch)");
        it = g_scratch.emplace(dev, static_cast<uint8_t *>(ptr)).first;
    }
    *out = it->second;
    return DFA_OK;
}
}  // namespace

extern "C" int dfa_match_noalloc(const dfa_t *d, const uint8_t *d_input, size_t len,
                                 uint32_t start_state, const dfa_match_opts_t *opts,
                                 void *stream, uint32_t *d_result, uint32_t *d_boundaries) {
    uint8_t *region = nullptr;
    int rc = scratch_region(&region);
    if (rc) return rc;
    return run_match(d, d_input, len, start_state, opts, (hipStream_t)stream, d_result,
                     d_boundaries, nullptr, region, kScratchBytes);
}

extern "C" int dfa_match_block(const dfa_t *d, const uint8_t *d_input, size_t offset, size_t len,
                               uint32_t start_state, const dfa_match_opts_t *opts, void *stream,
                               uint32_t *d_info, uint16_t *d_start, uint16_t *d_end,
                               uint32_t max_entries) {
    if (!d || !d_input || !d_info || !d_start || !d_end)
        return fail(DFA_E_INVAL, "dfa_match_block: NULL argument");
    const BlockReq req{offset, d_info, d_start, d_end, max_entries};
    return run_match(d, d_input + offset, len, start_state, opts, (hipStream_t)stream, nullptr,
                     nullptr, nullptr, nullptr, 0, &req);
}

extern "C" int dfa_compose_blocks(const dfa_t *d, uint32_t count, const uint32_t *d_infos,
                                  const uint16_t *d_starts, const uint16_t *d_ends,
                                  uint32_t max_entries, uint32_t start_state, void *stream,
                                  uint32_t *d_result, uint32_t *d_block_states) {
    if (!d || !d_result || (count && (!d_infos || !d_starts || !d_ends)))
        return fail(DFA_E_INVAL, "dfa_compose_blocks: NULL argument");
    if (start_state == DFA_Q0) start_state = d->dev.q0;
    if (start_state >= d->dev.nq) return fail(DFA_E_INVAL, "dfa_compose_blocks: start state out of range");
    return launch_compose_blocks(d, count, d_infos, d_starts, d_ends, max_entries, start_state,
                                 d_result, d_block_states, (hipStream_t)stream);
}

extern "C" int dfa_match_maps(const dfa_t *d, const uint8_t *d_input, size_t len,
                              uint32_t start_state, const dfa_match_opts_t *opts, void *stream,
                              uint32_t *d_result, uint32_t *d_first, uint16_t *d_pair_start,
                              uint16_t *d_pair_end, uint64_t max_pairs) {
    if (!d_first || (max_pairs && (!d_pair_start || !d_pair_end)))
        return fail(DFA_E_INVAL, "dfa_match_maps: NULL output");
    PackedBufs ro;
    ro.out_first = d_first;
    ro.out_start = d_pair_start;
    ro.out_end = d_pair_end;
    ro.out_cap = max_pairs;
    return run_match(d, d_input, len, start_state, opts, (hipStream_t)stream, d_result, nullptr,
                     &ro);
}

extern "C" int dfa_match_async(const dfa_t *d, const uint8_t *d_input, size_t len,
                               uint32_t start_state, void *stream, uint32_t *d_result) {
    return run_match(d, d_input, len, start_state, nullptr, (hipStream_t)stream, d_result,
                     nullptr);
}

extern "C" int dfa_plan_chunks(const dfa_t *d, size_t len, const dfa_match_opts_t *opts_in,
                               uint64_t *chunk_len, uint64_t *num_chunks) {
    if (!d) return fail(DFA_E_INVAL, "dfa_plan_chunks: NULL dfa");
    const dfa_match_opts_t o = resolve_opts(d, len, opts_in);
    uint64_t chunk = o.chunk_len ? o.chunk_len : env_chunk();
    MatchPlan p;
    int rc = plan_match(d, len, chunk, o.lookahead, &p, o.flags);
    if (rc) return rc;
    if (chunk_len) *chunk_len = p.chunk;
    if (num_chunks) *num_chunks = p.nch;
    return DFA_OK;
}

extern "C" int dfa_plan(const dfa_t *d, size_t len, const dfa_match_opts_t *opts_in,
                        dfa_plan_info_t *out) {
    if (!d || !out) return fail(DFA_E_INVAL, "dfa_plan: NULL argument");
    const dfa_match_opts_t o = resolve_opts(d, len, opts_in);
    uint64_t chunk = o.chunk_len ? o.chunk_len : env_chunk();
    MatchPlan p;
    int rc = plan_match(d, len, chunk, o.lookahead, &p, o.flags);
    if (rc) return rc;
    out->chunk_len = p.chunk;
    out->num_chunks = p.nch;
    out->kernel = p.packed ? 1u : 0u;
    out->lookahead = p.r;
    out->blocks = p.packed ? p.blocks2 : p.blocks;
    out->threads = p.packed ? p.threads2 : p.waves_per_block * 64u;
    out->symbols_per_step = p.pairs ? 2u : 1u;
    out->rounds = p.rounds;
    out->interleaved = p.ilv_nblk ? 1u : 0u;
    out->chunk_lanes = p.chunk_lanes ? 1u : 0u;
    out->set_max = p.stride;
    out->levels = p.levels;
    out->group0 = p.levels ? p.group_l[0] : 0u;
    out->group = p.levels > 1 ? p.group_l[1] : 0u;
    out->tail_lanes = p.tail ? p.tail_k : 0u;
    out->tail_start = p.tail ? p.tail_t0 : 0u;
    out->raw_input = p.packed && !p.pairs && !p.ilv_nblk && d->dev.direct && p.lookahead != 2;
    return DFA_OK;
}

extern "C" int dfa_match(const dfa_t *d, const uint8_t *input, size_t len, uint32_t start_state,
                         uint32_t *final_state, int *accepted) {
    if (!d || (len && !input)) return fail(DFA_E_INVAL, "dfa_match: NULL argument");
    hipStream_t s = nullptr;
    Workspace *ws = workspace_for(s);
    if (!ws) return fail(DFA_E_DEVICE, "no HIP device");
    int rc = ensure((void **)&ws->in, &ws->in_bytes, len + 256, s);
    if (rc) return rc;
    if (!ws->result) {
        hipError_t e = hipMalloc(&ws->result, 4 * sizeof(uint32_t));
        if (e != hipSuccess) return fail(DFA_E_NOMEM, "hipMalloc (result)");
    }
    if (len) {
        hipError_t e = hipMemcpyAsync(ws->in, input, len, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (input)");
    }
    rc = run_match(d, ws->in, len, start_state, nullptr, s, ws->result, nullptr);
    if (rc) return rc;
    uint32_t res[4];
    hipError_t e = hipMemcpyAsync(res, ws->result, sizeof(res), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "dfa_match readback");
    if (res[2] & DFA_FLAG_SYMBOL) return fail(DFA_E_SYMBOL, "input holds a byte outside Sigma");
    if (res[2] & DFA_FLAG_SPECULATION)
        return fail(DFA_E_SPECULATION, "speculation invariant violated");
    if (final_state) *final_state = res[0];
    if (accepted) *accepted = (int)res[1];
    return DFA_OK;
}

extern "C" int dfa_match_batch(const dfa_t *const *dfas, const uint8_t *const *d_inputs,
                               const size_t *lens, size_t count, void *stream,
                               uint32_t *d_results) {
    if (count && (!dfas || !d_inputs || !lens || !d_results))
        return fail(DFA_E_INVAL, "dfa_match_batch: NULL argument");
    if (!count) return DFA_OK;
    dfa_batch_t *b = nullptr;
    int rc = dfa_batch_create(dfas, d_inputs, lens, count, nullptr, &b);
    if (rc) return rc;
    rc = dfa_batch_run(b, stream, d_results);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    dfa_batch_destroy(b);
    if (rc) return rc;
    return e == hipSuccess ? DFA_OK : hip_fail(e, "dfa_match_batch: hipStreamSynchronize");
}

extern "C" int dfa_autotune(const dfa_t *d, const uint8_t *d_input, size_t len, void *stream,
                            dfa_match_opts_t *best, double *best_ms) {
    if (!d || (len && !d_input)) return fail(DFA_E_INVAL, "dfa_autotune: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = std::min<size_t>(len, 1ull << 30);
    uint32_t *res = nullptr;
    hipError_t e = hipMalloc(&res, 4 * sizeof(uint32_t));
    if (e != hipSuccess) return fail(DFA_E_NOMEM, "dfa_autotune: hipMalloc");
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    // candidates: r = 1 .. r0 + 2 (capped at 10), chunk = planner and powers of two
    // from 64 B (short chunks keep the walks short on small inputs; tables
    // without a packed layout support only r = 1; chunk counts are bounded so
    // that no candidate's maps exceed 1 GiB)
    std::vector<uint32_t> rs;
    const uint32_t rmax = d->dev.layout ? std::min<uint32_t>(d->dev.r0 + 2, 10) : 1u;
    for (uint32_t r = 1; r <= rmax; ++r) rs.push_back(r);
    std::vector<uint64_t> chunks = {0};
    const uint64_t per_chunk = 2ull * std::max<uint32_t>(d->setmax_host[0], 1u);
    for (uint64_t c = 64; c <= (1u << 20) && c <= std::max<size_t>(n, 256); c *= 2) {
        const uint64_t nch = (n + c - 1) / c;
        if (nch <= (1u << 20) && nch * per_chunk <= (1ull << 30)) chunks.push_back(c);
    }
    dfa_match_opts_t pick{};
    pick.lookahead = 1;
    double pick_ms = 1e30;
    int rc = DFA_OK;
    for (uint32_t r : rs) {
        for (uint64_t c : chunks) {
            dfa_match_opts_t o{};
            o.chunk_len = c;
            o.lookahead = r;
            double t_best = 1e30;
            for (int rep = 0; rep < 3 && rc == DFA_OK; ++rep) {
                if (rep > 0) (void)hipEventRecord(a, s);
                rc = run_match(d, d_input, n, DFA_Q0, &o, s, res, nullptr);
                if (rep > 0) {
                    (void)hipEventRecord(b, s);
                    (void)hipEventSynchronize(b);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, a, b);
                    t_best = std::min<double>(t_best, ms);
                }
            }
            if (rc) break;
            if (t_best < pick_ms) {
                pick_ms = t_best;
                pick = o;
            }
        }
        if (rc) break;
    }
    auto time_opts = [&](const dfa_match_opts_t &o) -> double {
        double t_best = 1e30;
        for (int rep = 0; rep < 3 && rc == DFA_OK; ++rep) {
            if (rep > 0) (void)hipEventRecord(a, s);
            rc = run_match(d, d_input, n, DFA_Q0, &o, s, res, nullptr);
            if (rep > 0) {
                (void)hipEventRecord(b, s);
                (void)hipEventSynchronize(b);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, a, b);
                t_best = std::min<double>(t_best, ms);
            }
        }
        return t_best;
    };
    // the best of each way of walking (flags) on the sample, for the whole-
    // input check below
    std::map<uint32_t, std::pair<double, dfa_match_opts_t>> family;
    family[pick.flags] = {pick_ms, pick};
    auto consider = [&](const dfa_match_opts_t &o) {
        const double t = time_opts(o);
        if (rc == DFA_OK) {
            auto it = family.find(o.flags);
            if (it == family.end() || t < it->second.first) family[o.flags] = {t, o};
        }
        if (rc == DFA_OK && t < pick_ms) {
            pick_ms = t;
            pick = o;
        }
    };
    // the ways of walking that change which chunk length is best (merged
    // rounds, interleaved codes, one chunk per lane), each at the best r and
    // the next, around the best chunk length
    if (rc == DFA_OK && d->dev.layout != 0) {
        const dfa_match_opts_t base = pick;
        uint64_t c0 = base.chunk_len;
        if (c0 == 0) {
            MatchPlan p0;
            if (plan_match(d, n, 0, base.lookahead, &p0, 0) == DFA_OK) c0 = p0.chunk;
        }
        std::vector<uint32_t> variants = {DFA_MATCH_ROUNDS(2), DFA_MATCH_ROUNDS(3), DFA_MATCH_ROUNDS(4),
                                          DFA_MATCH_INTERLEAVE, DFA_MATCH_INTERLEAVE | DFA_MATCH_ROUNDS(2),
                                          DFA_MATCH_INTERLEAVE | DFA_MATCH_ROUNDS(3),
                                          DFA_MATCH_INTERLEAVE | DFA_MATCH_ROUNDS(4),
                                          DFA_MATCH_CHUNK_LANES};
        // with a two-symbol table the variants above take two-symbol steps
        // (and so no one-chunk-per-lane last round); one symbol per step
        // with interleaved merged rounds reads the raw input in its last
        // round instead of a pair-code stream
        if (d->dev.pairs) {
            variants.push_back(DFA_MATCH_INTERLEAVE | DFA_MATCH_ROUNDS(2) | DFA_MATCH_SINGLE_STEP);
            variants.push_back(DFA_MATCH_INTERLEAVE | DFA_MATCH_ROUNDS(3) | DFA_MATCH_SINGLE_STEP);
        }
        // (merged rounds stop a walk at an absorbing state, so where the
        // input reaches one within a long chunk, lengths far above the
        // one-round best can win: up to 64 times it).  Besides r and r + 1
        // the largest precomputed r0 is tried: beyond it the window pass
        // needs per-byte codes, which may change the ranking.
        std::vector<uint32_t> vr = {base.lookahead};
        if (base.lookahead + 1 <= rmax) vr.push_back(base.lookahead + 1);
        if (d->dev.r0 >= 1 && d->dev.r0 <= rmax && d->dev.r0 != base.lookahead &&
            d->dev.r0 != base.lookahead + 1)
            vr.push_back(d->dev.r0);
        for (uint32_t r : vr) {
            for (uint32_t v : variants) {
                for (int sh : {-2, -1, 0, 1, 2, 4, 6}) {
                    if (rc != DFA_OK) break;
                    if (sh > 2 && !(v & 0xF00u)) continue;
                    const uint64_t c = sh < 0 ? c0 >> (-sh) : c0 << sh;
                    if (c < 256 || c % 32 != 0 || c > (1u << 20)) continue;
                    const uint64_t nch = (n + c - 1) / c;
                    if (nch > (1u << 20) || nch * per_chunk > (1ull << 30)) continue;
                    dfa_match_opts_t o{};
                    o.chunk_len = c;
                    o.lookahead = r;
                    o.flags = v;
                    consider(o);
                }
            }
        }
    }
    if (rc == DFA_OK && d->dev.pairs) {
        dfa_match_opts_t o = pick;
        o.flags |= DFA_MATCH_SINGLE_STEP;
        consider(o);
    }
    if (rc == DFA_OK && d->dev.nabs > 0 && d->dev.layout != 0) {
        // the best setting again with early exit at absorbing states
        dfa_match_opts_t o = pick;
        o.flags |= DFA_MATCH_EARLY_EXIT;
        double t_best = 1e30;
        for (int rep = 0; rep < 3 && rc == DFA_OK; ++rep) {
            if (rep > 0) (void)hipEventRecord(a, s);
            rc = run_match(d, d_input, n, DFA_Q0, &o, s, res, nullptr);
            if (rep > 0) {
                (void)hipEventRecord(b, s);
                (void)hipEventSynchronize(b);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, a, b);
                t_best = std::min<double>(t_best, ms);
            }
        }
        if (rc == DFA_OK && t_best < pick_ms) {
            pick_ms = t_best;
            pick = o;
        }
    }
    // On an input longer than the sample, the sample's best chunk length
    // gives more chunks than were measured (more lanes and tiles than the
    // device holds at once), and which way of walking wins can change with
    // the chunk count: the best setting of every way of walking, as measured
    // and with its chunk length scaled by len / n (the measured chunk count),
    // is timed on the whole input, and the fastest is kept.
    double full_ms = pick_ms * (double)len / (double)std::max<size_t>(n, 1);
    if (rc == DFA_OK && len > n) {
        auto time_full = [&](const dfa_match_opts_t &o) -> double {
            double t_best = 1e30;
            for (int rep = 0; rep < 3 && rc == DFA_OK; ++rep) {
                if (rep > 0) (void)hipEventRecord(a, s);
                rc = run_match(d, d_input, len, DFA_Q0, &o, s, res, nullptr);
                if (rep > 0) {
                    (void)hipEventRecord(b, s);
                    (void)hipEventSynchronize(b);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, a, b);
                    t_best = std::min<double>(t_best, ms);
                }
            }
            return t_best;
        };
        double best_full = 1e30;
        dfa_match_opts_t best_o = pick;
        for (const auto &f : family) {
            dfa_match_opts_t o = f.second.second;
            for (int scale = 0; scale < 2 && rc == DFA_OK; ++scale) {
                if (scale) {
                    if (o.chunk_len == 0) break;
                    uint64_t c = (uint64_t)((double)o.chunk_len * (double)len / (double)n);
                    c = std::max<uint64_t>(32, std::min<uint64_t>(c, (1ull << 31) - 32) / 32 * 32);
                    o.chunk_len = c;
                }
                const double t = time_full(o);
                if (rc == DFA_OK && t < best_full) {
                    best_full = t;
                    best_o = o;
                }
            }
        }
        // then halving and doubling the chunk length around the winner
        for (int sh : {-2, -1, 1}) {
            if (rc != DFA_OK || best_o.chunk_len == 0) break;
            dfa_match_opts_t o = best_o;
            const uint64_t c0 = best_o.chunk_len;
            const uint64_t c = sh < 0 ? c0 >> (-sh) : c0 << sh;
            if (c < 256 || c >= (1ull << 31) || ((o.flags & 0xF00u) && c % 32 != 0)) continue;
            o.chunk_len = c;
            const double t = time_full(o);
            if (rc == DFA_OK && t < best_full) {
                best_full = t;
                best_o = o;
            }
        }
        if (rc == DFA_OK) {
            full_ms = best_full;
            pick = best_o;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(res);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tuned[{d, length_bucket(len)}] = pick;
    }
    if (best) *best = pick;
    if (best_ms) *best_ms = full_ms;
    return DFA_OK;
}

extern "C" int dfa_batch_tune(const dfa_t *const *dfas, const uint8_t *const *d_inputs,
                              const size_t *lens, size_t count, void *stream,
                              dfa_match_opts_t *best, double *best_ms) {
    if (!best) return fail(DFA_E_INVAL, "dfa_batch_tune: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BatchPlan p0;
    int rc = plan_batch(dfas, d_inputs, lens, count, 0, &p0);
    if (rc) return rc;
    uint64_t base_chunk = p0.chunk;
    const bool packed = count > 0 && batch2_supported(dfas, count);
    if (packed) {
        Batch2Plan q0;
        rc = plan_batch2(dfas, d_inputs, lens, count, 0, 1, &q0);
        if (rc) return rc;
        base_chunk = q0.chunk;
    }
    uint32_t *res = nullptr;
    hipError_t e = hipMalloc(&res, std::max<size_t>(count, 1) * 4 * sizeof(uint32_t));
    if (e != hipSuccess) return fail(DFA_E_NOMEM, "dfa_batch_tune: hipMalloc");
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    dfa_match_opts_t pick{};
    pick.chunk_len = base_chunk;
    pick.lookahead = 1;
    double pick_ms = 1e30;
    // chunk candidates: the planner's and powers of two from 1 KiB to 64 KiB
    std::vector<uint64_t> cands = {std::max<uint64_t>(256, base_chunk / 64 * 64)};
    for (uint64_t c = 1024; c <= (64u << 10); c *= 2)
        if (c != cands[0]) cands.push_back(c);
    std::vector<uint32_t> looks = {1};
    if (packed) looks = {1, 2, 3, 4, 6, 8};
    for (uint32_t look : looks) {
        for (uint64_t c : cands) {
            dfa_match_opts_t o{};
            o.chunk_len = c;
            o.lookahead = look;
            dfa_batch_t *bt = nullptr;
            rc = dfa_batch_create(dfas, d_inputs, lens, count, &o, &bt);
            if (rc) break;
            double t_best = 1e30;
            for (int rep = 0; rep < 3 && rc == DFA_OK; ++rep) {
                if (rep > 0) (void)hipEventRecord(a, s);
                rc = dfa_batch_run(bt, stream, res);
                if (rep > 0) {
                    (void)hipEventRecord(b, s);
                    (void)hipEventSynchronize(b);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, a, b);
                    t_best = std::min<double>(t_best, ms);
                }
            }
            (void)hipStreamSynchronize(s);
            dfa_batch_destroy(bt);
            if (rc) break;
            if (t_best < pick_ms) {
                pick_ms = t_best;
                pick = o;
            }
        }
        if (rc) break;
    }
    bool any_abs = false;
    for (size_t i = 0; i < count; ++i) any_abs = any_abs || dfas[i]->dev.nabs > 0;
    if (rc == DFA_OK && packed && any_abs) {
        // the best setting again with early exit at absorbing states
        dfa_match_opts_t o = pick;
        o.flags |= DFA_MATCH_EARLY_EXIT;
        dfa_batch_t *bt = nullptr;
        rc = dfa_batch_create(dfas, d_inputs, lens, count, &o, &bt);
        double t_best = 1e30;
        for (int rep = 0; rep < 3 && rc == DFA_OK; ++rep) {
            if (rep > 0) (void)hipEventRecord(a, s);
            rc = dfa_batch_run(bt, stream, res);
            if (rep > 0) {
                (void)hipEventRecord(b, s);
                (void)hipEventSynchronize(b);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, a, b);
                t_best = std::min<double>(t_best, ms);
            }
        }
        (void)hipStreamSynchronize(s);
        if (bt) dfa_batch_destroy(bt);
        if (rc == DFA_OK && t_best < pick_ms) {
            pick_ms = t_best;
            pick = o;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(res);
    if (rc) return rc;
    *best = pick;
    if (best_ms) *best_ms = pick_ms;
    return DFA_OK;
}

namespace dfaspec {
bool timing_begin(hipStream_t s, hipEvent_t ev[4]) {
    Workspace *ws = workspace_for(s);
    if (!ws || !ws->timing) return false;
    for (int k = 0; k < 4; ++k) ev[k] = nullptr;
    for (int k = 0; k < 4; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(ev[j]);
            (void)hipGetLastError();
            return false;
        }
    (void)hipEventRecord(ev[0], s);
    return true;
}

int timing_end(hipStream_t s, hipEvent_t ev[4]) {
    Workspace *ws = workspace_for(s);
    if (!ws) return fail(DFA_E_DEVICE, "no HIP device");
    hipError_t e = hipEventRecord(ev[3], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ws->stamps.push_back({ev[0], ev[1], ev[2], ev[3], nullptr, nullptr});
    return DFA_OK;
}
}  // namespace dfaspec

extern "C" int dfa_timing_enable(void *stream, int on) {
    Workspace *ws = workspace_for((hipStream_t)stream);
    if (!ws) return fail(DFA_E_DEVICE, "no HIP device");
    ws->timing = on != 0;
    return DFA_OK;
}

extern "C" int dfa_timing_read_ex(void *stream, double *matcher_ms, double *call_ms,
                                  double *kernel_ms, uint32_t *calls) {
    Workspace *ws = workspace_for((hipStream_t)stream);
    if (!ws) return fail(DFA_E_DEVICE, "no HIP device");
    double m = 0.0, c = 0.0, k = 0.0;
    int rc = DFA_OK;
    for (auto &st : ws->stamps) {
        float a = 0.f, b = 0.f, x = 0.f;
        hipError_t e = hipEventSynchronize(st.end);
        if (e == hipSuccess) e = hipEventElapsedTime(&a, st.before_match, st.after_match);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, st.begin, st.end);
        if (e == hipSuccess && st.kern_begin) e = hipEventElapsedTime(&x, st.kern_begin, st.kern_end);
        else x = a;
        if (e != hipSuccess && rc == DFA_OK) rc = hip_fail(e, "dfa_timing_read");
        m += a;
        c += b;
        k += x;
        (void)hipEventDestroy(st.begin);
        (void)hipEventDestroy(st.before_match);
        (void)hipEventDestroy(st.after_match);
        (void)hipEventDestroy(st.end);
        if (st.kern_begin) (void)hipEventDestroy(st.kern_begin);
        if (st.kern_end) (void)hipEventDestroy(st.kern_end);
    }
    if (calls) *calls = (uint32_t)ws->stamps.size();
    ws->stamps.clear();
    if (matcher_ms) *matcher_ms = m;
    if (call_ms) *call_ms = c;
    if (kernel_ms) *kernel_ms = k;
    return rc;
}

extern "C" int dfa_timing_read(void *stream, double *matcher_ms, double *call_ms,
                               uint32_t *calls) {
    return dfa_timing_read_ex(stream, matcher_ms, call_ms, nullptr, calls);
}

extern "C" const char *dfa_strerror(int status) {
    switch (status) {
        case DFA_OK: return "ok";
        case DFA_E_INVAL: return "invalid argument";
        case DFA_E_NOMEM: return "out of memory";
        case DFA_E_DEVICE: return "HIP runtime error";
        case DFA_E_SYMBOL: return "input byte outside the alphabet";
        case DFA_E_TOOBIG: return "exceeds a device limit";
        case DFA_E_SPECULATION: return "speculation invariant violated";
        case DFA_E_BUSY: return "server busy";
        case DFA_E_NOTREADY: return "not ready";
        default: return "unknown status";
    }
}

extern "C" const char *dfa_last_error(void) { return dfaspec::g_last_error.c_str(); }
