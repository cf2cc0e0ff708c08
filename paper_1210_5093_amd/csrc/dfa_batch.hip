// Batched membership tests: many (DFA, string) pairs of uneven size in one
// persistent matcher launch.
//
// The paper's representation stores several DFAs in one table array and
// several strings in one input array, so one run can match many of them
// (Section 5, SBase/IBase).  Here a batch is planned once on the host: every
// string is cut into chunks, the (string, chunk) items are grouped into tasks
// of up to one chunk per wavefront of a workgroup, tasks of one DFA are
// adjacent (so a workgroup re-stages its LDS table only when the DFA
// changes), and DFAs with costlier chunks come first.  Persistent workgroups
// take tasks from a device counter.  Each chunk is matched from its one-symbol
// initial-state set exactly as in the single-string path; the per-string maps
// are then composed level by level (Eq. 9), all strings of a level in one
// launch, and each string's top map yields its final state.
//
// dfa_batch_run does no host work and allocates nothing, so it can be
// captured into a HIP graph and replayed.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>

#include "dfa_walk1.h"

namespace dfaspec {

constexpr uint32_t kBatchLevels = 12;
constexpr uint32_t kBatchWaves = 8;        // chunks per task = wavefronts per workgroup

struct BatchReq {
    const uint8_t *in;
    uint64_t n;
    uint64_t chunk;
    uint32_t nch;
    uint32_t dfa;          // index into the batch's DFA array
    uint32_t stride;       // map entries per chunk (the DFA's I_max, padded)
    uint32_t group;        // compose fan-in
    uint32_t levels;       // compose levels above level 0
    uint32_t start;
    uint32_t count[kBatchLevels];
    uint64_t map_off[kBatchLevels];
    uint64_t size_off[kBatchLevels];
};

struct BatchTask {
    uint32_t req;
    uint32_t chunk0;
    uint32_t nchunks;
    uint32_t dfa;
};

struct BatchGroup {
    uint32_t req;
    uint32_t g;
};

struct BatchArgs {
    const DevDFA *dfas;
    const BatchReq *reqs;
    const BatchTask *tasks;
    uint32_t ntasks;
    uint32_t *counter;
    uint16_t *maps;
    uint16_t *msize;
};

__global__ void k_batch_reset(uint32_t *counter) {
    if (threadIdx.x == 0) *counter = 0;
}

__global__ __launch_bounds__(512, 8) void k_batch_match(BatchArgs b) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_task;
    uint32_t cur_dfa = 0xFFFFFFFFu;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    while (true) {
        if (threadIdx.x == 0) s_task = atomicAdd(b.counter, 1u);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_task);   // uniform: scalar loads below
        __syncthreads();
        if (t >= b.ntasks) break;
        const BatchTask task = b.tasks[t];
        const DevDFA d = b.dfas[task.dfa];
        if (task.dfa != cur_dfa) {
            const uint4 *src = reinterpret_cast<const uint4 *>(d.table);
            uint4 *dst = reinterpret_cast<uint4 *>(smem);
            for (uint32_t i = threadIdx.x; i < d.table_bytes / 16; i += blockDim.x) dst[i] = src[i];
            const uint4 *lsrc = reinterpret_cast<const uint4 *>(d.lut);
            uint4 *ldst = reinterpret_cast<uint4 *>(smem + d.table_bytes);
            for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x) ldst[i] = lsrc[i];
            __syncthreads();
            cur_dfa = task.dfa;
        }
        if (wave < task.nchunks) {
            const BatchReq &rq = b.reqs[task.req];
            MatchArgs a;
            a.d = d;
            a.in = rq.in;
            a.n = rq.n;
            a.chunk = rq.chunk;
            a.nch = rq.nch;
            a.start = rq.start;
            a.mode = 1;
            a.stride = rq.stride;
            a.maps = b.maps + rq.map_off[0];
            a.msize = b.msize + rq.size_off[0];
            // 6 slots (384 states per pass) keep this kernel within 64 VGPRs
            match_one_chunk<6>(a, smem, reinterpret_cast<const uint32_t *>(smem + d.table_bytes),
                               task.chunk0 + wave, lane);
        }
        __syncthreads();   // every wave is done with this table before it may change
    }
}

// One workgroup per (string, group) of compose level l -> l + 1.
__global__ __launch_bounds__(256) void k_batch_compose(const BatchReq *__restrict__ reqs,
                                                       const BatchGroup *__restrict__ groups,
                                                       uint32_t l, uint16_t *__restrict__ maps,
                                                       uint16_t *__restrict__ msize) {
    extern __shared__ __align__(16) uint16_t sm[];
    __shared__ uint32_t flag;
    const BatchGroup gr = groups[blockIdx.x];
    const BatchReq &rq = reqs[gr.req];
    const uint32_t G = rq.group, stride = rq.stride;
    const uint32_t first = gr.g * G;
    const uint32_t cnt = min(G, rq.count[l] - first);
    const uint16_t *in_maps = maps + rq.map_off[l];
    const uint16_t *in_size = msize + rq.size_off[l];
    if (threadIdx.x == 0) flag = 0;
    __syncthreads();
    if (threadIdx.x < cnt && (in_size[first + threadIdx.x] & kFlagSymbol)) atomicOr(&flag, 1u);
    const uint16_t *src = in_maps + (size_t)first * stride;
    for (uint32_t i = threadIdx.x; i < cnt * stride; i += blockDim.x) sm[i] = src[i];
    __syncthreads();
    const uint32_t m = in_size[first] & 0x7FFFu;
    compose_staged(sm, cnt, stride, m, maps + rq.map_off[l + 1] + (size_t)gr.g * stride);
    if (threadIdx.x == 0)
        msize[rq.size_off[l + 1] + gr.g] = (uint16_t)(m | (flag ? kFlagSymbol : 0));
}

__global__ void k_batch_finalize(const DevDFA *__restrict__ dfas, const BatchReq *__restrict__ reqs,
                                 uint32_t count, const uint16_t *__restrict__ maps,
                                 const uint16_t *__restrict__ msize, uint32_t *__restrict__ results) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const BatchReq &rq = reqs[i];
    const DevDFA &d = dfas[rq.dfa];
    uint32_t fin = 0xFFFFFFFFu, acc = 0, flags = 0;
    if (rq.nch == 0) {
        fin = rq.start;
    } else {
        const uint32_t v = maps[rq.map_off[rq.levels]];
        if (msize[rq.size_off[rq.levels]] & kFlagSymbol)
            flags |= DFA_FLAG_SYMBOL;
        else if (!(v & kTerm) || (v & 0x7FFFu) >= d.nq)
            flags |= DFA_FLAG_SPECULATION;
        else
            fin = v & 0x7FFFu;
    }
    if (!flags) acc = (d.accept_bits[fin >> 5] >> (fin & 31)) & 1u;
    results[4 * i + 0] = fin;
    results[4 * i + 1] = acc;
    results[4 * i + 2] = flags;
    results[4 * i + 3] = rq.nch;
}

// ---------------------------------------------------------------------------
// Host side: planning (pure host work) and launching (device work only)
// ---------------------------------------------------------------------------
namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
bool g_batch_attr_set = false;
}  // namespace

int plan_batch(const dfa_t *const *dfas, const uint8_t *const *d_inputs, const size_t *lens,
               size_t count, uint64_t chunk_req, BatchPlan *out) {
    BatchPlan &P = *out;
    P = BatchPlan();
    if (count && (!dfas || !d_inputs || !lens)) return fail(DFA_E_INVAL, "batch plan: NULL argument");
    if (count > 0xFFFFFFFFull) return fail(DFA_E_TOOBIG, "batch plan: too many strings");
    const int lds = device_lds_bytes();
    const int cus = std::max(device_cu_count(), 1);
    if (lds <= 0) return fail(DFA_E_DEVICE, "no HIP device");
    P.count = (uint32_t)count;

    // distinct DFAs
    std::map<const dfa_t *, uint32_t> index;
    std::vector<const dfa_t *> uniq;
    for (size_t i = 0; i < count; ++i) {
        if (!dfas[i]) return fail(DFA_E_INVAL, "batch plan: NULL dfa");
        if (lens[i] && !d_inputs[i]) return fail(DFA_E_INVAL, "batch plan: NULL input");
        if (index.emplace(dfas[i], (uint32_t)uniq.size()).second) uniq.push_back(dfas[i]);
    }
    uint32_t max_table = 0;
    for (auto *d : uniq) max_table = std::max(max_table, d->dev.table_bytes);

    // chunk length: about four chunks per resident wavefront over the whole batch
    uint64_t total = 0;
    for (size_t i = 0; i < count; ++i) total += lens[i];
    const uint32_t per_cu =
        std::max<uint32_t>(1u, std::min<uint32_t>(4u, (uint32_t)lds / (max_table + 1024)));
    P.blocks = (uint32_t)cus * per_cu;
    P.threads = kBatchWaves * 64;
    P.lds_match = max_table + 1024;
    uint64_t chunk = chunk_req;
    if (!chunk) {
        const uint64_t target = 4ull * P.blocks * kBatchWaves;
        chunk = std::max<uint64_t>(1024, (total / std::max<uint64_t>(target, 1) + 63) / 64 * 64);
        chunk = std::min<uint64_t>(chunk, 1u << 20);
    }
    P.chunk = chunk;

    // per-string plan, arenas
    std::vector<BatchReq> reqs(count);
    uint64_t map_entries = 0, size_entries = 0;
    size_t compose_stage = 0;
    for (size_t i = 0; i < count; ++i) {
        const dfa_t *d = dfas[i];
        BatchReq &r = reqs[i];
        std::memset(&r, 0, sizeof(r));
        r.in = d_inputs[i];
        r.n = lens[i];
        r.chunk = chunk;
        const uint64_t nch = (lens[i] + chunk - 1) / chunk;
        if (nch > 0xFFFFFFFFull) return fail(DFA_E_TOOBIG, "batch plan: too many chunks");
        r.nch = (uint32_t)nch;
        r.dfa = index[d];
        r.start = d->dev.q0;
        r.stride = (std::max<uint32_t>(d->setmax_host[1], 1u) + 7u) & ~7u;
        r.group = (uint32_t)std::max<uint64_t>(
            2, std::min<uint64_t>(64, (96u * 1024u) / (2ull * r.stride)));
        compose_stage = std::max(compose_stage, (size_t)r.group * r.stride * 2);
        uint64_t c = nch;
        uint32_t L = 0;
        if (nch) {
            r.count[0] = (uint32_t)c;
            r.map_off[0] = map_entries;
            r.size_off[0] = size_entries;
            map_entries += c * r.stride;
            size_entries += c;
            while (c > 1) {
                if (L + 1 >= kBatchLevels) return fail(DFA_E_TOOBIG, "batch plan: too many levels");
                c = (c + r.group - 1) / r.group;
                ++L;
                r.count[L] = (uint32_t)c;
                r.map_off[L] = map_entries;
                r.size_off[L] = size_entries;
                map_entries += c * r.stride;
                size_entries += c;
            }
        }
        r.levels = L;
        P.max_levels = std::max(P.max_levels, L);
    }
    P.lds_compose = compose_stage;

    // tasks: strings grouped by DFA, DFAs with costlier chunks first
    std::vector<uint32_t> dorder(uniq.size());
    std::iota(dorder.begin(), dorder.end(), 0u);
    std::sort(dorder.begin(), dorder.end(), [&](uint32_t x, uint32_t y) {
        return uniq[x]->info.mean_iset > uniq[y]->info.mean_iset;
    });
    std::vector<std::vector<uint32_t>> by_dfa(uniq.size());
    for (size_t i = 0; i < count; ++i) by_dfa[reqs[i].dfa].push_back((uint32_t)i);
    std::vector<BatchTask> tasks;
    for (uint32_t di : dorder)
        for (uint32_t i : by_dfa[di])
            for (uint32_t c0 = 0; c0 < reqs[i].nch; c0 += kBatchWaves)
                tasks.push_back({i, c0, std::min<uint32_t>(kBatchWaves, reqs[i].nch - c0), di});
    if (tasks.size() > 0xFFFFFFFFull) return fail(DFA_E_TOOBIG, "batch plan: too many tasks");
    P.ntasks = (uint32_t)tasks.size();

    // compose groups per level
    std::vector<BatchGroup> groups;
    P.groups_per_level.assign(P.max_levels, 0);
    P.group_base.assign(P.max_levels, 0);
    for (uint32_t l = 0; l < P.max_levels; ++l) {
        P.group_base[l] = groups.size();
        for (size_t i = 0; i < count; ++i)
            if (reqs[i].levels > l)
                for (uint32_t g = 0; g < reqs[i].count[l + 1]; ++g)
                    groups.push_back({(uint32_t)i, g});
        P.groups_per_level[l] = (uint32_t)(groups.size() - P.group_base[l]);
    }

    // layout: descriptors (uploaded), counter, arenas (device only)
    std::vector<DevDFA> ddfas(uniq.size());
    for (size_t k = 0; k < uniq.size(); ++k) ddfas[k] = uniq[k]->dev;
    size_t at = 0;
    auto place = [&](size_t bytes) { size_t o = at; at = align256(at + bytes); return o; };
    P.o_dfas = place(std::max<size_t>(ddfas.size(), 1) * sizeof(DevDFA));
    P.o_reqs = place(std::max<size_t>(reqs.size(), 1) * sizeof(BatchReq));
    P.o_tasks = place(std::max<size_t>(tasks.size(), 1) * sizeof(BatchTask));
    P.o_groups = place(std::max<size_t>(groups.size(), 1) * sizeof(BatchGroup));
    P.desc_bytes = at;
    P.o_counter = place(sizeof(uint32_t));
    P.o_maps = place(std::max<uint64_t>(map_entries, 1) * 2);
    P.o_msize = place(std::max<uint64_t>(size_entries, 1) * 2);
    P.total_bytes = at;
    P.desc.assign(P.desc_bytes, 0);
    std::memcpy(P.desc.data() + P.o_dfas, ddfas.data(), ddfas.size() * sizeof(DevDFA));
    if (!reqs.empty()) std::memcpy(P.desc.data() + P.o_reqs, reqs.data(), reqs.size() * sizeof(BatchReq));
    if (!tasks.empty())
        std::memcpy(P.desc.data() + P.o_tasks, tasks.data(), tasks.size() * sizeof(BatchTask));
    if (!groups.empty())
        std::memcpy(P.desc.data() + P.o_groups, groups.data(), groups.size() * sizeof(BatchGroup));
    if (!g_batch_attr_set) {
        if (allow_dynamic_lds(reinterpret_cast<const void *>(&k_batch_match), lds) != DFA_OK ||
            allow_dynamic_lds(reinterpret_cast<const void *>(&k_batch_compose), lds) != DFA_OK)
            return fail(DFA_E_DEVICE, "batch plan: cannot enable the device's LDS size");
        g_batch_attr_set = true;
    }
    return DFA_OK;
}

int launch_batch(const BatchPlan &P, void *dev_base, hipStream_t s, uint32_t *d_results,
                 hipEvent_t ev_before_match, hipEvent_t ev_after_match) {
    if (!P.count) return DFA_OK;
    uint8_t *base = (uint8_t *)dev_base;
    const DevDFA *dfas = (const DevDFA *)(base + P.o_dfas);
    const BatchReq *reqs = (const BatchReq *)(base + P.o_reqs);
    const BatchGroup *groups = (const BatchGroup *)(base + P.o_groups);
    uint16_t *maps = (uint16_t *)(base + P.o_maps);
    uint16_t *msize = (uint16_t *)(base + P.o_msize);
    uint32_t *counter = (uint32_t *)(base + P.o_counter);
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, counter);
    BatchArgs a;
    a.dfas = dfas;
    a.reqs = reqs;
    a.tasks = (const BatchTask *)(base + P.o_tasks);
    a.ntasks = P.ntasks;
    a.counter = counter;
    a.maps = maps;
    a.msize = msize;
    if (ev_before_match) (void)hipEventRecord(ev_before_match, s);
    if (P.ntasks)
        hipLaunchKernelGGL(k_batch_match, dim3(P.blocks), dim3(P.threads), P.lds_match, s, a);
    if (ev_after_match) (void)hipEventRecord(ev_after_match, s);
    for (uint32_t l = 0; l < P.max_levels; ++l)
        if (P.groups_per_level[l])
            hipLaunchKernelGGL(k_batch_compose, dim3(P.groups_per_level[l]), dim3(256), P.lds_compose,
                               s, reqs, groups + P.group_base[l], l, maps, msize);
    hipLaunchKernelGGL(k_batch_finalize, dim3((P.count + 255) / 256), dim3(256), 0, s, dfas, reqs,
                       P.count, maps, msize, d_results);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DFA_OK : hip_fail(e, "batch launch");
}

}  // namespace dfaspec

using namespace dfaspec;

struct dfa_batch {
    int kind = 1;            // 1: one chunk per wavefront; 2: packed pairs (dfa_batch2.hip)
    BatchPlan plan;
    Batch2Plan plan2;
    void *blob = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t *graph_results = nullptr;
};

extern "C" int dfa_batch_create(const dfa_t *const *dfas, const uint8_t *const *d_inputs,
                                const size_t *lens, size_t count, const dfa_match_opts_t *opts,
                                dfa_batch_t **out) {
    if (!out) return fail(DFA_E_INVAL, "dfa_batch_create: out is NULL");
    *out = nullptr;
    const uint32_t look = opts ? opts->lookahead : 1u;
    if (look == 0 || look > 64)
        return fail(DFA_E_INVAL, "dfa_batch_create: lookahead must be 1 .. 64");
    std::unique_ptr<dfa_batch> b(new dfa_batch());
    // the packed-pair batch unless a DFA lacks a packed layout (or the
    // environment asks for the first-generation kernel: DFA_BATCH_KERNEL=1)
    const char *env = getenv("DFA_BATCH_KERNEL");
    const bool force1 = env && atoi(env) == 1;
    b->kind = (!force1 && (count == 0 || batch2_supported(dfas, count))) ? 2 : 1;
    if (b->kind == 1 && look != 1)
        return fail(DFA_E_INVAL, "dfa_batch_create: this batch needs one-symbol lookahead");
    int rc = b->kind == 2
                 ? plan_batch2(dfas, d_inputs, lens, count, opts ? opts->chunk_len : 0, look, &b->plan2,
                               opts ? opts->flags : 0u)
                 : plan_batch(dfas, d_inputs, lens, count, opts ? opts->chunk_len : 0, &b->plan);
    if (rc) return rc;
    const size_t total = b->kind == 2 ? b->plan2.total_bytes : b->plan.total_bytes;
    const size_t desc_bytes = b->kind == 2 ? b->plan2.desc_bytes : b->plan.desc_bytes;
    const void *desc = b->kind == 2 ? (const void *)b->plan2.desc.data() : (const void *)b->plan.desc.data();
    hipError_t e = hipMalloc(&b->blob, total);
    if (e != hipSuccess) return fail(DFA_E_NOMEM, "dfa_batch_create: hipMalloc failed");
    e = hipMemcpy(b->blob, desc, desc_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(b->blob);
        b->blob = nullptr;
        return hip_fail(e, "dfa_batch_create: hipMemcpy");
    }
    *out = b.release();
    return DFA_OK;
}

extern "C" int dfa_batch_run(dfa_batch_t *b, void *stream, uint32_t *d_results) {
    if (!b) return fail(DFA_E_INVAL, "dfa_batch_run: NULL batch");
    const uint32_t count = b->kind == 2 ? b->plan2.count : b->plan.count;
    if (count && !d_results) return fail(DFA_E_INVAL, "dfa_batch_run: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipEvent_t ev[4];
    const bool timed = hipStreamIsCapturing(s, &cap) == hipSuccess &&
                       cap == hipStreamCaptureStatusNone && timing_begin(s, ev);
    int rc = b->kind == 2 ? launch_batch2(b->plan2, b->blob, s, d_results, timed ? ev[1] : nullptr,
                                          timed ? ev[2] : nullptr)
                          : launch_batch(b->plan, b->blob, s, d_results, timed ? ev[1] : nullptr,
                                         timed ? ev[2] : nullptr);
    if (!timed) return rc;
    const int rc2 = timing_end(s, ev);
    return rc ? rc : rc2;
}

extern "C" int dfa_batch_graph_launch(dfa_batch_t *b, void *stream, uint32_t *d_results) {
    if (!b) return fail(DFA_E_INVAL, "dfa_batch_graph_launch: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(DFA_E_INVAL, "dfa_batch_graph_launch: capture needs a created stream, "
                                     "not the default stream");
    if (b->exec && b->graph_results != d_results) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    if (!b->exec) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        int rc = dfa_batch_run(b, stream, d_results);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        b->graph = g;
        b->graph_results = d_results;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    return e == hipSuccess ? DFA_OK : hip_fail(e, "hipGraphLaunch");
}

extern "C" void dfa_batch_destroy(dfa_batch_t *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->blob) (void)hipFree(b->blob);
    delete b;
}

extern "C" int dfa_batch_info(const dfa_batch_t *b, uint64_t *chunk_len, uint32_t *tasks) {
    if (!b) return fail(DFA_E_INVAL, "dfa_batch_info: NULL batch");
    if (chunk_len) *chunk_len = b->kind == 2 ? b->plan2.chunk : b->plan.chunk;
    if (tasks) *tasks = b->kind == 2 ? b->plan2.nchunks : b->plan.ntasks;
    return DFA_OK;
}
