// Host multicore speculative matcher (Section 4, Algorithm 3), with the
// capacity-weighted partition of Eqs. (1)-(7) and (10) and the ordered merge
// of Eq. (8).  One std::thread per processor.  This library is independent of
// the GPU library: it keeps its own class-compressed table and sets.
#include "../../include/dfa_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr int kOk = 0, kInval = -1, kNomem = -2, kSymbol = -4, kSpeculation = -6;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint8_t kNoClass = 0xFF;   // class numbers are < 256

}  // namespace

struct dfa_host {
    uint32_t nq = 0, q0 = 0, nclass = 0;
    uint8_t cls[256];                     // byte -> class, kNoClass outside Sigma
    uint16_t cls16[256];                  // same, 0xFFFF outside Sigma
    std::vector<uint32_t> table;          // class-major: table[c * nq + q] = delta(q, c)
    std::vector<uint8_t> accept, absorbing;
    std::vector<std::vector<uint32_t>> iset;   // per class: I_c (Eq. 11) without absorbing states
    uint32_t imax = 0;
};

namespace {

// Walks [b, e) from every state of `cur` at once; returns false on a byte
// outside Sigma.
bool walk_set(const dfa_host *d, const uint8_t *b, const uint8_t *e, uint32_t *cur, size_t m) {
    const uint32_t nq = d->nq;
    const uint32_t *T = d->table.data();
    constexpr size_t kBlock = 4096;
    uint16_t cbuf[kBlock];
    for (const uint8_t *p = b; p < e; p += kBlock) {
        const size_t len = std::min<size_t>(kBlock, (size_t)(e - p));
        uint16_t bad = 0;
        for (size_t i = 0; i < len; ++i) {
            const uint16_t c = d->cls16[p[i]];
            bad |= (uint16_t)(c >> 15);
            cbuf[i] = c;
        }
        if (bad) return false;
        if (m == 1) {
            uint32_t s = cur[0];
            for (size_t i = 0; i < len; ++i) s = T[(size_t)cbuf[i] * nq + s];
            cur[0] = s;
        } else {
            for (size_t i = 0; i < len; ++i) {
                const uint32_t *col = T + (size_t)cbuf[i] * nq;
                for (size_t j = 0; j < m; ++j) cur[j] = col[cur[j]];
            }
        }
    }
    return true;
}

}  // namespace

extern "C" int dfa_host_create(const uint32_t *delta, uint32_t num_states, uint32_t num_symbols,
                               uint32_t q0, const uint32_t *accepting, uint32_t num_accepting,
                               const uint8_t *byte_to_symbol, dfa_host_t **out) {
    if (!out) return kInval;
    *out = nullptr;
    if (!delta || num_states == 0 || num_symbols == 0 || num_symbols > 256 || q0 >= num_states)
        return kInval;
    if (num_accepting && !accepting) return kInval;
    if (!byte_to_symbol && num_symbols != 256) return kInval;
    const uint32_t nq = num_states;
    for (uint64_t i = 0; i < (uint64_t)nq * num_symbols; ++i)
        if (delta[i] >= nq) return kInval;
    dfa_host *d = new (std::nothrow) dfa_host();
    if (!d) return kNomem;
    d->nq = nq;
    d->q0 = q0;
    d->accept.assign(nq, 0);
    for (uint32_t k = 0; k < num_accepting; ++k) {
        if (accepting[k] >= nq) {
            delete d;
            return kInval;
        }
        d->accept[accepting[k]] = 1;
    }
    // classes: symbols with identical columns, numbered by first occurrence
    std::map<std::vector<uint32_t>, uint32_t> col_class;
    std::vector<int> sym_class(num_symbols, -1);
    std::vector<uint32_t> class_sym;
    for (int b = 0; b < 256; ++b) {
        const uint32_t a = byte_to_symbol ? byte_to_symbol[b] : (uint32_t)b;
        d->cls[b] = kNoClass;
        d->cls16[b] = 0xFFFF;
        if (a >= num_symbols) continue;
        if (sym_class[a] < 0) {
            std::vector<uint32_t> col(nq);
            for (uint32_t q = 0; q < nq; ++q) col[q] = delta[(uint64_t)q * num_symbols + a];
            auto it = col_class.find(col);
            if (it == col_class.end()) {
                it = col_class.emplace(std::move(col), (uint32_t)class_sym.size()).first;
                class_sym.push_back(a);
            }
            sym_class[a] = (int)it->second;
        }
        d->cls[b] = (uint8_t)sym_class[a];
        d->cls16[b] = (uint16_t)sym_class[a];
    }
    d->nclass = (uint32_t)class_sym.size();
    d->table.resize((size_t)d->nclass * nq);
    for (uint32_t c = 0; c < d->nclass; ++c)
        for (uint32_t q = 0; q < nq; ++q)
            d->table[(size_t)c * nq + q] = delta[(uint64_t)q * num_symbols + class_sym[c]];
    // absorbing states: every symbol of Sigma leads back to the state
    d->absorbing.assign(nq, 1);
    for (uint32_t q = 0; q < nq; ++q)
        for (uint32_t c = 0; c < d->nclass; ++c)
            if (d->table[(size_t)c * nq + q] != q) {
                d->absorbing[q] = 0;
                break;
            }
    // I_c: the image of Q under class c, absorbing states left out
    d->iset.resize(d->nclass);
    std::vector<uint8_t> seen(nq);
    for (uint32_t c = 0; c < d->nclass; ++c) {
        std::fill(seen.begin(), seen.end(), 0);
        for (uint32_t q = 0; q < nq; ++q) seen[d->table[(size_t)c * nq + q]] = 1;
        for (uint32_t q = 0; q < nq; ++q)
            if (seen[q] && !d->absorbing[q]) d->iset[c].push_back(q);
        d->imax = std::max<uint32_t>(d->imax, (uint32_t)d->iset[c].size());
    }
    *out = d;
    return kOk;
}

extern "C" void dfa_host_destroy(dfa_host_t *d) { delete d; }

extern "C" uint32_t dfa_host_imax(const dfa_host_t *d) { return d ? d->imax : 0; }

extern "C" int dfa_host_partition(uint64_t n, double m, const double *capacities, uint32_t P,
                                  uint64_t *starts) {
    if (!starts || P == 0 || !(m > 0.0)) return kInval;
    std::vector<double> w(P, 1.0);
    if (capacities) {
        double mean = 0.0;
        for (uint32_t k = 0; k < P; ++k) {
            if (!(capacities[k] > 0.0)) return kInval;
            mean += capacities[k];
        }
        mean /= P;
        for (uint32_t k = 0; k < P; ++k) w[k] = capacities[k] / mean;   // Eq. (1)
    }
    double rest = 0.0;
    for (uint32_t k = 1; k < P; ++k) rest += w[k];
    const double L0 = (double)n * m / (w[0] * m + rest);                 // Eq. (5) / (10)
    starts[0] = 0;
    double longer = 0.0;   // sum of L0 * w_i over chunks 1 .. k-1
    for (uint32_t k = 1; k < P; ++k) {
        // Eq. (6): chunk k starts after chunk 0 (length L0 * w_0) and chunks
        // 1 .. k-1 (length L0 * w_i / m each, Eq. (2) with weights)
        const double pos = std::floor(L0 * w[0] + longer / m);
        uint64_t s = pos <= 0.0 ? 0 : (uint64_t)pos;
        s = std::min<uint64_t>(std::max<uint64_t>(s, starts[k - 1]), n);
        starts[k] = s;
        longer += L0 * w[k];
    }
    starts[P] = n;
    return kOk;
}

extern "C" int dfa_host_profile(const dfa_host_t *d, const uint8_t *sample, size_t len,
                                uint32_t threads, double *capacities) {
    if (!d || !capacities || threads == 0 || (len && !sample)) return kInval;
    std::vector<std::thread> pool;
    std::vector<uint32_t> sink(threads);
    std::atomic<uint32_t> ready{0};
    for (uint32_t k = 0; k < threads; ++k)
        pool.emplace_back([&, k]() {
            ready.fetch_add(1);
            while (ready.load() < threads) std::this_thread::yield();
            const auto t0 = std::chrono::steady_clock::now();
            uint32_t s = d->q0;
            const uint32_t *T = d->table.data();
            for (size_t i = 0; i < len; ++i) {
                const uint16_t c = d->cls16[sample[i]];
                if (c != 0xFFFF) s = T[(size_t)c * d->nq + s];
            }
            const double sec =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            sink[k] = s;
            capacities[k] = (double)len / std::max(sec, 1e-9);
        });
    for (auto &t : pool) t.join();
    return kOk;
}

extern "C" int dfa_host_match(const dfa_host_t *d, const uint8_t *input, size_t len,
                              uint32_t threads, const double *capacities, uint32_t start_state,
                              uint32_t *final_state, int *accepted) {
    if (!d || !final_state || !accepted || (len && !input)) return kInval;
    if (start_state == kNone) start_state = d->q0;
    if (start_state >= d->nq) return kInval;
    if (threads == 0) threads = std::max(1u, std::thread::hardware_concurrency());
    if (len == 0) {
        *final_state = start_state;
        *accepted = d->accept[start_state];
        return kOk;
    }
    const uint32_t P = threads;
    std::vector<uint64_t> starts(P + 1);
    int rc = dfa_host_partition(len, std::max<double>(d->imax, 1.0), capacities, P, starts.data());
    if (rc) return rc;
    // the chunks in order, empty ones dropped; the first starts at 0
    std::vector<std::pair<uint64_t, uint64_t>> chunks;
    for (uint32_t k = 0; k < P; ++k)
        if (starts[k + 1] > starts[k]) chunks.push_back({starts[k], starts[k + 1]});
    const size_t nc = chunks.size();
    // per chunk i >= 1: its set I_sigma and the end state of each member (L_i)
    std::vector<const std::vector<uint32_t> *> sets(nc, nullptr);
    std::vector<std::vector<uint32_t>> ends(nc);
    std::vector<uint8_t> ok(nc, 1);
    uint32_t first_end = start_state;
    for (size_t i = 1; i < nc; ++i) {
        const uint8_t c = d->cls[input[chunks[i].first - 1]];
        if (c == kNoClass) return kSymbol;
        sets[i] = &d->iset[c];
        ends[i] = *sets[i];
    }
    std::vector<std::thread> pool;
    pool.reserve(nc);
    for (size_t i = 0; i < nc; ++i)
        pool.emplace_back([&, i]() {
            const uint8_t *b = input + chunks[i].first, *e = input + chunks[i].second;
            if (i == 0)
                ok[i] = walk_set(d, b, e, &first_end, 1);
            else
                ok[i] = walk_set(d, b, e, ends[i].data(), ends[i].size());
        });
    for (auto &t : pool) t.join();
    for (size_t i = 0; i < nc; ++i)
        if (!ok[i]) return kSymbol;
    // Eq. (8): the true start of chunk i is the end of chunk i-1
    uint32_t s = first_end;
    for (size_t i = 1; i < nc; ++i) {
        if (d->absorbing[s]) continue;            // an absorbing state maps to itself
        const auto &S = *sets[i];
        auto it = std::lower_bound(S.begin(), S.end(), s);
        if (it == S.end() || *it != s) return kSpeculation;
        s = ends[i][(size_t)(it - S.begin())];
    }
    *final_state = s;
    *accepted = d->accept[s];
    return kOk;
}
