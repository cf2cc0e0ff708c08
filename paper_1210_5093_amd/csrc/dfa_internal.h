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

// Device-resident compiled DFA, passed by value to kernels.
struct DevDFA {
    const uint16_t *table;       // [K][Qp] class-major; entry = 2 * delta(s, c)
    const uint32_t *lut;         // [256]: (class << 24) | class * colstride; kLutInvalid
    const uint32_t *set_off[2];  // [K+1] per lookahead mode (0: all states, 1: I_c)
    const uint16_t *set_st[2];   // states of each class's set, ascending
    const uint16_t *pos[2];      // [K][Q]: position of s in the class's set,
                                 //  kTerm|s for absorbing s, kBadPos otherwise
    const uint32_t *accept_bits; // ceil(Q/32) words
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
};

namespace dfaspec {

// Thread-local last-error message helpers (dfa_api.cpp).
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Kernel launchers (dfa_kernels.hip).
struct Workspace;
constexpr uint32_t kMaxLevels = 40;  // fan-in >= 2 and < 2^32 chunks need at most 32
struct MatchPlan {
    uint64_t n = 0;
    uint64_t chunk = 0;
    uint32_t nch = 0;
    uint32_t lookahead = 1;
    uint32_t stride = 0;         // map entries per chunk (>= largest set)
    uint32_t group = 0;          // maps combined per compose step
    uint32_t levels = 0;         // compose levels above level 0
    uint32_t level_count[kMaxLevels] = {};
    uint64_t level_off[kMaxLevels] = {};  // entry offsets of each level's maps
    uint64_t msize_off[kMaxLevels] = {};  // entry offsets of each level's sizes
    uint64_t map_entries = 0;    // total uint16 entries for maps
    uint64_t msize_entries = 0;
    uint32_t waves_per_block = 4;
    uint32_t blocks = 0;
};

int plan_match(const dfa *d, uint64_t n, uint64_t chunk_req, uint32_t lookahead, MatchPlan *p);
// ev_after_match (may be null) is recorded right after the matcher kernel.
int launch_match(const dfa *d, const uint8_t *d_in, uint32_t start, const MatchPlan &p,
                 uint16_t *maps, uint16_t *msize, uint16_t *bvals, uint32_t *d_result,
                 uint32_t *d_boundaries, hipStream_t s, hipEvent_t ev_after_match);
int device_lds_bytes();
int device_cu_count();

}  // namespace dfaspec
