// dfa_create / dfa_destroy / dfa_info: validate a DFA, compress its alphabet
// into equivalence classes, find its absorbing states and initial-state sets,
// and upload everything to the device once.
//
//  * Automaton (Q, Sigma, delta, q0, F) with a total delta: Section 2.1.
//  * Absorbing states: the paper assumes one error/sink state q_e and leaves
//    it out of every initial-state set (Section 2.1, Algorithm 3).  Here every
//    state with a self-loop on all symbols is treated that way: if the true
//    state at a chunk start is absorbing, it stays so through the chunk, and
//    the map combination carries it unchanged.
//  * Initial-state sets I_sigma = {delta(x, sigma) : x in Q} minus the
//    absorbing states: Eq. (11), first loop of Algorithm 3; I_max: Eq. (12).
//  * Alphabet classes: bytes whose delta-columns are identical share one
//    class (numbered by first byte occurrence).  I_sigma depends only on the
//    column, so I_class = I_sigma for any sigma of the class.  The paper
//    maps characters to symbol indices (Section 5, the IBase array); the
//    class compression is this library's addition, so the table fits LDS.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <unordered_map>

#include "dfa_internal.h"

using namespace dfaspec;

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

extern "C" int dfa_create(const uint32_t *delta, uint32_t nq, uint32_t nsym, uint32_t q0,
                          const uint32_t *accepting, uint32_t nacc,
                          const uint8_t *byte_to_symbol, dfa_t **out) {
    if (!out) return fail(DFA_E_INVAL, "dfa_create: out is NULL");
    *out = nullptr;
    if (!delta) return fail(DFA_E_INVAL, "dfa_create: delta is NULL");
    if (nq == 0 || nq > kMaxStates)
        return fail(DFA_E_INVAL, "dfa_create: num_states must be in 1..32767");
    if (nsym == 0 || nsym > 256)
        return fail(DFA_E_INVAL, "dfa_create: num_symbols must be in 1..256");
    if (q0 >= nq) return fail(DFA_E_INVAL, "dfa_create: q0 out of range");
    if (nacc && !accepting) return fail(DFA_E_INVAL, "dfa_create: accepting is NULL");
    if (!byte_to_symbol && nsym != 256)
        return fail(DFA_E_INVAL, "dfa_create: byte_to_symbol may be NULL only with 256 symbols");
    for (uint64_t i = 0; i < (uint64_t)nq * nsym; ++i)
        if (delta[i] >= nq) return fail(DFA_E_INVAL, "dfa_create: delta entry out of range");
    for (uint32_t k = 0; k < nacc; ++k)
        if (accepting[k] >= nq) return fail(DFA_E_INVAL, "dfa_create: accepting state out of range");

    uint8_t b2s[256];
    for (int b = 0; b < 256; ++b) b2s[b] = byte_to_symbol ? byte_to_symbol[b] : (uint8_t)b;

    // ---- absorbing states -------------------------------------------------
    std::vector<uint8_t> absorbing(nq, 1);
    for (uint32_t s = 0; s < nq; ++s)
        for (uint32_t a = 0; a < nsym; ++a)
            if (delta[(uint64_t)s * nsym + a] != s) { absorbing[s] = 0; break; }
    uint32_t nabs = 0;
    for (auto v : absorbing) nabs += v;

    // ---- alphabet classes over the bytes in Sigma ------------------------
    std::vector<int> sym_class(nsym, -1);
    std::vector<uint32_t> class_sym;  // representative symbol of each class
    std::unordered_map<std::string, int> col_id;
    std::string col(nq * sizeof(uint32_t), '\0');
    int byte_class[256];
    for (int b = 0; b < 256; ++b) {
        uint32_t a = b2s[b];
        if (a >= nsym) { byte_class[b] = -1; continue; }
        if (sym_class[a] < 0) {
            for (uint32_t s = 0; s < nq; ++s) {
                uint32_t t = delta[(uint64_t)s * nsym + a];
                std::memcpy(&col[s * 4], &t, 4);
            }
            auto it = col_id.find(col);
            if (it == col_id.end()) {
                int c = (int)class_sym.size();
                col_id.emplace(col, c);
                class_sym.push_back(a);
                sym_class[a] = c;
            } else {
                sym_class[a] = it->second;
            }
        }
        byte_class[b] = sym_class[a];
    }
    const uint32_t K = (uint32_t)std::max<size_t>(class_sym.size(), 1);
    const uint32_t Qp = (nq + 1) & ~1u;            // even, so columns stay 4-byte aligned
    const uint32_t colstride = 2 * Qp;
    const uint64_t table_bytes = align_up((uint64_t)K * colstride, 16);
    const int lds = device_lds_bytes();
    if (lds <= 0) return fail(DFA_E_DEVICE, "dfa_create: no HIP device");
    if (table_bytes + 1024 > (uint64_t)lds)
        return fail(DFA_E_TOOBIG, "dfa_create: compressed table (" + std::to_string(table_bytes) +
                                      " B) does not fit in LDS");

    // ---- class-major table, LUT ------------------------------------------
    std::vector<uint16_t> table(table_bytes / 2, 0);
    for (uint32_t c = 0; c < class_sym.size(); ++c)
        for (uint32_t s = 0; s < nq; ++s)
            table[(size_t)c * Qp + s] = (uint16_t)(2 * delta[(uint64_t)s * nsym + class_sym[c]]);
    std::vector<uint32_t> lut(256);
    for (int b = 0; b < 256; ++b)
        lut[b] = byte_class[b] < 0 ? kLutInvalid
                                   : ((uint32_t)byte_class[b] << 24) | ((uint32_t)byte_class[b] * colstride);

    // Fault injection for tests of the speculation check: with the
    // environment variable DFA_DROP_STATE=s, state s is left out of every
    // initial-state set (one-symbol and precomputed multi-symbol sets), so a
    // chunk whose true start state is s has no walk from it and the result
    // must carry DFA_FLAG_SPECULATION rather than a state.
    uint32_t dropped = 0xFFFFFFFFu;
    if (const char *ds = std::getenv("DFA_DROP_STATE")) dropped = (uint32_t)std::strtoul(ds, nullptr, 10);

    // ---- per-class sets: mode 1 = I_c (Eq. 11), mode 0 = all non-absorbing
    std::vector<uint32_t> off[2];
    std::vector<uint16_t> st[2], pos[2];
    uint32_t setmax[2] = {0, 0};
    double mean_iset = 0.0;
    int nvalid_bytes = 0;
    std::vector<uint32_t> class_size(K, 0);
    for (int mode = 0; mode < 2; ++mode) {
        off[mode].assign(K + 1, 0);
        pos[mode].assign((size_t)K * nq, kBadPos);
        for (uint32_t c = 0; c < K; ++c) {
            std::vector<uint8_t> in(nq, 0);
            if (mode == 1) {
                if (c < class_sym.size())
                    for (uint32_t x = 0; x < nq; ++x) in[delta[(uint64_t)x * nsym + class_sym[c]]] = 1;
            } else {
                std::fill(in.begin(), in.end(), 1);
            }
            off[mode][c] = (uint32_t)st[mode].size();
            for (uint32_t s = 0; s < nq; ++s) {
                if (absorbing[s]) {
                    pos[mode][(size_t)c * nq + s] = (uint16_t)(kTerm | s);
                } else if (in[s] && s != dropped) {
                    pos[mode][(size_t)c * nq + s] = (uint16_t)(st[mode].size() - off[mode][c]);
                    st[mode].push_back((uint16_t)s);
                }
            }
            uint32_t sz = (uint32_t)st[mode].size() - off[mode][c];
            setmax[mode] = std::max(setmax[mode], sz);
            if (mode == 1) class_size[c] = sz;
        }
        off[mode][K] = (uint32_t)st[mode].size();
        if (st[mode].empty()) st[mode].push_back(0);  // keep the device array non-empty
    }
    double slots = 0.0;   // wavefront slots the one-chunk-per-wave matcher would spend
    for (int b = 0; b < 256; ++b)
        if (byte_class[b] >= 0) {
            mean_iset += class_size[byte_class[b]];
            slots += 64.0 * ((class_size[byte_class[b]] + 63) / 64);
            ++nvalid_bytes;
        }
    const double wave_util = slots > 0 ? mean_iset / slots : 0.0;
    if (nvalid_bytes) mean_iset /= nvalid_bytes;

    // ---- multi-symbol initial-state sets (Eq. 13; Algorithm 4 generalised)
    // Level k holds I_{c_1..c_k} for every class string: level 1 is I_c, and
    // level k is delta(level k-1, c_k) without absorbing states (absorbing
    // states stay absorbing, so this is the exact image of Q).  Levels are
    // added while they fit a budget of 2M states and 256K sets (a few ms;
    // 8 classes reach six symbols).
    std::vector<uint32_t> mset_off;
    std::vector<uint16_t> mset_st;
    uint32_t moff[kMaxMsetLevel + 1] = {0}, mst[kMaxMsetLevel + 1] = {0};
    uint32_t r0 = 0;
    double mset_mean_k[kMaxMsetLevel + 1] = {0.0};
    uint32_t mset_max_k[kMaxMsetLevel + 1] = {0};
    {
        const uint32_t Kc = (uint32_t)class_sym.size();
        std::vector<uint32_t> prev_off, cur_off;
        std::vector<uint16_t> prev_st, cur_st;
        if (Kc > 0) {
            // level 1 as stored (I_c); the images that seed level 2 keep a
            // state left out by fault injection (each level is the exact image
            // of Q; only the stored sets lack it)
            std::vector<uint32_t> st_off(off[1].begin(), off[1].begin() + Kc + 1);
            std::vector<uint16_t> st_st(st[1].begin(), st[1].begin() + off[1][Kc]);
            prev_off.assign(1, 0);
            for (uint32_t c = 0; c < Kc; ++c) {
                std::vector<uint8_t> in(nq, 0);
                for (uint32_t x = 0; x < nq; ++x) in[delta[(uint64_t)x * nsym + class_sym[c]]] = 1;
                for (uint32_t q = 0; q < nq; ++q)
                    if (in[q] && !absorbing[q]) prev_st.push_back((uint16_t)q);
                prev_off.push_back((uint32_t)prev_st.size());
            }
            r0 = 1;
            mset_mean_k[1] = (double)st_st.size() / Kc;
            mset_max_k[1] = setmax[1];
            moff[1] = 0;
            mst[1] = 0;
            mset_off = st_off;
            mset_st = st_st;
            std::vector<uint32_t> mark(nq, 0);
            uint32_t stamp = 0;
            for (uint32_t k = 2; k <= kMaxMsetLevel; ++k) {
                const uint64_t nsets = (uint64_t)(prev_off.size() - 1) * Kc;
                if (nsets > (1u << 18)) break;
                cur_off.assign(1, 0);
                cur_st.clear();
                bool over = false;
                for (uint64_t parent = 0; parent + 1 < prev_off.size() && !over; ++parent) {
                    for (uint32_t c = 0; c < Kc; ++c) {
                        ++stamp;
                        const size_t base = cur_st.size();
                        for (uint32_t j = prev_off[parent]; j < prev_off[parent + 1]; ++j) {
                            const uint32_t t = delta[(uint64_t)prev_st[j] * nsym + class_sym[c]];
                            if (!absorbing[t] && mark[t] != stamp) {
                                mark[t] = stamp;
                                cur_st.push_back((uint16_t)t);
                            }
                        }
                        std::sort(cur_st.begin() + base, cur_st.end());
                        cur_off.push_back((uint32_t)cur_st.size());
                        if (mset_st.size() + cur_st.size() > (1u << 21)) { over = true; break; }
                    }
                }
                if (over) break;
                // stored sets: the images without a state left out by fault injection
                std::vector<uint32_t> keep_off(1, 0);
                std::vector<uint16_t> keep_st;
                keep_st.reserve(cur_st.size());
                for (size_t q = 0; q + 1 < cur_off.size(); ++q) {
                    for (uint32_t j = cur_off[q]; j < cur_off[q + 1]; ++j)
                        if (cur_st[j] != dropped) keep_st.push_back(cur_st[j]);
                    keep_off.push_back((uint32_t)keep_st.size());
                }
                mset_mean_k[k] = keep_off.size() > 1 ? (double)keep_st.size() / (keep_off.size() - 1) : 0.0;
                for (size_t q = 0; q + 1 < keep_off.size(); ++q)
                    mset_max_k[k] = std::max<uint32_t>(mset_max_k[k], keep_off[q + 1] - keep_off[q]);
                moff[k] = (uint32_t)mset_off.size();
                mst[k] = (uint32_t)mset_st.size();
                mset_off.insert(mset_off.end(), keep_off.begin(), keep_off.end());
                mset_st.insert(mset_st.end(), keep_st.begin(), keep_st.end());
                prev_off.swap(cur_off);
                prev_st.swap(cur_st);
                r0 = k;
            }
        }
        if (mset_off.empty()) mset_off.assign(2, 0);
        if (mset_st.empty()) mset_st.assign(1, 0);
    }

    // ---- packed-pair matcher layouts -------------------------------------
    // Layout 1 keeps the byte code small (2 * class, one byte) and puts the
    // class offset inside a state row; rows are an odd number of dwords so
    // that distinct states of one column fall into distinct LDS banks.
    // Layout 2 (class-major, 16-bit codes) serves alphabets with more classes.
    // The direct variant indexes rows by the byte itself when every byte of
    // Sigma is below 128 (code = 2 * byte fits one byte), so that the matcher
    // can read the raw input.  Rows of R bytes overlap outside [lo, hi], the
    // bytes of Sigma; the image spans R * (nq - 1) + 256 bytes, so that every
    // address R * s + c (c even, c <= 254) lies inside it, and every word of it
    // that is not a table entry holds 0 (state 0's offset).
    uint32_t layout = 0, rowbytes = 0, direct = 0;
    std::vector<uint16_t> stab;
    std::vector<uint16_t> code(256, kCodeInvalid);
    int lo = -1, hi = -1;
    for (int b = 0; b < 256; ++b)
        if (byte_class[b] >= 0) { if (lo < 0) lo = b; hi = b; }
    const char *no_direct = std::getenv("DFA_DIRECT");   // "0": class rows only (diagnostic)
    if (lo >= 0 && hi < 128 && !(no_direct && no_direct[0] == '0')) {
        const uint32_t W = (uint32_t)(hi - lo + 1);
        uint32_t R1 = (2 * W + 3) / 4 * 4;
        if ((R1 / 4) % 2 == 0) R1 += 4;
        for (uint32_t R : {R1, 2 * W}) {
            const uint64_t span = (uint64_t)(nq - 1) * R + 256;
            if (span > 0x10000 || span + (uint64_t)nq * R / 16 + 1024 > (uint64_t)lds) continue;
            layout = 1;
            direct = 1;
            rowbytes = R;
            stab.assign(align_up(span, 16) / 2, 0);
            for (uint32_t q = 0; q < nq; ++q)
                for (int b = lo; b <= hi; ++b)
                    if (byte_class[b] >= 0)
                        stab[((size_t)q * R + 2 * (uint32_t)b) / 2] =
                            (uint16_t)(R * delta[(uint64_t)q * nsym + class_sym[byte_class[b]]]);
            for (int b = 0; b < 256; ++b)
                if (byte_class[b] >= 0) code[b] = (uint16_t)(2 * b);
            break;
        }
    }
    if (!direct) {
        uint32_t R = (2 * K + 3) / 4 * 4;
        if ((R / 4) % 2 == 0) R += 4;
        if (2 * K <= 255 && (uint64_t)(nq - 1) * R <= 0xFFFF && (uint64_t)nq * R + 1024 <= (uint64_t)lds) {
            layout = 1;
            rowbytes = R;
            stab.assign(align_up((size_t)nq * R, 16) / 2, 0);
            for (uint32_t s = 0; s < nq; ++s)
                for (uint32_t c = 0; c < class_sym.size(); ++c)
                    stab[(size_t)s * (R / 2) + c] = (uint16_t)(R * delta[(uint64_t)s * nsym + class_sym[c]]);
            for (int b = 0; b < 256; ++b)
                if (byte_class[b] >= 0) code[b] = (uint16_t)(2 * byte_class[b]);
        } else if ((uint64_t)(K - 1) * colstride < kCodeInvalid) {
            layout = 2;
            for (int b = 0; b < 256; ++b)
                if (byte_class[b] >= 0) code[b] = (uint16_t)((uint32_t)byte_class[b] * colstride);
        }
    }
    // staged image of the packed matcher: table, then the absorbing-state
    // bitmap indexed by (LDS state offset >> shift): R * s / 4 for layout 1
    // (R * s / 2 when a direct row is not a whole number of dwords), 2 * s / 2
    // for layout 2
    uint32_t abs_off = 0, abs_shift = 0;
    if (layout != 0) {
        if (layout == 2) {   // the class-major table itself
            stab.assign(table.begin(), table.end());
        }
        stab.resize(align_up(stab.size() * 2, 16) / 2, 0);
        abs_off = (uint32_t)(stab.size() * 2);
        abs_shift = layout == 1 && rowbytes % 4 == 0 ? 2u : 1u;
        const uint32_t unit = layout == 1 ? rowbytes >> abs_shift : 1u;   // bitmap index per state
        std::vector<uint32_t> bits(((uint64_t)nq * unit + 31) / 32, 0);
        for (uint32_t q = 0; q < nq; ++q)
            if (absorbing[q]) bits[(q * unit) >> 5] |= 1u << ((q * unit) & 31);
        const size_t words = align_up(bits.size() * 4, 16) / 4;
        bits.resize(words, 0);
        for (uint32_t w : bits) {
            stab.push_back((uint16_t)(w & 0xFFFF));
            stab.push_back((uint16_t)(w >> 16));
        }
        if ((uint64_t)stab.size() * 2 + 16 > (uint64_t)lds) {
            layout = 0;   // no room for the bitmap: one chunk per wavefront only
            direct = 0;
            stab.clear();
            abs_off = abs_shift = 0;
        }
    }
    if (stab.empty()) stab.assign(8, 0);

    // ---- two-symbol steps --------------------------------------------------
    // delta2(s, c1 c2) = delta(delta(s, c1), c2) halves the lookups of a walk.
    // Pair columns are deduplicated; the table is laid out as layout 1 (rows
    // of an odd number of dwords, one-byte codes 2 * column) and exists when
    // there are at most 127 columns and its entries fit 16 bits.
    uint32_t pairs = 0, rowbytes2 = 0, abs_off2 = 0, npair = 0;
    std::vector<uint16_t> stab2;
    std::vector<uint8_t> pcode(256, 0xFF);
    std::vector<uint8_t> pcode2;   // direct tables: pair codes indexed by the bytes
    {
        const uint32_t Kc = (uint32_t)class_sym.size();
        if (layout != 0 && Kc >= 1 && Kc <= 63) {
            std::unordered_map<std::string, uint32_t> pid;
            std::vector<std::vector<uint32_t>> pcols;
            std::vector<uint8_t> pc((size_t)Kc * (Kc + 1), 0);
            std::string key(nq * sizeof(uint32_t), '\0');
            std::vector<uint32_t> colv(nq);
            bool ok = true;
            for (uint32_t c1 = 0; c1 < Kc && ok; ++c1)
                for (uint32_t c2 = 0; c2 <= Kc && ok; ++c2) {
                    for (uint32_t q = 0; q < nq; ++q) {
                        uint32_t t = delta[(uint64_t)q * nsym + class_sym[c1]];
                        if (c2 < Kc) t = delta[(uint64_t)t * nsym + class_sym[c2]];
                        colv[q] = t;
                    }
                    std::memcpy(&key[0], colv.data(), key.size());
                    auto it = pid.find(key);
                    uint32_t id;
                    if (it == pid.end()) {
                        id = (uint32_t)pcols.size();
                        if (id >= 127) { ok = false; break; }
                        pid.emplace(key, id);
                        pcols.push_back(colv);
                    } else {
                        id = it->second;
                    }
                    pc[(size_t)c1 * (Kc + 1) + c2] = (uint8_t)(2 * id);
                }
            uint32_t R2 = ok ? (2 * (uint32_t)pcols.size() + 3) / 4 * 4 : 0;
            if (ok && (R2 / 4) % 2 == 0) R2 += 4;
            const uint64_t img = align_up((uint64_t)nq * R2, 16);
            const uint64_t bits_bytes = align_up(((uint64_t)nq * (R2 / 4) + 31) / 32 * 4, 16);
            if (ok && (uint64_t)(nq - 1) * R2 <= 0xFFFF && img + bits_bytes + 16 <= (uint64_t)lds) {
                pairs = 1;
                npair = (uint32_t)pcols.size();
                rowbytes2 = R2;
                stab2.assign(img / 2, 0);
                for (uint32_t q = 0; q < nq; ++q)
                    for (size_t c = 0; c < pcols.size(); ++c)
                        stab2[(size_t)q * (R2 / 2) + c] = (uint16_t)(R2 * pcols[c][q]);
                abs_off2 = (uint32_t)img;
                std::vector<uint32_t> bits(bits_bytes / 4, 0);
                const uint32_t unit = R2 / 4;
                for (uint32_t q = 0; q < nq; ++q)
                    if (absorbing[q]) bits[(q * unit) >> 5] |= 1u << ((q * unit) & 31);
                for (uint32_t w : bits) {
                    stab2.push_back((uint16_t)(w & 0xFFFF));
                    stab2.push_back((uint16_t)(w >> 16));
                }
                for (int b = 0; b < 256; ++b)
                    if (byte_class[b] >= 0) pcode[b] = (uint8_t)byte_class[b];
                pcode.insert(pcode.end(), pc.begin(), pc.end());
                if (direct) {
                    // byte pairs below 128 -> code at b1 + 256 * b2, a lone
                    // last byte at 32768 + b; 0xFF (odd) for bytes outside Sigma
                    pcode2.assign(32768 + 128, 0xFF);
                    for (int b1 = 0; b1 < 128; ++b1) {
                        if (byte_class[b1] < 0) continue;
                        pcode2[32768 + b1] = pc[(size_t)byte_class[b1] * (Kc + 1) + Kc];
                        for (int b2 = 0; b2 < 128; ++b2)
                            if (byte_class[b2] >= 0)
                                pcode2[(size_t)b1 + 256 * b2] =
                                    pc[(size_t)byte_class[b1] * (Kc + 1) + byte_class[b2]];
                    }
                }
            }
        }
    }
    if (stab2.empty()) stab2.assign(8, 0);
    pcode.resize(align_up(pcode.size(), 16), 0);
    if (pcode2.empty()) pcode2.assign(16, 0);

    std::vector<uint32_t> accept_bits((nq + 31) / 32, 0);
    for (uint32_t k = 0; k < nacc; ++k) accept_bits[accepting[k] >> 5] |= 1u << (accepting[k] & 31);

    // ---- one device arena ---------------------------------------------------
    struct Piece { const void *src; size_t bytes; size_t at; };
    std::vector<Piece> pieces;
    size_t at = 0;
    auto add = [&](const void *src, size_t bytes) {
        at = align_up(at, 256);
        pieces.push_back({src, bytes, at});
        at += bytes;
        return pieces.size() - 1;
    };
    size_t i_table = add(table.data(), table.size() * 2);
    size_t i_lut = add(lut.data(), lut.size() * 4);
    size_t i_off[2], i_st[2], i_pos[2];
    for (int m = 0; m < 2; ++m) {
        i_off[m] = add(off[m].data(), off[m].size() * 4);
        i_st[m] = add(st[m].data(), st[m].size() * 2);
        i_pos[m] = add(pos[m].data(), pos[m].size() * 2);
    }
    size_t i_acc = add(accept_bits.data(), accept_bits.size() * 4);
    size_t i_code = add(code.data(), code.size() * 2);
    size_t i_moff = add(mset_off.data(), mset_off.size() * 4);
    size_t i_mst = add(mset_st.data(), mset_st.size() * 2);
    size_t i_stab = add(stab.data(), stab.size() * 2);
    size_t i_stab2 = add(stab2.data(), stab2.size() * 2);
    size_t i_pcode = add(pcode.data(), pcode.size());
    size_t i_pcode2 = add(pcode2.data(), pcode2.size());
    const size_t arena_bytes = align_up(at, 256);

    dfa *d = new (std::nothrow) dfa();
    if (!d) return fail(DFA_E_NOMEM, "dfa_create: host allocation failed");
    hipError_t e = hipGetDevice(&d->device);
    if (e != hipSuccess) { delete d; return hip_fail(e, "hipGetDevice"); }
    e = hipMalloc(&d->arena, arena_bytes);
    if (e != hipSuccess) { delete d; return fail(DFA_E_NOMEM, "dfa_create: hipMalloc failed"); }
    std::vector<uint8_t> staging(arena_bytes, 0);
    for (auto &p : pieces) std::memcpy(staging.data() + p.at, p.src, p.bytes);
    e = hipMemcpy(d->arena, staging.data(), arena_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d->arena);
        delete d;
        return hip_fail(e, "hipMemcpy (dfa_create)");
    }
    auto ptr = [&](size_t i) { return (const void *)((const uint8_t *)d->arena + pieces[i].at); };
    d->arena_bytes = arena_bytes;
    d->nsym = nsym;
    d->wave_util = wave_util;
    for (uint32_t k = 0; k <= kMaxMsetLevel; ++k) {
        d->mset_mean[k] = mset_mean_k[k];
        d->mset_max[k] = mset_max_k[k];
    }
    d->h_mset_off = mset_off;
    d->h_mset_st = mset_st;
    for (int b = 0; b < 256; ++b) d->h_byte_class[b] = (int16_t)byte_class[b];
    DevDFA &v = d->dev;
    v.table = (const uint16_t *)ptr(i_table);
    v.lut = (const uint32_t *)ptr(i_lut);
    for (int m = 0; m < 2; ++m) {
        v.set_off[m] = (const uint32_t *)ptr(i_off[m]);
        v.set_st[m] = (const uint16_t *)ptr(i_st[m]);
        v.pos[m] = (const uint16_t *)ptr(i_pos[m]);
        v.setmax[m] = setmax[m];
        d->setmax_host[m] = setmax[m];
    }
    v.accept_bits = (const uint32_t *)ptr(i_acc);
    v.code = (const uint16_t *)ptr(i_code);
    v.mset_off = (const uint32_t *)ptr(i_moff);
    v.mset_st = (const uint16_t *)ptr(i_mst);
    for (uint32_t k = 0; k <= kMaxMsetLevel; ++k) {
        v.moff[k] = moff[k];
        v.mst[k] = mst[k];
    }
    v.r0 = r0;
    v.stab = (const uint16_t *)ptr(i_stab);
    v.layout = layout;
    v.direct = direct;
    v.rowbytes = rowbytes;
    v.stab_bytes = layout != 0 ? (uint32_t)(stab.size() * 2) : (uint32_t)table_bytes;
    v.abs_off = abs_off;
    v.abs_shift = abs_shift;
    v.nabs = nabs;
    v.pairs = pairs;
    v.stab2 = (const uint16_t *)ptr(i_stab2);
    v.stab2_bytes = pairs ? (uint32_t)(stab2.size() * 2) : 0u;
    v.rowbytes2 = rowbytes2;
    v.abs_off2 = abs_off2;
    v.pcode = (const uint8_t *)ptr(i_pcode);
    v.pcode2 = pcode2.size() > 16 ? (const uint8_t *)ptr(i_pcode2) : nullptr;
    v.nq = nq;
    v.nclass = K;
    v.colstride = colstride;
    v.table_bytes = (uint32_t)table_bytes;
    v.q0 = q0;

    dfa_info_t &inf = d->info;
    inf.num_states = nq;
    inf.num_symbols = nsym;
    inf.num_classes = (uint32_t)class_sym.size();
    inf.num_absorbing = nabs;
    inf.imax = setmax[1];
    inf.q0 = q0;
    inf.mean_iset = mean_iset;
    inf.table_bytes = table_bytes;
    inf.device_bytes = arena_bytes;
    inf.packed_layout = direct ? 3u : layout;
    inf.lookahead_tables = r0;
    inf.pair_columns = npair;
    *out = d;
    return DFA_OK;
}

extern "C" void dfa_destroy(dfa_t *d) {
    if (!d) return;
    if (d->arena) (void)hipFree(d->arena);
    delete d;
}

extern "C" int dfa_lookahead_set(const dfa_t *d, const uint8_t *bytes, uint32_t k, uint16_t *out,
                                 uint32_t cap, uint32_t *count) {
    if (!d || (k && !bytes) || !count) return fail(DFA_E_INVAL, "dfa_lookahead_set: NULL argument");
    if (k == 0 || k > d->dev.r0) return fail(DFA_E_INVAL, "dfa_lookahead_set: k out of range");
    uint64_t id = 0;
    for (uint32_t j = 0; j < k; ++j) {
        const int c = d->h_byte_class[bytes[j]];
        if (c < 0) return fail(DFA_E_SYMBOL, "dfa_lookahead_set: byte outside Sigma");
        id = id * d->dev.nclass + (uint64_t)c;
    }
    const uint32_t lo = d->h_mset_off[d->dev.moff[k] + id];
    const uint32_t hi = d->h_mset_off[d->dev.moff[k] + id + 1];
    *count = hi - lo;
    for (uint32_t j = 0; j < hi - lo && j < cap; ++j) out[j] = d->h_mset_st[d->dev.mst[k] + lo + j];
    return DFA_OK;
}

extern "C" int dfa_info(const dfa_t *d, dfa_info_t *out) {
    if (!d || !out) return fail(DFA_E_INVAL, "dfa_info: NULL argument");
    *out = d->info;
    return DFA_OK;
}
