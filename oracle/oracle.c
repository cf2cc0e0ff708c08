/* ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU statement of what the DFA membership
 * test computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this file's library; the GPU library never links or calls
 * it, and the two share no code, header, table or helper.
 *
 * Sources (Ko, Jung, Han, Burgstaller, arXiv 1210.5093):
 *   - oracle_walk:       Algorithm 1 (sequential DFA matching) and the extended
 *                        transition function delta* of Section 2.1;
 *   - oracle_absorbing:  the error/sink state q_e of Section 2.1, read as "every
 *                        state e with delta(e, a) = e for all a";
 *   - oracle_isets:      Eq. (11) and the first loop of Algorithm 3 (initial
 *                        state sets I_sigma, the error state left out);
 *   - oracle_iset_word:  Eq. (13), initial state set for a string of reverse
 *                        lookahead symbols sigma_1..sigma_k;
 *   - oracle_chunk_map:  the state-map vector L_i of Section 4.1,
 *                        L_i[j] = delta*(q_j, c_i).
 *
 * The table is the caller's own 2-D layout delta[q * nsym + a] indexed by raw
 * symbol number; bytes become symbols through a 256-entry map.  A byte whose
 * map entry is >= |Sigma| is not in Sigma (so 0xFF marks such bytes whenever
 * |Sigma| <= 255; with |Sigma| = 256 every byte is a symbol).  No alphabet
 * classes, offsets, chunking or initial-state sets are used by the walk.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_BAD_SYMBOL 1
#define ORACLE_BAD_ARG (-1)

/* delta*(start, w[0..n)) by Algorithm 1's loop.  probe_pos (ascending, each
 * in [0, n]) asks for the prefix states delta*(start, w[0..p)).  On a byte
 * outside Sigma the walk stops, *bad_index receives its position and the
 * result is ORACLE_BAD_SYMBOL. */
int oracle_walk(const uint32_t *delta, uint32_t nq, uint32_t nsym,
                const uint8_t *byte_to_symbol, uint32_t start,
                const uint8_t *w, uint64_t n,
                const uint64_t *probe_pos, uint64_t nprobe, uint32_t *probe_state,
                uint32_t *final_state, uint64_t *bad_index)
{
    if (!delta || !byte_to_symbol || start >= nq || nsym == 0 || (n && !w))
        return ORACLE_BAD_ARG;
    uint32_t state = start;
    uint64_t next_probe = 0;
    for (uint64_t i = 0; i < n; ++i) {
        while (next_probe < nprobe && probe_pos[next_probe] == i)
            probe_state[next_probe++] = state;
        uint32_t a = byte_to_symbol[w[i]];
        if (a >= nsym) {
            if (bad_index) *bad_index = i;
            return ORACLE_BAD_SYMBOL;
        }
        state = delta[(uint64_t)state * nsym + a];
    }
    while (next_probe < nprobe && probe_pos[next_probe] == n)
        probe_state[next_probe++] = state;
    *final_state = state;
    return ORACLE_OK;
}

/* accepted = final state is in F (Algorithm 1, last lines). */
int oracle_accepts(uint32_t final_state, const uint32_t *accepting, uint32_t num_accepting)
{
    for (uint32_t k = 0; k < num_accepting; ++k)
        if (accepting[k] == final_state) return 1;
    return 0;
}

/* mask[e] = 1 iff delta(e, a) = e for every symbol a. */
void oracle_absorbing(const uint32_t *delta, uint32_t nq, uint32_t nsym, uint8_t *mask)
{
    for (uint32_t e = 0; e < nq; ++e) {
        uint8_t sink = 1;
        for (uint32_t a = 0; a < nsym; ++a)
            if (delta[(uint64_t)e * nsym + a] != e) { sink = 0; break; }
        mask[e] = sink;
    }
}

/* out[a * nq + s] = 1 iff s = delta(x, a) for some x in Q and s is not
 * excluded (excluded may be NULL). */
void oracle_isets(const uint32_t *delta, uint32_t nq, uint32_t nsym,
                  const uint8_t *excluded, uint8_t *out)
{
    memset(out, 0, (size_t)nsym * nq);
    for (uint32_t a = 0; a < nsym; ++a)
        for (uint32_t x = 0; x < nq; ++x) {
            uint32_t s = delta[(uint64_t)x * nsym + a];
            if (!excluded || !excluded[s]) out[(uint64_t)a * nq + s] = 1;
        }
}

/* out[s] = 1 iff s = delta*(x, sym[0..k)) for some x in Q, s not excluded. */
void oracle_iset_word(const uint32_t *delta, uint32_t nq, uint32_t nsym,
                      const uint8_t *excluded, const uint32_t *sym, uint32_t k, uint8_t *out)
{
    memset(out, 0, nq);
    for (uint32_t x = 0; x < nq; ++x) {
        uint32_t s = x;
        for (uint32_t t = 0; t < k; ++t) s = delta[(uint64_t)s * nsym + sym[t]];
        if (!excluded || !excluded[s]) out[s] = 1;
    }
}

/* out[j] = delta*(starts[j], w[begin..end)) for j < m.  Returns
 * ORACLE_BAD_SYMBOL if the chunk holds a byte outside Sigma. */
int oracle_chunk_map(const uint32_t *delta, uint32_t nq, uint32_t nsym,
                     const uint8_t *byte_to_symbol, const uint8_t *w,
                     uint64_t begin, uint64_t end,
                     const uint32_t *starts, uint32_t m, uint32_t *out)
{
    for (uint32_t j = 0; j < m; ++j) {
        uint32_t state = starts[j];
        if (state >= nq) return ORACLE_BAD_ARG;
        for (uint64_t i = begin; i < end; ++i) {
            uint32_t a = byte_to_symbol[w[i]];
            if (a >= nsym) return ORACLE_BAD_SYMBOL;
            state = delta[(uint64_t)state * nsym + a];
        }
        out[j] = state;
    }
    return ORACLE_OK;
}
