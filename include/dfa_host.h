/* Host multicore speculative DFA matcher: the paper's method on CPU cores.
 *
 * This is the paper's own CPU design (Section 4, Algorithm 3, one pthread per
 * processor), built as a second CPU yardstick beside the sequential walk.  It
 * is a separate library (libdfahost.so) with its own copy of the automaton;
 * the GPU library neither calls it nor falls back to it.
 *
 * Processor k walks one contiguous chunk.  Processor 0 walks its chunk from
 * the start state only; every other processor walks its chunk once from each
 * state of the reverse-lookahead set I_sigma of the symbol just before the
 * chunk (Eq. 11; absorbing states are left out and resolve to themselves).
 * Chunk lengths follow the capacity-weighted partition of Eqs. (1)-(7) with
 * |Q| replaced by I_max (Eq. 10), so that the single-state chunk 0 is longer
 * than the others; the per-processor maps are then merged in order (Eq. 8).
 * The result is exactly the sequential one.
 *
 * Status codes are those of dfa_spec.h (0 = ok, negative = error). */
#ifndef DFA_HOST_H
#define DFA_HOST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dfa_host dfa_host_t;

/* dfa_host_create -- copy a complete DFA (same arguments and validation as
 * dfa_create: delta[q * num_symbols + a], 1 <= num_symbols <= 256,
 * byte_to_symbol[256] with values >= num_symbols marking bytes outside Sigma,
 * NULL = identity for num_symbols == 256).  The caller keeps its arrays. */
int dfa_host_create(const uint32_t *delta, uint32_t num_states, uint32_t num_symbols, uint32_t q0,
                    const uint32_t *accepting, uint32_t num_accepting,
                    const uint8_t *byte_to_symbol, dfa_host_t **out);
void dfa_host_destroy(dfa_host_t *d);

/* I_max (Eq. 12: the largest |I_sigma| over the symbols of Sigma). */
uint32_t dfa_host_imax(const dfa_host_t *d);

/* dfa_host_partition -- Eqs. (1)-(7) with m in place of |Q| (Eq. 10 passes
 * I_max).  capacities: P measured speeds (NULL = all equal); the weights are
 * capacity / mean capacity (Eq. 1).  starts: out, P + 1 half-open chunk
 * boundaries, starts[0] = 0, starts[P] = n; chunk k = [starts[k],
 * starts[k+1]).  The inclusive end positions of Eq. (7) are starts[k+1] - 1.
 * Positions are floored as in Eqs. (6)-(7).  DFA_E_INVAL if P = 0, m = 0 or a
 * capacity is not positive. */
int dfa_host_partition(uint64_t n, double m, const double *capacities, uint32_t P,
                       uint64_t *starts);

/* dfa_host_profile -- offline profiling for Eq. (1): `threads` threads walk
 * `sample` (host, len bytes, bytes outside Sigma are skipped) from q0 at the
 * same time; capacities[k] receives thread k's bytes per second. */
int dfa_host_profile(const dfa_host_t *d, const uint8_t *sample, size_t len, uint32_t threads,
                     double *capacities);

/* dfa_host_match -- membership test of `input` (host, len bytes) on
 * `threads` threads (0 = hardware concurrency).  capacities: NULL (equal
 * weights) or `threads` speeds from dfa_host_profile.  start_state:
 * 0xFFFFFFFF = q0.  Outputs: *final_state (caller's numbering) and *accepted;
 * DFA_E_SYMBOL (-4) if a byte is outside Sigma, and then no state.  The
 * input is borrowed for the call. */
int dfa_host_match(const dfa_host_t *d, const uint8_t *input, size_t len, uint32_t threads,
                   const double *capacities, uint32_t start_state, uint32_t *final_state,
                   int *accepted);

#ifdef __cplusplus
}
#endif
#endif /* DFA_HOST_H */
