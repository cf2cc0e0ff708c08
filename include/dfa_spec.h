/* dfa_spec.h -- C ABI of the MI355X speculative DFA membership test.
 *
 * Method: Ko, Jung, Han, Burgstaller, "Speculative parallel DFA membership
 * tests for multicore, SIMD and cloud computing environments" (arXiv
 * 1210.5093).  The input string is cut into chunks; every chunk after the
 * first is matched from each state of its initial-state set I_sigma (Eq. 11),
 * where sigma is the last symbol of the preceding chunk (reverse lookahead,
 * Section 4.2, Algorithm 3); the per-chunk state maps L_i (Section 4.1) are
 * combined in order (Eqs. 8-9) into the exact sequential final state
 * delta*(q0, w) of Algorithm 1, and the string is accepted iff that state is
 * in F.
 *
 * Conventions for every entry point:
 *  - Status codes only (DFA_OK = 0, negative on error); no C++ exception
 *    crosses this boundary.  dfa_last_error() returns a message for the
 *    calling thread's most recent failure.
 *  - States are always reported in the caller's numbering 0..num_states-1.
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *    device allocations on the current device.  Host arrays passed to a call
 *    are only borrowed for the duration of the call.
 *  - A dfa_t is immutable after dfa_create: concurrent matches of one DFA on
 *    different streams are safe.
 *  - Streams are hipStream_t handles passed as void* (0 = the null stream).
 */
#ifndef DFA_SPEC_H
#define DFA_SPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DFA_OK = 0,
    DFA_E_INVAL = -1,       /* bad argument (null pointer, id out of range, ...) */
    DFA_E_NOMEM = -2,       /* host or device allocation failed */
    DFA_E_DEVICE = -3,      /* a HIP runtime call failed */
    DFA_E_SYMBOL = -4,      /* the input holds a byte outside Sigma */
    DFA_E_TOOBIG = -5,      /* table or request exceeds a device limit */
    DFA_E_SPECULATION = -6, /* internal invariant violated: a chunk's true start
                               state was not in its initial-state set */
    DFA_E_BUSY = -7,        /* server has no free slot / budget right now */
    DFA_E_NOTREADY = -8     /* server ticket not finished yet */
};

/* start_state value meaning "use the DFA's q0". */
#define DFA_Q0 0xFFFFFFFFu

/* Result record written by the asynchronous entry points (4 x uint32). */
typedef struct dfa_result {
    uint32_t final_state;   /* delta*(start, w), caller numbering */
    uint32_t accepted;      /* 1 iff final_state is in F */
    uint32_t flags;         /* DFA_FLAG_* bits; 0 on success */
    uint32_t num_chunks;    /* chunks the input was cut into */
} dfa_result_t;

#define DFA_FLAG_SYMBOL      1u  /* a byte outside Sigma was seen */
#define DFA_FLAG_SPECULATION 2u  /* internal invariant violated */

typedef struct dfa dfa_t;

/* Static properties of a compiled DFA (Eqs. 11-12 and the class compression). */
typedef struct dfa_info {
    uint32_t num_states;      /* |Q| */
    uint32_t num_symbols;     /* |Sigma| as given */
    uint32_t num_classes;     /* K: distinct delta-columns over the bytes in Sigma */
    uint32_t num_absorbing;   /* states with a self-loop on every symbol (the paper's q_e) */
    uint32_t imax;            /* I_max of Eq. 12 over the classes */
    uint32_t q0;
    double   mean_iset;       /* mean |I_c| over the bytes in Sigma (each byte weighted 1) */
    uint64_t table_bytes;     /* bytes of the class-major table staged in LDS */
    uint64_t device_bytes;    /* device memory held by this dfa_t */
    uint32_t packed_layout;   /* 0: one-chunk-per-wavefront matcher only;
                                 1: packed-pair matcher, state-major table;
                                 2: packed-pair matcher, class-major table;
                                 3: packed-pair matcher, state-major table with
                                    rows indexed by the byte itself (every byte
                                    of Sigma below 128): no translation pass */
    uint32_t lookahead_tables;/* r0: sets I_{c_1..c_k} precomputed for k <= r0 */
    uint32_t pair_columns;    /* distinct two-symbol columns delta(delta(., a), b) of the
                                 table that lets the packed matcher take two symbols
                                 per lookup; 0 = no such table */
} dfa_info_t;

/* Options for dfa_match_ex.  Zero-initialised means "library defaults". */
typedef struct dfa_match_opts {
    uint64_t chunk_len;       /* bytes per chunk; 0 = planner's choice */
    uint32_t lookahead;       /* reverse-lookahead symbols r:
                                 1 = one-symbol sets I_sigma (Algorithm 3, default);
                                 0 = every chunk from all non-absorbing states
                                     (Algorithm 2, the ablation);
                                 2..64 = the exact image of Q under the r bytes
                                     before each chunk (Eq. 13, computed per chunk
                                     on the device; DFAs without a packed layout
                                     use r = 1, with the same result) */
    uint32_t flags;           /* DFA_MATCH_* bits, 0 = none */
} dfa_match_opts_t;

/* flags bit: a wavefront stops walking its (chunk, state) pairs once every one
 * of them sits in an absorbing state (the paper's error state, Section 3: a
 * walk that reaches it can stop).  The result is unchanged; the saving depends
 * on the input.  Honoured by the packed-pair matchers (single string and
 * batch) for DFAs with an absorbing state; ignored otherwise. */
#define DFA_MATCH_EARLY_EXIT 1u

/* flags bit: walk one symbol per table lookup even where the DFA has a
 * two-symbol table (dfa_info_t::pair_columns > 0).  The two-symbol table
 * halves the lookups but needs a pass that turns byte pairs into codes; with
 * a direct table (packed_layout 3) the one-symbol walk reads the input as it
 * is.  Which is faster depends on how much walking is left after merging
 * (below); dfa_autotune tries both. */
#define DFA_MATCH_SINGLE_STEP 2u

/* flags bit: interleave the packed matcher's code stream: the 16-byte code
 * blocks of 64 consecutive chunks are stored side by side (block b of all 64
 * contiguous), so that the walks of consecutive chunks read whole cache lines
 * together.  Without it the stream is linear, chunk after chunk (with a
 * direct table, packed_layout 3: the raw input itself, no stream written).
 * Needs chunk lengths of a multiple of 32 and precomputed start sets; ignored
 * otherwise. */
#define DFA_MATCH_INTERLEAVE 4u

/* flags bit: one chunk per lane with merged walks.  A lane walks its chunk's
 * start states (sets of at most 128) four at a time over the first 32 code
 * positions,
 * keeps the distinct states reached (the walks of one chunk converge; at most
 * 4 are kept), walks only those to the chunk's end and gives every start state
 * the end of its group; a chunk that does not reduce that far is walked state
 * by state.  Implies DFA_MATCH_INTERLEAVE (chunk lengths of a multiple of 32,
 * precomputed start sets); ignored otherwise.  The maps, and every result,
 * are unchanged. */
#define DFA_MATCH_CHUNK_LANES 8u

/* flags field bits 8..11: walk rounds of the packed matcher.  Walks of one
 * chunk that reach the same state at the same position have the same future
 * (delta is a function), so after each round but the last the matcher keeps
 * one walk per distinct (chunk, state) and the others take its end state.
 * Round 1 walks the first 32 bytes of every chunk, each later round four
 * times as far, the last round to the chunk end.  The maps, and so every
 * result, are unchanged; the work after a round shrinks to the number of
 * distinct states, which for the automata measured here is about one per
 * chunk within a few dozen bytes.
 *   DFA_MATCH_ROUNDS(1) or 0 (the default): one round, every walk runs its
 *                        whole chunk (Algorithm 3 as written);
 *   DFA_MATCH_ROUNDS(2..6): that many rounds.
 * Rounds beyond one need chunk lengths that are multiples of 32 and no early
 * exit; otherwise a single round runs.  dfa_autotune tries them.
 * With DFA_MATCH_INTERLEAVE, one symbol per step and a 16-byte aligned input,
 * the last round runs one chunk per lane over the raw input (each chunk's
 * remaining walks side by side in one lane, bytes turned into codes in LDS),
 * and only the bytes before it are translated (dfa_plan_info_t::tail_lanes). */
#define DFA_MATCH_ROUNDS(k) (((uint32_t)(k) & 0xFu) << 8)
#define DFA_MATCH_ROUNDS_OF(flags) (((flags) >> 8) & 0xFu)

/* ---------------------------------------------------------------------------
 * dfa_create -- compile a DFA (Q, Sigma, delta, q0, F) (Section 2.1) and keep
 * it resident on the current device.
 *   delta:          host, num_states * num_symbols entries, row-major
 *                   delta[q * num_symbols + a]; every entry < num_states
 *                   (the automaton must be complete, as in the paper).
 *   num_states:     1 .. 32767.
 *   num_symbols:    1 .. 256.
 *   q0:             start state, < num_states.
 *   accepting:      host, num_accepting state ids (may be NULL if 0).
 *   byte_to_symbol: host, 256 entries mapping input bytes to symbols; an
 *                   entry >= num_symbols marks a byte outside Sigma (0xFF
 *                   is the usual marker).  NULL = identity (num_symbols must
 *                   be 256).
 *   out:            receives the handle (owned by the caller; dfa_destroy).
 * All inputs are copied.  Returns DFA_E_INVAL on an invalid automaton,
 * DFA_E_TOOBIG if the compressed table cannot be staged in LDS.
 * Fault injection (tests of the speculation check only): when the environment
 * variable DFA_DROP_STATE holds a state id s at dfa_create time, s is left
 * out of every one-symbol and precomputed multi-symbol initial-state set; a
 * match whose true state at a chunk boundary is s then reports
 * DFA_FLAG_SPECULATION (DFA_E_SPECULATION from dfa_match) instead of a
 * state. */
int dfa_create(const uint32_t *delta, uint32_t num_states, uint32_t num_symbols,
               uint32_t q0, const uint32_t *accepting, uint32_t num_accepting,
               const uint8_t *byte_to_symbol, dfa_t **out);

/* Release a DFA (device memory included).  Must not be called while a
 * match of it may still run on some stream.  NULL is ignored. */
void dfa_destroy(dfa_t *d);

/* Fill *out with the DFA's static properties. */
int dfa_info(const dfa_t *d, dfa_info_t *out);

/* ---------------------------------------------------------------------------
 * dfa_match -- synchronous membership test of a host string (Algorithm 1's
 * interface: transition function, string, start state, final states ->
 * true/false).  Copies the input to the device, runs the speculative path and
 * waits.
 *   input/len:    host bytes (len may be 0: the final state is the start).
 *   start_state:  DFA_Q0 or an explicit state (lets a long stream be matched
 *                 in segments: pass the previous segment's final state).
 *   final_state:  host out (may be NULL); accepted: host out (may be NULL).
 * Returns DFA_E_SYMBOL if a byte is outside Sigma (no state is returned). */
int dfa_match(const dfa_t *d, const uint8_t *input, size_t len, uint32_t start_state,
              uint32_t *final_state, int *accepted);

/* dfa_match_async -- the same test on device-resident input, enqueued on
 * `stream`.
 *   d_input:  device, len bytes; must stay valid until the stream passes
 *             this call.
 *   d_result: device, one dfa_result_t (4 x uint32), written on the stream.
 * Errors in the input (bytes outside Sigma) are reported in d_result->flags,
 * not by the return code.  The library keeps one scratch workspace per
 * (device, stream); a call that needs more than the stream's workspace holds
 * (the first call, or a larger input) waits for `stream` (never for other
 * streams) before it releases the old workspace, and allocates a larger one.
 * Calls that fit return without waiting. */
int dfa_match_async(const dfa_t *d, const uint8_t *d_input, size_t len,
                    uint32_t start_state, void *stream, uint32_t *d_result);

/* dfa_match_ex -- dfa_match_async with options and, optionally, the state at
 * every chunk boundary.
 *   opts:          may be NULL (defaults).
 *   d_boundaries:  NULL, or device, num_chunks + 1 uint32 entries where
 *                  num_chunks = ceil(len / chunk_len); entry i is the state
 *                  before chunk i (delta*(start, w[0 : i*chunk_len])), the
 *                  last entry the final state.  Use dfa_plan_chunks to learn
 *                  num_chunks beforehand. */
int dfa_match_ex(const dfa_t *d, const uint8_t *d_input, size_t len, uint32_t start_state,
                 const dfa_match_opts_t *opts, void *stream, uint32_t *d_result,
                 uint32_t *d_boundaries);

/* dfa_match_maps -- dfa_match_ex on the packed-pair matcher that also
 * returns the level-0 state maps: for every (chunk i, start state q) pair the
 * end state delta*(q, c_i) of its walk (Section 4.1's L_i[j], over the
 * chunk's initial-state set, Eq. 11 / Eq. 13), in the caller's numbering.
 * For tests and diagnostics: every entry of the maps the composition reads
 * can be checked against a direct walk.
 *   d_first:      device, num_chunks + 1 uint32: first pair of each chunk;
 *                 d_first[num_chunks] = number of pairs.
 *   d_pair_start, d_pair_end: device, max_pairs uint16 each: pair P's start
 *                 state and end state (0xFFFF: the end state is in no state
 *                 of the next chunk's set, an invariant violation that also
 *                 sets DFA_FLAG_SPECULATION).  Pairs >= max_pairs are not
 *                 written; the caller compares d_first[num_chunks] with
 *                 max_pairs (at most num_chunks * dfa_plan()'s set_max).
 * Returns DFA_E_INVAL when the plan does not use the packed-pair matcher
 * (dfa_plan's kernel 0) or len is 0. */
int dfa_match_maps(const dfa_t *d, const uint8_t *d_input, size_t len, uint32_t start_state,
                   const dfa_match_opts_t *opts, void *stream, uint32_t *d_result,
                   uint32_t *d_first, uint16_t *d_pair_start, uint16_t *d_pair_end,
                   uint64_t max_pairs);

/* dfa_match_block -- the block map of one shard of a longer string, and
 * dfa_compose_blocks -- the ordered composition of several shards' maps.
 * Together they are the one-GPU part of matching a string sharded over
 * several processors (Section 3: the input is cut into pieces whose lengths
 * follow the processors' measured capacities, Eqs. 1-7, with the first piece
 * lengthened by Eq. 10 since it starts from one state; each piece is matched
 * from its reverse-lookahead set, Eq. 11 / Eq. 13, and the pieces' maps are
 * combined in order, Eq. 9).  dfa_host_partition computes such boundaries.
 *
 * dfa_match_block matches bytes [offset, offset + len) of the string at
 * d_input (device; the `lookahead` bytes before offset must be readable,
 * they choose the start set).  offset = 0: the block starts from start_state
 * alone (DFA_Q0 = q0); otherwise from I of the r bytes before offset
 * (absorbing states left out).  Written on the stream:
 *   d_info:   device, 4 x uint32: number of entries m, flags (DFA_FLAG_SYMBOL
 *             if the shard holds a byte outside Sigma), chunks, 0;
 *   d_start:  device, max_entries uint16: the start states, ascending;
 *   d_end:    device, max_entries uint16: the state at the shard's end from
 *             each start state (0xFFFF: the walk left the chunks' start sets,
 *             an invariant violation; the composition then reports
 *             DFA_FLAG_SPECULATION if it needs that entry).
 * opts as for dfa_match_ex (boundaries are not offered); a lookahead beyond
 * the precomputed levels (dfa_info_t::lookahead_tables) is lowered to them.
 * Needs a packed layout (dfa_info_t::packed_layout != 0; DFA_E_INVAL
 * otherwise), len > 0, and max_entries >= dfa_plan()'s set_max for this
 * length (DFA_E_TOOBIG otherwise).
 *
 * dfa_compose_blocks follows start_state through `count` blocks in order:
 * block g's record at d_infos + 4 g, its entries at d_starts / d_ends +
 * g * max_entries.  Writes d_result (dfa_result_t: final state, accept bit,
 * flags, total chunks) and, if not NULL, d_block_states[0 .. count]: the
 * state before each block and the final state (0xFFFFFFFF after a flag). */
int dfa_match_block(const dfa_t *d, const uint8_t *d_input, size_t offset, size_t len,
                    uint32_t start_state, const dfa_match_opts_t *opts, void *stream,
                    uint32_t *d_info, uint16_t *d_start, uint16_t *d_end, uint32_t max_entries);
int dfa_compose_blocks(const dfa_t *d, uint32_t count, const uint32_t *d_infos,
                       const uint16_t *d_starts, const uint16_t *d_ends, uint32_t max_entries,
                       uint32_t start_state, void *stream, uint32_t *d_result,
                       uint32_t *d_block_states);

/* dfa_match_noalloc -- dfa_match_ex for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result record and boundaries as
 * dfa_match_ex (no timing instrumentation is recorded).  Every scratch
 * buffer of the call (maps, start-set sizes, scans, and on the packed-pair
 * path the code stream: about one byte per input byte when the input is
 * translated, none when the matcher reads the raw input) comes from one
 * fixed region of DFA_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
 * from the first call on that device until the process ends.  The call
 * allocates and frees no device memory.
 * Returns DFA_E_TOOBIG (nothing enqueued) when the plan needs more scratch
 * than the region holds.  All calls on one GPU share its region and leave
 * their contents in it: calls that overlap on one GPU (on different
 * streams, or from several host threads) race, and the caller must order
 * them (one stream, or events between them). */
#define DFA_NOALLOC_SCRATCH_BYTES (64u << 20)
int dfa_match_noalloc(const dfa_t *d, const uint8_t *d_input, size_t len, uint32_t start_state,
                      const dfa_match_opts_t *opts, void *stream, uint32_t *d_result,
                      uint32_t *d_boundaries);

/* lookahead value meaning "use what dfa_autotune chose for this DFA and a
 * length of this order (one symbol if it was never tuned)". */
#define DFA_LOOKAHEAD_AUTO 0xFFFFFFFFu

/* dfa_autotune -- time candidate (lookahead r, chunk length) settings on the
 * caller's device input and keep the fastest.  Every candidate gives the same
 * result (the method is exact); only speed differs.  Inputs beyond 1 GiB
 * are tuned on their first 1 GiB; the best setting of each way of walking is
 * then timed on the whole input, as measured and with its chunk length scaled
 * to the input (the chunk count measured on the sample), then the fastest
 * with a quarter, half and twice its chunk length, and the fastest kept.
 * The choice is cached per DFA and
 * power-of-two length bucket and used by calls with lookahead
 * DFA_LOOKAHEAD_AUTO.  Around the best (r, chunk) (r, r + 1 and r0, a quarter
 * to four times the chunk, and 16 and 64 times it for merged rounds, which
 * stop a walk at an absorbing state) it then times merged rounds (DFA_MATCH_ROUNDS 2-4),
 * interleaved codes (one to four rounds) and one chunk per lane, then the
 * best with DFA_MATCH_SINGLE_STEP where a two-symbol table exists, and for a
 * DFA with an absorbing state with DFA_MATCH_EARLY_EXIT; whichever is faster
 * is kept (in best->flags).
 *   d_input: device, len bytes.  best: out (may be NULL).  best_ms: out, the
 *   chosen setting's time per call on the whole input (may be NULL).
 *   Synchronises `stream`. */
int dfa_autotune(const dfa_t *d, const uint8_t *d_input, size_t len, void *stream,
                 dfa_match_opts_t *best, double *best_ms);

/* Chunk length the library would use for (d, len, opts), and the resulting
 * number of chunks. */
int dfa_plan_chunks(const dfa_t *d, size_t len, const dfa_match_opts_t *opts,
                    uint64_t *chunk_len, uint64_t *num_chunks);

/* Initial-state set for a string of k reverse-lookahead bytes (Eq. 13: the
 * image of Q under the string, absorbing states left out), read from the
 * tables dfa_create precomputed (k <= dfa_info.lookahead_tables).
 *   bytes: host, k bytes in matching order.  out: host, cap entries.
 *   *count receives the set size (states written in ascending order, at most
 *   cap).  Returns DFA_E_SYMBOL for a byte outside Sigma, DFA_E_INVAL if k is
 *   0 or beyond the tables. */
int dfa_lookahead_set(const dfa_t *d, const uint8_t *bytes, uint32_t k, uint16_t *out,
                      uint32_t cap, uint32_t *count);

/* What the planner picks for (d, len, opts). */
typedef struct dfa_plan_info {
    uint64_t chunk_len;       /* bytes per chunk */
    uint64_t num_chunks;
    uint32_t kernel;          /* 0: one chunk per wavefront; 1: packed (chunk, state) pairs */
    uint32_t lookahead;       /* effective reverse-lookahead symbols r */
    uint32_t blocks;          /* matcher grid */
    uint32_t threads;         /* threads per block */
    uint32_t symbols_per_step;/* 2: the packed matcher walks the two-symbol table (one
                                 lookup per two input bytes, after a pass that turns
                                 byte pairs into codes); 1 otherwise */
    uint32_t raw_input;       /* 1: the packed matcher reads the input bytes themselves
                                 (direct table: only a validation pass runs first) when
                                 the input is 16-byte aligned */
    uint32_t rounds;          /* walk rounds with merging (DFA_MATCH_ROUNDS); 1 = none */
    uint32_t interleaved;     /* 1: chunk-interleaved code stream (DFA_MATCH_INTERLEAVE) */
    uint32_t chunk_lanes;     /* 1: one chunk per lane with merged walks (DFA_MATCH_CHUNK_LANES) */
    uint32_t set_max;         /* largest start set a chunk can have (entries per strided map) */
    uint32_t levels;          /* composition levels (Eq. 9 applied as a tree) */
    uint32_t group0;          /* maps composed per workgroup on the first level */
    uint32_t group;           /* maps composed per workgroup on the later levels */
    uint32_t tail_lanes;      /* nonzero: merged walks whose last round runs one chunk per
                                 lane over the raw input (interleaved one-symbol codes,
                                 16-byte aligned input); the code stream then covers only
                                 each chunk's first tail_start bytes.  The value is the
                                 chunks each lane takes (1, or 2 side by side when one per
                                 lane would not fit the device at once) */
    uint32_t tail_start;      /* chunk bytes walked before that last round */
} dfa_plan_info_t;
int dfa_plan(const dfa_t *d, size_t len, const dfa_match_opts_t *opts, dfa_plan_info_t *out);

/* ---------------------------------------------------------------------------
 * Batches: many (DFA, string) pairs of uneven size in one persistent launch
 * (the paper's representation holds several DFAs and strings in one table and
 * input array, Section 5).  Every string is cut into chunks of one length;
 * one launch matches all (chunk, start state) pairs of all strings, each
 * chunk from its reverse-lookahead set (Eq. 11, or Eq. 13's I_{c1..ck} with
 * k = min(lookahead, the DFA's precomputed levels)), then the per-string maps
 * are composed (Eq. 9).  When every DFA has a packed layout (dfa_info_t::
 * packed_layout != 0) the pairs are packed onto lanes as in the single-string
 * packed matcher; otherwise one wavefront walks one chunk (one-symbol
 * lookahead only).  Each string's record equals what dfa_match_async writes
 * for it alone.
 *
 * dfa_batch_create -- plan a batch and upload its descriptors (synchronous).
 *   dfas:      host array of `count` handles (may repeat; must outlive the batch).
 *   d_inputs:  host array of `count` device pointers (must stay valid and may
 *              change contents between runs; the pointers are fixed).
 *   lens:      host array of `count` lengths.
 *   opts:      NULL (planner chunk length, lookahead 1) or chunk_len (0 =
 *              planner) and lookahead 1 .. 64 (above 1 only for packed
 *              layouts).
 * dfa_batch_run -- enqueue the whole batch on `stream`: no host work, no
 *   allocation, so it may be captured into a HIP graph.
 *   d_results: device, count dfa_result_t records.
 * dfa_batch_graph_launch -- capture dfa_batch_run into a HIP graph once (per
 *   d_results pointer) and replay it; `stream` must not be the null stream.
 * dfa_batch_info -- chunk length used and number of chunks (packed-pair
 *   batch) or matcher tasks (one chunk per wavefront). */
typedef struct dfa_batch dfa_batch_t;
int dfa_batch_create(const dfa_t *const *dfas, const uint8_t *const *d_inputs,
                     const size_t *lens, size_t count, const dfa_match_opts_t *opts,
                     dfa_batch_t **out);
int dfa_batch_run(dfa_batch_t *b, void *stream, uint32_t *d_results);
int dfa_batch_graph_launch(dfa_batch_t *b, void *stream, uint32_t *d_results);
int dfa_batch_info(const dfa_batch_t *b, uint64_t *chunk_len, uint32_t *tasks);
/* dfa_batch_tune -- time the batch at the planner's chunk length and at the
 * powers of two from 1 KiB to 64 KiB, with lookahead 1, 2, 3, 4, 6 and 8 (1
 * only when a DFA lacks a packed layout), then the best of them with
 * DFA_MATCH_EARLY_EXIT when a DFA has an absorbing state; *best receives the
 * fastest options (pass them to dfa_batch_create), *best_ms its time per run.
 * Allocates temporary plans; synchronises `stream`. */
int dfa_batch_tune(const dfa_t *const *dfas, const uint8_t *const *d_inputs, const size_t *lens,
                   size_t count, void *stream, dfa_match_opts_t *best, double *best_ms);
void dfa_batch_destroy(dfa_batch_t *b);

/* dfa_match_batch -- one-shot batch: plan, run on `stream`, wait for the
 *   stream, release the plan.  Returns once d_results holds every record. */
int dfa_match_batch(const dfa_t *const *dfas, const uint8_t *const *d_inputs,
                    const size_t *lens, size_t count, void *stream, uint32_t *d_results);

/* ---------------------------------------------------------------------------
 * Serving: DFAs registered once stay resident; clients submit (DFA id,
 * device string) requests at any time and poll or wait for their records.  A
 * dispatcher thread admits requests in arrival order while the in-flight
 * budget allows (input bytes plus the batch arena's estimate) and packs them
 * into batches that run concurrently on `streams` non-blocking streams
 * (continuous batching: requests arriving while batches run join the next
 * one).  Each record equals the request's result alone.  Dispatching
 * allocates nothing; the slots' device arenas and pinned buffers are made at
 * creation.
 *   dfa_server_create:   opts may be NULL (defaults below).
 *   dfa_server_register: the DFA must outlive the server; *id receives its id.
 *   dfa_server_submit:   d_input (device) must stay valid until the ticket is
 *                        done, and its contents must be complete when the
 *                        call is made (the server's streams do not wait for
 *                        the caller's); DFA_E_TOOBIG if one request exceeds
 *                        the budget or, alone in a batch, a slot's arena.
 *   dfa_server_submit_after: the same for an input still being produced on
 *                        `producer_stream` (a kernel or copy enqueued before
 *                        the call): an event recorded on that stream at
 *                        submit time is waited for on the server's stream
 *                        before the request's batch reads the input.
 *   dfa_server_poll:     DFA_OK and the record once done (the ticket is then
 *                        released), DFA_E_NOTREADY before.
 *   dfa_server_wait:     blocks until the ticket is done.
 *   dfa_server_destroy:  finishes every submitted request, then releases. */
typedef struct dfa_server dfa_server_t;
typedef struct dfa_server_opts {
    uint64_t budget_bytes;    /* in-flight device bytes (0 = 16 GiB) */
    uint32_t max_inflight;    /* in-flight requests (0 = 4096) */
    uint32_t streams;         /* concurrent batches (0 = 4) */
    uint32_t max_batch;       /* requests per batch (0 = 256) */
    uint32_t lookahead;       /* reverse-lookahead symbols of the batches (0 = 1).
                                 Batches run on the packed-pair path when every
                                 DFA has a packed layout and lookahead >= 2 or
                                 the batch holds >= 256 MiB; otherwise one chunk
                                 per wavefront (fewer launches) with lookahead 1 */
    uint64_t slot_bytes;      /* device arena per concurrent batch (0 = 1 GiB) */
} dfa_server_opts_t;
typedef struct dfa_server_stats {
    uint64_t submitted, completed, batches, bytes;
    uint64_t inflight, pending;
} dfa_server_stats_t;
int dfa_server_create(const dfa_server_opts_t *opts, dfa_server_t **out);
int dfa_server_register(dfa_server_t *srv, const dfa_t *d, uint32_t *id);
int dfa_server_submit(dfa_server_t *srv, uint32_t id, const uint8_t *d_input, size_t len,
                      uint64_t *ticket);
int dfa_server_submit_after(dfa_server_t *srv, uint32_t id, const uint8_t *d_input, size_t len,
                            void *producer_stream, uint64_t *ticket);
int dfa_server_poll(dfa_server_t *srv, uint64_t ticket, dfa_result_t *out);
int dfa_server_wait(dfa_server_t *srv, uint64_t ticket, dfa_result_t *out);
int dfa_server_stats(dfa_server_t *srv, dfa_server_stats_t *out);
/* dfa_server_drain -- move up to `cap` finished records into `out` (in no
 * particular order) and release their tickets; *count receives how many.
 * submit_ns is when dfa_server_submit accepted the request, done_ns when its
 * record became visible on the host, both CLOCK_MONOTONIC nanoseconds. */
typedef struct dfa_server_done {
    uint64_t ticket;
    dfa_result_t result;
    uint64_t submit_ns, done_ns;
} dfa_server_done_t;
int dfa_server_drain(dfa_server_t *srv, dfa_server_done_t *out, size_t cap, size_t *count);
void dfa_server_destroy(dfa_server_t *srv);

/* ---------------------------------------------------------------------------
 * Instrumentation.  With timing on for a stream, every match call and every
 * dfa_batch_run on it records HIP events around its chunk-matcher kernel (the
 * preparation kernels before it excluded) and around the whole call (no work
 * is skipped or reordered; graph launches are not instrumented).  dfa_timing_read waits for those
 * events, returns the summed milliseconds and the number of calls, and
 * clears the record. */
int dfa_timing_enable(void *stream, int on);
int dfa_timing_read(void *stream, double *matcher_ms, double *call_ms, uint32_t *calls);
/* dfa_timing_read_ex -- dfa_timing_read plus kernel_ms: the summed time of
 * each call's longest single matcher launch (the one-chunk-per-lane last
 * round when the plan has one, else the last merged round, else the packed
 * matcher; batches and the one-chunk-per-wave kernel: the matcher time). */
int dfa_timing_read_ex(void *stream, double *matcher_ms, double *call_ms, double *kernel_ms,
                       uint32_t *calls);

/* Message for a status code / for this thread's last failure. */
const char *dfa_strerror(int status);
const char *dfa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFA_SPEC_H */
