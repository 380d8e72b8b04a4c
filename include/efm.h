/*
 * efm.h -- C ABI of the MI355X (gfx950) exhaustive AND/OR pathway traversal.
 *
 * Method (paper "A system architecture for parallel analysis of flux-balanced
 * metabolic pathways"):
 *   - input: the stoichiometric matrix S (Section 2.1), reversibility per
 *     reaction and an external flag per metabolite; internal rows must balance
 *     (Definition 2), external rows are ignored for balancing;
 *   - output: the elementary flux modes (Definition 3) that produce a chosen
 *     external metabolite, each as a reaction-set bitset plus its primitive
 *     integer flux vector.
 *   Pathways are built as in Definitions 8-9 and Algorithm 3 (Section 4.1), made
 *   exhaustive (every output/input branch is taken, as in the proof of
 *   Theorem 1) and exact (an exact rank test replaces the topology-only
 *   acceptance that the paper's Discussion mentions).
 *
 * Conventions
 *   - Every call returns an efm_status (0 = EFM_OK, negative = error).  On error
 *     the output arguments are left untouched and efm_last_error() holds a
 *     message (thread-local, valid until the next call on the same thread).
 *   - No C++ exception crosses this boundary.
 *   - Bitsets are LSB-first: reaction r is bit (r & 63) of 64-bit word (r >> 6);
 *     W = ceil(n_rxn / 64) words per pathway.
 *   - Canonical order: a bitset read as an n_rxn-bit unsigned integer in which
 *     reaction r weighs 2^r; results are sorted ascending in that order, and a
 *     frontier that exceeds its cap keeps its smallest members in that order.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary process memory.  Streams are hipStream_t passed as
 *     void* (NULL = the null stream).
 */
#ifndef EFM_H
#define EFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t efm_status;

#define EFM_OK 0
#define EFM_EINVAL -1    /* bad dimension, null pointer, short buffer, bad target */
#define EFM_ENOMEM -2    /* workspace or a device capacity too small; see last_error */
#define EFM_EDEVICE -3   /* a HIP call failed; its text is in last_error */
#define EFM_EOVERFLOW -4 /* a flux entry does not fit the exact integer type */

/* result status flags (not errors) */
#define EFM_COMPLETE 0u
#define EFM_DEPTH_CAPPED 1u         /* an independent partial pathway reached the depth cap */
#define EFM_FRONTIER_TRUNCATED 2u   /* some level kept only frontier_cap members */

#define EFM_MAX_RXN 1024            /* reactions per network */
#define EFM_MAX_DEPTH 64            /* largest support size (depth cap) */

typedef struct efm_network efm_network;
typedef struct efm_result efm_result;

/* Options of one enumeration.  Zero-initialise and set what is needed. */
typedef struct {
  int32_t depth_cap;       /* largest support size D (0 = EFM_MAX_DEPTH, clamped to it) */
  int32_t reserved0;
  int64_t frontier_cap;    /* partial pathways kept per level (0 = no cap) */
  int64_t unique_cap;      /* distinct children per level the workspace holds (0 = default) */
  int64_t found_cap;       /* pathways the workspace holds (0 = default) */
  uint32_t flags;          /* EFM_OPT_* */
  uint32_t reserved1;
  void *stream;            /* hipStream_t the work is queued on (NULL = null stream) */
  void *workspace;         /* device memory of >= efm_workspace_query bytes, or NULL to let
                              the library allocate it for the duration of the call */
  size_t workspace_bytes;
} efm_enum_opts;

#define EFM_OPT_NO_PRUNE 1u      /* skip the found-set minimality prune (result unchanged) */
#define EFM_OPT_EXACT_RANK 2u    /* decide every row-closed child by fraction-free 128-bit
                                    elimination, skipping the modular tests and the modular
                                    null-vector lift (slower; result unchanged) */
#define EFM_OPT_NO_GF2 8u        /* skip the modulo-2 independence certificate, so every undecided
                                    rank test runs modulo the prime (result unchanged) */
#define EFM_OPT_AUTOTUNE 16u     /* batch only: time candidate tile shapes once at creation and keep
                                    the fastest */
#define EFM_OPT_TIME_KERNELS 4u  /* record HIP events around every kernel launch on the stream and
                                    report per-level kernel times in efm_level_stats */

/* Per-level counters (level k = partial pathways of k reactions). */
typedef struct {
  int64_t parents;      /* frontier members expanded at this level */
  int64_t children;     /* children generated (with repeats) */
  int64_t unique;       /* distinct children */
  int64_t row_closed;   /* distinct children that needed the rank test */
  int64_t pruned;       /* of those, removed by the found-set prune */
  int64_t independent;  /* distinct children with independent columns */
  int64_t emitted;      /* elementary pathways found */
  int64_t kept;         /* frontier members of the next level (after the cap) */
  double ms_expand;     /* kernel times on the stream (EFM_OPT_TIME_KERNELS only, else 0) */
  double ms_rank;
  double ms_exact;
  double ms_select;
  double ms_materialize;
} efm_level_stats;

/* Create a network from S (Section 2.1).
 *   S          host, row-major n_met x n_rxn int32, copied; S[i][j] > 0 when reaction j
 *              produces metabolite i, < 0 when it consumes it
 *   reversible host, n_rxn bytes (0/1), copied
 *   external   host, n_met bytes (0/1), copied; external rows are not balanced
 * Uploads the device tables to the current device.
 * Errors: EFM_EINVAL when n_met <= 0, n_rxn <= 0 or > EFM_MAX_RXN, or a pointer is NULL;
 *         EFM_EDEVICE on a HIP failure. */
efm_status efm_network_create(int32_t n_met, int32_t n_rxn, const int32_t *S,
                              const uint8_t *reversible, const uint8_t *external,
                              efm_network **out);
efm_status efm_network_destroy(efm_network *net);

/* Device bytes the enumeration needs for these options (the capacities given, or
 * their defaults). */
efm_status efm_workspace_query(const efm_network *net, const efm_enum_opts *opts,
                               size_t *bytes);

/* Enumerate the elementary pathways that produce the external metabolite
 * target_met (Proposition 1 with R_in = the reactions that can produce it).
 * The result holds every pair (E, v) with |E| <= depth_cap, S_int v = 0, v_r > 0
 * on irreversible r, S[target,:] v > 0, gcd(v) = 1, and no balanced mode on a
 * smaller support -- minus what a frontier cap cut (flagged).  Blocks until the
 * work queued on opts->stream has finished.
 * Errors: EFM_EINVAL (target not external, or no reaction can produce it);
 *         EFM_ENOMEM (workspace_bytes below the query, or a capacity overflowed:
 *         raise unique_cap / found_cap); EFM_EDEVICE; EFM_EOVERFLOW. */
efm_status efm_enumerate(const efm_network *net, int32_t target_met,
                         const efm_enum_opts *opts, efm_result **out);

/* Result accessors.  n_levels counts levels 1..L; stats may be NULL, otherwise it
 * receives min(max_levels, n_levels) entries (index 0 = level 1). */
efm_status efm_result_info(const efm_result *res, int64_t *n_pathways, int32_t *words,
                           uint32_t *status_flags, int32_t *n_levels);
efm_status efm_result_stats(const efm_result *res, efm_level_stats *stats, int32_t max_levels);
/* dst: host, n_pathways * W words, canonical order.  EFM_EINVAL if dst_words is short. */
efm_status efm_result_bitsets(const efm_result *res, uint64_t *dst, int64_t dst_words);
/* dst: host, n_pathways * n_rxn int64, dense fluxes in the same order. */
efm_status efm_result_fluxes(const efm_result *res, int64_t *dst, int64_t dst_len);
efm_status efm_result_destroy(efm_result *res);

/* ---------------------------------------------------------------- batches
 * Many independent networks, each with one target, traversed in one persistent
 * kernel launch: every workgroup pops a network from a device work queue and
 * runs its whole level loop (the same method as efm_enumerate).  The launch is
 * captured once in a HIP graph and replayed by efm_batch_run.  Per-network
 * results equal those of efm_enumerate with the same options.
 *
 * efm_batch_create: nets[i] (created by efm_network_create, at most 256
 *   reactions and 128 internal metabolites each) with targets[i] (an external
 *   metabolite of nets[i]); opts supplies depth_cap, frontier_cap (per network and
 *   level), unique_cap (distinct children per network and level, default 262144),
 *   found_cap (pathways per network, default 4096) and flags (EFM_OPT_NO_PRUNE,
 *   EFM_OPT_EXACT_RANK, EFM_OPT_NO_GF2, EFM_OPT_AUTOTUNE); opts->workspace and
 *   opts->stream are not used.  The batch owns its device memory and a private
 *   stream; the networks must outlive the call only.
 *   Errors: EFM_EINVAL (null, empty, too large, bad target), EFM_EDEVICE.
 * efm_batch_run: replays the graph on `stream` (NULL: the batch's stream) and
 *   blocks until it finishes; results and latencies then refer to this run.
 * efm_batch_result: network i's result (caller destroys it).  Its stats hold one
 *   summary entry (parents, children, emitted).  Errors: EFM_EINVAL before a run
 *   or for a bad index; EFM_ENOMEM / EFM_EOVERFLOW when that network overflowed a
 *   capacity or the exact arithmetic.
 * efm_batch_latency: ns[i] = device time from network i's start to its end
 *   (device wall clock), for count entries.
 * efm_batch_config_get: the tile shape in use. */
typedef struct efm_batch efm_batch;
typedef struct {
  int32_t waves_per_network;   /* waves of the workgroup that runs one network */
  int32_t networks_per_cu;     /* persistent workgroups per compute unit */
} efm_batch_config;

efm_status efm_batch_create(const efm_network *const *nets, const int32_t *targets, int32_t count,
                            const efm_enum_opts *opts, efm_batch **out);
efm_status efm_batch_run(efm_batch *batch, void *stream);
efm_status efm_batch_result(const efm_batch *batch, int32_t i, efm_result **out);
efm_status efm_batch_latency(const efm_batch *batch, int64_t *ns);
efm_status efm_batch_config_get(const efm_batch *batch, efm_batch_config *cfg);
efm_status efm_batch_destroy(efm_batch *batch);

const char *efm_status_string(efm_status s);
const char *efm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EFM_H */
