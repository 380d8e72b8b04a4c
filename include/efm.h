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
#define EFM_OPT_AUTOTUNE 16u     /* batch only: time candidate tile shapes once at creation (on every
                                    4th network of the batch) and keep the fastest */
#define EFM_OPT_TIME_KERNELS 4u  /* record HIP events around every kernel launch on the stream and
                                    report per-level kernel times in efm_level_stats */
#define EFM_OPT_LEARNED 32u      /* workspace layout of efm_enumerate_learned (adds one 4-byte score
                                    per distinct child); pass it to efm_workspace_query when sizing
                                    a workspace for that call */

/* Per-level counters (level k = partial pathways of k reactions). */
typedef struct {
  int64_t parents;      /* frontier members expanded at this level */
  int64_t children;     /* children generated (with repeats) */
  int64_t unique;       /* distinct children */
  int64_t row_closed;   /* distinct children that needed the rank test (depends on which parent
                           inserted a child first, so it may vary between runs) */
  int64_t pruned;       /* of those, removed by the found-set prune */
  int64_t independent;  /* distinct children with independent columns */
  int64_t emitted;      /* elementary pathways found */
  int64_t kept;         /* frontier members of the next level (after the cap) */
  double ms_expand;     /* kernel times on the stream (EFM_OPT_TIME_KERNELS only, else 0) */
  double ms_rank;
  double ms_exact;
  double ms_select;     /* truncation: scoring (learned ordering) and selection */
  double ms_materialize;
  int64_t rank_rows;    /* sum over the row-closed children tested of the rows their test
                           spans (the parent's touched internal metabolites) */
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
 *   blocks until it finishes; results and latencies then refer to this run.  The
 *   first run takes the networks largest first; every later run takes them in
 *   decreasing order of the previous run's latency.
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


/* ------------------------------------------------------- learned ordering
 * A three-layer perceptron scores partial pathways for whether they will close
 * into an elementary pathway; efm_enumerate_learned keeps, at every level whose
 * independent children exceed the budget, the `budget` best-scored ones (ties by
 * canonical order) instead of the canonically smallest.  Every pathway it
 * returns is still decided by the exact rank test, so the output is always a
 * subset of the exhaustive result; with a budget at least as large as every
 * level, it equals efm_enumerate's.  The ordering replaces the random choices of
 * the paper's Algorithm 3 under the search budget its Theorem 1 discusses.
 *
 * Input of a partial pathway P of a network, for target x: reactions and
 * internal metabolites are relabelled by breadth-first distance from the
 * reactions that touch x (then decreasing degree, then index).  One entry per
 * reaction of P (value 1 at its position, < in_bits) and one per internal
 * metabolite i whose imbalance count u_i = clamp(#{r in P: S_ir > 0} -
 * #{r in P: S_ir < 0}, -7, 7) is non-zero: metabolite position q owns rows
 * in_bits + 2q (surplus, u_i > 0) and in_bits + 2q + 1 (deficit), and the entry
 * is |u_i| / 8 on the row of its sign.  Entries are 16-bit words
 * (row << 4) | code: code 0 = a reaction (value 1), code c in 1..7 = an
 * imbalance of magnitude c (value c / 8).  At most EFM_FEAT_MAX entries.
 *
 * Model: s = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 with F = in_bits +
 * 2 * in_counts inputs and hidden = 256 units; fp32 master parameters, bf16 copies of
 * W1, W2 and w3 used by the kernels, fp32 accumulation.  Parameter vector order:
 * W1 [F][256] row-major, b1 [256], W2 [256 in][256 out], b2 [256], w3 [256], b3 [1].
 * Loss: mean over the batch of pw*y*softplus(-s) + (1-y)*softplus(s); Adam.
 */
#define EFM_FEAT_MAX 512
#define EFM_TRACE_WORDS 16   /* key words stored per trace record */

typedef struct efm_model efm_model;
typedef struct efm_traces efm_traces;

typedef struct {
  double neg_per_pos;    /* negatives kept per kept positive state at each level (<= 0: 4) */
  int64_t neg_min;       /* negatives kept at least per level, when there are any (<= 0: 64) */
  int64_t pos_max;       /* positives kept at most per level (<= 0: all) */
  uint64_t seed;         /* sampling seed */
} efm_trace_opts;

typedef struct {
  int64_t states;        /* frontier states seen */
  int64_t positives;     /* states contained in a pathway the plain run found (seen, not kept) */
  int64_t recorded;      /* records appended */
  int64_t pathways;      /* pathways the plain run found */
  uint32_t status;       /* status flags of the plain run */
  uint32_t reserved;
} efm_trace_info;

typedef struct {
  int32_t epochs;        /* passes over the traces (<= 0: 1) */
  int32_t batch;         /* records per step (<= 0: 1024), at most 65536 */
  float lr;              /* Adam step size (<= 0: 1e-3) */
  float beta1, beta2;    /* (<= 0: 0.9, 0.999) */
  float eps;             /* (<= 0: 1e-8) */
  float pos_weight;      /* weight of positive records (<= 0: #negatives / #positives) */
  uint32_t reserved;
  uint64_t seed;         /* shuffling seed */
  void *stream;          /* hipStream_t (NULL = null stream) */
} efm_train_opts;

typedef struct {
  int64_t steps;         /* Adam steps taken by this call */
  double loss_first;     /* mean loss over the first epoch */
  double loss_last;      /* mean loss over the last epoch */
  double ms;             /* wall time of the call */
} efm_train_stats;

/* Traces: labelled partial pathways in model-input form, in device memory.
 * efm_traces_create: room for `capacity` records.  EFM_EINVAL unless
 *   0 < in_bits <= EFM_MAX_RXN, 0 < in_counts <= 1024, capacity > 0.
 * efm_traces_info: records held and how many of them are positive.
 * efm_trace_collect (Section 4.1 traversal used as a teacher): runs the plain
 *   traversal of efm_enumerate with opts, then runs it again and, at every level
 *   (the first frontier holds the target's producing reactions), labels each
 *   frontier state 1 when a pathway found by the
 *   first run contains it, keeps the positives (a hashed sample of pos_max when
 *   there are more) and a hashed sample of the negatives (max(neg_min,
 *   neg_per_pos * kept positives) per level), and appends them.  EFM_EINVAL when
 *   the network does not fit in_bits / in_counts or a reaction touches more than
 *   16 internal metabolites; EFM_ENOMEM
 *   when the traces are full (records up to capacity are kept).
 * efm_traces_append: records from the host (entries count x EFM_FEAT_MAX words,
 *   lengths, labels 0/1); keys are stored as zero.
 * efm_traces_fetch: copies records [first, first + count) to the host; any
 *   pointer may be NULL (entries count x EFM_FEAT_MAX, keys count x
 *   EFM_TRACE_WORDS). */
efm_status efm_traces_create(int32_t in_bits, int32_t in_counts, int64_t capacity, efm_traces **out);
efm_status efm_traces_destroy(efm_traces *tr);
efm_status efm_traces_info(const efm_traces *tr, int64_t *count, int64_t *positives);
efm_status efm_trace_collect(efm_traces *tr, const efm_network *net, int32_t target_met,
                             const efm_enum_opts *opts, const efm_trace_opts *topts,
                             efm_trace_info *info);
efm_status efm_traces_append(efm_traces *tr, const uint16_t *entries, const uint16_t *lengths,
                             const uint8_t *labels, int64_t count);
efm_status efm_traces_fetch(const efm_traces *tr, int64_t first, int64_t count, uint16_t *entries,
                            uint16_t *lengths, uint8_t *labels, uint64_t *keys);

/* Model.  efm_model_create: hidden must be 256; weights uniform in +-sqrt(6/fan)
 *   (fan 32 for W1, 256 otherwise) from a seeded generator, biases 0.
 * efm_model_get_params / set_params: the fp32 parameter vector (len = n_params);
 *   set_params also rounds the bf16 copies (to nearest even) and clears Adam.
 * efm_model_save / load: a binary file (parameters, Adam moments and step).
 * efm_model_score: logits of records [first, first + count) (host output).
 * efm_model_score_keys: logits of partial pathways of `net` for target_met given as
 *   bitsets (host, count x W words of the network), with the traversal's own
 *   featurisation.
 * efm_model_grad: mean loss and its gradient (host, n_params floats) over
 *   records [first, first + count), count <= 65536, without an update.
 * efm_model_train: Adam over all records, shuffled per epoch.
 * All run on the null stream except train (opts->stream) and block until done. */
efm_status efm_model_create(int32_t in_bits, int32_t in_counts, int32_t hidden, uint64_t seed,
                            efm_model **out);
efm_status efm_model_destroy(efm_model *model);
efm_status efm_model_info(const efm_model *model, int64_t *n_params, int32_t *in_bits,
                          int32_t *in_counts, int32_t *hidden);
efm_status efm_model_get_params(const efm_model *model, float *dst, int64_t len);
efm_status efm_model_set_params(efm_model *model, const float *src, int64_t len);
efm_status efm_model_save(const efm_model *model, const char *path);
efm_status efm_model_load(const char *path, efm_model **out);
efm_status efm_model_score(const efm_model *model, const efm_traces *tr, int64_t first, int64_t count,
                           float *scores);
efm_status efm_model_score_keys(const efm_model *model, const efm_network *net, int32_t target_met,
                                const uint64_t *keys, int64_t count, float *scores);
efm_status efm_model_grad(const efm_model *model, const efm_traces *tr, int64_t first, int64_t count,
                          float pos_weight, float *grad, double *loss);
efm_status efm_model_train(efm_model *model, const efm_traces *tr, const efm_train_opts *opts,
                           efm_train_stats *stats);

/* efm_enumerate with frontier_cap = budget and the learned ordering of the
 * truncation.  opts as for efm_enumerate (its frontier_cap is ignored); a
 * caller-provided workspace must be sized by efm_workspace_query with
 * EFM_OPT_LEARNED set.  Errors as efm_enumerate, plus EFM_EINVAL when the model's
 * input does not fit the network or budget <= 0. */
efm_status efm_enumerate_learned(const efm_network *net, int32_t target_met, int64_t budget,
                                 const efm_model *model, const efm_enum_opts *opts, efm_result **out);

const char *efm_status_string(efm_status s);
const char *efm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EFM_H */
