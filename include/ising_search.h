/*
 * ising_search.h -- C ABI of the MI355X (gfx950) library for the synchronous
 * quantum-inspired (QI) low-energy search of classical Ising Hamiltonians
 * (Ueda, Otsuka, Yunoki, arXiv:2010.00180).
 *
 * Problem (Sec. I, Eq. 1): H0 = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i on a fully
 * connected graph of N spins.  A state is the integer psi = sum_i 2^i sigma_i
 * with sigma_i = 0 <=> s_i = +1 and sigma_i = 1 <=> s_i = -1 (Sec. III, Eq. 15).
 * Bit layout everywhere: W = ceil(N/64) little-endian uint64 words per state;
 * bit i of word i>>6 is sigma_i; bits at positions >= N must be zero.
 *
 * Method (Sec. II, Eqs. 9-14 in the infinitesimal-lambda limit, with the
 * one- and two-spin flip terms of H1, Eq. 16): every search keeps a set of at
 * most M distinct states.  One step replaces the set by the M lowest distinct
 * states of the union of the neighbourhoods (the state, its N single flips and
 * its N(N-1)/2 pair flips) of its states; the search is stable when a step
 * brings no new state.  Searches start from one initial state each; the L
 * searches of one instance are merged at the end into the M lowest distinct
 * states of their union (Alg. 4).  Ties in energy are broken by psi (smaller
 * first), which makes every kept set unique.
 *
 * Exact arithmetic: J_ij and h_i must be integer multiples of 2^-24 and
 * sum_{i<j} |J_ij| + sum_i |h_i| <= 2^24.  All energies, local fields and
 * energy changes are then exact in FP64 and independent of summation order.
 *
 * Errors: every call returns an ising_status_t; negative values are errors and
 * leave a message for ising_search_last_error().  No call aborts the process.
 * Calls on one handle must not overlap; different handles are independent.
 */
#ifndef ISING_SEARCH_H
#define ISING_SEARCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ising_search ising_search_t; /* opaque; owns all of its device memory */

typedef enum {
    ISING_OK = 0,
    ISING_NOT_CONVERGED = 1,   /* run() hit its step cap; the state is valid and can be continued */
    ISING_ERR_INVALID_ARG = -1,
    ISING_ERR_NO_DEVICE = -2,
    ISING_ERR_OUT_OF_MEMORY = -3,
    ISING_ERR_HIP = -4,
    ISING_ERR_BAD_STATE = -5,  /* NULL or destroyed handle, or a handle after a device error */
    ISING_ERR_CAPACITY = -6    /* a search produced more tied candidates than its buffer holds */
} ising_status_t;

typedef enum {
    ISING_FORM_PLAIN = 0,      /* exact local fields, FP64 energy-change scan */
    ISING_FORM_SPLIT_BF16 = 1, /* initial local fields from J = hi + lo (bf16) on MFMA with FP32
                                  accumulation, FP32 scan with a proven error slack, FP64 re-score */
    ISING_FORM_LEARNED = 2     /* pair flips ranked by a small network; only the best K per state are
                                  evaluated exactly (see the learned-form section below) */
} ising_form_t;

enum {
    ISING_FLAG_RECORD_PROPOSALS = 1,  /* learned form: keep each step's proposals for
                                         ising_search_get_proposals (B*L*M*K*4 bytes) */
    ISING_FLAG_SITE_BOUND = 2,        /* plain and split forms: skip pair flips that a bound proves
                                         cannot enter (not in the paper; see below) */
    ISING_FLAG_FP16_SCAN = 4,         /* split form: the pair scan in packed FP16 (two pairs per
                                         instruction) with a slack for FP16 rounding; every admitted
                                         pair is still re-scored in FP64, so the kept sets are the
                                         same (see the split-form section below) */
    ISING_FLAG_SINGLE_FLIPS = 8,      /* plain form: H1 = sum_i sigma^x_i only (the J = 1 choice of
                                         Sec. VI): the neighbourhood of a state is the state and its
                                         N single flips; O(N) per expanded state */
    ISING_FLAG_EXCHANGE = 16          /* plain form: H1 = sum_{i<j} (sigma^x_i sigma^x_j +
                                         sigma^y_i sigma^y_j), the XX interaction of Sec. VI: the
                                         neighbourhood is the state and the exchanges of two unequal
                                         spins (the pair flips with s_i != s_j); the number of down
                                         spins is conserved, so every initial state of an instance
                                         must have the same number (one sector per instance; give an
                                         instance again with other initial states for another
                                         sector), and ising_search_set_search keeps a search in its
                                         sector */
};

/*
 * Site bound (ISING_FLAG_SITE_BOUND).  The pair flip (i, j) of a state with
 * single-flip changes a_i = -2 s_i F_i changes the energy by
 * a_i + a_j + s_i s_j 4J_ij >= a_i + min_k a_k - max_k |4J_ik|, so it can pass
 * the step's cut T only if both of its sites satisfy
 * a_i + min_k a_k - max_k |4J_ik| <= T.  A state with at most 256 such sites has
 * exactly the pairs among them evaluated (FP64, the same arithmetic as the
 * scan) by a kernel of its own before the preparation and leaves the scan; the
 * others are prepared and scanned in full.  The kept sets are identical with and without the flag (every value
 * involved is exact on the 2^-24 grid); pair_evals then counts the pairs
 * actually evaluated and bounded_states the states resolved this way.
 */

typedef struct {
    int32_t M;                 /* states kept per search, >= 1 */
    int32_t max_iters;         /* default step cap used by ising_search_run when its cap is <= 0 */
    int32_t form;              /* ising_form_t */
    int32_t states_per_item;   /* scan tile: frontier states per work item; 0 = chosen by every step
                                  from its work (the largest power of two up to 256 that leaves each
                                  scan wave 16 items; 64 with the site bound or the learned form);
                                  ising_search_autotune keeps it only if it beats the tuned tiles */
    int32_t topk_factor;       /* learned form: K = topk_factor * N pairs per state (default 8) */
    int32_t persistent;        /* 1 = graph mode: ising_search_step replays a hipGraph of one step's
                                  kernels, ising_search_run a hipGraph of graph_steps steps (an internal
                                  stream is used when none is given) */
    int32_t timing;            /* 1 = time every kernel family with hipEvents on the handle's stream */
    int32_t flags;             /* ISING_FLAG_* bits; other bits must be zero */
    int32_t graph_steps;       /* graph mode: steps per replayed graph in ising_search_run, 1 .. 64
                                  (0 = 8).  A step that finds every search stable, or a search whose
                                  candidate buffer fills, makes the kernels of the graph's later steps
                                  return at once; the host reads the flags once per graph (not once per
                                  step) and finishes a full buffer's step with its retry passes.  The
                                  results are those of single steps. */
    int32_t surv_capacity;     /* candidate records per search (0 = 32768; 65536 for the learned form);
                                  otherwise between max(2M, 64) and 2^24.  A search whose candidates
                                  do not fit is re-scanned with the cut its stored candidates give
                                  (stats.retries); when that cut cannot move (the stored records are
                                  copies of fewer than M distinct states) every buffer doubles, a
                                  device allocation inside the step, up to 2^24 records
                                  (stats.surv_capacity); past that the step fails with CAPACITY */
    const char *tile_cache;    /* NULL, or a text file of tuned scan tiles that ising_search_autotune
                                  reads and appends to: one line per (device architecture, form,
                                  flags, N, M) with the states per item it chose.  Sizes found there
                                  are not timed again.  The path is copied; the file is created at
                                  init when missing (INVALID_ARG if it cannot be opened to append).
                                  Lines that do not parse are ignored. */
    const char *mlp_weights;   /* learned form: NULL, or a file of exactly ising_mlp_num_params()
                                  little-endian FP32 values (the parameter vector described with the
                                  learned form) that init installs as the network scorer, as
                                  ising_search_set_scorer(NETWORK, params, 0) would; INVALID_ARG if it
                                  cannot be read, has another size or holds a non-finite value */
} ising_config_t;

typedef struct {
    uint64_t steps;            /* steps executed (all searches advance together) */
    uint64_t pair_evals;       /* pair-flip energy changes evaluated by the scan */
    uint64_t single_evals;     /* single-flip energy changes evaluated */
    uint64_t frontier_states;  /* states expanded, summed over steps */
    uint64_t survivors;        /* candidates that passed the scan's cut, summed over steps */
    uint64_t retries;          /* re-scans of a search after its candidate buffer filled */
    uint64_t fallbacks;        /* split form: pairs admitted by the reduced-precision scan and then
                                  rejected by the FP64 re-score; learned form: full-enumeration steps
                                  (search-steps that evaluated every pair) */
    uint64_t scan_launches;    /* launches of the pair-scan kernel */
    double scan_ms;            /* device time of the pair-scan kernel (cfg.timing = 1), summed */
    double merge_ms;           /* device time of the per-search merge, summed */
    double frontier_ms;        /* device time of frontier listing, pilot cut and planning, summed */
    double prep_ms;            /* device time of the per-state preparation, summed */
    double init_ms;            /* device time of local fields and seeding (init and reset), summed */
    double step_ms;            /* persistent mode: device time of the replayed step graphs, summed */
    double split_field_err;    /* split form: max |F~ - F| of the initial states' bf16 hi+lo fields */
    uint64_t scored_pairs;     /* learned form: pair flips scored by the ranking kernel */
    uint64_t ranked_states;    /* learned form: states expanded with ranked pairs */
    uint64_t trace_samples;    /* samples offered to the trace buffer since ising_search_set_trace */
    double learn_ms;           /* learned form: device time of the ranking kernel, summed */
    uint64_t bounded_states;   /* site bound: expanded states whose pairs were evaluated among their
                                  bounded sites only */
    uint64_t surv_capacity;    /* candidate records per search now: cfg.surv_capacity or its
                                  default, doubled each time a step's candidates could not fit */
    double bound_ms;           /* site bound: device time of the site-bound kernel, summed (part of
                                  prep_ms) */
    uint64_t field_bytes;      /* bytes per stored local field: 4 when every instance's fields are
                                  held as 32-bit integers of its grid (|h_i| + sum_j |J_ij| below
                                  2^31 units of the coarsest power-of-two grid its values lie on),
                                  else 8 (FP64); exact either way */
} ising_stats_t;

/*
 * Create a handle and run the first part of the method: copy the instances to
 * the device, compute the local fields F = h + J s of every initial state
 * (FP64 MFMA GEMM, one per instance) and their energies (Eq. 1 through
 * E = (1/2) sum_i s_i (F_i + h_i)), and seed every search with S_0 = {x0}.
 *
 *   out        receives the handle (set to NULL on failure)
 *   cfg        configuration (see ising_config_t)
 *   n_inst     number of instances B >= 1
 *   N          [B] spins per instance, 1 <= N[b] <= 4096
 *   J          [B] host pointers to N[b]*N[b] row-major FP64 couplings; exactly
 *              symmetric, zero diagonal (Eq. 1 sums i<j, so an upper-triangle
 *              caller must mirror first)
 *   h          [B] host pointers to N[b] FP64 fields
 *   L          searches (initial states) per instance, >= 1
 *   init_bits  [B] host pointers to L*W[b] uint64 words (L initial states)
 *   stream     hipStream_t to order all device work on, or NULL for the
 *              default stream
 * Host inputs are copied; the caller keeps ownership.  Errors: INVALID_ARG
 * (sizes, asymmetry, nonzero diagonal, non-finite or off-grid values, stray
 * bits), NO_DEVICE, OUT_OF_MEMORY, HIP.
 */
int ising_search_init(ising_search_t **out, const ising_config_t *cfg, int32_t n_inst,
                      const int32_t *N, const double *const *J, const double *const *h,
                      int32_t L, const uint64_t *const *init_bits, void *stream);

/*
 * Restart every search from its initial state (the L states given to init,
 * kept on the device): local fields by the FP64 MFMA GEMM, energies, and
 * S_0 = {x0}.  Statistics counters are kept.  Lets a caller repeat a search
 * without copying the instances again.
 */
int ising_search_reset(ising_search_t *s);

/*
 * One synchronous step of every search still running (Sec. II): expand the
 * states that entered in the previous step by all single and pair flips,
 * evaluate their energies from local fields, and keep the M lowest distinct
 * states of the union with the current set.  States already kept never need
 * re-expansion: their neighbours were offered one step earlier.
 * n_active (may be NULL) receives the number of searches whose set changed.
 */
int ising_search_step(ising_search_t *s, int32_t *n_active);

/*
 * Step until every search is stable or max_iters steps were taken
 * (max_iters <= 0 uses cfg->max_iters).  iters_done (may be NULL) receives
 * the steps taken by this call, including the final one that found no new
 * state.  Returns ISING_OK when all searches are stable, ISING_NOT_CONVERGED
 * when the cap was reached first.
 */
int ising_search_run(ising_search_t *s, int32_t max_iters, int32_t *iters_done);

/*
 * Result of one instance (Alg. 4): the M lowest distinct states of the union
 * of its L kept sets, sorted by (E, psi).  bits_out: caller buffer of M*W
 * words; E_out: M doubles; count receives the number written (<= M).
 */
int ising_search_get_states(ising_search_t *s, int32_t instance, uint64_t *bits_out,
                            double *E_out, int32_t *count);

/*
 * The current kept set of one search (search = instance*L + l), sorted by
 * (E, psi), with front[k] = 1 for states that entered in the last step.
 * bits_out: M*W words; E_out: M doubles; front_out: M bytes (may be NULL).
 */
int ising_search_get_search(ising_search_t *s, int32_t search, uint64_t *bits_out,
                            double *E_out, uint8_t *front_out, int32_t *count);

/*
 * Replace the kept set of one search (checkpoint restore, or a test that
 * starts a step from a given set).  Up to M distinct states; energies and
 * local fields are recomputed on the device; front[k] marks states to expand
 * in the next step (NULL = all).  The search becomes active.
 */
int ising_search_set_search(ising_search_t *s, int32_t search, const uint64_t *bits,
                            const uint8_t *front, int32_t count);

int ising_search_get_stats(ising_search_t *s, ising_stats_t *out);

/*
 * One step (as ising_search_step) that first tunes the pair scan: for every
 * distinct N among the instances it times the scan for 16, 32, 64, 128 and 256
 * frontier states per work item on this step's frontier (coordinate descent
 * over the N buckets) and keeps the fastest; when the configuration leaves the
 * states per item to the steps (states_per_item 0), the tuned tiles are then
 * timed against that per-step choice and the faster is kept.  Results do not
 * depend on the choice; only the time does.  Best called once the frontier is
 * full (after the first step).  With cfg.tile_cache, sizes listed there for
 * this device, form, flags and M take the listed tiles untimed (the per-step
 * choice is then kept only if every listed size asks for it), and the sizes
 * tuned here are appended to the file.
 */
int ising_search_autotune(ising_search_t *s, int32_t *n_active);

/* The states per scan item in use for each instance (n_inst values; when
   chosen per step, those of the last step). */
int ising_search_get_tuning(ising_search_t *s, int32_t *states_per_item);

/*
 * ---------------------------------------------------------------- learned form
 * Not part of the paper (whose own lever for a cheaper step is a smaller
 * H1): a small network ranks the pair flips of each new state so that only
 * K = topk_factor * N of them (all of them if fewer) are evaluated exactly.
 * Features of the pair flip (i, j) of state x with local fields F = h + J s:
 *   (s_i F_i, s_j F_j, sqrt(N) J_ij, s_i s_j)
 * Network: 4 -> 64 -> 64 -> 1 with relu, evaluated on the bf16 matrix cores
 * with FP32 accumulation (weights, features and hidden activations rounded to
 * bf16, nearest even).  Parameter vector (ising_mlp_num_params() = 4545 FP32
 * values): W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3 (row-major).
 * A step of a search ranks the pairs of the states that entered in the last
 * step (their single flips are all offered) and keeps the M lowest distinct
 * states of the kept set and the offered children, exactly as the plain
 * step would for that candidate set.  When such a step brings nothing new,
 * the next step evaluates every pair flip of every kept state whose pairs
 * were not all evaluated before; if that finds nothing either, the set is a
 * fixed point of the exact step and the search stops.  stats.fallbacks counts
 * these full steps.
 */

/* Scorers of the learned form. */
enum {
    ISING_SCORER_NETWORK = 0,   /* the network with the given parameters */
    ISING_SCORER_FIELDS = 1,    /* s_i F_i + s_j F_j (the energy change without the coupling term) */
    ISING_SCORER_UNIFORM = 2    /* a hash of (seed, state, pair): a uniformly random ranking */
};

/*
 * Choose the scorer (required before the first step of a learned-form
 * handle).  params: host array of 4545 finite FP32 values for the network
 * scorer (copied), ignored otherwise; seed salts the uniform scorer.
 * Errors: INVALID_ARG (not the learned form, unknown scorer, NULL or
 * non-finite parameters).
 */
int ising_search_set_scorer(ising_search_t *s, int32_t scorer, const float *params, uint64_t seed);

/*
 * Capture training samples during later steps (any form).  For a fraction
 * `rate` of the states each step expands (chosen by a hash of seed, step and
 * state), one sample per pair flip of that state that entered the kept set
 * (label 1) and `pairs_per_state` uniformly drawn pairs i < j, labelled 1 iff
 * the child is a new member of the next kept set.  Sample k is written to
 * feat[4k .. 4k+3] (the four features above, FP32) and label[k] (0 or 1) while
 * k < capacity.  feat and label are device pointers owned by the caller and
 * must stay valid while tracing; NULL, NULL, 0 stops tracing.  The count of
 * samples offered (possibly above capacity) is reset here and read with
 * ising_search_get_trace_count.  Errors: BAD_STATE (a handle made with
 * ISING_FLAG_SITE_BOUND, which does not keep every expanded state's a row).
 */
int ising_search_set_trace(ising_search_t *s, float *feat, uint8_t *label, int64_t capacity,
                           int32_t pairs_per_state, float rate, uint64_t seed);
int ising_search_get_trace_count(ising_search_t *s, int64_t *count);

/*
 * Proposals of the last step of one search (handles created with
 * ISING_FLAG_RECORD_PROPOSALS).  For each ranked parent p < *n_parents:
 * its words in parent_bits[p*W .. p*W+W), its n_pairs[p] proposed pairs
 * (i | j << 16, i < j, in no particular order) in pairs[p*K .. p*K+n_pairs[p])
 * with K = ising_search_topk(s).  *mode is 0 when the step ranked pairs and 1
 * when it enumerated all pairs (then there are no ranked parents).  Call it
 * before the next step.  Errors: BAD_STATE (not recording), CAPACITY (more
 * than max_parents parents).
 */
int ising_search_get_proposals(ising_search_t *s, int32_t search, uint64_t *parent_bits, uint32_t *pairs,
                               int32_t *n_pairs, int32_t max_parents, int32_t *n_parents, int32_t *mode);

/* K of the largest instance (the row stride of get_proposals), or -1 for a bad handle. */
int32_t ising_search_topk(ising_search_t *s);

/*
 * Training of the network on the device, in FP32.  All array arguments are
 * device pointers owned by the caller; work is queued on `stream` (a
 * hipStream_t, NULL = default stream) and these calls do not synchronise.
 * Loss: the class-weighted binary cross-entropy with logits averaged over the
 * samples, L = mean(pos_weight * y * softplus(-z) + (1 - y) * softplus(z)).
 * feat: n x 4 FP32 features; label: n bytes (nonzero = 1).
 */
int32_t ising_mlp_num_params(void);
/* Bytes of the workspace that ising_mlp_loss_grad and ising_mlp_train need. */
int64_t ising_mlp_workspace_bytes(void);
/* logits[k] of sample k in FP32 (no rounding to bf16). */
int ising_mlp_forward(const float *params, const float *feat, int64_t n, float *logits, void *stream);
/* grad (4545) = dL/dparams over all n samples, and *loss (device, may be NULL). */
int ising_mlp_loss_grad(const float *params, const float *feat, const uint8_t *label, int64_t n,
                        float pos_weight, float *grad, float *loss, void *workspace,
                        int64_t workspace_bytes, void *stream);
/*
 * ising_mlp_loss_grad without a workspace argument and without any device
 * allocation, for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same loss, gradient and
 * pointer rules as ising_mlp_loss_grad; the per-block partial sums go to a
 * static device array of 256 rows (4,654,080 bytes per device, held until the
 * process ends), so the samples are spread over at most 256 blocks: for
 * n <= 16384 the result is bit-identical to ising_mlp_loss_grad, beyond that
 * it differs only in the FP32 summation order.  Every n >= 1 is accepted.
 * The array is shared by all calls on one device: calls that overlap on one
 * device (different streams or threads) race and must be serialised by the
 * caller.  `stream` must belong to the current device.  Errors: INVALID_ARG,
 * NO_DEVICE, HIP.
 */
int ising_mlp_loss_grad_noalloc(const float *params, const float *feat, const uint8_t *label, int64_t n,
                                float pos_weight, float *grad, float *loss, void *stream);
/* One Adam step (t >= 1): m, v and params updated in place (Kingma and Ba, Alg. 1). */
int ising_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t t, float lr,
                   float beta1, float beta2, float eps, void *stream);
/*
 * `steps` Adam steps (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, step numbers
 * t0+1 ..), each on a minibatch of `batch` samples drawn uniformly with
 * replacement by a hash of (seed, step, k).  *loss (device, may be NULL)
 * receives the last minibatch's loss.
 */
int ising_mlp_train(float *params, float *m, float *v, const float *feat, const uint8_t *label, int64_t n,
                    int32_t batch, int32_t steps, int32_t t0, float lr, float pos_weight, uint64_t seed,
                    float *loss, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * ---------------------------------------------------------------- exhaustive enumeration
 * The K lowest states of each instance over all 2^N states, sorted by
 * (E, psi): the brute-force reference of Sec. IV (Fig. 1) and the exact
 * low-energy spectra of Sec. V (ground energy, first gap, E_k).  Every state is
 * visited on the GPU in Gray-code order (one spin flip per state, the energy
 * updated from the flipped site's couplings); energies are exact on the 2^-24
 * grid.  Not a step of the search: a separate call for references and
 * spectra.
 *
 *   n_inst     instances, >= 1; N[b] in [1, 40] (2^N states are visited, so
 *              N = 30 takes about 10^9 state visits per instance)
 *   J, h       host pointers as for ising_search_init (symmetric, zero
 *              diagonal, multiples of 2^-24, sum |J_ij| + sum |h_i| <= 2^24)
 *   K          states wanted per instance, 1 <= K <= 4096 (fewer when 2^N < K)
 *   bits_out   caller buffer of n_inst*K words: instance b's states at
 *              b*K .. b*K+count[b]-1 (one word per state, bit i = sigma_i)
 *   E_out      caller buffer of n_inst*K doubles, the same layout
 *   count      caller buffer of n_inst ints: min(K, 2^N)
 *   stream     hipStream_t or NULL
 * The call allocates device memory for its own use and frees it before
 * returning; it synchronises the stream.  Errors: INVALID_ARG, NO_DEVICE,
 * OUT_OF_MEMORY, HIP, CAPACITY (more than 8192 states tie at the K-th lowest
 * energy of an instance).
 */
int ising_brute_lowest(int32_t n_inst, const int32_t *N, const double *const *J, const double *const *h,
                       int32_t K, uint64_t *bits_out, double *E_out, int32_t *count, void *stream);

/*
 * ---------------------------------------------------------------- best-first search (Alg. 2-4)
 * The paper's own sequential form of the method (Sec. III), one GPU block per
 * search: Alg. 3 (QI single search) keeps a list of K + 1 entries in energy
 * order (equal energies in order of arrival) and, I times, expands the first
 * entry not yet expanded, offering its single flips (sites 0 .. N-1) and then
 * its pair flips ((0,1), (0,2), .., (N-2,N-1)) one after the other with the
 * update of Alg. 2 (a state enters when the list does not hold it and its
 * energy is below the last entry's); Alg. 4 (QI multi search) runs L such
 * searches and merges their lists, in order, with the same update.  Readings:
 * placeholder entries are never expanded; the merge offers every state with
 * its own energy.  flags may hold ISING_FLAG_SINGLE_FLIPS or
 * ISING_FLAG_EXCHANGE (the other H1 choices of Sec. VI; exchanges of equal
 * spins give the parent back and are skipped).
 *
 *   n_inst, N, J, h   as for ising_search_init, with 1 <= N[b] <= 64
 *   L                 searches per instance, n_inst * L <= 2^24; init_bits[b]
 *                     holds L words (no bits at positions >= N[b])
 *   K, I              list of K + 1 entries (K + 1 <= 2^20), I >= 0 iterations;
 *                     a search keeps its list, the list's double buffer and
 *                     the hash of its states in LDS when they fit beside the
 *                     offered children in 160 KB, else in device memory
 *                     (about 58 (K+1) bytes per search, 78 (K+1) per instance
 *                     for the merge; the same result, more slowly)
 *   merged_bits/E     caller buffers of n_inst*(K+1): instance b's merged list
 *                     at b*(K+1), merged_count[b] real entries, in list order
 *   search_*          NULL, or caller buffers of n_inst*L*(K+1) (count: n_inst*L)
 *                     with each search's own final list, its expanded flags
 *                     and the iteration at which each entry arrived (0 = the
 *                     initial state); search_bits, search_E and search_count
 *                     go together, used and born may be NULL
 *   expanded          NULL or n_inst*L: iterations that expanded a state
 *   kernel_ms         NULL or the device time of the search and merge kernels
 * Device memory is allocated for the call and freed before it returns; the
 * call synchronises the stream.  Errors: INVALID_ARG, NO_DEVICE,
 * OUT_OF_MEMORY, HIP.
 */
int ising_bestfirst(int32_t n_inst, const int32_t *N, const double *const *J, const double *const *h, int32_t L,
                    const uint64_t *const *init_bits, int32_t K, int32_t I, int32_t flags, uint64_t *merged_bits,
                    double *merged_E, int32_t *merged_count, uint64_t *search_bits, double *search_E,
                    uint8_t *search_used, int32_t *search_born, int32_t *search_count, int32_t *expanded,
                    float *kernel_ms, void *stream);

/* Frees all device memory of the handle.  NULL is accepted. */
void ising_search_destroy(ising_search_t *s);

/* Message of the last error on the calling thread ("" if none). */
const char *ising_search_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_SEARCH_H */
