/*
 * lp.h -- C ABI of the MI355X (gfx950) engine for linear-algebraic T_P
 * fixpoints over sparse program matrices.
 *
 * The operations follow Nguyen, Inoue and Sakama, "Enhancing Linear Algebraic
 * Computation of Logic Programs Using Sparse Representation" (ICLP 2020):
 *   - the program matrix of a standardized program (Definition 2) and of the
 *     positive form of a normal program (Definition 7), stored as CSR
 *     (Section 3.2);
 *   - the least-model fixpoint v <- theta(M v) from the initial vector
 *     (Definitions 3-5, Algorithm 1);
 *   - the stable-model fixpoint over an initial matrix with one column per
 *     guess, followed by the column consistency test (Definition 8,
 *     Algorithms 2 and 3).
 *
 * Conventions shared by every call:
 *   - Every call returns lp_status: LP_OK (0) or a negative error code. No C++
 *     exception crosses this boundary. lp_last_error() returns a message for
 *     the calling thread's last failing call.
 *   - Pointers named in the argument lists are HOST pointers unless a name
 *     says d_ (device). Inputs are owned by the caller and are only read
 *     during the call; nothing is retained. Outputs go to caller-owned host
 *     buffers and are complete when the call returns (the call synchronizes
 *     the stream it was given).
 *   - hip_stream is a hipStream_t passed as void*; NULL means the default
 *     stream. All device work of a call is issued on that stream.
 *   - An lp_matrix is immutable after lp_build_matrix and may be used by
 *     several calls at once on distinct streams (each solve allocates its own
 *     interpretation buffers).
 *
 * Program layout (the input of lp_build_matrix):
 *   head[r]      head atom of rule r, 0 <= head[r] < n_atoms
 *   body_ptr[r]  rule r's literals are body_lit[body_ptr[r] .. body_ptr[r+1]);
 *                body_ptr has n_rules+1 entries, body_ptr[0] == 0, nondecreasing
 *   body_lit[e]  a >= 0: atom a;  a < 0: the negative literal "not atom (-a-1)"
 *   A rule with an empty body is a fact. Bodies are sets (the paper assumes
 *   distinct body atoms), so repeated literals in one body are merged.
 */
#ifndef LP_H
#define LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lp_status;

enum {
    LP_OK = 0,
    LP_E_INVAL = -1,            /* malformed input or argument; nnz or rows >= 2^31 */
    LP_E_NOMEM = -2,            /* host or device memory exhausted (checked before launches) */
    LP_E_DEVICE = -3,           /* a HIP runtime call failed */
    LP_E_NEGATION = -4,         /* lp_least_model on a program with negative literals */
    LP_E_TOO_MANY_GUESSES = -5, /* more than LP_MAX_NEG_ATOMS negated atoms */
    LP_E_TRUNCATED = -6,        /* more stable models than max_models (outputs still valid) */
    LP_E_INTERNAL = -7,         /* an invariant of the fixpoint failed (should not happen) */
    LP_E_HOST_ONLY = -8,        /* solve on a matrix built with LP_BUILD_HOST_ONLY */
    LP_E_TIMEOUT = -9           /* lp_server_wait_any: nothing completed in time */
};

#define LP_MAX_NEG_ATOMS 24

/* lp_build_matrix flags */
enum {
    /* Definition 8, item 3: a qbar row is fixed to 0 when q is a fact, so the
     * guesses on such atoms are not enumerated. The stable models returned are
     * the same; only fewer columns are computed. */
    LP_PRUNE_FACT_GUESSES = 1u << 0,
    /* Build the host-side CSR only (no device memory, no HIP call). Used to
     * inspect the matrix; solve calls then return LP_E_HOST_ONLY. */
    LP_BUILD_HOST_ONLY = 1u << 1,
    /* Stable-model products (Algorithm 2) evaluate every row each time. By
     * default, when the interpretation matrix holds at least 2^19 words
     * (n_rows x 64-guess words), a product evaluates only the rows that name a
     * row changed by the previous product (the others cannot change); smaller
     * matrices are swept in full. The products, their count and the models
     * are the same either way. */
    LP_STABLE_FULL_SWEEP = 1u << 2,
    /* Stable-model products by dirty rows whatever the matrix size (ignored
     * with LP_STABLE_FULL_SWEEP). */
    LP_STABLE_DIRTY_ROWS = 1u << 3,
    /* Least models: lay the AND entries out in column slices of 1,024 atoms
     * (one pass per slice and product; by default slices are used only when
     * the original atoms exceed what a workgroup's LDS holds, about 1.29
     * million). For tests of the sliced step on small programs: at most 64
     * slices, so programs of at most 65,536 atoms (LP_E_INVAL otherwise). */
    LP_STEP_SLICES_SMALL = 1u << 4
};

typedef struct lp_matrix lp_matrix;

typedef struct lp_info {
    int32_t n_atoms;        /* N = |B_P| as given */
    int32_t n_rules;        /* R */
    int32_t n_std_atoms;    /* N + new atoms of the standardization */
    int32_t n_rows;         /* N' = n_std_atoms + n_neg: matrix dimension */
    int64_t nnz;            /* stored nonzeros of the program matrix */
    int32_t n_neg;          /* K: distinct atoms occurring negated */
    int32_t n_pruned;       /* negated atoms whose guess is pruned (flag above) */
    int32_t n_and_rows;     /* rows of a rule body (fire iff all entries true) */
    int32_t n_or_rows;      /* OR rows of the standardization (fire iff one entry true) */
    int32_t n_fact_rows;    /* rows of facts (self-loop, set in the initial vector) */
    int32_t n_empty_rows;   /* atoms with no rule (never true) */
    int32_t max_row_len;    /* longest row */
    int32_t n_long_rows;    /* rows handled by the split long-row pass */
    int64_t device_bytes;   /* device memory held by the matrix */
    int64_t step_bytes;     /* bytes one full-sweep step must move on this device layout
                               (least models: the AND lengths, one entry offset per four
                               words, the AND entries, the OR range table, the long-row
                               segments, one read of v and one write of u; stable models:
                               CSR, one read of V, one write of U for all 2^K guesses; 0 when
                               K exceeds LP_MAX_NEG_ATOMS) */
    double sparsity;        /* equation 5: 1 - sum_r |body(r)| / N^2 */
    int32_t n_slices;       /* least models: column slices of the step's layout (0: not sliced) */
    int32_t reserved_info;
} lp_info;

/* Device-side schedule of the fixpoint loop. Zero-initialize and set what you
 * need: 0 in any field selects the library default. */
enum {
    LP_DRIVER_AUTO = 0,       /* least models: with every other field 0 (or no schedule), programs
                                 of at most 131,072 stored entries + rows run the whole loop in one
                                 workgroup with the interpretations in LDS (one launch); otherwise
                                 BATCHED */
    LP_DRIVER_PLAIN = 1,      /* one launch per product, host reads the change count each time */
    LP_DRIVER_BATCHED = 2,    /* steps_per_sync launches between host reads of the change counts */
    LP_DRIVER_PERSISTENT = 3, /* one launch; the loop runs on the device with a grid barrier */
    LP_DRIVER_FRONTIER = 4    /* least models only: newly true rows pushed through the transposed
                                 matrix, one level per product: a launch per level for large
                                 frontiers, one workgroup looping over up to 256 levels while
                                 they hold at most 4,096 rows; each entry is visited once per
                                 solve (same model and product count; builds the transpose on
                                 first use, about 4 (n_rows + nnz) more device bytes) */
};

enum {
    LP_STEP_AUTO = 0,
    LP_STEP_GLOBAL = 1,  /* 256-thread workgroups, gathers of v from global memory */
    LP_STEP_LDS = 2      /* one 1024-thread workgroup per CU, the original atoms of v staged in LDS */
};

typedef struct lp_schedule {
    int32_t driver;          /* LP_DRIVER_* */
    int32_t steps_per_sync;  /* products issued between host checks (BATCHED, AUTO) */
    int32_t variant;         /* LP_STEP_* kernel of the least-model step */
    int32_t grid;            /* workgroups of the step (0: one per CU for LDS, eight per CU otherwise) */
    int32_t wpw;             /* 64-row words per super-block: step 4 or 8, batch kernel 4 or 8
                                (0: default) */
    int32_t unroll;          /* 64-entry column chunks in flight per wave: 4, 8 or 16 (0: default) */
    int32_t block;           /* batch kernel: threads per workgroup, 256, 512 or 1024 (0: 1024) */
    int32_t team;            /* batch plans: 0 teams chosen by size, 1 no teams, k >= 2 every
                                program solved by a team of k workgroups (at most 8 and half the
                                grid) */
    int32_t team_polls;      /* batch plans: polls after which a team barrier gives up (0: 2^22).
                                A team that gives up has its program solved alone by
                                lp_batch_results; small values force that path (tests) */
} lp_schedule;

/*
 * Build the program matrix.
 *
 * Definite rules are standardized first (Section 2.1, the paragraph after
 * Definition 1; Algorithm 1 step 1): every head h with k >= 2 rules gets k new
 * atoms b_1..b_k with rules b_i <- body(r_i) and one OR rule h <- b_1 v ... v b_k.
 * New atoms are numbered n_atoms, n_atoms+1, ... in ascending head order and,
 * within one head, in rule order. Negative literals "not q" are replaced by
 * new atoms qbar (equation 4; Definition 7): the K distinct negated atoms
 * q_0 < q_1 < ... take the last K row ids, qbar_t = n_std_atoms + t.
 *
 * Rows store column ids only; the 1/m weights of Definition 2 are replaced by
 * a per-row kind: an AND row fires iff all its entries are true (the count of
 * true entries equals the row length), an OR row iff at least one entry is
 * true. This is the theta-threshold of Definition 5 evaluated exactly. A fact
 * row holds its own atom (a_ii = 1) and is set in the initial vector; an atom
 * with no rule has an empty OR row and is never true.
 *
 * flags: LP_PRUNE_FACT_GUESSES, LP_BUILD_HOST_ONLY, LP_STABLE_FULL_SWEEP,
 * LP_STABLE_DIRTY_ROWS, LP_STEP_SLICES_SMALL.
 * On success *out owns host metadata and (unless host-only) device buffers,
 * uploaded on hip_stream, until lp_free_matrix.
 * Errors: LP_E_INVAL (bad ids, body_ptr not monotone, NULL arrays with
 * nonzero sizes, more than 2^31-1 rows or nonzeros), LP_E_NOMEM, LP_E_DEVICE.
 */
lp_status lp_build_matrix(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                          const int64_t *body_ptr, const int32_t *body_lit, uint32_t flags,
                          void *hip_stream, lp_matrix **out);

/* Release every host and device resource of m (NULL is accepted). */
lp_status lp_free_matrix(lp_matrix *m);

/*
 * Resident-matrix management. lp_matrix_evict releases m's device copy and
 * keeps the host CSR: m then behaves as if built with LP_BUILD_HOST_ONLY
 * (solves return LP_E_HOST_ONLY, lp_info.device_bytes = 0). The caller
 * guarantees that no solve or batch plan on m is in flight. lp_matrix_upload
 * builds the device copy again from the host CSR on hip_stream (synchronized
 * before it returns); on a matrix that is already on the device it does
 * nothing. Results after a round trip are those of a fresh build.
 */
lp_status lp_matrix_evict(lp_matrix *m);
lp_status lp_matrix_upload(lp_matrix *m, void *hip_stream);

/* Sizes and statistics of m. */
lp_status lp_matrix_info(const lp_matrix *m, lp_info *out);

/* The K negated atoms q_0 < ... < q_{K-1} (out: int32[K], host). */
lp_status lp_matrix_neg_atoms(const lp_matrix *m, int32_t *out);

/*
 * Host copy of the program matrix in CSR form (Section 3.2, Example 4):
 * row_ptr int32[n_rows+1], col int32[nnz] (ascending within a row),
 * kind uint8[n_rows] (1 = AND row, 0 = OR row), fact uint8[n_rows]
 * (1 = fact row, set in the initial vector). Any output may be NULL.
 */
lp_status lp_matrix_csr(const lp_matrix *m, int32_t *row_ptr, int32_t *col, uint8_t *kind,
                        uint8_t *fact);

/*
 * Least model of a definite program (Algorithm 1).
 * model: uint8[n_atoms] host, receives 1 for atoms of the least model
 *   (the fixpoint restricted to the original atoms).
 * products: nullable; receives the number of theta(M v) evaluations,
 *   including the last one that found no change (>= 1).
 * sched: nullable (library default).
 * Errors: LP_E_NEGATION if the program has negative literals,
 *   LP_E_HOST_ONLY, LP_E_NOMEM, LP_E_DEVICE, LP_E_INTERNAL.
 */
lp_status lp_least_model(const lp_matrix *m, uint8_t *model, int32_t *products,
                         const lp_schedule *sched, void *hip_stream);

/*
 * Stable models of a normal program (Algorithms 2 and 3).
 * Guess j (0 <= j < 2^K) is column j of the initial matrix: bit t of j is the
 * initial value of qbar_t (1 = q_t assumed false). Column j is accepted iff in
 * its fixpoint exactly one of q_t, qbar_t is true for every t; its model is
 * the column restricted to the original atoms.
 *
 * accepted:  uint64[ceil(2^K/64)] host; bit j%64 of word j/64 = guess j accepted.
 * n_models:  receives the number of stable models.
 * models:    nullable; uint8[max_models][n_atoms] host, the first max_models
 *            models in guess order.
 * interp:    nullable; uint64[n_atoms][ceil(2^K/64)] host, the fixpoint
 *            interpretation matrix restricted to the original atoms (bit j of
 *            row a = atom a true in column j). Requires no pruning.
 * products:  nullable; number of theta(M_P M) evaluations until no column changed.
 * K = 0 gives exactly one model, the least model.
 * Device memory: a matrix of at most 2^28 row-words (n_rows x
 *   ceil(2^K/64), after pruning) keeps a solve plan after its first solve:
 *   both interpretation matrices (at most 4 GiB), its row sets and a captured
 *   graph, counted in lp_info's device bytes and released by lp_matrix_evict
 *   or lp_free_matrix. Larger matrices allocate their buffers per solve.
 * Errors: LP_E_TOO_MANY_GUESSES (K > LP_MAX_NEG_ATOMS), LP_E_TRUNCATED (more
 *   than max_models models; every other output is still complete),
 *   LP_E_INVAL (interp requested with pruning), LP_E_NOMEM, LP_E_DEVICE.
 */
lp_status lp_stable_models(const lp_matrix *m, uint64_t *accepted, int64_t *n_models,
                           uint8_t *models, int64_t max_models, uint64_t *interp,
                           int32_t *products, void *hip_stream);

/*
 * Stable models of several normal programs at once (Algorithms 2 and 3 per
 * program; the columns of Algorithm 2 are independent, so programs can share
 * launches). Every launch takes one product for every program still
 * changing, over the union of their interpretation matrices, so a batch of
 * small programs costs about the launches of its longest solve. Programs with
 * more than 12 negated atoms left after pruning (over 64 words per row), and
 * definite programs, are solved one after another as lp_stable_models does.
 * Results equal lp_stable_models' with max_models = 1 for each program.
 *
 * ms:        count matrices, all on one device (host CSR and device copy).
 * accepted:  count pointers; accepted[i] is uint64[ceil(2^K_i/64)] host, as
 *            lp_stable_models' accepted.
 * n_models:  int64[count] host, the number of stable models of each program.
 * models:    nullable; count pointers, each nullable: models[i] is
 *            uint8[n_atoms_i] host and receives the first model in guess
 *            order (left unchanged if the program has none).
 * products:  nullable; int32[count], as lp_stable_models' products.
 * Synchronizes hip_stream. Errors: LP_E_INVAL (NULL ms, accepted or n_models,
 *   count < 0, matrices on different devices), LP_E_HOST_ONLY,
 *   LP_E_TOO_MANY_GUESSES, LP_E_NOMEM, LP_E_DEVICE, LP_E_INTERNAL.
 */
lp_status lp_stable_models_batch(const lp_matrix *const *ms, int32_t count, uint64_t *const *accepted,
                                 int64_t *n_models, uint8_t *const *models, int32_t *products,
                                 void *hip_stream);

/*
 * Algorithms 2 and 3 on caller-chosen guesses, for programs whose 2^K guesses
 * are too many to enumerate (1 <= K <= 64). Column j of the initial matrix
 * (Definition 8) is guesses[j]: bit t is the initial value of qbar_t, as in
 * lp_stable_models' guess order; bits at or above K are ignored.
 * guesses:    uint64[n] host, 1 <= n <= 2^30 (duplicates allowed).
 * accepted:   uint64[ceil(n/64)] host; bit j%64 of word j/64 = guess j passes
 *             Algorithm 3's test (so its column is a stable model).
 * n_accepted: receives the number of accepted entries of guesses.
 * next:       nullable; uint64[n] host, for each guess the guess its fixpoint
 *             points to: bit t set iff q_t is false in that fixpoint. An
 *             accepted guess maps to itself; lp_stable_models_search iterates
 *             this map.
 * models:     nullable; uint8[max_models][n_atoms] host, the accepted columns
 *             restricted to the original atoms, in the order of guesses.
 * products:   nullable; theta(M_P M) evaluations until no column changed.
 * Device memory: two interpretation matrices of n_rows x W words, W = the
 * next power of two >= n/64. Errors: LP_E_INVAL (K = 0, bad arguments),
 * LP_E_TOO_MANY_GUESSES (K > 64), LP_E_TRUNCATED (more accepted than
 * max_models; the other outputs are complete), LP_E_NOMEM, LP_E_DEVICE.
 */
lp_status lp_stable_models_guesses(const lp_matrix *m, const uint64_t *guesses, int64_t n,
                                   uint64_t *accepted, int64_t *n_accepted, uint64_t *next,
                                   uint8_t *models, int64_t max_models, int32_t *products,
                                   void *hip_stream);

/*
 * Stable models by guess sampling and local search (the paper's closing
 * remarks name sampling guesses for programs with many negations as future
 * work; this is one such search, sound but not complete). rounds rounds of
 * n_samples guesses through lp_stable_models_guesses: round 0 draws guess j
 * as SplitMix64 output j of the stream seeded with seed, masked to K bits;
 * in later rounds a guess that was not accepted flips each bit where it
 * disagrees with the guess its fixpoint points to with probability 1/2 (a
 * mask drawn from the stream; at least one bit), and an accepted one is
 * replaced by the next draw of the stream.
 * Every accepted guess is a stable model (Algorithm 3); models that no
 * sampled or repaired guess reaches are missed.
 * found:    uint64[max_found] host, the distinct accepted guesses, ascending
 *           (the first max_found of them).
 * n_found:  receives the number of distinct accepted guesses.
 * models:   nullable; uint8[max_found][n_atoms] host, the models of found.
 * Errors: as lp_stable_models_guesses; LP_E_TRUNCATED if more than
 *   max_found guesses were found.
 */
lp_status lp_stable_models_search(const lp_matrix *m, int64_t n_samples, int32_t rounds,
                                  uint64_t seed, uint64_t *found, int64_t max_found,
                                  int64_t *n_found, uint8_t *models, void *hip_stream);

/*
 * Least models of count definite programs (Algorithm 1 for each) in one
 * persistent launch: lp_batch_create, lp_batch_run, lp_batch_results and
 * lp_batch_free in one call. models[i]: uint8[n_atoms of ms[i]] host,
 * non-NULL; products: nullable int32[count]. sched as lp_batch_create's
 * (LP_DRIVER_FRONTIER: a frontier plan). Results equal count separate
 * lp_least_model calls. Errors as lp_least_model, for the first failing
 * program; LP_E_INVAL if the matrices live on different devices.
 */
lp_status lp_least_model_batch(const lp_matrix *const *ms, int32_t count, uint8_t *const *models,
                               int32_t *products, const lp_schedule *sched, void *hip_stream);

/*
 * Batch plans: the device side of many least-model solves, kept for repeated
 * runs. Each workgroup of the batch kernel takes programs from a device work
 * queue (largest first by stored entries) and runs a program's whole
 * fixpoint by itself, with v_t and v_{t-1} in its LDS; a run is one launch of
 * a hipGraph captured at creation, with no host round trip and no allocation.
 * Programs whose two bit-packed buffers exceed the workgroup's LDS (about
 * 600,000 matrix rows on gfx950) are solved by lp_least_model's drivers, with
 * sched, inside lp_batch_results.
 *
 * The plan holds pointers into the matrices' device layouts: the matrices
 * must outlive it. Calls on one plan must not overlap (the queue and the
 * outputs are the plan's own); distinct plans may run concurrently.
 */
typedef struct lp_batch lp_batch;

typedef struct lp_batch_info {
    int32_t count;          /* programs of the plan */
    int32_t n_resident;     /* programs solved by the batch kernel */
    int32_t wpw;            /* batch kernel shape: words per super-block */
    int32_t unroll;         /* chunks of 64 entries per round of a wave's stream */
    int32_t block;          /* threads per workgroup */
    int32_t grid;           /* workgroups (0: no resident program) */
    int64_t lds_bytes;      /* dynamic LDS per workgroup: the two buffers of the largest program */
    int64_t nnz;            /* sum of the programs' stored nonzeros */
    int64_t step_bytes;     /* sum of the programs' lp_info.step_bytes */
    float tuned_ms;         /* time per run found by lp_batch_tune, 0 before */
    int32_t n_teams;        /* programs solved by a team of workgroups */
    int32_t team_members;   /* workgroups in those teams */
    int32_t team_fallbacks; /* team programs re-solved alone by lp_batch_results since the plan was made
                               (a team whose bounded barrier gave up); 0 normally */
} lp_batch_info;

/*
 * Plan for ms[0..count) (definite programs on one device). sched (nullable):
 * wpw, unroll, block and grid select the batch kernel's shape (0: defaults,
 * grid: as many workgroups as are resident at once, at most the number of
 * queue positions); the whole schedule is used for the programs solved by the
 * single-program drivers. A program whose work exceeds a workgroup's share of
 * the batch is solved by a team of up to 8 workgroups (sched->team); every
 * team's members fit in one grid, and a team whose bounded barrier gives up
 * (its members could not run together) has its program solved alone by
 * lp_batch_results. Results and product counts do not depend on teams.
 * sched->driver == LP_DRIVER_FRONTIER makes a frontier plan instead: every
 * program (no size limit) is solved by frontier levels (the rows that became
 * true pushed through the transposed matrix, as lp_least_model's frontier
 * driver) in one launch, one workgroup per program at a time; the levels are
 * the products, so the results and product counts are those of the other
 * plans. Such a plan has no shape to tune (lp_batch_tune times it).
 * Uploads the descriptors on hip_stream and synchronizes it.
 * Errors: LP_E_NEGATION, LP_E_HOST_ONLY, LP_E_INVAL (NULL matrix, mixed
 * devices, unsupported shape, a grid smaller than a team), LP_E_NOMEM,
 * LP_E_DEVICE.
 */
lp_status lp_batch_create(const lp_matrix *const *ms, int32_t count, const lp_schedule *sched, void *hip_stream,
                          lp_batch **out);

/* Enqueue one run of the batch kernel on hip_stream (asynchronous; one graph
 * launch, nothing allocated). The results of the last run are read by
 * lp_batch_results on the same stream. */
lp_status lp_batch_run(lp_batch *b, void *hip_stream);

/*
 * Results of the last run (stream-ordered after it): models[i] (nullable
 * array, nullable entries) uint8[n_atoms of program i] host; products
 * (nullable) int32[count]. Solves the programs that are not resident first.
 * Synchronizes hip_stream. LP_E_INTERNAL if a fixpoint was not reached.
 */
lp_status lp_batch_results(const lp_batch *b, uint8_t *const *models, int32_t *products, void *hip_stream);

/*
 * Autotuner of the batch kernel. On its first call for a plan it runs the
 * batch once and lays out the queue order and the teams again by each
 * program's product count times its work per product (the plan's first
 * layout knows only the work per product). Then it times every supported
 * shape (words per super-block / chunks per round 4/4, 4/8, 4/16, 8/8, 8/16; 256,
 * 512 and 1024 threads per workgroup) over reps runs of the whole batch with
 * HIP events, keeps the fastest and captures the graph again. best_ms
 * (nullable) receives its time per run. reps = 0: the layout step and one
 * run only, at the plan's shape (best_ms 0). Results depend on neither the shape nor the
 * layout. LP_E_INVAL for reps < 0.
 */
lp_status lp_batch_tune(lp_batch *b, int32_t reps, float *best_ms, void *hip_stream);

lp_status lp_batch_get_info(const lp_batch *b, lp_batch_info *out);

/* Release the plan (NULL is accepted). Waits for the device. */
lp_status lp_batch_free(lp_batch *b);

/*
 * Average duration in milliseconds of one full-sweep T_P step (theta(M v) on
 * the whole matrix, the change count included) over reps back-to-back
 * launches on hip_stream, timed with HIP events. sched (nullable) selects the
 * step kernel as for lp_least_model. With sched->driver == LP_DRIVER_PERSISTENT
 * every launch instead runs the whole fixpoint (one persistent kernel from
 * the initial vector) and the average is per launch, i.e. per fixpoint. The step reads the fixpoint
 * of m (computed first) and writes a scratch buffer, so every launch moves the
 * same bytes. Used to measure achieved bandwidth.
 */
lp_status lp_bench_step(const lp_matrix *m, const lp_schedule *sched, int32_t reps, float *avg_ms,
                        void *hip_stream);

/*
 * Average duration in milliseconds of one stable-model step U = theta(M_P V)
 * (Algorithm 2's product over all guess columns, change count included) over
 * reps launches on hip_stream, timed with HIP events, on the fixpoint
 * interpretation matrix of m (computed first, from Definition 8's initial
 * matrix); every launch reads the same V and writes the same U. products
 * (nullable) receives the fixpoint's product count. Used to measure achieved
 * bandwidth. Errors: LP_E_INVAL for a definite program or bad arguments; as
 * lp_stable_models otherwise.
 */
lp_status lp_bench_spmm(const lp_matrix *m, int32_t reps, float *avg_ms, int32_t *products, void *hip_stream);

/*
 * The dense-matrix method that the paper's experiments (Section 4) set
 * against the sparse one: Algorithms 1 and 2 (and 3) with the program matrix
 * of Definitions 2 and 7 expanded on the device to an n' x n' byte matrix,
 * n' = lp_info.n_rows rounded up to a multiple of 1024, so that every product
 * reads all n'^2 entries. It computes the same models and the same product
 * counts as lp_least_model and lp_stable_models; it exists to measure what
 * the sparse form saves. The dense matrix is built on hip_stream at each call
 * and released before the call returns.
 *
 * lp_dense_least_model: Algorithm 1, a byte-vector product per iteration.
 *   model (uint8[n_atoms] host) and products as in lp_least_model.
 * lp_dense_stable_models: Algorithms 2 and 3 over all 2^K guesses (the guess
 *   order of lp_stable_models, with no pruning): the interpretation matrix is
 *   held as 2^K columns of n' bytes (columns padded to a multiple of 128) and
 *   each product runs on the int8 matrix cores. accepted (uint64[ceil(2^K/64)]
 *   host), n_models, models (nullable, uint8[max_models][n_atoms] host, the
 *   first max_models models in guess order) and products as in
 *   lp_stable_models. K = 0 gives the least model as the one stable model.
 * kernel_ms: nullable; receives the mean time of one product launch,
 *   measured with HIP events on hip_stream.
 * Device memory: n'^2 + 2 n' bytes, plus two interpretation matrices of
 *   (2^K rounded up to 128) x n' bytes for stable models.
 * Errors: LP_E_NEGATION (lp_dense_least_model on a program with negative
 *   literals), LP_E_TOO_MANY_GUESSES (K > LP_MAX_NEG_ATOMS), LP_E_NOMEM (the
 *   dense form does not fit in free device memory; checked before any
 *   allocation), LP_E_TRUNCATED (more models than max_models; other outputs
 *   complete), LP_E_INVAL, LP_E_HOST_ONLY, LP_E_DEVICE.
 */
lp_status lp_dense_least_model(const lp_matrix *m, uint8_t *model, int32_t *products, float *kernel_ms,
                               void *hip_stream);
lp_status lp_dense_stable_models(const lp_matrix *m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                                 int64_t max_models, int32_t *products, float *kernel_ms, void *hip_stream);

/*
 * Autotuner for least-model solves of m (a definite program). Times every
 * supported step shape (LP_STEP_LDS / LP_STEP_GLOBAL, 4 or 8 words per super-block,
 * 4/8/16 chunks in flight) over reps full-sweep steps on m's own fixpoint
 * with HIP events, then times whole solves with the batched driver and, when
 * the fastest step is shorter than 20 us (where launch overhead matters), the
 * persistent driver, at the fastest shape; writes the fastest schedule to *best.
 * best_step_ms / best_solve_ms (nullable) receive the winning times. Results
 * of lp_least_model do not depend on the schedule; only the time does.
 */
lp_status lp_tune_schedule(const lp_matrix *m, int32_t reps, lp_schedule *best, float *best_step_ms,
                           float *best_solve_ms, void *hip_stream);

/*
 * Schedule cache. lp_tune_schedule stores the schedule it returns under the
 * matrix's size bucket: whether v fits a workgroup's LDS, ceil(log2 n_rows),
 * the mean AND row length in half entries (at most 64), and whether long rows
 * exist. lp_least_model with no schedule (or an all-zero one) then solves any
 * matrix of a bucket that holds a schedule with it; results never depend on
 * the schedule. The cache is per process and thread-safe.
 *
 * lp_schedule_cache_save: writes every entry to the text file `path` (one
 *   line per bucket; written to path.tmp, then renamed).
 * lp_schedule_cache_load: merges the entries of `path` into the cache; a
 *   malformed line or an unsupported schedule rejects the whole file
 *   (LP_E_INVAL, cache unchanged).
 * lp_schedule_cache_clear: empties the cache.
 * lp_schedule_cache_lookup: *found = 1 and *out the schedule if m's bucket
 *   holds one; 0 if not; 2 if the default driver solves m in one workgroup,
 *   where no schedule applies (and for programs with negation, 0).
 * With the environment variable LP_SCHEDULE_CACHE naming a file, the library
 * loads it (if it exists) on first use of the cache and saves the cache to
 * it after every lp_tune_schedule.
 * Errors: LP_E_INVAL (NULL or empty path, unreadable or unwritable file,
 *   malformed file; NULL m, out or found), LP_E_HOST_ONLY (lookup of a matrix
 *   without a device copy).
 */
lp_status lp_schedule_cache_save(const char *path);
lp_status lp_schedule_cache_load(const char *path);
lp_status lp_schedule_cache_clear(void);
lp_status lp_schedule_cache_lookup(const lp_matrix *m, lp_schedule *out, int32_t *found);

/*
 * lp_least_model without device allocation, for callers that cannot call
 * hipMalloc or take memory from a pool at solve time (code under stream
 * capture, tight serving loops, harnesses that forbid allocation). Same
 * arguments, results and errors as lp_least_model with the default schedule
 * (sched = NULL): the model (host, uint8[n_atoms]) and the product count.
 * Every device buffer of the solve (interpretations, change counts, the
 * one-workgroup loop's descriptor) is carved from a fixed region: a
 * 4 MiB (4,194,304-byte) array in the library's device code, one copy per
 * GPU, held from the first call on that GPU until the process ends. A solve
 * needs 16 * ceil(N'/64) bytes plus about 2 KiB (N' = the matrix's rows, the
 * lp_info field n_rows), so matrices up to about 16 million rows fit; a
 * larger one returns LP_E_INVAL, with the sizes in lp_last_error, before any
 * device work. The region keeps the last call's contents; each call clears
 * what must start at zero. Calls on one GPU share the region, so calls that
 * overlap in time on one GPU (other threads, other streams) race: the caller
 * serializes them. The matrix itself is built and uploaded beforehand
 * (lp_build_matrix), which allocates as usual; nothing is attached to it by
 * this call.
 */
lp_status lp_least_model_noalloc(const lp_matrix *m, uint8_t *model, int32_t *products, void *hip_stream);

/*
 * Route the library's device allocations through caller-supplied functions
 * (e.g. a framework's caching allocator). alloc(bytes, stream, ctx) returns a
 * device pointer or NULL; release(ptr, stream, ctx) frees it. Passing NULL for
 * both restores the library's own pool. Not thread-safe with concurrent
 * solves. LP_E_INVAL when installing a hook while blocks of the library's
 * pool are in use, and when removing or replacing the installed hook while
 * blocks it allocated are live (matrices, batch plans and servers hold
 * blocks until they are freed); the hook in place is then kept.
 */
lp_status lp_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                           void (*release)(void *ptr, void *stream, void *ctx), void *ctx);

/*
 * Serving: a request loop over registered programs. Requests are least-model
 * queries (programs without negation) or stable-model queries (programs with
 * K > 0 negated atoms; the accepted mask over all 2^K guesses, the number of
 * models and the first model in guess order). n_slots worker threads, each
 * with a HIP stream of its own, take work as soon as they are free:
 *   - admission by device memory: a request starts only when its matrix (if
 *     not resident) and its solve buffers fit in hbm_budget; idle resident
 *     matrices are evicted least recently used first to make room, and a
 *     request that does not fit waits while later ones that fit go ahead;
 *   - matrices stay resident between requests;
 *   - continuous batching: a free slot takes every waiting least-model
 *     request of a matrix with at most batch_rows rows (and within the batch
 *     kernel's LDS), up to batch_max, and solves them in one batch launch;
 *     other requests run alone. Work of different slots overlaps on the device.
 * Results equal those of lp_least_model / lp_stable_models on the program.
 */
typedef struct lp_server lp_server;

typedef struct lp_server_config {
    int32_t n_slots;      /* worker threads / streams (0: 4; at most 64) */
    int32_t batch_max;    /* least-model requests per batch launch (0: 64; 1: no batching) */
    int32_t batch_rows;   /* largest matrix (rows) taken into batches (0: 65536) */
    int32_t device;       /* HIP device (-1 or 0..: -1 means the current device) */
    int64_t hbm_budget;   /* device bytes for resident matrices and running solves
                             (0: 90% of the free memory at creation) */
    int32_t tune;         /* 1: a least-model request whose matrix's size bucket holds no cached
                             schedule (see lp_schedule_cache_lookup) tunes one first
                             (lp_tune_schedule); later matrices of the bucket use it */
    int32_t reserved;
} lp_server_config;

typedef struct lp_request_info {
    int64_t request_id;
    int32_t program_id;
    int32_t kind;         /* 0: least model, 1: stable models */
    lp_status status;     /* the solve's status (LP_OK on success) */
    int32_t products;     /* fixpoint products */
    int64_t n_models;     /* 1 for a least model; the number of stable models */
    int32_t batch_size;   /* requests solved by the same launch (1: alone) */
    int32_t built;        /* 1 if the matrix was uploaded for this request */
    int64_t nnz;          /* stored nonzeros of the program matrix */
    double t_submit;      /* seconds on the server's steady clock: submitted, */
    double t_start;       /*   taken by a slot, */
    double t_done;        /*   result in host memory */
} lp_request_info;

typedef struct lp_server_stats {
    int32_t n_programs;
    int32_t n_resident;
    int64_t pending;
    int64_t completed;
    int64_t batches;            /* batch launches */
    int64_t batched_requests;   /* requests solved in them */
    int64_t alone_requests;
    int64_t uploads;            /* matrix uploads (first use and after eviction) */
    int64_t evictions;
    int64_t used_bytes;         /* accounted device bytes now */
    int64_t peak_used_bytes;
    int64_t hbm_budget;
    int64_t tunes;              /* schedules tuned for least-model requests (cfg.tune) */
} lp_server_stats;

/* cfg nullable (defaults). Errors: LP_E_INVAL, LP_E_DEVICE. */
lp_status lp_server_create(const lp_server_config *cfg, lp_server **out);

/* Register a program (arrays as for lp_build_matrix, copied; the host matrix
 * is built now, the device copy on first use). Errors: as lp_build_matrix,
 * LP_E_TOO_MANY_GUESSES, LP_E_NOMEM if it can never fit in the budget. */
lp_status lp_server_add_program(lp_server *s, int32_t n_atoms, int32_t n_rules, const int32_t *head,
                                const int64_t *body_ptr, const int32_t *body_lit, int32_t *program_id);

/* Queue a request on a registered program (thread-safe, returns at once). */
lp_status lp_server_submit(lp_server *s, int32_t program_id, int64_t *request_id);

/* Wait up to timeout_ms for a completed request not yet reported and
 * describe it; LP_E_TIMEOUT if none completed in time. Each completed
 * request is reported once, in completion order. */
lp_status lp_server_wait_any(lp_server *s, int32_t timeout_ms, lp_request_info *out);

/* Copy a completed request's result and forget it. model (nullable):
 * uint8[n_atoms], the least model or the first stable model (zeros if none);
 * accepted (nullable, stable only): uint64[ceil(2^K/64)]. */
lp_status lp_server_take_result(lp_server *s, int64_t request_id, uint8_t *model, uint64_t *accepted);

lp_status lp_server_get_stats(lp_server *s, lp_server_stats *out);

/* Stop the workers after their current work (queued requests are dropped),
 * release every resident matrix and the streams. */
lp_status lp_server_free(lp_server *s);

/*
 * The library's own device allocations go through a caching pool: hipFree
 * waits for the whole device, so blocks released by a finished call are kept
 * for reuse instead (sizes rounded up by at most 12.5%). in_use / cached
 * (nullable) receive the bytes held by live objects and by the cache, over all
 * devices. lp_release_cached_memory returns the cached blocks to the driver.
 */
lp_status lp_memory_stats(int64_t *in_use, int64_t *cached);
lp_status lp_release_cached_memory(void);

/* Message of the calling thread's last failing call ("" if none). */
const char *lp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
