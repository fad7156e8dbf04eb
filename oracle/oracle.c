/*
 * oracle.c -- plain CPU oracle for least models and stable models.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the engine links, loads or calls this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it. It shares no code, header or table with the engine.
 *
 * What it computes, and from which passage of the paper:
 *
 *  O1 orc_least_model  -- the least model LM(P) of a definite program, i.e.
 *     the least fixpoint of the T_P operator (Section 2.1, the T_P definition
 *     and the van Emden-Kowalski result quoted after it). Algorithm: the
 *     linear-time forward chaining of Dowling and Gallier (1984): every rule
 *     keeps a count of body atoms not yet known true; an atom that becomes
 *     true decrements the counts of the rules it occurs in, and a rule whose
 *     count reaches zero makes its head true. Runs on the program as given,
 *     with no standardization and no matrix.
 *
 *  O2 orc_sd_fixpoint  -- the number of synchronous T_P applications the
 *     paper's Algorithm 1 performs. The program is first standardized into a
 *     singly-defined program plus OR-rules (Section 2.1, the paragraph after
 *     Definition 1; Algorithm 1, step 1) by this file's own rewrite. Then
 *     stage(a) = the first synchronous step at which atom a is true: facts
 *     have stage 0, an AND rule gives 1 + max of its body stages, an OR rule
 *     1 + min over its true children (layered forward chaining). Algorithm 1
 *     evaluates theta(M v) once per step plus once more to see that nothing
 *     changed, so products = 1 + max stage.
 *
 *  O3 orc_stable       -- stable models through the positive form (Section
 *     2.2, equation 4 and the Alferes et al. equivalence stated after it):
 *     for each guess j on the K negated atoms q_0 < ... < q_{K-1}, the guess
 *     G_j = { qbar_t : bit t of j is 1 } is added as facts, the least model
 *     L_j of P+ u G_j is taken (O1), and j is accepted iff for every t exactly
 *     one of q_t, qbar_t is in L_j (Algorithm 3's test a_l + a_j = 1). The
 *     model is L_j restricted to the original atoms. The per-guess synchronous
 *     step count (O2 on the standardized P+ with the guess) gives the number
 *     of matrix products of Algorithm 2 (max over guesses).
 *
 *  O4 orc_gl_check     -- the textbook Gelfond-Lifschitz test of a candidate I:
 *     the reduct P^I keeps h <- pos(r) for every rule r with neg(r) disjoint
 *     from I; I is stable iff LM(P^I) = I (computed with O1).
 *
 * Program layout (as in the engine's C-ABI): head[R], body_ptr[R+1] (int64,
 * body_ptr[0] = 0, nondecreasing), body_lit[...] with a >= 0 meaning atom a
 * and a < 0 meaning "not atom (-a-1)". Bodies are sets (the paper's footnote
 * to the definition of head/body), so repeated literals are merged.
 *
 * Return codes: 0 ok, -1 malformed input, -2 out of memory, -4 negation in a
 * definite-only call, -7 internal disagreement between O1 and O2.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_NEGATION (-4)
#define ORC_E_INTERNAL (-7)

/* A rule set over atoms [0, n_atoms): AND rules (fire when every body atom is
 * true) and OR rules (fire when some body atom is true). Bodies are deduped. */
typedef struct {
    int32_t n_atoms;
    int32_t n_rules;
    int32_t *head;
    int64_t *ptr;
    int32_t *body;
    uint8_t *is_or;
    /* occurrence index: rules containing atom a are occ[occ_ptr[a]..occ_ptr[a+1]) */
    int64_t *occ_ptr;
    int32_t *occ;
} ruleset;

static void rs_free(ruleset *r) {
    free(r->head); free(r->ptr); free(r->body); free(r->is_or);
    free(r->occ_ptr); free(r->occ);
    memset(r, 0, sizeof *r);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int validate(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                    const int64_t *body_ptr, const int32_t *body_lit) {
    if (n_atoms < 0 || n_rules < 0) return ORC_E_INVAL;
    if (n_rules > 0 && (!head || !body_ptr)) return ORC_E_INVAL;
    if (n_rules == 0) return ORC_OK;
    if (body_ptr[0] != 0) return ORC_E_INVAL;
    for (int32_t r = 0; r < n_rules; ++r) {
        if (head[r] < 0 || head[r] >= n_atoms) return ORC_E_INVAL;
        if (body_ptr[r + 1] < body_ptr[r]) return ORC_E_INVAL;
    }
    if (body_ptr[n_rules] > 0 && !body_lit) return ORC_E_INVAL;
    for (int64_t e = 0; e < body_ptr[n_rules]; ++e) {
        int64_t a = body_lit[e] >= 0 ? body_lit[e] : -(int64_t)body_lit[e] - 1;
        if (a >= n_atoms) return ORC_E_INVAL;
    }
    return ORC_OK;
}

/* Distinct negated atoms, ascending. Returns count; fills map[atom] = t or -1. */
static int32_t negated_atoms(int32_t n_atoms, int32_t n_rules, const int64_t *body_ptr,
                             const int32_t *body_lit, int32_t *map, int32_t *list) {
    for (int32_t a = 0; a < n_atoms; ++a) map[a] = -1;
    int64_t L = n_rules ? body_ptr[n_rules] : 0;
    for (int64_t e = 0; e < L; ++e)
        if (body_lit[e] < 0) map[-(int64_t)body_lit[e] - 1] = 1;
    int32_t k = 0;
    for (int32_t a = 0; a < n_atoms; ++a)
        if (map[a] == 1) { if (list) list[k] = a; map[a] = k++; }
    return k;
}

/* Build the positive form P+ (equation 4): 'not q_t' becomes atom n_atoms + t.
 * With neg_map == NULL the program must be definite. Bodies are deduped. */
static int make_ruleset(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                        const int64_t *body_ptr, const int32_t *body_lit,
                        const int32_t *neg_map, int32_t k, ruleset *out) {
    memset(out, 0, sizeof *out);
    out->n_atoms = n_atoms + k;
    out->n_rules = n_rules;
    int64_t L = n_rules ? body_ptr[n_rules] : 0;
    out->head = malloc(sizeof(int32_t) * (n_rules ? n_rules : 1));
    out->ptr = malloc(sizeof(int64_t) * (n_rules + 1));
    out->body = malloc(sizeof(int32_t) * (L ? L : 1));
    out->is_or = calloc(n_rules ? n_rules : 1, 1);
    if (!out->head || !out->ptr || !out->body || !out->is_or) { rs_free(out); return ORC_E_NOMEM; }
    int64_t w = 0;
    out->ptr[0] = 0;
    for (int32_t r = 0; r < n_rules; ++r) {
        out->head[r] = head[r];
        int64_t s = w;
        for (int64_t e = body_ptr[r]; e < body_ptr[r + 1]; ++e) {
            int32_t lit = body_lit[e];
            int32_t atom;
            if (lit >= 0) atom = lit;
            else {
                if (!neg_map) { rs_free(out); return ORC_E_NEGATION; }
                atom = n_atoms + neg_map[-(int64_t)lit - 1];
            }
            out->body[w++] = atom;
        }
        qsort(out->body + s, (size_t)(w - s), sizeof(int32_t), cmp_i32);
        int64_t u = s;
        for (int64_t e = s; e < w; ++e)
            if (e == s || out->body[e] != out->body[u - 1]) out->body[u++] = out->body[e];
        w = u;
        out->ptr[r + 1] = w;
    }
    return ORC_OK;
}

static int build_occ(ruleset *rs) {
    int32_t n = rs->n_atoms;
    int64_t L = rs->ptr[rs->n_rules];
    rs->occ_ptr = calloc((size_t)n + 1, sizeof(int64_t));
    rs->occ = malloc(sizeof(int32_t) * (L ? L : 1));
    if (!rs->occ_ptr || !rs->occ) return ORC_E_NOMEM;
    for (int64_t e = 0; e < L; ++e) rs->occ_ptr[rs->body[e] + 1]++;
    for (int32_t a = 0; a < n; ++a) rs->occ_ptr[a + 1] += rs->occ_ptr[a];
    int64_t *fill = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fill) return ORC_E_NOMEM;
    memcpy(fill, rs->occ_ptr, sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t r = 0; r < rs->n_rules; ++r)
        for (int64_t e = rs->ptr[r]; e < rs->ptr[r + 1]; ++e) rs->occ[fill[rs->body[e]]++] = r;
    free(fill);
    return ORC_OK;
}

/* Per-thread scratch for the chaining routines. */
typedef struct {
    int32_t *cnt;     /* [n_rules] */
    int32_t *queue;   /* [n_atoms] */
    int32_t *stage;   /* [n_atoms] */
    uint8_t *truth;   /* [n_atoms] */
} scratch;

static int scratch_init(scratch *s, const ruleset *rs) {
    s->cnt = malloc(sizeof(int32_t) * (rs->n_rules ? rs->n_rules : 1));
    s->queue = malloc(sizeof(int32_t) * (rs->n_atoms ? rs->n_atoms : 1));
    s->stage = malloc(sizeof(int32_t) * (rs->n_atoms ? rs->n_atoms : 1));
    s->truth = malloc(rs->n_atoms ? rs->n_atoms : 1);
    return (s->cnt && s->queue && s->stage && s->truth) ? ORC_OK : ORC_E_NOMEM;
}

static void scratch_free(scratch *s) { free(s->cnt); free(s->queue); free(s->stage); free(s->truth); }

/* O1: Dowling-Gallier forward chaining over AND rules (OR rules fire on their
 * first true child). extra_true: atoms given as facts (nullable). */
static void forward_chain(const ruleset *rs, const int32_t *extra, int32_t n_extra, scratch *s) {
    int32_t qh = 0, qt = 0;
    memset(s->truth, 0, (size_t)rs->n_atoms);
    for (int32_t r = 0; r < rs->n_rules; ++r) {
        int32_t len = (int32_t)(rs->ptr[r + 1] - rs->ptr[r]);
        s->cnt[r] = rs->is_or[r] ? 1 : len;
        if (len == 0 && !rs->is_or[r] && !s->truth[rs->head[r]]) {
            s->truth[rs->head[r]] = 1;
            s->queue[qt++] = rs->head[r];
        }
    }
    for (int32_t i = 0; i < n_extra; ++i)
        if (!s->truth[extra[i]]) { s->truth[extra[i]] = 1; s->queue[qt++] = extra[i]; }
    while (qh < qt) {
        int32_t a = s->queue[qh++];
        for (int64_t o = rs->occ_ptr[a]; o < rs->occ_ptr[a + 1]; ++o) {
            int32_t r = rs->occ[o];
            if (--s->cnt[r] == 0) {
                int32_t h = rs->head[r];
                if (!s->truth[h]) { s->truth[h] = 1; s->queue[qt++] = h; }
            }
        }
    }
}

/* O2: synchronous stages by layered chaining. Returns the max finite stage
 * (0 when only facts/extras are true, -1 when nothing is true). */
static int32_t layered_stages(const ruleset *rs, const int32_t *extra, int32_t n_extra, scratch *s) {
    const int32_t INF = INT32_MAX;
    for (int32_t a = 0; a < rs->n_atoms; ++a) s->stage[a] = INF;
    int32_t qt = 0;
    for (int32_t r = 0; r < rs->n_rules; ++r) {
        int32_t len = (int32_t)(rs->ptr[r + 1] - rs->ptr[r]);
        s->cnt[r] = rs->is_or[r] ? 1 : len;
        if (len == 0 && !rs->is_or[r] && s->stage[rs->head[r]] == INF) {
            s->stage[rs->head[r]] = 0;
            s->queue[qt++] = rs->head[r];
        }
    }
    for (int32_t i = 0; i < n_extra; ++i)
        if (s->stage[extra[i]] == INF) { s->stage[extra[i]] = 0; s->queue[qt++] = extra[i]; }
    int32_t maxst = qt ? 0 : -1;
    int32_t layer_begin = 0, t = 0;
    while (layer_begin < qt) {
        int32_t layer_end = qt;
        for (int32_t qi = layer_begin; qi < layer_end; ++qi) {
            int32_t a = s->queue[qi];
            for (int64_t o = rs->occ_ptr[a]; o < rs->occ_ptr[a + 1]; ++o) {
                int32_t r = rs->occ[o];
                if (--s->cnt[r] == 0) {
                    int32_t h = rs->head[r];
                    if (s->stage[h] == INF) { s->stage[h] = t + 1; s->queue[qt++] = h; maxst = t + 1; }
                }
            }
        }
        layer_begin = layer_end;
        ++t;
    }
    for (int32_t a = 0; a < rs->n_atoms; ++a) s->truth[a] = s->stage[a] != INF;
    return maxst;
}

/* Standardization (Section 2.1): every head with k >= 2 rules gets k new atoms
 * b_1..b_k, rules b_i <- body(r_i), and one OR rule h <- b_1 v ... v b_k.
 * This oracle numbers new atoms n_atoms, n_atoms+1, ... in rule-index order. */
static int sd_rewrite(const ruleset *in, ruleset *out) {
    memset(out, 0, sizeof *out);
    int32_t n = in->n_atoms, R = in->n_rules;
    int32_t *k = calloc((size_t)n + 1, sizeof(int32_t));
    if (!k) return ORC_E_NOMEM;
    for (int32_t r = 0; r < R; ++r) k[in->head[r]]++;
    int64_t n_new = 0, n_or = 0;
    for (int32_t a = 0; a < n; ++a) if (k[a] >= 2) { n_new += k[a]; n_or++; }
    if ((int64_t)n + n_new > INT32_MAX) { free(k); return ORC_E_INVAL; }
    int32_t R2 = (int32_t)(R + n_or);
    int64_t L2 = in->ptr[R] + n_new;
    out->n_atoms = (int32_t)(n + n_new);
    out->n_rules = R2;
    out->head = malloc(sizeof(int32_t) * (R2 ? R2 : 1));
    out->ptr = malloc(sizeof(int64_t) * (R2 + 1));
    out->body = malloc(sizeof(int32_t) * (L2 ? L2 : 1));
    out->is_or = calloc(R2 ? R2 : 1, 1);
    /* children of each OR head, collected in rule order */
    int64_t *or_start = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *or_child = malloc(sizeof(int32_t) * (n_new ? n_new : 1));
    int64_t *or_fill = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!out->head || !out->ptr || !out->body || !out->is_or || !or_start || !or_child || !or_fill) {
        free(k); free(or_start); free(or_child); free(or_fill); rs_free(out); return ORC_E_NOMEM;
    }
    int64_t acc = 0;
    for (int32_t a = 0; a < n; ++a) { or_start[a] = acc; or_fill[a] = acc; if (k[a] >= 2) acc += k[a]; }
    int32_t next_new = n;
    int64_t w = 0;
    out->ptr[0] = 0;
    for (int32_t r = 0; r < R; ++r) {
        int32_t h = in->head[r];
        int32_t nh = h;
        if (k[h] >= 2) { nh = next_new++; or_child[or_fill[h]++] = nh; }
        out->head[r] = nh;
        for (int64_t e = in->ptr[r]; e < in->ptr[r + 1]; ++e) out->body[w++] = in->body[e];
        out->ptr[r + 1] = w;
    }
    int32_t ri = R;
    for (int32_t a = 0; a < n; ++a) {
        if (k[a] < 2) continue;
        out->head[ri] = a;
        out->is_or[ri] = 1;
        for (int64_t c = or_start[a]; c < or_start[a] + k[a]; ++c) out->body[w++] = or_child[c];
        out->ptr[ri + 1] = w;
        ++ri;
    }
    free(k); free(or_start); free(or_child); free(or_fill);
    return ORC_OK;
}

/* ---------------------------------------------------------------- exports */

int orc_negated_atoms(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                      const int64_t *body_ptr, const int32_t *body_lit, int32_t *out, int32_t *k) {
    int rc = validate(n_atoms, n_rules, head, body_ptr, body_lit);
    if (rc) return rc;
    int32_t *map = malloc(sizeof(int32_t) * (n_atoms ? n_atoms : 1));
    if (!map) return ORC_E_NOMEM;
    *k = negated_atoms(n_atoms, n_rules, body_ptr, body_lit, map, out);
    free(map);
    return ORC_OK;
}

/* O1. model[n_atoms] receives 0/1. */
int orc_least_model(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                    const int64_t *body_ptr, const int32_t *body_lit, uint8_t *model) {
    int rc = validate(n_atoms, n_rules, head, body_ptr, body_lit);
    if (rc) return rc;
    ruleset rs;
    rc = make_ruleset(n_atoms, n_rules, head, body_ptr, body_lit, NULL, 0, &rs);
    if (rc) return rc;
    scratch s = {0};
    if ((rc = build_occ(&rs)) || (rc = scratch_init(&s, &rs))) { rs_free(&rs); scratch_free(&s); return rc ? rc : ORC_E_NOMEM; }
    forward_chain(&rs, NULL, 0, &s);
    memcpy(model, s.truth, (size_t)n_atoms);
    scratch_free(&s);
    rs_free(&rs);
    return ORC_OK;
}

/* O2. model[n_atoms]: LM(P^delta) restricted to the original atoms;
 * products: 1 + max stage; n_std_atoms: |B_{P^delta}|; n_true_std: |LM(P^delta)|.
 * Checks LM(P^delta) restricted to B_P against O1 and returns -7 on mismatch. */
int orc_sd_fixpoint(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                    const int64_t *body_ptr, const int32_t *body_lit, uint8_t *model,
                    int32_t *products, int32_t *n_std_atoms, int64_t *n_true_std) {
    int rc = validate(n_atoms, n_rules, head, body_ptr, body_lit);
    if (rc) return rc;
    ruleset p, sd;
    rc = make_ruleset(n_atoms, n_rules, head, body_ptr, body_lit, NULL, 0, &p);
    if (rc) return rc;
    rc = sd_rewrite(&p, &sd);
    if (rc) { rs_free(&p); return rc; }
    scratch s1 = {0}, s2 = {0};
    if ((rc = build_occ(&p)) || (rc = build_occ(&sd)) || (rc = scratch_init(&s1, &p)) ||
        (rc = scratch_init(&s2, &sd))) goto done;
    forward_chain(&p, NULL, 0, &s1);
    int32_t maxst = layered_stages(&sd, NULL, 0, &s2);
    int64_t cnt = 0;
    for (int32_t a = 0; a < sd.n_atoms; ++a) cnt += s2.truth[a];
    for (int32_t a = 0; a < n_atoms; ++a)
        if (s1.truth[a] != s2.truth[a]) { rc = ORC_E_INTERNAL; goto done; }
    memcpy(model, s2.truth, (size_t)n_atoms);
    if (products) *products = 1 + (maxst > 0 ? maxst : 0);
    if (n_std_atoms) *n_std_atoms = sd.n_atoms;
    if (n_true_std) *n_true_std = cnt;
done:
    scratch_free(&s1); scratch_free(&s2);
    rs_free(&p); rs_free(&sd);
    return rc;
}

/* O3. Guesses j in [guess_begin, guess_begin + guess_count), j < 2^K.
 * accept[guess_count]: 1 iff guess j passes the consistency test.
 * interp (nullable): [n_atoms][W], W = ceil(guess_count/64); bit (j-begin)%64
 *   of word (j-begin)/64 of row a is 1 iff a is in L_j.
 * products (nullable): max over the guesses of 1 + max stage on the
 *   standardized P+ with the guess added.
 * Checks the standardized fixpoint against O1 on P+ per guess (-7 on mismatch). */
int orc_stable(int32_t n_atoms, int32_t n_rules, const int32_t *head,
               const int64_t *body_ptr, const int32_t *body_lit,
               int64_t guess_begin, int64_t guess_count, int32_t n_threads,
               uint8_t *accept, uint64_t *interp, int32_t *products) {
    int rc = validate(n_atoms, n_rules, head, body_ptr, body_lit);
    if (rc) return rc;
    if (guess_begin < 0 || guess_count < 0) return ORC_E_INVAL;
    int32_t *map = malloc(sizeof(int32_t) * (n_atoms ? n_atoms : 1));
    int32_t *qlist = malloc(sizeof(int32_t) * (n_atoms ? n_atoms : 1));
    if (!map || !qlist) { free(map); free(qlist); return ORC_E_NOMEM; }
    int32_t K = negated_atoms(n_atoms, n_rules, body_ptr, body_lit, map, qlist);
    if (K > 30 || guess_begin + guess_count > ((int64_t)1 << K)) { free(map); free(qlist); return ORC_E_INVAL; }
    ruleset pp, sd;
    rc = make_ruleset(n_atoms, n_rules, head, body_ptr, body_lit, map, K, &pp);
    if (rc) { free(map); free(qlist); return rc; }
    rc = sd_rewrite(&pp, &sd);
    if (rc) { rs_free(&pp); free(map); free(qlist); return rc; }
    if ((rc = build_occ(&pp)) || (rc = build_occ(&sd))) goto out;
    int64_t W = (guess_count + 63) / 64;
    if (interp) memset(interp, 0, sizeof(uint64_t) * (size_t)n_atoms * (size_t)W);
    int32_t maxprod = 1;
    int err = ORC_OK;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
        scratch s1 = {0}, s2 = {0};
        int32_t *extra = malloc(sizeof(int32_t) * (K ? K : 1));
        int ok = extra && scratch_init(&s1, &pp) == ORC_OK && scratch_init(&s2, &sd) == ORC_OK;
        int32_t local_max = 1;
        /* one 64-guess word per iteration, so each thread owns whole interp words */
#pragma omp for schedule(dynamic)
        for (int64_t w = 0; w < W; ++w) {
            if (!ok) continue;
            for (int64_t b = 0; b < 64 && w * 64 + b < guess_count; ++b) {
                int64_t idx = w * 64 + b;
                int64_t j = guess_begin + idx;
                int32_t ne = 0;
                for (int32_t t = 0; t < K; ++t)
                    if ((j >> t) & 1) extra[ne++] = n_atoms + t;
                forward_chain(&pp, extra, ne, &s1);
                int32_t maxst = layered_stages(&sd, extra, ne, &s2);
                int bad = 0;
                for (int32_t a = 0; a < pp.n_atoms; ++a) bad |= s1.truth[a] != s2.truth[a];
                if (bad) {
#pragma omp critical
                    err = ORC_E_INTERNAL;
                }
                int32_t prod = 1 + (maxst > 0 ? maxst : 0);
                if (prod > local_max) local_max = prod;
                int acc = 1;
                for (int32_t t = 0; t < K; ++t)
                    if (s1.truth[qlist[t]] == s1.truth[n_atoms + t]) { acc = 0; break; }
                accept[idx] = (uint8_t)acc;
                if (interp)
                    for (int32_t a = 0; a < n_atoms; ++a)
                        if (s1.truth[a]) interp[(size_t)a * (size_t)W + (size_t)w] |= (uint64_t)1 << b;
            }
        }
        if (!ok) {
#pragma omp critical
            err = ORC_E_NOMEM;
        }
#pragma omp critical
        if (local_max > maxprod) maxprod = local_max;
        free(extra);
        scratch_free(&s1); scratch_free(&s2);
    }
    rc = err;
    if (products) *products = maxprod;
out:
    rs_free(&pp); rs_free(&sd);
    free(map); free(qlist);
    return rc;
}

/* O4. Returns 1 if interp (0/1 per atom) is a stable model, 0 if not, <0 on error. */
int orc_gl_check(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                 const int64_t *body_ptr, const int32_t *body_lit, const uint8_t *interp) {
    int rc = validate(n_atoms, n_rules, head, body_ptr, body_lit);
    if (rc) return rc;
    /* reduct P^I: drop rules with a negative literal true in I, strip the rest */
    int64_t L = n_rules ? body_ptr[n_rules] : 0;
    int32_t *h2 = malloc(sizeof(int32_t) * (n_rules ? n_rules : 1));
    int64_t *p2 = malloc(sizeof(int64_t) * ((size_t)n_rules + 1));
    int32_t *b2 = malloc(sizeof(int32_t) * (L ? L : 1));
    if (!h2 || !p2 || !b2) { free(h2); free(p2); free(b2); return ORC_E_NOMEM; }
    int32_t R2 = 0;
    int64_t w = 0;
    p2[0] = 0;
    for (int32_t r = 0; r < n_rules; ++r) {
        int blocked = 0;
        for (int64_t e = body_ptr[r]; e < body_ptr[r + 1]; ++e)
            if (body_lit[e] < 0 && interp[-(int64_t)body_lit[e] - 1]) { blocked = 1; break; }
        if (blocked) continue;
        for (int64_t e = body_ptr[r]; e < body_ptr[r + 1]; ++e)
            if (body_lit[e] >= 0) b2[w++] = body_lit[e];
        h2[R2++] = head[r];
        p2[R2] = w;
    }
    uint8_t *lm = malloc(n_atoms ? n_atoms : 1);
    rc = lm ? orc_least_model(n_atoms, R2, h2, p2, b2, lm) : ORC_E_NOMEM;
    int res = rc;
    if (rc == ORC_OK) {
        res = 1;
        for (int32_t a = 0; a < n_atoms; ++a)
            if ((lm[a] != 0) != (interp[a] != 0)) { res = 0; break; }
    }
    free(lm); free(h2); free(p2); free(b2);
    return res;
}
