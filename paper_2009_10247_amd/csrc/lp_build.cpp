// lp_build.cpp -- host construction of the program matrix.
//
// Steps, each O(R + total body length):
//   1. validation of ids and of body_ptr;
//   2. distinct negated atoms q_0 < ... < q_{K-1} (positive form, equation 4);
//   3. standardization (Section 2.1, after Definition 1): a head with k >= 2
//      rules gets k new atoms; new atoms are numbered by a counting sort over
//      heads, so the k children of an OR row are consecutive ids;
//   4. per-rule body dedupe (bodies are sets) with 'not q_t' mapped to qbar_t;
//   5. CSR with row kinds (Definitions 2 and 7, Section 3.2).
#include <algorithm>
#include <cstring>
#include <new>

#include "lp_internal.h"

namespace lp {

namespace {

inline void small_sort(int32_t *a, int64_t n) {
    if (n > 24) {
        std::sort(a, a + n);
        return;
    }
    for (int64_t i = 1; i < n; ++i) {
        int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = x;
    }
}

}  // namespace

lp_status build_host(int32_t n_atoms, int32_t n_rules, const int32_t *head, const int64_t *body_ptr,
                     const int32_t *body_lit, uint32_t flags, Matrix *m) {
    if (n_atoms < 0 || n_rules < 0) {
        set_error("n_atoms and n_rules must be >= 0");
        return LP_E_INVAL;
    }
    if (n_rules > 0 && (!head || !body_ptr)) {
        set_error("head and body_ptr must be non-NULL when n_rules > 0");
        return LP_E_INVAL;
    }
    const int64_t L = n_rules ? body_ptr[n_rules] : 0;
    if (n_rules > 0 && body_ptr[0] != 0) {
        set_error("body_ptr[0] must be 0");
        return LP_E_INVAL;
    }
    for (int32_t r = 0; r < n_rules; ++r) {
        if (head[r] < 0 || head[r] >= n_atoms) {
            set_error("head[" + std::to_string(r) + "] out of range");
            return LP_E_INVAL;
        }
        if (body_ptr[r + 1] < body_ptr[r]) {
            set_error("body_ptr not nondecreasing at rule " + std::to_string(r));
            return LP_E_INVAL;
        }
    }
    if (L > 0 && !body_lit) {
        set_error("body_lit must be non-NULL when bodies are non-empty");
        return LP_E_INVAL;
    }
    try {
        const int32_t N = n_atoms;
        std::vector<int32_t> k(N, 0);
        std::vector<uint8_t> has_fact(N, 0);
        for (int32_t r = 0; r < n_rules; ++r) {
            k[head[r]]++;
            if (body_ptr[r + 1] == body_ptr[r]) has_fact[head[r]] = 1;
        }
        // 2. negated atoms
        std::vector<int32_t> qidx(N, -1);
        for (int64_t e = 0; e < L; ++e) {
            int32_t lit = body_lit[e];
            int64_t a = lit >= 0 ? (int64_t)lit : -(int64_t)lit - 1;
            if (a >= N) {
                set_error("body_lit[" + std::to_string(e) + "] names an atom out of range");
                return LP_E_INVAL;
            }
            if (lit < 0) qidx[a] = 0;
        }
        m->neg_atoms.clear();
        for (int32_t a = 0; a < N; ++a)
            if (qidx[a] == 0) {
                qidx[a] = (int32_t)m->neg_atoms.size();
                m->neg_atoms.push_back(a);
            }
        const int32_t K = (int32_t)m->neg_atoms.size();
        // 3. standardization: counting sort of multi-rule heads
        std::vector<int64_t> sd_base(N, -1);
        int64_t n_new = 0;
        for (int32_t a = 0; a < N; ++a)
            if (k[a] >= 2) {
                sd_base[a] = n_new;
                n_new += k[a];
            }
        const int64_t n_std64 = (int64_t)N + n_new;
        const int64_t n_rows64 = n_std64 + K;
        if (n_rows64 >= INT32_MAX) {
            set_error("matrix dimension exceeds 2^31-1");
            return LP_E_INVAL;
        }
        const int32_t n_std = (int32_t)n_std64, n_rows = (int32_t)n_rows64;
        std::vector<int32_t> rule_row(n_rules);
        std::vector<int32_t> single_rule(N, -1);
        {
            std::vector<int64_t> fill(sd_base);
            for (int32_t r = 0; r < n_rules; ++r) {
                int32_t h = head[r];
                if (k[h] >= 2)
                    rule_row[r] = (int32_t)(N + fill[h]++);
                else {
                    rule_row[r] = h;
                    single_rule[h] = r;
                }
            }
        }
        // 4. dedupe bodies (in place in a copy), negatives mapped to qbar
        std::vector<int32_t> body(L > 0 ? L : 1);
        std::vector<int32_t> dlen(n_rules);
        int64_t sum_body = 0;
        for (int32_t r = 0; r < n_rules; ++r) {
            int64_t s = body_ptr[r], e = body_ptr[r + 1];
            for (int64_t i = s; i < e; ++i) {
                int32_t lit = body_lit[i];
                body[i] = lit >= 0 ? lit : n_std + qidx[-(int64_t)lit - 1];
            }
            small_sort(body.data() + s, e - s);
            int64_t w = s;
            for (int64_t i = s; i < e; ++i)
                if (i == s || body[i] != body[w - 1]) body[w++] = body[i];
            dlen[r] = (int32_t)(w - s);
            sum_body += w - s;
        }
        // 5. CSR
        std::vector<int32_t> &rp = m->row_ptr;
        rp.assign((size_t)n_rows + 1, 0);
        m->kind.assign(n_rows, 0);
        m->fact.assign(n_rows, 0);
        int64_t acc = 0;
        // a fact row holds one entry, its own atom
        auto rule_len = [&](int32_t r) -> int64_t { return dlen[r] == 0 ? 1 : dlen[r]; };
        std::vector<int64_t> len(n_rows, 0);
        for (int32_t i = 0; i < N; ++i) {
            if (k[i] == 1) len[i] = rule_len(single_rule[i]);
            else if (k[i] >= 2) len[i] = k[i];
        }
        for (int32_t r = 0; r < n_rules; ++r)
            if (k[head[r]] >= 2) len[rule_row[r]] = rule_len(r);
        for (int32_t i = n_std; i < n_rows; ++i) len[i] = 1;
        int32_t max_len = 0;
        for (int32_t i = 0; i < n_rows; ++i) {
            rp[i] = (int32_t)acc;
            acc += len[i];
            if (acc >= INT32_MAX) {
                set_error("number of nonzeros exceeds 2^31-1");
                return LP_E_INVAL;
            }
            max_len = std::max<int32_t>(max_len, (int32_t)len[i]);
        }
        rp[n_rows] = (int32_t)acc;
        m->col.assign(acc > 0 ? acc : 0, 0);
        int32_t n_and = 0, n_or = 0, n_fact = 0, n_empty = 0;
        for (int32_t r = 0; r < n_rules; ++r) {
            int32_t row = rule_row[r];
            int32_t *dst = m->col.data() + rp[row];
            m->kind[row] = 1;
            if (dlen[r] == 0) {
                dst[0] = row;  // fact: a_ii = 1 (Definition 2, item 3)
                m->fact[row] = 1;
            } else {
                std::memcpy(dst, body.data() + body_ptr[r], sizeof(int32_t) * dlen[r]);
            }
        }
        for (int32_t a = 0; a < N; ++a) {
            if (k[a] >= 2) {
                int32_t *dst = m->col.data() + rp[a];
                for (int32_t i = 0; i < k[a]; ++i) dst[i] = (int32_t)(N + sd_base[a] + i);
                m->kind[a] = 0;
            } else if (k[a] == 0) {
                m->kind[a] = 0;  // empty OR row: never fires (Definition 2, item 4)
            }
        }
        for (int32_t t = 0; t < K; ++t) {
            int32_t row = n_std + t;
            m->col[rp[row]] = row;  // qbar rows keep their guessed value (Definition 7, items 1-2)
            m->kind[row] = 1;
        }
        for (int32_t i = 0; i < n_rows; ++i) {
            if (len[i] == 0) n_empty++;
            else if (m->fact[i]) n_fact++;
            else if (m->kind[i]) n_and++;
            else n_or++;
        }
        // guesses pruned by Definition 8, item 3
        m->guess_pos.assign(K, 0);
        int32_t keff = 0, pruned = 0;
        for (int32_t t = 0; t < K; ++t) {
            if ((flags & LP_PRUNE_FACT_GUESSES) && has_fact[m->neg_atoms[t]]) {
                m->guess_pos[t] = -1;
                pruned++;
            } else {
                m->guess_pos[t] = keff++;
            }
        }
        m->n_atoms = N;
        m->n_rules = n_rules;
        m->n_std = n_std;
        m->n_rows = n_rows;
        m->K = K;
        m->K_eff = keff;
        m->nnz = acc;
        m->flags = flags;
        lp_info &I = m->info;
        std::memset(&I, 0, sizeof I);
        I.n_atoms = N;
        I.n_rules = n_rules;
        I.n_std_atoms = n_std;
        I.n_rows = n_rows;
        I.nnz = acc;
        I.n_neg = K;
        I.n_pruned = pruned;
        I.n_and_rows = n_and;
        I.n_or_rows = n_or;
        I.n_fact_rows = n_fact;
        I.n_empty_rows = n_empty;
        I.max_row_len = max_len;
        int32_t n_long = 0;
        for (int32_t i = 0; i < n_rows; ++i)
            n_long += m->kind[i] ? (!m->fact[i] && len[i] > kLongAnd) : (len[i] > kLongOrBits);
        I.n_long_rows = n_long;
        I.sparsity = N > 0 ? 1.0 - (double)sum_body / ((double)N * (double)N) : 1.0;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while building the matrix");
        return LP_E_NOMEM;
    }
    return LP_OK;
}

}  // namespace lp
