/* Sanitizer driver of the CPU oracle (oracle/oracle.c). Built by
 * tests/test_sanitize.py with gcc -fsanitize=address,undefined; for every
 * program in the file it prints one line: the negated-atom count, then for a
 * definite program the least-model status, its size, the synchronous
 * status and product count; for a normal program the stable-model status,
 * the number of accepted guesses, the product count and the Gelfond-Lifschitz
 * verdict of every accepted model. Malformed programs print their status.
 * Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "programs.h"

int orc_negated_atoms(int32_t, int32_t, const int32_t *, const int64_t *, const int32_t *, int32_t *, int32_t *);
int orc_least_model(int32_t, int32_t, const int32_t *, const int64_t *, const int32_t *, uint8_t *);
int orc_sd_fixpoint(int32_t, int32_t, const int32_t *, const int64_t *, const int32_t *, uint8_t *, int32_t *,
                    int32_t *, int64_t *);
int orc_stable(int32_t, int32_t, const int32_t *, const int64_t *, const int32_t *, int64_t, int64_t, int32_t,
               uint8_t *, uint64_t *, int32_t *);
int orc_gl_check(int32_t, int32_t, const int32_t *, const int64_t *, const int32_t *, const uint8_t *);

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    san_program p;
    int r;
    while ((r = san_read(f, &p)) == 1) {
        const int32_t n = p.n_atoms > 0 ? p.n_atoms : 1;
        int32_t *neg = malloc(sizeof(int32_t) * (size_t)n);
        int32_t K = 0;
        int rc = orc_negated_atoms(p.n_atoms, p.n_rules, p.head, p.body_ptr, p.body_lit, neg, &K);
        if (rc) {
            printf("%d\n", rc);
        } else if (K == 0) {
            uint8_t *lm = calloc((size_t)n, 1), *sd = calloc((size_t)n, 1);
            int32_t prods = 0, nstd = 0;
            int64_t ntrue = 0, size = 0;
            int rc1 = orc_least_model(p.n_atoms, p.n_rules, p.head, p.body_ptr, p.body_lit, lm);
            int rc2 = orc_sd_fixpoint(p.n_atoms, p.n_rules, p.head, p.body_ptr, p.body_lit, sd, &prods, &nstd,
                                      &ntrue);
            for (int32_t a = 0; a < p.n_atoms; ++a) size += lm[a];
            printf("0 %d %lld %d %d\n", rc1, (long long)size, rc2, prods);
            free(lm);
            free(sd);
        } else if (K <= 16) {
            const int64_t H = (int64_t)1 << K, W = (H + 63) / 64;
            uint8_t *acc = calloc((size_t)H, 1);
            uint64_t *interp = calloc((size_t)n * (size_t)W, 8);
            uint8_t *model = calloc((size_t)n, 1);
            int32_t prods = 0;
            int rc1 = orc_stable(p.n_atoms, p.n_rules, p.head, p.body_ptr, p.body_lit, 0, H, 1, acc, interp, &prods);
            int64_t n_acc = 0, n_gl = 0;
            for (int64_t j = 0; rc1 == 0 && j < H; ++j) {
                if (!acc[j]) continue;
                ++n_acc;
                for (int32_t a = 0; a < p.n_atoms; ++a) model[a] = (interp[(size_t)a * W + j / 64] >> (j % 64)) & 1;
                n_gl += orc_gl_check(p.n_atoms, p.n_rules, p.head, p.body_ptr, p.body_lit, model) == 1;
            }
            printf("%d %d %lld %d %lld\n", K, rc1, (long long)n_acc, prods, (long long)n_gl);
            free(acc);
            free(interp);
            free(model);
        } else {
            printf("%d skipped\n", K);
        }
        free(neg);
        san_free(&p);
    }
    fclose(f);
    return r < 0 ? 3 : 0;
}
