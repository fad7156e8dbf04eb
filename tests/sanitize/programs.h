/* Reader of the program file written by tests/test_sanitize.py: a sequence
 * of records
 *     int32 n_atoms, int32 n_rules, int64 n_lits,
 *     int32 head[n_rules], int64 body_ptr[n_rules + 1], int32 body_lit[n_lits]
 * (little-endian, no padding). Malformed programs are stored as they are;
 * only the record framing has to be consistent. Test infrastructure only. */
#pragma once
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t n_atoms, n_rules;
    int64_t n_lits;
    int32_t *head;
    int64_t *body_ptr;
    int32_t *body_lit;
} san_program;

/* 1 on a record read, 0 at end of file, -1 on a framing error. */
static int san_read(FILE *f, san_program *p) {
    if (fread(&p->n_atoms, 4, 1, f) != 1) return 0;
    if (fread(&p->n_rules, 4, 1, f) != 1 || fread(&p->n_lits, 8, 1, f) != 1) return -1;
    if (p->n_rules < 0 || p->n_lits < 0) return -1;
    p->head = (int32_t *)malloc(4 * (size_t)(p->n_rules + 1));
    p->body_ptr = (int64_t *)malloc(8 * (size_t)(p->n_rules + 1));
    p->body_lit = (int32_t *)malloc(4 * (size_t)(p->n_lits + 1));
    if (!p->head || !p->body_ptr || !p->body_lit) return -1;
    if (fread(p->head, 4, (size_t)p->n_rules, f) != (size_t)p->n_rules) return -1;
    if (fread(p->body_ptr, 8, (size_t)p->n_rules + 1, f) != (size_t)p->n_rules + 1) return -1;
    if (fread(p->body_lit, 4, (size_t)p->n_lits, f) != (size_t)p->n_lits) return -1;
    return 1;
}

static void san_free(san_program *p) {
    free(p->head);
    free(p->body_ptr);
    free(p->body_lit);
}
