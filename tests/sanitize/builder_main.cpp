// Sanitizer driver of the host matrix builder (csrc/lp_build.cpp: validation,
// body dedupe, standardization, positive form, CSR). Built by
// tests/test_sanitize.py with g++ -fsanitize=address,undefined; for every
// program in the file it builds the matrix without and with guess pruning and
// prints one line: status, then (on success) rows, nnz, K and pruned guesses
// of each build, and a checksum of the CSR. Test infrastructure only.
#include <cstdio>
#include <string>

#include "lp_internal.h"

extern "C" {
#include "programs.h"
}

namespace lp {
void set_error(const std::string &) {}  // the runtime's error slot is not linked into this driver
}  // namespace lp

static uint64_t checksum(const lp::Matrix &m) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
    for (int32_t x : m.row_ptr) mix((uint32_t)x);
    for (int32_t x : m.col) mix((uint32_t)x);
    for (uint8_t x : m.kind) mix(x);
    for (uint8_t x : m.fact) mix(x);
    return h;
}

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    san_program p;
    int r;
    while ((r = san_read(f, &p)) == 1) {
        for (uint32_t flags : {0u, (uint32_t)LP_PRUNE_FACT_GUESSES}) {
            lp::Matrix m;
            const lp_status rc = lp::build_host(p.n_atoms, p.n_rules, p.head, p.body_ptr, p.body_lit, flags, &m);
            if (rc) {
                std::printf("%d ", (int)rc);
            } else {
                std::printf("%d %d %lld %d %d %llu ", (int)rc, m.n_rows, (long long)m.nnz, m.K, m.info.n_pruned,
                            (unsigned long long)checksum(m));
            }
        }
        std::printf("\n");
        san_free(&p);
    }
    std::fclose(f);
    return r < 0 ? 3 : 0;
}
