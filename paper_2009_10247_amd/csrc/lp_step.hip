// lp_step.hip -- the least-model T_P step u = theta(M v) on gfx950.
//
// Interpretations are bit-packed: bit (i & 63) of word (i >> 6) is row i.
// theta (Definition 5) is evaluated exactly on the row kinds: an AND row fires
// iff every entry it names is 1 in v, an OR row iff at least one child is.
//
// Monotonicity: from the initial vector, v_t is a subset of v_{t+1}. The step
// ORs its result into the buffer holding v_{t-1} (a subset of the exact
// result), so several waves may contribute bits of one word with atomicOr, no
// clearing pass is needed, and fact rows (true in v_0) need no work at all.
// popcount(u & ~v) counts the new atoms; the fixpoint of Algorithm 1 is the
// first product whose count is 0.
//
// Layout (see WordMeta): per 64-row word the offset of its first AND entry,
// the index of its first OR row and the row-kind bits; per row an 8-bit AND
// length. The AND entries of a word's rows are consecutive in col, and those
// of consecutive words follow each other, so a wave that owns WPW words (a
// super-block) streams one contiguous stretch of col. OR rows store no
// entries: the children of an OR row are consecutive new atoms, so the row is
// the bit range [or_c0[i], or_c0[i+1]) of v.
//
// AND rows: the wave streams its stretch of col 64 entries (256 bytes,
// coalesced) per chunk with U chunks in flight, each lane gathers the v bit of
// its entry, and a 64-bit ballot per chunk is written to the wave's LDS slots;
// each row-owner lane then folds the one or two chunks its row overlaps. With
// LDS staging, the leading words of v (the original atoms, the only atoms AND
// bodies name) are copied into LDS per workgroup, so the gathers are ds_reads.
// OR rows are separate items, 64 per wave, one lane per row ORing the words
// of its bit range. Rows longer than kLongAnd entries or kLongOrBits children
// are evaluated by segments, one wave per segment.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "lp_dev.h"
#include "lp_kernels.h"

namespace lp {

namespace {

template <bool LDS>
__device__ __forceinline__ uint64_t vword(const StepParams &p, const lds_u32 *s_v, int64_t word) {
    if (LDS && word < p.lds_words) return ((const lds_u64 *)s_v)[word];
    return p.v[word];
}

// Row data of one super-block (WPW words of 64 rows from word sbw, a
// multiple of 4), loaded with vector loads only (scalar loads would share the
// lgkm counter with the LDS gathers, so every LDS wait would also wait for
// this prefetch): this lane's AND length in each word, four words per dword
// (lens4 stores them so), the first AND entry of the super-block's first word
// in the wave's range (the same in every lane) and the v words.
template <int WPW>
struct SbMeta {
    uint32_t lens[WPW / 4];
    int32_t b0;
    uint64_t vw;  // lane w < WPW: word w of the super-block in v (for the new-bit count)
    uint64_t pw;  // sliced passes, lane w < WPW: word w of and_all (pass 0) or of pacc (later passes)
};

template <int WPW, bool SLICE = false>
__device__ __forceinline__ void load_sb_meta(const StepParams &p, int32_t sbw, int32_t w_begin, int32_t n_words,
                                             SbMeta<WPW> &m) {
    // lens4 and words carry kWordPad empty words after the end, so every
    // super-block that starts before the last word loads in bounds
    const int lane = threadIdx.x & 63;
    const int64_t q0 = sbw >> 2;
#pragma unroll
    for (int k = 0; k < WPW / 4; ++k) m.lens[k] = p.lens4[(q0 + k) * 64 + lane];
    m.b0 = p.words[sbw > w_begin ? sbw : w_begin].and_base;
    const int32_t wv = sbw + (lane < WPW ? lane : WPW - 1);
    m.vw = p.v[wv < n_words ? wv : n_words - 1];
    if (SLICE) m.pw = (p.pass == 0 ? p.and_all : (const uint64_t *)p.pacc)[wv < n_words ? wv : n_words - 1];
}

template <int WPW>
__device__ __forceinline__ int32_t lane_len(const uint32_t (&lens)[WPW / 4], int w) {
    return (int32_t)((lens[w >> 2] >> ((w & 3) * 8)) & 0xffu);
}

// Loads the U chunks of 64 entries starting at entry base (a multiple of 64):
// col[base + 64 u + lane]. In bounds: base + 64 U is at most the number of
// entries rounded up to 64, or a small wave's first chunk + 64 U, and col
// carries kColPad zero entries after its end.
template <int U>
__device__ __forceinline__ void load_chunks(const StepParams &p, int32_t base, int32_t (&c)[U]) {
    const int32_t *cb = p.col + base;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = cb[64 * u + lane];
}

// State of the super-block being evaluated: each lane's first entry per
// word, the words' entry ranges (wave-uniform: word w covers [ws[w],
// ws[w + 1])) and this lane's AND results, one bit per word.
template <int WPW>
struct SbState {
    int32_t st[WPW];
    int32_t ws[WPW + 1];
    uint32_t lens[WPW / 4];
    uint32_t accm;
    uint64_t vw;
    uint64_t pw;
};

// Row starts from the 8-bit lengths of the words in [w_begin, w_end) (the
// others are masked to length 0: they belong to another wave). The lengths
// of words 4k and 4k + 2 (and of 4k + 1 and 4k + 3) are scanned together as
// the two 16-bit halves of one 32-bit DPP wave scan: a half's sum is at most
// 64 x 255 < 2^16, so no carry crosses between them. Two scans per four words.
template <int WPW>
__device__ __forceinline__ void sb_setup(const SbMeta<WPW> &m, int32_t sbw, int32_t w_begin, int32_t w_end,
                                         SbState<WPW> &S) {
    int32_t run = __builtin_amdgcn_readfirstlane(m.b0);
    S.accm = 0;
    S.vw = m.vw;
    S.pw = m.pw;
#pragma unroll
    for (int k = 0; k < WPW / 4; ++k) {
        // bytes of the words in [w_begin, w_end) (wave-uniform)
        const int32_t lo = min(max(w_begin - sbw - 4 * k, 0), 4);
        const int32_t hi = min(max(w_end - sbw - 4 * k, 0), 4);
        const uint32_t keep = (hi == 4 ? ~0u : (1u << (8 * hi)) - 1u) & (lo == 4 ? 0u : ~((1u << (8 * lo)) - 1u));
        const uint32_t L = m.lens[k] & keep;
        S.lens[k] = L;
        const int32_t pa = (int32_t)(L & 0x00ff00ffu);         // words 4k and 4k + 2
        const int32_t pb = (int32_t)((L >> 8) & 0x00ff00ffu);  // words 4k + 1 and 4k + 3
        const int32_t ea = wave_exclusive_scan(pa);
        const int32_t eb = wave_exclusive_scan(pb);
        const uint32_t ta = (uint32_t)__builtin_amdgcn_readlane(ea + pa, 63);
        const uint32_t tb = (uint32_t)__builtin_amdgcn_readlane(eb + pb, 63);
        const int32_t ex[4] = {ea & 0xffff, eb & 0xffff, (int32_t)((uint32_t)ea >> 16), (int32_t)((uint32_t)eb >> 16)};
        const int32_t tot[4] = {(int32_t)(ta & 0xffffu), (int32_t)(tb & 0xffffu), (int32_t)(ta >> 16),
                                (int32_t)(tb >> 16)};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int w = 4 * k + j;
            S.st[w] = run + ex[j];
            S.ws[w] = run;
            if ((L >> (8 * j)) & 0xffu) S.accm |= 1u << w;  // block AND rows are exactly the rows with a length
            run += tot[j];
        }
    }
    S.ws[WPW] = run;
}

// The v bits of the U chunks of one round, one ballot per chunk into the
// wave's LDS slots.
template <int MODE, int U>
__device__ __forceinline__ void round_ballots(const lds_u8 *s_v8, const uint8_t *v8, uint32_t lds_bytes,
                                              const int32_t (&c)[U], lds_u64 *s_ball) {
    const int lane = threadIdx.x & 63;
    uint32_t x[U];
    if (MODE == kStepLds || MODE == kStepSlice) {
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = entry_word(s_v8, c[u]);
    } else if (MODE == kStepGlobal) {
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = entry_word(v8, c[u]);
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (entry_byte(c[u]) >= lds_bytes) x[u] = entry_word(v8, c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (entry_byte(c[u]) < lds_bytes) x[u] = entry_word(s_v8, c[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t B = __ballot(__builtin_amdgcn_ubfe(x[u], (uint32_t)c[u], 1u));
        if (lane == 0) s_ball[u] = B;
    }
}

// Each row-owner lane's fold of the ballot bits of its entries in the round
// [base, base + 64 U) into its word bit of accm.
template <int WPW, int U>
__device__ __forceinline__ void fold_round(const lds_u64 *s_ball, int32_t base, SbState<WPW> &S) {
    const int32_t lim = base + 64 * U;
    const lds_u32 *b32 = (const lds_u32 *)s_ball;  // the round's ballot bits, 32 per word
#pragma unroll
    for (int w = 0; w < WPW; ++w) {
        if (S.ws[w + 1] <= base || S.ws[w] >= lim) continue;  // word outside the round (wave-uniform)
        int32_t lo = S.st[w] > base ? S.st[w] : base;
        const int32_t en = S.st[w] + lane_len<WPW>(S.lens, w);
        const int32_t hi = en < lim ? en : lim;
        uint32_t bad = 0;  // entries of the row that are 0
        while (lo < hi) {  // 32 entries per pass: one pass for rows of up to 32 entries
            const int32_t rel = lo - base;
            const int32_t n = hi - lo < 32 ? hi - lo : 32;
            const uint32_t win = __builtin_amdgcn_alignbit(b32[(rel >> 5) + 1], b32[rel >> 5], (uint32_t)rel);
            bad |= ~win & (0xffffffffu >> (32 - n));  // the window's first n bits
            lo += n;
        }
        if (bad) S.accm &= ~(1u << w);
    }
}

// Results of a finished super-block: one atomic OR per word with AND rows
// that fire, and the wave's count of new bits (counted in lane 0). The words
// of v came with the row data, so nothing here waits for memory.
template <int WPW>
__device__ __forceinline__ uint32_t sb_finish(const StepParams &p, int32_t sbw, int32_t n_words,
                                              const SbState<WPW> &S) {
    const int lane = threadIdx.x & 63;
    uint32_t n_new = 0;
    const uint32_t vlo = (uint32_t)S.vw, vhi = (uint32_t)(S.vw >> 32);
#pragma unroll
    for (int w = 0; w < WPW; ++w) {
        const int32_t wd = sbw + w;
        const uint64_t res = __ballot((S.accm >> w) & 1u);
        if (wd < n_words && res) {
            // readlane returns int: go through uint32_t so the low half is not sign-extended
            const uint64_t v = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(vhi, w) << 32) |
                               (uint64_t)(uint32_t)__builtin_amdgcn_readlane(vlo, w);
            n_new += (uint32_t)__popcll(res & ~v);
            if (lane == 0) atomicOr((unsigned long long *)&p.u[wd], (unsigned long long)res);
        }
    }
    return lane == 0 ? n_new : 0;
}

// Results of a finished super-block in a pass over one column slice. A row
// passes the slice if its entries there are all true or it has none there;
// per word of the wave's range, pass 0 stores the passing block AND rows in
// pacc, later passes AND theirs in, and the last pass ORs the rows that
// passed every slice into u and counts the new ones. The words of and_all
// (pass 0) or pacc came with the row data.
template <int WPW>
__device__ __forceinline__ uint32_t sb_finish_slice(const StepParams &p, int32_t sbw, int32_t w_begin, int32_t w_end,
                                                    const SbState<WPW> &S) {
    const int lane = threadIdx.x & 63;
    uint32_t n_new = 0;
    const uint32_t vlo = (uint32_t)S.vw, vhi = (uint32_t)(S.vw >> 32);
    const uint32_t plo = (uint32_t)S.pw, phi = (uint32_t)(S.pw >> 32);
    const bool last = p.pass == p.n_pass - 1;
#pragma unroll
    for (int w = 0; w < WPW; ++w) {
        const int32_t wd = sbw + w;
        if (wd < w_begin || wd >= w_end) continue;  // another wave's word (wave-uniform)
        const uint64_t res = __ballot((S.accm >> w) & 1u);
        const uint64_t has = __ballot(lane_len<WPW>(S.lens, w) != 0);
        const uint64_t pass_ok = res | ~has;
        const uint64_t prev = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(phi, w) << 32) |
                              (uint64_t)(uint32_t)__builtin_amdgcn_readlane(plo, w);
        const uint64_t acc = prev & pass_ok;  // pass 0: prev is and_all
        if (!last) {
            if (lane == 0) p.pacc[wd] = acc;
        } else if (acc) {
            const uint64_t v = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(vhi, w) << 32) |
                               (uint64_t)(uint32_t)__builtin_amdgcn_readlane(vlo, w);
            n_new += (uint32_t)__popcll(acc & ~v);
            if (lane == 0) atomicOr((unsigned long long *)&p.u[wd], (unsigned long long)acc);
        }
    }
    return lane == 0 ? n_new : 0;
}

// Block pass: AND rows of up to kLongAnd entries, as one stream per wave.
//
// Wave k owns the words [wave_part[2k], wave_part[2k + 2]) (a host-computed
// split with about the same number of AND entries per wave) and streams their
// AND entries, one contiguous stretch of col, in rounds of U chunks of 64
// entries (256 bytes per chunk, coalesced). The rows are taken in
// super-blocks of WPW words aligned to 4 words; words of a super-block outside
// the wave's range count as empty. The next round's chunks are always in
// flight while the current round is evaluated, and the next super-block's row
// data is loaded a super-block ahead. A round may end one super-block and
// continue into the next. The round body is written twice with the chunk
// buffers swapped, so no chunk register is copied (a copy would wait for its
// load).
//
// VALU economy (a wave64 VALU instruction takes 4 cycles on a CDNA SIMD):
//  * chunk loads are unconditional, from a wave-uniform base plus the lane
//    offset, so no per-entry predicate or address arithmetic;
//  * a gather is one shift (the 32-bit word of v), one word read and one
//    v_bfe_u32 (see entry_byte); v sits at LDS address 0, so the shifted entry
//    is the address;
//  * entries outside the wave's range are gathered like the others (they name
//    valid atoms) and simply fall outside every row's range;
//  * each row reads the 32-bit window of ballot bits starting at its first
//    entry (v_alignbit of two consecutive ballot dwords) and compares it with
//    a mask of its length: one step for rows of up to 32 entries in a round;
//  * row starts come from a DPP scan of 8-bit lengths; the AND row bits are
//    the rows with a nonzero length; per word a lane keeps one start and one
//    result bit.
template <int MODE, int WPW, int U>
struct BlockPass {
    int32_t w_begin, w_end;  // the wave's words
    int32_t sbw;             // first word of the current super-block
    int32_t sb_last;         // first word of the wave's last super-block
    int32_t n_words;
    int32_t base;            // first entry of the current round (a multiple of 64)
    int32_t last_base;       // start of the round that ends at the wave's last entry (rounded up to 64)
    SbMeta<WPW> cur, nxt;    // cur: the first super-block's row data, until start()
    SbState<WPW> S;
    int32_t ca[U], cb[U];

    // Issues the row data of the wave's first two super-blocks and its first
    // round of chunks. Called while v is being staged, so these loads overlap
    // the staging and everything else the wave does before the stream. False
    // if the wave has no words.
    __device__ __forceinline__ bool prefetch(const StepParams &p) {
        n_words = (p.n_rows + 63) >> 6;
        const int64_t k = grid_wave();
        // the wave's four split entries (the test names all four, so they are
        // read together rather than two of them after it)
        w_begin = p.wave_part[2 * k];
        const int32_t e_begin = p.wave_part[2 * k + 1];
        w_end = p.wave_part[2 * k + 2];
        const int32_t e_end = p.wave_part[2 * k + 3];
        // Every wave issues the same loads, also one with no words (its
        // range is empty and lies within the padded arrays), so the wait
        // counts of the loads issued after these are the same on every path.
        const bool has = w_begin < w_end && e_begin <= e_end;  // (e_begin <= e_end always)
        sbw = w_begin & ~3;
        sb_last = has ? sbw + ((w_end - 1 - sbw) / WPW) * WPW : sbw;
        base = e_begin & ~63;
        last_base = max(0, ((e_end + 63) & ~63) - 64 * U);
        load_sb_meta<WPW, MODE == kStepSlice>(p, sbw, w_begin, n_words, cur);
        load_sb_meta<WPW, MODE == kStepSlice>(p, sbw + WPW <= sb_last ? sbw + WPW : sb_last, w_begin, n_words, nxt);
        load_chunks<U>(p, base, ca);
        return has;
    }

    // Sets up the first super-block (its row data has landed by now).
    __device__ __forceinline__ void start() { sb_setup<WPW>(cur, sbw, w_begin, w_end, S); }

    __device__ __forceinline__ uint32_t run(const StepParams &p, const lds_u32 *s_v, lds_u64 *s_ball) {
        const uint32_t lds_bytes = MODE != kStepGlobal ? (uint32_t)p.lds_words * 8u : 0u;
        const lds_u8 *s_v8 = (const lds_u8 *)s_v;
        const uint8_t *v8 = reinterpret_cast<const uint8_t *>(p.v);
        uint32_t my_new = 0;
        // Let the loads issued so far land before the loop: otherwise the
        // compiler's wait counting merges them into the loop header's state
        // and waits for every load in flight at the top of each round.
        __builtin_amdgcn_s_waitcnt(0);
        // One round: prefetch the next round into cn, evaluate c, and finish
        // every super-block that ends in this round. At each such end the
        // next super-block is set up from nxt and the one after it is loaded
        // into nxt, to be used at the next end (normally a round or more
        // later; a round that ends several super-blocks waits for it). Row
        // data is thus read once per super-block. Returns false when the
        // wave's last super-block is done.
        auto round = [&](const int32_t (&c)[U], int32_t (&cn)[U]) -> bool {
            // Issue priority by the work left: the 16 waves of a workgroup
            // share a CU, and with equal priorities the ones that fell behind
            // stayed behind (measured: 5.7 us between the first and the last
            // wave of a workgroup to finish). A wave with more than three
            // rounds left gets priority 3, then 2, 1 and 0 for its last round.
            {
                const int32_t left = __builtin_amdgcn_readfirstlane(last_base - base);
                if (left > 3 * 64 * U) __builtin_amdgcn_s_setprio(3);
                else if (left > 2 * 64 * U) __builtin_amdgcn_s_setprio(2);
                else if (left > 64 * U) __builtin_amdgcn_s_setprio(1);
                else __builtin_amdgcn_s_setprio(0);
            }
            const int32_t lim = base + 64 * U;
            // The next round starts at lim, except that no round reads past
            // the wave's last entry (rounded up to 64): those entries belong to
            // the next wave, which read them long ago, so reading them again
            // would come from memory. The last round therefore starts earlier
            // and evaluates some entries twice (harmless: a row's fold only
            // clears bits), and the round after the last one reloads it.
            const int32_t nb = max(base, min(lim, last_base));
            load_chunks<U>(p, nb, cn);
            // keep the scheduler from hoisting this round's gathers (which
            // wait for its chunks) above the next round's loads
            __builtin_amdgcn_sched_barrier(0);
            round_ballots<MODE, U>(s_v8, v8, lds_bytes, c, s_ball);
            fold_round<WPW, U>(s_ball, base, S);
            while (__builtin_amdgcn_readfirstlane(S.ws[WPW]) <= lim) {
                if (MODE == kStepSlice)
                    my_new += sb_finish_slice<WPW>(p, sbw, w_begin, w_end, S);
                else
                    my_new += sb_finish<WPW>(p, sbw, n_words, S);
                if (sbw >= sb_last) return false;
                sbw += WPW;
                sb_setup<WPW>(nxt, sbw, w_begin, w_end, S);
                load_sb_meta<WPW, MODE == kStepSlice>(p, sbw + WPW <= sb_last ? sbw + WPW : sb_last, w_begin,
                                                      n_words, nxt);
                fold_round<WPW, U>(s_ball, base, S);
            }
            base = nb;
            return true;
        };
        for (;;) {
            if (!round(ca, cb)) break;
            if (!round(cb, ca)) break;
        }
        return my_new;
    }
};

// OR rows that are not long, 64 per wave: lane j takes OR row 64*tile + j,
// reads its child range from or_c0, ORs the words of v in that range and, if
// it fires, sets the row's bit. An OR row is evaluated by exactly one lane, so
// it is new iff its bit is 0 in v. A wave takes four of its tiles at a time
// (tiles t0 + g * stride) in three steps whose loads can be issued early:
// the range table, then the first and last word of every range (the words
// between them, rare for OR rows of at most kLongOrBits children, are read at
// the end), then the evaluation.
template <bool LDS>
struct OrTiles {
    static constexpr int G = 4;
    int32_t row[G], c0[G], c1[G];
    uint64_t a[G], z[G];
    bool any_tile;

    // The loads are issued in every wave, also one with no tile (clamped to
    // the table's first entries, which always exist), so the wait counts of
    // later loads are the same on every path.
    __device__ __forceinline__ void load_ranges(const StepParams &p, int64_t t0, int64_t stride) {
        const int lane = threadIdx.x & 63;
        any_tile = t0 < (((int64_t)p.n_or + 63) >> 6);  // wave-uniform
#pragma unroll
        for (int g = 0; g < G; ++g) {  // j clamped to the last OR row: in bounds, marked invalid below
            const int64_t j = (t0 + g * stride) * 64 + lane;
            const int64_t jc = j < p.n_or ? j : (p.n_or > 0 ? p.n_or - 1 : 0);
            const int32_t rr = p.or_row[jc];
            row[g] = j < p.n_or ? rr : -1;
            c0[g] = p.or_c0[jc];
            c1[g] = p.or_c0[jc + 1 <= p.n_or ? jc + 1 : p.n_or];
        }
    }

    __device__ __forceinline__ void load_words(const StepParams &p) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (c1[g] <= c0[g]) row[g] = -1;
            const int32_t w0 = row[g] >= 0 ? c0[g] >> 6 : 0;
            const int32_t w1 = row[g] >= 0 ? (c1[g] - 1) >> 6 : 0;
            a[g] = p.v[w0];
            z[g] = p.v[w1];
        }
    }

    __device__ __forceinline__ uint32_t finish(const StepParams &p, const lds_u32 *s_v) {
        uint32_t my_new = 0;
        if (!any_tile) return 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (row[g] < 0) continue;
            const int32_t w0 = c0[g] >> 6, w1 = (c1[g] - 1) >> 6;
            const int s = c0[g] & 63, t = ((c1[g] - 1) & 63) + 1;
            bool any;
            if (w0 == w1) {
                any = (a[g] & range_mask(s, t)) != 0;
            } else {
                any = (a[g] & range_mask(s, 64)) != 0 || (z[g] & range_mask(0, t)) != 0;
                for (int32_t wd = w0 + 1; wd < w1 && !any; ++wd) any = p.v[wd] != 0;
            }
            if (any) {
                const uint64_t bit = 1ull << (row[g] & 63);
                atomicOr((unsigned long long *)&p.u[row[g] >> 6], (unsigned long long)bit);
                if (!(vword<LDS>(p, s_v, row[g] >> 6) & bit)) my_new += 1;
            }
        }
        return my_new;
    }
};

// All of the wave's OR tiles, four at a time, each batch's loads issued
// together (the persistent kernel, whose loop state leaves no registers for
// issuing them earlier).
template <bool LDS>
__device__ __forceinline__ uint32_t or_rows(const StepParams &p, const lds_u32 *s_v) {
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t n_tiles = ((int64_t)p.n_or + 63) >> 6;
    uint32_t my_new = 0;
    for (int64_t t0 = grid_wave(); t0 < n_tiles; t0 += OrTiles<LDS>::G * stride) {
        OrTiles<LDS> ot;
        ot.load_ranges(p, t0, stride);
        ot.load_words(p);
        my_new += ot.finish(p, s_v);
    }
    return my_new;
}

// The wave's OR tiles after its first four (which the step kernel takes
// through OrTiles with its loads issued before staging v).
template <bool LDS>
__device__ __forceinline__ uint32_t or_rows_rest(const StepParams &p, const lds_u32 *s_v) {
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t n_tiles = ((int64_t)p.n_or + 63) >> 6;
    uint32_t my_new = 0;
    for (int64_t t0 = grid_wave() + OrTiles<LDS>::G * stride; t0 < n_tiles; t0 += OrTiles<LDS>::G * stride) {
        OrTiles<LDS> ot;
        ot.load_ranges(p, t0, stride);
        ot.load_words(p);
        my_new += ot.finish(p, s_v);
    }
    return my_new;
}

// Segments of long rows, one wave each: AND segments stream entries of
// long_col, OR segments scan a bit range of v.
template <bool LDS, int U>
__device__ __forceinline__ uint32_t long_rows(const StepParams &p, const lds_u32 *s_v) {
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * waves;
    const uint32_t lds_bytes = LDS ? (uint32_t)p.lds_words * 8u : 0u;
    const lds_u8 *s_v8 = (const lds_u8 *)s_v;
    const uint8_t *v8 = reinterpret_cast<const uint8_t *>(p.v);
    uint32_t my_new = 0;
    for (int64_t si = grid_wave(); si < p.n_segs; si += stride) {
        const LongSeg sg = p.segs[si];
        bool any = false, all = true;
        if (sg.is_and) {
            for (int32_t i0 = 0; i0 < sg.len; i0 += 64 * U) {
                int32_t c[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t i = i0 + 64 * u + lane;
                    c[u] = i < sg.len ? p.long_col[sg.begin + i] : -1;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (c[u] >= 0) {
                        const uint32_t x = (LDS && entry_byte(c[u]) < lds_bytes) ? entry_word(s_v8, c[u])
                                                                                : entry_word(v8, c[u]);
                        all &= __builtin_amdgcn_ubfe(x, (uint32_t)c[u], 1u) != 0;
                    }
                }
            }
        } else {
            // bits [begin, begin + len): lane l takes words l, l + 64, ... of the range
            const int64_t b0 = sg.begin, b1 = sg.begin + sg.len;
            for (int64_t wd = (b0 >> 6) + lane; wd <= (b1 - 1) >> 6; wd += 64) {
                const int s = wd == (b0 >> 6) ? (int)(b0 & 63) : 0;
                const int t = wd == ((b1 - 1) >> 6) ? (int)(((b1 - 1) & 63) + 1) : 64;
                any |= (p.v[wd] & range_mask(s, t)) != 0;
            }
        }
        any = __ballot(any) != 0;
        all = __ballot(!all) == 0;
        if (lane == 0) {
            bool fire;
            if (!sg.is_and) {
                fire = any;
            } else if (sg.nseg == 1) {
                fire = all;
            } else {
                // a split AND row fires when all of its segments were all-true
                uint32_t *cnt = p.and_cnt + (size_t)(p.step & 1) * p.n_long_and + sg.and_slot;
                fire = all && atomicAdd(cnt, 1u) == (uint32_t)(sg.nseg - 1);
                if (sg.seg == 0)  // clear the count the next product will use
                    p.and_cnt[(size_t)((p.step + 1) & 1) * p.n_long_and + sg.and_slot] = 0;
            }
            if (fire) {
                const uint64_t bit = 1ull << (sg.row & 63);
                const uint64_t old = atomicOr((unsigned long long *)&p.u[sg.row >> 6], (unsigned long long)bit);
                if (!(old & bit) && !(vword<LDS>(p, s_v, sg.row >> 6) & bit)) my_new += 1;
            }
        }
    }
    return my_new;
}

// Copies lds_words words of v from word stage_off (an even word: the copies
// are 16-byte loads) into LDS: 16-byte loads, up to
// eight in flight per thread before any is stored (one memory round trip for
// 128 KB with 1,024 threads).
__device__ __forceinline__ void stage_v(const StepParams &p, lds_u32 *s_v) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) u32x4 lds_u4;
    constexpr int kInFlight = 8;
    lds_u4 *d = (lds_u4 *)s_v;
    const u32x4 *src = reinterpret_cast<const u32x4 *>(p.v + p.stage_off);
    const int32_t n16 = p.lds_words >> 1;
    const int32_t bd = blockDim.x;
    for (int32_t i = threadIdx.x; i < n16; i += kInFlight * bd) {
        u32x4 x[kInFlight];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k)
            if (i + k * bd < n16) x[k] = src[i + k * bd];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k)
            if (i + k * bd < n16) d[i + k * bd] = x[k];
    }
    if ((p.lds_words & 1) && threadIdx.x == 0) ((lds_u64 *)s_v)[p.lds_words - 1] = p.v[p.stage_off + p.lds_words - 1];
}

// stage_v split in two: the first loads (up to eight 16-byte loads per
// thread, 128 KB per 1,024 threads) are issued before the wave's other
// prologue loads and written to LDS after them. Every thread issues all eight
// (indices past the end reload the last 16 bytes), so the wait counts of the
// loads issued in between are the same on every path.
struct StageV {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) u32x4 lds_u4;
    static constexpr int kInFlight = 8;
    u32x4 x[kInFlight];

    __device__ __forceinline__ void issue(const StepParams &p) {
        const int32_t n16 = p.lds_words >> 1;
        if (n16 == 0) return;  // the same in every thread of the launch
        const u32x4 *src = reinterpret_cast<const u32x4 *>(p.v + p.stage_off);
        const int32_t bd = blockDim.x;
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) {
            const int32_t i = threadIdx.x + k * bd;
            x[k] = src[i < n16 ? i : n16 - 1];
        }
    }

    __device__ __forceinline__ void commit(const StepParams &p, lds_u32 *s_v) {
        lds_u4 *d = (lds_u4 *)s_v;
        const u32x4 *src = reinterpret_cast<const u32x4 *>(p.v + p.stage_off);
        const int32_t n16 = p.lds_words >> 1;
        const int32_t bd = blockDim.x;
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) {
            const int32_t i = threadIdx.x + k * bd;
            if (i < n16) d[i] = x[k];
        }
        for (int32_t i = threadIdx.x + kInFlight * bd; i < n16; i += kInFlight * bd) {  // past 128 KB
            u32x4 y[kInFlight];
#pragma unroll
            for (int k = 0; k < kInFlight; ++k)
                if (i + k * bd < n16) y[k] = src[i + k * bd];
#pragma unroll
            for (int k = 0; k < kInFlight; ++k)
                if (i + k * bd < n16) d[i + k * bd] = y[k];
        }
        if ((p.lds_words & 1) && threadIdx.x == 0) ((lds_u64 *)s_v)[p.lds_words - 1] = p.v[p.stage_off + p.lds_words - 1];
    }
};

__device__ __forceinline__ void add_new_bits(uint32_t my_new, lds_u32 *s_new, unsigned long long *slot) {
    my_new = wave_sum(my_new);
    if ((threadIdx.x & 63) == 0 && my_new)
        __hip_atomic_fetch_add(s_new, my_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (threadIdx.x == 0 && *s_new) atomicAdd(slot, (unsigned long long)*s_new);
}

}  // namespace

// LDS of the staged forms, one static array so that v sits at LDS address 0
// and a gather's address is the shifted entry itself: [v: step_lds_v_words]
// [ballot slots: kMaxWaves x (U + 1) words][new-bit count]. The global form
// keeps only the ballot slots and the count.
template <int MODE, int U>
struct StepLds {
    static constexpr int kV = MODE == kStepGlobal ? 0 : kStepLdsBytes / 8 - kMaxWaves * (U + 1) - 2;
    static constexpr int kWords = kV + kMaxWaves * (U + 1) + 2;
    lds_u32 *v;
    lds_u64 *my_ball;
    lds_u32 *n_new;
    __device__ __forceinline__ explicit StepLds(lds_u64 *base) {
        v = (lds_u32 *)base;
        my_ball = base + kV + (threadIdx.x >> 6) * (U + 1);
        n_new = (lds_u32 *)(base + kV + kMaxWaves * (U + 1));
    }
};

template <int MODE, int WPW, int U>
__global__ __launch_bounds__(1024) void tp_step_kernel(StepParams p) {
    __shared__ uint64_t s_lds[StepLds<MODE, U>::kWords];
    const StepLds<MODE, U> L((lds_u64 *)s_lds);
    if ((threadIdx.x & 63) == 0) L.my_ball[U] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) p.counters[(p.step + 1) & (kRing - 1)] = 0;
    // Prologue loads, in this order: the previous product's count (early
    // exit past the fixpoint), the staging of v, the block pass's row data
    // and first chunks, the first OR tiles' ranges; then v goes to LDS, the
    // OR tiles' words are loaded, and they are evaluated after the barrier.
    // So the stream is in flight while v is staged and while the OR rows and
    // segments are evaluated, and no round trip of the prologue waits alone.
    const unsigned long long prev = p.counters[(p.step - 1) & (kRing - 1)];
    // OR rows and long rows read v from LDS in the staged forms; a sliced step
    // evaluates them in its last pass only, from v in global memory
    constexpr bool kOrLds = MODE == kStepLds || MODE == kStepMixed;
    StepParams q = p;
    if (MODE == kStepSlice && p.pass != p.n_pass - 1) {
        q.n_or = 0;
        q.n_segs = 0;
    }
    StageV sv;
    if (MODE != kStepGlobal) sv.issue(p);
    if (threadIdx.x == 0) *L.n_new = 0;
    BlockPass<MODE, WPW, U> bp;
    const bool blocks = bp.prefetch(p);
    OrTiles<kOrLds> ot;
    ot.load_ranges(q, grid_wave(), (int64_t)gridDim.x * (blockDim.x >> 6));
    if (MODE != kStepGlobal) sv.commit(p, L.v);
    if (p.early_exit && p.step >= 2 && prev == 0) return;
    ot.load_words(q);
    if (blocks) bp.start();
    __syncthreads();
    // long-row segments first: they are the longest items, so they start early
    uint32_t my_new = long_rows<kOrLds, U>(q, L.v);
    my_new += ot.finish(q, L.v);
    my_new += or_rows_rest<kOrLds>(q, L.v);
    if (blocks) my_new += bp.run(p, L.v, L.my_ball);
    add_new_bits(my_new, L.n_new, &p.counters[p.step & (kRing - 1)]);
}

// Grid-wide barrier of a cooperative launch (every workgroup is resident):
// each workgroup adds 1 to *count with an agent-scope release (its writes,
// made visible to the workgroup by __syncthreads, are written back past the
// XCD's L2 first), then its first thread polls *count with relaxed
// agent-scope loads until it reaches target and ends with one agent-scope
// acquire fence. The poll is bounded: after
// kBarrierPolls reads, or when another workgroup has given up, it sets
// *abort. Returns false (in every thread of the workgroup) if the barrier was
// abandoned.
constexpr uint32_t kBarrierPolls = 1u << 22;

__device__ __forceinline__ bool grid_barrier(uint32_t *count, uint32_t target, int32_t *abort, lds_u32 *s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        for (uint32_t polls = 0;; ++polls) {
            // relaxed polls (an acquire on each would invalidate the L2 every time)
            if (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (polls >= kBarrierPolls ||
                ((polls & 63) == 63 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// The whole Algorithm 1 loop in one cooperative launch. Each product: stage v
// in LDS, evaluate every row, add the new-bit count, grid-wide barrier
// (grid_barrier, which also orders the memory the other XCDs wrote), read the
// count. Every workgroup reads the same count after the barrier, so all leave
// the loop on the same product; max_steps (a monotone iteration needs at most
// n_rows + 1 products) guarantees the loop ends, and an abandoned barrier ends
// it with result -2.
template <int MODE, int WPW, int U>
__global__ __launch_bounds__(1024) void tp_fixpoint_persistent_kernel(PersistParams q) {
    __shared__ uint64_t s_lds[StepLds<MODE, U>::kWords];
    const StepLds<MODE, U> L((lds_u64 *)s_lds);
    lds_u32 *s_v = L.v;
    lds_u64 *my_ball = L.my_ball;
    lds_u32 *s_new_p = L.n_new;
    if ((threadIdx.x & 63) == 0) my_ball[U] = 0;
    StepParams p = q.p;
    for (int32_t step = 1;; ++step) {
        p.step = step;
        p.v = (step & 1) ? q.buf0 : q.buf1;
        p.u = (step & 1) ? q.buf1 : q.buf0;
        unsigned long long *slot = &p.counters[step & (kRing - 1)];
        if (blockIdx.x == 0 && threadIdx.x == 0) p.counters[(step + 1) & (kRing - 1)] = 0;
        if (threadIdx.x == 0) *s_new_p = 0;
        BlockPass<MODE, WPW, U> bp;
        const bool blocks = bp.prefetch(p);
        stage_v(p, s_v);
        if (blocks) bp.start();
        __syncthreads();
        uint32_t my_new = long_rows<true, U>(p, s_v);
        my_new += or_rows<true>(p, s_v);
        if (blocks) my_new += bp.run(p, s_v, my_ball);
        add_new_bits(my_new, s_new_p, slot);
        if (!grid_barrier(q.bar, gridDim.x * (uint32_t)step, q.abort, s_new_p + 1)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *q.result = -2;
            return;
        }
        const unsigned long long changed = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (changed == 0 || step >= q.max_steps) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *q.result = changed == 0 ? step : -1;
            return;
        }
    }
}

// ------------------------------------------------------------------ launchers

#define LP_STEP_SHAPES(X) X(4, 4) X(4, 8) X(4, 16) X(8, 4) X(8, 8) X(8, 16)

bool step_shape_supported(const StepShape &s) {
#define LP_X(W, U) \
    if (s.wpw == W && s.unroll == U) return true;
    LP_STEP_SHAPES(LP_X)
#undef LP_X
    return false;
}

// One product: one launch, or one launch per column slice of a sliced layout
// (pass k with slice k's layout and staged words).
hipError_t launch_step(const StepShape &s, const StepParams &p, hipStream_t st) {
    if (s.mode == kStepSlice) {
        if (s.n_slices < 2 || s.n_slices > kMaxSlices || !s.slice) return hipErrorInvalidValue;
        for (int k = 0; k < s.n_slices; ++k) {
            const SliceLayout &L = s.slice[k];
            StepParams q = p;
            q.words = L.words;
            q.and_len = L.and_len;
            q.lens4 = L.lens4;
            q.col = L.col;
            q.and_end = L.and_end;
            q.and_max_col = L.and_max_col;
            q.wave_part = s.slice_part[k];
            q.stage_off = L.first_word;
            q.lds_words = L.lds_words;
            q.pass = k;
            q.n_pass = s.n_slices;
            hipError_t e = launch_step_pass(s, q, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    return launch_step_pass(s, p, st);
}

hipError_t launch_step_pass(const StepShape &s, const StepParams &p, hipStream_t st) {
#define LP_X(W, U)                                                                                       \
    if (s.wpw == W && s.unroll == U) {                                                                   \
        if (s.mode == kStepSlice)                                                                        \
            hipLaunchKernelGGL((tp_step_kernel<kStepSlice, W, U>), dim3(s.grid), dim3(s.block), 0, st, p); \
        else if (s.mode == kStepLds)                                                                     \
            hipLaunchKernelGGL((tp_step_kernel<kStepLds, W, U>), dim3(s.grid), dim3(s.block), 0, st, p);   \
        else if (s.mode == kStepMixed)                                                                   \
            hipLaunchKernelGGL((tp_step_kernel<kStepMixed, W, U>), dim3(s.grid), dim3(s.block), 0, st, p); \
        else                                                                                             \
            hipLaunchKernelGGL((tp_step_kernel<kStepGlobal, W, U>), dim3(s.grid), dim3(s.block), 0, st, p); \
        return hipGetLastError();                                                                        \
    }
    LP_STEP_SHAPES(LP_X)
#undef LP_X
    return hipErrorInvalidValue;
}

static const void *persistent_fn(const StepShape &s) {
#define LP_X(W, U)                                                                                       \
    if (s.wpw == W && s.unroll == U) {                                                                   \
        if (s.mode == kStepLds) return (const void *)tp_fixpoint_persistent_kernel<kStepLds, W, U>;     \
        if (s.mode == kStepMixed) return (const void *)tp_fixpoint_persistent_kernel<kStepMixed, W, U>; \
        return nullptr;                                                                                  \
    }
    LP_STEP_SHAPES(LP_X)
#undef LP_X
    return nullptr;
}

hipError_t launch_persistent(const StepShape &s, const PersistParams &q, hipStream_t st) {
    const void *fn = persistent_fn(s);
    if (!fn) return hipErrorInvalidValue;
    PersistParams copy = q;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(s.grid), dim3(s.block), args, 0, st);
}

hipError_t persistent_occupancy(const StepShape &s, int *blocks_per_cu) {
    const void *fn = persistent_fn(s);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, s.block, 0);
}

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_words(void *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid), dim3(256), 0, st, (uint32_t *)p, n);
    return hipGetLastError();
}

}  // namespace lp
