// lp_batch.hip -- least models of many definite programs in one persistent
// launch (Algorithm 1 per program).
//
// Each workgroup takes programs from a device work queue (an atomic counter
// over programs sorted by decreasing size, so the longest start first) and
// runs a program's whole fixpoint by itself: both interpretation buffers of
// the program live in LDS, every product is evaluated by the workgroup's
// waves, products are separated by workgroup barriers, and no host round trip
// or grid-wide barrier is needed. The matrix layout is each program's own
// least-model layout (see WordMeta); programs whose two bit-packed buffers do
// not fit in LDS are solved by the single-program drivers instead.
//
// The evaluation of one product is the step of lp_step.hip with v and u in
// LDS: AND rows by super-blocks (coalesced column chunks, byte gathers from
// LDS, ballots, one window fold per row), OR rows as child bit ranges, long
// rows by segments. Results are ORed into the buffer holding v_{t-1}
// (monotone), and the new-bit count decides the loop.
//
// A program much larger than a workgroup's share of the batch is solved by a
// team of G workgroups (its G queue positions come first, so all members
// start at once). Member m evaluates the m-th of G contiguous ranges of
// words (about equal AND-stream work), every G-th block of OR rows and every
// G-th segment; after each product the members OR the rows they found new
// (true now, not in v_{t-1}) into a global delta buffer, meet at a bounded
// team barrier and take v_t as v_{t-1} OR the delta. The products are those
// of the one-workgroup loop.
//
// Within a workgroup (or a team member) the words are split among the waves
// by AND-stream work when the program starts, and each wave streams its stretch
// of the layout with a round of chunks always in flight; issue priority by
// the work left keeps the waves of a workgroup finishing together.
#include <hip/hip_runtime.h>

#include "lp_dev.h"
#include "lp_kernels.h"

namespace lp {

namespace {

// Descriptor pointers are loaded from memory, where the compiler cannot tell
// global from LDS addresses; the copies below carry the global address space
// so every access compiles to a global load (flat loads would also count
// against the LDS wait counter and serialize the LDS gathers).
template <class T>
using gp = const __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ gp<T> as_global(const T *p) {
    return (gp<T>)p;
}

typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) uint64_t g_u64;
typedef __attribute__((address_space(1))) int32_t g_i32;

template <class T>
using cp = const __attribute__((address_space(4))) T *;

template <class T>
__device__ __forceinline__ cp<T> as_const(const T *p) {
    return (cp<T>)p;
}

// A program descriptor read word by word through the constant address space.
__device__ __forceinline__ ProgDesc load_desc(const ProgDesc *p) {
    static_assert(sizeof(ProgDesc) % 4 == 0, "descriptor words");
    ProgDesc d;
    const cp<uint32_t> s = (cp<uint32_t>)(const void *)p;
    uint32_t *o = reinterpret_cast<uint32_t *>(&d);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(ProgDesc) / 4); ++i) o[i] = s[i];
    return d;
}

// A program's layout as the evaluation reads it: in global memory (AS = 1),
// or copied into the workgroup's LDS (AS = 3; see LdsLayout). Only the
// fields of WordMeta the workgroup loop reads are kept in the LDS form.
template <int AS>
struct Prog;

template <>
struct Prog<1> {
    gp<WordMeta> words;
    gp<uint8_t> and_len;
    gp<uint32_t> lens4;
    gp<int32_t> col;
    gp<int32_t> or_c0;
    gp<int32_t> or_row;
    gp<LongSeg> segs;
    gp<int32_t> long_col;
    int32_t n_rows, n_or, n_segs, and_end;
    static constexpr bool kLds = false;
    __device__ __forceinline__ int32_t and_base(int64_t w) const { return words[w].and_base; }
    __device__ __forceinline__ uint64_t and_bits(int64_t w) const { return words[w].and_bits; }
};

typedef __attribute__((address_space(3))) LongSeg lds_seg;

template <>
struct Prog<3> {
    const lds_u64 *andb;
    const lds_i32 *base;
    const lds_u8 *and_len;
    const lds_i32 *col;
    const lds_i32 *or_c0;
    const lds_i32 *or_row;
    const lds_seg *segs;
    const lds_i32 *long_col;
    int32_t n_rows, n_or, n_segs, and_end;
    static constexpr bool kLds = true;
    __device__ __forceinline__ int32_t and_base(int64_t w) const { return base[w]; }
    __device__ __forceinline__ uint64_t and_bits(int64_t w) const { return andb[w]; }
};

typedef Prog<1> GProg;

// Copies the layout of g into LDS at `dst` (offsets from lds_layout) with the
// whole workgroup; the caller synchronizes afterwards. The AND entries and
// lengths move in 16-byte pieces (their global arrays are padded past the
// ranges read), the small arrays in 4-byte pieces.
__device__ __forceinline__ Prog<3> copy_layout_to_lds(const GProg &g, int32_t long_nnz, const LdsLayout &L,
                                                      lds_u8 *dst) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) u32x4 lds_u32x4;
    const int32_t n_words = (g.n_rows + 63) >> 6;
    lds_u64 *andb = (lds_u64 *)(dst + L.andb);
    lds_i32 *base = (lds_i32 *)(dst + L.base);
    for (int32_t i = threadIdx.x; i < n_words; i += blockDim.x) {
        andb[i] = g.words[i].and_bits;
        base[i] = g.words[i].and_base;
    }
    {
        const gp<u32x4> src = (gp<u32x4>)(const void *)g.and_len;
        lds_u32x4 *d = (lds_u32x4 *)(dst + L.len);
        for (int32_t i = threadIdx.x; i < (g.n_rows + 15) / 16; i += blockDim.x) d[i] = src[i];
    }
    {
        // the global array holds and_end entries and 64 * 16 zeros
        const int32_t n = g.and_end + 64 * 16, n4 = n / 4;
        const gp<u32x4> src = (gp<u32x4>)(const void *)g.col;
        lds_u32x4 *d = (lds_u32x4 *)(dst + L.col);
        for (int32_t i = threadIdx.x; i < n4; i += blockDim.x) d[i] = src[i];
        lds_i32 *dc = (lds_i32 *)(dst + L.col);
        for (int32_t i = 4 * n4 + (int32_t)threadIdx.x; i < n; i += blockDim.x) dc[i] = g.col[i];
    }
    lds_i32 *or_c0 = (lds_i32 *)(dst + L.or_c0);
    lds_i32 *or_row = (lds_i32 *)(dst + L.or_row);
    for (int32_t i = threadIdx.x; i <= g.n_or; i += blockDim.x) or_c0[i] = g.or_c0[i];
    for (int32_t i = threadIdx.x; i < g.n_or; i += blockDim.x) or_row[i] = g.or_row[i];
    {
        const gp<uint32_t> src = (gp<uint32_t>)(const void *)g.segs;
        lds_u32 *d = (lds_u32 *)(dst + L.segs);
        const int32_t n = g.n_segs * (int32_t)(sizeof(LongSeg) / 4);
        for (int32_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = src[i];
    }
    lds_i32 *long_col = (lds_i32 *)(dst + L.long_col);
    for (int32_t i = threadIdx.x; i < long_nnz; i += blockDim.x) long_col[i] = g.long_col[i];
    Prog<3> p;
    p.andb = andb;
    p.base = base;
    p.and_len = dst + L.len;
    p.col = (const lds_i32 *)(dst + L.col);
    p.or_c0 = or_c0;
    p.or_row = or_row;
    p.segs = (const lds_seg *)(dst + L.segs);
    p.long_col = long_col;
    p.n_rows = g.n_rows;
    p.n_or = g.n_or;
    p.n_segs = g.n_segs;
    p.and_end = g.and_end;
    return p;
}

__device__ __forceinline__ bool lds_any_in_range(const lds_u64 *v, int64_t c0, int64_t c1) {
    bool any = false;
    for (int64_t wd = c0 >> 6; wd <= (c1 - 1) >> 6; ++wd) {
        const int s = wd == (c0 >> 6) ? (int)(c0 & 63) : 0;
        const int t = wd == ((c1 - 1) >> 6) ? (int)(((c1 - 1) & 63) + 1) : 64;
        any |= (v[wd] & range_mask(s, t)) != 0;
    }
    return any;
}

// Sets bit `row` of u; returns 1 if the row is new (in neither u before nor v).
__device__ __forceinline__ uint32_t lds_set_bit(lds_u64 *u, const lds_u64 *v, int32_t row) {
    const uint64_t bit = 1ull << (row & 63);
    const uint64_t old = __hip_atomic_fetch_or(&u[row >> 6], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return (!(old & bit) && !(v[row >> 6] & bit)) ? 1u : 0u;
}

// Work of the AND stream before word w: its AND entries plus kWordWork per
// word (the per-word part of a super-block's scan, folds and results).
// Nondecreasing in w.
constexpr int64_t kWordWork = 192;

__device__ __forceinline__ int64_t stream_work(const GProg &d, int32_t w) {
    return (int64_t)d.and_base(w) + kWordWork * w;
}

// First word w in [lo, hi] with stream_work(w) >= target (hi if none before
// it): a 64-way search, one probe per lane and round (three rounds reach a
// quarter million words).
__device__ __forceinline__ int32_t first_word_at(const GProg &d, int32_t lo, int32_t hi, int64_t target) {
    const int lane = threadIdx.x & 63;
    while (lo < hi) {
        const int32_t step = (hi - lo + 63) >> 6;
        const int32_t p = min(lo + lane * step, hi);
        const uint64_t ge = __ballot(p == hi || stream_work(d, p) >= target);
        if (ge == 0) {  // every probe below hi is short of the target
            lo = __builtin_amdgcn_readfirstlane(lo + 63 * step + 1);
            continue;
        }
        const int f = (int)__builtin_ctzll(ge);
        const int32_t pf = min(lo + f * step, hi);
        if (f == 0 || step == 1) return __builtin_amdgcn_readfirstlane(f == 0 ? lo : pf);
        lo = __builtin_amdgcn_readfirstlane(lo + (f - 1) * step + 1);
        hi = __builtin_amdgcn_readfirstlane(pf);
    }
    return lo;
}

// The AND stream of member `member` of a team of `team` workgroups (one
// workgroup alone: 0 of 1), split into the workgroup's waves: the member takes
// the words from the first word whose stream_work reaches member / team of
// the program's, and wave k of its waves from the first word reaching its
// member's start plus k / waves of the member's work. Every member finds the
// same boundaries. Written to split[0..waves] by the waves themselves; the
// caller synchronizes before reading it.
__device__ __forceinline__ void split_words(const GProg &d, int32_t n_words, int32_t member, int32_t team,
                                            lds_i32 *split) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int64_t total = stream_work(d, n_words);
    const int32_t mw0 = member == 0 ? 0 : first_word_at(d, 0, n_words, total * member / team);
    const int32_t mw1 = member + 1 == team ? n_words : first_word_at(d, 0, n_words, total * (member + 1) / team);
    int32_t w = mw0;
    if (wave > 0 && mw0 < mw1) {
        const int64_t k0 = stream_work(d, mw0), k1 = stream_work(d, mw1);
        w = first_word_at(d, mw0, mw1, k0 + (k1 - k0) * wave / waves);
    }
    if (lane == 0) {
        split[wave] = w;
        if (wave == waves - 1) split[waves] = mw1;
    }
}

// Row data of a super-block of WPW words from word sbw (a multiple of 4):
// this lane's AND length in each word, four words per dword as lens4 stores
// them, and the first AND entry of the super-block's first word in the
// wave's range (the same in every lane). Loaded a super-block ahead, so
// nothing here is made wave-uniform before it is used (that would wait for
// the load at once).
template <int WPW>
struct StreamMeta {
    uint32_t lens[WPW / 4];
    int32_t b0;
};

template <int WPW>
__device__ __forceinline__ void stream_meta(const GProg &d, int32_t sbw, int32_t w_begin, StreamMeta<WPW> &m) {
    // lens4 and words carry kWordPad empty words after the last, so every
    // super-block that starts before the last word loads in bounds
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < WPW / 4; ++k) m.lens[k] = d.lens4[(int64_t)((sbw >> 2) + k) * 64 + lane];
    m.b0 = d.and_base(sbw > w_begin ? sbw : w_begin);
}

template <int WPW>
__device__ __forceinline__ int32_t stream_len(const uint32_t (&lens)[WPW / 4], int w) {
    return (int32_t)((lens[w >> 2] >> ((w & 3) * 8)) & 0xffu);
}

// The super-block being evaluated: each lane's first entry per word, its
// lengths (packed as in StreamMeta, words outside the wave's range masked to
// 0), the words' entry ranges (wave-uniform: word w covers [ws[w],
// ws[w + 1])) and this lane's AND results, one bit per word (set for the rows
// with entries, cleared by the folds).
template <int WPW>
struct StreamSb {
    int32_t st[WPW];
    int32_t ws[WPW + 1];
    uint32_t lens[WPW / 4];
    uint32_t accm;
};

// Row starts by DPP scans of the lengths: those of words 4k and 4k + 2 (and
// of 4k + 1 and 4k + 3) are scanned together as the two 16-bit halves of one
// 32-bit scan (a half's sum is at most 64 x 255 < 2^16), two scans per four
// words. Words outside [w_begin, w_end) count as empty.
template <int WPW>
__device__ __forceinline__ void stream_setup(const StreamMeta<WPW> &m, int32_t sbw, int32_t w_begin, int32_t w_end,
                                             StreamSb<WPW> &S) {
    int32_t run = __builtin_amdgcn_readfirstlane(m.b0);
    S.accm = 0;
#pragma unroll
    for (int k = 0; k < WPW / 4; ++k) {
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

// Each row-owner lane's fold of the ballot bits of its entries in the round
// [base, base + 64 U): a 32-bit window of ballot bits from the row's first
// entry (v_alignbit of two consecutive ballot dwords) against a mask of its
// length; one step for rows of up to 32 entries in a round.
template <int WPW, int U>
__device__ __forceinline__ void stream_fold(const lds_u64 *s_ball, int32_t base, StreamSb<WPW> &S) {
    const int32_t lim = base + 64 * U;
    const lds_u32 *b32 = (const lds_u32 *)s_ball;
#pragma unroll
    for (int w = 0; w < WPW; ++w) {
        if (S.ws[w + 1] <= base || S.ws[w] >= lim) continue;  // word outside the round (wave-uniform)
        int32_t lo = S.st[w] > base ? S.st[w] : base;
        const int32_t en = S.st[w] + stream_len<WPW>(S.lens, w);
        const int32_t hi = en < lim ? en : lim;
        uint32_t bad = 0;
        while (lo < hi) {
            const int32_t rel = lo - base;
            const int32_t n = hi - lo < 32 ? hi - lo : 32;
            const uint32_t win = __builtin_amdgcn_alignbit(b32[(rel >> 5) + 1], b32[rel >> 5], (uint32_t)rel);
            bad |= ~win & (0xffffffffu >> (32 - n));
            lo += n;
        }
        if (bad) S.accm &= ~(1u << w);
    }
}

// Results of a finished super-block: one LDS OR per word of the wave's range
// with AND rows that fire, and the new ones (not in v) counted in lane 0.
template <int WPW>
__device__ __forceinline__ uint32_t stream_finish(const lds_u64 *v, lds_u64 *u, int32_t sbw, int32_t w_begin,
                                                  int32_t w_end, const StreamSb<WPW> &S) {
    const int lane = threadIdx.x & 63;
    uint32_t n_new = 0;
#pragma unroll
    for (int w = 0; w < WPW; ++w) {
        const int32_t wd = sbw + w;
        if (wd < w_begin || wd >= w_end) continue;  // another wave's word (wave-uniform)
        const uint64_t res = __ballot((S.accm >> w) & 1u);
        if (res && lane == 0) {
            __hip_atomic_fetch_or(&u[wd], res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            n_new += (uint32_t)__popcll(res & ~v[wd]);
        }
    }
    return n_new;
}

// A wave's part of the AND stream: words [w_begin, w_end) (split_words), the
// first round's start `base` and the start of the round that ends at its
// last entry (rounded up to 64). w_begin == w_end if it has no AND entries.
// Fixed for a program, so found once when the program starts.
struct StreamRange {
    int32_t w_begin, w_end, base, last_base;
};

template <int U>
__device__ __forceinline__ StreamRange stream_range(const GProg &d, int32_t w_begin, int32_t w_end) {
    StreamRange R{w_begin, w_begin, 0, 0};
    if (w_begin >= w_end) return R;
    const int32_t e_begin = __builtin_amdgcn_readfirstlane(d.and_base(w_begin));
    const int32_t e_end = __builtin_amdgcn_readfirstlane(d.and_base(w_end));
    if (e_begin == e_end) return R;
    R.w_end = w_end;
    R.base = e_begin & ~63;
    R.last_base = max(R.base, ((e_end + 63) & ~63) - 64 * U);
    return R;
}

// AND rows of a layout in global memory: the wave's words [w_begin, w_end)
// (split_words) as one stream of their AND entries, a contiguous stretch of
// col, in rounds of U chunks of 64 entries (256 bytes, coalesced). The next
// round's chunks are in flight while the current one is evaluated (byte
// gathers of v from LDS, one ballot per chunk into the wave's LDS slots, one
// window fold per row); the rows are taken in super-blocks of WPW words
// aligned to 4 words (words outside the wave's range count as empty), whose
// row data is loaded a super-block ahead, and a round may finish one
// super-block and go on into the next. No round starts past the wave's last
// entry (rounded up to 64): the last one starts early instead and folds some
// entries a second time, which leaves every row's result as it was. The round
// body is written twice with the chunk buffers swapped, so no chunk register
// is copied.
template <int WPW, int U, class F>
__device__ __forceinline__ uint32_t wg_stream_rows(const GProg &d, const lds_u64 *v, lds_u64 *u, lds_u64 *s_ball,
                                                   const StreamRange &R, F &&before) {
    if (R.w_begin >= R.w_end) return before();  // no AND entries in the wave's words
    const int32_t w_begin = R.w_begin, w_end = R.w_end, last_base = R.last_base;
    const int lane = threadIdx.x & 63;
    const lds_u8 *v8 = (const lds_u8 *)v;
    int32_t base = R.base;
    int32_t sbw = w_begin & ~3;
    const int32_t sb_last = sbw + ((w_end - 1 - sbw) / WPW) * WPW;
    // every load the first round needs is issued before the other work of
    // the product (`before`), so their latencies overlap
    StreamMeta<WPW> cur, nxt;
    stream_meta<WPW>(d, sbw, w_begin, cur);
    stream_meta<WPW>(d, sbw + WPW <= sb_last ? sbw + WPW : sb_last, w_begin, nxt);
    int32_t ca[U], cb[U];
#pragma unroll
    for (int k = 0; k < U; ++k) ca[k] = d.col[base + 64 * k + lane];
    uint32_t my_new = before();
    StreamSb<WPW> S;
    stream_setup<WPW>(cur, sbw, w_begin, w_end, S);
    auto round = [&](const int32_t (&c)[U], int32_t (&cn)[U]) -> bool {
        // waves with more rounds left issue first, so the waves of the
        // workgroup finish together
        {
            const int32_t left = last_base - base;
            if (left > 3 * 64 * U) __builtin_amdgcn_s_setprio(3);
            else if (left > 2 * 64 * U) __builtin_amdgcn_s_setprio(2);
            else if (left > 64 * U) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
        const int32_t lim = base + 64 * U;
        const int32_t nb = max(base, min(lim, last_base));
#pragma unroll
        for (int k = 0; k < U; ++k) cn[k] = d.col[nb + 64 * k + lane];
        // keep the scheduler from hoisting this round's gathers (which wait
        // for its chunks) above the next round's loads
        __builtin_amdgcn_sched_barrier(0);
        // gathers in groups of at most 8 chunks (fewer registers held)
        constexpr int H = U > 8 ? 8 : U;
        static_assert(U % H == 0, "a round's chunks must fill whole gather groups");
#pragma unroll
        for (int h = 0; h < U; h += H) {
            uint32_t x[H];
#pragma unroll
            for (int k = 0; k < H; ++k) x[k] = entry_word(v8, c[h + k]);
#pragma unroll
            for (int k = 0; k < H; ++k) {
                const uint64_t B = __ballot(__builtin_amdgcn_ubfe(x[k], (uint32_t)c[h + k], 1u));
                if (lane == 0) s_ball[h + k] = B;
            }
        }
        stream_fold<WPW, U>(s_ball, base, S);
        while (S.ws[WPW] <= lim) {
            my_new += stream_finish<WPW>(v, u, sbw, w_begin, w_end, S);
            if (sbw >= sb_last) return false;
            sbw += WPW;
            stream_setup<WPW>(nxt, sbw, w_begin, w_end, S);
            stream_meta<WPW>(d, sbw + WPW <= sb_last ? sbw + WPW : sb_last, w_begin, nxt);
            stream_fold<WPW, U>(s_ball, base, S);
        }
        base = nb;
        return true;
    };
    for (;;) {
        if (!round(ca, cb)) break;
        if (!round(cb, ca)) break;
    }
    __builtin_amdgcn_s_setprio(0);
    return my_new;
}

// AND rows of a layout in LDS, one lane per row: lane l of a wave takes row
// 64 w + l of each word w the wave owns (words wave, wave + waves, ...), finds
// its first entry by a scan of the lengths in the word and walks its own
// entries, four at a time, against v in LDS; a ballot gives the word's
// result. Coalescing does not matter in LDS, and each row's chain is a few
// LDS round trips, where the streaming form of wg_block_rows (made for
// entries in global memory) costs several per super-block. NW words are in
// flight per wave.
template <int NW>
__device__ __forceinline__ uint32_t wg_and_rows_by_lane(const Prog<3> &d, const lds_u64 *v, lds_u64 *u) {
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int64_t n_words = ((int64_t)d.n_rows + 63) >> 6;
    const lds_u8 *v8 = (const lds_u8 *)v;
    uint32_t my_new = 0;
    for (int64_t w0 = threadIdx.x >> 6; w0 < n_words; w0 += (int64_t)waves * NW) {
        int32_t len[NW], pos[NW];
        bool acc[NW];
        int32_t most = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t w = w0 + (int64_t)k * waves;
            const int64_t r = w * 64 + lane;
            const bool in = w < n_words;
            len[k] = in && r < d.n_rows ? (int32_t)d.and_len[r] : 0;
            const int32_t base = in ? d.and_base(w) : 0;
            acc[k] = in && ((d.and_bits(w) >> lane) & 1ull);
            pos[k] = base + wave_exclusive_scan(len[k]);
            most = len[k] > most ? len[k] : most;
        }
        // branch-free: every lane issues all NW x 4 entry loads, then all
        // gathers (a lane past its row's end reads entry 0 and ignores it),
        // so one wait covers each group of loads
        for (int32_t j = 0; __ballot(j < most) != 0; j += 4) {
            int32_t c[NW][4];
#pragma unroll
            for (int k = 0; k < NW; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) c[k][q] = d.col[j + q < len[k] ? pos[k] + j + q : 0];
            uint32_t x[NW][4];
#pragma unroll
            for (int k = 0; k < NW; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) x[k][q] = entry_word(v8, c[k][q]);
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                uint32_t all = 1u;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    all &= (uint32_t)(j + q >= len[k]) | __builtin_amdgcn_ubfe(x[k][q], (uint32_t)c[k][q], 1u);
                acc[k] = acc[k] & (all != 0u);
            }
        }
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int64_t w = w0 + (int64_t)k * waves;
            const uint64_t res = __ballot(acc[k]);
            if (lane == 0 && w < n_words && res) {
                __hip_atomic_fetch_or(&u[w], res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                my_new += (uint32_t)__popcll(res & ~v[w]);
            }
        }
    }
    return my_new;
}

// NQ OR rows of this thread, loaded together so that their loads are in
// flight at once.
template <int NQ>
struct OrRows {
    int32_t row[NQ], c0[NQ], c1[NQ];
};

template <int NQ, class P>
__device__ __forceinline__ void or_rows_load(const P &d, int64_t j0, int64_t ostride, OrRows<NQ> &o) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t j = j0 + q * ostride;
        const bool in = j < d.n_or;
        o.row[q] = in ? d.or_row[j] : -1;
        o.c0[q] = in ? d.or_c0[j] : 0;
        o.c1[q] = in ? d.or_c0[j + 1] : 0;
    }
}

// One OR row per row index, and u starts as a subset of v: a row that fires
// is new iff v does not hold it, so the OR needs no return value.
template <int NQ>
__device__ __forceinline__ uint32_t or_rows_eval(const OrRows<NQ> &o, const lds_u64 *v, lds_u64 *u) {
    uint32_t my_new = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (o.row[q] >= 0 && lds_any_in_range(v, o.c0[q], o.c1[q])) {
            const uint64_t bit = 1ull << (o.row[q] & 63);
            __hip_atomic_fetch_or(&u[o.row[q] >> 6], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            my_new += (v[o.row[q] >> 6] & bit) ? 0u : 1u;
        }
    return my_new;
}

// OR rows (one lane each, member `member` of a team of `team` workgroups
// takes every team-th block of them) and long rows (one wave per OR segment,
// one wave per whole long AND row, looping over its segments).
template <class P>
__device__ __forceinline__ uint32_t wg_or_and_long_rows(const P &d, const lds_u64 *v, lds_u64 *u,
                                                        int32_t member, int32_t team) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const lds_u8 *v8 = (const lds_u8 *)v;
    uint32_t my_new = 0;
    const int64_t ostride = (int64_t)team * blockDim.x;
    constexpr int NQ = 4;
    for (int64_t j0 = (int64_t)member * blockDim.x + threadIdx.x; j0 < d.n_or; j0 += NQ * ostride) {
        OrRows<NQ> o;
        or_rows_load<NQ>(d, j0, ostride, o);
        my_new += or_rows_eval<NQ>(o, v, u);
    }
    for (int64_t si = (int64_t)member * waves + wave; si < d.n_segs; si += (int64_t)team * waves) {
        const auto sg = d.segs + si;
        bool fire = false;
        if (!sg->is_and) {
            bool any = false;
            const int64_t b0 = sg->begin, b1 = sg->begin + sg->len;
            for (int64_t wd = (b0 >> 6) + lane; wd <= (b1 - 1) >> 6; wd += 64) {
                const int s = wd == (b0 >> 6) ? (int)(b0 & 63) : 0;
                const int t = wd == ((b1 - 1) >> 6) ? (int)(((b1 - 1) & 63) + 1) : 64;
                any |= (v[wd] & range_mask(s, t)) != 0;
            }
            fire = __ballot(any) != 0;
        } else if (sg->seg == 0) {
            // the whole row: its nseg segments are consecutive in segs and in long_col
            bool all = true;
            int64_t total = 0;
            const int32_t nseg = sg->nseg;
            const int64_t begin = sg->begin;
            for (int q = 0; q < nseg; ++q) total += sg[q].len;
            for (int64_t i = lane; i < total; i += 64) {
                const int32_t e = d.long_col[begin + i];
                all &= __builtin_amdgcn_ubfe(entry_word(v8, e), (uint32_t)e, 1u) != 0;
            }
            fire = __ballot(!all) == 0;
        }
        if (fire && lane == 0) my_new += lds_set_bit(u, v, sg->row);
    }
    return my_new;
}

// Barrier of one team: every wave first waits for its own global stores and
// atomics to complete (a workgroup barrier does not), then the first thread
// adds 1 to *count with an agent-scope release (the workgroup's global writes
// are written back past its XCD's L2), polls with relaxed agent-scope loads
// until *count reaches target and ends with one agent-scope acquire fence.
// Bounded: after max_polls reads, or when a member has given up (*abort), it
// sets *abort and returns false in every thread of the workgroup.
__device__ __forceinline__ bool team_barrier(g_u32 *count, uint32_t target, g_u32 *abort, uint32_t max_polls,
                                             lds_u32 *s_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        for (uint32_t polls = 0;; ++polls) {
            if (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (polls >= max_polls ||
                ((polls & 63) == 63 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Algorithm 1 on one program by this workgroup alone: cur holds v_t and nxt
// v_{t-1} (both start at the facts). Returns the product count (-1 past the
// n_rows + 1 bound) and leaves the fixpoint in *fix.
template <int WPW, int U, class P>
__device__ __forceinline__ int32_t solve_alone(const P &d, lds_u64 *cur, lds_u64 *nxt, lds_u64 *my_ball,
                                               uint32_t *s_new, const StreamRange &R, lds_u64 **fix) {
    int32_t step = 1, slot = 1;  // slot = step mod 3
    uint32_t changed = 0;
    for (;;) {
        if (threadIdx.x == 0) s_new[slot == 2 ? 0 : slot + 1] = 0;
        uint32_t my_new;
        if constexpr (P::kLds) {
            my_new = wg_and_rows_by_lane<4>(d, cur, nxt);
            my_new += wg_or_and_long_rows<P>(d, cur, nxt, 0, 1);
        } else {
            // OR and long rows while the stream's first loads are in flight
            my_new = wg_stream_rows<WPW, U>(d, cur, nxt, my_ball, R,
                                            [&]() { return wg_or_and_long_rows<P>(d, cur, nxt, 0, 1); });
        }
        my_new = wave_sum(my_new);
        if ((threadIdx.x & 63) == 0 && my_new) atomicAdd(&s_new[slot], my_new);
        __syncthreads();
        changed = s_new[slot];
        if (changed == 0 || step > d.n_rows) break;
        lds_u64 *t = cur;
        cur = nxt;
        nxt = t;
        ++step;
        slot = slot == 2 ? 0 : slot + 1;
    }
    // nxt holds the last product, equal to cur at the fixpoint
    *fix = nxt;
    return changed == 0 ? step : -1;
}

// Algorithm 1 on a program small enough that every lane keeps its rows in
// registers for the whole solve: at most NW words per wave (AND rows by
// lane: the first E entries of lane l's row in each word), at most NO OR rows
// per thread, no long rows; the layout is in LDS (entries past the E-th and
// the setup read it). A row that has fired is never evaluated again (the
// interpretations only grow); it is ORed into the result buffer of the
// product that fired it and of the next one, the two buffers then both hold
// it. Per product a wave issues only the gathers of rows still false and one
// LDS OR per word, and a product changed iff some row fired. The products and
// the fixpoint are those of solve_alone.
template <int NW, int NO, int E>
__device__ __forceinline__ int32_t solve_tiny(const Prog<3> &d, lds_u64 *cur, lds_u64 *nxt, uint32_t *s_new,
                                              lds_u64 **fix) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int32_t n_words = (d.n_rows + 63) >> 6;
    int32_t ent[NW][E], len[NW], tail[NW];
    bool todo[NW], pend[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int32_t w = wave + waves * k;
        const bool in = w < n_words;
        const int32_t r = w * 64 + lane;
        const int32_t l = in && r < d.n_rows ? (int32_t)d.and_len[r] : 0;
        const int32_t pos = (in ? d.and_base(w) : 0) + wave_exclusive_scan(l);
#pragma unroll
        for (int q = 0; q < E; ++q) ent[k][q] = d.col[q < l ? pos + q : 0];
        len[k] = l;
        tail[k] = pos + E;
        // facts (true in v0, both buffers) and rows that are not AND rows are never evaluated
        todo[k] = in && ((d.and_bits(w) >> lane) & 1ull) && !((cur[in ? w : 0] >> lane) & 1ull);
        pend[k] = false;
    }
    int32_t orow[NO], oc0[NO], oc1[NO];
    bool otodo[NO], opend[NO];
#pragma unroll
    for (int m = 0; m < NO; ++m) {
        const int32_t j = (int32_t)threadIdx.x + (int32_t)blockDim.x * m;
        orow[m] = j < d.n_or ? d.or_row[j] : -1;
        oc0[m] = j < d.n_or ? d.or_c0[j] : 0;
        oc1[m] = j < d.n_or ? d.or_c0[j + 1] : 0;
        otodo[m] = orow[m] >= 0 && !((cur[orow[m] >= 0 ? orow[m] >> 6 : 0] >> (orow[m] & 63)) & 1ull);
        opend[m] = false;
    }
    int32_t step = 1, slot = 1;  // slot = step mod 3
    uint32_t changed = 0;
    for (;;) {
        if (threadIdx.x == 0) s_new[slot == 2 ? 0 : slot + 1] = 0;
        const lds_u8 *v8 = (const lds_u8 *)cur;
        bool fired = false;
#pragma unroll
        for (int m = 0; m < NO; ++m) {
            bool f = false;
            if (otodo[m]) f = lds_any_in_range(cur, oc0[m], oc1[m]);
            if (f || opend[m])
                __hip_atomic_fetch_or(&nxt[orow[m] >> 6], 1ull << (orow[m] & 63), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            opend[m] = f;
            otodo[m] = otodo[m] && !f;
            fired |= f;
        }
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int32_t w = wave + waves * k;
            if (w >= n_words) continue;
            bool f = false;
            if (__ballot(todo[k]) != 0) {
                uint32_t x[E];
#pragma unroll
                for (int q = 0; q < E; ++q) x[q] = entry_word(v8, ent[k][q]);
                uint32_t all = 1u;
#pragma unroll
                for (int q = 0; q < E; ++q) all &= (uint32_t)(q >= len[k]) | __builtin_amdgcn_ubfe(x[q], (uint32_t)ent[k][q], 1u);
                if (todo[k] && all && len[k] > E) {
                    for (int32_t i = tail[k]; i < tail[k] + len[k] - E; ++i) {
                        const int32_t c = d.col[i];
                        all &= __builtin_amdgcn_ubfe(entry_word(v8, c), (uint32_t)c, 1u);
                    }
                }
                f = todo[k] && all != 0u;
            }
            const uint64_t bits = __ballot(f || pend[k]);
            if (lane == 0 && bits)
                __hip_atomic_fetch_or(&nxt[w], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            pend[k] = f;
            todo[k] = todo[k] && !f;
            fired |= f;
        }
        if (__ballot(fired) != 0 && lane == 0) s_new[slot] = 1u;
        __syncthreads();
        changed = s_new[slot];
        if (changed == 0 || step > d.n_rows) break;
        lds_u64 *t = cur;
        cur = nxt;
        nxt = t;
        ++step;
        slot = slot == 2 ? 0 : slot + 1;
    }
    *fix = nxt;
    return changed == 0 ? step : -1;
}

}  // namespace

template <int WPW, int U>
__global__ __launch_bounds__(1024) void tp_batch_kernel(BatchParams b) {
    extern __shared__ __attribute__((aligned(16))) uint64_t s_dyn[];
    __shared__ uint64_t s_ball[kMaxWaves * (U + 1)];
    // New-bit counts by product index mod 3: the slot of product t+1 is
    // cleared during product t, after every wave has read it for product t-2,
    // so one barrier per product suffices.
    __shared__ uint32_t s_new[3];
    __shared__ int32_t s_split[kMaxWaves + 1];  // the waves' words of the AND stream (split_words)
    __shared__ int32_t s_item;
    __shared__ uint32_t s_flag;
    lds_u64 *buf0 = (lds_u64 *)s_dyn;
    lds_u64 *buf1 = buf0 + b.lds_words;
    lds_u64 *my_ball = (lds_u64 *)s_ball + (threadIdx.x >> 6) * (U + 1);
    if ((threadIdx.x & 63) == 0) my_ball[U] = 0;
    for (int32_t round = 0;; ++round) {
        if (threadIdx.x == 0) s_item = b.single ? round : (int32_t)atomicAdd(&b.queue[0], 1u);
        if (threadIdx.x < 3) s_new[threadIdx.x] = 0;
        __syncthreads();
        const int32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= b.n_items) break;
        // The descriptor tables are written by the host only, so they are read
        // through the constant address space at a wave-uniform index: scalar
        // loads, and every layout pointer stays in scalar registers.
        const ProgDesc pd = b.single ? b.one : load_desc(b.progs + as_const(b.order)[item]);
        const int32_t team = pd.team_size;
        const int32_t member = team > 1 ? as_const(b.member)[item] : 0;
        GProg d;
        d.words = as_global(pd.words);
        d.and_len = as_global(pd.and_len);
        d.lens4 = as_global(pd.lens4);
        d.col = as_global(pd.col);
        d.or_c0 = as_global(pd.or_c0);
        d.or_row = as_global(pd.or_row);
        d.segs = as_global(pd.segs);
        d.long_col = as_global(pd.long_col);
        d.n_rows = pd.n_rows;
        d.n_or = pd.n_or;
        d.n_segs = pd.n_segs;
        d.and_end = pd.and_end;
        const gp<uint64_t> fact_bits = as_global(pd.fact_bits);
        const int32_t n_words = (d.n_rows + 63) >> 6;
        // a layout that fits beside the buffers is copied into LDS once, so
        // no product reads global memory; otherwise the member's words are
        // split among the waves for the AND stream
        const LdsLayout L = lds_layout(d.n_rows, d.and_end, d.n_or, d.n_segs, pd.long_nnz);
        const bool in_lds = team == 1 && L.end <= (int64_t)b.lds_layout_bytes;
        if (!in_lds)
            split_words(d, n_words, member, team, (lds_i32 *)s_split);
        for (int32_t i = threadIdx.x; i < n_words; i += blockDim.x) {
            const uint64_t f = fact_bits[i];
            buf0[i] = f;
            buf1[i] = f;
        }
        __syncthreads();
        const StreamRange R =
            in_lds ? StreamRange{0, 0, 0, 0}
                   : stream_range<U>(d, __builtin_amdgcn_readfirstlane(s_split[threadIdx.x >> 6]),
                                     __builtin_amdgcn_readfirstlane(s_split[(threadIdx.x >> 6) + 1]));
        lds_u64 *cur = buf0, *nxt = buf1;  // cur holds v_t, nxt holds v_{t-1}
        int32_t step = 1, slot = 1;        // slot = step mod 3
        uint32_t changed = 0;
        int32_t result;
        if (team == 1) {
            lds_u64 *fix;
            if (in_lds) {
                const Prog<3> dl = copy_layout_to_lds(d, pd.long_nnz, L, (lds_u8 *)(buf1 + b.lds_words));
                __syncthreads();
                result = solve_alone<WPW, U, Prog<3>>(dl, cur, nxt, my_ball, s_new, R, &fix);
            } else {
                result = solve_alone<WPW, U, GProg>(d, cur, nxt, my_ball, s_new, R, &fix);
            }
            cur = fix;
        } else {
            g_u32 *T = (g_u32 *)pd.team;  // [0] arrivals, [1] abort, [2 + t mod 3] new bits of product t
            g_u64 *xch = (g_u64 *)pd.xch;  // three delta buffers of n_words: D[t mod 3]
            // member m clears its share of a delta buffer
            const int32_t s0 = (int32_t)((int64_t)n_words * member / team);
            const int32_t s1 = (int32_t)((int64_t)n_words * (member + 1) / team);
            // member 0 clears D[1] (product 1's) and product 1's count before the first meeting
            if (member == 0) {
                for (int32_t i = threadIdx.x; i < n_words; i += blockDim.x) xch[n_words + i] = 0ull;
                if (threadIdx.x == 0) __hip_atomic_store(&T[2 + 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            bool ok = team_barrier(&T[0], (uint32_t)team, &T[1], b.team_polls, (lds_u32 *)&s_flag);
            result = -2;
            while (ok) {
                const int nslot = slot == 2 ? 0 : slot + 1;
                // the count and delta buffer of product t+1 are cleared during
                // product t, after every member has read them for product t-2
                if (member == 0 && threadIdx.x == 0)
                    __hip_atomic_store(&T[2 + nslot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                {
                    g_u64 *Dn = xch + (int64_t)nslot * n_words;
                    for (int32_t i = s0 + (int32_t)threadIdx.x; i < s1; i += blockDim.x) Dn[i] = 0ull;
                }
                uint32_t my_new = wg_stream_rows<WPW, U>(d, cur, nxt, my_ball, R, [&]() {
                    return wg_or_and_long_rows(d, cur, nxt, member, team);
                });
                my_new = wave_sum(my_new);
                if ((threadIdx.x & 63) == 0 && my_new)
                    __hip_atomic_fetch_add(&T[2 + slot], my_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                // publish the member's new rows (not in v_{t-1}) into D[t mod 3]
                g_u64 *Ds = xch + (int64_t)slot * n_words;
                for (int32_t i = threadIdx.x; i < n_words; i += blockDim.x) {
                    const uint64_t w = nxt[i] & ~cur[i];
                    if (w) __hip_atomic_fetch_or(&Ds[i], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                ok = team_barrier(&T[0], (uint32_t)team * (uint32_t)(step + 1), &T[1], b.team_polls,
                                  (lds_u32 *)&s_flag);
                if (!ok) break;
                changed = __hip_atomic_load(&T[2 + slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (changed == 0 || step > d.n_rows) {
                    result = changed == 0 ? step : -1;
                    break;
                }
                // nxt <- v_t = v_{t-1} | D[t mod 3]; then v_t is current and v_{t-1} the older buffer
                const gp<uint64_t> Dg = Ds;
                for (int32_t i = threadIdx.x; i < n_words; i += blockDim.x) nxt[i] = cur[i] | Dg[i];
                __syncthreads();
                lds_u64 *tmp = cur;
                cur = nxt;
                nxt = tmp;
                ++step;
                slot = nslot;
            }
            // at the fixpoint cur (v_{step-1}) equals v_step
        }
        if (member == 0) {
            g_u64 *out = (g_u64 *)pd.out_bits;
            const int32_t out_words = (pd.n_atoms + 63) >> 6;
            for (int32_t i = threadIdx.x; i < out_words; i += blockDim.x) out[i] = cur[i];
            if (threadIdx.x == 0) *(g_i32 *)pd.out_products = result;
        }
        __syncthreads();  // the buffers, s_item and s_new are reused by the next program
    }
    // The last workgroup to finish rewinds the queue and clears the team
    // states for the next launch (every other workgroup has left by then).
    if (threadIdx.x == 0 && !b.single) {
        __threadfence();
        if (atomicAdd(&b.queue[1], 1u) == gridDim.x - 1) {
            for (int32_t t = 0; t < b.n_teams; ++t)
                for (int k = 0; k < 5; ++k)
                    __hip_atomic_store(&b.teams[(int64_t)t * kTeamStateWords + k], 0u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            atomicExch(&b.queue[0], 0u);
            atomicExch(&b.queue[1], 0u);
        }
    }
}

// One program that tiny_fits accepts, by one workgroup of kTinyBlock
// threads (a kernel of its own, so its registers do not weigh on the batch
// kernel): facts into both LDS buffers, layout into LDS, solve_tiny, the
// model's words and the product count out.
__global__ __launch_bounds__(kTinyBlock) void tp_tiny_kernel(ProgDesc pd, int32_t lds_words) {
    extern __shared__ __attribute__((aligned(16))) uint64_t s_dyn[];
    __shared__ uint32_t s_new[3];
    lds_u64 *buf0 = (lds_u64 *)s_dyn;
    lds_u64 *buf1 = buf0 + lds_words;
    if (threadIdx.x < 3) s_new[threadIdx.x] = 0;
    GProg d;
    d.words = as_global(pd.words);
    d.and_len = as_global(pd.and_len);
    d.lens4 = as_global(pd.lens4);
    d.col = as_global(pd.col);
    d.or_c0 = as_global(pd.or_c0);
    d.or_row = as_global(pd.or_row);
    d.segs = as_global(pd.segs);
    d.long_col = as_global(pd.long_col);
    d.n_rows = pd.n_rows;
    d.n_or = pd.n_or;
    d.n_segs = pd.n_segs;
    d.and_end = pd.and_end;
    const gp<uint64_t> fact_bits = as_global(pd.fact_bits);
    const int32_t n_words = (d.n_rows + 63) >> 6;
    for (int32_t i = threadIdx.x; i < n_words; i += blockDim.x) {
        const uint64_t f = fact_bits[i];
        buf0[i] = f;
        buf1[i] = f;
    }
    const LdsLayout L = lds_layout(d.n_rows, d.and_end, d.n_or, d.n_segs, pd.long_nnz);
    const Prog<3> dl = copy_layout_to_lds(d, pd.long_nnz, L, (lds_u8 *)(buf1 + lds_words));
    __syncthreads();
    lds_u64 *fix;
    const int32_t result = solve_tiny<kTinyWords / (kTinyBlock / 64), kTinyOr / kTinyBlock, 4>(dl, buf0, buf1,
                                                                                              s_new, &fix);
    g_u64 *out = (g_u64 *)pd.out_bits;
    const int32_t out_words = (pd.n_atoms + 63) >> 6;
    for (int32_t i = threadIdx.x; i < out_words; i += blockDim.x) out[i] = fix[i];
    if (threadIdx.x == 0) *(g_i32 *)pd.out_products = result;
}

bool tiny_fits(int64_t n_rows, int64_t n_or, int64_t n_segs) {
    return n_segs == 0 && ((n_rows + 63) >> 6) <= kTinyWords && n_or <= kTinyOr;
}

hipError_t launch_tiny(const ProgDesc &pd, int32_t lds_words, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(tp_tiny_kernel, dim3(1), dim3(kTinyBlock), lds_bytes, st, pd, lds_words);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers

#define LP_BATCH_SHAPES(X) X(4, 4) X(4, 8) X(4, 16) X(8, 8) X(8, 16)

static const void *batch_fn(int wpw, int unroll) {
#define LP_X(W, U) \
    if (wpw == W && unroll == U) return (const void *)tp_batch_kernel<W, U>;
    LP_BATCH_SHAPES(LP_X)
#undef LP_X
    return nullptr;
}

bool batch_shape_supported(int wpw, int unroll) { return batch_fn(wpw, unroll) != nullptr; }

hipError_t launch_batch(int wpw, int unroll, int grid, int block, size_t lds_bytes, const BatchParams &b,
                        hipStream_t st) {
#define LP_X(W, U)                                                                                           \
    if (wpw == W && unroll == U) {                                                                           \
        hipLaunchKernelGGL((tp_batch_kernel<W, U>), dim3(grid), dim3(block), lds_bytes, st, b);              \
        return hipGetLastError();                                                                            \
    }
    LP_BATCH_SHAPES(LP_X)
#undef LP_X
    return hipErrorInvalidValue;
}

hipError_t batch_occupancy(int wpw, int unroll, int block, size_t lds_bytes, int *blocks_per_cu) {
    const void *fn = batch_fn(wpw, unroll);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, lds_bytes);
}

void batch_kernels_allow_lds(int max_dynamic_lds) {
#define LP_X(W, U)                                                                                      \
    (void)hipFuncSetAttribute((const void *)tp_batch_kernel<W, U>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              max_dynamic_lds);
    LP_BATCH_SHAPES(LP_X)
#undef LP_X
    (void)hipFuncSetAttribute((const void *)tp_tiny_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              max_dynamic_lds);
    (void)hipGetLastError();
}

}  // namespace lp
