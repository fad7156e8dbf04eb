"""Seeded synthetic logic programs.

This module only draws random rule lists; it holds none of the fixpoint
arithmetic. Both the CPU oracle (through the tests) and the HIP engine take
its output as plain arrays, so it is the one piece of code the two share.

A program is three flat arrays, the layout the C-ABI takes:

* ``head``     int32[R]    head atom of rule r, in [0, n_atoms)
* ``body_ptr`` int64[R+1]  rule r's literals are body_lit[body_ptr[r]:body_ptr[r+1]]
* ``body_lit`` int32[L]    a >= 0 is atom a; a < 0 is "not atom (-a-1)"

Rules have the form of the paper's definite rule (equation 1) or, with
negative literals, its normal rule (Definition 6). A rule with an empty body
is a fact.

All draws use ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GEN_VERSION = 1


@dataclasses.dataclass
class Program:
    n_atoms: int
    head: np.ndarray
    body_ptr: np.ndarray
    body_lit: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_rules(self) -> int:
        return int(self.head.shape[0])

    @property
    def n_literals(self) -> int:
        return int(self.body_lit.shape[0])

    def rules(self):
        """Yield (head, [literals]) per rule; for small programs and tests."""
        for r in range(self.n_rules):
            a, b = int(self.body_ptr[r]), int(self.body_ptr[r + 1])
            yield int(self.head[r]), [int(x) for x in self.body_lit[a:b]]

    def save(self, path: str) -> None:
        np.savez(path, n_atoms=np.int64(self.n_atoms), head=self.head,
                 body_ptr=self.body_ptr, body_lit=self.body_lit,
                 gen_version=np.int64(GEN_VERSION),
                 seed=np.int64(self.meta.get("seed", -1)))


def neg(atom: int) -> int:
    """Literal code of 'not atom'."""
    return -int(atom) - 1


def from_rules(n_atoms: int, rules, **meta) -> Program:
    """Build a Program from [(head, [literal, ...]), ...]."""
    heads = np.asarray([h for h, _ in rules], dtype=np.int32)
    ptr = np.zeros(len(rules) + 1, dtype=np.int64)
    lits = []
    for r, (_, body) in enumerate(rules):
        lits.extend(int(x) for x in body)
        ptr[r + 1] = len(lits)
    return Program(n_atoms, heads, ptr, np.asarray(lits, dtype=np.int32), dict(meta))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _assemble(n_atoms, heads, lengths, body_matrix, meta) -> Program:
    """Pack per-rule bodies (first lengths[r] entries of body_matrix[r]) into CSR."""
    heads = np.asarray(heads, dtype=np.int32)
    lengths = np.asarray(lengths, dtype=np.int64)
    ptr = np.zeros(heads.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=ptr[1:])
    if body_matrix.shape[1] == 0:
        lits = np.zeros(0, dtype=np.int32)
    else:
        keep = np.arange(body_matrix.shape[1])[None, :] < lengths[:, None]
        lits = body_matrix[keep].astype(np.int32)
    return Program(int(n_atoms), heads, ptr, lits, meta)


def _draw_bodies(rng, heads, lengths, max_len, pool_size, pool_map=None):
    """Bodies drawn without replacement from a pool of atoms, excluding the head.

    Returns an int64 matrix [R, max_len]; row r's first lengths[r] entries are
    its body. Pool index k maps to atom pool_map[k] (identity if None).
    Collisions (a repeated atom or the head) are redrawn until none remain.
    """
    R = heads.shape[0]
    out = np.zeros((R, max(max_len, 0)), dtype=np.int64)
    if max_len == 0 or R == 0:
        return out
    if int(lengths.max()) > pool_size - 1:
        raise ValueError("body length exceeds the atoms available (distinct, never the head)")
    todo = np.arange(R)
    while todo.size:
        draw = rng.integers(0, pool_size, size=(todo.size, max_len))
        if pool_map is not None:
            draw = pool_map[draw]
        out[todo] = draw
        L = lengths[todo]
        valid = np.arange(max_len)[None, :] < L[:, None]
        bad = np.zeros(todo.size, dtype=bool)
        bad |= np.any(valid & (draw == heads[todo][:, None]), axis=1)
        srt = np.sort(np.where(valid, draw, -1 - np.arange(max_len)[None, :]), axis=1)
        bad |= np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        todo = todo[bad]
    return out


def definite_uniform(seed: int, n_atoms: int = 1000, n_rules: int = 2000,
                     fact_frac: float = 0.05, max_body: int = 4) -> Program:
    """Definite program: uniform heads; the first fact_frac of the rules are
    facts; every other rule has a body length uniform in 1..max_body, body
    atoms uniform without replacement and never the rule's own head.

    At the defaults this is the 1,000-atom, 2,000-rule least-model workload.
    """
    rng = _rng(seed)
    heads = rng.integers(0, n_atoms, size=n_rules)
    n_facts = int(round(fact_frac * n_rules))
    lengths = rng.integers(1, max_body + 1, size=n_rules)
    lengths[:n_facts] = 0
    # a body has distinct atoms other than its head: at most n_atoms - 1 of them
    np.minimum(lengths, max(n_atoms - 1, 0), out=lengths)
    bodies = _draw_bodies(rng, heads, lengths, max_body, n_atoms)
    return _assemble(n_atoms, heads, lengths, bodies,
                     dict(kind="definite_uniform", seed=seed, gen_version=GEN_VERSION))


def _zipf_ranks(rng, count, n, s):
    """Ranks 0..n-1 with P(k) proportional to (k+1)^-s, by inverse CDF."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(count)
    return np.minimum(np.searchsorted(cdf, u, side="right"), n - 1)


def chain_zipf(seed: int, n_atoms: int = 1_000_000, n_rules: int = 5_000_000,
               chain_len: int = 2000, fact_frac: float = 0.01, zipf_s: float = 1.1,
               max_body: int = 8) -> Program:
    """Large definite program with skewed heads and a long derivation chain.

    * chain_len atoms c_0..c_{L-1} picked by a random permutation; c_0 is a
      fact and c_i <- c_{i-1}. No other rule has a chain atom as head or in
      its body, so the synchronous fixpoint takes exactly chain_len products.
    * fact_frac * n_rules facts in total (c_0 included), on distinct uniformly
      chosen non-chain atoms.
    * every remaining rule has a head drawn from a finite Zipf(zipf_s) over the
      non-chain atoms (rank -> atom through a random permutation) and a body of
      uniform length 1..max_body over the non-chain atoms.

    At the defaults: 1,000,000 atoms, 5,000,000 rules, a 2,000-long chain.
    """
    rng = _rng(seed)
    perm = rng.permutation(n_atoms)
    chain = perm[:chain_len]
    others = perm[chain_len:]
    n_other_atoms = others.shape[0]
    n_facts = int(round(fact_frac * n_rules))
    n_chain_rules = chain_len - 1
    n_rest = n_rules - n_chain_rules - n_facts
    assert n_rest >= 0 and n_facts >= 1
    fact_heads = np.concatenate([chain[:1], rng.choice(others, size=n_facts - 1, replace=False)])
    ranks = _zipf_ranks(rng, n_rest, n_other_atoms, zipf_s)
    zperm = rng.permutation(n_other_atoms)
    rest_heads = others[zperm[ranks]]
    lengths_rest = rng.integers(1, max_body + 1, size=n_rest)
    bodies_rest = _draw_bodies(rng, rest_heads, lengths_rest, max_body, n_other_atoms, others)

    heads = np.concatenate([chain[1:], fact_heads, rest_heads])
    lengths = np.concatenate([np.ones(n_chain_rules, np.int64),
                              np.zeros(n_facts, np.int64), lengths_rest])
    bodies = np.zeros((heads.shape[0], max_body), dtype=np.int64)
    bodies[:n_chain_rules, 0] = chain[:-1]
    bodies[n_chain_rules + n_facts:] = bodies_rest
    return _assemble(n_atoms, heads, lengths, bodies,
                     dict(kind="chain_zipf", seed=seed, chain_len=chain_len,
                          gen_version=GEN_VERSION))


def batch_sizes(seed_base: int, count: int, lo: float = 1e3, hi: float = 1e5):
    """Atom counts log-uniform in [lo, hi], one per program (own seed stream)."""
    rng = _rng(seed_base ^ 0x5EED)
    return [int(round(math.exp(x))) for x in rng.uniform(math.log(lo), math.log(hi), size=count)]


def batch_programs(seed_base: int = 0, count: int = 512, lo: float = 1e3, hi: float = 1e5,
                   rule_factor: int = 2, fact_frac: float = 0.02, max_body: int = 6):
    """Many independent definite programs of uneven size: program i uses seed
    seed_base + i, n_i log-uniform in [lo, hi], rule_factor * n_i rules,
    fact_frac facts, uniform heads, bodies of length 1..max_body."""
    sizes = batch_sizes(seed_base, count, lo, hi)
    return [definite_uniform(seed_base + i, n, rule_factor * n, fact_frac, max_body)
            for i, n in enumerate(sizes)]


def _negate_some(rng, prog: Program, neg_atoms, p_neg: float, max_neg: int) -> Program:
    """Replace body literals by negations of atoms from neg_atoms.

    Each rule with a non-empty body, with probability p_neg, has c ~ U{1..max_neg}
    (at most its body length) of its body literals replaced by 'not q' with the
    q distinct members of neg_atoms, q != head and q not positive in that body.
    """
    neg_atoms = np.asarray(neg_atoms, dtype=np.int64)
    lit = prog.body_lit.astype(np.int64).copy()
    R = prog.n_rules
    pick = rng.random(R) < p_neg
    for r in np.nonzero(pick)[0]:
        a, b = int(prog.body_ptr[r]), int(prog.body_ptr[r + 1])
        L = b - a
        if L == 0:
            continue
        c = min(int(rng.integers(1, max_neg + 1)), L)
        body = set(int(x) for x in lit[a:b])
        cand = [int(q) for q in neg_atoms if q != prog.head[r] and q not in body]
        if len(cand) < c:
            continue
        qs = rng.choice(np.asarray(cand), size=c, replace=False)
        slots = rng.choice(L, size=c, replace=False)
        for s, q in zip(slots, qs):
            lit[a + s] = -int(q) - 1
    return Program(prog.n_atoms, prog.head, prog.body_ptr, lit.astype(np.int32), dict(prog.meta))


def _negate_some_vec(rng, prog: Program, neg_atoms, p_neg: float, max_neg: int,
                     tries: int = 32) -> Program:
    """Array form of _negate_some for large programs (same constraints, other
    draws): each rule with a non-empty body, with probability p_neg, gets
    c ~ U{1..max_neg} (at most its body length) negations 'not q', q taken
    from neg_atoms as c consecutive entries from a random start, placed in c
    consecutive body slots (cyclically) from a random start; q != head and q
    not positive in the original body, redrawing the start up to `tries`
    times, else the rule keeps its positive body."""
    Q = np.asarray(neg_atoms, dtype=np.int64)
    K = Q.shape[0]
    lit = prog.body_lit.astype(np.int64).copy()
    if K == 0:
        return Program(prog.n_atoms, prog.head, prog.body_ptr, lit.astype(np.int32), dict(prog.meta))
    bp = prog.body_ptr.astype(np.int64)
    L = np.diff(bp)
    R = prog.n_rules
    pick = np.nonzero((rng.random(R) < p_neg) & (L > 0))[0]
    c = np.minimum(np.minimum(rng.integers(1, max_neg + 1, size=pick.shape[0]), L[pick]), K)
    Lm = int(L.max()) if R else 0
    body = np.full((pick.shape[0], max(Lm, 1)), -1, dtype=np.int64)
    for j in range(Lm):
        has = L[pick] > j
        body[has, j] = lit[bp[pick[has]] + j]
    head = prog.head.astype(np.int64)[pick]
    t0 = rng.integers(0, K, size=pick.shape[0])
    ok = np.zeros(pick.shape[0], dtype=bool)
    todo = np.arange(pick.shape[0])
    for _ in range(tries):
        if todo.shape[0] == 0:
            break
        good = np.ones(todo.shape[0], dtype=bool)
        for j in range(max_neg):
            act = c[todo] > j
            q = Q[(t0[todo] + j) % K]
            bad = (q == head[todo]) | (body[todo] == q[:, None]).any(axis=1)
            good &= ~(act & bad)
        ok[todo[good]] = True
        todo = todo[~good]
        t0[todo] = rng.integers(0, K, size=todo.shape[0])
    s0 = (rng.random(pick.shape[0]) * L[pick]).astype(np.int64)
    for j in range(max_neg):
        act = ok & (c > j)
        r = pick[act]
        slot = (s0[act] + j) % L[r]
        lit[bp[r] + slot] = -Q[(t0[act] + j) % K] - 1
    return Program(prog.n_atoms, prog.head, prog.body_ptr, lit.astype(np.int32), dict(prog.meta))


def normal_uniform(seed: int, n_atoms: int = 10_000, n_rules: int = 20_000, max_body: int = 5,
                   k_neg: int = 16, p_neg: float = 0.1, max_neg: int = 2,
                   fact_frac: float = 0.0, vectorized: bool = False) -> Program:
    """Normal program with k_neg atoms appearing negated.

    Uniform heads, bodies of length 1..max_body (fact_frac of the rules are
    facts), then k_neg uniformly chosen atoms Q and negations placed by
    _negate_some. Redrawn (next sub-seed) until every atom of Q occurs
    negated, so exactly k_neg atoms are negated and there are 2^k_neg guesses.

    At the defaults: 10,000 atoms, 20,000 rules, 16 negated atoms (65,536 guesses).
    vectorized=True places the negations with _negate_some_vec (for large programs).
    """
    attempt = 0
    while True:
        rng = _rng(seed * 1000 + attempt)
        base = definite_uniform(int(rng.integers(0, 2**62)), n_atoms, n_rules, fact_frac, max_body)
        Q = rng.choice(n_atoms, size=k_neg, replace=False) if k_neg > 0 else np.zeros(0, np.int64)
        prog = (_negate_some_vec if vectorized else _negate_some)(rng, base, Q, p_neg, max_neg)
        negs = np.unique(-prog.body_lit[prog.body_lit < 0].astype(np.int64) - 1)
        if negs.shape[0] == k_neg:
            prog.meta = dict(kind="normal_uniform", seed=seed, k_neg=k_neg, attempt=attempt,
                             gen_version=GEN_VERSION)
            return prog
        attempt += 1


def even_loops(n_loops: int) -> Program:
    """n independent even loops {a_i <- not b_i, b_i <- not a_i}: 2^n stable models."""
    rules = []
    for i in range(n_loops):
        a, b = 2 * i, 2 * i + 1
        rules.append((a, [neg(b)]))
        rules.append((b, [neg(a)]))
    return from_rules(2 * n_loops, rules, kind="even_loops", n_loops=n_loops)


def odd_loop() -> Program:
    """a <- not a: no stable model."""
    return from_rules(1, [(0, [neg(0)])], kind="odd_loop")


def transitive_closure(n_vertices: int, edges, grounding: str = "edges") -> Program:
    """Ground path/edge program: path(x,y) <- edge(x,y);
    path(x,y) <- edge(x,z) and path(z,y).

    Atom edge(x,y) = x*V + y, path(x,y) = V*V + x*V + y. Edge atoms are facts.
    grounding "edges" instantiates the rules only where edge(x, .) is a fact;
    "all" instantiates them for every x, y, z (V^3 + V^2 rules), the naive
    grounding whose matrix sizes match the transitive-closure table of the
    paper's section 4 (n' about V^3).
    """
    V = n_vertices
    E = V * V

    def e(x, y):
        return x * V + y

    def p(x, y):
        return E + x * V + y

    if grounding == "all":
        xs, ys = np.meshgrid(np.arange(V), np.arange(V), indexing="ij")
        xs, ys = xs.ravel(), ys.ravel()
        ed = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
        n_e = ed.shape[0]
        heads = [ed[:, 0] * V + ed[:, 1], E + xs * V + ys]               # facts, base rules
        bodies = [np.zeros((n_e, 2), np.int64), np.stack([xs * V + ys, np.zeros_like(xs)], 1)]
        lengths = [np.zeros(n_e, np.int64), np.ones(V * V, np.int64)]
        x3, z3, y3 = (a.ravel() for a in np.meshgrid(np.arange(V), np.arange(V), np.arange(V), indexing="ij"))
        heads.append(E + x3 * V + y3)
        bodies.append(np.stack([x3 * V + z3, E + z3 * V + y3], 1))
        lengths.append(np.full(V ** 3, 2, np.int64))
        return _assemble(2 * E, np.concatenate(heads), np.concatenate(lengths), np.concatenate(bodies),
                         dict(kind="transitive_closure", n_vertices=V, grounding="all"))
    if grounding != "edges":
        raise ValueError("grounding is 'edges' or 'all'")
    rules = []
    for (x, y) in edges:
        rules.append((e(x, y), []))
    for (x, y) in edges:
        rules.append((p(x, y), [e(x, y)]))
    for (x, z) in edges:
        for y in range(V):
            rules.append((p(x, y), [e(x, z), p(z, y)]))
    return from_rules(2 * E, rules, kind="transitive_closure", n_vertices=V)


# Body-length proportions of the non-fact rules in the paper's random
# programs (section 4, the table of rule proportions by body length 1..8).
PAPER_BODY_PROPORTIONS = (0.04, 0.04, 0.10, 0.40, 0.35, 0.04, 0.02, 0.01)


def paper_definite(seed: int, n_atoms: int, n_rules: int) -> Program:
    """Random definite program shaped like the paper's section 4 experiments:
    n = |B_P| atoms, m = |P| rules; fewer than n/3 facts (read as a count:
    floor((n - 1) / 3) fact rules with distinct heads); the other rules have
    uniform heads and body lengths 1..8 in the proportions of
    PAPER_BODY_PROPORTIONS (counts rounded, the remainder to length 4), body
    atoms distinct and never the head.
    """
    rng = _rng(seed)
    n_facts = min((n_atoms - 1) // 3, n_rules)
    n_body = n_rules - n_facts
    counts = [int(math.floor(q * n_body)) for q in PAPER_BODY_PROPORTIONS]
    counts[3] += n_body - sum(counts)
    lengths = np.concatenate([np.zeros(n_facts, np.int64)] +
                             [np.full(c, L + 1, np.int64) for L, c in enumerate(counts)])
    rng.shuffle(lengths[n_facts:])
    heads = np.concatenate([rng.permutation(n_atoms)[:n_facts],
                            rng.integers(0, n_atoms, size=n_body)]).astype(np.int64)
    np.minimum(lengths, max(n_atoms - 1, 0), out=lengths)
    bodies = _draw_bodies(rng, heads, lengths, 8, n_atoms)
    return _assemble(n_atoms, heads, lengths, bodies,
                     dict(kind="paper_definite", seed=seed, gen_version=GEN_VERSION))


def paper_normal(seed: int, n_atoms: int, n_rules: int, k: int) -> Program:
    """paper_definite with k body literals (distinct positions, uniform over
    all body literals) changed to negations, as in the paper's normal
    programs (4 <= k <= 8). The negated atoms are the atoms at those
    positions, so K <= k distinct atoms appear negated.
    """
    prog = paper_definite(seed, n_atoms, n_rules)
    rng = _rng(seed + 0x5EED)
    lits = prog.body_lit.copy()
    if k > lits.shape[0]:
        raise ValueError("more negations than body literals")
    pos = rng.choice(lits.shape[0], size=k, replace=False)
    lits[pos] = -lits[pos] - 1
    meta = dict(prog.meta, kind="paper_normal", k=k)
    return Program(prog.n_atoms, prog.head, prog.body_ptr, lits, meta)


def random_graph_edges(seed: int, n_vertices: int, n_edges: int):
    rng = _rng(seed)
    seen = set()
    while len(seen) < n_edges:
        x, y = (int(t) for t in rng.integers(0, n_vertices, size=2))
        if x != y:
            seen.add((x, y))
    return sorted(seen)


def tiny_random(seed: int, max_atoms: int = 16, max_rules: int = 40, max_body: int = 4,
                p_neg: float = 0.0, allow_dups: bool = True) -> Program:
    """Small messy programs for brute-force comparison: shared heads, facts,
    repeated body atoms (when allow_dups), h <- h, atoms with no rule, and
    (if p_neg > 0) negative literals, including 'b and not b' in one body."""
    rng = _rng(seed)
    n = int(rng.integers(1, max_atoms + 1))
    R = int(rng.integers(0, max_rules + 1))
    rules = []
    for _ in range(R):
        h = int(rng.integers(0, n))
        L = int(rng.integers(0, max_body + 1))
        body = []
        for _ in range(L):
            a = int(rng.integers(0, n))
            if not allow_dups and a in body:
                continue
            body.append(neg(a) if rng.random() < p_neg else a)
        rules.append((h, body))
    return from_rules(n, rules, kind="tiny_random", seed=seed)


def serving_pool(seed: int = 0, count: int = 256, lo: float = 1e3, hi: float = 1e6,
                 rule_factor: int = 3, max_body: int = 6, fact_frac: float = 0.02,
                 max_k: int = 12, p_neg: float = 0.1, max_neg: int = 2, progress=None):
    """Pool of request programs: n log-uniform in [lo, hi], rule_factor*n rules,
    bodies 1..max_body, fact_frac facts, k ~ U{0..max_k} negated atoms
    (k = 0 gives a least-model query, k > 0 a stable-model query).
    progress (nullable) is called with the number of programs drawn so far."""
    rng = _rng(seed ^ 0xC5C5)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        k = int(rng.integers(0, max_k + 1))
        sub = seed * 100_003 + i
        if k == 0:
            out.append(definite_uniform(sub, n, rule_factor * n, fact_frac, max_body))
        else:
            out.append(normal_uniform(sub, n, rule_factor * n, max_body, k, p_neg, max_neg,
                                      fact_frac, vectorized=True))
        if progress is not None:
            progress(i + 1)
    return out
