"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Each ``check_*`` takes an ``oracle.Oracle`` and raises AssertionError on a
mismatch.  They are run on the real oracle (test_oracle_pins.py) and on
copies of it with planted mistakes (test_oracle_mutants.py), which must each
fail at least one of them.

What pins what:
  - hand-worked golden cases (tests/golden): overlap counts, features, exact
    scores at z = 0, NW totals, paths and emitted pairs, including both tie
    rules and threshold equality;
  - overlap counts against a brute-force Python-set statement of the
    definitions on random tiny documents;
  - NW against exhaustive enumeration of every monotone path (Delannoy many)
    for n, m <= 6, folded left to right in float32 -- the DP value must equal
    the best fold bit for bit for any float input, and with dyadic inputs the
    traced path must be the lexicographically smallest optimal path read
    backwards with D < U < L;
  - NW with 0/1 scores and zero gap against LCS length from the bit-parallel
    algorithm of Allison & Dix / Hyyro (an independent routine);
  - closed forms: constant score matrices, sigmoid values via tanh;
  - invariants: path validity, threshold subsets, gap monotonicity (exchange
    argument), transposition without ties, identity documents, denormals and
    empty inputs.
"""
from __future__ import annotations

import json
import math
import os
from functools import lru_cache

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F32 = np.float32


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------- helpers
@lru_cache(None)
def all_paths(n: int, m: int) -> tuple:
    """Every forward move string from (0,0) to (n,m) over D (1,1), U (1,0), L (0,1)."""
    if n == 0 and m == 0:
        return ("",)
    out = []
    if n > 0 and m > 0:
        out += [p + "D" for p in all_paths(n - 1, m - 1)]
    if n > 0:
        out += [p + "U" for p in all_paths(n - 1, m)]
    if m > 0:
        out += [p + "L" for p in all_paths(n, m - 1)]
    return tuple(out)


def delannoy(n, m):
    return sum(math.comb(m, k) * math.comb(n, k) * 2 ** k for k in range(min(n, m) + 1))


def folds(S: np.ndarray, g, paths) -> np.ndarray:
    """float32 left fold of every path (0 + step1 + step2 + ...), vectorised over paths."""
    g = F32(g)
    P = len(paths)
    L = max((len(p) for p in paths), default=0)
    steps = np.zeros((P, L), np.float32)
    for k, p in enumerate(paths):
        i = j = 0
        for t, c in enumerate(p):
            if c == "D":
                steps[k, t] = S[i, j]
                i += 1
                j += 1
            elif c == "U":
                steps[k, t] = g
                i += 1
            else:
                steps[k, t] = g
                j += 1
    v = np.zeros(P, np.float32)
    for t in range(L):
        v = (v + steps[:, t]).astype(np.float32)  # adding +0 to padded slots is exact
    return v


def path_end(moves):
    i = j = 0
    for c in moves:
        if c == "D":
            i += 1
            j += 1
        elif c == "U":
            i += 1
        else:
            j += 1
    return i, j


def lcs_bitparallel(a, b) -> int:
    """LCS length by the bit-vector recurrence V' = (V + (V & M)) | (V & ~M)."""
    n = len(a)
    if n == 0:
        return 0
    full = (1 << n) - 1
    M = {}
    for i, c in enumerate(a):
        M[c] = M.get(c, 0) | (1 << i)
    V = full
    for c in b:
        Mc = M.get(c, 0)
        U = V & Mc
        V = ((V + U) | (V & ~Mc)) & full
    return n - bin(V).count("1")


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- overlap
def check_overlap_hand(O):
    G = _gold("overlap_hand_example.json")
    lx = G["lexicon"]
    L = O.lexicon(lx["src_ids"], lx["off"], lx["tgt_ids"])
    S, ms, mt = O.similarity(L, [G["src"]], [G["tgt"]], [0, 0, 0, 0])
    assert int(ms[0, 0]) == G["m_s"], (ms, G["m_s"])
    assert int(mt[0, 0]) == G["m_t"], (mt, G["m_t"])
    for c in G["score_cases"]:
        S, _, _ = O.similarity(L, [G["src"]], [G["tgt"]], c["w"])
        assert S[0, 0] == F32(c["S"]), (c, S)


def _py_counts(T, s, t):
    X = set()
    for x in s:
        X |= T.get(x, set())
    tset = set(t)
    mt = sum(1 for y in t if y in X)
    ms = sum(1 for x in s if T.get(x, set()) & tset)
    return ms, mt


def check_overlap_bruteforce(O, n_cases=40):
    r = rng(7)
    for case in range(n_cases):
        V = int(r.integers(4, 14))
        keys = r.choice(V + 3, size=int(r.integers(1, V + 3)), replace=False)  # some keys never occur
        src_ids, off, tgt = [], [0], []
        T = {}
        for k in keys:
            cnt = int(r.integers(0, 4))
            ys = [int(y) for y in r.integers(0, V, size=cnt)]  # duplicates allowed in the listing
            src_ids.append(int(k))
            tgt += ys
            off.append(len(tgt))
            T.setdefault(int(k), set()).update(ys)
        # repeat one key to exercise merging
        if len(keys) and r.random() < 0.5:
            k = int(keys[0])
            ys = [int(y) for y in r.integers(0, V, size=2)]
            src_ids.append(k)
            tgt += ys
            off.append(len(tgt))
            T.setdefault(k, set()).update(ys)
        L = O.lexicon(np.array(src_ids, np.int32), np.array(off, np.int64), np.array(tgt, np.int32))
        n, m = int(r.integers(0, 5)), int(r.integers(0, 5))
        src = [list(map(int, r.integers(0, V, size=int(r.integers(0, 7))))) for _ in range(n)]
        tg = [list(map(int, r.integers(0, V, size=int(r.integers(0, 7))))) for _ in range(m)]
        S, ms, mt = O.similarity(L, src, tg, [0, 0, 0, 0])
        for i in range(n):
            for j in range(m):
                e_ms, e_mt = _py_counts(T, src[i], tg[j])
                assert (int(ms[i, j]), int(mt[i, j])) == (e_ms, e_mt), (case, i, j, src[i], tg[j], T)


def check_score_closed_forms(O):
    # z = 0 exactly -> 0.5 exactly; each case isolates one feature
    cases = [
        ((-1.5, 2, 0, 0), (3, 4, 1, 4)),    # f1 = 3/4 only (f2 = 1/4 must not enter)
        ((-1.5, 0, 2, 0), (1, 4, 3, 4)),    # f2 = 3/4 only
        ((-0.5, 0, 0, 1), (0, 2, 0, 4)),    # f3 = min/max = 2/4
        ((-0.5, 0, 0, 1), (0, 4, 0, 2)),    # f3 symmetric in a, b
        ((0.0, 5, 5, 5), (0, 0, 0, 0)),     # empty sentences: all features 0
        ((-1.0, 1, 0, 0), (3, 3, 0, 7)),    # f1 = 1
    ]
    for w, (ms, a, mt, b) in cases:
        s = O.score(np.array(w, np.float32), ms, a, mt, b)
        assert s == F32(0.5), (w, ms, a, mt, b, s)
    # sign and value of the logistic: S(z0) = (1 + tanh(z0/2)) / 2
    for z0 in (2.0, -3.0, 0.75, 6.5, -20.0):
        s = O.score(np.array([z0, 0, 0, 0], np.float32), 0, 1, 0, 1)
        want = F32((1.0 + math.tanh(z0 / 2.0)) / 2.0)
        assert abs(int(np.float32(s).view(np.int32)) - int(want.view(np.int32))) <= 1, (z0, s, want)
    # S(-w) = 1 - S(w) (z negates exactly), within one ulp
    r = rng(3)
    for _ in range(50):
        w = r.normal(0, 3, 4).astype(np.float32)
        a, b = int(r.integers(1, 30)), int(r.integers(1, 30))
        ms, mt = int(r.integers(0, a + 1)), int(r.integers(0, b + 1))
        s1 = O.score(w, ms, a, mt, b)
        s2 = O.score(-w, ms, a, mt, b)
        assert abs(float(s1) + float(s2) - 1.0) <= 1.2e-7, (w, s1, s2)
    # monotone in each overlap count when its weight is positive
    w = np.array([-3, 2, 2, 1], np.float32)
    prev = -1.0
    for ms in range(0, 11):
        s = float(O.score(w, ms, 10, 4, 10))
        assert s >= prev
        prev = s


# --------------------------------------------------------------------- NW
def check_nw_hand(O):
    G = _gold("nw_hand_examples.json")
    for c in G["cases"]:
        S = np.array(c["S"], np.float32)
        h, mv, _ = O.nw(S, c["g"])
        assert h == F32(c["H"]), (c["name"], h)
        assert mv == c["moves"], (c["name"], mv)
        si, ti, sc = O.emit(S, mv, c["tau"])
        got = [[int(a), int(b), float(s)] for a, b, s in zip(si, ti, sc)]
        assert got == c["emitted"], (c["name"], got)


def check_nw_bruteforce(O, n_cases=60, max_dim=6, seed=11):
    r = rng(seed)
    assert len(all_paths(6, 6)) == delannoy(6, 6) == 8989
    for case in range(n_cases):
        n, m = int(r.integers(0, max_dim + 1)), int(r.integers(0, max_dim + 1))
        kind = case % 3
        if kind == 0:
            S = r.random((n, m)).astype(np.float32)
            g = F32(-r.random() * 0.6)
        elif kind == 1:
            S = r.normal(0.3, 0.5, (n, m)).astype(np.float32)  # arbitrary float scores, negative too
            g = F32(-0.2)
        else:
            S = (r.integers(0, 9, (n, m)) / 8.0).astype(np.float32)
            g = F32(-0.25)
        h, mv, H = O.nw(S, g, want_H=True)
        P = all_paths(n, m)
        v = folds(S, g, P)
        best = v.max()
        assert h == best and h.tobytes() == best.tobytes(), (case, n, m, h, best)
        # the traced path is a valid monotone path whose fold is the optimum
        assert path_end(mv) == (n, m)
        assert mv.count("D") + mv.count("U") == n and mv.count("D") + mv.count("L") == m
        assert folds(S, g, [mv])[0] == h
        # every prefix of the traced path is optimal for its end cell
        for k in range(len(mv) + 1):
            i, j = path_end(mv[:k])
            assert folds(S, g, [mv[:k]])[0] == H[i, j], (case, k)
        # H itself: every cell equals the brute-force optimum of its sub-problem
        if n <= 4 and m <= 4:
            for i in range(n + 1):
                for j in range(m + 1):
                    assert H[i, j] == folds(S, g, all_paths(i, j)).max()


def check_tie_rule_dyadic(O, n_cases=80, seed=5):
    order = {"D": 0, "U": 1, "L": 2}
    r = rng(seed)
    for case in range(n_cases):
        n, m = int(r.integers(1, 7)), int(r.integers(1, 7))
        S = (r.integers(0, 3, (n, m)) / 4.0).astype(np.float32)  # many exact ties
        g = F32(-0.25 * int(r.integers(0, 3)))
        h, mv, _ = O.nw(S, g)
        P = all_paths(n, m)
        v = folds(S, g, P)
        opt = [p for p, x in zip(P, v) if x == v.max()]
        want = min(opt, key=lambda p: [order[c] for c in reversed(p)])
        assert mv == want, (case, S.tolist(), float(g), mv, want, len(opt))


def check_lcs(O, n_cases=40, seed=13):
    r = rng(seed)
    for case in range(n_cases):
        la, lb = int(r.integers(0, 40)), int(r.integers(0, 40))
        k = int(r.integers(2, 6))
        a = list(map(int, r.integers(0, k, la)))
        b = list(map(int, r.integers(0, k, lb)))
        S = np.array([[1.0 if x == y else 0.0 for y in b] for x in a], np.float32).reshape(la, lb)
        h, mv, _ = O.nw(S, 0.0)
        assert int(h) == lcs_bitparallel(a, b) and float(h) == int(h), (case, h)


def check_constant_closed_form(O):
    for n in range(0, 9):
        for m in range(0, 9):
            for c, g in ((0.375, -0.25), (0.0, -0.125), (1.0, -0.5), (0.5, -0.125)):
                S = np.full((n, m), c, np.float32)
                h, mv, _ = O.nw(S, g)
                want = min(n, m) * c + abs(n - m) * g
                assert h == F32(want), (n, m, c, g, h, want)
                assert mv.count("D") == min(n, m)


# --------------------------------------------------------------- invariants
def check_threshold_and_edges(O):
    # equality accepted, the float just below rejected
    below = np.nextafter(F32(0.5), F32(0.0))
    S = np.array([[0.5, 0.0], [0.0, below]], np.float32)
    h, mv, _ = O.nw(S, -0.25)
    assert mv == "DD"
    si, ti, sc = O.emit(S, mv, 0.5)
    assert list(zip(si.tolist(), ti.tolist())) == [(0, 0)]
    # denormal scores are kept, not flushed
    d = F32(1e-40)
    assert 0 < d < np.finfo(np.float32).tiny
    h, mv, H = O.nw(np.array([[d]], np.float32), -0.5, want_H=True)
    assert h.tobytes() == d.tobytes() and mv == "D"
    si, ti, sc = O.emit(np.array([[d]], np.float32), mv, 0.0)
    assert sc.tobytes() == d.tobytes()
    # empty documents: an all-gap path and no pairs; boundary by repeated addition
    g = F32(-0.2)
    # (for g = -0.2f, 7*g differs from g+g+...+g in float32, so long boundaries tell them apart)
    for n, m in ((0, 0), (0, 5), (4, 0), (0, 12), (9, 0), (20, 1)):
        h, mv, _ = O.nw(np.zeros((n, m), np.float32), g)
        acc = F32(0.0)
        for _ in range(n + m):
            acc = F32(acc + g)
        if n == 0 or m == 0:
            assert h.tobytes() == acc.tobytes() and len(mv) == n + m and "D" not in mv
        si, _, _ = O.emit(np.zeros((n, m), np.float32), mv, 0.5)
        assert si.size == 0


def check_invariants(O, n_cases=40, seed=17):
    r = rng(seed)
    for case in range(n_cases):
        n, m = int(r.integers(1, 30)), int(r.integers(1, 30))
        S = r.random((n, m)).astype(np.float32)
        g = F32(-r.random() * 0.5)
        h, mv, _ = O.nw(S, g)
        assert mv.count("D") + mv.count("U") == n and mv.count("D") + mv.count("L") == m
        si, ti, sc = O.emit(S, mv, 0.5)
        assert np.all(np.diff(si) > 0) and np.all(np.diff(ti) > 0)
        assert np.all(sc >= F32(0.5)) and np.all(S[si, ti] == sc)
        # raising tau keeps a subset of the pairs, the path does not depend on tau
        si2, ti2, _ = O.emit(S, mv, 0.8)
        assert set(zip(si2.tolist(), ti2.tolist())) <= set(zip(si.tolist(), ti.tolist()))
    # gap monotonicity (exact arithmetic: dyadic scores and gaps)
    for case in range(n_cases):
        n, m = int(r.integers(1, 25)), int(r.integers(1, 25))
        S = (r.integers(0, 17, (n, m)) / 16.0).astype(np.float32)
        prev = None
        for g in (-0.0625, -0.125, -0.25, -0.5, -1.0):
            _, mv, _ = O.nw(S, g)
            gaps = mv.count("U") + mv.count("L")
            if prev is not None:
                assert gaps <= prev, (case, g, gaps, prev)
            prev = gaps
    # transposition: where the optimum is unique, NW on S^T traces the transposed path
    swap = str.maketrans("UL", "LU")
    done = 0
    for case in range(200):
        n, m = int(r.integers(1, 6)), int(r.integers(1, 6))
        S = r.random((n, m)).astype(np.float32)
        g = F32(-0.3)
        v = folds(S, g, all_paths(n, m))
        if (v == v.max()).sum() != 1:
            continue
        _, mv, _ = O.nw(S, g)
        _, mvT, _ = O.nw(np.ascontiguousarray(S.T), g)
        assert mvT == mv.translate(swap), (S, mv, mvT)
        done += 1
    assert done > 50


def check_identity_document(O, synth_mod, n_docs=3):
    """A document aligned with its exact translation recovers the diagonal."""
    cfg = synth_mod.Config("identity", vocab=3000, zipf_s=1.1, len_min=5, len_max=30, count_kind=0,
                           n_fixed=30, m_fixed=30, plant_frac=1.0, replace_p=0.0, indel_max=0,
                           primary_only=1, lex_translated=3000, lex_kmin=1, lex_kmax=3,
                           lex_pairs=0, n_pairs=n_docs, seed_offset=90)
    lex = synth_mod.make_lexicon(cfg)
    c = synth_mod.generate(cfg, lex)
    w = synth_mod.weights(synth_mod.CONFIGS[1].seed)
    L = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    for p in range(c.n_pairs):
        src, tgt = c.pair(p)
        S, ms, mt = O.similarity(L, src, tgt, w)
        n = len(src)
        # precondition: every sentence is fully covered by its translation and scores above tau
        assert all(int(ms[i, i]) == len(src[i]) and int(mt[i, i]) == len(tgt[i]) for i in range(n))
        assert np.all(np.diag(S) >= F32(0.5))
        h, mv, _ = O.nw(S, -0.2)
        assert mv == "D" * n, mv
        si, ti, _ = O.emit(S, mv, 0.5)
        assert si.tolist() == list(range(n)) and ti.tolist() == list(range(n))


def check_mine_composition(O, synth_mod):
    cfg = synth_mod.config(1, n_pairs=6, cmin=0, cmax=12)
    lex = synth_mod.make_lexicon(cfg)
    c = synth_mod.generate(cfg, lex)
    w = synth_mod.weights(cfg.seed)
    L = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    res = O.mine(L, c, w, -0.2, 0.5, want_S=True)
    base = 0
    for p in range(c.n_pairs):
        src, tgt = c.pair(p)
        S, _, _ = O.similarity(L, src, tgt, w)
        assert np.array_equal(S.reshape(-1), res["S"][base:base + S.size])
        base += S.size
        h, mv, _ = O.nw(S, -0.2)
        si, ti, sc = O.emit(S, mv, 0.5)
        a, b = res["pair_off"][p], res["pair_off"][p + 1]
        assert res["align_score"][p] == h
        assert np.array_equal(res["src_idx"][a:b], si) and np.array_equal(res["tgt_idx"][a:b], ti)


ALL = [
    check_overlap_hand, check_overlap_bruteforce, check_score_closed_forms, check_nw_hand,
    check_nw_bruteforce, check_tie_rule_dyadic, check_lcs, check_constant_closed_form,
    check_threshold_and_edges, check_invariants,
]


# ------------------------------------------------------------ A* (monotone)
def astar_monotone(S, g):
    """Best-first (A*) search for the best monotone alignment path.

    Section 4 notes that A* gives the NW result only when paths may not go up
    or left; this search walks the same DAG (moves D, U, L only).  Scores are
    turned into non-negative step costs that do not depend on path length:
    every path makes n + m units of progress (D counts 2, U and L count 1),
    and score = g(n+m) + sum over D of (S - 2g).  With K = (smax - 2g)/2,
    cost(D) = 2K - (S - 2g) >= 0 and cost(U) = cost(L) = K give
    cost = K(n+m) - (score - g(n+m)), so the cheapest path is the best one.
    Heuristic: K per unit of remaining progress minus the most a diagonal step
    could save, which never overestimates.  Exact in dyadic arithmetic.
    """
    import heapq
    S = np.asarray(S, dtype=np.float64)
    n, m = S.shape
    g = float(g)
    smax = float(S.max()) if S.size else 0.0
    K = max((smax - 2 * g) / 2.0, 0.0)
    gain = max(smax - 2 * g, 0.0)

    def h(i, j):
        rem_d = min(n - i, m - j)
        return K * ((n - i) + (m - j)) - rem_d * gain

    best = {(0, 0): 0.0}
    pq = [(h(0, 0), 0.0, 0, 0)]
    while pq:
        f, c, i, j = heapq.heappop(pq)
        if c > best.get((i, j), float("inf")):
            continue
        if (i, j) == (n, m):
            return g * (n + m) + (K * (n + m) - c)
        for di, dj in ((1, 1), (1, 0), (0, 1)):
            a, b = i + di, j + dj
            if a > n or b > m:
                continue
            step = 2 * K - (S[i, j] - 2 * g) if (di, dj) == (1, 1) else K
            nc = c + step
            if nc < best.get((a, b), float("inf")):
                best[(a, b)] = nc
                heapq.heappush(pq, (nc + h(a, b), nc, a, b))
    raise AssertionError("no path")


def check_astar_agrees(O, n_cases=60, seed=23):
    r = rng(seed)
    for case in range(n_cases):
        n, m = int(r.integers(0, 14)), int(r.integers(0, 14))
        S = (r.integers(0, 17, (n, m)) / 16.0).astype(np.float32)
        g = F32(-0.0625 * int(r.integers(0, 9)))
        h, _, _ = O.nw(S, g)
        a = astar_monotone(S, g)
        assert float(h) == a, (case, n, m, float(g), float(h), a)


ALL.append(check_astar_agrees)
