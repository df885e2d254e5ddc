"""Helpers shared by the GPU parity tests (comparison rules, input builders)."""
from __future__ import annotations

import json
import os

import numpy as np

import synth

TOL_S = 1e-6  # |S_gpu - S_oracle| bound for the similarity scores


def pairs_of(res, p):
    a, b = int(res["pair_off"][p]), int(res["pair_off"][p + 1])
    return list(zip(res["src_idx"][a:b].tolist(), res["tgt_idx"][a:b].tolist())), res["score"][a:b]


def compare_mined(O, olex, corpus, w, gap, tau, got, want, S_gpu_flat=None):
    """Mined results must match pair by pair: the same (source, target) index
    pairs in the same order, their scores within TOL_S, and H[n][m] equal bit
    for bit.  A pair that differs in any of these is admissible only as a tie:
    the GPU's whole score matrix agrees with the oracle's within TOL_S, and the
    oracle's own NW and threshold run on the GPU's scores reproduce the GPU's
    pairs, scores and H[n][m] exactly.  Returns the admissible ties as
    (pair index, cells where the two score matrices differ); every caller
    checks them against the committed list with `assert_ties`."""
    assert got["pair_off"].shape == want["pair_off"].shape
    n, m = corpus.nm()
    base = np.concatenate([[0], np.cumsum(n * m)])
    ties = []
    for p in range(corpus.n_pairs):
        gp, gs = pairs_of(got, p)
        wp, ws = pairs_of(want, p)
        h_same = np.float32(got["align_score"][p]).tobytes() == np.float32(want["align_score"][p]).tobytes()
        if gp == wp and h_same and np.max(np.abs(gs - ws), initial=0.0) <= TOL_S:
            continue
        assert S_gpu_flat is not None, f"pair {p}: GPU {gp} != oracle {wp} (H {got['align_score'][p]} vs {want['align_score'][p]})"
        Sg = S_gpu_flat[base[p]:base[p + 1]].reshape(int(n[p]), int(m[p]))
        src, tgt = corpus.pair(p)
        So, _, _ = O.similarity(olex, src, tgt, w)
        assert np.max(np.abs(Sg - So), initial=0.0) <= TOL_S, f"pair {p}: scores differ beyond tolerance"
        h, mv, _ = O.nw(Sg, gap)
        si, ti, sc = O.emit(Sg, mv, tau)
        assert list(zip(si.tolist(), ti.tolist())) == gp, f"pair {p}: not an admissible tie (pairs)"
        assert sc.tobytes() == np.asarray(gs, np.float32).tobytes(), f"pair {p}: not an admissible tie (scores)"
        assert np.float32(h).tobytes() == np.float32(got["align_score"][p]).tobytes(), f"pair {p}: not an admissible tie (H)"
        ties.append((p, np.argwhere(Sg != So).tolist()))
    return ties


_EXPECTED = None


def expected_ties(case):
    """The committed list of admissible ties of a test case (tests/golden/expected_ties.json)."""
    global _EXPECTED
    if _EXPECTED is None:
        with open(os.path.join(os.path.dirname(__file__), "golden", "expected_ties.json")) as f:
            _EXPECTED = json.load(f)["cases"]
    return [(int(p), [list(map(int, c)) for c in cells]) for p, cells in _EXPECTED.get(case, [])]


def assert_ties(case, ties):
    """Every admissible tie a comparison found must be listed, cell by cell,
    for its case; a listed tie that no longer occurs fails too."""
    got = [(int(p), [list(map(int, c)) for c in cells]) for p, cells in ties]
    assert got == expected_ties(case), f"{case}: ties {got} != listed {expected_ties(case)}"


def select_pairs(res, pairs):
    """The result entries of the listed pairs, in that order, as a result of its own."""
    off, si, ti, sc = [0], [], [], []
    for p in pairs:
        a, b = int(res["pair_off"][p]), int(res["pair_off"][p + 1])
        si.append(res["src_idx"][a:b])
        ti.append(res["tgt_idx"][a:b])
        sc.append(res["score"][a:b])
        off.append(off[-1] + b - a)
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    return dict(pair_off=np.array(off, np.int64), src_idx=cat(si, np.int32), tgt_idx=cat(ti, np.int32),
                score=cat(sc, np.float32), align_score=np.asarray(res["align_score"])[np.asarray(pairs, np.int64)])


def oracle_pair_banded(O, olex, src, tgt, w, gap, tau, workers=8, band=250):
    """The oracle's result for one large document pair, its score matrix
    computed in bands of source rows on worker threads (row i of S depends
    only on source sentence i and the target document), then the oracle's NW
    and threshold over the whole matrix.  Returns (result dict, S)."""
    from concurrent.futures import ThreadPoolExecutor
    n, m = len(src), len(tgt)
    S = np.zeros((n, m), np.float32)

    def run(i0):
        S[i0:i0 + band] = O.similarity(olex, src[i0:i0 + band], tgt, w)[0]
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(run, range(0, n, band)))
    h, mv, _ = O.nw(S, gap)
    si, ti, sc = O.emit(S, mv, tau)
    res = dict(pair_off=np.array([0, si.size], np.int64), src_idx=si, tgt_idx=ti, score=sc,
               align_score=np.array([h], np.float32))
    return res, S


def compare_result_fields(got, want, what=""):
    """Two results of the same pairs: every field equal (scores within TOL_S,
    H[n][m] bit for bit)."""
    assert np.array_equal(got["pair_off"], want["pair_off"]), what
    assert np.array_equal(got["src_idx"], want["src_idx"]), what
    assert np.array_equal(got["tgt_idx"], want["tgt_idx"]), what
    assert np.max(np.abs(got["score"] - want["score"]), initial=0.0) <= TOL_S, what
    assert np.asarray(got["align_score"], np.float32).tobytes() == np.asarray(want["align_score"], np.float32).tobytes(), what


def random_corpus(seed, n_pairs, nmax, mmax, lmax_src, lmax_tgt, vocab=60, neg_frac=0.02, empty_frac=0.1):
    """Ragged documents with empty docs / sentences, long sentences and odd ids."""
    r = np.random.default_rng(seed)
    srcs, tgts = [], []
    for _ in range(n_pairs):
        n = int(r.integers(0, nmax + 1))
        m = int(r.integers(0, mmax + 1))

        def sent(lmax):
            if r.random() < empty_frac:
                return np.zeros(0, np.int32)
            L = int(r.integers(1, lmax + 1))
            s = (r.zipf(1.3, L) - 1) % (vocab + 5)  # ids >= vocab are not lexicon keys
            neg = r.random(L) < neg_frac
            s[neg] = -int(r.integers(1, 5))
            return s.astype(np.int32)
        srcs.append([sent(lmax_src) for _ in range(n)])
        tgts.append([sent(lmax_tgt) for _ in range(m)])
    return synth.from_lists(srcs, tgts)


def random_lexicon(seed, vocab=60, kmax=4):
    r = np.random.default_rng(seed + 1)
    src, off, tgt = [], [0], []
    for x in range(vocab):
        if r.random() < 0.15:
            continue
        k = int(r.integers(1, kmax + 1))
        src.append(x)
        tgt += list(map(int, r.integers(0, vocab + 3, k)))
        off.append(len(tgt))
    return synth.Lexicon(np.array(src, np.int32), np.array(off, np.int64), np.array(tgt, np.int32))
