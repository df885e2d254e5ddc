"""Helpers shared by the GPU parity tests (comparison rules, input builders)."""
from __future__ import annotations

import numpy as np

import synth

TOL_S = 1e-6  # |S_gpu - S_oracle| bound for the similarity scores


def pairs_of(res, p):
    a, b = int(res["pair_off"][p]), int(res["pair_off"][p + 1])
    return list(zip(res["src_idx"][a:b].tolist(), res["tgt_idx"][a:b].tolist())), res["score"][a:b]


def compare_mined(O, olex, corpus, w, gap, tau, got, want, S_gpu_flat=None):
    """Mined sets must match pair by pair.  A mismatch is admissible only as a
    tie: the oracle's own NW run on the GPU's scores reproduces the GPU output
    and the two score matrices agree within TOL_S.  Returns the admissible
    ties (pair index, cells) so a test can list them."""
    assert got["pair_off"].shape == want["pair_off"].shape
    n, m = corpus.nm()
    base = np.concatenate([[0], np.cumsum(n * m)])
    ties = []
    for p in range(corpus.n_pairs):
        gp, gs = pairs_of(got, p)
        wp, ws = pairs_of(want, p)
        same = gp == wp and np.array_equal(gs, ws) and got["align_score"][p] == want["align_score"][p]
        if same:
            continue
        if gp == wp and np.max(np.abs(gs - ws), initial=0.0) <= TOL_S:
            # same pairs; scores within tolerance (the H value may differ by the same rounding)
            ties.append((p, "scores-within-tolerance", gp))
            continue
        assert S_gpu_flat is not None, f"pair {p}: GPU {gp} != oracle {wp}"
        Sg = S_gpu_flat[base[p]:base[p + 1]].reshape(int(n[p]), int(m[p]))
        src, tgt = corpus.pair(p)
        So, _, _ = O.similarity(olex, src, tgt, w)
        assert np.max(np.abs(Sg - So), initial=0.0) <= TOL_S, f"pair {p}: scores differ beyond tolerance"
        h, mv, _ = O.nw(Sg, gap)
        si, ti, sc = O.emit(Sg, mv, tau)
        assert list(zip(si.tolist(), ti.tolist())) == gp, f"pair {p}: not an admissible tie"
        diff = np.argwhere(Sg != So)
        ties.append((p, "admissible-tie", diff.tolist()))
    return ties


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
