"""Parameter sweep (tuned miner) and bidirectional mining against the oracle.

Both entry points are compositions of the miner: the sweep mines once per
gap penalty with every diagonal move kept and counts, per threshold, accepted
and reference pairs; bidirectional mining joins a forward run with a run on
the swapped batch.  The oracle side composes the oracle miner the same way.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

from . import parity

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def ym():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08639_amd import ymine
    return ymine


@pytest.fixture(scope="module")
def ctx(ym):
    return ym.Context(0)


@pytest.fixture(scope="module")
def O():
    return oracle.default()


def _counts(res, corpus, taus):
    """(accepted, correct) per threshold from a result mined with every move kept."""
    truth = set()
    for p in range(corpus.n_pairs):
        for e in range(int(corpus.truth_off[p]), int(corpus.truth_off[p + 1])):
            truth.add((p, int(corpus.truth_src[e]), int(corpus.truth_tgt[e])))
    pid = np.repeat(np.arange(corpus.n_pairs), np.diff(res["pair_off"]))
    hit = np.array([(int(p), int(i), int(j)) in truth
                    for p, i, j in zip(pid, res["src_idx"], res["tgt_idx"])], bool)
    sc = res["score"]
    return (np.array([(sc >= t).sum() for t in taus], np.int64),
            np.array([((sc >= t) & hit).sum() for t in taus], np.int64))


def _away_from(scores, taus, margin=1e-5):
    """Shift thresholds off any score closer than `margin` (GPU and oracle
    scores agree within 1e-6, so counts are then comparable exactly)."""
    out = []
    for t in taus:
        t = F32(t)
        while np.any(np.abs(scores - t) < margin):
            t = F32(t + 3 * margin)
        out.append(t)
    return np.array(out, np.float32)


def test_tune_matches_oracle_sweep(ym, ctx, O):
    cfg = synth.CONFIGS[1]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex, pair_ids=np.arange(0, 10000, 80))
    w = synth.weights(cfg.seed)
    gaps = np.array([0.0, -0.1, -0.2, -0.45], np.float32)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    S, _, _ = ym.similarity(ctx, L, c, w)
    taus = _away_from(S, [0.05, 0.2, 0.35, 0.5, 0.65, 0.8, 0.95])
    nm, nc = ym.tune(ctx, L, c, w, gaps, taus, c.truth_off, c.truth_src, c.truth_tgt)
    assert nm.shape == (len(gaps), len(taus))
    for gi, g in enumerate(gaps):
        got = ym.mine(ctx, L, c, w, g, -1.0)  # S >= 0 > -1: every diagonal move kept
        want = O.mine(OL, c, w, g, F32(-1.0))
        ties = parity.compare_mined(O, OL, c, w, F32(g), F32(-1.0), got, want, S)
        parity.assert_ties(f"tune_batch_10k_every_80th_gap{gi}", ties)
        gm, gc = _counts(got, c, taus)
        assert np.array_equal(nm[gi], gm) and np.array_equal(nc[gi], gc), (g, nm[gi], gm, nc[gi], gc)
        om, oc = _counts(want, c, taus)
        assert np.array_equal(nm[gi], om) and np.array_equal(nc[gi], oc), (g, nm[gi], om, nc[gi], oc)
    # precision rises with the threshold; counts never exceed the reference size
    assert np.all(nc <= nm) and np.all(np.diff(nm, axis=1) <= 0)
    assert np.all(nc <= int(c.truth_off[-1]))
    # the chosen (gap, threshold) is the oracle sweep's F1 argmax (exact
    # rationals, first entry on ties)
    truth = int(c.truth_off[-1])
    om_all = np.zeros_like(nm)
    oc_all = np.zeros_like(nc)
    for gi, g in enumerate(gaps):
        om_all[gi], oc_all[gi] = _counts(O.mine(OL, c, w, g, F32(-1.0)), c, taus)
    best = None
    for gi in range(len(gaps)):
        for ti in range(len(taus)):
            f = Fraction(2 * int(oc_all[gi, ti]), int(om_all[gi, ti]) + truth)
            if best is None or f > best[0]:
                best = (f, gi, ti)
    choice = ym.tune_select(nm, nc, truth)
    assert (choice["gap_index"], choice["tau_index"]) == best[1:]
    assert choice["f1"] == pytest.approx(float(best[0]), rel=1e-15, abs=0.0)


def test_tune_small_workspace_and_edges(ym, ctx, O):
    lex = parity.random_lexicon(9)
    c = parity.random_corpus(9, n_pairs=40, nmax=70, mmax=70, lmax_src=40, lmax_tgt=40)
    # a made-up reference: the main diagonal of every pair
    n, m = c.nm()
    k = np.minimum(n, m)
    c.truth_off = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    c.truth_src = np.concatenate([np.arange(x) for x in k] + [np.zeros(0)]).astype(np.int32)
    c.truth_tgt = c.truth_src.copy()
    w = np.array([-1.5, 3.0, 2.0, 0.5], np.float32)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    S, _, _ = ym.similarity(ctx, L, c, w)
    gaps = np.array([-0.3], np.float32)
    taus = _away_from(S, [0.5, 2.0])
    nm, nc = ym.tune(ctx, L, c, w, gaps, taus, c.truth_off, c.truth_src, c.truth_tgt)
    got = ym.mine(ctx, L, c, w, gaps[0], -1.0)
    gm, gc = _counts(got, c, taus)
    assert np.array_equal(nm[0], gm) and np.array_equal(nc[0], gc)
    assert nm[0, 1] == 0 and nc[0, 1] == 0  # no score reaches 2
    want = O.mine(OL, c, w, gaps[0], F32(-1.0))
    ties = parity.compare_mined(O, OL, c, w, gaps[0], F32(-1.0), got, want, S)
    parity.assert_ties("tune_ragged_40_seed9", ties)
    with pytest.raises(ym.YmError):
        ym.tune(ctx, L, c, w, np.zeros(0, np.float32), taus, c.truth_off, c.truth_src, c.truth_tgt)
    with pytest.raises(ym.YmError):
        ym.tune(ctx, L, c, w, np.array([np.nan], np.float32), taus, c.truth_off, c.truth_src, c.truth_tgt)


@pytest.mark.parametrize("large", [1, 0])
def test_tune_gaps_in_one_launch_with_large_pairs(ym, O, large):
    """Several gap penalties swept in one NW launch over a batch holding pairs
    of 449+ source sentences, in both sweeps of the large pairs: every gap's
    counts equal those of a plain mining run at that gap."""
    ctx = ym.Context(0)
    ym.set_tuning(ctx, 1, 128, 1, large)
    lex = parity.random_lexicon(11)
    c = parity.random_corpus(11, n_pairs=8, nmax=760, mmax=130, lmax_src=12, lmax_tgt=12)
    n, m = c.nm()
    k = np.minimum(n, m)
    c.truth_off = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    c.truth_src = np.concatenate([np.arange(x) for x in k] + [np.zeros(0)]).astype(np.int32)
    c.truth_tgt = c.truth_src.copy()
    w = np.array([-1.5, 3.0, 2.0, 0.5], np.float32)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    S, _, _ = ym.similarity(ctx, L, c, w)
    gaps = np.array([-0.2, -0.5, 0.0], np.float32)
    taus = _away_from(S, [0.3, 0.5, 0.7])
    nm, nc = ym.tune(ctx, L, c, w, gaps, taus, c.truth_off, c.truth_src, c.truth_tgt)
    for gi, g in enumerate(gaps):
        gm, gc = _counts(ym.mine(ctx, L, c, w, g, -1.0), c, taus)
        assert np.array_equal(nm[gi], gm) and np.array_equal(nc[gi], gc), gi


def _reverse_lexicon(lex):
    """The lexicon read the other way: every (x, y) entry becomes (y, x)."""
    pairs = sorted({(int(y), int(x)) for k, x in enumerate(lex.src_ids)
                    for y in lex.tgt_ids[lex.off[k]:lex.off[k + 1]]})
    src, off, tgt = [], [0], []
    for y, x in pairs:
        if not src or src[-1] != y:
            if src:
                off.append(len(tgt))
            src.append(y)
        tgt.append(x)
    off.append(len(tgt))
    if not src:
        off = [0]
    return synth.Lexicon(np.array(src, np.int32), np.array(off, np.int64), np.array(tgt, np.int32))


def _swap(c):
    return synth.Corpus(c.tgt_doc_off, c.tgt_sent_off, c.tgt_tok, c.src_doc_off, c.src_sent_off, c.src_tok)


def _union(fwd, rev, n_pairs):
    """Oracle composition: forward pairs plus reverse pairs mapped back, no
    duplicates (forward score kept), ordered by (source, target) index."""
    off, si, ti, sc = [0], [], [], []
    for p in range(n_pairs):
        d = {}
        a, b = int(rev["pair_off"][p]), int(rev["pair_off"][p + 1])
        for i, j, v in zip(rev["tgt_idx"][a:b], rev["src_idx"][a:b], rev["score"][a:b]):
            d[(int(i), int(j))] = v
        a, b = int(fwd["pair_off"][p]), int(fwd["pair_off"][p + 1])
        for i, j, v in zip(fwd["src_idx"][a:b], fwd["tgt_idx"][a:b], fwd["score"][a:b]):
            d[(int(i), int(j))] = v
        for (i, j) in sorted(d):
            si.append(i)
            ti.append(j)
            sc.append(d[(i, j)])
        off.append(len(si))
    return dict(pair_off=np.array(off, np.int64), src_idx=np.array(si, np.int32),
                tgt_idx=np.array(ti, np.int32), score=np.array(sc, np.float32), align_score=fwd["align_score"])


@pytest.mark.parametrize("which", ["planted", "ragged"])
def test_bidirectional_matches_oracle_union(ym, ctx, O, which):
    if which == "planted":
        cfg = synth.CONFIGS[1]
        lex = synth.make_lexicon(cfg)
        c = synth.generate(cfg, lex, pair_ids=np.arange(5, 10000, 97))
        wf = synth.weights(cfg.seed)
        wr = synth.weights(cfg.seed + 1)
    else:
        lex = parity.random_lexicon(11)
        c = parity.random_corpus(11, n_pairs=40, nmax=80, mmax=60, lmax_src=35, lmax_tgt=45)
        wf = np.array([-1.5, 3.0, 2.0, 0.5], np.float32)
        wr = np.array([-1.2, 2.0, 3.0, 0.4], np.float32)
    rlex = _reverse_lexicon(lex)
    g, tau = F32(-0.2), F32(0.5)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    R = ctx.lexicon(rlex.src_ids, rlex.off, rlex.tgt_ids)
    got = ym.mine_bidirectional(ctx, L, R, c, wf, wr, g, tau)
    # each direction on its own, on the GPU and in the oracle
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    OR = O.lexicon(rlex.src_ids, rlex.off, rlex.tgt_ids)
    cr = _swap(c)
    gf, gr = ym.mine(ctx, L, c, wf, g, tau), ym.mine(ctx, R, cr, wr, g, tau)
    of, orv = O.mine(OL, c, wf, g, tau), O.mine(OR, cr, wr, g, tau)
    Sf, _, _ = ym.similarity(ctx, L, c, wf)
    Sr, _, _ = ym.similarity(ctx, R, cr, wr)
    tf = parity.compare_mined(O, OL, c, wf, g, tau, gf, of, Sf)
    tr = parity.compare_mined(O, OR, cr, wr, g, tau, gr, orv, Sr)
    parity.assert_ties(f"bidirectional_{which}_forward", tf)
    parity.assert_ties(f"bidirectional_{which}_reverse", tr)
    # the joined result is exactly the union of the GPU's own directions ...
    mine_u = _union(gf, gr, c.n_pairs)
    for k in ("pair_off", "src_idx", "tgt_idx", "score", "align_score"):
        assert np.array_equal(got[k], mine_u[k]), k
    # ... and the oracle's union (no direction has a listed tie)
    want = _union(of, orv, c.n_pairs)
    for k in ("pair_off", "src_idx", "tgt_idx"):
        assert np.array_equal(got[k], want[k]), k
    assert np.max(np.abs(got["score"] - want["score"]), initial=0.0) <= parity.TOL_S
    assert got["align_score"].tobytes() == of["align_score"].tobytes()
    assert int(got["pair_off"][-1]) >= max(int(gf["pair_off"][-1]), int(gr["pair_off"][-1]))
