"""The multi-threaded CPU miner gives exactly the single-threaded oracle's result."""
import numpy as np

import oracle
import synth


def test_threads_equal_single():
    oracle.build(force=False)
    O = oracle.default()
    cfg = synth.config(1, n_pairs=60)
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex)
    w = synth.weights(cfg.seed)
    L = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    a = O.mine(L, c, w, -0.2, 0.5)
    for t in (1, 3, 8):
        b = O.mine_threads(L, c, w, -0.2, 0.5, t)
        for k in a:
            assert np.array_equal(a[k], b[k]), (t, k)


def test_banded_oracle_pair_equals_oracle_mine():
    """The banded composition used for very large pairs in the GPU tests (S
    by row bands, then NW and threshold on the whole matrix) is the oracle's
    own miner."""
    import numpy as np
    import synth
    from . import parity
    O = oracle.default()
    cfg = synth.config(3, count_kind=0, n_fixed=700, m_fixed=650, n_pairs=1)
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex)
    w = synth.weights(cfg.seed)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, np.float32(-0.2), np.float32(0.5))
    src, tgt = c.pair(0)
    got, _ = parity.oracle_pair_banded(O, OL, src, tgt, w, np.float32(-0.2), np.float32(0.5), workers=4, band=96)
    parity.compare_result_fields(got, want)
    assert np.array_equal(got["score"], want["score"])
