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
