"""Allocation-free device entry point (ym_mine_device_static) against the
device entry point with a caller workspace (ym_mine_device), through the C ABI:
identical results on two calls in a row, the second with a smaller batch, and
a batch too large for the static scratch rejected before any work."""
import numpy as np
import pytest

import oracle
import synth

from . import parity

pytestmark = pytest.mark.gpu

FIELDS = ("pair_off", "src_idx", "tgt_idx", "score", "align_score")


@pytest.fixture(scope="module")
def ym():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08639_amd import ymine
    return ymine


def _same(a, b):
    for k in FIELDS:
        assert a[k].dtype == b[k].dtype and np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def test_static_equals_workspace_form(ym):
    import torch
    ctx = ym.Context(0)
    cfg = synth.config(1, n_pairs=300)
    lex = synth.make_lexicon(cfg)
    w = synth.weights(cfg.seed)
    gap, tau = np.float32(-0.2), np.float32(0.5)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    O = oracle.default()
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    # a larger batch, then a smaller one: the second call reuses the scratch
    # that the first left filled
    for n_pairs in (300, 37):
        corpus = synth.generate(cfg, lex, pair_ids=np.arange(n_pairs))
        print(f"static entry point: {n_pairs} pairs, {corpus.cells()} cells", flush=True)
        ref = ym.DeviceMiner(ctx, L, corpus)
        ref.run(w, gap, tau)
        want = ref.result()
        dm = ym.DeviceMiner(ctx, L, corpus, workspace_bytes=0)
        dm.run_static(w, gap, tau)
        got = dm.result()
        _same(got, want)
        # and the oracle on a sample of the pairs
        for p in range(0, n_pairs, 7):
            o = O.mine(OL, corpus.slice(p, p + 1), w, gap, tau)
            parity.compare_result_fields(parity.select_pairs(got, [p]), o, f"pair {p} against the oracle")
        del ref, dm
        torch.cuda.synchronize()


def test_static_rejects_oversized_batch(ym):
    ctx = ym.Context(0)
    cfg = synth.config(0)
    lex = synth.make_lexicon(cfg)
    corpus = synth.generate(cfg, lex)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    dm = ym.DeviceMiner(ctx, L, corpus, workspace_bytes=0)
    # claim more source tokens than the scratch can translate (16 bytes each):
    # rejected on the host before anything is enqueued
    dm.b.n_src_tok = int(ym.STATIC_SCRATCH_BYTES // 16) + 1
    with pytest.raises(ym.YmError) as e:
        dm.run_static(synth.weights(cfg.seed), -0.2, 0.5)
    assert e.value.code == ym.YM_ENOMEM
