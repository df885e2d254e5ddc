"""GPU path (through the C ABI) against the CPU oracle, element by element.

Bars: overlap counts and NW results (H[n][m] bits, paths, emitted pairs)
bit-exact -- NW is fed the oracle's score matrices; scores within 1e-6; mined
pair sets identical, apart from explicitly listed admissible ties.
"""
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
def ctx_k(ym, ctx):
    """Contexts by similarity kernel: 1 (the default context), 2 (reads of
    target sentences longer than 32 tokens split over spare lanes), 3 and 4
    (bit-sliced tiles of four waves, 1,280- and 2,048-token chunks)."""
    made = {1: ctx}

    def get(k):
        if k not in made:
            c = ym.Context(0)
            ym.set_tuning(c, k, 128, 1)
            made[k] = c
        return made[k]
    return get


@pytest.fixture(scope="module")
def ctx_large(ym, ctx):
    """Contexts by sweep of the large pairs (449+ source sentences): 1 strips
    over every CU (the default context), 0 one 16-wave workgroup per pair."""
    made = {1: ctx}

    def get(v):
        if v not in made:
            c = ym.Context(0)
            ym.set_tuning(c, 1, 128, 1, v)
            made[v] = c
        return made[v]
    return get


@pytest.fixture(scope="module")
def O():
    return oracle.default()


def _similarity_check(ym, ctx, O, lex, corpus, w):
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    S, ms, mt = ym.similarity(ctx, L, corpus, w)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    base = 0
    worst = 0.0
    for p in range(corpus.n_pairs):
        src, tgt = corpus.pair(p)
        So, mso, mto = O.similarity(OL, src, tgt, w)
        k = So.size
        assert np.array_equal(ms[base:base + k], mso.reshape(-1)), f"m_s differs in pair {p}"
        assert np.array_equal(mt[base:base + k], mto.reshape(-1)), f"m_t differs in pair {p}"
        d = np.max(np.abs(S[base:base + k] - So.reshape(-1)), initial=0.0)
        worst = max(worst, float(d))
        base += k
    assert worst <= parity.TOL_S, worst
    return worst


def test_similarity_single_pair(ym, ctx, O):
    cfg = synth.CONFIGS[0]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex)
    _similarity_check(ym, ctx, O, lex, c, synth.weights(cfg.seed))


@pytest.mark.parametrize("seed,kernel", [(1, 1), (2, 1), (3, 1), (1, 2), (2, 2), (1, 3), (2, 3), (3, 3), (1, 4), (2, 4)])
def test_similarity_ragged_edges(ym, ctx_k, O, seed, kernel):
    # empty documents and sentences, negative / unknown ids, source sentences
    # of more than 31 and 63 tokens (one-row path, extra mask passes), > 128 source
    # sentences (several work items), > 256 target sentences (several chunks)
    lex = parity.random_lexicon(seed)
    c = parity.random_corpus(seed, n_pairs=12, nmax=150, mmax=300, lmax_src=70, lmax_tgt=40)
    w = np.array([-2.0, 3.0, 2.5, 0.75], np.float32)
    _similarity_check(ym, ctx_k(kernel), O, lex, c, w)


@pytest.mark.parametrize("kernel", [1, 2, 3, 4])
def test_similarity_long_sentences(ym, ctx_k, O, kernel):
    # source sentences of up to 200 tokens (up to four mask passes of 63
    # positions), target sentences of up to 130 (split reads: groups of up to
    # 8 lanes per sentence)
    lex = parity.random_lexicon(4, vocab=300)
    c = parity.random_corpus(4, n_pairs=8, nmax=70, mmax=90, lmax_src=200, lmax_tgt=130, vocab=300)
    _similarity_check(ym, ctx_k(kernel), O, lex, c, np.array([-2.0, 3.0, 2.5, 0.75], np.float32))


def test_similarity_key_ids_beyond_dense_table(ym, ctx, O):
    # a key of 2^25: the lexicon gets no dense record table, so the
    # translation pass probes the hash table
    lex = parity.random_lexicon(12, vocab=300)
    big = 1 << 25
    lex2 = synth.Lexicon(np.concatenate([lex.src_ids, [big]]).astype(np.int32),
                         np.concatenate([lex.off, [lex.off[-1] + 2]]).astype(np.int64),
                         np.concatenate([lex.tgt_ids, [5, 7]]).astype(np.int32))
    c = parity.random_corpus(12, n_pairs=10, nmax=60, mmax=80, lmax_src=40, lmax_tgt=40, vocab=300)
    c.src_tok[::7] = big
    _similarity_check(ym, ctx, O, lex2, c, np.array([-2.0, 3.0, 2.5, 0.75], np.float32))


@pytest.mark.parametrize("kernel", [1, 2, 3, 4])
def test_similarity_chunk_boundaries(ym, ctx_k, O, kernel):
    # target sentences near the chunk limits (1,024, 1,280 and 2,048 tokens)
    # and many short ones
    lex = parity.random_lexicon(9, vocab=400)
    r = np.random.default_rng(9)
    srcs = [[r.integers(0, 400, int(r.integers(1, 40))).astype(np.int32) for _ in range(7)]]
    tgts = [[r.integers(0, 400, L).astype(np.int32) for L in (1024, 1, 1023, 2, 600, 500, 0, 1024)]]
    srcs.append([r.integers(0, 400, 5).astype(np.int32) for _ in range(3)])
    tgts.append([r.integers(0, 400, 3).astype(np.int32) for _ in range(700)])
    srcs.append([r.integers(0, 400, int(r.integers(1, 60))).astype(np.int32) for _ in range(70)])
    tgts.append([r.integers(0, 400, L).astype(np.int32)
                 for L in (640, 640, 1, 700, 579, 1, 1024, 1024, 0, 3, 1024, 255, 1, 1, 1000, 47) + (60,) * 40])
    c = synth.from_lists(srcs, tgts)
    # one-sentence chunks of 1,024 tokens: with split reads, groups of all 64 lanes
    _similarity_check(ym, ctx_k(kernel), O, lex, c, np.array([-1.0, 2.0, 2.0, 0.5], np.float32))


def _nw_cases():
    r = np.random.default_rng(5)
    mats = []
    for (n, m) in [(1, 1), (0, 5), (6, 0), (0, 0), (3, 7), (64, 64), (65, 63), (127, 129), (200, 200),
                   # the last pair whose direction codes fit in LDS, and the first that does not
                   (168, 160), (169, 160),
                   (40, 45), (300, 17), (17, 300), (130, 600), (70, 520), (1000, 1100),
                   # pipelined sweep of large pairs: 8 strips (last of one row), 8 full, 17 strips
                   # (more strips than waves), a single target column, no target sentence
                   (449, 37), (512, 70), (1025, 90), (1100, 1), (700, 0), (1090, 3)]:
        mats.append(r.random((n, m)).astype(np.float32))
    # dyadic ties everywhere
    mats.append((r.integers(0, 3, (90, 77)) / 4.0).astype(np.float32))
    mats.append(np.full((33, 50), 0.375, np.float32))
    # denormals, exact threshold values, negative scores
    S = r.random((20, 25)).astype(np.float32)
    S[3, 4] = F32(1e-40)
    S[5, 6] = F32(0.5)
    S[7, 8] = np.nextafter(F32(0.5), F32(0))
    S[9, :] = -0.3
    mats.append(S)
    return mats


@pytest.mark.parametrize("large", [1, 0])
@pytest.mark.parametrize("gap", [-0.2, -0.25, 0.0, -1.5])
def test_nw_fed_oracle_scores(ym, ctx_large, O, gap, large):
    mats = _nw_cases()
    align, moves, res = ym.nw_align(ctx_large(large), mats, gap, 0.5)
    for k, S in enumerate(mats):
        h, mv, _ = O.nw(S, gap)
        assert align[k].tobytes() == h.tobytes(), (k, S.shape, align[k], h)
        assert moves[k] == mv, (k, S.shape)
        si, ti, sc = O.emit(S, mv, 0.5)
        gp, gs = parity.pairs_of(res, k)
        assert gp == list(zip(si.tolist(), ti.tolist())), k
        assert gs.tobytes() == sc.tobytes(), k


@pytest.mark.parametrize("large", [1, 0])
def test_nw_many_large_pairs(ym, ctx_large, O, large):
    """More strips of large pairs than the persistent grid has waves (so waves
    take several tickets), pairs of 8 to 10 strips with 0 to 40 target
    sentences, in both sweeps of the large pairs, against the oracle."""
    r = np.random.default_rng(77)
    mats = []
    for k in range(270):
        n = int(r.integers(449, 641))
        m = int(r.integers(0, 41)) if k % 9 else int(k % 2)
        mats.append(r.random((n, m)).astype(np.float32))
    mats.append((r.integers(0, 3, (520, 33)) / 4.0).astype(np.float32))  # dyadic ties
    assert sum((S.shape[0] + 63) // 64 for S in mats) > 2048
    align, moves, res = ym.nw_align(ctx_large(large), mats, -0.2, 0.5)
    for k, S in enumerate(mats):
        h, mv, _ = O.nw(S, F32(-0.2))
        assert align[k].tobytes() == h.tobytes(), (k, S.shape, align[k], h)
        assert moves[k] == mv, (k, S.shape)
        si, ti, sc = O.emit(S, mv, 0.5)
        gp, gs = parity.pairs_of(res, k)
        assert gp == list(zip(si.tolist(), ti.tolist())), k
        assert gs.tobytes() == sc.tobytes(), k


def test_nw_bruteforce_small(ym, ctx, O):
    from . import pins
    r = np.random.default_rng(21)
    mats, gaps = [], []
    for _ in range(40):
        n, m = int(r.integers(0, 7)), int(r.integers(0, 7))
        mats.append(r.random((n, m)).astype(np.float32))
    align, moves, _ = ym.nw_align(ctx, mats, -0.3, 0.5)
    for k, S in enumerate(mats):
        v = pins.folds(S, F32(-0.3), pins.all_paths(*S.shape))
        assert align[k] == v.max()


def test_mine_end_to_end_batch_sample(ym, ctx, O):
    cfg = synth.CONFIGS[1]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex, pair_ids=np.arange(0, 10000, 50))
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    got = ym.mine(ctx, L, c, w, -0.2, 0.5)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, -0.2, 0.5)
    S, _, _ = ym.similarity(ctx, L, c, w)
    ties = parity.compare_mined(O, OL, c, w, F32(-0.2), F32(0.5), got, want, S)
    parity.assert_ties("batch_10k_every_50th", ties)


def test_device_and_per_pair_forms_match(ym, ctx, O):
    cfg = synth.CONFIGS[1]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex, pair_ids=np.arange(300, 420))
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    a = ym.mine(ctx, L, c, w, -0.2, 0.5)
    b = ym.mine_per_pair(ctx, L, c, w, -0.2, 0.5)
    dm = ym.DeviceMiner(ctx, L, c)
    dm.run(w, -0.2, 0.5)
    d = dm.result()
    # a small workspace forces several chunks (token translations + 2 MiB)
    head = (c.src_tok.size * 16 + 255) // 256 * 256
    dm2 = ym.DeviceMiner(ctx, L, c, workspace_bytes=head + (2 << 20))
    dm2.run(w, -0.2, 0.5)
    e = dm2.result()
    for r in (b, d, e):
        for k in a:
            assert np.array_equal(a[k], r[k]), k
    # passes back to back on a second stream, two miners interleaved, no host
    # wait between them (plan uploads on the context's side stream, one
    # staging buffer)
    import torch
    s2 = torch.cuda.Stream()
    dm.run(w, -0.2, 0.5, stream=s2.cuda_stream)
    dm2.run(w, -0.2, 0.5, stream=s2.cuda_stream)
    dm.run(w, -0.2, 0.5, stream=s2.cuda_stream)
    s2.synchronize()
    for r in (dm.result(), dm2.result()):
        for k in a:
            assert np.array_equal(a[k], r[k]), k


def test_mine_ragged_edges_end_to_end(ym, ctx, O):
    lex = parity.random_lexicon(4)
    c = parity.random_corpus(4, n_pairs=30, nmax=90, mmax=90, lmax_src=40, lmax_tgt=35)
    w = np.array([-1.5, 3.0, 2.0, 0.5], np.float32)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    got = ym.mine(ctx, L, c, w, -0.2, 0.5)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, -0.2, 0.5)
    S, _, _ = ym.similarity(ctx, L, c, w)
    ties = parity.compare_mined(O, OL, c, w, F32(-0.2), F32(0.5), got, want, S)
    parity.assert_ties("ragged_30_pairs_seed4", ties)


@pytest.mark.parametrize("large", [1, 0])
def test_mine_large_pairs_end_to_end(ym, ctx_large, O, large):
    """A batch mixing pairs of 449+ source sentences with small ones, end to
    end in both sweeps of the large pairs, against the oracle."""
    lex = parity.random_lexicon(11)
    c = parity.random_corpus(11, n_pairs=8, nmax=760, mmax=130, lmax_src=12, lmax_tgt=12)
    n, _ = c.nm()
    assert (n >= 449).sum() >= 2
    w = np.array([-1.5, 3.0, 2.0, 0.5], np.float32)
    cx = ctx_large(large)
    L = cx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    got = ym.mine(cx, L, c, w, -0.2, 0.5)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, -0.2, 0.5)
    S, _, _ = ym.similarity(cx, L, c, w)
    ties = parity.compare_mined(O, OL, c, w, F32(-0.2), F32(0.5), got, want, S)
    parity.assert_ties("large_pairs_8_seed11", ties)


def test_long_pair(ym, ctx, O):
    cfg = synth.CONFIGS[2]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex, pair_ids=np.array([7]))
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    got = ym.mine(ctx, L, c, w, -0.2, 0.5)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, -0.2, 0.5)
    S, _, _ = ym.similarity(ctx, L, c, w)
    ties = parity.compare_mined(O, OL, c, w, F32(-0.2), F32(0.5), got, want, S)
    parity.assert_ties("long_64x2000x2200_pair7", ties)


def test_full_batch_sampled(ym, ctx, O):
    """The whole 10,000-pair batch in the benchmark's launch shape; the oracle
    checks a sample of pairs one by one and invariants hold everywhere."""
    cfg = synth.CONFIGS[1]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex)
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    dm = ym.DeviceMiner(ctx, L, c)
    dm.run(w, -0.2, 0.5)
    got = dm.result()
    n, m = c.nm()
    cnt = np.diff(got["pair_off"])
    assert np.all(cnt >= 0) and np.all(cnt <= np.minimum(n, m))
    assert np.all(got["score"] >= F32(0.5)) and np.all(got["score"] <= 1.0)
    for p in range(c.n_pairs):
        a, b = got["pair_off"][p], got["pair_off"][p + 1]
        assert np.all(np.diff(got["src_idx"][a:b]) > 0) and np.all(np.diff(got["tgt_idx"][a:b]) > 0)
    sample = np.random.default_rng(0).choice(c.n_pairs, 25, replace=False)
    sub = c.subset(sample)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, sub, w, -0.2, 0.5)
    got_sub = parity.select_pairs(got, sample)
    S, _, _ = ym.similarity(ctx, L, sub, w)
    ties = parity.compare_mined(O, OL, sub, w, F32(-0.2), F32(0.5), got_sub, want, S)
    parity.assert_ties("batch_10k_full_sample25", ties)
    # a second run gives the same bits
    dm.run(w, -0.2, 0.5)
    again = dm.result()
    for k in got:
        assert np.array_equal(got[k], again[k]), k


def test_errors(ym, ctx):
    L = ctx.lexicon(np.array([1], np.int32), np.array([0, 1]), np.array([2], np.int32))
    c = synth.from_lists([[[1, 2]]], [[[2]]])
    with pytest.raises(ym.YmError) as e:
        ym.mine(ctx, L, c, [np.nan, 0, 0, 0], -0.2, 0.5)
    assert e.value.code == ym.YM_EINVAL
    bad = synth.from_lists([[[1, 2], [3]]], [[[2]]])
    bad.src_sent_off = np.array([0, 2, 1], np.int64)  # decreasing sentence offsets
    with pytest.raises(ym.YmError) as e:
        ym.mine(ctx, L, bad, [0, 0, 0, 0], -0.2, 0.5)
    assert e.value.code == ym.YM_EINVAL
    with pytest.raises(ym.YmError) as e:
        ctx.lexicon(np.array([-1], np.int32), np.array([0, 1]), np.array([2], np.int32))
    assert e.value.code == ym.YM_EINVAL
    long_t = synth.from_lists([[[1]]], [[np.zeros(1025, np.int32)]])
    with pytest.raises(ym.YmError):
        ym.mine(ctx, L, long_t, [0, 0, 0, 0], -0.2, 0.5)
    long_s = synth.from_lists([[np.zeros(1025, np.int32)]], [[[1]]])
    with pytest.raises(ym.YmError):
        ym.mine(ctx, L, long_s, [0, 0, 0, 0], -0.2, 0.5)
    # empty batch
    empty = synth.from_lists([], [])
    r = ym.mine(ctx, L, empty, [0, 0, 0, 0], -0.2, 0.5)
    assert r["pair_off"].tolist() == [0]


@pytest.mark.parametrize("seed", [5, 6])
def test_similarity_variants_agree(ym, O, seed):
    """The bit-sliced tile kernels (one wave, four waves with both chunk
    sizes) and the lane-per-sentence kernel, with and without split reads,
    give the same counts and scores (all also match the oracle above)."""
    import os
    lex = parity.random_lexicon(seed, vocab=90)
    c = parity.random_corpus(seed, n_pairs=10, nmax=140, mmax=150, lmax_src=70, lmax_tgt=66)
    w = np.array([-2.0, 3.0, 2.5, 0.75], np.float32)
    outs = []
    for variant in ("tile", "lanes", "split", "bits", "bits2k"):
        old = os.environ.get("YM_SIM_KERNEL")
        os.environ["YM_SIM_KERNEL"] = variant
        try:
            cx = ym.Context(0)
        finally:
            if old is None:
                os.environ.pop("YM_SIM_KERNEL")
            else:
                os.environ["YM_SIM_KERNEL"] = old
        L = cx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
        outs.append(ym.similarity(cx, L, c, w))
        L.close()
        cx.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("kernel", [1, 2, 3, 4])
def test_scale_workload_sample(ym, ctx_k, O, kernel):
    """Pairs of the 1M-pair scale workload (3-60 token sentences, Zipf 1.05,
    1-4 translations per key): rows longer than 31 tokens take the one-row
    path, target sentences longer than 32 tokens the split reads (kernel 2);
    the mined sets match the oracle."""
    ctx = ctx_k(kernel)
    cfg = synth.CONFIGS[4]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex, pair_ids=np.arange(0, 1000000, 20000))
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    got = ym.mine(ctx, L, c, w, -0.2, 0.5)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, F32(-0.2), F32(0.5))
    S, _, _ = ym.similarity(ctx, L, c, w)
    ties = parity.compare_mined(O, OL, c, w, F32(-0.2), F32(0.5), got, want, S)
    parity.assert_ties("scale_1M_every_20000th", ties)
    lens = np.diff(c.src_sent_off)
    assert lens.max() > 31  # the long-row path is exercised


def test_single_pair_end_to_end(ym, ctx, O):
    """The single 40 x 45 pair (vocabulary 5k, 4,000 translated ids, 60%
    planted) through every entry point, against the oracle."""
    cfg = synth.CONFIGS[0]
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex)
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    want = O.mine(OL, c, w, F32(-0.2), F32(0.5))
    S, _, _ = ym.similarity(ctx, L, c, w)
    got = ym.mine(ctx, L, c, w, -0.2, 0.5)
    parity.assert_ties("single_40x45", parity.compare_mined(O, OL, c, w, F32(-0.2), F32(0.5), got, want, S))
    assert int(got["pair_off"][-1]) > 0
    dm = ym.DeviceMiner(ctx, L, c)
    dm.run(w, -0.2, 0.5)
    for r in (ym.mine_per_pair(ctx, L, c, w, -0.2, 0.5), dm.result()):
        parity.compare_result_fields(r, got, "single pair: forms differ")


def test_served_tail_pair_4000x4000(ym, ctx, O):
    """The largest request of the served stream (4,000 x 4,000 sentences,
    vocabulary 200k, 1M lexicon pairs), through the batch entry point and the
    server, against the oracle (scores computed in row bands)."""
    cfg = synth.config(3, count_kind=0, n_fixed=4000, m_fixed=4000, n_pairs=1)
    lex = synth.make_lexicon(cfg)
    c = synth.generate(cfg, lex)
    w = synth.weights(cfg.seed)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    src, tgt = c.pair(0)
    want, So = parity.oracle_pair_banded(O, OL, src, tgt, w, F32(-0.2), F32(0.5))
    got = ym.mine(ctx, L, c, w, -0.2, 0.5)
    if not (np.array_equal(got["src_idx"], want["src_idx"]) and np.array_equal(got["tgt_idx"], want["tgt_idx"])
            and got["align_score"].tobytes() == want["align_score"].tobytes()):
        S, _, _ = ym.similarity(ctx, L, c, w)
        assert np.max(np.abs(S - So.reshape(-1))) <= parity.TOL_S
        h, mv, _ = O.nw(S.reshape(4000, 4000), F32(-0.2))
        si, ti, _ = O.emit(S.reshape(4000, 4000), mv, F32(0.5))
        tie = [(0, np.argwhere(S.reshape(4000, 4000) != So).tolist())]
        assert np.array_equal(si, got["src_idx"]) and np.array_equal(ti, got["tgt_idx"]) and h == got["align_score"][0]
        parity.assert_ties("served_tail_4000x4000", tie)
    else:
        parity.compare_result_fields(got, want, "4000 x 4000")
        parity.assert_ties("served_tail_4000x4000", [])
    srv = ym.Server(ctx, L, w, -0.2, 0.5, max_pairs_per_step=8, use_graph=1)
    try:
        r = srv.poll(srv.submit(c))
    finally:
        srv.stop()
    parity.compare_result_fields(r, got, "served 4000 x 4000")


@pytest.mark.parametrize("large", [1, 0])
def test_pipelined_sweep_give_up_is_an_error(ym, O, large):
    """A bounded wait of the pipelined sweep that gives up (forced from the
    host: a zero wait limit makes every such wait give up at once, and every
    kernel still runs to its end) fails the call with YM_EDEVICE; pairs that
    do not need the pipelined sweep are not affected, and the default limit
    restores normal results.  Both sweeps of the large pairs."""
    ctx = ym.Context(0)
    ym.set_tuning(ctx, 1, 128, 1, large)
    r = np.random.default_rng(31)
    big = [r.random((700, 90)).astype(np.float32)]
    small = [r.random((60, 70)).astype(np.float32)]
    ym.set_wait_limit(ctx, 0)
    with pytest.raises(ym.YmError) as e:
        ym.nw_align(ctx, big + small, -0.2, 0.5)
    assert e.value.code == ym.YM_EDEVICE
    align, moves, res = ym.nw_align(ctx, small, -0.2, 0.5)
    assert align[0].tobytes() == O.nw(small[0], F32(-0.2))[0].tobytes()
    lex = parity.random_lexicon(3)
    c = parity.random_corpus(3, n_pairs=3, nmax=40, mmax=40, lmax_src=20, lmax_tgt=20)
    big_pair = synth.from_lists([[np.array([1, 2, 3], np.int32)] * 500], [[np.array([2, 3], np.int32)] * 60])
    w = np.array([-1.5, 3.0, 2.0, 0.5], np.float32)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    with pytest.raises(ym.YmError) as e:
        ym.mine(ctx, L, big_pair, w, -0.2, 0.5)
    assert e.value.code == ym.YM_EDEVICE
    dm = ym.DeviceMiner(ctx, L, big_pair)
    dm.run(w, -0.2, 0.5)
    with pytest.raises(ym.YmError) as e:
        dm.result()
    assert e.value.code == ym.YM_EDEVICE
    srv = ym.Server(ctx, L, w, -0.2, 0.5, max_pairs_per_step=4)
    try:
        t_small = srv.submit(c.subset([0]))
        t_big = srv.submit(big_pair)
        t_small2 = srv.submit(c.subset([1]))
        with pytest.raises(ym.YmError) as e:
            srv.poll(t_big)
        assert e.value.code == ym.YM_EDEVICE
        assert srv.poll(t_small) is not None and srv.poll(t_small2) is not None
    finally:
        srv.stop()
    ym.set_wait_limit(ctx, -1)
    got = ym.mine(ctx, L, big_pair, w, -0.2, 0.5)
    OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    parity.compare_result_fields(got, O.mine(OL, big_pair, w, F32(-0.2), F32(0.5)), "after the limit is restored")
    dm.run(w, -0.2, 0.5)
    parity.compare_result_fields(dm.result(), got, "device form after the limit is restored")
