"""Seeded synthetic comparable corpora (test and benchmark input only).

The paper's inputs (comparable Wikipedia article pairs, Table 3; the corpora
of Table 1) are not available, so every run draws documents, a bilingual
lexicon and classifier weights from this generator.  It contains none of the
miner's arithmetic; the GPU path and the CPU oracle both receive its arrays.

The generator itself is plain C (``synth.c``) behind ctypes; ``build()``
compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

BASE_SEED = 150908639


def build(force: bool = True) -> str:
    """Compile libsynth.so next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-pthread", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("vocab", C.c_int32),
        ("zipf_s", C.c_double),
        ("len_min", C.c_int32),
        ("len_max", C.c_int32),
        ("count_kind", C.c_int32),
        ("n_fixed", C.c_int32),
        ("m_fixed", C.c_int32),
        ("cmin", C.c_int32),
        ("cmax", C.c_int32),
        ("ln_median", C.c_double),
        ("ln_sigma", C.c_double),
        ("ln_cap", C.c_int32),
        ("plant_frac", C.c_double),
        ("replace_p", C.c_double),
        ("indel_max", C.c_int32),
        ("shuffle_block", C.c_int32),
        ("primary_only", C.c_int32),
    ]


class _Corpus(C.Structure):
    _fields_ = [
        ("n_pairs", C.c_int64),
        ("src_doc_off", C.POINTER(C.c_int64)),
        ("src_sent_off", C.POINTER(C.c_int64)),
        ("src_tok", C.POINTER(C.c_int32)),
        ("tgt_doc_off", C.POINTER(C.c_int64)),
        ("tgt_sent_off", C.POINTER(C.c_int64)),
        ("tgt_tok", C.POINTER(C.c_int32)),
        ("n_src_sent", C.c_int64),
        ("n_tgt_sent", C.c_int64),
        ("n_src_tok", C.c_int64),
        ("n_tgt_tok", C.c_int64),
        ("truth_off", C.POINTER(C.c_int64)),
        ("truth_src", C.POINTER(C.c_int32)),
        ("truth_tgt", C.POINTER(C.c_int32)),
        ("n_truth", C.c_int64),
    ]


class _Lex(C.Structure):
    _fields_ = [
        ("n_src", C.c_int64),
        ("src_ids", C.POINTER(C.c_int32)),
        ("off", C.POINTER(C.c_int64)),
        ("tgt_ids", C.POINTER(C.c_int32)),
        ("n_tgt", C.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        lib.synth_generate.argtypes = [
            C.POINTER(_Cfg), C.c_uint64, C.POINTER(C.c_int64), C.c_int64,
            C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(_Corpus),
        ]
        lib.synth_free.argtypes = [C.POINTER(_Corpus)]
        lib.synth_generate_mt.argtypes = [
            C.POINTER(_Cfg), C.c_uint64, C.POINTER(C.c_int64), C.c_int64,
            C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int,
            C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]
        lib.synth_collect.argtypes = [C.c_void_p] + [C.c_void_p] * 9
        lib.synth_make_lexicon.argtypes = [
            C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int64, C.c_uint64, C.POINTER(_Lex)]
        lib.synth_free_lexicon.argtypes = [C.POINTER(_Lex)]
        lib.synth_weights.argtypes = [C.c_uint64, C.POINTER(C.c_float)]
        lib.synth_arrivals.argtypes = [C.c_uint64, C.c_double, C.c_int64, C.POINTER(C.c_double)]
        lib.synth_uniform_ints.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int64,
                                           C.POINTER(C.c_int64)]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


@dataclass
class Lexicon:
    """CSR lexicon: target ids tgt_ids[off[k]:off[k+1]] translate source id src_ids[k]."""
    src_ids: np.ndarray  # int32 [n_src]
    off: np.ndarray  # int64 [n_src+1]
    tgt_ids: np.ndarray  # int32 [off[-1]]

    @property
    def n_src(self) -> int:
        return int(self.src_ids.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.tgt_ids.shape[0])

    def dense(self, vocab: int):
        """first/count arrays indexed by source id < vocab (for planting)."""
        first = np.zeros(vocab, dtype=np.int64)
        count = np.zeros(vocab, dtype=np.int32)
        ids = self.src_ids
        keep = ids < vocab
        first[ids[keep]] = self.off[:-1][keep]
        count[ids[keep]] = (self.off[1:] - self.off[:-1])[keep].astype(np.int32)
        return first, count


@dataclass
class Corpus:
    """A batch of document pairs in packed ragged (three-level CSR) form.

    Pair p's source document is sentences src_doc_off[p]..src_doc_off[p+1];
    sentence s holds tokens src_tok[src_sent_off[s]:src_sent_off[s+1]].
    Same for the target side.  truth_* lists the planted (src, tgt) sentence
    index pairs of each pair (ground truth for recall, not for parity).
    """
    src_doc_off: np.ndarray
    src_sent_off: np.ndarray
    src_tok: np.ndarray
    tgt_doc_off: np.ndarray
    tgt_sent_off: np.ndarray
    tgt_tok: np.ndarray
    truth_off: np.ndarray = field(default=None)
    truth_src: np.ndarray = field(default=None)
    truth_tgt: np.ndarray = field(default=None)
    pair_ids: np.ndarray = field(default=None)

    @property
    def n_pairs(self) -> int:
        return int(self.src_doc_off.shape[0] - 1)

    def nm(self):
        n = np.diff(self.src_doc_off).astype(np.int64)
        m = np.diff(self.tgt_doc_off).astype(np.int64)
        return n, m

    def cells(self) -> int:
        n, m = self.nm()
        return int((n * m).sum())

    def pair(self, p: int):
        """(src sentences, tgt sentences) of pair p as lists of int32 arrays."""
        def side(doc, sent, tok):
            s0, s1 = int(doc[p]), int(doc[p + 1])
            return [tok[sent[s]:sent[s + 1]] for s in range(s0, s1)]
        return (side(self.src_doc_off, self.src_sent_off, self.src_tok),
                side(self.tgt_doc_off, self.tgt_sent_off, self.tgt_tok))

    def slice(self, p0: int, p1: int) -> "Corpus":
        """Pairs [p0, p1) as a new packed corpus (array slices, rebased offsets)."""
        def side(doc, sent, tok):
            s0, s1 = int(doc[p0]), int(doc[p1])
            t0, t1 = int(sent[s0]), int(sent[s1])
            return doc[p0:p1 + 1] - s0, sent[s0:s1 + 1] - t0, tok[t0:t1].copy()
        a = side(self.src_doc_off, self.src_sent_off, self.src_tok)
        b = side(self.tgt_doc_off, self.tgt_sent_off, self.tgt_tok)
        return Corpus(a[0], a[1], a[2], b[0], b[1], b[2])

    def subset(self, pairs) -> "Corpus":
        """A new packed corpus holding the listed pairs, in that order."""
        srcs, tgts = [], []
        for p in pairs:
            s, t = self.pair(int(p))
            srcs.append(s)
            tgts.append(t)
        return from_lists(srcs, tgts)


def from_lists(src_docs, tgt_docs) -> Corpus:
    """Pack lists of documents (lists of token-id sequences) into a Corpus."""
    def pack(docs):
        doc_off = [0]
        sent_off = [0]
        toks = []
        for d in docs:
            for s in d:
                s = np.asarray(s, dtype=np.int32).reshape(-1)
                toks.append(s)
                sent_off.append(sent_off[-1] + s.shape[0])
            doc_off.append(len(sent_off) - 1)
        tok = np.concatenate(toks).astype(np.int32) if toks else np.zeros(0, np.int32)
        return (np.asarray(doc_off, np.int64), np.asarray(sent_off, np.int64), tok)
    a = pack(src_docs)
    b = pack(tgt_docs)
    return Corpus(a[0], a[1], a[2], b[0], b[1], b[2])


@dataclass
class Config:
    name: str
    vocab: int
    zipf_s: float
    len_min: int
    len_max: int
    count_kind: int  # 0 fixed, 1 uniform, 2 lognormal
    n_fixed: int = 0
    m_fixed: int = 0
    cmin: int = 0
    cmax: int = 0
    ln_median: float = 0.0
    ln_sigma: float = 0.0
    ln_cap: int = 0
    plant_frac: float = 0.4
    replace_p: float = 0.2
    indel_max: int = 2
    shuffle_block: int = 0
    primary_only: int = 0
    # lexicon
    lex_translated: int = 0
    lex_kmin: int = 1
    lex_kmax: int = 3
    lex_pairs: int = 0
    n_pairs: int = 1
    seed_offset: int = 0
    arrival_rate: float = 0.0
    arrival_seconds: float = 0.0

    @property
    def seed(self) -> int:
        return BASE_SEED + self.seed_offset

    def _c(self) -> _Cfg:
        return _Cfg(self.vocab, self.zipf_s, self.len_min, self.len_max, self.count_kind,
                    self.n_fixed, self.m_fixed, self.cmin, self.cmax, self.ln_median,
                    self.ln_sigma, self.ln_cap, self.plant_frac, self.replace_p,
                    self.indel_max, self.shuffle_block, self.primary_only)


# The five workloads.  Sizes follow the evaluation setting chosen for this
# miner (document-pair batches shaped like comparable article pairs).
CONFIGS = {
    # one pair, 40 x 45 sentences, vocab 5k, 4k translated ids
    0: Config("single_40x45", vocab=5000, zipf_s=1.1, len_min=5, len_max=30, count_kind=0,
              n_fixed=40, m_fixed=45, plant_frac=0.6, lex_translated=4000, lex_kmin=1,
              lex_kmax=3, lex_pairs=0, n_pairs=1, seed_offset=0),
    # 10,000 pairs, 20-200 sentences per side
    1: Config("batch_10k_u20_200", vocab=50000, zipf_s=1.1, len_min=5, len_max=30, count_kind=1,
              cmin=20, cmax=200, plant_frac=0.4, lex_translated=50000, lex_kmin=1, lex_kmax=3,
              lex_pairs=100000, n_pairs=10000, seed_offset=1),
    # 64 long pairs, 2000 x 2200 sentences, planted targets locally shuffled
    2: Config("long_64x2000x2200", vocab=200000, zipf_s=1.1, len_min=5, len_max=30, count_kind=0,
              n_fixed=2000, m_fixed=2200, plant_frac=0.3, shuffle_block=5,
              lex_translated=200000, lex_kmin=1, lex_kmax=3, lex_pairs=500000, n_pairs=64,
              seed_offset=2),
    # served stream: lognormal sentence counts, Poisson arrivals
    3: Config("served_lognormal80", vocab=200000, zipf_s=1.1, len_min=5, len_max=30, count_kind=2,
              ln_median=80.0, ln_sigma=1.0, ln_cap=4000, plant_frac=0.4,
              lex_translated=200000, lex_kmin=1, lex_kmax=3, lex_pairs=1000000,
              n_pairs=120000, seed_offset=3, arrival_rate=2000.0, arrival_seconds=60.0),
    # 1M pairs, lognormal(60, 0.8) counts, 3-60 token sentences
    4: Config("scale_1M_lognormal60", vocab=1000000, zipf_s=1.05, len_min=3, len_max=60,
              count_kind=2, ln_median=60.0, ln_sigma=0.8, ln_cap=1500, plant_frac=0.25,
              lex_translated=1000000, lex_kmin=1, lex_kmax=4, lex_pairs=4000000,
              n_pairs=1000000, seed_offset=4),
}


def make_lexicon(cfg: Config) -> Lexicon:
    lib = _load()
    L = _Lex()
    rc = lib.synth_make_lexicon(cfg.vocab, cfg.lex_translated, cfg.lex_kmin, cfg.lex_kmax,
                                cfg.lex_pairs, cfg.seed, C.byref(L))
    if rc != 0:
        raise RuntimeError(f"synth_make_lexicon failed ({rc})")
    try:
        src = np.ctypeslib.as_array(L.src_ids, shape=(L.n_src,)).copy()
        off = np.ctypeslib.as_array(L.off, shape=(L.n_src + 1,)).copy()
        tgt = np.ctypeslib.as_array(L.tgt_ids, shape=(max(L.n_tgt, 1),))[:L.n_tgt].copy()
    finally:
        lib.synth_free_lexicon(C.byref(L))
    return Lexicon(src, off, tgt)


def weights(seed: int) -> np.ndarray:
    lib = _load()
    w = (C.c_float * 4)()
    lib.synth_weights(seed, w)
    return np.array(list(w), dtype=np.float32)


def arrivals(seed: int, rate: float, n: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(n, dtype=np.float64)
    lib.synth_arrivals(seed, rate, n, _ptr(out, C.c_double))
    return out


def uniform_ints(seed: int, stream: int, n: int, lo: int, hi: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(n, dtype=np.int64)
    lib.synth_uniform_ints(seed, stream, n, lo, hi, _ptr(out, C.c_int64))
    return out


def generate(cfg: Config, lex: Lexicon, pair_ids=None, seed: int | None = None, threads: int | None = None) -> Corpus:
    """Documents for the listed pair ids (default: 0..cfg.n_pairs-1), drawn by
    `threads` worker threads (default: the CPUs this process may use, at most
    16); the result does not depend on the thread count."""
    lib = _load()
    if pair_ids is None:
        pair_ids = np.arange(cfg.n_pairs, dtype=np.int64)
    pair_ids = np.ascontiguousarray(pair_ids, dtype=np.int64)
    if threads is None:
        threads = min(16, len(os.sched_getaffinity(0)))
    first, count = lex.dense(cfg.vocab)
    tgt = np.ascontiguousarray(lex.tgt_ids if lex.tgt_ids.size else np.zeros(1, np.int32))
    c = cfg._c()
    job = C.c_void_p()
    tot = (C.c_int64 * 5)()
    rc = lib.synth_generate_mt(C.byref(c), cfg.seed if seed is None else seed,
                               _ptr(pair_ids, C.c_int64), pair_ids.shape[0],
                               _ptr(first, C.c_int64), _ptr(count, C.c_int32), _ptr(tgt, C.c_int32),
                               int(threads), C.byref(job), tot)
    if rc != 0:
        raise RuntimeError(f"synth_generate_mt failed ({rc})")
    P = pair_ids.shape[0]
    ns, nt, nts, ntt, ntr = (int(x) for x in tot)
    out = [np.empty(P + 1, np.int64), np.empty(ns + 1, np.int64), np.empty(max(nts, 1), np.int32),
           np.empty(P + 1, np.int64), np.empty(nt + 1, np.int64), np.empty(max(ntt, 1), np.int32),
           np.empty(P + 1, np.int64), np.empty(max(ntr, 1), np.int32), np.empty(max(ntr, 1), np.int32)]
    rc = lib.synth_collect(job, *[a.ctypes.data_as(C.c_void_p) for a in out])
    if rc != 0:
        raise RuntimeError(f"synth_collect failed ({rc})")
    return Corpus(out[0], out[1], out[2][:nts], out[3], out[4], out[5][:ntt], out[6], out[7][:ntr], out[8][:ntr],
                  pair_ids.copy())


def config(k: int, **over) -> Config:
    """A copy of workload k with fields overridden."""
    import dataclasses
    return dataclasses.replace(CONFIGS[k], **over)
