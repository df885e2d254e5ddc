"""CPU oracle of the comparable-corpus miner -- test infrastructure only.

Plain single-threaded C (``oracle.c``) behind ctypes.  It states what the
miner computes (Section 4 of the paper: a probability score for every
source/target sentence pair, Needleman-Wunsch alignment of the score matrix
with a monotone path and a skip penalty, and a confidence threshold) and is
used only by the test suite, the smoke check and the benchmark's CPU-baseline
leg.  The GPU library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]


def build(force: bool = True, extra=(), out: str | None = None) -> str:
    """Compile liboracle.so (or `out`) from oracle.c with gcc."""
    out = out or _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *extra, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str | None = None):
        if path is None:
            path = _LIB
            if not os.path.exists(path):
                build(force=False)
        lib = C.CDLL(path)
        lib.oracle_lex_build.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                         C.c_int64, C.POINTER(C.c_void_p)]
        lib.oracle_lex_free.argtypes = [C.c_void_p]
        lib.oracle_score.argtypes = [C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        lib.oracle_score.restype = C.c_float
        lib.oracle_similarity.argtypes = [
            C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int32,
            C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_float),
            C.POINTER(C.c_float), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.oracle_nw.argtypes = [C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_float,
                                  C.POINTER(C.c_float), C.c_char_p, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_float)]
        lib.oracle_emit.argtypes = [C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_char_p, C.c_int32,
                                    C.c_float, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_float), C.POINTER(C.c_int32)]
        lib.oracle_mine_threads.argtypes = [
            C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
            C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_float),
            C.c_float, C.c_float, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
            C.POINTER(C.c_float), C.POINTER(C.c_float)]
        lib.oracle_mine.argtypes = [
            C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
            C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_float),
            C.c_float, C.c_float, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
            C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float)]
        self.lib = lib

    # -- lexicon -----------------------------------------------------------
    def lexicon(self, src_ids, off, tgt_ids) -> "OLex":
        src_ids = np.ascontiguousarray(src_ids, np.int32)
        off = np.ascontiguousarray(off, np.int64)
        tgt_ids = np.ascontiguousarray(tgt_ids if len(tgt_ids) else np.zeros(1), np.int32)
        h = C.c_void_p()
        rc = self.lib.oracle_lex_build(_p(src_ids, C.c_int32), _p(off, C.c_int64), _p(tgt_ids, C.c_int32),
                                       src_ids.shape[0], C.byref(h))
        if rc:
            raise MemoryError("oracle_lex_build")
        return OLex(self, h)

    # -- single pieces ---------------------------------------------------------
    def score(self, w, ms, a, mt, b) -> np.float32:
        w = np.ascontiguousarray(w, np.float32)
        return np.float32(self.lib.oracle_score(_p(w, C.c_float), ms, a, mt, b))

    def similarity(self, lex: "OLex", src_sents, tgt_sents, w):
        """S, m_s, m_t for one document pair given as lists of token arrays."""
        so, st = _flat(src_sents)
        to, tt = _flat(tgt_sents)
        n, m = len(src_sents), len(tgt_sents)
        S = np.zeros((n, m), np.float32)
        ms = np.zeros((n, m), np.int32)
        mt = np.zeros((n, m), np.int32)
        w = np.ascontiguousarray(w, np.float32)
        rc = self.lib.oracle_similarity(lex.h, _p(so, C.c_int64), _p(st, C.c_int32), n, _p(to, C.c_int64),
                                        _p(tt, C.c_int32), m, _p(w, C.c_float), _p(S, C.c_float),
                                        _p(ms, C.c_int32), _p(mt, C.c_int32))
        if rc:
            raise MemoryError("oracle_similarity")
        return S, ms, mt

    def nw(self, S, g, want_H=False):
        """(H[n][m], forward move string, full H or None)."""
        S = np.ascontiguousarray(S, np.float32)
        n, m = S.shape
        H = np.zeros((n + 1, m + 1), np.float32) if want_H else None
        mv = C.create_string_buffer(n + m + 1)
        nmv = C.c_int32()
        h = C.c_float()
        Sp = _p(S, C.c_float) if S.size else _p(np.zeros(1, np.float32), C.c_float)
        rc = self.lib.oracle_nw(Sp, n, m, np.float32(g), _p(H, C.c_float) if want_H else None, mv,
                                C.byref(nmv), C.byref(h))
        if rc:
            raise MemoryError("oracle_nw")
        return np.float32(h.value), mv.raw[: nmv.value].decode(), H

    def emit(self, S, moves: str, tau):
        S = np.ascontiguousarray(S, np.float32)
        n, m = S.shape
        cap = max(min(n, m), 1)
        si = np.zeros(cap, np.int32)
        ti = np.zeros(cap, np.int32)
        sc = np.zeros(cap, np.float32)
        cnt = C.c_int32()
        Sp = _p(S, C.c_float) if S.size else _p(np.zeros(1, np.float32), C.c_float)
        self.lib.oracle_emit(Sp, n, m, moves.encode(), len(moves), np.float32(tau), _p(si, C.c_int32),
                             _p(ti, C.c_int32), _p(sc, C.c_float), C.byref(cnt))
        k = cnt.value
        return si[:k], ti[:k], sc[:k]

    def mine(self, lex: "OLex", corpus, w, g, tau, want_S=False):
        """Whole miner over a packed corpus: dict of numpy arrays."""
        n, m = corpus.nm()
        cap = int(np.minimum(n, m).sum()) + 1
        P = corpus.n_pairs
        pair_off = np.zeros(P + 1, np.int64)
        si = np.zeros(cap, np.int32)
        ti = np.zeros(cap, np.int32)
        sc = np.zeros(cap, np.float32)
        al = np.zeros(max(P, 1), np.float32)
        S = np.zeros(max(corpus.cells(), 1), np.float32) if want_S else None
        w = np.ascontiguousarray(w, np.float32)
        c = corpus
        rc = self.lib.oracle_mine(
            lex.h, P, _p(c.src_doc_off, C.c_int64), _p(c.src_sent_off, C.c_int64),
            _p(_nz(c.src_tok), C.c_int32), _p(c.tgt_doc_off, C.c_int64), _p(c.tgt_sent_off, C.c_int64),
            _p(_nz(c.tgt_tok), C.c_int32), _p(w, C.c_float), np.float32(g), np.float32(tau),
            _p(pair_off, C.c_int64), _p(si, C.c_int32), _p(ti, C.c_int32), _p(sc, C.c_float),
            _p(al, C.c_float), _p(S, C.c_float) if want_S else None)
        if rc:
            raise MemoryError("oracle_mine")
        k = int(pair_off[-1])
        out = dict(pair_off=pair_off, src_idx=si[:k], tgt_idx=ti[:k], score=sc[:k], align_score=al[:P])
        if want_S:
            out["S"] = S[: corpus.cells()]
        return out


def _mine_threads(self, lex, corpus, w, g, tau, threads):
    """oracle_mine_threads: the per-pair oracle over `threads` worker threads."""
    n, m = corpus.nm()
    cap = int(np.minimum(n, m).sum()) + 1
    P = corpus.n_pairs
    pair_off = np.zeros(P + 1, np.int64)
    si = np.zeros(cap, np.int32)
    ti = np.zeros(cap, np.int32)
    sc = np.zeros(cap, np.float32)
    al = np.zeros(max(P, 1), np.float32)
    w = np.ascontiguousarray(w, np.float32)
    c = corpus
    rc = self.lib.oracle_mine_threads(
        lex.h, P, _p(c.src_doc_off, C.c_int64), _p(c.src_sent_off, C.c_int64), _p(_nz(c.src_tok), C.c_int32),
        _p(c.tgt_doc_off, C.c_int64), _p(c.tgt_sent_off, C.c_int64), _p(_nz(c.tgt_tok), C.c_int32),
        _p(w, C.c_float), np.float32(g), np.float32(tau), int(threads), _p(pair_off, C.c_int64),
        _p(si, C.c_int32), _p(ti, C.c_int32), _p(sc, C.c_float), _p(al, C.c_float))
    if rc:
        raise MemoryError("oracle_mine_threads")
    k = int(pair_off[-1])
    return dict(pair_off=pair_off, src_idx=si[:k], tgt_idx=ti[:k], score=sc[:k], align_score=al[:P])


Oracle.mine_threads = _mine_threads


class OLex:
    def __init__(self, owner: Oracle, h):
        self.owner = owner
        self.h = h

    def __del__(self):
        try:
            self.owner.lib.oracle_lex_free(self.h)
        except Exception:
            pass


def _nz(a):
    a = np.ascontiguousarray(a)
    return a if a.size else np.zeros(1, a.dtype)


def _flat(sents):
    off = [0]
    for s in sents:
        off.append(off[-1] + len(s))
    tok = np.concatenate([np.asarray(s, np.int32).reshape(-1) for s in sents]) if off[-1] else np.zeros(1, np.int32)
    return np.asarray(off, np.int64), np.ascontiguousarray(tok, np.int32)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
