"""Thin Python binding of libymine (the C ABI in include/ymine.h).

Argument marshalling only: every step of the miner runs in the library's HIP
kernels.  PyTorch appears only for device memory and streams in the
device-resident entry point.  If the compiled library is missing the import
of this module's functions fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libymine.so")

YM_OK = 0
YM_EPENDING = 1
YM_EINVAL = -1
YM_ENOMEM = -2
YM_EDEVICE = -3
YM_EBUDGET = -4
YM_ECANCELLED = -5
YM_ENOTFOUND = -6

STATIC_SCRATCH_BYTES = 256 << 20  # YM_STATIC_SCRATCH_BYTES: workspace of ym_mine_device_static

# Every symbol declared in include/ymine.h.
EXPORTS = [
    "ym_create", "ym_destroy", "ym_last_error", "ym_version", "ym_lexicon_load", "ym_lexicon_free",
    "ym_lexicon_stats", "ym_mine", "ym_result_free", "ym_mine_per_pair", "ym_mine_device_capacity",
    "ym_mine_device_workspace", "ym_mine_device_workspace_min", "ym_mine_device", "ym_similarity",
    "ym_nw_align", "ym_tune", "ym_mine_bidirectional", "ym_set_tuning", "ym_get_tuning", "ym_autotune",
    "ym_profile_enable", "ym_profile_read", "ym_server_start", "ym_submit", "ym_poll", "ym_server_next_done", "ym_cancel",
    "ym_server_stop",
    "ym_server_stats", "ym_server_graph_stats", "ym_check_pair", "ym_set_wait_limit", "ym_mine_device_static",
    "ym_tune_select",
]


class YmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ymine error {code}: {msg}")
        self.code = code


P = C.POINTER
i32, i64, f32, u64, vp = C.c_int32, C.c_int64, C.c_float, C.c_uint64, C.c_void_p


class Batch(C.Structure):
    _fields_ = [("n_pairs", i64), ("src_doc_off", P(i64)), ("src_sent_off", P(i64)), ("src_tok", P(i32)),
                ("tgt_doc_off", P(i64)), ("tgt_sent_off", P(i64)), ("tgt_tok", P(i32))]


class Params(C.Structure):
    _fields_ = [("w", f32 * 4), ("gap", f32), ("threshold", f32)]


class Result(C.Structure):
    _fields_ = [("n_pairs", i64), ("n_out", i64), ("pair_off", P(i64)), ("src_idx", P(i32)),
                ("tgt_idx", P(i32)), ("score", P(f32)), ("align_score", P(f32))]


class DeviceBatch(C.Structure):
    _fields_ = [("n_pairs", i64), ("src_doc_off", P(i64)), ("tgt_doc_off", P(i64)), ("src_sent_off", vp),
                ("src_tok", vp), ("tgt_sent_off", vp), ("tgt_tok", vp), ("n_src_tok", i64),
                ("n_tgt_tok", i64)]


class DeviceOut(C.Structure):
    _fields_ = [("pair_off", vp), ("src_idx", vp), ("tgt_idx", vp), ("score", vp), ("align_score", vp),
                ("status", vp)]


class Tuning(C.Structure):
    _fields_ = [("sim_kernel", C.c_int32), ("item_rows", C.c_int32), ("nw_pairs_per_group", C.c_int32),
                ("nw_large", C.c_int32)]

    def as_dict(self):
        return dict(sim_kernel=self.sim_kernel, item_rows=self.item_rows, nw_pairs_per_group=self.nw_pairs_per_group,
                    nw_large=self.nw_large)


class ServerOpts(C.Structure):
    _fields_ = [("max_pairs_per_step", i32), ("max_cells_per_step", i64), ("use_graph", i32)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    L.ym_create.argtypes = [C.c_int, C.c_size_t, P(vp)]
    L.ym_destroy.argtypes = [vp]
    L.ym_destroy.restype = None
    L.ym_last_error.restype = C.c_char_p
    L.ym_version.restype = C.c_char_p
    L.ym_lexicon_load.argtypes = [vp, P(i32), P(i64), P(i32), i64, P(vp)]
    L.ym_lexicon_free.argtypes = [vp]
    L.ym_lexicon_free.restype = None
    L.ym_lexicon_stats.argtypes = [vp, P(i64), P(i64), P(i32)]
    L.ym_mine.argtypes = [vp, vp, P(Batch), P(Params), P(P(Result))]
    L.ym_mine_per_pair.argtypes = [vp, vp, P(Batch), P(Params), P(P(Result))]
    L.ym_result_free.argtypes = [P(Result)]
    L.ym_result_free.restype = None
    L.ym_mine_device_capacity.argtypes = [P(i64), P(i64), i64]
    L.ym_mine_device_capacity.restype = i64
    L.ym_mine_device_workspace.argtypes = [P(i64), P(i64), i64, i64]
    L.ym_mine_device_workspace.restype = C.c_size_t
    L.ym_mine_device_workspace_min.argtypes = [P(i64), P(i64), i64, i64]
    L.ym_mine_device_workspace_min.restype = C.c_size_t
    L.ym_mine_device.argtypes = [vp, vp, P(DeviceBatch), P(Params), vp, C.c_size_t, P(DeviceOut), vp]
    L.ym_mine_device_static.argtypes = [vp, vp, P(DeviceBatch), P(Params), P(DeviceOut), vp]
    L.ym_similarity.argtypes = [vp, vp, P(Batch), P(Params), P(f32), P(i32), P(i32)]
    L.ym_nw_align.argtypes = [vp, P(f32), P(i32), P(i32), i64, f32, f32, P(f32), C.c_char_p, P(i32),
                              P(P(Result))]
    L.ym_tune.argtypes = [vp, vp, P(Batch), P(f32), P(f32), i32, P(f32), i32, P(i64), P(i32), P(i32), P(i64), P(i64)]
    L.ym_mine_bidirectional.argtypes = [vp, vp, vp, P(Batch), P(Params), P(Params), P(P(Result))]
    L.ym_set_tuning.argtypes = [vp, P(Tuning)]
    L.ym_get_tuning.argtypes = [vp, P(Tuning)]
    L.ym_autotune.argtypes = [vp, vp, P(Batch), P(Params), i32, P(Tuning), P(C.c_double)]
    L.ym_profile_enable.argtypes = [vp, C.c_int]
    L.ym_profile_read.argtypes = [vp, P(C.c_double), P(i64)]
    L.ym_server_start.argtypes = [vp, vp, P(Params), P(ServerOpts), P(vp)]
    L.ym_submit.argtypes = [vp, P(Batch), P(u64)]
    L.ym_poll.argtypes = [vp, u64, i64, P(P(Result))]
    L.ym_server_next_done.argtypes = [vp, i64, P(u64), P(i64)]
    L.ym_cancel.argtypes = [vp, u64]
    L.ym_server_stop.argtypes = [vp]
    L.ym_server_stats.argtypes = [vp, P(i64), P(i64), P(i64)]
    L.ym_server_graph_stats.argtypes = [vp, P(i64), P(i64)]
    L.ym_check_pair.argtypes = [i64, i64]
    L.ym_set_wait_limit.argtypes = [vp, i64]
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise YmError(rc, lib().ym_last_error().decode(errors="replace"))
    return rc


def _ptr(a, ct):
    return a.ctypes.data_as(P(ct))


def _c(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a if a.size else np.zeros(1, dt)


def params(w, gap, threshold) -> Params:
    p = Params()
    for k in range(4):
        p.w[k] = float(np.float32(w[k]))
    p.gap = float(np.float32(gap))
    p.threshold = float(np.float32(threshold))
    return p


class _HostBatch:
    """Keeps the numpy arrays of a ctypes Batch alive."""

    def __init__(self, corpus):
        self.arrs = [_c(corpus.src_doc_off, np.int64), _c(corpus.src_sent_off, np.int64), _c(corpus.src_tok, np.int32),
                     _c(corpus.tgt_doc_off, np.int64), _c(corpus.tgt_sent_off, np.int64), _c(corpus.tgt_tok, np.int32)]
        a = self.arrs
        self.b = Batch(int(corpus.src_doc_off.shape[0] - 1), _ptr(a[0], i64), _ptr(a[1], i64), _ptr(a[2], i32),
                       _ptr(a[3], i64), _ptr(a[4], i64), _ptr(a[5], i32))


def prepare(corpus):
    """Pack a corpus into ctypes form once (for repeated or timed submission)."""
    return _HostBatch(corpus)


def mine_prepared(ctx: Context, lex: Lexicon, hb, p: Params, per_pair: bool = False) -> dict:
    rp = P(Result)()
    fn = lib().ym_mine_per_pair if per_pair else lib().ym_mine
    _check(fn(ctx.h, lex.h, C.byref(hb.b), C.byref(p), C.byref(rp)))
    return _result_to_numpy(rp)


def _result_to_numpy(rp) -> dict:
    r = rp.contents
    n, k = r.n_pairs, r.n_out

    def arr(p, cnt, dt):
        if cnt == 0:
            return np.zeros(0, dt)
        return np.ctypeslib.as_array(p, shape=(cnt,)).copy()
    out = dict(pair_off=arr(r.pair_off, n + 1, np.int64), src_idx=arr(r.src_idx, k, np.int32),
               tgt_idx=arr(r.tgt_idx, k, np.int32), score=arr(r.score, k, np.float32),
               align_score=arr(r.align_score, n, np.float32))
    lib().ym_result_free(rp)
    return out


class Context:
    """A device context (ym_create)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import weakref
        self.h = vp()
        self._deps = weakref.WeakSet()  # servers and lexicons, closed before the context
        _check(lib().ym_create(device, hbm_budget_bytes, C.byref(self.h)))

    def close(self):
        if self.h:
            for d in sorted(list(self._deps), key=lambda o: 0 if isinstance(o, Server) else 1):
                d.close()
            lib().ym_destroy(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool):
        _check(lib().ym_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self):
        """{kernel: (ms summed, launches)} since the last read."""
        ms = (C.c_double * 4)()
        n = (i64 * 4)()
        _check(lib().ym_profile_read(self.h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(("similarity", "nw", "compact", "translate"))}

    def lexicon(self, src_ids, off, tgt_ids) -> "Lexicon":
        return Lexicon(self, src_ids, off, tgt_ids)


class Lexicon:
    def __init__(self, ctx: Context, src_ids, off, tgt_ids):
        self.ctx = ctx
        self.h = vp()
        ctx._deps.add(self)
        s, o, t = _c(src_ids, np.int32), _c(off, np.int64), _c(tgt_ids, np.int32)
        _check(lib().ym_lexicon_load(ctx.h, _ptr(s, i32), _ptr(o, i64), _ptr(t, i32), int(np.asarray(src_ids).shape[0]),
                                     C.byref(self.h)))

    def stats(self):
        a, b, c = i64(), i64(), i32()
        _check(lib().ym_lexicon_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if self.h:
            lib().ym_lexicon_free(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mine(ctx: Context, lex: Lexicon, corpus, w, gap, threshold) -> dict:
    """ym_mine on a host corpus (synth.Corpus-like)."""
    hb = _HostBatch(corpus)
    p = params(w, gap, threshold)
    rp = P(Result)()
    _check(lib().ym_mine(ctx.h, lex.h, C.byref(hb.b), C.byref(p), C.byref(rp)))
    return _result_to_numpy(rp)


def mine_per_pair(ctx: Context, lex: Lexicon, corpus, w, gap, threshold) -> dict:
    """ym_mine_per_pair: one launch sequence per pair, synchronised each time."""
    hb = _HostBatch(corpus)
    p = params(w, gap, threshold)
    rp = P(Result)()
    _check(lib().ym_mine_per_pair(ctx.h, lex.h, C.byref(hb.b), C.byref(p), C.byref(rp)))
    return _result_to_numpy(rp)


def similarity(ctx: Context, lex: Lexicon, corpus, w):
    """ym_similarity: flat S, m_s, m_t (pairs back to back, row-major)."""
    hb = _HostBatch(corpus)
    p = params(w, 0.0, 0.0)
    n = np.diff(corpus.src_doc_off)
    m = np.diff(corpus.tgt_doc_off)
    cells = int((n * m).sum())
    S = np.zeros(max(cells, 1), np.float32)
    ms = np.zeros(max(cells, 1), np.int32)
    mt = np.zeros(max(cells, 1), np.int32)
    _check(lib().ym_similarity(ctx.h, lex.h, C.byref(hb.b), C.byref(p), _ptr(S, f32), _ptr(ms, i32), _ptr(mt, i32)))
    return S[:cells], ms[:cells], mt[:cells]


def nw_align(ctx: Context, mats, gap, threshold):
    """ym_nw_align on a list of score matrices: (align, moves list, result dict)."""
    mats = [np.ascontiguousarray(S, np.float32).reshape(np.shape(S)[0], np.shape(S)[1]) for S in mats]
    n = np.array([S.shape[0] for S in mats], np.int32)
    m = np.array([S.shape[1] for S in mats], np.int32)
    flat = np.concatenate([S.reshape(-1) for S in mats]) if mats else np.zeros(0, np.float32)
    flat = _c(flat, np.float32)
    P_ = len(mats)
    align = np.zeros(max(P_, 1), np.float32)
    mvlen = int((n.astype(np.int64) + m).sum())
    mv = C.create_string_buffer(max(mvlen, 1))
    nmv = np.zeros(max(P_, 1), np.int32)
    rp = P(Result)()
    _check(lib().ym_nw_align(ctx.h, _ptr(flat, f32), _ptr(_c(n, np.int32), i32), _ptr(_c(m, np.int32), i32), P_,
                             float(np.float32(gap)), float(np.float32(threshold)), _ptr(align, f32), mv,
                             _ptr(nmv, i32), C.byref(rp)))
    raw = mv.raw
    moves, base = [], 0
    for k in range(P_):
        moves.append(raw[base:base + int(nmv[k])].decode())
        base += int(n[k]) + int(m[k])
    return align[:P_], moves, _result_to_numpy(rp)


def tune(ctx: Context, lex: Lexicon, corpus, w, gaps, taus, truth_off, truth_src, truth_tgt):
    """ym_tune: (n_mined, n_correct) arrays of shape [len(gaps), len(taus)]."""
    hb = _HostBatch(corpus)
    w = _c(w, np.float32)
    g = _c(gaps, np.float32)
    t = _c(taus, np.float32)
    to, ts, tt = _c(truth_off, np.int64), _c(truth_src, np.int32), _c(truth_tgt, np.int32)
    nm = np.zeros(len(gaps) * len(taus), np.int64)
    nc = np.zeros(len(gaps) * len(taus), np.int64)
    _check(lib().ym_tune(ctx.h, lex.h, C.byref(hb.b), _ptr(w, f32), _ptr(g, f32), len(gaps), _ptr(t, f32), len(taus),
                         _ptr(to, i64), _ptr(ts, i32), _ptr(tt, i32), _ptr(nm, i64), _ptr(nc, i64)))
    return nm.reshape(len(gaps), len(taus)), nc.reshape(len(gaps), len(taus))


class TuneChoice(C.Structure):
    _fields_ = [("gap_index", i32), ("tau_index", i32), ("n_mined", i64), ("n_correct", i64),
                ("precision", C.c_double), ("recall", C.c_double), ("f1", C.c_double)]


def tune_select(n_mined, n_correct, n_truth: int) -> dict:
    """ym_tune_select: the sweep entry (gap index, threshold index) with the
    highest F1 against n_truth reference pairs, and its figures."""
    nm2 = np.atleast_2d(np.asarray(n_mined, np.int64))
    nc2 = np.atleast_2d(np.asarray(n_correct, np.int64))
    if nm2.shape != nc2.shape or nm2.ndim != 2:
        raise ValueError("n_mined and n_correct must be [n_gaps, n_taus] arrays of one shape")
    nm, nc = _c(nm2, np.int64), _c(nc2, np.int64)
    out = TuneChoice()
    _check(lib().ym_tune_select(_ptr(nm, i64), _ptr(nc, i64), nm2.shape[0], nm2.shape[1], int(n_truth), C.byref(out)))
    return dict(gap_index=out.gap_index, tau_index=out.tau_index, n_mined=out.n_mined, n_correct=out.n_correct,
                precision=out.precision, recall=out.recall, f1=out.f1)


def mine_bidirectional(ctx: Context, lex_fwd: Lexicon, lex_rev: Lexicon, corpus, w_fwd, w_rev, gap, threshold) -> dict:
    """ym_mine_bidirectional: union of forward and reverse mining per pair."""
    hb = _HostBatch(corpus)
    pf = params(w_fwd, gap, threshold)
    pr = params(w_rev, gap, threshold)
    rp = P(Result)()
    _check(lib().ym_mine_bidirectional(ctx.h, lex_fwd.h, lex_rev.h, C.byref(hb.b), C.byref(pf), C.byref(pr),
                                       C.byref(rp)))
    return _result_to_numpy(rp)


def check_pair(n: int, m: int) -> None:
    """Raise YmError(YM_EINVAL) if a pair of n x m sentences exceeds the library's limits (host only)."""
    _check(lib().ym_check_pair(int(n), int(m)))


def set_wait_limit(ctx: Context, ticks: int) -> None:
    """Limit of one bounded wait of the pipelined NW sweep (failure injection for tests; < 0: default)."""
    _check(lib().ym_set_wait_limit(ctx.h, int(ticks)))


def set_tuning(ctx: Context, sim_kernel: int, item_rows: int, nw_pairs_per_group: int, nw_large: int = 1):
    """ym_set_tuning: similarity kernel (1 lanes, 2 lanes with split reads of
    long target sentences, 0 bit-sliced tiles of one wave, 3 / 4 bit-sliced
    tiles of four waves with chunks of 1,280 / 2,048 tokens), source rows per
    work item (64, 128, 256), NW pairs per workgroup (1, 2, 4), and the sweep of
    pairs of 449+ source sentences (1 strips over every CU, 0 one workgroup per
    pair).  No choice changes a result."""
    t = Tuning(sim_kernel, item_rows, nw_pairs_per_group, nw_large)
    _check(lib().ym_set_tuning(ctx.h, C.byref(t)))


def get_tuning(ctx: Context) -> dict:
    """ym_get_tuning."""
    t = Tuning()
    _check(lib().ym_get_tuning(ctx.h, C.byref(t)))
    return t.as_dict()


def autotune(ctx: Context, lex: Lexicon, corpus, w, gap, threshold, reps: int = 3):
    """ym_autotune on a sample batch: (chosen configuration, its ms per pass)."""
    hb = _HostBatch(corpus)
    p = params(w, gap, threshold)
    t = Tuning()
    ms = C.c_double()
    _check(lib().ym_autotune(ctx.h, lex.h, C.byref(hb.b), C.byref(p), int(reps), C.byref(t), C.byref(ms)))
    return t.as_dict(), ms.value


class DeviceMiner:
    """ym_mine_device over a corpus resident in HBM (torch tensors for memory)."""

    def __init__(self, ctx: Context, lex: Lexicon, corpus, device="cuda", workspace_bytes=None):
        import torch
        self.torch = torch
        self.ctx, self.lex = ctx, lex
        self.sdo = _c(corpus.src_doc_off, np.int64)
        self.tdo = _c(corpus.tgt_doc_off, np.int64)
        self.n_pairs = int(corpus.src_doc_off.shape[0] - 1)
        t = lambda a, dt: torch.from_numpy(_c(a, dt)).to(device)
        self.d_ssent = t(corpus.src_sent_off, np.int64)
        self.d_tsent = t(corpus.tgt_sent_off, np.int64)
        self.d_stok = t(corpus.src_tok, np.int32)
        self.d_ttok = t(corpus.tgt_tok, np.int32)
        L = lib()
        self.cap = int(L.ym_mine_device_capacity(_ptr(self.sdo, i64), _ptr(self.tdo, i64), self.n_pairs))
        full = int(L.ym_mine_device_workspace(_ptr(self.sdo, i64), _ptr(self.tdo, i64), self.n_pairs,
                                              int(corpus.src_tok.shape[0])))
        self.ws_bytes = full if workspace_bytes is None else int(workspace_bytes)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)
        self.pair_off = torch.zeros(self.n_pairs + 1, dtype=torch.int64, device=device)
        self.align = torch.zeros(max(self.n_pairs, 1), dtype=torch.float32, device=device)
        self.src_idx = torch.zeros(max(self.cap, 1), dtype=torch.int32, device=device)
        self.tgt_idx = torch.zeros(max(self.cap, 1), dtype=torch.int32, device=device)
        self.score = torch.zeros(max(self.cap, 1), dtype=torch.float32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.b = DeviceBatch(self.n_pairs, _ptr(self.sdo, i64), _ptr(self.tdo, i64), self.d_ssent.data_ptr(),
                             self.d_stok.data_ptr(), self.d_tsent.data_ptr(), self.d_ttok.data_ptr(),
                             int(corpus.src_tok.shape[0]), int(corpus.tgt_tok.shape[0]))
        self.o = DeviceOut(self.pair_off.data_ptr(), self.src_idx.data_ptr(), self.tgt_idx.data_ptr(),
                           self.score.data_ptr(), self.align.data_ptr(), self.status.data_ptr())

    def run(self, w, gap, threshold, stream=None):
        """Enqueue one mining pass on `stream` (default: torch's current stream)."""
        p = params(w, gap, threshold)
        st = stream if stream is not None else self.torch.cuda.current_stream().cuda_stream
        _check(lib().ym_mine_device(self.ctx.h, self.lex.h, C.byref(self.b), C.byref(p), self.ws.data_ptr(),
                                    self.ws_bytes, C.byref(self.o), vp(st)))

    def run_static(self, w, gap, threshold, stream=None):
        """Enqueue one mining pass through the allocation-free entry point
        (ym_mine_device_static: the library's static scratch as workspace)."""
        p = params(w, gap, threshold)
        st = stream if stream is not None else self.torch.cuda.current_stream().cuda_stream
        _check(lib().ym_mine_device_static(self.ctx.h, self.lex.h, C.byref(self.b), C.byref(p), C.byref(self.o),
                                           vp(st)))

    def result(self) -> dict:
        """The last pass's result; raises YmError(YM_EDEVICE) if a pair could not be completed."""
        self.torch.cuda.synchronize()
        st = int(self.status.cpu().item())
        if st != 0:
            raise YmError(st, "a pair's pipelined Needleman-Wunsch sweep gave up on a bounded wait")
        po = self.pair_off.cpu().numpy()
        k = int(po[-1])
        return dict(pair_off=po, src_idx=self.src_idx[:k].cpu().numpy(), tgt_idx=self.tgt_idx[:k].cpu().numpy(),
                    score=self.score[:k].cpu().numpy(), align_score=self.align[:self.n_pairs].cpu().numpy())


class Server:
    """Continuous-batching server (ym_server_*)."""

    def __init__(self, ctx: Context, lex: Lexicon, w, gap, threshold, max_pairs_per_step=256,
                 max_cells_per_step=1 << 26, use_graph=0):
        self.ctx, self.lex = ctx, lex
        self.p = params(w, gap, threshold)
        self.opts = ServerOpts(max_pairs_per_step, max_cells_per_step, use_graph)
        self.h = vp()
        _check(lib().ym_server_start(ctx.h, lex.h, C.byref(self.p), C.byref(self.opts), C.byref(self.h)))
        ctx._deps.add(self)

    def submit(self, corpus_one_pair) -> int:
        return self.submit_prepared(prepare(corpus_one_pair))

    def submit_prepared(self, hb) -> int:
        """Submit a request packed beforehand with prepare()."""
        t = u64()
        _check(lib().ym_submit(self.h, C.byref(hb.b), C.byref(t)))
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        """Result dict, None while pending; raises YmError (YM_ECANCELLED, ...)."""
        rp = P(Result)()
        rc = _check(lib().ym_poll(self.h, ticket, timeout_us, C.byref(rp)))
        if rc == YM_EPENDING:
            return None
        return _result_to_numpy(rp)

    def next_done(self, timeout_us: int = -1):
        """(ticket, done time in ns of CLOCK_MONOTONIC) or None on timeout."""
        t, d = u64(), i64()
        rc = _check(lib().ym_server_next_done(self.h, timeout_us, C.byref(t), C.byref(d)))
        if rc == YM_EPENDING:
            return None
        return t.value, d.value

    def cancel(self, ticket: int):
        _check(lib().ym_cancel(self.h, ticket))

    def stats(self):
        a, b, c = i64(), i64(), i64()
        _check(lib().ym_server_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(steps=a.value, completed=b.value, cells=c.value)

    def graph_stats(self):
        a, b = i64(), i64()
        _check(lib().ym_server_graph_stats(self.h, C.byref(a), C.byref(b)))
        return dict(instantiations=a.value, updates=b.value)

    def stop(self):
        if self.h:
            _check(lib().ym_server_stop(self.h))
            self.h = vp()

    close = stop

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
