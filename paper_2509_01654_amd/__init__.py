"""Python binding of libnw (all-pairs Needleman-Wunsch scoring on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libnw.so`` behind the C ABI of ``include/nw.h``.  PyTorch provides
device memory (the caller-owned buffers the library works in) and streams.
There is no fallback: if the library has not been built, every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NW_LIBRARY names another build of the same library (the host-sanitizer build
# of the CPU tests); by default the in-tree libnw.so
LIB_PATH = os.environ.get("NW_LIBRARY") or os.path.join(_HERE, "libnw.so")

NW_OK, NW_EINVAL, NW_ERANGE, NW_ENOMEM, NW_EDEVICE, NW_ESTOPPED = 0, -1, -2, -3, -4, -5
NW_I8, NW_I16 = 1, 2

_lib = None


class NwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnw error {code}: {msg}")
        self.code = code


class _Scoring(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_int32), ("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap", ctypes.c_int32), ("submat", ctypes.c_void_p)]


class _EdgeFilter(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("lo", ctypes.c_int32), ("hi", ctypes.c_int32), ("den", ctypes.c_int32)]


NW_EDGE_RAW, NW_EDGE_NORMALISED = 0, 1


# nw_chunk_fn: int (*)(void *user, uint64_t idx_begin, uint64_t count, const void *h_chunk)
_CHUNK_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p)


class _BatchOptions(ctypes.Structure):
    _fields_ = [("class_width", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("pairs_per_item", ctypes.c_uint32), ("use_graph", ctypes.c_uint32)]


def load_library(path: str = LIB_PATH):
    """Load libnw.so (after torch, so both use the one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2509_01654_amd.build.build()")
    try:
        import torch  # noqa: F401  (binds libamdhip64 first)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    sig = {
        "nw_last_error": (ctypes.c_char_p, []),
        "nw_max_word_length": (ctypes.c_int, []),
        "nw_vocab_bytes": (ctypes.c_int, [u64, u64, u32, ctypes.POINTER(u64)]),
        "nw_load_vocab": (ctypes.c_int, [P, P, u64, ctypes.POINTER(_Scoring), P, u64, P, ctypes.POINTER(P)]),
        "nw_free_vocab": (None, [P]),
        "nw_vocab_info": (ctypes.c_int, [P, ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(u64),
                                         ctypes.POINTER(u64)]),
        "nw_score_bounds": (ctypes.c_int, [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "nw_all_pairs_scores": (ctypes.c_int, [P, u64, u64, ctypes.c_int, P, P]),
        "nw_all_pairs_scores_naive": (ctypes.c_int, [P, u64, u64, ctypes.c_int, P, P]),
        "nw_all_pairs_scores_diag": (ctypes.c_int, [P, u64, u64, ctypes.c_int, P, P]),
        "nw_topk_workspace_bytes": (ctypes.c_int, [P, u32, ctypes.POINTER(u64)]),
        "nw_all_pairs_topk": (ctypes.c_int, [P, u32, P, P, P, P, u64, P]),
        "nw_all_pairs_topk_async": (ctypes.c_int, [P, u32, P, P, P, P, u64, P]),
        "nw_topk_finish": (ctypes.c_int, [P, u32, P, P, P, u64, P]),
        "nw_all_pairs_scores_batched": (ctypes.c_int, [P, u32, P, ctypes.c_int, P]),
        "nw_query_workspace_bytes": (ctypes.c_int, [P, u64, u64, u32, ctypes.POINTER(u64)]),
        "nw_topk_phase_times": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                               ctypes.POINTER(ctypes.c_float)]),
        "nw_query": (ctypes.c_int, [P, P, P, u64, u32, P, P, P, u64, P]),
        "nw_topk_overflow_words": (ctypes.c_int, [P, ctypes.POINTER(u32)]),
        "nw_all_pairs_edges": (ctypes.c_int, [P, u64, u64, ctypes.POINTER(_EdgeFilter), P, P, P, u64, P, P]),
        "nw_export_triangle": (ctypes.c_int, [P, u64, u64, ctypes.c_int, u64, P, P, _CHUNK_FN, P, P]),
        "nw_graph_workspace_bytes": (ctypes.c_int, [u64, ctypes.POINTER(u64)]),
        "nw_packed_issue_rate": (ctypes.c_int, [u32, u32, ctypes.POINTER(u64), P]),
        "nw_graph_csr": (ctypes.c_int, [u64, P, P, u64, P, P, P, u64, P]),
        "nw_ego_network": (ctypes.c_int, [u64, P, P, P, u32, u32, P, P]),
    }
    sig.update({
        "nw_server_workspace_bytes": (ctypes.c_int, [P, u32, u32, u32, ctypes.POINTER(u64)]),
        "nw_server_create": (ctypes.c_int, [P, u32, u32, u32, P, u64, ctypes.POINTER(P)]),
        "nw_server_submit": (ctypes.c_int, [P, P, u32, u64, ctypes.c_int64]),
        "nw_server_poll": (ctypes.c_int, [P, u32, ctypes.c_int32, P, P, P, P, ctypes.POINTER(u32)]),
        "nw_server_replay": (ctypes.c_int, [P, P, P, u64, P, P, P, P]),
        "nw_server_stats": (ctypes.c_int, [P, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "nw_server_min_workspace_bytes": (ctypes.c_int, [P, u32, ctypes.POINTER(u64)]),
        "nw_server_memory_stats": (ctypes.c_int, [P, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "nw_server_inject_failure": (ctypes.c_int, [P]),
        "nw_server_destroy": (None, [P]),
        "nw_clock_ns": (ctypes.c_int64, []),
        "nw_batch_workspace_bytes": (ctypes.c_int, [P, u32, ctypes.POINTER(_BatchOptions), ctypes.POINTER(u64)]),
        "nw_batch_create": (ctypes.c_int, [P, u32, P, ctypes.c_int, ctypes.POINTER(_BatchOptions), P, u64,
                                           ctypes.POINTER(P)]),
        "nw_batch_run": (ctypes.c_int, [P, P]),
        "nw_batch_info": (ctypes.c_int, [P, ctypes.POINTER(u64), ctypes.POINTER(u32)]),
        "nw_batch_destroy": (None, [P]),
        "nw_batch_autotune": (ctypes.c_int, [P, u32, P, ctypes.c_int, P, u64, P, ctypes.c_char_p,
                                             ctypes.POINTER(_BatchOptions), ctypes.POINTER(ctypes.c_float)]),
    })
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != NW_OK:
        raise NwError(rc, _lib.nw_last_error().decode())


# Objects that own library resources.  At interpreter exit they are released
# in dependency order (servers, then batches, then dictionaries) by an atexit
# handler, while the HIP runtime and this module are still intact; each object
# keeps its own reference to the library, so a late __del__ never needs the
# module's globals.
_live = weakref.WeakSet()
_CLOSE_ORDER = {"Server": 0, "Batch": 1, "Vocab": 2}


def _close_all():
    for obj in sorted(list(_live), key=lambda o: _CLOSE_ORDER.get(type(o).__name__, 3)):
        try:
            obj.close()
        except Exception:  # nothing useful can be done with an error at exit
            pass


atexit.register(_close_all)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def max_word_length() -> int:
    return load_library().nw_max_word_length()


def vocab_bytes(n: int, total_symbols: int, max_len: int) -> int:
    lib = load_library()
    out = ctypes.c_uint64()
    _check(lib.nw_vocab_bytes(n, total_symbols, max_len, ctypes.byref(out)))
    return out.value


def packed_issue_rate(blocks: int, trips: int, stream=None) -> int:
    """Enqueue the packed-instruction issue-rate microbenchmark on `stream`;
    returns the lane-instructions that launch issues (time it with events)."""
    lib = load_library()
    out = ctypes.c_uint64()
    _check(lib.nw_packed_issue_rate(blocks, trips, ctypes.byref(out), _stream_handle(stream)))
    return out.value


def graph_csr(n: int, i, j, stream=None):
    """Compressed rows of the undirected graph with edges {i[e], j[e]} on n nodes
    (nw_graph_csr): (row_ptr int64 [n+1], adj int32 [2m]) on the edges' device."""
    import torch
    lib = load_library()
    m = i.numel()
    assert j.numel() == m and i.dtype == j.dtype == torch.int32 and i.is_contiguous() and j.is_contiguous()
    dev = i.device
    nbytes = ctypes.c_uint64()
    _check(lib.nw_graph_workspace_bytes(n, ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    adj = torch.empty(max(2 * m, 1), dtype=torch.int32, device=dev)
    _check(lib.nw_graph_csr(n, ctypes.c_void_p(i.data_ptr()), ctypes.c_void_p(j.data_ptr()), m,
                            ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(adj.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), nbytes.value, _stream_handle(stream)))
    return row_ptr, adj[:2 * m]


def ego_network(row_ptr, adj, seeds, depth: int, out=None, stream=None):
    """Hop distance of every node from the seed set, -1 beyond `depth` (nw_ego_network)."""
    import torch
    lib = load_library()
    n = row_ptr.numel() - 1
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.int32))
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    ap = ctypes.c_void_p(adj.data_ptr()) if adj.numel() else None
    _check(lib.nw_ego_network(n, ctypes.c_void_p(row_ptr.data_ptr()), ap,
                              seeds.ctypes.data if seeds.size else None, seeds.size, depth,
                              ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


class Scoring:
    """Similarity and gap penalty of Algorithm 1 (see nw_scoring in nw.h)."""

    def __init__(self, alphabet: int, match: int = 1, mismatch: int = -1, gap: int = -1, submat=None):
        self.alphabet, self.match, self.mismatch, self.gap = alphabet, match, mismatch, gap
        self.submat = None if submat is None else np.ascontiguousarray(np.asarray(submat, dtype=np.int8))

    def _c(self):
        sp = self.submat.ctypes.data if self.submat is not None else None
        return _Scoring(self.alphabet, self.match, self.mismatch, self.gap, sp)


class Vocab:
    """A dictionary resident on the current GPU (nw_load_vocab)."""

    def __init__(self, symbols, offsets, scoring: Scoring, device="cuda", stream=None):
        import torch
        lib = load_library()
        self.symbols = np.ascontiguousarray(np.asarray(symbols, dtype=np.uint8))
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        self.scoring = scoring
        n = self.offsets.shape[0] - 1
        lengths = np.diff(self.offsets)
        max_len = int(lengths.max()) if n > 0 else 0
        nbytes = vocab_bytes(n, int(self.offsets[-1]), max_len)
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=device)
        handle = ctypes.c_void_p()
        sc = scoring._c()
        _check(lib.nw_load_vocab(self.symbols.ctypes.data, self.offsets.ctypes.data, n, ctypes.byref(sc),
                                 ctypes.c_void_p(self.mem.data_ptr()), nbytes, _stream_handle(stream),
                                 ctypes.byref(handle)))
        self._h = handle
        self._lib = lib
        _live.add(self)
        self.device = self.mem.device
        N, L, E, C = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib.nw_vocab_info(self._h, ctypes.byref(N), ctypes.byref(L), ctypes.byref(E), ctypes.byref(C)))
        self.n, self.max_len, self.num_pairs, self.num_cells = N.value, L.value, E.value, C.value
        lo, hi = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.nw_score_bounds(self._h, ctypes.byref(lo), ctypes.byref(hi)))
        self.bounds = (lo.value, hi.value)

    def close(self):
        """Release the host descriptor (the device memory is a torch tensor)."""
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h is not None and h.value and lib is not None:
            lib.nw_free_vocab(h)
        self._h = None

    def __del__(self):
        self.close()

    def _triangle(self, fn, idx_begin, idx_end, dtype, out, stream):
        import torch
        if idx_end is None:
            idx_end = self.num_pairs
        dt = {torch.int8: NW_I8, torch.int16: NW_I16}[dtype]
        if out is None:
            out = torch.empty(max(0, idx_end - idx_begin), dtype=dtype, device=self.device)
        assert out.dtype == dtype and out.is_contiguous() and out.numel() >= idx_end - idx_begin
        _check(fn(self._h, idx_begin, idx_end, dt, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def all_pairs_scores(self, idx_begin: int = 0, idx_end: int | None = None, dtype=None, out=None, stream=None):
        """Row-major upper-triangle scores for pair indices [idx_begin, idx_end)."""
        import torch
        return self._triangle(_lib.nw_all_pairs_scores, idx_begin, idx_end, dtype or torch.int8, out, stream)

    def all_pairs_scores_naive(self, idx_begin: int = 0, idx_end: int | None = None, dtype=None, out=None,
                               stream=None):
        """Same output through the one-thread-per-pair kernel."""
        import torch
        return self._triangle(_lib.nw_all_pairs_scores_naive, idx_begin, idx_end, dtype or torch.int8, out, stream)

    def all_pairs_scores_diag(self, idx_begin: int = 0, idx_end: int | None = None, dtype=None, out=None,
                              stream=None):
        """Same output through the intra-pair anti-diagonal kernel."""
        import torch
        return self._triangle(_lib.nw_all_pairs_scores_diag, idx_begin, idx_end, dtype or torch.int8, out, stream)

    # ----------------------------------------------------------------- export
    def export_triangle(self, fn, dtype=None, chunk_pairs: int = 1 << 28, idx_begin: int = 0,
                        idx_end: int | None = None, ws=None, host=None, stream=None):
        """Stream the triangle of pair indices [idx_begin, idx_end) to the host in
        chunks (nw_export_triangle): fn(idx_begin, scores) is called once per chunk,
        in index order, with a numpy view that is valid only during the call;
        a truthy return value stops the export (NwError NW_ESTOPPED).  ws (device)
        and host (page-locked) buffers of 2*chunk_pairs elements are allocated
        when not given."""
        import torch
        dtype = dtype or torch.int8
        if idx_end is None:
            idx_end = self.num_pairs
        dt = {torch.int8: NW_I8, torch.int16: NW_I16}[dtype]
        np_dtype = np.int8 if dt == NW_I8 else np.int16
        es = 1 if dt == NW_I8 else 2
        chunk_pairs = max(1, min(chunk_pairs, max(1, idx_end - idx_begin)))
        nbytes = 2 * chunk_pairs * es
        if ws is None or ws.numel() * ws.element_size() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if host is None or host.numel() * host.element_size() < nbytes:
            host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        raised = []

        def chunk(_user, b0, count, ptr):
            try:
                view = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_int8 if es == 1
                                                                              else ctypes.c_int16)), (count,))
                return 1 if fn(b0, view.view(np_dtype)) else 0
            except BaseException as exc:  # stop the export and re-raise below
                raised.append(exc)
                return 1

        cb = _CHUNK_FN(chunk)
        rc = _lib.nw_export_triangle(self._h, idx_begin, idx_end, dt, chunk_pairs, ctypes.c_void_p(ws.data_ptr()),
                                     ctypes.c_void_p(host.data_ptr()), cb, None, _stream_handle(stream))
        if raised:
            raise raised[0]
        _check(rc)

    # ------------------------------------------------------------------ edges
    def all_pairs_edges(self, lo: int, hi: int, normalised: bool = False, den: int = 1, cap: int | None = None,
                        idx_begin: int = 0, idx_end: int | None = None, out=None, count=None, stream=None):
        """Pairs (i < j) whose raw score, or normalised weight 100*s/max(len i, len j)
        when `normalised`, lies in the closed slice [lo/den, hi/den] (nw_all_pairs_edges).

        Returns (i int32, j int32, score int16, count): the arrays hold the first
        min(count, cap) edges, in no particular order; count is the number of pairs
        that passed (it exceeds cap when the arrays were too small).  With cap=None
        a counting call sizes the arrays first.  `count` may pass a one-element int64
        device tensor to reuse for the count.  Synchronises the stream.
        """
        import torch
        if idx_end is None:
            idx_end = self.num_pairs
        f = _EdgeFilter(NW_EDGE_NORMALISED if normalised else NW_EDGE_RAW, lo, hi, den)
        cnt = count if count is not None else torch.empty(1, dtype=torch.int64, device=self.device)
        sh = _stream_handle(stream)

        def run(i, j, sc, c):
            P = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None)
            _check(_lib.nw_all_pairs_edges(self._h, idx_begin, idx_end, ctypes.byref(f), P(i), P(j), P(sc), c,
                                           ctypes.c_void_p(cnt.data_ptr()), sh))
            (stream or torch.cuda.current_stream()).synchronize()
            return int(cnt.item())

        if cap is None:
            cap = run(None, None, None, 0) if out is None else out[0].numel()
        if out is None:
            out = (torch.empty(cap, dtype=torch.int32, device=self.device),
                   torch.empty(cap, dtype=torch.int32, device=self.device),
                   torch.empty(cap, dtype=torch.int16, device=self.device))
        i, j, sc = out
        assert i.numel() >= cap and j.numel() >= cap and sc.numel() >= cap
        count = run(i, j, sc, cap)
        m = min(count, cap)
        return i[:m], j[:m], sc[:m], count

    # ------------------------------------------------------------------ top-k
    def topk_overflow_words(self) -> int:
        """Words of the last all_pairs_topk call that were recomputed exactly."""
        out = ctypes.c_uint32()
        _check(_lib.nw_topk_overflow_words(self._h, ctypes.byref(out)))
        return out.value

    def topk_workspace_bytes(self, k: int) -> int:
        out = ctypes.c_uint64()
        _check(_lib.nw_topk_workspace_bytes(self._h, k, ctypes.byref(out)))
        return out.value

    def all_pairs_topk(self, k: int = 32, hist: bool = True, ws=None, out=None, stream=None):
        """Per-word top-k neighbours over all other words and the score histogram.

        Returns (score int16 [n, k], index int32 [n, k], hist int64 [hi-lo+1] or None);
        the histogram bin b counts unordered pairs with score lo + b.
        """
        import torch
        nbytes = self.topk_workspace_bytes(k)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if out is None:
            out = (torch.empty((self.n, k), dtype=torch.int16, device=self.device),
                   torch.empty((self.n, k), dtype=torch.int32, device=self.device),
                   torch.empty(self.bounds[1] - self.bounds[0] + 1, dtype=torch.int64, device=self.device)
                   if hist else None)
        sc, ix, h = out
        hp = ctypes.c_void_p(h.data_ptr()) if h is not None else None
        _check(_lib.nw_all_pairs_topk(self._h, k, ctypes.c_void_p(sc.data_ptr()), ctypes.c_void_p(ix.data_ptr()), hp,
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
        return sc, ix, h

    def all_pairs_topk_async(self, k: int, ws, out, stream=None):
        """Enqueue the top-k passes and return (nw_all_pairs_topk_async); call
        topk_finish with the same k, ws and out before using the lists."""
        sc, ix, h = out
        hp = ctypes.c_void_p(h.data_ptr()) if h is not None else None
        _check(_lib.nw_all_pairs_topk_async(self._h, k, ctypes.c_void_p(sc.data_ptr()),
                                            ctypes.c_void_p(ix.data_ptr()), hp, ctypes.c_void_p(ws.data_ptr()),
                                            ws.numel(), _stream_handle(stream)))
        return out

    def topk_finish(self, k: int, ws, out, stream=None):
        """Complete an enqueued top-k pass (nw_topk_finish; blocks)."""
        sc, ix, _ = out
        _check(_lib.nw_topk_finish(self._h, k, ctypes.c_void_p(sc.data_ptr()), ctypes.c_void_p(ix.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
        return out

    def topk_phase_times(self):
        """(pre-pass, main pass, select) GPU milliseconds of the last all_pairs_topk."""
        a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        _check(_lib.nw_topk_phase_times(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    # ------------------------------------------------------------------ queries
    def query_workspace_bytes(self, n_q: int, k: int) -> int:
        out = ctypes.c_uint64()
        _check(_lib.nw_query_workspace_bytes(self._h, n_q, 0, k, ctypes.byref(out)))
        return out.value

    def query(self, qsymbols, qoffsets, k: int = 16, ws=None, out=None, stream=None):
        """Top-k dictionary neighbours of each query word: (score int16 [nq,k], index int32 [nq,k])."""
        import torch
        qsymbols = np.ascontiguousarray(np.asarray(qsymbols, dtype=np.uint8))
        qoffsets = np.ascontiguousarray(np.asarray(qoffsets, dtype=np.uint64))
        nq = qoffsets.shape[0] - 1
        nbytes = self.query_workspace_bytes(nq, k)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int16, device=self.device),
                   torch.empty((nq, k), dtype=torch.int32, device=self.device))
        sc, ix = out
        _check(_lib.nw_query(self._h, qsymbols.ctypes.data, qoffsets.ctypes.data, nq, k,
                             ctypes.c_void_p(sc.data_ptr()), ctypes.c_void_p(ix.data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
        return sc, ix


class Server:
    """Continuous-batching query server over a resident dictionary (nw_server_*)."""

    def __init__(self, vocab: Vocab, k: int = 16, max_batch: int = 256, num_slots: int = 4, ws_bytes=None):
        """ws_bytes caps the device memory pool batches are admitted against
        (default: enough for every slot to hold a max_batch batch at once)."""
        import torch
        lib = load_library()
        self.vocab, self.k = vocab, k
        nbytes = ctypes.c_uint64()
        _check(lib.nw_server_workspace_bytes(vocab._h, k, max_batch, num_slots, ctypes.byref(nbytes)))
        size = nbytes.value if ws_bytes is None else int(ws_bytes)
        self.ws = torch.empty(max(size, 256), dtype=torch.uint8, device=vocab.device)
        torch.cuda.synchronize(vocab.device)
        h = ctypes.c_void_p()
        _check(lib.nw_server_create(vocab._h, k, max_batch, num_slots, ctypes.c_void_p(self.ws.data_ptr()),
                                    size, ctypes.byref(h)))
        self._h = h
        self._lib = lib
        _live.add(self)

    def submit(self, symbols, tag: int, t_arrival_ns: int = 0):
        sym = np.ascontiguousarray(np.asarray(symbols, dtype=np.uint8))
        _check(_lib.nw_server_submit(self._h, sym.ctypes.data, sym.shape[0], tag, t_arrival_ns))

    def poll(self, max_results: int = 1024, timeout_us: int = 1000):
        tags = np.zeros(max_results, np.uint64)
        sc = np.zeros((max_results, self.k), np.int16)
        ix = np.zeros((max_results, self.k), np.int32)
        lat = np.zeros(max_results, np.int64)
        n = ctypes.c_uint32()
        _check(_lib.nw_server_poll(self._h, max_results, timeout_us, tags.ctypes.data, sc.ctypes.data, ix.ctypes.data,
                                   lat.ctypes.data, ctypes.byref(n)))
        m = n.value
        return tags[:m], sc[:m], ix[:m], lat[:m]

    def replay(self, qsymbols, qoffsets, arrival_s):
        """Open-loop replay; returns (scores [nq,k], index [nq,k], latency_s [nq])."""
        qsymbols = np.ascontiguousarray(np.asarray(qsymbols, dtype=np.uint8))
        qoffsets = np.ascontiguousarray(np.asarray(qoffsets, dtype=np.uint64))
        arrival_s = np.ascontiguousarray(np.asarray(arrival_s, dtype=np.float64))
        nq = qoffsets.shape[0] - 1
        sc = np.zeros((nq, self.k), np.int16)
        ix = np.zeros((nq, self.k), np.int32)
        lat = np.zeros(nq, np.float64)
        _check(_lib.nw_server_replay(self._h, qsymbols.ctypes.data, qoffsets.ctypes.data, nq, arrival_s.ctypes.data,
                                     sc.ctypes.data, ix.ctypes.data, lat.ctypes.data))
        return sc, ix, lat

    def stats(self):
        b, q = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.nw_server_stats(self._h, ctypes.byref(b), ctypes.byref(q)))
        return b.value, q.value

    def memory_stats(self):
        """(pool bytes, peak bytes reserved at once, batches that waited or shrank for memory)."""
        p, k, w = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.nw_server_memory_stats(self._h, ctypes.byref(p), ctypes.byref(k), ctypes.byref(w)))
        return p.value, k.value, w.value

    def inject_failure(self):
        """Make the next admitted batch fail on the host (tests of the error path)."""
        _check(_lib.nw_server_inject_failure(self._h))

    @staticmethod
    def min_workspace_bytes(vocab, k: int = 16) -> int:
        out = ctypes.c_uint64()
        _check(load_library().nw_server_min_workspace_bytes(vocab._h, k, ctypes.byref(out)))
        return out.value

    def close(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h is not None and h.value and lib is not None:
            lib.nw_server_destroy(h)
        self._h = None

    def __del__(self):
        self.close()


def clock_ns() -> int:
    return load_library().nw_clock_ns()


def all_pairs_scores_batched(vocabs, dtype=None, outs=None, stream=None):
    """Whole triangles of several dictionaries in one call (nw_all_pairs_scores_batched);
    returns the output tensors (row-major, one per dictionary)."""
    import torch
    lib = load_library()
    dtype = dtype or torch.int16
    dt = {torch.int8: NW_I8, torch.int16: NW_I16}[dtype]
    vocabs = list(vocabs)
    if outs is None:
        outs = [torch.empty(max(1, v.num_pairs), dtype=dtype, device=v.device) for v in vocabs]
    for v, o in zip(vocabs, outs):
        assert o.dtype == dtype and o.is_contiguous() and o.numel() >= v.num_pairs
    nv = len(vocabs)
    vh = (ctypes.c_void_p * max(1, nv))(*[v._h.value for v in vocabs])
    oh = (ctypes.c_void_p * max(1, nv))(*[o.data_ptr() for o in outs])
    _check(lib.nw_all_pairs_scores_batched(vh, nv, oh, dt, _stream_handle(stream)))
    return outs


class Batch:
    """Triangles of several dictionaries in one graph-captured persistent sequence (nw_batch_*)."""

    def __init__(self, vocabs, dtype=None, class_width=8, wg_per_cu=4, pairs_per_item=64, use_graph=True,
                 outs=None, autotune=False, cache_path=None, stream=None):
        import torch
        lib = load_library()
        dtype = dtype or torch.int16
        self.vocabs = list(vocabs)
        self.dtype = dtype
        self.dt = {torch.int8: NW_I8, torch.int16: NW_I16}[dtype]
        nv = len(self.vocabs)
        self._vh = (ctypes.c_void_p * nv)(*[v._h.value for v in self.vocabs])
        dev = self.vocabs[0].device
        self.outs = outs or [torch.empty(max(1, v.num_pairs), dtype=dtype, device=dev) for v in self.vocabs]
        self._oh = (ctypes.c_void_p * nv)(*[o.data_ptr() for o in self.outs])
        # workspace for the largest plan any option could need (finest items)
        probe = _BatchOptions(1, 1, 16, 1)
        need = ctypes.c_uint64()
        _check(lib.nw_batch_workspace_bytes(self._vh, nv, ctypes.byref(probe), ctypes.byref(need)))
        self.ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        opt = _BatchOptions(class_width, wg_per_cu, pairs_per_item, 1 if use_graph else 0)
        self.tuned_ms = None
        if autotune:
            ms = ctypes.c_float()
            cp = cache_path.encode() if cache_path else None
            _check(lib.nw_batch_autotune(self._vh, nv, self._oh, self.dt, ctypes.c_void_p(self.ws.data_ptr()),
                                         self.ws.numel(), _stream_handle(stream), cp, ctypes.byref(opt),
                                         ctypes.byref(ms)))
            if not use_graph:   # the caller forbids graphs; otherwise keep the tuner's choice
                opt.use_graph = 0
            self.tuned_ms = ms.value
        self.options = dict(class_width=opt.class_width, wg_per_cu=opt.wg_per_cu,
                            pairs_per_item=opt.pairs_per_item, use_graph=opt.use_graph)
        h = ctypes.c_void_p()
        _check(lib.nw_batch_create(self._vh, nv, self._oh, self.dt, ctypes.byref(opt),
                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        _live.add(self)

    def run(self, stream=None):
        _check(_lib.nw_batch_run(self._h, _stream_handle(stream)))
        return self.outs

    def info(self):
        items, launches = ctypes.c_uint64(), ctypes.c_uint32()
        _check(_lib.nw_batch_info(self._h, ctypes.byref(items), ctypes.byref(launches)))
        return items.value, launches.value

    def close(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        if h is not None and h.value and lib is not None:
            lib.nw_batch_destroy(h)
        self._h = None

    def __del__(self):
        self.close()
