"""The C ABI on the CPU: the library loads, exports every declared symbol, and
rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2509_01654_amd as nw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        text = open(os.path.join(ROOT, "include", h), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(nw_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol():
    lib = nw.load_library()
    names = _declared_functions()
    assert "nw_load_vocab" in names and "nw_all_pairs_scores" in names
    for name in names:
        assert hasattr(lib, name), name


def test_vocab_bytes_and_limits():
    assert nw.max_word_length() == 255
    assert nw.vocab_bytes(0, 0, 0) > 0
    b1 = nw.vocab_bytes(2000, 14000, 20)
    b2 = nw.vocab_bytes(50000, 350000, 20)
    assert b2 > b1
    assert nw.vocab_bytes(2000, 14000, 200) > b1
    with pytest.raises(nw.NwError) as e:
        nw.vocab_bytes(10, 10, 256)
    assert e.value.code == nw.NW_EINVAL


def _load(symbols, offsets, sc, d_bytes=1 << 30, d_mem=1 << 20):
    lib = nw.load_library()
    symbols = np.ascontiguousarray(symbols, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    h = ctypes.c_void_p()
    c = sc._c()
    rc = lib.nw_load_vocab(symbols.ctypes.data, offsets.ctypes.data, offsets.shape[0] - 1, ctypes.byref(c),
                           ctypes.c_void_p(d_mem), d_bytes, None, ctypes.byref(h))
    return rc, lib.nw_last_error().decode()


def test_load_vocab_rejects_bad_input_before_any_device_call():
    ok_syms = np.array([1, 2, 3, 4], np.uint8)
    ok_offs = np.array([0, 2, 4], np.uint64)
    pm = nw.Scoring(40, 1, -1, -1)
    rc, msg = _load(np.array([1, 40], np.uint8), np.array([0, 2], np.uint64), pm)
    assert rc == nw.NW_EINVAL and "alphabet" in msg
    long_word = np.zeros(256, np.uint8)
    rc, msg = _load(long_word, np.array([0, 256], np.uint64), pm)
    assert rc == nw.NW_EINVAL and "maximum" in msg
    rc, _ = _load(ok_syms, ok_offs, nw.Scoring(40, 1, -1, +1))
    assert rc == nw.NW_EINVAL
    rc, _ = _load(ok_syms, ok_offs, nw.Scoring(0, 1, -1, -1))
    assert rc == nw.NW_EINVAL
    rc, _ = _load(ok_syms, ok_offs, nw.Scoring(256, 1, -1, -1))
    assert rc == nw.NW_EINVAL
    rc, _ = _load(ok_syms, np.array([0, 3, 2], np.uint64), pm)
    assert rc == nw.NW_EINVAL
    # DP values beyond the exact 16-bit range: 48 * (100 + 2) > 2048
    big = np.full((8, 8), -5, np.int8)
    np.fill_diagonal(big, 100)
    rc, msg = _load(np.zeros(48, np.uint8), np.array([0, 48], np.uint64), nw.Scoring(8, submat=big, gap=-1))
    assert rc == nw.NW_ERANGE, msg
    # a too-small device buffer
    need = nw.vocab_bytes(2, 4, 2)
    rc, msg = _load(ok_syms, ok_offs, pm, d_bytes=need - 1)
    assert rc == nw.NW_ENOMEM, msg
    # misaligned device memory
    rc, _ = _load(ok_syms, ok_offs, pm, d_mem=(1 << 20) + 8)
    assert rc == nw.NW_EINVAL


def test_graph_and_export_arguments_rejected_on_the_host():
    """Argument checks that fail before any device call (fake non-NULL pointers
    are never dereferenced on these paths)."""
    lib = nw.load_library()
    need = ctypes.c_uint64()
    assert lib.nw_graph_workspace_bytes(1000, ctypes.byref(need)) == nw.NW_OK and need.value > 8 * 1000
    assert lib.nw_graph_workspace_bytes(1 << 31, ctypes.byref(need)) == nw.NW_EINVAL
    fake = ctypes.c_void_p(1 << 20)
    assert lib.nw_graph_csr(1 << 31, fake, fake, 1, fake, fake, fake, 1 << 30, None) == nw.NW_EINVAL
    assert lib.nw_graph_csr(10, None, None, 1, fake, fake, fake, 1 << 30, None) == nw.NW_EINVAL
    assert lib.nw_graph_csr(10, fake, fake, 1, fake, fake, ctypes.c_void_p((1 << 20) + 8), 1 << 30,
                            None) == nw.NW_EINVAL
    assert lib.nw_graph_csr(10, fake, fake, 1, fake, fake, fake, 8, None) == nw.NW_ENOMEM
    seeds = np.array([3, 10], np.int32)
    assert lib.nw_ego_network(10, fake, fake, seeds.ctypes.data, 2, 3, fake, None) == nw.NW_EINVAL
    assert "seed 10" in lib.nw_last_error().decode()
    seeds = np.array([-1], np.int32)
    assert lib.nw_ego_network(10, fake, fake, seeds.ctypes.data, 1, 3, fake, None) == nw.NW_EINVAL
    assert lib.nw_ego_network(10, fake, fake, None, 1, 3, fake, None) == nw.NW_EINVAL
    assert lib.nw_ego_network(10, fake, fake, None, 0, 2_000_000, fake, None) == nw.NW_EINVAL
    # export and edges: a NULL dictionary is refused first
    assert lib.nw_export_triangle(None, 0, 1, nw.NW_I8, 1, fake, fake, nw._CHUNK_FN(lambda *a: 0), None,
                                  None) == nw.NW_EINVAL
    f = nw._EdgeFilter(0, 0, 1, 1)
    assert lib.nw_all_pairs_edges(None, 0, 1, ctypes.byref(f), fake, fake, fake, 1, fake, None) == nw.NW_EINVAL


def test_packed_rate_arguments_rejected_on_the_host():
    lib = nw.load_library()
    n = ctypes.c_uint64()
    assert lib.nw_packed_issue_rate(0, 1, ctypes.byref(n), None) == nw.NW_EINVAL
    assert lib.nw_packed_issue_rate(1, 0, ctypes.byref(n), None) == nw.NW_EINVAL
    assert lib.nw_packed_issue_rate(1, 1, None, None) == nw.NW_EINVAL
