"""Interpreter shutdown with live library objects: a child process builds a
dictionary, a batch and a server (with a query still queued) and exits without
closing any of them.  The binding's exit handler must release them in
dependency order, with no traceback and a clean exit status."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
import paper_2509_01654_amd as nw
from synth import zipf_vocab

v = zipf_vocab(600, seed=7, mean_len=8.0, max_len=32)
sc = nw.Scoring(alphabet=40, match=1, mismatch=-1, gap=-1)
dv = nw.Vocab(v.symbols, v.offsets, sc, device="cuda:0")
dv2 = nw.Vocab(v.symbols, v.offsets, sc, device="cuda:0")
b = nw.Batch([dv, dv2], torch.int16, use_graph=True)
b.run()
srv = nw.Server(dv, k=8, max_batch=16, num_slots=2)
srv.submit(v.symbols[:5], tag=1)
torch.cuda.synchronize()
print("objects live at exit", flush=True)
"""


@pytest.mark.gpu
def test_exit_with_live_objects_is_clean():
    print("teardown child: Vocab x2 + Batch(graph) + Server with a queued query", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], cwd=ROOT, capture_output=True, text=True, timeout=120)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "objects live at exit" in r.stdout, out
    assert "Traceback" not in r.stderr and "Exception ignored" not in r.stderr, out
