"""The two forms of the top-k threshold pre-pass give the same keys.

Each word's pre-pass key is its key of rank k+1 against the probe subset.  The
selection form (byte-wide score codes: a histogram and a rank-ordered code
array in LDS) replaces the list form (wavefront lists, then a merge) wherever
it applies; NW_PREPASS=lists keeps the list form.  A child process runs the
list form and the test the selection form on the same dictionaries.  Since
everything after the pre-pass is deterministic, both must leave the same final
thresholds and candidate counts in the workspace (the thresholds at its
start, the per-word counts at the next 256-byte boundary) and the same
lists.  The dictionaries stress what the selection decides: heavy score
ties (three- and four-symbol alphabets), k = 1, n not a multiple of the probe
count M = 8192 (probe i is word floor(i n / M)), and n < 256 (a probe array
with unused tail slots).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# name -> (generator args, scoring (alphabet, match, mismatch, gap), k)
CASES = {
    "zipf40_20001": (("zipf", 20001, 11), (40, 1, -1, -1), 32),
    "uni4_30000": (("uniform", 30000, 7, 4, 1, 12), (4, 1, -1, -1), 16),
    "uni4_k1": (("uniform", 9000, 8, 4, 1, 6), (4, 2, -1, -2), 1),
    "uni3_300": (("uniform", 300, 9, 3, 1, 5), (3, 1, -1, -1), 8),
    "uni2_200": (("uniform", 200, 10, 2, 0, 3), (2, 1, -1, -1), 63),
}

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
import paper_2509_01654_amd as nw
sys.path.insert(0, sys.argv[1] + "/tests")
from test_gpu_prepass import CASES, run_case
out = sys.argv[2]
for name in CASES:
    thr, cnt, s, i = run_case(name)
    np.savez(f"{out}/{name}.npz", thr=thr, cnt=cnt, s=s, i=i)
    print("child done", name, flush=True)
"""


def make_vocab(gen):
    if gen[0] == "zipf":
        return synth.zipf_vocab(gen[1], seed=gen[2], mean_len=8.0, max_len=32)
    _, n, seed, alphabet, lo, hi = gen
    return synth.uniform_vocab(n, seed=seed, alphabet=alphabet, min_len=lo, max_len=hi)


def run_case(name):
    import paper_2509_01654_amd as nw
    gen, (alphabet, match, mismatch, gap), k = CASES[name]
    v = make_vocab(gen)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(alphabet, match, mismatch, gap))
    n = v.n
    ws = torch.zeros(dv.topk_workspace_bytes(k), dtype=torch.uint8, device="cuda")
    s, i, _ = dv.all_pairs_topk(k, hist=False, ws=ws)
    torch.cuda.synchronize()
    a = ws.cpu().numpy()
    o = (8 * n + 255) // 256 * 256
    return (a[:8 * n].view(np.uint64).copy(), a[o:o + 4 * n].view(np.uint32).copy(), s.cpu().numpy(),
            i.cpu().numpy())


def test_selection_prepass_matches_list_prepass(tmp_path):
    print("[gpu case] pre-pass forms: child with NW_PREPASS=lists", flush=True)
    env = dict(os.environ, NW_PREPASS="lists")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(tmp_path)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert os.environ.get("NW_PREPASS") != "lists"
    for name in CASES:
        print(f"[gpu case] pre-pass forms: {name}", flush=True)
        want = np.load(tmp_path / f"{name}.npz")
        thr, cnt, s, i = run_case(name)
        np.testing.assert_array_equal(thr, want["thr"], err_msg=name)
        np.testing.assert_array_equal(cnt, want["cnt"], err_msg=name)
        np.testing.assert_array_equal(s, want["s"], err_msg=name)
        np.testing.assert_array_equal(i, want["i"], err_msg=name)


@pytest.mark.parametrize("name", ["uni3_300", "uni2_200", "uni4_k1"])
def test_selection_prepass_lists_against_oracle(name):
    print(f"[gpu case] selection pre-pass top-k vs oracle: {name}", flush=True)
    gen, (alphabet, match, mismatch, gap), k = CASES[name]
    v = make_vocab(gen)
    _, _, s, i = run_case(name)
    ws, wi, _ = oracle.topk_rows(v.symbols, v.offsets, oracle.sim_matrix(alphabet, match, mismatch), gap, k)
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s.astype(np.int32), ws)
