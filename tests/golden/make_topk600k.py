"""Write the whole-workload top-32 fixture of the 600,000-word dictionary from
the CPU oracle alone.

For every word i of the dictionary (40-symbol Zipf(1.1) symbols, lengths
clip(Poisson(8), 1, 32), seed 3; scoring +1 / -1 / gap -1) the oracle scores i
against all 599,999 other words and keeps the first 32 under (score
descending, index ascending); it also counts every unordered pair's score.
The fixture stores, per block of 1,024 consecutive rows, the SHA-256 of

    scores  as little-endian int16, rows x 32, row-major, then
    indices as little-endian int32, rows x 32, row-major,

and the full 65-bin histogram (scores -32 .. 32).  This is the paper's own
check of comparing the CPU and GPU output files byte for byte (Section 5),
kept small enough to commit.

The run costs about 2.3e13 cell updates (every ordered pair), an hour or two
on a few host cores.  It is resumable: finished blocks are appended to a
cache file named after the dataset's SHA-256, and a new run skips them.

    python tests/golden/make_topk600k.py [--threads T] [--cache DIR] [--blocks A:B]

Only the oracle and the seeded input generator are used here.
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

K = 32
BLOCK = 1024
LO, HI = -32, 32
FIXTURE = os.path.join(HERE, "topk600k_paper.txt")


def block_digest(scores: np.ndarray, index: np.ndarray) -> str:
    """SHA-256 of one block's lists: int16 scores, then int32 indices (little-endian, row-major)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(scores, dtype="<i2").tobytes())
    h.update(np.ascontiguousarray(index, dtype="<i4").tobytes())
    return h.hexdigest()


def read_fixture(path: str = FIXTURE) -> dict:
    """{'dataset_sha256', 'n', 'k', 'block_rows', 'hist_lo', 'hist' (np.uint64), 'blocks' {b: hex}}."""
    out = {"blocks": {}}
    with open(path, encoding="ascii") as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "block":
                out["blocks"][int(vals[0])] = vals[1]
            elif key == "hist":
                out["hist"] = np.array([int(x) for x in vals], dtype=np.uint64)
            elif key == "dataset_sha256":
                out[key] = vals[0]
            else:
                out[key] = int(vals[0])
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--cache", default=os.path.join(os.environ.get("TMPDIR", "/tmp"), "nw_oracle_cache"))
    ap.add_argument("--blocks", default=None, help="A:B, only blocks A .. B-1 (the fixture is written once all are done)")
    ap.add_argument("--out", default=FIXTURE)
    args = ap.parse_args()

    v = synth.plain_config("paper")
    n = v.n
    sha = synth.sha256_vocab(v)
    sim = oracle.sim_matrix(40, 1, -1)
    nblocks = (n + BLOCK - 1) // BLOCK
    os.makedirs(args.cache, exist_ok=True)
    part = os.path.join(args.cache, f"{sha}_k{K}_b{BLOCK}.partial")

    done = {}
    if os.path.exists(part):
        with open(part, encoding="ascii") as f:
            for line in f:
                vals = line.split()
                if len(vals) == 2 + (HI - LO + 1):
                    done[int(vals[0])] = (vals[1], [int(x) for x in vals[2:]])
    a, b = 0, nblocks
    if args.blocks:
        a, b = (int(x) for x in args.blocks.split(":"))
    todo = [blk for blk in range(a, b) if blk not in done]
    print(f"dataset {sha}: {nblocks} blocks, {len(done)} cached, {len(todo)} to run on {args.threads} threads",
          flush=True)
    t0 = time.time()
    for c, blk in enumerate(todo):
        r0, r1 = blk * BLOCK, min(n, (blk + 1) * BLOCK)
        sc, ix, hist = oracle.topk_rows(v.symbols, v.offsets, sim, -1, K, r0=r0, r1=r1, hist_range=(LO, HI),
                                        threads=args.threads)
        dig = block_digest(sc, ix)
        with open(part, "a", encoding="ascii") as f:
            f.write(f"{blk} {dig} " + " ".join(str(int(x)) for x in hist) + "\n")
        done[blk] = (dig, [int(x) for x in hist])
        el = time.time() - t0
        print(f"block {blk} done ({c + 1}/{len(todo)}, {el:.0f} s, ~{el / (c + 1) * (len(todo) - c - 1):.0f} s left)",
              flush=True)

    if len(done) < nblocks:
        print(f"{nblocks - len(done)} blocks still missing; fixture not written", flush=True)
        return
    hist = np.zeros(HI - LO + 1, dtype=np.uint64)
    for blk in range(nblocks):
        hist += np.array(done[blk][1], dtype=np.uint64)
    assert int(hist.sum()) == n * (n - 1) // 2
    with open(args.out, "w", encoding="ascii") as f:
        f.write("# Top-32 neighbour lists and the score histogram of the 600,000-word workload\n"
                "# (Zipf-40, clip(Poisson(8), 1, 32), seed 3; +1 / -1 / gap -1), computed by the CPU\n"
                "# oracle over every row; written by tests/golden/make_topk600k.py.\n"
                "# block b covers rows [1024 b, 1024 b + 1024): SHA-256 of its int16 scores then\n"
                "# int32 indices, little-endian, row-major.  hist: unordered pairs per score -32 .. 32.\n")
        f.write(f"dataset_sha256 {sha}\nn {n}\nk {K}\nblock_rows {BLOCK}\nhist_lo {LO}\n")
        f.write("hist " + " ".join(str(int(x)) for x in hist) + "\n")
        for blk in range(nblocks):
            f.write(f"block {blk} {done[blk][0]}\n")
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
