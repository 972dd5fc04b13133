"""GPU parity of the triangle kernels against the CPU oracle (bit-exact).

Every case prints its name before the GPU work starts.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PM1 = dict(match=1, mismatch=-1, gap=-1)


def _nw():
    import paper_2509_01654_amd as nw
    return nw


def _gpu_triangle(v, sc_kw, dtype, idx=(0, None), naive=False, submat=None):
    nw = _nw()
    sc = nw.Scoring(v.alphabet, submat=submat, **sc_kw)
    dv = nw.Vocab(v.symbols, v.offsets, sc)
    fn = dv.all_pairs_scores_naive if naive else dv.all_pairs_scores
    out = fn(idx[0], idx[1], dtype=dtype)
    torch.cuda.synchronize()
    return dv, out.cpu().numpy().astype(np.int32)


def _oracle_triangle(v, sc_kw, idx=(0, None), submat=None):
    sim = oracle.sim_matrix(v.alphabet, sc_kw.get("match", 1), sc_kw.get("mismatch", -1), submat)
    return oracle.triangle(v.symbols, v.offsets, sim, sc_kw["gap"], idx[0], idx[1])


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.mark.parametrize("naive", [False, True])
@pytest.mark.parametrize("dtype", ["int8", "int16"])
def test_small_config_full_triangle(dtype, naive):
    """2,000 Zipf-40 words, clip(Poisson 7, 1, 20), +1/-1/-1: all 1,999,000 pairs."""
    _report(f"small config dtype={dtype} naive={naive}")
    v = synth.plain_config("small")
    _, got = _gpu_triangle(v, PM1, getattr(torch, dtype), naive=naive)
    want = _oracle_triangle(v, PM1)
    assert got.shape == want.shape == (1_999_000,)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n", [2, 3, 17, 255, 256, 257, 511, 700])
def test_ragged_sizes(n):
    _report(f"ragged n={n}")
    v = synth.zipf_vocab(n, seed=1000 + n, mean_len=8.0, max_len=32)
    _, got = _gpu_triangle(v, PM1, torch.int8)
    np.testing.assert_array_equal(got, _oracle_triangle(v, PM1))


@pytest.mark.parametrize("n", [16384, 16385])
def test_launch_form_switch(n):
    """Both sides of the switch between one launch per class of 8 row lengths
    (at most 16,384 words, 256-word blocks) and one launch per length (larger
    dictionaries, 1,024-word blocks): the whole triangle against the oracle."""
    _report(f"launch-form switch n={n}")
    v = synth.zipf_vocab(n, seed=2000 + n, mean_len=7.0, max_len=20)
    _, got = _gpu_triangle(v, PM1, torch.int8)
    np.testing.assert_array_equal(got, _oracle_triangle(v, PM1))


def test_empty_and_single_word():
    nw = _nw()
    for n in (0, 1):
        _report(f"degenerate n={n}")
        v = synth.zipf_vocab(n, seed=5)
        dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, **PM1))
        assert dv.num_pairs == 0
        out = dv.all_pairs_scores(dtype=torch.int8)
        assert out.numel() == 0


def test_edge_words_empty_long_duplicates():
    """Empty words, words of the maximum length 48, duplicates, one-symbol words."""
    _report("edge words")
    rng = np.random.default_rng(77)
    words = [[], [], [3], [3], [5], list(range(40)) + list(range(8)), [7] * 48, [7] * 48]
    words += [list(rng.integers(0, 40, size=rng.integers(0, 49))) for _ in range(300)]
    words += [[], [1, 2, 3], [1, 2, 3]]
    v = synth.vocab_from_words(words, 40)
    _, got = _gpu_triangle(v, PM1, torch.int16)
    np.testing.assert_array_equal(got, _oracle_triangle(v, PM1))
    _, got8 = _gpu_triangle(v, PM1, torch.int8)
    np.testing.assert_array_equal(got8, _oracle_triangle(v, PM1))


def test_submatrix_scoring_uniform_lengths():
    """64-symbol alphabet, seeded symmetric matrix in [-3,3] (diag +3), gap -2, lengths 1..48, int16."""
    _report("submatrix 64 gap -2")
    v = synth.uniform_vocab(600, seed=44, alphabet=64, min_len=1, max_len=48)
    S = synth.random_submat(64, seed=4)
    kw = dict(gap=-2)
    _, got = _gpu_triangle(v, kw, torch.int16, submat=S)
    np.testing.assert_array_equal(got, _oracle_triangle(v, kw, submat=S))
    _, naive = _gpu_triangle(v, kw, torch.int16, submat=S, naive=True)
    np.testing.assert_array_equal(naive, got)


@pytest.mark.parametrize("scoring", [dict(match=0, mismatch=-1, gap=-1), dict(match=1, mismatch=0, gap=0),
                                     dict(match=2, mismatch=-5, gap=-1), dict(match=1, mismatch=-1, gap=-2)])
def test_other_linear_scorings(scoring):
    _report(f"scoring {scoring}")
    v = synth.zipf_vocab(400, seed=31, mean_len=8.0, max_len=32)
    _, got = _gpu_triangle(v, scoring, torch.int16)
    np.testing.assert_array_equal(got, _oracle_triangle(v, scoring))


def test_index_ranges_are_slices_of_the_triangle():
    _report("index ranges")
    v = synth.zipf_vocab(1500, seed=9, mean_len=7.0, max_len=20)
    _, full = _gpu_triangle(v, PM1, torch.int8)
    E = full.shape[0]
    for a, b in [(0, 1), (0, 1499), (1499, 2998), (12345, 12346), (E - 1, E), (E // 3, 2 * E // 3), (E, E)]:
        _, part = _gpu_triangle(v, PM1, torch.int8, idx=(a, b))
        np.testing.assert_array_equal(part, full[a:b])
    np.testing.assert_array_equal(full, _oracle_triangle(v, PM1))


def test_block_size_1024_sampled():
    """20,000 words take the 1024-word blocks: GPU triangle vs the oracle on
    whole blocks of rows and a random pair sample."""
    _report("n=20000 sampled")
    v = synth.zipf_vocab(20000, seed=21, mean_len=7.0, max_len=20)
    _, got = _gpu_triangle(v, PM1, torch.int8)
    n = v.n
    rng = np.random.default_rng(0)
    i = rng.integers(0, n, size=300_000)
    j = rng.integers(0, n, size=300_000)
    keep = i != j
    i, j = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
    idx = i * (2 * n - i - 1) // 2 + (j - i - 1)
    sim = oracle.sim_matrix(40, 1, -1)
    want = oracle.pairs(v.symbols, v.offsets, sim, -1, i, j)
    np.testing.assert_array_equal(got[idx], want)
    # rows 0..39 and 10230..10249 in full (straddling block boundaries)
    for r0, r1 in [(0, 40), (1015, 1035), (10230, 10250), (n - 30, n - 1)]:
        a = r0 * (2 * n - r0 - 1) // 2
        b = r1 * (2 * n - r1 - 1) // 2
        want = oracle.triangle(v.symbols, v.offsets, sim, -1, a, b)
        np.testing.assert_array_equal(got[a:b], want)
