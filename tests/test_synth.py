"""The seeded generators: determinism and the laws the workloads state."""
import numpy as np

import synth


def test_deterministic_and_hashed():
    a = synth.zipf_vocab(3000, seed=1)
    b = synth.zipf_vocab(3000, seed=1)
    c = synth.zipf_vocab(3000, seed=2)
    assert synth.sha256_vocab(a) == synth.sha256_vocab(b) != synth.sha256_vocab(c)


def test_small_config_laws():
    v = synth.plain_config("small")
    assert v.n == 2000 and v.alphabet == 40
    L = v.lengths
    assert L.min() >= 1 and L.max() <= 20 and abs(L.mean() - 7.0) < 0.3
    assert v.symbols.max() < 40
    # Zipf(1.1) over 40 symbols: P(symbol 0) ~ 0.272
    p0 = np.mean(v.symbols == 0)
    assert abs(p0 - synth.zipf_probs(40, 1.1)[0]) < 0.02
    assert int(v.offsets[-1]) == int(L.sum())


def test_batched_configs():
    vocabs, S = synth.batched_configs(scale=0.01)
    assert synth.BATCHED_LMAX == (8, 14, 19, 25, 31, 37, 42, 48)
    assert S.shape == (64, 64) and (S == S.T).all() and (np.diag(S) == 3).all()
    assert S.min() >= -3 and S.max() <= 3
    for v, lmax in zip(vocabs, synth.BATCHED_LMAX):
        assert v.lengths.max() <= lmax and v.lengths.min() >= 1 and v.symbols.max() < 64


def test_poisson_arrivals():
    t = synth.poisson_arrivals(10000.0, 20000, seed=50)
    assert np.all(np.diff(t) > 0)
    assert abs(20000 / t[-1] - 10000) < 300
