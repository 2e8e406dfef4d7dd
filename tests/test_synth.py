"""The seeded input generators: reproducible, well-formed, and of the stated shapes."""
import numpy as np

import synth

M64 = (1 << 64) - 1


def _splitmix64(state):
    state = (state + 0x9E3779B97F4A7C15) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def _xoshiro256ss(seed, n):
    # published xoshiro256** (Blackman & Vigna) seeded by SplitMix64
    s, x = [], seed
    for _ in range(4):
        x, v = _splitmix64(x)
        s.append(v)
    rotl = lambda v, k: ((v << k) | (v >> (64 - k))) & M64
    out = []
    for _ in range(n):
        out.append((rotl((s[1] * 5) & M64, 7) * 9) & M64)
        t = (s[1] << 17) & M64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = rotl(s[3], 45)
    return out


def test_rng_is_the_published_generator():
    for seed in (0, 1, 2108050381):
        assert synth.raw(seed, 16).tolist() == _xoshiro256ss(seed, 16)


def _well_formed(o, it, ni):
    assert o[0] == 0 and np.all(np.diff(o.astype(np.int64)) >= 0) and o[-1] == len(it)
    assert len(it) == 0 or int(it.max()) < ni
    for t in range(0, len(o) - 1, max(1, (len(o) - 1) // 500)):
        row = it[o[t]:o[t + 1]]
        assert np.all(np.diff(row.astype(np.int64)) > 0)  # sorted, no duplicates


def test_basket_reproducible_and_shaped():
    a = synth.basket(42, 5000, 300, 10.0, 600, 4.0)
    b = synth.basket(42, 5000, 300, 10.0, 600, 4.0)
    c = synth.basket(43, 5000, 300, 10.0, 600, 4.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1], c[1])
    _well_formed(*a)
    mean = np.diff(a[0].astype(np.int64)).mean()
    assert 9.0 < mean < 14.0  # target Poisson mean 10; the last pattern is added whole


def test_dense_reproducible_and_shaped():
    a = synth.dense(7, 3000, 120)
    b = synth.dense(7, 3000, 120)
    assert np.array_equal(a[1], b[1])
    _well_formed(*a)
    lens = np.diff(a[0].astype(np.int64))
    assert lens.mean() > 48  # Beta(4,6) background (mean 0.4 * 120) plus planted groups


def test_named_workloads_sizes():
    d = synth.make("basket-10k")
    assert d.n_tx == 10_000 and d.n_items == 1_000 and d.minsup == 100
    _well_formed(d.offsets, d.items, d.n_items)


def test_batch_params_ranges():
    for i in range(64):
        p = synth.batch_params(i)
        assert 1000 <= p["n_tx"] <= 200000 and 200 <= p["n_items"] <= 5000
        assert 8 <= p["mean_len"] <= 30 and 0.002 <= p["rel_minsup"] <= 0.05
        assert p["minsup"] == max(1, int(np.ceil(p["rel_minsup"] * p["n_tx"])))
    assert synth.batch_params(3) == synth.batch_params(3)
