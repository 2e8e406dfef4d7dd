"""The C ABI without a GPU: symbols, status handling and the estimator's host parts."""
import itertools
import math
import os
import re

import numpy as np
import pytest

import paper_2108_05038_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fim_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = F.lib()
    declared = _declared()
    assert len(declared) >= 25
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(F.EXPORTED)


def test_status_strings_and_version():
    L = F.lib()
    assert L.fim_status_str(0) == b"FIM_OK"
    assert L.fim_status_str(F.FIM_E_OUTPUT_LIMIT) == b"FIM_E_OUTPUT_LIMIT"
    assert L.fim_status_str(-999) == b"FIM_E_UNKNOWN"
    assert "gfx950" in F.fim_version()


def test_minsup_from_relative():
    assert F.fim_minsup_from_relative(10000, 0.01) == 100
    assert F.fim_minsup_from_relative(200000, 0.001) == 200
    assert F.fim_minsup_from_relative(50000, 0.4) == 20000
    assert F.fim_minsup_from_relative(1000, 0.0001) == 1  # at least one transaction
    assert F.fim_minsup_from_relative(7, 0.5) == 4        # rounded up
    for bad in (0.0, -0.1, 1.5):
        with pytest.raises(F.FimError):
            F.fim_minsup_from_relative(100, bad)


def test_no_gpu_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(F.FimError) as e:
        F.fim_ctx_create(0)
    assert e.value.status == F.FIM_E_NO_DEVICE


# ---------------------------------------------------------------- sample sizes

def _kl(x, y):
    from scipy.special import rel_entr
    return float(rel_entr(x, y) + rel_entr(1 - x, 1 - y))


@pytest.mark.parametrize("eps,delta", [(0.02, 0.05), (0.01, 0.01), (0.05, 0.1)])
def test_database_sample_size_is_the_smallest_meeting_the_chernoff_bound(eps, delta):
    n, _ = F.fim_estimate_sample_sizes(eps, delta, 0.001, 0.0005, 0.05)
    assert 2 * math.exp(-2 * eps * eps * n) <= delta
    assert 2 * math.exp(-2 * eps * eps * (n - 1)) > delta


@pytest.mark.parametrize("rho,eps,delta", [(0.001, 0.0005, 0.05), (0.01, 0.005, 0.01)])
def test_reservoir_size_is_the_smallest_meeting_the_kl_bound(rho, eps, delta):
    _, n = F.fim_estimate_sample_sizes(0.02, 0.05, rho, eps, delta)
    d = _kl(rho + eps, rho)  # Bernoulli KL divergence from scipy
    assert 2 * math.exp(-n * d) <= delta * (1 + 1e-12)
    assert 2 * math.exp(-(n - 1) * d) > delta
    # the thesis's recommended sizes are of this order (tens of thousands)
    if rho == 0.001:
        assert 10000 < n < 60000


def test_sample_size_arguments_checked():
    with pytest.raises(F.FimError):
        F.fim_estimate_sample_sizes(0.0, 0.05, 0.001, 0.0005, 0.05)
    with pytest.raises(F.FimError):
        F.fim_estimate_sample_sizes(0.02, 0.05, 0.9, 0.2, 0.05)


# ---------------------------------------------------------------- reservoir

def test_reservoir_short_stream_keeps_everything():
    assert sorted(F.fim_reservoir_sample(5, 10, 1).tolist()) == [0, 1, 2, 3, 4]
    assert len(F.fim_reservoir_sample(0, 10, 1)) == 0


def test_reservoir_is_uniform_without_replacement():
    L, n, trials = 20, 5, 4000
    counts = np.zeros(L)
    for s in range(trials):
        r = F.fim_reservoir_sample(L, n, 1000 + s)
        assert len(set(r.tolist())) == n and r.max() < L
        counts[r] += 1
    expected = trials * n / L
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 19 degrees of freedom: the 99.9 % quantile is about 43.8
    assert chi2 < 43.8, chi2


# ---------------------------------------------------------------- LPT and Partition

def _opt_makespan(w, p):
    best = float("inf")
    for assign in itertools.product(range(p), repeat=len(w)):
        loads = [0.0] * p
        for j, k in enumerate(assign):
            loads[k] += w[j]
        best = min(best, max(loads))
    return best


def test_lpt_within_graham_bound_of_optimal():
    rng = np.random.default_rng(0)
    for _ in range(60):
        p = int(rng.integers(2, 4))
        w = rng.integers(1, 30, int(rng.integers(3, 8))).astype(float)
        wk, ms = F.fim_lpt_schedule(w, p)
        loads = np.bincount(wk, weights=w, minlength=p)
        assert math.isclose(ms, loads.max())
        opt = _opt_makespan(list(w), p)
        assert ms <= (4.0 / 3.0 - 1.0 / (3 * p)) * opt + 1e-9


def test_lpt_known_schedule():
    # the classic tight example for two workers: 3, 3, 2, 2, 2 -> LPT 7, optimum 6
    wk, ms = F.fim_lpt_schedule([3, 3, 2, 2, 2], 2)
    assert ms == 7.0


def _check_cover(n_atoms, tasks):
    seen = {}
    for c, r0, r1 in tasks.tolist():
        assert r0 < r1 <= n_atoms[c] - 1
        for r in range(r0, r1):
            assert (c, r) not in seen
            seen[(c, r)] = 1
    want = {(c, r) for c, a in enumerate(n_atoms) for r in range(max(0, a - 1))}
    assert set(seen) == want


def test_partition_covers_every_class_once_and_splits_large_ones():
    rng = np.random.default_rng(3)
    n_atoms = rng.integers(0, 30, 40)
    w = rng.exponential(1.0, int(n_atoms.sum()))
    w[: n_atoms[0]] *= 200  # one dominant class
    tasks, ms = F.fim_partition_lpt(n_atoms, w, 0.3, 16)
    _check_cover(list(n_atoms), tasks)
    # LPT order: estimates decrease along the task list
    off = np.concatenate([[0], np.cumsum(n_atoms)])
    est = [w[off[c] + r0: off[c] + r1].sum() for c, r0, r1 in tasks.tolist()]
    assert all(a >= b - 1e-9 for a, b in zip(est, est[1:]))
    theta = 0.3 * sum(w[off[c]: off[c] + max(0, a - 1)].sum() for c, a in enumerate(n_atoms)) / 16
    for (c, r0, r1), e in zip(tasks.tolist(), est):
        assert e <= theta + 1e-9 or r1 - r0 == 1 or (r0 == 0 and r1 == n_atoms[c] - 1
                                                      and e <= theta)
    assert sum(1 for c, _, _ in tasks.tolist() if c == 0) > 1  # the dominant class was split
    nosplit, _ = F.fim_partition_lpt(n_atoms, w, 0.3, 16, flags=F.FIM_FLAG_NO_SPLIT)
    _check_cover(list(n_atoms), nosplit)
    assert len(nosplit) == int((n_atoms >= 2).sum())
