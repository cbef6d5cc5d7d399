"""The hybrid split of section 4.4 (eq:costwo), host logic of the library.

The returned n minimises c_HY(n) = t_CG(m_n^2) + sum_{i>n} t_MG over n = 1..N for the
CG iteration bound 0.5 sqrt(kappa) ln(2/tol); where lambda_min lies far above the
smallest shifts the multi-shift solve costs the same for every n and all shifts stay
with it; near the critical point, with a cheap multigrid, the smallest shifts move to
the multigrid; inconsistent arguments are refused.
"""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


def _cost(sig, n, lmin, lmax, tol, ms_it, ms_mg):
    s = sig[n - 1]
    return 0.5 * np.sqrt((lmax + s) / (lmin + s)) * np.log(2 / tol) * ms_it + (len(sig) - n) * ms_mg


def test_regime_of_the_bench_fields(nd):
    sig = synth.geometric_shifts(12, 1e-5)
    # 0.19 ms per iteration, about 45 ms per multigrid shift started from Lagrange guesses
    assert nd.hybrid_split(sig, 0.011, 28.0, 1e-10, 0.19, 45.0) == 12


def test_near_critical_moves_small_shifts_to_multigrid(nd):
    sig = synth.geometric_shifts(12, 1e-5)
    n = nd.hybrid_split(sig, 1e-7, 28.0, 1e-10, 0.19, 2.0)
    assert n < 12
    assert _cost(sig, n, 1e-7, 28.0, 1e-10, 0.19, 2.0) < _cost(sig, 12, 1e-7, 28.0, 1e-10, 0.19, 2.0)
    # a dearer multigrid never moves more shifts to it
    assert nd.hybrid_split(sig, 1e-7, 28.0, 1e-10, 0.19, 20.0) >= n


def test_argmin_over_random_inputs(nd):
    rng = np.random.default_rng(3)
    for _ in range(200):
        N = int(rng.integers(1, 17))
        sig = np.sort(np.exp(rng.uniform(np.log(1e-7), 0, N)))[::-1]
        sig = sig[np.concatenate([[True], np.diff(sig) < 0])]
        lmin = 10 ** rng.uniform(-8, -1)
        lmax = lmin * 10 ** rng.uniform(1, 6)
        ms_it, ms_mg = 10 ** rng.uniform(-2, 0), 10 ** rng.uniform(-2, 2)
        n = nd.hybrid_split(sig, lmin, lmax, 1e-10, ms_it, ms_mg)
        costs = [_cost(sig, k, lmin, lmax, 1e-10, ms_it, ms_mg) for k in range(1, len(sig) + 1)]
        assert 1 <= n <= len(sig)
        assert costs[n - 1] <= min(costs) * (1 + 1e-12)


def test_bad_arguments(nd):
    with pytest.raises(nd.NdtmError):
        nd.hybrid_split([1e-3, 1e-2], 0.01, 1.0, 1e-10, 0.1, 1.0)  # not descending
    with pytest.raises(nd.NdtmError):
        nd.hybrid_split([1.0, 0.1], 0.01, 1.0, 0.0, 0.1, 1.0)
    with pytest.raises(nd.NdtmError):
        nd.hybrid_split([1.0, 0.1], -1.0, 1.0, 1e-10, 0.1, 1.0)
