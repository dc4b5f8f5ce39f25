"""Host-side logic of the package (no GPU): Doerfler marking against the
oracle's independent implementation."""

import numpy as np

import oracle


def test_host_doerfler_matches_oracle():
    from paper_1901_08393_amd.adaptive import doerfler

    rng = np.random.default_rng(0)
    for _ in range(50):
        n = int(rng.integers(1, 300))
        eta2 = rng.choice([0.1, 0.2, 0.5], n) if rng.random() < 0.3 else rng.exponential(1.0, n)
        th = float(rng.uniform(0.05, 1.0))
        assert np.array_equal(doerfler(eta2, th), oracle.doerfler(eta2, th))
