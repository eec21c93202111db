"""Host logic of the statistics campaign (no GPU): the batch-means error bar
of a correlated series."""
import math

import numpy as np

from paper_1701_02005_amd.campaign import batch_means


def test_batch_means_of_independent_samples():
    rng = np.random.default_rng(3)
    ses = []
    for _ in range(200):
        x = 2.0 + 0.5 * rng.standard_normal(1000)
        m, se = batch_means(x, 10)
        assert abs(m - x.mean()) < 1e-12
        ses.append(se)
    # standard error of the mean of 1000 iid samples of sd 0.5
    assert abs(np.mean(ses) / (0.5 / math.sqrt(1000)) - 1.0) < 0.1


def test_batch_means_sees_correlation():
    """An AR(1) series with correlation time ~50 samples: batch means over
    batches of 1000 give the larger, correct standard error."""
    rng = np.random.default_rng(5)
    phi, n = 0.98, 20000
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    _, se = batch_means(x, 20)
    naive = x.std() / math.sqrt(n)
    exact = math.sqrt(1 / (1 - phi ** 2)) * math.sqrt((1 + phi) / (1 - phi)) / math.sqrt(n)
    assert se > 3 * naive
    assert 0.5 < se / exact < 1.6
