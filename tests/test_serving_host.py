"""Host side of serving, on the CPU: the admission charge of a request
(rhg_server_estimate_bytes), the server's refusal without a device, and the
benchmark's request stream and Poisson arrivals, reproducible from their seeds."""
import math
import os
import sys

import numpy as np
import pytest

from paper_1606_09481_amd import rhg

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_estimate_kbar_given():
    for n, kbar in [(5000, 10.0), (2_000_000, 64.0), (1000, 6.0)]:
        want = int(n * kbar / 2 * 8 * 1.25) + n * 256 + (1 << 20)
        assert rhg.rhg_server_estimate_bytes(rhg.params(n, 0.8, kbar=kbar)) == want


def test_estimate_R_given_uses_expected_degree():
    n, alpha, kbar = 100_000, 0.9, 20.0
    R = rhg.rhg_target_radius(n, alpha, kbar)
    a = rhg.rhg_server_estimate_bytes(rhg.params(n, alpha, R=R))
    b = rhg.rhg_server_estimate_bytes(rhg.params(n, alpha, kbar=kbar))
    assert abs(a - b) <= 1e-6 * b  # the radius for kbar has expected degree kbar
    # a smaller disk is denser: larger charge
    assert rhg.rhg_server_estimate_bytes(rhg.params(n, alpha, R=R - 1.0)) > a


def test_estimate_monotone_and_refusals():
    e = lambda n, k: rhg.rhg_server_estimate_bytes(rhg.params(n, 1.0, kbar=k))
    assert e(20_000, 10) < e(40_000, 10) and e(20_000, 10) < e(20_000, 20)
    for bad in (rhg.params(1, 1.0, kbar=10), rhg.params(1000, 0.4, kbar=10), rhg.params(1000, 1.0, kbar=-1.0),
                rhg.params(1000, 1.0, R=float("nan"))):
        with pytest.raises(rhg.RhgError) as ei:
            rhg.rhg_server_estimate_bytes(bad)
        assert ei.value.status == rhg.RHG_EINVAL


def test_server_without_device_is_refused():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(rhg.RhgError) as ei:
        rhg.rhg_server_create(0, 1 << 30)
    assert ei.value.status in (rhg.RHG_EDEVICE, rhg.RHG_EINVAL)


def test_request_stream_reproducible():
    a = bench.serving_requests(rhg, 300, 5)
    b = bench.serving_requests(rhg, 300, 5)
    c = bench.serving_requests(rhg, 300, 6)
    key = lambda reqs: [(p.n, p.alpha, p.kbar, p.seed) for p in reqs]
    assert key(a) == key(b) and key(a) != key(c)
    n = np.array([p.n for p in a])
    assert n.min() >= 1000 and n.max() <= 2_000_000
    assert all(0.55 <= p.alpha <= 1.5 and p.kbar == int(p.kbar) and 6 <= p.kbar <= 64 for p in a)
    assert [p.seed for p in a] == [1000 + i for i in range(300)]
    # log-uniform n: about a third of the requests below 10^4 ... 2 * 10^4
    frac = np.mean(np.log(n) < math.log(1e3) + (math.log(2e6) - math.log(1e3)) / 3)
    assert 0.2 < frac < 0.45


def test_poisson_arrivals_reproducible():
    t1 = bench.poisson_arrivals(20_000, 500.0, 8)
    t2 = bench.poisson_arrivals(20_000, 500.0, 8)
    assert np.array_equal(t1, t2) and np.all(np.diff(t1) > 0)
    gaps = np.diff(np.concatenate([[0.0], t1]))
    assert abs(gaps.mean() * 500.0 - 1.0) < 0.03          # mean gap 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05     # exponential: cv = 1
