"""The iteration-count agreement rule of the GPU parity tests, on made-up
residual histories (threshold 1e-10 * ||b|| with ||b|| = 1)."""
from types import SimpleNamespace

from parity_rules import iters_agree

TOL = 1e-10


def _info(resnorms):
    # the oracle stops at the first residual at or below the threshold
    iters = next(k for k, r in enumerate(resnorms) if r <= TOL)
    return SimpleNamespace(iters=iters, resnorms=list(resnorms))


def test_equal_counts_agree():
    assert iters_agree(3, _info([1.0, 1e-4, 1e-8, 5e-11]), TOL, 1.0)


def test_one_fewer_only_if_the_oracle_nearly_stopped_earlier():
    # oracle stops at 3; its residual after 2 iterations was just above the threshold
    assert iters_agree(2, _info([1.0, 1e-4, 1.1e-10, 5e-11]), TOL, 1.0)
    assert not iters_agree(2, _info([1.0, 1e-4, 1.3e-10, 5e-11]), TOL, 1.0)


def test_one_more_only_if_the_oracle_barely_stopped():
    assert iters_agree(4, _info([1.0, 1e-4, 1e-8, 0.9e-10]), TOL, 1.0)
    assert not iters_agree(4, _info([1.0, 1e-4, 1e-8, 0.5e-10]), TOL, 1.0)


def test_two_apart_never_agree():
    assert not iters_agree(1, _info([1.0, 1.05e-10, 1.01e-10, 0.99e-10]), TOL, 1.0)
    assert not iters_agree(5, _info([1.0, 1e-4, 1e-8, 0.99e-10]), TOL, 1.0)
