"""CPU: the bench's host-side arithmetic -- how many evaluations one graph
holds (whole replays time exactly the requested number) and the algorithmic
flop count of one evaluation that the roofline fraction divides by."""
import pytest

import bench


@pytest.mark.parametrize("steps,n", [(200, 10), (50, 10), (25, 5), (20, 10), (7, 7), (13, 1), (1, 1), (99, 9)])
def test_evals_per_graph_divides_steps(steps, n):
    got = bench.evals_per_graph(steps)
    assert got == n
    assert steps % got == 0 and 1 <= got <= bench.EVALS_PER_GRAPH


def test_flops_per_eval_headline():
    """Three passes of N(N+1)/2 exponentials at 16 flops: 25.19 MFLOP at N = 1024."""
    assert bench.flops_per_eval(1024) == 3 * 1024 * 1025 // 2 * 16
    assert abs(bench.flops_per_eval(1024) / 1e6 - 25.19) < 0.01


@pytest.mark.parametrize("steps,warmup,replays", [(200, 50, 5), (20, 5, 5), (20, 60, 6), (7, 0, 8), (1, 1, 50)])
def test_warmup_covers_at_least_the_minimum(steps, warmup, replays):
    n = bench.evals_per_graph(steps)
    got = bench.warmup_replays(steps, warmup)
    assert got == replays
    assert got * n >= max(warmup, bench.MIN_WARMUP_EVALS)
    assert (got - 1) * n < max(warmup, bench.MIN_WARMUP_EVALS)
