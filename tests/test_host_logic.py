"""Host-side logic that needs no device: the autotuner's candidate launch
shapes and cache keys."""
import types

import pytest

from paper_2305_18025_amd import _lib
from paper_2305_18025_amd.tune import SPLITS, _bucket, cache_key, candidates


def _abi_accepts(threads, per, nmax):
    """The rules pimdb_set_tuning enforces (include/pimdb.h)."""
    return (threads in (64, 128, 256, 512, 1024) and per in (1, 2, 4, 8)
            and not (per >= 4 and threads > 512) and threads * per >= nmax)


@pytest.mark.parametrize("nmax", [1, 2, 63, 64, 65, 511, 512, 1024, 1025, 2047, 2048, 2049, 4095, 4096])
def test_candidates_are_valid_launch_shapes(nmax):
    c = candidates(nmax)
    assert c, "every supported size has a candidate"
    assert len(set(c)) == len(c)
    whole = [(t, p) for t, p, g in c if g == 0]
    split = [g for t, p, g in c if g > 0]
    assert whole, "whole recursions are always a candidate"
    # split recursions only where a system has blocks beyond its first two
    assert split == (list(SPLITS) if nmax > 128 else [])
    for threads, per in whole:
        assert _abi_accepts(threads, per, nmax), (threads, per)
        # no shape that leaves three quarters of the lanes idle, except the
        # narrowest workgroup
        assert threads == 64 or threads * per < 4 * nmax


def test_candidates_up_to_the_largest_system():
    for nmax in range(1, _lib.MAX_N + 1, 37):
        assert candidates(nmax)
    # above 2048 particles only the 8-rows-per-thread shape holds a whole
    # recursion; large batches are never split
    assert candidates(_lib.MAX_N, S=256) == [(512, 8, 0)]
    assert [g for _, _, g in candidates(_lib.MAX_N, S=1) if g] == list(SPLITS)


def test_cache_key_buckets():
    assert [_bucket(x) for x in (1, 2, 3, 64, 65, 1000, 1024, 1025)] == [1, 2, 4, 64, 128, 1024, 1024, 2048]
    eng = types.SimpleNamespace(N=[95, 1930, 700], S=64, precision="fp64", box=0.0)
    assert cache_key(eng) == "N2048_S64_fp64_open"
    eng2 = types.SimpleNamespace(N=[4096], S=1, precision="mixed", box=16.0)
    assert cache_key(eng2) == "N4096_S1_mixed_box"
    # batches of the same bucketed shape share an entry
    eng3 = types.SimpleNamespace(N=[1100, 2000], S=40, precision="fp64", box=0.0)
    assert cache_key(eng3) == cache_key(types.SimpleNamespace(N=[1500], S=64, precision="fp64", box=0.0))
