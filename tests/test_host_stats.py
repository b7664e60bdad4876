"""Host-side statistics of the time-to-satisfy comparisons (no GPU).

The comparison at equal solve rate (Sec. VII, learned seeds and the
Sampling baseline) takes, for each method, the time by which it has solved
the common fraction of scenes."""
import itertools

import pytest

from paper_2411_11833_amd import seeds as SD


def test_equal_rate_times_picks_the_kth_solved_time():
    a = [3.0, None, 1.0, 2.0]          # 3 of 4 solved
    b = [None, 5.0, None, 4.0]         # 2 of 4 solved
    ca, cb, r, ta, tb = SD.equal_rate_times(a, b)
    assert (ca, cb, r) == (0.75, 0.5, 0.5)
    assert (ta, tb) == (2.0, 5.0)      # 2nd fastest of each


def test_equal_rate_times_none_when_one_side_never_solves():
    assert SD.equal_rate_times([None, None], [1.0, 2.0]) == (0.0, 1.0, 0.0, None, None)


@pytest.mark.parametrize("n", [25, 50, 100])
def test_equal_rate_times_exact_for_every_count(n):
    # Counts whose fraction times n rounds above the count in floating point
    # (7/25 * 25 and many more) must still index the k-th solved time.
    for sa, sb in itertools.product(range(n + 1), repeat=2):
        a = [float(i) for i in range(sa)] + [None] * (n - sa)
        b = [10.0 + i for i in range(sb)] + [None] * (n - sb)
        ca, cb, r, ta, tb = SD.equal_rate_times(a, b)
        k = min(sa, sb)
        if k == 0:
            assert ta is None and tb is None
        else:
            assert ta == float(k - 1) and tb == 10.0 + k - 1
