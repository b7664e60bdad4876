"""The oracle's Philox4x32-10 against the generator's published known-answer
vectors, and the uniform initializer's definition against plain properties."""
import os

import numpy as np

from oracle.philox import philox4x32_10, uniform_init

HERE = os.path.dirname(os.path.abspath(__file__))


def test_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        got = philox4x32_10(np.array(w[0:4], np.uint32), np.array(w[4:6], np.uint32))
        assert [int(v) for v in got] == w[6:10]


def test_uniform_init_properties():
    lo = np.array([-2.8, 0.1, -np.pi, 0.25], np.float64)
    hi = np.array([2.8, 0.3, np.pi, 0.55], np.float64)
    x = uniform_init(lo, hi, 20000, seed=42)
    assert x.dtype == np.float32 and x.shape == (20000, 4)
    assert np.all(x >= lo.astype(np.float32)) and np.all(x <= hi.astype(np.float32))
    u = (x - lo) / (hi - lo)
    assert np.all(np.abs(u.mean(0) - 0.5) < 0.01) and np.all(np.abs(u.var(0) - 1 / 12) < 0.005)
    # distinct seeds and distinct particles draw different numbers
    assert not np.array_equal(x, uniform_init(lo, hi, 20000, seed=43))
    assert len(np.unique(x[:, 0])) > 19000
