"""The CPU oracle against its pins (see tests/pins.py for what each checks)."""
import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(oracle.load())


def test_threads_do_not_change_results():
    import numpy as np
    import synth
    t = synth.config1_tables()
    q = synth.config1_queries(20_000)
    a = oracle.lookup(t, q.E, q.mat)
    b = oracle.lookup(t, q.E, q.mat, threads=4)
    assert np.array_equal(a, b)
