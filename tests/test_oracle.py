"""The FP64 oracle against its pins (closed forms, invariants, brute force, the
published radix-2 error bound, an independent library routine)."""
import pytest

import oracle
from tests import oracle_pins


@pytest.fixture(scope="module")
def o():
    oracle.build()
    return oracle.default()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS + [oracle_pins.pin_bad_arguments],
                         ids=lambda f: f.__name__)
def test_pin(o, pin):
    pin(o)


def test_split_reading_is_exact():
    """hi + 2^-11 lo is formed exactly in FP64 (both halves are FP16)."""
    import numpy as np

    hi = np.array([[1.0, -0.5]], dtype=np.float16)
    lo = np.array([[1.0, 3.0]], dtype=np.float16)
    z = oracle.from_split(hi, lo)
    assert z[0] == complex(1.0 + 2.0 ** -11, -0.5 + 3.0 * 2.0 ** -11)


def test_rel_l2_conventions():
    import numpy as np

    ref = np.array([[1 + 0j, 0], [0, 0]])
    y = np.array([[1 + 0j, 0.5], [0, 0]])
    e = oracle.rel_l2(y, ref)
    assert abs(e[0] - 0.5) < 1e-15 and e[1] == 0.0
    e2 = oracle.rel_l2(np.array([[0, 1e-3]]), np.zeros((1, 2)))
    assert e2[0] == float("inf")
