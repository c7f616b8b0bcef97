"""The FP64 oracle against its pins (CPU only)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(None)


def test_oracle_rejects_bad_input():
    import numpy as np
    import oracle
    m = np.ones(3)
    x = np.eye(3)
    v = np.zeros((3, 3))
    with pytest.raises(ValueError):
        oracle.regular_force(m, x, v, [3], 1.0, 0.0)
    with pytest.raises(ValueError):
        oracle.regular_force(m, x, v, [0], 0.0, 0.0)
