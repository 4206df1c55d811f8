"""The oracle against the paper's worked example, closed forms and invariants."""
import pytest

import oracle
import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(oracle.default())


def test_oracle_rejects_non_binary_bytes():
    import numpy as np
    with pytest.raises(ValueError):
        oracle.counts(np.full((1, 4), 2, np.uint8), np.zeros((1, 4), np.uint8), oracle.MIXTURE)
