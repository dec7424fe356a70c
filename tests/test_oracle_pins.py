"""The FP64 oracle against its pins (closed forms, library routines, brute force, invariants)."""
import pytest

from oracle import bfly_oracle
from tests.pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin):
    pin(bfly_oracle)
