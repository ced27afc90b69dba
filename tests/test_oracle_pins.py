"""The CPU oracle against the paper's worked example, closed forms,
brute force and spectral invariants (no GPU)."""
import pytest

from oracle import oracle as O

from oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin):
    pin(O.load())
