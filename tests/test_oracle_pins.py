"""The oracle against its pins (closed forms, brute force, invariants, library routines)."""
import pytest

import oracle
from pins import ALL_PINS


@pytest.fixture(scope="module")
def lib():
    oracle.build(force=False)
    return oracle.load_library()


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin, lib):
    pin(lib)
