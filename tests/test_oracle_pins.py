"""The CPU oracle against the paper's closed forms, invariants and brute force."""
import pytest

import oracle
from tests import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


@pytest.mark.parametrize("pin", pins.PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)
