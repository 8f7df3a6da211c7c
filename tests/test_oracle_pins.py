"""The CPU oracle against its pins (closed forms, invariants, brute force, textbook
special cases, dense direct solves, Theorem 2.1, jump independence)."""
import pytest

from oracle import psl_oracle as O
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(O)
