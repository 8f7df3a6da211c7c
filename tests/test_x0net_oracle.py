"""The start-vector network's float64 reference against its pins (tests/x0net_pins.py)."""
import pytest

from oracle import x0net_oracle as N
from tests import x0net_pins as P

PINS = sorted(k for k in dir(P) if k.startswith("pin_"))


@pytest.mark.parametrize("name", PINS)
def test_pin(name):
    fn = getattr(P, name)
    if name == "pin_network_gradient_finite_differences":
        fn(N, False)
        fn(N, True)
    else:
        fn(N)
