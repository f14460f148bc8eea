"""CPU pins of the oracle's bridge ranking (Sec. IV-B), maximum-speed step
(Eq. 8), path validator, capacity reading and learned draw; the checks
themselves live in oracle_pins.py so that the mutant tests can rerun them."""
import pytest

from tests import oracle_pins


@pytest.mark.parametrize("name", sorted(oracle_pins.PINS))
def test_oracle_pin(oracle_lib, name):
    oracle_pins.PINS[name](oracle_lib)

