"""Pins of the oracle's robot contact rows, door / drawer joints and their
limit rows, implicit PD drive and joint damping, explicit gyroscopic term,
sliding sensitivity of the adjoint and robot contact cap (the physics each
pin states is in tests/_pins.py)."""
import pytest

import oracle
from _pins import ALL


def _mk(b, **kw):
    return oracle.Oracle(b, **kw)


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__[4:] for p in ALL])
def test_pin(pin):
    pin(_mk)
