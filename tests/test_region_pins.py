"""The oracle's region-I subtraction and Gaussian-charge correction against
hand-summed images, point-charge clusters, the tin-foil surface term,
invariance, finite differences and the limits of the Gaussian exponent."""
import pytest

from tests import _region_pins


@pytest.mark.parametrize("name", list(_region_pins.REGION_PINS))
def test_region_pin(name):
    fn, tol = _region_pins.REGION_PINS[name]
    err = fn()
    assert err <= tol, f"{name}: deviation {err:.3e} > {tol:.0e}"
