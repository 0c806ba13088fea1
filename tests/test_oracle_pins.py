"""The CPU oracle against closed forms, brute-force lattice sums, alpha
independence, finite differences and invariants (no GPU needed)."""
import pytest

from tests import _pins


@pytest.mark.parametrize("name", list(_pins.ALL_PINS))
def test_oracle_pin(name):
    fn, tol = _pins.ALL_PINS[name]
    err = fn()
    assert err <= tol, f"{name}: relative deviation {err:.3e} > {tol:.0e}"


def test_golden_constants_readable():
    assert abs(_pins.lattice_constant("nacl_madelung") - 1.7475645946) < 1e-9
    assert abs(_pins.lattice_constant("cscl_madelung") - 1.7626747731) < 1e-9
    assert abs(_pins.lattice_constant("sc_wigner_xi") + 2.8372974795) < 1e-9
