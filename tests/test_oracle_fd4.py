"""The oracle's finite-difference reference solver (Sec. III) against the
checks in fd4_pins: RK4 amplification of every Fourier mode, the RK4 of the
local ODE, the mirror extension, conservation, fourth-order convergence and
an independent NumPy implementation."""
import pytest

import fd4_pins
import oracle


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("check", fd4_pins.FAST_FD4_CHECKS, ids=lambda f: f.__name__)
def test_fd4_pin(orc, check):
    check(orc)
