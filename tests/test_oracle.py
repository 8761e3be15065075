"""The CPU oracle against its pins (CPU only)."""
import pytest

import oracle
from tests import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(oracle.default())


def test_config1_reference_values():
    """100 x 100 triangulated grid in natural order: the values the oracle gives
    (First-Fit 4 colours; the round-synchronous schedule needs 149 recolouring
    rounds because a defect front sweeps the grid one diagonal at a time)."""
    import graphgen as gg
    rp, ci = gg.tri_grid(100)
    assert len(ci) == 2 * 29601
    c, K = oracle.seq_ff(rp, ci)
    assert K == 4
    r = oracle.rsync(rp, ci)
    assert r["K"] == 4 and r["rounds"] == 149 and r["conflicts"] == 828300
    assert oracle.check(rp, ci, r["colors"]) == 0
