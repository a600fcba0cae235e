"""Host-side logic that needs no GPU: the time-to-loss target and its
first crossing (the library is not loaded)."""

import pytest

from paper_2508_10743_amd import warmstart as WS


def test_loss_target_for_negative_and_positive_losses():
    """Equal final loss within 0.5 %: LNCC's negative F must come within
    0.5 % of |F| from above, not beat F by it."""
    assert WS.loss_target(-0.2) == pytest.approx(-0.199)
    assert WS.loss_target(0.2) == pytest.approx(0.201)
    t, k = WS.first_reach([1.0, 2.0, 3.0], [-0.1, -0.1995, -0.2], WS.loss_target(-0.2))
    assert (t, k) == (2.0, 2)
    assert WS.first_reach([1.0], [0.5], WS.loss_target(0.2)) == (None, None)
