"""Reconstruction of initial modes through the hand-written reverse mode on a
small instance: starting from zero modes, gradient descent (pm_adam) on the
final-density loss against a seeded target run lowers the loss and moves the
estimate towards the true modes."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_reconstruction_descends(dev):
    from paper_2007_13394_amd import reconstruct
    res = reconstruct.reconstruct("C5_fd32", target_seed=303, iters=15, lr=0.05, pool=1, log=say)
    say("loss", res["loss"][0], "->", res["loss"][-1], "corr", res["corr_modes"],
        "corr (k < k_Nyq / 4)", res["corr_modes_k_below_quarter_nyquist"])
    assert res["loss"][-1] < 0.5 * res["loss"][0]
    assert res["corr_modes_k_below_quarter_nyquist"] > 0.3
