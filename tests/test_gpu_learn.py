"""The learned force correction trained on the GPU by libpm's own forward and
reverse kernels (force matching against 4x-finer-mesh forces, Adam; the
radial filter also calibrated on fine-mesh power spectra), and what it gains
over the plain coarse particle-mesh method on a held-out seed: the force error
against the fine mesh and the power-spectrum error of a full run against a
fine-mesh run.  Small instance of the C4 setting (64^3 CDM + 8^3 x 70
neutrinos, 64^3 coarse mesh, 256^3 fine mesh, 10 steps from z = 19)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_training_gain_on_held_out_seed(dev):
    from paper_2007_13394_amd import learn
    res = learn.evaluate("C4s_coarse", "C4s_fine", [151, 152, 153], 160, snap_every=2, iters=200,
                      log=lambda *m: say(*m), calib_rounds=4)
    fl, pk = res["force_loss"], res["pk_max_rel_err"]
    say("force loss plain/learned (train)", fl["plain_train"], fl["learned_train"])
    say("force loss plain/learned (held-out)", fl["plain_test"], fl["learned_test"])
    say("P(k) max rel err plain coarse / calibrated / force-matched", pk["plain_coarse"], pk["learned"],
        pk["learned_force_matched"], "k range", res["k_range_hMpc"])
    say("calibration, training-seed error per round", res["calibration"]["train_seed_err"])
    say("r_min plain / learned", res["r_min"]["plain_coarse"], res["r_min"]["learned"])
    say("particle-steps/s", res["particle_steps_per_s"])
    pk_ = res["pk"]
    for i, kk in enumerate(res["k"]):
        say("k %.3f learned/fine %.4f plain/fine %.4f" % (kk, pk_["learned"][i] / pk_["fine"][i],
                                                         pk_["plain_coarse"][i] / pk_["fine"][i]))
    assert np.isfinite(fl["learned_test"])
    assert fl["learned_train"] < 0.8 * fl["plain_train"]
    assert fl["learned_test"] < 0.8 * fl["plain_test"]
    hist = res["calibration"]["train_seed_err"]
    assert min(hist[1:]) < hist[0]          # the calibration improves on the force-matched start
    assert pk["learned"] < 0.5 * pk["plain_coarse"]
