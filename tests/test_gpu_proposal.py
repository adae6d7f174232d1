"""What the trained proposal network gains over plain random starts.

The learned-proposal workload at a quarter of its size (64x64x16 open
BaTiO3 boxes, films of 8..16 layers, T ~ U(250, 450) K, starts of
U(-0.1, 0.1) C/m^2 noise on 8^3 blocks; 256 training starts relaxed for at
most 8000 steps, 32 held-out samples): relax the training starts into a
dataset, train the network on the GPU through the library's own kernels on
the states that relaxed (no symmetry augmentation: with this few states it
lowers the gain), then relax the held-out samples from their random starts
and from the network's proposals to the same energy criterion (relaxed
instances retired, so each ends in the state it relaxed in).  The gain is
asserted over all held-out samples and over those where the proposal-started
run ends at an equal (within 1e-6) or lower energy than the plain run.  The
run is seeded and the kernels are deterministic, so the numbers repeat on
the same build."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import tdgl_inputs as I  # noqa: E402
from tests.gpu_helpers import announce  # noqa: E402


@pytest.mark.timeout(400)
def test_trained_proposal_relaxes_in_fewer_steps():
    from paper_2605_28800_amd import relaxation as R
    shape, noise_div, width = (16, 64, 64), 8, 32
    n_train, n_test, eval_cap = 256, 32, 20000
    announce("proposal gain: %d training starts, %d held-out" % (n_train, n_test))
    T, th, noise = I.net_conditions(n_train + n_test, shape, noise_div, seed=7,
                                    T_range=(250.0, 450.0), thickness_range=(8, 16))
    starts = torch.from_numpy(I.noise_start(noise, th, shape)).cuda()
    r = R.proposal_experiment(lambda k: I.c5_recipe(int(k), shape), shape, noise_div, T, th,
                              noise, starts, n_train, I.net_params(width, seed=7), width,
                              data_steps=8000, eval_steps=eval_cap, train_steps=2000, batch=8,
                              seed=7, log=announce, augment=False)
    capped = lambda s: np.where(s > 0, s, eval_cap)
    plain, prop = capped(r["plain_steps"]), capped(r["proposal_steps"])
    print("[gain] plain mean %.0f, proposal mean %.0f; relaxed %d / %d of %d; losses %.3e -> %.3e"
          % (plain.mean(), prop.mean(), (r["plain_steps"] > 0).sum(),
             (r["proposal_steps"] > 0).sum(), n_test, r["losses"][:20].mean(),
             r["losses"][-20:].mean()), flush=True)
    assert np.isfinite(r["losses"]).all() and r["losses"][-20:].mean() < r["losses"][:20].mean()
    assert (r["proposal_steps"] > 0).sum() >= (r["plain_steps"] > 0).sum()
    assert prop.mean() < 0.85 * plain.mean()
    # at equal final-energy accuracy: the samples whose proposal-started run
    # ends within 1e-6 of, or below, the plain run's energy, both relaxed
    dF = (r["proposal_F"] - r["plain_F"]) / np.maximum(np.abs(r["plain_F"]), r["energy_floor"])
    m = (dF <= 1e-6) & (r["plain_steps"] > 0) & (r["proposal_steps"] > 0)
    print("[gain at equal energy] %d samples: plain mean %.0f, proposal mean %.0f"
          % (m.sum(), r["plain_steps"][m].mean(), r["proposal_steps"][m].mean()), flush=True)
    # (measured: 15-17 of 32 samples; the rest end in another minimum, mostly
    # at a higher energy).  With 90 relaxed training states the network, and
    # with it this ratio, follows rounding-level differences between builds
    # of the kernels (which change the training set): 0.80, 0.85 and 0.86
    # measured (8333 -> 6687, 8013 -> 6769, 9076 -> 7812 steps), so the bar
    # asks for a gain beyond that spread, 0.9; with 4096 training starts the
    # same ratio is 0.44-0.46
    assert m.sum() >= n_test // 4
    assert r["proposal_steps"][m].mean() < 0.9 * r["plain_steps"][m].mean()
