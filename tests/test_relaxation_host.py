"""Host logic of the relaxation driver (no GPU): the energy criterion, the
recorded relax step of each instance and the step cap, on a stand-in
context whose energies follow known sequences."""
import numpy as np

from paper_2605_28800_amd import relaxation as R


class FakeBatch:
    """energies(k) of each instance after k calls of step(check)."""

    def __init__(self, curves):
        self.curves = curves
        self.k = 0
        self.steps = 0

    def step(self, n):
        self.k += 1
        self.steps += n

    def energies_batch(self):
        F = np.zeros((len(self.curves), 5))
        F[:, 4] = [c(self.k) for c in self.curves]
        return F, np.zeros((len(self.curves), 3))


def test_relax_records_the_first_check_below_the_tolerance():
    floor = 1e-20
    curves = [
        lambda k: -1.0 - 0.5 ** k,           # change 0.5^k: below 1e-6 once 0.5^k < ~1e-6
        lambda k: -2.0,                       # already stationary: relaxed at the first check
        lambda k: -1.0 - 1e-3 * k,            # never relaxes
    ]
    ctx = FakeBatch(curves)
    done, steps = R.relax(ctx, floor, check=100, max_steps=5000)
    # instance 0: |F(k) - F(k-1)| = 0.5^k < 1e-6 * |F(k)| first at k = 20
    k0 = next(k for k in range(1, 100) if 0.5 ** k < 1e-6 * (1.0 + 0.5 ** k))
    assert done[0] == 100 * k0
    assert done[1] == 100
    assert done[2] == -1
    assert steps == 5000 and ctx.steps == 5000


def test_relax_stops_when_all_have_relaxed_and_uses_the_floor():
    # |F| tiny: the floor decides (paraelectric instance near F = 0)
    curves = [lambda k: 1e-12 * 0.5 ** k, lambda k: -3.0]
    ctx = FakeBatch(curves)
    done, steps = R.relax(ctx, floor=1e-3, check=50, max_steps=10000)
    assert list(done) == [50, 50]
    assert steps == 50


def test_relax_floor_scales_with_the_volume():
    import tdgl_inputs as I
    c = I.c5_recipe(8, (16, 64, 64))
    f = R.relax_floor(c)
    assert np.isclose(f, c["scales"]["alpha_ref"] * 1e-3 * 64 * 64 * 16 * 1e-27)
