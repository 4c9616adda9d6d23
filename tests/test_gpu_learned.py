"""The learned refinement indicator end to end on a small decaying-vortex
grid (4^3 roots of 8^3 cells, levels 0..3): snapshots of plain-criterion
runs with two blob placements train the MLP on the GPU; a third placement is
then run with static refinement (the paper's method), plain-criterion regrid
and MLP regrid.

What the trained network must show: it reproduces the criterion's decisions
on held-out snapshots (never the opposite decision), it needs the fallback
for few blocks, and its run stays as close to the plain-criterion run as
that run is to the static one, at a fraction of the static run's cell
updates."""

import pytest

from paper_1508_07982_amd import learned

pytestmark = pytest.mark.gpu


def test_learned_indicator_gain():
    print("learned indicator: n=8 roots=4 max_level=3 60 steps, regrid every 10", flush=True)
    rep = learned.gain_experiment(n=8, roots=4, max_level=3, steps=60, every=10, train_seeds=(11, 12), test_seed=5,
                                  snapshots=20000, epochs=40, log=lambda m: print(m, flush=True))
    tr = rep["training"]
    assert tr["samples"] == 20000 and tr["test"] == 2000
    assert tr["loss_last_epoch"] < tr["loss_first_epoch"]
    assert tr["test_misclassification"] < 0.05
    assert tr["test_opposite_decisions"] < 0.005
    mlp, plain, static = rep["mlp"], rep["plain"], rep["static"]
    assert mlp["fallback_blocks"] < 0.05 * mlp["decided_blocks"]
    assert mlp["rel_l2_velocity_vs_plain"] < static["rel_l2_velocity_vs_plain"]
    assert mlp["cell_updates"] < 0.7 * static["cell_updates"]
    assert abs(mlp["cell_updates"] - plain["cell_updates"]) < 0.1 * plain["cell_updates"]
