"""What the trained proposer gains over uniform proposals (the sampling comparison at a
reduced size: thousands of minima instead of a million).

Minima are collected with uniform proposals relaxed by FIRE to |F| < 1e-4 eV/A, the
proposer is trained on the distinct ones (IMLE), then both proposal forms run the same
number of proposals against fresh archives (distinct within 0.01 eV).  Asserted: the
training loss falls; learned proposals land nearer to minima (more of them converge, and
relaxation moves their atoms less, RMS over the molecule) while still reaching most of the
distinct minima.  Minima/s and mean FIRE steps of both forms are reported.
"""
import numpy as np
import pytest

from paper_2508_15522_amd import configs, device as D, sampling as SM, synth as S
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def test_learned_proposals_land_near_minima():
    D.require_gpu()
    cfg = configs.GRID_SMALL
    grid = D.build_physical_grid(cfg.substrate(), D.spec_for(cfg))
    res = SM.compare_learned_vs_uniform(grid, S.mol_chain24(), collect_minima=6000, collect_rep=2048,
                                        train_steps=300, eval_rounds=3, eval_rep=1024, log=announce)
    announce(f"  result: {res}")
    tr = res["training"]
    assert tr["loss_last"] < 0.8 * tr["loss_first"]
    assert res["learned"]["converged"] > 0.5 * res["learned"]["proposals"]
    L, U = res["learned"], res["uniform"]
    assert L["converged"] > U["converged"]
    assert L["mean_rms_move"] < 0.95 * U["mean_rms_move"]
    assert L["distinct_minima"] >= 0.75 * U["distinct_minima"]
