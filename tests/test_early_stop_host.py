"""Host logic of the learned early stop (no GPU): the stop threshold is the smallest
candidate whose first confident checkpoint costs at most the target on every
validation run, and a run that never reaches the threshold costs nothing."""
import numpy as np

from paper_2004_03972_amd import early_stop as E


def test_pick_threshold_smallest_safe_candidate():
    per = [[(0.6, 0.01), (0.8, 0.0005), (0.95, 0.0)],
           [(0.7, 0.002), (0.9, 0.0)]]
    cands = np.linspace(0.50, 0.999, 200)
    c = E.pick_threshold(per, 1e-3, cands)
    # run 2 must not stop at 0.7 (cost 0.002): c > 0.7; run 1 then stops at 0.8 (0.0005)
    assert c == cands[cands > 0.7][0]
    # a looser target lets run 2 stop at its first checkpoint
    assert E.pick_threshold(per, 0.002, cands) == cands[cands > 0.6][0]
    # and the loosest stops both at once
    assert E.pick_threshold(per, 0.01, cands) == cands[0]


def test_pick_threshold_no_stop_costs_nothing_and_inf_when_unsafe():
    per = [[(0.3, 0.5)]]                      # never confident: always the full run
    assert E.pick_threshold(per, 0.0) == 0.5
    per = [[(0.9995, 0.2)]]                   # confident beyond every candidate, and wrong
    assert E.pick_threshold(per, 0.1) == float("inf")
