"""The single-view workload's depth complexity (mean fragments per covered
pixel, from the oracle's statistics): the literal distribution of centres
in the unit ball gives about 3, and the variant with the ball radius set for
a depth complexity of 8 gives 8."""
from oracle import oracle as O
from paper_2603_27151_amd import workloads as W


def _dc(wl):
    _, _, _, st = O.forward(wl.scene, wl.views[0], O.Opts(seed=wl.seed, mode=1), want_logp=False)
    return st["covering_fragments"] / st["covered_pixels"]


def test_literal_single_view_depth_complexity():
    assert abs(_dc(W.single(with_targets=False)) - 2.97) < 0.05


def test_dc8_single_view_depth_complexity():
    assert abs(_dc(W.single_dc8(with_targets=False)) - 8.0) < 0.05
