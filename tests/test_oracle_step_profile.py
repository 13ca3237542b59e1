"""The step-profile advection test of Table 3 on the oracle's compound-only
step: the outcome the paper reports for the first opening of the source
channel. At Pe ~ 4100 (cases a, b) the front carries overshoots that do not
decay; at Pe ~ 800 (cases c, d) they are smoothed out; a tenfold smaller
time step (b against a, d against c) changes neither picture. Besides, the
front at the channel's centre travels U T (200 nodes in every case) and C
stays bounded. These hold for the scheme itself, so they pin the oracle's
run of the experiment (and through the GPU parity tests, the kernels')."""
import numpy as np
import pytest

from paper_1307_4703_amd import workloads as W
from tests.parity_util import make_oracle


def _run(case, n_records=10):
    wl, fld = W.step_profile(case)
    o = make_oracle(wl)
    o.init()
    steps = W.STEP_PROFILE_CASES[case][2]
    fl = wl.mask == 0
    over, under = [], []
    for _ in range(n_records):
        o.cde_step(steps // n_records, [fld])
        C = o.fields()[3]
        over.append(C[fl].max() - 1.0)
        under.append(C[fl].min())
    return wl, o, np.array(over), np.array(under)


@pytest.fixture(scope="module")
def runs():
    return {c: _run(c) for c in "abcd"}


def test_high_peclet_overshoot_persists(runs):
    for c in "ab":
        _, _, over, _ = runs[c]
        assert over.max() > 0.3, c
        assert over[-1] > 0.15, (c, over[-1])  # not decayed at the end


def test_low_peclet_overshoot_smoothed(runs):
    for c in "cd":
        _, _, over, _ = runs[c]
        assert over.max() > 0.1, c          # present at the first opening
        assert over[-1] < 0.01, (c, over[-1])


def test_tenfold_time_step_changes_little(runs):
    for fine, coarse in (("b", "a"), ("d", "c")):
        of, oc = runs[fine][2], runs[coarse][2]
        assert abs(of.max() - oc.max()) < 0.1
        assert (of[-1] > 0.15) == (oc[-1] > 0.15)


def test_front_travels_U_T(runs):
    for c in "abcd":
        wl, o, _, under = runs[c]
        C = o.fields()[3]
        centre = C[wl.ny // 2, 1:-1]
        front = int(np.argmax(centre < 0.5))
        assert 180 <= front <= 205, (c, front)
        assert under.min() > -0.1, c
