"""Host checks of the seeded input generators for the paper's simulation
set-up (Sec. VI-A, Table I; Sec. V, Fig. 4): quarter-sphere Fibonacci poses plus poses
from above, Gaussian-mixture initialisation, and the table in the collision
cloud.  These generators hold none of the method's arithmetic."""
import math

import numpy as np
import pytest

import oracle
from paper_2412_08346_amd import synth

ANCHOR = np.array([0.01, -0.02, 0.03])
TIP = np.array([0.0, 0.0, 0.0164])


def frames(th):
    th = th.astype(np.float64)
    out = []
    for j in range(th.shape[1]):
        Rm = oracle.quat_to_rot(th[3:, j])
        out.append((Rm, Rm @ TIP + th[:3, j]))
    return out


@pytest.mark.parametrize("k", [1, 5, 24, 64])
def test_quarter_sphere_directions(k):
    d = synth.quarter_sphere_dirs(k)
    assert d.shape == (k, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    assert (d[:, 2] >= 0).all() and (d[:, 0] <= 0).all()  # above the table, arm side (-x)
    # the points are Fibonacci points: distinct and roughly evenly spread
    g = d @ d.T - 2 * np.eye(k)
    assert g.max() < 1.0 - 1e-9


def test_paper_initialisation_is_quarter_plus_six_from_above():
    K, dist = 30, 0.12
    th = synth.tabletop_poses(K, ANCHOR, TIP, dist)
    assert th.shape == (7, K)
    rolls = []
    for j, (Rm, p_tip) in enumerate(frames(th)):
        assert np.linalg.norm(p_tip - ANCHOR) == pytest.approx(dist, abs=1e-6)
        u = (p_tip - ANCHOR) / dist
        assert np.allclose(Rm[:, 2], -u, atol=1e-6)  # looks at the object
        if j >= K - 6:
            assert np.allclose(u, [0, 0, 1], atol=1e-6)  # straight above
            rolls.append(math.atan2(Rm[1, 0], Rm[0, 0]))
        else:
            assert u[2] >= -1e-7 and u[0] <= 1e-7
    # six distinct rolls, pi/6 apart modulo the half turn a parallel gripper repeats
    r = np.sort(np.mod(np.array(rolls) - rolls[0], math.pi))
    assert np.allclose(np.diff(r), math.pi / 6, atol=1e-6)


def test_gmm_initialisation_concentrates_on_the_means():
    means = [(0.0, 0.0, 1.0), (-1.0, 0.0, 0.0)]
    th = synth.gmm_poses(400, ANCHOR, TIP, 0.1, means, 0.1, np.random.default_rng(0))
    us = np.array([(p - ANCHOR) / 0.1 for _, p in frames(th)])
    assert np.allclose(np.linalg.norm(us, axis=1), 1.0, atol=1e-5)
    near = np.maximum(us @ np.array(means[0]), us @ np.array(means[1]))
    assert (near > math.cos(math.radians(40))).mean() > 0.97
    assert 0.4 < (us[:, 2] > 0.7).mean() < 0.6  # equal weights


def test_table_plane_and_tabletop_workload():
    pb, st = synth.workload_tabletop()
    M = pb.r_off[1]
    assert 1100 <= len(pb.C) <= 1900  # object with table (Table I)
    assert np.array_equal(pb.C[:M], pb.R)
    table = pb.C[M:].astype(np.float64)
    assert np.ptp(table[:, 2]) == 0 and table[0, 2] < pb.R[:, 2].min()
    sp = np.diff(np.unique(np.round(table[:, 0], 6)))
    assert np.allclose(sp, 0.005, atol=1e-6)
    assert pb.n_pre == 10 and pb.K == 30
    assert st.k_stein == 15 and st.k_max == 40 and st.minibatch == 1
