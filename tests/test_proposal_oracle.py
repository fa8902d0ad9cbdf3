"""Pins of the FP64 oracle of the learned grasp proposal (CPU).

Checks against facts the definitions fix: finite differences of the loss,
the invariances of a max-pooled point encoder, hand cases of the set loss,
and the BF16 format."""
import math

import numpy as np
import pytest

from oracle import proposal as P

NP, NS = 2, 4


def rand_targets(rng, T=5):
    tg = np.concatenate([rng.uniform(-0.1, 0.1, (NP, T, 3)), rng.standard_normal((NP, T, 4))], -1)
    tg[..., 3:] /= np.linalg.norm(tg[..., 3:], axis=-1, keepdims=True)
    return tg


def total_loss(th, cloud, tg, bf=False):
    o, I = P.forward(th, cloud, NP, NS, bf=bf)
    return P.loss(o, I["com"], tg, NP, NS)[0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_is_finite_difference_of_loss(seed):
    rng = np.random.default_rng(seed)
    th = P.init_params(NP, NS, rng)
    cloud = rng.uniform(-0.05, 0.05, (60, 3))
    tg = rand_targets(rng)
    o, I = P.forward(th, cloud, NP, NS)
    _, do = P.loss(o, I["com"], tg, NP, NS)
    g = P.backward(th, I, do, NP, NS)
    # every layer: a few parameters each
    sizes = [int(np.prod(s)) for s in P.layer_shapes(NP, NS)]
    starts = np.cumsum([0] + sizes[:-1])
    h = 1e-6
    for st, n in zip(starts, sizes):
        for i in rng.choice(n, min(n, 4), replace=False) + st:
            e = np.zeros_like(th)
            e[i] = h
            fd = (total_loss(th + e, cloud, tg) - total_loss(th - e, cloud, tg)) / (2 * h)
            assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-7), (i, fd, g[i])


def test_loss_gradient_in_outputs_is_finite_difference():
    rng = np.random.default_rng(7)
    o = rng.standard_normal(NP * NS * 7)
    com = rng.uniform(-0.02, 0.02, 3)
    tg = rand_targets(rng, T=6)
    L, do = P.loss(o, com, tg, NP, NS)
    for i in range(len(o)):
        e = np.zeros_like(o)
        e[i] = 1e-7
        fd = (P.loss(o + e, com, tg, NP, NS)[0] - P.loss(o - e, com, tg, NP, NS)[0]) / 2e-7
        assert fd == pytest.approx(do[i], rel=1e-5, abs=1e-6)


def test_encoder_is_invariant_to_point_order_and_translation():
    rng = np.random.default_rng(3)
    th = P.init_params(NP, NS, rng)
    cloud = rng.uniform(-0.05, 0.05, (80, 3))
    o, I = P.forward(th, cloud, NP, NS)
    o2, _ = P.forward(th, cloud[rng.permutation(80)], NP, NS)
    assert np.allclose(o, o2, rtol=0, atol=1e-12)
    shift = np.array([0.3, -0.2, 0.1])
    o3, I3 = P.forward(th, cloud + shift, NP, NS)
    assert np.allclose(o, o3, rtol=0, atol=1e-10)
    s1, s3 = P.seeds(o, I["com"], NP, NS), P.seeds(o3, I3["com"], NP, NS)
    assert np.allclose(s3[..., :3] - s1[..., :3], shift, atol=1e-12)
    assert np.allclose(s3[..., 3:], s1[..., 3:], atol=1e-12)


def test_max_pool_takes_lowest_index_on_ties():
    rng = np.random.default_rng(4)
    th = P.init_params(NP, NS, rng)
    pts = rng.uniform(-0.05, 0.05, (10, 3))
    cloud = np.concatenate([pts, pts])  # every point twice
    _, I = P.forward(th, cloud, NP, NS)
    live = I["g"] > 0
    assert np.all(I["am"][live] < 10)


def test_set_loss_hand_cases():
    com = np.zeros(3)
    q = np.array([0.5, 0.5, 0.5, 0.5])
    # one seed, one target: L = d + d, d = |dt|^2 / 0.01 + beta (1 - c^2)
    o = np.concatenate([[0.2, 0.0, 0.0], q])  # t = 0.02 m
    tq = np.array([math.cos(0.3), math.sin(0.3), 0.0, 0.0])
    tg = np.concatenate([[0.0, 0.0, 0.0], tq])[None, None, :]
    L, _ = P.loss(o, com, tg, 1, 1)
    c = q @ tq
    d = 0.02 ** 2 / 0.01 + P.BETA * (1 - c * c)
    assert L == pytest.approx(2 * d, rel=1e-13)
    # seeds equal to the targets (as a set, any order, either quaternion sign)
    rng = np.random.default_rng(5)
    tg = rand_targets(rng, T=NS)
    o = np.zeros((NP, NS, 7))
    for p in range(NP):
        perm = rng.permutation(NS)
        o[p, :, :3] = (tg[p, perm, :3] - com) / P.UNIT
        o[p, :, 3:] = tg[p, perm, 3:] * np.where(rng.random(NS) < 0.5, -1.0, 2.5)[:, None]
    L, do = P.loss(o.ravel(), com, tg, NP, NS)
    assert L == pytest.approx(0.0, abs=1e-12)
    assert np.allclose(do, 0.0, atol=1e-10)


def test_bf16_rounding_follows_the_format():
    # BF16 keeps the top 16 bits of an IEEE single; round to nearest, ties to even
    one = 1.0
    ulp = 2.0 ** -7  # spacing of BF16 values in [1, 2)
    assert P.bf16(np.array([one]))[0] == one
    assert P.bf16(np.array([one + ulp / 2]))[0] == one           # tie -> even (1.0)
    assert P.bf16(np.array([one + 3 * ulp / 2]))[0] == one + 2 * ulp  # tie -> even
    assert P.bf16(np.array([one + 0.6 * ulp]))[0] == one + ulp
    assert P.bf16(np.array([-3.0]))[0] == -3.0
    x = np.random.default_rng(0).standard_normal(1000)
    r = P.bf16(x)
    assert np.all(np.abs(r - x) <= (2.0 ** -8 + 2.0 ** -24) * np.abs(x))  # 8 significant bits
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
