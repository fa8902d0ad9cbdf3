"""GPU (HIP, gfx950) vs FP64 oracle for the learned grasp proposal.

The oracle runs in its BF16 mode (the operands of the kernel's BF16 matrix
products rounded the same way), so the remaining differences are FP32 versus
FP64 accumulation.  No input and no expected value comes from the HIP path."""
import numpy as np
import pytest

from oracle import proposal as OP
import paper_2412_08346_amd.proposal as PP

pytestmark = pytest.mark.gpu
NPRE, NSEED = 3, 8


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)


def random_params(rng):
    th = OP.init_params(NPRE, NSEED, rng)
    # non-zero biases everywhere, output layer at a useful scale
    sizes = [int(np.prod(s)) for s in OP.layer_shapes(NPRE, NSEED)]
    o = 0
    for k, n in enumerate(sizes):
        if k % 2 == 1:
            th[o:o + n] = rng.normal(0.0, 0.1, n)
        if k == 10:
            th[o:o + n] *= 30.0
        o += n
    return th.astype(np.float32).astype(np.float64)


def clouds_for(rng, sizes):
    return [(rng.standard_normal((m, 3)) * [0.04, 0.03, 0.02] + rng.uniform(-0.2, 0.2, 3)).astype(np.float32)
            for m in sizes]


def test_forward_matches_oracle_ragged_objects():
    torch = _gpu()
    rng = np.random.default_rng(11)
    th = random_params(rng)
    clouds = clouds_for(rng, [1, 63, 64, 65, 300, 5000])
    net = PP.ProposalNet(NPRE, NSEED, max_obj=len(clouds), params=th.astype(np.float32))
    seeds, raw = net.forward(clouds)
    torch.cuda.synchronize()
    raw = raw.cpu().numpy().astype(np.float64)
    seeds = seeds.cpu().numpy().astype(np.float64)
    for i, c in enumerate(clouds):
        o, I = OP.forward(th, c.astype(np.float64), NPRE, NSEED, bf=True)
        scale = max(np.abs(o).mean(), 1e-6)
        err = np.abs(raw[i] - o).max()
        say(f"[proposal] object {i} ({len(c)} points): max |raw - oracle| {err:.3g}, scale {scale:.3g}")
        assert err <= 1e-3 * scale
        s_or = OP.seeds(o, I["com"], NPRE, NSEED).reshape(-1, 7)
        k = NPRE * NSEED
        s_gpu = seeds[:, i * k:(i + 1) * k].T
        assert np.abs(s_gpu[:, :3] - s_or[:, :3]).max() <= 1e-4 * (1 + np.abs(s_or[:, :3]).max())
        assert np.abs(s_gpu[:, 3:] - s_or[:, 3:]).max() <= 2e-3
        assert np.all(s_gpu[:, 3] >= 0)


def gap_ok(th, c):
    """True if no channel's max is nearly tied with another point's value
    (the argmax, and so the gradient's route, would then be ambiguous)."""
    _, I = OP.forward(th, c.astype(np.float64), NPRE, NSEED, bf=True)
    h3 = I["h3"]
    if h3.shape[0] < 2:
        return True
    top2 = np.sort(h3, axis=0)[-2:]
    live = top2[1] > 0
    gap = (top2[1] - top2[0])[live] / np.maximum(top2[1][live], 1e-30)
    return bool(np.all(gap > 1e-4))


def test_loss_and_gradient_match_oracle():
    torch = _gpu()
    rng = np.random.default_rng(12)
    th = random_params(rng)
    sizes = [2, 64, 130, 700, 2000]
    clouds = []
    while len(clouds) < len(sizes):
        c = clouds_for(rng, [sizes[len(clouds)]])[0]
        if gap_ok(th, c):
            clouds.append(c)
    T = 5
    tg = np.concatenate([rng.uniform(-0.3, 0.3, (len(clouds), NPRE, T, 3)),
                         rng.standard_normal((len(clouds), NPRE, T, 4))], -1)
    tg[..., 3:] /= np.linalg.norm(tg[..., 3:], axis=-1, keepdims=True)
    tg = tg.astype(np.float32)
    net = PP.ProposalNet(NPRE, NSEED, max_obj=8, params=th.astype(np.float32))
    loss = net.loss_grad(clouds, tg).cpu().numpy().astype(np.float64)
    g_gpu = net.grad.cpu().numpy().astype(np.float64)
    g_or = np.zeros_like(th)
    for i, c in enumerate(clouds):
        o, I = OP.forward(th, c.astype(np.float64), NPRE, NSEED, bf=True)
        L, do = OP.loss(o, I["com"], tg[i].astype(np.float64), NPRE, NSEED)
        assert loss[i] == pytest.approx(L, rel=1e-4, abs=1e-6)
        g_or += OP.backward(th, I, do, NPRE, NSEED, bf=True) / len(clouds)
    sizes_l = [int(np.prod(s)) for s in OP.layer_shapes(NPRE, NSEED)]
    o = 0
    for k, n in enumerate(sizes_l):
        a, b = g_gpu[o:o + n], g_or[o:o + n]
        scale = max(np.abs(b).max(), 1e-12)
        err = np.abs(a - b).max()
        say(f"[proposal] grad block {k}: max err {err:.3g} scale {scale:.3g}")
        assert err <= 2e-3 * scale, k
        o += n
    # repeated calls are bitwise identical (fixed-order sums)
    net.loss_grad(clouds, tg)
    assert np.array_equal(net.grad.cpu().numpy(), g_gpu.astype(np.float32))


def test_adam_step_matches_closed_form():
    torch = _gpu()
    rng = np.random.default_rng(13)
    net = PP.ProposalNet(1, 1, max_obj=1)
    n = net.n
    p0 = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m0 = rng.standard_normal(n).astype(np.float32) * 0.1
    v0 = np.abs(rng.standard_normal(n)).astype(np.float32) * 0.1
    net.params.copy_(torch.as_tensor(p0))
    net.grad.copy_(torch.as_tensor(g))
    net.m.copy_(torch.as_tensor(m0))
    net.v.copy_(torch.as_tensor(v0))
    net.step_count = 2
    net.adam(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8)
    b1, b2, t = 0.9, 0.99, 3
    m = b1 * m0.astype(np.float64) + (1 - b1) * g
    v = b2 * v0.astype(np.float64) + (1 - b2) * g.astype(np.float64) ** 2
    p = p0 - 1e-2 * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + 1e-8)
    assert np.allclose(net.params.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_training_on_solver_grasps_beats_no_network():
    """Trained on grasps the solver itself finds, the network's seeds are
    closer (set loss on held-out objects) to plain AS-ICP's grasps than the
    untrained network's Fibonacci seeds, and a short seeded solve returns
    collision-free grasps."""
    torch = _gpu()
    from paper_2412_08346_amd import synth
    train_objs = synth.random_objects(128, 1024, 2048, seed=31)
    eval_objs = synth.random_objects(16, 1024, 2048, seed=32)
    tg = []
    for b in range(0, 128, 64):
        pb, r, _ = PP.solve(train_objs[b:b + 64], K=64, k_max=60, warm=False)
        tg.append(PP.targets_from(pb, r, 8))
    tg = np.concatenate(tg)
    pb_e, r_e, _ = PP.solve(eval_objs, K=64, k_max=60, warm=False)
    tg_e = PP.targets_from(pb_e, r_e, 8)
    net = PP.ProposalNet(3, 16, max_obj=64, seed=3)
    before = float(net.loss_grad(eval_objs, tg_e).mean().item())
    PP.train(net, train_objs, tg, steps=600, batch=64, lr=1e-3, seed=3)
    after = float(net.loss_grad(eval_objs, tg_e).mean().item())
    say(f"[proposal] held-out set loss: untrained {before:.3f}, trained {after:.3f}")
    assert after < 0.7 * before
    # 3 cm retraction along the approach axis, the pipeline's default.  A
    # sanity floor only: with this little training the count moves with the
    # FP32 rounding of the solves that make the targets (7 to 12 of 16
    # measured); the gain over the method without the network is tested at a
    # useful training size below
    seeds, _ = net.forward(eval_objs, retract=0.03)
    pb_l, r_l, _ = PP.solve(eval_objs, K=16, k_max=30, theta0=seeds.cpu().numpy(), warm=False)
    best = PP.best_per_object(pb_l, r_l)
    say(f"[proposal] seeded solve: {int(np.isfinite(best).sum())} of 16 objects with a collision-free grasp")
    assert np.isfinite(best).sum() >= 4


def test_learned_seeds_reach_plain_cost_more_often_than_no_network():
    """What the trained network gains over the method without it.  The
    network is trained on the GPU by the library's kernels on grasps plain
    AS-ICP finds (384 random objects of 2k-8k points, 1500 Adam steps); on
    64 held-out objects its seeds (32 per preshape, 50 SGD-ICP iterations:
    16x fewer particle-iterations than plain's 256 x 100) must end within 2 %
    of plain's best collision-free cost on more objects than the same budget
    from Fibonacci seeds, by at least 8 objects (0.125), and the median
    object must reach plain's cost."""
    _gpu()
    r = PP.run_learned(n_train=384, n_eval=64, steps=1500, m_hi=8192, log=lambda m: say(f"[proposal] {m}"))
    l, f = r["learned"], r["fibonacci_same_budget"]
    ratio = (r["plain"]["particles_per_preshape"] * r["plain"]["iterations"]) / (
        l["particles_per_preshape"] * l["iterations"])
    say(f"[proposal] within 2 % of plain: learned {l['matched_fraction']:.3f} (median cost ratio "
        f"{l['median_cost_ratio']:.3f}), no network {f['matched_fraction']:.3f} (median "
        f"{f['median_cost_ratio']:.3f}); {ratio:.0f}x fewer particle-iterations")
    assert ratio >= 5
    assert l["matched_fraction"] >= f["matched_fraction"] + 0.125
    assert l["median_cost_ratio"] <= 1.0
