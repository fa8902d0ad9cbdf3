"""Learned grasp proposal: seeds for the AS-ICP iteration from a point-cloud
encoder (kernels in csrc/k_proposal.hip, C calls asicp_pn_*).

The paper points to learned priors and data-driven seeding as the way to
need fewer initialisations (Sec. V, the ablation; Sec. VII).  Here a max-pooled
point encoder is trained on grasps the solver itself finds: each training
object is solved with plain Fibonacci AS-ICP, and the lowest-cost
collision-free final poses per preshape are the targets of a set loss.  The
trained network then seeds a short AS-ICP run with few particles; plain
AS-ICP stays the fallback and the judge.

Everything computed runs in the library's kernels; torch only holds device
memory and supplies the stream.
"""
from __future__ import annotations

import math

import numpy as np

from . import (Solver, asicp_pn_adam, asicp_pn_forward, asicp_pn_loss_grad, asicp_pn_param_count,
               asicp_pn_workspace_bytes, synth)

H1, H2, H3, HH = 64, 128, 256, 256


def layer_shapes(n_pre: int, n_seed: int):
    O = n_pre * n_seed * 7
    return [(H1, 3), (H1,), (H2, H1), (H2,), (H3, H2), (H3,), (HH, H3), (HH,), (HH, HH), (HH,), (O, HH), (O,)]


def init_params(n_pre: int, n_seed: int, rng: np.random.Generator, radius: float = 1.5) -> np.ndarray:
    """He-style random weights; the output bias places seed s of every preshape
    on a Fibonacci sphere `radius` units (0.1 m each) from the object's mean
    point, gripper +z looking at it, so an untrained network already proposes
    the plain method's initial poses."""
    ps = []
    for s in layer_shapes(n_pre, n_seed):
        ps.append(rng.standard_normal(s) * math.sqrt(2.0 / s[1]) if len(s) == 2 else np.zeros(s))
    ps[-2] *= 0.01
    fib = synth.fibonacci_poses(n_seed, np.zeros(3), np.zeros(3), radius * 0.1).astype(np.float64)
    b = np.zeros((n_pre, n_seed, 7))
    b[:, :, :3] = fib[:3].T / 0.1
    b[:, :, 3:] = fib[3:].T
    ps[-1] = b.ravel()
    return np.concatenate([p.ravel() for p in ps]).astype(np.float32)


class ProposalNet:
    """Parameters, Adam moments and a workspace on the device."""

    def __init__(self, n_pre: int, n_seed: int, max_obj: int, params=None, seed: int = 0, device="cuda"):
        import torch
        self.torch = torch
        self.n_pre, self.n_seed, self.max_obj = n_pre, n_seed, max_obj
        self.n = asicp_pn_param_count(n_pre, n_seed)
        p0 = init_params(n_pre, n_seed, np.random.default_rng(seed)) if params is None else np.asarray(params, np.float32)
        assert p0.size == self.n
        self.params = torch.as_tensor(p0).to(device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.ws_bytes = asicp_pn_workspace_bytes(max_obj, n_pre, n_seed)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.step_count = 0
        self.device = device

    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def _clouds(self, clouds):
        torch = self.torch
        off = np.cumsum([0] + [len(c) for c in clouds]).astype(np.int32)
        allp = np.concatenate(clouds).astype(np.float32)
        xyz = [torch.as_tensor(np.ascontiguousarray(allp[:, a])).to(self.device) for a in range(3)]
        return off, xyz

    def forward(self, clouds, retract: float = 0.0):
        """Seeds (7, n_obj * n_pre * n_seed) float32 device tensor, solver
        order, backed off `retract` metres along each approach axis; and the
        raw outputs."""
        torch = self.torch
        assert len(clouds) <= self.max_obj
        off, xyz = self._clouds(clouds)
        n_obj = len(clouds)
        seeds = torch.empty(7, n_obj * self.n_pre * self.n_seed, dtype=torch.float32, device=self.device)
        raw = torch.empty(n_obj, self.n_pre * self.n_seed * 7, dtype=torch.float32, device=self.device)
        asicp_pn_forward(self.params.data_ptr(), self.n_pre, self.n_seed, n_obj, off.ctypes.data,
                         xyz[0].data_ptr(), xyz[1].data_ptr(), xyz[2].data_ptr(), retract, seeds.data_ptr(),
                         raw.data_ptr(), self.ws_ptr, self.ws_bytes, self._stream())
        return seeds, raw

    def loss_grad(self, clouds, targets):
        """Mean loss over the objects; fills self.grad.  targets: (n_obj,
        n_pre, T, 7) float32 (device tensor or array)."""
        torch = self.torch
        off, xyz = self._clouds(clouds)
        n_obj = len(clouds)
        tg = torch.as_tensor(np.asarray(targets, np.float32) if not isinstance(targets, torch.Tensor) else targets)
        tg = tg.to(self.device).float().contiguous()
        loss = torch.empty(n_obj, dtype=torch.float32, device=self.device)
        asicp_pn_loss_grad(self.params.data_ptr(), self.n_pre, self.n_seed, n_obj, off.ctypes.data,
                           xyz[0].data_ptr(), xyz[1].data_ptr(), xyz[2].data_ptr(), tg.data_ptr(),
                           tg.shape[2], loss.data_ptr(), self.grad.data_ptr(), self.ws_ptr, self.ws_bytes,
                           self._stream())
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        asicp_pn_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.grad.data_ptr(),
                      self.n, lr, beta1, beta2, eps, self.step_count, self._stream())


# ---------------------------------------------------------------------------
# self-supervised data, training and evaluation

def solve(objs, K: int, k_max: int, theta0=None, T0: float = 1.0, T1: float = 0.01, launch=None,
          warm: bool = True, k_stein: int | None = None):
    """Plain (Fibonacci) or seeded AS-ICP on the objects with the paper-scale
    preshapes; returns (problem, per-particle result, wall seconds of the
    timed solve).  With warm, one untimed solve runs first."""
    import time
    import torch
    pb = synth.workload_objects(objs, K, k_max, theta0=theta0)
    st = synth.Settings(k_max=k_max, k_stein=k_max if k_stein is None else k_stein, T0=T0, T1=T1)
    s = Solver(pb, st)
    if launch is not None:
        s.set_launch(**launch)
    if warm:
        s.solve()
        s.result(per_particle=False)
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve()
    r = s.result(per_particle=True)
    wall = time.perf_counter() - t0
    s.close()
    return pb, r, wall


def targets_from(pb, r, n_targets: int) -> np.ndarray:
    """Per (object, preshape): the n_targets lowest-cost final poses among the
    collision-free particles (all particles if fewer are free), repeated to
    fill; returns (n_obj, n_pre, n_targets, 7) float32."""
    K, P = pb.K, pb.n_pre
    th = np.asarray(r["theta"], np.float64).T  # (Ktot, 7)
    cost = np.asarray(r["cost"], np.float64)
    ncol = np.asarray(r["ncol"])
    out = np.zeros((pb.n_obj, P, n_targets, 7), np.float32)
    for o in range(pb.n_obj):
        for p in range(P):
            sl = slice((o * P + p) * K, (o * P + p + 1) * K)
            c, nc = cost[sl], ncol[sl]
            key = np.where(nc == 0, c, c + 1e9)  # collision-free first, then cost
            order = np.argsort(key, kind="stable")
            sel = [order[i % len(order)] for i in range(n_targets)]
            out[o, p] = th[sl][sel]
    return out


def _quat_rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _quat_mul(a, b):
    """Hamilton products a (x) b[i] for one quaternion a and rows b."""
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def rotate_sample(cloud, targets, rng):
    """The same random rotation about the cloud's mean point applied to the
    cloud and to its target grasps (a valid training sample for the rotated
    object): data augmentation for an encoder that is not rotation
    invariant."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    Rm = _quat_rot(q)
    c = np.asarray(cloud, np.float64)
    com = c.mean(0)
    tg = np.asarray(targets, np.float64).copy()
    sh = tg.shape
    flat = tg.reshape(-1, 7)
    flat[:, :3] = (flat[:, :3] - com) @ Rm.T + com
    qq = _quat_mul(q, flat[:, 3:])
    qq[qq[:, 0] < 0] *= -1
    flat[:, 3:] = qq
    return (((c - com) @ Rm.T + com).astype(np.float32), flat.reshape(sh).astype(np.float32))


def train(net: ProposalNet, clouds, targets, steps: int, batch: int, lr: float, seed: int = 0,
          augment: bool = True, log_every: int = 0):
    """Adam on random batches of objects, each object and its targets turned
    by a random rotation when `augment`; returns (step, mean loss) pairs."""
    rng = np.random.default_rng(seed)
    n = len(clouds)
    losses = []
    for it in range(steps):
        idx = rng.choice(n, size=min(batch, n), replace=False)
        cl, tg = [clouds[i] for i in idx], targets[idx]
        if augment:
            pairs = [rotate_sample(c, t, rng) for c, t in zip(cl, tg)]
            cl, tg = [p[0] for p in pairs], np.stack([p[1] for p in pairs])
        loss = net.loss_grad(cl, tg)
        net.adam(lr=lr)
        if log_every and (it % log_every == 0 or it == steps - 1):
            losses.append((it, float(loss.mean().item())))
    return losses


def best_per_object(pb, r):
    """Per object: the lowest cost among collision-free particles (inf if none)."""
    per = pb.n_pre * pb.K
    cost = np.asarray(r["cost"], np.float64)
    free = np.asarray(r["ncol"]) == 0
    out = np.full(pb.n_obj, np.inf)
    for o in range(pb.n_obj):
        sl = slice(o * per, (o + 1) * per)
        c = np.where(free[sl], cost[sl], np.inf)
        out[o] = c.min()
    return out


def run_learned(n_train: int = 1024, n_eval: int = 64, steps: int = 3000, n_seed: int = 32,
                seeded_iters: int = 50, seeded_k_stein: int = 0, retract: float = 0.03,
                m_lo: int = 2048, m_hi: int = 16384,
                plain_k: int = 256, plain_iters: int = 100, n_targets: int = 16, seed: int = 0, log=None):
    """Self-supervised pipeline and the comparison at matched final cost.

    1. Training data: n_train random objects solved by plain AS-ICP (128
       Fibonacci particles per preshape, 100 iterations); targets are the
       lowest-cost collision-free final poses.
    2. Training: Adam with rotation augmentation.
    3. Held-out objects: plain AS-ICP (plain_k particles x plain_iters
       iterations per preshape) against learned seeds (n_seed x
       seeded_iters, backed off `retract`) and against the same small budget
       from Fibonacci seeds (no network), and the two seed sets together in
       one run (2 n_seed per preshape).  The seeded runs refine with the
       first seeded_k_stein iterations Stein and the rest SGD-ICP (eq. 3,
       with the convergence freeze): good seeds need local refinement, not
       exploration.  Per object the lowest collision-free cost; a run is
       matched when it is within 2 % of plain's.
    Returns a dict of the measured numbers."""
    import time
    import torch
    say = log or (lambda *a: None)
    t_all = time.perf_counter()
    train_objs = synth.random_objects(n_train, m_lo, m_hi, seed=1000 + seed)
    targets = []
    for b in range(0, n_train, 64):
        pb, r, _ = solve(train_objs[b:b + 64], K=128, k_max=100, warm=False)
        targets.append(targets_from(pb, r, n_targets))
    targets = np.concatenate(targets)
    t_data = time.perf_counter() - t_all
    say(f"training data: {n_train} objects in {t_data:.1f} s")
    net = ProposalNet(3, n_seed, max_obj=max(64, n_eval), seed=seed)
    eval_objs = synth.random_objects(n_eval, m_lo, m_hi, seed=2000 + seed)
    pb_p, r_p, w_p = solve(eval_objs, K=plain_k, k_max=plain_iters)
    best_p = best_per_object(pb_p, r_p)
    eval_tg = targets_from(pb_p, r_p, n_targets)
    held0 = float(net.loss_grad(eval_objs, eval_tg).mean().item())
    t0 = time.perf_counter()
    losses = train(net, train_objs, targets, steps=steps, batch=64, lr=1e-3, seed=seed, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    held = float(net.loss_grad(eval_objs, eval_tg).mean().item())
    say(f"training: {steps} steps in {t_train:.1f} s, held-out loss {held0:.3f} -> {held:.3f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seeds, _ = net.forward(eval_objs, retract=retract)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    iters_list = seeded_iters if isinstance(seeded_iters, (list, tuple)) else [seeded_iters]
    extra = {}
    for it in iters_list[1:]:
        pb_x, r_x, w_x = solve(eval_objs, K=n_seed, k_max=it, theta0=seeds.cpu().numpy(), k_stein=seeded_k_stein)
        rx = best_per_object(pb_x, r_x) / best_p
        extra[f"learned_{it}_iterations"] = {"solve_s": w_x, "grasps_per_s": n_eval / (w_x + t_fwd),
                                             "median_cost_ratio": float(np.median(rx)),
                                             "matched_fraction": float(np.mean(rx <= 1.02))}
    seeded_iters = iters_list[0]
    pb_l, r_l, w_l = solve(eval_objs, K=n_seed, k_max=seeded_iters, theta0=seeds.cpu().numpy(),
                           k_stein=seeded_k_stein)
    best_l = best_per_object(pb_l, r_l)
    pb_f, r_f, w_f = solve(eval_objs, K=n_seed, k_max=seeded_iters, k_stein=seeded_k_stein)
    best_f = best_per_object(pb_f, r_f)
    # hybrid: each group starts from its learned seeds and its Fibonacci
    # particles together (twice the particles of either)
    G = pb_f.theta0.shape[1] // n_seed
    th_l = seeds.cpu().numpy().reshape(7, G, n_seed)
    th_f = np.asarray(pb_f.theta0, np.float32).reshape(7, G, n_seed)
    th_h = np.ascontiguousarray(np.concatenate([th_l, th_f], axis=2).reshape(7, G * 2 * n_seed))
    pb_h, r_h, w_h = solve(eval_objs, K=2 * n_seed, k_max=seeded_iters, theta0=th_h, k_stein=seeded_k_stein)
    best_h = best_per_object(pb_h, r_h)

    def cmp(best):
        ratio = best / best_p
        return {"median_cost_ratio": float(np.median(ratio)), "matched_fraction": float(np.mean(ratio <= 1.02)),
                "collision_free_objects": int(np.isfinite(best).sum())}

    P = pb_p.n_pre
    out = {
        "objects": n_eval, "train_objects": n_train, "train_steps": steps,
        "held_out_loss_untrained": held0, "held_out_loss_trained": held,
        "train_loss_log": losses, "data_s": t_data, "train_s": t_train,
        "plain": {"particles_per_preshape": plain_k, "iterations": plain_iters, "solve_s": w_p,
                  "grasps_per_s": n_eval / w_p,
                  "particle_iters_per_s": n_eval * P * plain_k * plain_iters / w_p,
                  "collision_free_objects": int(np.isfinite(best_p).sum())},
        "learned": {"particles_per_preshape": n_seed, "iterations": seeded_iters, "stein_iterations": seeded_k_stein,
                    "retract_m": retract,
                    "solve_s": w_l, "forward_s": t_fwd, "grasps_per_s": n_eval / (w_l + t_fwd),
                    "particle_iters_per_s": n_eval * P * n_seed * seeded_iters / w_l, **cmp(best_l)},
        "fibonacci_same_budget": {"particles_per_preshape": n_seed, "iterations": seeded_iters,
                                  "stein_iterations": seeded_k_stein, "solve_s": w_f,
                                  "grasps_per_s": n_eval / w_f, **cmp(best_f)},
        "learned_plus_fibonacci": {"particles_per_preshape": 2 * n_seed, "iterations": seeded_iters,
                                   "stein_iterations": seeded_k_stein, "solve_s": w_h,
                                   "grasps_per_s": n_eval / (w_h + t_fwd), **cmp(best_h)},
        **extra,
    }
    return out
