"""GPU (HIP, gfx950) vs FP64 oracle parity, through the C ABI.

Teacher forcing: the oracle runs its own trajectory; its pose at iteration k,
rounded to float32, is the input of one step on both sides.  No input and no
expected value comes from the HIP path.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2412_08346_amd import synth
import parity_util as pu

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_08346_amd as A
    return A, torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def col_scales(pb, theta_soa, or_rev):
    """Scales of the collision terms: mean |e| and mean |R s| |e| over the
    colliding points (e = s' - c), and bounds of the FP32 rounding the
    kernel's arithmetic allows in (col_cost, g_t, g_w).  The kernel forms
    e = s - R^T (c - t) in the gripper frame; each component then carries an
    error of a few units of 2^-24 times |c - t| + |s| (a subtraction, a
    three-term dot product, a subtraction), taken here as
    delta = 16 * 2^-24 * (|c - t| + |s|) per component.  Near convergence a
    colliding point sits on its contact point (|e| of micrometres), where
    this absolute error dominates any relative tolerance."""
    S = pb.S.astype(np.float64)
    Cc = pb.C.astype(np.float64)
    th = np.asarray(theta_soa, np.float64)
    n_p = th.shape[1]
    st, sw = np.zeros(n_p), np.zeros(n_p)
    xc, xt, xw = np.zeros(n_p), np.zeros(n_p), np.zeros(n_p)
    eps = 16 * 2.0 ** -24
    for i in range(n_p):
        g = i // pb.K
        o, p = g // pb.n_pre, g % pb.n_pre
        c0, c1 = pb.c_off[o], pb.c_off[o + 1]
        r = np.asarray(or_rev[i][: c1 - c0])
        sel = np.nonzero(r >= 0)[0]
        if len(sel) == 0:
            continue
        Rm = oracle.quat_to_rot(th[3:, i])
        s_loc = S[pb.s_off[p] + r[sel]]
        u = s_loc @ Rm.T
        e = u + th[:3, i] - Cc[c0 + sel]
        ne = np.linalg.norm(e, axis=1)
        ns = np.linalg.norm(s_loc, axis=1)
        st[i] = ne.mean()
        sw[i] = (ns * ne).mean()
        dv = math.sqrt(3) * eps * (np.linalg.norm(Cc[c0 + sel] - th[:3, i], axis=1) + ns)
        xc[i] = (2 * ne * dv + dv * dv).mean() / 2
        xt[i] = dv.mean()
        xw[i] = (ns * dv).mean()
    return st, sw, xc, xt, xw


def gate_excusal_bounds(pb, theta, gpu_rev, r, rows):
    """Bounds on what excused gate decisions (points with |phi| < 1e-6 m that
    collide on one side only) move in the collision terms of particles
    `rows`.  With D the points decided differently, N_gpu >= n the GPU's
    colliding count and e_c = s'(c) - c the residual of a point against its
    nearest transformed contact point:
      g_gpu - g_or = ((N_or - N_gpu) g_or +- sum_D e_c) / N_gpu,
    so |g_gpu - g_or| <= (|D| |g_or| + sum_D |e_c|) / n, and likewise for the
    moment (R s) x e_c and for 1/2 L_col with |e_c|^2 / 2.  A particle whose
    colliding set is empty on one side switches between the contact and the
    collision gradient: it has no bound (inf)."""
    S = pb.S.astype(np.float64)
    Cc = pb.C.astype(np.float64)
    th = np.asarray(theta, np.float64)
    n = th.shape[1]
    bc, bt, bw = np.zeros(n), np.zeros(n), np.zeros(n)
    for i in np.nonzero(rows)[0]:
        gi = i // pb.K
        o, p = gi // pb.n_pre, gi % pb.n_pre
        c0, c1 = pb.c_off[o], pb.c_off[o + 1]
        n0, n1 = pb.s_off[p], pb.s_off[p + 1]
        gg = np.asarray(gpu_rev[i][: c1 - c0]) >= 0
        go = np.asarray(r["gate"][i][: c1 - c0]) > 0
        diff = np.nonzero(gg != go)[0]
        nmin = min(int(gg.sum()), int(go.sum()))
        if nmin == 0:
            bc[i] = bt[i] = bw[i] = np.inf
            continue
        Rm = oracle.quat_to_rot(th[3:, i])
        u_all = S[n0:n1] @ Rm.T
        c = Cc[c0 + diff]
        d2 = ((c[:, None, :] - (u_all + th[:3, i])[None, :, :]) ** 2).sum(-1)
        nn = d2.argmin(1)
        e = u_all[nn] + th[:3, i] - c
        mom = np.cross(u_all[nn], e)
        gcol = np.asarray(r["g_col"][i])
        bt[i] = (np.abs(e).max(1).sum() + len(diff) * np.abs(gcol[:3]).max()) / nmin
        bw[i] = (np.abs(mom).max(1).sum() + len(diff) * np.abs(gcol[3:]).max()) / nmin
        bc[i] = (0.5 * (e ** 2).sum() + len(diff) * r["col_cost"][i]) / nmin
    return bc, bt, bw


def stein_scales(pb, st, k, th64, r, setup, gs_t, gs_w, xb_t, xb_w):
    """Scales of the Stein direction phi of eqs. (8)-(10), per particle i, with
    the kernel weights of the configured mode (product: k_t k_r on the driving
    terms and the translation repulsion, k_t sign(q_i.q_j) on the rotation
    repulsion; block: k_t, k_t, |q_i.q_j| and sign(q_i.q_j)):
    - ph_t, ph_w: mean over j of |weight| times the magnitude of summand j,
      the gradient's magnitude taken as max(|g_j|, gs_j), the scale its own
      parity tolerance uses, so that the gradients' allowed rounding is
      carried into phi;
    - ex_t, ex_w: the same weights applied to xb (what excused ties may move
      in g_j);
    - fq_w: the FP32 rounding floor of the rotation repulsion.  Each
      component of vec(q_i (x) conj q_j) is a sum of four products of
      unit-bounded numbers, so its FP32 error is a few units of 2^-24 however
      small the result (nearly equal rotations cancel); 8 * 2^-24 is used.
    r is the oracle's step record at th64."""
    n = pb.k_tot
    ph_t, ph_w, ex_t, ex_w, fq_w = (np.zeros(n) for _ in range(5))
    gam, tau = oracle.schedule(st, k)
    # driving gradient: the cost gradient minus the log-prior gradient
    gdrive = r["g_fin"].copy()
    if getattr(pb, "prior", None) is not None:
        for i in range(n):
            gdrive[i] -= oracle.log_prior(pb.prior[i // pb.K].astype(np.float64), th64[:, i])[1]
    G_t = np.maximum(np.abs(gdrive[:, :3]).max(1), gs_t)
    G_w = np.maximum(np.abs(gdrive[:, 3:]).max(1), gs_w)
    block = st.kernel_mode == synth.KERNEL_BLOCK
    for gi in range(pb.n_obj * pb.n_pre):
        p = gi % pb.n_pre
        sl = slice(gi * pb.K, (gi + 1) * pb.K)
        t = th64[:3, sl].T
        q = th64[3:, sl].T
        d = t[:, None, :] - t[None, :, :]
        kt = np.exp(-(d ** 2).sum(-1) / r["h"][gi])
        dot = q @ q.T
        kr = np.abs(dot)
        # vector part of q_i (x) conj(q_j): w_j v_i - w_i v_j - v_i x v_j
        vec = (q[None, :, :1] * q[:, None, 1:] - q[:, None, :1] * q[None, :, 1:]
               - np.cross(q[:, None, 1:], q[None, :, 1:]))
        if block:
            wdt, wrt, wdw, wrw = kt, kt, kr, np.ones_like(kt)
        else:
            wdt = wrt = wdw = kt * kr
            wrw = kt
        a_t, a_w = setup["a_t"][p], setup["a_w"][p]
        ph_t[sl] = (wdt * gam * a_t * G_t[sl][None, :] + tau * wrt * np.abs(d).max(-1)).mean(1)
        ph_w[sl] = (wdw * gam * a_w * G_w[sl][None, :] + tau * wrw * 0.5 * np.abs(vec).max(-1)).mean(1)
        ex_t[sl] = (wdt * gam * a_t * xb_t[sl][None, :]).mean(1)
        ex_w[sl] = (wdw * gam * a_w * xb_w[sl][None, :]).mean(1)
        fq_w[sl] = (tau * wrw * 0.5 * 8 * 2.0 ** -24).mean(1)
    return ph_t, ph_w, ex_t, ex_w, fq_w


def gpu_step(pb, st, theta, k, prev_cost=None, converged=None, label="", debug=True):
    """One step on the GPU from float32 `theta` (7, Ktot), with the per-point
    NN and gate records."""
    A, torch = _gpu()
    theta = np.ascontiguousarray(theta, np.float32)
    say(f"[parity] {label} k={k} Ktot={pb.k_tot} n_obj={pb.n_obj} n_pre={pb.n_pre}")
    pc32 = None if prev_cost is None else np.asarray(prev_cost, np.float32)
    sol = A.Solver(pb, st, debug=debug, theta0=theta, k_start=k, prev_cost=pc32, converged=converged)
    sol.step(1)
    g = sol.result()
    sol.close()
    return g


def compare(pb, st, theta, k, g, prev_cost=None, converged=None):
    """The GPU's step record `g` (with debug records) against the oracle's
    step from the same float32 poses, on problem `pb`.  Returns stats."""
    theta = np.ascontiguousarray(theta, np.float32)
    pc32 = None if prev_cost is None else np.asarray(prev_cost, np.float32)
    o = oracle.Oracle(pb, st)
    r = o.step(k, theta, prev_cost=None if pc32 is None else pc32.astype(np.float64),
               converged=converged, full=True)
    setup = o.setup()
    ties = pu.check_nn(pb, theta, g["nn_idx"], r["nn_idx"])
    excused = pu.check_gate(pb, g["rev_idx"], r["gate"], r["phi_c"])
    rties = pu.check_rev(pb, theta, g["rev_idx"], r["rev_idx"])
    mcs = np.diff(pb.c_off)
    obj_of = (np.arange(pb.k_tot) // pb.K) // pb.n_pre
    gate_gpu = np.array([(g["rev_idx"][i, :mcs[obj_of[i]]] >= 0).sum() for i in range(pb.k_tot)])
    gate_or = r["gate"].astype(np.int64).sum(1)
    gate_diff = gate_gpu != gate_or  # only where a decision within 1e-6 m of phi = 0 was excused
    assert np.array_equal(g["ncol"], gate_gpu), "ncol disagrees with the GPU's own gate record"
    assert np.array_equal(g["ncol"][~gate_diff], r["ncol"][~gate_diff]), "collision counts differ"
    assert np.abs(gate_gpu - gate_or).sum() <= excused
    s_t, s_w = pu.scales(pb, theta, r["nn_idx"], st.lam, setup)
    pu.close(g["cost"], r["cost"], r["cost"], what="cost")
    b_t, b_w = pu.tie_bounds(pb, theta, g["nn_idx"], r["nn_idx"])
    pu.close(g["grad_ct"][:3].T, r["g_ct"][:, :3], s_t[:, None], what="g_t", extra=b_t[:, None])
    pu.close(g["grad_ct"][3:].T, r["g_ct"][:, 3:], s_w[:, None], what="g_w", extra=b_w[:, None])
    gx_c, gx_t, gx_w = gate_excusal_bounds(pb, theta, g["rev_idx"], r, gate_diff)
    switched = ~np.isfinite(gx_t)  # contact <-> collision gradient: no bound
    both = (g["ncol"] > 0) & (r["ncol"] > 0)
    rb_t, rb_w = pu.rev_tie_bounds(pb, theta, g["rev_idx"], r["rev_idx"])
    c_t, c_w, x_c, x_t, x_w = col_scales(pb, theta, r["rev_idx"])
    if both.any():
        pu.close(g["col_cost"][both], r["col_cost"][both], r["col_cost"][both], what="col_cost",
                 extra=rb_t[both] * 0.05 + x_c[both] + gx_c[both])
        pu.close(g["grad_col"][:3].T[both], r["g_col"][both, :3], c_t[both, None], what="gcol_t",
                 extra=(rb_t + x_t + gx_t)[both, None])
        pu.close(g["grad_col"][3:].T[both], r["g_col"][both, 3:], c_w[both, None], what="gcol_w",
                 extra=(rb_w + x_w + gx_w)[both, None])
    # the gradient the update uses: its tolerance scale, and what excused ties,
    # excused gate decisions and the collision terms' FP32 floor may move in it
    colliding = r["ncol"] > 0
    gs_t = np.where(colliding, c_t, s_t)
    gs_w = np.where(colliding, c_w, s_w)
    xb_t = np.where(colliding, rb_t + x_t + np.where(switched, 0.0, gx_t), b_t)
    xb_w = np.where(colliding, rb_w + x_w + np.where(switched, 0.0, gx_w), b_w)
    # particles whose update is compared: all, except the Stein groups (phi
    # mixes the group's gradients) or, in the SGD phase, the particles where
    # an excused gate decision switched a particle between the contact and
    # the collision gradient
    svgd = k < st.k_stein
    grp = np.arange(pb.k_tot) // pb.K
    if svgd:
        sel = ~np.isin(grp, np.unique(grp[switched]))
    else:
        sel = ~switched
    th64 = theta.astype(np.float64)
    if svgd:
        pu.close(g["h"], r["h"], r["h"], what="h")
        ph_t, ph_w, ex_t, ex_w, fq_w = stein_scales(pb, st, k, th64, r, setup, gs_t, gs_w, xb_t, xb_w)
        pu.close(g["phi"][:3].T[sel], r["phi"][sel, :3], ph_t[sel, None], what="phi_t", extra=ex_t[sel, None])
        pu.close(g["phi"][3:].T[sel], r["phi"][sel, 3:], ph_w[sel, None], what="phi_w",
                 extra=(ex_w + fq_w)[sel, None])
        step_t, step_w = st.eta * ph_t, st.eta * ph_w
        ext_t, ext_w = st.eta * ex_t, st.eta * (ex_w + fq_w)
    else:
        p_of = (np.arange(pb.k_tot) // pb.K) % pb.n_pre
        step_t = st.eta * setup["a_t"][p_of] * np.maximum(np.abs(r["g_fin"][:, :3]).max(1), gs_t)
        step_w = st.eta * setup["a_w"][p_of] * np.maximum(np.abs(r["g_fin"][:, 3:]).max(1), gs_w)
        ext_t = st.eta * setup["a_t"][p_of] * xb_t
        ext_w = st.eta * setup["a_w"][p_of] * xb_w
        conv_or = r["converged"].astype(bool)
        conv_gpu = g["converged"].astype(bool)
        pcv = np.asarray(prev_cost if prev_cost is not None else np.full(pb.k_tot, -1.0), np.float64)
        near = np.abs(np.abs(r["cost"] - pcv) - st.conv_tol * pcv) <= 1e-3 * st.conv_tol * np.abs(pcv)
        bad = (conv_or != conv_gpu) & ~near & sel
        assert not bad.any(), f"converged flags differ for particles {np.nonzero(bad)[0][:8]}"
        sel &= conv_or == conv_gpu
    dt_err = np.abs(g["theta"][:3].astype(np.float64) - r["theta"][:3]).max(0)
    tol_t = 1e-4 * step_t + 2e-7 * np.maximum(np.abs(th64[:3]).max(0), 1e-2) + ext_t
    assert (dt_err[sel] <= tol_t[sel]).all(), f"translation update: worst {(dt_err / tol_t)[sel].max():.3g}x tol"
    ang = pu.angle_between(g["theta"][3:], r["theta"][3:])
    tol_w = 1e-4 * step_w + 2e-6 + ext_w
    assert (ang[sel] <= tol_w[sel]).all(), f"rotation update: worst {(ang / tol_w)[sel].max():.3g}x tol"
    assert g["status"] == 0
    return dict(ties=ties, gate_excused=excused, rev_ties=rties, ncol=int(g["ncol"].sum()),
                update_checked=int(sel.sum()), of=int(pb.k_tot))


def compare_step(pb, st, theta, k, prev_cost=None, converged=None, label=""):
    """One teacher-forced step from float32 `theta` (7, Ktot) on both sides."""
    g = gpu_step(pb, st, theta, k, prev_cost, converged, label=label)
    return compare(pb, st, theta, k, g, prev_cost, converged)


def oracle_trajectory(pb, st, ks):
    o = oracle.Oracle(pb, st)
    th = pb.theta0.astype(np.float64)
    pc, cv = None, None
    snaps = {}
    for k in range(max(ks) + 1):
        if k in ks:
            snaps[k] = (th.astype(np.float32), None if pc is None else pc.copy(),
                        None if cv is None else cv.copy())
        r = o.step(k, th, pc, cv)
        th, pc, cv = r["theta"], r["prev_cost"], r["converged"]
    return snaps


# ---------------------------------------------------------------------------

def test_small_first_step():
    pb, st = synth.workload_small()
    out = compare_step(pb, st, pb.theta0, 0, label="small first step")
    say("[parity] small first step", out)


@pytest.mark.parametrize("K", [2, 128, 160, 255, 256, 257, 300, 512, 1024])
def test_bandwidth_on_both_sides_of_one_workgroup(K):
    """The median bandwidth (eq. 9) comes from one workgroup per group up to
    K = 256 (of 256 threads up to K = 128, 512 up to K = 181, 1024 above) and
    from the sliced four-launch select above, up to the largest group the
    interface accepts (K = 1024); all must give the oracle's lower median.
    Checked on the first step and one later step."""
    pb, st = synth.workload_small(K=K)
    out = compare_step(pb, st, pb.theta0, 0, label=f"bandwidth K={K}")
    say(f"[parity] bandwidth K={K}", out)
    th, pc, cv = oracle_trajectory(pb, st, [3])[3]
    compare_step(pb, st, th, 3, pc, cv, label=f"bandwidth K={K} k=3")


def test_exact_ties_give_one_valid_nearest_point_for_every_launch():
    """A mirror-symmetric object seen from its mirror plane: every query's two
    nearest points (a point and its mirror image, 1024 indices apart in the
    input) have bit-identical squared distances, in FP32 as
    in FP64, so eq. (1) has two minimisers.  The oracle takes the lowest
    original index (the first copy); the GPU takes the lowest index of the
    prepared (k-d ordered) cloud, which is the other copy as often as not.
    Both are valid: the GPU's point must lie at exactly the oracle's minimal
    distance, and every launch choice, pruned or not, must return the same
    index whatever order it visits the chunks in."""
    A, torch = _gpu()
    rng = np.random.default_rng(5)
    half = synth.ellipsoid(1024, (0.04, 0.03, 0.02), rng)
    half[:, 0] = np.abs(half[:, 0]) + 1e-3  # no point on the plane itself
    obj = np.concatenate([half, half * np.array([-1.0, 1.0, 1.0], np.float32)]).astype(np.float32)
    S = synth.gripper_contact_cloud(0.06, 512, np.random.default_rng(2))
    S[:, 0] = 0.0  # the contact points lie in the mirror plane ...
    grid = synth.gripper_sdf_grid(0.06, 64, 0.002)
    K = 8
    pb = synth._assemble([obj], [S], [grid], K, [0.10])
    th = np.zeros((7, K), np.float32)
    th[1] = rng.uniform(-0.03, 0.03, K)
    th[2] = rng.uniform(-0.03, 0.03, K)
    th[3] = 1.0  # ... and stay there: identity rotation, no x translation
    pb.theta0 = th
    st = synth.Settings(k_max=3, k_stein=3)
    r = oracle.Oracle(pb, st).step(0, th.astype(np.float64), full=True)
    n = len(S)
    ref = np.asarray(r["nn_idx"])[:, :n]
    assert (ref < len(half)).all(), "the oracle must pick the first copy"
    sp = S.astype(np.float64)[None, :, :] + th[:3].T.astype(np.float64)[:, None, :]  # (K, n, 3)
    R = obj.astype(np.float64)
    d_ref = ((sp - R[ref]) ** 2).sum(-1)
    first = None
    for prune in (True, False):
        for v in range(A.ASICP_LAUNCH_CHOICES):
            ch = A.launch_choice(v)
            if not prune and (ch["fine"] or ch["chunk_points"] == 64):
                continue  # the full scan has neither test
            sol = A.Solver(pb, st, debug=True, theta0=th, prune=prune)
            sol.set_launch(**ch)
            sol.step(1)
            g = sol.result()
            sol.close()
            got = np.asarray(g["nn_idx"])[:, :n]
            assert ((got >= 0) & (got < len(obj))).all()
            d_got = ((sp - R[got]) ** 2).sum(-1)
            mirror = int((got != ref).sum())
            say(f"[ties] prune={prune} launch={ch}: other copy for {mirror} of {got.size}")
            assert np.array_equal(d_got, d_ref), "not a nearest point"
            if first is None:
                first = got
            assert np.array_equal(got, first), "launch choices disagree on a tie"


def test_small_teacher_forced_steps():
    pb, st = synth.workload_small()
    ks = [1, 5, 9, 14, 20, 29]
    snaps = oracle_trajectory(pb, st, ks)
    for k in ks:
        th, pc, cv = snaps[k]
        out = compare_step(pb, st, th, k, pc, cv, label="small teacher-forced")
        say("[parity] k", k, out)


def test_paper_preset_sgd_phase_with_collisions():
    pb, _ = synth.workload_small()
    st = synth.paper_settings(k_max=40, k_stein=15)
    ks = [0, 14, 15, 16, 20, 33]
    snaps = oracle_trajectory(pb, st, ks)
    total_col = 0
    for k in ks:
        th, pc, cv = snaps[k]
        out = compare_step(pb, st, th, k, pc, cv, label="paper preset")
        total_col += out["ncol"]
        say("[parity] paper preset k", k, out)
    assert total_col > 1000  # the collision branch was exercised


@pytest.mark.parametrize("init", ["quarter", "gmm"])
def test_tabletop_paper_setup(init):
    """Sec. VI-A set-up: collision cloud = object + table (C differs from R),
    10 preshapes of 96 points, 30 poses each, Table I schedule with the
    mini-batch."""
    pb, st = synth.workload_tabletop(init=init)
    ks = [0, 9, 15, 27, 39]
    snaps = oracle_trajectory(pb, st, ks)
    total_col = 0
    for k in ks:
        th, pc, cv = snaps[k]
        out = compare_step(pb, st, th, k, pc, cv, label=f"tabletop {init}")
        total_col += out["ncol"]
        say("[parity] tabletop", init, "k", k, out)
    assert total_col > 0


def test_priors_in_the_stein_update():
    """Gaussian translation and von Mises rotation priors (eq. 8) on the
    small workload and the tabletop set-up (Stein phase and SGD phase)."""
    pb, st = synth.workload_small()
    pb.prior = synth.grasp_prior(pb, sigma=0.05, kappa=2.0, sigma_n=0.01)
    ks = [0, 5, 17]
    snaps = oracle_trajectory(pb, st, ks)
    for k in ks:
        th, pc, cv = snaps[k]
        say("[parity] prior small k", k, compare_step(pb, st, th, k, pc, cv, label="prior small"))
    pb, st = synth.workload_tabletop()
    pb.prior = synth.grasp_prior(pb, sigma=0.03, kappa=5.0, sigma_n=0.005)
    ks = [1, 14, 20]
    snaps = oracle_trajectory(pb, st, ks)
    for k in ks:
        th, pc, cv = snaps[k]
        say("[parity] prior tabletop k", k, compare_step(pb, st, th, k, pc, cv, label="prior tabletop"))


def test_block_kernel_identity_preconditioner_fixed_bandwidth():
    pb, st = synth.workload_small()
    st.kernel_mode = synth.KERNEL_BLOCK
    st.precond = synth.PRECOND_IDENTITY
    st.eta = 0.5
    th = oracle_trajectory(pb, st, [4])[4]
    compare_step(pb, st, th[0], 4, th[1], th[2], label="block kernel")
    st.bw_mode, st.h_fixed = synth.BW_FIXED, 0.003
    compare_step(pb, st, th[0], 4, th[1], th[2], label="fixed bandwidth")


def pulled_in(pb, frac):
    """Poses moved a fraction of the way towards the object (collisions)."""
    th = pb.theta0.astype(np.float64).copy()
    com = pb.R.astype(np.float64).mean(0)
    th[:3] = th[:3] + frac * (com[:, None] - th[:3])
    return th.astype(np.float32)


def test_paper_scale_step_full_size():
    pb, st = synth.workload_paper_scale()
    out = compare_step(pb, st, pb.theta0, 0, label="paper scale theta0")
    say("[parity] paper scale theta0", out)
    out = compare_step(pb, st, pulled_in(pb, 0.75), 50, label="paper scale pulled in")
    say("[parity] paper scale pulled in", out)
    assert out["ncol"] > 0


def test_paper_scale_minibatch_steps():
    """Table I mini-batch at full size: both sides draw the same batch of the
    8192-point cloud (keyed permutation), so the nearest neighbours agree."""
    pb, _ = synth.workload_paper_scale()
    st = synth.paper_settings(k_max=100, k_stein=100, seed=21)
    for k in (1, 30):
        out = compare_step(pb, st, pb.theta0, k, label="paper scale mini-batch")
        say("[parity] paper scale mini-batch k", k, out)
    out = compare_step(pb, st, pulled_in(pb, 0.75), 45, label="paper scale mini-batch pulled in")
    say("[parity] paper scale mini-batch pulled in", out)


def test_pruned_and_brute_force_nn_agree():
    """Skipping chunks never changes a nearest distance: the pruned and the
    plain scan return the same index, or (FP32 ties across chunks visited in
    a different order) a point whose distance rounds to the same value."""
    A, torch = _gpu()
    pb, st = synth.workload_paper_scale()
    for theta in (pb.theta0, pulled_in(pb, 0.75), pulled_in(pb, 0.95)):
        res = []
        for prune in (True, False):
            s = A.Solver(pb, st, debug=True, theta0=theta, prune=prune)
            s.step(1)
            res.append(s.result())
            s.close()
        a, b = res[0]["nn_idx"], res[1]["nn_idx"]
        diff = np.argwhere(a != b)
        say("[parity] pruned vs plain index differences:", len(diff))
        assert len(diff) <= 1e-4 * a.size
        S = pb.S.astype(np.float64)
        R = pb.R.astype(np.float64)
        th = np.asarray(theta, np.float64)
        for i, n in diff[:200]:
            p = (i // pb.K) % pb.n_pre
            sp = oracle.quat_to_rot(th[3:, i]) @ S[pb.s_off[p] + n] + th[:3, i]
            da = ((sp - R[a[i, n]]) ** 2).sum()
            db = ((sp - R[b[i, n]]) ** 2).sum()
            # both round to the same FP32 value of |r|^2 - 2 r.s (a few ulp of ~0.01 m^2)
            assert abs(da - db) <= 1e-8
        assert np.array_equal(res[0]["ncol"], res[1]["ncol"])


def ragged_problem(seed, n_obj, ms, ns, K, mcs=None):
    rng = np.random.default_rng(seed)
    objs = [synth.superquadric(m, rng) if m > 8 else rng.uniform(-0.03, 0.03, (m, 3)).astype(np.float32)
            for m in ms]
    pre = [synth.gripper_contact_cloud(0.04 + 0.02 * j, n, rng) for j, n in enumerate(ns)]
    grids = [synth.gripper_sdf_grid(0.04 + 0.02 * j, 48, 0.003) for j in range(len(ns))]
    pb = synth._assemble(objs, pre, grids, K, [0.07] * n_obj)
    if mcs is not None:
        cs = [o[:mc] for o, mc in zip(objs, mcs)]
        pb.C = np.concatenate(cs) if sum(mcs) else np.zeros((0, 3), np.float32)
        pb.c_off = np.cumsum([0] + list(mcs)).astype(np.int32)
    return pb


def test_ragged_sizes_and_edges():
    st = synth.Settings(k_max=6, k_stein=3)
    # ragged M (77, 1, 130), ragged N (100, 65), K = 3; object 1 has one point
    pb = ragged_problem(5, 3, [77, 1, 130], [100, 65], 3)
    for k, frac in [(0, 0.0), (2, 0.6), (4, 0.8)]:
        compare_step(pb, st, pulled_in(pb, frac), k, label=f"ragged k={k}")
    # a single particle, an empty collision cloud for one object
    pb = ragged_problem(6, 2, [200, 64], [64], 1, mcs=[0, 64])
    compare_step(pb, st, pulled_in(pb, 0.7), 0, label="K=1 empty collision cloud")
    compare_step(pb, st, pulled_in(pb, 0.7), 4, label="K=1 SGD")


@pytest.mark.parametrize("case", ["cropped", "no_negative_node", "all_negative"])
def test_sdf_grid_shapes_and_degenerate_grids(case):
    """The collision gate's cull tables (one bit per cell, prefix counts of
    4^3-cell bricks) on grids that a cubic grid would not exercise: a grid
    cropped to 63 x 40 x 37 nodes (per axis a different cell count, none a
    multiple of 4 or 32, cutting through the fingers), a grid without any
    negative node (nothing collides) and one with every node negative (every
    collision point inside the grid collides).  One teacher-forced step
    against the oracle, poses pulled in so that the gripper meets the
    object."""
    pb, st = synth.workload_small(k_max=8)
    g = pb.grids[0]
    if case == "cropped":
        x0, y0, z0 = 1, 7, 3
        vals = np.ascontiguousarray(g.values[z0:z0 + 37, y0:y0 + 40, x0:x0 + 63])
        origin = (g.origin + np.float32(g.cell) * np.array([x0, y0, z0], np.float32)).astype(np.float32)
        grid = synth.Grid(values=vals, origin=origin, cell=g.cell)
    elif case == "no_negative_node":
        grid = synth.Grid(values=(np.abs(g.values) + np.float32(1e-3)).astype(np.float32), origin=g.origin, cell=g.cell)
    else:
        grid = synth.Grid(values=(-np.abs(g.values) - np.float32(1e-3)).astype(np.float32), origin=g.origin, cell=g.cell)
    pb = dataclasses.replace(pb, grids=[grid])
    for k, frac in [(0, 0.6), (2, 0.8)]:
        out = compare_step(pb, st, pulled_in(pb, frac), k, label=f"sdf {case} k={k}")
        say(f"[parity] sdf {case} k={k}", out)


@pytest.mark.parametrize("offset", [(1.0, -0.7, 0.5), (-3.0, 2.5, 4.0)])
def test_scene_away_from_the_origin(offset):
    """The whole scene -- object and collision clouds and every pose -- moved
    by a few metres: the poses of Sec. IV-A are in the object's frame, but
    the interface accepts any frame.  The library works relative to each
    object's centroid, so the bar is the same as at the origin (ties within
    1e-6 m^2, 1e-4 relative)."""
    pb, st = synth.workload_small()
    shift = np.asarray(offset, np.float32)
    pb.R = (pb.R + shift).astype(np.float32)
    pb.C = pb.R
    pb.theta0 = pb.theta0.copy()
    pb.theta0[:3] += shift[:, None]
    for k, frac in [(0, 0.0), (5, 0.7)]:
        out = compare_step(pb, st, pulled_in(pb, frac), k, label=f"offset {offset} k={k}")
        say(f"[parity] offset {offset} k={k}", out)
    # a later step of the oracle's own trajectory (Stein and SGD phases)
    st2 = synth.paper_settings(k_max=20, k_stein=8)
    snaps = oracle_trajectory(pb, st2, [6, 12])
    for k in (6, 12):
        th_k, pc, cv = snaps[k]
        say(f"[parity] offset {offset} paper preset k={k}", compare_step(pb, st2, th_k, k, pc, cv, label="offset"))


def test_largest_object_cloud():
    """An object of 2^22 points, the most the interface accepts per cloud
    (its collision cloud too), with a ragged 200-point contact cloud: one
    teacher-forced Stein step of 4 particles against the oracle, and the
    pruned and full scans give the same nearest points."""
    A, torch = _gpu()
    rng = np.random.default_rng(11)
    m = 1 << 22
    v = rng.normal(size=(m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    obj = (v * 0.035 + rng.normal(scale=0.001, size=(m, 3))).astype(np.float32)  # a 3.5 cm shell
    pre = [synth.gripper_contact_cloud(0.06, 200, rng)]
    grids = [synth.gripper_sdf_grid(0.06, 48, 0.003)]
    pb = synth._assemble([obj], pre, grids, 4, [0.07])
    st = synth.Settings(k_max=4, k_stein=2)
    th = pulled_in(pb, 0.6)
    out = compare_step(pb, st, th, 0, label="largest object cloud")
    say("[parity] largest object cloud", out)
    assert out["ncol"] > 0
    assert out["update_checked"] == out["of"]  # excused gate decisions are bounded, not skipped
    res = []
    for prune in (True, False):
        s = A.Solver(pb, st, debug=True, theta0=th, prune=prune)
        s.step(1)
        res.append(s.result())
        s.close()
    a, b = res[0]["nn_idx"], res[1]["nn_idx"]
    diff = np.argwhere(a != b)
    say("[parity] largest object cloud, pruned vs plain index differences:", len(diff))
    S = pb.S.astype(np.float64)
    R = pb.R.astype(np.float64)
    th64 = th.astype(np.float64)
    for i, n in diff:
        sp = oracle.quat_to_rot(th64[3:, i]) @ S[n] + th64[:3, i]
        assert abs(((sp - R[a[i, n]]) ** 2).sum() - ((sp - R[b[i, n]]) ** 2).sum()) <= 1e-8


def test_batched_objects_first_steps():
    pb, st = synth.workload_batched(n_obj=4, K=16, k_max=10, m_lo=512, m_hi=4096, n=640, grid_n=64)
    compare_step(pb, st, pb.theta0, 0, label="batched")
    compare_step(pb, st, pulled_in(pb, 0.7), 3, label="batched pulled in")


def subset_record(g, sel, groups):
    """The GPU record of particles `sel` (and bandwidths of `groups`), laid out
    as a record of the sub-problem holding only those particles."""
    out = dict(g)
    for key in ("theta", "cost", "col_cost", "ncol", "converged", "prev_cost", "grad", "grad_ct", "grad_col",
                "phi"):
        out[key] = np.asarray(g[key])[..., sel]
    for key in ("nn_idx", "rev_idx"):
        out[key] = np.asarray(g[key])[sel]
    out["h"] = np.asarray(g["h"])[groups]
    return out


def sub_problem(pb, objs, theta):
    """The objects `objs` of pb alone, with their particles' poses: groups
    never mix objects, so their step is the same computation."""
    R_parts = [pb.R[pb.r_off[o]:pb.r_off[o + 1]] for o in objs]
    C_parts = [pb.C[pb.c_off[o]:pb.c_off[o + 1]] for o in objs]
    per_obj = pb.n_pre * pb.K
    sel = np.concatenate([np.arange(o * per_obj, (o + 1) * per_obj) for o in objs])
    groups = np.concatenate([np.arange(o * pb.n_pre, (o + 1) * pb.n_pre) for o in objs])
    sub = synth.Problem(R=np.concatenate(R_parts), r_off=np.cumsum([0] + [len(r) for r in R_parts]).astype(np.int32),
                        C=np.concatenate(C_parts), c_off=np.cumsum([0] + [len(c) for c in C_parts]).astype(np.int32),
                        S=pb.S, s_off=pb.s_off, grids=pb.grids, theta0=np.ascontiguousarray(theta[:, sel]), K=pb.K)
    return sub, sel, groups


def test_batched_workload_full_size_sampled():
    """The full batched workload (64 objects of 2k-32k points, 24,576
    particles, 3 x 4096 contact points) stepped once on the GPU in its own
    launch layout, with the per-point NN and gate records; every particle of
    its smallest and its largest object is held to the bar of the other
    parity tests (exact tie and gate excusal) against the oracle run on those
    two objects alone.  Poses are pulled 0-70 % of the way towards each
    object's centre, so both collision-free and colliding particles occur."""
    pb, st = synth.workload_batched()
    m = np.diff(pb.r_off)
    sub_objs = [int(np.argmin(m)), int(np.argmax(m))]
    per_obj = pb.n_pre * pb.K
    th = pb.theta0.astype(np.float64)
    frac = np.linspace(0.0, 0.7, per_obj)
    for o in range(pb.n_obj):
        com = pb.R[pb.r_off[o]:pb.r_off[o + 1]].astype(np.float64).mean(0)
        c = slice(o * per_obj, (o + 1) * per_obj)
        th[:3, c] += frac * (com[:, None] - th[:3, c])
    th = th.astype(np.float32)
    say(f"[parity] batched full size: objects {sub_objs} of {pb.n_obj}, M = {m[sub_objs].tolist()}")
    g = gpu_step(pb, st, th, 0, label="batched full size")
    sub, sel, groups = sub_problem(pb, sub_objs, th)
    out = compare(sub, st, sub.theta0, 0, subset_record(g, sel, groups))
    say("[parity] batched full size:", out)
    assert 0 < (np.asarray(g["ncol"])[sel] > 0).sum() < len(sel)


def test_determinism_and_resume():
    A, torch = _gpu()
    pb, st = synth.workload_small()
    runs = []
    for _ in range(2):
        s = A.Solver(pb, st)
        s.solve()
        runs.append(s.result())
        s.close()
    assert np.array_equal(runs[0]["theta"], runs[1]["theta"])
    assert np.array_equal(runs[0]["cost"], runs[1]["cost"])
    # 12 + 18 iterations through a new context equal 30 straight
    s = A.Solver(pb, st)
    s.step(12)
    mid = s.result()
    s.close()
    s = A.Solver(pb, st, theta0=mid["theta"], k_start=12, prev_cost=mid["prev_cost"],
                 converged=mid["converged"])
    s.solve()
    res = s.result()
    s.close()
    assert np.array_equal(res["theta"], runs[0]["theta"])
    assert np.array_equal(res["best_particle"], runs[0]["best_particle"])


def test_graph_replay_matches_solve():
    """asicp_replay (whole solve as one captured HIP graph) gives bitwise the
    result of asicp_solve, on every replay, also after the initial particles
    are rewritten in place."""
    A, torch = _gpu()
    pb, st = synth.workload_small(k_max=8)
    ref = A.Solver(pb, st)
    ref.solve()
    r0 = ref.result()
    ref.close()
    g = A.Solver(pb, st)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()  # eager work between replays
        r = g.result()
        assert np.array_equal(r["theta"], r0["theta"]) and np.array_equal(r["cost"], r0["cost"])
        assert np.array_equal(r["best_particle"], r0["best_particle"])
    # new initial particles written into the borrowed buffer
    th2 = pb.theta0.copy()
    th2[:3] += np.float32(0.003)
    g._keep["theta0"].copy_(torch.as_tensor(th2))
    g.replay()
    r2 = g.result()
    g.close()
    ref2 = A.Solver(pb, st, theta0=th2)
    ref2.solve()
    e2 = ref2.result()
    ref2.close()
    assert np.array_equal(r2["theta"], e2["theta"])
    assert not np.array_equal(r2["theta"], r0["theta"])


def _final_selection(pb, st, th):
    """GPU final evaluation and selection only (k_start = k_max) at float32
    poses `th`; returns the result record."""
    A, torch = _gpu()
    s = A.Solver(pb, st, theta0=th, k_start=st.k_max)
    s.solve()
    r = s.result()
    s.close()
    return r


def test_selection_fallback_and_tie_rule():
    """The returned grasp (Algorithm 1 return; Sec. VI-A): the lowest-cost
    collision-free particle; with none collision free, the lowest-cost
    particle, flagged; equal costs go to the lowest particle index.  Poses
    are built so that the oracle's costs are separated by far more than FP32
    rounding, except for bit-identical copies of one pose (equal costs on both
    sides)."""
    pb, st = synth.workload_small(K=8, k_max=3)
    o = oracle.Oracle(pb, st)
    th = pulled_in(pb, 1.0)  # every gripper at the object's centre: all collide
    ev = o.evaluate(th)
    assert (ev["ncol"] > 0).all()
    j = int(np.argmin(ev["cost"]))
    dups = [i for i in range(pb.k_tot) if i != j][:2] if j >= 2 else [pb.k_tot - 2, pb.k_tot - 1]
    th[:, dups] = th[:, [j]]
    ev = o.evaluate(th)
    tied = sorted(dups + [j])
    c = ev["cost"]
    rest = np.setdiff1d(np.arange(pb.k_tot), tied)
    assert c[rest].min() > c[j] * (1 + 1e-3), "precondition: a clear minimum"
    exp = o.solve(th, k_start=st.k_max)
    assert exp["best"][0] == tied[0] and exp["best_free"][0] == 0
    r = _final_selection(pb, st, th)
    say("[select] all colliding: tie", tied, "->", r["best_particle"][0], "free", r["best_free"][0])
    assert r["best_free"][0] == 0 and r["best_particle"][0] == tied[0]
    assert np.array_equal(r["best_theta"][0], th[:, tied[0]])
    # one particle left at its far initial pose: collision free with a higher
    # cost than the colliding ones, and it must be the one returned
    far = rest[-1]
    th[:, far] = pb.theta0[:, far]
    ev = o.evaluate(th)
    assert ev["ncol"][far] == 0 and (ev["ncol"][np.arange(pb.k_tot) != far] > 0).all()
    assert ev["cost"][far] > ev["cost"][j]
    exp = o.solve(th, k_start=st.k_max)
    assert exp["best"][0] == far and exp["best_free"][0] == 1
    r = _final_selection(pb, st, th)
    assert r["best_free"][0] == 1 and r["best_particle"][0] == far
    assert r["best_cost"][0] == r["cost"][far]


@pytest.mark.parametrize("wl", ["paper", "batched"])
def test_graph_replay_matches_solve_full_size(wl):
    """asicp_replay on the full paper-scale and batched workloads returns
    bitwise what asicp_solve returns, on two replays in a row."""
    A, torch = _gpu()
    pb, st = synth.workload_paper_scale() if wl == "paper" else synth.workload_batched()
    ref = A.Solver(pb, st)
    ref.solve()
    r0 = ref.result()
    ref.close()
    g = A.Solver(pb, st)
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        r = g.result()
        for key in ("theta", "cost", "ncol", "grad", "best_particle", "best_free", "best_theta", "best_cost"):
            assert np.array_equal(np.asarray(r[key]), np.asarray(r0[key])), (wl, rep, key)
        say(f"[replay] {wl} replay {rep}: bit-identical to the solve")
    g.close()


def test_free_running_solve_small():
    """Free-running trajectories: while every correspondence agrees the poses
    agree to 1e-3 rad / 0.5 mm; the selected grasp is valid either way."""
    A, torch = _gpu()
    pb, st = synth.workload_small()
    o = oracle.Oracle(pb, st)
    s = A.Solver(pb, st, debug=True)
    th = pb.theta0.astype(np.float64)
    pc = cv = None
    agreed = 0
    for k in range(st.k_max):
        s.step(1)
        g = s.result()
        r = o.step(k, th, pc, cv, full=True)
        try:  # correspondences and gate decisions equal up to ties
            pu.check_nn(pb, th, g["nn_idx"], r["nn_idx"])
            pu.check_gate(pb, g["rev_idx"], r["gate"], r["phi_c"])
        except AssertionError:
            break
        th, pc, cv = r["theta"], r["prev_cost"], r["converged"]
        dt = np.abs(g["theta"][:3] - th[:3]).max()
        ang = pu.angle_between(g["theta"][3:], th[3:]).max()
        assert dt < 5e-4 and ang < 1e-3, (k, dt, ang)
        agreed = k + 1
    say("[parity] iterations with correspondences equal up to ties:", agreed)
    s.close()
    s = A.Solver(pb, st)
    s.solve()
    res = s.result()
    s.close()
    assert agreed >= 5
    b = res["best_particle"][0]
    assert 0 <= b < pb.k_tot
    if res["best_free"][0]:
        assert res["ncol"][b] == 0
        assert res["cost"][b] == res["cost"][res["ncol"] == 0].min()
    assert np.allclose(res["best_theta"][0], res["theta"][:, b])


def test_abi_state_and_numeric_errors():
    A, torch = _gpu()
    pb, st = synth.workload_small(k_max=3)
    s = A.Solver(pb, st)
    s.step(3)
    with pytest.raises(A.AsicpError) as e:
        s.step(1)
    assert e.value.status == A.ASICP_E_STATE
    s.solve()
    with pytest.raises(A.AsicpError) as e:
        s.solve()
    assert e.value.status == A.ASICP_E_STATE
    s.close()
    bad = pb.theta0.copy()
    bad[0, 5] = np.nan
    s = A.Solver(pb, st, theta0=bad)
    s.solve()
    r = s.result(check=False)
    assert r["status"] == A.ASICP_E_NUMERIC
    s.close()


def test_timing_hook_counts_launches():
    A, torch = _gpu()
    pb, st = synth.workload_small(k_max=4)
    s = A.Solver(pb, st, timing=True)
    s.solve()
    s.result(per_particle=False)
    ms, n, pairs = s.kernel_time()
    assert n == 5 and ms > 0
    # every launch compares each contact point with at most every object point
    assert 0 < pairs <= 5 * pb.k_tot * (pb.s_off[1] - pb.s_off[0]) * (pb.r_off[1] - pb.r_off[0])
    s.close()
    s = A.Solver(pb, st, timing=True, prune=False)
    s.solve()
    s.result(per_particle=False)
    ms, n, pairs = s.kernel_time()
    assert pairs == 5 * pb.k_tot * (pb.s_off[1] - pb.s_off[0]) * (pb.r_off[1] - pb.r_off[0])
    s.close()



def test_reset_repeats_the_solve_exactly():
    """asicp_reset starts the solve again on the same context: a second solve
    returns bitwise what the first did, the timing records accumulate over
    both, and a captured graph replayed after an eager solve (an odd number
    of iterations, so the double-buffered poses end on the other buffer)
    still reads back its own final poses."""
    A, torch = _gpu()
    pb, st = synth.workload_small(k_max=5)
    keys = ("theta", "cost", "ncol", "grad", "h", "best_theta", "best_particle")
    s = A.Solver(pb, st, timing=True)
    s.solve()
    first = s.result()
    t1 = s.kernel_time()
    s.reset()
    s.solve()
    second = s.result()
    t2 = s.kernel_time()
    for key in keys:
        assert np.array_equal(np.asarray(first[key]), np.asarray(second[key])), key
    assert t2[1] == 2 * t1[1] and t2[2] == 2 * t1[2]
    s.close()
    g = A.Solver(pb, st)
    g.replay()
    rep = g.result()
    g.reset()
    g.step(2)
    part = g.result()
    assert part["iterations_done"] == 2
    g.solve()
    eager = g.result()
    g.replay()
    rep2 = g.result()
    g.close()
    for key in keys:
        assert np.array_equal(np.asarray(rep[key]), np.asarray(first[key])), ("replay", key)
        assert np.array_equal(np.asarray(eager[key]), np.asarray(first[key])), ("eager after replay", key)
        assert np.array_equal(np.asarray(rep2[key]), np.asarray(first[key])), ("replay after eager", key)
    assert not np.array_equal(np.asarray(part["theta"]), np.asarray(first["theta"]))

def test_reset_reads_a_rewritten_sdf():
    """The set-up rebuilds the SDF cull tables from the borrowed grid: after
    the grid is rewritten in place (a gripper inflated by 3 cm, then the
    original again), asicp_reset and a solve return bitwise what a fresh
    context on that grid returns, and collisions do occur on the inflated
    grid."""
    A, torch = _gpu()
    pb, st = synth.workload_small(k_max=8)
    keys = ("theta", "cost", "col_cost", "ncol", "grad", "best_theta", "best_particle")
    fat = dataclasses.replace(pb.grids[0], values=(pb.grids[0].values - np.float32(0.03)).astype(np.float32))
    pb_fat = dataclasses.replace(pb, grids=[fat])

    def fresh(problem):
        f = A.Solver(problem, st)
        f.solve()
        r = f.result()
        f.close()
        return r

    ref_thin, ref_fat = fresh(pb), fresh(pb_fat)
    assert int(np.sum(ref_fat["ncol"])) > int(np.sum(ref_thin["ncol"]))
    s = A.Solver(pb, st)
    grid = s._keep["grids"][0]
    for values, ref, name in ((fat.values, ref_fat, "inflated"), (pb.grids[0].values, ref_thin, "original")):
        grid.copy_(torch.as_tensor(values).to(grid.device))
        s.reset()
        s.solve()
        r = s.result()
        for key in keys:
            assert np.array_equal(np.asarray(r[key]), np.asarray(ref[key])), (name, key)
    s.close()


def _run(pb, st, launch=None, tune=False, steps=3):
    A, torch = _gpu()
    s = A.Solver(pb, st, debug=True)
    chosen = None
    if launch is not None:
        s.set_launch(**launch)
    if tune:
        chosen, ms = s.autotune(reps=2)
        say("[parity] autotune", chosen, ms)
        assert all(v > 0 for v in ms)
    s.step(steps)
    r = s.result()
    s.close()
    return r, chosen


@pytest.mark.parametrize("wl", ["small", "paper", "batched"])
def test_launch_choices_are_bit_identical(wl):
    """Every XCD placement and chunk-test choice, and autotuning itself,
    return exactly the same outputs (they only change speed)."""
    if wl == "small":
        pb, st = synth.workload_small()
    elif wl == "paper":
        pb, st = synth.workload_paper_scale()
    else:
        pb, st = synth.workload_batched(n_obj=8, K=32, m_lo=1024, m_hi=8192, grid_n=64)
    A, torch = _gpu()
    ref, _ = _run(pb, st, launch=A.launch_choice(0))
    for v in range(1, A.ASICP_LAUNCH_CHOICES):
        launch = A.launch_choice(v)
        r, _ = _run(pb, st, launch=launch)
        for key in ("theta", "cost", "ncol", "grad", "nn_idx", "rev_idx", "h"):
            assert np.array_equal(np.asarray(r[key]), np.asarray(ref[key])), (launch, key)
    r, chosen = _run(pb, st, tune=True)
    assert A.launch_index(**chosen) in range(A.ASICP_LAUNCH_CHOICES)
    for key in ("theta", "cost", "ncol", "grad", "nn_idx", "rev_idx", "h"):
        assert np.array_equal(np.asarray(r[key]), np.asarray(ref[key])), ("tuned", key)


def test_launch_choices_rejected_on_the_host():
    A, torch = _gpu()
    pb, st = synth.workload_small(k_max=2)
    s = A.Solver(pb, st)
    assert s.launch() == {"xcd_map": 1, "fine": 1, "query_blocks": 4, "chunk_points": 128}
    for bad in (dict(xcd_map=2, fine=0), dict(xcd_map=0, fine=0, query_blocks=3),
                dict(xcd_map=0, fine=0, chunk_points=96)):
        with pytest.raises(A.AsicpError) as e:
            s.set_launch(**bad)
        assert e.value.status == A.ASICP_E_INVALID
    assert s.launch() == {"xcd_map": 1, "fine": 1, "query_blocks": 4, "chunk_points": 128}
    s.close()


def test_autotune_leaves_the_pair_counter():
    """The pairs evaluated depend on the launch choice (the chunk test skips
    work), so compare a tuned context with an untuned one set to the same
    choice: the tuning launches must not be counted."""
    A, torch = _gpu()
    pb, st = synth.workload_small()
    s = A.Solver(pb, st, timing=True)
    chosen, _ = s.autotune(reps=2)
    s.step(3)
    tuned = s.kernel_time()[1:]
    s.close()
    s = A.Solver(pb, st, timing=True)
    s.set_launch(**chosen)
    s.step(3)
    plain = s.kernel_time()[1:]
    s.close()
    assert tuned == plain
