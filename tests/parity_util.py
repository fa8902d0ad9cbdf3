"""Comparison helpers for GPU-vs-oracle parity (tolerances of the build).

- NN indices: equal, or the GPU's choice is within 1e-6 m^2 of the oracle's
  nearest distance (FP64, same pose): a tie.
- Gate decisions: equal, or the oracle's SDF value is within 1e-6 m of 0.
- Costs / gradients: |gpu - oracle| <= 1e-4 * max(|oracle|, scale), the scale
  being the mean magnitude of the summed terms (so that cancellation near a
  converged pose does not turn rounding into a failure).
"""
import numpy as np

import oracle

TIE_M2 = 1e-6
GATE_M = 1e-6
REL = 1e-4


def poses(theta_soa):
    th = np.asarray(theta_soa, np.float64)
    return [(th[:3, i], oracle.quat_to_rot(th[3:, i])) for i in range(th.shape[1])]


def tie_bounds(pb, theta_soa, gpu_idx, or_idx, K=None):
    """Per-particle bound on what tie-excused NN mismatches may change in g_t
    and g_w: (1/N) sum |r_gpu - r_or| and (1/N) sum |R s| |r_gpu - r_or| over
    the mismatched points (both choices are nearest neighbours within the tie
    tolerance, so either gradient is a correct result)."""
    S = pb.S.astype(np.float64)
    R = pb.R.astype(np.float64)
    th = np.asarray(theta_soa, np.float64)
    K = pb.K if K is None else K
    bt = np.zeros(th.shape[1])
    bw = np.zeros(th.shape[1])
    for i in range(th.shape[1]):
        g = i // K
        o, p = g // pb.n_pre, g % pb.n_pre
        n0, n1 = pb.s_off[p], pb.s_off[p + 1]
        a = np.asarray(gpu_idx[i][: n1 - n0])
        b = np.asarray(or_idx[i][: n1 - n0])
        bad = np.nonzero(a != b)[0]
        if len(bad) == 0:
            continue
        m0 = pb.r_off[o]
        dr = np.linalg.norm(R[m0 + a[bad]] - R[m0 + b[bad]], axis=1)
        u = np.linalg.norm(S[n0 + bad] @ oracle.quat_to_rot(th[3:, i]).T, axis=1)
        bt[i] = dr.sum() / (n1 - n0)
        bw[i] = (u * dr).sum() / (n1 - n0)
    return bt, bw


def rev_tie_bounds(pb, theta_soa, gpu_rev, or_rev):
    """Like tie_bounds for the collision gradient: (1/ncol) sum |s_gpu - s_or|
    and (1/ncol) sum |R s| |s_gpu - s_or| over colliding points whose reverse
    matches differ."""
    S = pb.S.astype(np.float64)
    th = np.asarray(theta_soa, np.float64)
    bt = np.zeros(th.shape[1])
    bw = np.zeros(th.shape[1])
    for i in range(th.shape[1]):
        g = i // pb.K
        o, p = g // pb.n_pre, g % pb.n_pre
        c0, c1 = pb.c_off[o], pb.c_off[o + 1]
        a = np.asarray(gpu_rev[i][: c1 - c0])
        b = np.asarray(or_rev[i][: c1 - c0])
        ncol = max(1, int((b >= 0).sum()))
        bad = np.nonzero((a >= 0) & (b >= 0) & (a != b))[0]
        if len(bad) == 0:
            continue
        n0 = pb.s_off[p]
        ds = np.linalg.norm(S[n0 + a[bad]] - S[n0 + b[bad]], axis=1)
        # s x (s - c') = -s x c', so a different match moves that term by |ds x c'|
        cl = np.linalg.norm(pb.C.astype(np.float64)[c0 + bad] - th[:3, i], axis=1)
        bt[i] = ds.sum() / ncol
        bw[i] = (ds * cl).sum() / ncol
    return bt, bw


def check_nn(pb, theta_soa, gpu_idx, or_idx, K=None, particles=None):
    """Returns the number of tie-excused mismatches; raises on a real one."""
    S = pb.S.astype(np.float64)
    R = pb.R.astype(np.float64)
    th = np.asarray(theta_soa, np.float64)
    n_pre = pb.n_pre
    K = pb.K if K is None else K
    ties = 0
    idxs = range(th.shape[1]) if particles is None else particles
    for i in idxs:
        g = i // K
        o, p = g // n_pre, g % n_pre
        n0, n1 = pb.s_off[p], pb.s_off[p + 1]
        m0 = pb.r_off[o]
        a = np.asarray(gpu_idx[i][: n1 - n0])
        b = np.asarray(or_idx[i][: n1 - n0])
        bad = np.nonzero(a != b)[0]
        if len(bad) == 0:
            continue
        Rm = oracle.quat_to_rot(th[3:, i])
        sp = S[n0 + bad] @ Rm.T + th[:3, i]
        assert (a[bad] >= 0).all() and (a[bad] < pb.r_off[o + 1] - m0).all(), "GPU NN index out of range"
        da = ((sp - R[m0 + a[bad]]) ** 2).sum(1)
        db = ((sp - R[m0 + b[bad]]) ** 2).sum(1)
        worst = float((da - db).max())
        assert worst <= TIE_M2, f"particle {i}: NN mismatch {worst:.3g} m^2 beyond the tie tolerance"
        ties += len(bad)
    return ties


def check_gate(pb, gpu_rev, or_gate, or_phi, particles=None):
    """Gate decisions (rev index >= 0 on the GPU means colliding)."""
    gg = np.asarray(gpu_rev) >= 0
    go = np.asarray(or_gate).astype(bool)
    n_obj_pts = np.diff(pb.c_off)
    excused = 0
    rows = range(gg.shape[0]) if particles is None else particles
    for i in rows:
        o = (i // pb.K) // pb.n_pre
        mc = n_obj_pts[o]
        diff = np.nonzero(gg[i, :mc] != go[i, :mc])[0]
        if len(diff):
            phi = np.abs(np.asarray(or_phi)[i, diff])
            assert np.all(phi < GATE_M), f"particle {i}: gate mismatch with |phi| up to {phi.max():.3g} m"
            excused += len(diff)
    return excused


def check_rev(pb, theta_soa, gpu_rev, or_rev, particles=None):
    """Reverse NN indices of points both sides call colliding."""
    S = pb.S.astype(np.float64)
    Cc = pb.C.astype(np.float64)
    th = np.asarray(theta_soa, np.float64)
    ties = 0
    rows = range(th.shape[1]) if particles is None else particles
    for i in rows:
        g = i // pb.K
        o, p = g // pb.n_pre, g % pb.n_pre
        n0 = pb.s_off[p]
        c0, c1 = pb.c_off[o], pb.c_off[o + 1]
        a = np.asarray(gpu_rev[i][: c1 - c0])
        b = np.asarray(or_rev[i][: c1 - c0])
        both = (a >= 0) & (b >= 0)
        bad = np.nonzero(both & (a != b))[0]
        if len(bad) == 0:
            continue
        Rm = oracle.quat_to_rot(th[3:, i])
        c = Cc[c0 + bad]
        sa = S[n0 + a[bad]] @ Rm.T + th[:3, i]
        sb = S[n0 + b[bad]] @ Rm.T + th[:3, i]
        worst = float((((sa - c) ** 2).sum(1) - ((sb - c) ** 2).sum(1)).max())
        assert worst <= TIE_M2, f"particle {i}: reverse NN mismatch {worst:.3g} m^2"
        ties += len(bad)
    return ties


def scales(pb, theta_soa, or_nn_idx, lam, setup):
    """Per-particle mean magnitudes of the summed terms of g_t and g_w
    (contact terms plus the lambda-weighted TCP-CoM term)."""
    S = pb.S.astype(np.float64)
    R = pb.R.astype(np.float64)
    th = np.asarray(theta_soa, np.float64)
    st = np.zeros(th.shape[1])
    sw = np.zeros(th.shape[1])
    for i in range(th.shape[1]):
        g = i // pb.K
        o, p = g // pb.n_pre, g % pb.n_pre
        n0, n1 = pb.s_off[p], pb.s_off[p + 1]
        Rm = oracle.quat_to_rot(th[3:, i])
        u = S[n0:n1] @ Rm.T
        e = u + th[:3, i] - R[pb.r_off[o] + np.asarray(or_nn_idx[i][: n1 - n0])]
        ne = np.linalg.norm(e, axis=1)
        uT = Rm @ setup["tcp"][p]
        eT = np.linalg.norm(uT + th[:3, i] - setup["com"][o])
        st[i] = ne.mean() + lam * eT
        sw[i] = (np.linalg.norm(u, axis=1) * ne).mean() + lam * np.linalg.norm(uT) * eT
    return st, sw


def close(gpu, ref, scale, rel=REL, what="", extra=0.0):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = rel * np.maximum(np.abs(ref), scale) + extra
    err = np.abs(gpu - ref)
    ok = err <= tol
    assert ok.all(), f"{what}: {int((~ok).sum())} entries beyond tolerance, worst ratio {float((err / tol).max()):.3g}"


def angle_between(qa, qb):
    """Rotation angle between quaternion columns, well conditioned for small
    angles: both normalised in FP64, signs aligned, angle = 4 asin(|qa - qb| / 2)."""
    a = np.asarray(qa, np.float64)
    b = np.asarray(qb, np.float64)
    a = a / np.linalg.norm(a, axis=0)
    b = b / np.linalg.norm(b, axis=0)
    b = np.where(np.sum(a * b, axis=0) < 0, -b, b)
    return 4 * np.arcsin(np.clip(np.linalg.norm(a - b, axis=0) / 2, 0, 1))
