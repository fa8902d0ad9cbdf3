"""Seeded synthetic inputs for the AS-ICP grasp iteration.

This module only *generates data*: object clouds, box-built parallel-jaw
grippers (contact cloud and signed distance grid), Fibonacci initial poses and
the named workload presets.  It holds none of the method's arithmetic, so both
the HIP path and the CPU oracle may read what it produces.

The paper's objects (KIT / Google Scanned Objects meshes), its gripper meshes
and its SDFs built with Open3D are not available; the workloads here stand in
for them with shapes of the same kind and size.  Every array is float32 (the
precision the solver receives); units are metres.

Quaternions are (w, x, y, z), scalar first, with w >= 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------
# Solver settings (plain numbers; the method itself lives elsewhere)
# ----------------------------------------------------------------------------

PRECOND_GN_DIAG, PRECOND_IDENTITY = 0, 1
SCHED_GEOMETRIC, SCHED_PAPER_CYCLIC = 0, 1
KERNEL_PRODUCT, KERNEL_BLOCK = 0, 1
BW_MEDIAN, BW_FIXED = 0, 1


@dataclasses.dataclass
class Settings:
    """Iteration settings (Table I of the paper for the cyclic preset)."""

    k_max: int = 30
    k_stein: int = 30
    eta: float = 1.0
    lam: float = 1.0
    precond: int = PRECOND_GN_DIAG
    schedule: int = SCHED_GEOMETRIC
    T0: float = 1.0
    T1: float = 0.01
    cyc_C: float = 5.0
    cyc_p: float = 2.0
    kernel_mode: int = KERNEL_PRODUCT
    bw_mode: int = BW_MEDIAN
    h_fixed: float = 1.0
    h_min: float = 1e-8
    conv_tol: float = 2e-4
    w_pen: float = 0.0  # optional SDF penetration term (0: the paper's cost)
    minibatch: int = 0  # 1: Table I mini-batch schedule of the object cloud
    seed: int = 0       # mini-batch sampling seed


def paper_settings(k_max: int = 40, k_stein: int = 15, minibatch: int = 1, seed: int = 7) -> Settings:
    """Table I: 15 SVGD + 25 SGD iterations, cyclic annealing C=5, p=2,
    learning rate and cost weights 1, convergence 0.02 %, mini-batch size
    growing linearly to the whole cloud at 2 k_max / 3."""
    return Settings(k_max=k_max, k_stein=k_stein, schedule=SCHED_PAPER_CYCLIC, cyc_C=5.0,
                    cyc_p=2.0, eta=1.0, lam=1.0, conv_tol=2e-4, minibatch=minibatch, seed=seed)


@dataclasses.dataclass
class Grid:
    values: np.ndarray  # (nz, ny, nx) float32, x fastest
    origin: np.ndarray  # (3,) float32, position of node (0, 0, 0)
    cell: float         # node spacing (a float32 value)


@dataclasses.dataclass
class Problem:
    """Host copy of one batch: objects x preshapes x K particles."""

    R: np.ndarray        # (Mtot, 3) float32 object clouds, concatenated
    r_off: np.ndarray    # (n_obj + 1,) int32
    C: np.ndarray        # (Mctot, 3) float32 collision clouds, concatenated
    c_off: np.ndarray    # (n_obj + 1,) int32
    S: np.ndarray        # (Ntot, 3) float32 gripper contact clouds, concatenated
    s_off: np.ndarray    # (n_pre + 1,) int32
    grids: list          # [Grid] per preshape
    theta0: np.ndarray   # (7, Ktot) float32 SoA: tx ty tz qw qx qy qz
    K: int               # particles per (object, preshape) group
    prior: np.ndarray | None = None  # optional (n_obj*n_pre, 9) float32 per group:
    #   mu_t (3), translation precision 1/sigma^2, mu_q (4, unit), kappa

    @property
    def n_obj(self) -> int:
        return len(self.r_off) - 1

    @property
    def n_pre(self) -> int:
        return len(self.s_off) - 1

    @property
    def k_tot(self) -> int:
        return self.n_obj * self.n_pre * self.K


# ----------------------------------------------------------------------------
# Box-built parallel gripper
# ----------------------------------------------------------------------------

def gripper_boxes(gap: float):
    """Palm plus two fingers, gripper origin at the palm centre, +z from the
    palm towards the fingertips.  For gap 0.06 m the palm is 8 x 2 x 1 cm and
    each finger 1 x 1 x 5 cm, the fingers' inner faces 6 cm apart.
    Returns a list of (centre, half_extents) in float64."""
    palm = (np.array([0.0, 0.0, 0.0]), np.array([(gap + 0.02) / 2, 0.01, 0.005]))
    f1 = (np.array([gap / 2 + 0.005, 0.0, 0.030]), np.array([0.005, 0.005, 0.025]))
    f2 = (np.array([-(gap / 2 + 0.005), 0.0, 0.030]), np.array([0.005, 0.005, 0.025]))
    return [palm, f1, f2]


def gripper_contact_cloud(gap: float, n: int, rng: np.random.Generator) -> np.ndarray:
    """Inner (contact) surface of the box gripper: the two finger inner faces
    and the palm face between the fingers, sampled uniformly by area."""
    faces = [  # (area, sampler)
        (0.01 * 0.05, lambda k: np.stack([np.full(k, gap / 2), rng.uniform(-0.005, 0.005, k),
                                          rng.uniform(0.005, 0.055, k)], 1)),
        (0.01 * 0.05, lambda k: np.stack([np.full(k, -gap / 2), rng.uniform(-0.005, 0.005, k),
                                          rng.uniform(0.005, 0.055, k)], 1)),
        (gap * 0.02, lambda k: np.stack([rng.uniform(-gap / 2, gap / 2, k),
                                         rng.uniform(-0.01, 0.01, k), np.full(k, 0.005)], 1)),
    ]
    area = np.array([f[0] for f in faces])
    which = rng.choice(len(faces), size=n, p=area / area.sum())
    pts = np.empty((n, 3))
    for fi, (_, sampler) in enumerate(faces):
        sel = np.nonzero(which == fi)[0]
        if len(sel):
            pts[sel] = sampler(len(sel))
    return pts.astype(np.float32)


def box_union_sdf(points: np.ndarray, boxes) -> np.ndarray:
    """Signed distance to a union of axis-aligned boxes (negative inside):
    the minimum over boxes of the textbook box distance
    |max(q, 0)| + min(max_k q_k, 0), q = |p - c| - h.  float64."""
    out = np.full(points.shape[:-1], np.inf)
    for c, h in boxes:
        q = np.abs(points - c) - h
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        inside = np.minimum(q.max(axis=-1), 0.0)
        out = np.minimum(out, outside + inside)
    return out


_GRID_CACHE: dict = {}


def gripper_sdf_grid(gap: float, n: int, cell: float) -> Grid:
    """n^3 grid of the box gripper's signed distance, centred on the
    gripper's bounding box; values computed in float64, stored float32.
    Grids are kept per (gap, n, cell) for the process; each call returns its
    own copy of the values."""
    key = (float(gap), int(n), float(cell))
    if key not in _GRID_CACHE:
        _GRID_CACHE[key] = _gripper_sdf_grid(gap, n, cell)
    g = _GRID_CACHE[key]
    return Grid(values=g.values.copy(), origin=g.origin.copy(), cell=g.cell)


def _gripper_sdf_grid(gap: float, n: int, cell: float) -> Grid:
    boxes = gripper_boxes(gap)
    lo = np.min([c - h for c, h in boxes], axis=0)
    hi = np.max([c + h for c, h in boxes], axis=0)
    centre = 0.5 * (lo + hi)
    cell32 = float(np.float32(cell))
    origin = (centre - cell32 * (n - 1) / 2.0).astype(np.float32)
    ax = np.arange(n, dtype=np.float64) * cell32
    z, y, x = np.meshgrid(ax + origin[2], ax + origin[1], ax + origin[0], indexing="ij")
    vals = box_union_sdf(np.stack([x, y, z], -1), boxes).astype(np.float32)
    return Grid(values=np.ascontiguousarray(vals), origin=origin, cell=cell32)


# ----------------------------------------------------------------------------
# Objects
# ----------------------------------------------------------------------------

def _unit_vectors(rng: np.random.Generator, k: int) -> np.ndarray:
    v = rng.standard_normal((k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def ellipsoid(m: int, axes, rng: np.random.Generator) -> np.ndarray:
    """m points uniform by area on an ellipsoid (rejection from the sphere map)."""
    a, b, c = sorted([float(x) for x in axes], reverse=True)
    ax = np.array([float(x) for x in axes])
    out = []
    need = m
    while need > 0:
        u = _unit_vectors(rng, 4 * need + 64)
        stretch = np.sqrt((ax[1] * ax[2] * u[:, 0]) ** 2 + (ax[0] * ax[2] * u[:, 1]) ** 2 +
                          (ax[0] * ax[1] * u[:, 2]) ** 2) / (a * b)
        keep = rng.uniform(size=len(u)) < stretch
        pts = u[keep] * ax
        out.append(pts[:need])
        need -= len(out[-1])
    return np.concatenate(out).astype(np.float32)


def _signed_pow(x, e):
    return np.sign(x) * np.abs(x) ** e


def superquadric(m: int, rng: np.random.Generator, noise: float = 0.001,
                 eps=None, axes=None) -> np.ndarray:
    """m points of a random superquadric surface, approximately uniform by
    area (8x oversampling in (eta, omega), weighted draw without replacement),
    plus isotropic Gaussian noise."""
    e1, e2 = eps if eps is not None else rng.uniform(0.3, 1.5, 2)
    a1, a2, a3 = axes if axes is not None else rng.uniform(0.02, 0.08, 3)

    def surf(eta, om):
        ce, se = _signed_pow(np.cos(eta), e1), _signed_pow(np.sin(eta), e1)
        return np.stack([a1 * ce * _signed_pow(np.cos(om), e2),
                         a2 * ce * _signed_pow(np.sin(om), e2), a3 * se], -1)

    k = 8 * m
    eta = rng.uniform(-np.pi / 2, np.pi / 2, k)
    om = rng.uniform(-np.pi, np.pi, k)
    hstep = 1e-5
    de = (surf(eta + hstep, om) - surf(eta - hstep, om)) / (2 * hstep)
    do = (surf(eta, om + hstep) - surf(eta, om - hstep)) / (2 * hstep)
    w = np.linalg.norm(np.cross(de, do), axis=1) + 1e-300
    # weighted sampling without replacement (exponential keys)
    key = np.log(rng.uniform(size=k)) / w
    pick = np.argpartition(-key, m - 1)[:m]
    pts = surf(eta[pick], om[pick]) + noise * rng.standard_normal((m, 3))
    return pts.astype(np.float32)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def box_union_object(m: int, rng: np.random.Generator, noise: float = 0.001) -> np.ndarray:
    """Union of 1-3 randomly rotated boxes: faces sampled by area, points
    strictly inside another box dropped, m kept, Gaussian noise added."""
    nb = int(rng.integers(1, 4))
    boxes = [(rng.uniform(-0.02, 0.02, 3), rng.uniform(0.01, 0.04, 3), _random_rotation(rng))
             for _ in range(nb)]
    pts = []
    for c, h, Rb in boxes:
        k = 6 * m
        face_area = np.array([h[1] * h[2], h[1] * h[2], h[0] * h[2], h[0] * h[2],
                              h[0] * h[1], h[0] * h[1]])
        f = rng.choice(6, size=k, p=face_area / face_area.sum())
        loc = rng.uniform(-1, 1, (k, 3)) * h
        ax = f // 2
        loc[np.arange(k), ax] = np.where(f % 2 == 0, h[ax], -h[ax])
        pts.append(loc @ Rb.T + c)
    allp = np.concatenate(pts)
    keep = np.ones(len(allp), bool)
    for c, h, Rb in boxes:
        local = (allp - c) @ Rb
        keep &= ~np.all(np.abs(local) < h - 1e-9, axis=1)
    allp = allp[keep]
    sel = rng.choice(len(allp), size=m, replace=len(allp) < m)
    return (allp[sel] + noise * rng.standard_normal((m, 3))).astype(np.float32)


# ----------------------------------------------------------------------------
# Initial poses
# ----------------------------------------------------------------------------

def _rot_to_quat(Rm: np.ndarray) -> np.ndarray:
    tr = Rm[0, 0] + Rm[1, 1] + Rm[2, 2]
    if tr > 0:
        s = 2.0 * math.sqrt(tr + 1.0)
        q = [0.25 * s, (Rm[2, 1] - Rm[1, 2]) / s, (Rm[0, 2] - Rm[2, 0]) / s, (Rm[1, 0] - Rm[0, 1]) / s]
    elif Rm[0, 0] > Rm[1, 1] and Rm[0, 0] > Rm[2, 2]:
        s = 2.0 * math.sqrt(1.0 + Rm[0, 0] - Rm[1, 1] - Rm[2, 2])
        q = [(Rm[2, 1] - Rm[1, 2]) / s, 0.25 * s, (Rm[0, 1] + Rm[1, 0]) / s, (Rm[0, 2] + Rm[2, 0]) / s]
    elif Rm[1, 1] > Rm[2, 2]:
        s = 2.0 * math.sqrt(1.0 + Rm[1, 1] - Rm[0, 0] - Rm[2, 2])
        q = [(Rm[0, 2] - Rm[2, 0]) / s, (Rm[0, 1] + Rm[1, 0]) / s, 0.25 * s, (Rm[1, 2] + Rm[2, 1]) / s]
    else:
        s = 2.0 * math.sqrt(1.0 + Rm[2, 2] - Rm[0, 0] - Rm[1, 1])
        q = [(Rm[1, 0] - Rm[0, 1]) / s, (Rm[0, 2] + Rm[2, 0]) / s, (Rm[1, 2] + Rm[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def _cross3(a, b) -> np.ndarray:
    """Cross product of two 3-vectors (numpy's formula, without its per-call
    overhead)."""
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _look_at(u: np.ndarray, anchor: np.ndarray, tip: np.ndarray, dist: float,
             roll: float = 0.0):
    """Pose whose gripper +z axis points along -u (back at `anchor`), with the
    gripper-frame point `tip` at `anchor + dist u`; the roll about +z is fixed
    by a look-at frame (up = world z, or world y when the approach is nearly
    vertical) and then turned by `roll`.  Returns (t, q) in float64."""
    ez = -u
    w = np.array([0.0, 0.0, 1.0]) if abs(ez[2]) <= 0.9 else np.array([0.0, 1.0, 0.0])
    ex = _cross3(w, ez)
    ex /= np.linalg.norm(ex)
    ey = _cross3(ez, ex)
    if roll != 0.0:
        ex, ey = math.cos(roll) * ex + math.sin(roll) * ey, -math.sin(roll) * ex + math.cos(roll) * ey
    Rm = np.stack([ex, ey, ez], axis=1)
    return anchor + dist * u - Rm @ tip, _rot_to_quat(Rm)


def _fibonacci_dirs(k: int) -> np.ndarray:
    """Fibonacci sphere: z_j = 1 - (2j+1)/k, azimuth j*pi*(3 - sqrt 5)."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    out = np.zeros((k, 3))
    for j in range(k):
        z = 1.0 - (2.0 * j + 1.0) / k
        r = math.sqrt(max(0.0, 1.0 - z * z))
        out[j] = (r * math.cos(j * golden), r * math.sin(j * golden), z)
    return out


def _poses(dirs, anchor, tip, dist, rolls=None) -> np.ndarray:
    out = np.zeros((7, len(dirs)))
    for j, u in enumerate(dirs):
        t, q = _look_at(np.asarray(u, np.float64), anchor, tip, dist, 0.0 if rolls is None else rolls[j])
        out[:3, j] = t
        out[3:, j] = q
    return out.astype(np.float32)


def fibonacci_poses(k: int, anchor: np.ndarray, tip: np.ndarray, dist: float) -> np.ndarray:
    """k poses on a Fibonacci sphere around `anchor` (the paper initialises
    with the Fibonacci sequence, Sec. V): direction u_j, the gripper's +z
    axis pointing back at the anchor and the gripper-frame point `tip` at
    distance `dist` from the anchor.  Returns (7, k) float32."""
    return _poses(_fibonacci_dirs(k), anchor, tip, dist)


def quarter_sphere_dirs(k: int, arm=(-1.0, 0.0, 0.0)) -> np.ndarray:
    """Exactly k Fibonacci directions on the quarter sphere that faces the
    robot arm (Sec. V, Fig. 4(b); Sec. VI-A): above the table (u_z >= 0) and on the
    arm's side (u . arm >= 0).  The Fibonacci count is the smallest whose
    quarter holds k points."""
    a = np.asarray(arm, np.float64)
    a = a / np.linalg.norm(a)
    for n in range(k, 16 * k + 64):
        d = _fibonacci_dirs(n)
        keep = d[(d[:, 2] >= 0.0) & (d @ a >= 0.0)]
        if len(keep) == k:
            return keep
    raise ValueError(f"no Fibonacci count gives {k} quarter-sphere points")


def top_poses(k: int, anchor: np.ndarray, tip: np.ndarray, dist: float) -> np.ndarray:
    """k poses straight above the object (Sec. VI-A adds six of them): gripper
    +z pointing down, rolls j*pi/k, j < k (a parallel gripper repeats itself
    after half a turn)."""
    dirs = np.tile([0.0, 0.0, 1.0], (k, 1))
    return _poses(dirs, anchor, tip, dist, [j * math.pi / k for j in range(k)])


def tabletop_poses(k: int, anchor: np.ndarray, tip: np.ndarray, dist: float, n_top: int = 6,
                   arm=(-1.0, 0.0, 0.0)) -> np.ndarray:
    """The paper's simulation initialisation (Sec. VI-A): k - n_top
    quarter-sphere Fibonacci poses plus n_top poses from above."""
    quarter = _poses(quarter_sphere_dirs(k - n_top, arm), anchor, tip, dist)
    return np.concatenate([quarter, top_poses(n_top, anchor, tip, dist)], axis=1)


def gmm_poses(k: int, anchor: np.ndarray, tip: np.ndarray, dist: float, means, sigma: float,
              rng: np.random.Generator) -> np.ndarray:
    """Initialisation from a mixture of Gaussians (Fig. 4(a), Sec. V):
    approach directions drawn from equal-weight isotropic Gaussians of
    standard deviation `sigma` around the unit directions `means`, projected
    to the unit sphere; the gripper looks at the anchor from `dist`."""
    mu = np.asarray(means, np.float64)
    mu = mu / np.linalg.norm(mu, axis=1, keepdims=True)
    comp = rng.integers(0, len(mu), k)
    d = mu[comp] + sigma * rng.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return _poses(d, anchor, tip, dist)


def table_plane(obj: np.ndarray, spacing: float = 0.005, margin: float = 0.05) -> np.ndarray:
    """Points of the supporting table (the collision cloud C holds the object
    and the table, Sec. IV-A): a square grid at `spacing` (Table I's 5 mm
    voxels) in the plane just below the object's lowest point, extending
    `margin` beyond the object's footprint."""
    o = obj.astype(np.float64)
    lo, hi = o.min(0) - margin, o.max(0) + margin
    xs = np.arange(lo[0], hi[0] + 1e-12, spacing)
    ys = np.arange(lo[1], hi[1] + 1e-12, spacing)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    Z = np.full(X.shape, o[:, 2].min() - 0.002)
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def _assemble(objects, preshapes, grids, K, dists):
    """Concatenate clouds and build Fibonacci poses for every (object,
    preshape) group.  The placement anchor is the object's mean point and the
    gripper point placed at distance `dist` is the contact cloud's mean."""
    r_off = np.cumsum([0] + [len(o) for o in objects]).astype(np.int32)
    s_off = np.cumsum([0] + [len(s) for s in preshapes]).astype(np.int32)
    thetas = []
    for oi, obj in enumerate(objects):
        anchor = obj.astype(np.float64).mean(0)
        for s in preshapes:
            thetas.append(fibonacci_poses(K, anchor, s.astype(np.float64).mean(0), dists[oi]))
    R = np.ascontiguousarray(np.concatenate(objects).astype(np.float32))
    return Problem(R=R, r_off=r_off, C=R, c_off=r_off.copy(),
                   S=np.ascontiguousarray(np.concatenate(preshapes).astype(np.float32)),
                   s_off=s_off, grids=list(grids), theta0=np.ascontiguousarray(np.concatenate(thetas, 1)),
                   K=K)


def standoff(obj: np.ndarray) -> float:
    """Start distance: 10 cm, or 6 cm beyond the object's farthest point from
    its mean, so the fingertips start clear of the object."""
    c = obj.astype(np.float64).mean(0)
    rb = float(np.linalg.norm(obj.astype(np.float64) - c, axis=1).max())
    return max(0.10, rb + 0.06)


def workload_small(K: int = 32, k_max: int = 30):
    """One object of 1024 points on an ellipsoid (semi-axes 4, 3, 2 cm); one
    preshape of 512 contact points on a box gripper (palm 8x2x1 cm, 1x1x5 cm
    fingers 6 cm apart); 64^3 SDF at 2 mm; 32 Fibonacci particles 10 cm away;
    30 iterations, geometric annealing 1 -> 0.01, median bandwidth."""
    obj = ellipsoid(1024, (0.04, 0.03, 0.02), np.random.default_rng(1))
    S = gripper_contact_cloud(0.06, 512, np.random.default_rng(2))
    grid = gripper_sdf_grid(0.06, 64, 0.002)
    pb = _assemble([obj], [S], [grid], K, [0.10])
    return pb, Settings(k_max=k_max, k_stein=k_max)


def workload_paper_scale(K: int = 256, k_max: int = 100, m: int = 8192, n: int = 4096,
                         grid_n: int = 128):
    """Object of 8192 points from a random superquadric (exponents U[0.3, 1.5],
    semi-axes U[2, 8] cm) with 1 mm Gaussian noise; 3 preshapes (finger gaps
    4 / 6 / 8 cm, 4096 contact points each, 128^3 SDF at 1.5 mm); 256
    Fibonacci particles per preshape; 100 iterations."""
    rng = np.random.default_rng(3)
    obj = superquadric(m, rng, noise=0.001)
    gaps = (0.04, 0.06, 0.08)
    pre = [gripper_contact_cloud(g, n, np.random.default_rng((3, i))) for i, g in enumerate(gaps)]
    grids = [gripper_sdf_grid(g, grid_n, 0.0015) for g in gaps]
    pb = _assemble([obj], pre, grids, K, [standoff(obj)])
    return pb, Settings(k_max=k_max, k_stein=k_max)


def workload_batched(n_obj: int = 64, K: int = 128, k_max: int = 100, m_lo: int = 2048,
                     m_hi: int = 32768, n: int = 4096, grid_n: int = 128, seed: int = 4):
    """Many objects of uneven size in one batch: point counts log-uniform in
    [m_lo, m_hi], superquadrics and unions of 1-3 boxes alternating, 1 mm
    noise; the three preshapes of the paper-scale workload; K particles each."""
    objs = random_objects(n_obj, m_lo, m_hi, seed)
    return workload_objects(objs, K, k_max, n, grid_n), Settings(k_max=k_max, k_stein=k_max)


def random_objects(n_obj: int, m_lo: int, m_hi: int, seed: int) -> list:
    """n_obj clouds of log-uniform size in [m_lo, m_hi]: superquadrics and
    unions of 1-3 boxes alternating, 1 mm noise."""
    rng = np.random.default_rng(seed)
    objs = []
    for o in range(n_obj):
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        objs.append(superquadric(m, rng) if o % 2 == 0 else box_union_object(m, rng))
    return objs


def workload_objects(objs: list, K: int, k_max: int = 100, n: int = 4096, grid_n: int = 128,
                     theta0: np.ndarray | None = None) -> Problem:
    """The given object clouds with the three preshapes of the paper-scale
    workload (finger gaps 4 / 6 / 8 cm, n contact points, grid_n^3 SDF at
    1.5 mm) and K Fibonacci particles per (object, preshape), or the poses
    theta0 (7, n_obj * 3 * K) when given."""
    gaps = (0.04, 0.06, 0.08)
    pre = [gripper_contact_cloud(g, n, np.random.default_rng((3, i))) for i, g in enumerate(gaps)]
    grids = [gripper_sdf_grid(g, grid_n, 0.0015) for g in gaps]
    pb = _assemble(objs, pre, grids, K, [standoff(o) for o in objs])
    if theta0 is not None:
        pb.theta0 = np.ascontiguousarray(theta0, np.float32)
    return pb


def random_poses(k: int, anchor: np.ndarray, radius: float, rng: np.random.Generator) -> np.ndarray:
    """k poses with uniformly random rotations and the gripper origin
    uniformly in a ball of `radius` around `anchor`.  Returns (7, k) float32."""
    q = rng.standard_normal((k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    u = _unit_vectors(rng, k) * (radius * rng.uniform(0, 1, (k, 1)) ** (1 / 3))
    return np.concatenate([(anchor + u).T, q.T]).astype(np.float32)


def workload_adjoint(n_obj: int = 16, K: int = 512, m: int = 4096, n: int = 4096, grid_n: int = 128,
                     seed: int = 5, w_pen: float = 1.0):
    """Cost-and-gradient workload: n_obj superquadrics of m points, one
    preshape (finger gap 6 cm, n contact points, grid_n^3 SDF at 1.5 mm), K
    particles per object at random poses near the object (some colliding,
    some free)."""
    rng = np.random.default_rng(seed)
    objs = [superquadric(m, rng) for _ in range(n_obj)]
    S = gripper_contact_cloud(0.06, n, np.random.default_rng((seed, 1)))
    grid = gripper_sdf_grid(0.06, grid_n, 0.0015)
    pb = _assemble(objs, [S], [grid], K, [0.1] * n_obj)
    th = []
    for o in objs:
        c = o.astype(np.float64).mean(0)
        rb = float(np.linalg.norm(o.astype(np.float64) - c, axis=1).max())
        th.append(random_poses(K, c, rb + 0.03, rng))
    pb.theta0 = np.ascontiguousarray(np.concatenate(th, 1))
    return pb, Settings(k_max=1, k_stein=1, w_pen=w_pen)


def grasp_prior(pb: Problem, sigma: float = 0.03, kappa: float = 5.0, sigma_n: float = 0.005) -> np.ndarray:
    """A prior per group (Sec. III-C names Gaussian translation and von Mises
    rotation priors without parameters): the translation mean places the
    contact cloud's centroid on the object's mean point from straight above,
    the rotation mean points the gripper down.  sigma (m) is the translation
    spread and kappa the von Mises concentration; both are expressed in the
    cost's units by the likelihood scale sigma_n (m): the cost C stands for
    sigma_n^2 times a negative log likelihood, so the stored weights are
    w_t = sigma_n^2 / sigma^2 and sigma_n^2 kappa."""
    out = np.zeros((pb.n_obj * pb.n_pre, 9), np.float32)
    for o in range(pb.n_obj):
        anchor = pb.R[pb.r_off[o]:pb.r_off[o + 1]].astype(np.float64).mean(0)
        for p in range(pb.n_pre):
            tip = pb.S[pb.s_off[p]:pb.s_off[p + 1]].astype(np.float64).mean(0)
            t, q = _look_at(np.array([0.0, 0.0, 1.0]), anchor, tip, 0.0)
            out[o * pb.n_pre + p] = np.concatenate([t, [sigma_n ** 2 / sigma ** 2], q,
                                                    [sigma_n ** 2 * kappa]])
    return out


def workload_tabletop(n_pre: int = 10, K: int = 30, m: int = 800, n: int = 96, grid_n: int = 64,
                      seed: int = 8, init: str = "quarter"):
    """The paper's simulation set-up (Sec. VI-A, Table I) at its own scale: a
    superquadric of m points resting on a table; the collision cloud C is the
    object plus a 5 mm table grid 2 cm beyond its footprint (about 1100-1900
    points in all); n_pre preshapes of a parallel gripper with finger gaps
    3-8 cm and n contact points each (5 mm spacing); per preshape K poses:
    K - 6 quarter-sphere Fibonacci poses facing the arm plus 6 from above
    (init="quarter"), or a mixture of four Gaussians around the up, arm-side
    and two lateral directions (init="gmm"); Table I settings (15 Stein + 25
    SGD iterations, cyclic annealing, mini-batch schedule)."""
    rng = np.random.default_rng(seed)
    obj = superquadric(m, rng, noise=0.001).astype(np.float64)
    obj[:, 2] -= obj[:, 2].min()  # resting on the table plane z = -2 mm
    obj = obj.astype(np.float32)
    table = table_plane(obj, 0.005, 0.02)
    gaps = np.linspace(0.03, 0.08, n_pre)
    pre = [gripper_contact_cloud(float(g), n, np.random.default_rng((seed, i))) for i, g in enumerate(gaps)]
    grids = [gripper_sdf_grid(float(g), grid_n, 0.002) for g in gaps]
    anchor = obj.astype(np.float64).mean(0)
    dist = standoff(obj)
    th = []
    for i, s in enumerate(pre):
        tip = s.astype(np.float64).mean(0)
        if init == "quarter":
            th.append(tabletop_poses(K, anchor, tip, dist))
        elif init == "gmm":
            means = [(0.0, 0.0, 1.0), (-1.0, 0.0, 0.3), (0.0, 1.0, 0.3), (0.0, -1.0, 0.3)]
            th.append(gmm_poses(K, anchor, tip, dist, means, 0.25, np.random.default_rng((seed, 100 + i))))
        else:
            raise ValueError(init)
    C = np.ascontiguousarray(np.concatenate([obj, table]).astype(np.float32))
    pb = Problem(R=np.ascontiguousarray(obj), r_off=np.array([0, len(obj)], np.int32),
                 C=C, c_off=np.array([0, len(C)], np.int32),
                 S=np.ascontiguousarray(np.concatenate(pre).astype(np.float32)),
                 s_off=np.cumsum([0] + [len(s) for s in pre]).astype(np.int32),
                 grids=grids, theta0=np.ascontiguousarray(np.concatenate(th, 1)), K=K)
    return pb, paper_settings()
