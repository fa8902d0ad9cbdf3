"""FP64 oracle of the learned grasp proposal (test infrastructure only).

A point-cloud encoder in the style of PointNet (the paper points to learned
priors and data-driven seeding as ways to need fewer initialisations,
Sec. V, the ablation, and Sec. VII) maps an object cloud to S seed poses per
preshape, which then start the AS-ICP iteration of Algorithm 1:

  x_m   = (r_m - mean(r)) / 0.1                       centred, 10 cm units
  h1_m  = relu(W1 x_m + b1)            3 -> 64
  h2_m  = relu(W2 h1_m + b2)          64 -> 128
  h3_m  = relu(W3 h2_m + b3)         128 -> 256
  g     = max_m h3_m                   channel-wise, lowest m on ties
  u     = relu(W4 g + b4)            256 -> 256
  v     = relu(W5 u + b5)            256 -> 256
  o     = W6 v + b6                  256 -> P * S * 7
  seed (p, s): t = mean(r) + 0.1 o[0:3], q = o[3:7] / |o[3:7]|

Set loss per (object, preshape) against T target poses (t_g, q_g):
  d(a, g) = |t_a - t_g|^2 / 0.01 + beta (1 - (q_a . q_g)^2)
  L = (1/T) sum_g min_a d(a, g) + (1/S) sum_a min_g d(a, g)
(a symmetric Chamfer distance; 1 - (q.q')^2 is blind to the sign of q.)
The object's loss is the mean over preshapes.

With bf16=True the operands the kernel feeds to its BF16 matrix products
(h1, h2 and W2, W3) are rounded to BF16 (round to nearest even) before the
products; everything else stays FP64.

Parameters are one flat array in the order W1 (64x3), b1, W2 (128x64), b2,
W3 (256x128), b3, W4 (256x256), b4, W5 (256x256), b5, W6 (O x 256), b6,
matrices row-major (output index first).
"""
import numpy as np

H1, H2, H3, HH = 64, 128, 256, 256
UNIT = 0.1
BETA = 1.0


def layer_shapes(n_pre, n_seed):
    O = n_pre * n_seed * 7
    return [(H1, 3), (H1,), (H2, H1), (H2,), (H3, H2), (H3,), (HH, H3), (HH,), (HH, HH), (HH,), (O, HH), (O,)]


def n_params(n_pre, n_seed):
    return int(sum(np.prod(s) for s in layer_shapes(n_pre, n_seed)))


def unpack(params, n_pre, n_seed):
    out, o = [], 0
    for s in layer_shapes(n_pre, n_seed):
        n = int(np.prod(s))
        out.append(np.asarray(params[o:o + n], np.float64).reshape(s))
        o += n
    return out


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, cloud, n_pre, n_seed, bf=False):
    """One object: returns the raw outputs o (P*S*7) and the intermediates."""
    W1, b1, W2, b2, W3, b3, W4, b4, W5, b5, W6, b6 = unpack(params, n_pre, n_seed)
    r = np.asarray(cloud, np.float64)
    com = r.mean(0)
    x = (r - com) / UNIT
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    A1, B2 = (bf16(h1), bf16(W2)) if bf else (h1, W2)
    z2 = A1 @ B2.T + b2
    h2 = np.maximum(z2, 0.0)
    A2, B3 = (bf16(h2), bf16(W3)) if bf else (h2, W3)
    z3 = A2 @ B3.T + b3
    h3 = np.maximum(z3, 0.0)
    am = np.argmax(h3, axis=0)  # first index of the maximum
    g = h3[am, np.arange(H3)]
    zu = W4 @ g + b4
    u = np.maximum(zu, 0.0)
    zv = W5 @ u + b5
    v = np.maximum(zv, 0.0)
    o = W6 @ v + b6
    return o, dict(com=com, x=x, z1=z1, h1=h1, A1=A1, z2=z2, h2=h2, A2=A2, z3=z3, h3=h3, am=am, g=g,
                   zu=zu, u=u, zv=zv, v=v)


def seeds(o, com, n_pre, n_seed):
    """Raw outputs -> (P, S, 7) poses (t, unit q with q_w >= 0)."""
    a = o.reshape(n_pre, n_seed, 7)
    t = com + UNIT * a[..., :3]
    q = a[..., 3:] / np.linalg.norm(a[..., 3:], axis=-1, keepdims=True)
    q = np.where(q[..., :1] < 0, -q, q)
    return np.concatenate([t, q], -1)


def loss(o, com, targets, n_pre, n_seed, beta=BETA):
    """Set loss of one object and its gradient with respect to o.
    targets: (P, T, 7) poses (t, unit q)."""
    a = o.reshape(n_pre, n_seed, 7)
    tg = np.asarray(targets, np.float64)
    T = tg.shape[1]
    L = 0.0
    do = np.zeros_like(a)
    for p in range(n_pre):
        ta = com + UNIT * a[p, :, :3]
        qr = a[p, :, 3:]
        nq = np.linalg.norm(qr, axis=1)
        qa = qr / nq[:, None]
        dt = ta[:, None, :] - tg[p][None, :, :3]          # (S, T, 3)
        c = qa @ tg[p][:, 3:].T                          # (S, T)
        D = (dt ** 2).sum(-1) / (UNIT * UNIT) + beta * (1.0 - c * c)
        ga = np.argmin(D, axis=0)   # per target, nearest seed (lowest index)
        sa = np.argmin(D, axis=1)   # per seed, nearest target
        L += D[ga, np.arange(T)].mean() + D[np.arange(n_seed), sa].mean()
        w = np.zeros((n_seed, T))
        np.add.at(w, (ga, np.arange(T)), 1.0 / T)
        np.add.at(w, (np.arange(n_seed), sa), 1.0 / n_seed)
        # dD/dt_a = 2 dt / UNIT^2, dt_a/do = UNIT
        dta = (w[..., None] * 2.0 * dt / (UNIT * UNIT)).sum(1) * UNIT
        # dD/dq_a(raw) = -2 beta c (q_g - c q_a) / |q_raw|
        dqa = (w[..., None] * (-2.0 * beta * c[..., None]) *
               (tg[p][None, :, 3:] - c[..., None] * qa[:, None, :])).sum(1) / nq[:, None]
        do[p, :, :3] = dta
        do[p, :, 3:] = dqa
    return L / n_pre, do.reshape(-1) / n_pre


def backward(params, inter, do, n_pre, n_seed, bf=False):
    """Gradient of the loss with respect to the flat parameters, given
    dL/do; the max-pool routes each channel's gradient to its argmax point."""
    W1, b1, W2, b2, W3, b3, W4, b4, W5, b5, W6, b6 = unpack(params, n_pre, n_seed)
    I = inter
    dW6 = np.outer(do, I["v"]); db6 = do.copy()
    dv = W6.T @ do
    dzv = dv * (I["zv"] > 0)
    dW5 = np.outer(dzv, I["u"]); db5 = dzv
    du = W5.T @ dzv
    dzu = du * (I["zu"] > 0)
    dW4 = np.outer(dzu, I["g"]); db4 = dzu
    dg = W4.T @ dzu
    M = I["x"].shape[0]
    dh3 = np.zeros((M, H3))
    dh3[I["am"], np.arange(H3)] = dg
    dz3 = dh3 * (I["z3"] > 0)
    B3 = bf16(W3) if bf else W3
    dW3 = dz3.T @ I["A2"]; db3 = dz3.sum(0)
    dh2 = dz3 @ B3
    dz2 = dh2 * (I["z2"] > 0)
    B2 = bf16(W2) if bf else W2
    dW2 = dz2.T @ I["A1"]; db2 = dz2.sum(0)
    dh1 = dz2 @ B2
    dz1 = dh1 * (I["z1"] > 0)
    dW1 = dz1.T @ I["x"]; db1 = dz1.sum(0)
    return np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3, dW4, db4, dW5, db5, dW6, db6)])


def init_params(n_pre, n_seed, rng):
    """He-style random weights, zero biases, a small output layer (for tests)."""
    ps = []
    for s in layer_shapes(n_pre, n_seed):
        if len(s) == 2:
            ps.append(rng.standard_normal(s) * np.sqrt(2.0 / s[1]))
        else:
            ps.append(np.zeros(s))
    ps[-2] *= 0.01
    return np.concatenate([p.ravel() for p in ps])
