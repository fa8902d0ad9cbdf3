"""ctypes face of the FP64 CPU oracle (asicp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product package never imports it.

Inputs arrive as the float32 arrays the GPU receives (a synth.Problem) and
are widened exactly to float64 here; all arithmetic happens in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asicp_oracle.c")
_LIB = os.path.join(_HERE, "libasicp_oracle.so")
# A test may point the face at a library built from a deliberately altered copy
# of the source, to show that the pins catch the alteration.
_VARIANT = os.environ.get("ASICP_ORACLE_VARIANT_LIB")


def build(force: bool = False) -> str:
    """Compile the oracle with the system C compiler (plain -O2, OpenMP)."""
    if _VARIANT:
        return _VARIANT
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("n_obj", C.c_int32), ("n_pre", C.c_int32), ("K", C.c_int32),
                ("R", C.c_void_p), ("r_off", C.c_void_p), ("C", C.c_void_p), ("c_off", C.c_void_p),
                ("S", C.c_void_p), ("s_off", C.c_void_p), ("sdf", C.c_void_p),
                ("sdf_off", C.c_void_p), ("sdf_n", C.c_void_p), ("sdf_origin", C.c_void_p),
                ("sdf_cell", C.c_void_p), ("prior", C.c_void_p)]


class _Config(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("k_stein", C.c_int32), ("eta", C.c_double),
                ("lam", C.c_double), ("precond", C.c_int32), ("schedule", C.c_int32),
                ("T0", C.c_double), ("T1", C.c_double), ("cyc_C", C.c_double), ("cyc_p", C.c_double),
                ("kernel_mode", C.c_int32), ("bw_mode", C.c_int32), ("h_fixed", C.c_double),
                ("h_min", C.c_double), ("conv_tol", C.c_double), ("w_pen", C.c_double),
                ("minibatch", C.c_int32), ("seed", C.c_uint64)]


class _EvalOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("cost", "g_ct", "g_q", "ncol", "col_cost", "g_col",
                                          "g_fin", "nn_idx", "gate", "phi_c", "rev_idx", "pen")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp, i32, f64 = C.c_void_p, C.c_int32, C.c_double
        L.or_quat_to_rot.argtypes = [vp, vp]
        L.or_quat_mul.argtypes = [vp, vp, vp]
        L.or_quat_exp.argtypes = [vp, vp]
        L.or_nn_brute.argtypes = [vp, i32, vp, vp]
        L.or_nn_brute.restype = i32
        L.or_sdf_trilinear.argtypes = [vp, vp, vp, f64, vp, vp]
        L.or_sdf_trilinear.restype = f64
        L.or_sdf_trilinear_grad.argtypes = [vp, vp, vp, f64, vp, vp, vp]
        L.or_sdf_trilinear_grad.restype = f64
        L.or_setup.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.or_schedule.argtypes = [vp, i32, vp, vp]
        L.or_eval.argtypes = [vp, vp, i32, vp, vp]
        L.or_splitmix64.argtypes = [C.c_uint64]
        L.or_splitmix64.restype = C.c_uint64
        L.or_batch_size.argtypes = [vp, i32, C.c_int64]
        L.or_batch_size.restype = C.c_int64
        L.or_batch_perm.argtypes = [C.c_int64, C.c_int64, C.c_uint64]
        L.or_batch_perm.restype = C.c_int64
        L.or_batch_key.argtypes = [vp, i32, i32]
        L.or_batch_key.restype = C.c_uint64
        L.or_bandwidth.argtypes = [vp, i32, vp]
        L.or_bandwidth.restype = f64
        L.or_svgd_direction.argtypes = [vp, vp, i32, f64, f64, f64, f64, f64, i32, vp, vp]
        L.or_retract.argtypes = [vp, vp, vp]
        L.or_step.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp]
        L.or_step.restype = i32
        L.or_solve.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.or_solve.restype = i32
        L.or_select.argtypes = [vp, vp, vp, vp, vp]
        L.or_log_prior.argtypes = [vp, vp, vp]
        L.or_log_prior.restype = f64
        L.or_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def threads() -> int:
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Threads of the parallel loops from now on (results do not depend on it)."""
    lib().or_set_threads(int(n))


# ---------------------------------------------------------------------------
# small helpers (exposed for the pinning tests)
# ---------------------------------------------------------------------------

def quat_to_rot(q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float64)
    out = np.zeros(9)
    lib().or_quat_to_rot(_p(q), _p(out))
    return out.reshape(3, 3)


def quat_mul(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    out = np.zeros(4)
    lib().or_quat_mul(_p(a), _p(b), _p(out))
    return out


def quat_exp(v) -> np.ndarray:
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros(4)
    lib().or_quat_exp(_p(v), _p(out))
    return out


def nn_brute(points, x):
    pts = np.ascontiguousarray(points, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    d2 = np.zeros(1)
    j = lib().or_nn_brute(_p(pts), len(pts), _p(x), _p(d2))
    return int(j), float(d2[0])


def sdf_trilinear(grid, origin, cell, p):
    g = np.ascontiguousarray(grid, np.float64)
    n = np.array([g.shape[2], g.shape[1], g.shape[0]], np.int32)
    o = np.ascontiguousarray(origin, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    inside = np.zeros(1, np.int32)
    v = lib().or_sdf_trilinear(_p(g), _p(n), _p(o), float(cell), _p(p), _p(inside))
    return float(v), bool(inside[0])


def sdf_trilinear_grad(grid, origin, cell, p):
    g = np.ascontiguousarray(grid, np.float64)
    n = np.array([g.shape[2], g.shape[1], g.shape[0]], np.int32)
    o = np.ascontiguousarray(origin, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    inside = np.zeros(1, np.int32)
    grad = np.zeros(3)
    v = lib().or_sdf_trilinear_grad(_p(g), _p(n), _p(o), float(cell), _p(p), _p(inside), _p(grad))
    return float(v), bool(inside[0]), grad


def splitmix64(x: int) -> int:
    return int(lib().or_splitmix64(x & 0xFFFFFFFFFFFFFFFF))


def batch_size(settings, k, M) -> int:
    cfg = _config(settings)
    return int(lib().or_batch_size(C.byref(cfg), int(k), int(M)))


def batch_key(settings, k, o) -> int:
    cfg = _config(settings)
    return int(lib().or_batch_key(C.byref(cfg), int(k), int(o)))


def batch_perm(j, M, key) -> int:
    return int(lib().or_batch_perm(int(j), int(M), int(key)))


def log_prior(prior9, theta7):
    """Log prior of one pose (up to a constant) and its (t, w) gradient."""
    pr = np.ascontiguousarray(prior9, np.float64)
    th = np.ascontiguousarray(theta7, np.float64)
    g = np.zeros(6)
    v = lib().or_log_prior(_p(pr), _p(th), _p(g))
    return float(v), g


def bandwidth(theta_aos, settings) -> float:
    th = np.ascontiguousarray(theta_aos, np.float64)
    cfg = _config(settings)
    return float(lib().or_bandwidth(_p(th), len(th), C.byref(cfg)))


def svgd_direction(theta_aos, g, h, gamma, tau, a_t, a_w, kernel_mode=0):
    th = np.ascontiguousarray(theta_aos, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    K = len(th)
    kmat = np.zeros((K, K))
    phi = np.zeros((K, 6))
    lib().or_svgd_direction(_p(th), _p(g), K, h, gamma, tau, a_t, a_w, kernel_mode, _p(kmat), _p(phi))
    return phi, kmat


def retract(theta7, dt, dw) -> np.ndarray:
    th = np.array(theta7, np.float64)
    dt = np.ascontiguousarray(dt, np.float64)
    dw = np.ascontiguousarray(dw, np.float64)
    lib().or_retract(_p(th), _p(dt), _p(dw))
    return th


def _config(st) -> _Config:
    return _Config(int(st.k_max), int(st.k_stein), float(st.eta), float(st.lam), int(st.precond),
                   int(st.schedule), float(st.T0), float(st.T1), float(st.cyc_C), float(st.cyc_p),
                   int(st.kernel_mode), int(st.bw_mode), float(st.h_fixed), float(st.h_min),
                   float(st.conv_tol), float(getattr(st, "w_pen", 0.0)),
                   int(getattr(st, "minibatch", 0)), int(getattr(st, "seed", 0)))


def schedule(settings, k):
    cfg = _config(settings)
    g = np.zeros(1)
    t = np.zeros(1)
    lib().or_schedule(C.byref(cfg), int(k), _p(g), _p(t))
    return float(g[0]), float(t[0])


# ---------------------------------------------------------------------------
# whole-problem calls
# ---------------------------------------------------------------------------

class Oracle:
    """FP64 oracle bound to one synth.Problem and its Settings."""

    def __init__(self, pb, settings):
        self.pb = pb
        self.settings = settings
        self._keep = []
        keep = self._keep.append

        def arr(a, dt):
            a = np.ascontiguousarray(a, dt)
            keep(a)
            return a.ctypes.data

        grids = pb.grids
        sdf = np.concatenate([g.values.astype(np.float64).ravel() for g in grids])
        sizes = [g.values.size for g in grids]
        sdf_off = np.cumsum([0] + sizes[:-1]).astype(np.int64)
        sdf_n = np.array([[g.values.shape[2], g.values.shape[1], g.values.shape[0]] for g in grids],
                         np.int32).ravel()
        sdf_origin = np.array([g.origin for g in grids], np.float64).ravel()
        sdf_cell = np.array([g.cell for g in grids], np.float64)
        self.n_pre = pb.n_pre
        self.n_obj = pb.n_obj
        self.K = pb.K
        self.k_tot = pb.k_tot
        self.n_max = int(np.max(np.diff(pb.s_off)))
        self.mc_max = int(np.max(np.diff(pb.c_off)))
        self._pb = _Problem(pb.n_obj, pb.n_pre, pb.K, arr(pb.R, np.float64), arr(pb.r_off, np.int32),
                            arr(pb.C, np.float64), arr(pb.c_off, np.int32), arr(pb.S, np.float64),
                            arr(pb.s_off, np.int32), arr(sdf, np.float64), arr(sdf_off, np.int64),
                            arr(sdf_n, np.int32), arr(sdf_origin, np.float64), arr(sdf_cell, np.float64),
                            None if getattr(pb, "prior", None) is None else arr(pb.prior, np.float64))
        self._cfg = _config(settings)

    def setup(self):
        com = np.zeros((self.n_obj, 3))
        tcp = np.zeros((self.n_pre, 3))
        rho2 = np.zeros(self.n_pre)
        a_t = np.zeros(self.n_pre)
        a_w = np.zeros(self.n_pre)
        lib().or_setup(C.byref(self._pb), C.byref(self._cfg), _p(com), _p(tcp), _p(rho2), _p(a_t), _p(a_w))
        return dict(com=com, tcp=tcp, rho2=rho2, a_t=a_t, a_w=a_w)

    def _alloc_eval(self, full: bool):
        K = self.k_tot
        d = dict(cost=np.zeros(K), g_ct=np.zeros((K, 6)), g_q=np.zeros((K, 4)),
                 ncol=np.zeros(K, np.int32), col_cost=np.zeros(K), g_col=np.zeros((K, 6)),
                 g_fin=np.zeros((K, 6)), pen=np.zeros(K))
        if full:
            d.update(nn_idx=np.full((K, self.n_max), -1, np.int32),
                     gate=np.zeros((K, self.mc_max), np.uint8),
                     phi_c=np.zeros((K, self.mc_max)),
                     rev_idx=np.full((K, self.mc_max), -1, np.int32))
        out = _EvalOut(*[_p(d.get(n)) for n, _ in _EvalOut._fields_])
        return d, out

    @staticmethod
    def aos(theta_soa) -> np.ndarray:
        """(7, Ktot) SoA pose array (any float type) -> (Ktot, 7) float64, always
        a fresh copy (the C calls update poses in place)."""
        return np.array(np.asarray(theta_soa, np.float64).T, order="C", copy=True)

    def evaluate(self, theta_soa, full: bool = True, k=None) -> dict:
        """Evaluation at poses theta; k selects the iteration's mini-batch
        (default k_max: the whole cloud)."""
        th = self.aos(theta_soa)
        d, out = self._alloc_eval(full)
        k = self.settings.k_max if k is None else k
        lib().or_eval(C.byref(self._pb), C.byref(self._cfg), int(k), _p(th), C.byref(out))
        return d

    def step(self, k, theta_soa, prev_cost=None, converged=None, full: bool = False) -> dict:
        """One iteration from the given state; returns the evaluation, h per
        group, phi per particle and the next state (theta as (7, Ktot))."""
        th = self.aos(theta_soa)
        pc = np.full(self.k_tot, -1.0) if prev_cost is None else np.array(prev_cost, np.float64)
        cv = np.zeros(self.k_tot, np.int32) if converged is None else np.array(converged, np.int32)
        d, out = self._alloc_eval(full)
        h = np.zeros(self.n_obj * self.n_pre)
        phi = np.zeros((self.k_tot, 6))
        lib().or_step(C.byref(self._pb), C.byref(self._cfg), int(k), _p(th), _p(pc), _p(cv),
                      C.byref(out), _p(h), _p(phi))
        d.update(h=h, phi=phi, theta=np.ascontiguousarray(th.T), prev_cost=pc, converged=cv)
        return d

    def solve(self, theta_soa=None, k_start=0, k_end=None, prev_cost=None, converged=None) -> dict:
        th = self.aos(self.pb.theta0 if theta_soa is None else theta_soa)
        k_end = self.settings.k_max if k_end is None else k_end
        pc = np.full(self.k_tot, -1.0) if prev_cost is None else np.array(prev_cost, np.float64)
        cv = np.zeros(self.k_tot, np.int32) if converged is None else np.array(converged, np.int32)
        d, out = self._alloc_eval(False)
        best = np.zeros(self.n_obj, np.int32)
        free = np.zeros(self.n_obj, np.int32)
        it = lib().or_solve(C.byref(self._pb), C.byref(self._cfg), int(k_start), int(k_end), _p(th),
                            _p(pc), _p(cv), C.byref(out), _p(best), _p(free))
        d.update(theta=np.ascontiguousarray(th.T), prev_cost=pc, converged=cv, best=best,
                 best_free=free, iters=int(it))
        return d
