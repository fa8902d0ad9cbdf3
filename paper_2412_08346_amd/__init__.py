"""MI355X-native batched Annealed Stein ICP (arXiv 2412.08346).

Thin Python face of libasicp.so (C ABI in include/asicp.h).  The functions
named asicp_* marshal arguments to the C calls of the same name; `Solver`
packs a synth.Problem into torch device tensors and drives them.  Every step
of the iteration runs in the library's HIP kernels; nothing here computes
any part of the method, and there is no CPU fallback: if the library is
missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasicp.so")

ASICP_OK, ASICP_E_INVALID, ASICP_E_STATE, ASICP_E_HIP, ASICP_E_NUMERIC, ASICP_E_HOST = 0, -1, -2, -3, -4, -5
ASICP_FLAG_DEBUG, ASICP_FLAG_TIMING, ASICP_FLAG_NO_PRUNE = 1, 2, 4

EXPORTS = ("asicp_workspace_bytes", "asicp_create", "asicp_step", "asicp_solve", "asicp_replay",
           "asicp_cost_grad", "asicp_result", "asicp_kernel_time", "asicp_get_launch",
           "asicp_set_launch", "asicp_autotune", "asicp_destroy", "asicp_last_error",
           "asicp_pn_param_count", "asicp_pn_workspace_bytes", "asicp_pn_forward",
           "asicp_pn_loss_grad", "asicp_pn_adam", "asicp_pn_last_error", "asicp_pn_forward_noalloc",
           "asicp_pose_vjp", "asicp_reset")
ASICP_GRAD_TANGENT, ASICP_GRAD_POSE = 0, 1


class AsicpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"asicp status {status}: {msg}")
        self.status = status


class asicp_sdf(C.Structure):
    _fields_ = [("values", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("origin", C.c_float * 3), ("cell", C.c_float)]


class asicp_problem(C.Structure):
    _fields_ = [("n_objects", C.c_int32), ("n_preshapes", C.c_int32),
                ("particles_per_group", C.c_int32),
                ("rx", C.c_void_p), ("ry", C.c_void_p), ("rz", C.c_void_p), ("r_off", C.c_void_p),
                ("cx", C.c_void_p), ("cy", C.c_void_p), ("cz", C.c_void_p), ("c_off", C.c_void_p),
                ("sx", C.c_void_p), ("sy", C.c_void_p), ("sz", C.c_void_p), ("s_off", C.c_void_p),
                ("sdf", C.c_void_p), ("theta0", C.c_void_p), ("prev_cost", C.c_void_p),
                ("converged", C.c_void_p), ("k_start", C.c_int32), ("prior", C.c_void_p)]


class asicp_config(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("k_stein", C.c_int32), ("eta", C.c_float),
                ("lambda_", C.c_float), ("precond", C.c_int32), ("schedule", C.c_int32),
                ("T0", C.c_float), ("T1", C.c_float), ("cyc_C", C.c_float), ("cyc_p", C.c_float),
                ("kernel_mode", C.c_int32), ("bw_mode", C.c_int32), ("h_fixed", C.c_float),
                ("h_min", C.c_float), ("conv_tol", C.c_float), ("w_pen", C.c_float),
                ("minibatch", C.c_int32), ("seed", C.c_uint64), ("flags", C.c_uint32)]


class asicp_launch_t(C.Structure):
    _fields_ = [("xcd_map", C.c_int32), ("fine", C.c_int32), ("query_blocks", C.c_int32),
                ("chunk_points", C.c_int32)]


ASICP_LAUNCH_CHOICES = 24


def launch_index(xcd_map: int, fine: int, query_blocks: int = 4, chunk_points: int = 128) -> int:
    """Index of a launch choice in asicp_autotune's timings (asicp.h)."""
    qi = {1: 0, 2: 1, 4: 2}[int(query_blocks)]
    return ((qi * 2 + (int(chunk_points) == 128)) * 2 + int(xcd_map)) * 2 + int(fine)


def launch_choice(v: int) -> dict:
    """The launch choice with index v (inverse of launch_index)."""
    return {"xcd_map": (v >> 1) & 1, "fine": v & 1, "query_blocks": 1 << (v >> 3),
            "chunk_points": 128 if (v >> 2) & 1 else 64}


class asicp_result_t(C.Structure):
    _fields_ = [("best_particle", C.c_void_p), ("best_free", C.c_void_p), ("best_theta", C.c_void_p),
                ("best_cost", C.c_void_p), ("iterations_done", C.c_int32),
                ("final_evaluated", C.c_int32)] + [
                   (n, C.c_void_p) for n in ("theta", "cost", "col_cost", "ncol", "converged",
                                             "prev_cost", "grad", "grad_ct", "grad_col", "phi", "h",
                                             "nn_idx", "rev_idx")]


_lib = None


def load():
    """Load libasicp.so (built by build_lib); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2412_08346_amd.build_lib` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.asicp_workspace_bytes.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.asicp_workspace_bytes.restype = i32
        L.asicp_create.argtypes = [vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.asicp_create.restype = i32
        L.asicp_reset.argtypes = [vp, vp]
        L.asicp_reset.restype = i32
        L.asicp_step.argtypes = [vp, i32, vp]
        L.asicp_step.restype = i32
        L.asicp_solve.argtypes = [vp, vp]
        L.asicp_solve.restype = i32
        L.asicp_cost_grad.argtypes = [vp, vp, vp, vp, i32, vp]
        L.asicp_cost_grad.restype = i32
        L.asicp_pose_vjp.argtypes = [vp, vp, vp, i32, vp]
        L.asicp_pose_vjp.restype = i32
        L.asicp_replay.argtypes = [vp, vp]
        L.asicp_replay.restype = i32
        L.asicp_result.argtypes = [vp, vp, vp]
        L.asicp_result.restype = i32
        L.asicp_kernel_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i32), C.POINTER(C.c_double)]
        L.asicp_kernel_time.restype = i32
        L.asicp_get_launch.argtypes = [vp, vp]
        L.asicp_get_launch.restype = i32
        L.asicp_set_launch.argtypes = [vp, vp]
        L.asicp_set_launch.restype = i32
        L.asicp_autotune.argtypes = [vp, i32, vp, vp, vp]
        L.asicp_autotune.restype = i32
        L.asicp_pn_param_count.argtypes = [i32, i32]
        L.asicp_pn_param_count.restype = C.c_int64
        L.asicp_pn_workspace_bytes.argtypes = [i32, i32, i32, C.POINTER(C.c_size_t)]
        L.asicp_pn_workspace_bytes.restype = i32
        L.asicp_pn_forward.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, C.c_float, vp, vp, vp, C.c_size_t, vp]
        L.asicp_pn_forward.restype = i32
        L.asicp_pn_forward_noalloc.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, C.c_float, vp, vp, vp]
        L.asicp_pn_forward_noalloc.restype = i32
        L.asicp_pn_loss_grad.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, C.c_size_t, vp]
        L.asicp_pn_loss_grad.restype = i32
        L.asicp_pn_adam.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                    i32, vp]
        L.asicp_pn_adam.restype = i32
        L.asicp_pn_last_error.argtypes = []
        L.asicp_pn_last_error.restype = C.c_char_p
        L.asicp_destroy.argtypes = [vp]
        L.asicp_destroy.restype = None
        L.asicp_last_error.argtypes = []
        L.asicp_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def asicp_last_error() -> str:
    return load().asicp_last_error().decode()


def _check(st):
    if st != ASICP_OK:
        raise AsicpError(st, asicp_last_error())
    return st


def asicp_workspace_bytes(pb: asicp_problem, cfg: asicp_config) -> int:
    n = C.c_size_t(0)
    _check(load().asicp_workspace_bytes(C.byref(pb), C.byref(cfg), C.byref(n)))
    return int(n.value)


def asicp_create(pb, cfg, workspace_ptr: int, workspace_bytes: int, stream: int):
    ctx = C.c_void_p()
    _check(load().asicp_create(C.byref(pb), C.byref(cfg), C.c_void_p(workspace_ptr), workspace_bytes,
                               C.c_void_p(stream), C.byref(ctx)))
    return ctx


def asicp_reset(ctx, stream: int):
    return _check(load().asicp_reset(ctx, C.c_void_p(stream)))


def asicp_step(ctx, n_iters: int, stream: int):
    return _check(load().asicp_step(ctx, int(n_iters), C.c_void_p(stream)))


def asicp_solve(ctx, stream: int):
    return _check(load().asicp_solve(ctx, C.c_void_p(stream)))


def asicp_cost_grad(ctx, theta_ptr: int, cost_ptr, grad_ptr, stream: int, grad_form: int = ASICP_GRAD_TANGENT):
    return _check(load().asicp_cost_grad(ctx, C.c_void_p(theta_ptr), C.c_void_p(cost_ptr),
                                         C.c_void_p(grad_ptr), int(grad_form), C.c_void_p(stream)))


def asicp_pose_vjp(grad_ptr: int, gout_ptr: int, dtheta_ptr: int, ktot: int, stream: int):
    return _check(load().asicp_pose_vjp(C.c_void_p(grad_ptr), C.c_void_p(gout_ptr), C.c_void_p(dtheta_ptr),
                                        int(ktot), C.c_void_p(stream)))


def asicp_replay(ctx, stream: int):
    return _check(load().asicp_replay(ctx, C.c_void_p(stream)))


def asicp_result(ctx, out: asicp_result_t, stream: int, check: bool = True):
    st = load().asicp_result(ctx, C.byref(out), C.c_void_p(stream))
    return _check(st) if check else st


def asicp_kernel_time(ctx):
    """(total ms, launches, distance evaluations) of the forward-NN launches."""
    ms = C.c_double(0.0)
    n = C.c_int32(0)
    pairs = C.c_double(0.0)
    _check(load().asicp_kernel_time(ctx, C.byref(ms), C.byref(n), C.byref(pairs)))
    return float(ms.value), int(n.value), float(pairs.value)


def _launch_dict(out) -> dict:
    return {"xcd_map": int(out.xcd_map), "fine": int(out.fine), "query_blocks": int(out.query_blocks),
            "chunk_points": int(out.chunk_points)}


def asicp_get_launch(ctx) -> dict:
    out = asicp_launch_t()
    _check(load().asicp_get_launch(ctx, C.byref(out)))
    return _launch_dict(out)


def asicp_set_launch(ctx, xcd_map: int, fine: int, query_blocks: int = 4, chunk_points: int = 128):
    return _check(load().asicp_set_launch(
        ctx, C.byref(asicp_launch_t(int(xcd_map), int(fine), int(query_blocks), int(chunk_points)))))


def asicp_autotune(ctx, reps: int, stream: int):
    """Time every launch choice; returns (chosen dict, ms per evaluation of
    each choice, indexed as launch_index)."""
    out = asicp_launch_t()
    ms = (C.c_float * ASICP_LAUNCH_CHOICES)()
    _check(load().asicp_autotune(ctx, int(reps), C.c_void_p(stream), C.byref(out), ms))
    return _launch_dict(out), [float(v) for v in ms]


def asicp_destroy(ctx):
    load().asicp_destroy(ctx)


def _pn_check(st):
    if st != ASICP_OK:
        raise AsicpError(st, load().asicp_pn_last_error().decode())
    return st


def asicp_pn_param_count(n_pre: int, n_seed: int) -> int:
    n = int(load().asicp_pn_param_count(int(n_pre), int(n_seed)))
    if n < 0:
        raise AsicpError(ASICP_E_INVALID, "n_pre * n_seed * 7 must be in 7..1024")
    return n


def asicp_pn_workspace_bytes(n_obj: int, n_pre: int, n_seed: int) -> int:
    out = C.c_size_t(0)
    _pn_check(load().asicp_pn_workspace_bytes(int(n_obj), int(n_pre), int(n_seed), C.byref(out)))
    return int(out.value)


def asicp_pn_forward(params, n_pre, n_seed, n_obj, off, x, y, z, retract, seeds, raw, ws, ws_bytes, stream):
    return _pn_check(load().asicp_pn_forward(params, int(n_pre), int(n_seed), int(n_obj), off, x, y, z,
                                             float(retract), seeds, raw, ws, int(ws_bytes), C.c_void_p(stream)))


def asicp_pn_forward_noalloc(params, n_pre, n_seed, n_obj, off, x, y, z, retract, seeds, raw, stream):
    return _pn_check(load().asicp_pn_forward_noalloc(params, int(n_pre), int(n_seed), int(n_obj), off, x, y, z,
                                                     float(retract), seeds, raw, C.c_void_p(stream)))


def asicp_pn_loss_grad(params, n_pre, n_seed, n_obj, off, x, y, z, targets, n_targets, loss, grad, ws,
                       ws_bytes, stream):
    return _pn_check(load().asicp_pn_loss_grad(params, int(n_pre), int(n_seed), int(n_obj), off, x, y, z,
                                               targets, int(n_targets), loss, grad, ws, int(ws_bytes),
                                               C.c_void_p(stream)))


def asicp_pn_adam(params, m, v, grad, count, lr, beta1, beta2, eps, step, stream):
    return _pn_check(load().asicp_pn_adam(params, m, v, grad, int(count), float(lr), float(beta1),
                                          float(beta2), float(eps), int(step), C.c_void_p(stream)))


def make_config(st: "synth.Settings", flags: int = 0) -> asicp_config:
    return asicp_config(int(st.k_max), int(st.k_stein), float(st.eta), float(st.lam), int(st.precond),
                        int(st.schedule), float(st.T0), float(st.T1), float(st.cyc_C), float(st.cyc_p),
                        int(st.kernel_mode), int(st.bw_mode), float(st.h_fixed), float(st.h_min),
                        float(st.conv_tol), float(getattr(st, "w_pen", 0.0)),
                        int(getattr(st, "minibatch", 0)), int(getattr(st, "seed", 0)), int(flags))


class Solver:
    """One batch on the current HIP device: uploads a synth.Problem, owns the
    workspace and the context.  All methods enqueue on torch's current stream
    (or `stream`), like the C calls."""

    def __init__(self, pb: "synth.Problem", st: "synth.Settings", debug: bool = False,
                 timing: bool = False, theta0=None, k_start: int = 0, prev_cost=None,
                 converged=None, device: str = "cuda", stream=None, prune: bool = True):
        import torch

        load()
        self.torch = torch
        self.pb, self.st = pb, st
        self.dev = torch.device(device)
        dv = self.dev

        def f32(a):
            return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dv)

        R, Cc, S = np.asarray(pb.R, np.float32), np.asarray(pb.C, np.float32), np.asarray(pb.S, np.float32)
        self._keep = dict(
            rx=f32(R[:, 0]), ry=f32(R[:, 1]), rz=f32(R[:, 2]),
            sx=f32(S[:, 0]), sy=f32(S[:, 1]), sz=f32(S[:, 2]),
            grids=[f32(g.values) for g in pb.grids])
        if Cc is R or (Cc.shape == R.shape and np.array_equal(Cc, R) and np.array_equal(pb.c_off, pb.r_off)):
            cx, cy, cz = self._keep["rx"], self._keep["ry"], self._keep["rz"]
        else:
            cx, cy, cz = f32(Cc[:, 0]), f32(Cc[:, 1]), f32(Cc[:, 2])
        self._keep.update(cx=cx, cy=cy, cz=cz)
        th0 = pb.theta0 if theta0 is None else theta0
        self._keep["theta0"] = th0.to(dv).float().contiguous() if isinstance(th0, torch.Tensor) else f32(th0)
        if prev_cost is not None:
            self._keep["prev_cost"] = f32(prev_cost)
        if converged is not None:
            self._keep["converged"] = torch.as_tensor(np.asarray(converged, np.int32)).to(dv)
        self._offs = dict(r=np.ascontiguousarray(pb.r_off, np.int32), c=np.ascontiguousarray(pb.c_off, np.int32),
                          s=np.ascontiguousarray(pb.s_off, np.int32))
        pr = getattr(pb, "prior", None)
        self._prior = None if pr is None else np.ascontiguousarray(pr, np.float32).reshape(-1, 9)
        sdfs = (asicp_sdf * pb.n_pre)()
        for p, g in enumerate(pb.grids):
            nz, ny, nx = g.values.shape
            sdfs[p] = asicp_sdf(self._keep["grids"][p].data_ptr(), nx, ny, nz,
                                (C.c_float * 3)(*[float(v) for v in g.origin]), float(g.cell))
        self._sdfs = sdfs
        k = self._keep
        self.problem = asicp_problem(
            pb.n_obj, pb.n_pre, pb.K, k["rx"].data_ptr(), k["ry"].data_ptr(), k["rz"].data_ptr(),
            self._offs["r"].ctypes.data, k["cx"].data_ptr(), k["cy"].data_ptr(), k["cz"].data_ptr(),
            self._offs["c"].ctypes.data, k["sx"].data_ptr(), k["sy"].data_ptr(), k["sz"].data_ptr(),
            self._offs["s"].ctypes.data, C.cast(sdfs, C.c_void_p).value, k["theta0"].data_ptr(),
            k["prev_cost"].data_ptr() if "prev_cost" in k else None,
            k["converged"].data_ptr() if "converged" in k else None, int(k_start),
            self._prior.ctypes.data if self._prior is not None else None)
        flags = ((ASICP_FLAG_DEBUG if debug else 0) | (ASICP_FLAG_TIMING if timing else 0) |
                 (0 if prune else ASICP_FLAG_NO_PRUNE))
        self.config = make_config(st, flags)
        self.ws_bytes = asicp_workspace_bytes(self.problem, self.config)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dv)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ctx = asicp_create(self.problem, self.config, self._ws_ptr, self.ws_bytes, self._stream(stream))
        self.k_tot, self.G = pb.k_tot, pb.n_obj * pb.n_pre
        self.n_max = int(np.max(np.diff(pb.s_off)))
        self.mc_max = max(1, int(np.max(np.diff(pb.c_off))))
        self.debug = debug

    def _stream(self, stream):
        if stream is None:
            return self.torch.cuda.current_stream(self.dev).cuda_stream
        return int(stream)

    def reset(self, stream=None):
        """Start the solve again from the initial poses on the same context
        (asicp_reset: the set-up kernels run again; the launch choice, the
        captured graph and the timing records are kept)."""
        asicp_reset(self.ctx, self._stream(stream))

    def step(self, n: int = 1, stream=None):
        asicp_step(self.ctx, n, self._stream(stream))

    def solve(self, stream=None):
        asicp_solve(self.ctx, self._stream(stream))

    def cost_grad(self, theta, stream=None, pose: bool = False):
        """Cost and gradient per particle at poses `theta` (7, Ktot) on the
        device (the adjoint of the cost; pairs and gates held at theta): the
        6-D tangent gradient (6, Ktot), or with `pose` the gradient with
        respect to the 7 pose numbers (7, Ktot)."""
        torch = self.torch
        th = torch.as_tensor(theta, dtype=torch.float32, device=self.dev).contiguous()
        cost = torch.empty(self.k_tot, device=self.dev)
        grad = torch.empty((7 if pose else 6, self.k_tot), device=self.dev)
        asicp_cost_grad(self.ctx, th.data_ptr(), cost.data_ptr(), grad.data_ptr(), self._stream(stream),
                        ASICP_GRAD_POSE if pose else ASICP_GRAD_TANGENT)
        return cost, grad

    def replay(self, stream=None):
        asicp_replay(self.ctx, self._stream(stream))

    def result(self, per_particle: bool = True, stream=None, check: bool = True) -> dict:
        torch = self.torch
        dv = self.dev
        n_obj = self.pb.n_obj
        host = dict(best_particle=np.zeros(n_obj, np.int32), best_free=np.zeros(n_obj, np.int32),
                    best_theta=np.zeros((n_obj, 7), np.float32), best_cost=np.zeros(n_obj, np.float32))
        out = asicp_result_t()
        for n, a in host.items():
            setattr(out, n, a.ctypes.data)
        dev = {}
        if per_particle:
            K, G = self.k_tot, self.G
            dev = dict(theta=torch.empty((7, K), device=dv), cost=torch.empty(K, device=dv),
                       col_cost=torch.empty(K, device=dv), ncol=torch.empty(K, dtype=torch.int32, device=dv),
                       converged=torch.empty(K, dtype=torch.int32, device=dv),
                       prev_cost=torch.empty(K, device=dv), grad=torch.empty((6, K), device=dv),
                       grad_ct=torch.empty((6, K), device=dv), grad_col=torch.empty((6, K), device=dv),
                       phi=torch.empty((6, K), device=dv), h=torch.empty(G, device=dv))
            if self.debug:
                dev["nn_idx"] = torch.empty((K, self.n_max), dtype=torch.int32, device=dv)
                dev["rev_idx"] = torch.empty((K, self.mc_max), dtype=torch.int32, device=dv)
            for n, t in dev.items():
                setattr(out, n, t.data_ptr())
        st = asicp_result(self.ctx, out, self._stream(stream), check=check)
        res = {n: a for n, a in host.items()}
        res.update({n: t.cpu().numpy() for n, t in dev.items()})
        res["iterations_done"] = out.iterations_done
        res["final_evaluated"] = out.final_evaluated
        res["status"] = st
        return res

    def kernel_time(self):
        return asicp_kernel_time(self.ctx)

    def launch(self) -> dict:
        return asicp_get_launch(self.ctx)

    def set_launch(self, xcd_map: int, fine: int, query_blocks: int = 4, chunk_points: int = 128):
        asicp_set_launch(self.ctx, xcd_map, fine, query_blocks, chunk_points)
        self._launch = {"xcd_map": int(xcd_map), "fine": int(fine), "query_blocks": int(query_blocks),
                        "chunk_points": int(chunk_points)}

    def autotune(self, reps: int = 3, stream=None):
        chosen, ms = asicp_autotune(self.ctx, reps, self._stream(stream))
        self._launch = chosen
        return chosen, ms

    def close(self):
        if getattr(self, "ctx", None) is not None:
            asicp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _pose_autograd():
    import torch

    class PoseCost(torch.autograd.Function):
        """cost_i(theta_i) of the grasp iteration with a hand-written backward.

        Input: poses (7, Ktot) on the device (translation, unit quaternion).
        Forward runs the library's kernels (asicp_cost_grad, pose form: the
        gradient with respect to the 7 pose numbers); backward is the
        library's vector-Jacobian product (asicp_pose_vjp)."""

        @staticmethod
        def forward(ctx, theta, solver):
            cost, grad = solver.cost_grad(theta.detach(), pose=True)
            ctx.save_for_backward(grad)
            ctx.solver = solver
            return cost

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            solver = ctx.solver
            gout = gout.to(torch.float32).contiguous()
            dtheta = torch.empty_like(grad)
            asicp_pose_vjp(grad.data_ptr(), gout.data_ptr(), dtheta.data_ptr(), grad.shape[1],
                           solver._stream(None))
            return dtheta, None

    return PoseCost


def pose_cost(theta, solver):
    """Differentiable per-particle cost at poses `theta` (see PoseCost)."""
    return _pose_autograd().apply(theta, solver)
