"""Learned grasp proposal: seeds for the AS-ICP iteration from a point-cloud
encoder (kernels in csrc/k_proposal.hip, C calls asicp_pn_*).

The paper points to learned priors and data-driven seeding as the way to
need fewer initialisations (Sec. V-A ablation, Sec. VI).  Here a max-pooled
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

from . import (ASICP_OK, AsicpError, Solver, asicp_pn_adam, asicp_pn_forward, asicp_pn_loss_grad,
               asicp_pn_param_count, asicp_pn_workspace_bytes, synth)

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

    def forward(self, clouds):
        """Seeds (7, n_obj * n_pre * n_seed) float32 device tensor, solver order."""
        torch = self.torch
        assert len(clouds) <= self.max_obj
        off, xyz = self._clouds(clouds)
        n_obj = len(clouds)
        seeds = torch.empty(7, n_obj * self.n_pre * self.n_seed, dtype=torch.float32, device=self.device)
        raw = torch.empty(n_obj, self.n_pre * self.n_seed * 7, dtype=torch.float32, device=self.device)
        asicp_pn_forward(self.params.data_ptr(), self.n_pre, self.n_seed, n_obj, off.ctypes.data,
                         xyz[0].data_ptr(), xyz[1].data_ptr(), xyz[2].data_ptr(), seeds.data_ptr(),
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
