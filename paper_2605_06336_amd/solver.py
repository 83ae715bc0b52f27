"""Python handle of the native NL-RMM-GKS driver (nlrmm_solver_* in the C ABI).

The outer iteration (rebase, Enlarge, Compress, Gauss-Newton angles, residual append)
runs entirely in the library on the current torch stream; this class only owns the
handle and marshals tensors.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib, ops
from ._lib import SolverCfg, check


@dataclasses.dataclass
class Config:
    kmin: int = 5
    kmax: int = 30
    solves: int = 0              # <= 0: kmax - kmin
    eps: float = 1e-3
    tau: float = 1.01
    lam_fix: float = -1.0        # < 0: discrepancy principle
    param_update: int = 1        # 0 none, 1 Gauss-Newton (AltMin), 2 VarPro, 3 sensitivity
    param_mode: int = 0          # 0 per-view, 1 global shift
    maxiter_p: int = 1
    mu_rel: float = 1e-6
    c1: float = 1e-4
    beta: float = 0.5
    alpha0: float = 1.0
    armijo_trials: int = 10
    breakdown_tol: float = 1e-10
    temporal: int = 0            # 0 none, 1 frame differences, 2 optical-flow motion rows
    gram_precision: int = 0      # 0 FP64, 1 FP32 MFMA, 2 BF16 MFMA
    compress_precision: int = 0  # compression basis products: 0 FP32 (FP64 accumulate), 2 BF16 MFMA
    lam_hi: float = 0.0          # > 0: high-regularisation solve feeding the parameter update
    sens_iters: int = 50         # CG steps of the sensitivity solve (param_update 3)
    of_iters: int = 200          # temporal 2: CG steps of the velocity estimation
    of_gamma: float = 0.05       # temporal 2: smoothness weight of the velocity problem
    of_ridge: float = 1e-3       # temporal 2: ridge of the velocity problem
    of_every: int = 1            # temporal 2: velocities re-estimated every of_every outer its

    def struct(self) -> SolverCfg:
        return SolverCfg(**dataclasses.asdict(self))


class Solver:
    def __init__(self, g: ops.Geom, nframes: int, max_views: int, cfg: Config, device: int = 0):
        self.g = g
        self.nframes = nframes
        self.cfg = cfg
        self.device = torch.device("cuda", device)
        self.n = nframes * g.nx * g.ny
        h = ctypes.c_void_p()
        c = cfg.struct()
        check(_lib.lib().nlrmm_solver_create(ops.context(device), ctypes.byref(g), nframes,
                                             max_views, ctypes.byref(c), ctypes.byref(h)),
              "nlrmm_solver_create")
        self.h = h.value

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize(self.device)
            _lib.lib().nlrmm_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_per_frame(self, view_off_host=None) -> None:
        """Plain per-frame launches (view_off_host given) or batched launches (None)."""
        import numpy as np
        if view_off_host is None:
            check(_lib.lib().nlrmm_solver_set_launch(self.h, 0, None, self.nframes),
                  "nlrmm_solver_set_launch")
            return
        self._vo = np.ascontiguousarray(view_off_host, dtype=np.int64)
        check(_lib.lib().nlrmm_solver_set_launch(
            self.h, 1, self._vo.ctypes.data_as(ctypes.c_void_p), self.nframes),
            "nlrmm_solver_set_launch")

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def init(self, theta: torch.Tensor, b: torch.Tensor, frames=None) -> None:
        bt = ops._batch(frames, theta.numel())
        check(_lib.lib().nlrmm_solver_init(self.h, ctypes.byref(bt), theta.data_ptr(),
                                           b.data_ptr(), self._stream()), "nlrmm_solver_init")

    def grid_search(self, theta: torch.Tensor, b: torch.Tensor, shifts: torch.Tensor,
                    ell0: int = 10, frames=None):
        """Coarse grid search of one global angle offset (nlrmm_solver_grid_search): theta
        (float64, device) is shifted in place by the best candidate; returns (res2 [ncand]
        float64, best [1] int32) device tensors.  Call init() at the new angles afterwards."""
        bt = ops._batch(frames, theta.numel())
        shifts = shifts.to(device=theta.device, dtype=torch.float64).contiguous()
        res2 = torch.empty(shifts.numel(), dtype=torch.float64, device=theta.device)
        best = torch.empty(1, dtype=torch.int32, device=theta.device)
        check(_lib.lib().nlrmm_solver_grid_search(self.h, ctypes.byref(bt), theta.data_ptr(),
                                                  b.data_ptr(), shifts.data_ptr(),
                                                  int(shifts.numel()), int(ell0),
                                                  res2.data_ptr(), best.data_ptr(),
                                                  self._stream()),
              "nlrmm_solver_grid_search")
        return res2, best

    def offset_sensitivity(self, theta: torch.Tensor, b: torch.Tensor, iters: int = 100,
                           frames=None):
        """Full-space sensitivity for one global angle offset at the current image
        (nlrmm_solver_offset_sensitivity): returns ([g, h, dp] float64, u_p float32) device
        tensors."""
        bt = ops._batch(frames, theta.numel())
        out = torch.empty(3, dtype=torch.float64, device=theta.device)
        up = torch.empty(self.n, dtype=torch.float32, device=theta.device)
        check(_lib.lib().nlrmm_solver_offset_sensitivity(self.h, ctypes.byref(bt),
                                                         theta.data_ptr(), b.data_ptr(),
                                                         int(iters), out.data_ptr(),
                                                         up.data_ptr(), self._stream()),
              "nlrmm_solver_offset_sensitivity")
        return out, up

    def outer(self, theta: torch.Tensor, b: torch.Tensor, delta: float, frames=None) -> None:
        """One outer iteration; theta (float64, device) is updated in place."""
        bt = ops._batch(frames, theta.numel())
        check(_lib.lib().nlrmm_solver_outer(self.h, ctypes.byref(bt), theta.data_ptr(),
                                            b.data_ptr(), float(delta), self._stream()),
              "nlrmm_solver_outer")

    def read(self):
        """(u [n] float32, scalars [16] float64, status [1] int32) as new device tensors."""
        u = torch.empty(self.n, dtype=torch.float32, device=self.device)
        sc = torch.empty(16, dtype=torch.float64, device=self.device)
        st = torch.empty(1, dtype=torch.int32, device=self.device)
        check(_lib.lib().nlrmm_solver_read(self.h, u.data_ptr(), sc.data_ptr(), st.data_ptr(),
                                           self._stream()), "nlrmm_solver_read")
        return u, sc, st


class OuterGraph:
    """One outer iteration captured as a HIP graph (torch.cuda.CUDAGraph) and replayed.

    The solver's state, theta and b live at fixed device addresses, so every replay
    performs the next outer iteration.  An eager outer iteration must have run first so
    that every workspace is allocated before capture (allocation is refused while a stream
    is capturing)."""

    def __init__(self, solver: Solver, theta: torch.Tensor, b: torch.Tensor, delta: float,
                 frames=None):
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize(solver.device)
        with torch.cuda.graph(self.graph):
            solver.outer(theta, b, delta, frames)
        torch.cuda.synchronize(solver.device)

    def replay(self) -> None:
        self.graph.replay()
