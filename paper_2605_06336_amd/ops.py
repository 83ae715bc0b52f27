"""Python entry points with the C ABI's names, over torch device tensors.

Each function checks dtypes, devices and shapes, then calls the library on the
current torch stream.  torch provides device memory and streams only.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import torch

from . import _lib
from ._lib import Batch, Geom, PatGeom, check

_ctx = {}


def context(device: int = 0) -> int:
    """Library context for a device (created once per process and device)."""
    if device not in _ctx:
        h = ctypes.c_void_p()
        check(_lib.lib().nlrmm_ctx_create(ctypes.byref(h), device), "nlrmm_ctx_create")
        _ctx[device] = h.value
    return _ctx[device]


def set_kernel_timing(enable, device: int = 0) -> None:
    """Event timing of the forward-weights and backprojection kernels (measurement): False
    off, True on, an int R > 1 launches each timed kernel R times between its events, an int
    -P < 0 records every P-th eligible single launch for kernel_avg."""
    check(_lib.lib().nlrmm_ctx_set_timing(context(device), int(enable)), "nlrmm_ctx_set_timing")


def kernel_ms(which: str, device: int = 0) -> float:
    """Duration per launch of the most recent 'project' (forward-weights) or 'backproject'
    (pixel-tile) kernel, from HIP events on its launch stream; waits for that launch."""
    ms = ctypes.c_float()
    check(_lib.lib().nlrmm_ctx_kernel_ms(context(device), {"project": 0, "backproject": 1}[which],
                                         ctypes.byref(ms)), "nlrmm_ctx_kernel_ms")
    return float(ms.value)


def kernel_avg(which: str, device: int = 0):
    """Per-launch accumulation mode (set_kernel_timing(-P)): (average ms of the recorded
    single launches of the 'project' or 'backproject' kernel, their number); resets."""
    ms = ctypes.c_float()
    n = ctypes.c_int32()
    check(_lib.lib().nlrmm_ctx_kernel_avg(context(device),
                                          {"project": 0, "backproject": 1}[which],
                                          ctypes.byref(ms), ctypes.byref(n)),
          "nlrmm_ctx_kernel_avg")
    return float(ms.value), int(n.value)


def geom(N: int, nb: int, ny: Optional[int] = None, half: float = 1.0,
         s_half: float = 1.42) -> Geom:
    """Square-pixel grid on [-half, half] along x (N pixels) and detector [-s_half, s_half]."""
    ny = N if ny is None else ny
    d = 2.0 * half / N
    return Geom(nx=N, ny=ny, x0=-half, y0=-half * ny / N, d=d, nbins=nb, s0=-s_half,
                ds=2.0 * s_half / nb)


class Frames:
    """Frame structure of a batch: view offsets on the device plus the host count."""

    def __init__(self, view_off, device="cuda"):
        vo = torch.as_tensor(view_off, dtype=torch.int64)
        self.nframes = int(vo.numel() - 1)
        self.nviews = int(vo[-1])
        self.view_off = vo.to(device)
        self.host = vo.cpu().numpy()

    def struct(self) -> Batch:
        return Batch(nframes=self.nframes, nviews=self.nviews,
                     view_off=self.view_off.data_ptr() if self.nframes > 1 else None)


def single(nviews: int) -> Batch:
    return Batch(nframes=1, nviews=nviews, view_off=None)


def _batch(frames, nviews):
    if frames is None:
        return single(nviews)
    if isinstance(frames, Frames):
        return frames.struct()
    return frames


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _need(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous CUDA tensor of {dtype}")


def project(x: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A(theta) x.  x: [..., F, ny, nx] float32 (leading dims = columns); y: [..., V, nb]."""
    _need(x, torch.float32, "x")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    npix = b.nframes * g.nx * g.ny
    if x.numel() % npix:
        raise ValueError("x size is not a multiple of frames*ny*nx")
    ncols = x.numel() // npix
    if out is None:
        out = torch.empty((ncols, V, g.nbins), dtype=torch.float32, device=x.device)
    _need(out, torch.float32, "out")
    check(_lib.lib().nlrmm_project(context(x.device.index or 0), ctypes.byref(g), ctypes.byref(b),
                                   ncols, x.data_ptr(), theta.data_ptr(), out.data_ptr(),
                                   _stream(x.device)), "nlrmm_project")
    return out


def backproject(y: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = A(theta)^T y.  y: [..., V, nb] float32; x: [ncols, F, ny, nx]."""
    _need(y, torch.float32, "y")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    if y.numel() % (V * g.nbins):
        raise ValueError("y size is not a multiple of V*nb")
    ncols = y.numel() // (V * g.nbins)
    if out is None:
        out = torch.empty((ncols, b.nframes, g.ny, g.nx), dtype=torch.float32, device=y.device)
    _need(out, torch.float32, "out")
    check(_lib.lib().nlrmm_backproject(context(y.device.index or 0), ctypes.byref(g),
                                       ctypes.byref(b), ncols, y.data_ptr(), theta.data_ptr(),
                                       out.data_ptr(), _stream(y.device)), "nlrmm_backproject")
    return out


def _fan_forward(name, x, theta, g, R, frames, out):
    _need(x, torch.float32, "x")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    npix = b.nframes * g.nx * g.ny
    if x.numel() % npix:
        raise ValueError("x size is not a multiple of frames*ny*nx")
    ncols = x.numel() // npix
    if out is None:
        out = torch.empty((ncols, V, g.nbins), dtype=torch.float32, device=x.device)
    _need(out, torch.float32, "out")
    check(getattr(_lib.lib(), name)(context(x.device.index or 0), ctypes.byref(g),
                                    ctypes.byref(b), ncols, x.data_ptr(), theta.data_ptr(),
                                    float(R), out.data_ptr(), _stream(x.device)), name)
    return out


def _fan_transpose(name, y, theta, g, R, frames, out):
    _need(y, torch.float32, "y")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    if y.numel() % (V * g.nbins):
        raise ValueError("y size is not a multiple of V*nb")
    ncols = y.numel() // (V * g.nbins)
    if out is None:
        out = torch.empty((ncols, b.nframes, g.ny, g.nx), dtype=torch.float32, device=y.device)
    _need(out, torch.float32, "out")
    check(getattr(_lib.lib(), name)(context(y.device.index or 0), ctypes.byref(g),
                                    ctypes.byref(b), ncols, y.data_ptr(), theta.data_ptr(),
                                    float(R), out.data_ptr(), _stream(y.device)), name)
    return out


def fan_project(x: torch.Tensor, theta: torch.Tensor, g: Geom, R: float, frames=None,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Fan-beam y = A_fan(theta) x, source at distance R (nlrmm_fan_project).  Shapes as
    ``project``."""
    return _fan_forward("nlrmm_fan_project", x, theta, g, R, frames, out)


def fan_backproject(y: torch.Tensor, theta: torch.Tensor, g: Geom, R: float, frames=None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Fan-beam x = A_fan(theta)^T y (nlrmm_fan_backproject).  Shapes as ``backproject``."""
    return _fan_transpose("nlrmm_fan_backproject", y, theta, g, R, frames, out)


def fan_project_dtheta(x: torch.Tensor, theta: torch.Tensor, g: Geom, R: float, frames=None,
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-view angle derivative of the fan-beam projection (nlrmm_fan_project_dtheta)."""
    return _fan_forward("nlrmm_fan_project_dtheta", x, theta, g, R, frames, out)


def fan_backproject_dtheta(r: torch.Tensor, theta: torch.Tensor, g: Geom, R: float,
                           frames=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Transpose of ``fan_project_dtheta`` (nlrmm_fan_backproject_dtheta)."""
    return _fan_transpose("nlrmm_fan_backproject_dtheta", r, theta, g, R, frames, out)


def pat_geom(n_sensors: int, n_radii: int, n_samples: int, sensor_radius: float = 1.5,
             radius_step: Optional[float] = None) -> PatGeom:
    """Circular-means geometry: radii (j + 1) radius_step + p (default step 2 / n_radii)."""
    return PatGeom(n_sensors=n_sensors, n_radii=n_radii, n_samples=n_samples,
                   sensor_radius=sensor_radius,
                   radius_step=2.0 / n_radii if radius_step is None else radius_step)


def _pat(name, src, g, pg, p, out, out_shape):
    _need(src, torch.float32, "input")
    if out is None:
        out = torch.empty(out_shape, dtype=torch.float32, device=src.device)
    _need(out, torch.float32, "out")
    ncols = out_shape[0]
    check(getattr(_lib.lib(), name)(context(src.device.index or 0), ctypes.byref(g),
                                    ctypes.byref(pg), ncols, src.data_ptr(), float(p),
                                    out.data_ptr(), _stream(src.device)), name)
    return out


def pat_project(x: torch.Tensor, g: Geom, pg: PatGeom, p: float,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Circle integrals y = A_pat(p) x: x [..., ny, nx] -> [ncols, n_sensors, n_radii]."""
    ncols = x.numel() // (g.nx * g.ny)
    if x.numel() != ncols * g.nx * g.ny:
        raise ValueError("x size is not a multiple of ny*nx")
    return _pat("nlrmm_pat_project", x, g, pg, p, out, (ncols, pg.n_sensors, pg.n_radii))


def pat_project_dp(x: torch.Tensor, g: Geom, pg: PatGeom, p: float,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """d(A_pat(p) x)/dp, same shapes as ``pat_project``."""
    ncols = x.numel() // (g.nx * g.ny)
    if x.numel() != ncols * g.nx * g.ny:
        raise ValueError("x size is not a multiple of ny*nx")
    return _pat("nlrmm_pat_project_dp", x, g, pg, p, out, (ncols, pg.n_sensors, pg.n_radii))


def pat_backproject(y: torch.Tensor, g: Geom, pg: PatGeom, p: float,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = A_pat(p)^T y: y [..., n_sensors, n_radii] -> [ncols, ny, nx]."""
    per = pg.n_sensors * pg.n_radii
    ncols = y.numel() // per
    if y.numel() != ncols * per:
        raise ValueError("y size is not a multiple of n_sensors*n_radii")
    return _pat("nlrmm_pat_backproject", y, g, pg, p, out, (ncols, g.ny, g.nx))


def backproject_noalloc(y: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = A(theta)^T y without any device allocation by the library
    (nlrmm_backproject_noalloc: partial images in its fixed scratch).  Same shapes and results
    as ``backproject``; pass ``out`` to allocate nothing here either."""
    _need(y, torch.float32, "y")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    if y.numel() % (V * g.nbins):
        raise ValueError("y size is not a multiple of V*nb")
    ncols = y.numel() // (V * g.nbins)
    if out is None:
        out = torch.empty((ncols, b.nframes, g.ny, g.nx), dtype=torch.float32, device=y.device)
    _need(out, torch.float32, "out")
    check(_lib.lib().nlrmm_backproject_noalloc(context(y.device.index or 0), ctypes.byref(g),
                                               ctypes.byref(b), ncols, y.data_ptr(),
                                               theta.data_ptr(), out.data_ptr(),
                                               _stream(y.device)), "nlrmm_backproject_noalloc")
    return out


def backproject_dtheta(r: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None,
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = D(theta)^T r, the transpose of the angle derivative (nlrmm_backproject_dtheta).
    r: [..., V, nb] float32; x: [ncols, F, ny, nx]."""
    _need(r, torch.float32, "r")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    if r.numel() % (V * g.nbins):
        raise ValueError("r size is not a multiple of V*nb")
    ncols = r.numel() // (V * g.nbins)
    if out is None:
        out = torch.empty((ncols, b.nframes, g.ny, g.nx), dtype=torch.float32, device=r.device)
    _need(out, torch.float32, "out")
    check(_lib.lib().nlrmm_backproject_dtheta(context(r.device.index or 0), ctypes.byref(g),
                                              ctypes.byref(b), ncols, r.data_ptr(),
                                              theta.data_ptr(), out.data_ptr(),
                                              _stream(r.device)), "nlrmm_backproject_dtheta")
    return out


def autotune_project(x: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None,
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Same result as project(); also times the forward block shapes for this shape and
    keeps the fastest in the device's context (synchronizes the stream)."""
    _need(x, torch.float32, "x")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    ncols = x.numel() // (b.nframes * g.nx * g.ny)
    if out is None:
        out = torch.empty((ncols, V, g.nbins), dtype=torch.float32, device=x.device)
    check(_lib.lib().nlrmm_autotune_project(context(x.device.index or 0), ctypes.byref(g),
                                            ctypes.byref(b), ncols, x.data_ptr(),
                                            theta.data_ptr(), out.data_ptr(), _stream(x.device)),
          "nlrmm_autotune_project")
    return out


def autotune_backproject(y: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None,
                         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Same result as backproject(); also times the view splits for this shape and keeps the
    fastest in the device's context (synchronizes the stream)."""
    _need(y, torch.float32, "y")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    ncols = y.numel() // (V * g.nbins)
    if out is None:
        out = torch.empty((ncols, b.nframes, g.ny, g.nx), dtype=torch.float32, device=y.device)
    check(_lib.lib().nlrmm_autotune_backproject(context(y.device.index or 0), ctypes.byref(g),
                                                ctypes.byref(b), ncols, y.data_ptr(),
                                                theta.data_ptr(), out.data_ptr(),
                                                _stream(y.device)), "nlrmm_autotune_backproject")
    return out


def tune_query(kind: str, g: Geom, nviews: int, ncols: int = 1, frames=None,
               device: int = 0) -> int:
    """Tuned launch shape for 'project' (waves per forward block) or 'backproject' (view
    split) at this shape; 0 when none is stored."""
    b = _batch(frames, nviews)
    c = ctypes.c_int32()
    check(_lib.lib().nlrmm_tune_query(context(device), {"project": 0, "backproject": 1}[kind],
                                      ctypes.byref(g), ctypes.byref(b), ncols, ctypes.byref(c)),
          "nlrmm_tune_query")
    return int(c.value)


def set_tune_file(path: Optional[str], device: int = 0) -> None:
    """Load tuned shapes from `path` and append new ones there (None: stop appending)."""
    check(_lib.lib().nlrmm_ctx_set_tune_file(context(device),
                                             None if path is None else path.encode()),
          "nlrmm_ctx_set_tune_file")


def project_dtheta(x: torch.Tensor, theta: torch.Tensor, g: Geom, frames=None, *,
                   want_dy: bool = True, want_y: bool = False, gres: Optional[torch.Tensor] = None,
                   want_gdot: bool = False, want_dnorm2: bool = False):
    """Angle derivative D = d(A(theta)x)/d theta_v (per view row) with optional fused outputs.

    Returns a dict with any of: 'dy' [ncols, V, nb], 'y' [ncols, V, nb], 'gdot' [ncols, V]
    (= <D_v, gres_v>, float64), 'dnorm2' [ncols, V] (= ||D_v||^2, float64)."""
    _need(x, torch.float32, "x")
    _need(theta, torch.float64, "theta")
    V = theta.numel()
    b = _batch(frames, V)
    ncols = x.numel() // (b.nframes * g.nx * g.ny)
    dev = x.device
    res = {}
    dy = torch.empty((ncols, V, g.nbins), dtype=torch.float32, device=dev) if want_dy else None
    yp = torch.empty((ncols, V, g.nbins), dtype=torch.float32, device=dev) if want_y else None
    gd = torch.empty((ncols, V), dtype=torch.float64, device=dev) if want_gdot else None
    dn = torch.empty((ncols, V), dtype=torch.float64, device=dev) if want_dnorm2 else None
    if want_gdot:
        _need(gres, torch.float32, "gres")
    ptr = lambda t: t.data_ptr() if t is not None else None
    check(_lib.lib().nlrmm_project_dtheta(context(dev.index or 0), ctypes.byref(g),
                                          ctypes.byref(b), ncols, x.data_ptr(), theta.data_ptr(),
                                          ptr(dy), ptr(yp), ptr(gres), ptr(gd), ptr(dn),
                                          _stream(dev)), "nlrmm_project_dtheta")
    for k, t in (("dy", dy), ("y", yp), ("gdot", gd), ("dnorm2", dn)):
        if t is not None:
            res[k] = t
    return res


# ---------------------------------------------------------------------------
# Krylov primitives
# ---------------------------------------------------------------------------
def _p(t):
    return None if t is None else t.data_ptr()


def tv_weights(u: torch.Tensor, g: Geom, nframes: int = 1, temporal: bool = False,
               eps: float = 1e-3, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """w = ((Psi u)^2 + eps^2)^(-1/2) over the anisotropic TV differences."""
    _need(u, torch.float32, "u")
    npsi = nframes * (g.ny * (g.nx - 1) + (g.ny - 1) * g.nx)
    if temporal and nframes > 1:
        npsi += (nframes - 1) * g.nx * g.ny
    if out is None:
        out = torch.empty(npsi, dtype=torch.float32, device=u.device)
    check(_lib.lib().nlrmm_tv_weights(context(u.device.index or 0), ctypes.byref(g), nframes,
                                      int(temporal), u.data_ptr(), eps, out.data_ptr(),
                                      _stream(u.device)), "nlrmm_tv_weights")
    return out


def gram_psi(V: torch.Tensor, w: torch.Tensor, g: Geom, ell: int, nframes: int = 1,
             temporal: bool = False, precision: int = 0) -> torch.Tensor:
    """(Psi V)^T diag(w) (Psi V) for the first ell columns of V ([>=ell, n] float32).
    precision: 0 FP64, 1 FP32 MFMA, 2 BF16 MFMA."""
    _need(V, torch.float32, "V")
    G = torch.empty((ell, ell), dtype=torch.float64, device=V.device)
    check(_lib.lib().nlrmm_gram_psi(context(V.device.index or 0), ctypes.byref(g), nframes,
                                    int(temporal), ell, V.data_ptr(), w.data_ptr(), G.data_ptr(),
                                    ell, precision, _stream(V.device)), "nlrmm_gram_psi")
    return G


def theta_rows(g: Geom, nframes: int, temporal: int) -> int:
    """Length of Theta u: spatial rows plus the temporal rows of mode `temporal` (0 none,
    1 frame differences, 2 optical-flow motion rows)."""
    n = nframes * (g.ny * (g.nx - 1) + (g.ny - 1) * g.nx)
    if nframes > 1 and temporal == 1:
        n += (nframes - 1) * g.nx * g.ny
    if nframes > 1 and temporal == 2:
        n += 2 * (nframes - 1) * g.nx * g.ny
    return n


def _flow_ptr(flow):
    if flow is None:
        return None
    _need(flow, torch.float32, "flow")
    return flow.data_ptr()


def of_estimate(u: torch.Tensor, g: Geom, nframes: int, gamma: float = 0.05,
                ridge: float = 1e-3, iters: int = 200,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Velocities of every frame pair of u ([nframes, ny, nx]) by nlrmm_of_estimate:
    [nframes-1, 2, ny, nx] float32 (s_x, s_y)."""
    _need(u, torch.float32, "u")
    if out is None:
        out = torch.empty((max(nframes - 1, 0), 2, g.ny, g.nx), dtype=torch.float32,
                          device=u.device)
    check(_lib.lib().nlrmm_of_estimate(context(u.device.index or 0), ctypes.byref(g), nframes,
                                       u.data_ptr(), gamma, ridge, iters, out.data_ptr(),
                                       _stream(u.device)), "nlrmm_of_estimate")
    return out


def theta_apply(u: torch.Tensor, g: Geom, nframes: int, temporal: int,
                flow: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Theta u (nlrmm_theta_apply)."""
    _need(u, torch.float32, "u")
    out = torch.empty(theta_rows(g, nframes, temporal), dtype=torch.float32, device=u.device)
    check(_lib.lib().nlrmm_theta_apply(context(u.device.index or 0), ctypes.byref(g), nframes,
                                       temporal, _flow_ptr(flow), u.data_ptr(), out.data_ptr(),
                                       _stream(u.device)), "nlrmm_theta_apply")
    return out


def theta_weights(u: torch.Tensor, g: Geom, nframes: int, temporal: int,
                  flow: Optional[torch.Tensor] = None, eps: float = 1e-3) -> torch.Tensor:
    """w = ((Theta u)^2 + eps^2)^(-1/2) (nlrmm_theta_weights)."""
    _need(u, torch.float32, "u")
    out = torch.empty(theta_rows(g, nframes, temporal), dtype=torch.float32, device=u.device)
    check(_lib.lib().nlrmm_theta_weights(context(u.device.index or 0), ctypes.byref(g), nframes,
                                         temporal, _flow_ptr(flow), u.data_ptr(), eps,
                                         out.data_ptr(), _stream(u.device)),
          "nlrmm_theta_weights")
    return out


def theta_grad_add(u: torch.Tensor, r: torch.Tensor, lam: torch.Tensor, g: Geom, nframes: int,
                   temporal: int, flow: Optional[torch.Tensor] = None,
                   w: Optional[torch.Tensor] = None, eps: float = 1e-3) -> torch.Tensor:
    """r += lam Theta^T (w * Theta u) in place (nlrmm_theta_grad_add); lam a device float64
    scalar tensor; w None: the weights of u."""
    _need(u, torch.float32, "u")
    _need(r, torch.float32, "r")
    _need(lam, torch.float64, "lam")
    check(_lib.lib().nlrmm_theta_grad_add(context(u.device.index or 0), ctypes.byref(g),
                                          nframes, temporal, _flow_ptr(flow), u.data_ptr(),
                                          None if w is None else w.data_ptr(), eps,
                                          lam.data_ptr(), r.data_ptr(), _stream(u.device)),
          "nlrmm_theta_grad_add")
    return r


def gram_theta(V: torch.Tensor, w: torch.Tensor, g: Geom, ell: int, nframes: int, temporal: int,
               flow: Optional[torch.Tensor] = None, precision: int = 0) -> torch.Tensor:
    """(Theta V)^T diag(w) (Theta V) for the first ell columns (nlrmm_gram_theta)."""
    _need(V, torch.float32, "V")
    G = torch.empty((ell, ell), dtype=torch.float64, device=V.device)
    check(_lib.lib().nlrmm_gram_theta(context(V.device.index or 0), ctypes.byref(g), nframes,
                                      temporal, _flow_ptr(flow), ell, V.data_ptr(), w.data_ptr(),
                                      G.data_ptr(), ell, precision, _stream(V.device)),
          "nlrmm_gram_theta")
    return G


def gks_solve(GA, GP, rb, scal, ell, lam_fix=-1.0, status=None):
    """Projected solve with the discrepancy principle; returns (z [ell], out [2], status)."""
    dev = GA.device
    z = torch.empty(ell, dtype=torch.float64, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    check(_lib.lib().nlrmm_gks_solve(context(dev.index or 0), ell, GA.data_ptr(), GP.data_ptr(),
                                     GA.shape[1], rb.data_ptr(), scal.data_ptr(), lam_fix,
                                     z.data_ptr(), out.data_ptr(), status.data_ptr(),
                                     _stream(dev)), "nlrmm_gks_solve")
    return z, out, status


def gks_expand(V, AV, z, b, w, lam, GA, rb, theta, g: Geom, ell: int, frames=None,
               temporal=False, breakdown_tol=1e-10, status=None):
    """Append GKS direction ell to V / AV and extend GA, rb in place (see nlrmm_gks_expand)."""
    dev = V.device
    bt = _batch(frames, theta.numel())
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    check(_lib.lib().nlrmm_gks_expand(context(dev.index or 0), ctypes.byref(g), ctypes.byref(bt),
                                      theta.data_ptr(), ell, int(temporal), V.data_ptr(),
                                      AV.data_ptr(), z.data_ptr(), b.data_ptr(), w.data_ptr(),
                                      lam.data_ptr(), GA.data_ptr(), GA.shape[1], rb.data_ptr(),
                                      breakdown_tol, status.data_ptr(), _stream(dev)),
          "nlrmm_gks_expand")
    return status


def recycle_compress(V, AV, GA, GP, rb, lam, z, ell: int, kmin: int, status=None,
                     precision: int = 0):
    """Compress the basis to kmin columns in place (see nlrmm_recycle_compress); precision 2
    forms the basis products with BF16 operands on the matrix cores."""
    dev = V.device
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    check(_lib.lib().nlrmm_recycle_compress(context(dev.index or 0), V.shape[1], AV.shape[1], ell,
                                            kmin, V.data_ptr(), AV.data_ptr(), GA.data_ptr(),
                                            GP.data_ptr(), GA.shape[1], rb.data_ptr(),
                                            lam.data_ptr(), z.data_ptr(), precision,
                                            status.data_ptr(), _stream(dev)),
          "nlrmm_recycle_compress")
    return status


def project_residual(x: torch.Tensor, theta: torch.Tensor, b: torch.Tensor, g: Geom, frames=None,
                     want_r: bool = True, want_rnorm2: bool = True):
    """r = A(theta) x - b and/or per-view ||r_v||^2 (float64), one image."""
    _need(x, torch.float32, "x")
    _need(theta, torch.float64, "theta")
    _need(b, torch.float32, "b")
    V = theta.numel()
    bt = _batch(frames, V)
    r = torch.empty((V, g.nbins), dtype=torch.float32, device=x.device) if want_r else None
    rn = torch.empty(V, dtype=torch.float64, device=x.device) if want_rnorm2 else None
    check(_lib.lib().nlrmm_project_residual(context(x.device.index or 0), ctypes.byref(g),
                                            ctypes.byref(bt), x.data_ptr(), theta.data_ptr(),
                                            b.data_ptr(), _p(r), _p(rn), _stream(x.device)),
          "nlrmm_project_residual")
    return r, rn


def backproject_into(y: torch.Tensor, theta: torch.Tensor, g: Geom, out: torch.Tensor,
                     frames=None, accumulate: bool = True) -> torch.Tensor:
    """out (+)= A(theta)^T y."""
    _need(y, torch.float32, "y")
    _need(out, torch.float32, "out")
    V = theta.numel()
    bt = _batch(frames, V)
    ncols = y.numel() // (V * g.nbins)
    check(_lib.lib().nlrmm_backproject_acc(context(y.device.index or 0), ctypes.byref(g),
                                           ctypes.byref(bt), ncols, y.data_ptr(),
                                           theta.data_ptr(), out.data_ptr(), int(accumulate),
                                           _stream(y.device)), "nlrmm_backproject_acc")
    return out
