"""Photometric loss of fitted pair similarities as a differentiable torch function, and the
Gauss-Newton refinement; argument marshalling over the library's vs_photometric_* entry points
(all arithmetic runs in the HIP kernels).

Parameters follow the library: T(x) = x + [[a, -b], [b, a]] (x - c) / rho + t, theta = (a, b, tx, ty),
c = ((W-1)/2, (H-1)/2), rho = max(W, H) / 2; a fitted similarity (A, B, TX, TY) in centred
coordinates is theta = (rho (A - 1), rho B, TX, TY).
"""
from __future__ import annotations

import math

import torch

from . import vstab as V


def frame_geometry(width: int, height: int) -> tuple:
    return (width - 1) / 2.0, (height - 1) / 2.0, max(width, height) / 2.0


def theta_from_fit(params: torch.Tensor, width: int, height: int) -> torch.Tensor:
    """[n, 4] fitted (a, b, tx, ty) -> [n, 4] theta (float64, same device)."""
    rho = frame_geometry(width, height)[2]
    p = params.to(torch.float64)
    return torch.stack([rho * (p[:, 0] - 1.0), rho * p[:, 1], p[:, 2], p[:, 3]], dim=1)


def omega_for(theta: torch.Tensor, width: int, height: int, extra: int = 0) -> V.vs_rect:
    """Inner rectangle with margin ceil(max |T(x) - x|) + 2 + extra over all pairs (the displacement of
    this transform is largest at a frame corner). Reads theta on the host."""
    cx, cy, rho = frame_geometry(width, height)
    th = theta.detach().to("cpu", torch.float64).reshape(-1, 4)
    best = 0.0
    for x in (0.0, width - 1.0):
        for y in (0.0, height - 1.0):
            dx, dy = (x - cx) / rho, (y - cy) / rho
            mx = th[:, 0] * dx - th[:, 1] * dy + th[:, 2]
            my = th[:, 1] * dx + th[:, 0] * dy + th[:, 3]
            if len(th):
                best = max(best, float(torch.sqrt(mx * mx + my * my).max()))
    m = int(math.ceil(best)) + 2 + extra
    return V.vs_rect(m, m, width - m, height - m)


def _workspace(n: int, width: int, height: int, device) -> tuple:
    wsb = V.vs_photometric_workspace(n, width, height)
    return torch.empty(max(wsb, 256), dtype=torch.uint8, device=device), wsb


def _sums(prev, nxt, theta, omega, grad: bool) -> torch.Tensor:
    n, H, W = prev.shape
    cx, cy, rho = frame_geometry(W, H)
    th = theta.detach().to(torch.float64).contiguous()
    out = torch.empty((n, V.VS_PHOTO_SUMS), dtype=torch.float64, device=prev.device)
    ws, wsb = _workspace(n, W, H, prev.device)
    fn = V.vs_photometric_bwd if grad else V.vs_photometric_fwd
    fn(prev, nxt, W * H, W, H, W, n, th, 4, cx, cy, rho, omega, out, ws, wsb)
    return out


def _features(prev, nxt, u, d, win_half: int, grad: bool):
    n, H, W = prev.shape
    m = u.shape[1]
    loss = torch.empty((n, m), dtype=torch.float64, device=prev.device)
    g = torch.empty((n, m, 2), dtype=torch.float64, device=prev.device) if grad else None
    V.vs_photometric_features(prev, nxt, W * H, W, H, W, n, u.detach().to(torch.float32).contiguous(),
                              d.detach().to(torch.float32).contiguous(), m, win_half, loss, g)
    return loss, g


class PhotometricLoss(torch.autograd.Function):
    """The photometric residual of n frame pairs, differentiable in the similarity parameters and in
    the per-feature displacements:

    * loss_g[i] = sum over omega of (S(next_i, T_theta_i(x)) - prev_i(x))^2, theta float64 [n, 4];
    * loss_f[i, k] = sum over the (2 win_half + 1)^2 window q of (S(next_i, u + d + q) - S(prev_i, u + q))^2
      for the k-th feature u = u[i, k] of pair i displaced by d = d[i, k] ([n, m, 2]; the kernels read
      u and d as float32, so gradients are taken at the float32 values).

    prev, nxt: uint8 [n, H, W] device tensors; omega: vs_rect (fixed); u, d may be None (then loss_f is
    [n, 0]). Backward runs the hand-written kernels: vs_photometric_bwd for dL/dtheta and
    vs_photometric_features for dL/dd."""

    @staticmethod
    def forward(ctx, theta, d, prev, nxt, omega, u=None, win_half: int = 10):
        ctx.save_for_backward(theta, d, u)
        ctx.frames = (prev, nxt, omega, win_half)
        loss_g = _sums(prev, nxt, theta, omega, grad=False)[:, 0].clone()
        if d is None or u is None:
            loss_f = torch.zeros((prev.shape[0], 0), dtype=torch.float64, device=prev.device)
        else:
            loss_f, _ = _features(prev, nxt, u, d, win_half, grad=False)
        return loss_g, loss_f

    @staticmethod
    def backward(ctx, g_g, g_f):
        theta, d, u = ctx.saved_tensors
        prev, nxt, omega, win_half = ctx.frames
        grad_theta = grad_d = None
        if ctx.needs_input_grad[0] and g_g is not None:
            s = _sums(prev, nxt, theta, omega, grad=True)
            grad_theta = (g_g.to(torch.float64)[:, None] * s[:, 1:5]).to(theta.dtype)
        if d is not None and u is not None and ctx.needs_input_grad[1] and g_f is not None:
            _, gd = _features(prev, nxt, u, d, win_half, grad=True)
            grad_d = (g_f.to(torch.float64)[..., None] * gd).to(d.dtype)
        return grad_theta, grad_d, None, None, None, None, None


def photometric_loss(theta, prev, nxt, omega):
    """loss_g only (differentiable in theta)."""
    return PhotometricLoss.apply(theta, None, prev, nxt, omega)[0]


def photometric_losses(theta, d, prev, nxt, omega, u, win_half: int = 10):
    """(loss_g [n], loss_f [n, m]), differentiable in theta and d."""
    return PhotometricLoss.apply(theta, d, prev, nxt, omega, u, win_half)


def gauss_newton_terms(theta, prev, nxt, omega) -> dict:
    """J^T J [n, 4, 4], J^T r [n, 4], loss [n] and dL/dtheta [n, 4] in one pass."""
    s = _sums(prev, nxt, theta, omega, grad=True)
    n = s.shape[0]
    jtj = torch.zeros((n, 4, 4), dtype=torch.float64, device=s.device)
    t = 5
    for i in range(4):
        for j in range(i, 4):
            jtj[:, i, j] = s[:, t]
            jtj[:, j, i] = s[:, t]
            t += 1
    return {"loss": s[:, 0], "grad": s[:, 1:5], "jtj": jtj, "jtr": s[:, 15:19]}


def refine(prev, nxt, theta0, omega, max_steps: int = 5):
    """Gauss-Newton refinement of every pair; returns (theta [n, 4], loss [n, 2] = initial/final,
    accepted [n])."""
    n, H, W = prev.shape
    cx, cy, rho = frame_geometry(W, H)
    th0 = theta0.detach().to(torch.float64).contiguous()
    out = torch.empty_like(th0)
    loss = torch.empty((n, 2), dtype=torch.float64, device=prev.device)
    acc = torch.empty(n, dtype=torch.int32, device=prev.device)
    ws, wsb = _workspace(n, W, H, prev.device)
    V.vs_photometric_refine(prev, nxt, W * H, W, H, W, n, th0, out, 4, V.VS_PHOTO_THETA, None, 0, cx, cy, rho, omega,
                            max_steps, loss, acc, ws, wsb)
    return out, loss, acc


def feature_loss(prev, nxt, u, d, win_half: int = 10):
    """Per-point window loss and its gradient with respect to the displacement d: prev, nxt uint8
    [H, W] (one pair) with u, d [m, 2], or [n, H, W] with u, d [n, m, 2]."""
    if prev.dim() == 2:
        loss, g = _features(prev[None], nxt[None], u[None], d[None], win_half, grad=True)
        return loss[0], g[0]
    return _features(prev, nxt, u, d, win_half, grad=True)
