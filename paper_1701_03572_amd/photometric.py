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


def _sums(prev, nxt, theta, omega, grad: bool) -> torch.Tensor:
    n, H, W = prev.shape
    cx, cy, rho = frame_geometry(W, H)
    th = theta.detach().to(torch.float64).contiguous()
    out = torch.empty((n, V.VS_PHOTO_SUMS), dtype=torch.float64, device=prev.device)
    fn = V.vs_photometric_bwd if grad else V.vs_photometric_fwd
    fn(prev, nxt, W * H, W, H, W, n, th, 4, cx, cy, rho, omega, out)
    return out


class PhotometricLoss(torch.autograd.Function):
    """loss[i] = sum over omega of (S(next_i, T_theta_i(x)) - prev_i(x))^2; differentiable in theta.

    prev, nxt: uint8 [n, H, W] device tensors; theta: float64 [n, 4]; omega: vs_rect (fixed)."""

    @staticmethod
    def forward(ctx, theta, prev, nxt, omega):
        ctx.save_for_backward(theta)
        ctx.frames = (prev, nxt, omega)
        return _sums(prev, nxt, theta, omega, grad=False)[:, 0].clone()

    @staticmethod
    def backward(ctx, g):
        (theta,) = ctx.saved_tensors
        prev, nxt, omega = ctx.frames
        s = _sums(prev, nxt, theta, omega, grad=True)
        return g.to(torch.float64)[:, None] * s[:, 1:5], None, None, None


def photometric_loss(theta, prev, nxt, omega):
    return PhotometricLoss.apply(theta, prev, nxt, omega)


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
    wsb = V.vs_photometric_workspace(n)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=prev.device)
    V.vs_photometric_refine(prev, nxt, W * H, W, H, W, n, th0, out, 4, V.VS_PHOTO_THETA, None, 0, cx, cy, rho, omega,
                            max_steps, loss, acc, ws, wsb)
    return out, loss, acc


def feature_loss(prev, nxt, u, d, win_half: int = 10):
    """Per-point window loss and its gradient with respect to the displacement d (one frame pair)."""
    H, W = prev.shape
    m = u.shape[0]
    loss = torch.empty(m, dtype=torch.float64, device=prev.device)
    grad = torch.empty((m, 2), dtype=torch.float64, device=prev.device)
    V.vs_photometric_features(prev, nxt, W, H, W, u.to(torch.float32).contiguous(), d.to(torch.float32).contiguous(),
                              m, win_half, loss, grad)
    return loss, grad
