"""torch.autograd binding of TSDF integration and its hand-written adjoint.

Forward: integrate keyframes k at poses T_k Exp(xi_k) into an empty volume
(running weighted average, Sec. 3) with libscsurf; returns the field over the
allocated blocks in pool order.  Backward: tsdf_integrate_backward, with the
pixel and band decisions of the forward held fixed.  The pose gradient is that
of a right perturbation at the integrated pose, i.e. exact at xi = 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import scsurf


def so3_exp(phi):
    phi = np.asarray(phi, np.float64)
    th = float(np.sqrt(phi @ phi))
    K = np.array([[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K, np.eye(3) + 0.5 * K
    a = np.sin(th) / th
    b = (1 - np.cos(th)) / th**2
    c = (th - np.sin(th)) / th**3
    return np.eye(3) + a * K + b * K @ K, np.eye(3) + b * K + c * K @ K


def perturbed_poses(R, t, xi):
    """T_k Exp(xi_k) for every keyframe."""
    R = np.asarray(R, np.float64)
    t = np.asarray(t, np.float64)
    xi = np.asarray(xi, np.float64).reshape(-1, 6)
    Ro, to = np.empty_like(R), np.empty_like(t)
    for k in range(len(R)):
        Re, V = so3_exp(xi[k, 3:])
        Ro[k] = R[k] @ Re
        to[k] = R[k] @ (V @ xi[k, :3]) + t[k]
    return Ro, to


class TsdfIntegrate(torch.autograd.Function):
    """(depth (K,H,W), color (K,H,W,3) in [0,1], weight (K,H,W), xi (K,6)) ->
    (D (n,512), C (n,3,512), W (n,512)) over the allocated blocks of `volume`
    (an F32-colour scsurf.Volume, reset by the forward)."""

    @staticmethod
    def forward(ctx, depth, color, weight, xi, volume, intr, R, t):
        Rp, tp = perturbed_poses(R, t, xi.detach().cpu().numpy())
        volume.reset()
        kfs = [scsurf.Keyframe(depth[k].contiguous(), weight[k].contiguous(), color[k].contiguous())
               for k in range(depth.shape[0])]
        for k, kf in enumerate(kfs):
            volume.integrate(kf, intr, Rp[k], tp[k])
        volume.check_error()
        f = volume.export()
        ctx.volume = volume
        ctx.intr = intr
        ctx.poses = (Rp, tp)
        ctx.kfs = kfs
        ctx.shapes = (depth.shape, color.shape)
        ctx.mark_non_differentiable(f["W"])
        ctx.blocks = f["blocks"]
        return f["D"], f["C"], f["W"]

    @staticmethod
    def backward(ctx, gD, gC, gW):
        dshape, cshape = ctx.shapes
        dev = gD.device if gD is not None else gC.device
        n = ctx.blocks.shape[0]
        gD = gD.contiguous() if gD is not None else torch.zeros((n, 512), device=dev)
        gC = gC.contiguous() if gC is not None else torch.zeros((n, 3, 512), device=dev)
        g_depth = torch.zeros(dshape, dtype=torch.float32, device=dev)
        g_color = torch.zeros(cshape, dtype=torch.float32, device=dev)
        g_xi = torch.zeros((dshape[0], 6), dtype=torch.float32, device=dev)
        ctx.volume.integrate_backward(ctx.kfs, ctx.intr, *ctx.poses, gD, gC, g_depth, g_color, g_xi)
        return g_depth, g_color, None, g_xi, None, None, None, None


def integrate(depth, color, weight, xi, volume, intr, R, t):
    return TsdfIntegrate.apply(depth, color, weight, xi, volume, intr, R, t)
