"""torch.autograd binding of TSDF integration and its hand-written adjoint.

Forward: integrate keyframes k at poses T_k Exp(xi_k) (Sec. 3 running
weighted average) with libscsurf, into an empty volume or onto a given prior
field (D0, C0, W0); returns the field over the allocated blocks in pool
order.  Backward: tsdf_integrate_backward with the pixel and band decisions
of the forward held fixed.  The library returns the gradient of a right
perturbation at the integrated pose T_k Exp(xi_k); the gradient with respect
to xi_k is that vector times the SE(3) right Jacobian J_r(xi_k), since
T Exp(xi + delta) = T Exp(xi) Exp(J_r(xi) delta) to first order.
"""
from __future__ import annotations

import numpy as np
import torch

from . import scsurf


def _skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def so3_exp(phi):
    """(exp([phi]_x), J_l(phi)): the rotation and the SO(3) left Jacobian."""
    phi = np.asarray(phi, np.float64)
    th = float(np.sqrt(phi @ phi))
    K = _skew(phi)
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K, np.eye(3) + 0.5 * K + K @ K / 6.0
    a = np.sin(th) / th
    b = 2.0 * np.sin(0.5 * th) ** 2 / th**2  # (1 - cos th) / th^2 without the cancellation
    c = (th - np.sin(th)) / th**3
    return np.eye(3) + a * K + b * K @ K, np.eye(3) + b * K + c * K @ K


def se3_left_jacobian(xi):
    """6x6 left Jacobian of SE(3) at xi = (rho, phi), Exp(xi) = [[exp(phi^),
    J_l(phi) rho], [0, 1]]: Exp(xi + d) = Exp(J_l(xi) d) Exp(xi) to first
    order.  Block form [[J_l(phi), Q(rho, phi)], [0, J_l(phi)]] with the
    closed-form Q of the SE(3) series (Barfoot, State Estimation for
    Robotics, Sec. 7.1)."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    _, J = so3_exp(phi)
    P, Rh = _skew(phi), _skew(rho)
    th = float(np.sqrt(phi @ phi))
    if th < 1e-6:
        # the coefficients' limits at phi -> 0: 1/6, 1/24, 1/120
        Q = (0.5 * Rh + (P @ Rh + Rh @ P + P @ Rh @ P) / 6.0
             + (P @ P @ Rh + Rh @ P @ P - 3.0 * P @ Rh @ P) / 24.0 + (P @ Rh @ P @ P + P @ P @ Rh @ P) / 120.0)
    else:
        s, c = np.sin(th), np.cos(th)
        Q = (0.5 * Rh + (th - s) / th**3 * (P @ Rh + Rh @ P + P @ Rh @ P)
             + (th * th + 2.0 * c - 2.0) / (2.0 * th**4) * (P @ P @ Rh + Rh @ P @ P - 3.0 * P @ Rh @ P)
             + (2.0 * th - 3.0 * s + th * c) / (2.0 * th**5) * (P @ Rh @ P @ P + P @ P @ Rh @ P))
    out = np.zeros((6, 6))
    out[:3, :3] = J
    out[3:, 3:] = J
    out[:3, 3:] = Q
    return out


def se3_right_jacobian(xi):
    """J_r(xi) = J_l(-xi): Exp(xi + d) = Exp(xi) Exp(J_r(xi) d) to first order."""
    return se3_left_jacobian(-np.asarray(xi, np.float64))


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
    """(depth (K,H,W), color (K,H,W,3) in [0,1], weight (K,H,W), xi (K,6),
    D0 (n0,512), C0 (n0,3,512), W0 (n0,512), blocks0 (n0,3)) ->
    (D (n,512), C (n,3,512), W (n,512)) over the allocated blocks of `volume`
    (an F32-colour scsurf.Volume, reset by the forward).  Without a prior
    (D0 None) the keyframes are integrated into an empty field."""

    @staticmethod
    def forward(ctx, depth, color, weight, xi, D0, C0, W0, blocks0, volume, intr, R, t):
        xin = xi.detach().cpu().numpy().astype(np.float64)
        Rp, tp = perturbed_poses(R, t, xin)
        volume.reset()
        if D0 is not None:
            prior = {"blocks": blocks0, "D": D0.detach(), "W": W0}
            if C0 is not None:
                prior["C"] = C0.detach()
            volume.import_field(prior)
        kfs = [scsurf.Keyframe(depth[k].contiguous(), weight[k].contiguous(), color[k].contiguous())
               for k in range(depth.shape[0])]
        for k, kf in enumerate(kfs):
            volume.integrate(kf, intr, Rp[k], tp[k])
        volume.check_error()
        f = volume.export()
        ctx.volume = volume
        ctx.intr = intr
        ctx.poses = (Rp, tp)
        ctx.xi = xin
        ctx.kfs = kfs
        ctx.shapes = (depth.shape, color.shape)
        ctx.prior = (blocks0, D0 is not None, C0 is not None)
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
        g_right = torch.zeros((dshape[0], 6), dtype=torch.float32, device=dev)
        blocks0, has_d0, has_c0 = ctx.prior
        need_d0 = has_d0 and ctx.needs_input_grad[4]
        need_c0 = has_c0 and ctx.needs_input_grad[5]
        g_D0p = torch.empty((n, 512), dtype=torch.float32, device=dev) if (need_d0 or need_c0) else None
        g_C0p = torch.empty((n, 3, 512), dtype=torch.float32, device=dev) if need_c0 else None
        ctx.volume.integrate_backward(ctx.kfs, ctx.intr, *ctx.poses, gD, gC, g_depth, g_color, g_right, g_D0p, g_C0p)
        # the pose gradient with respect to xi: J_r(xi)^T times the right-perturbation gradient
        Jr = np.stack([se3_right_jacobian(x) for x in ctx.xi])
        g_xi = torch.einsum("kij,ki->kj", torch.from_numpy(Jr).to(dev), g_right.double()).float()
        g_D0 = g_C0 = None
        if g_D0p is not None:
            # prior blocks in their given order: their pool slots, as the library's hash lookup finds them
            slots = ctx.volume.hash_alloc(blocks0.to(torch.int32).contiguous()).long()
            g_D0 = g_D0p[slots] if need_d0 else None
            g_C0 = g_C0p[slots] if need_c0 else None
        return g_depth, g_color, None, g_xi, g_D0, g_C0, None, None, None, None, None, None


def integrate(depth, color, weight, xi, volume, intr, R, t, prior=None):
    """Differentiable integration of K keyframes at T_k Exp(xi_k).  `prior`
    is an optional dict {"blocks" (n0,3) int32, "D" (n0,512), "C" (n0,3,512),
    "W" (n0,512)} of device tensors, the field integrated onto (its D and C
    may require gradients)."""
    if prior is None:
        return TsdfIntegrate.apply(depth, color, weight, xi, None, None, None, None, volume, intr, R, t)
    return TsdfIntegrate.apply(depth, color, weight, xi, prior["D"], prior.get("C"), prior["W"], prior["blocks"],
                               volume, intr, R, t)
