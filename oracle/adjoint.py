"""Adjoint of TSDF integration — oracle side, FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward (Sec. 3 running weighted average, quantities of Sec. 4.3): after
integrating keyframes k = 1..K at poses T_k into a field with prior (D0, W0),
every voxel holds
    D(v) = (W0 D0 + sum_k w_k d_k) / (W0 + sum_k w_k),
    C(v) = (W0 C0 + sum_k w_k c_k) / (W0 + sum_k w_k),
    d_k  = Z_k(u_k(v)) - p_z,   p = T_k^-1 x_v,
with u_k(v) the nearest pixel and w_k = q(W*_k(u_k)) the keyframe weight.
Pixel choice and band membership are piecewise constant; the derivative is
that of the active smooth piece ("frozen decisions").  Perturbing the pose on
the right, T_k Exp(xi) with xi = (rho, phi):
    p(xi) = Exp(-xi) p  =>  dp/drho = -I,  dp/dphi = [p]_x,
    d d_k / d xi = -d p_z / d xi = (0, 0, 1, p_y, -p_x, 0).
Hence, with g_D = dL/dD and g_C = dL/dC,
    dL/dZ_k(u)  = sum_{v: u_k(v) = u} g_D(v) w_k / W(v)
    dL/dC_k(u)  = sum_{v: u_k(v) = u} g_C(v) w_k / W(v)
    dL/dxi_k    = sum_v g_D(v) (w_k / W(v)) (0, 0, 1, p_y, -p_x, 0)
    dL/dD0(v)   = g_D(v) W0(v) / W(v).
"""
from __future__ import annotations

import math

import numpy as np

from . import Volume


def so3_exp(phi):
    phi = np.asarray(phi, float)
    th = math.sqrt(float(phi @ phi))
    K = np.array([[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K, np.eye(3) + 0.5 * K + K @ K / 6.0
    A = math.sin(th) / th
    B = (1.0 - math.cos(th)) / th**2
    Cc = (th - math.sin(th)) / th**3
    return np.eye(3) + A * K + B * K @ K, np.eye(3) + B * K + Cc * K @ K


def right_perturb(R, t, xi):
    """T Exp(xi) for T = (R, t)."""
    Re, V = so3_exp(xi[3:])
    te = V @ np.asarray(xi[:3], float)
    return R @ Re, R @ te + t


class FrozenIntegration:
    """Decisions of integrating K keyframes, frozen at the given poses."""

    def __init__(self, voxel_size, trunc, kfs, intr, R, t):
        self.s = float(np.float32(voxel_size))
        probe = Volume(voxel_size, trunc, color_f32=True)
        self.K = len(kfs)
        self.shape = kfs[0]["depth"].shape
        recs = [probe.record(kfs[k], intr, R[k], t[k]) for k in range(self.K)]
        alln = np.concatenate([r["n"] for r in recs]).astype(np.int64)
        self.vox, inv = np.unique(alln, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        off = 0
        self.vid, self.pix, self.w = [], [], []
        for r in recs:
            m = len(r["pix"])
            self.vid.append(inv[off:off + m])
            self.pix.append(r["pix"].astype(np.int64))
            self.w.append(r["w"].astype(np.float64))
            off += m
        self.V = len(self.vox)
        self.xv = self.s * self.vox.astype(np.float64)  # voxel centres s*n

    def camera_points(self, k, R, t):
        e = self.xv[self.vid[k]] - np.asarray(t, float)
        return e @ np.asarray(R, float)  # rows: R^T e

    def field(self, depths, colors, R, t, prior=None):
        """(D, C, W) over the recorded voxels, FP64."""
        V = self.V
        if prior is None:
            D0 = np.zeros(V)
            C0 = np.zeros((V, 3))
            W0 = np.zeros(V)
        else:
            D0, C0, W0 = prior
        numD = W0 * D0
        numC = W0[:, None] * C0
        den = W0.copy()
        for k in range(self.K):
            p = self.camera_points(k, R[k], t[k])
            z = np.asarray(depths[k], np.float64).reshape(-1)[self.pix[k]]
            d = z - p[:, 2]
            c = np.asarray(colors[k], np.float64).reshape(-1, 3)[self.pix[k]]
            w = self.w[k]
            numD = numD + np.bincount(self.vid[k], w * d, minlength=V)
            for ch in range(3):
                numC[:, ch] = numC[:, ch] + np.bincount(self.vid[k], w * c[:, ch], minlength=V)
            den = den + np.bincount(self.vid[k], w, minlength=V)
        return numD / den, numC / den[:, None], den

    def grad(self, gD, gC, R, t, W, W0=None):
        """Closed-form adjoint at the recorded decisions."""
        H, Wd = self.shape
        gZ = np.zeros((self.K, H * Wd))
        gCol = np.zeros((self.K, H * Wd, 3))
        gxi = np.zeros((self.K, 6))
        for k in range(self.K):
            a = self.w[k] / W[self.vid[k]]
            gd = gD[self.vid[k]] * a
            gZ[k] = np.bincount(self.pix[k], gd, minlength=H * Wd)
            for ch in range(3):
                gCol[k, :, ch] = np.bincount(self.pix[k], gC[self.vid[k], ch] * a, minlength=H * Wd)
            p = self.camera_points(k, R[k], t[k])
            J = np.stack([np.zeros_like(gd), np.zeros_like(gd), np.ones_like(gd), p[:, 1], -p[:, 0],
                          np.zeros_like(gd)], axis=1)
            gxi[k] = gd @ J
        out = {"depth": gZ.reshape(self.K, H, Wd), "color": gCol.reshape(self.K, H, Wd, 3), "xi": gxi}
        if W0 is not None:
            out["D0"] = gD * W0 / W
        return out


def sdf_loss(D, C, target, color_ref=None, lam=0.0):
    """L = sum (D - target)^2 + lam * sum |C - C_ref|^2 and its (g_D, g_C)."""
    r = D - target
    L = float(np.sum(r * r))
    gD = 2.0 * r
    gC = np.zeros_like(C)
    if color_ref is not None and lam > 0:
        rc = C - color_ref
        L += lam * float(np.sum(rc * rc))
        gC = 2.0 * lam * rc
    return L, gD, gC
