"""FP64 reference of the one-level variational refinement that follows the
interpolation (Sec. 4 of the paper, "Variational Energy Minimization").

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library's
refinement.  Only tests, the smoke check and the benchmark's CPU-baseline
leg use it.  Plain numpy, float64, written for reading, not speed.

What the paper fixes: an energy of a data term plus a smoothness term that
penalises the flow gradient norm with a local weight alpha(x) =
exp(-kappa ||grad I||), kappa = 5; minimised from the interpolated field,
without coarse-to-fine, by 5 fixed-point iterations (the non-linear weights
of the Euler-Lagrange equations recomputed, then the flow update solved) with
30 successive-over-relaxation iterations per linear system.  The data term
is only cited (colour and gradient constancy with a normalisation); its form
here is this repository's reading of that description:

  I2w(x)   = I2(x + u0(x)), bilinear, coordinates clamped to the image
  derivatives: central differences with the border pixel repeated; second
           derivatives Ixx = I(x+1) - 2 I(x) + I(x-1) (likewise Iyy) and
           Ixy = (I(x+1,y+1) - I(x-1,y+1) - I(x+1,y-1) + I(x-1,y-1)) / 4,
           all of I2w; Iz = I2w - I1; Ixz, Iyz = d/dx, d/dy of I2w minus the
           same of I1
  colour:   r_c  = Iz + Ix du + Iy dv,     theta_c  = 1 / (Ix^2 + Iy^2 + zeta^2)
  gradient: rx_c = Ixz + Ixx du + Ixy dv,  thetax_c = 1 / (Ixx^2 + Ixy^2 + zeta^2)
            ry_c = Iyz + Ixy du + Iyy dv,  thetay_c = 1 / (Ixy^2 + Iyy^2 + zeta^2)
  E = sum_x  delta psi(sum_c theta_c r_c^2)
           + gamma psi(sum_c thetax_c rx_c^2 + thetay_c ry_c^2)
      + sum over edges (i, j) between 4-neighbours of
             lam (alpha_i + alpha_j) / 2 psi(|U_j - U_i|^2 + |V_j - V_i|^2)
  with U = u0 + du, V = v0 + dv: the flow gradient's norm penalised along
  each grid direction (forward differences), which makes the discrete
  Euler-Lagrange equations exactly the linear system below;
  psi(s^2) = sqrt(s^2 + eps^2), alpha(x) = exp(-kappa ||grad I1(x)||).
The data term is linearised once about u0 (one level, one warp); each
fixed-point iteration evaluates psi' (= 1 / (2 sqrt(s^2 + eps^2))) at the
current (du, dv) -- per pixel for the data term, per edge for the
smoothness term, g_ij = lam (alpha_i + alpha_j) / 2 psi'(...) -- and solves
   (A11 + sum_j g_ij) du_i + A12 dv_i = b1 + sum_j g_ij (U_j - u0_i)
   A12 du_i + (A22 + sum_j g_ij) dv_i = b2 + sum_j g_ij (V_j - v0_i)
by 30 red-black SOR sweeps (red: x + y even, then black; du before dv at
each pixel); an equation whose diagonal is zero (no image gradient and no
neighbour weight) leaves its unknown unchanged.  The result is u0 + du.

Pinning: the tests pin this code to the mathematics of the energy above
(closed forms of the warp and derivatives, the SOR solve against a direct
sparse solve, stationarity of the linearised energy at the converged
iterate, the exact field staying put).  The paper itself fixes only
alpha, kappa and the iteration counts: the data term's form and the
weights delta, gamma, lam, zeta, eps and omega are this reading, so for
the data term parity with the paper's method is partly unpinned.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Params:
    lam: float = 0.1        # smoothness weight (global)
    delta: float = 0.1      # colour-constancy weight
    gamma: float = 0.7      # gradient-constancy weight
    kappa: float = 5.0      # alpha(x) = exp(-kappa ||grad I1||) (paper: 5)
    eps: float = 1e-3       # psi(s^2) = sqrt(s^2 + eps^2)
    zeta: float = 0.1       # normalisation floor
    omega: float = 1.6      # over-relaxation
    fixed_point: int = 5    # paper: 5
    sor: int = 30           # paper: 30


def _pad(a):
    """Repeat the border pixel once on every side (first two axes)."""
    return np.pad(a, [(1, 1), (1, 1)] + [(0, 0)] * (a.ndim - 2), mode="edge")


def grad_c(a):
    """Central differences (a(x+1) - a(x-1)) / 2, border repeated."""
    p = _pad(a)
    return (p[1:-1, 2:] - p[1:-1, :-2]) / 2.0, (p[2:, 1:-1] - p[:-2, 1:-1]) / 2.0


def second(a):
    p = _pad(a)
    xx = p[1:-1, 2:] - 2.0 * p[1:-1, 1:-1] + p[1:-1, :-2]
    yy = p[2:, 1:-1] - 2.0 * p[1:-1, 1:-1] + p[:-2, 1:-1]
    xy = (p[2:, 2:] - p[2:, :-2] - p[:-2, 2:] + p[:-2, :-2]) / 4.0
    return xx, xy, yy


def warp(I2, u):
    """I2 sampled at x + u(x), bilinear, with the coordinates clamped to the
    image."""
    H, W = I2.shape[:2]
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    x = np.clip(xs + u[..., 0], 0.0, W - 1.0)
    y = np.clip(ys + u[..., 1], 0.0, H - 1.0)
    x0 = np.minimum(np.floor(x).astype(np.int64), W - 2 if W > 1 else 0)
    y0 = np.minimum(np.floor(y).astype(np.int64), H - 2 if H > 1 else 0)
    x1, y1 = np.minimum(x0 + 1, W - 1), np.minimum(y0 + 1, H - 1)
    fx, fy = (x - x0)[..., None], (y - y0)[..., None]
    return ((1 - fy) * ((1 - fx) * I2[y0, x0] + fx * I2[y0, x1])
            + fy * ((1 - fx) * I2[y1, x0] + fx * I2[y1, x1]))


def coefficients(I1, I2, u0, p: Params):
    """Per pixel: the colour and gradient systems J (each the entries 11, 12,
    22, 13, 23, 33 of sum theta [a b c]^T [a b c]) and alpha(x)."""
    I1 = np.asarray(I1, np.float32).astype(np.float64)
    I2 = np.asarray(I2, np.float32).astype(np.float64)
    if I1.ndim == 2:
        I1, I2 = I1[..., None], I2[..., None]
    u0 = np.asarray(u0, np.float32).astype(np.float64)
    I2w = warp(I2, u0)
    Ix, Iy = grad_c(I2w)
    Iz = I2w - I1
    g1x, g1y = grad_c(I1)
    Ixx, Ixy, Iyy = second(I2w)
    Ixz, Iyz = Ix - g1x, Iy - g1y
    z2 = p.zeta ** 2
    th = 1.0 / (Ix ** 2 + Iy ** 2 + z2)
    thx = 1.0 / (Ixx ** 2 + Ixy ** 2 + z2)
    thy = 1.0 / (Ixy ** 2 + Iyy ** 2 + z2)

    def J(terms):
        out = np.zeros(I1.shape[:2] + (6,))
        for w, a, b, c in terms:
            out[..., 0] += (w * a * a).sum(-1)
            out[..., 1] += (w * a * b).sum(-1)
            out[..., 2] += (w * b * b).sum(-1)
            out[..., 3] += (w * a * c).sum(-1)
            out[..., 4] += (w * b * c).sum(-1)
            out[..., 5] += (w * c * c).sum(-1)
        return out
    JC = J([(th, Ix, Iy, Iz)])
    JG = J([(thx, Ixx, Ixy, Ixz), (thy, Ixy, Iyy, Iyz)])
    gn = np.sqrt((g1x ** 2 + g1y ** 2).sum(-1))
    alpha = np.exp(-p.kappa * gn)
    return JC, JG, alpha


def psi_d(s2, eps):
    """psi'(s^2) = 1 / (2 sqrt(s^2 + eps^2)) for psi(s^2) = sqrt(s^2 + eps^2).
    (The factor 2 of d(s^2) appears in every Euler-Lagrange term and is
    divided out of all of them.)"""
    return 0.5 / np.sqrt(s2 + eps * eps)


def quad(J, du, dv):
    """[du dv 1] J [du dv 1]^T."""
    return (J[..., 0] * du * du + 2 * J[..., 1] * du * dv + J[..., 2] * dv * dv
            + 2 * J[..., 3] * du + 2 * J[..., 4] * dv + J[..., 5])


def weights(JC, JG, alpha, u0, du, dv, p: Params):
    """One fixed-point step's linear system: per pixel A11, A12, A22, b1, b2
    (data term); per edge gx (pixel and its right neighbour, H x W-1) and
    gy (pixel and the one below, H-1 x W) (smoothness)."""
    wc = p.delta * psi_d(quad(JC, du, dv), p.eps)
    wg = p.gamma * psi_d(quad(JG, du, dv), p.eps)
    A11 = wc * JC[..., 0] + wg * JG[..., 0]
    A12 = wc * JC[..., 1] + wg * JG[..., 1]
    A22 = wc * JC[..., 2] + wg * JG[..., 2]
    b1 = -(wc * JC[..., 3] + wg * JG[..., 3])
    b2 = -(wc * JC[..., 4] + wg * JG[..., 4])
    U, V = u0[..., 0] + du, u0[..., 1] + dv
    gx = p.lam * 0.5 * (alpha[:, 1:] + alpha[:, :-1]) * psi_d(
        (U[:, 1:] - U[:, :-1]) ** 2 + (V[:, 1:] - V[:, :-1]) ** 2, p.eps)
    gy = p.lam * 0.5 * (alpha[1:, :] + alpha[:-1, :]) * psi_d(
        (U[1:, :] - U[:-1, :]) ** 2 + (V[1:, :] - V[:-1, :]) ** 2, p.eps)
    return A11, A12, A22, b1, b2, gx, gy


def _neighbour_sums(gx, gy, u0, du, dv):
    """sum_j g_ij, sum_j g_ij (U_j - u0_i), sum_j g_ij (V_j - v0_i)."""
    H, W = du.shape
    U, V = u0[..., 0] + du, u0[..., 1] + dv
    sw, su, sv = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W))
    # right neighbour (edge gx[:, x]) and left neighbour (gx[:, x-1])
    sw[:, :-1] += gx
    su[:, :-1] += gx * (U[:, 1:] - u0[:, :-1, 0])
    sv[:, :-1] += gx * (V[:, 1:] - u0[:, :-1, 1])
    sw[:, 1:] += gx
    su[:, 1:] += gx * (U[:, :-1] - u0[:, 1:, 0])
    sv[:, 1:] += gx * (V[:, :-1] - u0[:, 1:, 1])
    # neighbour below and above
    sw[:-1, :] += gy
    su[:-1, :] += gy * (U[1:, :] - u0[:-1, :, 0])
    sv[:-1, :] += gy * (V[1:, :] - u0[:-1, :, 1])
    sw[1:, :] += gy
    su[1:, :] += gy * (U[:-1, :] - u0[1:, :, 0])
    sv[1:, :] += gy * (V[:-1, :] - u0[1:, :, 1])
    return sw, su, sv


def sor_sweep(A11, A12, A22, b1, b2, gx, gy, u0, du, dv, p: Params, color):
    """Update every pixel of one colour (x + y even = 0, odd = 1) in place,
    du first, then dv with the new du.  A pixel's neighbours all have the
    other colour, so updating one colour at once is the sequential order."""
    H, W = du.shape
    ys, xs = np.mgrid[0:H, 0:W]
    sel = ((xs + ys) & 1) == color
    sw, su, sv = _neighbour_sums(gx, gy, u0, du, dv)
    # a zero diagonal (no image gradient and no neighbour weight: a flat
    # 1 x 1 image, or lam = 0 on a flat region) leaves the equation empty:
    # that unknown keeps its value
    du_u = sel & (A11 + sw > 0)
    nu = (b1 - A12 * dv + su) / np.where(du_u, A11 + sw, 1.0)
    du_new = np.where(du_u, (1 - p.omega) * du + p.omega * nu, du)
    dv_u = sel & (A22 + sw > 0)
    nv = (b2 - A12 * du_new + sv) / np.where(dv_u, A22 + sw, 1.0)
    dv_new = np.where(dv_u, (1 - p.omega) * dv + p.omega * nv, dv)
    du[...] = du_new
    dv[...] = dv_new


def refine(I1, I2, u0, p: Params | None = None, return_du=False):
    """The refined flow u0 + du (H, W, 2) in float64."""
    p = Params() if p is None else p
    u0 = np.asarray(u0, np.float32).astype(np.float64)
    JC, JG, alpha = coefficients(I1, I2, u0, p)
    H, W = u0.shape[:2]
    du, dv = np.zeros((H, W)), np.zeros((H, W))
    for _ in range(p.fixed_point):
        A11, A12, A22, b1, b2, gx, gy = weights(JC, JG, alpha, u0, du, dv, p)
        for _ in range(p.sor):
            sor_sweep(A11, A12, A22, b1, b2, gx, gy, u0, du, dv, p, 0)
            sor_sweep(A11, A12, A22, b1, b2, gx, gy, u0, du, dv, p, 1)
    out = u0 + np.stack([du, dv], -1)
    return (out, du, dv) if return_du else out


def energy_lin(JC, JG, alpha, u0, du, dv, p: Params):
    """The linearised energy whose stationary point the iteration seeks."""
    U, V = u0[..., 0] + du, u0[..., 1] + dv
    ps = lambda s2: np.sqrt(s2 + p.eps ** 2)
    e = (p.delta * ps(quad(JC, du, dv)) + p.gamma * ps(quad(JG, du, dv))).sum()
    e += (p.lam * 0.5 * (alpha[:, 1:] + alpha[:, :-1])
          * ps((U[:, 1:] - U[:, :-1]) ** 2 + (V[:, 1:] - V[:, :-1]) ** 2)).sum()
    e += (p.lam * 0.5 * (alpha[1:, :] + alpha[:-1, :])
          * ps((U[1:, :] - U[:-1, :]) ** 2 + (V[1:, :] - V[:-1, :]) ** 2)).sum()
    return float(e)
