"""Pins for the FP64 reference of the variational refinement (Sec. 4):
closed forms of the warp and the derivatives, a pair whose initial flow is
already exact (nothing moves), the direction of the update on a translated
texture, the SOR sweeps against a direct sparse solve, and the iterate as a
stationary point of the linearised energy (finite differences).  CPU only.

The data term's exact form is only cited by the paper; these pins check the
reference against its stated reading, not against the cited method."""
from __future__ import annotations

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.linalg import spsolve

from oracle import variational as va


def _texture(rng, H, W, ch=3):
    from scipy import ndimage
    return np.clip(0.5 + 0.25 * ndimage.gaussian_filter(rng.standard_normal((H, W, ch)), (1.5, 1.5, 0)),
                   0, 1).astype(np.float32)


def test_warp_and_derivatives_closed_forms():
    H, W = 9, 11
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    I = (0.25 * xs - 0.125 * ys + 1.0)[..., None]
    gx, gy = va.grad_c(I)
    np.testing.assert_allclose(gx[:, 1:-1], 0.25)
    np.testing.assert_allclose(gy[1:-1, :], -0.125)
    np.testing.assert_allclose(gx[:, 0], 0.125)          # one-sided at the border
    xx, xy, yy = va.second(I)
    np.testing.assert_allclose(xx[:, 1:-1], 0, atol=1e-15)
    np.testing.assert_allclose(yy[1:-1, :], 0, atol=1e-15)
    np.testing.assert_allclose(xy[1:-1, 1:-1], 0, atol=1e-15)
    u = np.zeros((H, W, 2))
    u[..., 0], u[..., 1] = 0.3, -0.7                     # bilinear of a plane is exact
    w = va.warp(I, u)
    inside = (xs + 0.3 <= W - 1) & (ys - 0.7 >= 0)
    np.testing.assert_allclose(w[..., 0][inside], (0.25 * (xs + 0.3) - 0.125 * (ys - 0.7) + 1.0)[inside])


def _shifted_pair(t, H=40, W=48):
    """A textured bump, constant 0.5 within 8 px of the border, and the same
    image moved by the integer displacement t: I2(x) = I1(x - t)."""
    rng = np.random.default_rng(1)
    I1 = np.full((H, W, 3), 0.5, np.float32)
    I1[8:-8, 8:-8] = _texture(rng, H - 16, W - 16)
    I2 = np.full_like(I1, 0.5)
    tx, ty = t
    I2[max(0, ty):H + min(0, ty), max(0, tx):W + min(0, tx)] = \
        I1[max(0, -ty):H - max(0, ty), max(0, -tx):W - max(0, tx)]
    return I1, I2


def test_exact_initial_flow_stays():
    """u0 = the true translation: I2 warped by u0 is I1, every residual and
    right-hand side is zero, and the refinement returns u0 exactly."""
    I1, I2 = _shifted_pair((3, -2))
    u0 = np.zeros(I1.shape[:2] + (2,), np.float32)
    u0[..., 0], u0[..., 1] = 3.0, -2.0
    np.testing.assert_array_equal(va.refine(I1, I2, u0), u0.astype(np.float64))


def test_update_moves_towards_the_translation():
    """From u0 off by (0.4, -0.3) px, the refinement moves the flow towards
    the true translation wherever the texture constrains it."""
    I1, I2 = _shifted_pair((3, -2))
    u0 = np.zeros(I1.shape[:2] + (2,), np.float32)
    u0[..., 0], u0[..., 1] = 3.4, -2.3
    out = va.refine(I1, I2, u0)
    inner = (slice(12, -12), slice(12, -12))
    e0 = np.linalg.norm(u0[inner] - [3.0, -2.0], axis=-1).mean()
    e1 = np.linalg.norm(out[inner] - [3.0, -2.0], axis=-1).mean()
    assert e1 < 0.5 * e0, (e0, e1)


def _assemble(A11, A12, A22, b1, b2, gx, gy, u0):
    """The linear system the SOR sweeps solve, as a sparse matrix over the
    unknowns (du, dv) of every pixel."""
    H, W = A11.shape
    n = H * W
    idx = np.arange(n).reshape(H, W)
    rows, cols, vals = [], [], []
    rhs = np.concatenate([b1.ravel(), b2.ravel()])
    diag_s = np.zeros((H, W))

    def add(r, c, v):
        rows.append(r.ravel()), cols.append(c.ravel()), vals.append(v.ravel())
    for g, a, b in ((gx, idx[:, :-1], idx[:, 1:]), (gy, idx[:-1, :], idx[1:, :])):
        for comp in (0, 1):
            add(a + comp * n, b + comp * n, -g)
            add(b + comp * n, a + comp * n, -g)
        np.add.at(diag_s, np.unravel_index(a.ravel(), (H, W)), g.ravel())
        np.add.at(diag_s, np.unravel_index(b.ravel(), (H, W)), g.ravel())
        # right-hand side: g (u0_j - u0_i) on both ends
        for comp in (0, 1):
            d = u0[..., comp].ravel()
            np.add.at(rhs, a.ravel() + comp * n, g.ravel() * (d[b.ravel()] - d[a.ravel()]))
            np.add.at(rhs, b.ravel() + comp * n, g.ravel() * (d[a.ravel()] - d[b.ravel()]))
    add(idx, idx, A11 + diag_s)
    add(idx + n, idx + n, A22 + diag_s)
    add(idx, idx + n, A12)
    add(idx + n, idx, A12)
    M = coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(2 * n, 2 * n))
    return M.tocsr(), rhs


def test_sor_sweeps_solve_the_linear_system():
    """With the weights of one fixed-point step held, many red-black sweeps
    converge to scipy's direct solution of the assembled system."""
    rng = np.random.default_rng(2)
    H, W = 10, 13
    I1 = _texture(rng, H, W)
    I2 = _texture(rng, H, W)
    u0 = rng.normal(0, 0.5, (H, W, 2))
    p = va.Params()
    JC, JG, alpha = va.coefficients(I1, I2, u0, p)
    du, dv = np.zeros((H, W)), np.zeros((H, W))
    A11, A12, A22, b1, b2, gx, gy = va.weights(JC, JG, alpha, u0, du, dv, p)
    for _ in range(3000):
        va.sor_sweep(A11, A12, A22, b1, b2, gx, gy, u0, du, dv, p, 0)
        va.sor_sweep(A11, A12, A22, b1, b2, gx, gy, u0, du, dv, p, 1)
    M, rhs = _assemble(A11, A12, A22, b1, b2, gx, gy, u0)
    x = spsolve(M, rhs)
    np.testing.assert_allclose(du.ravel(), x[:H * W], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(dv.ravel(), x[H * W:], rtol=1e-8, atol=1e-10)


def test_iterate_is_a_stationary_point_of_the_energy():
    """Run to convergence, the iterate zeroes the gradient of the linearised
    energy, checked by central finite differences at sampled unknowns
    against the gradient's size at du = 0."""
    rng = np.random.default_rng(3)
    H, W = 12, 14
    I1 = _texture(rng, H, W)
    I2 = _texture(rng, H, W)
    u0 = rng.normal(0, 0.5, (H, W, 2))
    p = va.Params(fixed_point=200, sor=200)
    _, du, dv = va.refine(I1, I2, u0, p, return_du=True)
    JC, JG, alpha = va.coefficients(I1, I2, u0, p)
    u0d = np.asarray(u0, np.float32).astype(np.float64)

    def grad_at(du, dv, y, x, comp, h=1e-7):
        a, b = du.copy(), dv.copy()
        tgt = a if comp == 0 else b
        tgt[y, x] += h
        ep = va.energy_lin(JC, JG, alpha, u0d, a, b, p)
        tgt[y, x] -= 2 * h
        em = va.energy_lin(JC, JG, alpha, u0d, a, b, p)
        return (ep - em) / (2 * h)
    z = np.zeros((H, W))
    pts = [(int(rng.integers(0, H)), int(rng.integers(0, W)), c) for c in (0, 1) for _ in range(6)]
    g0 = max(abs(grad_at(z, z, y, x, c)) for y, x, c in pts)
    g1 = max(abs(grad_at(du, dv, y, x, c)) for y, x, c in pts)
    assert g0 > 1e-3 and g1 <= 1e-4 * g0, (g0, g1)


def test_empty_equations_keep_the_initial_flow():
    """An equation with a zero diagonal says nothing about its unknown: a
    1 x 1 image (no gradient, no neighbour) and a flat image with lam = 0
    return the initial field unchanged, without NaN."""
    rng = np.random.default_rng(11)
    I1 = rng.uniform(0, 1, (1, 1, 3))
    u0 = np.array([[[1.5, -2.0]]])
    out = va.refine(I1, I1 + 0.1, u0)
    assert np.array_equal(out, u0.astype(np.float32).astype(np.float64))
    flat = np.full((6, 9), 0.4)
    u0 = rng.normal(0, 1, (6, 9, 2))
    out = va.refine(flat, flat + 0.2, u0, va.Params(lam=0.0))
    assert np.array_equal(out, u0.astype(np.float32).astype(np.float64))
    # with lam > 0 the flat image's field is smoothed, and stays finite
    out = va.refine(flat, flat + 0.2, u0)
    assert np.isfinite(out).all() and np.std(out[..., 0]) < np.std(u0[..., 0])
