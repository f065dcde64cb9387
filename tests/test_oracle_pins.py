"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Every pin is chosen so that a plausible slip (a dropped term, a wrong sign or
index, a transposed operand) fails one of them:
* complex-step derivatives of the oracle's own energies (exact to rounding for
  analytic functions) check the hand-derived gradients and Hessians;
* textbook linear-elasticity stiffness matrices (Voigt B^T C B) check the rest
  Hessians and the Stable Neo-Hookean re-parametrisation;
* closed forms (rest energy, uniaxial stretch, rotating one hinge wing) and
  invariants (translation, rotation, relabelling, symmetry);
* brute force for the sparsity pattern and closed-form block counts;
* matrices with known eigen-decomposition for the PSD projection;
* a direct sparse solve and exact rigid-motion solutions for the Newton step.
"""
import itertools

import numpy as np
import pytest

import scenegen as sg
from oracle import contact, assembly, elements, newton, projection, rest


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _cs_grad(f, x, h=1e-30):
    """Complex-step gradient of a batched scalar function f(x) -> (E,)."""
    E, k, _ = x.shape
    g = np.zeros((E, k, 3))
    for a in range(k):
        for i in range(3):
            xc = x.astype(complex)
            xc[:, a, i] += 1j * h
            g[:, a, i] = np.imag(f(xc)) / h
    return g


def _cs_jac(gf, x, h=1e-30):
    """Complex-step Jacobian of a batched gradient function -> (E,k,3,k,3)."""
    E, k, _ = x.shape
    H = np.zeros((E, k, 3, k, 3))
    for b in range(k):
        for j in range(3):
            xc = x.astype(complex)
            xc[:, b, j] += 1j * h
            H[:, :, :, b, j] = np.imag(gf(xc)) / h
    return H


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ----------------------------------------------------------------------------
# Stable Neo-Hookean tet4
# ----------------------------------------------------------------------------
MU, LAM = rest.lame(1e5, 0.4)


def _snh(x, X, **kw):
    n = x.shape[0]
    return elements.snh_tet4(x, X, np.full(n, MU), np.full(n, LAM), **kw)


def test_lame_c1_values():
    # E = 1e5, nu = 0.4: mu = E/2.8, lambda = 0.4E/0.28
    assert MU == pytest.approx(1e5 / 2.8, rel=1e-15)
    assert LAM == pytest.approx(0.4e5 / 0.28, rel=1e-15)
    mu_, lam_ = rest.snh_reparam(MU, LAM)
    assert mu_ == pytest.approx(47619.047619047619, rel=1e-14)
    assert lam_ == pytest.approx(172619.04761904762, rel=1e-14)


def test_snh_gradient_complex_step():
    x, X = sg.random_tets(40, seed=11)
    _, g, _ = _snh(x, X, want_hess=False)
    gc = _cs_grad(lambda xc: _snh(xc, X, want_hess=False)[0], x)
    assert _rel(g, gc) < 1e-12


def test_snh_hessian_complex_step():
    x, X = sg.random_tets(40, seed=12)
    _, _, H = _snh(x, X)
    Hc = _cs_jac(lambda xc: _snh(xc, X, want_hess=False)[1], x)
    assert _rel(H, Hc) < 1e-12


def test_snh_central_differences():
    x, X = sg.random_tets(5, seed=13)
    E, g, _ = _snh(x, X, want_hess=False)
    h = 1e-8
    for a, i in [(0, 0), (1, 2), (3, 1)]:
        xp = x.copy(); xp[:, a, i] += h
        xm = x.copy(); xm[:, a, i] -= h
        fd = (_snh(xp, X, want_hess=False)[0] - _snh(xm, X, want_hess=False)[0]) / (2 * h)
        assert np.allclose(fd, g[:, a, i], rtol=1e-5, atol=1e-6 * np.abs(g).max())


def _tet_rest():
    _, X = sg.random_tets(8, seed=14)
    return X


def test_snh_rest_energy_closed_form():
    # psi(I) = lam'/2 (1-alpha)^2 - mu'/2 log 4 with 1 - alpha = -3 mu'/(4 lam')
    X = _tet_rest()
    E, g, _ = _snh(X, X, want_hess=False)
    mu_ = 4.0 / 3.0 * MU
    lam_ = LAM + 5.0 / 6.0 * MU
    psi_I = 9.0 * mu_ ** 2 / (32.0 * lam_) - 0.5 * mu_ * np.log(4.0)
    assert psi_I == pytest.approx(-29312.4, abs=0.05)            # E=1e5, nu=0.4
    V = np.abs(np.linalg.det(np.stack([X[:, a] - X[:, 0] for a in (1, 2, 3)], 2))) / 6
    assert np.allclose(E, V * psi_I, rtol=1e-13)
    # zero rest gradient (relative to a typical nodal force scale mu*h^2)
    assert np.max(np.abs(g)) < 1e-9 * MU * 1e-4


def _voigt_C3(mu, lam):
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[[0, 1, 2], [0, 1, 2]] = lam + 2 * mu
    C[[3, 4, 5], [3, 4, 5]] = mu
    return C


def _cst_tet_stiffness(X, mu, lam):
    """Textbook constant-strain tet: K = V B^T C B (Voigt, engineering shear)."""
    Dm = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    V = abs(np.linalg.det(Dm)) / 6.0
    # shape-function gradients from the 4x4 system [1 X] c = I
    M = np.hstack([np.ones((4, 1)), X])
    grads = np.linalg.inv(M)[1:, :].T          # (4,3): dN_a/dX
    B = np.zeros((6, 12))
    for a in range(4):
        dx, dy, dz = grads[a]
        B[0, 3 * a + 0] = dx
        B[1, 3 * a + 1] = dy
        B[2, 3 * a + 2] = dz
        B[3, 3 * a + 1] = dz; B[3, 3 * a + 2] = dy      # gamma_yz
        B[4, 3 * a + 0] = dz; B[4, 3 * a + 2] = dx      # gamma_xz
        B[5, 3 * a + 0] = dy; B[5, 3 * a + 1] = dx      # gamma_xy
    return V * B.T @ _voigt_C3(mu, lam) @ B


def test_snh_rest_hessian_is_linear_elasticity():
    X = _tet_rest()
    _, _, H = _snh(X, X)
    for e in range(X.shape[0]):
        K = _cst_tet_stiffness(X[e], MU, LAM)
        assert _rel(H[e].reshape(12, 12), K) < 1e-12
        ev = np.linalg.eigvalsh(K)
        assert np.sum(np.abs(ev) < 1e-9 * ev.max()) == 6        # rigid modes


def test_snh_invariances_and_symmetry():
    x, X = sg.random_tets(20, seed=15)
    E, g, H = _snh(x, X)
    Hm = H.reshape(-1, 12, 12)
    assert _rel(Hm, np.swapaxes(Hm, 1, 2)) < 1e-13
    # translation: sum of nodal forces = 0, H (1 (x) t) = 0
    assert np.max(np.abs(g.sum(axis=1))) < 1e-12 * np.abs(g).max()
    t = np.tile(np.array([0.3, -0.7, 0.2]), 4)
    assert np.max(np.abs(Hm @ t)) < 1e-11 * np.abs(Hm).max()
    # rotation
    R = _rot(3)
    E2, g2, H2 = _snh(x @ R.T, X)
    assert np.allclose(E2, E, rtol=1e-12, atol=1e-12 * np.abs(E).max())
    assert _rel(g2, g @ R.T) < 1e-11
    RR = np.kron(np.eye(4), R)
    assert _rel(H2.reshape(-1, 12, 12), RR @ Hm @ RR.T) < 1e-11
    # relabelling the vertices (same permutation of x and X) leaves E unchanged
    for perm in ([1, 2, 3, 0], [2, 0, 1, 3], [3, 2, 1, 0]):
        E3, g3, _ = _snh(x[:, perm], X[:, perm], want_hess=False)
        assert np.allclose(E3, E, rtol=1e-12, atol=1e-12 * np.abs(E).max())
        assert _rel(g3, g[:, perm]) < 1e-11


# ----------------------------------------------------------------------------
# StVK membrane
# ----------------------------------------------------------------------------
# ----------------------------------------------------------------------------
# Other App. B materials on tets (classic NH, StVK, fixed co-rotational, ARAP)
# ----------------------------------------------------------------------------
def _mat(kind, x, X, R=None, **kw):
    n = x.shape[0]
    mu, lam = np.full(n, MU), np.full(n, LAM)
    if kind == "nh":
        return elements.nh_tet4(x, X, mu, lam, **kw)
    if kind == "stvk":
        return elements.stvk_tet4(x, X, mu, lam, **kw)
    if kind == "fcr":
        return elements.fcr_tet4(x, X, mu, lam, R, **kw)
    return elements.arap_tet4(x, X, mu, lam, R, **kw)


@pytest.mark.parametrize("kind", ["nh", "stvk", "fcr", "arap"])
def test_material_derivatives_complex_step(kind):
    x, X = sg.random_tets(25, seed=31, inverted_frac=0.0)    # log J needs J > 0
    R = np.stack([_rot(s) for s in range(25)])
    E, g, H = _mat(kind, x, X, R)
    gc = _cs_grad(lambda xc: _mat(kind, xc, X, R, want_hess=False)[0], x)
    Hc = _cs_jac(lambda xc: _mat(kind, xc, X, R, want_hess=False)[1], x)
    assert _rel(g, gc) < 1e-12
    assert _rel(H, Hc) < 1e-12


@pytest.mark.parametrize("kind", ["nh", "stvk"])
def test_nh_and_stvk_rest_is_linear_elasticity(kind):
    X = _tet_rest()
    E, g, H = _mat(kind, X, X)
    assert np.max(np.abs(E)) < 1e-12 * MU * 1e-6
    assert np.max(np.abs(g)) < 1e-9 * MU * 1e-4
    for e in range(X.shape[0]):
        assert _rel(H[e].reshape(12, 12), _cst_tet_stiffness(X[e], MU, LAM)) < 1e-12


@pytest.mark.parametrize("kind,c", [("fcr", 2.0), ("arap", 1.0)])
def test_lagged_rotation_rest_hessian_closed_form(kind, c):
    """With R = I at rest: E = 0, g = 0 and d2psi = c mu d_ik d_jl + lam d_ij d_kl,
    so block (a,b) = V (c mu (b_a . b_b) I + lam b_a b_b^T), b_a the shape
    gradients (rows of Dm^-1 and minus their sum)."""
    X = _tet_rest()
    R = np.broadcast_to(np.eye(3), (X.shape[0], 3, 3))
    E, g, H = _mat(kind, X, X, R)
    assert np.max(np.abs(E)) < 1e-12 * MU * 1e-6
    assert np.max(np.abs(g)) < 1e-9 * MU * 1e-4
    for e in range(X.shape[0]):
        M = np.hstack([np.ones((4, 1)), X[e]])
        bg = np.linalg.inv(M)[1:, :].T                       # dN_a/dX, (4,3)
        V = abs(np.linalg.det(np.stack([X[e][a] - X[e][0] for a in (1, 2, 3)], 1))) / 6
        K = np.zeros((4, 3, 4, 3))
        for a in range(4):
            for b in range(4):
                K[a, :, b, :] = V * (c * MU * (bg[a] @ bg[b]) * np.eye(3)
                                     + LAM * np.outer(bg[a], bg[b]))
        assert _rel(H[e], K) < 1e-12


@pytest.mark.parametrize("kind", ["fcr", "arap"])
def test_lagged_rotation_energies_rotate_with_r(kind):
    """Rotating positions and the lagged rotation together leaves E unchanged
    and rotates g and H; translation leaves everything unchanged."""
    x, X = sg.random_tets(20, seed=32, inverted_frac=0.2)
    R = np.stack([_rot(s + 40) for s in range(20)])
    E, g, H = _mat(kind, x, X, R)
    Q = _rot(5)
    E2, g2, H2 = _mat(kind, x @ Q.T, X, Q[None] @ R)
    assert np.allclose(E2, E, rtol=1e-12, atol=1e-12 * np.abs(E).max())
    assert _rel(g2, g @ Q.T) < 1e-11
    QQ = np.kron(np.eye(4), Q)
    assert _rel(H2.reshape(-1, 12, 12), QQ @ H.reshape(-1, 12, 12) @ QQ.T) < 1e-11
    E3, g3, _ = _mat(kind, x + np.array([0.2, -0.1, 0.3]), X, R)
    assert np.allclose(E3, E, rtol=1e-12) and _rel(g3, g) < 1e-12


def test_closest_rotation():
    rng = np.random.default_rng(33)
    Q = np.stack([_rot(s + 60) for s in range(30)])
    A = rng.normal(size=(30, 3, 3))
    S = A @ np.swapaxes(A, 1, 2) + 0.5 * np.eye(3)
    R = elements.closest_rotation(Q @ S)                    # polar factor of Q S is Q
    assert _rel(R, Q) < 1e-12
    F = rng.normal(size=(30, 3, 3))                        # some with det F < 0
    R = elements.closest_rotation(F)
    assert np.max(np.abs(R @ np.swapaxes(R, 1, 2) - np.eye(3))) < 1e-13
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-13)
    best = np.einsum("eij,eij->e", R, F)
    for s in range(300):                                  # no rotation does better
        T = _rot(s + 100)
        assert np.all(np.einsum("ij,eij->e", T, F) <= best + 1e-12)


# ----------------------------------------------------------------------------
# Conditional contact barrier: point against the plane of a triangle
# ----------------------------------------------------------------------------
def _contact_elems(n, seed, d_lo=0.1, d_hi=2.0):
    """Random triangles and points at signed distance in [d_lo, d_hi] * 1e-3
    above them (plus an in-plane offset)."""
    rng = np.random.default_rng(seed)
    t = rng.normal(size=(n, 3, 3)) * 0.01
    N = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    nrm = N / np.linalg.norm(N, axis=1, keepdims=True)
    d = rng.uniform(d_lo, d_hi, n) * 1e-3
    p = t.mean(axis=1) + rng.normal(size=(n, 3)) * 0.003
    p = p - np.einsum("ei,ei->e", p - t[:, 0], nrm)[:, None] * nrm + d[:, None] * nrm
    return np.concatenate([p[:, None], t], axis=1), d


def test_point_plane_distance_closed_form_and_derivatives():
    x, d_true = _contact_elems(30, 101)
    d, dd, d2d = contact.point_plane_distance(x)
    assert np.allclose(d, d_true, rtol=1e-12)
    # complex-step gradient and Hessian of the distance
    gc = _cs_grad(lambda xc: contact.point_plane_distance(xc)[0], x).reshape(30, 12)
    Hc = _cs_jac(lambda xc: contact.point_plane_distance(xc)[1].reshape(-1, 4, 3), x)
    assert _rel(dd, gc) < 1e-12
    assert _rel(d2d, Hc.reshape(30, 12, 12)) < 1e-10
    # translation and rotation invariance; the gradient of p is the unit normal
    Q = _rot(102)
    d2, _, _ = contact.point_plane_distance(x @ Q.T + 0.3)
    assert np.allclose(d2, d, rtol=1e-12)
    assert np.allclose(np.linalg.norm(dd[:, :3], axis=1), 1.0)


def test_contact_barrier_and_activation():
    """b(d) vanishes with its first two derivatives at d = d_hat (the
    conditional energy is C2 across the activation boundary); complex-step
    derivatives of b and of the element energy; inactive elements give zero,
    a point through the plane gives +inf."""
    kc, dhat = 1e3, 1e-3
    dv = np.linspace(0.05, 0.999, 25) * dhat
    b, b1, b2 = contact.barrier(dv, kc, dhat)
    h = 1e-30
    assert np.allclose(b1, np.imag(contact.barrier(dv + 1j * h, kc, dhat)[0]) / h, rtol=1e-12)
    assert np.allclose(b2, np.imag(contact.barrier(dv + 1j * h, kc, dhat)[1]) / h, rtol=1e-12)
    bb = contact.barrier(np.array([dhat]), kc, dhat)
    assert all(abs(v[0]) < 1e-18 for v in bb)
    x, d = _contact_elems(40, 103, d_lo=0.2, d_hi=1.8)            # about half active
    E, g, H, act = contact.point_plane_barrier(x, kc, dhat)
    assert np.array_equal(act, d < dhat) and 5 < act.sum() < 35
    assert np.all(E[~act] == 0) and np.all(g[~act] == 0) and np.all(H[~act] == 0)
    assert np.all(E[act] > 0)
    xa = x[act]
    gc = _cs_grad(lambda xc: contact.point_plane_barrier(xc, kc, dhat, False)[0], xa)
    Hc = _cs_jac(lambda xc: contact.point_plane_barrier(xc, kc, dhat, False)[1], xa)
    assert _rel(g[act], gc) < 1e-11
    assert _rel(H[act], Hc) < 1e-9
    xin = x[:1].copy()
    d0, dd0, _ = contact.point_plane_distance(xin)
    xin[0, 0] -= (d0[0] + 1e-4) * dd0[0, :3]                      # through the plane
    E2, _, _, act2 = contact.point_plane_barrier(xin, kc, dhat)
    assert act2[0] and np.isinf(E2[0])


# ----------------------------------------------------------------------------
# Stable Neo-Hookean tet4 with the density Hessian filtered to PSD
# ----------------------------------------------------------------------------
def _signed_svd(F):
    U, s, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U) * np.linalg.det(Vt))
    U[:, :, 2] *= np.where(np.linalg.det(U) < 0, -1.0, 1.0)[:, None]
    Vt[:, 2, :] *= np.where(np.linalg.det(Vt) < 0, -1.0, 1.0)[:, None]
    return U, s * np.stack([np.ones_like(d), np.ones_like(d), d], 1), Vt


def test_snh_density_hessian_eigensystem():
    """The eigenvalues of d2psi/dF2 (9x9) are, with the rotation-variant SVD
    F = U diag(s) V^T (s3 < 0 when inverted): 2 psi_2 + psi_3 s_k (twists) and
    2 psi_2 - psi_3 s_k (flips) for each pair, and those of the 3x3 scaling
    block 2 psi_2 I + 4 psi_22 s s^T + psi_3 offdiag(s_k) + psi_33 c c^T with
    c = (s2 s3, s1 s3, s1 s2) (Smith et al. 2019, for psi(I2, I3))."""
    x, X = sg.random_tets(40, seed=81, inverted_frac=0.3)
    mu_, lam_ = rest.snh_reparam(np.full(40, MU), np.full(40, LAM))
    F = elements._cols(x) @ np.linalg.inv(elements._cols(X))
    _, _, d2 = elements._snh_density(F, mu_, lam_)
    ev = np.linalg.eigvalsh(d2().reshape(-1, 9, 9))
    _, s, _ = _signed_svd(F)
    I2 = np.sum(s * s, 1)
    J = np.prod(s, 1)
    alpha = 1.0 + mu_ / lam_ - mu_ / (4.0 * lam_)
    p2 = 0.5 * mu_ * (1.0 - 1.0 / (I2 + 1.0))
    p22 = 0.5 * mu_ / (I2 + 1.0) ** 2
    p3 = lam_ * (J - alpha)
    c = np.stack([s[:, 1] * s[:, 2], s[:, 0] * s[:, 2], s[:, 0] * s[:, 1]], 1)
    A = (2 * p2[:, None, None] * np.eye(3) + 4 * p22[:, None, None] * np.einsum("ei,ej->eij", s, s)
         + lam_[:, None, None] * np.einsum("ei,ej->eij", c, c))
    for i, j, k in [(0, 1, 2), (0, 2, 1), (1, 2, 0)]:
        A[:, i, j] += p3 * s[:, k]
        A[:, j, i] += p3 * s[:, k]
    closed = np.concatenate([np.linalg.eigvalsh(A), 2 * p2[:, None] + p3[:, None] * s,
                             2 * p2[:, None] - p3[:, None] * s], 1)
    assert np.allclose(np.sort(closed, 1), ev, rtol=1e-10, atol=1e-10 * np.abs(ev).max())


def test_snh_filtered_hessian_properties():
    """The filtered element Hessian is PSD, exceeds the raw one by a PSD
    matrix (only negative directions are removed from d2psi), keeps the
    gradient, matches the raw Hessian where d2psi is PSD (the rest state),
    and rotates with the positions."""
    x, X = sg.random_tets(60, seed=82, inverted_frac=0.3)
    n = 60
    mu, lam = np.full(n, MU), np.full(n, LAM)
    E, g, H = elements.snh_tet4(x, X, mu, lam)
    Ef, gf, Hf = elements.snh_tet4_filtered(x, X, mu, lam)
    assert np.allclose(Ef, E, rtol=1e-13) and _rel(gf, g) < 1e-13
    Hm, Hfm = H.reshape(n, 12, 12), Hf.reshape(n, 12, 12)
    scale = np.abs(Hm).max()
    assert np.linalg.eigvalsh(Hfm).min() > -1e-10 * scale
    assert np.linalg.eigvalsh(Hfm - Hm).min() > -1e-10 * scale
    assert np.linalg.eigvalsh(Hm).min() < -1e-3 * scale          # the raw one is indefinite
    Xr = _tet_rest()
    _, _, H0 = elements.snh_tet4(Xr, Xr, np.full(8, MU), np.full(8, LAM))
    _, _, H0f = elements.snh_tet4_filtered(Xr, Xr, np.full(8, MU), np.full(8, LAM))
    assert _rel(H0f, H0) < 1e-12
    Q = _rot(83)
    _, _, Hq = elements.snh_tet4_filtered(x @ Q.T, X, mu, lam)
    QQ = np.kron(np.eye(4), Q)
    assert _rel(Hq.reshape(n, 12, 12), QQ @ Hfm @ QQ.T) < 1e-11


# ----------------------------------------------------------------------------
# Quadratic tet (tet10), Eq. 12 with the App. A interpolation
# ----------------------------------------------------------------------------
def _tet10_random(n, seed, curved=0.1):
    """Straight-sided rest tet10s (edge nodes at midpoints), and current
    states: an affine map plus node noise (curved = noise / edge length)."""
    x4, X4 = sg.random_tets(n, seed, inverted_frac=0.0)
    E = [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]
    X = np.concatenate([X4, np.stack([0.5 * (X4[:, i] + X4[:, j]) for i, j in E], 1)], 1)
    x = np.concatenate([x4, np.stack([0.5 * (x4[:, i] + x4[:, j]) for i, j in E], 1)], 1)
    x = x + np.random.default_rng(seed + 1).uniform(-curved, curved, x.shape) * 0.01
    return x, X


def _snh10(x, X, **kw):
    n = x.shape[0]
    return elements.snh_tet10(x, X, np.full(n, MU), np.full(n, LAM), **kw)


def test_tet10_rule_is_degree_two():
    """The 4-point rule integrates every monomial of degree <= 2 over the
    reference tet exactly (int xi^a = a!b!c!/(a+b+c+3)!), and not degree 3."""
    from math import factorial
    rule = elements.TET10_RULE

    def exact(p):
        return factorial(p[0]) * factorial(p[1]) * factorial(p[2]) / factorial(sum(p) + 3)
    for p in itertools.product(range(4), repeat=3):
        q = sum(w * xi[0] ** p[0] * xi[1] ** p[1] * xi[2] ** p[2] for w, xi in rule)
        if sum(p) <= 2:
            assert q == pytest.approx(exact(p), rel=1e-14)
    cubic = sum(w * xi[0] ** 3 for w, xi in rule)
    assert abs(cubic - exact((3, 0, 0))) > 1e-6


def test_tet10_shape_derivatives():
    """dN/dxi matches the complex-step derivative of the App. A interpolation
    written out here, the functions are a partition of unity (derivatives sum
    to zero) and interpolate: N_a(node b) = delta_ab."""
    nodes = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [.5, 0, 0], [.5, .5, 0],
                      [0, .5, 0], [0, 0, .5], [.5, 0, .5], [0, .5, .5]])

    def N(xi):
        L0, L1, L2, L3 = 1 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]
        return np.array([L0 * (2 * L0 - 1), L1 * (2 * L1 - 1), L2 * (2 * L2 - 1), L3 * (2 * L3 - 1),
                         4 * L0 * L1, 4 * L1 * L2, 4 * L2 * L0, 4 * L0 * L3, 4 * L1 * L3,
                         4 * L2 * L3])
    assert np.allclose(np.stack([N(p) for p in nodes]), np.eye(10), atol=1e-15)
    rng = np.random.default_rng(50)
    for _ in range(10):
        xi = rng.dirichlet(np.ones(4))[1:]
        dN = elements.tet10_shape_derivatives(xi)
        cs = np.stack([np.imag(N(xi + 1e-30j * np.eye(3)[k])) / 1e-30 for k in range(3)], 1)
        assert np.allclose(dN, cs, rtol=0, atol=1e-13)
        assert np.allclose(dN.sum(axis=0), 0.0, atol=1e-14)


def test_tet10_affine_patch_equals_tet4():
    """Under an affine map every quadrature point sees the same F, so the
    quadratic element's energy is V psi(F) of its corner tet (the linear
    element, pinned separately), and its gradient sums to zero."""
    _, X = _tet10_random(12, 51)
    A = np.eye(3)[None] + np.random.default_rng(52).uniform(-0.3, 0.3, (12, 3, 3))
    x = np.einsum("eij,eaj->eai", A, X) + 0.3
    E10, g10, _ = _snh10(x, X, want_hess=False)
    E4, _, _ = _snh(x[:, :4], X[:, :4], want_hess=False)
    assert _rel(E10, E4) < 1e-12
    assert np.max(np.abs(g10.sum(axis=1))) < 1e-9 * np.max(np.abs(g10))


def test_tet10_derivatives_complex_step():
    x, X = _tet10_random(6, 53)
    E, g, H = _snh10(x, X)
    gc = _cs_grad(lambda xc: _snh10(xc, X, want_hess=False)[0], x)
    Hc = _cs_jac(lambda xc: _snh10(xc, X, want_hess=False)[1], x)
    assert _rel(g, gc) < 1e-12
    assert _rel(H, Hc) < 1e-11
    Hm = H.reshape(6, 30, 30)
    assert _rel(Hm, np.swapaxes(Hm, 1, 2)) < 1e-13


def test_tet10_invariances():
    """Translation leaves E and g unchanged, rotation rotates g, and relabelling
    the corners (edge nodes following their edges) permutes g: the symmetric
    rule maps onto itself, so E is unchanged."""
    x, X = _tet10_random(10, 54)
    E, g, H = _snh10(x, X)
    E2, g2, _ = _snh10(x + np.array([0.3, -0.2, 0.1]), X, want_hess=False)
    assert np.allclose(E2, E, rtol=1e-12) and _rel(g2, g) < 1e-12
    Q = _rot(55)
    E3, g3, _ = _snh10(x @ Q.T, X, want_hess=False)
    assert np.allclose(E3, E, rtol=1e-12) and _rel(g3, g @ Q.T) < 1e-11
    edges = [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]
    for sigma in itertools.permutations(range(4)):
        perm = list(sigma)
        for i, j in edges:
            a, b = sigma[i], sigma[j]
            perm.append(4 + next(k for k, e in enumerate(edges) if set(e) == {a, b}))
        E4, g4, H4 = _snh10(x[:, perm], X[:, perm])
        assert np.allclose(E4, E, rtol=1e-12)
        assert _rel(g4, g[:, perm]) < 1e-11
        assert _rel(H4, H[:, perm][:, :, :, perm]) < 1e-11


def test_tet10_hrz_masses():
    """HRZ lumping: int N_a^2 over a straight-sided tet by a brute-force
    tensor Gauss rule on the collapsed cube, scaled to rho V, gives rho V/36
    per corner and 4 rho V/27 per edge node."""
    t, w = np.polynomial.legendre.leggauss(8)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    total = np.zeros(10)
    for u, wu in zip(t, w):
        for v, wv in zip(t, w):
            for r, wr in zip(t, w):
                xi = np.array([u, v * (1 - u), r * (1 - u) * (1 - v)])   # Duffy map
                jac = (1 - u) ** 2 * (1 - v)
                L = np.array([1 - xi.sum(), *xi])
                N = [L[c] * (2 * L[c] - 1) for c in range(4)]
                N += [4 * L[i] * L[j] for i, j in [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]]
                total += wu * wv * wr * jac * np.array(N) ** 2
    frac = total / total.sum()
    assert np.allclose(frac[:4], 1 / 36, rtol=1e-12) and np.allclose(frac[4:], 4 / 27, rtol=1e-12)
    s = sg.tet_cube_scene(2, h=0.01, kind=sg.SNH_TET10)
    m = rest.lumped_mass(s)
    assert np.sum(m) == pytest.approx(1000.0 * 0.02 ** 3, rel=1e-12)
    V = 0.01 ** 3 / 6
    e = s.energies[0].conn[0]
    own = np.zeros(s.n_nodes)
    np.add.at(own, e, 1000.0 * V * np.array([1 / 36] * 4 + [4 / 27] * 6))
    assert np.all(m[e] >= own[e] - 1e-18)


# ----------------------------------------------------------------------------
# Cubic tet (tet20)
# ----------------------------------------------------------------------------
_E6 = [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]
_F4 = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]


def _tet20_nodes(P4):
    """Straight-sided cubic node positions from corner positions (E,4,3)."""
    e = []
    for i, j in _E6:
        e += [(2 * P4[:, i] + P4[:, j]) / 3, (P4[:, i] + 2 * P4[:, j]) / 3]
    f = [P4[:, list(fc)].mean(axis=1) for fc in _F4]
    return np.concatenate([P4, np.stack(e, 1), np.stack(f, 1)], 1)


def _tet20_random(n, seed, curved=0.1):
    x4, X4 = sg.random_tets(n, seed, inverted_frac=0.0)
    X, x = _tet20_nodes(X4), _tet20_nodes(x4)
    return x + np.random.default_rng(seed + 1).uniform(-curved, curved, x.shape) * 0.01, X


def _tet20_relabel(sigma):
    """Original node of each position after relabelling the corners by sigma."""
    perm = list(sigma)
    for i, j in _E6:
        a, b = sigma[i], sigma[j]
        m = next(k for k, e in enumerate(_E6) if set(e) == {a, b})
        near_a = 4 + 2 * m if _E6[m][0] == a else 5 + 2 * m
        perm += [near_a, near_a + 1 if near_a == 4 + 2 * m else near_a - 1]
    perm += [16 + sigma[c] for c in range(4)]
    return perm


def _snh20(x, X, **kw):
    n = x.shape[0]
    return elements.snh_tet20(x, X, np.full(n, MU), np.full(n, LAM), **kw)


def test_tet20_rule_is_degree_four_and_symmetric():
    """Every monomial of degree <= 4 integrated exactly (not degree 5), and
    the point set maps onto itself under every vertex permutation (what the
    row-wise relabelling of the elements relies on)."""
    from math import factorial
    rule = elements.TET20_RULE
    for p in itertools.product(range(6), repeat=3):
        q = sum(w * xi[0] ** p[0] * xi[1] ** p[1] * xi[2] ** p[2] for w, xi in rule)
        exact = factorial(p[0]) * factorial(p[1]) * factorial(p[2]) / factorial(sum(p) + 3)
        if sum(p) <= 4:
            assert q == pytest.approx(exact, rel=1e-13)
        if p == (5, 0, 0):
            assert abs(q - exact) > 1e-6 * exact
    bary = [np.concatenate([[1 - xi.sum()], xi]) for _, xi in rule]
    for sigma in itertools.permutations(range(4)):
        for (w, _), L in zip(rule, bary):
            Ls = L[list(sigma)]
            assert any(abs(w - w2) < 1e-15 and np.allclose(Ls, L2, atol=1e-15)
                       for (w2, _), L2 in zip(rule, bary))


def test_tet20_shape_functions():
    """Interpolation at the 20 nodes, partition of unity, and derivatives by
    the complex step of the interpolation written out here."""
    nodes = _tet20_nodes(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]]))[0]

    def N(xi):
        L = [1 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]]
        out = [0.5 * L[c] * (3 * L[c] - 1) * (3 * L[c] - 2) for c in range(4)]
        for i, j in _E6:
            out += [4.5 * L[i] * L[j] * (3 * L[i] - 1), 4.5 * L[i] * L[j] * (3 * L[j] - 1)]
        out += [27 * L[a] * L[b] * L[c] for a, b, c in _F4]
        return np.array(out)
    assert np.allclose(np.stack([N(p) for p in nodes]), np.eye(20), atol=1e-14)
    rng = np.random.default_rng(56)
    for _ in range(10):
        xi = rng.dirichlet(np.ones(4))[1:]
        dN = elements.tet20_shape_derivatives(xi)
        cs = np.stack([np.imag(N(xi + 1e-30j * np.eye(3)[k])) / 1e-30 for k in range(3)], 1)
        assert np.allclose(dN, cs, rtol=0, atol=1e-12)
        assert abs(N(xi).sum() - 1) < 1e-14 and np.allclose(dN.sum(0), 0.0, atol=1e-13)


def test_tet20_affine_patch_and_derivatives():
    _, X = _tet20_random(6, 57)
    A = np.eye(3)[None] + np.random.default_rng(58).uniform(-0.3, 0.3, (6, 3, 3))
    xa = np.einsum("eij,eaj->eai", A, X) - 0.2
    E20, _, _ = _snh20(xa, X, want_hess=False)
    E4, _, _ = _snh(xa[:, :4], X[:, :4], want_hess=False)
    assert _rel(E20, E4) < 1e-12
    x, X = _tet20_random(2, 59)
    E, g, H = _snh20(x, X)
    gc = _cs_grad(lambda xc: _snh20(xc, X, want_hess=False)[0], x)
    Hc = _cs_jac(lambda xc: _snh20(xc, X, want_hess=False)[1], x)
    assert _rel(g, gc) < 1e-12
    assert _rel(H, Hc) < 1e-11


def test_tet20_relabelling_invariance():
    x, X = _tet20_random(4, 60)
    E, g, H = _snh20(x, X)
    for sigma in [(1, 0, 2, 3), (2, 3, 0, 1), (3, 1, 2, 0), (1, 2, 3, 0)]:
        perm = _tet20_relabel(sigma)
        assert sorted(perm) == list(range(20))
        E2, g2, H2 = _snh20(x[:, perm], X[:, perm])
        assert np.allclose(E2, E, rtol=1e-12)
        assert _rel(g2, g[:, perm]) < 1e-11
        assert _rel(H2, H[:, perm][:, :, :, perm]) < 1e-10


def test_tet20_hrz_masses():
    t, w = np.polynomial.legendre.leggauss(8)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    total = np.zeros(20)
    for u, wu in zip(t, w):
        for v, wv in zip(t, w):
            for r, wr in zip(t, w):
                xi = np.array([u, v * (1 - u), r * (1 - u) * (1 - v)])
                jac = (1 - u) ** 2 * (1 - v)
                L = [1 - xi.sum(), *xi]
                N = [0.5 * L[c] * (3 * L[c] - 1) * (3 * L[c] - 2) for c in range(4)]
                for i, j in _E6:
                    N += [4.5 * L[i] * L[j] * (3 * L[i] - 1), 4.5 * L[i] * L[j] * (3 * L[j] - 1)]
                N += [27 * L[a] * L[b] * L[c] for a, b, c in _F4]
                total += wu * wv * wr * jac * np.array(N) ** 2
    frac = total / total.sum()
    assert np.allclose(frac[:4], 1 / 193, rtol=1e-12)
    assert np.allclose(frac[4:16], 27 / 772, rtol=1e-12)
    assert np.allclose(frac[16:], 27 / 193, rtol=1e-12)
    s = sg.tet_cube_scene(2, h=0.01, kind=sg.SNH_TET20)
    assert np.sum(rest.lumped_mass(s)) == pytest.approx(1000.0 * 0.02 ** 3, rel=1e-12)


def _random_tris(n, seed, stretch=0.2):
    rng = np.random.default_rng(seed)
    base = np.array([[0, 0, 0], [1, 0, 0], [0.2, 0.9, 0]], dtype=np.float64) * 0.01
    X = base[None] + rng.uniform(-0.002, 0.002, size=(n, 3, 3))
    X = np.einsum("ij,eaj->eai", _rot(seed), X)
    A = np.eye(3)[None] + rng.uniform(-stretch, stretch, size=(n, 3, 3))
    x = np.einsum("eij,eaj->eai", A, X) + rng.uniform(-1, 1, size=(n, 1, 3))
    return x, X


MU2, LAM2 = rest.lame(1e4, 0.3)


def _stvk(x, X, **kw):
    n = x.shape[0]
    return elements.stvk_tri3(x, X, np.full(n, MU2), np.full(n, LAM2), 1e-3, **kw)


def test_stvk_derivatives_complex_step():
    x, X = _random_tris(30, 21)
    _, g, H = _stvk(x, X)
    gc = _cs_grad(lambda xc: _stvk(xc, X, want_hess=False)[0], x)
    Hc = _cs_jac(lambda xc: _stvk(xc, X, want_hess=False)[1], x)
    assert _rel(g, gc) < 1e-12
    assert _rel(H, Hc) < 1e-12


def test_stvk_uniaxial_stretch_closed_form():
    # stretch s along the first rest edge: psi = (mu + lam/2) ((s^2 - 1)/2)^2
    _, X = _random_tris(6, 22)
    d1 = X[:, 1] - X[:, 0]
    e1 = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    for s in (1.1, 0.8):
        x = X + (s - 1.0) * np.einsum("ea,ei->eai", np.einsum("eai,ei->ea", X - X[:, :1], e1), e1)
        E, _, _ = _stvk(x, X, want_hess=False)
        A = 0.5 * np.linalg.norm(np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), axis=1)
        psi = (MU2 + 0.5 * LAM2) * ((s * s - 1.0) / 2.0) ** 2
        assert np.allclose(E, 1e-3 * A * psi, rtol=1e-12)


def _cst_membrane_stiffness(X, mu, lam, h):
    """Textbook plane CST in the triangle's own 2D frame, rotated to 3D."""
    d1 = X[1] - X[0]
    d2 = X[2] - X[0]
    n = np.cross(d1, d2); n /= np.linalg.norm(n)
    t1 = d1 / np.linalg.norm(d1)
    t2 = np.cross(n, t1)
    P = np.stack([t1, t2])                     # (2,3) projection to the plane
    p = (X - X[0]) @ P.T                       # (3,2) local coordinates
    A = 0.5 * abs(np.linalg.det(np.stack([p[1], p[2]], 1)))
    M = np.hstack([np.ones((3, 1)), p])
    grads = np.linalg.inv(M)[1:, :].T          # (3,2)
    B = np.zeros((3, 6))
    for a in range(3):
        dx, dy = grads[a]
        B[0, 2 * a] = dx
        B[1, 2 * a + 1] = dy
        B[2, 2 * a] = dy; B[2, 2 * a + 1] = dx
    C = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
    K2 = h * A * B.T @ C @ B
    T = np.kron(np.eye(3), P)                  # (6,9) 3D -> local displacements
    return T.T @ K2 @ T


def test_stvk_rest_is_plane_cst():
    _, X = _random_tris(6, 23)
    E, g, H = _stvk(X, X)
    assert np.max(np.abs(E)) < 1e-20
    assert np.max(np.abs(g)) < 1e-14
    for e in range(X.shape[0]):
        K = _cst_membrane_stiffness(X[e], MU2, LAM2, 1e-3)
        assert _rel(H[e].reshape(9, 9), K) < 1e-12
        ev = np.linalg.eigvalsh(K)
        assert np.sum(ev > 1e-9 * ev.max()) == 3


def test_stvk_invariances():
    x, X = _random_tris(10, 24)
    E, g, H = _stvk(x, X)
    R = _rot(5)
    E2, g2, _ = _stvk(x @ R.T, X)
    assert np.allclose(E2, E, rtol=1e-12)
    assert _rel(g2, g @ R.T) < 1e-11
    # rotating the rest triangle does not change anything (frame choice)
    E3, g3, H3 = _stvk(x, X @ _rot(6).T)
    assert np.allclose(E3, E, rtol=1e-11)
    assert _rel(H3, H) < 1e-10
    E4, g4, _ = _stvk(x[:, [1, 2, 0]], X[:, [1, 2, 0]], want_hess=False)
    assert np.allclose(E4, E, rtol=1e-12)
    assert _rel(g4, g[:, [1, 2, 0]]) < 1e-11


# ----------------------------------------------------------------------------
# Bending hinge
# ----------------------------------------------------------------------------
def _flat_hinges(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 4, 3))
    X[:, 1, 0] = rng.uniform(0.5, 1.5, n)
    X[:, 2, :2] = np.stack([rng.uniform(0.1, 0.9, n), rng.uniform(0.3, 1.0, n)], 1)
    X[:, 3, :2] = np.stack([rng.uniform(0.1, 0.9, n), -rng.uniform(0.3, 1.0, n)], 1)
    X = np.einsum("ij,eaj->eai", _rot(seed), X) + rng.normal(size=(n, 1, 3))
    return X * 0.01


def test_hinge_flat_rest_and_translation():
    X = _flat_hinges(20, 31)
    K, c = elements.hinge_rest(X)
    assert np.max(np.abs(K.sum(1))) < 1e-12 * np.abs(K).max()
    E, g, H = elements.hinge4(X, X, 1e-3)
    assert np.max(np.abs(E)) < 1e-30 + 1e-24
    assert np.max(np.abs(g)) < 1e-14


def test_hinge_wing_rotation_closed_form():
    # rotating one wing by theta about the edge: E = k_b/2 * 3|e|^2/(A0+A1) * (2 sin(theta/2))^2
    X = _flat_hinges(10, 32)
    kb = 2e-3
    e = X[:, 1] - X[:, 0]
    eh = e / np.linalg.norm(e, axis=1, keepdims=True)
    A0 = 0.5 * np.linalg.norm(np.cross(e, X[:, 2] - X[:, 0]), axis=1)
    A1 = 0.5 * np.linalg.norm(np.cross(e, X[:, 3] - X[:, 0]), axis=1)
    for wing in (2, 3):
        for theta in (0.3, -1.1):
            x = X.copy()
            r = X[:, wing] - X[:, 0]
            par = np.einsum("ei,ei->e", r, eh)[:, None] * eh
            perp = r - par
            x[:, wing] = X[:, 0] + par + np.cos(theta) * perp + np.sin(theta) * np.cross(eh, perp)
            E, _, _ = elements.hinge4(x, X, kb, want_hess=False)
            ref = 0.5 * kb * 3 * np.sum(e * e, 1) / (A0 + A1) * (2 * np.sin(theta / 2)) ** 2
            assert np.allclose(E, ref, rtol=1e-11)


def test_hinge_derivatives():
    X = _flat_hinges(10, 33)
    x = X + np.random.default_rng(1).normal(scale=1e-3, size=X.shape)
    _, g, H = elements.hinge4(x, X, 1e-3)
    assert _rel(g, _cs_grad(lambda xc: elements.hinge4(xc, X, 1e-3, want_hess=False)[0], x)) < 1e-12
    assert _rel(H, _cs_jac(lambda xc: elements.hinge4(xc, X, 1e-3, want_hess=False)[1], x)) < 1e-12
    _, _, H2 = elements.hinge4(x * 1.7 + 0.2, X, 1e-3)
    assert _rel(H2, H) < 1e-15                        # constant quadratic form
    ev = np.linalg.eigvalsh(H.reshape(-1, 12, 12))
    assert np.all(ev > -1e-12 * ev.max())
    assert np.all(np.sum(ev > 1e-9 * ev.max(axis=1, keepdims=True), axis=1) == 3)


# ----------------------------------------------------------------------------
# inertia, masses
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [sg.SNH_TET4, sg.NH_TET4, sg.STVK_TET4, sg.FCR_TET4,
                                  sg.ARAP_TET4])
def test_tet_masses_every_material(kind):
    """Mass does not depend on the material: every tet kind lumps rho V / 4,
    so a box of side L carries rho L^3, split equally among a tet's nodes."""
    s = sg.tet_cube_scene(3, h=0.01, seed=1, kind=kind)
    m = rest.lumped_mass(s)
    assert np.sum(m) == pytest.approx(1000.0 * (0.03) ** 3, rel=1e-12)
    assert np.all(m > 0)
    # and node by node the same as the Stable Neo-Hookean box
    ref = rest.lumped_mass(sg.tet_cube_scene(3, h=0.01, seed=1))
    assert np.array_equal(m, ref)


def test_inertia_and_masses():
    s = sg.tet_cube_scene(3, h=0.01, seed=1)
    m = rest.lumped_mass(s)
    assert np.sum(m) == pytest.approx(1000.0 * (0.03) ** 3, rel=1e-12)
    assert np.all(m > 0)
    cs = sg.cloth_scene(4)
    mc = rest.lumped_mass(cs)
    assert np.sum(mc) == pytest.approx(1000.0 * 1e-3 * 1.0, rel=1e-12)
    xt = s.x0 + 0.001
    E, g, w = elements.inertia(s.x0, xt, m, 0.01)
    assert np.allclose(E, 0.5 * m / 1e-4 * 3e-6, rtol=1e-12)
    assert np.allclose(g, -m[:, None] / 1e-4 * 1e-3, rtol=1e-12)


# ----------------------------------------------------------------------------
# projection
# ----------------------------------------------------------------------------
def test_projection_known_spectrum():
    rng = np.random.default_rng(41)
    for n in (9, 12):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        d = rng.normal(size=n)
        d[:3] = [-2.0, -1e-3, 0.0]
        H = (Q * d) @ Q.T
        ref = (Q * np.maximum(d, 0)) @ Q.T
        P = projection.project_psd(H[None])[0]
        assert _rel(P, ref) < 1e-13
        assert _rel(projection.project_psd(P[None])[0], P) < 1e-13        # idempotent
        S = (Q * np.abs(d)) @ Q.T                                          # PSD input
        assert _rel(projection.project_psd(S[None])[0], S) < 1e-13
        # nearest: no random PSD matrix is closer
        for _ in range(20):
            B = rng.normal(size=(n, n))
            T = P + 0.1 * B @ B.T
            assert np.linalg.norm(H - P) <= np.linalg.norm(H - T) + 1e-14


# ----------------------------------------------------------------------------
# pattern, scatter map, assembly
# ----------------------------------------------------------------------------
def _tet_nnzb(n):
    return (n + 1) ** 3 + 2 * (3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tet_pattern_closed_form(n):
    s = sg.tet_cube_scene(n, seed=1)
    rp, ci = assembly.pattern(s)
    assert ci.size == _tet_nnzb(n)
    upper = np.sum(ci >= np.repeat(np.arange(s.n_nodes), np.diff(rp)))
    assert upper == (2 * n + 1) ** 3
    rp2, ci2 = assembly.pattern_fast(s)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)


@pytest.mark.parametrize("m", [2, 4])
def test_cloth_pattern_closed_form(m):
    s = sg.cloth_scene(m)
    assert s.energies[1].conn.shape[0] == 3 * m * m - 2 * m
    rp, ci = assembly.pattern(s)
    assert ci.size == (m + 1) ** 2 + 12 * m * m
    rp2, ci2 = assembly.pattern_fast(s)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)


def test_c1_block_count():
    s = sg.config_c1()
    rp, ci = assembly.pattern_fast(s)
    assert ci.size == 17191 == _tet_nnzb(10)
    assert np.all(np.diff(rp) <= 15)


def test_scatter_map_brute_force():
    s = sg.tet_cube_scene(2, seed=1)
    rp, ci = assembly.pattern(s)
    sm = assembly.scatter_map(s, rp, ci)[0]
    fast = assembly._block_index(s.energies[0].conn, rp, ci)
    assert np.array_equal(sm, fast)
    rows = np.repeat(np.arange(s.n_nodes), np.diff(rp))
    c = s.energies[0].conn
    for a in range(4):
        for b in range(4):
            assert np.array_equal(rows[sm[:, a, b]], c[:, a])
            assert np.array_equal(ci[sm[:, a, b]], c[:, b])


def _small_mixed_scene():
    s = sg.tet_cube_scene(2, seed=7, perturb=0.05)
    c = sg.cloth_scene(2, perturb=0.1)
    # merge: tets first, cloth nodes after
    N = s.n_nodes
    es = [s.energies[0]] + [sg.EnergySet(e.kind, e.conn + N, young=e.young, poisson=e.poisson,
                                         thickness=e.thickness, bend_kb=e.bend_kb,
                                         density=e.density) for e in c.energies]
    X = np.concatenate([s.X, c.X])
    x0 = np.concatenate([s.x0, c.x0])
    fixed = np.concatenate([s.fixed, c.fixed])
    return sg.Scene("mixed", X, es, fixed, x0, np.zeros_like(X))


def test_assembly_matches_complex_step_of_total_energy():
    s = _small_mixed_scene()
    rng = np.random.default_rng(3)
    x = s.x0 + rng.uniform(-1e-3, 1e-3, size=s.x0.shape)
    xt = x + rng.normal(scale=1e-3, size=x.shape)
    dt = 0.01
    a = assembly.assemble(s, x, xt, dt, dirichlet=False)
    N = s.n_nodes
    A = assembly.to_scipy(a["row_ptr"], a["col_idx"], a["vals"]).toarray()
    h = 1e-30
    for k in rng.choice(3 * N, size=12, replace=False):
        xc = x.astype(complex)
        xc.reshape(-1)[k] += 1j * h
        Ec = assembly.energy(s, xc, xt, dt) if False else _energy_complex(s, xc, xt, dt)
        assert np.imag(Ec) / h == pytest.approx(a["g"].reshape(-1)[k], rel=1e-10,
                                                abs=1e-12 * np.abs(a["g"]).max())
        col = _grad_complex(s, xc, xt, dt).reshape(-1)
        assert np.allclose(np.imag(col) / h, A[:, k], rtol=1e-10, atol=1e-10 * np.abs(A).max())
    # block symmetry
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())


def _energy_complex(s, x, xt, dt):
    E = 0.0
    for es in s.energies:
        E = E + np.sum(elements.element_eval(es, x, s.X, want_hess=False)[0])
    m = rest.lumped_mass(s)
    return E + np.sum(elements.inertia(x, xt, m, dt)[0])


def _grad_complex(s, x, xt, dt):
    g = np.zeros(x.shape, dtype=complex)
    for es in s.energies:
        _, ge, _ = elements.element_eval(es, x, s.X, want_hess=False)
        np.add.at(g, es.conn.ravel(), ge.reshape(-1, 3))
    m = rest.lumped_mass(s)
    return g + elements.inertia(x, xt, m, dt)[1]


def test_dirichlet_and_matrix_free_product():
    s = _small_mixed_scene()
    x = s.x0
    a = assembly.assemble(s, x, s.x0, 0.01, dirichlet=True)
    rp, ci, vals = a["row_ptr"], a["col_idx"], a["vals"]
    fixed = s.fixed.astype(bool)
    assert np.all(a["g"][fixed] == 0)
    rows = np.repeat(np.arange(s.n_nodes), np.diff(rp))
    for b in range(ci.size):
        if fixed[rows[b]] or fixed[ci[b]]:
            ref = np.eye(3) if rows[b] == ci[b] else np.zeros((3, 3))
            assert np.array_equal(vals[b], ref)
    # without Dirichlet: BSR p == sum_e R_e^T H_e R_e p + M/dt^2 p
    a2 = assembly.assemble(s, x, s.x0, 0.01, dirichlet=False)
    p = np.random.default_rng(5).normal(size=x.shape)
    y = (assembly.to_scipy(rp, ci, a2["vals"]) @ p.ravel()).reshape(-1, 3)
    ref = rest.lumped_mass(s)[:, None] / 1e-4 * p
    for es in s.energies:
        _, _, He = elements.element_eval(es, x, s.X)
        k = es.conn.shape[1]
        ye = np.einsum("emn,en->em", He.reshape(-1, 3 * k, 3 * k), p[es.conn].reshape(-1, 3 * k))
        np.add.at(ref, es.conn.ravel(), ye.reshape(-1, 3))
    assert _rel(y, ref) < 1e-12


# ----------------------------------------------------------------------------
# solver
# ----------------------------------------------------------------------------
def test_pcg_matches_direct_solve():
    s = sg.config_c1()
    xt = elements.x_tilde(s.x0, s.v0, 0.01, (0, 0, -9.81))
    a = assembly.assemble(s, s.x0, xt, 0.01)
    A = assembly.to_scipy(a["row_ptr"], a["col_idx"], a["vals"])
    b = -a["g"].ravel()
    import scipy.sparse.linalg as spla
    ref = spla.spsolve(A.tocsc(), b)
    D = newton.diag_inverse(a["row_ptr"], a["col_idx"], a["vals"])
    x, it, ok = newton.pcg(A, D, b, 1e-13, 2000)
    assert ok and it > 1
    assert _rel(x, ref) < 1e-10


def test_newton_rigid_translation_is_exact():
    # no gravity, no fixed nodes, uniform velocity: E_elastic is translation
    # invariant, so x(t+dt) = x(t) + dt v exactly
    s = sg.tet_cube_scene(2, seed=2, perturb=0.0)
    s.fixed[:] = 0
    v = np.tile(np.array([[0.3, -0.1, 0.2]]), (s.n_nodes, 1))
    prm = newton.StepParams(dt=0.01, gravity=(0, 0, 0))
    st = newton.Stepper(s, prm, solver="direct")
    x1, v1, rep = st.step(s.X.copy(), v)
    assert rep["status"] == "ok"
    assert np.allclose(x1, s.X + 0.01 * v, rtol=0, atol=1e-12)
    assert np.allclose(v1, v, atol=1e-9)


def test_x_tilde_free_fall_closed_form():
    # Eq. 2-3 for a body in free fall: a uniform translation leaves every
    # elastic energy at its rest value, so each implicit-Euler step moves all
    # nodes as one particle, v_{k+1} = v_k + dt g and x_{k+1} = x_k + dt v_{k+1}.
    # Summed over K steps: v_K = v_0 + K dt g, x_K = x_0 + K dt v_0 +
    # dt^2 g K (K + 1) / 2 (explicit Euler would give K (K - 1) / 2, the exact
    # flow K^2 / 2).  A slip in the prediction x_tilde (dt g for dt^2 g, a
    # half, a sign, a component) moves x_K off this closed form.
    s = sg.tet_cube_scene(2, seed=3, perturb=0.0)
    s.fixed[:] = 0
    grav = np.array([0.7, -0.4, -9.81])
    v0 = np.array([0.05, 0.02, -0.1])
    dt, K = 0.01, 5
    prm = newton.StepParams(dt=dt, gravity=tuple(grav))
    st = newton.Stepper(s, prm, solver="direct")
    x, v = s.X.copy(), np.tile(v0, (s.n_nodes, 1))
    for _ in range(K):
        x, v, rep = st.step(x, v)
        assert rep["status"] == "ok" and rep["dt_halvings"] == 0
    x_ref = s.X + K * dt * v0 + dt * dt * grav * K * (K + 1) / 2
    v_ref = v0 + K * dt * grav
    assert np.max(np.abs(x - x_ref)) <= 1e-12
    assert np.max(np.abs(v - v_ref[None, :])) <= 1e-9


def test_block_jacobi_is_exact_on_block_diagonal_systems():
    # With every off-diagonal block removed the matrix is its own block-Jacobi
    # preconditioner, so preconditioned CG reaches the exact solution in one
    # iteration.  The diagonal blocks (inertia + elastic, fully populated 3x3)
    # are split between the mesh matrix and the contact blocks, whose diagonal
    # blocks the preconditioner must add in; a wrong block, a missing contact
    # part or a wrong inverse needs more iterations.
    s = sg.config_c1()
    xt = elements.x_tilde(s.x0, s.v0, 0.01, s.gravity)
    a = assembly.assemble(s, s.x0, xt, 0.01)
    rp, ci = a["row_ptr"], a["col_idx"]
    N = rp.size - 1
    rows = np.repeat(np.arange(N), np.diff(rp))
    diag = rows == ci
    # free nodes' diagonal blocks couple their components (fixed ones are I)
    assert np.mean(np.abs(a["vals"][diag][:, 0, 1]) > 0) > 0.8
    vals = np.where(diag[:, None, None], a["vals"], 0.0)
    # contact part: a random symmetric matrix per node (not a multiple of the
    # block, since CG does not see a uniform scaling of the preconditioner)
    R = np.random.default_rng(4).normal(size=(N, 3, 3))
    R = 0.3 * (R + np.transpose(R, (0, 2, 1))) * np.abs(vals[diag]).max(axis=(1, 2))[:, None, None]
    cb = {(i, i): R[i] for i in range(N)}
    part = vals.copy()
    part[diag] -= R
    A = assembly.to_scipy(rp, ci, part, cb)
    D = newton.diag_inverse(rp, ci, part, cb)
    b = np.random.default_rng(5).normal(size=3 * N)
    x, it, ok = newton.pcg(A, D, b, 1e-13, 50)
    assert ok and it == 1
    ref = np.concatenate([np.linalg.solve(vals[d], b[3 * i:3 * i + 3])
                          for i, d in zip(rows[diag], np.nonzero(diag)[0])])
    assert _rel(x, ref) < 1e-12
    # and the full matrix needs many iterations with the same preconditioner
    Af = assembly.to_scipy(rp, ci, a["vals"])
    _, it_full, _ = newton.pcg(Af, newton.diag_inverse(rp, ci, a["vals"]), b, 1e-13, 2000)
    assert it_full > 10


def test_newton_quadratic_energy_one_iteration():
    # inertia + bending only: E_BE is quadratic, so one exact Newton step solves it
    c = sg.cloth_scene(3, perturb=0.2)
    c.energies = [c.energies[1]]
    prm = newton.StepParams(dt=1 / 60)
    rec = []
    ok, x, rep = newton.newton_solve(c, c.x0, c.v0, prm.dt, prm, solver="direct", record=rec)
    assert ok and rep["newton_iters"] == 1
    assert rep["residual"] <= 1e-9 * rep["residual0"]


def test_newton_c1_converges_and_descends():
    s = sg.config_c1()
    prm = newton.StepParams(dt=0.01)
    rec = []
    ok, x, rep = newton.newton_solve(s, s.x0, s.v0, 0.01, prm, solver="pcg", record=rec)
    assert ok
    assert rep["residual"] <= 1e-6 * rep["residual0"]
    Es = [r["E"] for r in rec] + [rep["energy"]]
    assert all(b <= a for a, b in zip(Es, Es[1:]))


def test_dt_halving_control():
    s = sg.tet_cube_scene(2, seed=1)
    prm = newton.StepParams(dt=0.01, max_newton=0, max_halvings=3)
    st = newton.Stepper(s, prm)
    x, v, rep = st.step(s.x0, s.v0)
    assert rep["dt_halvings"] == 3 and rep["status"] == "not_converged"
    prm2 = newton.StepParams(dt=0.01)
    st2 = newton.Stepper(s, prm2)
    st2.dt_cur = 0.0025
    for k in range(3):
        st2.step(s.x0, s.v0)
    assert st2.dt_cur == 0.005
    # no step control (max_halvings 0): exactly prm.dt, state untouched
    st3 = newton.Stepper(s, newton.StepParams(dt=0.01, max_halvings=0))
    st3.dt_cur = 0.0025
    _, _, rep = st3.step(s.x0, s.v0)
    assert rep["dt_used"] == 0.01 and st3.dt_cur == 0.0025 and st3.successes == 0


def test_line_search_takes_full_steps_within_energy_rounding(monkeypatch):
    # Newton's line search compares float64 energy sums, whose rounding grows
    # with the number of elements (1e-14 relative and more); close to the
    # minimiser the decrease of a full Newton step falls below it.  Planted
    # here: every trial energy comes back 1e-13 relative too high, and the
    # step is solved to 1e-8.  With the rounding allowance of the Armijo test
    # it converges on full Newton steps to the same point as without the
    # noise; with no allowance the line search fails on the same noise.
    s = sg.tet_cube_scene(3, seed=4, perturb=0.05)
    dt = s.dt
    base = newton.StepParams(dt=dt, newton_rtol=1e-8)
    ok0, x0, rep0 = newton.newton_solve(s, s.x0, s.v0, dt, base, solver="direct")
    assert ok0 and rep0["ls_backtracks"] == 0
    true_energy = newton.assembly.energy

    def noisy(*a, **k):
        e = true_energy(*a, **k)
        return e + 1e-13 * abs(e)

    monkeypatch.setattr(newton.assembly, "energy", noisy)
    ok1, x1, rep1 = newton.newton_solve(s, s.x0, s.v0, dt, base, solver="direct")
    assert ok1 and rep1["ls_backtracks"] == 0
    assert rep1["newton_iters"] == rep0["newton_iters"]
    assert np.max(np.abs(x1 - x0)) == 0.0
    strict = newton.StepParams(dt=dt, newton_rtol=1e-8, energy_round=0.0)
    ok2, _, rep2 = newton.newton_solve(s, s.x0, s.v0, dt, strict, solver="direct")
    assert not ok2 and rep2["status"] == "line_search"
