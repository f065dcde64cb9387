"""Per-element energies with hand-derived gradients and Hessians (oracle).

TEST INFRASTRUCTURE ONLY.  Arrays are batched over elements: positions x and X
have shape (E, k, 3); gradients (E, k, 3); Hessians (E, k, 3, k, 3) with index
order (node a, coord i, node b, coord k).  All functions accept complex x so
that tests can differentiate them with the complex step; rest data are real.

Energies:
* Stable Neo-Hookean tet4 -- App. B (Stable Neo-Hookean branch, after Smith et
  al. 2018 Eq. 14), integrated over a linear tet as E_e = V_e psi(F_e)
  (Sec. 3.1, element energy by volume integration).  F = Ds Dm^-1.
* StVK triangle membrane -- App. B (Saint Venant-Kirchhoff branch) applied to
  the 3x2 deformation gradient of a triangle in its rest frame, times rest area
  and thickness (Sec. 6.3 uses a 2D FEM integrator for cloth).
* Quadratic bending hinge -- Eq. 13 (Bergou et al. 2006): E = k_b/2 x^T Q x with
  the constant Q = 3/(A0+A1) (K K^T) (x) I3 built from the rest cotangents.
* Inertia -- Eq. 2: m/(2 dt^2) |x - x_tilde|^2 per node.
* The other App. B constitutive models on linear tets, E_e = V_e psi(F_e):
  classic Neo-Hookean (Eq. 6 with the rest-stable sign of the log term),
  Saint Venant-Kirchhoff, fixed co-rotational and as-rigid-as-possible with a
  volume term, the last two with the rotation R held constant over a time step
  (lagged, Sec. 6.1); R is the rotation closest to F at the lag positions.
* Stable Neo-Hookean tet4 with the density Hessian filtered to PSD: the
  element Hessian V B^T d2psi B is rebuilt from the 9x9 density Hessian
  d2psi/dF2 with its negative eigenvalues set to zero (the eigensystem
  approach of Smith et al. 2019, an alternative to projecting the 12x12
  element Hessian; it differs from the nearest-PSD element Hessian unless B
  is orthogonal up to scale).
* Stable Neo-Hookean cubic tet (tet20) -- Eq. 12 with the cubic Lagrange
  interpolation (corners L(3L-1)(3L-2)/2, edge nodes 9/2 L_i L_j (3L_i - 1),
  face nodes 27 L_i L_j L_k) and Keast's symmetric 11-point rule of degree 4
  (centroid weight -74/5625; points (11/14, 1/14, 1/14, 1/14) with 343/45000;
  points (c, c, d, d), c, d = (1 +- sqrt(5/14))/4, with 56/2250).
* Stable Neo-Hookean quadratic tet (tet10) -- Eq. 12: E_e = sum over the
  quadrature points xi_q of w_q |det J_X(xi_q)| psi(F(xi_q)), F = J_x J_X^-1,
  with the tet10 interpolation of App. A and a symmetric 4-point rule of
  degree 2 (Sec. 5.2 fixed value summation: the same density at each point).
"""
from __future__ import annotations

import numpy as np

from .rest import snh_reparam

# Levi-Civita symbol eps[i,j,k]
_EPS = np.zeros((3, 3, 3))
_EPS[0, 1, 2] = _EPS[1, 2, 0] = _EPS[2, 0, 1] = 1.0
_EPS[0, 2, 1] = _EPS[2, 1, 0] = _EPS[1, 0, 2] = -1.0


def _cols(P):
    """Stack edge vectors of nodes 1.. relative to node 0 as matrix columns."""
    return np.stack([P[:, a] - P[:, 0] for a in range(1, P.shape[1])], axis=2)


def _shape_gradients(Dinv):
    """b_a = d F / d x_a contraction vectors: rows of Dm^-1, b_0 = -sum of rows.

    With F = Ds Dm^-1 and Ds columns x_a - x_0, dF_ij/dx_{a,m} = delta_im b_a[j].
    Returns (E, k, d) for Dinv of shape (E, d, d) with k = d + 1 nodes.
    """
    rows = [Dinv[:, r, :] for r in range(Dinv.shape[1])]
    return np.stack([-sum(rows)] + rows, axis=1)


# ----------------------------------------------------------------------------
# Stable Neo-Hookean tet4
# ----------------------------------------------------------------------------
def snh_tet4(x, X, mu, lam, want_hess=True):
    """Energy, gradient and Hessian of V psi_SNH(F) for linear tets.

    mu, lam are the linear-elasticity Lame parameters per element (E,); the
    energy applies the Stable Neo-Hookean re-parametrisation itself.
    psi = mu'/2 (Ic - 3) + lam'/2 (J - alpha)^2 - mu'/2 log(Ic + 1),
    alpha = 1 + mu'/lam' - mu'/(4 lam').
    """
    mu_, lam_ = snh_reparam(np.asarray(mu, dtype=np.float64), np.asarray(lam, dtype=np.float64))
    Dm = _cols(X)
    Dinv = np.linalg.inv(Dm)
    V = np.abs(np.linalg.det(Dm)) / 6.0
    F = _cols(x) @ Dinv
    Ic = np.einsum("eij,eij->e", F, F)
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    J = np.einsum("ei,ei->e", f0, np.cross(f1, f2))
    cof = np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=2)
    alpha = 1.0 + mu_ / lam_ - mu_ / (4.0 * lam_)
    psi = 0.5 * mu_ * (Ic - 3.0) + 0.5 * lam_ * (J - alpha) ** 2 - 0.5 * mu_ * np.log(Ic + 1.0)
    E = V * psi
    s1 = mu_ * (1.0 - 1.0 / (Ic + 1.0))                 # coefficient of F in dpsi/dF
    s2 = lam_ * (J - alpha)                             # coefficient of cof F
    P = s1[:, None, None] * F + s2[:, None, None] * cof
    b = _shape_gradients(Dinv)                          # (E,4,3)
    g = V[:, None, None] * np.einsum("eij,eaj->eai", P, b)
    if not want_hess:
        return E, g, None
    # d2psi/dF_ij dF_kl
    I3 = np.eye(3)
    d2 = (s1[:, None, None, None, None] * np.einsum("ik,jl->ijkl", I3, I3)[None]
          + (2.0 * mu_ / (Ic + 1.0) ** 2)[:, None, None, None, None]
          * np.einsum("eij,ekl->eijkl", F, F)
          + lam_[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", cof, cof)
          + s2[:, None, None, None, None] * np.einsum("ikm,jln,emn->eijkl", _EPS, _EPS, F))
    H = V[:, None, None, None, None] * np.einsum("eaj,ebl,eijkl->eaibk", b, b, d2)
    return E, g, H


# ----------------------------------------------------------------------------
# Other App. B materials on linear tets
# ----------------------------------------------------------------------------
def _tet_kinematics(x, X):
    Dm = _cols(X)
    Dinv = np.linalg.inv(Dm)
    V = np.abs(np.linalg.det(Dm)) / 6.0
    F = _cols(x) @ Dinv
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    J = np.einsum("ei,ei->e", f0, np.cross(f1, f2))
    cof = np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=2)
    return V, F, J, cof, _shape_gradients(Dinv)


def _tet_element(V, psi, P, d2, b, want_hess):
    """E = V psi, g_a = V P b_a, H_ab = V sum b_aj b_bl d2_ijkl."""
    E = V * psi
    g = V[:, None, None] * np.einsum("eij,eaj->eai", P, b)
    if not want_hess:
        return E, g, None
    return E, g, V[:, None, None, None, None] * np.einsum("eaj,ebl,eijkl->eaibk", b, b, d2())


def _hess_J(F):
    """d2 J / dF_ij dF_kl = eps_ikm eps_jln F_mn."""
    return np.einsum("ikm,jln,emn->eijkl", _EPS, _EPS, F)


def _I4(n):
    I3 = np.eye(3)
    return np.broadcast_to(np.einsum("ik,jl->ijkl", I3, I3)[None], (n, 3, 3, 3, 3))


def nh_tet4(x, X, mu, lam, want_hess=True):
    """Classic Neo-Hookean: psi = mu/2 (Ic - 3) - mu log J + lam/2 log^2 J.
    P = mu F + (lam log J - mu) F^-T; with Fi = F^-T,
    d2psi_ijkl = mu d_ik d_jl + lam Fi_ij Fi_kl - (lam log J - mu) Fi_il Fi_kj."""
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    V, F, J, cof, b = _tet_kinematics(x, X)
    Ic = np.einsum("eij,eij->e", F, F)
    logJ = np.log(J)
    psi = 0.5 * mu * (Ic - 3.0) - mu * logJ + 0.5 * lam * logJ ** 2
    Fi = cof / J[:, None, None]
    c = lam * logJ - mu
    P = mu[:, None, None] * F + c[:, None, None] * Fi
    return _tet_element(V, psi, P, lambda: (
        mu[:, None, None, None, None] * _I4(len(V))
        + lam[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", Fi, Fi)
        - c[:, None, None, None, None] * np.einsum("eil,ekj->eijkl", Fi, Fi)), b, want_hess)


def stvk_tet4(x, X, mu, lam, want_hess=True):
    """Saint Venant-Kirchhoff: psi = mu |E|^2 + lam/2 tr(E)^2, E = (F^T F - I)/2.
    P = F S, S = 2 mu E + lam tr(E) I;
    d2psi_ijkl = d_ik S_lj + mu (F_il F_kj + (F F^T)_ik d_jl) + lam F_ij F_kl."""
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    V, F, J, cof, b = _tet_kinematics(x, X)
    Eg = 0.5 * (np.einsum("eki,ekj->eij", F, F) - np.eye(3)[None])
    trE = np.einsum("eii->e", Eg)
    psi = mu * np.einsum("eij,eij->e", Eg, Eg) + 0.5 * lam * trE ** 2
    S = 2.0 * mu[:, None, None] * Eg + (lam * trE)[:, None, None] * np.eye(3)[None]
    P = F @ S
    I3 = np.eye(3)

    def d2():
        FFt = np.einsum("eim,ekm->eik", F, F)
        return (np.einsum("ik,elj->eijkl", I3, S)
                + mu[:, None, None, None, None] * (np.einsum("eil,ekj->eijkl", F, F)
                                                   + np.einsum("eik,jl->eijkl", FFt, I3))
                + lam[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", F, F))
    return _tet_element(V, psi, P, d2, b, want_hess)


def fcr_tet4(x, X, mu, lam, R, want_hess=True):
    """Fixed co-rotational with lagged R: psi = mu |F - R|^2 + lam/2 (J - 1)^2.
    P = 2 mu (F - R) + lam (J - 1) cof F;
    d2psi = 2 mu d_ik d_jl + lam cof_ij cof_kl + lam (J - 1) d2J."""
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    V, F, J, cof, b = _tet_kinematics(x, X)
    D = F - R
    psi = mu * np.einsum("eij,eij->e", D, D) + 0.5 * lam * (J - 1.0) ** 2
    P = 2.0 * mu[:, None, None] * D + (lam * (J - 1.0))[:, None, None] * cof
    return _tet_element(V, psi, P, lambda: (
        2.0 * mu[:, None, None, None, None] * _I4(len(V))
        + lam[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", cof, cof)
        + (lam * (J - 1.0))[:, None, None, None, None] * _hess_J(F)), b, want_hess)


def arap_tet4(x, X, mu, lam, R, want_hess=True):
    """As-rigid-as-possible with a volume term, lagged R:
    psi = mu/2 (Ic - 2 tr(F^T R) + 3) + lam/2 (J - 1)^2 = mu/2 |F - R|^2 + ...
    P = mu (F - R) + lam (J - 1) cof F;
    d2psi = mu d_ik d_jl + lam cof_ij cof_kl + lam (J - 1) d2J."""
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    V, F, J, cof, b = _tet_kinematics(x, X)
    Ic = np.einsum("eij,eij->e", F, F)
    trFR = np.einsum("eij,eij->e", F, R)
    psi = 0.5 * mu * (Ic - 2.0 * trFR + 3.0) + 0.5 * lam * (J - 1.0) ** 2
    P = mu[:, None, None] * (F - R) + (lam * (J - 1.0))[:, None, None] * cof
    return _tet_element(V, psi, P, lambda: (
        mu[:, None, None, None, None] * _I4(len(V))
        + lam[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", cof, cof)
        + (lam * (J - 1.0))[:, None, None, None, None] * _hess_J(F)), b, want_hess)


def closest_rotation(F):
    """The rotation R maximising tr(R^T F) (orthogonal Procrustes on SO(3)):
    with F = U S V^T, R = U diag(1, 1, det(U V^T)) V^T."""
    U, _, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U @ Vt))
    D = np.ones((F.shape[0], 3))
    D[:, 2] = d
    return np.einsum("eij,ej,ejk->eik", U, D, Vt)


def lagged_rotations(x_lag, X):
    """Rotations of the deformation gradients at the lag positions (E,k,3)."""
    return closest_rotation(_cols(x_lag) @ np.linalg.inv(_cols(X)))


# ----------------------------------------------------------------------------
# Stable Neo-Hookean quadratic tet (tet10)
# ----------------------------------------------------------------------------
# Symmetric 4-point rule of degree 2 on the reference tet {xi >= 0, sum <= 1}
# (Hammer, Marlowe and Stroud 1956): barycentric points (a, b, b, b) and their
# permutations, a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20, weights 1/24 (the
# reference volume 1/6 split evenly).  xi = (L1, L2, L3).
_Q4_A = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_Q4_B = (5.0 - np.sqrt(5.0)) / 20.0
TET10_RULE = [(1.0 / 24.0, np.array([_Q4_B if j != i else _Q4_A for j in range(4)])[1:])
              for i in range(4)]


def tet10_shape_derivatives(xi):
    """dN_a/dxi_k (10, 3) of the App. A quadratic interpolation at xi:
    corners N_c = L_c (2 L_c - 1), edge (i, j) N = 4 L_i L_j, L0 = 1 - sum xi."""
    L = np.array([1.0 - xi.sum(), xi[0], xi[1], xi[2]])
    dL = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    dN = np.empty((10, 3))
    for c in range(4):
        dN[c] = (4.0 * L[c] - 1.0) * dL[c]
    edges = ((0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3))
    for k, (i, j) in enumerate(edges):
        dN[4 + k] = 4.0 * (L[i] * dL[j] + L[j] * dL[i])
    return dN


def tet20_shape_derivatives(xi):
    """dN_a/dxi_k (20, 3) of the cubic interpolation at xi (node order of
    scenegen's cubic grids)."""
    L = np.array([1.0 - xi.sum(), xi[0], xi[1], xi[2]])
    dL = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    dN = np.empty((20, 3))
    for c in range(4):
        # d/dL [L (3L-1)(3L-2) / 2] = (27 L^2 - 18 L + 2) / 2
        dN[c] = 0.5 * (27.0 * L[c] ** 2 - 18.0 * L[c] + 2.0) * dL[c]
    edges = ((0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3))
    for k, (i, j) in enumerate(edges):
        for slot, (u, v) in enumerate(((i, j), (j, i))):
            # N = 9/2 L_u L_v (3 L_u - 1)
            dN[4 + 2 * k + slot] = 4.5 * ((6.0 * L[u] - 1.0) * L[v] * dL[u]
                                          + L[u] * (3.0 * L[u] - 1.0) * dL[v])
    faces = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
    for c, (i, j, k) in enumerate(faces):
        dN[16 + c] = 27.0 * (L[j] * L[k] * dL[i] + L[i] * L[k] * dL[j] + L[i] * L[j] * dL[k])
    return dN


def _keast11():
    """Keast's 11-point rule of degree 4 on the reference tet (weights sum to
    the volume 1/6); symmetric under the vertex permutations."""
    rule = [(-74.0 / 5625.0, np.array([0.25, 0.25, 0.25]))]
    a, b = 11.0 / 14.0, 1.0 / 14.0
    for i in range(4):
        L = np.full(4, b)
        L[i] = a
        rule.append((343.0 / 45000.0, L[1:].copy()))
    c = (1.0 + np.sqrt(5.0 / 14.0)) / 4.0
    d = (1.0 - np.sqrt(5.0 / 14.0)) / 4.0
    for i in range(4):
        for j in range(i + 1, 4):
            L = np.full(4, d)
            L[i] = L[j] = c
            rule.append((56.0 / 2250.0, L[1:].copy()))
    return rule


TET20_RULE = _keast11()


def _snh_density(F, mu_, lam_):
    """psi, dpsi/dF and (lazily) d2psi/dF2 of Stable Neo-Hookean (App. B)."""
    Ic = np.einsum("eij,eij->e", F, F)
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    J = np.einsum("ei,ei->e", f0, np.cross(f1, f2))
    cof = np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=2)
    alpha = 1.0 + mu_ / lam_ - mu_ / (4.0 * lam_)
    psi = 0.5 * mu_ * (Ic - 3.0) + 0.5 * lam_ * (J - alpha) ** 2 - 0.5 * mu_ * np.log(Ic + 1.0)
    s1 = mu_ * (1.0 - 1.0 / (Ic + 1.0))
    s2 = lam_ * (J - alpha)
    P = s1[:, None, None] * F + s2[:, None, None] * cof

    def d2():
        return (s1[:, None, None, None, None] * _I4(F.shape[0])
                + (2.0 * mu_ / (Ic + 1.0) ** 2)[:, None, None, None, None]
                * np.einsum("eij,ekl->eijkl", F, F)
                + lam_[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", cof, cof)
                + s2[:, None, None, None, None] * _hess_J(F))
    return psi, P, d2


def snh_tet4_filtered(x, X, mu, lam):
    """E, g and the filtered Hessian V sum b_aj b_bl [d2psi]+_ijkl of linear
    SNH tets, [.]+ clamping the eigenvalues of the 9x9 matrix d2psi_(ij),(kl)
    at zero (eigh)."""
    mu_, lam_ = snh_reparam(np.asarray(mu, dtype=np.float64), np.asarray(lam, dtype=np.float64))
    V, F, _, _, b = _tet_kinematics(x, X)
    psi, P, d2 = _snh_density(F, mu_, lam_)
    A = d2().reshape(-1, 9, 9)
    w, Q = np.linalg.eigh(0.5 * (A + np.swapaxes(A, 1, 2)))
    Ap = np.einsum("eij,ej,ekj->eik", Q, np.maximum(w, 0.0), Q).reshape(-1, 3, 3, 3, 3)
    E = V * psi
    g = V[:, None, None] * np.einsum("eij,eaj->eai", P, b)
    H = V[:, None, None, None, None] * np.einsum("eaj,ebl,eijkl->eaibk", b, b, Ap)
    return E, g, H


def snh_tet20(x, X, mu, lam, want_hess=True):
    """Cubic tets: as snh_tet10 with the cubic interpolation and its rule."""
    return _snh_high_order(x, X, mu, lam, want_hess, TET20_RULE, tet20_shape_derivatives)


def snh_tet10(x, X, mu, lam, want_hess=True, rule=None):
    """Energy, gradient (E,10,3) and Hessian (E,10,3,10,3) of a quadratic tet:
    at each quadrature point the shape gradients b_a = J_X^-T dN_a/dxi give
    dF_ij/dx_{a,m} = delta_im b_a[j], and the point adds w |det J_X| times
    psi, P b_a and b_a d2psi b_b to E, g_a and H_ab."""
    return _snh_high_order(x, X, mu, lam, want_hess, TET10_RULE if rule is None else rule,
                           tet10_shape_derivatives)


def _snh_high_order(x, X, mu, lam, want_hess, rule, shape_derivatives):
    mu_, lam_ = snh_reparam(np.asarray(mu, dtype=np.float64), np.asarray(lam, dtype=np.float64))
    n, k = x.shape[0], x.shape[1]
    E = np.zeros(n, dtype=x.dtype)
    g = np.zeros((n, k, 3), dtype=x.dtype)
    H = np.zeros((n, k, 3, k, 3), dtype=x.dtype) if want_hess else None
    for w, xi in rule:
        dN = shape_derivatives(xi)
        JX = np.einsum("eai,ak->eik", X, dN)
        Jx = np.einsum("eai,ak->eik", x, dN)
        JXinv = np.linalg.inv(JX)
        wdet = w * np.abs(np.linalg.det(JX))
        F = Jx @ JXinv
        b = np.einsum("ak,ekj->eaj", dN, JXinv)
        psi, P, d2 = _snh_density(F, mu_, lam_)
        E = E + wdet * psi
        g = g + wdet[:, None, None] * np.einsum("eij,eaj->eai", P, b)
        if want_hess:
            H = H + wdet[:, None, None, None, None] * np.einsum("eaj,ebl,eijkl->eaibk", b, b, d2())
    return E, g, H


# ----------------------------------------------------------------------------
# StVK triangle membrane
# ----------------------------------------------------------------------------
def tri_rest_frame(X):
    """2x2 rest matrix Dm of a triangle in the orthonormal frame (e1, e2) of its
    plane: e1 along X1-X0, e2 = n x e1.  Returns (Dm, area)."""
    d1 = X[:, 1] - X[:, 0]
    d2 = X[:, 2] - X[:, 0]
    e1 = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    n = np.cross(d1, d2)
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    e2 = np.cross(n, e1)
    Dm = np.empty((X.shape[0], 2, 2))
    Dm[:, 0, 0] = np.einsum("ei,ei->e", d1, e1)
    Dm[:, 0, 1] = np.einsum("ei,ei->e", d2, e1)
    Dm[:, 1, 0] = np.einsum("ei,ei->e", d1, e2)
    Dm[:, 1, 1] = np.einsum("ei,ei->e", d2, e2)
    area = 0.5 * np.abs(np.linalg.det(Dm))
    return Dm, area


def stvk_tri3(x, X, mu, lam, thickness, want_hess=True):
    """Energy, gradient and Hessian of h A psi_StVK(F) for a membrane triangle.

    F = [x1-x0, x2-x0] Dm^-1 (3x2), Green strain Eg = (F^T F - I)/2,
    psi = mu |Eg|_F^2 + lam/2 tr(Eg)^2, first Piola P = F S with
    S = 2 mu Eg + lam tr(Eg) I.
    """
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    Dm, A = tri_rest_frame(X)
    Dinv = np.linalg.inv(Dm)
    F = _cols(x) @ Dinv                                  # (E,3,2)
    C = np.einsum("eki,ekj->eij", F, F)
    Eg = 0.5 * (C - np.eye(2)[None])
    trE = Eg[:, 0, 0] + Eg[:, 1, 1]
    psi = mu * np.einsum("eij,eij->e", Eg, Eg) + 0.5 * lam * trE ** 2
    hA = thickness * A
    E = hA * psi
    S = 2.0 * mu[:, None, None] * Eg + (lam * trE)[:, None, None] * np.eye(2)[None]
    P = F @ S
    b = _shape_gradients(Dinv)                           # (E,3,2)
    g = hA[:, None, None] * np.einsum("eij,eaj->eai", P, b)
    if not want_hess:
        return E, g, None
    # d(F S)_ij / dF_kl = delta_ik S_lj + mu (F_il F_kj + (F F^T)_ik delta_jl) + lam F_ij F_kl
    I2 = np.eye(2)
    I3 = np.eye(3)
    FFt = np.einsum("eim,ekm->eik", F, F)
    d2 = (np.einsum("ik,elj->eijkl", I3, S)
          + mu[:, None, None, None, None] * (np.einsum("eil,ekj->eijkl", F, F)
                                             + np.einsum("eik,jl->eijkl", FFt, I2))
          + lam[:, None, None, None, None] * np.einsum("eij,ekl->eijkl", F, F))
    H = hA[:, None, None, None, None] * np.einsum("eaj,ebl,eijkl->eaibk", b, b, d2)
    return E, g, H


# ----------------------------------------------------------------------------
# Quadratic bending hinge (Bergou et al. 2006)
# ----------------------------------------------------------------------------
def _cot(u, v):
    return np.einsum("ei,ei->e", u, v) / np.linalg.norm(np.cross(u, v), axis=1)


def hinge_rest(X):
    """Cotangent weights K (E,4) and scale 3/(A0+A1) of rest hinges.

    Nodes 0,1 span the shared edge, 2 and 3 are the wing tips of triangles
    (0,1,2) and (0,1,3).  a_t, b_t are the interior angles at X0 and X1 of
    triangle t; K = [cot b0 + cot b1, cot a0 + cot a1, -(cot a0 + cot b0),
    -(cot a1 + cot b1)].
    """
    X0, X1, X2, X3 = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
    ca0 = _cot(X1 - X0, X2 - X0)
    cb0 = _cot(X0 - X1, X2 - X1)
    ca1 = _cot(X1 - X0, X3 - X0)
    cb1 = _cot(X0 - X1, X3 - X1)
    K = np.stack([cb0 + cb1, ca0 + ca1, -(ca0 + cb0), -(ca1 + cb1)], axis=1)
    A0 = 0.5 * np.linalg.norm(np.cross(X1 - X0, X2 - X0), axis=1)
    A1 = 0.5 * np.linalg.norm(np.cross(X1 - X0, X3 - X0), axis=1)
    return K, 3.0 / (A0 + A1)


def hinge4(x, X, kb, want_hess=True):
    """E = k_b/2 x^T Q x, g = k_b Q x, H = k_b Q with Q = c (K K^T) (x) I3."""
    K, c = hinge_rest(X)
    kb = np.broadcast_to(np.asarray(kb, dtype=np.float64), c.shape)
    s = np.einsum("ea,eai->ei", K, x)                    # sum_a K_a x_a
    E = 0.5 * kb * c * np.einsum("ei,ei->e", s, s)
    g = (kb * c)[:, None, None] * K[:, :, None] * s[:, None, :]
    if not want_hess:
        return E, g, None
    H = (kb * c)[:, None, None, None, None] * np.einsum("ea,eb,ik->eaibk", K, K, np.eye(3))
    return E, g, H


# ----------------------------------------------------------------------------
# Inertia (per node)
# ----------------------------------------------------------------------------
def inertia(x, x_tilde, m, dt):
    """E_i = m_i/(2 dt^2)|x_i - x~_i|^2, g_i = m_i/dt^2 (x_i - x~_i), H_ii = m_i/dt^2 I."""
    d = x - x_tilde
    w = m / dt ** 2
    E = 0.5 * w * np.einsum("ni,ni->n", d, d)
    g = w[:, None] * d
    return E, g, w


def x_tilde(x_t, v_t, dt, gravity):
    """Predicted position x(t) + dt v(t) + dt^2 g (Eq. 2; gravity enters here)."""
    return x_t + dt * v_t + dt ** 2 * np.asarray(gravity, dtype=np.float64)[None, :]


def element_eval(es, x, X, want_hess=True, x_lag=None):
    """Dispatch on the energy kind of an EnergySet (element arrays gathered).
    x_lag: positions the lagged rotations are taken at (default: rest)."""
    from .rest import lame, young_array
    xe = x[es.conn]
    Xe = X[es.conn]
    if es.kind == 1:
        mu, lam = lame(young_array(es), es.poisson)
        return stvk_tri3(xe, Xe, mu, lam, es.thickness, want_hess)
    if es.kind == 2:
        return hinge4(xe, Xe, es.bend_kb, want_hess)
    mu, lam = lame(young_array(es), es.poisson)
    if es.kind == 0:
        return snh_tet4(xe, Xe, mu, lam, want_hess)
    if es.kind == 3:
        return nh_tet4(xe, Xe, mu, lam, want_hess)
    if es.kind == 4:
        return stvk_tet4(xe, Xe, mu, lam, want_hess)
    if es.kind in (5, 6):
        R = lagged_rotations(Xe if x_lag is None else x_lag[es.conn], Xe)
        f = fcr_tet4 if es.kind == 5 else arap_tet4
        return f(xe, Xe, mu, lam, R, want_hess)
    if es.kind == 7:
        return snh_tet10(xe, Xe, mu, lam, want_hess)
    if es.kind == 8:
        return snh_tet20(xe, Xe, mu, lam, want_hess)
    raise ValueError(f"unknown energy kind {es.kind}")
