"""Conditional contact energy: IPC barrier between a point and the plane of a
triangle (oracle).

TEST INFRASTRUCTURE ONLY.
* Conditional evaluation (Sec. 5.2, extensions; Eq. 9): the energy of an
  element is E_e+ when its activation c_e > 0 and zero otherwise.
* Contact barrier (Sec. 5.4): E_c(d) = -k_c (d - d_hat)^2 ln(d / d_hat).
* Element (p, t0, t1, t2): d = (p - t0) . N / |N|, N = (t1 - t0) x (t2 - t0),
  the signed distance of node p to the plane through the triangle; activation
  c = d_hat - d.  Positions with d <= 0 are outside the barrier's domain: the
  energy is +inf there (a line search backs off), derivatives are not taken.

The derivatives are hand-derived: with u = p - t0, e1 = t1 - t0, e2 = t2 - t0
(z = (u, e1, e2) = L q), s = u . N is trilinear and m = |N| a norm of the
bilinear N; d = s / m follows by the quotient rule, and the barrier by the
chain rule, g = b'(d) grad d, H = b''(d) grad d grad d^T + b'(d) hess d.
"""
from __future__ import annotations

import numpy as np


def _skew(a):
    """[a]_x for a batch of vectors (E,3): [a]_x b = a x b."""
    z = np.zeros(a.shape[:-1], dtype=a.dtype)
    return np.stack([np.stack([z, -a[..., 2], a[..., 1]], -1),
                     np.stack([a[..., 2], z, -a[..., 0]], -1),
                     np.stack([-a[..., 1], a[..., 0], z], -1)], -2)


# dz = L dq for q = (p, t0, t1, t2) and z = (u, e1, e2)
_L = np.zeros((9, 12))
for _k, (_plus, _minus) in enumerate([(0, 1), (2, 1), (3, 1)]):
    _L[3 * _k:3 * _k + 3, 3 * _plus:3 * _plus + 3] = np.eye(3)
    _L[3 * _k:3 * _k + 3, 3 * _minus:3 * _minus + 3] = -np.eye(3)


def point_plane_distance(x):
    """d (E,), grad d (E,12) and hess d (E,12,12) for elements x (E,4,3)."""
    u = x[:, 0] - x[:, 1]
    e1 = x[:, 2] - x[:, 1]
    e2 = x[:, 3] - x[:, 1]
    N = np.cross(e1, e2)
    m = np.sqrt(np.einsum("ei,ei->e", N, N))
    n = N / m[:, None]
    s = np.einsum("ei,ei->e", u, N)
    d = s / m
    n_el = x.shape[0]
    # first derivatives with respect to z = (u, e1, e2)
    ds = np.concatenate([N, np.cross(e2, u), np.cross(u, e1)], axis=1)
    JN = np.concatenate([-_skew(e2), _skew(e1)], axis=2)          # dN/d(e1, e2): (E,3,6)
    dm = np.concatenate([np.zeros((n_el, 3), dtype=x.dtype), np.einsum("eki,ek->ei", JN, n)], axis=1)
    # second derivatives
    d2s = np.zeros((n_el, 9, 9), dtype=x.dtype)
    d2s[:, 0:3, 3:6] = -_skew(e2)
    d2s[:, 3:6, 0:3] = _skew(e2)
    d2s[:, 0:3, 6:9] = _skew(e1)
    d2s[:, 6:9, 0:3] = -_skew(e1)
    d2s[:, 3:6, 6:9] = -_skew(u)
    d2s[:, 6:9, 3:6] = _skew(u)
    P = (np.eye(3)[None] - np.einsum("ei,ej->eij", n, n)) / m[:, None, None]
    d2m = np.zeros((n_el, 9, 9), dtype=x.dtype)
    d2m[:, 3:9, 3:9] = np.einsum("eki,ekl,elj->eij", JN, P, JN)
    # sum_k n_k d2 N_k / d e1 d e2 = -[n]_x (and its transpose)
    d2m[:, 3:6, 6:9] += -_skew(n)
    d2m[:, 6:9, 3:6] += _skew(n)
    dd = ds / m[:, None] - s[:, None] * dm / m[:, None] ** 2
    d2d = (d2s / m[:, None, None]
           - (np.einsum("ei,ej->eij", ds, dm) + np.einsum("ei,ej->eij", dm, ds)) / m[:, None, None] ** 2
           + 2.0 * s[:, None, None] * np.einsum("ei,ej->eij", dm, dm) / m[:, None, None] ** 3
           - s[:, None, None] * d2m / m[:, None, None] ** 2)
    return d, dd @ _L, np.einsum("ai,eab,bj->eij", _L, d2d, _L)


def barrier(d, kc, dhat):
    """b(d) = -k_c (d - d_hat)^2 ln(d / d_hat) and its first two derivatives."""
    t = d - dhat
    lg = np.log(d / dhat)
    b = -kc * t * t * lg
    b1 = -kc * (2.0 * t * lg + t * t / d)
    b2 = -kc * (2.0 * lg + 4.0 * t / d - t * t / (d * d))
    return b, b1, b2


def activation(x, dhat):
    """c_e = d_hat - d for elements x (E,4,3)."""
    u = x[:, 0] - x[:, 1]
    N = np.cross(x[:, 2] - x[:, 1], x[:, 3] - x[:, 1])
    return dhat - np.einsum("ei,ei->e", u, N) / np.sqrt(np.einsum("ei,ei->e", N, N))


def point_plane_barrier(x, kc, dhat, want_hess=True):
    """E (E,), g (E,4,3), H (E,4,3,4,3) of the conditional barrier; inactive
    elements contribute zero, active ones with d <= 0 have E = +inf."""
    n_el = x.shape[0]
    E = np.zeros(n_el, dtype=x.dtype)
    g = np.zeros((n_el, 4, 3), dtype=x.dtype)
    H = np.zeros((n_el, 4, 3, 4, 3), dtype=x.dtype) if want_hess else None
    act = np.real(activation(x, dhat)) > 0.0
    if not np.any(act):
        return E, g, H, act
    d, dd, d2d = point_plane_distance(x[act])
    inside = np.real(d) > 0.0
    b, b1, b2 = barrier(np.where(inside, d, dhat), kc, dhat)
    Ea = np.where(inside, b, np.inf)
    E[act] = Ea
    g[act] = (b1[:, None] * dd).reshape(-1, 4, 3)
    if want_hess:
        Ha = b2[:, None, None] * np.einsum("ei,ej->eij", dd, dd) + b1[:, None, None] * d2d
        H[act] = Ha.reshape(-1, 4, 3, 4, 3)
    return E, g, H, act
