"""TT basics (paper Sec. 2.1-2.2), FP64 numpy.

Conventions (Sec. 2.1): the multi-index has its last index fastest, so the
horizontal unfolding H(T) of a core T (r0 x n x r1) is the row-major reshape
to r0 x (n r1) and the vertical unfolding V(T) the row-major reshape to
(r0 n) x r1.  A full tensor is the row-major array over (i_1, ..., i_d).
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

TT = List[np.ndarray]


def H(core: np.ndarray) -> np.ndarray:
    """Horizontal unfolding, r0 x (n r1) (mode-1 matricization)."""
    return core.reshape(core.shape[0], -1)


def V(core: np.ndarray) -> np.ndarray:
    """Vertical unfolding, (r0 n) x r1."""
    return core.reshape(-1, core.shape[2])


def ranks(tt: Sequence[np.ndarray]) -> List[int]:
    return [int(tt[0].shape[0])] + [int(c.shape[2]) for c in tt]


def modes(tt: Sequence[np.ndarray]) -> List[int]:
    return [int(c.shape[1]) for c in tt]


def full(tt: Sequence[np.ndarray]) -> np.ndarray:
    """The full tensor of eq. (tt_decom_element): entry = product of the core
    slices T_1(i_1) ... T_d(i_d)."""
    acc = tt[0].reshape(tt[0].shape[1], tt[0].shape[2])
    for c in tt[1:]:
        acc = acc @ c.reshape(c.shape[0], -1)
        acc = acc.reshape(-1, c.shape[2])
    return acc.reshape(modes(tt))


def pkp_core(y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Partial Kronecker product along modes 1 and 3 (Sec. 2.1):
    A(ab, i, a'b') = Y(a, i, a') Z(b, i, b') with the Y index slow, i.e.
    slice i of A is kron(Y(:, i, :), Z(:, i, :))."""
    r0, n, r1 = y.shape
    s0, n2, s1 = z.shape
    assert n == n2
    out = np.empty((r0 * s0, n, r1 * s1))
    for i in range(n):
        out[:, i, :] = np.kron(y[:, i, :], z[:, i, :])
    return out


def pkp(y: Sequence[np.ndarray], z: Sequence[np.ndarray]) -> TT:
    """TT cores of the Hadamard product y (.) z, ranks r_k s_k (Sec. 2.2)."""
    if modes(y) != modes(z):
        raise ValueError("mode sizes differ")
    return [pkp_core(a, b) for a, b in zip(y, z)]


def _qr_pos(a: np.ndarray):
    """Economy Householder QR (LAPACK) with diag(R) >= 0."""
    q, r = np.linalg.qr(a, mode="reduced")
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q * sg[None, :], r * sg[:, None]


def orthogonalize_rl(tt: Sequence[np.ndarray]) -> TT:
    """Right-to-left orthogonalization, the first loop of Alg. 1: for
    k = d..2, QR of H(B_k)^T, H(B_k) <- Q^T, V(B_{k-1}) <- V(B_{k-1}) R^T.
    Returns cores 2..d right-orthogonal; the norm sits in core 1."""
    b = [c.copy() for c in tt]
    for k in range(len(b) - 1, 0, -1):
        r0, n, r1 = b[k].shape
        q, r = _qr_pos(H(b[k]).T)               # (n r1) x r0' ... r0' = min
        m = q.shape[1]
        b[k] = q.T.reshape(m, n, r1)
        p0, pn, _ = b[k - 1].shape
        b[k - 1] = (V(b[k - 1]) @ r.T).reshape(p0, pn, m)
    return b


def orthogonalize_lr(tt: Sequence[np.ndarray]) -> TT:
    """Left-to-right orthogonalization: cores 1..d-1 left-orthogonal."""
    b = [c.copy() for c in tt]
    for k in range(len(b) - 1):
        r0, n, r1 = b[k].shape
        q, r = _qr_pos(V(b[k]))
        m = q.shape[1]
        b[k] = q.reshape(r0, n, m)
        _, pn, p1 = b[k + 1].shape
        b[k + 1] = (r @ H(b[k + 1])).reshape(m, pn, p1)
    return b


def norm(tt: Sequence[np.ndarray]) -> float:
    """Frobenius norm (Sec. 2.1) as ||B_1||_F after right-to-left
    orthogonalization (the norm identity used in Alg. 1)."""
    return float(np.linalg.norm(orthogonalize_rl(tt)[0]))


def add(a: Sequence[np.ndarray], b: Sequence[np.ndarray], alpha: float = 1.0, beta: float = 1.0) -> TT:
    """TT of alpha*a + beta*b: first cores side by side, interior cores
    block-diagonal, last cores stacked (ranks add)."""
    d = len(a)
    if modes(a) != modes(b):
        raise ValueError("mode sizes differ")
    if d == 1:
        return [alpha * a[0] + beta * b[0]]
    out = []
    for k in range(d):
        ca, cb = a[k], b[k]
        if k == 0:
            out.append(np.concatenate([alpha * ca, beta * cb], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([ca, cb], axis=0))
        else:
            c = np.zeros((ca.shape[0] + cb.shape[0], ca.shape[1], ca.shape[2] + cb.shape[2]))
            c[:ca.shape[0], :, :ca.shape[2]] = ca
            c[ca.shape[0]:, :, ca.shape[2]:] = cb
            out.append(c)
    return out


def rel_err(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """||a - b||_F / ||b||_F (the error measure of Sec. 5), with the
    difference formed as a TT and its norm taken by orthogonalization, so
    errors far below sqrt(machine eps) are resolved."""
    nb = norm(b)
    diff = norm(add(a, b, 1.0, -1.0))
    return diff / nb if nb > 0 else diff


def inner_gram(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """<a, b> by the left-to-right Gram transfer
    G_k = sum_i A_k(i)^T G_{k-1} B_k(i) (an independent route to norms)."""
    g = np.ones((1, 1))
    for ca, cb in zip(a, b):
        g = np.einsum("ab,aic,bid->cd", g, ca, cb)
    return float(g[0, 0])
