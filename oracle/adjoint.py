"""Reference gradients of the weighted loss L = sum w |g_mn nu(k,q)|^2.

TEST INFRASTRUCTURE ONLY.  Plain NumPy FP64, written from the chain rule of
the nested loop (Eqs. (9)-(10)) and the textbook perturbation formula for a
Hermitian eigendecomposition; independent of the HIP adjoint kernels.

Conventions: the gradient of the real loss with respect to a complex array z
is dL/dRe z + i dL/dIm z (so dL = Re sum conj(zbar) dz); the gradient with
respect to the real coordinates of k and q is an ordinary real gradient.
k+q is evaluated directly (no grid lookup), so dL/dk and dL/dq include the
dependence of V(k+q) on both.
"""
from __future__ import annotations

import numpy as np

from . import core

TWO_PI = 2.0 * np.pi


def _mode_mass(system):
    return np.repeat(np.asarray(system.mass, dtype=np.float64), 3)


def _weights(seed, nq, nk, nm, nw, q_offset=0):
    iq = np.repeat(np.arange(nq), nk) + q_offset
    ik = np.tile(np.arange(nk), nq)
    w = core.splitmix64_weights(seed, core.element_index(iq, ik, nk, nm, nw))
    return w.reshape(nq, nk, nm, nw, nw)


def eigvec_derivative(mat, dmat, vals, vecs):
    """First-order change of the eigenvector columns of a Hermitian matrix:
    dV = V (F o (V^H dM V)) with F_ij = 1/(l_j - l_i) off the diagonal and 0 on
    it (the phase of each column is held fixed)."""
    a = np.conj(np.swapaxes(vecs, -1, -2)) @ dmat @ vecs
    diff = vals[..., None, :] - vals[..., :, None]
    n = vals.shape[-1]
    eye = np.eye(n, dtype=bool)
    f = np.where(eye, 0.0, 1.0 / np.where(eye, 1.0, diff))
    return vecs @ (f * a)


def eigh_backward(vals, vecs, vbar):
    """Gradient with respect to a Hermitian matrix M = V diag(l) V^H of a loss
    that depends on M only through V (and is invariant to column phases):
    Mbar = V (F o (V^H Vbar - Vbar^H V) / 2) V^H, F_ij = 1/(l_j - l_i)."""
    vh = np.conj(np.swapaxes(vecs, -1, -2))
    s = vh @ vbar
    skew = 0.5 * (s - np.conj(np.swapaxes(s, -1, -2)))
    diff = vals[..., None, :] - vals[..., :, None]
    n = vals.shape[-1]
    eye = np.eye(n, dtype=bool)
    f = np.where(eye, 0.0, 1.0 / np.where(eye, 1.0, diff))
    return vecs @ (f * skew) @ vh


def _phase_derivative_matrix(points, r, w, mats):
    """dM/dp_d = sum_R 2 pi i R_d w_R exp(2 pi i p.R) M(R) for d = 0, 1, 2: [3][N][n][n]."""
    ph = core.phases(points, r, w)
    out = []
    for d in range(3):
        out.append(np.einsum("kr,rab->kab", ph * (2j * np.pi * r[:, d].astype(np.float64))[None, :], mats))
    return np.stack(out)


def loss_and_grads(system, k, q, seed, q_offset=0):
    """L, dL/dg(Re,Rp) [Np][Ne][Nm][Nw][Nw], dL/dk [Nk][3], dL/dq [Nq][3]."""
    k = np.asarray(k, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nk, nq, nw, nm = len(k), len(q), system.nw, system.nm
    f = core.interpolate(system, k, q, return_all=True)
    w = _weights(seed, nq, nk, nm, nw, q_offset)
    ghat = f["ghat"]
    loss = float(np.sum(w * np.abs(ghat) ** 2))

    # Y = A^H X B with A = V(k+q), B = V(k), X = gw_nu
    ybar = 2.0 * w * ghat
    a = f["v_kq"][:, :, None]                       # [q][k][1][nw][nw]
    b = f["v_k"][None, :, None]                      # [1][k][1][nw][nw]
    ah = np.conj(np.swapaxes(a, -1, -2))
    bh = np.conj(np.swapaxes(b, -1, -2))
    x = f["gw_nu"]
    xbar = a @ ybar @ bh                             # [q][k][nu][m'][n']
    vk_bar = np.sum(np.conj(np.swapaxes(x, -1, -2)) @ a @ ybar, axis=(0, 2))     # [k][nw][nw]
    vkq_bar = np.sum(x @ b @ np.conj(np.swapaxes(ybar, -1, -2)), axis=2)         # [q][k][nw][nw]

    # mode vectors: gw_nu = sum_ka gw_ka u_{ka,nu}
    u = f["u"]                                       # [q][ka][nu]
    gwbar = np.einsum("qkvmn,qav->qkamn", xbar, np.conj(u))
    ubar = np.einsum("qkamn,qkvmn->qav", np.conj(f["gw"]), xbar)

    # Re sum: gw(k,q) = sum_e Pk[k,e] G(e,q)
    pk = core.phases(k, system.r_e, system.w_e)      # [k][e]
    g_req = f["g_req"]                               # [q][e][ka][m][n]
    nq_, ne = g_req.shape[:2]
    gflat = g_req.reshape(nq, ne, -1)
    gwflat = gwbar.reshape(nq, nk, -1)
    g_req_bar = np.einsum("ke,qkx->qex", np.conj(pk), gwflat)                   # [q][e][X]
    pk_bar = np.einsum("qkx,qex->ke", gwflat, np.conj(gflat))

    # Rp sum: G(e,q) = sum_p Pq[q,p] g(e,p)
    pq = core.phases(q, system.r_p, system.w_p)      # [q][p]
    g = system.g.astype(np.complex128).reshape(system.g.shape[0], -1)           # [p][eX]
    gbar = (np.conj(pq).T @ g_req_bar.reshape(nq, -1)).reshape(system.g.shape)
    pq_bar = g_req_bar.reshape(nq, -1) @ np.conj(g).T                          # [q][p]

    # k, q through the phase factors
    re_f = system.r_e.astype(np.float64)
    rp_f = system.r_p.astype(np.float64)
    dk = np.real(np.einsum("ke,ke,ed->kd", np.conj(pk_bar), pk, 2j * np.pi * re_f))
    dq = np.real(np.einsum("qp,qp,pd->qd", np.conj(pq_bar), pq, 2j * np.pi * rp_f))

    # k through V(k); k and q through V(k+q)
    h_r = system.h_r.astype(np.complex128)
    hbar_k = eigh_backward(f["eps_k"], f["v_k"], vk_bar)
    dh_k = _phase_derivative_matrix(k, system.r_h, system.w_h, h_r)            # [3][k][nw][nw]
    dk += np.real(np.einsum("kab,dkab->kd", np.conj(hbar_k), dh_k))
    kq = (q[:, None, :] + k[None, :, :]).reshape(-1, 3)
    hbar_kq = eigh_backward(f["eps_kq"].reshape(-1, nw), f["v_kq"].reshape(-1, nw, nw),
                            vkq_bar.reshape(-1, nw, nw))
    dh_kq = _phase_derivative_matrix(kq, system.r_h, system.w_h, h_r)
    s_kq = np.real(np.einsum("pab,dpab->pd", np.conj(hbar_kq), dh_kq)).reshape(nq, nk, 3)
    dk += s_kq.sum(axis=0)
    dq += s_kq.sum(axis=1)

    # q through u(q) = e(q) / sqrt(M)
    ebar = ubar / np.sqrt(_mode_mass(system))[None, :, None]
    dbar = eigh_backward(f["lam"], f["e"], ebar)
    m = _mode_mass(system)
    c_scaled = np.asarray(system.c_r, dtype=np.float64) / np.sqrt(m[:, None] * m[None, :])[None]
    dd = _phase_derivative_matrix(q, system.r_c, system.w_c, c_scaled.astype(np.complex128))
    dq += np.real(np.einsum("qab,dqab->qd", np.conj(dbar), dd))
    return dict(loss=loss, dg=gbar, dk=dk, dq=dq)


def loss_only(system, k, q, seed, q_offset=0):
    k = np.asarray(k, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    ghat = core.interpolate(system, k, q)
    w = _weights(seed, len(q), len(k), system.nm, system.nw, q_offset)
    return float(np.sum(w * np.abs(ghat) ** 2))
