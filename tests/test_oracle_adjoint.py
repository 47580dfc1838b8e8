"""Pins of the oracle's reference gradients: finite differences of the loss
(exact for the quadratic dependence on g; Richardson-extrapolated central
differences for k and q) and the eigenvector-derivative formula."""
import numpy as np
import pytest

import synth
from oracle import adjoint


def tiny(nw=3, na=2, seed=4):
    s = synth.make_system(nw, na, synth.box((3, 2, 2)), synth.box((3, 3, 1)), [seed, 7],
                          mass=np.linspace(1.0, 2.5, na))
    gen = np.random.default_rng(seed)
    k = gen.random((3, 3))
    q = gen.random((2, 3))
    return s, k, q


def richardson(f, x0, h):
    d1 = (f(x0 + h) - f(x0 - h)) / (2 * h)
    d2 = (f(x0 + h / 2) - f(x0 - h / 2)) / h
    return (4 * d2 - d1) / 3


def test_gradient_in_g_matches_directional_difference():
    s, k, q = tiny()
    res = adjoint.loss_and_grads(s, k, q, seed=5)
    gen = np.random.default_rng(1)
    dg = gen.standard_normal(s.g.shape) + 1j * gen.standard_normal(s.g.shape)
    g0 = s.g.copy()
    t = 1e-3

    def loss_at(tt):
        s.g = g0 + tt * dg
        return adjoint.loss_only(s, k, q, seed=5)

    fd = (loss_at(t) - loss_at(-t)) / (2 * t)       # exact for a quadratic, up to rounding
    s.g = g0
    an = float(np.real(np.sum(np.conj(res["dg"]) * dg)))
    assert abs(fd - an) < 1e-9 * abs(an)
    assert res["loss"] == pytest.approx(adjoint.loss_only(s, k, q, seed=5), rel=1e-14)


@pytest.mark.parametrize("which", ["k", "q"])
def test_gradient_in_k_and_q_matches_finite_differences(which):
    s, k, q = tiny()
    res = adjoint.loss_and_grads(s, k, q, seed=9)
    pts = k if which == "k" else q
    grad = res["dk"] if which == "k" else res["dq"]
    worst = 0.0
    for i in range(len(pts)):
        for d in range(3):
            def f(x):
                p = pts.copy()
                p[i, d] = x
                return adjoint.loss_only(s, p if which == "k" else k, q if which == "k" else p, seed=9)
            fd = richardson(f, pts[i, d], 1e-5)
            worst = max(worst, abs(fd - grad[i, d]) / max(1.0, np.abs(grad).max()))
    assert worst < 1e-7, worst


def test_gradient_with_nontrivial_masses_and_q_offset():
    s, k, q = tiny(nw=2, na=3, seed=8)
    res = adjoint.loss_and_grads(s, k, q, seed=2, q_offset=5)
    def f(x):
        p = q.copy()
        p[1, 0] = x
        return adjoint.loss_only(s, k, p, seed=2, q_offset=5)
    fd = richardson(f, q[1, 0], 1e-5)
    assert abs(fd - res["dq"][1, 0]) < 1e-7 * max(1.0, abs(fd))


def test_eigenvector_derivative_formula():
    gen = np.random.default_rng(3)
    a = gen.standard_normal((5, 5)) + 1j * gen.standard_normal((5, 5))
    h = a + a.conj().T
    b = gen.standard_normal((5, 5)) + 1j * gen.standard_normal((5, 5))
    dh = b + b.conj().T
    lam, v = np.linalg.eigh(h)
    dv = adjoint.eigvec_derivative(h, dh, lam, v)
    eps = 1e-6
    lam2, v2 = np.linalg.eigh(h + eps * dh)
    # align phases of the perturbed columns with the unperturbed ones
    ph = np.sum(np.conj(v) * v2, axis=0)
    v2 = v2 * (np.conj(ph) / np.abs(ph))[None, :]
    fd = (v2 - v) / eps
    # the gauge-fixed derivative has no component along v itself
    assert np.abs(fd - dv).max() < 1e-4
    # first-order perturbation: eigenvector derivative satisfies (H - l) dv = -(dH - dl) v
    dl = np.real(np.einsum("ai,ab,bi->i", np.conj(v), dh, v))
    lhs = h @ dv - dv * lam[None, :]
    rhs = -(dh @ v - v * dl[None, :])
    assert np.abs(lhs - rhs).max() < 1e-10
