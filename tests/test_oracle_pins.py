"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, invariants, inverse transforms, brute force, published
generator vectors).  Each test would fail for a plausible slip in the oracle:
a dropped term, a flipped phase sign, a transposed or conjugated operand."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.core import element_index

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_system(nw=3, na=1, ne_box=(3, 2, 2), np_box=(2, 2, 1), seed=11, mass=None):
    r_e = synth.box(ne_box)
    r_p = synth.box(np_box)
    return synth.make_system(nw, na, r_e, r_p, [seed, 99], mass=mass)


def rand_pts(n, seed):
    return np.random.default_rng(seed).random((n, 3))


# --------------------------------------------------------------------------
# a1: phase convention, single-R closed form (Eq. (7) with one nonzero term)
# --------------------------------------------------------------------------

def test_single_r_term_gives_pure_phase():
    s = synth.si_toy().system
    e0, p0 = 37, 91                        # two arbitrary lattice vectors of the 5^3 box
    g0 = s.g[p0, e0].copy()
    s.g = np.zeros_like(s.g)
    s.g[p0, e0] = g0
    k, q = rand_pts(5, 1), rand_pts(4, 2)
    res = oracle.interpolate(s, k, q, return_all=True)
    re0, rp0 = s.r_e[e0].astype(float), s.r_p[p0].astype(float)
    for iq in range(len(q)):
        for ik in range(len(k)):
            ang = 2 * np.pi * (k[ik] @ re0 + q[iq] @ rp0)
            expect = complex(np.cos(ang), np.sin(ang)) * g0
            np.testing.assert_allclose(res["gw"][iq, ik], expect, rtol=0, atol=1e-14)


def test_phase_reduction_is_exact_for_large_vectors():
    # exp(2 pi i k.R) for |R| ~ 1e6 must equal the phase of the reduced argument
    k = np.array([[0.25, 0.5, 0.125]])
    r = np.array([[1000000, 3, -2000001]], dtype=np.int32)
    ph = oracle.phases(k, r)[0, 0]
    # k.R = 250000 + 1.5 - 250000.125 = 1.375 -> reduced 0.375 -> angle 3 pi / 4
    assert abs(ph - complex(-np.sqrt(0.5), np.sqrt(0.5))) < 1e-15


# --------------------------------------------------------------------------
# a2: H(k), D(q) closed forms, Hermiticity, periodicity
# --------------------------------------------------------------------------

def test_tight_binding_chain_closed_form():
    # one orbital, on-site e0, hopping t*exp(i a) to R=+x (and its conjugate to -x):
    # H(k) = e0 + 2|t| cos(2 pi k_x + a).  The sign of a pins the phase sign.
    t, a, e0 = 0.7, 0.4, -0.3
    s = synth.System(nw=1, na=1, r_e=synth.box((3, 1, 1)), r_p=synth.box((1, 1, 1)),
                     r_h=np.array([[-1, 0, 0], [0, 0, 0], [1, 0, 0]], dtype=np.int32),
                     r_c=np.zeros((1, 3), dtype=np.int32),
                     h_r=np.array([[[t * np.exp(-1j * a)]], [[e0]], [[t * np.exp(1j * a)]]]),
                     c_r=np.eye(3)[None], mass=np.ones(1),
                     g=np.zeros((1, 3, 3, 1, 1), dtype=np.complex128))
    k = np.zeros((7, 3))
    k[:, 0] = np.linspace(-0.4, 0.9, 7)
    eps, v = oracle.bands(s, k)
    np.testing.assert_allclose(eps[:, 0], e0 + 2 * t * np.cos(2 * np.pi * k[:, 0] + a), atol=1e-14)
    np.testing.assert_allclose(np.abs(v[:, 0, 0]), 1.0, atol=1e-15)


def test_phonon_chain_closed_form_and_mass_scaling():
    # one atom of mass M, springs K_a along x: C(0) = 2 diag(K), C(+-x) = -diag(K)
    # lambda_a(q) = 2 K_a (1 - cos 2 pi q_x) / M, omega = 2 sqrt(K_a/M) |sin pi q_x|
    kk = np.array([0.5, 1.3, 2.9])
    m_atom = 2.5
    r_c = np.array([[-1, 0, 0], [0, 0, 0], [1, 0, 0]], dtype=np.int32)
    c_r = np.stack([-np.diag(kk), 2 * np.diag(kk), -np.diag(kk)])
    s = synth.System(nw=1, na=1, r_e=synth.box((1, 1, 1)), r_p=r_c, r_h=synth.box((1, 1, 1)),
                     r_c=r_c, h_r=np.ones((1, 1, 1), complex), c_r=c_r,
                     mass=np.array([m_atom]), g=np.zeros((3, 1, 3, 1, 1), complex))
    q = np.zeros((6, 3))
    q[:, 0] = np.linspace(0.05, 0.95, 6)
    lam, om, e = oracle.phonons(s, q)
    exp_lam = np.sort(2 * kk[None, :] * (1 - np.cos(2 * np.pi * q[:, :1])) / m_atom, axis=1)
    np.testing.assert_allclose(lam, exp_lam, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(om, np.sqrt(exp_lam), rtol=1e-13)
    u = oracle.mode_vectors(s, e)
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1 / np.sqrt(m_atom), rtol=1e-14)


def test_dynamical_matrix_phase_sign():
    # a single off-diagonal force constant a between atoms 0 and 1 at R=+x (and its
    # transpose at -x) gives D(q)[0,3] = a exp(+2 pi i q_x): pins the sign reading
    a = 0.8
    r_c = np.array([[-1, 0, 0], [0, 0, 0], [1, 0, 0]], dtype=np.int32)
    c = np.zeros((3, 6, 6))
    c[2, 0, 3] = a
    c[0, 3, 0] = a
    c[1] = np.eye(6)
    s = synth.System(nw=1, na=2, r_e=synth.box((1, 1, 1)), r_p=r_c, r_h=synth.box((1, 1, 1)),
                     r_c=r_c, h_r=np.ones((1, 1, 1), complex), c_r=c, mass=np.ones(2),
                     g=np.zeros((3, 1, 6, 1, 1), complex))
    q = np.array([[0.13, 0.0, 0.0], [0.71, 0.2, 0.0]])
    d = oracle.dynamical_q(s, q)
    np.testing.assert_allclose(d[:, 0, 3], a * np.exp(2j * np.pi * q[:, 0]), atol=1e-15)
    np.testing.assert_allclose(d[:, 3, 0], a * np.exp(-2j * np.pi * q[:, 0]), atol=1e-15)


def test_hermiticity_and_time_reversal():
    s = synth.si_toy().system
    k = rand_pts(9, 3)
    h = oracle.hamiltonian_k(s, k)
    np.testing.assert_allclose(h, np.conj(np.swapaxes(h, 1, 2)), atol=1e-14)
    d = oracle.dynamical_q(s, k)
    np.testing.assert_allclose(d, np.conj(np.swapaxes(d, 1, 2)), atol=1e-14)
    # real force constants: D(-q) = D(q)^*
    np.testing.assert_allclose(oracle.dynamical_q(s, -k), np.conj(d), atol=1e-14)


def test_periodicity_k_plus_G():
    w = synth.si_toy()
    s = w.system
    k, q = w.k[:4], w.q[:3]
    gk = np.array([[1, -2, 3]] * len(k), dtype=float)
    gq = np.array([[-1, 0, 2]] * len(q), dtype=float)
    a = oracle.interpolate(s, k, q, return_all=True)
    b = oracle.interpolate(s, k + gk, q + gq, return_all=True)
    np.testing.assert_allclose(b["gw"], a["gw"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["eps_k"], a["eps_k"], atol=1e-12)
    np.testing.assert_allclose(b["lam"], a["lam"], atol=1e-12)
    sa = oracle.block_sums(np.abs(a["ghat"]) ** 2, a["eps_kq"], a["eps_k"], a["lam"])
    sb = oracle.block_sums(np.abs(b["ghat"]) ** 2, a["eps_kq"], a["eps_k"], a["lam"])
    assert oracle.compare_block_sums(sb, sa)[0] < 1e-12


# --------------------------------------------------------------------------
# a3: eigensolves (library-routine pin)
# --------------------------------------------------------------------------

def test_eigh_residual_orthogonality_order():
    s = synth.mos2_2d(nk=4, nq=4).system
    k = rand_pts(20, 4)
    h = oracle.hamiltonian_k(s, k)
    eps, v = oracle.bands(s, k)
    hn = np.linalg.norm(h, axis=(1, 2))
    res = np.linalg.norm(h @ v - v * eps[:, None, :], axis=(1, 2))
    assert np.all(res <= 1e-12 * hn)
    eye = np.eye(s.nw)[None]
    assert np.abs(np.conj(np.swapaxes(v, 1, 2)) @ v - eye).max() < 1e-13
    assert np.all(np.diff(eps, axis=1) >= 0)


# --------------------------------------------------------------------------
# a4 + a6 (+ a5, a7): the coarse-grid round trip, Eq. (6) o Eq. (7)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nw,na", [(2, 1), (3, 2)])
def test_coarse_round_trip_wannier_to_bloch_to_wannier(nw, na):
    ne_box, np_box = (4, 3, 2), (2, 2, 2)
    s = tiny_system(nw=nw, na=na, ne_box=ne_box, np_box=np_box, seed=5 + nw,
                    mass=np.linspace(1.0, 3.0, na))
    kc = synth.uniform_grid(ne_box)
    qc = synth.uniform_grid(np_box)
    a = oracle.interpolate(s, kc, qc, return_all=True)
    back = oracle.coarse_transform(a["ghat"], kc, qc, a["v_k"], a["v_kq"], a["u"], s.r_e, s.r_p)
    np.testing.assert_allclose(back, s.g, rtol=0, atol=1e-13 * np.abs(s.g).max())


def test_coarse_round_trip_bloch_to_wannier_to_bloch():
    ne_box, np_box = (3, 2, 2), (2, 1, 2)
    s = tiny_system(nw=2, na=1, ne_box=ne_box, np_box=np_box, seed=21)
    kc = synth.uniform_grid(ne_box)
    qc = synth.uniform_grid(np_box)
    ref = oracle.interpolate(s, kc, qc, return_all=True)
    gen = np.random.default_rng(3)
    g_kq = gen.standard_normal(ref["ghat"].shape) + 1j * gen.standard_normal(ref["ghat"].shape)
    s.g = oracle.coarse_transform(g_kq, kc, qc, ref["v_k"], ref["v_kq"], ref["u"], s.r_e, s.r_p)
    again = oracle.interpolate(s, kc, qc)
    np.testing.assert_allclose(again, g_kq, rtol=0, atol=1e-12)


def test_nested_equals_single_loop_brute_force():
    w = synth.si_toy()
    k, q = w.k[:2], w.q[:2]
    nested = oracle.interpolate(w.system, k, q)
    brute = oracle.interpolate_single_loop(w.system, k, q)
    np.testing.assert_allclose(nested, brute, rtol=0, atol=1e-12 * np.abs(brute).max())


# --------------------------------------------------------------------------
# a5 + a7: gauge-free band sums, Nw = 1, linearity
# --------------------------------------------------------------------------

def test_band_sum_is_rotation_free():
    w = synth.si_toy()
    a = oracle.interpolate(w.system, w.k[:5], w.q[:3], return_all=True)
    t_after = oracle.band_sums(a["ghat"])
    t_before = np.sum(np.abs(a["gw_nu"]) ** 2, axis=(-2, -1))
    np.testing.assert_allclose(t_after, t_before, rtol=1e-12)
    # unit masses: u(q) is unitary, so the sum over modes equals the raw Wannier norm
    np.testing.assert_allclose(t_after.sum(-1), np.sum(np.abs(a["gw"]) ** 2, axis=(-3, -2, -1)),
                               rtol=1e-12)


def test_single_band_only_phases():
    s = tiny_system(nw=1, na=2, seed=8)
    k, q = rand_pts(4, 5), rand_pts(3, 6)
    a = oracle.interpolate(s, k, q, return_all=True)
    np.testing.assert_allclose(np.abs(a["ghat"]), np.abs(a["gw_nu"]), rtol=1e-13)


def test_linearity_in_g():
    s = tiny_system(nw=3, na=1, seed=9)
    k, q = rand_pts(3, 7), rand_pts(2, 8)
    g1 = s.g.copy()
    gen = np.random.default_rng(4)
    g2 = gen.standard_normal(g1.shape) + 1j * gen.standard_normal(g1.shape)
    r1 = oracle.interpolate(s, k, q)
    s.g = g2
    r2 = oracle.interpolate(s, k, q)
    s.g = (0.3 - 1.1j) * g1 + 2.0 * g2
    r3 = oracle.interpolate(s, k, q)
    np.testing.assert_allclose(r3, (0.3 - 1.1j) * r1 + 2.0 * r2, atol=1e-12)


# --------------------------------------------------------------------------
# O7: gauge invariance of the block sums under unitary mixing of degenerate bands
# --------------------------------------------------------------------------

def test_block_sums_invariant_under_degenerate_mixing():
    # H(R) = h(R) (x) 1_2 gives exactly two-fold degenerate bands
    base = tiny_system(nw=2, na=1, seed=13)
    s = tiny_system(nw=4, na=1, seed=13)
    s.h_r = np.kron(base.h_r, np.eye(2)).reshape(len(base.h_r), 4, 4)
    k, q = rand_pts(3, 9), rand_pts(2, 10)
    a = oracle.interpolate(s, k, q, return_all=True)
    gen = np.random.default_rng(6)

    def mix(v):
        out = v.copy()
        for i in range(0, 4, 2):
            z = gen.standard_normal((2, 2)) + 1j * gen.standard_normal((2, 2))
            qm, _ = np.linalg.qr(z)
            out[..., :, i:i + 2] = out[..., :, i:i + 2] @ qm
        return out

    vk2 = np.stack([mix(v) for v in a["v_k"]])
    vkq2 = np.stack([[mix(v) for v in row] for row in a["v_kq"]])
    ghat2 = np.matmul(np.matmul(np.conj(np.swapaxes(vkq2, -1, -2))[:, :, None], a["gw_nu"]),
                      vk2[None, :, None])
    assert np.abs(ghat2 - a["ghat"]).max() > 1e-3       # the gauge really changed
    s1 = oracle.block_sums(np.abs(a["ghat"]) ** 2, a["eps_kq"], a["eps_k"], a["lam"])
    s2 = oracle.block_sums(np.abs(ghat2) ** 2, a["eps_kq"], a["eps_k"], a["lam"])
    assert oracle.compare_block_sums(s2, s1)[0] < 1e-13


def test_degenerate_blocks():
    assert oracle.degenerate_blocks(np.array([0.0, 1.0, 1.0 + 1e-9, 2.0])).tolist() == [0, 1, 3]
    assert oracle.degenerate_blocks(np.array([-5.0, -5.0, 3.0])).tolist() == [0, 2]


# --------------------------------------------------------------------------
# loss weights: the published SplitMix64 vectors
# --------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64.txt"))
            if l.strip() and not l.startswith("#")]
    for seed, idx, val in rows:
        w = oracle.splitmix64_weights(int(seed), np.array([int(idx)]))[0]
        assert w == 0.5 + (int(val) >> 40) * 2.0 ** -24
        assert np.float32(w) == w                     # exact in single precision
        assert 0.5 <= w < 1.5


def test_element_index_layout():
    idx = element_index(np.array([2]), np.array([3]), nk=5, nm=4, nw=3)
    assert idx.shape == (1, 4, 3, 3)
    assert int(idx[0, 1, 2, 0]) == ((((2 * 5 + 3) * 4 + 1) * 3 + 2) * 3 + 0)


# --------------------------------------------------------------------------
# Downstream reduction (linewidth): components against library routines and
# closed forms, the reduction through a sum rule and its invariances
# --------------------------------------------------------------------------

def test_linewidth_components():
    from scipy import integrate, special
    sigma = 0.037
    norm = integrate.quad(lambda x: oracle.gauss(x, sigma), -1, 1, points=[0.0])[0]
    var = integrate.quad(lambda x: x * x * oracle.gauss(x, sigma), -1, 1, points=[0.0])[0]
    assert abs(norm - 1.0) < 1e-12 and abs(var - sigma ** 2) < 1e-12
    e = np.linspace(-1.0, 1.0, 41)
    np.testing.assert_allclose(oracle.fermi(e, 0.2, 0.05), special.expit(-(e - 0.2) / 0.05), rtol=1e-14)
    t = 0.025
    assert abs(oracle.bose(t * np.log(2.0), t) - 1.0) < 1e-14                # e^{w/T} = 2
    w = np.linspace(0.01, 0.2, 9)
    np.testing.assert_allclose(oracle.bose(w, t) + 1.0, oracle.bose(w, t) * np.exp(w / t), rtol=1e-12)


def _linewidth_case(seed, nq=2, nk=3, nm=3, nw=4):
    gen = np.random.default_rng(seed)
    g = gen.standard_normal((nq, nk, nm, nw, nw)) + 1j * gen.standard_normal((nq, nk, nm, nw, nw))
    eps_k = np.sort(gen.uniform(-0.5, 0.5, (nk, nw)), axis=1)
    eps_kq = np.sort(gen.uniform(-0.5, 0.5, (nq, nk, nw)), axis=2)
    omega = gen.uniform(0.02, 0.08, (nq, nm))
    return g, eps_k, eps_kq, omega


def test_linewidth_sum_rule_over_the_initial_energy():
    """Integrating Gamma over the energy of the initial state turns both
    Gaussians into 1, so the occupations add to N + f + N + 1 - f = 2N + 1
    whatever the electron occupations are."""
    from scipy import integrate
    g, eps_k, eps_kq, omega = _linewidth_case(5, nk=1)
    temp, mu, sigma = 0.03, 0.1, 0.02

    def gamma_at(e):
        ek = eps_k.copy()
        ek[0, 0] = e
        return oracle.linewidth(g, ek, eps_kq, omega, temp, mu, sigma, 0.0, 7)[0, 0]

    peaks = np.sort(np.concatenate([(eps_kq[:, 0, :, None] + s * omega[:, None, :]).reshape(-1)
                                    for s in (-1.0, 1.0)]))
    total = integrate.quad(gamma_at, -2.0, 2.0, points=peaks, limit=400)[0]
    n_b = oracle.bose(omega, temp)                                      # [q][nu]
    expect = np.pi / 7 * np.sum(np.abs(g[:, 0, :, :, 0]) ** 2 * ((2.0 * n_b + 1.0) / (2.0 * omega))[:, :, None])
    assert abs(total - expect) < 1e-9 * abs(expect)


def test_linewidth_invariances():
    """Unchanged by a unitary mixing of exactly degenerate final states (m)
    or of modes of equal frequency; linear in |g|^2; additive over q; a mode
    below omega_min contributes nothing."""
    g, eps_k, eps_kq, omega = _linewidth_case(9)
    args = (0.03, 0.05, 0.04, 0.0, 11)
    base = oracle.linewidth(g, eps_k, eps_kq, omega, *args)
    # degenerate m block {1, 2} at every (q, k): rotate g's m index inside it
    ekq = eps_kq.copy()
    ekq[..., 2] = ekq[..., 1]
    ref = oracle.linewidth(g, eps_k, ekq, omega, *args)
    th = 0.7
    rot = np.array([[np.cos(th), np.sin(th) * np.exp(0.3j)], [-np.sin(th) * np.exp(-0.3j), np.cos(th)]])
    g2 = g.copy()
    g2[:, :, :, 1:3, :] = np.einsum("ab,qkvbn->qkvan", rot, g[:, :, :, 1:3, :])
    np.testing.assert_allclose(oracle.linewidth(g2, eps_k, ekq, omega, *args), ref, rtol=1e-12)
    # modes 0 and 1 of equal frequency: rotate g's nu index inside them
    om = omega.copy()
    om[:, 1] = om[:, 0]
    ref = oracle.linewidth(g, eps_k, eps_kq, om, *args)
    g3 = g.copy()
    g3[:, :, 0:2] = np.einsum("ab,qkbmn->qkamn", rot, g[:, :, 0:2])
    np.testing.assert_allclose(oracle.linewidth(g3, eps_k, eps_kq, om, *args), ref, rtol=1e-12)
    # linear in |g|^2, additive over q
    np.testing.assert_allclose(oracle.linewidth(2.0 * g, eps_k, eps_kq, omega, *args), 4.0 * base, rtol=1e-13)
    parts = sum(oracle.linewidth(g[i:i + 1], eps_k, eps_kq[i:i + 1], omega[i:i + 1], *args) for i in range(len(g)))
    np.testing.assert_allclose(parts, base, rtol=1e-13)
    # omega_min removes mode 2 entirely: same as zeroing its g
    cut = omega[:, 2].max() + 1e-3
    om2 = omega.copy()
    om2[:, 2] = 0.5 * cut
    om2[:, :2] = np.maximum(om2[:, :2], cut)
    g4 = g.copy()
    g4[:, :, 2] = 0.0
    np.testing.assert_allclose(oracle.linewidth(g, eps_k, eps_kq, om2, 0.03, 0.05, 0.04, cut, 11),
                               oracle.linewidth(g4, eps_k, eps_kq, om2, 0.03, 0.05, 0.04, cut, 11), rtol=1e-13)


def test_linewidth_zero_temperature_empty_final_states():
    """At T -> 0 with every final state empty (mu far below), no phonon can be
    absorbed and emission needs e_n = e_m + omega: Gamma vanishes for an
    initial state below every e_m + omega and is positive on a resonance."""
    g, eps_k, eps_kq, omega = _linewidth_case(13, nq=1, nk=1, nm=2, nw=3)
    temp, mu, sigma = 1e-4, -50.0, 0.002
    floor = float((eps_kq[0, 0, :, None] + omega[0][None, :]).min())
    ek = eps_k.copy()
    ek[0, 0] = floor - 20 * sigma
    ek[0, 1] = float(eps_kq[0, 0, 1] + omega[0, 0])                     # emission resonance
    ek[0, 2] = float(eps_kq[0, 0, 1] - omega[0, 0])                     # absorption resonance
    gam = oracle.linewidth(g, ek, eps_kq, omega, temp, mu, sigma, 0.0, 1)[0]
    assert gam[0] < 1e-30
    assert gam[1] > 1.0
    off = ek[0, 2] - (eps_kq[0, 0, :, None] + omega[0][None, :])       # distance to every emission resonance
    if np.abs(off).min() > 20 * sigma:
        assert gam[2] < 1e-30


def test_linewidth_zero_frequency_mode_is_dropped():
    """A mode with omega = 0 has no zero-point amplitude: it contributes
    nothing (rather than an infinite Bose factor) even with omega_min = 0."""
    g, eps_k, eps_kq, omega = _linewidth_case(17)
    om = omega.copy()
    om[:, 0] = 0.0
    g0 = g.copy()
    g0[:, :, 0] = 0.0
    a = oracle.linewidth(g, eps_k, eps_kq, om, 0.03, 0.05, 0.04, 0.0, 5)
    assert np.all(np.isfinite(a))
    np.testing.assert_allclose(a, oracle.linewidth(g0, eps_k, eps_kq, om, 0.03, 0.05, 0.04, 0.0, 5), rtol=1e-14)
