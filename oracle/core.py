"""Plain FP64 evaluation of the interpolation, Eqs. (6), (7), (9), (10).

TEST INFRASTRUCTURE ONLY (see the package docstring). Nothing here is tuned:
every sum is written the way the paper states it, with NumPy matmul/einsum as
the only library steps and LAPACK eigh for the Hermitian eigenproblems.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


# ---------------------------------------------------------------------------
# Phase factors (the exponentials of Eq. (7))
# ---------------------------------------------------------------------------

def phases(points: np.ndarray, r: np.ndarray, w=None) -> np.ndarray:
    """exp(+2 pi i p.R) * w_R for every point p and lattice vector R, [Np][NR].

    Eq. (7) multiplies g(Re,Rp) by exp(i(q.Rp + k.Re)); with fractional
    points and integer vectors the argument is 2 pi p.R.  The product p.R is
    reduced to (-1/2, 1/2] before the exponential so the phase is accurate
    for large |R|.
    """
    t = np.asarray(points, dtype=np.float64) @ np.asarray(r, dtype=np.float64).T
    t = t - np.rint(t)
    ph = np.exp(1j * TWO_PI * t)
    if w is not None:
        ph = ph * np.asarray(w, dtype=np.float64)[None, :]
    return ph


# ---------------------------------------------------------------------------
# Electrons: H(k), eigenvalues and the gauge matrices (Eqs. (4)-(5))
# ---------------------------------------------------------------------------

def hamiltonian_k(system, k: np.ndarray) -> np.ndarray:
    """H(k) = sum_R w_R exp(2 pi i k.R) H(R), [Nk][Nw][Nw].  Not symmetrised."""
    ph = phases(k, system.r_h, system.w_h)
    return np.einsum("kr,rab->kab", ph, system.h_r.astype(np.complex128))


def bands(system, k: np.ndarray):
    """Eigenvalues (ascending) and eigenvector columns V(k) of H(k).

    In the gauge of Eq. (5), U(k) = V(k)^dagger.
    """
    h = hamiltonian_k(system, k)
    eps, v = np.linalg.eigh(h)
    return eps, v


# ---------------------------------------------------------------------------
# Phonons: D(q), frequencies and the mode vectors u of Eq. (2)
# ---------------------------------------------------------------------------

def _mode_mass(system) -> np.ndarray:
    return np.repeat(np.asarray(system.mass, dtype=np.float64), 3)


def dynamical_q(system, q: np.ndarray) -> np.ndarray:
    """D(q) = sum_R w_R exp(2 pi i q.R) C(R) / sqrt(M_kappa M_kappa'), [Nq][Nm][Nm]."""
    ph = phases(q, system.r_c, system.w_c)
    d = np.einsum("qr,rab->qab", ph, np.asarray(system.c_r, dtype=np.float64))
    m = _mode_mass(system)
    return d / np.sqrt(m[:, None] * m[None, :])[None]


def phonons(system, q: np.ndarray):
    """(lambda, omega, e): eigenvalues, sqrt(|lambda|), eigenvector columns of D(q)."""
    lam, e = np.linalg.eigh(dynamical_q(system, q))
    return lam, np.sqrt(np.abs(lam)), e


def mode_vectors(system, e: np.ndarray) -> np.ndarray:
    """u_{kappa alpha, nu}(q) = e_{kappa alpha, nu}(q) / sqrt(M_kappa)."""
    return e / np.sqrt(_mode_mass(system))[None, :, None]


# ---------------------------------------------------------------------------
# The nested loop, Eqs. (9) and (10)
# ---------------------------------------------------------------------------

def g_re_q(system, q: np.ndarray) -> np.ndarray:
    """Eq. (9): g(Re, q) = sum_Rp exp(i q.Rp) g(Re, Rp), [Nq][Ne][Nm][Nw][Nw]."""
    ph = phases(q, system.r_p, system.w_p)                      # [Nq][Np]
    g = system.g
    flat = g.reshape(g.shape[0], -1)
    out = np.zeros((len(q), flat.shape[1]), dtype=np.complex128)
    # a few Rp slabs of g at a time keep the complex128 upcast small
    step = max(1, int(2e7 // max(1, flat.shape[1])))
    for p0 in range(0, flat.shape[0], step):
        p1 = min(flat.shape[0], p0 + step)
        out += ph[:, p0:p1] @ flat[p0:p1].astype(np.complex128)
    return out.reshape((len(q),) + g.shape[1:])


def wannier_gauge_pairs(system, k: np.ndarray, g_req: np.ndarray) -> np.ndarray:
    """The Re sum of Eq. (10) before any rotation:
    gW[q][k][ka][m'][n'] = sum_Re exp(i k.Re) g(Re, q)."""
    ph = phases(k, system.r_e, system.w_e)                      # [Nk][Ne]
    nq = g_req.shape[0]
    flat = g_req.reshape(nq, g_req.shape[1], -1)                # [Nq][Ne][E]
    out = np.matmul(ph[None, :, :], flat)                       # [Nq][Nk][E]
    return out.reshape((nq, len(k)) + g_req.shape[2:])


def interpolate(system, k: np.ndarray, q: np.ndarray, return_all: bool = False):
    """Eq. (7) evaluated with the nested loop of Eqs. (9)-(10).

    Returns g_hat[q][k][nu][m][n] = sum_{m'n' ka} V(k+q)*_{m'm} gW_{ka m'n'}
    u_{ka nu}(q) V(k)_{n'n}, with k+q = k_i + q_j computed directly (no grid
    lookup) and its own eigensolve.
    """
    k = np.asarray(k, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nk, nq = len(k), len(q)
    eps_k, v_k = bands(system, k)
    lam, omega, e = phonons(system, q)
    u = mode_vectors(system, e)                                  # [Nq][Nm][Nm]
    kq = (q[:, None, :] + k[None, :, :]).reshape(-1, 3)
    eps_kq, v_kq = bands(system, kq)
    eps_kq = eps_kq.reshape(nq, nk, -1)
    v_kq = v_kq.reshape(nq, nk, system.nw, system.nw)
    g_req = g_re_q(system, q)                                    # Eq. (9)
    gw = wannier_gauge_pairs(system, k, g_req)                   # Re sum of Eq. (10)
    # phonon factor u_{ka,nu}(q) of Eq. (10) (no conjugate)
    gw_nu = np.einsum("qkamn,qav->qkvmn", gw, u)
    # electron factors U(k+q) g U(k)^dagger = V(k+q)^dagger g V(k)
    vkq_h = np.conj(np.swapaxes(v_kq, -1, -2))                   # [Nq][Nk][Nw][Nw]
    ghat = np.matmul(np.matmul(vkq_h[:, :, None], gw_nu), v_k[None, :, None])
    if not return_all:
        return ghat
    return dict(ghat=ghat, eps_k=eps_k, v_k=v_k, eps_kq=eps_kq, v_kq=v_kq,
                lam=lam, omega=omega, e=e, u=u, g_req=g_req, gw=gw, gw_nu=gw_nu)


def interpolate_single_loop(system, k: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Eq. (7) as written: for every (k, q) pair, one sum over all (Re, Rp)
    of g(Re,Rp) exp(i(q.Rp + k.Re)) followed by the three rotations.
    For tiny inputs only (cost Eq. (8))."""
    k = np.asarray(k, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nw, nm = system.nw, system.nm
    out = np.zeros((len(q), len(k), nm, nw, nw), dtype=np.complex128)
    g = system.g.astype(np.complex128)
    for iq in range(len(q)):
        ph_p = phases(q[iq:iq + 1], system.r_p, system.w_p)[0]
        _, _, e = phonons(system, q[iq:iq + 1])
        u = mode_vectors(system, e)[0]
        for ik in range(len(k)):
            ph_e = phases(k[ik:ik + 1], system.r_e, system.w_e)[0]
            _, v_k = bands(system, k[ik:ik + 1])
            _, v_kq = bands(system, (k[ik] + q[iq])[None, :])
            tot = np.einsum("p,e,peamn->amn", ph_p, ph_e, g)
            for nu in range(nm):
                x = np.einsum("amn,a->mn", tot, u[:, nu])
                out[iq, ik, nu] = v_kq[0].conj().T @ x @ v_k[0]
    return out


# ---------------------------------------------------------------------------
# Eq. (6): coarse Bloch -> Wannier transform (used for the round-trip pin)
# ---------------------------------------------------------------------------

def coarse_transform(g_kq: np.ndarray, k: np.ndarray, q: np.ndarray, v_k: np.ndarray,
                     v_kq: np.ndarray, u: np.ndarray, r_e: np.ndarray, r_p: np.ndarray) -> np.ndarray:
    """Eq. (6): g(Re,Rp) = 1/(Ne Np) sum_{k'q'} sum_{mn nu} g_{mn nu}(k',q')
    U*_{mm'}(k'+q') U_{nn'}(k') u^-1_{nu, ka}(q') exp(-i(q'.Rp + k'.Re)).

    With U = V^dagger:  sum_mn U*_{mm'} g_mn U_{nn'} = [V(k'+q') g V(k')^dagger]_{m'n'}.
    g_kq is [Nq'][Nk'][Nm][Nw][Nw]; returns [Np][Ne][Nm][Nw][Nw].
    """
    ne, npp = len(r_e), len(r_p)
    uinv = np.linalg.inv(u)                                          # [Nq][Nm(nu)][Nm(ka)]
    back = np.matmul(np.matmul(v_kq[:, :, None], g_kq),
                     np.conj(np.swapaxes(v_k, -1, -2))[None, :, None])  # [q][k][nu][m'][n']
    back = np.einsum("qkvmn,qva->qkamn", back, uinv)
    ph_e = np.conj(phases(k, r_e))                                   # [Nk][Ne]
    ph_p = np.conj(phases(q, r_p))                                   # [Nq][Np]
    out = np.einsum("qp,ke,qkamn->peamn", ph_p, ph_e, back)
    return out / (ne * npp)


# ---------------------------------------------------------------------------
# Gauge-invariant observables
# ---------------------------------------------------------------------------

def degenerate_blocks(vals: np.ndarray, rel_tol: float = 1e-6):
    """Start indices of blocks of (ascending) eigenvalues whose consecutive gaps
    are <= rel_tol * max(1, max|vals|).  Vectors within a block are only defined
    up to a unitary mixing, so observables must be summed over each block."""
    vals = np.asarray(vals)
    tol = rel_tol * max(1.0, float(np.max(np.abs(vals))) if vals.size else 1.0)
    starts = [0]
    for i in range(1, len(vals)):
        if vals[i] - vals[i - 1] > tol:
            starts.append(i)
    return np.array(starts, dtype=np.int64)


def block_sums(g2: np.ndarray, eps_kq: np.ndarray, eps_k: np.ndarray, lam: np.ndarray) -> list:
    """S[M,N,Nu] = sum over m in M, n in N, nu in Nu of |g_mn nu|^2 for every pair.

    g2 is |g_hat|^2 with shape [Nq][Nk][Nm][Nw][Nw]; the blocks come from the
    given eigenvalues (the caller passes the oracle's eigenvalues to both sides).
    Returns a list (one entry per pair, q-major) of 3-D arrays.
    """
    out = []
    nq, nk = g2.shape[:2]
    for iq in range(nq):
        bnu = degenerate_blocks(lam[iq])
        for ik in range(nk):
            bm = degenerate_blocks(eps_kq[iq, ik])
            bn = degenerate_blocks(eps_k[ik])
            s = np.add.reduceat(g2[iq, ik], bnu, axis=0)
            s = np.add.reduceat(s, bm, axis=1)
            s = np.add.reduceat(s, bn, axis=2)
            out.append(s)
    return out


def compare_block_sums(s_test: list, s_ref: list):
    """Normwise relative error ||S_test - S_ref|| / ||S_ref|| over all blocks, and
    the largest blockwise relative error over blocks with S_ref >= 1e-6 max S_ref."""
    a = np.concatenate([x.reshape(-1) for x in s_test])
    b = np.concatenate([x.reshape(-1) for x in s_ref])
    norm = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    big = b >= 1e-6 * b.max()
    blk = float(np.max(np.abs(a[big] - b[big]) / b[big]))
    return norm, blk


def band_sums(ghat: np.ndarray) -> np.ndarray:
    """T_nu = sum_mn |g_mn nu|^2 (gauge free), [Nq][Nk][Nm]."""
    return np.sum(np.abs(ghat) ** 2, axis=(-2, -1))


# ---------------------------------------------------------------------------
# Loss weights: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014)
# ---------------------------------------------------------------------------

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_weights(seed: int, index: np.ndarray) -> np.ndarray:
    """w = 0.5 + (x >> 40) * 2^-24 with x the index-th output of SplitMix64
    seeded with ``seed``: x = mix(seed + (index + 1) * gamma).

    ``index`` is the linear position ((((iq*Nk + ik)*Nm + nu)*Nw + m)*Nw + n)
    of the element in the whole (q, k) workload.  The values are exact in both
    single and double precision.
    """
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(index, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return 0.5 + (z >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def element_index(iq: np.ndarray, ik: np.ndarray, nk: int, nm: int, nw: int) -> np.ndarray:
    """Linear index of every (nu, m, n) element of the pairs (iq, ik): [len][Nm][Nw][Nw]."""
    iq = np.asarray(iq, dtype=np.uint64).reshape(-1, 1, 1, 1)
    ik = np.asarray(ik, dtype=np.uint64).reshape(-1, 1, 1, 1)
    nu = np.arange(nm, dtype=np.uint64).reshape(1, -1, 1, 1)
    m = np.arange(nw, dtype=np.uint64).reshape(1, 1, -1, 1)
    n = np.arange(nw, dtype=np.uint64).reshape(1, 1, 1, -1)
    nk_, nm_, nw_ = np.uint64(nk), np.uint64(nm), np.uint64(nw)
    return ((((iq * nk_ + ik) * nm_ + nu) * nw_ + m) * nw_ + n)


def weighted_loss(ghat: np.ndarray, seed: int, iq: np.ndarray, ik: np.ndarray, nk: int) -> float:
    """L = sum w_{mn nu}(k,q) |g_mn nu(k,q)|^2 over the given pairs.
    ghat is [Npairs][Nm][Nw][Nw] for the pairs (iq[i], ik[i])."""
    nm, nw = ghat.shape[1], ghat.shape[2]
    w = splitmix64_weights(seed, element_index(iq, ik, nk, nm, nw))
    return float(np.sum(w * np.abs(ghat) ** 2))


# ---------------------------------------------------------------------------
# Downstream reduction: phonon-limited electron linewidth (not printed in the
# paper, which runs an electron self-energy on the interpolated g; this is the
# textbook imaginary part of the Fan-Migdal self-energy with Gaussian
# broadening, the reading recorded in the design notes)
# ---------------------------------------------------------------------------

def bose(omega: np.ndarray, temp: float) -> np.ndarray:
    """Bose-Einstein occupation 1 / (exp(omega / T) - 1)."""
    return 1.0 / np.expm1(np.asarray(omega, dtype=np.float64) / temp)


def fermi(eps: np.ndarray, mu: float, temp: float) -> np.ndarray:
    """Fermi-Dirac occupation 1 / (exp(x) + 1), x = (eps - mu) / T, evaluated
    as exp(-x) / (1 + exp(-x)) for x > 0 so that it neither overflows nor
    loses its relative precision in the tail."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / temp
    e = np.exp(-np.abs(x))
    return np.where(x > 0, e / (1.0 + e), 1.0 / (1.0 + e))


def gauss(x: np.ndarray, sigma: float) -> np.ndarray:
    """Normalised Gaussian exp(-x^2 / (2 sigma^2)) / (sigma sqrt(2 pi))."""
    return np.exp(-0.5 * (np.asarray(x) / sigma) ** 2) / (sigma * np.sqrt(2.0 * np.pi))


def linewidth(ghat: np.ndarray, eps_k: np.ndarray, eps_kq: np.ndarray, omega: np.ndarray, temp: float,
              mu: float, sigma: float, omega_min: float, nq_total: int) -> np.ndarray:
    """Gamma[k][n] = (pi / Nq) sum over q, m and modes nu with omega >= omega_min
    and omega > 0 of
    |g_mn nu(k,q)|^2 / (2 omega) * [ (N + f_m) delta(e_n - e_m + omega)
                                  + (N + 1 - f_m) delta(e_n - e_m - omega) ],
    N = bose(omega), f_m = fermi(e_m(k+q)), e_n = eps_k[k][n]: phonon absorption
    and emission by the state n at k into the states m at k+q.  The 1/(2 omega)
    supplies the zero-point amplitude that the mode vectors u = e/sqrt(M) of
    Eq. (2) leave out.  ghat [Nq][Nk][Nm][Nw][Nw] (nu, m, n); returns [Nk][Nw]."""
    om = np.asarray(omega, dtype=np.float64)                          # [q][nu]
    keep = (om >= omega_min) & (om > 0.0)                             # omega = 0: no zero-point amplitude
    om_safe = np.where(keep, om, 1.0)
    n_b = np.where(keep, bose(om_safe, temp), 0.0)
    amp = np.where(keep, 1.0 / (2.0 * om_safe), 0.0)
    f_m = fermi(eps_kq, mu, temp)                                     # [q][k][m]
    g2 = np.abs(ghat) ** 2                                            # [q][k][nu][m][n]
    de = eps_k[None, :, None, :] - eps_kq[:, :, :, None]              # [q][k][m][n] = e_n - e_m
    absorb = (n_b[:, None, :, None, None] + f_m[:, :, None, :, None]) * \
        gauss(de[:, :, None, :, :] + om[:, None, :, None, None], sigma)
    emit = (n_b[:, None, :, None, None] + 1.0 - f_m[:, :, None, :, None]) * \
        gauss(de[:, :, None, :, :] - om[:, None, :, None, None], sigma)
    w = amp[:, None, :, None, None] * (absorb + emit)                 # [q][k][nu][m][n]
    return np.pi / nq_total * np.einsum("qkvmn,qkvmn->kn", g2, w)
