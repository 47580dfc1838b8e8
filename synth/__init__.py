"""Seeded synthetic inputs for the Wannier-to-Bloch e-ph interpolation.

This module only *draws data*: lattice-vector boxes, Wannier-space tensors
g(Re,Rp), H(R), C(R), masses and fine k/q lists with the shapes of the
paper's workloads (bulk Si, a 2D MoS2-like sheet, a quasi-1D nanoribbon).
It performs none of the interpolation arithmetic. Both the CPU oracle and
the GPU path consume what it returns, so they see identical inputs.

Random streams: every tensor draws from its own numpy PCG64 stream
``default_rng(SeedSequence([*base, stream]))`` with stream ids
1 = g(Re,Rp), 2 = H(R), 3 = C(R), 4 = k list, 5 = q list,
7 = per-system shapes of the multi-system batch.

Lattice boxes: an axis of n cells holds the integers
-floor(n/2) .. ceil(n/2)-1 (a complete residue system modulo n), listed in
lexicographic (x, y, z) order.

Tensor recipes (decay envelopes mimic maximally localised Wannier
functions, whose matrix elements fall off with |Re| and |Rp|):

* g[p, e, ka, m', n'] = (x + i y)/sqrt(2) * exp(-(|Re| + |Rp|)/2),
  x, y iid N(0, 1).
* H(R) = Z[R] for R >lex 0, Z[-R]^dagger for R <lex 0, (Z0 + Z0^dagger)/2
  at R = 0, zero where -R lies outside the box; Z complex normal times
  exp(-|R|). Hence H(-R) = H(R)^dagger.
* C(R): the same pairing with a real normal Z and transposes, so
  C(-R) = C(R)^T.  Masses are 1 unless a workload says otherwise.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

STREAM_G, STREAM_H, STREAM_C, STREAM_K, STREAM_Q, STREAM_SHAPE = 1, 2, 3, 4, 5, 7


def rng(base: Sequence[int], stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([*base, stream]))


def box(n: Sequence[int]) -> np.ndarray:
    """Integer lattice vectors of an n0 x n1 x n2 box, int32 [N][3]."""
    axes = [np.arange(-(ni // 2), -(ni // 2) + ni, dtype=np.int32) for ni in n]
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.reshape(-1) for a in grid], axis=1).astype(np.int32)


def axis_box(lo: int, hi: int, axis: int) -> np.ndarray:
    """Lattice vectors lo..hi along one axis (quasi-1D systems)."""
    r = np.zeros((hi - lo + 1, 3), dtype=np.int32)
    r[:, axis] = np.arange(lo, hi + 1, dtype=np.int32)
    return r


def uniform_grid(m: Sequence[int]) -> np.ndarray:
    """Fractional points (i/m0, j/m1, l/m2) in lexicographic order, f64 [N][3]."""
    axes = [np.arange(mi, dtype=np.float64) / mi for mi in m]
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.reshape(-1) for a in grid], axis=1)


def grid_index_of_sum(m: Sequence[int]) -> np.ndarray:
    """For a lexicographic grid of size m: idx[iq, ik] = grid index of k_ik + q_iq
    folded back into the grid (integer lookup table, int32 [Nq][Nk])."""
    m = [int(x) for x in m]
    n = m[0] * m[1] * m[2]
    flat = np.arange(n, dtype=np.int32)
    digits = [flat // (m[1] * m[2]), (flat // m[2]) % m[1], flat % m[2]]
    scale = [m[1] * m[2], m[2], 1]
    out = np.zeros((n, n), dtype=np.int32)
    for d in range(3):
        out += ((digits[d][:, None] + digits[d][None, :]) % m[d]) * np.int32(scale[d])
    return out


def _lex_sign(r: np.ndarray) -> np.ndarray:
    """+1 if the first nonzero component is positive, -1 if negative, 0 for R=0."""
    s = np.zeros(len(r), dtype=np.int64)
    for ax in range(3):
        undecided = s == 0
        s[undecided] = np.sign(r[undecided, ax])
    return s


def _partner_index(r: np.ndarray) -> np.ndarray:
    """Index of -R in the list, or -1 when -R is absent."""
    lut = {tuple(v): i for i, v in enumerate(r.tolist())}
    return np.array([lut.get(tuple((-v).tolist()), -1) for v in r], dtype=np.int64)


def _norms(r: np.ndarray) -> np.ndarray:
    return np.sqrt((r.astype(np.float64) ** 2).sum(axis=1))


def hermitian_paired(r: np.ndarray, n: int, gen: np.random.Generator, complex_: bool) -> np.ndarray:
    """Draw Z[R] * exp(-|R|) and pair it so that M(-R) = M(R)^dagger."""
    nr = len(r)
    if complex_:
        z = gen.standard_normal((nr, n, n, 2))
        z = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    else:
        z = gen.standard_normal((nr, n, n))
    z = z * np.exp(-_norms(r))[:, None, None]
    sgn = _lex_sign(r)
    partner = _partner_index(r)
    out = np.zeros_like(z)
    for i in range(nr):
        if partner[i] < 0:
            continue
        if sgn[i] > 0:
            out[i] = z[i]
        elif sgn[i] < 0:
            out[i] = z[partner[i]].conj().T
        else:
            out[i] = 0.5 * (z[i] + z[i].conj().T)
    return out


def decaying_g(r_e: np.ndarray, r_p: np.ndarray, nm: int, nw: int,
               gen: np.random.Generator, dtype) -> np.ndarray:
    """g[p, e, ka, m', n'] complex normal times exp(-(|Re|+|Rp|)/2)."""
    ne, npp = len(r_e), len(r_p)
    env = np.exp(-0.5 * (_norms(r_p)[:, None] + _norms(r_e)[None, :]))
    real_t = np.float32 if np.dtype(dtype) == np.complex64 else np.float64
    out = np.empty((npp, ne, nm, nw, nw), dtype=dtype)
    inv = real_t(1.0 / np.sqrt(2.0))
    # draw one Rp slab at a time to bound host memory on large systems
    for p in range(npp):
        x = gen.standard_normal((ne, nm, nw, nw, 2), dtype=real_t)
        # the trailing (re, im) pairs read as complex values in place
        slab = x.view(dtype)[..., 0] * inv
        out[p] = slab * env[p][:, None, None, None].astype(real_t)
    return out


@dataclasses.dataclass
class System:
    """Wannier-space description of one material (all host numpy arrays)."""
    nw: int
    na: int
    r_e: np.ndarray          # int32 [ne][3]  electron WS vectors
    r_p: np.ndarray          # int32 [np][3]  phonon WS vectors
    r_h: np.ndarray          # int32 [nh][3]  vectors of H(R)
    r_c: np.ndarray          # int32 [nc][3]  vectors of C(R)
    h_r: np.ndarray          # c128 [nh][nw][nw]
    c_r: np.ndarray          # f64  [nc][nm][nm]
    mass: np.ndarray         # f64  [na]
    g: np.ndarray            # [np][ne][nm][nw][nw] complex128 or complex64
    w_e: Optional[np.ndarray] = None   # f64 weights (None = all 1)
    w_p: Optional[np.ndarray] = None
    w_h: Optional[np.ndarray] = None
    w_c: Optional[np.ndarray] = None

    @property
    def nm(self) -> int:
        return 3 * self.na

    @property
    def ne(self) -> int:
        return len(self.r_e)

    @property
    def np_(self) -> int:
        return len(self.r_p)


@dataclasses.dataclass
class Workload:
    name: str
    system: System
    k: np.ndarray                      # f64 [nk][3] fractional
    q: np.ndarray                      # f64 [nq][3] fractional
    kq_index: Optional[np.ndarray]     # int32 [nq][nk] grid index of k+q, or None
    precision: str                     # "fp64" | "fp32"
    seed: int = 0
    loss_seed: int = 0


def make_system(nw: int, na: int, r_e: np.ndarray, r_p: np.ndarray, base: Sequence[int],
                g_dtype=np.complex128, mass: Optional[np.ndarray] = None, with_g: bool = True) -> System:
    """with_g False leaves g None (its stream is then not drawn): for systems
    whose g is generated on the device instead."""
    nm = 3 * na
    h_r = hermitian_paired(r_e, nw, rng(base, STREAM_H), complex_=True)
    c_r = hermitian_paired(r_p, nm, rng(base, STREAM_C), complex_=False)
    g = decaying_g(r_e, r_p, nm, nw, rng(base, STREAM_G), g_dtype) if with_g else None
    if mass is None:
        mass = np.ones(na, dtype=np.float64)
    return System(nw=nw, na=na, r_e=r_e, r_p=r_p, r_h=r_e.copy(), r_c=r_p.copy(),
                  h_r=h_r, c_r=c_r, mass=np.asarray(mass, dtype=np.float64), g=g)


def random_points(n: int, gen: np.random.Generator, axes=(0, 1, 2)) -> np.ndarray:
    pts = gen.random((n, 3))
    keep = np.zeros(3, dtype=bool)
    keep[list(axes)] = True
    pts[:, ~keep] = 0.0
    return pts


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the paper's systems: bulk Si (Nb=8, Nm=6),
# a MoS2-like monolayer (2D grids), stanene nanoribbons (quasi-1D, large Nb/Nm).
# ---------------------------------------------------------------------------

def si_toy(seed: int = 0, nk: int = 16, nq: int = 16) -> Workload:
    """Si-like toy, FP64: Nw=8, Na=2, 5x5x5 boxes, 16 random k x 16 random q."""
    base = [seed]
    r = box((5, 5, 5))
    sys_ = make_system(8, 2, r, r, base)
    k = random_points(nk, rng(base, STREAM_K))
    q = random_points(nq, rng(base, STREAM_Q))
    return Workload("si_toy_nw8_nm6_r5x5x5_16kx16q_fp64", sys_, k, q, None, "fp64", seed)


def mos2_2d(seed: int = 0, nk: int = 1000, nq: int = 1000) -> Workload:
    """MoS2-like 2D, FP64: Nw=11, Na=3, 18x18 in-plane boxes, 1000 k x 1000 q."""
    base = [seed]
    r = box((18, 18, 1))
    sys_ = make_system(11, 3, r, r, base)
    k = random_points(nk, rng(base, STREAM_K), axes=(0, 1))
    q = random_points(nq, rng(base, STREAM_Q), axes=(0, 1))
    return Workload("mos2_2d_nw11_nm9_r18x18_1000kx1000q_fp64", sys_, k, q, None, "fp64", seed)


def si_dense(seed: int = 0, m: int = 20, g_dtype=np.complex64) -> Workload:
    """Si-like dense precision workload: Nw=8, Na=2, 10x10x10 boxes (Ne=Np=1000),
    k = q = m^3 uniform grid (8000 at m=20); g stored complex64."""
    base = [seed]
    r = box((10, 10, 10))
    sys_ = make_system(8, 2, r, r, base, g_dtype=g_dtype)
    pts = uniform_grid((m, m, m))
    return Workload(f"si_dense_nw8_nm6_r10x10x10_grid{m}^3_c64", sys_, pts, pts.copy(),
                    grid_index_of_sum((m, m, m)), "fp32", seed)


G_CAP_BYTES = 2 * 2 ** 30


def batch_shape(seed: int, s: int, max_grid: int = 16, g_cap_bytes: Optional[int] = G_CAP_BYTES):
    """Shape of system s of the multi-system batch: Nw in [4,32], Na in [1,8],
    a 3D box with n_i in [4,10] and Ne=Np<=800, grid m in [4, max_grid].
    Draws whose complex64 g would exceed g_cap_bytes are redrawn from the same
    ranges (None: no cap; the unrestricted 32-system batch holds about 207 GB
    of g)."""
    gen = rng([seed, STREAM_SHAPE, s], 0)
    while True:
        nw = int(gen.integers(4, 33))
        na = int(gen.integers(1, 9))
        while True:
            n = [int(x) for x in gen.integers(4, 11, size=3)]
            if n[0] * n[1] * n[2] <= 800:
                break
        m = int(gen.integers(4, max_grid + 1))
        ne = n[0] * n[1] * n[2]
        if g_cap_bytes is None or 8 * ne * ne * 3 * na * nw * nw <= g_cap_bytes:
            return nw, na, n, m


def batch_system(seed: int, s: int, max_grid: int = 16, g_cap_bytes: Optional[int] = G_CAP_BYTES,
                 with_g: bool = True) -> Workload:
    """System s of the multi-system batch (see batch_shape); complex64 g, k = q =
    the m^3 grid of the system."""
    base = [seed, STREAM_SHAPE, s]
    nw, na, n, m = batch_shape(seed, s, max_grid, g_cap_bytes)
    r = box(n)
    sys_ = make_system(nw, na, r, r, base, g_dtype=np.complex64, with_g=with_g)
    pts = uniform_grid((m, m, m))
    return Workload(f"batch{s}_nw{nw}_nm{3*na}_r{n[0]}x{n[1]}x{n[2]}_grid{m}^3",
                    sys_, pts, pts.copy(), grid_index_of_sum((m, m, m)), "fp32", seed)


def batch_systems(seed: int = 0, count: int = 32, max_grid: int = 16,
                  g_cap_bytes: int = G_CAP_BYTES) -> list:
    """The whole heterogeneous batch (list of Workloads)."""
    return [batch_system(seed, s, max_grid, g_cap_bytes) for s in range(count)]


def ribbon_1d(seed: int = 0, nw: int = 200, na: int = 50, nk: int = 256, half: int = 5,
              g_dtype=np.complex64) -> Workload:
    """Stanene-nanoribbon-like quasi-1D system: Nw=200, Nm=150, R = -5..5 along the
    ribbon (b) axis, k = q = i/256 along that axis, complex64 g."""
    base = [seed]
    r = axis_box(-half, half, axis=1)
    sys_ = make_system(nw, na, r, r, base, g_dtype=g_dtype)
    pts = np.zeros((nk, 3))
    pts[:, 1] = np.arange(nk) / nk
    kq = ((np.arange(nk)[None, :] + np.arange(nk)[:, None]) % nk).astype(np.int32)
    return Workload(f"ribbon_1d_nw{nw}_nm{3*na}_r1d{2*half+1}_{nk}kx{nk}q_c64", sys_, pts,
                    pts.copy(), kq, "fp32", seed)


WORKLOADS = {
    "si_toy": si_toy,
    "mos2_2d": mos2_2d,
    "si_dense": si_dense,
    "ribbon_1d": ribbon_1d,
}
