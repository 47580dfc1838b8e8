"""Write the oracle's expected values for the ribbon-shaped GPU parity tests.

    python tests/golden/make_ribbon_c4.py

The system has the band and mode counts of the stanene-nanoribbon workload
(Nw = 200 Wannier functions, Nm = 150 modes, the sizes Table 3 of the paper
lists for its wider ribbons) on a short 1D lattice (R = -1..1 along the
ribbon axis) and 4 k x 4 q points k = q = i/4 on that axis, so every band
product the GPU runs has the full 200 x 200 shape while the oracle still
finishes on a CPU.  Both outputs come from `oracle/` only (NumPy complex128
and LAPACK eigh); the inputs come from the seeded generators in `synth/`.

Stored (ribbon_c4_nw200_nm150.npz):
  fp32_*  complex64 g (the FP32 path's input, upcast by the oracle):
          eigenvalues, the loss with seed LOSS_SEED, band sums T[q][k][nu],
          and the eigenvector-dependent reductions R[q][k][n] = sum_{nu,m}
          |g_mn nu|^2 (depends on V(k)) and C[q][k][m] = sum_{nu,n} |g_mn nu|^2
          (depends on V(k+q)), each summed over degenerate blocks of its band
          index so that it is gauge invariant;
  fp64_*  complex128 g: the loss and its gradients with respect to g(Re,Rp)
          (sampled at SAMPLES seeded positions, with its largest magnitude and
          per-(Rp, Re) slab norms), k and q, from the oracle's adjoint.
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import adjoint  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ribbon_c4_nw200_nm150.npz")
SHAPE = dict(nw=200, na=50, nk=4, half=1)
LOSS_SEED = 41
SAMPLES = 4096


def workload(g_dtype):
    return synth.ribbon_1d(g_dtype=g_dtype, **SHAPE)


def block_reduce(x: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """Sum the last axis of x over the degenerate blocks of vals (same leading shape)."""
    out = np.zeros_like(x)
    for idx in np.ndindex(x.shape[:-1]):
        starts = oracle.degenerate_blocks(vals[idx])
        s = np.add.reduceat(x[idx], starts)
        ends = list(starts[1:]) + [x.shape[-1]]
        for b, (a, e) in enumerate(zip(starts, ends)):
            out[idx][a:e] = s[b]
    return out


def reductions(ghat: np.ndarray, eps_k: np.ndarray, eps_kq: np.ndarray):
    """(T, R, C) of the module docstring from g_hat [q][k][nu][m][n]."""
    g2 = np.abs(ghat) ** 2
    t = g2.sum(axis=(3, 4))
    r = g2.sum(axis=(2, 3))
    c = g2.sum(axis=(2, 4))
    nq = ghat.shape[0]
    r = block_reduce(r, np.broadcast_to(eps_k[None], (nq,) + eps_k.shape))
    c = block_reduce(c, eps_kq)
    return t, r, c


def sample_positions(size: int) -> np.ndarray:
    gen = np.random.default_rng([LOSS_SEED, 99])
    return np.sort(gen.choice(size, SAMPLES, replace=False))


def main():
    out = {}
    w = workload(np.complex64)
    s = w.system
    f = oracle.interpolate(s, w.k, w.q, return_all=True)
    nq, nk = len(w.q), len(w.k)
    iq, ik = np.divmod(np.arange(nq * nk), nk)
    out["fp32_loss"] = oracle.weighted_loss(f["ghat"].reshape(nq * nk, *f["ghat"].shape[2:]), LOSS_SEED, iq, ik, nk)
    out["fp32_T"], out["fp32_R"], out["fp32_C"] = reductions(f["ghat"], f["eps_k"], f["eps_kq"])
    out["eps_k"], out["eps_kq"], out["lam"] = f["eps_k"], f["eps_kq"], f["lam"]
    del f, w, s
    print("fp32 forward done", flush=True)

    w = workload(np.complex128)
    r = adjoint.loss_and_grads(w.system, w.k, w.q, seed=LOSS_SEED)
    dg = r["dg"]
    pos = sample_positions(dg.size)
    out["fp64_loss"] = r["loss"]
    out["fp64_dk"] = r["dk"]
    out["fp64_dq"] = r["dq"]
    out["fp64_dg_pos"] = pos
    out["fp64_dg_val"] = dg.reshape(-1)[pos]
    out["fp64_dg_max"] = np.abs(dg).max()
    out["fp64_dg_slab_norm"] = np.linalg.norm(dg.reshape(dg.shape[0], dg.shape[1], -1), axis=2)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
