"""GPU parity at the band and mode counts of the stanene-nanoribbon workload
(Nw = 200, Nm = 150; Table 3 of the paper lists ribbons of that size) on a
short 1D lattice and 4 k x 4 q points, so that every band product runs at its
full 200 x 200 shape: the pair-stacked rotation GEMMs (Nm*Nw = 30000 rows,
N = K = 200), the n = 200 and n = 150 eigensolves, and in the adjoint the
eigenvector-gradient GEMMs that contract K = Nm*Nw = 30000 over a pair.

The expected values were written by tests/golden/make_ribbon_c4.py, which
calls only the oracle (its oracle run takes minutes on a CPU)."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ribbon_c4_nw200_nm150.npz")
SHAPE = dict(nw=200, na=50, nk=4, half=1)
LOSS_SEED = 41


@pytest.fixture(scope="module")
def run():
    from gpu_run import Runner
    return Runner()


@pytest.fixture(scope="module")
def golden():
    with np.load(GOLDEN) as z:
        return {k: z[k] for k in z.files}


def block_reduce(x, vals):
    """sum the last axis of x over the degenerate blocks of vals (oracle's blocks)"""
    import oracle
    out = np.zeros_like(x)
    for idx in np.ndindex(x.shape[:-1]):
        starts = oracle.degenerate_blocks(vals[idx])
        s = np.add.reduceat(x[idx], starts)
        ends = list(starts[1:]) + [x.shape[-1]]
        for b, (a, e) in enumerate(zip(starts, ends)):
            out[idx][a:e] = s[b]
    return out


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_ribbon_shape_fp32_forward(run, golden):
    import torch
    from paper_2603_10295_amd import ephw
    w = synth.ribbon_1d(g_dtype=np.complex64, **SHAPE)
    s = w.system
    sysh = run.system(s)
    out = run.interpolate(sysh, w.k, w.q, ephw.FP32, kq_index=w.kq_index, loss_seed=LOSS_SEED,
                          flags=ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS)
    h_norm = np.abs(golden["eps_k"]).max()
    assert np.abs(out["eps_k"] - golden["eps_k"]).max() < 1e-12 * h_norm        # n = 200 Jacobi vs LAPACK
    assert np.abs(out["eps_kq"] - golden["eps_kq"]).max() < 1e-12 * h_norm
    lam, _, _ = run.phonons(sysh, w.q)                                            # n = 150
    assert np.abs(lam - golden["lam"]).max() < 1e-12 * np.abs(golden["lam"]).max()
    g2 = np.abs(out["g"].astype(np.complex128)) ** 2
    nq = g2.shape[0]
    t = g2.sum(axis=(3, 4))
    r = block_reduce(g2.sum(axis=(2, 3)), np.broadcast_to(golden["eps_k"][None], (nq,) + golden["eps_k"].shape))
    c = block_reduce(g2.sum(axis=(2, 4)), golden["eps_kq"])
    errs = dict(T=relnorm(t, golden["fp32_T"]), R=relnorm(r, golden["fp32_R"]), C=relnorm(c, golden["fp32_C"]),
                band_sum=relnorm(out["band_sum"], golden["fp32_T"]),
                loss=abs(out["loss"] - float(golden["fp32_loss"])) / float(golden["fp32_loss"]))
    print("ribbon-shape FP32 forward vs oracle:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < 1e-5, (k, v)
    sysh.close()


def test_ribbon_shape_fp64_backward(run, golden):
    import torch
    from paper_2603_10295_amd import ephw
    w = synth.ribbon_1d(g_dtype=np.complex128, **SHAPE)
    s = w.system
    sysh = run.system(s)
    k = torch.from_numpy(w.k).to("cuda:0")
    q = torch.from_numpy(w.q).to("cuda:0")
    kqi = torch.from_numpy(w.kq_index).to("cuda:0")
    ks = ephw.KSet(sysh, k, ephw.FP64)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    dg = torch.zeros(s.g.shape, dtype=torch.complex128, device="cuda:0")
    dk = torch.zeros((len(w.k), 3), dtype=torch.float64, device="cuda:0")
    dq = torch.zeros((len(w.q), 3), dtype=torch.float64, device="cuda:0")
    ephw.loss_backward(ks, q, kqi, loss_seed=LOSS_SEED, loss=loss, dL_dg=dg, dL_dk=dk, dL_dq=dq)
    run.ctx.check()
    got_loss = float(loss.cpu()[0])
    dgh = dg.cpu().numpy()
    dkh, dqh = dk.cpu().numpy(), dq.cpu().numpy()
    ref_loss = float(golden["fp64_loss"])
    e_l = abs(got_loss - ref_loss) / ref_loss
    dg_max = float(golden["fp64_dg_max"])
    e_g = float(np.abs(dgh.reshape(-1)[golden["fp64_dg_pos"]] - golden["fp64_dg_val"]).max() / dg_max)
    slab = np.linalg.norm(dgh.reshape(dgh.shape[0], dgh.shape[1], -1), axis=2)
    e_s = float(np.abs(slab - golden["fp64_dg_slab_norm"]).max() / golden["fp64_dg_slab_norm"].max())
    scale = max(np.abs(golden["fp64_dk"]).max(), np.abs(golden["fp64_dq"]).max())
    e_k = float(np.abs(dkh - golden["fp64_dk"]).max() / scale)
    e_q = float(np.abs(dqh - golden["fp64_dq"]).max() / scale)
    print(f"ribbon-shape FP64 adjoint vs oracle: loss {e_l:.2e} dL/dg {e_g:.2e} (slabs {e_s:.2e}) "
          f"dL/dk {e_k:.2e} dL/dq {e_q:.2e}")
    assert e_l < 1e-11
    assert e_g < 1e-10 and e_s < 1e-10
    assert e_k < 1e-8 and e_q < 1e-8

    # Central differences (Richardson) of the GPU forward along the ribbon
    # axis.  Above 32 bands the forward takes V(k+q) from a k grid, so the
    # moved point k_i + h (or q_j + h) is evaluated with a k-set holding the
    # grid and the grid shifted by h: every k + q of the moved configuration
    # is then a point of the set.  The loss of the moved configuration is
    # summed from the stored g with the loss weights of the unmoved one.
    import oracle
    from oracle import core
    nk = len(w.k)
    k8 = np.concatenate([w.k, w.k])
    iq, ik = np.divmod(np.arange(nk * nk), nk)
    wts = oracle.splitmix64_weights(LOSS_SEED, core.element_index(iq, ik, nk, s.nm, s.nw))

    def loss_moved(which, idx, x):
        kk = k8.copy()
        kk[nk:, 1] += x                                       # the shifted copy of the grid
        qq = w.q.copy()
        kqi8 = np.zeros((nk, 2 * nk), dtype=np.int32)
        for j in range(nk):
            for a in range(2 * nk):
                kqi8[j, a] = (a % nk + j) % nk + (nk if a >= nk else 0)
        sel = np.arange(nk)                                   # set position of each k_i
        if which == "k":
            sel[idx] = nk + idx
        else:
            qq[idx, 1] += x
            kqi8[idx, :nk] += nk                              # k_a + q_idx + x = shifted grid point
        ks2 = ephw.KSet(sysh, torch.from_numpy(kk).to("cuda:0"), ephw.FP64)
        g = torch.empty((nk, 2 * nk, s.nm, s.nw, s.nw), dtype=torch.complex128, device="cuda:0")
        ephw.interpolate(ks2, torch.from_numpy(qq).to("cuda:0"), kq_index=torch.from_numpy(kqi8).to("cuda:0"),
                         flags=ephw.OUT_G, g_out=g)
        run.ctx.check()
        gh = g[:, torch.from_numpy(sel).to("cuda:0")].cpu().numpy()       # [q][k_i]
        ks2.close()
        return float(np.sum(wts * np.abs(gh.reshape(wts.shape)) ** 2))

    assert abs(loss_moved("k", 0, 0.0) - got_loss) < 1e-11 * got_loss
    h = 1e-5
    worst = 0.0
    for which, idx in [("k", 1), ("k", 3), ("q", 0), ("q", 2)]:
        d1 = (loss_moved(which, idx, h) - loss_moved(which, idx, -h)) / (2 * h)
        d2 = (loss_moved(which, idx, h / 2) - loss_moved(which, idx, -h / 2)) / h
        fd = (4 * d2 - d1) / 3
        an = (dkh if which == "k" else dqh)[idx, 1]
        worst = max(worst, abs(fd - an) / scale)
    print(f"ribbon-shape FP64 adjoint vs finite differences of the GPU forward: {worst:.2e}")
    assert worst < 1e-6
    ks.close()
    sysh.close()
