"""GPU adjoint of the weighted loss: against the oracle's reference gradients,
against central differences of the GPU forward, FP64 and FP32."""
import numpy as np
import pytest

import oracle
import synth
from oracle import adjoint

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    from gpu_run import Runner
    return Runner()


def grid_system(nw=5, na=2, m=(3, 2, 2), seed=3, g_dtype=np.complex128):
    s = synth.make_system(nw, na, synth.box((3, 3, 2)), synth.box((3, 2, 2)), [seed, 40], g_dtype=g_dtype,
                          mass=np.linspace(1.0, 2.0, na))
    pts = synth.uniform_grid(m)
    return s, pts, synth.grid_index_of_sum(m)


def gpu_backward(run, s, pts, kqi, prec, seed, q_batch=0, k_tile=0):
    import torch
    from paper_2603_10295_amd import ephw
    sysh = run.system(s)
    sysh.set_q_batch(q_batch)
    sysh.set_k_tile(k_tile)
    k = torch.from_numpy(pts).to("cuda:0")
    ks = ephw.KSet(sysh, k, prec)
    dt = torch.complex128 if prec == ephw.FP64 else torch.complex64
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    dg = torch.zeros(s.g.shape, dtype=dt, device="cuda:0")
    dk = torch.zeros((len(pts), 3), dtype=torch.float64, device="cuda:0")
    dq = torch.zeros((len(pts), 3), dtype=torch.float64, device="cuda:0")
    ephw.loss_backward(ks, k, torch.from_numpy(kqi).to("cuda:0"), loss_seed=seed, loss=loss, dL_dg=dg, dL_dk=dk,
                       dL_dq=dq)
    run.ctx.check()
    out = dict(loss=float(loss.cpu()[0]), dg=dg.cpu().numpy(), dk=dk.cpu().numpy(), dq=dq.cpu().numpy())
    ks.close()
    return out, sysh


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# (40, 6, 2, 3): the per-pair Vbar GEMMs (K = Nm Nw = 720) split K in two and
# the k row dot products split each row over column chunks
@pytest.mark.parametrize("nw,na,q_batch,k_tile", [(5, 2, 0, 0), (3, 1, 5, 7), (36, 1, 4, 5), (40, 6, 2, 3)])
def test_fp64_backward_matches_oracle(run, nw, na, q_batch, k_tile):
    s, pts, kqi = grid_system(nw=nw, na=na, seed=nw)
    got, _ = gpu_backward(run, s, pts, kqi, 0, seed=21, q_batch=q_batch, k_tile=k_tile)
    ref = adjoint.loss_and_grads(s, pts, pts, seed=21)
    assert abs(got["loss"] - ref["loss"]) < 1e-11 * ref["loss"]
    assert rel(got["dg"], ref["dg"]) < 1e-10
    assert rel(got["dk"], ref["dk"]) < 1e-8, (got["dk"][:3], ref["dk"][:3])
    assert rel(got["dq"], ref["dq"]) < 1e-8, (got["dq"][:3], ref["dq"][:3])


def test_fp64_backward_matches_finite_differences_of_the_gpu_forward(run):
    """dL/dk, dL/dq of the GPU adjoint vs central differences (Richardson) of the
    GPU forward, which evaluates H(k+q) directly at the moved points."""
    import torch
    from paper_2603_10295_amd import ephw
    s, pts, kqi = grid_system(nw=4, na=1, seed=12)
    got, sysh = gpu_backward(run, s, pts, kqi, 0, seed=5)

    def loss_at(k, q):
        ks = ephw.KSet(sysh, torch.from_numpy(k).to("cuda:0"), ephw.FP64)
        out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ephw.interpolate(ks, torch.from_numpy(q).to("cuda:0"), flags=ephw.OUT_LOSS, loss=out, loss_seed=5)
        run.ctx.check()
        v = float(out.cpu()[0])
        ks.close()
        return v

    assert abs(loss_at(pts, pts) - got["loss"]) < 1e-12 * got["loss"]
    h = 1e-5
    worst = 0.0
    for which, idx, d in [("k", 0, 0), ("k", 5, 1), ("k", 11, 2), ("q", 3, 0), ("q", 7, 1), ("q", 10, 2)]:
        def f(x):
            k, q = pts.copy(), pts.copy()
            (k if which == "k" else q)[idx, d] = x
            return loss_at(k, q)
        x0 = pts[idx, d]
        d1 = (f(x0 + h) - f(x0 - h)) / (2 * h)
        d2 = (f(x0 + h / 2) - f(x0 - h / 2)) / h
        fd = (4 * d2 - d1) / 3
        an = (got["dk"] if which == "k" else got["dq"])[idx, d]
        scale = max(np.abs(got["dk"]).max(), np.abs(got["dq"]).max())
        worst = max(worst, abs(fd - an) / scale)
    print(f"adjoint vs finite differences (FP64): max rel err {worst:.2e}")
    assert worst < 1e-6
    # g: exact directional derivative (the loss is quadratic in g)
    gen = np.random.default_rng(2)
    dgdir = gen.standard_normal(s.g.shape) + 1j * gen.standard_normal(s.g.shape)
    g0 = s.g.copy()
    t = 1e-3
    vals = []
    for sign in (1, -1):
        s.g = g0 + sign * t * dgdir
        sysh_t = run.system(s)
        ks = ephw.KSet(sysh_t, torch.from_numpy(pts).to("cuda:0"), ephw.FP64)
        out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ephw.interpolate(ks, torch.from_numpy(pts).to("cuda:0"), kq_index=torch.from_numpy(kqi).to("cuda:0"),
                         flags=ephw.OUT_LOSS, loss=out, loss_seed=5)
        run.ctx.check()
        vals.append(float(out.cpu()[0]))
        ks.close()
    s.g = g0
    fd = (vals[0] - vals[1]) / (2 * t)
    an = float(np.real(np.sum(np.conj(got["dg"]) * dgdir)))
    assert abs(fd - an) < 1e-9 * abs(an)


def test_fp32_backward_error_vs_fp64_oracle(run):
    s, pts, kqi = grid_system(nw=6, na=2, seed=17, g_dtype=np.complex64)
    got, _ = gpu_backward(run, s, pts, kqi, 1, seed=8)
    ref = adjoint.loss_and_grads(s, pts, pts, seed=8)
    e_l = abs(got["loss"] - ref["loss"]) / ref["loss"]
    e_g, e_k, e_q = rel(got["dg"], ref["dg"]), rel(got["dk"], ref["dk"]), rel(got["dq"], ref["dq"])
    print(f"FP32 adjoint vs FP64 oracle: loss {e_l:.2e} dL/dg {e_g:.2e} dL/dk {e_k:.2e} dL/dq {e_q:.2e}")
    assert e_l < 1e-5 and e_g < 1e-4 and e_k < 1e-4 and e_q < 1e-4


@pytest.mark.parametrize("prec,nw,na,k_tile", [(0, 36, 1, 5), (0, 40, 3, 0), (1, 33, 2, 7)])
def test_large_band_forward_matches_oracle(run, prec, nw, na, k_tile):
    """nw > 32: the band rotations run as batched GEMMs per (q batch, k tile)."""
    from paper_2603_10295_amd import ephw
    g_dtype = np.complex128 if prec == 0 else np.complex64
    s, pts, kqi = grid_system(nw=nw, na=na, seed=nw + na, g_dtype=g_dtype)
    sysh = run.system(s)
    sysh.set_k_tile(k_tile)
    out = run.interpolate(sysh, pts, pts, prec, kq_index=kqi, loss_seed=13, q_batch=5,
                          flags=ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS)
    ref = oracle.interpolate(s, pts, pts, return_all=True)
    tol = 1e-10 if prec == 0 else 1e-5
    sg = oracle.block_sums(np.abs(out["g"].astype(np.complex128)) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
    sr = oracle.block_sums(np.abs(ref["ghat"]) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
    assert oracle.compare_block_sums(sg, sr)[0] < tol
    assert rel(out["band_sum"], oracle.band_sums(ref["ghat"])) < tol
    nq, nk = len(pts), len(pts)
    iq, ik = np.divmod(np.arange(nq * nk), nk)
    l_ref = oracle.weighted_loss(ref["ghat"].reshape(nq * nk, *ref["ghat"].shape[2:]), 13, iq, ik, nk)
    assert abs(out["loss"] - l_ref) < tol * l_ref
    np.testing.assert_allclose(out["eps_kq"], ref["eps_kq"], atol=1e-12 * np.abs(ref["eps_kq"]).max())


def test_autograd_function_matches_oracle(run):
    import torch
    from paper_2603_10295_amd import ephw
    from paper_2603_10295_amd.autograd import eph_loss
    # quasi-1D ribbon-like slice: R along b only, k = q = i/8 on that axis, 36 bands
    w = synth.ribbon_1d(nw=36, na=2, nk=8, half=2, g_dtype=np.complex128)
    s = w.system
    sysh = run.system(s)
    g = torch.from_numpy(s.g).to("cuda:0").requires_grad_(True)
    k = torch.from_numpy(w.k).to("cuda:0").requires_grad_(True)
    q = torch.from_numpy(w.q).to("cuda:0").requires_grad_(True)
    kqi = torch.from_numpy(w.kq_index).to("cuda:0")
    L = eph_loss(sysh, g, k, q, kqi, seed=31)
    L.backward()
    ref = adjoint.loss_and_grads(s, w.k, w.q, seed=31)
    assert abs(float(L.detach().cpu()) - ref["loss"]) < 1e-11 * ref["loss"]
    assert rel(g.grad.cpu().numpy(), ref["dg"]) < 1e-10
    assert rel(k.grad.cpu().numpy(), ref["dk"]) < 1e-8
    assert rel(q.grad.cpu().numpy(), ref["dq"]) < 1e-8
    # only the ribbon axis carries a derivative
    assert np.abs(k.grad.cpu().numpy()[:, [0, 2]]).max() == 0.0
