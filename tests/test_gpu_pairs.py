"""GPU parity of the pair-list path of the energy-window pre-screening.

ephw_window_pairs must list exactly the pairs the oracle's eigenvalues keep
(integer output, compared exactly, window edges placed in gaps of the
spectrum so rounding cannot move a state across them);
ephw_interpolate_pairs must give, on every kept pair, the g of
ephw_interpolate at the same (k, q) (same k-set, same V) and the oracle's g
in degenerate-block sums; its loss equals the oracle's weighted loss over the
kept pairs with the full-grid element indices.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL_W = 1e-12      # FP64: same V on both sides, sums of a few hundred terms
RTOL_S = 1e-10      # FP64 block sums against the oracle
RTOL_32 = 1e-5      # FP32


@pytest.fixture(scope="module")
def run():
    from gpu_run import Runner
    return Runner()


def gap_edge(vals, target):
    """A value between the two sorted neighbours of target in vals (a gap)."""
    v = np.unique(vals)
    i = int(np.searchsorted(v, target))
    i = min(max(i, 1), len(v) - 1)
    return 0.5 * (v[i - 1] + v[i])


def window_case(prec, seed=71, m=(4, 4, 2), frac=0.4, nw=6):
    s = synth.make_system(nw, 2, synth.box((3, 3, 2)), synth.box((2, 2, 2)), [seed, 2])
    if prec != 0:
        s = dataclasses.replace(s, g=s.g.astype(np.complex64))
    kg = synth.uniform_grid(m)
    kqi = synth.grid_index_of_sum(m)
    eps, _ = oracle.bands(s, kg)
    lo = float(eps.min()) - 1.0
    hi = gap_edge(eps, np.quantile(eps[:, 0], frac))
    kact = np.any((eps >= lo) & (eps <= hi), axis=1)
    keep = kact[None, :] & kact[kqi]          # [q][k]
    return s, kg, kg.copy(), kqi, lo, hi, keep


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
def test_window_pairs_match_the_oracle_window(run, prec, order):
    """Both groupings (by q: each q's k ascending; by k: each k's q ascending)."""
    from paper_2603_10295_amd import ephw
    from gpu_run import dev
    s, kg, qg, kqi, lo, hi, keep = window_case(prec)
    assert 0 < keep.sum() < keep.size and not keep.all(axis=1).any() and (~keep).all(axis=1).any()
    ks = ephw.KSet(run.system(s), dev(kg), prec)
    used, start, other, pkq, _ = ephw.window_pairs(ks, dev(kqi), lo, hi, order=order)
    run.ctx.check()
    ks.close()
    assert used == order
    if order == ephw.PAIRS_BY_Q:
        want_start = np.concatenate([[0], np.cumsum(keep.sum(axis=1))])
        iq, ik = np.nonzero(keep)             # q-major, ascending k within each q
        want_other = ik
    else:
        want_start = np.concatenate([[0], np.cumsum(keep.sum(axis=0))])
        ik, iq = np.nonzero(keep.T)           # k-major, ascending q within each k
        want_other = iq
    np.testing.assert_array_equal(start, want_start)
    np.testing.assert_array_equal(other.cpu().numpy()[:len(ik)], want_other)
    np.testing.assert_array_equal(pkq.cpu().numpy()[:len(ik)], kqi[iq, ik])


def test_window_pairs_auto_picks_the_smaller_grouping(run):
    """A window that keeps few k (every q keeps some pair) is listed by k, and
    with a k+q table that sends every k to one kept point the list is by q
    when fewer q than k own pairs."""
    from paper_2603_10295_amd import ephw
    from gpu_run import dev
    s, kg, qg, kqi, lo, hi, keep = window_case(0, frac=0.1)
    ks = ephw.KSet(run.system(s), dev(kg), 0)
    ak, aq = int(keep.any(axis=0).sum()), int(keep.any(axis=1).sum())
    used, start, _, _, _ = ephw.window_pairs(ks, dev(kqi), lo, hi)
    assert used == (ephw.PAIRS_BY_K if ak < aq else ephw.PAIRS_BY_Q), (ak, aq)
    assert int(start[-1]) == int(keep.sum())
    # k+q of q row j is always k point j: q row j keeps pairs only when k_j is
    # active, so as many q as active k own pairs, each with every active k
    eps = oracle.bands(s, kg)[0]
    kact = np.any((eps >= lo) & (eps <= hi), axis=1)
    tab = np.repeat(np.arange(len(kg), dtype=np.int32)[:, None], len(kg), axis=1)
    tab_keep = kact[None, :] & kact[tab]
    used2, start2, _, _, _ = ephw.window_pairs(ks, dev(tab), lo, hi)
    ak2, aq2 = int(tab_keep.any(axis=0).sum()), int(tab_keep.any(axis=1).sum())
    assert used2 == (ephw.PAIRS_BY_K if ak2 < aq2 else ephw.PAIRS_BY_Q), (ak2, aq2)
    assert int(start2[-1]) == int(tab_keep.sum())
    run.ctx.check()
    ks.close()


@pytest.mark.parametrize("prec,order,nw", [(0, 0, 6), (0, 1, 6), (1, 0, 6), (1, 1, 6), (1, 0, 12), (0, 1, 20)])
def test_interpolate_pairs_matches_full_path_and_oracle(run, prec, order, nw):
    """Both nesting orders: by q (Eq. (9) first, the Re sum per q on its kept
    k) and by k (the Re sum first, the Rp sum per k on its kept q, mode
    vectors per pair); Nw = 12 and 20 run the pair rotations on the matrix
    cores."""
    import torch
    from paper_2603_10295_amd import ephw
    from gpu_run import dev, cplx_dtype
    s, kg, qg, kqi, lo, hi, keep = window_case(prec, nw=nw)
    nk, nq = len(kg), len(qg)
    sysh = run.system(s)
    ks = ephw.KSet(sysh, dev(kg), prec)
    used, start, other, pkq, _ = ephw.window_pairs(ks, dev(kqi), lo, hi, order=order)
    npairs = int(start[-1])
    q_off, seed = 5, 23
    g = torch.empty((npairs, s.nm, s.nw, s.nw), dtype=cplx_dtype(prec), device="cuda:0")
    t = torch.empty((npairs, s.nm), dtype=torch.float64, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ephw.interpolate_pairs(ks, dev(qg), used, start, other, pkq, q_offset=q_off,
                           flags=ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS, g_out=g, band_sum=t, loss=loss,
                           loss_seed=seed)
    # the full path on every pair of the same k-set
    gf = torch.empty((nq, nk, s.nm, s.nw, s.nw), dtype=cplx_dtype(prec), device="cuda:0")
    ephw.interpolate(ks, dev(qg), kq_index=dev(kqi), q_offset=q_off, flags=ephw.OUT_G, g_out=gf)
    run.ctx.check()
    ks.close()
    if order == ephw.PAIRS_BY_Q:
        iq, ik = np.nonzero(keep)
    else:
        ik, iq = np.nonzero(keep.T)
    gp = g.cpu().numpy().astype(np.complex128)
    full = gf.cpu().numpy().astype(np.complex128)[iq, ik]
    err_full = float(np.abs(gp - full).max() / np.abs(full).max())
    # against the oracle (its own k+q eigensolves: block sums)
    ref = oracle.interpolate(s, kg, qg, return_all=True)
    s_gpu = []
    s_ref = []
    for p_, (a, b) in enumerate(zip(iq, ik)):
        s_gpu += oracle.block_sums(np.abs(gp[p_])[None, None] ** 2, ref["eps_kq"][a, b][None, None],
                                   ref["eps_k"][b][None], ref["lam"][a][None])
        s_ref += oracle.block_sums(np.abs(ref["ghat"][a, b])[None, None] ** 2, ref["eps_kq"][a, b][None, None],
                                   ref["eps_k"][b][None], ref["lam"][a][None])
    norm, _ = oracle.compare_block_sums(s_gpu, s_ref)
    t_ref = oracle.band_sums(ref["ghat"])[iq, ik]
    t_err = float(np.abs(t.cpu().numpy() - t_ref).max() / np.abs(t_ref).max())
    l_ref = oracle.weighted_loss(ref["ghat"][iq, ik], seed, iq + q_off, ik, nk)
    l_err = abs(float(loss.cpu().numpy()[0]) - l_ref) / l_ref
    print(f"pairs prec={prec} order={order}: {npairs} of {nq * nk}; vs full path {err_full:.2e}, "
          f"block sums {norm:.2e}, band sums {t_err:.2e}, loss {l_err:.2e}")
    # by q runs the full path's arithmetic; by k sums in the other order
    tol_full = (RTOL_W if prec == 0 else RTOL_32) if order == 1 else (RTOL_W if prec == 0 else 1e-6)
    tol = RTOL_S if prec == 0 else RTOL_32
    assert err_full < tol_full and norm < tol and t_err < tol and l_err < tol


@pytest.mark.parametrize("order", [0, 1])
def test_interpolate_pairs_edge_cases(run, order):
    """Empty window (no pair: nothing enqueued, outputs untouched), a window
    holding every pair (equal to the full path) in small chunks, the Wannier
    gauge, groups without pairs between groups with pairs, and invalid CSR
    offsets refused on the host."""
    import torch
    from paper_2603_10295_amd import ephw
    from gpu_run import dev
    s, kg, qg, kqi, lo, hi, keep = window_case(0, seed=72)
    nk, nq = len(kg), len(qg)
    sysh = run.system(s)
    ks = ephw.KSet(sysh, dev(kg), 0)
    eps = oracle.bands(s, kg)[0]
    # empty window
    used, start, other, pkq, _ = ephw.window_pairs(ks, dev(kqi), float(eps.max()) + 1.0, float(eps.max()) + 2.0,
                                                order=order)
    assert int(start[-1]) == 0 and not start.any()
    loss = torch.full((1,), 7.0, dtype=torch.float64, device="cuda:0")
    ephw.interpolate_pairs(ks, dev(qg), used, start, other, pkq, flags=ephw.OUT_LOSS, loss=loss)
    run.ctx.check()
    assert float(loss.cpu()[0]) == 7.0
    # every pair kept; by q in batches of 3 q
    used, start, other, pkq, _ = ephw.window_pairs(ks, dev(kqi), float(eps.min()) - 1.0, float(eps.max()) + 1.0,
                                                order=order)
    assert int(start[-1]) == nq * nk
    sysh.set_q_batch(3)
    g = torch.empty((nq * nk, s.nm, s.nw, s.nw), dtype=torch.complex128, device="cuda:0")
    ephw.interpolate_pairs(ks, dev(qg), used, start, other, pkq, flags=ephw.OUT_G, g_out=g)
    gw = torch.empty_like(g)
    ephw.interpolate_pairs(ks, dev(qg), used, start, other, pkq, flags=ephw.OUT_G | ephw.OUT_WANNIER, g_out=gw)
    sysh.set_q_batch(0)
    gf = torch.empty((nq, nk, s.nm, s.nw, s.nw), dtype=torch.complex128, device="cuda:0")
    ephw.interpolate(ks, dev(qg), kq_index=dev(kqi), flags=ephw.OUT_G, g_out=gf)
    run.ctx.check()
    perm = (lambda a: a) if order == 0 else (lambda a: np.swapaxes(a, 0, 1))
    full = perm(gf.cpu().numpy()).reshape(nq * nk, s.nm, s.nw, s.nw)
    assert np.abs(g.cpu().numpy() - full).max() < RTOL_W * np.abs(full).max()
    ref = oracle.interpolate(s, kg, qg, return_all=True)
    gw_ref = perm(ref["gw"]).reshape(nq * nk, s.nm, s.nw, s.nw)   # sums before the mode and band rotations
    np.testing.assert_allclose(gw.cpu().numpy(), gw_ref, rtol=0, atol=RTOL_W * np.abs(gw_ref).max())
    # only groups 1 and 30 own pairs (every other group skipped)
    n = nq if order == 0 else nk
    start = np.zeros(n + 1, dtype=np.int64)
    start[2:] = 3
    start[31:] = 3 + 32
    sel_major = np.concatenate([[1, 1, 1], np.full(32, 30)])
    sel_other = np.concatenate([[0, 5, 9], np.arange(32)]).astype(np.int32)
    sel_q, sel_k = (sel_major, sel_other) if order == 0 else (sel_other, sel_major)
    po = dev(sel_other)
    pkq = dev(kqi[sel_q, sel_k].astype(np.int32))
    g2 = torch.empty((35, s.nm, s.nw, s.nw), dtype=torch.complex128, device="cuda:0")
    ephw.interpolate_pairs(ks, dev(qg), order, start, po, pkq, flags=ephw.OUT_G, g_out=g2)
    run.ctx.check()
    full = gf.cpu().numpy()[sel_q, sel_k]
    assert np.abs(g2.cpu().numpy() - full).max() < RTOL_W * np.abs(full).max()
    # invalid offsets are refused before anything is enqueued
    bad = start.copy()
    bad[5] = 10
    with pytest.raises(ephw.EphwError):
        ephw.interpolate_pairs(ks, dev(qg), order, bad, po, pkq, flags=ephw.OUT_G, g_out=g2)
    bad = start.copy()
    bad[0] = 1
    with pytest.raises(ephw.EphwError):
        ephw.interpolate_pairs(ks, dev(qg), order, bad, po, pkq, flags=ephw.OUT_G, g_out=g2)
    ks.close()


@pytest.mark.parametrize("prec,order,nw", [(0, 0, 6), (1, 1, 6), (0, 1, 6), (1, 0, 12)])
def test_interpolate_pairs_band_window(run, prec, order, nw):
    """The band window: the screen's band range equals the range of the bands
    the oracle's eigenvalues put in the window; g, band sums and loss on that
    range equal the sub-blocks of the all-band pair path (same V, same sums;
    bit for bit where both run the row kernel, to rounding where the all-band
    rotations run on the matrix cores) and the oracle's weighted loss over
    those elements."""
    import torch
    from paper_2603_10295_amd import ephw
    from gpu_run import dev, cplx_dtype
    s, kg, qg, kqi, lo, hi, keep = window_case(prec, nw=nw)
    eps = oracle.bands(s, kg)[0]
    # a window around the second band (inside gaps): bands 1.. of the range
    hi = gap_edge(eps, np.quantile(eps[:, 2], 0.5))
    lo = gap_edge(eps, np.quantile(eps[:, 1], 0.5))
    inwin = (eps >= lo) & (eps <= hi)
    kact = inwin.any(axis=1)
    keep = kact[None, :] & kact[kqi]
    bset = np.flatnonzero(inwin.any(axis=0))
    b0, nb = int(bset.min()), int(bset.max() - bset.min() + 1)
    assert 0 < nb < s.nw and keep.any()
    nk = len(kg)
    ks = ephw.KSet(run.system(s), dev(kg), prec)
    used, start, other, pkq, band_range = ephw.window_pairs(ks, dev(kqi), lo, hi, order=order)
    assert band_range == (b0, nb)
    npairs = int(start[-1])
    assert npairs == int(keep.sum())
    flags = ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS
    gfull = torch.empty((npairs, s.nm, s.nw, s.nw), dtype=cplx_dtype(prec), device="cuda:0")
    ephw.interpolate_pairs(ks, dev(qg), used, start, other, pkq, flags=ephw.OUT_G, g_out=gfull)
    g = torch.empty((npairs, s.nm, nb, nb), dtype=cplx_dtype(prec), device="cuda:0")
    t = torch.empty((npairs, s.nm), dtype=torch.float64, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ephw.interpolate_pairs(ks, dev(qg), used, start, other, pkq, flags=flags, bands=band_range, g_out=g,
                           band_sum=t, loss=loss, loss_seed=31)
    run.ctx.check()
    ks.close()
    sub = gfull.cpu().numpy()[:, :, b0:b0 + nb, b0:b0 + nb]
    if nw <= 8:
        assert np.array_equal(g.cpu().numpy(), sub)
    else:
        assert np.abs(g.cpu().numpy() - sub).max() < (RTOL_W if prec == 0 else RTOL_32) * np.abs(sub).max()
    np.testing.assert_allclose(t.cpu().numpy(), (np.abs(sub.astype(np.complex128)) ** 2).sum(axis=(2, 3)),
                               rtol=1e-12 if prec == 0 else 1e-6)
    if order == ephw.PAIRS_BY_Q:
        iq, ik = np.nonzero(keep)
    else:
        ik, iq = np.nonzero(keep.T)
    ref = oracle.interpolate(s, kg, qg, return_all=True)
    w = oracle.splitmix64_weights(31, oracle.element_index(iq, ik, nk, s.nm, s.nw))[:, :, b0:b0 + nb, b0:b0 + nb]
    ghat = ref["ghat"][iq, ik][:, :, b0:b0 + nb, b0:b0 + nb]
    # the window's bands sit in gaps of the spectrum, so the sub-block sums are
    # gauge invariant when no degenerate block straddles the range edges
    l_ref = float(np.sum(w * np.abs(ghat) ** 2))
    l_err = abs(float(loss.cpu().numpy()[0]) - l_ref) / l_ref
    print(f"band window prec={prec} order={order}: bands {b0}..{b0 + nb - 1}, {npairs} pairs, loss {l_err:.2e}")
    assert l_err < (1e-10 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec,nw,na", [(1, 9, 3), (0, 16, 4), (1, 17, 5), (0, 20, 6), (1, 20, 6), (0, 31, 8)])
def test_row_kernel_and_matrix_cores_agree(run, prec, nw, na):
    """For 8 < Nw <= 32 the rotations run on the matrix cores; a band window
    holding every band sends the same pairs through the row kernel instead
    (its work splits: several pairs per workgroup, one pair in mode chunks
    with a ragged last chunk, and the 160 KB LDS form at FP64, Nw = 31,
    Nm = 24).  g, band sums and loss of both against each other and the
    oracle."""
    import torch
    from paper_2603_10295_amd import ephw
    from gpu_run import dev, cplx_dtype
    s = synth.make_system(nw, na, synth.box((2, 2, 1)), synth.box((2, 1, 1)), [nw, na, 5],
                          g_dtype=np.complex64 if prec else np.complex128)
    m = (3, 2, 1)
    kg = synth.uniform_grid(m)
    kqi = synth.grid_index_of_sum(m)
    nk = len(kg)
    ks = ephw.KSet(run.system(s), dev(kg), prec)
    eps = oracle.bands(s, kg)[0]
    used, start, other, pkq, band_range = ephw.window_pairs(ks, dev(kqi), float(eps.min()) - 1.0,
                                                            float(eps.max()) + 1.0, order=ephw.PAIRS_BY_Q)
    assert band_range == (0, nw) and int(start[-1]) == nk * nk
    flags = ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS
    outs = []
    for bands in ((0, 0), band_range):
        g = torch.empty((nk * nk, s.nm, nw, nw), dtype=cplx_dtype(prec), device="cuda:0")
        t = torch.empty((nk * nk, s.nm), dtype=torch.float64, device="cuda:0")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ephw.interpolate_pairs(ks, dev(kg), used, start, other, pkq, flags=flags, bands=bands, g_out=g,
                               band_sum=t, loss=loss, loss_seed=17)
        run.ctx.check()
        outs.append((g.cpu().numpy().astype(np.complex128), t.cpu().numpy(), float(loss.cpu()[0])))
    ks.close()
    (gm, tm, lm), (gr, tr, lr) = outs
    tol = RTOL_W if prec == 0 else RTOL_32
    assert np.abs(gm - gr).max() < tol * np.abs(gr).max()
    ref = oracle.interpolate(s, kg, kg, return_all=True)
    iq, ik = np.divmod(np.arange(nk * nk), nk)
    t_ref = oracle.band_sums(ref["ghat"]).reshape(nk * nk, s.nm)
    l_ref = oracle.weighted_loss(ref["ghat"].reshape(nk * nk, *ref["ghat"].shape[2:]), 17, iq, ik, nk)
    tol_s = RTOL_S if prec == 0 else RTOL_32
    for g_, t_, l_ in outs:
        sg = oracle.block_sums(np.abs(g_.reshape(nk, nk, *g_.shape[1:])) ** 2, ref["eps_kq"], ref["eps_k"],
                               ref["lam"])
        sr = oracle.block_sums(np.abs(ref["ghat"]) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
        assert oracle.compare_block_sums(sg, sr)[0] < tol_s
        assert np.abs(t_ - t_ref).max() < tol_s * np.abs(t_ref).max()
        assert abs(l_ - l_ref) < tol_s * l_ref
    print(f"rows vs matrix cores prec={prec} nw={nw}: g {np.abs(gm - gr).max() / np.abs(gr).max():.2e}")
