"""GPU parity of the multi-system batch (one grouped launch per stage over all
systems, graph-captured pass) against the oracle and the single-system path."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
# largest relative error of one degenerate block with S >= 1e-6 max S: FP32
# rounding of sums whose terms are up to 1e3 times the block's own size
FP32_BLOCK_TOL = 1e-2


@pytest.fixture(scope="module")
def run():
    from gpu_run import Runner
    return Runner()


def small_batch(count=6, seed=3, max_grid=5, cap_mib=24):
    # heterogeneous shapes from the batch generator, capped small for the oracle
    return synth.batch_systems(seed=seed, count=count, max_grid=max_grid, g_cap_bytes=cap_mib * 2 ** 20)


def make_items(run, works, flags):
    import torch
    from paper_2603_10295_amd import ephw
    items, keep = [], []
    for i, w in enumerate(works):
        s = w.system
        sysh = run.system(s)
        k = torch.from_numpy(w.k).to("cuda:0")
        q = torch.from_numpy(w.q).to("cuda:0")
        ks = ephw.KSet(sysh, k, ephw.FP32)
        nk, nq = len(w.k), len(w.q)
        it = dict(ks=ks, q=q, kq_index=torch.from_numpy(w.kq_index).to("cuda:0"), flags=flags,
                  band_sum=torch.zeros((nq, nk, s.nm), dtype=torch.float64, device="cuda:0"),
                  loss=torch.zeros(1, dtype=torch.float64, device="cuda:0"), loss_seed=100 + i)
        if flags & ephw.OUT_G:
            it["g_out"] = torch.zeros((nq, nk, s.nm, s.nw, s.nw), dtype=torch.complex64, device="cuda:0")
        items.append(it)
        keep.append((sysh, k))
    return items, keep


@pytest.mark.parametrize("seed,max_grid,count,cap_mib", [(3, 5, 6, 24), (25, 4, 6, 24), (50, 4, 4, 96)])
def test_batch_matches_oracle_and_replays(run, tmp_path, seed, max_grid, count, cap_mib):
    """Every item of a heterogeneous batch against the oracle on ALL of its
    pairs, through quantities that depend on the eigenvectors V(k), V(k+q):
    the gauge-invariant block sums of the batch's own stored g (a wrong V,
    k+q index or item offset mixes non-degenerate blocks) and the batch's own
    weighted loss (the weights differ per (nu, m, n) element).  The band sums
    T_nu, which any unitary V leaves unchanged, are checked beside them.
    Seed 3 draws band counts 4..7 (row kernel), seed 25 also Nw = 9 and 13
    (the one-wave matrix-core rotations, one grouped launch for both), seed 50
    Nw = 22 (the rotations split over a workgroup's four waves) beside Nw = 9."""
    import torch
    from paper_2603_10295_amd import ephw
    works = small_batch(seed=seed, max_grid=max_grid, count=count, cap_mib=cap_mib)
    if seed == 25:
        assert sorted(w.system.nw for w in works if w.system.nw > 8) == [9, 13]
    if seed == 50:
        assert sorted(w.system.nw for w in works if w.system.nw > 8) == [9, 22]
    assert len({(w.system.nw, w.system.nm, w.system.ne) for w in works}) > 3   # heterogeneous
    items, keep = make_items(run, works, ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS)
    cache = str(tmp_path / "tune.jsonl")
    b = ephw.Batch(run.ctx, items, tune=True, tune_cache=cache)
    b.run()
    run.ctx.check()
    first = [(it["g_out"].cpu().numpy(), it["band_sum"].cpu().numpy(), float(it["loss"].cpu()[0]))
             for it in items]
    b.run()
    run.ctx.check()
    for it, (g1, t1, l1) in zip(items, first):
        assert np.array_equal(it["g_out"].cpu().numpy(), g1)              # replay is deterministic
        assert np.array_equal(it["band_sum"].cpu().numpy(), t1)
        assert float(it["loss"].cpu()[0]) == 2 * l1                       # loss accumulates
    print("batch stats", b.stats(), [b.shape(i) for i in range(len(items))])
    for i, w in enumerate(works):
        s = w.system
        nk, nq = len(w.k), len(w.q)
        ref = oracle.interpolate(s, w.k, w.q, return_all=True)
        g_gpu = first[i][0].astype(np.complex128)
        sg = oracle.block_sums(np.abs(g_gpu) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
        sr = oracle.block_sums(np.abs(ref["ghat"]) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
        norm, blk = oracle.compare_block_sums(sg, sr)
        print(f"item {i} {w.name}: block sums normwise {norm:.2e}, max blockwise {blk:.2e}")
        assert norm < FP32_TOL, (i, w.name, norm)
        assert blk < FP32_BLOCK_TOL, (i, w.name, blk)
        t_ref = oracle.band_sums(ref["ghat"])
        err = float(np.abs(first[i][1] - t_ref).max() / np.abs(t_ref).max())
        assert err < FP32_TOL, (i, w.name, err)
        # the batch's own loss over every pair of the item
        gh = ref["ghat"].reshape(nq * nk, *ref["ghat"].shape[2:])
        iq = np.repeat(np.arange(nq), nk)
        ik = np.tile(np.arange(nk), nq)
        l_ref = oracle.weighted_loss(gh, 100 + i, iq, ik, nk)
        assert abs(first[i][2] - l_ref) < FP32_TOL * l_ref, (i, w.name, first[i][2], l_ref)
    # the tuned shapes were cached and are reused
    lines = [json.loads(l) for l in open(cache)]
    assert len(lines) >= len({w.name.split("_", 1)[1] for w in works}) - 1
    b2 = ephw.Batch(run.ctx, items, tune=True, tune_cache=cache)
    assert [b2.shape(i) for i in range(len(items))] == [b.shape(i) for i in range(len(items))]
    assert len(open(cache).readlines()) == len(lines)
    b2.close()
    b.close()


def test_batch_solo_items_equal_grouped(run):
    """A workspace budget below what the items' sweep buffers want sends the
    largest items to rounds of their own, sharing one sweep region, with their
    phase sums as plain GEMMs (the tile or streaming kernel of their own
    shape): with every item solo (a 1-byte budget), with some solo (3 GiB: the
    1 GiB floor caps of six items leave the last two grouped) and with none,
    the shapes are the same and the outputs agree to FP32 rounding (the plain
    and grouped GEMMs tile the same sums differently), the sweep region shared
    by items run one after another included."""
    from paper_2603_10295_amd import ephw
    works = small_batch()
    flags = ephw.OUT_G | ephw.OUT_BAND_SUM | ephw.OUT_LOSS
    outs, solos = [], []
    for budget in (0, 3 << 30, 1):
        items, keep = make_items(run, works, flags)
        b = ephw.Batch(run.ctx, items, workspace_budget_bytes=budget)
        b.run()
        b.run()
        run.ctx.check()
        solos.append([b.solo(i) for i in range(len(items))])
        shapes = [b.shape(i) for i in range(len(items))]
        outs.append((shapes, [(it["g_out"].cpu().numpy(), it["band_sum"].cpu().numpy(),
                               float(it["loss"].cpu()[0])) for it in items]))
        b.close()
    print("solo items per budget", solos)
    assert not any(solos[0]) and all(solos[2]) and 0 < sum(solos[1]) < len(works)
    for shapes, res in outs[1:]:
        assert shapes == outs[0][0]
        for (g, t, l), (g0, t0, l0) in zip(res, outs[0][1]):
            assert np.abs(g - g0).max() <= FP32_TOL * np.abs(g0).max()
            assert np.abs(t - t0).max() <= FP32_TOL * np.abs(t0).max()
            assert abs(l - l0) <= FP32_TOL * abs(l0)


def test_batch_without_graph_equals_graph(run):
    from paper_2603_10295_amd import ephw
    works = small_batch(count=4, seed=9)
    items_a, keep_a = make_items(run, works, ephw.OUT_BAND_SUM)
    items_b, keep_b = make_items(run, works, ephw.OUT_BAND_SUM)
    import torch
    a = ephw.Batch(run.ctx, items_a, use_graph=True)
    b = ephw.Batch(run.ctx, items_b, use_graph=False)
    b.run()
    run.ctx.check()
    eager = [y["band_sum"].cpu().numpy() for y in items_b]
    # several graph replays, with eager device work and synchronisation in
    # between; every replay must equal the eager pass (the work-queue
    # counters are re-zeroed by a kernel node on each replay)
    for rep in range(3):
        for x in items_a:
            x["band_sum"].fill_(-1.0)
        torch.cuda.synchronize()
        a.run()
        run.ctx.check()
        scratch = torch.randn(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        for x, e in zip(items_a, eager):
            assert np.array_equal(x["band_sum"].cpu().numpy(), e), rep
    a.close()
    b.close()


def test_batch_rejects_missing_index(run):
    import torch
    from paper_2603_10295_amd import ephw
    w = small_batch(count=1)[0]
    items, keep = make_items(run, [w], ephw.OUT_LOSS)
    items[0]["kq_index"] = None
    with pytest.raises(ephw.EphwError) as e:
        ephw.Batch(run.ctx, items)
    assert e.value.status == ephw.EINVAL
