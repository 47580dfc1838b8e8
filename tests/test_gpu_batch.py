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


@pytest.fixture(scope="module")
def run():
    from gpu_run import Runner
    return Runner()


def small_batch(count=6, seed=3):
    # heterogeneous shapes from the batch generator, capped small for the oracle
    return synth.batch_systems(seed=seed, count=count, max_grid=5, g_cap_bytes=24 * 2 ** 20)


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
        items.append(it)
        keep.append((sysh, k))
    return items, keep


def test_batch_matches_oracle_and_replays(run, tmp_path):
    import torch
    from paper_2603_10295_amd import ephw
    works = small_batch()
    assert len({(w.system.nw, w.system.nm, w.system.ne) for w in works}) > 3   # heterogeneous
    items, keep = make_items(run, works, ephw.OUT_BAND_SUM | ephw.OUT_LOSS)
    cache = str(tmp_path / "tune.jsonl")
    b = ephw.Batch(run.ctx, items, tune=True, tune_cache=cache)
    b.run()
    run.ctx.check()
    first = [(it["band_sum"].cpu().numpy(), float(it["loss"].cpu()[0])) for it in items]
    b.run()
    run.ctx.check()
    for it, (t1, l1) in zip(items, first):
        assert np.array_equal(it["band_sum"].cpu().numpy(), t1)          # replay is deterministic
        assert float(it["loss"].cpu()[0]) == 2 * l1                       # loss accumulates
    print("batch stats", b.stats(), [b.shape(i) for i in range(len(items))])
    for i, w in enumerate(works):
        s = w.system
        nk = len(w.k)
        sample = np.unique(np.array([0, len(w.q) // 2, len(w.q) - 1]))
        ref = oracle.interpolate(s, w.k, w.q[sample], return_all=True)
        t_ref = oracle.band_sums(ref["ghat"])
        t_gpu = first[i][0][sample]
        err = float(np.abs(t_gpu - t_ref).max() / np.abs(t_ref).max())
        assert err < FP32_TOL, (i, w.name, err)
        # loss of the sampled q rows only: recompute with the oracle and with the single path
        gh = ref["ghat"].reshape(len(sample) * nk, *ref["ghat"].shape[2:])
        iq = np.repeat(sample, nk)
        ik = np.tile(np.arange(nk), len(sample))
        l_ref = oracle.weighted_loss(gh, 100 + i, iq, ik, nk)
        single = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for qi in sample:
            ephw.interpolate(items[i]["ks"], items[i]["q"][qi:qi + 1], kq_index=items[i]["kq_index"][qi:qi + 1],
                             q_offset=int(qi), flags=ephw.OUT_LOSS, loss=single, loss_seed=100 + i)
        run.ctx.check()
        assert abs(float(single.cpu()[0]) - l_ref) < FP32_TOL * l_ref
    # the tuned shapes were cached and are reused
    lines = [json.loads(l) for l in open(cache)]
    assert len(lines) >= len({w.name.split("_", 1)[1] for w in works}) - 1
    b2 = ephw.Batch(run.ctx, items, tune=True, tune_cache=cache)
    assert [b2.shape(i) for i in range(len(items))] == [b.shape(i) for i in range(len(items))]
    assert len(open(cache).readlines()) == len(lines)
    b2.close()
    b.close()


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
