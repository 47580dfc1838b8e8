"""Failure paths forced from the host: a context's device-memory cap
(EPHW_ENOMEM before any allocation) and its Jacobi sweep limit (EPHW_ENOCONV
through the status word; the eigensolve kernels still exit normally)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def small_system(nw=8, na=2, seed=5):
    return synth.make_system(nw, na, synth.box((3, 3, 2)), synth.box((3, 2, 2)), [seed, 70])


def test_memory_cap_gives_enomem_and_releases():
    from paper_2603_10295_amd import ephw
    ctx = ephw.Context(0)
    s = small_system()
    g_bytes = s.g.nbytes
    ctx.set_limits(max_device_bytes=g_bytes // 2)
    assert ctx.memory() == (0, g_bytes // 2)
    with pytest.raises(ephw.EphwError) as e:
        ephw.System.from_synth(ctx, s)
    assert e.value.status == ephw.ENOMEM
    assert "limit" in str(e.value)
    assert ctx.memory()[0] == 0                 # the partial system was released
    ctx.set_limits(max_device_bytes=0)
    sysh = ephw.System.from_synth(ctx, s)
    used = ctx.memory()[0]
    assert used == sysh.bytes() and used >= g_bytes
    # a workspace that would pass the cap fails the call, not the process
    import torch
    ctx.set_limits(max_device_bytes=used + 4096)
    k = torch.from_numpy(synth.uniform_grid((2, 2, 2))).to("cuda:0")
    with pytest.raises(ephw.EphwError) as e:
        ephw.KSet(sysh, k, ephw.FP64)
    assert e.value.status == ephw.ENOMEM
    assert ctx.memory()[0] == used
    ctx.set_limits(max_device_bytes=0)
    ks = ephw.KSet(sysh, k, ephw.FP64)
    assert ctx.memory()[0] > used
    ks.close()
    sysh.close()
    assert ctx.memory()[0] == 0
    ctx.close()


@pytest.mark.parametrize("nw", [8, 36])
def test_sweep_limit_gives_enoconv(nw):
    """nw = 8 runs the one-wave LDS solver, nw = 36 the global-memory one."""
    import torch
    from paper_2603_10295_amd import ephw
    ctx = ephw.Context(0)
    sysh = ephw.System.from_synth(ctx, small_system(nw=nw, na=1))
    k = torch.from_numpy(synth.uniform_grid((2, 2, 2))).to("cuda:0")
    eps = torch.empty((len(k), nw), dtype=torch.float64, device="cuda:0")
    ctx.set_limits(max_sweeps=0)
    ephw.bands(sysh, k, eps)
    with pytest.raises(ephw.EphwError) as e:
        ctx.check()
    assert e.value.status == ephw.ENOCONV
    ctx.check()                                  # the status word was cleared
    ctx.set_limits(max_sweeps=40)
    ephw.bands(sysh, k, eps)
    ctx.check()
    ref = oracle.bands(small_system(nw=nw, na=1), synth.uniform_grid((2, 2, 2)))[0]
    assert np.abs(eps.cpu().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    sysh.close()
    ctx.close()
