"""Helpers that drive the HIP library through its C ABI for the GPU tests.

They marshal numpy inputs to torch device tensors, call the binding and
return numpy results; they contain none of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np


def torch_mod():
    import torch
    return torch


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def cplx_dtype(prec):
    torch = torch_mod()
    return torch.complex128 if prec == 0 else torch.complex64


class Runner:
    def __init__(self):
        from paper_2603_10295_amd import ephw
        self.ephw = ephw
        self.ctx = ephw.Context(0)

    def system(self, s):
        return self.ephw.System.from_synth(self.ctx, s)

    def bands(self, sysh, k):
        torch = torch_mod()
        kt = dev(k)
        eps = torch.empty((len(k), sysh.nw), dtype=torch.float64, device="cuda:0")
        vec = torch.empty((len(k), sysh.nw, sysh.nw), dtype=torch.complex128, device="cuda:0")
        self.ephw.bands(sysh, kt, eps, vec)
        self.ctx.check()
        return eps.cpu().numpy(), vec.cpu().numpy()

    def phonons(self, sysh, q):
        torch = torch_mod()
        qt = dev(q)
        lam = torch.empty((len(q), sysh.nm), dtype=torch.float64, device="cuda:0")
        om = torch.empty_like(lam)
        ev = torch.empty((len(q), sysh.nm, sysh.nm), dtype=torch.complex128, device="cuda:0")
        self.ephw.phonons(sysh, qt, lam, om, ev)
        self.ctx.check()
        return lam.cpu().numpy(), om.cpu().numpy(), ev.cpu().numpy()

    def phase_sum_rp(self, sysh, q, prec):
        torch = torch_mod()
        out = torch.empty((len(q), sysh.ne, sysh.nm, sysh.nw, sysh.nw), dtype=cplx_dtype(prec), device="cuda:0")
        self.ephw.phase_sum_rp(sysh, dev(q), prec, out)
        self.ctx.check()
        return out.cpu().numpy()

    def interpolate(self, sysh, k, q, prec, *, kq_index=None, flags=None, q_offset=0, loss_seed=0,
                    q_batch=0, want_eps_kq=True):
        torch = torch_mod()
        E = self.ephw
        if flags is None:
            flags = E.OUT_G | E.OUT_BAND_SUM | E.OUT_LOSS
        sysh.set_q_batch(q_batch)
        kt, qt = dev(k), dev(q)
        ks = E.KSet(sysh, kt, prec)
        nk, nq = len(k), len(q)
        g = torch.empty((nq, nk, sysh.nm, sysh.nw, sysh.nw), dtype=cplx_dtype(prec), device="cuda:0") \
            if flags & E.OUT_G else None
        t = torch.empty((nq, nk, sysh.nm), dtype=torch.float64, device="cuda:0") \
            if flags & E.OUT_BAND_SUM else None
        loss = torch.zeros(1, dtype=torch.float64, device="cuda:0") if flags & E.OUT_LOSS else None
        ekq = torch.empty((nq, nk, sysh.nw), dtype=torch.float64, device="cuda:0") if want_eps_kq else None
        om = torch.empty((nq, sysh.nm), dtype=torch.float64, device="cuda:0")
        kqi = dev(kq_index) if kq_index is not None else None
        E.interpolate(ks, qt, kq_index=kqi, q_offset=q_offset, flags=flags, g_out=g, band_sum=t, loss=loss,
                      loss_seed=loss_seed, eps_kq=ekq, omega=om)
        self.ctx.check()
        eps_k = torch.empty((nk, sysh.nw), dtype=torch.float64, device="cuda:0")
        ks.bands(eps_k)
        torch.cuda.synchronize()
        out = dict(omega=om.cpu().numpy(), eps_k=eps_k.cpu().numpy())
        if g is not None:
            out["g"] = g.cpu().numpy()
        if t is not None:
            out["band_sum"] = t.cpu().numpy()
        if loss is not None:
            out["loss"] = float(loss.cpu().numpy()[0])
        if ekq is not None:
            out["eps_kq"] = ekq.cpu().numpy()
        ks.close()
        return out


def scaled_block_error(s_gpu, s_ref):
    """Largest |S_gpu - S_ref| / sqrt(S_ref * max S_ref) over the degenerate-block
    sums of |g|^2 (blocks with S_ref >= 1e-10 max S_ref).  An absolute error
    eta * |g|max in the elements of g changes a block sum S by about
    2 eta sqrt(S * max S), so this bounds eta; the plain relative error of
    blocks far below the largest is not something an FP32 sum can bound."""
    a = np.concatenate([x.reshape(-1) for x in s_gpu])
    b = np.concatenate([x.reshape(-1) for x in s_ref])
    keep = b >= 1e-10 * b.max()
    return float(np.max(np.abs(a[keep] - b[keep]) / np.sqrt(b[keep] * b.max())))
