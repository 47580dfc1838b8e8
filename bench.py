#!/usr/bin/env python3
"""Throughput of the e-ph Wannier interpolation on one MI355X.

Workload (default): the dense Si-like precision system - Nw=8 bands, Nm=6
modes, 10x10x10 boxes (Ne=Np=1000), k = q = the 20^3 uniform grid (8000
each), g stored complex64.  One step is the whole path on that input:
k-side phases + H(k) eigensolves, then every q in chunks: phases, D(q)
eigensolves, the Rp phase GEMM (Eq. 9), mode rotation, the Re phase GEMM
(Eq. 10), band rotations, storing every g_{mn nu}(k,q) (complex64) into a
q-chunk output buffer.  Inputs are resident in HBM before timing starts.

Reported: g(k,q) elements/s of the FP32-MFMA path (the value), the same
workload on the FP64 path and the speedup, the error of both against the
CPU oracle on a q sample, per-stage times from HIP events, the roofline of
the dominant kernel, and the oracle's own throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="si_dense",
                    choices=["si_dense", "mos2_2d", "si_toy", "batch32", "ribbon", "coarse_si", "si_window", "si_linewidth"])
    ap.add_argument("--ribbon-nk", type=int, default=256, help="k = q = i/n along the ribbon axis")
    ap.add_argument("--ribbon-nw", type=int, default=200)
    ap.add_argument("--ribbon-na", type=int, default=50)
    ap.add_argument("--batch-count", type=int, default=32)
    ap.add_argument("--batch-max-grid", type=int, default=16)
    ap.add_argument("--batch-uncapped", action="store_true",
                    help="batch32: the systems as drawn, no cap on the size of g (g drawn on the device)")
    ap.add_argument("--tune-cache", default="")
    ap.add_argument("--grid", type=int, default=20, help="k = q = grid^3 for si_dense")
    ap.add_argument("--q-chunk", type=int, default=1024)
    ap.add_argument("--no-band-window", action="store_true", help="si_window: keep all bands of the kept pairs")
    ap.add_argument("--pair-order", type=int, default=-1,
                    help="si_window pair lists: 0 by q, 1 by k, -1 the cheaper (fewer groups owning pairs)")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-sample-q", type=int, default=12, help="q points of the oracle sample (about 15 s of host work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-one-thread-q", type=int, default=1,
                    help="q points of the oracle's one-thread sample (0 skips it)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-comp", action="store_true",
                    help="skip the compensated FP32 (K-blocked accumulation) measurement")
    ap.add_argument("--comp-steps", type=int, default=2)
    ap.add_argument("--q-batch", type=int, default=0)
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="first run a plain device copy of this many GiB (HBM counter calibration)")
    return ap.parse_args(argv)


def workload(args):
    import synth
    if args.workload == "si_dense":
        return synth.si_dense(m=args.grid)
    w = synth.mos2_2d() if args.workload == "mos2_2d" else synth.si_toy()
    # g stored complex64 so that the FP32 leg can run; the FP64 leg and the
    # oracle take the same (exactly widened) values
    w.system.g = w.system.g.astype(np.complex64)
    w.precision = "fp32"
    w.name = w.name.replace("_fp64", "") + "_g_c64"
    return w


class Path:
    """One precision of the GPU path on a resident system."""

    def __init__(self, ctx, system, prec, k, q, kqi, q_chunk, q_batch):
        import torch
        from paper_2603_10295_amd import ephw
        self.ephw = ephw
        self.ctx = ctx
        self.sys = ephw.System.from_synth(ctx, system)
        if q_batch:
            self.sys.set_q_batch(q_batch)
        self.prec = prec
        self.k, self.q, self.kqi = k, q, kqi
        self.q_chunk = min(q_chunk, q.shape[0])
        s = system
        dt = torch.complex128 if prec == ephw.FP64 else torch.complex64
        self.out = torch.empty((self.q_chunk, k.shape[0], s.nm, s.nw, s.nw), dtype=dt, device="cuda:0")

    def step(self):
        E = self.ephw
        ks = E.KSet(self.sys, self.k, self.prec)
        nq = self.q.shape[0]
        for q0 in range(0, nq, self.q_chunk):
            q1 = min(nq, q0 + self.q_chunk)
            E.interpolate(ks, self.q[q0:q1], kq_index=None if self.kqi is None else self.kqi[q0:q1],
                          q_offset=q0, flags=E.OUT_G, g_out=self.out[: q1 - q0])
        ks.close()

    def sample(self, qs_idx):
        """g for the sampled q (all k), copied to the host."""
        import torch
        E = self.ephw
        ks = E.KSet(self.sys, self.k, self.prec)
        n = len(qs_idx)
        idx = torch.as_tensor(qs_idx, device="cuda:0")
        out = torch.empty((n,) + tuple(self.out.shape[1:]), dtype=self.out.dtype, device="cuda:0")
        E.interpolate(ks, self.q[idx].contiguous(),
                      kq_index=None if self.kqi is None else self.kqi[idx].contiguous(),
                      flags=E.OUT_G, g_out=out)
        self.ctx.check()
        res = out.cpu().numpy()
        ks.close()
        return res


def timed(path, steps, warmup, profile=False):
    import torch
    for _ in range(warmup):
        path.step()
    path.ctx.check()
    if profile:
        path.sys.profile_read()
        path.sys.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        path.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = None
    if profile:
        path.sys.profile(False)
        stages = path.sys.profile_read()
    path.ctx.check()
    return (t1 - t0) / steps, stages


def measured_traffic(kernel_tag: str, workgroups: int):
    """HBM bytes per dispatch of a kernel from the committed counter summary,
    or None when the GEMM source changed since the counters were taken."""
    from paper_2603_10295_amd import rocprof_summary as rs
    path = os.path.join(ROOT, "profiles", "cgemm_si_dense_nw8_nm6_ne1000_8000k_8000q_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    lines = open(path).read().splitlines()
    if not lines or f"digest {rs.source_digest()}" not in lines[0]:
        return None
    for l in lines:
        if l.startswith("#") or kernel_tag not in l or f"[{workgroups} x" not in l:
            continue
        parts = l.split()
        return (float(parts[3]) + float(parts[4])) * 1e9
    return None


def block_error(g_gpu, ref):
    """(normwise, max blockwise, max scaled blockwise) errors of the degenerate-
    block sums of |g|^2; the scaled form divides each block's error by
    sqrt(S_block * max S) (blocks with S >= 1e-10 max S), the size that an
    absolute error of g proportional to the largest |g| gives, so that blocks
    far below the largest are not held to a relative bound no FP32 sum meets."""
    import oracle
    s_gpu = oracle.block_sums(np.abs(g_gpu.astype(np.complex128)) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
    s_ref = oracle.block_sums(np.abs(ref["ghat"]) ** 2, ref["eps_kq"], ref["eps_k"], ref["lam"])
    norm, blk = oracle.compare_block_sums(s_gpu, s_ref)
    a = np.concatenate([x.reshape(-1) for x in s_gpu])
    b = np.concatenate([x.reshape(-1) for x in s_ref])
    keep = b >= 1e-10 * b.max()
    scaled = float(np.max(np.abs(a[keep] - b[keep]) / np.sqrt(b[keep] * b.max())))
    return norm, blk, scaled


def cpu_baseline(w, qs_idx):
    """The oracle as it stands on a q sample (all k): returns (elems/s, seconds, ref)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = None
    t0 = time.perf_counter()
    ref = oracle.interpolate(w.system, w.k, w.q[qs_idx], return_all=True)
    dt = time.perf_counter() - t0
    s = w.system
    elems = len(qs_idx) * len(w.k) * s.nm * s.nw * s.nw
    return elems / dt, dt, ref, threads


def device_g(s, seed: int):
    """complex64 g(Re,Rp) of system s drawn on the device: complex normal
    (re, im iid N(0, 1/2)) times exp(-(|Re| + |Rp|)/2), the value distribution
    of the host generator, from torch's counter-based device generator (for
    systems too large to draw on the host; nothing compares them with the
    host-drawn values)."""
    import torch
    dev_ = "cuda:0"
    ne, npp = len(s.r_e), len(s.r_p)
    nre = torch.from_numpy(np.linalg.norm(s.r_e.astype(np.float64), axis=1)).to(dev_)
    nrp = torch.from_numpy(np.linalg.norm(s.r_p.astype(np.float64), axis=1)).to(dev_)
    env = torch.exp(-0.5 * (nrp[:, None] + nre[None, :])).to(torch.float32)
    out = torch.empty((npp, ne, s.nm, s.nw, s.nw), dtype=torch.complex64, device=dev_)
    gen = torch.Generator(device=dev_)
    gen.manual_seed(seed)
    per = max(1, int(2 ** 28 // max(1, ne * s.nm * s.nw * s.nw)))   # Rp rows per draw
    for p0 in range(0, npp, per):
        p1 = min(npp, p0 + per)
        x = torch.randn((p1 - p0, ne, s.nm, s.nw, s.nw, 2), generator=gen, device=dev_, dtype=torch.float32)
        x.mul_(0.7071067811865476 * env[p0:p1, :, None, None, None, None])
        out[p0:p1] = torch.view_as_complex(x)
        del x
    return out


def bench_batch(args):
    """Many heterogeneous systems in one graph-captured pass (one grouped launch
    per stage), against the same items run one system at a time (each system
    timed on its own after a warm-up call, its workspace released before the
    next).  --batch-uncapped draws the 32 systems with no cap on the size of
    g (about 207 GB of complex64 g in all, generated on the device)."""
    import torch
    import synth
    from paper_2603_10295_amd import ephw, model
    t_gen = time.perf_counter()
    ctx = ephw.Context(0)
    items, keep, names = [], [], []
    elems = 0.0
    cnt_tot = None
    cap = None if args.batch_uncapped else synth.G_CAP_BYTES
    g_bytes = 0
    for i in range(args.batch_count):
        # generated, uploaded, freed one by one
        w = synth.batch_system(0, i, max_grid=args.batch_max_grid, g_cap_bytes=cap, with_g=cap is not None)
        names.append(w.name)
        s = w.system
        if cap is None:
            sysh = ephw.System.from_synth(ctx, s, g_dtype=ephw.C64)
            g = device_g(s, seed=1000 + i)
            sysh.set_g(g)
            torch.cuda.synchronize()
            g_bytes += g.numel() * 8
            del g
            log(f"system {i}: {w.name}, g {g_bytes / 1e9:.1f} GB so far")
        else:
            sysh = ephw.System.from_synth(ctx, s)
            g_bytes += s.g.nbytes
        k = torch.from_numpy(w.k).to("cuda:0")
        q = torch.from_numpy(w.q).to("cuda:0")
        ks = ephw.KSet(sysh, k, ephw.FP32)
        items.append(dict(ks=ks, q=q, kq_index=torch.from_numpy(w.kq_index).to("cuda:0"), flags=ephw.OUT_LOSS,
                          loss=torch.zeros(1, dtype=torch.float64, device="cuda:0"), loss_seed=i))
        keep.append(sysh)
        c = model.stage_counts(s.nw, s.nm, s.ne, s.np_, len(w.k), len(w.q))
        elems += c.elems
        cnt_tot = c if cnt_tot is None else model.StageCounts(*(getattr(cnt_tot, f) + getattr(c, f)
                                                               for f in ("rp", "modes", "re", "rot", "hkq", "elems")))
        del w, s
    log(f"batch of {len(names)} systems generated and uploaded in {time.perf_counter() - t_gen:.1f}s")
    torch.cuda.synchronize()
    t_tune = time.perf_counter()
    b = ephw.Batch(ctx, items, tune=True, tune_cache=args.tune_cache or None)
    log(f"planned in {time.perf_counter() - t_tune:.1f}s: {b.stats()}, "
        f"{sum(b.solo(i) for i in range(len(items)))} of {len(items)} systems in rounds of their own")
    for _ in range(max(1, args.warmup)):
        b.run()
    ctx.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    ctx.check()
    stats, shapes = b.stats(), [dict(b.shape(i), solo=b.solo(i)) for i in range(len(items))]
    b.close()   # release the batch's sweep buffers before the one-at-a-time runs allocate theirs
    # the same items, one system at a time (no grouping, no graph): each
    # system warmed up and timed on its own, its workspace then released
    ts = 0.0
    per_system_ms = []
    for it, sysh in zip(items, keep):
        def one():
            ephw.interpolate(it["ks"], it["q"], kq_index=it["kq_index"], flags=ephw.OUT_LOSS, loss=it["loss"],
                             loss_seed=it["loss_seed"])
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ts += dt
        per_system_ms.append(round(dt * 1e3, 3))
        ctx.check()
        sysh.trim()
    log(f"one at a time: {ts * 1e3:.1f} ms; batched {tb * 1e3:.1f} ms")
    gemm_tf = 8.0 * cnt_tot.gemm / tb / 1e12
    line = {
        "metric": "g(k,q) elems/s (FP32 MFMA path, 32-system batch)", "value": elems / tb, "unit": "elems/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tb * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"batch{len(names)}_{'uncapped' if cap is None else 'capped2GiB'}"
                               f"_maxgrid{args.batch_max_grid}", "systems": len(names),
                   "g_bytes": g_bytes, "g_source": "device generator" if cap is None else "host generator",
                   "output": "weighted |g|^2 loss per system", **stats},
        "one_system_at_a_time_per_system_ms": per_system_ms,
        "one_system_at_a_time_ms": ts * 1e3, "batch_speedup": ts / tb,
        "phase_gemm_tflops_lower_bound": gemm_tf,
        "algorithmic_flops_per_step": 8.0 * cnt_tot.total,
        "shapes": [dict(system=names[i], **shapes[i]) for i in range(len(items))],
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_ribbon(args):
    """Differentiation workload: weighted |g|^2 loss over all pairs and its
    gradients dL/dg(Re,Rp), dL/dk, dL/dq (hand-written adjoint), FP32 MFMA."""
    import torch
    import synth
    from paper_2603_10295_amd import ephw, model
    t_gen = time.perf_counter()
    w = synth.ribbon_1d(nw=args.ribbon_nw, na=args.ribbon_na, nk=args.ribbon_nk)
    s = w.system
    nk, nq = len(w.k), len(w.q)
    log(f"workload {w.name}: generated in {time.perf_counter() - t_gen:.1f}s, g {s.g.nbytes / 1e9:.2f} GB")
    ctx = ephw.Context(0)
    sysh = ephw.System.from_synth(ctx, s)
    k = torch.from_numpy(w.k).to("cuda:0")
    q = torch.from_numpy(w.q).to("cuda:0")
    kqi = torch.from_numpy(w.kq_index).to("cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    dg = torch.zeros(s.g.shape, dtype=torch.complex64, device="cuda:0")
    dk = torch.zeros((nk, 3), dtype=torch.float64, device="cuda:0")
    dq = torch.zeros((nq, 3), dtype=torch.float64, device="cuda:0")
    del w.system.g

    def fwd():
        ks = ephw.KSet(sysh, k, ephw.FP32)
        ephw.interpolate(ks, q, kq_index=kqi, flags=ephw.OUT_LOSS, loss=loss, loss_seed=1)
        ks.close()

    def bwd():
        ks = ephw.KSet(sysh, k, ephw.FP32)
        ephw.loss_backward(ks, q, kqi, loss_seed=1, loss=loss, dL_dg=dg, dL_dk=dk, dL_dq=dq)
        ks.close()

    def timed_call(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for _ in range(args.warmup):
        fwd()
    sysh.profile_read()
    sysh.profile(True)
    t_f = min(timed_call(fwd) for _ in range(args.steps))
    sysh.profile(False)
    st_f = sysh.profile_read()
    ctx.check()
    log(f"forward: {t_f:.3f} s")
    t_b = timed_call(bwd)
    ctx.check()
    log(f"backward (recompute + gradients): {t_b:.3f} s")
    c = model.stage_counts(s.nw, s.nm, s.ne, s.np_, nk, nq)
    line = {
        "metric": "g(k,q) elems/s (FP32 MFMA path, loss forward; ribbon differentiation workload)",
        "value": c.elems / t_f, "unit": "elems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_f * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": w.name, "nw": s.nw, "nm": s.nm, "ne": s.ne, "np": s.np_, "nk": nk, "nq": nq},
        "forward_s": t_f, "backward_s": t_b,
        "forward_algorithmic_tflops": 8.0 * c.total / t_f / 1e12,
        "rotation_share_of_flops": c.rot / c.total,
        "stages_forward_ms": {k_: round(v[0], 3) for k_, v in st_f.items()},
        "gradient_norms": {"dL_dg": float(torch.linalg.vector_norm(dg).cpu()),
                           "dL_dk": float(torch.linalg.vector_norm(dk).cpu()),
                           "dL_dq": float(torch.linalg.vector_norm(dq).cpu())},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_coarse(args):
    """Eq. (6), the coarse Bloch -> Wannier transform, on a Si-like system:
    Nw 8, Nm 6, Re box 8^3 and Rp box 4^3 with the coarse k' = 8^3 and
    q' = 4^3 grids they are complete residue systems of.  The Bloch input is
    Eq. (7) on those grids; parity is the round trip back to g(Re,Rp)."""
    import torch
    import synth
    from paper_2603_10295_amd import ephw
    ne_box, np_box = (8, 8, 8), (4, 4, 4)
    t_gen = time.perf_counter()
    s = synth.make_system(8, 2, synth.box(ne_box), synth.box(np_box), [0, 11])
    kc, qc = synth.uniform_grid(ne_box), synth.uniform_grid(np_box)
    mk = np.asarray(ne_box)
    ik, iq = np.rint(kc * mk).astype(np.int64), np.rint(qc * mk).astype(np.int64)
    sm = (ik[None] + iq[:, None]) % mk
    kqi_np = (sm[..., 0] * mk[1] * mk[2] + sm[..., 1] * mk[2] + sm[..., 2]).astype(np.int32)
    nk, nq, E = len(kc), len(qc), s.nm * s.nw * s.nw
    log(f"coarse workload: nk'={nk} nq'={nq} ne={s.ne} np={s.np_} E={E}, generated in "
        f"{time.perf_counter() - t_gen:.1f}s")
    ctx = ephw.Context(0)
    k = torch.from_numpy(kc).to("cuda:0")
    q = torch.from_numpy(qc).to("cuda:0")
    kqi = torch.from_numpy(kqi_np).to("cuda:0")
    # algorithmic flops: two band rotations per pair, the Re and Rp sums, the mode contraction
    flops = 8.0 * (2 * nk * nq * s.nm * s.nw ** 3 + s.ne * nq * E * nk + nq * s.ne * s.nm * s.nm * s.nw ** 2
                   + s.np_ * s.ne * E * nq)
    results = {}
    for prec, g_dtype, t_dtype in ((ephw.FP32, np.complex64, torch.complex64),
                                   (ephw.FP64, np.complex128, torch.complex128)):
        s.g = s.g.astype(g_dtype)
        sysh = ephw.System.from_synth(ctx, s)
        ks = ephw.KSet(sysh, k, prec)
        g_b = torch.empty((nq, nk, s.nm, s.nw, s.nw), dtype=t_dtype, device="cuda:0")
        ephw.interpolate(ks, q, kq_index=kqi, flags=ephw.OUT_G, g_out=g_b)
        out = torch.empty((s.np_, s.ne, s.nm, s.nw, s.nw), dtype=t_dtype, device="cuda:0")
        for _ in range(args.warmup):
            ephw.wannier_transform(ks, q, kqi, g_b, out)
        torch.cuda.synchronize()
        steps = args.steps if prec == ephw.FP32 else max(1, args.fp64_steps)
        t0 = time.perf_counter()
        for _ in range(steps):
            ephw.wannier_transform(ks, q, kqi, g_b, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ctx.check()
        ref = torch.from_numpy(s.g).to("cuda:0")
        err = float((out.to(torch.complex128) - ref.to(torch.complex128)).abs().max() / ref.abs().max())
        name = "fp32" if prec == ephw.FP32 else "fp64"
        results[name] = {"ms": dt * 1e3, "tflops": flops / dt / 1e12, "round_trip_error": err}
        log(f"{name}: {dt * 1e3:.2f} ms per transform, {flops / dt / 1e12:.1f} TFLOP/s algorithmic, "
            f"round-trip error {err:.2e}")
        ks.close()
        sysh.close()
        del g_b, out, ref
    f32 = results["fp32"]
    line = {
        "metric": "Bloch elements/s through Eq. (6) (FP32 MFMA path, coarse Bloch -> Wannier transform)",
        "value": nk * nq * E / (f32["ms"] * 1e-3), "unit": "elems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f32["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "coarse_si_nw8_nm6_re8x8x8_rp4x4x4_k8x8x8_q4x4x4", "nw": s.nw, "nm": s.nm,
                   "ne": s.ne, "np": s.np_, "nk": nk, "nq": nq},
        "roofline": {"bound": "mfma", "achieved": f32["tflops"], "peak": 157.3, "unit": "TFLOP/s",
                     "frac": f32["tflops"] / 157.3, "traffic": None, "kernel": "whole transform (GEMM-dominated)"},
        "algorithmic_flops_per_step": flops,
        "round_trip_error_fp32": f32["round_trip_error"],
        "fp64": results["fp64"],
        "fp32_vs_fp64_speedup": results["fp64"]["ms"] / f32["ms"],
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_window(args):
    """Energy-window prescreening on the dense-Si grids (8000 k x 8000 q, Nw 8,
    Nm 6, Ne = Np = 1000, FP32): the window takes the lowest tenth of the
    lowest band's energies.  Two forms of one step, each from the k-set's
    bands to g stored on the kept pairs: (1) pair lists: ephw_window_pairs,
    then Eq. (7) on the kept pairs only (ephw_interpolate_pairs, q chunks of
    the pair list); (2) compacted sets: ephw_window_screen, then Eq. (7) on
    every active k x active q pair with a mask of the kept ones.  Both against
    the same pass over the whole grids (the headline workload)."""
    import torch
    import synth
    from paper_2603_10295_amd import ephw, model
    w = synth.si_dense(m=args.grid)
    s = w.system
    nk, nq = len(w.k), len(w.q)
    E = s.nm * s.nw * s.nw
    ctx = ephw.Context(0)
    sysh = ephw.System.from_synth(ctx, s)
    k = torch.from_numpy(w.k).to("cuda:0")
    q = torch.from_numpy(w.q).to("cuda:0")
    kqi = torch.from_numpy(w.kq_index).to("cuda:0")
    ks = ephw.KSet(sysh, k, ephw.FP32)
    eps = torch.empty((nk, s.nw), dtype=torch.float64, device="cuda:0")
    ks.bands(eps)
    e0 = eps[:, 0].cpu().numpy()
    ks.close()
    lo, hi = float(e0.min()) - 1.0, float(np.quantile(e0, 0.1))

    def timed_steps(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ctx.check()
        return (time.perf_counter() - t0) / args.steps

    # ---- (1) pair lists ----------------------------------------------------
    ks_f = ephw.KSet(sysh, k, ephw.FP32)
    order, start, po, pkq, bands = ephw.window_pairs(ks_f, kqi, lo, hi, order=args.pair_order)
    ks_f.close()
    npairs = int(start[-1])
    if args.no_band_window:
        bands = (0, 0)
    b0, nb = bands[0], (bands[1] or s.nw)
    gp = torch.empty((max(npairs, 1), s.nm, nb, nb), dtype=torch.complex64, device="cuda:0")
    qc = min(args.q_chunk, nq)
    order_name = {ephw.PAIRS_BY_Q: "by q", ephw.PAIRS_BY_K: "by k"}[order]

    def step_pairs():
        ks_p = ephw.KSet(sysh, k, ephw.FP32)
        o, st, _, _, _ = ephw.window_pairs(ks_p, kqi, lo, hi, order=order, pair_other=po, pair_kq=pkq)
        if o == ephw.PAIRS_BY_K:
            # the whole list at once: every k's q are in one group
            ephw.interpolate_pairs(ks_p, q, o, st, po, pkq, flags=ephw.OUT_G, bands=bands, g_out=gp)
        else:
            for q0 in range(0, nq, qc):
                q1 = min(nq, q0 + qc)
                p0 = int(st[q0])
                ephw.interpolate_pairs(ks_p, q[q0:q1], o, st[q0:q1 + 1] - p0, po[p0:], pkq[p0:], q_offset=q0,
                                       flags=ephw.OUT_G, bands=bands, g_out=gp[p0:])
        ks_p.close()

    sysh.profile_read()
    sysh.profile(True)
    dt_pairs = timed_steps(step_pairs)
    sysh.profile(False)
    stages_pairs = {k_: round(v[0] / (args.steps + args.warmup), 3) for k_, v in sysh.profile_read().items()}
    log(f"pairs ({order_name}, bands {b0}..{b0 + nb - 1}): {npairs} kept of {nk * nq}; "
        f"{dt_pairs * 1e3:.1f} ms per pass; stages {stages_pairs}")

    # ---- (2) compacted sets with a pair mask -------------------------------
    k_out = torch.empty((nk, 3), dtype=torch.float64, device="cuda:0")
    q_out = torch.empty((nq, 3), dtype=torch.float64, device="cuda:0")
    kq_out = torch.empty((nq, nk), dtype=torch.int32, device="cuda:0")
    mask = torch.empty((nq, nk), dtype=torch.uint8, device="cuda:0")
    out = torch.empty((qc, nk, s.nm, s.nw, s.nw), dtype=torch.complex64, device="cuda:0")
    state = {}

    def step_masked():
        ks_m = ephw.KSet(sysh, k, ephw.FP32)
        nks, nqs = ephw.window_screen(ks_m, q, kqi, lo, hi, k_out, q_out, kq_out, mask)
        ks_m.close()
        kq2 = kq_out.reshape(-1)[:nqs * nks].reshape(nqs, nks)
        ks2 = ephw.KSet(sysh, k_out[:nks], ephw.FP32)
        for q0 in range(0, nqs, qc):
            q1 = min(nqs, q0 + qc)
            g = out.reshape(-1)[:(q1 - q0) * nks * E].reshape(q1 - q0, nks, s.nm, s.nw, s.nw)
            ephw.interpolate(ks2, q_out[q0:q1], kq_index=kq2[q0:q1].contiguous(), q_offset=q0, flags=ephw.OUT_G,
                             g_out=g)
        ks2.close()
        state.update(nks=nks, nqs=nqs)

    dt_masked = timed_steps(step_masked)
    nks, nqs = state["nks"], state["nqs"]
    kept = int(mask.reshape(-1)[:nqs * nks].sum().item())
    log(f"compacted sets: {nks}/{nk} k, {nqs}/{nq} q, {nks * nqs} pairs computed, {kept} kept; "
        f"{dt_masked * 1e3:.1f} ms per pass")
    del out

    # parity of the pair path on two q against the oracle (kept pairs only)
    import oracle
    # every pair's (q, k) from the list, then all kept pairs of two q
    other = po[:npairs].cpu().numpy()
    major = np.repeat(np.arange(len(start) - 1), np.diff(start))
    pair_q, pair_k = (major, other) if order == ephw.PAIRS_BY_Q else (other, major)
    pick = [int(pair_q.min()), int(np.median(pair_q))]
    pick = sorted(set(pick))
    sel_p = np.flatnonzero(np.isin(pair_q, pick))
    sel_q, sel_k = pair_q[sel_p], pair_k[sel_p]
    got = gp[torch.as_tensor(sel_p, device="cuda:0")].cpu().numpy().astype(np.complex128)
    ref = oracle.interpolate(s, w.k, w.q[pick], return_all=True)
    qpos = {j: i for i, j in enumerate(pick)}
    s_gpu, s_ref = [], []
    bs = slice(b0, b0 + nb)   # the band window's block (its edges lie in gaps of the spectrum)
    for p_, (a, b) in enumerate(zip(sel_q, sel_k)):
        a = qpos[a]
        s_gpu += oracle.block_sums(np.abs(got[p_])[None, None] ** 2, ref["eps_kq"][a, b][bs][None, None],
                                   ref["eps_k"][b][bs][None], ref["lam"][a][None])
        s_ref += oracle.block_sums(np.abs(ref["ghat"][a, b][:, bs, bs])[None, None] ** 2,
                                   ref["eps_kq"][a, b][bs][None, None], ref["eps_k"][b][bs][None],
                                   ref["lam"][a][None])
    err = oracle.compare_block_sums(s_gpu, s_ref)
    log(f"kept pairs of {len(pick)} q vs oracle: normwise {err[0]:.2e}, max blockwise {err[1]:.2e}")
    line = {
        "metric": "full-grid g(k,q) elems/s covered by the energy-window pass (FP32 MFMA path)",
        "value": nk * nq * E / dt_pairs, "unit": "elems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt_pairs * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"si_dense_window_nw8_nm6_ne1000_{nk}kx{nq}q_lowest10pct_band0", "nk": nk, "nq": nq,
                   "window": [lo, hi],
                   "form": f"pair lists grouped {order_name} (ephw_window_pairs + ephw_interpolate_pairs)",
                   "band_window": [b0, nb]},
        "kept_pairs": npairs, "computed_pairs": npairs, "kept_elems_per_s": npairs * E / dt_pairs,
        "stages_ms_per_step": stages_pairs,
        "compacted_sets": {"ms_per_step": dt_masked * 1e3, "active_k": nks, "active_q": nqs,
                           "computed_pairs": nks * nqs, "kept_pairs": kept},
        "pairs_vs_compacted_sets_speedup": dt_masked / dt_pairs,
        "err_vs_oracle_kept_pairs": {"normwise": err[0], "max_blockwise": err[1], "sample_q": len(pick)},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_linewidth(args):
    """The downstream reduction on the dense-Si grids (8000 k x 8000 q, FP32),
    two ways: fused (ephw_interpolate_linewidth: the band rotations and the
    linewidth terms in the Eq. (10) GEMM's epilogue, g never stored) and
    stored (per q chunk, Eq. (7) stores g and ephw_linewidth reduces it).
    Both gammas are compared; the fused pass is the headline of the line."""
    import torch
    import synth
    from paper_2603_10295_amd import ephw, model
    w = synth.si_dense(m=args.grid)
    s = w.system
    nk, nq = len(w.k), len(w.q)
    ctx = ephw.Context(0)
    sysh = ephw.System.from_synth(ctx, s)
    k = torch.from_numpy(w.k).to("cuda:0")
    q = torch.from_numpy(w.q).to("cuda:0")
    kqi = torch.from_numpy(w.kq_index).to("cuda:0")
    qc = min(args.q_chunk, nq)
    eps_k = torch.empty((nk, s.nw), dtype=torch.float64, device="cuda:0")
    gamma = torch.zeros((nk, s.nw), dtype=torch.float64, device="cuda:0")
    ks0 = ephw.KSet(sysh, k, ephw.FP32)
    ks0.bands(eps_k)
    e = eps_k.cpu().numpy()
    ks0.close()
    temp, mu, sigma = 0.02 * float(np.ptp(e)), float(np.median(e)), 0.01 * float(np.ptp(e))
    cnt = model.stage_counts(s.nw, s.nm, s.ne, s.np_, nk, nq, nh=len(s.r_h), kq_on_grid=True)

    def fused_step():
        gamma.zero_()
        ks = ephw.KSet(sysh, k, ephw.FP32)
        for q0 in range(0, nq, qc):
            q1 = min(nq, q0 + qc)
            ephw.interpolate_linewidth(ks, q[q0:q1], gamma, kq_index=kqi[q0:q1], temperature=temp, mu=mu,
                                       sigma=sigma, nq_total=nq)
        ks.close()

    for _ in range(args.warmup):
        fused_step()
    torch.cuda.synchronize()
    sysh.profile_read()
    sysh.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fused_step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.check()
    stages = sysh.profile_read()
    sysh.profile(False)
    gamma_fused = gamma.cpu().numpy()
    re_ms, re_n = stages["re_gemm"]
    re_tflops = 8.0 * cnt.re * args.steps / (re_ms * 1e-3) / 1e12
    log(f"fused pass {dt * 1e3:.1f} ms (Re GEMM with rotations and linewidth terms {re_ms / args.steps:.1f} ms)")

    # the stored-g reference: Eq. (7) per q chunk into g, then ephw_linewidth
    g = torch.empty((qc, nk, s.nm, s.nw, s.nw), dtype=torch.complex64, device="cuda:0")
    ekq = torch.empty((qc, nk, s.nw), dtype=torch.float64, device="cuda:0")
    om = torch.empty((qc, s.nm), dtype=torch.float64, device="cuda:0")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    lw_ms = []

    def stored_step():
        gamma.zero_()
        ks = ephw.KSet(sysh, k, ephw.FP32)
        t = 0.0
        for q0 in range(0, nq, qc):
            q1 = min(nq, q0 + qc)
            b = q1 - q0
            ephw.interpolate(ks, q[q0:q1], kq_index=kqi[q0:q1], q_offset=q0, flags=ephw.OUT_G, g_out=g[:b],
                             eps_kq=ekq[:b], omega=om[:b])
            ev[0].record()
            ephw.linewidth(ephw.FP32, g[:b], eps_k, ekq[:b], om[:b], gamma, temperature=temp, mu=mu, sigma=sigma,
                           nq_total=nq)
            ev[1].record()
            ev[1].synchronize()
            t += ev[0].elapsed_time(ev[1])
        ks.close()
        lw_ms.append(t)

    stored_step()
    torch.cuda.synchronize()
    lw_ms.clear()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        stored_step()
    torch.cuda.synchronize()
    dt_stored = (time.perf_counter() - t0) / max(1, args.steps // 2)
    ctx.check()
    gamma_stored = gamma.cpu().numpy()
    lw = sum(lw_ms) / len(lw_ms)
    diff = float(np.abs(gamma_fused - gamma_stored).max() / np.abs(gamma_stored).max())
    E = s.nm * s.nw * s.nw
    elems = nk * nq * E
    log(f"stored-g pass {dt_stored * 1e3:.1f} ms, of which the linewidth reduction {lw:.1f} ms; "
        f"fused vs stored gamma: {diff:.2e} of the largest")
    line = {
        "metric": "g(k,q) elems/s reduced into linewidths (FP32 MFMA interpolation, rotations and "
                  "FP64-weighted reduction fused, g not stored)",
        "value": elems / dt, "unit": "elems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"si_dense_linewidth_nw8_nm6_ne1000_{nk}kx{nq}q", "nk": nk, "nq": nq,
                   "temperature": temp, "mu": mu, "sigma": sigma, "q_chunk": qc},
        "roofline": {"bound": "mfma", "achieved": re_tflops, "peak": model.PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": re_tflops / model.PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "cgemm_kernel<float> Re phase sum (Eq. 10) with the band rotations and linewidth "
                               "terms in its epilogue (Re-sum flops credited only)",
                     "avg_launch_ms": re_ms / max(1, re_n), "launches": re_n},
        "stages_ms_per_step": {k_: round(v[0] / args.steps, 3) for k_, v in stages.items()},
        "stored_g": {"ms_per_step": dt_stored * 1e3, "linewidth_ms_per_step": lw,
                     "linewidth_read_GBps": elems * 8 / (lw * 1e-3) / 1e9},
        "fused_vs_stored_gamma_rel": diff,
        "gamma_norm": float(np.linalg.norm(gamma_fused)),
    }
    print(json.dumps(line), flush=True)
    return 0


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards over q across GPUs by design, see the design notes)", file=sys.stderr)
        return 2
    if args.workload == "ribbon":
        return bench_ribbon(args)
    if args.workload == "batch32":
        return bench_batch(args)
    if args.workload == "coarse_si":
        return bench_coarse(args)
    if args.workload == "si_window":
        return bench_window(args)
    if args.workload == "si_linewidth":
        return bench_linewidth(args)
    import torch
    from paper_2603_10295_amd import ephw, model
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2

    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * 2 ** 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 4} bytes read and written")
        del src, dst

    t_gen = time.perf_counter()
    w = workload(args)
    s = w.system
    nk, nq = len(w.k), len(w.q)
    log(f"workload {w.name}: nk={nk} nq={nq} nw={s.nw} nm={s.nm} ne={s.ne} np={s.np_} "
        f"(generated in {time.perf_counter() - t_gen:.1f}s)")
    k = torch.from_numpy(w.k).to("cuda:0")
    q = torch.from_numpy(w.q).to("cuda:0")
    kqi = torch.from_numpy(w.kq_index).to("cuda:0") if w.kq_index is not None else None
    ctx = ephw.Context(0)
    cnt = model.stage_counts(s.nw, s.nm, s.ne, s.np_, nk, nq, nh=len(s.r_h), kq_on_grid=w.kq_index is not None)

    # ---- FP32 MFMA path (the headline) -----------------------------------
    p32 = Path(ctx, s, ephw.FP32, k, q, kqi, args.q_chunk, args.q_batch)
    log("FP32 path: warmup + timed steps")
    t32, stages = timed(p32, args.steps, args.warmup, profile=True)
    v32 = cnt.elems / t32
    log(f"FP32: {t32 * 1e3:.1f} ms/step, {v32:.4e} elems/s")
    re_ms, re_n = stages["re_gemm"]
    qb32 = min(128, nq)
    re_wg = -(-nk // 128) * -(-(qb32 * s.nm * s.nw * s.nw) // 128)   # workgroups of a full-batch Re GEMM
    # with the band rotations in the Re-sum GEMM's epilogue (no separate
    # rotation launches) the dominant kernel also does the rotation flops
    fused = stages["band_rot"][1] == 0
    re_flops = 8.0 * (cnt.re + (cnt.rot if fused else 0.0)) * args.steps
    re_tflops = re_flops / (re_ms * 1e-3) / 1e12
    # algorithmic HBM bytes of one full-batch launch: the phase rows P_k and
    # G_nu read once, g stored (the fused kernel) or W stored (unfused)
    E = s.nm * s.nw * s.nw
    algo_bytes = 8.0 * (nk * s.ne + s.ne * qb32 * E + nk * qb32 * E)
    rp_ms, rp_n = stages["rp_gemm"]
    rp_tflops = 8.0 * cnt.rp * args.steps / (rp_ms * 1e-3) / 1e12
    gemm_tflops = 8.0 * cnt.gemm * args.steps / ((re_ms + rp_ms) * 1e-3) / 1e12

    # ---- oracle sample: CPU baseline and the error of the GPU paths -------
    rng = np.random.default_rng(1234)
    qs_idx = np.sort(rng.choice(nq, size=min(args.cpu_sample_q, nq), replace=False))
    cpu = None
    err32 = err64 = None
    if not args.no_cpu_baseline:
        log(f"oracle on {len(qs_idx)} q x {nk} k")
        c_val, c_dt, ref, threads = cpu_baseline(w, qs_idx)
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": c_val, "unit": "elems/s", "cores": cores, "blas_threads": threads, "kind": "oracle",
               "seconds": round(c_dt, 2),
               "sample": f"{len(qs_idx)} q (of {nq}) x all {nk} k of the same workload, "
                         f"NumPy complex128 + LAPACK eigh, nested loop Eqs. (9)-(10)"}
        log(f"oracle: {c_val:.4e} elems/s in {c_dt:.1f}s")
        if args.cpu_one_thread_q > 0:
            # the same oracle on one host thread (BLAS limited to 1), smaller sample
            from threadpoolctl import threadpool_limits
            q1 = qs_idx[:args.cpu_one_thread_q]
            with threadpool_limits(limits=1):
                v1, dt1, _, _ = cpu_baseline(w, q1)
            cpu["one_thread"] = {"value": v1, "unit": "elems/s", "seconds": round(dt1, 2),
                                 "sample": f"{len(q1)} q x all {nk} k, BLAS limited to 1 thread"}
            log(f"oracle, 1 thread: {v1:.4e} elems/s in {dt1:.1f}s")
        g32 = p32.sample(qs_idx)
        err32 = block_error(g32, ref)
        log(f"FP32 vs oracle: normwise {err32[0]:.2e}, max blockwise {err32[1]:.2e}, scaled {err32[2]:.2e}")

    # ---- compensated FP32: K-blocked accumulation in the phase GEMMs ------
    comp = None
    if not args.no_comp:
        del p32.out
        pc = Path(ctx, s, ephw.FP32_COMP, k, q, kqi, args.q_chunk, args.q_batch)
        log("compensated FP32 path: warmup + timed steps")
        tc, stc = timed(pc, args.comp_steps, 1 if args.warmup else 0, profile=True)
        comp = {"value": cnt.elems / tc, "ms_per_step": tc * 1e3,
                "re_gemm_ms_per_step": round(stc["re_gemm"][0] / args.comp_steps, 3),
                "note": "both phase GEMMs accumulate in K blocks of 32 (fresh FP32 MFMA accumulators per "
                        "block, block sums added in FP32); g stored, band rotations unfused"}
        log(f"compensated FP32: {tc * 1e3:.1f} ms/step")
        if cpu is not None:
            e = block_error(pc.sample(qs_idx), ref)
            comp["err_vs_oracle"] = {"normwise": e[0], "max_blockwise": e[1], "max_scaled_blockwise": e[2]}
            log(f"compensated FP32 vs oracle: normwise {e[0]:.2e}, max blockwise {e[1]:.2e}, scaled {e[2]:.2e}")
        del pc.out
        pc.sys.close()

    # ---- FP64 path on the same values (complex64 g upcast) ----------------
    fp64 = None
    if not args.no_fp64:
        if hasattr(p32, "out"):
            del p32.out
        s64 = type(s)(**{**s.__dict__, "g": s.g.astype(np.complex128)})
        p64 = Path(ctx, s64, ephw.FP64, k, q, kqi, args.q_chunk, args.q_batch)
        log("FP64 path: warmup + timed steps")
        t64, st64 = timed(p64, args.fp64_steps, 1 if args.warmup else 0, profile=True)
        fp64 = {"value": cnt.elems / t64, "ms_per_step": t64 * 1e3,
                "re_gemm_tflops": 8.0 * cnt.re * args.fp64_steps / (st64["re_gemm"][0] * 1e-3) / 1e12,
                "rp_gemm_tflops": 8.0 * cnt.rp * args.fp64_steps / (st64["rp_gemm"][0] * 1e-3) / 1e12,
                "stages_ms": {k_: round(v[0] / args.fp64_steps, 3) for k_, v in st64.items()}}
        log(f"FP64: {t64 * 1e3:.1f} ms/step")
        if cpu is not None:
            g64 = p64.sample(qs_idx)
            err64 = block_error(g64, ref)
            fp64["err_vs_oracle"] = {"normwise": err64[0], "max_blockwise": err64[1],
                                     "max_scaled_blockwise": err64[2]}
        p64.sys.close()

    line = {
        "metric": "g(k,q) elems/s (FP32 MFMA path)",
        "value": v32,
        "unit": "elems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": w.name, "nw": s.nw, "nm": s.nm, "ne": s.ne, "np": s.np_, "nk": nk, "nq": nq,
                   "g_dtype": "complex64", "eig": "fp64", "output": "g stored complex64, q-chunked",
                   "q_chunk": p32.q_chunk},
        "roofline": {"bound": "mfma", "achieved": re_tflops, "peak": model.PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": re_tflops / model.PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic("cgemm_kernel<float", re_wg),
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes": algo_bytes,
                     "kernel": "cgemm_kernel<float> Re phase sum (Eq. 10)"
                               + (" with the band rotations and the g store in its epilogue" if fused else ""),
                     "flops_per_launch": re_flops / max(1, re_n), "avg_launch_ms": re_ms / max(1, re_n),
                     "launches": re_n},
        "cpu_baseline": cpu,
        "phase_gemm_tflops": {"re": re_tflops, "rp": rp_tflops, "both": gemm_tflops,
                              "frac_of_fp32_peak": gemm_tflops / model.PEAK_FP32_TFLOPS},
        "stages_ms_per_step": {k_: round(v[0] / args.steps, 3) for k_, v in stages.items()},
        "err_vs_oracle": None if err32 is None else {"normwise": err32[0], "max_blockwise": err32[1],
                                                     "max_scaled_blockwise": err32[2],
                                                     "sample_q": len(qs_idx)},
        "fp64_gpu": fp64,
        "fp32_vs_fp64_speedup": None if fp64 is None else fp64["ms_per_step"] / (t32 * 1e3),
        "fp32_comp": comp,
        "fp32_comp_vs_fp64_speedup": None if (fp64 is None or comp is None)
        else fp64["ms_per_step"] / comp["ms_per_step"],
        "algorithmic_flops_per_step": 8.0 * cnt.total,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
