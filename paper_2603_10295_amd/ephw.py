"""ctypes binding of libephw (include/ephw.h).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch tensors on a ROCm device (their ``data_ptr()`` is passed
through); the stream is torch's current stream unless one is given.  If the
shared library is missing, importing the binding succeeds but every call
raises ``EphwError`` - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EPHW_LIB", os.path.join(_HERE, "libephw.so"))

# status codes, precisions, flags (mirror include/ephw.h)
OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EUNSUPPORTED, EINDEX = range(7)
FP64, FP32, FP32_COMP = 0, 1, 2
PAIRS_BY_Q, PAIRS_BY_K, PAIRS_AUTO = 0, 1, -1
C128, C64 = 0, 1
OUT_G, OUT_BAND_SUM, OUT_LOSS, OUT_WANNIER = 1, 2, 4, 8

EXPORTS = [
    "ephw_ctx_create", "ephw_ctx_destroy", "ephw_ctx_check", "ephw_ctx_set_limits", "ephw_ctx_memory", "ephw_system_load",
    "ephw_system_free", "ephw_system_set_g", "ephw_system_trim", "ephw_system_bytes", "ephw_bands", "ephw_phonons", "ephw_phase_sum_rp",
    "ephw_kset_create", "ephw_kset_free", "ephw_kset_bands", "ephw_interpolate", "ephw_interpolate_noalloc", "ephw_interpolate_linewidth", "ephw_degenerate_sums", "ephw_wannier_transform",
    "ephw_window_screen", "ephw_window_pairs", "ephw_interpolate_pairs", "ephw_linewidth",
    "ephw_loss_backward", "ephw_set_q_batch", "ephw_set_k_tile", "ephw_profile_enable", "ephw_profile_read", "ephw_batch_create",
    "ephw_batch_run", "ephw_batch_shape", "ephw_batch_stats", "ephw_batch_solo", "ephw_batch_free", "ephw_status_string",
    "ephw_last_error", "ephw_version",
]

STAGES = ["phase", "eig", "kq_eig", "rp_gemm", "mode_rot", "re_gemm", "band_rot", "other"]


class EphwError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: status {status} ({_status_name(status)}) {detail}".strip())


def _status_name(s: int) -> str:
    names = {OK: "ok", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOCONV: "ENOCONV",
             EUNSUPPORTED: "EUNSUPPORTED", EINDEX: "EINDEX"}
    return names.get(s, "unknown")


class SystemDesc(ctypes.Structure):
    _fields_ = [
        ("nw", ctypes.c_int32), ("na", ctypes.c_int32),
        ("ne", ctypes.c_int64), ("np", ctypes.c_int64), ("nh", ctypes.c_int64), ("nc", ctypes.c_int64),
        ("r_e", ctypes.c_void_p), ("r_p", ctypes.c_void_p), ("r_h", ctypes.c_void_p), ("r_c", ctypes.c_void_p),
        ("w_e", ctypes.c_void_p), ("w_p", ctypes.c_void_p), ("w_h", ctypes.c_void_p), ("w_c", ctypes.c_void_p),
        ("h_r", ctypes.c_void_p), ("c_r", ctypes.c_void_p), ("mass", ctypes.c_void_p), ("g", ctypes.c_void_p),
        ("g_dtype", ctypes.c_int32),
    ]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("ks", ctypes.c_void_p), ("q", ctypes.c_void_p), ("nq", ctypes.c_int64),
        ("kq_index", ctypes.c_void_p), ("flags", ctypes.c_uint32), ("g_out", ctypes.c_void_p),
        ("band_sum", ctypes.c_void_p), ("loss", ctypes.c_void_p), ("loss_seed", ctypes.c_uint64),
    ]


class BatchOptions(ctypes.Structure):
    _fields_ = [("tune", ctypes.c_int32), ("tune_cache", ctypes.c_char_p), ("use_graph", ctypes.c_int32),
                ("item_workspace_bytes", ctypes.c_int64), ("workspace_budget_bytes", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libephw.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise EphwError(EDEVICE, "load", f"{LIB_PATH} not found; run `python -m paper_2603_10295_amd.build`")
    # torch bundles its own HIP runtime under the same soname as ROCm's; loading
    # torch first makes libephw bind to that one runtime instead of a second copy
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "ephw_ctx_create": [ctypes.c_int, pp],
        "ephw_ctx_destroy": [vp],
        "ephw_ctx_check": [vp, vp],
        "ephw_ctx_set_limits": [vp, i64, i32],
        "ephw_ctx_memory": [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
        "ephw_system_load": [vp, ctypes.POINTER(SystemDesc), pp],
        "ephw_system_free": [vp],
        "ephw_system_set_g": [vp, vp, vp],
        "ephw_system_trim": [vp],
        "ephw_system_bytes": [vp, ctypes.POINTER(ctypes.c_int64)],
        "ephw_bands": [vp, vp, i64, vp, vp, vp],
        "ephw_phonons": [vp, vp, i64, vp, vp, vp, vp],
        "ephw_phase_sum_rp": [vp, vp, i64, i32, vp, vp],
        "ephw_kset_create": [vp, vp, i64, i32, vp, pp],
        "ephw_kset_free": [vp],
        "ephw_kset_bands": [vp, vp, vp, vp],
        "ephw_interpolate": [vp, vp, i64, vp, i64, i32, u32, vp, vp, vp, u64, vp, vp, vp],
        "ephw_interpolate_noalloc": [vp, vp, i64, vp, i64, i32, u32, vp, vp, vp, u64, vp, vp, vp],
        "ephw_interpolate_linewidth": [vp, vp, i64, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, i64, vp, vp],
        "ephw_degenerate_sums": [i32, vp, i64, i64, i32, i32, vp, vp, vp, ctypes.c_double, vp, vp],
        "ephw_wannier_transform": [vp, vp, i64, vp, vp, vp, vp],
        "ephw_linewidth": [i32, vp, i64, i64, i32, i32, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, i64, vp, vp],
        "ephw_window_screen": [vp, vp, i64, vp, ctypes.c_double, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_int64),
                               vp, ctypes.POINTER(ctypes.c_int64), vp, vp, vp],
        "ephw_window_pairs": [vp, vp, i64, ctypes.c_double, ctypes.c_double, i32, vp, vp, vp, vp, i64, vp, vp],
        "ephw_interpolate_pairs": [vp, vp, i64, i32, vp, vp, vp, i64, i32, u32, i32, i32, vp, vp, vp, u64, vp],
        "ephw_set_q_batch": [vp, i32],
        "ephw_set_k_tile": [vp, i32],
        "ephw_loss_backward": [vp, vp, i64, vp, i64, u64, vp, vp, vp, vp, vp],
        "ephw_profile_enable": [vp, i32],
        "ephw_profile_read": [vp, vp, vp],
        "ephw_batch_create": [vp, ctypes.POINTER(BatchItem), i32, ctypes.POINTER(BatchOptions), vp, pp],
        "ephw_batch_run": [vp, vp],
        "ephw_batch_shape": [vp, i32, vp, vp, vp, vp],
        "ephw_batch_stats": [vp, vp, vp],
        "ephw_batch_solo": [vp, i32, vp],
        "ephw_batch_free": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.ephw_status_string.argtypes = [ctypes.c_int32]
    L.ephw_status_string.restype = ctypes.c_char_p
    L.ephw_last_error.argtypes = []
    L.ephw_last_error.restype = ctypes.c_char_p
    L.ephw_version.argtypes = []
    L.ephw_version.restype = ctypes.c_int32
    _lib = L
    return L


def _check(status: int, where: str):
    if status != OK:
        detail = lib().ephw_last_error().decode(errors="replace")
        raise EphwError(status, where, detail)


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return t.data_ptr()


def _g_shape(prec: int, g, where: str):
    """(nq, nk, nm, nw) of a stored g [nq][nk][nm][nw][nw], after checking that
    its element type is the one `prec` reads (c128 at FP64, c64 otherwise):
    the kernels size their reads from prec, not from the tensor."""
    import torch
    want = torch.complex128 if prec == FP64 else torch.complex64
    if g.dtype != want:
        raise ValueError(f"{where}: g is {g.dtype}, precision {prec} reads {want}")
    if g.dim() != 5 or g.shape[3] != g.shape[4]:
        raise ValueError(f"{where}: g must be [nq][nk][nm][nw][nw], got {tuple(g.shape)}")
    return g.shape[0], g.shape[1], g.shape[2], g.shape[3]


def _expect(t, shape, name: str):
    """A float64 device buffer of the given shape."""
    import torch
    if t.dtype != torch.float64 or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be float64 {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ----------------------------------------------------------------------------
# thin object wrappers over the handles
# ----------------------------------------------------------------------------

class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().ephw_ctx_create(device, ctypes.byref(h)), "ephw_ctx_create")
        self.handle = h
        self.device = device

    def check(self, stream=None):
        _check(lib().ephw_ctx_check(self.handle, _stream(stream)), "ephw_ctx_check")

    def set_limits(self, max_device_bytes: int = 0, max_sweeps: int = 40):
        """Cap the device memory the context's objects may hold (0 = none) and
        the Jacobi sweeps per eigensolve (see ephw_ctx_set_limits)."""
        _check(lib().ephw_ctx_set_limits(self.handle, int(max_device_bytes), int(max_sweeps)), "ephw_ctx_set_limits")

    def memory(self):
        """(bytes held by the context's objects, cap or 0)"""
        u, l = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ephw_ctx_memory(self.handle, ctypes.byref(u), ctypes.byref(l)), "ephw_ctx_memory")
        return u.value, l.value

    def close(self):
        if self.handle:
            lib().ephw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host(a, dtype):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dtype)


class System:
    """Library-owned device copy of a Wannier-space system (host numpy inputs)."""

    def __init__(self, ctx: Context, *, nw, na, r_e, r_p, r_h, r_c, h_r, c_r, mass, g,
                 w_e=None, w_p=None, w_h=None, w_c=None, g_dtype=None):
        """g None: the device copy is allocated but not written (fill it with
        set_g); g_dtype (C128 or C64) then gives its element type."""
        g_arr = None if g is None else np.asarray(g)
        if g_arr is None:
            if g_dtype not in (C128, C64):
                raise ValueError("without g, g_dtype must be C128 or C64")
            gdt = g_dtype
        elif g_arr.dtype == np.complex128:
            gdt = C128
        elif g_arr.dtype == np.complex64:
            gdt = C64
        else:
            raise ValueError("g must be complex128 or complex64")
        keep = dict(
            r_e=_host(r_e, np.int32), r_p=_host(r_p, np.int32), r_h=_host(r_h, np.int32),
            r_c=_host(r_c, np.int32), w_e=_host(w_e, np.float64), w_p=_host(w_p, np.float64),
            w_h=_host(w_h, np.float64), w_c=_host(w_c, np.float64),
            h_r=_host(h_r, np.complex128), c_r=_host(c_r, np.float64), mass=_host(mass, np.float64),
            g=None if g_arr is None else np.ascontiguousarray(g_arr))
        d = SystemDesc()
        d.nw, d.na = int(nw), int(na)
        d.ne, d.np, d.nh, d.nc = (len(keep["r_e"]), len(keep["r_p"]), len(keep["r_h"]), len(keep["r_c"]))
        for name in ("r_e", "r_p", "r_h", "r_c", "w_e", "w_p", "w_h", "w_c", "h_r", "c_r", "mass", "g"):
            arr = keep[name]
            setattr(d, name, None if arr is None else arr.ctypes.data)
        d.g_dtype = gdt
        h = ctypes.c_void_p()
        _check(lib().ephw_system_load(ctx.handle, ctypes.byref(d), ctypes.byref(h)), "ephw_system_load")
        self.handle = h
        self.ctx = ctx
        self.nw, self.na, self.nm = int(nw), int(na), 3 * int(na)
        self.ne, self.np, self.nh, self.nc = d.ne, d.np, d.nh, d.nc
        self.g_dtype = gdt

    @classmethod
    def from_synth(cls, ctx: Context, s, g_dtype=None) -> "System":
        return cls(ctx, nw=s.nw, na=s.na, r_e=s.r_e, r_p=s.r_p, r_h=s.r_h, r_c=s.r_c, h_r=s.h_r,
                   c_r=s.c_r, mass=s.mass, g=s.g, w_e=s.w_e, w_p=s.w_p, w_h=s.w_h, w_c=s.w_c, g_dtype=g_dtype)

    def trim(self):
        """Release the system's workspaces (see ephw_system_trim)."""
        _check(lib().ephw_system_trim(self.handle), "ephw_system_trim")

    def set_g(self, g, stream=None):
        """Copy a device tensor (same shape/dtype as the loaded g) into the system."""
        _check(lib().ephw_system_set_g(self.handle, _ptr(g), _stream(stream)), "ephw_system_set_g")

    def bytes(self) -> int:
        v = ctypes.c_int64()
        _check(lib().ephw_system_bytes(self.handle, ctypes.byref(v)), "ephw_system_bytes")
        return v.value

    def set_q_batch(self, qb: int):
        _check(lib().ephw_set_q_batch(self.handle, int(qb)), "ephw_set_q_batch")

    def set_k_tile(self, kt: int):
        _check(lib().ephw_set_k_tile(self.handle, int(kt)), "ephw_set_k_tile")

    def profile(self, enable: bool):
        _check(lib().ephw_profile_enable(self.handle, 1 if enable else 0), "ephw_profile_enable")

    def profile_read(self) -> dict:
        """{stage: (milliseconds, launches)} summed since the last read."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(lib().ephw_profile_read(self.handle, ms, n), "ephw_profile_read")
        return {s: (ms[i], int(n[i])) for i, s in enumerate(STAGES)}

    def close(self):
        if self.handle:
            lib().ephw_system_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bands(sys: System, k, eps=None, vecs=None, stream=None):
    _check(lib().ephw_bands(sys.handle, _ptr(k), k.shape[0], _ptr(eps), _ptr(vecs), _stream(stream)),
           "ephw_bands")


def phonons(sys: System, q, lam=None, omega=None, evecs=None, stream=None):
    _check(lib().ephw_phonons(sys.handle, _ptr(q), q.shape[0], _ptr(lam), _ptr(omega), _ptr(evecs),
                              _stream(stream)), "ephw_phonons")


def phase_sum_rp(sys: System, q, prec: int, out, stream=None):
    _check(lib().ephw_phase_sum_rp(sys.handle, _ptr(q), q.shape[0], prec, _ptr(out), _stream(stream)),
           "ephw_phase_sum_rp")


class KSet:
    def __init__(self, sys: System, k, prec: int, stream=None):
        h = ctypes.c_void_p()
        _check(lib().ephw_kset_create(sys.handle, _ptr(k), k.shape[0], prec, _stream(stream), ctypes.byref(h)),
               "ephw_kset_create")
        self.handle = h
        self.sys = sys
        self.nk = k.shape[0]
        self.prec = prec

    def bands(self, eps=None, vecs=None, stream=None):
        _check(lib().ephw_kset_bands(self.handle, _ptr(eps), _ptr(vecs), _stream(stream)), "ephw_kset_bands")

    def close(self):
        if self.handle:
            lib().ephw_kset_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def interpolate(ks: KSet, q, *, kq_index=None, q_offset: int = 0, flags: int = OUT_G, g_out=None,
                band_sum=None, loss=None, loss_seed: int = 0, eps_kq=None, omega=None, stream=None):
    _check(lib().ephw_interpolate(ks.handle, _ptr(q), q.shape[0], _ptr(kq_index), int(q_offset), ks.prec,
                                  int(flags), _ptr(g_out), _ptr(band_sum), _ptr(loss), int(loss_seed),
                                  _ptr(eps_kq), _ptr(omega), _stream(stream)), "ephw_interpolate")


def interpolate_noalloc(ks: KSet, q, *, kq_index=None, q_offset: int = 0, flags: int = OUT_G, g_out=None,
                        band_sum=None, loss=None, loss_seed: int = 0, eps_kq=None, omega=None, stream=None):
    """ephw_interpolate with every intermediate in the library's static scratch
    (no device allocation; see ephw_interpolate_noalloc)."""
    _check(lib().ephw_interpolate_noalloc(ks.handle, _ptr(q), q.shape[0], _ptr(kq_index), int(q_offset), ks.prec,
                                          int(flags), _ptr(g_out), _ptr(band_sum), _ptr(loss), int(loss_seed),
                                          _ptr(eps_kq), _ptr(omega), _stream(stream)), "ephw_interpolate_noalloc")


def interpolate_linewidth(ks: KSet, q, gamma, *, kq_index=None, temperature: float, mu: float, sigma: float,
                          omega_min: float = 0.0, nq_total: int = 0, stream=None):
    """gamma[k][n] += the linewidth terms of Eq. (7)'s g for the k-set and q
    list, with g never stored (see ephw_interpolate_linewidth); nq_total
    defaults to this call's q count."""
    _expect(gamma, (ks.nk, ks.sys.nw), "gamma")
    _check(lib().ephw_interpolate_linewidth(ks.handle, _ptr(q), q.shape[0], _ptr(kq_index), float(temperature),
                                            float(mu), float(sigma), float(omega_min), int(nq_total or q.shape[0]),
                                            _ptr(gamma), _stream(stream)), "ephw_interpolate_linewidth")


def window_screen(ks: KSet, q, kq_index, e_lo: float, e_hi: float, k_out, q_out, kq_out, pair_mask=None,
                  stream=None):
    """Active k and q points of an energy window (see ephw_window_screen);
    returns (nk_active, nq_active).  Synchronises the stream."""
    nk = ctypes.c_int64(0)
    nq = ctypes.c_int64(0)
    _check(lib().ephw_window_screen(ks.handle, _ptr(q), q.shape[0], _ptr(kq_index), float(e_lo), float(e_hi),
                                    _ptr(k_out), ctypes.byref(nk), _ptr(q_out), ctypes.byref(nq), _ptr(kq_out),
                                    _ptr(pair_mask), _stream(stream)), "ephw_window_screen")
    return nk.value, nq.value


def window_pairs(ks: KSet, kq_index, e_lo: float, e_hi: float, order: int = PAIRS_AUTO, pair_other=None,
                 pair_kq=None, stream=None):
    """Kept (k, q) pairs of an energy window as CSR lists (see
    ephw_window_pairs).  Returns (order, pair_start, pair_other, pair_kq,
    band_range): the grouping used, a host int64 array of group offsets, int32
    device tensors (the other index of each pair, the k+q index), allocated
    here when not given or too small, and (first band, band count) of the
    window's bands.  Synchronises the stream."""
    import numpy as np
    import torch
    nq = kq_index.shape[0]
    start = np.zeros(max(nq, ks.nk) + 1, dtype=np.int64)
    cap = 0 if pair_other is None else min(pair_other.numel(), pair_kq.numel())
    used = ctypes.c_int32(-2)
    bands = (ctypes.c_int32 * 2)(0, 0)

    def call(cap_, po, pkq):
        return lib().ephw_window_pairs(ks.handle, _ptr(kq_index), nq, float(e_lo), float(e_hi), int(order),
                                       ctypes.byref(used), start.ctypes.data_as(ctypes.c_void_p), _ptr(po),
                                       _ptr(pkq), cap_, bands, _stream(stream))
    st = call(cap, pair_other, pair_kq)
    n = ks.nk if used.value == PAIRS_BY_K else nq
    total = int(start[n])
    if st == EINVAL and total > cap:
        pair_other = torch.empty(max(total, 1), dtype=torch.int32, device=kq_index.device)
        pair_kq = torch.empty(max(total, 1), dtype=torch.int32, device=kq_index.device)
        st = call(total, pair_other, pair_kq)
    _check(st, "ephw_window_pairs")
    if pair_other is None:
        pair_other = torch.empty(0, dtype=torch.int32, device=kq_index.device)
        pair_kq = torch.empty(0, dtype=torch.int32, device=kq_index.device)
    return used.value, start[:n + 1].copy(), pair_other, pair_kq, (int(bands[0]), int(bands[1]))


def interpolate_pairs(ks: KSet, q, order: int, pair_start, pair_other, pair_kq, *, q_offset: int = 0,
                      flags: int = OUT_G, bands=(0, 0), g_out=None, band_sum=None, loss=None, loss_seed: int = 0,
                      stream=None):
    """Eq. (7) on the kept pairs of a CSR pair list (see ephw_interpolate_pairs);
    pair_start is a host int64 array of group offsets (nq + 1 by q, nk + 1 by k);
    bands = (first band, count) of the band window ((0, 0): all bands)."""
    import numpy as np
    import torch
    start = np.ascontiguousarray(pair_start, dtype=np.int64)
    n = q.shape[0] if order == PAIRS_BY_Q else ks.nk
    if start.shape != (n + 1,):
        raise ValueError(f"pair_start must hold {n + 1} offsets for this grouping, got {start.shape}")
    npairs = int(start[-1])
    for name, t in (("pair_other", pair_other), ("pair_kq", pair_kq)):
        if t.dtype != torch.int32 or t.numel() < npairs:
            raise ValueError(f"{name} must be int32 with at least {npairs} entries")
    s = ks.sys
    nb = int(bands[1]) if int(bands[1]) > 0 else s.nw
    if g_out is not None:
        want = torch.complex128 if ks.prec == FP64 else torch.complex64
        if g_out.dtype != want or tuple(g_out.shape[1:]) != (s.nm, nb, nb) or g_out.shape[0] < npairs:
            raise ValueError(f"g_out must be {want} [>= {npairs}][{s.nm}][{nb}][{nb}]")
    if band_sum is not None and (band_sum.dtype != torch.float64 or band_sum.numel() < npairs * s.nm):
        raise ValueError(f"band_sum must be float64 with at least {npairs * s.nm} entries")
    _check(lib().ephw_interpolate_pairs(ks.handle, _ptr(q), q.shape[0], int(order),
                                        start.ctypes.data_as(ctypes.c_void_p), _ptr(pair_other), _ptr(pair_kq),
                                        int(q_offset), ks.prec, int(flags), int(bands[0]), int(bands[1]),
                                        _ptr(g_out), _ptr(band_sum), _ptr(loss), int(loss_seed), _stream(stream)),
           "ephw_interpolate_pairs")


def linewidth(prec: int, g, eps_k, eps_kq, omega, gamma, *, temperature: float, mu: float, sigma: float,
              omega_min: float = 0.0, nq_total: int = 0, stream=None):
    """gamma[k][n] += phonon-limited linewidth from g [nq][nk][nm][nw][nw]
    (see ephw_linewidth); nq_total defaults to this chunk's q count."""
    nq, nk, nm, nw = _g_shape(prec, g, "linewidth")
    _expect(eps_k, (nk, nw), "eps_k")
    _expect(eps_kq, (nq, nk, nw), "eps_kq")
    _expect(omega, (nq, nm), "omega")
    _expect(gamma, (nk, nw), "gamma")
    _check(lib().ephw_linewidth(int(prec), _ptr(g), nq, nk, nm, nw, _ptr(eps_k), _ptr(eps_kq), _ptr(omega),
                                float(temperature), float(mu), float(sigma), float(omega_min),
                                int(nq_total or nq), _ptr(gamma), _stream(stream)), "ephw_linewidth")


def wannier_transform(ks: KSet, q, kq_index, g_bloch, g_out, stream=None):
    """Eq. (6): g_out[Rp][Re][ka][m'][n'] from g_bloch[q][k][nu][m][n] on the
    coarse grids (the k-set's points and q, k+q on the set's grid)."""
    _check(lib().ephw_wannier_transform(ks.handle, _ptr(q), q.shape[0], _ptr(kq_index), _ptr(g_bloch), _ptr(g_out),
                                        _stream(stream)), "ephw_wannier_transform")


def degenerate_sums(prec: int, g, eps_kq, eps_k, lam, out, rel_tol: float = 1e-6, stream=None):
    """out[q][k][nu][m][n] = |g|^2 summed over the degenerate blocks of nu, m, n.
    g [nq][nk][nm][nw][nw] (c128 at FP64, c64 otherwise), eps_kq [nq][nk][nw],
    eps_k [nk][nw], lam [nq][nm], out f64 shaped like g."""
    nq, nk, nm, nw = _g_shape(prec, g, "degenerate_sums")
    _expect(eps_kq, (nq, nk, nw), "eps_kq")
    _expect(eps_k, (nk, nw), "eps_k")
    _expect(lam, (nq, nm), "lam")
    _expect(out, (nq, nk, nm, nw, nw), "out")
    _check(lib().ephw_degenerate_sums(int(prec), _ptr(g), nq, nk, nm, nw, _ptr(eps_kq), _ptr(eps_k), _ptr(lam),
                                      float(rel_tol), _ptr(out), _stream(stream)), "ephw_degenerate_sums")


class Batch:
    """Many (k-set, q list) items interpolated in one pass (see ephw_batch_create).

    items: list of dicts with keys ks, q, kq_index, flags and the output tensors
    g_out / band_sum / loss, plus loss_seed.  Tensors must stay alive as long as
    the batch (their pointers are baked into the captured pass).
    """

    def __init__(self, ctx: Context, items, *, tune: bool = False, tune_cache: Optional[str] = None,
                 use_graph: bool = True, item_workspace_bytes: int = 0, workspace_budget_bytes: int = 0,
                 stream=None):
        arr = (BatchItem * len(items))()
        self._keep = []
        for i, it in enumerate(items):
            arr[i].ks = it["ks"].handle
            arr[i].q = _ptr(it["q"])
            arr[i].nq = it["q"].shape[0]
            arr[i].kq_index = _ptr(it["kq_index"])
            arr[i].flags = int(it.get("flags", OUT_LOSS))
            arr[i].g_out = _ptr(it.get("g_out"))
            arr[i].band_sum = _ptr(it.get("band_sum"))
            arr[i].loss = _ptr(it.get("loss"))
            arr[i].loss_seed = int(it.get("loss_seed", 0))
            self._keep.append(it)
        opt = BatchOptions(1 if tune else 0, tune_cache.encode() if tune_cache else None, 1 if use_graph else 0,
                           int(item_workspace_bytes), int(workspace_budget_bytes))
        h = ctypes.c_void_p()
        _check(lib().ephw_batch_create(ctx.handle, arr, len(items), ctypes.byref(opt), _stream(stream),
                                       ctypes.byref(h)), "ephw_batch_create")
        self.handle = h
        self.n = len(items)

    def run(self, stream=None):
        _check(lib().ephw_batch_run(self.handle, _stream(stream)), "ephw_batch_run")

    def shape(self, i: int):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().ephw_batch_shape(self.handle, i, *[ctypes.byref(x) for x in v]), "ephw_batch_shape")
        return dict(q_batch=v[0].value, k_tile=v[1].value, cfg_rp=v[2].value, cfg_re=v[3].value)

    def solo(self, i: int) -> bool:
        v = ctypes.c_int32()
        _check(lib().ephw_batch_solo(self.handle, i, ctypes.byref(v)), "ephw_batch_solo")
        return bool(v.value)

    def stats(self):
        r, l = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ephw_batch_stats(self.handle, ctypes.byref(r), ctypes.byref(l)), "ephw_batch_stats")
        return dict(rounds=r.value, launches=l.value)

    def close(self):
        if self.handle:
            lib().ephw_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def loss_backward(ks: KSet, q, kq_index, *, q_offset: int = 0, loss_seed: int = 0, loss=None, dL_dg=None,
                  dL_dk=None, dL_dq=None, stream=None):
    """L += sum w |g|^2 and the gradients (accumulated) for the k-set and q list."""
    _check(lib().ephw_loss_backward(ks.handle, _ptr(q), q.shape[0], _ptr(kq_index), int(q_offset), int(loss_seed),
                                    _ptr(loss), _ptr(dL_dg), _ptr(dL_dk), _ptr(dL_dq), _stream(stream)),
           "ephw_loss_backward")


def version() -> int:
    return int(lib().ephw_version())
