"""CPU-side checks of the C ABI and the host accounting (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_10295_amd import ephw, model

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ephw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ephw_[a-z_0-9]+)\s*\(", text)))


def test_header_declarations_are_exported():
    names = declared_functions()
    assert len(names) >= 15
    assert sorted(ephw.EXPORTS) == names
    L = ephw.lib()
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    L = ephw.lib()
    for s in range(7):
        assert L.ephw_status_string(s)
    assert L.ephw_status_string(99) == b"unknown status"
    assert ephw.version() == 200


def test_null_arguments_rejected_before_any_device_call():
    L = ephw.lib()
    assert L.ephw_interpolate(None, None, 1, None, 0, 0, 1, None, None, None, 0, None, None, None) == ephw.EINVAL
    assert b"invalid" in L.ephw_last_error()
    assert L.ephw_system_load(None, None, None) == ephw.EINVAL
    assert L.ephw_set_q_batch(None, 4) == ephw.EINVAL
    assert L.ephw_ctx_check(None, None) == ephw.EINVAL
    assert L.ephw_kset_create(None, None, 4, 0, None, None) == ephw.EINVAL
    assert L.ephw_bands(None, None, 3, None, None, None) == ephw.EINVAL
    # degenerate-block sums: precision, sizes, tolerance and buffers are checked on the host
    assert L.ephw_degenerate_sums(7, None, 1, 1, 3, 4, None, None, None, 1e-6, None, None) == ephw.EINVAL
    assert L.ephw_degenerate_sums(0, None, 1, 1, 3, 0, None, None, None, 1e-6, None, None) == ephw.EINVAL
    assert L.ephw_degenerate_sums(0, None, 1, 1, 3, 4, None, None, None, -1.0, None, None) == ephw.EINVAL
    assert L.ephw_degenerate_sums(0, None, 1, 1, 3, 4, None, None, None, float("nan"), None, None) == ephw.EINVAL
    assert L.ephw_degenerate_sums(0, None, 2, 3, 3, 4, None, None, None, 1e-6, None, None) == ephw.EINVAL
    assert b"NULL" in L.ephw_last_error()
    assert L.ephw_degenerate_sums(1, None, 0, 3, 3, 4, None, None, None, 1e-6, None, None) == ephw.OK
    assert L.ephw_wannier_transform(None, None, 4, None, None, None, None) == ephw.EINVAL
    assert L.ephw_window_screen(None, None, 4, None, 0.0, 1.0, None, None, None, None, None, None, None) == ephw.EINVAL
    # linewidth: temperature and width must be positive, buffers present
    assert L.ephw_linewidth(0, None, 1, 1, 3, 4, None, None, None, 0.0, 0.0, 0.01, 0.0, 1, None, None) == ephw.EINVAL
    assert L.ephw_linewidth(0, None, 1, 1, 3, 4, None, None, None, 0.02, 0.0, -1.0, 0.0, 1, None, None) == ephw.EINVAL
    assert L.ephw_linewidth(0, None, 1, 1, 3, 4, None, None, None, 0.02, 0.0, 0.01, 0.0, 0, None, None) == ephw.EINVAL
    assert L.ephw_linewidth(0, None, 1, 1, 3, 4, None, None, None, 0.02, 0.0, 0.01, 0.0, 1, None, None) == ephw.EINVAL
    assert L.ephw_linewidth(1, None, 0, 1, 3, 4, None, None, None, 0.02, 0.0, 0.01, 0.0, 1, None, None) == ephw.OK
    assert L.ephw_phonons(None, None, 3, None, None, None, None) == ephw.EINVAL
    assert L.ephw_phase_sum_rp(None, None, 3, 0, None, None) == ephw.EINVAL
    assert L.ephw_ctx_create(0, None) == ephw.EINVAL
    assert L.ephw_ctx_set_limits(None, 0, 40) == ephw.EINVAL
    assert L.ephw_ctx_memory(None, None, None) == ephw.EINVAL
    # freeing NULL handles is a no-op
    assert L.ephw_system_free(None) == ephw.OK
    assert L.ephw_kset_free(None) == ephw.OK
    assert L.ephw_ctx_destroy(None) == ephw.OK


def test_system_desc_layout_matches_header():
    # int32 nw, na; int64 ne, np, nh, nc; 12 pointers; int32 g_dtype (+ padding)
    assert ctypes.sizeof(ephw.SystemDesc) == 8 + 4 * 8 + 12 * 8 + 8


# ----------------------------------------------------------------------------
# accounting against the paper's printed numbers
# ----------------------------------------------------------------------------

def test_si_g_size_is_0p4_gb():
    # bulk Si: Nb=8, Nm=6, Ne=617, Np=93 -> "0.4 GB" in double-complex
    b = model.g_bytes(8, 6, 617, 93)
    assert round(b / 1e9, 1) == 0.4


def test_zsnr_table_sizes():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "zsnr_g_size.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 11
    for w, nb, nm, ne, np_, printed in rows:
        gib = model.g_bytes(int(nb), int(nm), int(ne), int(np_)) / 2 ** 30
        digits = len(printed.split(".")[1]) if "." in printed else 0
        assert round(gib, digits) == pytest.approx(float(printed)), (w, gib, printed)


def test_nested_over_single_ratio_si():
    # Eq. (12) for Si (Ne=617, Np=93, Nm=6) with Nk >> Np: about 1/93
    r = model.nested_over_single(8, 6, 617, 93, nk=10 ** 7)
    assert 1 / 95 < r < 1 / 90
    # and it is the ratio of the two printed counts in that limit
    exact = model.nested_loop_cmul(8, 6, 617, 93, 10 ** 7, 50) / model.single_loop_cmul(8, 6, 617, 93, 10 ** 7, 50)
    assert exact == pytest.approx(r, rel=2e-2)


def test_stage_counts_sum_to_the_reassociated_nested_loop():
    c = model.stage_counts(8, 6, 1000, 1000, 8000, 8000)
    assert c.rp == 8000 * 1000 * 1000 * 384
    assert c.re == 8000 * 8000 * 1000 * 384
    assert c.rot == 8000 * 8000 * 2 * 512 * 6
    assert c.elems == 8000 * 8000 * 384
    # the Re sum dominates the dense Si workload (about 88 % of the cMAC)
    assert 0.85 < c.re / c.total < 0.9


def test_wrappers_check_buffer_types_before_the_call():
    """The kernels size their reads of g from the precision argument: the
    binding refuses a g whose element type that precision does not read, and
    side buffers of the wrong shape or type, before calling the library."""
    import torch
    g = torch.zeros((2, 3, 6, 4, 4), dtype=torch.complex64)
    eps_k = torch.zeros((3, 4), dtype=torch.float64)
    eps_kq = torch.zeros((2, 3, 4), dtype=torch.float64)
    om = torch.zeros((2, 6), dtype=torch.float64)
    gamma = torch.zeros((3, 4), dtype=torch.float64)
    with pytest.raises(ValueError, match="reads"):
        ephw.linewidth(ephw.FP64, g, eps_k, eps_kq, om, gamma, temperature=0.1, mu=0.0, sigma=0.1)
    with pytest.raises(ValueError, match="eps_kq"):
        ephw.linewidth(ephw.FP32, g, eps_k, eps_kq[:, :2], om, gamma, temperature=0.1, mu=0.0, sigma=0.1)
    with pytest.raises(ValueError, match="gamma"):
        ephw.linewidth(ephw.FP32, g, eps_k, eps_kq, om, gamma.float(), temperature=0.1, mu=0.0, sigma=0.1)
    out = torch.zeros((2, 3, 6, 4, 4), dtype=torch.float64)
    with pytest.raises(ValueError, match="reads"):
        ephw.degenerate_sums(ephw.FP64, g, eps_kq, eps_k, om, out)
    with pytest.raises(ValueError, match="lam"):
        ephw.degenerate_sums(ephw.FP32, g, eps_kq, eps_k, om[:, :3], out)


def test_host_validation_under_address_and_ub_sanitizers(tmp_path):
    """The host side of every .hip source, compiled without device code and
    with AddressSanitizer and UndefinedBehaviorSanitizer, linked with a C
    driver that calls each entry point with invalid arguments
    (tests/abi_host_check.c): every call returns its status with no invalid
    access, overflow, undefined operation or leak."""
    import concurrent.futures as cf
    import glob
    import shutil
    import subprocess
    from paper_2603_10295_amd import build as b

    hipcc = b.hipcc()
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    host_only = [f"--offload-arch={b.ARCH}", "--offload-host-only", "-fgpu-rdc"]
    inc = ["-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [hipcc, *host_only, "-x", "hip", "-std=c++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer",
               *san, *inc, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2603_10295_amd", "csrc", "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "drv.o")
    r = subprocess.run([gcc, "-std=c11", "-O1", "-g", "-fsanitize=address", "-fsanitize=undefined",
                        "-fno-sanitize-recover=all", *inc, "-c", os.path.join(ROOT, "tests", "abi_host_check.c"),
                        "-o", drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_host_check")
    r = subprocess.run([hipcc, *host_only, *san, drv, *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "abi_host_check: ok" in r.stdout


def test_jacobi_lds_layout(tmp_path):
    """The LDS map of the one-task-per-lane Jacobi solves (n <= 12), checked on
    the host from the kernel source (tests/jacobi_layout_check.hip): every
    entry of A (upper triangle, transposes sharing a slot) and of V in its own
    slot inside the data region, task t's loads at e RS + t (what keeps a
    round's loads free of LDS bank conflicts), the stores to the moved
    positions covering every slot the next round reads, and every position
    back in place after a sweep."""
    import subprocess
    from paper_2603_10295_amd import build as b

    host_only = [b.hipcc(), f"--offload-arch={b.ARCH}", "--offload-host-only", "-fgpu-rdc"]
    obj, exe = str(tmp_path / "jacobi_layout_check.o"), str(tmp_path / "jacobi_layout_check")
    r = subprocess.run([*host_only, "-x", "hip", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2603_10295_amd", "csrc"),
                        os.path.join(ROOT, "tests", "jacobi_layout_check.hip"), "-c", "-o", obj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([*host_only, obj, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "jacobi_layout_check: ok" in r.stdout
