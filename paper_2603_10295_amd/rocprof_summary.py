"""Summarise rocprofv3 result databases (SQLite) of libephw runs as text.

    python -m paper_2603_10295_amd.rocprof_summary stats RESULTS.db [--command CMD]
    python -m paper_2603_10295_amd.rocprof_summary traffic FETCH.db WRITE.db \
        --copy-bytes BYTES [--command CMD]
    python -m paper_2603_10295_amd.rocprof_summary util COUNTERS.db [--command CMD]
    python -m paper_2603_10295_amd.rocprof_summary lds COUNTERS.db [--match NAME] [--command CMD]

`stats` groups kernel dispatches by (kernel, grid) - the phase GEMMs of
Eqs. (9) and (10) share one kernel but differ in grid - and prints calls,
total/average/min/max duration.  `traffic` reads FETCH_SIZE and WRITE_SIZE
(KiB per dispatch) from two counter runs, scales each by the factor that
makes a plain device copy of `--copy-bytes` bytes read and write exactly that
many bytes, and prints HBM bytes per dispatch per (kernel, grid) group.
`lds` prints, per (kernel, grid) group, VALU and LDS instructions per
wavefront (SQ_INSTS_VALU, SQ_INSTS_LDS over SQ_WAVES), the VALU issue time
they imply (4 cycles per wave64 instruction over the SIMDs) as a share of the
kernel's cycles, and the LDS-active and bank-conflict cycles
(SQ_ACTIVE_INST_LDS, SQ_LDS_BANK_CONFLICT) per CU cycle and per LDS-active
cycle.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def short_name(name: str) -> str:
    """Kernel name without namespaces and parameter list, keeping template arguments."""
    n = name.replace("(anonymous namespace)::", "")
    n = re.sub(r"^void ", "", n)
    if n.endswith(")") and "(" in n:
        n = n[: n.rfind("(")] if n.count("(") == 1 else n[: n.index("(")]
    return n.replace("ephw::", "").strip()


def source_digest() -> str:
    """Hash of the GEMM source: the traffic figures hold only for this kernel."""
    h = hashlib.sha256()
    with open(os.path.join(HERE, "csrc", "gemm.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def stats(db: str, command: str = "") -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select name, grid_x, grid_y, grid_z, workgroup_x, duration from kernels").fetchall()
    groups = collections.defaultdict(list)
    for name, gx, gy, gz, wx, dur in rows:
        groups[(short_name(name), gx // max(1, wx), gy, gz)].append(dur)
    total = sum(sum(v) for v in groups.values())
    out = [f"# rocprofv3 kernel-trace stats: {os.path.basename(db)}",
           f"# command: {command}" if command else "# command: (not recorded)",
           "# grouped by (kernel, workgroups x, grid y, grid z); durations in ms",
           f"{'calls':>6} {'total_ms':>11} {'avg_ms':>10} {'min_ms':>10} {'max_ms':>10} {'pct':>6}  kernel [wg_x x grid_y x grid_z]"]
    for (name, bx, gy, gz), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{len(v):6d} {sum(v) / 1e6:11.3f} {sum(v) / len(v) / 1e6:10.4f} {min(v) / 1e6:10.4f} "
                   f"{max(v) / 1e6:10.4f} {100 * sum(v) / total:6.2f}  {name} [{bx} x {gy} x {gz}]")
    return "\n".join(out) + "\n"


def _counter_groups(db: str, counter: str):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, grid_size_x, grid_size_y, workgroup_size_x, counter_name, value "
                     "from counters_collection").fetchall()
    groups = collections.defaultdict(list)
    for name, gx, gy, wx, cname, val in rows:
        if cname == counter:
            groups[(short_name(name), gx // max(1, wx), gy)].append(val)
    return groups


def traffic(fetch_db: str, write_db: str, copy_bytes: int, command: str = "") -> str:
    fg = _counter_groups(fetch_db, "FETCH_SIZE")
    wg = _counter_groups(write_db, "WRITE_SIZE")

    def copy_value(groups):
        vals = [v for (n, _, _), vs in groups.items() if "copyBuffer" in n for v in vs]
        return max(vals) if vals else None

    kib = copy_bytes / 1024.0
    cf, cw = copy_value(fg), copy_value(wg)
    ff = kib / cf if cf else None
    fw = kib / cw if cw else None
    out = [f"# HBM traffic per dispatch from rocprofv3 counters (gemm.hip digest {source_digest()})",
           f"# command: {command}" if command else "# command: (not recorded)",
           f"# calibration: device copy of {copy_bytes} bytes read FETCH_SIZE={cf} KiB, WRITE_SIZE={cw} KiB",
           f"# scale factors: fetch x{ff:.4f}, write x{fw:.4f}" if ff and fw else "# scale factors: unavailable",
           f"{'disp':>5} {'fetch_KiB':>13} {'write_KiB':>13} {'read_GB':>9} {'write_GB':>9}  kernel [workgroups x grid_y]"]
    keys = sorted(set(fg) | set(wg), key=lambda k: -(sum(fg.get(k, [0])) + sum(wg.get(k, [0]))))
    for k in keys:
        f = fg.get(k, [])
        w = wg.get(k, [])
        fa = sum(f) / len(f) if f else float("nan")
        wa = sum(w) / len(w) if w else float("nan")
        rd = fa * 1024 * (ff or float("nan")) / 1e9
        wr = wa * 1024 * (fw or float("nan")) / 1e9
        out.append(f"{max(len(f), len(w)):5d} {fa:13.1f} {wa:13.1f} {rd:9.3f} {wr:9.3f}  {k[0]} [{k[1]} x {k[2]}]")
    return "\n".join(out) + "\n"


def utilisation(db: str, simds: int = 1024, xcds: int = 8, command: str = "") -> str:
    """Per (kernel, grid): MFMA busy share and clock from SQ_VALU_MFMA_BUSY_CYCLES
    (summed over SIMDs) and GRBM_GUI_ACTIVE (summed over XCDs), with the
    kernel's duration; plus LDS bank-conflict and LDS-wait cycles relative to
    the MFMA busy cycles when present."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, grid_size_x, grid_size_y, workgroup_size_x, counter_name, "
                     "value, start, end from counters_collection").fetchall()
    per = collections.defaultdict(dict)
    meta = {}
    for d, name, gx, gy, wx, cname, val, t0, t1 in rows:
        per[d][cname] = per[d].get(cname, 0.0) + val
        meta[d] = (short_name(name), gx // max(1, wx), gy, (t1 - t0) * 1e-9)
    groups = collections.defaultdict(list)
    for d, v in per.items():
        groups[meta[d][:3]].append((v, meta[d][3]))
    out = [f"# MFMA utilisation per dispatch from rocprofv3 counters: {os.path.basename(db)}",
           f"# command: {command}" if command else "# command: (not recorded)",
           f"# mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / {simds} SIMDs / (GRBM_GUI_ACTIVE / {xcds} XCDs); "
           f"clock = (GRBM_GUI_ACTIVE / {xcds}) / duration",
           f"{'disp':>5} {'mfma_busy':>9} {'clock_GHz':>9} {'lds_conf':>9} {'lds_wait':>9} {'mfma_insts':>11}  "
           f"kernel [workgroups x grid_y]"]
    def avg(xs):
        return sum(xs) / len(xs) if xs else float("nan")
    keys = sorted(groups, key=lambda k: -sum(v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) for v, _ in groups[k]))
    for k in keys:
        vs = groups[k]
        busy = avg([v.get("SQ_VALU_MFMA_BUSY_CYCLES", float("nan")) for v, _ in vs])
        gui = avg([v.get("GRBM_GUI_ACTIVE", float("nan")) for v, _ in vs])
        dur = avg([t for _, t in vs])
        conf = avg([v.get("SQ_LDS_BANK_CONFLICT", float("nan")) for v, _ in vs])
        lw = avg([v.get("SQ_WAIT_INST_LDS", float("nan")) for v, _ in vs])
        ins = avg([v.get("SQ_INSTS_MFMA", float("nan")) for v, _ in vs])
        util = busy / simds / (gui / xcds) if gui else float("nan")
        clk = (gui / xcds) / dur / 1e9 if dur else float("nan")
        out.append(f"{len(vs):5d} {util:9.3f} {clk:9.3f} {conf / busy if busy else float('nan'):9.4f} "
                   f"{lw / busy if busy else float('nan'):9.4f} {ins:11.4g}  {k[0]} [{k[1]} x {k[2]}]")
    return "\n".join(out) + "\n"


def lds(db: str, match: str = "", simds: int = 1024, cus: int = 256, xcds: int = 8, command: str = "") -> str:
    """VALU and LDS figures per (kernel, grid) group from SQ_WAVES, SQ_INSTS_VALU,
    SQ_INSTS_LDS, SQ_ACTIVE_INST_LDS, SQ_LDS_BANK_CONFLICT and GRBM_GUI_ACTIVE
    (each summed over the chip)."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, grid_size_x, grid_size_y, workgroup_size_x, counter_name, "
                     "value, start, end from counters_collection").fetchall()
    per = collections.defaultdict(dict)
    meta = {}
    for d, name, gx, gy, wx, cname, val, t0, t1 in rows:
        if match and match not in name:
            continue
        per[d][cname] = per[d].get(cname, 0.0) + val
        meta[d] = (short_name(name), gx // max(1, wx), gy, (t1 - t0) * 1e-9)
    groups = collections.defaultdict(list)
    for d, v in per.items():
        groups[meta[d][:3]].append((v, meta[d][3]))
    out = [f"# VALU and LDS counters per dispatch: {os.path.basename(db)}",
           f"# command: {command}" if command else "# command: (not recorded)",
           f"# valu_issue = SQ_INSTS_VALU x 4 cycles / {simds} SIMDs / (GRBM_GUI_ACTIVE / {xcds} XCDs); "
           f"lds_active, conflict = SQ_ACTIVE_INST_LDS, SQ_LDS_BANK_CONFLICT / {cus} CUs / (GRBM_GUI_ACTIVE / {xcds})",
           f"{'disp':>5} {'avg_ms':>8} {'valu/wave':>10} {'lds/wave':>9} {'valu_issue':>10} {'lds_active':>10} "
           f"{'conflict':>9} {'conf/lds':>9}  kernel [workgroups x grid_y]"]
    def avg(xs):
        return sum(xs) / len(xs) if xs else float("nan")
    for k in sorted(groups, key=lambda k: -sum(t for _, t in groups[k])):
        vs = groups[k]
        def field(n):
            return avg([v.get(n, float("nan")) for v, _ in vs])
        waves, gui = field("SQ_WAVES"), field("GRBM_GUI_ACTIVE") / xcds
        valu, ldsi = field("SQ_INSTS_VALU"), field("SQ_INSTS_LDS")
        act, conf = field("SQ_ACTIVE_INST_LDS"), field("SQ_LDS_BANK_CONFLICT")
        out.append(f"{len(vs):5d} {avg([t for _, t in vs]) * 1e3:8.3f} {valu / waves:10.0f} {ldsi / waves:9.0f} "
                   f"{valu * 4 / simds / gui:10.3f} {act / cus / gui:10.3f} {conf / cus / gui:9.3f} "
                   f"{conf / act if act else float('nan'):9.3f}  {k[0]} [{k[1]} x {k[2]}]")
    return "\n".join(out) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--command", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command", default="")
    u = sub.add_parser("util")
    u.add_argument("db")
    u.add_argument("--command", default="")
    lp = sub.add_parser("lds")
    lp.add_argument("db")
    lp.add_argument("--match", default="")
    lp.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        sys.stdout.write(stats(a.db, a.command))
    elif a.cmd == "util":
        sys.stdout.write(utilisation(a.db, command=a.command))
    elif a.cmd == "lds":
        sys.stdout.write(lds(a.db, match=a.match, command=a.command))
    else:
        sys.stdout.write(traffic(a.fetch_db, a.write_db, a.copy_bytes, a.command))
    return 0


if __name__ == "__main__":
    sys.exit(main())
