"""rocprofv3 helpers for the headline kernel: a short counter workload and the
summaries kept beside the sources.

    python -m paper_2602_23434_amd.profiling workload [--steps 4]
        a 256 MiB device-to-device copy (the calibration kernel), then the
        benchmark's float32 run-based configuration on the 128^3 turbulent
        box: one sort and `steps` fused steps, launched eagerly so that every
        dispatch carries its own counters.  Run it under
        `rocprofv3 --pmc FETCH_SIZE` and again under `--pmc WRITE_SIZE`.

    python -m paper_2602_23434_amd.profiling trace-md DB TITLE COMMAND [--split K=label:n,...]
        markdown table of the top kernels of a `--kernel-trace --stats`
        database; --split adds the average of one kernel's dispatches per
        consecutive group (the workloads of the benchmark, in order).

    python -m paper_2602_23434_amd.profiling traffic FETCH_CSV WRITE_CSV COMMAND
        HBM bytes per launch of the run kernel as JSON: each counter's mean
        over the kernel's dispatches, scaled by the known bytes of the copy
        over what the same counter reads for the copy.

    python -m paper_2602_23434_amd.profiling instructions SQ_CSV COMMAND
        VALU and LDS instruction counts per launch of the run kernel (from a
        `rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT`
        run of the same workload) as JSON.

    python -m paper_2602_23434_amd.profiling lds LDS_A_CSV LDS_B_CSV AGENT_CSV COMMAND
        LDS occupancy and bytes per launch of the run kernel as JSON, from a
        `--pmc SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE`
        run and a `--pmc SQ_INSTS_LDS_LOAD_BANDWIDTH SQ_INSTS_LDS_STORE_BANDWIDTH
        SQ_INSTS_LDS_ATOMIC_BANDWIDTH GRBM_GUI_ACTIVE` run of the same workload
        (AGENT_CSV: rocprofv3's agent_info.csv of either run, for the CU and
        XCD counts).

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  The JSON carries
the digest of the kernel sources, so a reader can tell whether the figures
still describe the built kernel.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
# sources that define the float32 run kernel and the particle order it reads
DIGEST_FILES = ("k_runs_impl.h", "k_runs_f32.hip", "k_step_impl.h", "pl_device.h", "pl_internal.h", "k_sort.hip")
COPY_BYTES = 1 << 28          # the calibration copy reads and writes 256 MiB
COPY_ELEMS = 1 << 26         # float32 elements of the copy


def src_digest():
    h = hashlib.sha256()
    for f in DIGEST_FILES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(steps=4):
    import torch

    from . import benchcfg as BC
    from . import binding as B
    from . import driver, inputs
    src = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    cfg = BC.headline()
    wl = inputs.turbulent_box(n=BC.TURB_N, npart=BC.TURB_NP, steps=steps)
    run = driver.Run(wl, **BC.run_kwargs(cfg))
    run.sort()
    for _ in range(steps):
        run.zero_moments()
        run.step(flags=BC.STEP_FLAGS & ~B.PL_GRAPH)
    st = run.sync()
    stats = B.pl_part_stats(run.ctx)
    run.close()
    if st != B.PL_OK or stats[4] == 0 or stats[5] != 0:
        raise RuntimeError(f"status {st}, stats {stats}")
    print(f"profiling workload done: {steps} steps, stats {stats}", flush=True)


def trace_md(db, title, command):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = [f"# {title}\n", f"Command (run from the repository root on one MI355X):\n\n```\n{command}\n```\n",
           "Durations from `rocprofv3 --kernel-trace --stats` (top_kernels of the trace database).\n",
           "| kernel | calls | average (ms) | total (ms) | share |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:20]:
        out.append(f"| `{name.split('(')[0]}` | {calls} | {avg / 1e3:.4f} | {tot / 1e3:.2f} | {pct:.1f}% |")
    return "\n".join(out) + "\n"


def split_md(db, kernel, parts):
    """Markdown rows for the dispatches of one kernel split into consecutive
    groups, in dispatch order: parts is a list of (label, count)."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    durs = [d for n, d in rows if n.split("(")[0].replace("void ", "") == kernel]
    if sum(c for _, c in parts) != len(durs):
        raise RuntimeError(f"{len(durs)} dispatches of {kernel}, parts {parts}")
    out = [f"\nDispatches of `{kernel}` by workload, in order:\n", "| workload | calls | average (ms) |",
           "|---|---:|---:|"]
    i = 0
    for label, cnt in parts:
        seg = durs[i:i + cnt]
        i += cnt
        out.append(f"| {label} | {cnt} | {sum(seg) / len(seg) / 1e6:.4f} |")
    return "\n".join(out) + "\n"


def _rows(path, counter):
    with open(path) as fh:
        return [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]


def _kernel_and_copy(rows):
    runs = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith("void pl::k_runs<")]
    names = {r["Kernel_Name"].split("(")[0] for r in rows if r["Kernel_Name"].startswith("void pl::k_runs<")}
    # the calibration copy: torch's device-to-device copy kernel, dispatched first
    copy = [float(r["Counter_Value"]) for r in rows if "direct_copy_kernel" in r["Kernel_Name"]]
    if not runs or len(names) != 1 or not copy:
        raise RuntimeError(f"expected run-kernel dispatches of one kernel and one copy: {names}, {len(copy)}")
    return runs, names.pop(), copy[0]


def workload_config():
    """Particle order and tile of the counter workload (the benchmark's
    headline configuration): the counters depend on them as well as on the
    kernel sources."""
    from . import benchcfg as BC
    cfg = BC.headline()
    return {"key_mode": int(cfg["key_mode"]), "tile": [int(t) for t in cfg["tile"]]}


def traffic(fetch_csv, write_csv, command):
    fr, name, fc = _kernel_and_copy(_rows(fetch_csv, "FETCH_SIZE"))
    wr, name2, wc = _kernel_and_copy(_rows(write_csv, "WRITE_SIZE"))
    if name != name2:
        raise RuntimeError(f"different kernels: {name} / {name2}")
    f_factor = COPY_BYTES / (fc * 1024.0)
    w_factor = COPY_BYTES / (wc * 1024.0)
    f_kib = sum(fr) / len(fr)
    w_kib = sum(wr) / len(wr)
    fetch_b = f_kib * 1024.0 * f_factor
    write_b = w_kib * 1024.0 * w_factor
    return {
        "kernel": name.replace("void ", ""),
        "src_digest": src_digest(),
        "config": workload_config(),
        "launches": len(fr),
        "fetch_kib_per_launch_raw": f_kib,
        "write_kib_per_launch_raw": w_kib,
        "copy_fetch_kib_raw": fc,
        "copy_write_kib_raw": wc,
        "copy_bytes": COPY_BYTES,
        "fetch_factor": f_factor,
        "write_factor": w_factor,
        "fetch_bytes_per_launch": fetch_b,
        "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b,
        "command": command,
    }


# chip figures for the instruction ceilings: a wave64 VALU instruction
# occupies a 16-lane SIMD for 4 cycles
SIMDS, CUS, CLOCK_HZ, VALU_CYCLES = 1024, 256, 2.4e9, 4


def instructions(sq_csv, command):
    vals = {}
    with open(sq_csv) as fh:
        for r in csv.DictReader(fh):
            if r["Kernel_Name"].startswith("void pl::k_runs<"):
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                name = r["Kernel_Name"].split("(")[0].replace("void ", "")
    need = ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAVES")
    if not all(k in vals for k in need):
        raise RuntimeError(f"missing counters: {sorted(vals)}")
    mean = {k: sum(v) / len(v) for k, v in vals.items()}
    return {
        "kernel": name,
        "src_digest": src_digest(),
        "config": workload_config(),
        "launches": len(vals["SQ_INSTS_VALU"]),
        "valu_wave_insts": mean["SQ_INSTS_VALU"],
        "lds_wave_insts": mean["SQ_INSTS_LDS"],
        "lds_bank_conflict_cycles": mean["SQ_LDS_BANK_CONFLICT"],
        "waves": mean["SQ_WAVES"],
        "valu_floor_ms": mean["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * CLOCK_HZ) * 1e3,
        "lds_conflict_ms_per_cu": mean["SQ_LDS_BANK_CONFLICT"] / CUS / CLOCK_HZ * 1e3,
        "command": command,
    }


# LDS: 128 bytes per clock per CU (32 banks of 4 bytes)
LDS_BYTES_PER_CLK = 128


def _kernel_means(path):
    vals, name = {}, None
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Kernel_Name"].startswith("void pl::k_runs<"):
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                name = r["Kernel_Name"].split("(")[0].replace("void ", "")
    return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}, name


def _gpu_agent(path):
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Agent_Type") == "GPU":
                return int(r["Cu_Count"]), int(r["Num_Xcc"])
    raise RuntimeError("no GPU agent in " + path)


def lds(a_csv, b_csv, agent_csv, command):
    """LDS occupancy of the run kernel (cycles the LDS serves indexed
    operations over the launch's cycles on every CU) and its LDS bytes per
    launch against what 128 bytes per clock per CU would move in the same
    cycles.  GRBM_GUI_ACTIVE is summed over the XCDs in the CSV; one XCD's
    count is the launch's length in clocks."""
    ma, na, name = _kernel_means(a_csv)
    mb, nb, name2 = _kernel_means(b_csv)
    need_a = ("SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "GRBM_GUI_ACTIVE")
    need_b = ("SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH",
              "GRBM_GUI_ACTIVE")
    if not all(k in ma for k in need_a) or not all(k in mb for k in need_b) or name != name2:
        raise RuntimeError(f"missing counters or different kernels: {sorted(ma)} {sorted(mb)} {name} {name2}")
    cus, xcc = _gpu_agent(agent_csv)
    clk_a = ma["GRBM_GUI_ACTIVE"] / xcc
    clk_b = mb["GRBM_GUI_ACTIVE"] / xcc
    load = mb["SQ_INSTS_LDS_LOAD_BANDWIDTH"] * 64
    store = mb["SQ_INSTS_LDS_STORE_BANDWIDTH"] * 64
    atomic = mb["SQ_INSTS_LDS_ATOMIC_BANDWIDTH"] * 64
    total = load + store + atomic
    return {
        "kernel": name,
        "src_digest": src_digest(),
        "config": workload_config(),
        "launches": na["SQ_LDS_IDX_ACTIVE"],
        "cu_count": cus,
        "xcc_count": xcc,
        "launch_clocks": clk_a,
        "lds_active_cycles_per_cu": ma["SQ_LDS_IDX_ACTIVE"] / cus,
        "lds_util": ma["SQ_LDS_IDX_ACTIVE"] / (clk_a * cus),
        "bank_conflict_share_of_active": ma["SQ_LDS_BANK_CONFLICT"] / ma["SQ_LDS_IDX_ACTIVE"],
        "lds_load_bytes": load,
        "lds_store_bytes": store,
        "lds_atomic_bytes": atomic,
        "lds_bytes": total,
        "lds_bw_frac": total / (LDS_BYTES_PER_CLK * cus * clk_b),
        "command": command,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    w = sub.add_parser("workload")
    w.add_argument("--steps", type=int, default=4)
    t = sub.add_parser("trace-md")
    t.add_argument("db")
    t.add_argument("title")
    t.add_argument("command")
    t.add_argument("--split", default=None,
                   help="KERNEL=label:count,label:count,... per-workload averages of one kernel's dispatches")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("command")
    i = sub.add_parser("instructions")
    i.add_argument("sq_csv")
    i.add_argument("command")
    ld = sub.add_parser("lds")
    ld.add_argument("a_csv")
    ld.add_argument("b_csv")
    ld.add_argument("agent_csv")
    ld.add_argument("command")
    a = ap.parse_args(argv)
    if a.cmd == "workload":
        workload(a.steps)
    elif a.cmd == "trace-md":
        sys.stdout.write(trace_md(a.db, a.title, a.command))
        if a.split:
            kern, spec = a.split.split("=", 1)
            parts = [(p.rsplit(":", 1)[0], int(p.rsplit(":", 1)[1])) for p in spec.split(",")]
            sys.stdout.write(split_md(a.db, kern, parts))
    elif a.cmd == "instructions":
        print(json.dumps(instructions(a.sq_csv, a.command), indent=1))
    elif a.cmd == "lds":
        print(json.dumps(lds(a.a_csv, a.b_csv, a.agent_csv, a.command), indent=1))
    else:
        print(json.dumps(traffic(a.fetch_csv, a.write_csv, a.command), indent=1))


if __name__ == "__main__":
    main()
