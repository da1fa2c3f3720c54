"""Summaries of rocprofv3 databases (rocpd SQLite) for the files under profiles/.

    python -m paper_2010_15069_amd.profile_summary trace DB [TOP]
        per kernel name and launch shape: calls and mean / median / min / max duration in us,
        largest total time first (a markdown table)
    python -m paper_2010_15069_amd.profile_summary counters DB
        per kernel: the median over its dispatches of each counter, summed over the counter's
        instances in a dispatch
    python -m paper_2010_15069_amd.profile_summary traffic KERNEL_FETCH KERNEL_WRITE COPY_FETCH COPY_WRITE OUT
        HBM bytes per launch of the 1024^2 step kernels from four --pmc runs (FETCH_SIZE and
        WRITE_SIZE of bench.py's headline kernels, and of bench.py --copy-reference 256), each
        scaled by what the counter reads for the plain 256 MiB copy; writes OUT (the JSON record
        bench.py reports as roofline.traffic while the kernel sources and the schedule match)

Only reads databases; it does not run or profile anything.
"""
from __future__ import annotations

import collections
import json
import sqlite3
import statistics
import sys

COPY_MIB = 256
BYTES_PER_POINT_PASS = 32


def _short(name: str) -> str:
    return name.replace("void sgpe::", "").replace("sgpe::", "").split("(")[0]


def trace_table(db: str, top: int = 40) -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select name, grid_x, grid_y, workgroup_x, vgpr_count, lds_size, scratch_size, end - start "
                     "from kernels").fetchall()
    groups = collections.defaultdict(list)
    for name, gx, gy, wx, vg, lds, scr, dur in rows:
        wgs = gx // max(wx, 1) * max(gy, 1)
        groups[(name, wgs, wx, vg, lds, scr)].append(dur / 1000.0)
    items = sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]
    out = ["| kernel | workgroups | threads/WG | VGPRs | LDS B | scratch B | calls | mean us | median us | min us | max us |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for (name, wgs, wx, vg, lds, scr), ds in items:
        out.append(f"| `{_short(name)}` | {wgs} | {wx} | {vg} | {lds} | {scr} | {len(ds)} | {statistics.fmean(ds):.2f} | "
                   f"{statistics.median(ds):.2f} | {min(ds):.2f} | {max(ds):.2f} |")
    return "\n".join(out)


def counter_medians(db: str) -> dict:
    """{kernel: {counter: median per dispatch}}, and the dispatch count under key '_dispatches'."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    name_of = {}
    for d, k, cn, v in rows:
        per[d][cn] += v
        name_of[d] = k
    byk = collections.defaultdict(lambda: collections.defaultdict(list))
    for d, cs in per.items():
        for cn, v in cs.items():
            byk[_short(name_of[d])][cn].append(v)
    res = {}
    for k, cs in byk.items():
        res[k] = {cn: statistics.median(v) for cn, v in cs.items()}
        res[k]["_dispatches"] = len(next(iter(cs.values())))
    return res


def traffic_record(kf: str, kw: str, cf: str, cw: str) -> dict:
    from paper_2010_15069_amd.build import kernel_hash

    copy_bytes = COPY_MIB << 20
    cfm, cwm = counter_medians(cf), counter_medians(cw)
    copy_fetch = max(v["FETCH_SIZE"] for v in cfm.values())
    copy_write = max(v["WRITE_SIZE"] for v in cwm.values())
    fetch_scale = copy_bytes / (copy_fetch * 1024)
    write_scale = copy_bytes / (copy_write * 1024)
    kfm, kwm = counter_medians(kf), counter_medians(kw)
    alg = BYTES_PER_POINT_PASS * 1024 * 1024
    want = {"row_pass": "row_kernel<1024, 2, true, false, 1, 16>", "col_pass": "col_kernel<1024, 1, 1, 16>",
            "row_pass_real": "row_kernel<1024, 2, false, false, 1, 16>", "col_pass_real": "col_kernel<1024, 0, 1, 16>"}
    rec = {"workload": "metric_1024", "kernel_hash": kernel_hash(),
           "schedule": {"col_tile": 4, "row_iters": 1, "col_iters": 1, "row_points": 16, "col_points": 16,
                        "row_tile": 1},
           "calibration": {"copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes,
                           "copy_fetch_size_kib": copy_fetch, "copy_write_size_kib": copy_write,
                           "fetch_scale": fetch_scale, "write_scale": write_scale},
           "kernels": {}}
    for key, kname in want.items():
        if kname not in kfm or kname not in kwm:
            continue
        rb = kfm[kname]["FETCH_SIZE"] * 1024 * fetch_scale
        wb = kwm[kname]["WRITE_SIZE"] * 1024 * write_scale
        rec["kernels"][key] = {"kernel": kname, "dispatches": kfm[kname]["_dispatches"],
                               "fetch_size_kib": kfm[kname]["FETCH_SIZE"], "write_size_kib": kwm[kname]["WRITE_SIZE"],
                               "read_bytes": int(rb), "written_bytes": int(wb), "bytes_per_launch": int(rb + wb),
                               "alg_bytes": alg, "ratio_to_alg": (rb + wb) / alg}
    return rec


def main(argv):
    if len(argv) >= 2 and argv[0] == "trace":
        print(trace_table(argv[1], int(argv[2]) if len(argv) > 2 else 40))
    elif len(argv) == 2 and argv[0] == "counters":
        for k, cs in sorted(counter_medians(argv[1]).items(), key=lambda kv: -kv[1]["_dispatches"]):
            print(k, json.dumps(cs))
    elif len(argv) == 6 and argv[0] == "traffic":
        rec = traffic_record(*argv[1:5])
        with open(argv[5], "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        print(json.dumps(rec, indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
