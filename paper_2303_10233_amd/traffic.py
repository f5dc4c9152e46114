"""Bytes a kernel moves between L2 and memory, from two rocprofv3 counter
runs of `bench.py --counters` (one with FETCH_SIZE, one with WRITE_SIZE, both
in KiB per dispatch), each scaled by what the same counter reads for a plain
copy of known size (n = 2048: 336 MB per vector, beyond every cache).

    python -m paper_2303_10233_amd.traffic --fetch F.csv --write W.csv \\
        --launches counters.json --kernel k_mq_cheb_fused --out profiles/...json

(--kernel k_apply with the record of `bench.py --counters --counters-kernel
apply`: the FP64 saddle apply at n = 2048; --kernel k_apply_oseen or
k_cd_step --precision fp64|mixed with the record of `--counters-kernel
oseen`: the Oseen apply and the damped-Jacobi F smoothing step at n = 2048.)

The result records the sha256 of the kernel's source file, so a reader can
tell when the counters no longer describe the code.
"""
import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = {"k_mq_cheb_fused": "k_mq.hip", "k_apply": "k_apply.hip", "k_cheb_step": "k_gmg.hip",
           "k_apply_oseen": "k_apply.hip", "k_cd_step": "k_oseen.hip"}


def per_dispatch(path, counter):
    """{(kernel name, grid size): [values]} of one counter."""
    out = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            out[(row["Kernel_Name"], int(row["Grid_Size"]))].append(float(row["Counter_Value"]))
    return out


def pick(groups, name_part, grid_size):
    """Mean counter value over the dispatches of one kernel with one grid."""
    v = [x for (name, gs), vals in groups.items() if name_part in name and gs == grid_size for x in vals]
    if not v:
        raise SystemExit(f"no dispatch of {name_part!r} with {grid_size} work-items")
    return sum(v) / len(v), len(v)


def modal_grid(groups, name_part):
    """The grid size most dispatches of a kernel share (the profile loop's)."""
    count = {}
    for (name, gs), vals in groups.items():
        if name_part in name:
            count[gs] = count.get(gs, 0) + len(vals)
    if not count:
        raise SystemExit(f"no dispatch of {name_part!r}")
    return max(count, key=count.get)


def vector_length(n):
    return 2 * (2 * n + 1) ** 2 + (n + 1) ** 2 + n * n


def copy_grid(n):
    """work-items of the profile loop's k_copy (256 per block, one per value)"""
    return -(-vector_length(n) // 256) * 256


def mq_grid(n, tile, steps=1):
    """work-items of k_mq_cheb_fused<T, tile, steps> on one right-hand side
    (ceil(n / tile) blocks per side, the last ones owning node n; one thread
    per entry of a parity array of the staged region for tiles below 32)"""
    qw = tile // 2 + 10 * steps
    threads = 1024 if tile >= 32 else 64 * (-(-qw * qw // 64))
    return (-(-n // tile)) ** 2 * threads


def apply_grid(n):
    """work-items of k_apply (64 x 4 threads per 64 x 16 velocity-node tile)"""
    nq = 2 * n + 1
    return (-(-nq // 64)) * (-(-nq // 16)) * 256


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--launches", required=True, help="the JSON line printed by bench.py --counters")
    ap.add_argument("--kernel", default="k_mq_cheb_fused")
    ap.add_argument("--precision", default=None, help="fp64 or mixed (records with several)")
    ap.add_argument("--commands", nargs=2, metavar=("FETCH_CMD", "WRITE_CMD"), default=None)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    with open(a.launches) as f:
        rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
    n = 2048 if a.kernel in ("k_apply", "k_apply_oseen", "k_cd_step") else rec["n"]
    target = [x for x in rec["launches"] if x["kernel"] == a.kernel and x["n"] == n and
              (a.precision is None or x.get("precision") == a.precision)][0]
    big_copy = [x for x in rec["launches"] if x["kernel"] == "k_copy" and x["n"] == 2048][0]
    small_copy = [x for x in rec["launches"] if x["kernel"] == "k_copy" and x["n"] == n][0]
    fetch = per_dispatch(a.fetch, "FETCH_SIZE")
    write = per_dispatch(a.write, "WRITE_SIZE")
    if a.kernel == "k_mq_cheb_fused":
        steps = target.get("mq_steps_per_launch", 1)
        name = f"{a.kernel}<float, {target['mq_tile']}, {steps}>"
        grid = mq_grid(n, target["mq_tile"], steps)
        workload = f"Stokes cavity {n}x{n}, mixed precision, one launch of the profile loop"
    elif a.kernel == "k_apply":
        name = "k_apply<true, false, false>"
        grid = apply_grid(n)
        workload = f"Stokes saddle apply with its fused dot, FP64, {n}x{n} (one 336 MB vector in, one out)"
    elif a.kernel == "k_apply_oseen":
        name = "k_apply<true, true, false>"
        grid = modal_grid(fetch, name)
        workload = f"Oseen saddle apply with its fused dot, FP64, {n}x{n} (336 MB vector in, one out, wind)"
    elif a.kernel == "k_cd_step":
        t = "float" if target.get("precision") == "mixed" else "double"
        name = f"k_cd_step<{t}, 0, false>"
        grid = modal_grid(fetch, name)
        workload = f"damped-Jacobi F smoothing step, finest level, {t}, {n}x{n}, both velocity planes"
    else:
        raise SystemExit("kernels described here: k_mq_cheb_fused, k_apply, k_apply_oseen, k_cd_step")
    f_kib, nf = pick(fetch, name, grid)
    w_kib, nw = pick(write, name, grid)
    cf_big, _ = pick(fetch, "k_copy", copy_grid(2048))
    cw_big, _ = pick(write, "k_copy", copy_grid(2048))
    cf_small, _ = pick(fetch, "k_copy", copy_grid(n))
    cw_small, _ = pick(write, "k_copy", copy_grid(n))
    half = big_copy["bytes_per_launch"] / 2.0          # bytes read = bytes written
    sf = half / (cf_big * 1024.0)
    sw = half / (cw_big * 1024.0)
    traffic = f_kib * 1024.0 * sf + w_kib * 1024.0 * sw
    src = SOURCES[a.kernel]
    with open(os.path.join(ROOT, "paper_2303_10233_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out = {
        "kernel": name, "source": src, "source_sha256": sha,
        "workload": workload,
        "bytes_per_launch": round(traffic, 1),
        "algorithmic_bytes_per_launch": target["bytes_per_launch"],
        "fetch_kib_per_dispatch": round(f_kib, 3), "write_kib_per_dispatch": round(w_kib, 3),
        "dispatches": {"fetch": nf, "write": nw},
        "copy_calibration": {
            "bytes_read_and_written_each": half, "n": 2048,
            "fetch_kib": round(cf_big, 3), "write_kib": round(cw_big, 3),
            "fetch_scale": round(sf, 5), "write_scale": round(sw, 5),
            "copy_at_workload_size": {"bytes_each": small_copy["bytes_per_launch"] / 2.0,
                                      "fetch_kib": round(cf_small, 3), "write_kib": round(cw_small, 3)},
        },
        "commands": a.commands,
    }
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
