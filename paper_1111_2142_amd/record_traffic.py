"""Record counter-derived figures of a kernel in measured_traffic.json.

    python -m paper_1111_2142_amd.record_traffic --kernel 'k_fwd_march2<128,false>' \
        --workload '...' --profile profiles/....md \
        --fetch F.csv --write W.csv [--valu V.csv] --copy-fetch CF.csv --copy-write CW.csv

Each CSV is the counter_collection.csv of one `rocprofv3 --pmc <counter>
--output-format csv` run: --fetch / --write of FETCH_SIZE and WRITE_SIZE over
a run that launches the kernel, --valu of SQ_INSTS_VALU, and --copy-fetch /
--copy-write of the same two counters over `bench.py --copy-calibration`
(a copy of 256 MiB, read and written once).  The copy fixes the scale of each
counter: bytes read = fetch_scale x FETCH_SIZE x 1024 with fetch_scale =
copied bytes / (its FETCH_SIZE x 1024), and likewise for writes.  The entry
stores the kernel's per-dispatch means, the scaled HBM bytes per launch and
a SHA-256 over the kernel's source files (its .hip file and every local
header it includes, followed transitively), so bench.py reports the figure
only while those sources are unchanged.
"""
import argparse
import csv
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 * 1024 * 1024  # bench.py --copy-calibration: 64 Mi floats

# the .hip file that defines each kernel
KERNEL_SOURCE = {
    "k_fwd_march2": "csrc/lwacm_march2.hip",
    "k_fwd_march_rolled": "csrc/lwacm_march.hip",
    "k_adj_march2": "csrc/lwacm_adjoint_march2.hip",
    "k_adj_march": "csrc/lwacm_adjoint_march.hip",
    "k_fwd_generic": "csrc/lwacm_generic.hip",
    "k_thermal_march": "csrc/lwacm_thermal.hip",
    "k_wall_correction": "csrc/lwacm_walls.hip",
    "k_fwd_d2q9_multi": "csrc/lwacm_d2q9_multi.hip",
}


def kernel_key(name: str) -> str:
    """'void lwacm::(anonymous namespace)::k_x<float, 64>(...)' -> 'k_x<float,64>'."""
    m = re.search(r"(k_\w+)(<[^()]*>)?\(", name)
    if not m:
        return name.strip()
    return (m.group(1) + (m.group(2) or "")).replace(" ", "")


def sources_of(hip: str):
    """The .hip file and the local headers it includes, transitively."""
    out, todo = [], [hip]
    while todo:
        f = todo.pop(0)
        if f in out:
            continue
        out.append(f)
        with open(os.path.join(PKG, f)) as fh:
            for inc in re.findall(r'^#include "([^"]+)"', fh.read(), re.M):
                g = os.path.join(os.path.dirname(f), inc)
                if os.path.exists(os.path.join(PKG, g)):
                    todo.append(g)
    return out


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(PKG, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def mean_counter(path: str, counter: str, key=None):
    """Mean per dispatch of `counter` over the dispatches of kernel `key`
    (all dispatches when key is None), and the number of dispatches."""
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            k = kernel_key(r["Kernel_Name"])
            if key is not None and k != key:
                continue
            d = (k, r.get("Dispatch_Id") or r.get("Correlation_Id") or len(per))
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"{path}: no {counter} rows for {key}")
    return sum(per.values()) / len(per), len(per)


def largest_kernel(path: str, counter: str):
    """The kernel with the largest mean `counter` in a run (the copy)."""
    best = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                best.setdefault(kernel_key(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return max(best, key=lambda k: sum(best[k]) / len(best[k]))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--profile", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--valu")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    a = ap.parse_args()
    base = a.kernel.split("<")[0]
    if base not in KERNEL_SOURCE:
        raise SystemExit(f"unknown kernel {base}")
    copy_k = largest_kernel(a.copy_fetch, "FETCH_SIZE")
    cf, _ = mean_counter(a.copy_fetch, "FETCH_SIZE", copy_k)
    cw, _ = mean_counter(a.copy_write, "WRITE_SIZE", copy_k)
    fetch_scale = round(COPY_BYTES / (cf * 1024.0), 3)
    write_scale = round(COPY_BYTES / (cw * 1024.0), 3)
    f, nf = mean_counter(a.fetch, "FETCH_SIZE", a.kernel)
    w, nw = mean_counter(a.write, "WRITE_SIZE", a.kernel)
    files = sources_of(KERNEL_SOURCE[base])
    rec = {
        "workload": a.workload,
        "sources": files,
        "sources_sha256": sources_sha256(files),
        "fetch_size_kib": round(f, 2),
        "write_size_kib": round(w, 2),
        "dispatches": [nf, nw],
        "copy_kernel": copy_k,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "hbm_bytes_per_launch": int(round(fetch_scale * f * 1024 + write_scale * w * 1024)),
        "profile": a.profile,
    }
    if a.valu:
        v, _ = mean_counter(a.valu, "SQ_INSTS_VALU", a.kernel)
        rec["valu_insts_per_launch"] = int(round(v))
    path = os.path.join(PKG, "measured_traffic.json")
    try:
        db = json.load(open(path))
    except (OSError, ValueError):
        db = {}
    db[a.kernel] = rec
    with open(path, "w") as fh:
        json.dump(db, fh, indent=1)
        fh.write("\n")
    print(json.dumps({a.kernel: rec}))


if __name__ == "__main__":
    main()
