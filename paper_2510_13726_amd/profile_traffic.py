"""HBM traffic of the sweep kernel from two rocprofv3 counter passes.

    python -m paper_2510_13726_amd.profile_traffic --fetch F.csv --write W.csv \
        --workload rotor_array_1536x768x256 --cells 301989888 --out profiles \
        --fetch-cmd "..." --write-cmd "..."

F.csv / W.csv: run_counter_collection.csv of a FETCH_SIZE pass and of a
WRITE_SIZE pass over the same program, which also copies a 2 GiB tensor
(__amd_rocclr_copyBuffer).  The counters read KiB per dispatch; each is
scaled by what it reads for that copy of known size (2 GiB read, 2 GiB
written).  For every storage type and velocity set of k_sweep found, the
script writes sweep_traffic_<workload>[_d3q19]_<storage>.json (bytes per
launch, with the hash of the kernel sources it was taken on) and one
markdown table k_sweep_<workload>_traffic.md holding both commands.
"""
import argparse
import collections
import csv
import json
import os

from paper_2510_13726_amd.provenance import kernel_hash

ELEM = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
COPY_KIB = 2 * 1024 * 1024  # the 2 GiB reference copy, read once and written once


def classify(name):
    """(storage, q) of a k_sweep dispatch name, or None for other kernels."""
    if "k_sweep" not in name or "adj" in name:
        return None
    if "bf16_t" in name:
        st = "bf16"
    elif "DF16_" in name or "_Float16" in name:
        st = "f16"
    elif "k_sweep<float" in name:
        st = "f32"
    elif "k_sweep<double" in name:
        st = "f64"
    else:
        return None
    q = 19 if (", 19>" in name or "Li19E" in name) else 27
    return st, q


def load(path, counter):
    rows = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                rows[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return rows


def copy_factor(rows):
    vals = [v for k, vs in rows.items() if "copyBuffer" in k for v in vs]
    if not vals:
        raise SystemExit("no __amd_rocclr_copyBuffer dispatch: the program must copy a 2 GiB tensor")
    top = max(vals)
    big = [v for v in vals if v >= 0.9 * top]
    return COPY_KIB / (sum(big) / len(big)), len(big)


def sweep_groups(rows):
    """(storage, q) -> per-variant lists of counter values."""
    out = collections.defaultdict(dict)
    for k, vs in rows.items():
        c = classify(k)
        if c:
            out[c][k] = vs
    return out


def dominant(variants):
    """The variant with the most dispatches (the steady-state launch) and its mean."""
    k = max(variants, key=lambda n: len(variants[n]))
    v = variants[k]
    return k, len(v), sum(v) / len(v)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--cells", type=int, required=True)
    ap.add_argument("--out", default="profiles")
    ap.add_argument("--fetch-cmd", default="")
    ap.add_argument("--write-cmd", default="")
    a = ap.parse_args()
    fr, wr = load(a.fetch, "FETCH_SIZE"), load(a.write, "WRITE_SIZE")
    ff, nf = copy_factor(fr)
    wf, nw = copy_factor(wr)
    fg, wg = sweep_groups(fr), sweep_groups(wr)
    h = kernel_hash()
    md = os.path.join(a.out, f"k_sweep_{a.workload}_traffic.md")
    lines = [f"# HBM traffic of k_sweep, {a.workload} ({a.cells:,} cells per launch)", "",
             "Two counter passes of the same program (one counter each):", "",
             f"    {a.fetch_cmd}", f"    {a.write_cmd}", "",
             f"Calibration on the 2 GiB copy of the same runs (__amd_rocclr_copyBuffer, {nf} / {nw} dispatches): "
             f"FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {wf:.4f}.  Kernel sources hash {h}.", "",
             "| storage | velocities | variant dispatches | FETCH_SIZE KiB | bytes read | algorithmic read | "
             "WRITE_SIZE KiB | bytes written | algorithmic write | total / algorithmic |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for key in sorted(set(fg) & set(wg)):
        st, q = key
        _, n1, fk = dominant(fg[key])
        _, n2, wk = dominant(wg[key])
        rd, wt = fk * ff * 1024, wk * wf * 1024
        algo_half = q * ELEM[st] * a.cells
        ratio = (rd + wt) / (2 * algo_half)
        lines.append(f"| {st} | D3Q{q} | {n1}/{n2} | {fk:.1f} | {rd:,.0f} | {algo_half:,} | {wk:.1f} | {wt:,.0f} | "
                     f"{algo_half:,} | {ratio:.4f} |")
        tag = "" if q == 27 else "_d3q19"
        rec = {"kernel_hash": h, "bytes_per_launch": int(round(rd + wt)), "read_bytes": int(round(rd)),
               "write_bytes": int(round(wt)), "fetch_kib": fk, "write_kib": wk, "fetch_factor": ff,
               "write_factor": wf, "algorithmic_bytes": 2 * algo_half, "dispatches": [n1, n2], "source": md}
        with open(os.path.join(a.out, f"sweep_traffic_{a.workload}{tag}_{st}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(f"{st} D3Q{q}: {ratio:.4f} x algorithmic")
    lines += ["", "Each row averages the sweep variant launched most often (the steady-state step)."]
    with open(md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
