"""Instruction counts per wave of the sweep from a rocprofv3 counter pass.

    python -m paper_2510_13726_amd.profile_counters --csv run_counter_collection.csv \
        --workload rotor_channel_256x128x128 --cells 4194304 --cmd "..." \
        --out profiles/k_sweep_<workload>_instructions.md

For every storage type and velocity set of k_sweep in the pass, the mean
value per dispatch of each counter of the steady-state variant (the one
launched most often), per wave of 64 cells.
"""
import argparse
import collections
import csv

from paper_2510_13726_amd.profile_traffic import classify


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--csv", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--cells", type=int, required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--skip", default="", help="comma-separated counters to leave out of the table")
    ap.add_argument("--note", default="")
    a = ap.parse_args()
    skip = set(x for x in a.skip.split(",") if x)
    vals = collections.defaultdict(lambda: collections.defaultdict(list))  # (st, q) -> name -> counter -> [v]
    counters = []
    with open(a.csv) as fh:
        for r in csv.DictReader(fh):
            c = classify(r["Kernel_Name"])
            if not c:
                continue
            name = r["Counter_Name"]
            if name in skip:
                continue
            if name not in counters:
                counters.append(name)
            vals[c][(r["Kernel_Name"], name)].append(float(r["Counter_Value"]))
    lines = [f"# Vector and scalar instructions per wave of k_sweep, {a.workload} ({a.cells:,} cells per launch)", "",
             "Command (one counter pass):", "", f"    {a.cmd}", "",
             "Mean per dispatch of the steady-state variant. SQ_INSTS_* are wave instructions per wave (one wave "
             "updates 64 cells, one per lane; a vector instruction is executed by every lane).", "",
             *([a.note, ""] if a.note else []),
             "| storage | velocities | " + " | ".join(counters) + " |",
             "|---|---|" + "---|" * len(counters)]
    for key in sorted(vals):
        st, q = key
        by = vals[key]
        names = collections.Counter(k for (k, _c) in by)
        kern = max(names, key=lambda n: len(by[(n, counters[0])]) if (n, counters[0]) in by else 0)
        row = []
        for cn in counters:
            v = by.get((kern, cn), [])
            if not v:
                row.append("—")
                continue
            mean = sum(v) / len(v)
            if cn == "SQ_WAVES":
                row.append(f"{a.cells / mean:.1f} cells per wave")
                continue
            per = mean / a.cells
            if cn.startswith("SQ_INSTS") and "FLOPS" not in cn:
                per *= 64.0  # per wave: 64 cells
            row.append(f"{per:.1f}")
        lines.append(f"| {st} | D3Q{q} | " + " | ".join(row) + " |")
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
