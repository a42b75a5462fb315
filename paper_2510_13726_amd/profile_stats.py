"""Markdown summary of a rocprofv3 --kernel-trace --stats run.

    python -m paper_2510_13726_amd.profile_stats --stats run_kernel_stats.csv \
        --title "..." --cmd "..." --out profiles/k_sweep_<workload>_kernel_stats.md

Lists the kernels above 0.1 % of the GPU time with calls and durations in
microseconds, and the command that produced the run.
"""
import argparse
import csv


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--note", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    with open(a.stats) as fh:
        rows = list(csv.DictReader(fh))
    lines = [f"# {a.title}", "", "Command (from the repository root, MI355X):", "", f"    {a.cmd}", ""]
    if a.note:
        lines += [a.note, ""]
    lines += ["run_kernel_stats.csv, kernels above 0.1 % of the GPU time (durations in microseconds):", "",
              "| kernel | calls | average us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["Percentage"])):
        if float(r["Percentage"]) < 0.1:
            continue
        name = r["Name"].replace("|", "\\|")
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
