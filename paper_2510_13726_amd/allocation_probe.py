"""Sweep time on several allocations of one workload, and a per-allocation
summary of a rocprofv3 counter pass over the same program.

    python -m paper_2510_13726_amd.allocation_probe --config 5 --trials 4
    python -m paper_2510_13726_amd.allocation_probe --summary CSV LOG --title ... --cmd ... --out FILE.md

The first form creates the lattice `trials` times (each time after holding
one more 512 MiB block, so that its buffers land elsewhere), steps it 3 + 6
times and prints one JSON line per allocation: the buffer addresses, the
sweep launches and their mean duration from HIP events over the last 6.
The second form splits the sweep dispatches of the counter CSV into the
allocations in launch order and writes each counter's mean per dispatch
next to that allocation's sweep time.
"""
import argparse
import collections
import csv
import json


def run(config, trials, storage):
    import torch
    from paper_2510_13726_amd import hlbm, workloads as W
    w = W.ALL[config]()
    hold = []
    for t in range(trials):
        lat = hlbm.setup(w, storage=storage, diag_every=0, check_nonfinite=0)
        lat.step(3)
        hlbm.profile_enable(lat, True)
        lat.step(6)
        n, ms = hlbm.profile_read(lat, hlbm.KERNEL_SWEEP)
        hlbm.profile_enable(lat, False)
        print(json.dumps(dict(trial=t, workload=w.name, storage=storage, a=hex(lat.pop_a.data_ptr()),
                              b=hex(lat.pop_b.data_ptr()), sweeps=n + 3, sweep_ms=round(ms / n, 4))), flush=True)
        lat.close()
        del lat
        torch.cuda.empty_cache()
        hold.append(torch.empty((t + 1) << 29, dtype=torch.uint8, device="cuda"))


def summary(csv_path, log_path, kernel, title, cmd, out):
    trials = [json.loads(line) for line in open(log_path) if line.startswith('{"trial"')]
    rows = collections.defaultdict(dict)
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if kernel in r["Kernel_Name"]:
                rows[int(r["Dispatch_Id"])][r["Counter_Name"]] = float(r["Counter_Value"])
    ids = sorted(rows)
    per = len(ids) // max(len(trials), 1)
    names = sorted({k for v in rows.values() for k in v})
    lines = [f"# {title}", "", "Command (from the repository root, MI355X):", "", f"    {cmd}", "",
             f"Sweep dispatches `{kernel}`: {len(ids)}, {per} per allocation; counters as the mean per dispatch.", "",
             "| allocation | buffer a | sweep ms (HIP events) | " + " | ".join(names) + " |",
             "|---|---|---|" + "---|" * len(names)]
    for t, tr in enumerate(trials):
        grp = ids[t * per:(t + 1) * per]
        cells = []
        for nm in names:
            v = [rows[i][nm] for i in grp if nm in rows[i]]
            cells.append(f"{sum(v) / len(v):.4g}" if v else "—")
        lines.append(f"| {tr['trial']} | {tr['a']} | {tr['sweep_ms']} | " + " | ".join(cells) + " |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="5")
    ap.add_argument("--trials", type=int, default=4)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--summary", nargs=2, metavar=("CSV", "LOG"))
    ap.add_argument("--kernel", default="k_sweep<float, float, false, false, 27>")
    ap.add_argument("--title", default="")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    if a.summary:
        summary(a.summary[0], a.summary[1], a.kernel, a.title, a.cmd, a.out)
    else:
        run(a.config, a.trials, a.storage)


if __name__ == "__main__":
    main()
