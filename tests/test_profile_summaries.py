"""Host logic of the profile summary writers on small synthetic counter
files: dispatches of the sweep split per allocation in launch order, means
per dispatch, and the copy calibration of the traffic summary."""
import json

from paper_2510_13726_amd import allocation_probe as AP
from paper_2510_13726_amd import profile_traffic as PT

KERNEL = "void hlbm::k_sweep<float, float, false, false, 27>(hlbm::SweepArgs<float>)"


def _csv(path, rows):
    with open(path, "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for r in rows:
            fh.write(f'{r[0]},"{r[1]}",{r[2]},{r[3]}\n')


def test_allocation_summary_splits_dispatches_in_launch_order(tmp_path):
    rows = []
    for d in range(6):  # two allocations of three sweeps, another kernel in between
        rows.append((2 * d, KERNEL, "TCP_UTCL1_TRANSLATION_MISS_sum", 10.0 * (d // 3 + 1) + d % 3))
        rows.append((2 * d + 1, "hlbm::k_wall_geometry", "TCP_UTCL1_TRANSLATION_MISS_sum", 1e9))
    _csv(tmp_path / "c.csv", rows)
    with open(tmp_path / "log", "w") as fh:
        fh.write("noise\n")
        for t, ms in enumerate((11.5, 11.0)):
            fh.write(json.dumps({"trial": t, "a": f"0x{t}", "sweep_ms": ms}) + "\n")
    out = tmp_path / "s.md"
    AP.summary(str(tmp_path / "c.csv"), str(tmp_path / "log"), "k_sweep<float, float, false, false, 27>", "T", "cmd",
               str(out))
    table = [l for l in out.read_text().splitlines() if l.startswith("| 0") or l.startswith("| 1")]
    assert table[0].split("|")[3].strip() == "11.5" and table[0].split("|")[4].strip() == "11"
    assert table[1].split("|")[3].strip() == "11.0" and table[1].split("|")[4].strip() == "21"


def test_traffic_calibration_uses_the_copy_of_known_size():
    rows = {"__amd_rocclr_copyBuffer": [1048576.0, 1048576.0, 3.0], KERNEL: [5.0]}
    f, n = PT.copy_factor(rows)
    assert n == 2 and f == 2.0  # 2 GiB counted as 1 GiB: the counter is scaled by 2
    assert PT.classify(KERNEL) == ("f32", 27)
    assert PT.classify("void hlbm::k_adj_sweep<float, float, false, 27>(hlbm::AdjArgs<float>)") is None
