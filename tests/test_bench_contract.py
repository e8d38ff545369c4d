"""Host-side checks of bench.py and the profile summaries that need no GPU: the one-GPU rule, the
algorithmic bytes of a plain pressure sweep per node, the ALU peak derived
from the unit counts, and that the committed counter summaries are used only
while they were taken on the current sweep sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_algorithmic_bytes_per_node():
    # Q - 1 deviations read and written, 1/tau_f and the base pressure read
    assert bench.f_sweep_bytes("D2Q5", "fp32") == 2 * 4 * 4 + 8 == 40
    assert bench.f_sweep_bytes("D2Q5", "fp16") == 2 * 4 * 2 + 8
    assert bench.f_sweep_bytes("D3Q7", "fp32") == 2 * 6 * 4 + 8
    assert bench.f_sweep_bytes("D2Q9", "bf16") == 2 * 8 * 2 + 8


def test_method_flops_per_node_sweep():
    # D2Q5: P (3 adds, 1 mul), w1 P (1 mul), 4 x BGK (sub, mul, add);
    # D2Q9: P (7 adds, 1 mul), w1 P, w2 P, 8 x BGK
    assert bench.BLOCK_FLOPS_PER_NODE_SWEEP == {"D2Q5": 3 + 1 + 1 + 4 * 3, "D3Q7": 5 + 1 + 1 + 6 * 3,
                                                "D2Q9": 7 + 1 + 2 + 8 * 3}


def test_alu_peak_from_unit_counts():
    # 256 compute units x 64 lanes x one FMA (2 flops) per clock x 2.4 GHz
    assert abs(bench.ALU_PEAK_TFLOPS - 78.6432) < 1e-9
    assert bench.HBM_PEAK_GBS == 8000.0


def test_traffic_only_for_matching_sources(monkeypatch, tmp_path):
    path = tmp_path / "traffic_{}.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("fp32") is None                  # no summary
    (tmp_path / "traffic_fp32.txt").write_text(
        f"bytes_per_launch: 8.0e+08\nsource_sha256: {bench.source_digest()}  (sources)\n")
    assert bench.measured_traffic("fp32") == 8.0e8
    monkeypatch.setattr(bench, "TRAFFIC_FILE_Q9", str(tmp_path / "q9_{}.txt"))
    assert bench.measured_traffic("fp32", "D2Q9") is None          # none for the other lattice
    monkeypatch.setattr(bench, "source_digest", lambda *a: "0" * 64)  # sources changed since
    assert bench.measured_traffic("fp32") is None


def _counter_csv(path, counter, rows):
    lines = ["Kernel_Name,Counter_Name,Counter_Value"] + [f'"{k}",{counter},{v}' for k, v in rows]
    path.write_text("\n".join(lines) + "\n")


def test_step_traffic_summary(tmp_path):
    """The per-kernel summary of the saturation step and moments scales each
    counter by the plain copy's bytes per count and divides by the kernel's
    algorithmic bytes (D2Q5, 52 + 20 B per node in fp32 for the saturation
    step, 28 + 8 B for the moments)."""
    from paper_1808_07554_amd import profile_sweep as ps
    n = 64
    cells = n * n
    cf, cw = ps.COPY_BYTES / 2048.0, ps.COPY_BYTES / 1024.0      # copy counts: 2048 / 1024 B per count
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [("lbtp_copy_probe", cf), ("g_sweep_kernel<2, float, false, false>",
                                       52 * cells * 1.5 / 2048.0), ("moments_kernel<2, false, float>",
                                                                     28 * cells / 2048.0)])
    _counter_csv(write, "WRITE_SIZE", [("lbtp_copy_probe", cw), ("g_sweep_kernel<2, float, false, false>",
                                       20 * cells / 1024.0), ("moments_kernel<2, false, float>",
                                                               8 * cells / 1024.0)])
    out = tmp_path / "out.txt"
    ps.summarize_step(str(fetch), str(write), str(out), "fp32", n, "cmd")
    text = out.read_text()
    assert "g_sweep_kernel (1 dispatches)" in text and "ratio 1.500" in text and "ratio 1.000" in text
    assert "algorithmic 52 B/node" in text and "algorithmic 28 B/node" in text


def test_mangled_kernel_names_read():
    from paper_1808_07554_amd import profile_sweep as ps
    assert ps._short_name("_ZN4lbtp12_GLOBAL__N_114f_block_kernelIDF16_Lb0ELi8ELi9EEEvNS_2KCENS_5FPtrsES3_PKf"
                          ) == "f_block_kernel<_Float16, false, 8, 9>"
    assert ps._short_name("_ZN4lbtp12_GLOBAL__N_114f_block_kernelINS0_6bf16_tELb1ELi8ELi8EEEvNS_2KC"
                          ) == "f_block_kernel<bf16_t, true, 8, 8>"
    assert ps._short_name("void lbtp::(anonymous namespace)::g_sweep_kernel<2, float, false, false>(lbtp::KC)"
                          ) == "g_sweep_kernel<2, float, false, false>"
