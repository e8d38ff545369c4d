"""Profiling workload and per-layer summary of the warm-start network.

Run under rocprofv3:
    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run -- python -m paper_1808_07554_amd.profile_nn
The workload: inference of the 4-level, 32-channel network on one 1024 x 1024
field (factor 1: every layer at full resolution; one warm-up pass and three
timed ones), then three training steps on 32 fields of 64 x 64.  Then, on any
machine:
    python -m paper_1808_07554_amd.profile_nn --summarize DIR/.../run_kernel_trace.csv OUT.txt
lists every convolution of an inference pass with its duration (mean of the
three timed passes), its flops, its algorithmic bytes (input and output
activations in bf16, weights in bf16, read or written once), and achieved
TFLOP/s against min(2.5 PFLOP/s, 8 TB/s x flops/byte): the bf16 matrix-core
peak or the HBM roof at that arithmetic intensity.
"""
import argparse
import csv
import os
import sys

BASE, LEVELS, SCALE = 32, 4, 3.2
PEAK_TFLOPS = 2500.0       # dense bf16 matrix cores
HBM_GBPS = 8000.0
INFER = (1, 1024, 1024)    # N, H, W
TRAIN = (32, 64, 64)


def pad16(c):
    return (c + 15) // 16 * 16


def layers(N, H, W, base=BASE, levels=LEVELS):
    """(name, N, h, w, ci, co) of every 3x3 convolution of one forward pass, in
    launch order (the order of lbtp_nn's forward)."""
    c = [base << lv for lv in range(levels)]
    out, h, w, prev = [], H, W, 3
    for lv in range(levels):
        if lv > 0:
            h, w = h // 2, w // 2
        out.append((f"enc{lv}a", N, h, w, prev, c[lv]))
        out.append((f"enc{lv}b", N, h, w, c[lv], c[lv]))
        prev = c[lv]
    for lv in range(levels - 2, -1, -1):
        h, w = h * 2, w * 2
        out.append((f"dec{lv}a", N, h, w, c[lv + 1] + c[lv], c[lv]))
        out.append((f"dec{lv}b", N, h, w, c[lv], c[lv]))
    out.append(("head", N, h, w, c[0], 1))
    return out


def _run():
    import numpy as np
    import torch

    from . import lbtp
    torch.cuda.set_device(0)
    net = lbtp.WarmStartNet(BASE, LEVELS, SCALE)
    rng = np.random.default_rng(5)
    # He-scaled random weights (the layer order and sizes of the network)
    theta = []
    for (_, _, _, _, ci, co) in layers(1, 64, 64):
        theta.append(rng.standard_normal(co * 9 * ci) * np.sqrt(2.0 / (9 * ci)))
        theta.append(np.zeros(co))
    theta = np.concatenate(theta).astype(np.float32)
    assert theta.size == net.n_params, (theta.size, net.n_params)
    net.set_params(theta)
    N, H, W = INFER
    lnK = torch.from_numpy(rng.standard_normal((N, H, W)).astype(np.float32)).cuda()
    S = torch.from_numpy(rng.uniform(0, 1, (N, H, W)).astype(np.float32)).cuda()
    for _ in range(4):
        net.predict(lnK, S, 1)
        torch.cuda.synchronize()
    N, H, W = TRAIN
    lnK = torch.from_numpy(rng.standard_normal((N, H, W)).astype(np.float32)).cuda()
    S = torch.from_numpy(rng.uniform(0, 1, (N, H, W)).astype(np.float32)).cuda()
    P = torch.from_numpy((1.0 - (np.arange(W) + 0.5) / W)[None, None, :].repeat(N, 0).repeat(H, 1)
                         .astype(np.float32)).cuda()
    for _ in range(3):
        net.train_step(lnK, S, P, 1e-4)
        torch.cuda.synchronize()
    net.close()
    print("profile_nn: done", flush=True)


def summarize(trace_csv, out_path):
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    conv = [r for r in rows if "conv3x3_kernel" in r["Kernel_Name"]]
    ls = layers(*INFER)
    n = len(ls)
    passes = [conv[i * n:(i + 1) * n] for i in range(4)]
    lines = ["Warm-start network, per-layer convolution (implicit GEMM on v_mfma_f32_16x16x32_bf16, LDS-tiled), "
             f"inference of one {INFER[1]}x{INFER[2]} field at full resolution",
             "command: cd /tmp && export TMPDIR=/tmp; rocprofv3 --kernel-trace --stats --output-format csv -d DIR "
             "-o run -- python -m paper_1808_07554_amd.profile_nn; summary: python -m "
             "paper_1808_07554_amd.profile_nn --summarize DIR/.../run_kernel_trace.csv OUT.txt",
             "flops = 2 N h w 9 ci co (real channels); bytes = bf16 input + output activations + bf16 weights, "
             "each once; roof = min(2500 TFLOP/s, 8 TB/s x flops/byte)",
             "",
             f"{'layer':8s} {'h x w':>11s} {'ci':>4s} {'co':>4s} {'us':>9s} {'GFLOP':>8s} {'flop/B':>7s} "
             f"{'TFLOP/s':>8s} {'roof':>8s} {'frac':>6s}"]
    tot_t = tot_f = 0.0
    for i, (name, N, h, w, ci, co) in enumerate(ls):
        ds = [(int(p[i]["End_Timestamp"]) - int(p[i]["Start_Timestamp"])) / 1e3 for p in passes[1:]]
        us = sum(ds) / len(ds)
        flops = 2.0 * N * h * w * 9 * ci * co
        byts = 2.0 * N * h * w * (ci + co) + 2.0 * 9 * ci * co
        ai = flops / byts
        roof = min(PEAK_TFLOPS, HBM_GBPS * ai / 1e3)
        ach = flops / (us * 1e-6) / 1e12
        tot_t += us
        tot_f += flops
        lines.append(f"{name:8s} {h:5d}x{w:<5d} {ci:4d} {co:4d} {us:9.1f} {flops / 1e9:8.2f} {ai:7.1f} "
                     f"{ach:8.2f} {roof:8.1f} {ach / roof:6.3f}")
    lines.append(f"{'total':8s} {'':11s} {'':4s} {'':4s} {tot_t:9.1f} {tot_f / 1e9:8.2f} {'':7s} "
                 f"{tot_f / (tot_t * 1e-6) / 1e12:8.2f}")
    # training steps: every kernel of the three steps, by name
    train = [r for r in rows if int(r["Start_Timestamp"]) > int(passes[-1][-1]["End_Timestamp"])]
    agg = {}
    for r in train:
        nm = r["Kernel_Name"].replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        agg.setdefault(nm, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines += ["", f"Training: 3 Adam steps on {TRAIN[0]} fields of {TRAIN[1]}x{TRAIN[2]} (forward, loss, "
              "backward-data, weight gradients, Adam), kernel time per step:"]
    step_us = 0.0
    for nm, ds in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"  {nm[:60]:60s} {len(ds) // 3:4d} calls  {sum(ds) / 3:9.1f} us")
        step_us += sum(ds) / 3
    fwd_f = sum(2.0 * N * h * w * 9 * ci * co for (_, N, h, w, ci, co) in layers(*TRAIN))
    lines.append(f"  total {step_us:.1f} us per step; forward {fwd_f / 1e9:.2f} GFLOP, forward + backward "
                 f"about 3x that: {3 * fwd_f / (step_us * 1e-6) / 1e12:.2f} TFLOP/s over the step")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize", nargs=2, metavar=("TRACE_CSV", "OUT"))
    a = ap.parse_args()
    if a.summarize:
        summarize(*a.summarize)
    else:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        _run()
