"""Profiling workload and counter summary for the pressure sweep.

Run under rocprofv3 (one counter per run):
    rocprofv3 --pmc FETCH_SIZE -d DIR -o run -- python -m paper_1808_07554_amd.profile_sweep
    rocprofv3 --pmc WRITE_SIZE -d DIR -o run -- python -m paper_1808_07554_amd.profile_sweep
The workload is a 1 GiB plain copy (lbtp_copy_probe, the known-size
reference) followed by a burst of launches of the blocked plain pressure
sweep (lbtp_probe_sweeps) on the 4096 x 4096 injection problem, on D2Q5 or
(--lattice D2Q9) on D2Q9, 9 sweeps per launch, or (--lattice D3Q7) on the
512^3 injection problem, 3 sweeps per launch.  Then, on any machine:
    python -m paper_1808_07554_amd.profile_sweep --summarize FETCH.csv WRITE.csv OUT.txt [--storage S] [--lattice L]
converts the counters of the sweep into HBM bytes per launch with the
copy's bytes-per-count scale and writes a short text summary, and
    python -m paper_1808_07554_amd.profile_sweep --summarize-trace TRACE.csv OUT.txt --title T --command C [--lattice L]
turns the kernel trace of a bench run (rocprofv3 --kernel-trace --output-format
csv) into a per-kernel table with the blocked sweep's achieved rate against the
vector ALU peak, and
    python -m paper_1808_07554_amd.profile_sweep --summarize-counters CSV OUT.txt [--lattice L]
summarises one instruction-counter run of this workload (SQ_* and GRBM_*
counters of one rocprofv3 --pmc pass) for the blocked sweep.
"""
import argparse
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30
# the sources the sweep kernels are compiled from
SWEEP_SOURCES = ("lbtp_kernels.hip", "lbtp_device.h", "lbtp_internal.h", "lbtp_block.hip", "lbtp_block.h")
SWEEP_SOURCES_Q9 = ("lbtp_d2q9.hip", "lbtp_device.h", "lbtp_internal.h")
SWEEP_SOURCES_Q7 = ("lbtp_block3.hip", "lbtp_device.h", "lbtp_internal.h")
# plain sweeps per blocked launch (the library default) and populations
# moved per node (the rest population is not stored)
SWEEPS_PER_LAUNCH = {"D2Q5": 9, "D2Q9": 9, "D3Q7": 3}
MOVING = {"D2Q5": 4, "D2Q9": 8, "D3Q7": 6}


def default_n(lattice):
    return 512 if lattice == "D3Q7" else 4096


def cells_of(lattice, n):
    return n ** 3 if lattice == "D3Q7" else n * n


def grid_name(lattice, n):
    return f"3-D {n}^3" if lattice == "D3Q7" else f"2-D {n}x{n}"


# flops the method itself does in one plain pressure sweep per node (eq. 3-1,
# eq. 3-9a): D2Q5: P = sum of 4 populations / (1 - w0) (3 adds, 1 multiply),
# w1 P (1 multiply), 4 BGK relaxations f - (f - w P)/tau (sub, mul, add each)
# = 17.  D3Q7: P (5 adds, 1 multiply), w1 P, 6 BGK relaxations = 25.  D2Q9:
# P (7 adds, 1 multiply), w1 P and w2 P (2 multiplies), 8 BGK relaxations
# = 34.  The pull corrections of the stored deviations,
# w (P_b(src) - P_b(node)), are a cost of the storage form, not of the
# method, and are not counted.
METHOD_FLOPS_PER_NODE_SWEEP = {"D2Q5": 17, "D3Q7": 25, "D2Q9": 34}
# one fp32 fused multiply-add (two flops) per lane per clock, 64 lanes per
# compute unit, 256 compute units at 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def sweep_sources(lattice="D2Q5"):
    return {"D2Q9": SWEEP_SOURCES_Q9, "D3Q7": SWEEP_SOURCES_Q7}.get(lattice, SWEEP_SOURCES)


def source_digest(lattice="D2Q5"):
    """sha256 over the sweep kernel sources of the lattice (in order): a
    counter summary is valid only for the kernels it was taken on."""
    h = hashlib.sha256()
    for name in sweep_sources(lattice):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def sweep_kernel_name(storage, dim=2, lattice=None, sweeps_per_launch=9):
    """The kernel that runs the plain pull-form pressure sweeps of a full
    chunk with nx % 4 == 0: the blocked kernels (several sweeps per launch:
    the region kernels on D2Q5 and D2Q9, the z-streaming one on D3Q7), else
    the 4-nodes-per-thread sweep."""
    if lattice == "D2Q9":
        return "q9_f_block_kernel" if sweeps_per_launch > 1 else "q9_f_sweep_vec_kernel"
    if dim == 3 and sweeps_per_launch > 1:
        return "f_zstream_kernel"
    if dim == 2 and sweeps_per_launch > 1:
        return "f_block_kernel"
    return "f_sweep_vec_kernel"


def run(storage, n, launches, lattice="D2Q5", coupled_steps=0):
    import ctypes

    import torch

    from . import inputs, lbtp
    dev = torch.device("cuda", 0)
    lib = lbtp.load()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        rc = lib.lbtp_copy_probe(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), COPY_BYTES,
                                 ctypes.c_void_p(stream))
        assert rc == 0, rc
    torch.cuda.synchronize()
    del a, b
    params, fl = inputs.injection_3d(n) if lattice == "D3Q7" else inputs.injection_2d(n)
    if lattice == "D2Q9":
        # the equilibrium of eq. 3-4 needs max(phi)/2 <= beta <= 2 min(phi)
        params = dict(params, lattice="D2Q9", beta=0.2)
    s = lbtp.from_problem(params, m=64, storage=storage)
    s.set_fields(torch.from_numpy(inputs.f32(fl["K"]).ravel()).to(dev),
                 torch.from_numpy(inputs.f32(fl["phi"]).ravel()).to(dev))
    s.set_state(torch.from_numpy(inputs.f32(fl["P0"]).ravel()).to(dev),
                torch.from_numpy(inputs.f32(fl["S0"]).ravel()).to(dev))
    s.update_coefficients()
    s.pressure_solve(-1.0, 20)
    H = s.probe_sweeps(launches)
    # coupled steps (coefficients, one chunk of the pressure solve, the
    # saturation step): the other kernels of a warm step, for their counters
    for _ in range(coupled_steps):
        s.update_coefficients()
        s.pressure_solve(-1.0, 64)
        s.saturation_step()
    torch.cuda.synchronize()
    print(f"profile workload done: copy {COPY_BYTES} B x3, {launches} launches of {H} plain sweeps at "
          f"{grid_name(lattice, n)} "
          f"({lattice}, {storage}), {coupled_steps} coupled steps", flush=True)


# Algorithmic bytes per node of the once-per-step kernels on D2Q5 (read,
# written): the saturation step reads g (5 populations), the pressure
# deviations (4) and their base, 1/tau_f, K and phi, and writes g; with 16-bit
# storage it also reads the input's base saturation and S^n and writes the
# output's base.  The moments read g (and its base), K and phi and write S and
# 1/tau_f.
STEP_BYTES = {
    ("g_sweep", "fp32"): (5 * 4 + 4 * 4 + 4 + 12, 5 * 4),
    ("g_sweep", "16"): (5 * 2 + 4 * 2 + 4 + 12 + 4 + 4, 5 * 2 + 4),
    ("moments_kernel", "fp32"): (5 * 4 + 8, 8),
    ("moments_kernel", "16"): (5 * 2 + 4 + 8, 8),
}


def summarize_step(fetch_csv, write_csv, out_txt, storage, n, command):
    """HBM traffic of the saturation step and the moments (D2Q5) from one
    FETCH_SIZE and one WRITE_SIZE run of the workload with coupled steps,
    scaled by the plain copy's bytes per count, against their algorithmic
    bytes."""
    f_rows = _counter_rows(fetch_csv)
    w_rows = _counter_rows(write_csv)
    copy_f, _ = _per_dispatch(f_rows, "copy_probe")
    copy_w, _ = _per_dispatch(w_rows, "copy_probe")
    scale_f, scale_w = COPY_BYTES / copy_f, COPY_BYTES / copy_w
    cells = n * n
    lines = [f"HBM traffic of the once-per-step kernels, heterogeneous injection {grid_name('D2Q5', n)}, "
             f"D2Q5, {storage} storage",
             f"command: {command}",
             "counters: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own rocprofv3 --pmc run; "
             f"scaled by the plain copy's {scale_f:.2f} / {scale_w:.2f} B per count"]
    for k in ("g_sweep", "moments_kernel"):
        fv, nf = _per_dispatch(f_rows, k)
        wv, _ = _per_dispatch(w_rows, k)
        if fv is None or wv is None:
            continue
        # the kernel's own name (the saturation step runs one or four nodes per thread)
        name = next(_short_name(n).split("<")[0] for n, _, _ in f_rows if k in n)
        ar, aw = STEP_BYTES[(k, "fp32" if storage == "fp32" else "16")]
        fb, wb = fv * scale_f, wv * scale_w
        lines.append(f"{name} ({nf} dispatches): {fb / 1e6:.1f} MB read (algorithmic {ar} B/node = "
                     f"{ar * cells / 1e6:.1f} MB, ratio {fb / (ar * cells):.3f}), {wb / 1e6:.1f} MB written "
                     f"(algorithmic {aw} B/node = {aw * cells / 1e6:.1f} MB, ratio {wb / (aw * cells):.3f})")
    text = "\n".join(lines) + "\n"
    with open(out_txt, "w") as f:
        f.write(text)
    print(text)


def _counter_rows(path):
    with open(path) as f:
        rows = list(csv.DictReader(f))
    out = []
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
        val = r.get("Counter_Value") or r.get("Counter-Value")
        cname = r.get("Counter_Name") or r.get("Counter-Name")
        if val is None:
            continue
        out.append((name, cname, float(val)))
    return out


def _per_dispatch(rows, pattern, exclude=None):
    vals = [v for (k, _, v) in rows if pattern in k and (exclude is None or exclude not in k)]
    return sum(vals) / len(vals) if vals else None, len(vals)


def summarize(fetch_csv, write_csv, out_txt, storage, n, command, lattice="D2Q5"):
    f_rows = _counter_rows(fetch_csv)
    w_rows = _counter_rows(write_csv)
    copy_f, ncf = _per_dispatch(f_rows, "copy_probe")
    copy_w, ncw = _per_dispatch(w_rows, "copy_probe")
    # launches of the blocked plain sweep (each moves the state in and out once)
    kname = sweep_kernel_name(storage, 3 if lattice == "D3Q7" else 2, lattice, SWEEPS_PER_LAUNCH[lattice])
    sw_f, nsf = _per_dispatch(f_rows, kname)
    sw_w, nsw = _per_dispatch(w_rows, kname)
    scale_f = COPY_BYTES / copy_f
    scale_w = COPY_BYTES / copy_w
    fetch_b = sw_f * scale_f
    write_b = sw_w * scale_w
    q1, pop = MOVING[lattice], (4 if storage == "fp32" else 2)
    cells = cells_of(lattice, n)
    alg_read = cells * (q1 * pop + 8)
    alg_write = cells * q1 * pop
    sha = source_digest(lattice)
    text = f"""Blocked pressure sweep HBM traffic per launch ({SWEEPS_PER_LAUNCH[lattice]} plain sweeps), heterogeneous injection {grid_name(lattice, n)}, {lattice}, {storage} storage
command: {command}
counters: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own rocprofv3 --pmc run
calibration: lbtp_copy_probe of {COPY_BYTES} B: FETCH_SIZE {copy_f:.1f} ({ncf} dispatches), WRITE_SIZE {copy_w:.1f} ({ncw}) -> {scale_f:.2f} / {scale_w:.2f} B per count
{kname} ({nsf} dispatches): FETCH_SIZE {sw_f:.1f} -> {fetch_b / 1e6:.1f} MB read (algorithmic {alg_read / 1e6:.1f} MB, ratio {fetch_b / alg_read:.3f})
{kname} ({nsw} dispatches): WRITE_SIZE {sw_w:.1f} -> {write_b / 1e6:.1f} MB written (algorithmic {alg_write / 1e6:.1f} MB, ratio {write_b / alg_write:.3f})
bytes_per_launch: {fetch_b + write_b:.6e}
algorithmic_bytes_per_launch: {alg_read + alg_write:.6e}
source_sha256: {sha}  (csrc/{", csrc/".join(sweep_sources(lattice))})
"""
    with open(out_txt, "w") as f:
        f.write(text)
    print(text)


def _demangle_lbtp(name):
    """Readable form of a mangled kernel name of this library that the
    profiler left mangled (it does so where a template argument is
    _Float16): name<args> for the argument kinds the kernels use (types,
    bools, ints); None for anything else."""
    import re
    m = re.match(r"_ZN4lbtp12_GLOBAL__N_1(\d+)", name)
    if not m:
        return None
    k = m.end()
    ident = name[k:k + int(m.group(1))]
    k += int(m.group(1))
    if k >= len(name) or name[k] != "I":
        return ident
    k += 1
    args = []
    simple = {"f": "float", "d": "double", "i": "int", "b": "bool"}
    while k < len(name) and name[k] != "E":
        if name.startswith("DF16_", k):
            args.append("_Float16")
            k += 5
        elif name[k] in simple:
            args.append(simple[name[k]])
            k += 1
        elif name[k] == "L":
            lit = re.match(r"L([bi])(n?\d+)E", name[k:])
            if not lit:
                return None
            v = lit.group(2).replace("n", "-")
            args.append(("true" if v == "1" else "false") if lit.group(1) == "b" else v)
            k += lit.end()
        elif name[k] == "N":
            nested = re.match(r"NS\d*_(\d+)", name[k:])
            if not nested:
                return None
            j = k + nested.end()
            args.append(name[j:j + int(nested.group(1))])
            k = j + int(nested.group(1)) + 1   # the closing E
        else:
            return None
    return f"{ident}<{', '.join(args)}>"


def _short_name(name):
    """Kernel name without return type, namespaces and argument list."""
    if name.startswith("_Z"):
        name = _demangle_lbtp(name) or name
    name = name.replace("void ", "").replace("lbtp::", "").replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def d2q5_block_length(grid_x, n, rows=72):
    """Sweeps per launch of a D2Q5 blocked launch (regions of 64 columns x
    `rows` rows, 512 threads, tiles of (64 - 2H) x (rows - 2H) nodes; 72 rows
    without a pressure source) on an n x n grid, from its grid size; None if
    no block length gives it."""
    for h in range(3, 25, 2):
        tx = -(-n // (64 - 2 * h))
        ty = -(-n // (rows - 2 * h))
        if tx * ty * 512 == grid_x:
            return h
    return None


def summarize_trace(trace_csv, out_txt, title, command, lattice="D2Q5", n=4096, sweeps_per_launch=None):
    sweeps_per_launch = sweeps_per_launch or SWEEPS_PER_LAUNCH[lattice]
    with open(trace_csv) as f:
        rows = list(csv.DictReader(f))
    agg = {}
    for r in rows:
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        name = _short_name(r["Kernel_Name"])
        # D2Q5 chunks mix block lengths: one row per length
        if lattice == "D2Q5" and name.split("<")[0] in ("f_block_kernel", "f_block_first_kernel"):
            h = d2q5_block_length(int(r["Grid_Size_X"]), n)
            if h is not None:
                name = f"{name} H={h}"
        agg.setdefault(name, []).append(us)
    total = sum(sum(v) for v in agg.values())
    lines = [title, f"command: {command}", "",
             f"{'kernel':66s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k[:66]:66s} {len(v):6d} {sum(v) / len(v):9.2f} {min(v):9.2f} {max(v):9.2f} "
                     f"{100 * sum(v) / total:6.2f}")
    kname = sweep_kernel_name("fp32", 3 if lattice == "D3Q7" else 2, lattice, sweeps_per_launch)
    blk = [v for k, v in agg.items() if k.split("<")[0] == kname and
           (lattice != "D2Q5" or k.endswith(f" H={sweeps_per_launch}"))]
    if blk:
        d = blk[0]
        avg = sum(d) / len(d)
        fl = METHOD_FLOPS_PER_NODE_SWEEP[lattice] * cells_of(lattice, n) * sweeps_per_launch
        lines += ["", f"{kname} runs {sweeps_per_launch} plain pressure sweeps per launch; average launch "
                  f"{avg:.1f} us = {avg / sweeps_per_launch:.2f} us per sweep;",
                  f"{METHOD_FLOPS_PER_NODE_SWEEP[lattice]} method flops per node and sweep (eq. 3-1, eq. 3-9a) x "
                  f"{cells_of(lattice, n)} nodes x {sweeps_per_launch} = {fl / 1e9:.2f} GFLOP per launch",
                  f"-> {fl / (avg * 1e-6) / 1e12:.2f} TFLOP/s against {ALU_PEAK_TFLOPS:.2f} TFLOP/s (one fp32 fused "
                  "multiply-add per lane and clock, 64 lanes per CU, 256 CUs, 2.4 GHz), frac "
                  f"{fl / (avg * 1e-6) / 1e12 / ALU_PEAK_TFLOPS:.3f}"]
    text = "\n".join(lines) + "\n"
    with open(out_txt, "w") as f:
        f.write(text)
    print(text)


def summarize_counters(csv_path, out_txt, command, lattice="D2Q5", n=4096, sweeps_per_launch=None):
    """Per-dispatch averages of the counters of one --pmc run over the blocked
    sweep's launches, and the vector issue they imply: a wave64 fp32
    instruction occupies its SIMD (16 lanes) for 4 cycles, and the chip has
    1024 SIMDs; the launch time comes from the same dispatches' timestamps."""
    sweeps_per_launch = sweeps_per_launch or SWEEPS_PER_LAUNCH[lattice]
    kname = sweep_kernel_name("fp32", 3 if lattice == "D3Q7" else 2, lattice, sweeps_per_launch)
    with open(csv_path) as f:
        rows = [r for r in csv.DictReader(f) if _short_name(r["Kernel_Name"]).split("<")[0] == kname]
    per = {}
    times = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        times[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    dur = sum(times.values()) / len(times)
    avg = {k: sum(v) / len(v) for k, v in per.items()}
    lines = [f"Instruction counters of {kname} ({sweeps_per_launch} plain pressure sweeps per launch), "
             f"heterogeneous injection {grid_name(lattice, n)}, {lattice}, fp32 storage",
             f"command: {command}", f"dispatches: {len(times)}, mean duration {dur * 1e6:.1f} us", ""]
    for k in sorted(avg):
        lines.append(f"{k:24s} {avg[k]:16.6e} per dispatch")
    if "SQ_INSTS_VALU" in avg:
        issue = avg["SQ_INSTS_VALU"] * 4 / 1024 / 2.4e9
        node_sweeps = cells_of(lattice, n) * sweeps_per_launch
        lines += ["", f"vector issue: {avg['SQ_INSTS_VALU']:.3e} wave instructions x 4 cycles / 1024 SIMDs = "
                  f"{issue * 1e6:.1f} us at 2.4 GHz = {issue / dur:.2f} of the launch",
                  f"per tile node and sweep: {avg['SQ_INSTS_VALU'] * 64 / node_sweeps:.2f} lane instructions "
                  f"(method flops {METHOD_FLOPS_PER_NODE_SWEEP[lattice]})"]
    if "GRBM_GUI_ACTIVE" in avg:
        # the GRBM counters sum over the 8 XCDs
        clk = avg["GRBM_GUI_ACTIVE"] / 8 / dur
        lines.append(f"clock held: GRBM_GUI_ACTIVE / 8 XCDs / duration = {clk / 1e9:.2f} GHz; vector issue at that "
                     f"clock {avg['SQ_INSTS_VALU'] * 4 / 1024 / clk / dur:.2f} of the launch")
    if "SQ_BUSY_CYCLES" in avg and "GRBM_GUI_ACTIVE" in avg:
        lines.append(f"SQ_BUSY_CYCLES / GRBM_GUI_ACTIVE = {avg['SQ_BUSY_CYCLES'] / avg['GRBM_GUI_ACTIVE']:.3f}")
    if "SQ_ACTIVE_INST_VALU" in avg and "SQ_WAVE_CYCLES" in avg:
        lines.append(f"SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES = {avg['SQ_ACTIVE_INST_VALU'] / avg['SQ_WAVE_CYCLES']:.3f} "
                     "(share of a wavefront's cycles spent issuing vector instructions)")
    text = "\n".join(lines) + "\n"
    with open(out_txt, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--n", type=int, default=None, help="grid size (default 4096, 512 on D3Q7)")
    ap.add_argument("--launches", type=int, default=20)
    ap.add_argument("--lattice", default="D2Q5", choices=["D2Q5", "D2Q9", "D3Q7"])
    ap.add_argument("--summarize", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_TXT"))
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_CSV", "OUT_TXT"))
    ap.add_argument("--summarize-counters", nargs=2, metavar=("CSV", "OUT_TXT"))
    ap.add_argument("--coupled-steps", type=int, default=0,
                    help="coupled steps after the sweep burst (their kernels' counters; D2Q5)")
    ap.add_argument("--summarize-step", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_TXT"))
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default=None, help="command line recorded in the summary (default: the one "
                    "that profiles this module with --storage and --n as given)")
    a = ap.parse_args()
    if a.n is None:
        a.n = default_n(a.lattice)
    if a.summarize_trace:
        summarize_trace(*a.summarize_trace, a.title, a.command or "", a.lattice, a.n)
    elif a.summarize_counters:
        summarize_counters(*a.summarize_counters, a.command or "", a.lattice, a.n)
    elif a.summarize_step:
        args = f"--storage {a.storage} --coupled-steps 10"
        command = a.command or (
            "cd /tmp && export TMPDIR=/tmp; rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o run -- "
            f"python -u -m paper_1808_07554_amd.profile_sweep {args}  (then the same with --pmc WRITE_SIZE); "
            "summary: python -m paper_1808_07554_amd.profile_sweep --summarize-step FETCH.csv WRITE.csv OUT.txt "
            f"--storage {a.storage}")
        summarize_step(*a.summarize_step, a.storage, a.n, command)
    elif a.summarize:
        args = (f"--storage {a.storage}" + (f" --n {a.n}" if a.n != default_n(a.lattice) else "")
                + (f" --lattice {a.lattice}" if a.lattice != "D2Q5" else ""))
        command = a.command or (
            "cd /tmp && export TMPDIR=/tmp; rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o run -- "
            f"python -u -m paper_1808_07554_amd.profile_sweep {args}  (then the same with --pmc WRITE_SIZE); "
            f"summary: python -m paper_1808_07554_amd.profile_sweep --summarize FETCH.csv WRITE.csv OUT.txt {args}")
        summarize(*a.summarize, a.storage, a.n, command, a.lattice)
    else:
        run(a.storage, a.n, a.launches, a.lattice, a.coupled_steps)
        sys.exit(0)
