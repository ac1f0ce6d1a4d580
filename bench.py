"""Throughput benchmark of the fused LTNE MRT lattice Boltzmann step.

Workload (one GPU): the 8192 x 8192 periodic-x / walled-y porous layer
heated from below (Ra = 1e5, Da = 1e-3, per-node porosity from seeded
smoothed noise, seeded initial temperature noise), all three lattices fused
into one kernel.  The headline number is the FP32 form (shifted binary32
populations; binary32 arithmetic for the flow lattice, binary64 for the two
temperature lattices); the FP64, FP16-storage and FP32-storage /
FP64-arithmetic (stochastic rounding) forms, and the FP32 form with the
Eq. 52 correlation and the Sec. 3.2 correction term, are timed on the same
lattice and reported under "variants".

A step is one time step of all three lattices over the whole lattice.  The
FP32 forms advance two steps per launch (an odd last step of a call
alone; the call's last launch also writes the macroscopic fields); the
other forms one.  Inputs are
resident in device memory before timing starts.  The time of K steps (one
call) is taken with HIP events on the stream the library queues on, between
two device synchronisations.

Prints one JSON line:  value = MLUPS (10^6 lattice-node updates of all three
lattices per second), plus the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (all 3 populations fused) + % HBM peak, FP32 vs FP64; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
N = 8192
WORKLOAD = ("porous layer 8192x8192, periodic x, walls y (bottom T=1, top T=0), Ra=1e5, "
            "Da=1e-3, Pr=1, H_v=10, per-node porosity clip(0.65+0.1 z, 0.4, 0.9), "
            "initial T 0.5 +- 0.05")
# Algorithmic HBM bytes per lattice-node update: 19 populations read and 19
# written in the storage type, plus the per-node porosity in the compute type.
BYTES_PER_LUP = {"f32": 19 * 4 * 2 + 4, "f64": 19 * 8 * 2 + 8, "f16s": 19 * 2 * 2 + 4, "f32sr": 19 * 4 * 2 + 8,
                 "f32ext": 19 * 4 * 2 + 4}
PRECISION = {"f32": 1, "f64": 0, "f16s": 2, "f32sr": 3, "f32ext": 1}
FORM_ARITHMETIC = {
    "f32": "binary32 storage; binary32 flow arithmetic, binary64 temperature arithmetic",
    "f32ext": "binary32 storage; binary32 flow arithmetic, binary64 temperature arithmetic",
    "f64": "binary64 storage and arithmetic",
    "f16s": "binary16 storage (scaled, stochastically rounded); binary32 arithmetic",
    "f32sr": "binary32 storage (stochastically rounded); binary64 arithmetic"}
# f32ext: the FP32 form with both model extensions on -- h_v of every node
# from the correlation of Eq. 52 (D_p = 0.0135 L, the paper's pore size) and
# the correction term of Sec. 3.2 -- at no extra memory traffic.
EXTRA = {"f32ext": dict(thermal_correction=1, pore_size=0.0135)}
KERNEL_SOURCES = ["paper_1608_04118_amd/csrc/step_kernel.hpp", "paper_1608_04118_amd/csrc/step2_kernel.hpp",
                  "paper_1608_04118_amd/csrc/common.hpp",
                  "paper_1608_04118_amd/csrc/host_common.hpp", "paper_1608_04118_amd/csrc/lbm_ltne.hip",
                  "paper_1608_04118_amd/build.py"]


def kernel_hash() -> str:
    """Hash of the kernel sources; in C++ sources, // comments and blank
    lines are left out, so a comment edit keeps counter runs valid."""
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            text = f.read()
        if not s.endswith(".py"):
            lines = (re.sub(rb"//.*$", b"", ln).rstrip() for ln in text.split(b"\n"))
            text = b"\n".join(ln for ln in lines if ln)
        h.update(text)
    return h.hexdigest()[:16]


def _counters(tag: str, name: str):
    """Entry `tag` of a committed counter summary (profiles/<name>.json),
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(tag)
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e


def measured_traffic(tag: str):
    """HBM bytes per launch from committed rocprofv3 counter runs
    (FETCH_SIZE, WRITE_SIZE), if taken on the current kernel sources."""
    e = _counters(tag, "traffic")
    return e.get("bytes_per_launch") if e else None


def measured_valu(tag: str):
    """Wavefront vector instructions per launch (SQ_INSTS_VALU) from a
    committed rocprofv3 counter run, if taken on the current kernel
    sources."""
    e = _counters(tag, "sq")
    return e.get("valu_per_launch") if e else None


# Vector instruction issue: each CU's four SIMDs issue one wavefront
# instruction every four clocks each (a wave64 instruction occupies a 16-lane
# SIMD for four clocks), i.e. one wavefront instruction per clock per CU.
CUS, CLOCK_HZ = 256, 2.4e9
VALU_ISSUE_PER_S = CUS * CLOCK_HZ


# Forms whose steps run two to a launch on the 8192^2 layer (an odd last step
# of a call alone)
TWO_STEP = ("f32", "f32ext", "f64")


def _events_ms(stream, fn):
    import torch
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


def time_form(tag: str, steps: int, warmup: int, inputs):
    """Whole-job rate over `steps` steps of one call (every launch the call
    makes).  For the two-step forms, also the average duration of one
    two-step launch: a call of 2m + 1 steps (m two-step launches and the
    final single step that writes the macros) minus a call of one step."""
    import torch
    from paper_1608_04118_amd import binding as B
    p, phi, Tf0, Ts0 = inputs
    p = dict(p, precision=PRECISION[tag], **EXTRA.get(tag, {}))
    lat = B.Lattice(p, phi=phi, Tf0=Tf0, Ts0=Ts0)
    stream = lat.stream
    if warmup:
        lat.step(warmup)
    ms = _events_ms(stream, lambda: lat.step(steps))
    launch_ms, steps_per_launch = ms / steps, 1
    if tag in TWO_STEP:
        m = max(1, steps // 2)
        t_call = _events_ms(stream, lambda: lat.step(2 * m + 1))
        t_one = _events_ms(stream, lambda: lat.step(1))
        launch_ms, steps_per_launch = (t_call - t_one) / m, 2
    mass, energy, _ = lat.diagnostics()
    if not (np.isfinite(mass) and np.isfinite(energy)):
        raise RuntimeError("%s run diverged" % tag)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    cells = p["nx"] * p["ny"]
    ms_step = ms / steps
    mlups = cells * steps / (ms * 1e-3) / 1e6
    # HBM bytes one launch must move: every population read and written once
    # and the porosity read once per node, whether the launch advances one
    # step or two (the intermediate level of a two-step launch stays on chip)
    bytes_launch = BYTES_PER_LUP[tag] * cells
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    return dict(ms_per_step=ms_step, mlups=mlups, achieved_gbs=achieved,
                frac=achieved / HBM_PEAK_GBS, bytes_per_launch=bytes_launch, launch_ms=launch_ms,
                steps_per_launch=steps_per_launch)


def time_batch(steps: int, warmup: int, autotune: bool = True):
    """The 256-cavity batch (sides 64..512, seeded parameters), FP32: tile
    widths, chunk heights and launch mode chosen by the autotuner, then both
    launch modes timed (launches over all lattices, two steps per launch but
    the last of a call; or one persistent launch); ms_per_step is the mode
    the autotuner chose.  Aggregate node updates per second."""
    import torch
    from paper_1608_04118_amd import binding as B
    from paper_1608_04118_amd import inputs as I
    ps = I.batch()
    bt = B.Batch(ps)
    tuned_ms = bt.autotune(reps=3) if autotune else None
    chosen = bt.info()["persistent"]
    if warmup:
        bt.step(warmup)

    def timed(mode):
        bt.set_mode(mode)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(bt.stream)
        bt.step(steps)
        t1.record(bt.stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps

    ms_launches = timed(0)
    info = bt.info()
    ms_persistent = timed(1)
    bt.macros(0)  # synchronizes and checks the barrier flag
    bt.close()
    nodes = info["nodes"]
    ms_step = ms_persistent if chosen else ms_launches
    # one read and one write of the state (19 binary32 populations, uniform
    # porosity) per two-step launch: 152 B per node per two steps
    achieved = 152 * nodes / (2 * ms_step * 1e-3) / 1e9
    return dict(ms_per_step=ms_step, mlups=nodes / (ms_step * 1e-3) / 1e6, achieved_gbs=achieved,
                frac=achieved / HBM_PEAK_GBS, nodes=nodes, lattices=len(ps), grid=info["grid"],
                mode=("one persistent launch per call" if chosen else
                      "launches over all lattices, two steps per launch (an odd last step alone)"),
                mode_chosen_by="autotuner" if autotune else "default",
                bytes_note="152 B per node per pair of steps (state read and written once)",
                launches_ms_per_step=ms_launches, persistent_ms_per_step=ms_persistent,
                autotune_ms=tuned_ms)


ADJ_WORKLOAD = ("adjoint: 512x512 cavity, FP32, per-node porosity clip(0.65+0.1 z_a, 0.4, 0.9) and "
                "interphase coefficient 10 (1 + 0.5 clip(z_b, -1, 1)), Ra=1e5, Da=1e-3, loss = mean hot-wall "
                "Nu_f after 4000 steps, checkpoints every 200")


def time_adjoint(n_side: int = 512, steps: int = 4000, ckpt: int = 200):
    """Cost of the gradient: lbm_ltne_adjoint over `steps` steps (its own
    forward with checkpoints, the per-segment recompute and the reverse
    sweep) against the plain forward of the same steps, both wall-clock
    around synchronizing calls from a fresh lattice."""
    import torch
    from paper_1608_04118_amd import binding as B
    from paper_1608_04118_amd import inputs as I
    p, phi, Hv = I.adjoint_cavity(n_side, precision=I.FP32)
    B.Lattice(p, phi=phi, Hv=Hv).adjoint(20, 10)  # loads the kernels
    fwd = B.Lattice(p, phi=phi, Hv=Hv)
    torch.cuda.synchronize()
    t = time.perf_counter()
    fwd.step(steps)
    nu = fwd.nusselt()[0]  # synchronizes
    t_fwd = time.perf_counter() - t
    lat = B.Lattice(p, phi=phi, Hv=Hv)
    torch.cuda.synchronize()
    t = time.perf_counter()
    loss, gp, gh = lat.adjoint(steps, ckpt)
    t_adj = time.perf_counter() - t
    fwd.close()
    lat.close()
    if loss != nu or not (np.isfinite(gp).all() and np.isfinite(gh).all()):
        raise RuntimeError("adjoint run inconsistent with the forward")
    return {"workload": ADJ_WORKLOAD, "forward_ms": round(t_fwd * 1e3, 2), "adjoint_ms": round(t_adj * 1e3, 2),
            "cost_ratio": round((t_adj - t_fwd) / t_fwd, 3), "cost_ratio_with_forward": round(t_adj / t_fwd, 3),
            "note": "cost_ratio = (adjoint call - forward) / forward: recompute + reverse sweep per forward; "
                    "the adjoint call also runs the forward itself"}


def copy_bandwidth(gib: float = 1.0, reps: int = 5):
    """Plain device copy of a known size (torch's copy kernel): the
    reference kernel for the rocprofv3 byte counters, and a practical
    bandwidth ceiling next to the published peak."""
    import torch
    n = int(gib * 2 ** 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read": n * 4, "bytes_written": n * 4, "ms": ms, "gbs": 2 * n * 4 / ms / 1e6}


# element type of each two-step form's kernel, as rocprofv3 names it
TWO_STEP_TYPE = {"f32": "float", "f64": "double"}


def is_two_step_kernel(name: str, tag: str = "f32") -> bool:
    """The two-step kernel of form `tag` with the porosity field (the 8192^2
    layer's), by its demangled or mangled name in a rocprofv3 record."""
    t = TWO_STEP_TYPE[tag]
    return ("step2_kernel<%s, 1>" % t) in name or ("step2_kernelI%sLi1E" % t[0]) in name


def _merge_record(out_path: str, tag: str, rec: dict):
    """Writes rec as entry `tag` of a counter summary, keeping the others."""
    try:
        with open(out_path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        t = {}
    t[tag] = rec
    with open(out_path, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps({tag: rec}, indent=1))


def ingest_counters(fetch_csv: str, write_csv: str, copy_bytes: int, out_path: str, tag: str = "f32"):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) of `bench.py --forms <tag>` into HBM bytes per launch of that
    form's two-step kernel (two node updates per node), each scaled by the
    same counter's reading on the plain copy of copy_bytes read and
    copy_bytes written that bench.py times in the same run."""
    import csv

    def per_kernel(path, counter):
        rows = list(csv.DictReader(open(path)))
        vals = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals = per_kernel(path, counter)
        copy = [v for k, vs in vals.items() if "copy" in k.lower()
                for v in vs if v * 1024 > 0.25 * copy_bytes]
        step = [v for k, vs in vals.items() if is_two_step_kernel(k, tag) for v in vs]
        if not copy or not step:
            raise SystemExit("counters for the copy or the step kernel not found in %s" % path)
        scale = copy_bytes / (np.median(copy) * 1024.0)
        out[counter] = {"step_kib_median": float(np.median(step)), "copy_kib_median": float(np.median(copy)),
                        "scale": float(scale), "step_bytes": float(np.median(step) * 1024.0 * scale)}
    total = out["FETCH_SIZE"]["step_bytes"] + out["WRITE_SIZE"]["step_bytes"]
    _merge_record(out_path, tag, {"kernel_hash": kernel_hash(), "bytes_per_launch": total,
                                  "must_move_bytes_per_launch": BYTES_PER_LUP[tag] * N * N,
                                  "one_step_equivalent_bytes_per_launch": BYTES_PER_LUP[tag] * N * N * 2,
                                  "counters": out})


def ingest_sq(csv_path: str, out_path: str, tag: str = "f32"):
    """Turns a rocprofv3 --pmc run with SQ_INSTS_VALU (and SQ_WAVES) of
    `bench.py --forms <tag>` into wavefront vector instructions per launch of
    that form's two-step kernel (median over its dispatches)."""
    import csv
    vals = {}
    for row in csv.DictReader(open(csv_path)):
        k = row["Kernel_Name"]
        if is_two_step_kernel(k, tag):
            vals.setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    if "SQ_INSTS_VALU" not in vals:
        raise SystemExit("SQ_INSTS_VALU of the two-step kernel not found in %s" % csv_path)
    _merge_record(out_path, tag, {"kernel_hash": kernel_hash(),
                                  "valu_per_launch": float(np.median(vals["SQ_INSTS_VALU"])),
                                  "counters": {k: float(np.median(v)) for k, v in vals.items()},
                                  "dispatches": len(vals["SQ_INSTS_VALU"])})


def clock_probe(forms=("f32", "f16s", "f64"), samples: int = 6, interval_s: float = 0.4):
    """Shader and memory clocks (rocm-smi --showclocks) while one form steps
    the 8192^2 layer continuously (400 steps per call, in a loop on a second
    thread), sampled after one second of running; idle first."""
    import subprocess
    import threading
    import torch
    from paper_1608_04118_amd import binding as B
    from paper_1608_04118_amd import inputs as I

    def sample(n):
        out = []
        for _ in range(n):
            r = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True, timeout=30)
            out.append([ln.split(":", 1)[1].strip() for ln in r.stdout.splitlines() if "sclk" in ln or "mclk" in ln])
            time.sleep(interval_s)
        return out

    res = {"idle": sample(2)}
    for tag in forms:
        p, phi, Tf0, Ts0 = I.throughput(n=N, precision=PRECISION[tag])
        lat = B.Lattice(dict(p, **EXTRA.get(tag, {})), phi=phi, Tf0=Tf0, Ts0=Ts0)
        lat.step(20)
        torch.cuda.synchronize()
        stop = threading.Event()

        def run():
            while not stop.is_set():
                lat.step(400)
                torch.cuda.synchronize()
        th = threading.Thread(target=run)
        th.start()
        time.sleep(1.0)
        try:
            res[tag] = sample(samples)
        finally:
            stop.set()
            th.join()
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return res


def persist_probe(mode: int, steps: int = 200):
    """16 cavities of 64^2 (FP32; the single-step batch kernel) stepped in one
    call in the given launch mode (0: a launch per step, 1: persistent), for
    counter runs comparing the modes."""
    import torch
    from paper_1608_04118_amd import binding as B
    from paper_1608_04118_amd import inputs as I
    ps = [I.cavity_small(nx=64, ny=64, precision=I.FP32, Ra=1e4 * (1 + 0.1 * i)) for i in range(16)]
    bt = B.Batch(ps)
    bt.set_mode(mode)
    ms = _events_ms(bt.stream, lambda: bt.step(steps))
    bt.macros(0)  # synchronizes and checks the barrier flag
    info = bt.info()
    bt.close()
    torch.cuda.synchronize()
    return {"mode": mode, "steps": steps, "us_per_step": round(1e3 * ms / steps, 2), "grid": info["grid"],
            "tiles": info["tiles"]}


def cpu_model() -> str:
    """CPU model name of the host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_STRIP_COLS = 512


def _oracle_strip_rate(inputs, budget_s: float):
    import oracle as O
    p, phi, Tf0, Ts0 = inputs
    cols = np.arange(_STRIP_COLS)
    ps = dict(p, nx=len(cols), L=p["ny"] - 1.0)
    o = O.Oracle(ps, phi=phi[:, cols], Tf0=Tf0[:, cols], Ts0=Ts0[:, cols])
    t = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t
    steps = max(1, min(200, int(budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t
    return ps["nx"] * ps["ny"] * steps / dt / 1e6, steps, dt, O.threads()


def _single_thread_rate(budget_s: float):
    """The oracle on the same strip with one OpenMP thread, in a child
    process (the thread count is fixed when the oracle library loads)."""
    import subprocess
    code = ("import sys, json; sys.path.insert(0, %r); import bench; from paper_1608_04118_amd import inputs as I; "
            "r = bench._oracle_strip_rate(I.throughput(n=%d, precision=I.FP32), %r); print(json.dumps(r))"
            % (ROOT, N, budget_s))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                             timeout=10 * budget_s + 120)
        rate, steps, dt, threads = json.loads(out.stdout.strip().splitlines()[-1])
        return {"value": rate, "threads": threads, "steps": steps, "seconds": round(dt, 2)}
    except Exception as e:  # reported, never fatal for the benchmark
        return {"error": str(e)[:200]}


def cpu_baseline(inputs, budget_s: float = 12.0):
    """The FP64 oracle on a periodic strip of the same layer: all 8192 rows,
    512 columns, timed over as many steps as fit the budget, on all host
    threads and (a shorter sample) on one."""
    rate, steps, dt, threads = _oracle_strip_rate(inputs, budget_s)
    return {"value": rate, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 oracle, 8192 rows x 512 columns strip of the same layer, %d steps, "
                      "%.1f s" % (steps, dt),
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "single_thread": _single_thread_rate(budget_s / 3)}


EXTRA_WORKLOADS = {
    "cavity64_fp64": ("64x64 cavity, FP64 (phi 0.6, Da 1e-2, Ra 1e4)", lambda I: (I.cavity_small(), 2000)),
    "cavity1024_fp32": ("1024x1024 cavity, FP32 (phi 0.4, Da 1e-4, Ra 1e6, gamma_sf 10, H_v 100)",
                        lambda I: (I.cavity_large(), 2000)),
    "channel1024x256_fp32": ("1024x256 Brinkman-Forchheimer channel, FP32 (Da 1e-4, Re 10)",
                             lambda I: (I.channel(), 2000)),
    "paper_cavity128_fp64": ("the paper's cavity, 128x128, Ra 1e6, FP64, h_v from Eq. 52",
                             lambda I: (I.paper_cavity(n=128, Ra=1e6), 4000)),
    "paper_cavity192_fp64": ("the paper's cavity, 192x192, Ra 1e9, FP64, h_v from Eq. 52",
                             lambda I: (I.paper_cavity(n=192, Ra=1e9), 4000)),
    "adjoint_cavity512_fp32": ("512x512 cavity of the adjoint workload (Ra 1e5, Da 1e-3; uniform phi 0.65, H_v 10), FP32",
                               lambda I: (I.adjoint_cavity(512)[0], 2000)),
}


def time_extras():
    """Rates of the smaller workloads: the 64^2 FP64 cavity (launch-bound),
    the 1024^2 FP32 cavity (its 159 MB of populations fit in the MI355X's
    256 MB last-level cache) and the 1024 x 256 FP32 channel; one call of
    the stated steps after a warm-up call, HIP events on the library's
    stream."""
    import torch
    from paper_1608_04118_amd import binding as B
    from paper_1608_04118_amd import inputs as I
    out = {}
    for key, (desc, make) in EXTRA_WORKLOADS.items():
        p, steps = make(I)
        lat = B.Lattice(p)
        lat.step(100)
        ms = _events_ms(lat.stream, lambda: lat.step(steps))
        lat.close()
        del lat
        torch.cuda.empty_cache()
        nodes = p["nx"] * p["ny"]
        out[key] = {"workload": desc, "steps": steps, "us_per_step": round(ms * 1e3 / steps, 3),
                    "mlups": round(nodes * steps / (ms * 1e-3) / 1e6, 1)}
    return out


def counter_figures(tag: str, r: dict) -> dict:
    """HBM traffic and vector-issue fractions of a two-step form's launch from
    its committed counter runs (only those taken on the current sources)."""
    out = {}
    launch_s = r["launch_ms"] * 1e-3
    traffic = measured_traffic(tag)
    if traffic:
        out["traffic_bytes_per_launch"] = traffic
        out["traffic_frac"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    valu = measured_valu(tag)
    if valu:
        out["valu_per_node_update"] = round(valu * 64 / (2 * N * N), 1)
        out["valu_issue_frac"] = round(valu / VALU_ISSUE_PER_S / launch_s, 4)
    return out


def roofline(head: str, r: dict, traffic):
    """Roofline of the dominant kernel.  achieved = the HBM bytes one launch
    must move (per node: every population read once and written once in the
    storage type, the porosity read once -- BYTES_PER_LUP; a two-step launch
    moves these once for its two steps) over the launch time measured live.
    The two-step kernel is also put against its vector-instruction issue
    (SQ_INSTS_VALU per launch from the committed counter run), the resource
    that binds it, and its bytes are restated as if every step went to HBM
    (one_step_equivalent: what the same node updates would cost one step per
    launch)."""
    nodes = N * N
    launch_s = r["launch_ms"] * 1e-3
    must = BYTES_PER_LUP[head] * nodes
    achieved = must / launch_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "traffic_gbs": (round(traffic / launch_s / 1e9, 1) if traffic else None),
           "traffic_frac": (round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None),
           "bytes_per_launch": must, "launch_ms": round(r["launch_ms"], 4)}
    if r["steps_per_launch"] == 2:
        eq = must * 2 / launch_s / 1e9
        out["kernel"] = ("step2_kernel<float, kPhiField>: two time steps per launch over %d^2 nodes; %d B per node "
                         "per launch (state read and written once)" % (N, BYTES_PER_LUP[head]))
        out["one_step_equivalent"] = {"bytes_per_launch": must * 2, "gbs": round(eq, 1),
                                      "frac": round(eq / HBM_PEAK_GBS, 4)}
        valu = measured_valu(head)
        if valu:
            floor_ms = valu / VALU_ISSUE_PER_S * 1e3
            out["valu_issue"] = {"wave_instructions_per_launch": valu,
                                 "per_node_update": round(valu * 64 / (2 * nodes), 1),
                                 "issue_floor_ms": round(floor_ms, 4),
                                 "frac": round(floor_ms / r["launch_ms"], 4),
                                 "peak": "one wavefront instruction per clock per CU, 256 CUs, 2.4 GHz"}
        else:
            out["valu_issue"] = None
    else:
        out["kernel"] = "step_kernel: one time step per launch over %d^2 nodes, %d B per node" % (
            N, BYTES_PER_LUP[head])
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="f32,f64,f16s,f32sr,f32ext")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-cavity batch workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint cost measurement (one JSON object)")
    ap.add_argument("--no-copy-check", action="store_true",
                    help="skip the plain 1 GiB device copy (bandwidth reference and counter calibration)")
    ap.add_argument("--copy-check", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the small-workload rates (64^2 FP64 cavity, 1024^2 FP32 cavity, 1024x256 channel)")
    ap.add_argument("--persist-probe", type=int, choices=(0, 1), default=None,
                    help="only step a small batch in launch mode 0 or 1 (for counter runs)")
    ap.add_argument("--clock-probe", action="store_true",
                    help="only sample the shader clock (rocm-smi) while each form runs (one JSON object)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="convert rocprofv3 FETCH_SIZE / WRITE_SIZE runs into profiles/traffic.json")
    ap.add_argument("--ingest-sq", metavar="SQ_CSV",
                    help="convert a rocprofv3 SQ_INSTS_VALU run into profiles/sq.json")
    ap.add_argument("--counters-form", default="f32", choices=sorted(TWO_STEP_TYPE),
                    help="the two-step form whose kernel the ingested counter runs measured")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(args.ingest_counters[0], args.ingest_counters[1], 2 ** 30,
                        os.path.join(ROOT, "profiles", "traffic.json"), args.counters_form)
        return
    if args.ingest_sq:
        ingest_sq(args.ingest_sq, os.path.join(ROOT, "profiles", "sq.json"), args.counters_form)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the step would shard as horizontal slabs with a halo exchange per step); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(2)
    if args.adjoint_only:
        print(json.dumps(time_adjoint()), flush=True)
        return
    if args.clock_probe:
        print(json.dumps(clock_probe()), flush=True)
        return
    if args.persist_probe is not None:
        print(json.dumps(persist_probe(args.persist_probe)), flush=True)
        return
    from paper_1608_04118_amd import inputs as I
    inputs = I.throughput(n=N, precision=I.FP32)
    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for tag in forms:
        print("[bench] timing %s: %d warmup + %d steps on %dx%d" % (tag, args.warmup, args.steps, N, N),
              file=sys.stderr, flush=True)
        res[tag] = time_form(tag, args.steps, args.warmup, inputs)
        print("[bench] %s: %.3f ms/step, %.0f MLUPS, %.0f GB/s algorithmic (%.3f ms per launch of %d step%s)" % (
            tag, res[tag]["ms_per_step"], res[tag]["mlups"], res[tag]["achieved_gbs"], res[tag]["launch_ms"],
            res[tag]["steps_per_launch"], "s" if res[tag]["steps_per_launch"] > 1 else ""),
            file=sys.stderr, flush=True)
    batch = None
    if not args.no_batch:
        print("[bench] timing the 256-cavity batch (FP32)", file=sys.stderr, flush=True)
        batch = time_batch(args.steps, args.warmup)
        print("[bench] batch: %.3f ms/step, %.0f MLUPS, %.0f GB/s" % (
            batch["ms_per_step"], batch["mlups"], batch["achieved_gbs"]), file=sys.stderr, flush=True)
    adjoint = None
    if not args.no_adjoint:
        print("[bench] timing the adjoint (512^2 FP32, 4000 steps)", file=sys.stderr, flush=True)
        adjoint = time_adjoint()
        print("[bench] adjoint: %.1f ms vs forward %.1f ms, cost ratio %.2f" % (
            adjoint["adjoint_ms"], adjoint["forward_ms"], adjoint["cost_ratio"]), file=sys.stderr, flush=True)
    copy = None
    if not args.no_copy_check:
        print("[bench] timing a plain 1 GiB device copy", file=sys.stderr, flush=True)
        copy = copy_bandwidth()
    extras = None
    if not args.no_extras:
        print("[bench] timing the small workloads", file=sys.stderr, flush=True)
        extras = time_extras()
    head = "f32" if "f32" in res else forms[0]
    r = res[head]
    traffic = measured_traffic(head)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(inputs)
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": WORKLOAD + ", %s form" % head, "nx": N, "ny": N,
                   "nodes": N * N, "parallelism": "single GPU",
                   "arithmetic": FORM_ARITHMETIC.get(head)},
        "roofline": roofline(head, r, traffic),
        "cpu_baseline": cpu,
        "copy_reference": copy,
        "extras": extras,
        "variants": {k: dict({kk: (round(vv, 4) if isinstance(vv, float) else vv)
                              for kk, vv in v.items()}, **counter_figures(k, v)) for k, v in res.items()},
        "batch256_f32": batch,
        "adjoint": adjoint,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
