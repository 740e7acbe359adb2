"""Benchmark of the MacLAB time step on one MI355X.

Default workload: D3Q19 lid-driven cube, 256^3 nodes including walls,
Re = 400 (lid u = (0.1, 0, 0) on z = 1), FP32 storage and arithmetic. One
step is one launch of the step kernel over the lattice; MLUPS counts the
updated (non-wall) nodes, 254^3 per step. The split-storage variants (S16 =
scaled binary16 with stochastic rounding, HILO = bfloat16 hi+lo) are timed on
the same lattice and reported beside it.

Output: one JSON line with
  - the metric and `value` (MLUPS of the FP32 step, inputs resident in HBM);
  - `roofline`: algorithmic bytes per launch / measured launch time against
    8 TB/s, and the HBM bytes per launch from the committed rocprofv3
    counters when they were taken on the current sources;
  - `copy_ceiling`: the library's streaming copy of the same state buffer
    back and forth, the memory rate a step can reach on this device;
  - `cpu_baseline`: the FP64 CPU oracle timed on a bounded sample of the
    same workload, one single-threaded oracle process per host core (at
    most 16), each on its own copy; `small_configs` beside it: the oracle on
    one core over the whole 64^2 Taylor-Green run and a 10-step window of
    the 1024^2 cavity;
  - `variants` (S16, HILO), `adjoint` (the 512^2 D2Q9 reverse mode against
    the forward), `batch` (512 D2Q9 cavities in one launch per step against
    one launch per cavity), `launch_bound` (a 64^2 lattice),
    `steady_state` (the paper's 2-D cavity run to a steady state),
    `cavity1024` (the 1024^2 2-D cavity in FP64 and FP32), `bgk` (the tau = 1
    population scheme on the same cube, 152 against 32 bytes per update), `parity_cube64`
    (each storage against the oracle's stored 64^3 run) and `conservation`
    (mass and momentum drift on a periodic box).
Every timed run starts after ADVANCE untimed steps from rest, then the
autotuner, then --warmup steps.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    "cube256": dict(desc="D3Q19 lid-driven cube 256^3 Re=400", q=19, n=256, Re=400.0, U=0.1),
    "cube64": dict(desc="D3Q19 lid-driven cube 64^3 Re=98.8", q=19, n=64, Re=98.8, U=0.1),
    "cavity1024": dict(desc="D2Q9 lid-driven cavity 1024^2 Re=1000", q=9, n=1024, Re=1000.0, U=0.1),
}
BYTES = {"fp64": 8, "fp32": 4, "hilo": 4, "s16": 2}


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) of the sources that define the kernels and
    their launches (csrc/ without the C ABI file maclab_api.hip, which holds
    host code only), with comments and blank lines removed, so that an edit
    of a comment or of host code keeps the counter figures taken on the same
    kernels."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1901_02716_amd", "csrc", "*"))):
        if os.path.basename(p) == "maclab_api.hip":
            continue
        text = open(p, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def make_case(wl):
    from paper_1901_02716_amd import workloads

    if wl["q"] == 19:
        return workloads.cavity_3d(n=wl["n"], Re=wl["Re"], U=wl["U"])
    return workloads.cavity_2d(n=wl["n"], Re=wl["Re"], U=wl["U"])


def updated_nodes(case) -> int:
    n = 1
    for ax in range(case.d):
        walled = any(f[0] == "xyz"[ax] for f in case.fixed)
        n *= case.n[ax] - 2 if walled else case.n[ax]
    return n


# Untimed steps before every timed run, whatever --warmup says: the lattice
# starts at rest (mostly exact zeros, which the memory system moves faster),
# so every figure is taken on the same partly developed state.
ADVANCE = 1000


def time_variant(case, precision, steps, warmup, autotune=True, tiling=None, copy=False):
    import torch

    from paper_1901_02716_amd import Simulation

    sim = Simulation(case.q, case.n, case.dx, case.nu, precision=precision, seed=1)
    sim.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        sim.set_bc(face, rb, ub)
    sim.step(ADVANCE)
    if tiling is not None:
        sim.set_tiling(*tiling)
    elif autotune:
        sim.autotune(reps=5)
    sim.tiling_used = sim.tiling()
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    t0 = time.perf_counter()
    sim.step(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    d = sim.diagnostics()
    d = {"diag": d, "tiling": sim.tiling_used}
    if copy:
        d["copy_ms"], d["copy_bytes"] = copy_rate(sim, steps, warmup)
    sim.close()
    return ms / steps, wall, d


def copy_rate(sim, steps: int, warmup: int):
    """The library's streaming copy of a state buffer back and forth between
    two buffers of the step's size, as many times as the step was timed: the
    memory rate of a step without its arithmetic. Returns ms per copy and the
    bytes each copy moves (read + write)."""
    import torch

    nb = sim.state_bytes()
    a = torch.zeros(nb, dtype=torch.uint8, device=sim.device)
    b = torch.zeros_like(a)
    sim.save_state(a)
    for i in range(max(warmup, 2)):
        sim.copy(a, b) if i % 2 == 0 else sim.copy(b, a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    for i in range(steps):
        sim.copy(a, b) if i % 2 == 0 else sim.copy(b, a)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps, 2 * nb


def time_adjoint(T: int, precision: str = "fp32", reps: int = 3):
    """Reverse-mode cost on the periodic D2Q9 512^2 box (nu = 0.005, Fourier-
    mode initial field and target): the backward of a T-step rollout with
    sqrt(T) checkpointing (recompute + reverse steps) against T forward steps.
    Also the bare reverse-step kernel against the bare forward kernel."""
    import math

    import torch

    from paper_1901_02716_amd import Simulation, rollout, workloads

    case, tgt = workloads.adjoint_case(steps=T)
    sim = Simulation(9, case.n, case.dx, case.nu, precision=precision)
    dev = sim.device
    tg = torch.tensor(tgt, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def fwd_ms(n):
        sim.set_fields(case.rho, case.u)
        sim.step(10)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(sim.stream)
        sim.step(n)
        b.record(sim.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    fwd_ms(T)  # warm-up
    fwd = min(fwd_ms(T) for _ in range(reps)) / T
    bwd = []
    for _ in range(reps):
        u0 = torch.tensor(case.u, device=dev, requires_grad=True)
        G = torch.zeros(3, dtype=torch.float64, requires_grad=True)
        uT = rollout(sim, case.rho, u0, G, T)
        loss = ((uT - tg) ** 2).sum()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(sim.stream)
        t0 = time.perf_counter()
        loss.backward()
        b.record(sim.stream)
        torch.cuda.synchronize()
        bwd.append(max(a.elapsed_time(b), (time.perf_counter() - t0) * 1e3))
    # bare kernels: the reverse step alone on resident buffers
    sim.set_fields(case.rho, case.u)
    s0 = sim.save_state()
    adj = [sim.new_adjoint(), sim.new_adjoint()]
    sim.adjoint_seed(s0, torch.zeros_like(tg), adj[0])
    sim.adjoint_reset()
    n = 500
    for i in range(20):
        sim.adjoint_step(s0, adj[i & 1], adj[(i & 1) ^ 1])
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(sim.stream)
    for i in range(n):
        sim.adjoint_step(s0, adj[i & 1], adj[(i & 1) ^ 1])
    b.record(sim.stream)
    torch.cuda.synchronize()
    adj_kernel = a.elapsed_time(b) / n
    bwd_ms = min(bwd)
    out = {"workload": f"D2Q9 periodic 512^2 nu=0.005 T={T} {precision}, K={math.ceil(math.sqrt(T))}",
           "forward_ms_per_step": round(fwd, 5), "backward_ms": round(bwd_ms, 3),
           "backward_over_T_forward": round(bwd_ms / (T * fwd), 3),
           "reverse_step_ms": round(adj_kernel, 5), "reverse_over_forward_step": round(adj_kernel / fwd, 3),
           "adjoint_tiling": sim.adjoint_tiling(), "forward_tiling": sim.tiling()}
    sim.close()
    return out


def time_batch(steps: int, sep_steps: int):
    """512 D2Q9 lid-driven cavities of the seeded draw (N uniform in
    [64, 512], Re log-uniform in [100, 5000], lid speed uniform in
    [0.05, 0.1]; seed 4), FP32: aggregate MLUPS of one launch per step over
    all cavities (HIP graphs, autotuned tiling) against one launch per cavity
    per step."""
    import torch

    from paper_1901_02716_amd import cavities, workloads

    draws = workloads.batch_draw()
    b = cavities(draws, precision="fp32")
    # tune on a developed state: at the start most of each cavity holds
    # exact zeros, which the memory system moves faster than the later state
    b.step(200)
    tune_ms = b.autotune(reps=3)
    lu = b.updated_nodes()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed(fn, n):
        fn(2)
        torch.cuda.synchronize()
        a, c = ev(), ev()
        a.record(b.stream)
        fn(n)
        c.record(b.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(c) / n

    ms = timed(b.step, steps)
    ms_sep = timed(b.step_separate, sep_steps)
    nonfinite = sum(1 for i in range(len(b)) if b[i].diagnostics()[6] > 0)
    out = {"workload": "512 D2Q9 lid-driven cavities, seed 4 draw, FP32",
           "nodes_per_step": sum(N * N for N, _, _ in draws), "updated_nodes_per_step": lu,
           "mlups": round(lu / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
           "hbm_frac": round(24 * lu / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "separate_launches_mlups": round(lu / (ms_sep * 1e-3) / 1e6, 1),
           "separate_ms_per_step": round(ms_sep, 5), "speedup_vs_separate": round(ms_sep / ms, 3),
           "tiling": b.tiling(), "autotune_best_ms": round(tune_ms, 5),
           "nonfinite_cavities_after": nonfinite, "steps_timed": steps}
    b.close()
    return out


def time_small(steps: int = 2000):
    """The launch-bound case: the 64^2 periodic Taylor-Green vortex in FP64
    (4096 nodes), one launch per step."""
    import torch

    from paper_1901_02716_amd import Simulation, workloads

    case = workloads.taylor_green(n=64, nu=0.01, U0=0.01)
    sim = Simulation(9, case.n, case.dx, case.nu, precision="fp64")
    sim.set_fields(case.rho, case.u)
    sim.step(100)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(sim.stream)
    sim.step(steps)
    b.record(sim.stream)
    torch.cuda.synchronize()
    us = a.elapsed_time(b) / steps * 1e3
    sim.close()
    return {"workload": "D2Q9 Taylor-Green vortex 64^2 FP64 (launch-bound)", "steps_timed": steps,
            "us_per_step": round(us, 3), "mlups": round(case.n[0] * case.n[1] / us, 1)}


def time_steady(tol: float = 1e-10, check_every: int = 5000):
    """The steady-state driver on the paper's 2-D cavity (400 x 400 lattices,
    u0 = 1, Re = 1000), FP64: steps until the per-step change of u is below
    `tol`, with the residual evaluated every `check_every` steps."""
    import torch

    from paper_1901_02716_amd import Simulation, workloads

    case = workloads.cavity_2d(n=401, Re=1000.0, U=1.0)
    sim = Simulation(9, case.n, case.dx, case.nu, precision="fp64")
    sim.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        sim.set_bc(face, rb, ub)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, r = sim.run_to_steady(tol, 2000000, check_every)
    wall = time.perf_counter() - t0
    lu = updated_nodes(case) * steps
    sim.close()
    return {"workload": "D2Q9 lid-driven cavity 401^2 (400 x 400 lattices), u0 = 1, Re = 1000, FP64",
            "tol_per_step": tol, "check_every": check_every, "steps": steps, "residual": r,
            "wall_s": round(wall, 3), "mlups": round(lu / wall / 1e6, 1)}


def time_cavity1024(steps: int, warmup: int):
    """The 2-D lid-driven cavity of 1024^2 nodes (Re = 1000, lid 0.1) in FP64
    and FP32 storage. Its state (12.6 MB in FP32, 25 MB in FP64) stays in the
    256 MB last-level cache, so the rate is an effective one, not HBM."""
    case = make_case(WORKLOADS["cavity1024"])
    lu = updated_nodes(case)
    out = {"workload": WORKLOADS["cavity1024"]["desc"], "updated_nodes_per_step": lu}
    for prec in ("fp64", "fp32"):
        ms, _, info = time_variant(case, prec, steps, warmup)
        b_lu = 2 * 3 * BYTES[prec]
        out[prec] = {"mlups": round(lu / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
                     "bytes_per_lattice_update": b_lu,
                     "effective_gbs": round(b_lu * lu / (ms * 1e-3) / 1e9, 1), "tiling": info["tiling"]}
    return out


def time_bgk(steps: int, warmup: int, maclab_ms: float):
    """The tau = 1 lattice BGK scheme (populations stored and streamed) on
    the benchmark cube, FP32: 2 Q x 4 = 152 bytes per lattice update where
    the MacLAB step moves 2 (d + 1) x 4 = 32. Same advance and warmup as the
    MacLAB figures."""
    import torch

    from paper_1901_02716_amd import BGK

    case = make_case(WORKLOADS["cube256"])
    lu = updated_nodes(case)
    b = BGK(case.q, case.n, case.dx, case.nu, precision="fp32")
    b.set_fields(case.rho, case.u)
    for face, (rb, ub) in case.fixed.items():
        b.set_bc(face, rb, ub)
    b.step(ADVANCE + warmup)
    torch.cuda.synchronize()
    a, c = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(b.stream)
    b.step(steps)
    c.record(b.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(c) / steps
    b.close()
    b_lu = 2 * 19 * 4
    return {"workload": WORKLOADS["cube256"]["desc"] + " fp32, lattice BGK tau = 1 (populations stored)",
            "bytes_per_lattice_update": b_lu, "maclab_bytes_per_lattice_update": 32,
            "mlups": round(lu / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
            "hbm_frac": round(b_lu * lu / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "maclab_speedup": round(ms / maclab_ms, 3)}


def parity_cube64(precisions=("fp32", "hilo", "s16")):
    """Error of each storage against the FP64 oracle's 5000-step run of the
    64^3 lid-driven cube at Re = 98.8 (the lattice Reynolds number of the
    256^3 Re = 400 cube), stored in tests/golden/cube64_re98.8.npz (every 4th
    node per axis): relative L2 of u and of the density deviation rho - 1."""
    import numpy as np

    from paper_1901_02716_amd import Simulation

    path = os.path.join(ROOT, "tests", "golden", "cube64_re98.8.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    case = make_case(WORKLOADS["cube64"])
    out = {"workload": WORKLOADS["cube64"]["desc"] + ", 5000 steps, every 4th node per axis"}
    for prec in precisions:
        sim = Simulation(case.q, case.n, case.dx, case.nu, precision=prec, seed=5)
        sim.set_fields(case.rho, case.u)
        for face, (rb, ub) in case.fixed.items():
            sim.set_bc(face, rb, ub)
        sim.step(int(ref["steps"]))
        rho, u = sim.fields()
        sim.close()
        st = int(ref["stride"])
        r, v = rho[::st, ::st, ::st], u[:, ::st, ::st, ::st]
        rr, rv = ref["rho"], ref["u"]
        rel = lambda a, b: float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))  # noqa: E731
        out[prec] = {"rel_l2_u": rel(v, rv), "rel_l2_drho": rel(r - 1.0, rr - 1.0)}
    return out


def conservation(steps: int = 2000):
    """Mass and momentum drift of the periodic 512^2 D2Q9 box (the adjoint
    workload, no force): Eqs. (4)-(5) conserve both exactly, so the drift is
    the storage's rounding."""
    import numpy as np

    from paper_1901_02716_amd import Simulation, workloads

    case, _ = workloads.adjoint_case()
    out = {"workload": f"D2Q9 periodic 512^2 nu=0.005 Fourier-mode field, {steps} steps"}
    for prec in ("fp64", "fp32", "s16"):
        sim = Simulation(9, case.n, case.dx, case.nu, precision=prec, seed=2)
        sim.set_fields(case.rho, case.u)
        d0 = np.array(sim.diagnostics())
        sim.step(steps)
        d1 = np.array(sim.diagnostics())
        sim.close()
        pscale = float(np.sqrt(2.0 * d0[0] * d0[4]))  # bounds sum |rho u_i|
        out[prec] = {"mass_rel_drift": float(abs(d1[0] - d0[0]) / d0[0]),
                     "momentum_drift_over_sqrt_2ME": float(np.max(np.abs(d1[1:3] - d0[1:3])) / pscale)}
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(workload: str, steps: int, core: int = -1) -> float:
    """Seconds the FP64 oracle (single-threaded C) takes for `steps` steps of
    a workload lattice, from its initial state, pinned to host core `core`
    (if >= 0)."""
    if core >= 0:
        os.sched_setaffinity(0, {core})
    import oracle

    case = make_case(WORKLOADS[workload])
    p = oracle.Problem(case.q, case.n, case.dx, case.nu)
    for face, (rb, ub) in case.fixed.items():
        p.set_fixed(face, rb, ub)
    t0 = time.perf_counter()
    oracle.run(p, case.rho, case.u, steps)
    return time.perf_counter() - t0


def _oracle_small(kind: str, steps: int, core: int) -> float:
    """Seconds the FP64 oracle takes for `steps` steps of a small config
    (`tgv64`: the 64^2 Taylor-Green vortex; `cavity1024`: the 1024^2 cavity
    from rest), pinned to host core `core`."""
    os.sched_setaffinity(0, {core})
    import oracle
    from paper_1901_02716_amd import workloads

    if kind == "tgv64":
        case = workloads.taylor_green(64, 0.01, 0.01, e=oracle.particle_speed(0.01, 1.0 / 64))
    else:
        case = workloads.cavity_2d(n=1024, Re=1000.0, U=0.1)
    p = oracle.Problem(case.q, case.n, case.dx, case.nu)
    for face, (rb, ub) in case.fixed.items():
        p.set_fixed(face, rb, ub)
    t0 = time.perf_counter()
    oracle.run(p, case.rho, case.u, steps)
    return time.perf_counter() - t0


def oracle_configs(core: int) -> dict:
    """The FP64 oracle timed on the small configs, one single-threaded child
    process each on one host core: the whole 1000-step 64^2 Taylor-Green run
    and 10 steps of the 1024^2 cavity (a window of its 50000-step run)."""
    import subprocess

    out = {}
    for kind, steps, nodes in (("tgv64", 1000, 64 * 64), ("cavity1024", 10, 1022 * 1022)):
        code = (f"import sys; sys.path.insert(0, {ROOT!r}); import bench; "
                f"print(bench._oracle_small({kind!r}, {steps}, {core}))")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS="1"))
        if r.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {r.returncode}")
        sec = float(r.stdout.strip().splitlines()[-1])
        out[kind] = {"steps": steps, "seconds": round(sec, 3), "mlups": round(nodes * steps / sec / 1e6, 3),
                     "cores": 1}
    return out


def host_cores() -> list:
    """Host cores to run the oracle on: those this process may use, at most
    16 (the host share of one GPU)."""
    try:
        cores = sorted(os.sched_getaffinity(0))
    except AttributeError:
        cores = list(range(os.cpu_count() or 1))
    return cores[:16] or [0]


def cpu_baseline(workload: str, steps: int, cores: list):
    """The FP64 oracle on `steps` steps of the workload lattice, as one
    independent process per listed host core at once, each pinned to its core
    and working on its own copy. They are child processes that import only
    the oracle and the input generators, so none of them touches the GPU.
    Returns the aggregate MLUPS, the slowest process's seconds and the
    per-process seconds."""
    import subprocess

    import oracle

    oracle.build()  # once, before the workers load it
    procs = len(cores)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    workers = []
    for c in cores:
        code = (f"import sys; sys.path.insert(0, {ROOT!r}); import bench; "
                f"print(bench._oracle_steps({workload!r}, {steps}, {c}))")
        workers.append(subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, text=True, env=env))
    secs = []
    for w in workers:
        out, _ = w.communicate()
        if w.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {w.returncode}")
        secs.append(float(out.strip().splitlines()[-1]))
    lu = updated_nodes(make_case(WORKLOADS[workload])) * steps
    return procs * lu / max(secs) / 1e6, max(secs), secs


def load_traffic(workload: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}:{precision}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cube256", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=sorted(BYTES))
    ap.add_argument("--variants", default="s16,hilo", help="extra storage variants to time ('' for none)")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes of the CPU baseline (0: host cores, at most 16)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 1024^2 cavity, the 64^3 parity run and the conservation run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-steady", action="store_true", help="skip the steady-state run of the 2-D cavity")
    ap.add_argument("--no-autotune", action="store_true", help="use the default tiling")
    ap.add_argument("--tiling", default="", help="W,nyb,nzb,pf[,kernel] of the fast kernel (skips autotuning)")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="T of the reverse-mode cost measurement (0 to skip)")
    ap.add_argument("--batch-steps", type=int, default=200,
                    help="steps of the 512-cavity batch measurement (0 to skip)")
    ap.add_argument("--profile-copy-mib", type=int, default=0,
                    help="after timing, run one torch copy of this many MiB (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the step would shard as z-slabs with one-plane halo exchange).", file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    wl = WORKLOADS[args.workload]
    case = make_case(wl)
    lu = updated_nodes(case)
    d = case.d
    tiling = None
    if args.tiling:
        parts = args.tiling.split(",")
        tiling = tuple(int(v) for v in parts[:4]) + ((parts[4],) if len(parts) > 4 else ())
    ms, wall, info = time_variant(case, args.precision, args.steps, args.warmup, not args.no_autotune, tiling,
                                  copy=True)
    diag = info["diag"]
    mlups = lu / (ms * 1e-3) / 1e6
    b_lu = 2 * (d + 1) * BYTES[args.precision]
    achieved = b_lu * lu / (ms * 1e-3) / 1e9
    copy_gbs = info["copy_bytes"] / (info["copy_ms"] * 1e-3) / 1e9
    traffic = load_traffic(args.workload, args.precision)

    variants = {}
    for v in [s for s in args.variants.split(",") if s and s != args.precision]:
        vms, _, vd = time_variant(case, v, args.steps, args.warmup, not args.no_autotune, tiling)
        vm = lu / (vms * 1e-3) / 1e6
        variants[v] = {"mlups": round(vm, 1), "ms_per_step": round(vms, 5), "tiling": vd["tiling"],
                       "vs_" + args.precision: round(vm / mlups, 3),
                       "hbm_frac": round(2 * (d + 1) * BYTES[v] * lu / (vms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    adjoint = time_adjoint(args.adjoint_steps) if args.adjoint_steps > 0 else None
    batch = time_batch(args.batch_steps, max(10, args.batch_steps // 4)) if args.batch_steps > 0 else None
    small = time_small() if args.batch_steps > 0 else None
    steady = time_steady() if args.batch_steps > 0 and not args.no_steady else None
    extras = not args.no_extras and args.workload == "cube256"
    cavity = time_cavity1024(args.steps, args.warmup) if extras else None
    bgk = time_bgk(args.steps, args.warmup, ms) if extras and args.precision == "fp32" else None
    parity = parity_cube64() if extras else None
    drift = conservation() if extras else None

    cpu = None
    if not args.no_cpu_baseline:
        cores = host_cores()
        if args.cpu_procs:
            cores = cores[:args.cpu_procs]
        procs = len(cores)
        cm, cdt, csecs = cpu_baseline(args.workload, args.cpu_steps, cores)
        cpu = {"value": round(cm, 3), "unit": "MLUPS", "cores": procs, "kind": "oracle",
               "sample": f"{args.cpu_steps} FP64 steps of the same {wl['desc']} lattice in each of {procs} "
                         f"single-threaded oracle processes at once, each pinned to its own core "
                         f"({procs} x {args.cpu_steps * lu} lattice "
                         f"updates; slowest {cdt:.1f} s, fastest {min(csecs):.1f} s; one process alone: "
                         f"about {args.cpu_steps * lu / min(csecs) / 1e6:.2f} MLUPS)",
               "cpu_model": cpu_model(), "pinned_cores": cores}
        if extras:
            cpu["small_configs"] = oracle_configs(cores[0])

    if args.profile_copy_mib > 0:
        n = args.profile_copy_mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": "MLUPS + HBM-roofline fraction, D3Q19 256^3 FP32 vs split-BF16; adjoint/fwd cost",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "hilo": "f32 (bf16x2 storage)", "s16": "f32 (f16 storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{wl['desc']} {args.precision}", "lattice": "D3Q19" if d == 3 else "D2Q9",
                   "nodes": list(case.n), "updated_nodes_per_step": lu, "storage": args.precision,
                   "bytes_per_lattice_update": b_lu, "tiling": info["tiling"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "copy_ceiling": {"kernel": "maclab_copy: the state buffer copied back and forth (non-temporal "
                                   "16-byte loads, device-scope stores)",
                         "bytes_per_copy": info["copy_bytes"], "ms_per_copy": round(info["copy_ms"], 5),
                         "gbs": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                         "step_frac_of_copy": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
        "variants": variants,
        "adjoint": adjoint,
        "batch": batch,
        "launch_bound": small,
        "steady_state": steady,
        "cavity1024": cavity,
        "bgk": bgk,
        "parity_cube64": parity,
        "conservation": drift,
        "untimed_advance_steps": ADVANCE,
        "diagnostics_after": {"mass": diag[0], "max_u_over_e": diag[5], "nonfinite": diag[6]},
        "wall_s": round(wall, 3),
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
