"""Writes the long-run oracle references used by the GPU parity tests.

Every value stored here comes from the FP64 CPU oracle (``oracle/``) on inputs
from ``paper_1901_02716_amd.workloads``; nothing is taken from the GPU path.
The runs are too long for the test suite (minutes to hours on one core), so
their results are stored in compact form:

* ``cube64_re98.8.npz`` -- D3Q19 lid-driven cube, 64^3 nodes, Re = 98.8
  (lattice Reynolds number 1.57, the value of the 256^3 Re = 400 cube), lid
  (0.1, 0, 0), 5000 steps: every 4th node per axis of rho and u, the
  centre-line profile u_x(z) at x = y = 1/2, and the diagnostics.
* ``cube64_re400.json`` -- the same cube at the literal Re = 400 (lattice
  Reynolds number 6.35, so the lid itself moves at |u|/e = 1.06): the first
  step at which the state holds a non-finite value, and max |u|/e every 10
  steps until then.
* ``cavity1024_re1000.npz`` -- D2Q9 lid-driven cavity, 1024^2 nodes,
  Re = 1000, lid 0.1: after 1000, 5000, 20000 and 50000 steps, the
  diagnostics, the centre-line profiles u_x(y) at x = 1/2 and u_y(x) at
  y = 1/2 (mean of the two node columns / rows either side of the centre),
  and every 16th node per axis of rho and u.

* ``adjoint512_fd.json`` -- D2Q9 periodic 512^2 box, nu = 0.005, initial
  velocity a sum of 8 random Fourier modes (seed 1), target the same
  construction with seed 2, G = 0, 2000 steps, loss sum (u(T) - u_target)^2:
  the loss and central differences of it along 16 unit directions in u0 and
  16 in G (seed 3), each at h = 1e-4 and at 2h. Their difference bounds the
  error of the difference at h (the truncation error of a central difference
  falls by 4 from 2h to h, so it is about a third of the difference; rounding
  in the loss adds a part that grows as 1/h). Two directions (the smallest
  |derivative| in u0 and in G) are also differenced at h = 1e-5 and 1e-6, to
  show the rounding floor that rules out the smaller steps.
* ``cavity1024_re1000_ext.npz`` -- the same cavity and checkpoints with the
  oracle built in x87 extended precision (oracle.run_extended).
* ``batch512_stable.npz`` -- the three largest cavities of the 512-cavity
  draw (seed 4) whose lattice Reynolds number U dx / nu is at most 2.5,
  2000 steps each: diagnostics and every 4th node per axis of rho and u;
  ``batch512_stable_10000.npz`` the same after 10000 steps
  (``batch512 10000``).

Usage: python tests/golden/make_references.py {cube64,cube64_re400,cavity1024,cavity1024_extended,adjoint512 [workers],batch512 [steps]}
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1901_02716_amd import workloads  # noqa: E402


def problem(case):
    p = oracle.Problem(case.q, case.n, case.dx, case.nu, G=tuple(case.G))
    for face, (rb, ub) in case.fixed.items():
        p.set_fixed(face, rb, ub)
    return p


def cube64():
    case = workloads.cavity_3d(n=64, Re=98.8, U=0.1)
    p = problem(case)
    t0 = time.time()
    rho, u = oracle.run(p, case.rho, case.u, 5000)
    d = oracle.diagnostics(p, rho, u)
    c = case.n[0] // 2
    np.savez_compressed(os.path.join(HERE, "cube64_re98.8.npz"), steps=5000, stride=4,
                        rho=rho[::4, ::4, ::4], u=u[:, ::4, ::4, ::4],
                        centre_ux=0.5 * (u[0, :, c - 1, c - 1] + u[0, :, c, c]), diagnostics=d,
                        seconds=time.time() - t0)


def cube64_re400():
    case = workloads.cavity_3d(n=64, Re=400.0, U=0.1)
    p = problem(case)
    rho, u = case.rho, case.u
    blow = None
    trace = []
    for step in range(1, 1001):
        rho, u = oracle.run(p, rho, u, 1)
        d = oracle.diagnostics(p, rho, u)
        if step % 10 == 0:
            trace.append([step, d[5]])
        if d[6] > 0:
            blow = step
            break
    json.dump({"case": "D3Q19 cube 64^3, Re 400, lid 0.1", "lattice_reynolds": 0.1 * case.dx / case.nu,
               "lid_mach": 0.1 / oracle.particle_speed(case.nu, case.dx),
               "first_nonfinite_step": blow, "max_u_over_e_every_10_steps": trace},
              open(os.path.join(HERE, "cube64_re400.json"), "w"), indent=1)


def cavity1024(resume=None):
    """Long run; the full state is saved every 2500 steps to `resume` (a
    scratch file outside the repository) so an interrupted run continues."""
    import tempfile

    resume = resume or os.path.join(tempfile.gettempdir(), "maclab_cavity1024_state.npz")
    case = workloads.cavity_2d(n=1024, Re=1000.0, U=0.1)
    p = problem(case)
    rho, u = case.rho, case.u
    out = {}
    done = 0
    elapsed = 0.0
    if os.path.exists(resume):
        z = np.load(resume)
        rho, u, done, elapsed = z["rho"], z["u"], int(z["done"]), float(z["elapsed"])
        out = {k[4:]: z[k] for k in z.files if k.startswith("out_")}
        print(f"cavity1024: resuming at step {done}", flush=True)
    t0 = time.time() - elapsed
    c = case.n[0] // 2
    for target in (1000, 5000, 20000, 50000):
        while done < target:
            n = min(2500, target - done)
            rho, u = oracle.run(p, rho, u, n)
            done += n
            if done < target:
                np.savez(resume, rho=rho, u=u, done=done, elapsed=time.time() - t0,
                         **{"out_" + k: v for k, v in out.items()})
        if f"diag_{target}" in out:
            continue
        d = oracle.diagnostics(p, rho, u)
        out[f"diag_{target}"] = d
        out[f"ux_centre_{target}"] = 0.5 * (u[0, 0, :, c - 1] + u[0, 0, :, c])
        out[f"uy_centre_{target}"] = 0.5 * (u[1, 0, c - 1, :] + u[1, 0, c, :])
        out[f"rho_sub_{target}"] = rho[0, ::16, ::16]
        out[f"u_sub_{target}"] = u[:, 0, ::16, ::16]
        out[f"seconds_{target}"] = time.time() - t0
        np.savez_compressed(os.path.join(HERE, "cavity1024_re1000.npz"), stride=16, **out)
        np.savez(resume, rho=rho, u=u, done=done, elapsed=time.time() - t0,
                 **{"out_" + k: v for k, v in out.items()})
        print(f"cavity1024: {target} steps after {time.time() - t0:.0f} s", flush=True)


def cavity1024_extended(resume=None, targets=(1000, 5000, 20000, 50000)):
    """The 1024^2 cavity of cavity1024() with the oracle built in x87
    extended precision (run_extended): the same checkpoints, written to
    cavity1024_re1000_ext.npz as float64 after each target is reached (the
    state itself stays in extended precision between chunks; `resume` keeps
    it on disk so an interrupted run continues)."""
    import tempfile

    resume = resume or os.path.join(tempfile.gettempdir(), "maclab_cavity1024_ext_state.npz")
    case = workloads.cavity_2d(n=1024, Re=1000.0, U=0.1)
    p = problem(case)
    rho, u, done, elapsed, out = case.rho, case.u, 0, 0.0, {}
    if os.path.exists(resume):
        z = np.load(resume)
        rho, u = z["rho"].view(np.longdouble).reshape(case.rho.shape), z["u"].view(np.longdouble).reshape(case.u.shape)
        done, elapsed = int(z["done"]), float(z["elapsed"])
        out = {k[4:]: z[k] for k in z.files if k.startswith("out_")}
        print(f"cavity1024_extended: resuming at step {done}", flush=True)
    t0 = time.time() - elapsed

    def save_state():
        np.savez(resume, rho=np.asarray(rho, dtype=np.longdouble).view(np.uint8), u=np.asarray(u, dtype=np.longdouble).view(np.uint8),
                 done=done, elapsed=time.time() - t0, **{"out_" + k: v for k, v in out.items()})

    c = case.n[0] // 2
    for target in targets:
        while done < target:
            n = min(1000, target - done)
            rho, u = oracle.run_extended(p, rho, u, n)
            done += n
            save_state()
            print(f"cavity1024_extended: {done} steps after {time.time() - t0:.0f} s", flush=True)
        if f"u_sub_{target}" in out:
            continue
        r64, u64 = rho.astype(np.float64), u.astype(np.float64)
        out[f"diag_{target}"] = oracle.diagnostics(p, r64, u64)
        out[f"ux_centre_{target}"] = 0.5 * (u64[0, 0, :, c - 1] + u64[0, 0, :, c])
        out[f"uy_centre_{target}"] = 0.5 * (u64[1, 0, c - 1, :] + u64[1, 0, c, :])
        out[f"rho_sub_{target}"] = r64[0, ::16, ::16]
        out[f"u_sub_{target}"] = u64[:, 0, ::16, ::16]
        out[f"seconds_{target}"] = time.time() - t0
        np.savez_compressed(os.path.join(HERE, "cavity1024_re1000_ext.npz"), stride=16, **out)
        save_state()


def _loss(args):
    which, k, sign, h = args
    case, tgt = workloads.adjoint_case()
    du, dG = workloads.adjoint_directions()
    u0 = case.u.copy()
    G = np.zeros(3)
    if which == "u":
        u0 = u0 + sign * h * du[k]
    elif which == "G":
        G = G + sign * h * dG[k]
    case.G = tuple(G)
    p = problem(case)
    rho, u = oracle.run(p, case.rho, u0, case.steps)
    return args, float(np.sum((u - tgt) ** 2))


def adjoint512(workers=6):
    from multiprocessing import Pool

    h = 1e-4
    ref = json.load(open(os.path.join(HERE, "adjoint512_fd.json")))
    small = (("u", int(np.argmin(np.abs(ref["fd_u"])))), ("G", int(np.argmin(np.abs(ref["fd_G"])))))
    jobs = [("base", 0, 0, 0.0)]
    jobs += [(w, k, s, hh) for hh in (h, 2 * h) for w in ("u", "G") for k in range(16) for s in (1, -1)]
    jobs += [(w, k, s, hh) for hh in (1e-5, 1e-6) for w, k in small for s in (1, -1)]
    t0 = time.time()
    res = {}
    with Pool(workers) as pool:
        for args, L in pool.imap_unordered(_loss, jobs):
            res[args] = L
            print(f"adjoint512: {len(res)}/{len(jobs)} after {time.time() - t0:.0f} s", flush=True)

    def fd(w, k, hh):
        return (res[(w, k, 1, hh)] - res[(w, k, -1, hh)]) / (2 * hh)

    out = {"case": "D2Q9 periodic 512^2, nu 0.005, 2000 steps, modes seed 1, target seed 2, G = 0",
           "h": h, "loss": res[("base", 0, 0, 0.0)],
           "fd_u": [fd("u", k, h) for k in range(16)],
           "fd_G": [fd("G", k, h) for k in range(16)],
           "fd_u_2h": [fd("u", k, 2 * h) for k in range(16)],
           "fd_G_2h": [fd("G", k, 2 * h) for k in range(16)],
           "small_h": [{"dir": w, "index": k, "h": hh, "fd": fd(w, k, hh)} for hh in (1e-5, 1e-6) for w, k in small],
           "seconds": time.time() - t0}
    json.dump(out, open(os.path.join(HERE, "adjoint512_fd.json"), "w"), indent=1)


def _batch_run(args):
    i, steps = args
    N, Re, U = workloads.batch_draw()[i]
    case = workloads.cavity_2d(n=N, Re=Re, U=U)
    p = problem(case)
    rho, u = oracle.run(p, case.rho, case.u, steps)
    return i, oracle.diagnostics(p, rho, u), rho[0, ::4, ::4], u[:, 0, ::4, ::4]


def batch512(steps=2000, workers=3):
    from multiprocessing import Pool

    draws = workloads.batch_draw()
    stable = sorted(((N, i) for i, (N, Re, U) in enumerate(draws) if Re / (N - 1) <= 2.5), reverse=True)[:3]
    idx = [i for _, i in stable]
    t0 = time.time()
    with Pool(workers) as pool:
        res = pool.map(_batch_run, [(i, steps) for i in idx])
    out = {"index": np.array(idx), "steps": steps, "stride": 4, "seconds": time.time() - t0}
    for i, d, r, u in res:
        out[f"diag_{i}"] = d
        out[f"rho_sub_{i}"] = r
        out[f"u_sub_{i}"] = u
    name = "batch512_stable.npz" if steps == 2000 else f"batch512_stable_{steps}.npz"
    np.savez_compressed(os.path.join(HERE, name), **out)


if __name__ == "__main__":
    oracle.build()
    if sys.argv[1] == "adjoint512":
        adjoint512(int(sys.argv[2]) if len(sys.argv) > 2 else 6)
    elif sys.argv[1] == "batch512":
        batch512(int(sys.argv[2]) if len(sys.argv) > 2 else 2000)
    elif sys.argv[1] == "cavity1024_extended":
        cavity1024_extended()
    else:
        {"cube64": cube64, "cube64_re400": cube64_re400, "cavity1024": cavity1024}[sys.argv[1]]()
