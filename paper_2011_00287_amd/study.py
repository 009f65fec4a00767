"""Accuracy of the reduced-precision variants against the FP64 GPU path.

python -m paper_2011_00287_amd.study droplet64 [--out FILE]
python -m paper_2011_00287_amd.study droplet128 [--out FILE]

droplet64  : 64^3 droplet (R = 16, q0 = 2 pi/16), zeta in {0, 0.005, 0.01},
             2000 steps, FP64 and FP32 side by side; every 100 steps the
             per-field error of FP32 against FP64, the droplet-centre
             trajectory of both, and (at zeta = 0) F_h + E_kin.
droplet128 : 128^3 droplet (R = 32, q0 = 2 pi/24, zeta = 0.008), 5000 steps,
             FP32 and FP16 population storage against FP64, every 500 steps.

Per-field error: ||X - X64||_2 / ||X64||_2 and max|X - X64| / max|X64| for
X in rho - rho0, u, phi, Q.  Droplet velocity: displacement of the
circular-mean centre over the last 1000 steps / 1000.  The FP64 GPU path is
the reference (it matches the FP64 oracle to 1e-12 per field on the 16^3
droplet over 100 steps and on 64^3 over 30 steps).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs
from .sim import Sim


def _err(a, b):
    d = a - b
    n2 = np.linalg.norm(b)
    m = np.abs(b).max()
    return [float(np.linalg.norm(d) / n2) if n2 > 0 else float(np.linalg.norm(d)),
            float(np.abs(d).max() / m) if m > 0 else float(np.abs(d).max())]


def field_errors(sim, ref, rho0=1.0):
    r1, u1, p1, q1 = sim.moments()
    r0, u0, p0, q0 = ref.moments()
    return {"rho-rho0": _err(r1 - rho0, r0 - rho0), "u": _err(u1, u0), "phi": _err(p1, p0), "Q": _err(q1, q0)}


def _unwrap(prev, new, n):
    """Unwrap a periodic coordinate series."""
    d = new - prev
    return prev + (d - n * np.round(d / n))


class Track:
    def __init__(self, shape):
        self.n = np.array(shape[::-1], dtype=float)  # x, y, z sizes
        self.pos = None
        self.hist = []

    def add(self, t, sim):
        _, circ, _ = sim.centre()
        c = np.asarray(circ, dtype=float)
        self.pos = c if self.pos is None else _unwrap(self.pos, c, self.n)
        self.hist.append((t, self.pos.tolist()))

    def velocity(self, window):
        t1, p1 = self.hist[-1]
        for t0, p0 in self.hist:
            if t1 - t0 <= window:
                return (np.array(p1) - np.array(p0)) / (t1 - t0)
        return np.zeros(3)


def run_pair(workload, precisions, steps, every, zeta=None, log=print):
    p = inputs.params_for(workload) if zeta is None else inputs.params_for(workload, zeta=zeta)
    phi, q5 = inputs.workload_fields(workload)
    sims = {pr: Sim(p, phi, q5, precision=pr) for pr in ("fp64",) + tuple(precisions)}
    tracks = {pr: Track(phi.shape) for pr in sims}
    rows = []
    t0 = time.time()
    for t in range(0, steps + 1, every):
        if t:
            for s in sims.values():
                s.step(every)
        row = {"step": t}
        for pr, s in sims.items():
            tracks[pr].add(t, s)
            tot = s.totals()
            row[pr] = {"centre": tracks[pr].pos.tolist(), "mass": tot["mass"], "phi_total": tot["phi_total"],
                       "free_energy": tot["free_energy"], "kinetic_energy": tot["kinetic_energy"]}
            if pr != "fp64":
                row[pr]["errors"] = field_errors(s, sims["fp64"], p["rho0"])
                row[pr]["centre_error"] = float(np.linalg.norm(tracks[pr].pos - tracks["fp64"].pos))
        rows.append(row)
        log(f"# {workload} zeta={p['zeta']} step {t}/{steps} ({time.time() - t0:.1f}s)")
    vel = {pr: tracks[pr].velocity(1000).tolist() for pr in sims}
    for s in sims.values():
        s.close()
    return {"workload": workload, "zeta": p["zeta"], "steps": steps, "every": every, "rows": rows,
            "velocity_last_1000": vel}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["droplet64", "droplet128"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--steps", type=int, default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    out = []
    if args.workload == "droplet64":
        steps = args.steps or inputs.WORKLOADS["droplet64"]["steps"]
        for z in inputs.WORKLOADS["droplet64"]["zetas"]:
            out.append(run_pair("droplet64", ("fp32",), steps, 100, zeta=z, log=log))
    else:
        steps = args.steps or inputs.WORKLOADS["droplet128"]["steps"]
        out.append(run_pair("droplet128", ("fp32", "fp16s"), steps, 500, log=log))
    text = json.dumps(out)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
