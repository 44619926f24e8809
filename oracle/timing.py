"""Wall-clock timing of the FP64 oracle (test infrastructure).

    python -m oracle.timing [--repeats 3]

Times the oracle's step on the 64x32x32 canopy case (200 steps) and on the
128x64x64 crop (1000 steps at all threads; 100 steps on one thread) in child
processes with OMP_NUM_THREADS = 1 and = all host CPUs, median of the
repeats, and prints one JSON line per case: wall seconds, CPU-seconds
(wall x threads) and oracle MLUPS, with the CPU model and core count.
"""
import argparse
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _child(case, steps, repeats):
    sys.path.insert(0, ROOT)
    from oracle import ref
    from paper_2206_15454_amd import inputs

    w = {"c1": inputs.C1, "crop": inputs.CROP}[case]
    walls = []
    for _ in range(repeats):
        sim = ref.RefLBM(w.nx, w.ny, w.nz, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi)
        sim.set_canopy(w.cd, inputs.lad_constant(w))
        rho, u = inputs.init_fields(w)
        sim.init(rho, u)
        t0 = time.perf_counter()
        sim.step(steps)
        walls.append(time.perf_counter() - t0)
        sim.close()
    print(json.dumps({"threads": ref.threads(), "walls": walls}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--child", nargs=3, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.child:
        _child(args.child[0], int(args.child[1]), int(args.child[2]))
        return
    ncpu = len(os.sched_getaffinity(0))
    for case, steps, threads, reps in (("c1", 200, 1, args.repeats),
                                       ("c1", 200, ncpu, args.repeats),
                                       ("crop", 1000, ncpu, args.repeats),
                                       ("crop", 100, 1, 1)):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, "-m", "oracle.timing", "--child", case, str(steps),
                              str(reps)], cwd=ROOT, env=env, capture_output=True, text=True,
                             check=True).stdout
        r = json.loads(out.strip().splitlines()[-1])
        cells = {"c1": 64 * 32 * 32, "crop": 128 * 64 * 64}[case]
        wall = statistics.median(r["walls"])
        print(json.dumps({"case": case, "steps": steps, "threads": r["threads"],
                          "repeats": len(r["walls"]), "wall_s": round(wall, 3),
                          "cpu_s": round(wall * r["threads"], 3),
                          "MLUPS": round(cells * steps / wall / 1e6, 3), "cpu": cpu_model(),
                          "host_cpus": ncpu}), flush=True)


if __name__ == "__main__":
    main()
