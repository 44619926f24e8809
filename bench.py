"""Throughput of the fused LBM-LES-canopy step on one MI355X.

A step is one lattice-Boltzmann time step of the whole hot path over the
production canopy boundary layer (512x128x256 cells, FP32 storage,
Smagorinsky closure, Lalic-Mihailovic LAD with h = 12, LAI 2, C_D = 0.15,
bounce-back ground, free-slip top): one fused kernel launch that streams in
place, applies the walls, computes the moments, the canopy drag, the eddy
viscosity, the forced BGK collision, stores in place and accumulates the FP64
impulse; every 10th step also accumulates the plane statistics, the last
step writes the moments and the timed region ends with the FP64
diagnostics reduction.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  value = cells * steps / time / 1e6 (MLUPS).
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS and % of HBM roofline; low-precision+learned vs plain FP32 at "
          "≤1% profile error")
HBM_PEAK_GBS = 8000.0
# The paper's own MLUPS (Table tab:mesh_cost: whole-program time per 10^6
# steps on one RTX 2070 SUPER, constant-LAD forest, precision unstated) for
# the workloads that are exactly its meshes; context from another machine.
PAPER_MLUPS = {"paper-abl-200x80x160-case1": 83.7, "paper-abl-250x100x200-case1": 99.0,
               "paper-abl-350x140x280-case1": 97.7}
BYTES_PER_ELT = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2, "bf16sr": 2}
KERNEL_SOURCES = ("paper_2206_15454_amd/csrc/lbm_kernels.hip",
                  "paper_2206_15454_amd/csrc/lbm_device.h",
                  "paper_2206_15454_amd/csrc/lbm_api.hip")


def kernel_hash():
    """Hash of the step kernels' source with its comments removed (an edit
    of a comment leaves the compiled kernels, and so their counters, as they
    were; the sources hold no comment markers inside string literals)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(l.rstrip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(storage, w):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, only if it was taken on the current kernel source and
    the same workload."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("entries", {}).get(f"{w.name}/{storage}")
    if not ent or ent.get("kernel_hash") != kernel_hash() or ent.get("cells") != w.n:
        return None
    return ent.get("bytes_per_launch")


def workload_lad(w, lad_fn, inputs):
    """LAD per row from a workload, with the given Eq. (af_theory) routine"""
    if w.lad_lalic is not None:
        h, ym, lai = w.lad_lalic
        return lad_fn(h, ym, w.ny, lai=lai)
    if w.lad_profile is not None:
        h, ym, afm = w.lad_profile
        return lad_fn(h, ym, w.ny, afm=afm)
    return inputs.lad_constant(w)


_FOREST_CODES = {}


def forest_codes(w, lbm, inputs):
    """Per-cell forest codes of a heterogeneous-forest workload (the library's
    routine on the workload's seeded point cloud), built once per workload."""
    if w.name not in _FOREST_CODES:
        pts = inputs.forest_points(w)
        _FOREST_CODES[w.name] = lbm.forest_codes(pts, w.nx, w.ny, w.nz, w.forest[4])[0]
    return _FOREST_CODES[w.name]


def make_sim(w, storage, lbm, inputs):
    sim = lbm.LBM(w.nx, w.ny, w.nz, storage, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi,
                  u_wall=w.u_wall, forest_map=w.forest is not None)
    if w.forest is not None:
        sim.set_forest(w.cd, w.forest[3], forest_codes(w, lbm, inputs))
        return sim
    sim.set_canopy(w.cd, workload_lad(w, lbm.lad_lalic, inputs))
    return sim


def time_steps(sim, steps, warmup, torch):
    """(total_ms, step_ms): events on the stream the kernels run on (torch's
    current stream, handed to the library)."""
    sim.stats_reset()
    sim.stats_enable(10)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    sim.step(steps)
    e1.record()
    d = sim.diag()  # FP64 reductions; synchronises
    e2.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e2), e0.elapsed_time(e1), d


def time_training(torch, lbm, batch=8192, steps=200, big=1 << 20):
    """Closure training throughput on synthetic samples of the training
    set's shape (X [n][9] FP32, y [n]): Adam steps at the training batch, and
    one gradient evaluation over `big` samples (no update).  Algorithmic
    work: forward + backward = 3 x 9472 flop per sample."""
    import numpy as np

    from paper_2206_15454_amd import closure

    g = torch.Generator(device="cuda").manual_seed(5)
    X = torch.randn(big, 9, device="cuda", generator=g)
    y = torch.rand(big, device="cuda", generator=g) * 1e-3
    p, mean, std, _, _, s, _ = closure.read_blob(closure.trained_blob())
    tr = lbm.Trainer(p, np.zeros(9), np.ones(9), s, max_batch=big)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for b in range(20):
        tr.step(X[b * batch:(b + 1) * batch], y[b * batch:(b + 1) * batch], update=True, loss=False)
    torch.cuda.synchronize()
    ev[0].record()
    for b in range(steps):
        o = (b % 100) * batch
        tr.step(X[o:o + batch], y[o:o + batch], update=True, loss=False)
    ev[1].record()
    tr.step(X, y, update=False, loss=False)
    torch.cuda.synchronize()
    ev[2].record()
    tr.step(X, y, update=False, loss=False)
    ev[3].record()
    torch.cuda.synchronize()
    tr.close()
    t_steps = ev[0].elapsed_time(ev[1]) * 1e-3
    t_big = ev[2].elapsed_time(ev[3]) * 1e-3
    flop = 3 * 9472
    return {"adam_steps_batch": batch, "samples_per_s": round(steps * batch / t_steps),
            "us_per_step": round(t_steps / steps * 1e6, 1),
            "gradient_pass_samples": big, "gradient_samples_per_s": round(big / t_big),
            "gradient_tflops": round(big * flop / t_big / 1e12, 2)}


def cpu_baseline(w, target_s=10.0):
    """The FP64 oracle on a z-slab of the same workload (all host cores)."""
    import numpy as np

    from oracle import ref
    from paper_2206_15454_amd import inputs

    nz = max(1, min(w.nz, 16))
    ws = inputs.scaled(w, w.nx, w.ny, nz)
    sim = ref.RefLBM(ws.nx, ws.ny, ws.nz, ws.tau0, ws.c_smag, ws.g, ws.bc_lo, ws.bc_hi)
    sim.set_wall_velocity(w.u_wall)
    if w.forest is not None:
        # the oracle's own codes of the whole point cloud, first nz planes
        codes, _ = ref.forest_codes(inputs.forest_points(w), w.nx, w.ny, w.nz, w.forest[4])
        sim.set_forest(ws.cd, w.forest[3], codes[:nz])
    else:
        sim.set_canopy(ws.cd, workload_lad(w, ref.lad_lalic, inputs))
    rho, u = inputs.init_fields(ws)
    sim.init(rho, u)
    t0 = time.perf_counter()
    sim.step(2)
    per = (time.perf_counter() - t0) / 2
    steps = int(max(2, min(500, target_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    del np
    return {"value": round(ws.n * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": ref.threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, {ws.nx}x{ws.ny}x{ws.nz} z-slab of the same workload, "
                      f"{steps} steps, {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=list(BYTES_PER_ELT))
    ap.add_argument("--variants", default="f64,f16s,bf16s,bf16sr",
                    help="other storage types timed on the same workload ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mlp", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the learned closure on the same workload (default on)")
    ap.add_argument("--mlp-storage", default="bf16sr", choices=list(BYTES_PER_ELT))
    ap.add_argument("--mlp-every", default="1,4,8",
                    help="closure intervals timed with the learned closure (1 = every step)")
    ap.add_argument("--mlp-canopy-every", default="1,8",
                    help="intervals timed with the closure restricted to the canopy layer "
                         "(y/h <= 4, Smagorinsky above)")
    ap.add_argument("--mlp-also", default="f16s",
                    help="other storage types timed with the learned closure every step, "
                         "everywhere and in the canopy layer ('' for none)")
    ap.add_argument("--c5", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 1024x256x512 pair of the learned-closure comparison: "
                         "FP32 + Smagorinsky against low-precision storage + learned closure")
    ap.add_argument("--train", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the closure training kernels (Adam steps at batch 8192 and "
                         "a gradient pass over 1M samples)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c3", "c5", "abl1", "abl2", "abl3", "abl_coarse", "abl_medium",
                             "channel", "forest", "slab"],
                    help="c2: production canopy 512x128x256 (default); c3/c5: 1024x256x512 "
                         "with the 64x32x32 case's physics; abl1-3: the paper's ABL fine mesh "
                         "350x140x280 with LAD cases 1-3; abl_coarse/abl_medium: its "
                         "200x80x160 and 250x100x200 meshes (case 1); channel: the paper's Re_tau=180 "
                         "channel 372x62x124; forest: heterogeneous forest from a synthetic "
                         "point cloud (per-cell forest codes) on 512x128x256; slab: one GPU's "
                         "128x256x512 share of 1024x256x512 split 8 ways along x")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the method here is a single-GPU kernel "
              "(multi-GPU slab decomposition is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2206_15454_amd import inputs, lbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel(), "copy_bytes_written": y.numel(),
                          "launches": 3}), flush=True)
        return
    w = {"c2": inputs.C2, "c3": inputs.C3, "c5": inputs.C5, "abl1": inputs.ABL1,
         "abl2": inputs.ABL2, "abl3": inputs.ABL3, "channel": inputs.CHANNEL,
         "forest": inputs.FOREST, "slab": inputs.SLAB, "abl_coarse": inputs.ABL_COARSE,
         "abl_medium": inputs.ABL_MEDIUM}[args.workload]
    if args.workload == "c2":
        rho, u = inputs.init_fields(w)
        rho_d = torch.from_numpy(rho).cuda()
        u_d = torch.from_numpy(u).cuda()
    else:
        rho_d, u_d = inputs.init_fields_torch(w, torch.device("cuda"))

    def run(storage, steps, warmup):
        sim = make_sim(w, storage, lbm, inputs)
        sim.init(rho_d, u_d)
        total, step_ms, d = time_steps(sim, steps, warmup, torch)
        sim.close()
        return total, step_ms, d

    total_ms, step_ms, diag = run(args.storage, args.steps, args.warmup)
    mlups = w.n * args.steps / (total_ms * 1e-3) / 1e6
    per_launch_s = step_ms * 1e-3 / args.steps
    # populations read and written once; a heterogeneous forest adds its
    # 16-bit table index per cell
    extra = 2 if w.forest is not None else 0
    algo_bytes = (2 * 19 * BYTES_PER_ELT[args.storage] + extra) * w.n
    achieved = algo_bytes / per_launch_s / 1e9
    traffic = measured_traffic(args.storage, w)

    variants = {}
    for st in [s for s in args.variants.split(",") if s and s != args.storage]:
        k = max(50, args.steps // 4)
        t_ms, s_ms, _ = run(st, k, 20)
        b = (2 * 19 * BYTES_PER_ELT[st] + extra) * w.n
        v = w.n * k / (t_ms * 1e-3) / 1e6
        variants[st] = {"MLUPS": round(v, 1), "vs_" + args.storage: round(v / mlups, 3),
                        "hbm_frac": round(b / (s_ms * 1e-3 / k) / 1e9 / HBM_PEAK_GBS, 4)}

    if args.mlp:
        from paper_2206_15454_amd import closure

        # the network trained on the canopy case at twice the resolution, used
        # everywhere and restricted to the canopy layer (a wavefront whose cells
        # all fall back skips the network, so the restriction is faster)
        st = args.mlp_storage
        runs = [(st, closure.trained_blob(), int(e), "") for e in args.mlp_every.split(",") if e]
        runs += [(st, closure.canopy_layer_blob(), int(e), "(y<4h)")
                 for e in args.mlp_canopy_every.split(",") if e]
        for other in (x for x in args.mlp_also.split(",") if x and x != st):
            if other not in BYTES_PER_ELT:
                raise SystemExit(f"--mlp-also: unknown storage {other!r}")
            runs += [(other, closure.trained_blob(), 1, ""),
                     (other, closure.canopy_layer_blob(), 1, "(y<4h)")]
        for st, blob, every, tag in runs:
            sim = make_sim(w, st, lbm, inputs)
            sim.init(rho_d, u_d)
            sim.set_closure(blob)
            sim.set_closure_interval(every)
            k = max(50, args.steps // 4)
            t_ms, s_ms, d = time_steps(sim, k, 24, torch)
            sim.close()
            # steps that reuse nu_t also read it (4 B/cell FP32, 8 B FP64);
            # evaluating steps write it when it is reused
            nb = 8 if st == "f64" else 4
            b = (2 * 19 * BYTES_PER_ELT[st] + extra) * w.n
            b += (nb * w.n if every > 1 else 0)
            name = st + "+mlp" + tag + ("" if every == 1 else f"/{every}")
            v = w.n * k / (t_ms * 1e-3) / 1e6
            variants[name] = {"MLUPS": round(v, 1), "vs_" + args.storage: round(v / mlups, 3),
                              "hbm_frac": round(b / (s_ms * 1e-3 / k) / 1e9 / HBM_PEAK_GBS, 4),
                              "closure_every": every, "mlp_fallback": d["mlp_fallback"]}

    if args.c5 and args.workload == "c2":
        # the learned-closure comparison at its configured size (1024x256x512,
        # the 64x32x32 case's physics): FP32 + Smagorinsky, then the
        # low-precision storage without the network, and with it evaluated
        # every step and every 4th step.  The trained network with its input
        # ranges opened, so that every cell evaluates it here too.
        from paper_2206_15454_amd import closure

        net = closure.everywhere(closure.trained_blob())
        w5 = inputs.C5
        rho5, u5 = inputs.init_fields_torch(w5, torch.device("cuda"))
        k = max(50, args.steps // 10)
        c5 = {}
        for name, st, blob, every in (("f32", "f32", None, 1),
                                      (args.mlp_storage, args.mlp_storage, None, 1),
                                      (args.mlp_storage + "+mlp", args.mlp_storage, net, 1),
                                      (args.mlp_storage + "+mlp/4", args.mlp_storage, net, 4)):
            sim = make_sim(w5, st, lbm, inputs)
            sim.init(rho5, u5)
            if blob is not None:
                sim.set_closure(blob)
                sim.set_closure_interval(every)
            t_ms, s_ms, d = time_steps(sim, k, 10, torch)
            sim.close()
            c5[name] = {"MLUPS": round(w5.n * k / (t_ms * 1e-3) / 1e6, 1),
                        "hbm_frac": round((2 * 19 * BYTES_PER_ELT[st] + (4 if every > 1 else 0))
                                          * w5.n / (s_ms * 1e-3 / k) / 1e9 / HBM_PEAK_GBS, 4)}
            if blob is not None:
                c5[name]["mlp_fallback"] = d["mlp_fallback"]
        for name in c5:
            c5[name]["vs_f32"] = round(c5[name]["MLUPS"] / c5["f32"]["MLUPS"], 3)
        variants["c5:1024x256x512"] = c5
        del rho5, u5

    if args.train and args.workload == "c2":
        variants["train:9-64-64-1"] = time_training(torch, lbm)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (round(mlups / PAPER_MLUPS[w.name], 1) if w.name in PAPER_MLUPS else None),
        "dtype": "f32" if args.storage != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "nz": w.nz,
                   "storage": args.storage, "closure": "smagorinsky",
                   "canopy": ("forest codes: %d trees/1000 ground cells, h %g-%g, a_fm %g" % (
                                  round(1000 * w.forest[0]), w.forest[1], w.forest[2], w.forest[3])
                              if w.forest else
                              "lalic h=%g LAI=%g" % (w.lad_lalic[0], w.lad_lalic[2])
                              if w.lad_lalic else
                              "lalic h=%g a_fm=%g" % (w.lad_profile[0], w.lad_profile[2])
                              if w.lad_profile else
                              "LAD %g below row %d" % (w.lad_const, w.canopy_rows)),
                   "stats_every": 10},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "variants": variants,
        "diag": {"mass": diag["mass"], "max_u": diag["max_u"], "t": diag["t"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
