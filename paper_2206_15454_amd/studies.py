"""Drivers of the studies the metric names (GPU only; results as JSON).

  python -m paper_2206_15454_amd.studies closure   --out DIR
      learned closure: a run at twice the resolution (1024x256x512, FP32,
      h = 24) -> training samples at three snapshots -> GPU training (MFMA
      forward/backward + Adam) -> closure blob -> the production canopy case
      (512x128x256) with BF16S storage + learned closure against FP32 storage
      + Smagorinsky (and a perturbed FP32 run for the chaotic noise floor),
      profiles averaged in time and over x-z; throughput of both forms.
  python -m paper_2206_15454_amd.studies interval --out DIR
      the trained closure evaluated every k = 1, 2, 4, 8 steps (nu_t reused
      in between) on the production canopy case against FP32 + Smagorinsky.
  python -m paper_2206_15454_amd.studies layer --out DIR
      the trained closure restricted to the canopy layer (y/h <= 4, through
      its feature range; Smagorinsky above) against the unrestricted one.
  python -m paper_2206_15454_amd.studies abl --out DIR
      the paper's ABL cases 1-3 (350x140x280): mean profiles, u_* at y/h = 2.
  python -m paper_2206_15454_amd.studies aposteriori --out DIR
      the whole learned-closure pipeline at half size (fine 512x128x256 ->
      filter -> GPU training -> coarse 256x64x128 with each closure) and the
      profile errors of both closures against the filtered fine statistics.
  python -m paper_2206_15454_amd.studies precision --out DIR
      storage precision on 1024x256x512 (physics of the 64x32x32 canopy
      case): FP32 / FP16S / BF16S fields after 1000 steps against the GPU FP64
      run (itself pinned to the CPU oracle by the parity tests); mean and RMS
      profiles after a long run; throughput per storage type.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import closure, inputs, lbm

MEAN_COLS = {"u": 0, "v": 1, "w": 2}


def _log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def _lad(w):
    if w.lad_lalic is not None:
        h, ym, lai = w.lad_lalic
        return lbm.lad_lalic(h, ym, w.ny, lai=lai)
    if w.lad_profile is not None:
        h, ym, afm = w.lad_profile
        return lbm.lad_lalic(h, ym, w.ny, afm=afm)
    return inputs.lad_constant(w)


def make(w, storage, rho, u, blob=None):
    sim = lbm.LBM(w.nx, w.ny, w.nz, storage, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi,
                  u_wall=w.u_wall)
    sim.set_canopy(w.cd, _lad(w))
    sim.init(rho, u)
    if blob is not None:
        sim.set_closure(blob)
    return sim


def timed_steps(sim, n, torch, chunk=1000, label=""):
    """n steps in chunks (progress lines); returns GPU ms."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    total = 0.0
    done = 0
    while done < n:
        k = min(chunk, n - done)
        e0.record()
        sim.step(k)
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
        done += k
        if label:
            _log(f"{label}: {done}/{n} steps")
    return total


def profiles(prof):
    """mean and RMS profiles from the [ny][10] means"""
    u, v, w = prof[:, 0], prof[:, 1], prof[:, 2]
    var = np.maximum(prof[:, 3:6] - prof[:, 0:3] ** 2, 0.0)
    return {"u": u, "v": v, "w": w, "u_rms": np.sqrt(var[:, 0]), "v_rms": np.sqrt(var[:, 1]),
            "w_rms": np.sqrt(var[:, 2]), "uv": prof[:, 6] - u * v, "vw": prof[:, 8] - v * w,
            "nu_t": prof[:, 9]}


def friction_velocity(prof, y):
    """u_* = (<u'v'>^2 + <v'w'>^2)^(1/4) at height y (cell centres j + 1/2,
    linear interpolation between rows), the definition of Sec. 5.1."""
    p = profiles(prof)
    yc = np.arange(prof.shape[0]) + 0.5
    uv = float(np.interp(y, yc, p["uv"]))
    vw = float(np.interp(y, yc, p["vw"]))
    return (uv * uv + vw * vw) ** 0.25


def coarsen_profile(prof):
    """[2m][10] means on a fine grid -> [m][10] means on the 2x coarser rows"""
    return 0.5 * (prof[0::2] + prof[1::2])


def profile_errors(a, b):
    """max_y |a - b| / max_y |b| for the mean and RMS profiles"""
    pa, pb = profiles(a), profiles(b)
    out = {}
    for k in ("u", "u_rms", "v_rms", "w_rms", "uv"):
        den = np.max(np.abs(pb[k]))
        out[k] = float(np.max(np.abs(pa[k] - pb[k])) / den) if den > 0 else 0.0
    return out


def field_errors(a, b):
    """per-field max and RMS error of a against b (normalised by max |b|)"""
    den = float(np.max(np.abs(b)))
    d = np.abs(a - b)
    return {"max": float(d.max() / den), "rms": float(np.sqrt(np.mean(d * d)) / den)}


# ---------------------------------------------------------------------------
# learned closure
# ---------------------------------------------------------------------------

def closure_study(out, fine_steps=40000, snapshots=(20000, 30000, 40000), coarse_steps=20000,
                  avg_from=10000, n_train=None, epochs=3, batch=8192, lr=1e-3):
    import torch

    dev = torch.device("cuda")
    res = {"fine": {}, "train": {}, "aposteriori": {}, "mlups": {}}
    wf, wc = inputs.C4, inputs.C2
    lad_c = _lad(wc)
    h_c = wc.lad_lalic[0]

    # 1. the run at twice the resolution, with its own statistics
    rho, u = inputs.init_fields_torch(wf, dev)
    fine = make(wf, "f32", rho, u)
    del rho, u
    Xs, ys = [], []
    done = 0
    ms = 0.0
    for snap in snapshots:
        if done < fine_steps // 2 <= snap:
            ms += timed_steps(fine, fine_steps // 2 - done, torch, 2000, "fine")
            done = fine_steps // 2
            fine.stats_reset()
            fine.stats_enable(20)
        ms += timed_steps(fine, snap - done, torch, 2000, "fine")
        done = snap
        X, y = fine.closure_samples(wc.tau0, h_c, lad_c)
        Xs.append(X)
        ys.append(y)
        _log(f"snapshot at fine step {snap}: {y.numel()} samples, "
             f"mean target {float(y.mean()):.3e}, nonzero {float((y > 0).float().mean()):.3f}")
    prof_f, nsf = fine.stats_read()
    d = fine.diag()
    res["fine"] = {"cells": wf.n, "steps": done, "ms": ms, "MLUPS": wf.n * done / ms / 1e3,
                   "stat_samples": nsf, "max_u": d["max_u"]}
    fine.close()
    prof_ref = coarsen_profile(prof_f)

    # 2. training set (90/10 split by z slabs of every snapshot), statistics
    nz = wc.nz
    per = Xs[0].shape[0]
    cut = per * 9 // 10
    Xtr = torch.cat([x[:cut] for x in Xs]).cpu().numpy()
    ytr = torch.cat([y[:cut] for y in ys]).cpu().numpy()
    Xva = torch.cat([x[cut:] for x in Xs])
    yva = torch.cat([y[cut:] for y in ys])
    del Xs, ys
    mean = Xtr.mean(axis=0, dtype=np.float64)
    std = Xtr.std(axis=0, dtype=np.float64)
    std[std <= 0] = 1.0
    lo = Xtr.min(axis=0).astype(np.float64)
    hi = Xtr.max(axis=0).astype(np.float64)
    s = float(ytr.mean()) if ytr.mean() > 0 else 1e-5
    rng = np.random.default_rng(7)
    n_train = Xtr.shape[0] if n_train is None else min(int(n_train), Xtr.shape[0])
    idx = rng.permutation(Xtr.shape[0])[:n_train]
    Xd = torch.from_numpy(np.ascontiguousarray(Xtr[idx])).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(ytr[idx])).to(dev)
    var = float(np.var(ytr / s))
    del Xtr, ytr
    p0 = closure.join(rng.normal(size=(64, 9)) / 3.0, np.zeros(64),
                      rng.normal(size=(64, 64)) / 8.0, np.zeros(64),
                      rng.normal(size=64) / 8.0, math.log(math.e - 1.0))
    tr = lbm.Trainer(p0, mean, std, s, lr=lr, max_batch=batch)
    nb = Xd.shape[0] // batch
    t0 = time.time()
    hist = []
    for ep in range(epochs):
        for b in range(nb):
            want = (b % 500 == 0)
            l = tr.step(Xd[b * batch:(b + 1) * batch], yd[b * batch:(b + 1) * batch],
                        update=True, loss=want)
            if want:
                hist.append(l)
                _log(f"epoch {ep} batch {b}/{nb} loss {l:.4e}")
    torch.cuda.synchronize()
    train_s = time.time() - t0

    def val_loss():
        tot, cnt = 0.0, 0
        for b in range(0, yva.numel() - batch + 1, batch * 8):
            tot += tr.step(Xva[b:b + batch], yva[b:b + batch], update=False) * batch
            cnt += batch
        return tot / max(cnt, 1)

    vl = val_loss()
    p, _ = tr.get()
    tr.close()
    blob = closure.make_blob(p, mean, std, lo, hi, s, h_c)
    res["train"] = {"samples_train": int(n_train), "epochs": epochs, "batch": batch, "lr": lr,
                    "seconds": train_s, "steps": epochs * nb,
                    "samples_per_s": epochs * nb * batch / train_s, "loss_history": hist,
                    "val_loss": vl, "val_target_variance": var,
                    "val_explained_variance": 1.0 - vl / var if var > 0 else None,
                    "out_scale": s, "mean": mean.tolist(), "std": std.tolist(),
                    "lo": lo.tolist(), "hi": hi.tolist()}
    with open(os.path.join(out, "closure_blob.bin"), "wb") as f:
        f.write(blob)
    _log("training done", json.dumps({k: res["train"][k] for k in ("val_loss", "val_target_variance")}))
    del Xd, yd, Xva, yva

    # 3. a-posteriori: the production canopy case with each closure/storage
    rho, u = inputs.init_fields_torch(wc, dev)
    runs = {"f32_smag": ("f32", None, 0.0), "f32_smag_perturbed": ("f32", None, 1e-7),
            "f32_mlp": ("f32", blob, 0.0),
            "bf16s_smag": ("bf16s", None, 0.0), "bf16s_mlp": ("bf16s", blob, 0.0),
            "bf16sr_smag": ("bf16sr", None, 0.0), "bf16sr_mlp": ("bf16sr", blob, 0.0),
            "f16s_smag": ("f16s", None, 0.0), "f16s_mlp": ("f16s", blob, 0.0)}
    profs = {}
    for name, (st, b, eps) in runs.items():
        uu = u if eps == 0.0 else u * (1.0 + eps)
        sim = make(wc, st, rho, uu, b)
        try:
            ms = timed_steps(sim, avg_from, torch, 5000, name)
            sim.stats_reset()
            sim.stats_enable(10)
            ms += timed_steps(sim, coarse_steps - avg_from, torch, 5000, name)
            prof, ns = sim.stats_read()
            d = sim.diag()
        except lbm.LBMError as e:
            res["aposteriori"][name] = {"error": str(e)}
            _log(name, "failed:", e)
            sim.close()
            continue
        profs[name] = prof
        res["aposteriori"][name] = {"MLUPS": wc.n * coarse_steps / ms / 1e3, "stat_samples": ns,
                                    "mlp_fallback_last_step": d["mlp_fallback"],
                                    "fallback_fraction": d["mlp_fallback"] / wc.n,
                                    "max_u": d["max_u"], "profile": profiles(prof)["u"].tolist()}
        sim.close()
    A = res["aposteriori"]
    for x in runs:
        if x != "f32_smag" and x in profs and "f32_smag" in profs:
            A[f"e_{x}_vs_f32_smag"] = profile_errors(profs[x], profs["f32_smag"])
    A["noise_floor_f32_perturbed"] = A.pop("e_f32_smag_perturbed_vs_f32_smag", None)
    for x in runs:
        if x in profs:
            A[f"e_{x}_vs_filtered_fine"] = profile_errors(profs[x], prof_ref)
            A[x]["nu_t_mean"] = float(np.mean(profiles(profs[x])["nu_t"]))
    A["filtered_fine_profile"] = profiles(prof_ref)["u"].tolist()
    A["u_tau"] = math.sqrt(wc.g[0] * wc.ny)

    # 4. throughput of both forms at 1024x256x512 (the network with its input
    # ranges opened: on this workload's physics the trained ranges would make
    # most wavefronts fall back and skip it)
    w5 = inputs.C5
    rho, u = inputs.init_fields_torch(w5, dev)
    net = closure.everywhere(blob)
    for name, (st, b) in {"f32_smag": ("f32", None), "bf16s_mlp": ("bf16s", net),
                          "bf16sr_mlp": ("bf16sr", net), "bf16s_smag": ("bf16s", None),
                          "f16s_mlp": ("f16s", net), "bf16sr_smag": ("bf16sr", None)}.items():
        sim = make(w5, st, rho, u, b)
        sim.step(20)
        ms = timed_steps(sim, 200, torch, 200)
        res["mlups"][name + "_1024x256x512"] = w5.n * 200 / ms / 1e3
        sim.close()
    with open(os.path.join(out, "closure_study.json"), "w") as f:
        json.dump(res, f, indent=1)
    _log("closure study:", json.dumps({"aposteriori": {k: v["u"] for k, v in A.items()
                                                      if k.startswith(("e_", "noise")) and v},
                                      "mlups": res["mlups"]}))
    return res


# ---------------------------------------------------------------------------
# precision
# ---------------------------------------------------------------------------

def precision_study(out, steps=1000, long_steps=20000, avg_from=10000,
                    storages=("f32", "f16s", "bf16s", "bf16sr")):
    import torch

    dev = torch.device("cuda")
    w = inputs.C3
    rho, u = inputs.init_fields_torch(w, dev)
    res = {"workload": w.name, "steps": steps, "fields": {}, "mlups": {}, "profiles": {}}
    ref = make(w, "f64", rho, u)
    ms = timed_steps(ref, steps, torch, 500, "f64")
    res["mlups"]["f64"] = w.n * steps / ms / 1e3
    r0, u0, n0, _ = ref.moments(device=True)
    ref.close()
    for st in storages:
        sim = make(w, st, rho, u)
        ms = timed_steps(sim, steps, torch, 500, st)
        res["mlups"][st] = w.n * steps / ms / 1e3
        r1, u1, n1, _ = sim.moments(device=True)
        sim.close()
        fe = {}
        for name, a, b in (("rho", r1, r0), ("u", u1, u0), ("nu_t", n1, n0)):
            d = (a - b).abs()
            den = float(b.abs().max())
            fe[name] = {"max": float(d.max()) / den, "rms": float(d.pow(2).mean().sqrt()) / den}
        res["fields"][st] = fe
        _log(st, json.dumps(fe))
        del r1, u1, n1
    del r0, u0, n0
    if long_steps:
        profs = {}
        for st, eps in (("f32", 0.0), ("bf16s", 0.0), ("bf16sr", 0.0), ("f16s", 0.0),
                        ("f32_perturbed", 1e-7)):
            sim = make(w, st.split("_")[0], rho, u if eps == 0.0 else u * (1.0 + eps))
            timed_steps(sim, avg_from, torch, 5000, st)
            sim.stats_reset()
            sim.stats_enable(10)
            timed_steps(sim, long_steps - avg_from, torch, 5000, st)
            profs[st] = sim.stats_read()[0]
            sim.close()
        for st in ("bf16s", "bf16sr", "f16s", "f32_perturbed"):
            res["profiles"][st + "_vs_f32"] = profile_errors(profs[st], profs["f32"])
        _log("profiles:", json.dumps(res["profiles"]))
    with open(os.path.join(out, "precision_study.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


# ---------------------------------------------------------------------------
# learned closure evaluated every k steps
# ---------------------------------------------------------------------------

def interval_study(out, coarse_steps=20000, avg_from=10000, intervals=(1, 2, 4, 8)):
    """A-posteriori error of the trained closure when it is evaluated only on
    every k-th step (nu_t reused in between), on the production canopy case,
    against FP32 + Smagorinsky, with the perturbed-start noise floor."""
    import torch

    dev = torch.device("cuda")
    wc = inputs.C2
    blob = closure.trained_blob()
    rho, u = inputs.init_fields_torch(wc, dev)
    runs = {"f32_smag": ("f32", None, 0.0, 1), "f32_smag_perturbed": ("f32", None, 1e-7, 1),
            "f32_smag_perturbed2": ("f32", None, -1e-7, 1), "f32_mlp": ("f32", blob, 0.0, 1)}
    for k in intervals:
        runs[f"bf16sr_mlp_every{k}"] = ("bf16sr", blob, 0.0, k)
    runs["f16s_mlp_every4"] = ("f16s", blob, 0.0, 4)
    res = {"workload": wc.name, "steps": coarse_steps, "avg_from": avg_from, "runs": {},
           "errors": {}, "profiles": {}}
    profs = {}
    for name, (st, b, eps, every) in runs.items():
        sim = make(wc, st, rho, u if eps == 0.0 else u * (1.0 + eps), b)
        if b is not None:
            sim.set_closure_interval(every)
        ms = timed_steps(sim, avg_from, torch, 5000, name)
        sim.stats_reset()
        sim.stats_enable(10)
        ms += timed_steps(sim, coarse_steps - avg_from, torch, 5000, name)
        prof, ns = sim.stats_read()
        d = sim.diag()
        sim.close()
        profs[name] = prof
        h = wc.lad_lalic[0]
        res["runs"][name] = {"MLUPS": wc.n * coarse_steps / ms / 1e3, "closure_every": every,
                             "stat_samples": ns, "max_u": d["max_u"],
                             "mlp_fallback_last_eval": d["mlp_fallback"],
                             "u_star_2h": friction_velocity(prof, 2 * h)}
        res["profiles"][name] = {k: v.tolist() for k, v in profiles(prof).items()}
        _log(name, json.dumps(res["runs"][name]))
    for name in runs:
        if name != "f32_smag":
            res["errors"][name] = profile_errors(profs[name], profs["f32_smag"])
    _log("errors vs f32_smag:", json.dumps({k: round(v["u"], 5) for k, v in res["errors"].items()}))
    with open(os.path.join(out, "interval_study.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


def layer_study(out, cut=4.0, coarse_steps=20000, avg_from=10000):
    """The trained closure restricted to the canopy layer (y/h <= cut through
    its feature range; Smagorinsky above) against the unrestricted closure
    and FP32 + Smagorinsky on the production canopy case: mean and RMS
    profile errors, with the perturbed-start noise floor."""
    import torch

    dev = torch.device("cuda")
    wc = inputs.C2
    full = closure.trained_blob()
    low = closure.with_range(full, "y_over_h", hi=cut)
    rho, u = inputs.init_fields_torch(wc, dev)
    runs = {"f32_smag": ("f32", None, 0.0, 1), "f32_smag_perturbed": ("f32", None, 1e-7, 1),
            "bf16sr_mlp_every1": ("bf16sr", full, 0.0, 1),
            f"bf16sr_mlp_below{cut:g}h_every1": ("bf16sr", low, 0.0, 1),
            f"bf16sr_mlp_below{cut:g}h_every8": ("bf16sr", low, 0.0, 8),
            f"f32_mlp_below{cut:g}h_every1": ("f32", low, 0.0, 1),
            "f16s_mlp_every1": ("f16s", full, 0.0, 1),
            f"f16s_mlp_below{cut:g}h_every1": ("f16s", low, 0.0, 1)}
    res = {"workload": wc.name, "cut_y_over_h": cut, "steps": coarse_steps,
           "avg_from": avg_from, "runs": {}, "errors": {}, "profiles": {}}
    profs = {}
    for name, (st, b, eps, every) in runs.items():
        sim = make(wc, st, rho, u if eps == 0.0 else u * (1.0 + eps), b)
        if b is not None:
            sim.set_closure_interval(every)
        ms = timed_steps(sim, avg_from, torch, 5000, name)
        sim.stats_reset()
        sim.stats_enable(10)
        ms += timed_steps(sim, coarse_steps - avg_from, torch, 5000, name)
        prof, ns = sim.stats_read()
        d = sim.diag()
        sim.close()
        profs[name] = prof
        res["runs"][name] = {"MLUPS": wc.n * coarse_steps / ms / 1e3, "closure_every": every,
                             "fallback_fraction_last_eval": d["mlp_fallback"] / wc.n}
        res["profiles"][name] = {k: v.tolist() for k, v in profiles(prof).items()}
        _log(name, json.dumps(res["runs"][name]))
    for name in runs:
        if name != "f32_smag":
            res["errors"][name] = profile_errors(profs[name], profs["f32_smag"])
            _log("error vs f32_smag", name, json.dumps({k: round(v, 4)
                                                        for k, v in res["errors"][name].items()}))
    with open(os.path.join(out, "layer_study.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


# ---------------------------------------------------------------------------
# the paper's ABL over a homogeneous forest (Sec. 5), fine mesh
# ---------------------------------------------------------------------------

def abl_study(out, steps=20000, avg_from=10000):
    """LAD cases 1-3 of Table tab:forest_cases on 350x140x280: mean velocity
    profile over y/h, u_* at y/h = 2 (Sec. 5.1) and throughput."""
    import torch

    dev = torch.device("cuda")
    res = {"steps": steps, "avg_from": avg_from, "cases": {}}
    for w in (inputs.ABL1, inputs.ABL2, inputs.ABL3):
        rho, u = inputs.init_fields_torch(w, dev)
        sim = make(w, w.storage, rho, u)
        ms = timed_steps(sim, avg_from, torch, 5000, w.name)
        sim.stats_reset()
        sim.stats_enable(10)
        ms += timed_steps(sim, steps - avg_from, torch, 5000, w.name)
        prof, ns = sim.stats_read()
        d = sim.diag()
        sim.close()
        h = 7.0
        p = profiles(prof)
        ustar = friction_velocity(prof, 2 * h)
        res["cases"][w.name] = {"MLUPS": w.n * steps / ms / 1e3, "stat_samples": ns,
                                "max_u": d["max_u"], "u_star_2h": ustar,
                                "y_over_h": ((np.arange(w.ny) + 0.5) / h).tolist(),
                                "u_over_ustar": (p["u"] / ustar).tolist(),
                                "u_rms_over_ustar": (p["u_rms"] / ustar).tolist()}
        _log(w.name, json.dumps({k: res["cases"][w.name][k]
                                 for k in ("MLUPS", "u_star_2h", "max_u")}))
    with open(os.path.join(out, "abl_study.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


# ---------------------------------------------------------------------------
# the small oracle-size cases on the GPU
# ---------------------------------------------------------------------------

def small_cases(out, repeats=5):
    """GPU time of the 64x32x32 canopy case (200 steps) and the 128x64x64 crop
    (1000 steps) per storage type, median of the repeats: the same runs the
    oracle timing covers on the host."""
    import torch

    res = {}
    for w, steps in ((inputs.C1, 200), (inputs.CROP, 1000)):
        rho, u = inputs.init_fields(w)
        for st in ("f64", "f32", "bf16sr"):
            ms = []
            for _ in range(repeats):
                sim = make(w, st, rho, u)
                sim.step(10)
                torch.cuda.synchronize()
                ms.append(timed_steps(sim, steps, torch, steps))
                sim.close()
            m = float(np.median(ms))
            res[f"{w.name}/{st}"] = {"steps": steps, "ms": m, "MLUPS": w.n * steps / m / 1e3}
            _log(w.name, st, json.dumps(res[f"{w.name}/{st}"]))
    with open(os.path.join(out, "small_cases.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


def apriori_study(out, fine_steps=20000, batch=8192):
    """What the trained closure gains over the Smagorinsky closure a priori:
    both predict the filtered target nu_t of fresh samples (a new run of the
    canopy case at twice the resolution, box-filtered 2x2x2) from the same
    features.  Score: explained variance 1 - L / var(y/s) with the training
    loss L = mean((nu_t,pred - nu_t,target)^2) / s^2.  Smagorinsky (Sec. 2.2)
    needs only |P| = sqrt(tr P^2), P = Pi_neq / (rho c_s^2): X = 6 sqrt(2)
    C_s |P|, nu_t = X / (6 (sqrt(tau0^2 + X) + tau0)), the form of the step."""
    import torch

    dev = torch.device("cuda")
    wf, wc = inputs.C4, inputs.C2
    lad_c = _lad(wc)
    h_c = wc.lad_lalic[0]
    rho, u = inputs.init_fields_torch(wf, dev)
    fine = make(wf, "f32", rho, u)
    del rho, u
    ms = timed_steps(fine, fine_steps, torch, 2000, "fine")
    X, y = fine.closure_samples(wc.tau0, h_c, lad_c)
    fine.close()
    p, mean, std, lo, hi, s, _ = closure.read_blob(closure.trained_blob())
    ys = y.double() / s
    var = float(ys.var())
    # the network (its BF16 weights, the training forward pass)
    tr = lbm.Trainer(p, mean, std, s, max_batch=batch)
    n = (y.numel() // batch) * batch
    tot = 0.0
    for b in range(0, n, batch):
        tot += tr.step(X[b:b + batch], y[b:b + batch], update=False) * batch
    tr.close()
    l_net = tot / n
    # Smagorinsky from the same samples
    tau0, cs = wc.tau0, wc.c_smag
    xs = 6.0 * math.sqrt(2.0) * cs * X[:n, 5].double()
    nu_s = xs / (6.0 * (torch.sqrt(tau0 * tau0 + xs) + tau0))
    l_smag = float(((nu_s - y[:n].double()) / s).pow(2).mean())
    Xl = X[:n].double().cpu().numpy()
    inr = np.all((Xl >= lo) & (Xl <= hi), axis=1)
    res = {"fine": {"cells": wf.n, "steps": fine_steps, "MLUPS": wf.n * fine_steps / ms / 1e3},
           "samples": int(n), "target_mean": float(y.mean()), "target_variance_scaled": var,
           "in_training_range": float(inr.mean()),
           "network": {"loss": l_net, "explained_variance": 1.0 - l_net / var},
           "smagorinsky": {"loss": l_smag, "explained_variance": 1.0 - l_smag / var,
                           "mean_nu_t": float(nu_s.mean())}}
    _log("apriori", json.dumps(res))
    with open(os.path.join(out, "apriori_study.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


def aposteriori_pipeline(fine_steps=20000, tau0=0.5005, epochs=3, batch=8192, lr=1e-3,
                         storages=("f32", "bf16sr"), out=None):
    """The whole learned-closure pipeline at half the production size, and
    what the trained network gains a posteriori over the Smagorinsky closure
    of Sec. 2.2.  Coarse case: the production canopy set-up on 256x64x128
    cells (h = 6 cells, LAI 2, C_D = 0.15, u_tau = 0.01, g = u_tau^2 / ny,
    bounce-back ground, free-slip top); reference: the same physics at twice
    the resolution, 512x128x256 (h = 12, acoustic scaling: tau0_f = 1/2 +
    2 (tau0 - 1/2), g_f = g/2), FP32 + Smagorinsky, fine_steps steps with
    statistics over the second half (every 20 steps) and training samples at
    three snapshots of that half (2x2x2 box filter; 90/10 split by z slab).
    The network is trained on the GPU (Adam, `epochs` passes).  The coarse
    runs (fine_steps / 2 steps, statistics over the second half every 10
    steps) start from one seeded field, with each closure in each storage.
    Returns the profile errors of each coarse run against the box-filtered
    fine statistics, split at y/h = 4 (canopy layer and upper layer), and the
    x-z RMS density fluctuation per row at the end of each run, which shows
    the grid-scale mode that the BGK collision carries in the upper layer at
    this tau0 and Mach number."""
    import torch
    from dataclasses import replace

    dev = torch.device("cuda")
    ut = 0.01
    wc = replace(inputs.C2, name="canopy-abl-256x64x128", nx=256, ny=64, nz=128, tau0=tau0,
                 g=(ut ** 2 / 64, 0.0, 0.0), lad_lalic=(6.0, 4.2, 2.0), y_ref=64.0, seed=12)
    wf = replace(inputs.C2, name="canopy-abl-fine-512x128x256", nx=512, ny=128, nz=256,
                 tau0=0.5 + 2.0 * (tau0 - 0.5), g=(ut ** 2 / 64 / 2.0, 0.0, 0.0),
                 lad_lalic=(12.0, 8.4, 2.0), y_ref=128.0, seed=13)
    h_c = wc.lad_lalic[0]
    lad_c = _lad(wc)
    res = {"coarse": wc.name, "fine": wf.name, "u_tau": ut, "fine_steps": fine_steps}
    t0 = time.time()
    rho, u = inputs.init_fields_torch(wf, dev)
    fine = make(wf, "f32", rho, u)
    del rho, u
    half = fine_steps // 2
    fine.step(half)
    fine.stats_reset()
    fine.stats_enable(20)
    Xs, ys = [], []
    done = half
    for snap in (half + half // 3, half + 2 * half // 3, fine_steps):
        fine.step(snap - done)
        done = snap
        X, y = fine.closure_samples(wc.tau0, h_c, lad_c)
        Xs.append(X)
        ys.append(y)
    prof_f, _ = fine.stats_read()
    r, _, _, d = fine.moments()
    rho_rms_fine = 0.5 * (r.std(axis=(0, 2))[0::2] + r.std(axis=(0, 2))[1::2])
    fine.close()
    ref = coarsen_profile(prof_f)
    _log(f"fine run {time.time() - t0:.1f} s, max |u| {d['max_u']:.3f}")

    per = Xs[0].shape[0]
    cut = per * 9 // 10
    Xtr = torch.cat([x[:cut] for x in Xs]).cpu().numpy()
    ytr = torch.cat([y[:cut] for y in ys]).cpu().numpy()
    Xva = torch.cat([x[cut:] for x in Xs])
    yva = torch.cat([y[cut:] for y in ys])
    del Xs, ys
    mean = Xtr.mean(axis=0, dtype=np.float64)
    std = Xtr.std(axis=0, dtype=np.float64)
    std[std <= 0] = 1.0
    lo = Xtr.min(axis=0).astype(np.float64)
    hi = Xtr.max(axis=0).astype(np.float64)
    s = float(ytr.mean()) if ytr.mean() > 0 else 1e-5
    var = float(np.var(ytr / s))
    rng = np.random.default_rng(7)
    idx = rng.permutation(Xtr.shape[0])
    Xd = torch.from_numpy(np.ascontiguousarray(Xtr[idx])).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(ytr[idx])).to(dev)
    del Xtr, ytr
    p0 = closure.join(rng.normal(size=(64, 9)) / 3.0, np.zeros(64),
                      rng.normal(size=(64, 64)) / 8.0, np.zeros(64),
                      rng.normal(size=64) / 8.0, math.log(math.e - 1.0))
    tr = lbm.Trainer(p0, mean, std, s, lr=lr, max_batch=batch)
    nb = Xd.shape[0] // batch
    for _ in range(epochs):
        for b in range(nb):
            tr.step(Xd[b * batch:(b + 1) * batch], yd[b * batch:(b + 1) * batch], update=True,
                    loss=False)
    vls = [tr.step(Xva[b:b + batch], yva[b:b + batch], update=False)
           for b in range(0, yva.numel() - batch + 1, batch * 4)]
    p, _ = tr.get()
    tr.close()
    blob = closure.make_blob(p, mean, std, lo, hi, s, h_c)
    res["train"] = {"samples": int(Xd.shape[0]), "epochs": epochs, "target_mean": s,
                    "val_explained_variance": 1.0 - float(np.mean(vls)) / var}
    del Xd, yd, Xva, yva
    _log(f"trained {time.time() - t0:.1f} s: {res['train']}")

    yh = (np.arange(wc.ny) + 0.5) / h_c
    layers = {"canopy": yh <= 4.0, "upper": yh > 4.0}
    pr = profiles(ref)
    res["reference_rho_rms"] = rho_rms_fine.tolist()
    rho, u = inputs.init_fields_torch(wc, dev)
    cs = fine_steps // 2
    runs = {}
    for st in storages:
        for name, b in (("smag", None), ("mlp", blob)):
            sim = make(wc, st, rho, u, b)
            sim.step(cs // 2)
            sim.stats_reset()
            sim.stats_enable(10)
            sim.step(cs - cs // 2)
            prof, _ = sim.stats_read()
            r, _, _, d = sim.moments()
            sim.close()
            pa = profiles(prof)
            errs = {}
            for ln, m in layers.items():
                errs[ln] = {k: float(np.max(np.abs(pa[k][m] - pr[k][m])) / np.max(np.abs(pr[k])))
                            for k in ("u", "u_rms", "v_rms", "w_rms", "uv")}
            runs[f"{st}_{name}"] = {"errors_vs_filtered_fine": errs,
                                    "rho_rms": r.std(axis=(0, 2)).tolist(),
                                    "nu_t_mean": float(np.mean(pa["nu_t"])),
                                    "mlp_fallback": d["mlp_fallback"], "max_u": d["max_u"],
                                    "u": pa["u"].tolist()}
    res["runs"] = runs
    res["y_over_h"] = yh.tolist()
    _log(f"coarse runs {time.time() - t0:.1f} s")
    if out:
        with open(os.path.join(out, "aposteriori_pipeline.json"), "w") as f:
            json.dump(res, f, indent=1)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["closure", "precision", "interval", "abl", "small", "layer",
                                      "apriori", "aposteriori"])
    ap.add_argument("--out", default="studies_out")
    ap.add_argument("--fine-steps", type=int, default=40000)
    ap.add_argument("--coarse-steps", type=int, default=20000)
    ap.add_argument("--long-steps", type=int, default=20000)
    ap.add_argument("--avg-from", type=int, default=None,
                    help="first step of the statistics window (default: half the run)")
    args = ap.parse_args()
    import torch

    if not torch.cuda.is_available():
        sys.exit("the studies need a GPU")
    torch.cuda.set_device(0)
    os.makedirs(args.out, exist_ok=True)
    if args.study == "closure":
        f = args.fine_steps
        closure_study(args.out, fine_steps=f, snapshots=(f // 2, 3 * f // 4, f),
                      coarse_steps=args.coarse_steps, avg_from=args.coarse_steps // 2)
    elif args.study == "precision":
        precision_study(args.out, long_steps=args.long_steps, avg_from=args.long_steps // 2)
    elif args.study == "interval":
        interval_study(args.out, coarse_steps=args.coarse_steps,
                       avg_from=args.avg_from or args.coarse_steps // 2)
    elif args.study == "small":
        small_cases(args.out)
    elif args.study == "layer":
        layer_study(args.out, coarse_steps=args.coarse_steps,
                    avg_from=args.avg_from or args.coarse_steps // 2)
    elif args.study == "apriori":
        apriori_study(args.out, fine_steps=args.fine_steps // 2)
    elif args.study == "aposteriori":
        aposteriori_pipeline(fine_steps=args.fine_steps // 2, out=args.out)
    else:
        abl_study(args.out, steps=args.long_steps, avg_from=args.avg_from or args.long_steps // 2)


if __name__ == "__main__":
    main()
