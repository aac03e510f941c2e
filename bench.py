#!/usr/bin/env python3
"""Benchmark of the fused D3Q19 stream-collide path on one MI355X.

Workload: D3Q19 on the unit cube with 512 nodes per axis, full-way Dirichlet
walls on all six faces (data from four random cosines, seed 3),
u = (0.05, 0.1, 0.08), R = 1, tau = 1/2, third-order initialisation, fourth-order
walls.  One step is one time step of the whole lattice (bulk kernel + wall
kernel); `value` is the throughput of the float32-split storage mode (float32
g_k, float64 phi: the float32 storage that keeps the float64 discretisation
error, so the one that counts at fixed L2 error) in million lattice updates
per second with all state resident in HBM.  Plain float32 (`value_fp32`, whose
storage rounding exceeds the discretisation error), float64 and hi/lo (float32
arithmetic, phi as a float32 pair) are measured on the same workload for the
precision comparison.

The roofline entry is for the dominant kernel (the bulk stream-collide; it
advances two time steps per launch, keeping the intermediate state in LDS):
its algorithmic bytes per launch (per node of the (n-2)^2 rows off the y/z
walls: 2 q sizeof(float) plus 16 B of phi in the split modes, times the steps
per launch) divided by its
average duration from HIP events recorded around every launch on the
library's stream during the timed region.  Because the two-step kernel moves
fewer bytes than two single steps, the measured HBM traffic (from the
committed counter profile) is reported beside it, with the bandwidth of a plain
device copy measured in the same run.  The CPU baseline is the
float64 oracle on a bounded sample of the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "D3Q19 MLUPS & % HBM peak, FP32 vs FP64 at fixed L2 error; adjoint/fwd ratio"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_fused2_d3q19_512_{mode}_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2410_13165_amd", "csrc", f)
                  for f in ("kernels.hip", "kernels.hpp", "fuse.hpp", "engine.hpp",
                            "lattice.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(mode: str):
    """HBM bytes per bulk launch of one storage mode from the committed
    rocprofv3 counter summary, or None when it is missing or was taken on
    other kernel sources."""
    path = PROFILE_TRAFFIC.format(mode=mode)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def run_mode(precision: str, steps: int, warmup: int, n: int, scheme: str = "fullway", u=None,
             keep_phi: bool = False):
    """The benchmark workload in one storage mode; `scheme` / `u` switch to
    half-way walls (dx = 1/n, cell-centred nodes) and another velocity (the
    same four cosines, seed 3).  keep_phi: also return phi at the end (a float64
    device tensor) under "phi"."""
    import torch
    from paper_2410_13165_amd import Lattice, inputs
    w = inputs.BENCH_D3Q19
    u = list(w["u"]) if u is None else list(u)
    spec = inputs.bench_field() if u == list(w["u"]) else inputs.random_cosines(3, u, w["R"],
                                                                               w["seed"])
    dx = 1.0 / (n - 1) if scheme == "fullway" else 1.0 / n
    lat = Lattice(3, (n, n, n), 0.5, dx=dx, u=u, R=w["R"],
                  bc=[scheme] * 3, P=4, K=3, precision=precision, field=spec)
    try:
        info = lat.info()
        lat.step(warmup)
        torch.cuda.synchronize()
        lat.profile_begin(steps)
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = lat.profile_end()
        diag = lat.diagnostics()
        phi = lat.phi().clone() if keep_phi else None
    finally:
        lat.close()
        torch.cuda.empty_cache()
    seconds = t1 - t0
    nodes = n ** 3
    # the bulk kernel updates every row that is not on a y/z wall, x_1-face
    # nodes included: (n - 2)^2 rows of n nodes
    bulk_nodes = (n - 2) ** 2 * n
    q = info["q"]
    esize = 8 if precision == "fp64" else 4
    bulk_bytes_step = bulk_nodes * 2 * q * esize + (
        bulk_nodes * 16 if precision in ("fp32_split", "fp32_hilo") else 0)
    # a bulk launch covers steps_per_launch time steps (two when the lattice
    # advances in fused pairs); its algorithmic bytes are those of its steps
    steps_per_launch = prof["steps"] / prof["launches"]
    bulk_bytes = bulk_bytes_step * steps_per_launch
    bulk_s = prof["bulk_ms"] / prof["launches"] / 1e3
    wall_s = prof["wall_ms"] / prof["steps"] / 1e3
    return {
        "precision": precision,
        "mlups": nodes * steps / seconds / 1e6,
        "ms_per_step": seconds / steps * 1e3,
        "seconds": seconds,
        "bytes_per_lu": info["bytes_per_lu"],
        "hbm_frac_step": nodes * steps * info["bytes_per_lu"] / seconds / (HBM_PEAK_GBS * 1e9),
        "steps_per_launch": steps_per_launch,
        "bulk_ms": bulk_s * 1e3,
        "wall_ms": wall_s * 1e3,
        "bulk_bytes_per_launch": bulk_bytes,
        "bulk_gbs": bulk_bytes / bulk_s / 1e9,
        "rmse": diag["rmse"],
        "t_final": diag["t"],
        "nonfinite": diag["nonfinite"],
        "phi": phi,
    }


def run_adjoint(precision: str = "fp32", n=None, steps=None):
    """Forward with checkpoint tape, then the adjoint gradient (dL/dphi0 and
    dL/dtau) on the gradient workload; returns the backward / forward time ratio."""
    import numpy as np
    import torch
    from paper_2410_13165_amd import Lattice, inputs
    w = inputs.ADJOINT_D3Q19
    n = n or w["n"]
    steps = steps or w["steps"]
    dx = 1.0 / n
    phi0 = torch.from_numpy(inputs.gaussian_random_field(n, 3, w["seed_init"], w["corr"]).ravel())
    tgt = torch.from_numpy(inputs.gaussian_random_field(n, 3, w["seed_target"], w["corr"]))
    lat = Lattice(3, (n, n, n), 0.5, dx=dx, u=w["u"], precision=precision)
    try:
        # one untimed forward + gradient first: the checkpoints and the
        # segment states then come from the caching allocator, as in every
        # iteration of an optimisation loop after the first
        lat.set_initial(phi0)
        lat.tape_begin(w["every"])
        lat.step(steps)
        phiN = lat.phi()
        t_w0 = time.perf_counter()
        lat.tape_gradient((phiN - tgt.to(phiN.device)) * dx ** 3, want_phi0=True, want_tau=True)
        torch.cuda.synchronize()
        cold_backward = time.perf_counter() - t_w0
        lat.tape_end()
        lat.set_initial(phi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.tape_begin(w["every"])
        lat.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        phiN = lat.phi()
        seed = (phiN - tgt.to(phiN.device)) * dx ** 3
        loss = 0.5 * float((phiN - tgt.to(phiN.device)).pow(2).sum()) * dx ** 3
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g = lat.tape_gradient(seed, want_phi0=True, want_tau=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g2 = lat.tape_gradient(seed, want_phi0=True, want_tau=False)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        gnorm = float(g["phi0"].norm())
        lat.tape_end()
        # the same forward without recording checkpoints
        lat.set_initial(phi0)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        t6 = time.perf_counter()
    finally:
        lat.close()
        torch.cuda.empty_cache()
    fwd = t1 - t0
    return {
        "forward_untaped_s": t6 - t5,
        "ratio_vs_untaped_forward": (t3 - t2) / (t6 - t5),
        "workload": (f"D3Q19 {n}^3 periodic, {precision}, {steps} steps, checkpoints every "
                     f"{w['every']}, Gaussian random fields (corr {w['corr']})"),
        "forward_s": fwd,
        "backward_s": t3 - t2,
        "ratio": (t3 - t2) / fwd,
        "backward_phi0_only_s": t4 - t3,
        "ratio_phi0_only": (t4 - t3) / fwd,
        "backward_first_call_s": cold_backward,
        "loss": loss,
        "dL_dtau": g["tau"],
        "grad_phi0_norm": gnorm,
    }


def run_fixed_error(target=1e-6, sizes=(64, 96, 128, 192, 256, 384, 512)):
    """Smallest grid of the benchmark family (D3Q19 full-way, same field, final
    time t = 2000/511) whose RMSE relative to the RMS of phi reaches `target`,
    per storage mode, and the time to solution there (one timed run per size,
    no warm-up, so the small sizes include launch overhead)."""
    import torch
    from paper_2410_13165_amd import Lattice, inputs
    w = inputs.BENCH_D3Q19
    T = w["steps"] / (w["n"] - 1)
    spec = inputs.bench_field()
    out = {}
    for mode in ("fp64", "fp32_split", "fp32_hilo", "fp32"):
        tried = []
        hit = None
        for n in sizes:
            steps = int(round(T * (n - 1)))
            lat = Lattice(3, (n, n, n), 0.5, dx=1.0 / (n - 1), u=w["u"], R=w["R"],
                          bc=["fullway"] * 3, precision=mode, field=spec)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lat.step(steps)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                dg = lat.diagnostics()
            finally:
                lat.close()
                torch.cuda.empty_cache()
            rmse = dg["rmse"]
            rel = rmse / math.sqrt(dg["sum_phi2"] / n ** 3)
            rec = {"n": n, "steps": steps, "rmse": float(f"{rmse:.4g}"),
                   "rel_rmse": float(f"{rel:.4g}"), "seconds": round(sec, 4),
                   "mlups": round(n ** 3 * steps / sec / 1e6, 1)}
            tried.append(rec)
            print(f"# fixed error {mode}: n={n} rmse={rmse:.3e} relative {rel:.3e} {sec:.3f} s",
                  file=sys.stderr, flush=True)
            if rel <= target:
                hit = rec
                break
        out[mode] = {"reached": hit, "runs": tried}
    return {"target_rmse": target, "t_final": T, "modes": out}


def run_d2q9(n=2048):
    """D2Q9 periodic plane wave phi0 = sin(2 pi x) sin(2 pi y), u = (0.1, 0.2),
    tau = 1/2, n^2 nodes, n steps (t = 1): MLUPS with two steps per bulk pass and
    with one, and the RMSE against the transported exact solution."""
    import torch
    from paper_2410_13165_amd import Lattice, inputs
    spec = inputs.plane_sine(2, [0.1, 0.2])
    out = {"workload": f"D2Q9 {n}^2 periodic, sin(2 pi x) sin(2 pi y), u=(0.1,0.2), {n} steps"}
    for prec in ("fp64", "fp32"):
        for spp in (2, 1):
            lat = Lattice(2, (n, n), 0.5, dx=1.0 / n, u=spec["u"], precision=prec, field=spec,
                          steps_per_pass=spp)
            try:
                lat.step(4)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lat.step(n)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                rmse = lat.diagnostics()["rmse"]
            finally:
                lat.close()
                torch.cuda.empty_cache()
            out[f"{prec}_pass{spp}"] = {"mlups": round(n * n * n / sec / 1e6, 1),
                                        "rmse": float(f"{rmse:.4g}")}
            print(f"# d2q9 {prec} steps/pass {spp}: {n * n * n / sec / 1e6:.0f} MLUPS, "
                  f"rmse {rmse:.3e}", file=sys.stderr, flush=True)
    return out


def run_d4q33(n=96, steps=32):
    """Example 3 (Sec. 5) at benchmark size: D4Q33, phi* = sin[pi (sum_i x_i - u_i t)]
    on [-1, 1]^4 with u = (0.05, 0.2, 0.08, 0.1), tau = 1/2, K = 3, n^4 nodes,
    periodic and full-way (P = 4), float32 and float64, one step per pass.
    Reports MLUPS, the bulk kernel's mean launch time (HIP events) and its
    algorithmic rate, 2 q sizeof(T) bytes per node and step over the rows off
    the walls of x_2..x_4, and the RMSE against the exact solution."""
    import torch
    from paper_2410_13165_amd import Lattice, inputs
    u = [0.05, 0.2, 0.08, 0.1]
    spec = inputs.diagonal_sine(4, u)
    out = {"workload": (f"D4Q33 {n}^4, Example 3 field sin(pi (sum x_i - u_i t)) on [-1,1]^4, "
                        f"u=(0.05,0.2,0.08,0.1), tau=1/2, K=3, P=4, {steps} steps")}
    for bc in ("periodic", "fullway"):
        dx = 2.0 / n if bc == "periodic" else 2.0 / (n - 1)
        bulk_nodes = n ** 4 if bc == "periodic" else (n - 2) ** 3 * n
        for prec in ("fp32", "fp64"):
            lat = Lattice(4, (n,) * 4, 0.5, dx=dx, u=u, origin=[-1.0] * 4, bc=[bc] * 4, P=4,
                          K=3, precision=prec, field=spec)
            try:
                q = lat.info()["q"]
                lat.step(4)
                torch.cuda.synchronize()
                lat.profile_begin(steps)
                t0 = time.perf_counter()
                lat.step(steps)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                prof = lat.profile_end()
                rmse = lat.diagnostics()["rmse"]
            finally:
                lat.close()
                torch.cuda.empty_cache()
            esize = 8 if prec == "fp64" else 4
            bulk_s = prof["bulk_ms"] / prof["launches"] / 1e3
            bulk_bytes = bulk_nodes * 2 * q * esize * prof["steps"] / prof["launches"]
            rec = {"mlups": round(n ** 4 * steps / sec / 1e6, 1),
                   "steps_per_launch": prof["steps"] / prof["launches"],
                   "bulk_ms": round(bulk_s * 1e3, 4),
                   "bulk_gbs": round(bulk_bytes / bulk_s / 1e9, 1),
                   "bulk_frac": round(bulk_bytes / bulk_s / 1e9 / HBM_PEAK_GBS, 4),
                   "rmse": float(f"{rmse:.4g}")}
            out[f"{bc}_{prec}"] = rec
            print(f"# d4q33 {bc} {prec}: {rec['mlups']:.0f} MLUPS, bulk {rec['bulk_gbs']:.0f} GB/s"
                  f", rmse {rmse:.3e}", file=sys.stderr, flush=True)
    return out


def run_d2q9_convergence(sizes=(64, 128, 256, 512, 1024, 2048)):
    """The grid-refinement study of the D2Q9 plane wave: phi0 = sin(2 pi x)
    sin(2 pi y), u = (0.1, 0.2), periodic unit square, n^2 nodes and n steps
    (t = 1), per storage mode at tau = 1/2, plus float64 at one tau drawn from
    U[0.6, 1.5] (seed 2); RMSE against the transported exact solution and the
    observed order log2(e_n / e_2n) per grid."""
    import numpy as np
    import torch
    from paper_2410_13165_amd import Lattice, inputs
    spec = inputs.plane_sine(2, [0.1, 0.2])
    tau_draw = float(np.random.default_rng(2).uniform(0.6, 1.5))
    cases = [("fp64", 0.5), ("fp32", 0.5), ("fp32_split", 0.5), ("fp64", tau_draw)]
    out = {"workload": "D2Q9 periodic plane wave sin(2 pi x) sin(2 pi y), u=(0.1,0.2), "
                       "n^2 nodes, n steps (t = 1)", "cases": []}
    for prec, tau in cases:
        runs = []
        for n in sizes:
            lat = Lattice(2, (n, n), tau, dx=1.0 / n, u=spec["u"], precision=prec, field=spec)
            try:
                lat.step(n)
                rmse = lat.diagnostics()["rmse"]
            finally:
                lat.close()
                torch.cuda.empty_cache()
            order = math.log2(runs[-1]["rmse"] / rmse) if runs and rmse > 0 else None
            runs.append({"n": n, "rmse": float(f"{rmse:.5g}"),
                         "order": round(order, 3) if order is not None else None})
        print(f"# d2q9 convergence {prec} tau={tau:.4f}: " +
              " ".join(f"{r['n']}:{r['rmse']:.3e}" + (f"({r['order']:.2f})" if r["order"] else "")
                       for r in runs), file=sys.stderr, flush=True)
        out["cases"].append({"precision": prec, "tau": tau, "runs": runs})
    # crossover N*: the smallest grid at which a storage mode's error exceeds
    # the float64 (discretisation) error of the same grid by 10%
    ref = {r["n"]: r["rmse"] for r in out["cases"][0]["runs"]}
    out["crossover_n"] = {}
    for c in out["cases"][1:3]:
        hit = [r["n"] for r in c["runs"] if r["rmse"] > 1.1 * ref[r["n"]]]
        out["crossover_n"][c["precision"]] = hit[0] if hit else None
    return out


def run_sweep(steps=None, count=None, precision="fp32"):
    """512 independent D2Q9 lattices advanced together (tuned launch form);
    per-instance growth of the L2 norm of phi."""
    import numpy as np
    import torch
    from paper_2410_13165_amd import Batch, inputs
    w = inputs.SWEEP_D2Q9
    steps = steps or w["steps"]
    specs = inputs.sweep_specs(count)
    phi0 = torch.from_numpy(inputs.sweep_phi0(specs))
    nodes = sum(int(np.prod(sp["dims"])) for sp in specs)
    print(f"# sweep: {len(specs)} lattices, {nodes} nodes", file=sys.stderr, flush=True)
    with Batch(2, specs, precision=precision) as b:
        b.set_initial(phi0)
        print("# sweep: initialised", file=sys.stderr, flush=True)
        cfg = b.tune(10)
        print(f"# sweep: tuned {cfg}", file=sys.stderr, flush=True)
        m0 = b.moments()
        torch.cuda.synchronize()
        # sum phi^2 after every chunk gives the late-time growth rates; those
        # readouts sit between timed chunks, outside the timed work
        marks = [(0, m0[:, 1])]
        elapsed = 0.0
        done = 0
        chunk = 500
        while done < steps:
            todo = min(chunk, steps - done)
            t0 = time.perf_counter()
            b.step(todo)
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            done += todo
            marks.append((done, b.moments()[:, 1]))
            print(f"# sweep: {done} steps", file=sys.stderr, flush=True)
        m1 = b.moments()
        min_om = np.array([b.instance(i).info()["min_omega"] for i in range(len(specs))])
    taus = np.array([sp["tau"] for sp in specs])
    growth = np.sqrt(m1[:, 1] / m0[:, 1])
    finite = np.isfinite(growth)
    pred = sweep_prediction(specs, growth, m0[:, 3], m1[:, 3], min_om, steps,
                            late_rate=late_growth_rates(marks))
    return {
        "workload": (f"{len(specs)} periodic D2Q9 lattices (sizes 64^2..512^2), {precision}, "
                     f"{steps} steps, tau~U(0.5,2), sigma~U(-0.75,0.75)^2, noise init"),
        "nodes": nodes,
        "seconds": elapsed,
        "mlups": nodes * steps / elapsed / 1e6,
        "config": cfg,
        "grew_1e3": int(np.sum(~finite | (growth > 1e3))),
        "bounded": int(np.sum(finite & (growth <= 1.0 + 1e-6))),
        "entropy_stable_instances": int(np.sum(min_om > 0)),
        "prediction": pred,
    }


def late_growth_rates(marks):
    """Per instance, log of the growth of ||phi|| per step over the second half
    of its readable run: marks is a list of (step, sum phi^2 per instance); an
    instance whose norm overflowed is read up to its last finite readout S_e,
    from the readout nearest S_e / 2 (NaN where fewer than two readouts apart)."""
    import numpy as np
    steps = np.array([m[0] for m in marks])
    ss = np.stack([m[1] for m in marks])  # (readouts, instances)
    ok = np.isfinite(ss) & (ss > 0)
    rate = np.full(ss.shape[1], np.nan)
    for i in range(ss.shape[1]):
        good = np.nonzero(ok[:, i])[0]
        if good.size < 2:
            continue
        e = good[-1]
        b = good[np.argmin(np.abs(steps[good] - steps[e] / 2))]
        if b >= e:
            b = good[-2]
        rate[i] = 0.5 * np.log(ss[e, i] / ss[b, i]) / (steps[e] - steps[b])
    return rate


def sweep_prediction(specs, growth, ent0, ent1, min_om, steps, late_rate=None):
    """Per instance, the growth of ||phi|| and of the total entropy over the run
    against what the parameters predict: the largest spectral radius of the
    amplification matrix over the instance's wave numbers (a grid of
    min(n, 256)^2 of them, a subset of the instance's own when n > 256),
    computed on the GPU by lbm_stability_map, and the entropy criterion
    min omega > 0 (Prop. 1).

    The rate log(growth)/steps over the whole run carries log c / steps, where
    c is the share of the noise initial data in the fastest-growing modes (about
    1/n for n^2 modes).  late_rate (late_growth_rates) starts where those modes
    already dominate and also covers instances whose norm overflowed before the
    end, so it is compared with log rho as well (growth_rate_late_*)."""
    import numpy as np
    import torch
    from paper_2410_13165_amd import lbm
    count = len(specs)
    rho = np.zeros(count)
    for m in sorted({min(sp["dims"][0], 256) for sp in specs}):
        idx = [i for i, sp in enumerate(specs) if min(sp["dims"][0], 256) == m]
        sig = np.array([specs[i]["u"] for i in idx], dtype=np.float64)
        s = np.array([1.0 / specs[i]["tau"] for i in idx], dtype=np.float64)
        out = lbm.stability_map(sig, s, m=m)
        rho[idx] = out["rho"].cpu().numpy()
        torch.cuda.synchronize()
    unstable = rho > 1.0 + 1e-9
    finite = np.isfinite(growth)
    grew = ~finite | (growth > 1.0 + 1e-6)
    rate = np.where(finite & (growth > 0), np.log(np.where(finite & (growth > 0), growth, 1.0)) / steps,
                    np.inf)
    logrho = np.log(np.maximum(rho, 1e-300))
    # growing instances: the measured rate log(growth)/steps tends to log rho
    sel = unstable & grew & finite
    rel_rate = np.abs(rate[sel] - logrho[sel]) / logrho[sel] if np.any(sel) else np.zeros(0)
    late = {}
    if late_rate is not None:
        sel_l = unstable & grew & np.isfinite(late_rate)
        rel_l = (np.abs(late_rate[sel_l] - logrho[sel_l]) / logrho[sel_l]
                 if np.any(sel_l) else np.zeros(0))
        late = {
            "growth_rate_instances": int(sel.sum()),
            "growth_rate_late_instances": int(sel_l.sum()),
            "growth_rate_late_rel_err_median": float(np.median(rel_l)) if rel_l.size else None,
            "growth_rate_late_rel_err_max": float(np.max(rel_l)) if rel_l.size else None,
        }
    ent_ratio = ent1 / ent0
    pos = min_om > 0
    return {
        "predicted_unstable": int(unstable.sum()),
        "grew": int(grew.sum()),
        "agree": int(np.sum(unstable == grew)),
        "unstable_not_grown": int(np.sum(unstable & ~grew)),
        "grown_not_unstable": int(np.sum(~unstable & grew)),
        "growth_rate_rel_err_median": float(np.median(rel_rate)) if rel_rate.size else None,
        "growth_rate_rel_err_max": float(np.max(rel_rate)) if rel_rate.size else None,
        "min_omega_positive": int(pos.sum()),
        "entropy_grew_where_min_omega_positive": int(np.sum(pos & ~(ent_ratio <= 1.0 + 1e-9))),
        "rho_max": float(np.max(rho)),
        **late,
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(n_sample: int, steps: int):
    """The FP64 oracle on a bounded sample: a cube of n_sample^3 nodes with the
    benchmark's spacing, field and walls, for `steps` steps."""
    from oracle import lbm_oracle as O
    from paper_2410_13165_amd import inputs
    from tests.pairs import oracle_problem
    w = inputs.BENCH_D3Q19
    spec = inputs.bench_field()
    prob = oracle_problem(3, (n_sample,) * 3, 1.0 / (w["n"] - 1), spec, bc=["fullway"] * 3)
    run = O.Run(prob)
    t0 = time.perf_counter()
    run.step(steps)
    dt = time.perf_counter() - t0
    return {
        "value": n_sample ** 3 * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"D3Q19 full-way, {n_sample}^3 nodes at dx=1/{w['n'] - 1}, same field, "
                   f"{steps} steps, {dt:.1f} s, numpy float64 single thread; host: "
                   f"{cpu_model()}, {os.cpu_count()} logical CPUs"),
    }


def measure_copy_gbs(gib: float = 2.0, reps: int = 10) -> float:
    """Bandwidth of a plain device-to-device copy (torch's copy kernel) of `gib`
    GiB: bytes read plus bytes written per launch over the mean duration."""
    import torch
    nbytes = int(gib * (1 << 30))
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / sec / 1e9


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="nodes per axis")
    ap.add_argument("--modes", default="fp32_split,fp32,fp64,fp32_hilo",
                    help="storage modes; the first one gives `value`")
    ap.add_argument("--cpu-nodes", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-fixed-error", action="store_true")
    ap.add_argument("--no-d2q9", action="store_true")
    ap.add_argument("--no-d4q33", action="store_true")
    ap.add_argument("--no-halfway", action="store_true")
    ap.add_argument("--halfway-steps", type=int, default=200)
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          f"--gpus {args.gpus} is not supported"}), flush=True)
        return 2

    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)

    if args.calib_copy_gib > 0:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
        # give the scale between the counters and bytes
        nbytes = int(args.calib_copy_gib * (1 << 30))
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"# calibration copy: {nbytes} bytes read and written per launch", file=sys.stderr)
        del a, b
        torch.cuda.empty_cache()

    # (not in counter-calibration runs, whose only large copies must be the
    # calibration copies)
    copy_gbs = measure_copy_gbs() if args.calib_copy_gib <= 0 else None
    ceiling = None
    if copy_gbs:
        from paper_2410_13165_amd import lbm
        ceiling = {k: round(v, 1) for k, v in lbm.stream_ceiling().items()}
        print(f"# device copy (torch): {copy_gbs:.0f} GB/s; float4 probes {ceiling}",
              file=sys.stderr, flush=True)

    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    results = {}
    phis = {}
    for m in modes:
        results[m] = run_mode(m, args.steps, args.warmup, args.n, keep_phi=True)
        phis[m] = results[m].pop("phi")
        print(f"# {m}: {results[m]['mlups']:.0f} MLUPS, bulk {results[m]['bulk_gbs']:.0f} GB/s, "
              f"rmse {results[m]['rmse']:.3e}", file=sys.stderr, flush=True)
    # per-run precision: each reduced-precision mode against the float64 run of
    # the same workload and step count, and the discretisation error of that run
    precision = None
    if "fp64" in phis:
        ref = phis["fp64"]
        ref_norm = float(ref.norm())
        disc = results["fp64"]["rmse"] * math.sqrt(args.n ** 3) / ref_norm
        precision = {"steps": args.steps, "fp64_rel_discretisation_error": float(f"{disc:.4g}"),
                     "drift_vs_fp64": {}, "below_discretisation_error": {}}
        for m, ph in phis.items():
            if m == "fp64":
                continue
            drift = float((ph - ref).norm()) / ref_norm
            precision["drift_vs_fp64"][m] = float(f"{drift:.4g}")
            precision["below_discretisation_error"][m] = bool(drift < disc)
    del phis
    torch.cuda.empty_cache()
    for m in modes:
        tr = committed_traffic(m)
        r = results[m]
        r["traffic_bytes_per_launch"] = tr
        r["phys_gbs"] = tr / (r["bulk_ms"] / 1e3) / 1e9 if tr else None
        r["phys_frac"] = r["phys_gbs"] / HBM_PEAK_GBS if tr else None
    head = results[modes[0]]
    fixed = None
    if not args.no_fixed_error:
        fixed = run_fixed_error()
    halfway = None
    if not args.no_halfway:
        # half-way walls diverge at the benchmark's u (Table 1's pattern), so
        # they are timed at u = 1e-3 in every component
        halfway = {"workload": (f"D3Q19 {args.n}^3 half-way Dirichlet on all faces, same "
                                "cosines, u=(1e-3,1e-3,1e-3), R=1, tau=1/2, K=3, P=4, "
                                f"{args.halfway_steps} steps")}
        for m in ("fp32", "fp64", "fp32_split"):
            r = run_mode(m, args.halfway_steps, 4, args.n, scheme="halfway", u=[1e-3] * 3)
            halfway[m] = {"mlups": round(r["mlups"], 1), "bulk_gbs": round(r["bulk_gbs"], 1),
                          "steps_per_launch": r["steps_per_launch"],
                          "rmse": float(f"{r['rmse']:.4g}")}
            print(f"# halfway {m}: {r['mlups']:.0f} MLUPS, bulk {r['bulk_gbs']:.0f} GB/s, "
                  f"rmse {r['rmse']:.3e}", file=sys.stderr, flush=True)
    d2q9 = None if args.no_d2q9 else run_d2q9()
    conv = None if args.no_d2q9 else run_d2q9_convergence()
    d4q33 = None if args.no_d4q33 else run_d4q33()
    sweep = None
    if not args.no_sweep:
        sweep = run_sweep()
        print(f"# sweep: {sweep['mlups']:.0f} MLUPS, config {sweep['config']}", file=sys.stderr,
              flush=True)
    adj = None
    adj32 = None
    if not args.no_adjoint:
        # the gradient workload is specified with split storage; plain float32 beside it
        adj = run_adjoint("fp32_split")
        adj32 = run_adjoint("fp32")
        for name, a in (("fp32_split", adj), ("fp32", adj32)):
            print(f"# adjoint {name}: forward {a['forward_s']:.3f} s, backward "
                  f"{a['backward_s']:.3f} s, ratio {a['ratio']:.3f}", file=sys.stderr, flush=True)

    traffic = head["traffic_bytes_per_launch"]
    kname = {"fp32": "k_fused2<float, false>", "fp64": "k_fused2<double, false>",
             "fp32_split": "k_fused2_split<false, false>",
             "fp32_hilo": "k_fused2_split<false, true>"}[modes[0]]
    if head["steps_per_launch"] == 2:
        kernel = f"{kname} (two stream-collide steps per pass)"
    else:
        kernel = f"k_step<3,{'float' if modes[0] != 'fp64' else 'double'}> (bulk stream-collide)"
    roofline = {
        "bound": "hbm",
        "achieved": round(head["bulk_gbs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(head["bulk_gbs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": kernel,
        "steps_per_launch": head["steps_per_launch"],
        "bytes_per_launch": head["bulk_bytes_per_launch"],
        "avg_launch_ms": round(head["bulk_ms"], 4),
    }
    # a plain device copy measured in the same process, for scale
    roofline["copy_gbs_measured"] = round(copy_gbs, 1) if copy_gbs else None
    roofline["stream_ceiling_gbs"] = ceiling
    if traffic:
        # measured HBM bytes per launch (committed counters) over the same
        # duration: the physical rate, against the peak and the float4 copy
        roofline["hbm_gbs_measured"] = round(head["phys_gbs"], 1)
        roofline["phys_frac"] = round(head["phys_frac"], 4)
        if ceiling:
            roofline["phys_frac_of_copy_ceiling"] = round(head["phys_gbs"] / ceiling["copy"], 4)
    else:
        roofline["phys_frac"] = None
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_nodes, args.cpu_steps)

    dtype = {"fp32": "f32", "fp64": "f64", "fp32_split": "f32+f64", "fp32_hilo": "f32"}[modes[0]]
    line = {
        "metric": METRIC,
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"D3Q19 {args.n}^3 full-way Dirichlet on all faces, 4 random cosines "
                         "(seed 3), u=(0.05,0.1,0.08), R=1, tau=1/2, K=3, P=4, "
                         f"{modes[0]} storage"),
            "nodes": args.n ** 3,
            "global_batch": 1,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_frac_step": round(head["hbm_frac_step"], 4),
        "value_fp32": round(results["fp32"]["mlups"], 1) if "fp32" in results else None,
        "value_fp32_split": round(results["fp32_split"]["mlups"], 1) if "fp32_split" in results
        else None,
        "value_fp32_hilo": round(results["fp32_hilo"]["mlups"], 1) if "fp32_hilo" in results
        else None,
        "value_fp64": round(results["fp64"]["mlups"], 1) if "fp64" in results else None,
        "precision": precision,
        "modes": {m: {k: (float(f"{v:.6g}") if isinstance(v, float) else v)
                      for k, v in r.items()}
                  for m, r in results.items()},
        "fixed_error": fixed,
        "halfway": halfway,
        "d2q9": d2q9,
        "d2q9_convergence": conv,
        "d4q33": d4q33,
        "sweep": sweep,
        "adjoint_fwd_ratio": round(adj["ratio"], 4) if adj else None,
        "adjoint": ({k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in adj.items()}
                    if adj else None),
        "adjoint_fp32": ({k: (float(f"{v:.6g}") if isinstance(v, float) else v)
                          for k, v in adj32.items()} if adj32 else None),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
