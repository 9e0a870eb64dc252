"""Benchmark: H|psi> band-applies/s and embedding-cycle time on one MI355X.

Workload (default): the slab + molecule cell -- 10.2 x 10.2 x 40 bohr,
60 x 60 x 240 grid, E_cut = 40 Ha (about 50 300 plane waves per k); slab of
36 Gaussian ions with one s projector each, 40 bands, 4 Monkhorst-Pack
k-points, Fermi-Dirac 0.01 Ha; a 6-atom molecule at Gamma with 8 bands.
Synthetic seeded inputs of that shape (the paper's systems need
pseudopotential files that are not available).

A step is one embedding cycle: embedding potential of both subsystems, per
subsystem and k-point one H application + Rayleigh-Ritz then 4 Davidson
iterations (preconditioner, H application, Rayleigh-Ritz), occupations,
densities and mixing. `value` is band-applies per cycle / cycle time.

The roofline object covers one H application (stick inverse FFT, plane pass
with V_eff, stick forward FFT + kinetic term, Kleinman-Bylander projector
products and update), timed with HIP events on the stream the kernels run on,
over an isolated resident batch of all 40 slab bands at one k-point with the
slab's 36 projectors. Algorithmic bytes per call (complex of `cs` bytes, V_eff
real of `rs` bytes; V_eff and the projectors counted once per call, whatever the
launch shape re-reads):
    nb * (3*cs*npw + 4*cs*ncol*N3) + rs*N + nproj*cs*npw.

`--workload 64-subsystems` times the cycle of the 20 bohr cube holding 64 uneven
subsystems (72^3 grid, E_cut 15 Ha, 4-128 bands and 1-8 k-points each) instead;
that line is context, without CPU baseline or counter traffic.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of the kernels one fde_apply_h call runs (the counter summary is tied to them)
APPLY_SOURCES = ["common.hpp", "kernels_gemm.hpp", "kernels_plane.hpp", "kernels_pw.hpp", "pw.hip"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-bands", type=int, default=40)
    ap.add_argument("--also-fp64", action="store_true", help="also time the FP64 cycle")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-1e-6 Ha comparison")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--streams", type=int, default=3, help="concurrent band-solver groups")
    ap.add_argument("--gemm", choices=["fp64", "bf16x3", "bf16x6"], default="fp64",
                    help="arithmetic of the Rayleigh-Ritz subspace products (FP32 plan)")
    ap.add_argument("--workload", choices=["slab-molecule", "64-subsystems"], default="slab-molecule",
                    help="slab + molecule cell (the benchmark line) or the cube of 64 uneven subsystems "
                         "(timed for context: no CPU baseline, no counter traffic)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only time a plain device-to-device copy of MIB MiB (stream bandwidth and "
                         "the calibration of the HBM byte counters), then exit")
    return ap.parse_args()


def copy_probe(mib, reps=10):
    """Plain device copy of a known size: attainable stream bandwidth."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps + 1,
            "copy_GBps": 2 * 4 * n / t / 1e9}


def apply_bytes(plan, ik, nb, nproj):
    cs = 16 if plan.prec == 0 else 8
    rs = cs // 2
    N1, N2, N3 = plan.grid
    npw, ncol = plan.npw(ik), plan.ncol(ik)
    per_band = 3 * cs * npw + 4 * cs * ncol * N3
    return per_band * nb + rs * N1 * N2 * N3 + cs * npw * nproj


def measured_traffic():
    """HBM bytes per fde_apply_h call from the committed counter summary, or None
    when the sources of its kernels changed since the counters were taken."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "apply_h_slab_molecule_60x60x240.traffic.txt")
    if not os.path.exists(f):
        return None
    kv = dict(line.split()[:2] for line in open(f) if line.strip() and not line.startswith("#"))
    h = hashlib.sha256()
    for src in sorted(os.path.join(ROOT, "paper_1406_7803_amd", "csrc", n) for n in APPLY_SOURCES):
        h.update(os.path.basename(src).encode())
        h.update(open(src, "rb").read())
    if h.hexdigest() != kv.get("sources_sha256"):
        return None
    return float(kv["traffic_bytes_per_call"])


def time_cycles(eng, steps, warmup, graph=False):
    """Time `steps` cycles (eager launches, or replays of one captured HIP graph)."""
    import torch
    for _ in range(warmup):
        eng.cycle()
    if graph:
        eng.capture()
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    t0 = time.perf_counter()
    for k in range(steps):
        if graph:
            eng.replay()
        else:
            eng.cycle()
        print(f"# cycle {k + 1}/{steps} enqueued", file=sys.stderr, flush=True)
    s1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return s0.elapsed_time(s1) / 1e3, wall


def time_to_accuracy(be, max_cycles=300):
    """Wall time until the two-subsystem cube's occupied eigenvalues are within 1e-6 Ha
    and every subsystem density within 1e-5 (integrated |drho|) of the converged FP64
    result, per precision mode (engine set-up excluded; each cycle is followed by the
    same device-to-host check in every mode)."""
    import numpy as np
    import torch

    import fde_synth
    from paper_1406_7803_amd import driver, fde

    s = fde_synth.config1()
    dv = float(np.prod(s.L)) / float(np.prod(s.grid))

    def state(e):
        torch.cuda.synchronize()
        return [x.double().cpu().numpy().copy() for x in e.eps], e.rho_out.double().cpu().numpy().copy()

    ref = driver.Engine(s, prec=fde.F64, backend=be)
    prev = None
    for c in range(max_cycles):
        ref.cycle()
        eps, rho = state(ref)
        if prev is not None and max(np.max(np.abs(a - b)) for a, b in zip(eps, prev[0])) < 1e-11 \
                and np.sum(np.abs(rho - prev[1])) * dv < 1e-10:
            break
        prev = (eps, rho)
    ref_cycles = c + 1
    occ = [o.cpu().numpy() > 1e-8 for o in ref.occw]
    out = {"system": "two-subsystem 10 bohr cube, 24^3, E_cut 7 Ha", "reference": f"FP64, {ref_cycles} cycles"}
    for name, prec, gemm in (("fp64", fde.F64, fde.GEMM_FP64), ("fp32", fde.F32, fde.GEMM_FP64),
                             ("fp32_bf16x6", fde.F32, fde.GEMM_BF16X6)):
        warm = driver.Engine(s, prec=prec, backend=be, gemm=gemm)  # first launches of this mode's kernels
        warm.cycle()
        del warm
        eng = driver.Engine(s, prec=prec, backend=be, gemm=gemm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hit = None
        for c in range(max_cycles):
            eng.cycle()
            e, r = state(eng)
            de = max(np.max(np.abs(a[o] - b[o])) for a, b, o in zip(e, eps, occ))
            dr = max(np.sum(np.abs(r[I] - rho[I])) * dv for I in range(len(s.subsystems)))
            if de <= 1e-6 and dr <= 1e-5:
                hit = (c + 1, time.perf_counter() - t0)
                break
        out[name] = None if hit is None else {"cycles": hit[0], "seconds": hit[1]}
    if out["fp64"] and out["fp32"]:
        out["speedup_fp32_over_fp64"] = out["fp64"]["seconds"] / out["fp32"]["seconds"]
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": a.gpus}))
        return 2
    if a.copy_probe:
        print(json.dumps(copy_probe(a.copy_probe)))
        return 0
    import numpy as np
    import torch

    import fde_synth
    from paper_1406_7803_amd import driver, fde

    prec = fde.F32 if a.prec == "fp32" else fde.F64
    be = fde.gpu_backend("cuda:0")
    many = a.workload == "64-subsystems"
    system = fde_synth.config3() if many else fde_synth.config2()
    print("# building engine", file=sys.stderr, flush=True)
    gemm = {"fp64": fde.GEMM_FP64, "bf16x3": fde.GEMM_BF16X3, "bf16x6": fde.GEMM_BF16X6}[a.gemm]
    eng = driver.Engine(system, prec=prec, backend=be, gemm=gemm, streams=a.streams)
    torch.cuda.synchronize()
    print("# engine ready", file=sys.stderr, flush=True)
    tuned = None
    if not a.no_autotune:
        eng.cycle()  # a potential and bands to time with
        tuned = eng.autotune()
        print(f"# autotune: {tuned}", file=sys.stderr, flush=True)
    secs, wall = time_cycles(eng, a.steps, a.warmup, graph=not a.eager)
    per_cycle = eng.band_applies_per_cycle()
    ms_step = secs / a.steps * 1e3
    value = per_cycle * a.steps / secs
    eps_err_ok = all(int(b.info.item()) == 0 for row in eng.blocks for b in row)

    # ---- isolated H application on a resident batch (roofline object)
    plan = eng.plan
    b = eng.blocks[0][0]
    nb = b.nb
    X = b.V[:nb].clone()
    HX = torch.empty_like(X)
    veff = eng.veff[0]
    for _ in range(3):
        plan.apply_h(b.ik, X, veff, b.beta, b.dkb, out=HX)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.apply_reps):
        plan.apply_h(b.ik, X, veff, b.beta, b.dkb, out=HX)
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / 1e3 / a.apply_reps
    N3 = plan.grid[2]
    nproj = 0 if b.beta is None else b.beta.shape[0]
    alg_bytes = apply_bytes(plan, b.ik, nb, nproj)
    achieved = alg_bytes / t_apply / 1e9
    isolated = nb / t_apply

    fp64 = None
    if a.also_fp64 and prec == fde.F32:
        eng64 = driver.Engine(system, prec=fde.F64, backend=be)
        s64, _ = time_cycles(eng64, max(2, a.steps // 2), 1)
        fp64 = {"ms_per_cycle": s64 / max(2, a.steps // 2) * 1e3}
        del eng64

    tta = None if a.no_tta else time_to_accuracy(be)

    cpu = None
    if not a.no_cpu_baseline and not many:
        from oracle import basis, hamiltonian as oham, pseudo as opseudo
        cell = basis.Cell(system.L, system.grid)
        sph = basis.sphere(cell, system.ecut, system.subsystems[0].kfrac[0])
        vl = veff.double().cpu().numpy()
        psi = X[:a.cpu_bands].to(torch.complex128).cpu().numpy()
        beta, dkb = opseudo.kb_projectors(cell, sph, system.subsystems[0].atoms)
        t0 = time.perf_counter()
        oham.apply_h(cell, sph, psi, vl, beta, dkb)
        tc = time.perf_counter() - t0
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": a.cpu_bands / tc, "unit": "band-applies/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 oracle H application (naive DFTs) of {a.cpu_bands} slab bands at one k-point "
                         f"of the same cell, {tc:.1f} s"}

    out = {
        "metric": "H|psi> band-applies/s and embedding-cycle time",
        "value": value,
        "unit": "band-applies/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == fde.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": ("64 uneven subsystems in a 20 bohr cube, 72x72x72 grid, Ecut 15 Ha, "
                                "4-128 bands and 1-8 k-points each" if many else
                                "slab+molecule 10.2x10.2x40 bohr, 60x60x240 grid, Ecut 40 Ha, "
                                "slab 36 ions/40 bands/4 k + molecule 6 ions/8 bands/Gamma"),
                   "band_applies_per_cycle": per_cycle, "davidson_per_cycle": system.n_david,
                   "subspace_products": a.gemm, "launch": "eager" if a.eager else "one HIP graph per cycle",
                   "apply_bands_per_plane_workgroup": None if tuned is None else tuned["bpw"],
                   "z_pass": "four-step register FFT" if system.grid[2] in (240, 120) else "LDS Stockham",
                   "solver_streams": len(eng.groups),
                   "parallelism": "single GPU"},
        "isolated_apply_h": {"band_applies_per_s": isolated, "bands": nb, "projectors": nproj,
                             "ms_per_call": t_apply * 1e3},
        "roofline": {"kernel": "fde_apply_h: FFT sandwich (KZInv, KPlaneHReg, KZFwd) + projectors "
                               "(KAhBAll, KKbReduce, KKbAdd)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if many else measured_traffic(), "algorithmic_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "stream_copy_GBps": copy_probe(1024)["copy_GBps"],
        "time_to_1e-6Ha": tta,
        "fp64_cycle": fp64,
        "device_info_ok": eps_err_ok,
        "wall_s_timed": wall,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
