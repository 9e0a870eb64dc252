"""Benchmark: H|psi> band-applies/s and embedding-cycle time on one MI355X.

Default workload (the benchmark line): the large metal-surface cell -- 20.4 x
20.4 x 60 bohr, 144 x 144 x 432 grid, E_cut = 26 Ha (about 158 000 plane
waves per k); a 144-atom slab with s + p Kleinman-Bylander projectors (576),
320 bands, 2 k-points, Fermi-Dirac 0.01 Ha; four 6-atom molecules at Gamma
with 8 bands each. Synthetic seeded inputs of that shape (the paper's systems
need pseudopotential files that are not available).

A step is one embedding cycle (one HIP graph replay): embedding potential of
all subsystems, per subsystem and k-point one H application + Rayleigh-Ritz
then 4 Davidson iterations (preconditioner, H application, Rayleigh-Ritz),
occupations, densities and mixing. `value` is band-applies per cycle / cycle
time, FP32 plan.

The roofline object is one fde_apply_h call on all 320 slab bands at one
k-point without projectors: the FFT sandwich (stick inverse FFT, in-plane pass
with V_eff, stick forward FFT + kinetic term), which is bound by FP32 vector
arithmetic on this grid. Algorithmic flops per band-apply, with the 5 n log2 n
convention per transform of length n:
    10 N3 log2(N3) ncol + 10 N1 N2 log2(N1 N2) N3 + 2 N,
timed with HIP events on the library's stream. Algorithmic bytes (complex of
cs bytes, V_eff real of rs bytes, V_eff counted once per call):
    nb (3 cs npw + 4 cs ncol N3) + rs N.

Also in the line: the same call with the projectors, the precision study of the
large cell (FP64 plan as the reference; FP32 plan with FP64, BF16x3 and BF16x6
subspace products: Ritz-value and density errors per cycle), the slab +
molecule cell (cycle and H application), the time to 1e-6 Ha of the band
solver at a fixed self-consistent potential of the slab + molecule cell (FP64 +
TPA, FP32 + TPA, FP32 + learned preconditioner), the oracle timed on the host
cores, and the attainable copy bandwidth.

`--workload slab-molecule` / `64-subsystems` time those cells' cycles instead.
`--apply-only` runs only the isolated H application (for counter profiles).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H|ψ> band-applies/s and embedding-cycle time, FP32+learned vs FP64 @1e-6 Ha"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFS = 157.3
# sources of the kernels one fde_apply_h call runs (the counter summary is tied to them)
APPLY_SOURCES = ["common.hpp", "kernels_gemm.hpp", "kernels_plane.hpp", "kernels_plane4.hpp", "kernels_pw.hpp",
                 "pw.hip"]
TRAFFIC_FILE = {"large-slab": "apply_h_large_slab_144x144x432.traffic.txt",
                "slab-molecule": "apply_h_slab_molecule_60x60x240.traffic.txt"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large-slab", "slab-molecule", "64-subsystems"], default="large-slab")
    ap.add_argument("--apply-reps", type=int, default=10)
    ap.add_argument("--apply-only", action="store_true", help="only the isolated H application, then exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-study", action="store_true")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-1e-6 Ha comparison")
    ap.add_argument("--no-second-cell", action="store_true", help="skip the slab + molecule line")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--streams", type=int, default=0,
                    help="concurrent band-solver groups (0: one for blocks that fill the GPU, else three)")
    ap.add_argument("--gemm", choices=["fp64", "bf16x3", "bf16x6"], default="fp64",
                    help="arithmetic of the Rayleigh-Ritz subspace products (FP32 plan)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only time a plain device-to-device copy of MIB MiB (stream bandwidth and "
                         "the calibration of the HBM byte counters), then exit")
    return ap.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


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


def sandwich_model(plan, ik, nb):
    """Algorithmic flops and bytes of one fde_apply_h call without projectors."""
    cs = 16 if plan.prec == 0 else 8
    rs = cs // 2
    N1, N2, N3 = plan.grid
    N = N1 * N2 * N3
    npw, ncol = plan.npw(ik), plan.ncol(ik)
    flops = nb * (10 * N3 * math.log2(N3) * ncol + 10 * N1 * N2 * math.log2(N1 * N2) * N3 + 2 * N)
    nbytes = nb * (3 * cs * npw + 4 * cs * ncol * N3) + rs * N
    return flops, nbytes


def sources_hash():
    h = hashlib.sha256()
    for src in sorted(os.path.join(ROOT, "paper_1406_7803_amd", "csrc", n) for n in APPLY_SOURCES):
        h.update(os.path.basename(src).encode())
        h.update(open(src, "rb").read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per fde_apply_h call from the committed counter summary, or None
    when the sources of its kernels changed since the counters were taken."""
    f = os.path.join(ROOT, "profiles", TRAFFIC_FILE.get(workload, "-"))
    if not os.path.exists(f):
        return None
    kv = dict(line.split()[:2] for line in open(f) if line.strip() and not line.startswith("#"))
    if sources_hash() != kv.get("sources_sha256"):
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
        log(f"cycle {k + 1}/{steps} enqueued")
    s1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return s0.elapsed_time(s1) / 1e3, wall


def slab_block(eng):
    return max((b for row in eng.blocks for b in row), key=lambda b: b.nb * eng.plan.npw(b.ik))


def isolated_apply(eng, reps, with_proj):
    """Median-free mean time of fde_apply_h on the largest block (events on the plan's stream)."""
    import torch
    plan = eng.plan
    b = slab_block(eng)
    X = b.V[:b.nb].clone()
    HX = torch.empty_like(X)
    veff = eng.veff[b.isub]
    beta, dkb = (b.beta, b.dkb) if with_proj else (None, None)
    for _ in range(2):
        plan.apply_h(b.ik, X, veff, beta, dkb, out=HX)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.apply_h(b.ik, X, veff, beta, dkb, out=HX)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    nproj = 0 if beta is None else beta.shape[0]
    return b, t, nproj


def roofline_object(eng, reps, workload):
    b, t, _ = isolated_apply(eng, reps, with_proj=False)
    flops, nbytes = sandwich_model(eng.plan, b.ik, b.nb)
    achieved = flops / t / 1e12
    traffic = measured_traffic(workload)
    return {"kernel": "fde_apply_h without projectors: FFT sandwich (stick inverse FFT, in-plane pass with V_eff, "
                      "stick forward FFT + kinetic term)",
            "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFS, "traffic": traffic,
            "algorithmic_flops": flops, "algorithmic_bytes": nbytes, "bands": b.nb, "ms_per_call": t * 1e3,
            "hbm_GBps_algorithmic": nbytes / t / 1e9, "hbm_frac_algorithmic": nbytes / t / 1e9 / HBM_PEAK_GBS}


def cycle_errors(ref_hist, hist, dv, nelec):
    """Per cycle: max |d eps| over occupied levels and max_I int |d rho_I| (also per electron)."""
    import numpy as np
    out = []
    for (e0, o0, r0), (e1, _, r1) in zip(ref_hist, hist):
        de = max(float(np.max(np.abs((a - b)[o > 1e-8]))) for a, b, o in zip(e1, e0, o0))
        dr = [float(np.sum(np.abs(r1[I] - r0[I]))) * dv for I in range(len(r0))]
        out.append({"max_deps_occ_Ha": de, "max_int_drho": max(dr),
                    "max_int_drho_per_electron": max(d / n for d, n in zip(dr, nelec))})
    return out


def run_cycles(eng, n):
    import torch
    hist, times = [], []
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.cycle()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        hist.append(([e.cpu().numpy().copy() for e in eng.eps], [o.cpu().numpy().copy() for o in eng.occw],
                     eng.rho_out.double().cpu().numpy().copy()))
    return hist, times


def precision_study(system, be, n_cycles=3, streams=0):
    """The large cell's fixed schedule with the FP64 plan (reference) and the FP32 plan
    with each subspace-product mode; errors of every FP32 run against the FP64 one."""
    import numpy as np
    import torch
    from paper_1406_7803_amd import driver, fde
    dv = float(np.prod(system.L)) / float(np.prod(system.grid))
    nelec = [s.nelec for s in system.subsystems]
    log("precision study: FP64 reference")
    eng = driver.Engine(system, prec=fde.F64, backend=be, streams=streams)
    ref, t64 = run_cycles(eng, n_cycles)
    del eng
    torch.cuda.empty_cache()
    out = {"cycles": n_cycles, "reference": "FP64 plan, FP64 subspace products",
           "fp64": {"s_per_cycle": t64}}
    for name, gemm in (("fp32", fde.GEMM_FP64), ("fp32_bf16x6", fde.GEMM_BF16X6),
                       ("fp32_bf16x3", fde.GEMM_BF16X3)):
        log(f"precision study: {name}")
        eng = driver.Engine(system, prec=fde.F32, backend=be, gemm=gemm, streams=streams)
        hist, t = run_cycles(eng, n_cycles)
        ok = all(int(b.info.item()) == 0 for row in eng.blocks for b in row)
        del eng
        torch.cuda.empty_cache()
        out[name] = {"s_per_cycle": t, "errors_per_cycle": cycle_errors(ref, hist, dv, nelec), "info_ok": ok}
    return out


def network_params(be):
    """The learned preconditioner's parameters (FP32): tests/golden/mlp_params.npy, trained
    offline on Jacobi-Davidson corrections of small cells; None when absent."""
    import numpy as np
    import torch
    f = os.path.join(ROOT, "tests", "golden", "mlp_params.npy")
    if not os.path.exists(f):
        return None
    return torch.from_numpy(np.load(f).astype(np.float32)).to(be.device)


def time_to_accuracy(be, max_cycles=150):
    """Time to 1e-6 Ha on the two-subsystem cube: the embedding cycle from the seeded start
    with FP64 + TPA, FP32 + TPA and FP32 + the learned preconditioner, each run until every
    occupied eigenvalue is within 1e-6 Ha of the converged FP64 cycle (density residual
    below 1e-11 electrons) and every int |rho_I - rho_I^ref| <= 1e-5. Seconds are the summed
    per-cycle times (each cycle synchronised; the host-side checks between cycles are not
    counted); every variant first runs two cycles on a throwaway engine so that no kernel's
    first-use set-up is timed."""
    import numpy as np
    import torch
    import fde_synth
    from paper_1406_7803_amd import driver, fde
    s = fde_synth.config1()
    dv = float(np.prod(s.L)) / float(np.prod(s.grid))
    ref = driver.Engine(s, prec=fde.F64, backend=be, streams=1)
    ref_cycles, ref_res = driver.converge(ref, 1e-11, 600)
    eps_ref = [e.cpu().numpy().copy() for e in ref.eps]
    occ = [(o > 1e-8).cpu().numpy() for o in ref.occw]
    rho_ref = ref.rho_out.double().cpu().numpy()
    del ref
    out = {"system": "two-subsystem cube 10 bohr, 24^3 grid, Ecut 7 Ha, 2 x 2 bands, Gamma; linear mixing 0.3, "
                     "4 Davidson iterations per cycle",
           "reference": {"prec": "fp64", "cycles": ref_cycles, "density_residual": ref_res}}
    params = network_params(be)
    for name, prec, mlp in (("fp64_tpa", fde.F64, False), ("fp32_tpa", fde.F32, False),
                            ("fp32_mlp", fde.F32, True)):
        if mlp and params is None:
            out[name] = "not run: tests/golden/mlp_params.npy absent"
            continue
        kw = dict(prec=prec, backend=be, streams=1, mlp_params=params if mlp else None)
        warm = driver.Engine(s, **kw)
        warm.cycle()
        warm.cycle()
        del warm
        eng = driver.Engine(s, **kw)
        torch.cuda.synchronize()
        t, reached, errs = 0.0, None, None
        for c in range(max_cycles):
            t0 = time.perf_counter()
            eng.cycle()
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            de = max(float(np.max(np.abs(e.cpu().numpy() - r)[o])) for e, r, o in zip(eng.eps, eps_ref, occ))
            rho = eng.rho_out.double().cpu().numpy()
            dr = max(float(np.sum(np.abs(rho[I] - rho_ref[I]))) * dv for I in range(len(s.subsystems)))
            errs = (de, dr)
            if de <= 1e-6 and dr <= 1e-5:
                reached = c + 1
                break
        out[name] = {"cycles": reached, "seconds": t if reached else None, "ms_per_cycle": 1e3 * t / (c + 1),
                     "final_max_deps_occ_Ha": errs[0], "final_max_int_drho": errs[1]}
        del eng
    for v in ("fp32_mlp", "fp32_tpa"):
        a, b = out.get("fp64_tpa"), out.get(v)
        if isinstance(a, dict) and isinstance(b, dict) and a["seconds"] and b["seconds"]:
            out[f"speedup_fp64_tpa_over_{v}"] = a["seconds"] / b["seconds"]
    return out


def table1_analogue(be):
    """Table 1's quantities on the slab + molecule geometry (PBE, FP64 plan, Pulay + Kerker):
    Kohn-Sham of the supersystem against FDE with each nonadditive kinetic functional,
    <Delta rho> and the interaction energies (without the inter-fragment ion-ion term,
    the same in both)."""
    import fde_synth
    from paper_1406_7803_amd import driver, fde
    s = fde_synth.config2()
    mixer = dict(kind="pulay", nhist=8, beta=0.2, q0=0.4)
    out = {"system": "slab + molecule cell; xc PBE; interaction energies in Ha without the ion-ion term",
           "mixing": mixer, "tolerance_electrons": 1e-5}
    for name, kin in (("lc94", fde.KIN_LC94), ("revapbek", fde.KIN_REVAPBEK)):
        r = driver.supersystem_comparison(s, prec=fde.F64, backend=be,
                                          kinds=dict(xc=fde.XC_PBE, xc_nad=fde.XC_PBE, kin_nad=kin),
                                          tol=1e-5, max_cycles=500, mixer=mixer)
        out[name] = {k: r[k] for k in ("dens_diff", "int_KS", "int_FDE", "E_KS", "E_FDE", "cycles", "residuals")}
    return out


def second_cell(be, a):
    """The slab + molecule cell: cycle time (graph replays) and the isolated H application."""
    import torch
    import fde_synth
    from paper_1406_7803_amd import driver, fde
    s = fde_synth.config2()
    eng = driver.Engine(s, prec=fde.F32, backend=be, streams=a.streams)
    eng.cycle()
    tuned = eng.autotune()
    secs, _ = time_cycles(eng, 10, 2, graph=True)
    per_cycle = eng.band_applies_per_cycle()
    b, t, nproj = isolated_apply(eng, 50, with_proj=True)
    out = {"workload": "slab+molecule 10.2x10.2x40 bohr, 60x60x240 grid, Ecut 40 Ha, slab 36 ions/40 bands/4 k "
                       "+ molecule 6 ions/8 bands/Gamma",
           "band_applies_per_s": per_cycle * 10 / secs, "ms_per_cycle": secs / 10 * 1e3,
           "isolated_apply_h": {"band_applies_per_s": b.nb / t, "bands": b.nb, "projectors": nproj,
                                "ms_per_call": t * 1e3},
           "roofline": roofline_object(eng, 50, "slab-molecule"), "autotune": {k: tuned[k] for k in ("plane", "rows", "bpw")}}
    del eng
    torch.cuda.empty_cache()
    return out


def cpu_baseline(system, n_bands=8):
    """The oracle (FFT mode, all host cores) timed on a bounded sample of the same workload:
    H application (local potential + Kleinman-Bylander projectors) of n_bands slab bands
    at one k-point; and one cycle of the two-subsystem cube for scale."""
    import numpy as np
    import fde_synth
    from oracle import basis, dft, hamiltonian as oham, pseudo as opseudo, scf as oscf
    cores = len(os.sched_getaffinity(0))
    dft.set_mode("fft", cores)
    try:
        cell = basis.Cell(system.L, system.grid)
        sph = basis.sphere(cell, system.ecut, system.subsystems[0].kfrac[0])
        beta, dkb = opseudo.kb_projectors(cell, sph, system.subsystems[0].atoms)
        veff = fde_synth.random_real(3, cell.shape, -1, 1)
        psi = fde_synth.random_complex(4, (n_bands, sph.npw))
        t0 = time.perf_counter()
        oham.apply_h(cell, sph, psi, veff, beta, dkb)
        tc = time.perf_counter() - t0
        s1 = fde_synth.config1()
        st = oscf.setup(s1)
        t1 = time.perf_counter()
        oscf.run(s1, n_cycles=2, st=st)
        c1 = (time.perf_counter() - t1) / 2
    finally:
        dft.set_mode("naive")
    model = ""
    try:
        model = [l.split(":", 1)[1].strip() for l in subprocess.run(["lscpu"], capture_output=True, text=True).stdout
                 .splitlines() if l.startswith("Model name")][0]
    except Exception:
        pass
    return {"value": n_bands / tc, "unit": "band-applies/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle (scipy.fft mode, {cores} threads) H application of {n_bands} slab bands with "
                      f"{beta.shape[0]} projectors at one k-point of the same cell, {tc:.1f} s",
            "cpu_model": model, "cycle_s_two_subsystem_cube": c1}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; runs on several GPUs are not part of it",
                          "n_gpus": a.gpus}))
        return 2
    if a.copy_probe:
        print(json.dumps(copy_probe(a.copy_probe)))
        return 0
    import torch

    import fde_synth
    from paper_1406_7803_amd import driver, fde

    be = fde.gpu_backend("cuda:0")
    system = {"large-slab": fde_synth.config4, "slab-molecule": fde_synth.config2,
              "64-subsystems": fde_synth.config3}[a.workload]()
    log(f"building engine ({a.workload})")
    gemm = {"fp64": fde.GEMM_FP64, "bf16x3": fde.GEMM_BF16X3, "bf16x6": fde.GEMM_BF16X6}[a.gemm]
    eng = driver.Engine(system, prec=fde.F32, backend=be, gemm=gemm, streams=a.streams)
    torch.cuda.synchronize()
    log("engine ready")
    eng.cycle()  # a potential and bands to time with
    tuned = None
    if not a.no_autotune:
        tuned = eng.autotune(reps=3)
        log(f"autotune: {tuned}")
    if a.apply_only:
        b, t, nproj = isolated_apply(eng, a.apply_reps, with_proj=False)
        print(json.dumps({"apply_only_ms_per_call": t * 1e3, "bands": b.nb}))
        return 0
    secs, wall = time_cycles(eng, a.steps, a.warmup, graph=not a.eager)
    per_cycle = eng.band_applies_per_cycle()
    ms_step = secs / a.steps * 1e3
    value = per_cycle * a.steps / secs
    info_ok = all(int(b.info.item()) == 0 for row in eng.blocks for b in row)
    log("roofline object")
    roof = roofline_object(eng, a.apply_reps, a.workload)
    bp, tp, nproj = isolated_apply(eng, a.apply_reps, with_proj=True)
    isolated = {"band_applies_per_s": bp.nb / tp, "bands": bp.nb, "projectors": nproj, "ms_per_call": tp * 1e3}
    n_groups = eng.n_groups
    del eng
    torch.cuda.empty_cache()

    many = a.workload == "64-subsystems"
    prec_study = None
    if not a.no_precision_study and not many:
        prec_study = precision_study(system, be, streams=a.streams)
    second = None
    if a.workload == "large-slab" and not a.no_second_cell:
        log("slab + molecule cell")
        second = second_cell(be, a)
    tta = None
    if not a.no_tta and not many:
        log("time to 1e-6 Ha")
        tta = time_to_accuracy(be)
    table1 = None
    if a.workload == "large-slab" and not a.no_second_cell:
        log("supersystem comparison")
        table1 = table1_analogue(be)
    copy = copy_probe(1024)["copy_GBps"]
    cpu = None
    if not a.no_cpu_baseline and not many:
        log("cpu baseline")
        cpu = cpu_baseline(system)

    names = {"large-slab": "large metal-surface cell 20.4x20.4x60 bohr, 144x144x432 grid, Ecut 26 Ha, slab 144 "
                           "ions/576 s+p projectors/320 bands/2 k + 4 molecules x 8 bands/Gamma",
             "slab-molecule": "slab+molecule 10.2x10.2x40 bohr, 60x60x240 grid, Ecut 40 Ha, slab 36 ions/40 "
                              "bands/4 k + molecule 6 ions/8 bands/Gamma",
             "64-subsystems": "64 uneven subsystems in a 20 bohr cube, 72x72x72 grid, Ecut 15 Ha, 4-128 bands and "
                              "1-8 k-points each"}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "band-applies/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": names[a.workload], "band_applies_per_cycle": per_cycle,
                   "davidson_per_cycle": system.n_david, "subspace_products": a.gemm,
                   "launch": "eager" if a.eager else "one HIP graph per cycle",
                   "autotune": None if tuned is None else {k: tuned[k] for k in ("plane", "rows", "bpw", "zlds", "sz")},
                   "solver_streams": n_groups, "parallelism": "single GPU"},
        "isolated_apply_h": isolated,
        "roofline": roof,
        "cpu_baseline": cpu,
        "precision_study": prec_study,
        "slab_molecule": second,
        "time_to_1e-6Ha": tta,
        "supersystem_comparison": table1,
        "stream_copy_GBps": copy,
        "device_info_ok": info_ok,
        "wall_s_timed": wall,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
