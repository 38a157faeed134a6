"""Benchmark: converged Sternheimer solves per second of the chi0 apply on one GPU.

Headline workload: the large cell at full size (L = 32 bohr, 512 atoms, 30 Ry: 91,047 plane
waves, 128^3 grid, 1,024 occupied bands). A step is one stern_apply_chi0 over 4 fields x 1,024
bands = 4,096 Sternheimer solves (the one-GPU share of a 32-field Davidson block spread over 8
GPUs), FP64 true residual <= 1e-8, inputs already resident in HBM. The headline path is fixed
before anything is timed: the learned diagonal preconditioner (net trained, untimed, on fields
4-5 of the same cell, disjoint from the timed fields 0-3) with mixed-precision defect correction
(FP32 FFTs, split-BF16 MFMA GEMMs, FP64 outer residual). The plain FP64 path runs the same call
as the baseline, with its own step count. The occupied states come from the input generator's
GPU eigensolver (Chebyshev-filtered subspace iteration on the library's own H apply, untimed).

Timed steps run without the per-launch profile; one extra profiled step of the headline path,
the last apply of the run, gives the kernel breakdown and the roofline of the dominant kernel
(HIP events on the library's stream). Secondary entries (fewer steps, same metric): the mid
cell (72^3, 128 bands x 64 fields) and the 32 uneven cells of the batched workload in one
stern_apply_chi0_many call. The CPU oracle is timed on a seeded uniform sample of the headline's
(band, field) pairs, solved as one batch; its mean iterations are stated beside the GPU's.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--fp64-steps F] [--no-cpu-baseline]
                    [--no-secondary] [--cpu-pairs P] [--headline-only] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6    # MI355X dense FP64 matrix
BF16_MFMA_PEAK_TFS = 2500.0  # MI355X dense BF16 matrix
FP32_VALU_PEAK_TFS = 157.3   # MI355X FP32 vector (256 CUs, 2.4 GHz; counts dual-issue/packed FP32)
FP64_VALU_PEAK_TFS = 78.6    # MI355X FP64 vector
# kernels whose work is vector-ALU arithmetic (FFT butterflies) rather than matrix-core products
ALU_KERNELS = {"plane_h32": FP32_VALU_PEAK_TFS, "plane_h": FP64_VALU_PEAK_TFS}
MFMA_KERNELS = {"gemm_bf16": BF16_MFMA_PEAK_TFS, "pc_reduce": FP64_MFMA_PEAK_TFS, "pc_expand": FP64_MFMA_PEAK_TFS,
                "kb_reduce": FP64_MFMA_PEAK_TFS, "kb_expand": FP64_MFMA_PEAK_TFS, "net": BF16_MFMA_PEAK_TFS}
FFT_KERNELS = ("plane_h32", "x32", "plane_h", "xinv", "xfwd")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
METRIC = "converged Sternheimer solves/s at resid≤1e-8 (learned+mixed vs plain FP64)"


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel: str, algorithmic_bytes_per_launch: float, workload: str):
    """HBM bytes per launch of `kernel` in this run: the ratio of measured (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, calibrated on a plain copy) to algorithmic bytes over the same launches of a
    committed counter run of this workload, times this run's algorithmic bytes per launch; None
    when there is no such run or the kernel source has changed since the counters were taken."""
    from paper_2607_14025_amd.rocprof_summary import source_hash
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE)).get(f"{workload}:{kernel}")
    if not t or t.get("source_sha1") != source_hash(kernel) or not t.get("measured_over_algorithmic"):
        return None
    return t["measured_over_algorithmic"] * algorithmic_bytes_per_launch


def timed_steps(fn, steps, warmup, label):
    """Runs fn() warmup times, then `steps` times between device synchronisations; returns
    (solves/s over the timed steps, seconds, list of infos)."""
    import torch
    for w in range(warmup):
        info = fn()
        log(f"{label} warmup {w}: {info['n_converged']}/{info['n_solves']} converged in {info['wall_s']:.2f} s")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(steps):
        info = fn()
        infos.append(info)
        log(f"{label} step {k}: {info['n_converged']}/{info['n_solves']} converged, {info['wall_s']:.3f} s, "
            f"mean iterations {info['total_iters'] / max(1, info['n_solves']):.1f}, max {info['max_iters']}, "
            f"max true resid {info['max_true_resid']:.2e}, fallback {info['n_fallback']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    conv = sum(i["n_converged"] for i in infos)
    return conv / dt, dt, infos


def summary(infos, dt, value):
    import numpy as np
    return dict(solves_per_s=value, steps=len(infos), seconds=dt,
                mean_iters=float(np.mean([i["total_iters"] / max(1, i["n_solves"]) for i in infos])),
                max_iters=int(max(i["max_iters"] for i in infos)),
                fallback_solves=int(sum(i["n_fallback"] for i in infos)),
                max_true_resid=float(max(i["max_true_resid"] for i in infos)))


def rel_err(a, ref):
    n = ref.shape[0]
    return ((a - ref).reshape(n, -1).norm(dim=1) / ref.reshape(n, -1).norm(dim=1)).max().item()


def roofline(kern, workload):
    dom = max(kern, key=lambda n: kern[n]["ms"])
    d = kern[dom]
    per_launch_s = d["ms"] / d["launches"] / 1e3
    traffic = measured_traffic(dom, d["bytes"] / d["launches"], workload)
    if dom in ALU_KERNELS or dom in MFMA_KERNELS:
        peak = ALU_KERNELS.get(dom) or MFMA_KERNELS[dom]
        achieved = d["flops"] / d["launches"] / per_launch_s / 1e12
        roof = dict(bound="alu" if dom in ALU_KERNELS else "mfma", achieved=achieved, peak=peak, unit="TFLOP/s",
                    frac=achieved / peak, traffic=traffic, kernel=dom,
                    hbm_GBps=d["bytes"] / d["launches"] / per_launch_s / 1e9)
        if dom == "gemm_bf16":
            # the split-BF16 products issue three BF16 MFMA products per complex multiply-add
            roof["bf16_mfma_TFLOPs_issued"] = 3.0 * achieved
    else:
        achieved = d["bytes"] / d["launches"] / per_launch_s / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel=dom)
    roof["launches"] = d["launches"]
    roof["ms_per_launch"] = d["ms"] / d["launches"]
    roof["traffic_source"] = ("profiles/traffic.json: rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel on this "
                              "workload, calibrated on a 1 GiB copy, as a ratio to the algorithmic bytes, scaled to "
                              "this run's launches") if traffic is not None else None
    return roof


def breakdown(kern):
    total_ms = sum(v["ms"] for v in kern.values())
    return {n: dict(share=round(v["ms"] / total_ms, 4), launches=v["launches"],
                    bytes_per_launch=round(v["bytes"] / v["launches"]), ms_per_launch=round(v["ms"] / v["launches"], 4),
                    GBps=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                    TFLOPs=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2) if v["flops"] > 0 else None)
            for n, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])}


def fft_stage(kern):
    """HBM rate of the FFT stage (x pencils and yz planes) of the profiled step."""
    ks = [k for k in FFT_KERNELS if k in kern]
    ms = sum(kern[k]["ms"] for k in ks)
    b = sum(kern[k]["bytes"] for k in ks)
    if ms <= 0:
        return None
    gbs = b / (ms / 1e3) / 1e9
    return dict(kernels=ks, ms=ms, algorithmic_GB=b / 1e9, GBps=gbs, frac_of_hbm_peak=gbs / HBM_PEAK_GBS,
                target_frac=0.6)


def cpu_baseline(wl, pairs, tol, gpu_x):
    """The oracle on a seeded sample of the headline's (band, field) pairs, solved together as
    one vectorised batch (RHS, projected Teter-PCG to true residual `tol`, dn), numpy/scipy FP64;
    also the residual of the GPU's solutions of the same pairs under the oracle's operator."""
    import numpy as np
    from oracle import OracleCell, project
    from oracle.sternheimer import band_kinetic, delta_n, pcg_solve, rhs
    spec = wl["spec"]
    cell = OracleCell(spec.L, spec.ecut, wl["pos"])
    psi = cell.take(wl["psi"].cpu().numpy() if hasattr(wl["psi"], "cpu") else wl["psi"], wl["miller"])
    bands = [v for v, _ in pairs]
    perts = [i for _, i in pairs]
    tk = band_kinetic(cell, psi)
    t0 = time.perf_counter()
    b = rhs(cell, psi, wl["dv"], bands, perts)
    xo, its, _ = pcg_solve(cell, psi, wl["eps"][bands], tk[bands], b, tol)
    delta_n(cell, psi, xo, bands, perts, max(perts) + 1)
    dt = time.perf_counter() - t0
    x = cell.take(gpu_x, wl["miller"])
    px = project(psi, x)
    ax = project(psi, cell.h_apply(px) - wl["eps"][bands][:, None] * px)
    res = np.linalg.norm(b - ax, axis=1) / np.linalg.norm(b, axis=1)
    dx = np.linalg.norm(x - xo, axis=1) / np.linalg.norm(xo, axis=1)
    return dict(value=len(pairs) / dt, unit="solves/s", cores=len(os.sched_getaffinity(0)), kind="oracle",
                sample=f"{len(pairs)} (band, field) pairs of the headline cell drawn uniformly with a seeded "
                       f"generator: {pairs}; solved as one vectorised batch (RHS + projected Teter-PCG to true "
                       f"residual {tol:g} + dn), numpy/scipy FP64, {dt:.1f} s",
                mean_iters=float(np.mean(its)), iters=[int(i) for i in its],
                gpu_x_true_resid_under_oracle_max=float(res.max()),
                gpu_x_vs_oracle_x_rel_max=float(dx.max()))


def large_entry(args, dev):
    import numpy as np
    import torch
    from paper_2607_14025_amd import Model, STERN_FP64, STERN_MIXED
    from synth.cells import LARGE
    from synth.ground_gpu import large_workload
    log("large cell: ground state on the GPU (Chebyshev-filtered subspace iteration on the library's H)")
    wl = large_workload(LARGE, n_pert=8, verbose=True)  # a line per pass on stderr
    log(f"ground state: {wl['passes']} passes, {wl['wall_s']:.1f} s, gap {wl['gap']:.2e} Ha, "
        f"max eigen-residual {wl['resid'].max():.2e}")
    s = wl["system"]
    s.set_occupied(wl["psi"], torch.from_numpy(wl["eps"]).to(dev))
    dv_all = torch.from_numpy(wl["dv"]).to(dev)
    dv = dv_all[:4].contiguous()
    n_timed, tuned = s.autotune(n_vec=1024)
    tune_ms = s.autotune_report()
    log(f"autotuned {n_timed} kernel candidates: {tuned}")
    log("training the learned preconditioner on fields 4-5")
    model = Model(seed=0, device=0)
    train = model.train([s], [dv_all[4:6].contiguous()], epochs=2, batch=16, lr=1e-3, max_solves=1024, tol=1e-10,
                        seed=1, prec_epochs=4, prec_max_solves=512)
    log(f"training done: {train}")
    dn = torch.empty_like(dv)
    ref = torch.empty_like(dv)

    def call(prec, out, mdl=None, **kw):
        return s.apply_chi0(dv, tol=args.tol, dn_out=out, precision=prec, model=mdl, prec_only=mdl is not None,
                            **kw)[1]

    plain = mixed = None
    if not args.headline_only:
        # plain FP64 baseline (the training's FP64 solves have already run every FP64 kernel)
        v64, t64, i64 = timed_steps(lambda: call(STERN_FP64, ref), args.fp64_steps, 0, "large fp64")
        plain = summary(i64, t64, v64)
        vmx, tmx, imx = timed_steps(lambda: call(STERN_MIXED, dn), 1, 0, "large mixed")
        mixed = summary(imx, tmx, vmx)
        mixed["dn_rel_err_vs_fp64"] = rel_err(dn, ref)
    # headline: learned preconditioner + mixed
    vh, th, ih = timed_steps(lambda: call(STERN_MIXED, dn, model), args.steps, args.warmup, "large learnedK-mixed")
    head = summary(ih, th, vh)
    if plain is not None:
        head["dn_rel_err_vs_fp64"] = rel_err(dn, ref)
    # pairs of the oracle sample: uniform over the step's 4,096 (band, field) pairs, seeded
    rng = np.random.default_rng(np.random.SeedSequence([LARGE.config_id, 0, 7]))
    pick = rng.choice(4 * s.n_occ, size=args.cpu_pairs, replace=False)
    pairs = [(int(k % s.n_occ), int(k // s.n_occ)) for k in pick]
    # the last apply of the run: the headline step once more with the per-launch profile
    _, pinfo = s.apply_chi0(dv, tol=args.tol, dn_out=dn, precision=STERN_MIXED, model=model, prec_only=True,
                            profile=True, samples=pairs)
    torch.cuda.synchronize()
    log(f"profiled step: {pinfo['wall_s']:.3f} s")
    kern = pinfo["kernels"]
    cfg = dict(workload=LARGE.name, L_bohr=LARGE.L, ecut_ry=LARGE.ecut, atoms=LARGE.n_atoms, n_pw=s.n_pw,
               grid=s.fft_n, n_occ=s.n_occ, n_pert=4, solves_per_step=4 * s.n_occ, tol=args.tol,
               share="4 of a 32-field Davidson block x all 1,024 bands: one GPU's share on 8 GPUs",
               ground_state=dict(method="Chebyshev-filtered subspace iteration on the library's FP64 H apply",
                                 passes=wl["passes"], seconds=wl["wall_s"], gap_Ha=wl["gap"],
                                 max_eigen_residual=float(wl["resid"].max())),
               autotuned=tuned, autotune_ms=tune_ms,
               path="learned diagonal preconditioner (x0 = 0) from the BF16 MFMA conv net on the coarse grid, "
                    "FP32 FFTs + split-BF16 MFMA GEMMs in FP64 defect correction; Teter FP64 PCG fallback",
               headline=head, plain_fp64=plain, mixed=mixed,
               training=dict(fields="4-5 of the same cell (timed: 0-3)", **train),
               speedup_vs_plain_fp64=head["solves_per_s"] / plain["solves_per_s"] if plain else None,
               mixed_speedup_vs_plain_fp64=mixed["solves_per_s"] / plain["solves_per_s"] if plain else None)
    out = dict(value=vh, dt=th, steps=args.steps, cfg=cfg, kern=kern, wl=wl, pairs=pairs,
               gpu_x=pinfo["samples"], roof=roofline(kern, LARGE.name), fft=fft_stage(kern))
    model.close()
    del dv_all, dv, dn, ref
    return out, s


def mid_entry(args, dev):
    """Secondary: the mid cell (72^3, 128 bands x 64 fields), mixed and plain FP64."""
    import numpy as np
    import torch
    from paper_2607_14025_amd import System, STERN_FP64, STERN_MIXED
    from synth.cells import MID
    from synth.inputs import load_workload
    wl = load_workload(MID)
    sp = wl["spec"]
    s = System(sp.L, sp.ecut, wl["pos"], sp.vloc_amp, sp.vloc_sigma, sp.kb_D, sp.kb_width, device=0)
    s.set_occupied(torch.from_numpy(np.ascontiguousarray(wl["psi"])).to(dev), torch.from_numpy(wl["eps"]).to(dev))
    s.autotune(n_vec=1024)
    dv = torch.from_numpy(wl["dv"]).to(dev)
    dn, ref = torch.empty_like(dv), torch.empty_like(dv)
    v64, t64, i64 = timed_steps(lambda: s.apply_chi0(dv, tol=args.tol, dn_out=ref, precision=STERN_FP64)[1], 2, 1,
                                "mid fp64")
    vmx, tmx, imx = timed_steps(lambda: s.apply_chi0(dv, tol=args.tol, dn_out=dn, precision=STERN_MIXED)[1], 2, 1,
                                "mid mixed")
    r = dict(workload=sp.name, n_pw=s.n_pw, grid=s.fft_n, solves_per_step=dv.shape[0] * s.n_occ,
             plain_fp64=summary(i64, t64, v64), mixed=summary(imx, tmx, vmx))
    r["mixed"]["dn_rel_err_vs_fp64"] = rel_err(dn, ref)
    r["mixed_speedup_vs_plain_fp64"] = vmx / v64
    r["tddft"] = tddft_entry(s)
    s.close()
    return r


def tddft_entry(s, n_exc=8, reps=3):
    """The Liouville superoperator of TDDFT (Tamm-Dancoff, Hartree kernel) on the same system:
    applies of n_exc excitations on device arrays, the lowest excitation energies by Davidson,
    Z-vector solves, and a Lanczos chain with its absorption spectrum. The grid stage's algorithmic bytes per excitation: n_occ full grids written
    (a_v(r)), read twice (density, products) and written once more (V psi_v), plus psi_v(r) read
    twice: 6 n_occ N^3 complex FP64 values."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(5)
    shape = (n_exc, s.n_occ, s.n_pw)
    a = torch.complex(torch.randn(shape, generator=g, dtype=torch.float64),
                      torch.randn(shape, generator=g, dtype=torch.float64)).to("cuda")
    s.liouville_apply(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.liouville_apply(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    grid_bytes = 6.0 * s.n_occ * s.fft_n ** 3 * 16 * n_exc
    log(f"tddft: L apply of {n_exc} excitations {dt * 1e3:.1f} ms")
    t0 = time.perf_counter()
    w, _, dinfo = s.liouville_davidson(4, tol=1e-4, block=8, max_basis=64, max_iter=300, seed=1)
    tdav = time.perf_counter() - t0
    log(f"tddft: Davidson {dinfo['n_iter']} iterations, {tdav:.2f} s, w {w}")
    b = a[:2].cpu().numpy()
    t0 = time.perf_counter()
    _, it, res, rc = s.liouville_solve(b, tol=1e-8)
    tsol = time.perf_counter() - t0
    log(f"tddft: Z-vector solves {it.tolist()} iterations, {tsol:.2f} s, residuals {res.tolist()}")
    import numpy as np
    N = s.fft_n
    j = np.arange(N) * (2.0 * np.pi / N)
    dvl = np.cos(j)[:, None, None] * np.ones((1, N, N))  # the longest wave along x
    t0 = time.perf_counter()
    al, be, n2 = s.liouville_lanczos(dvl, 100)
    tlan = time.perf_counter() - t0
    om = np.linspace(0.0, 3.0, 601)
    spec = s.lanczos_spectrum(al, be, n2, om, 0.01)
    log(f"tddft: Lanczos 100 steps {tlan:.2f} s, spectrum peak at {om[int(np.argmax(spec))]:.3f} Ha")
    return dict(apply=dict(n_exc=n_exc, ms=dt * 1e3, excitations_per_s=n_exc / dt,
                           grid_GB=grid_bytes / 1e9, grid_GBps_whole_apply=grid_bytes / dt / 1e9),
                davidson=dict(n_eig=4, tol=1e-4, block=8, max_basis=64, iterations=dinfo["n_iter"], seconds=tdav, rc=dinfo["rc"],
                              w_Ha=[float(x) for x in w]),
                zvector=dict(n_exc=2, tol=1e-8, iterations=[int(x) for x in it], seconds=tsol, rc=int(rc),
                             true_resid=[float(x) for x in res]),
                lanczos=dict(field="cos(2 pi x / L)", steps=100, seconds=tlan, ms_per_step=tlan / 100 * 1e3,
                             eta_Ha=0.01, peak_Ha=float(om[int(np.argmax(spec))])))


def batched_entry(args, dev):
    """Secondary: the 32 uneven cells (L ~ U[10, 18], 8-48 atoms, 20 Ry, 16 fields each) in one
    stern_apply_chi0_many call, mixed and plain FP64."""
    import numpy as np
    import torch
    from paper_2607_14025_amd import System, STERN_FP64, STERN_MIXED, apply_chi0_many
    from synth.cells import batched_specs
    from synth.inputs import load_workload
    systems, dvs = [], []
    for sp0 in batched_specs(32):
        w = load_workload(sp0)
        sp = w["spec"]
        s = System(sp.L, sp.ecut, w["pos"], sp.vloc_amp, sp.vloc_sigma, sp.kb_D, sp.kb_width, device=0)
        s.set_occupied(torch.from_numpy(np.ascontiguousarray(w["psi"])).to(dev), torch.from_numpy(w["eps"]).to(dev))
        systems.append(s)
        dvs.append(torch.from_numpy(w["dv"]).to(dev))
    outs64 = [torch.empty_like(d) for d in dvs]
    outs = [torch.empty_like(d) for d in dvs]
    v64, t64, i64 = timed_steps(lambda: apply_chi0_many(systems, dvs, tol=args.tol, dn_outs=outs64,
                                                        precision=STERN_FP64)[1], 2, 1, "batched fp64")
    vmx, tmx, imx = timed_steps(lambda: apply_chi0_many(systems, dvs, tol=args.tol, dn_outs=outs,
                                                        precision=STERN_MIXED)[1], 2, 1, "batched mixed")
    err = max(rel_err(a, b) for a, b in zip(outs, outs64))
    r = dict(workload="batched_32_cells_L10-18_8-48at_20Ry_16fields", systems=len(systems),
             grids=sorted({s.fft_n for s in systems}), solves_per_step=i64[0]["n_solves"],
             plain_fp64=summary(i64, t64, v64), mixed=summary(imx, tmx, vmx), mixed_speedup_vs_plain_fp64=vmx / v64)
    r["mixed"]["dn_rel_err_vs_fp64"] = err
    for s in systems:
        s.close()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-pairs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline path (setup, its steps and the profiled step): for profiler runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the chi0 apply of one cell runs on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).normal_()
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)  # one elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("copied 1 GiB device to device (counter reference)")
        del a, b
    secondary = {}
    if args.headline_only:
        args.no_secondary = args.no_cpu_baseline = True
    if not args.no_secondary:  # before the headline, so that its profiled step is the run's last apply
        log("secondary: batched cells")
        secondary["batched"] = batched_entry(args, dev)
        log("secondary: mid cell")
        secondary["mid"] = mid_entry(args, dev)
        torch.cuda.empty_cache()
    r, s = large_entry(args, dev)
    cfg = r["cfg"]
    if secondary:
        cfg["secondary"] = secondary
    cfg["fft_stage"] = r["fft"]
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(r["wl"], r["pairs"], args.tol, r["gpu_x"])
        cpu["gpu_mean_iters_headline"] = cfg["headline"]["mean_iters"]
    line = dict(metric=METRIC, value=r["value"], unit="solves/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=r["dt"] / args.steps * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32+bf16/f64", data="synthetic", config=cfg, roofline=r["roof"], cpu_baseline=cpu,
                kernels=breakdown(r["kern"]), kernels_steps=1)
    s.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
