"""Benchmark: converged Sternheimer solves per second of one chi0 apply on one GPU.

A step is one stern_apply_chi0 call on the mid cell (L = 20 bohr, 64 atoms,
25 Ry: 16,879 plane waves, 72^3 grid, 128 occupied bands x 64 band-limited
fields = 8,192 Sternheimer solves, FP64 true residual <= 1e-8), inputs already
resident in HBM. The headline path is the learned guess and preconditioner
(trained beforehand, untimed, on two other seeded cells of the same model and
size) with mixed-precision defect correction; the plain FP64 path is timed
on the same cell as the baseline. Prints one JSON line with the throughput,
the roofline of the dominant kernel (per-launch HIP events on the library's
stream) and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--path learned-mixed|mixed|fp64]
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel: str, algorithmic_bytes_per_launch: float):
    """HBM bytes per launch of `kernel` in this run: the ratio of measured (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, calibrated on a plain copy) to algorithmic bytes over the same launches of a
    committed counter run, times this run's algorithmic bytes per launch; None when the kernel
    source has changed since the counters were taken."""
    from paper_2607_14025_amd.rocprof_summary import source_hash
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE)).get(kernel)
    if not t or t.get("source_sha1") != source_hash(kernel) or not t.get("measured_over_algorithmic"):
        return None
    return t["measured_over_algorithmic"] * algorithmic_bytes_per_launch


def cpu_baseline(wl, n_bands: int, tol: float):
    """The oracle on `n_bands` solves (bands 0.. of field 0): RHS, PCG and dn."""
    from oracle import OracleCell, apply_chi0
    spec = wl["spec"]
    cell = OracleCell(spec.L, spec.ecut, wl["pos"])
    psi = cell.take(wl["psi"], wl["miller"])
    t0 = time.perf_counter()
    out = apply_chi0(cell, psi, wl["eps"], wl["dv"][:1], tol=tol, bands=range(n_bands), perts=[0])
    dt = time.perf_counter() - t0
    return dict(value=n_bands / dt, unit="solves/s", cores=len(os.sched_getaffinity(0)), kind="oracle",
                sample=f"{n_bands} (band, field) pairs of the same cell (bands 0-{n_bands - 1} of field 0): "
                       f"RHS + projected Teter-PCG to true residual {tol:g} + dn, numpy/scipy FP64, "
                       f"{dt:.1f} s, mean {out['iters'].mean():.1f} CG iterations")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-bands", type=int, default=48)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path", choices=["learned-mixed", "mixed", "fp64"], default="learned-mixed")
    ap.add_argument("--train-solves", type=int, default=8192)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the chi0 apply of one cell runs on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2607_14025_amd import Model, System, STERN_FP64, STERN_MIXED, STERN_INNER_PROJECTED
    from synth.cells import MID
    from synth.inputs import load_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).normal_()
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)  # one elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print("bench: copied 1 GiB device to device (counter reference)", file=sys.stderr, flush=True)
        del a, b
    print("bench: loading mid cell inputs", file=sys.stderr, flush=True)
    wl = load_workload(MID)
    spec = wl["spec"]

    def make_system(w):
        sp = w["spec"]
        sy = System(sp.L, sp.ecut, w["pos"], sp.vloc_amp, sp.vloc_sigma, sp.kb_D, sp.kb_width, device=0)
        sy.set_occupied(torch.from_numpy(np.ascontiguousarray(w["psi"])).to(dev), torch.from_numpy(w["eps"]).to(dev))
        return sy

    s = make_system(wl)
    dv = torch.from_numpy(wl["dv"]).to(dev)
    n_timed, tuned = s.autotune(n_vec=1024)  # setup, like init and set_occupied: not timed
    tune_ms = s.autotune_report()
    print(f"bench: autotuned {n_timed} kernel candidates: {tuned}; ms per candidate on 1,024 rows: {tune_ms}",
          file=sys.stderr, flush=True)
    dn = torch.empty_like(dv)
    n_pert = dv.shape[0]
    n_solves = n_pert * s.n_occ

    model = None
    train = None
    if args.path == "learned-mixed":
        print("bench: training the learned guess and preconditioner on two other mid cells", file=sys.stderr,
              flush=True)
        tr_sys, tr_dv = [], []
        for sid in (1, 2):
            w = load_workload(MID.with_system(sid))
            tr_sys.append(make_system(w))
            tr_dv.append(torch.from_numpy(w["dv"]).to(dev))
        model = Model(seed=0, device=0)
        train = model.train(tr_sys, tr_dv, epochs=4, batch=16, lr=1e-3, max_solves=args.train_solves, tol=1e-10,
                            seed=1, prec_epochs=4)
        for t in tr_sys:
            t.close()
        del tr_dv
        torch.cuda.synchronize()
        print(f"bench: training done: {train}", file=sys.stderr, flush=True)

    def run(precision, steps, warmup, label, mdl=None, prec_only=False, inner_op=STERN_INNER_PROJECTED):
        kw = dict(precision=precision, model=mdl, prec_only=prec_only, inner_op=inner_op)
        for w in range(warmup):
            _, info = s.apply_chi0(dv, tol=args.tol, dn_out=dn, **kw)
            print(f"bench: {label} warmup {w}: {info['n_converged']}/{info['n_solves']} converged in "
                  f"{info['wall_s']:.2f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        conv = 0
        kern = {}
        iters = []
        fallback = 0
        t0 = time.perf_counter()
        for k in range(steps):
            _, info = s.apply_chi0(dv, tol=args.tol, dn_out=dn, profile=True, **kw)
            conv += info["n_converged"]
            fallback += info["n_fallback"]
            iters.append(info["total_iters"] / max(1, info["n_solves"]))
            for name, v in info["kernels"].items():
                a = kern.setdefault(name, dict(launches=0, ms=0.0, bytes=0.0, flops=0.0))
                for f in a:
                    a[f] += v[f]
            print(f"bench: {label} step {k}: {info['n_converged']}/{info['n_solves']} converged, "
                  f"{info['wall_s']:.3f} s, max true resid {info['max_true_resid']:.2e}, "
                  f"fallback {info['n_fallback']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = dict(value=conv / dt, dt=dt, kern=kern, iters=float(np.mean(iters)), fallback=fallback)
        if label != "fp64":  # dn against the plain FP64 path at the same tolerance
            s.apply_chi0(dv, tol=args.tol, dn_out=dn, **kw)
            torch.cuda.synchronize()
            r["dn_rel_err_vs_fp64"] = ((dn - ref).reshape(n_pert, -1).norm(dim=1)
                                       / ref.reshape(n_pert, -1).norm(dim=1)).max().item()
        return r

    ref = torch.empty_like(dv)
    s.apply_chi0(dv, tol=args.tol, dn_out=ref, precision=STERN_FP64)
    torch.cuda.synchronize()
    plain = run(STERN_FP64, args.steps, args.warmup, "fp64")
    head = plain
    mixed = learned = learned_fp64 = learned_k = None
    if args.path in ("mixed", "learned-mixed"):
        mixed = run(STERN_MIXED, args.steps, args.warmup, "mixed")
        head = mixed
    if args.path == "learned-mixed":
        learned_fp64 = run(STERN_FP64, args.steps, args.warmup, "learned-fp64", model)
        learned = run(STERN_MIXED, args.steps, args.warmup, "learned-mixed", model)
        learned_k = run(STERN_MIXED, args.steps, args.warmup, "learnedK-mixed", model, prec_only=True)
        head = learned_k if learned_k["value"] > learned["value"] else learned
    value = head["value"]
    dt = head["dt"]
    kern = head["kern"]

    dom = max(kern, key=lambda n: kern[n]["ms"])
    d = kern[dom]
    per_launch_s = d["ms"] / d["launches"] / 1e3
    traffic = measured_traffic(dom, d["bytes"] / d["launches"])
    if dom in ALU_KERNELS or dom in MFMA_KERNELS:
        peak = ALU_KERNELS.get(dom) or MFMA_KERNELS[dom]
        achieved = d["flops"] / d["launches"] / per_launch_s / 1e12
        roof = dict(bound="alu" if dom in ALU_KERNELS else "mfma", achieved=achieved, peak=peak, unit="TFLOP/s",
                    frac=achieved / peak, traffic=traffic, kernel=dom,
                    hbm_GBps=d["bytes"] / d["launches"] / per_launch_s / 1e9)
    else:
        achieved = d["bytes"] / d["launches"] / per_launch_s / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel=dom)
    roof["launches"] = d["launches"]
    roof["ms_per_launch"] = d["ms"] / d["launches"]
    total_ms = sum(v["ms"] for v in kern.values())
    breakdown = {n: dict(share=round(v["ms"] / total_ms, 4), launches=v["launches"],
                         bytes_per_launch=round(v["bytes"] / v["launches"]), ms_per_launch=round(v["ms"] / v["launches"], 4),
                         GBps=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                         TFLOPs=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2) if v["flops"] > 0 else None)
                 for n, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_bands, args.tol)

    cfg = dict(workload=spec.name, L_bohr=spec.L, ecut_ry=spec.ecut, atoms=spec.n_atoms, n_pw=s.n_pw,
               grid=s.fft_n, n_occ=s.n_occ, n_pert=n_pert, solves_per_step=n_solves, tol=args.tol, autotuned=tuned,
               autotune_ms=tune_ms,
               plain_fp64=dict(solves_per_s=plain["value"], mean_cg_iters=plain["iters"]))
    if mixed is not None:
        cfg.update(path="FP32 FFT + split-BF16 MFMA GEMMs in FP64 defect correction (fallback: FP64 PCG)",
                   mixed=dict(solves_per_s=mixed["value"], mean_inner_iters=mixed["iters"],
                              fallback_solves=mixed["fallback"], dn_rel_err_vs_fp64=mixed["dn_rel_err_vs_fp64"]),
                   speedup_vs_plain_fp64=mixed["value"] / plain["value"])
        dtype = "f32+bf16/f64"
    if learned is not None:
        which = ("learned diagonal preconditioner (x0 = 0)" if head is learned_k else
                 "learned guess + learned diagonal preconditioner")
        cfg.update(path=which + " from the BF16 MFMA conv net on the coarse grid, FP32 FFT + split-BF16 MFMA GEMMs "
                            "in FP64 defect correction; Teter FP64 PCG fallback",
                   learned_fp64=dict(solves_per_s=learned_fp64["value"], mean_cg_iters=learned_fp64["iters"],
                                     fallback_solves=learned_fp64["fallback"],
                                     dn_rel_err_vs_fp64=learned_fp64["dn_rel_err_vs_fp64"]),
                   learned_mixed=dict(solves_per_s=learned["value"], mean_inner_iters=learned["iters"],
                                      fallback_solves=learned["fallback"],
                                      dn_rel_err_vs_fp64=learned["dn_rel_err_vs_fp64"]),
                   learned_k_mixed=dict(solves_per_s=learned_k["value"], mean_inner_iters=learned_k["iters"],
                                        fallback_solves=learned_k["fallback"],
                                        dn_rel_err_vs_fp64=learned_k["dn_rel_err_vs_fp64"]),
                   training=dict(cells="two other seeded mid cells (same L, Ecut, atom count)", **train),
                   speedup_vs_plain_fp64=head["value"] / plain["value"])
    if mixed is None:
        cfg.update(path="plain FP64 projected Teter-PCG")
        dtype = "f64"
    line = dict(metric="converged Sternheimer solves/s at resid≤1e-8 (learned+mixed vs plain FP64)", value=value, unit="solves/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=dt / args.steps * 1e3, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype=dtype, data="synthetic", config=cfg,
                roofline=roof, cpu_baseline=cpu, kernels=breakdown)
    s.close()
    if model is not None:
        model.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
