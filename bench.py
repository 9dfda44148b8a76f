"""Benchmark: ms/frame to a 1e-6 relative residual at N = 8,192 (BF16 batched
method vs FP32 plain method vs Jacobi-PCG) on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic frames:
network inference (features, encoder, both attention stacks with highways,
heads, packed factors) and PCG with the learned H-matrix preconditioner until
every frame reaches ||r|| <= 1e-6 ||b|| on a true residual.  Inputs (density,
right-hand side, assembled operator, weights) are resident in HBM before the
timed region; assembly is timed separately, as the paper leaves it out.

Prints one JSON line.  Run with no flags for the default (1 GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_FRAMES = 20            # frames per batch (seeds 2000..2019, the precision workload)
GRID = (32, 16, 16)      # N = 8,192
TOL = 1e-6
PEAK_HBM_GBS = 8000.0    # MI355X HBM3E, published
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 MFMA, published


def _weights(cfg):
    from paper_2605_13343_amd import hp, inputs
    path = os.path.join(ROOT, "paper_2605_13343_amd", "weights", f"trained_L{cfg.leaf}.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return {k: z[k] for k in z.files}, "trained"
    return inputs.init_weights(cfg, 7), "seeded-init"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=N_FRAMES)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--method-only", action="store_true",
                    help="time only the BF16 batched method (for counter runs under rocprofv3)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU design is "
                                   "documented but not built (frames shard with no communication)"}))
        return 2

    import torch
    from paper_2605_13343_amd import hp, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    hp.lib()  # fails loudly if the HIP library is missing
    cfg = inputs.MODEL_DEFAULT
    w, wkind = _weights(cfg)
    frames = [inputs.make_frame("precision8192", 2000 + f) for f in range(args.frames)]
    dims = [(f.nx, f.ny, f.nz) for f in frames]
    perms = [hp.morton_order(*d) for d in dims]
    stream = torch.cuda.current_stream()

    def upload(fs, ps):
        rho = torch.tensor(np.concatenate([f.rho[p] for f, p in zip(fs, ps)]).astype(np.float32), device="cuda")
        b = torch.tensor(np.concatenate([f.b[p] for f, p in zip(fs, ps)]).astype(np.float32), device="cuda")
        return rho, b

    wt = torch.tensor(hp.pack_weights(cfg, w), device="cuda")
    if args.calib_copy_mib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # scale the same counters of the library's kernels to HBM bytes
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------------------------------------------------------- batched BF16 method
    B = hp.Batch(cfg, dims, stream)
    rho, b = upload(frames, perms)
    sys_ = B.new_sys()
    fac = B.new_factors(hp.HP_BF16)
    x = torch.zeros(B.ntot, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        B.assemble(rho, sys_)
    torch.cuda.synchronize()
    assemble_ms = (time.perf_counter() - t0) / 5 * 1e3

    def step():
        B.infer_factors(wt, rho, sys_, fac, hp.HP_BF16)
        x.zero_()
        return B.pcg_solve(sys_, fac, b, x, hp.PRECOND_HMAT, fdtype=hp.HP_BF16, tol=TOL, use_graph=True)

    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        res = step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    ms_per_step = evs[0].elapsed_time(evs[-1]) / args.steps
    iters = [r[0] for r in res]
    flags = [r[1] for r in res]
    relres = [r[2] for r in res]
    ms_frame = ms_per_step / len(frames)
    # inference share
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        B.infer_factors(wt, rho, sys_, fac, hp.HP_BF16)
    e1.record(stream)
    torch.cuda.synchronize()
    infer_ms = e0.elapsed_time(e1) / 3

    if args.method_only:
        print(json.dumps({"metric": "ms/frame (BF16 batched method only; counter run)", "value": round(ms_frame, 4),
                          "unit": "ms/frame", "steps": args.steps, "iterations_mean": float(np.mean(iters)),
                          "inference_ms_per_batch": round(infer_ms, 4)}))
        return 0

    # ---------------------------------------------------------------- rooflines
    # GEMMs (BF16 MFMA): every GEMM launch of one inference, timed with HIP
    # events on the batch stream, once counting the algorithmic flops (2 M N K
    # per launch) and once the algorithmic HBM bytes (X, W, bias, outputs and
    # residual once each).  The bound is whichever peak the work needs longer
    # for; at these shapes (K <= 512, N <= 512, M ~ 10^5) that is HBM.
    B.profile_enable("gemm")
    B.infer_factors(wt, rho, sys_, fac, hp.HP_BF16)
    n_gemm, gemm_ms, gemm_flops = B.profile_read()
    B.profile_enable("gemm_bytes")
    B.infer_factors(wt, rho, sys_, fac, hp.HP_BF16)
    n_gemm_b, gemm_ms_b, gemm_bytes = B.profile_read()
    B.profile_enable("none")
    gemm_tf = gemm_flops / (gemm_ms * 1e-3) / 1e12
    gemm_gbs = gemm_bytes / (gemm_ms_b * 1e-3) / 1e9
    hbm_bound = gemm_bytes / (PEAK_HBM_GBS * 1e9) >= gemm_flops / (PEAK_BF16_TFLOPS * 1e12)
    gemm_kernel = "k_gemm_dl<..> / k_gemm_bt<..> / k_gemm<bf16> (MFMA 32x32x16, FP32 accumulation)"
    gemm_common = {"traffic": None, "kernel": gemm_kernel, "launches": n_gemm,
                   "avg_launch_us": round(gemm_ms * 1e3 / max(n_gemm, 1), 2), "ms_per_inference": round(gemm_ms, 4),
                   "flops_per_inference": gemm_flops, "bytes_per_inference": gemm_bytes,
                   "tflops": round(gemm_tf, 2), "mfma_frac": round(gemm_tf / PEAK_BF16_TFLOPS, 4)}
    if hbm_bound:
        gemm_roof = {"bound": "hbm", "achieved": round(gemm_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gemm_gbs / PEAK_HBM_GBS, 4), **gemm_common}
    else:
        gemm_roof = {"bound": "mfma", "achieved": round(gemm_tf, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(gemm_tf / PEAK_BF16_TFLOPS, 4), **gemm_common}
    # PCG kernels (HBM): an eager 20-iteration solve with every frame active,
    # each k_update_hmat / k_spmv_p launch timed with HIP events; algorithmic
    # bytes per launch as stated in the library header.
    pcg_roofs = {}
    for fam, kname in (("update", "k_update_hmat<64, 16, bf16>"), ("spmv", "k_spmv_p<false>")):
        x.zero_()
        B.profile_enable(fam)
        B.pcg_solve(sys_, fac, b, x, hp.PRECOND_HMAT, fdtype=hp.HP_BF16, tol=0.0, max_iter=20, fallback=False,
                    use_graph=False, stagnation=False, raise_on_fail=False)
        n_l, l_ms, l_bytes = B.profile_read()
        B.profile_enable("none")
        gbs = l_bytes / (l_ms * 1e-3) / 1e9
        pcg_roofs[fam] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None, "kernel": kname, "launches": n_l,
                          "avg_launch_us": round(l_ms * 1e3 / max(n_l, 1), 2),
                          "bytes_per_launch": l_bytes / max(n_l, 1)}
    # the dominant kernel of a step: GEMM time per inference against the
    # update kernel's time over the step's iterations
    upd_ms_step = pcg_roofs["update"]["avg_launch_us"] * 1e-3 * float(np.max(iters))
    for r in [gemm_roof] + list(pcg_roofs.values()):
        r["traffic"] = _traffic(r["kernel"])
    roofline = dict(gemm_roof) if gemm_ms >= upd_ms_step else dict(pcg_roofs["update"])
    roofline["others"] = {"gemm": gemm_roof, "pcg_update": pcg_roofs["update"], "pcg_spmv": pcg_roofs["spmv"]}
    roofline["others"] = {k: v for k, v in roofline["others"].items() if v["kernel"] != roofline["kernel"]}

    # ---------------------------------------------------------------- Jacobi, batched
    def jac_step():
        x.zero_()
        return B.pcg_solve(sys_, None, b, x, hp.PRECOND_JACOBI, tol=TOL, use_graph=True)

    jac_step()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        jres = jac_step()
    e1.record(stream)
    torch.cuda.synchronize()
    jac_ms_frame = e0.elapsed_time(e1) / args.steps / len(frames)

    # ---------------------------------------------------------------- FP32 plain, frame by frame
    plain = []
    nplain = min(len(frames), 5)
    for f in range(nplain):
        B1 = hp.Batch(cfg, [dims[f]], stream)
        r1, b1 = upload([frames[f]], [perms[f]])
        s1 = B1.new_sys()
        B1.assemble(r1, s1)
        f1 = B1.new_factors(hp.HP_F32)
        x1 = torch.zeros(B1.ntot, dtype=torch.float64, device="cuda")

        def pstep():
            B1.infer_factors(wt, r1, s1, f1, hp.HP_F32)
            x1.zero_()
            return B1.pcg_solve(s1, f1, b1, x1, hp.PRECOND_HMAT, fdtype=hp.HP_F32, tol=TOL, use_graph=True)

        pstep()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(3):
            pres = pstep()
        e1.record(stream)
        torch.cuda.synchronize()
        plain.append((e0.elapsed_time(e1) / 3, pres[0][0]))
        del B1
    plain_ms = float(np.mean([p[0] for p in plain]))

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        cpu = _cpu_baseline(cfg, w, frames[0])

    out = {
        "metric": "ms/frame to 1e-6 rel. residual at N=8192: BF16 batched vs FP32 plain vs Jacobi",
        "value": round(ms_frame, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": f"precision-8192: {len(frames)} frames of a 32x16x16 grid, 8 spheres at 100:1, "
                        f"L=64, L_s=16, d=128, 4 layers, 4 heads, {wkind} weights, rtol 1e-6",
            "frames_per_batch": len(frames),
            "n": 8192,
        },
        "legs": {
            "bf16_batched_ms_per_frame": round(ms_frame, 4),
            "bf16_ms_per_frame_p50_p90": [round(float(np.percentile(step_ms, q)) / len(frames), 4) for q in (50, 90)],
            "bf16_inference_ms_per_batch": round(infer_ms, 4),
            "bf16_iterations_mean": float(np.mean(iters)),
            "bf16_iterations_max": int(max(iters)),
            "bf16_converged": int(sum(1 for fl in flags if fl & hp.CONVERGED)),
            "bf16_fell_back": int(sum(1 for fl in flags if fl & hp.FELL_BACK)),
            "bf16_max_true_relres": float(max(relres)),
            "fp32_plain_ms_per_frame": round(plain_ms, 4),
            "fp32_plain_iterations_mean": float(np.mean([p[1] for p in plain])),
            "jacobi_batched_ms_per_frame": round(jac_ms_frame, 4),
            "jacobi_iterations_mean": float(np.mean([r[0] for r in jres])),
            "assemble_ms_per_batch": round(assemble_ms, 4),
            "wall_ms_per_step": round(wall, 4),
        },
        "roofline": roofline,
        "autotune": B.autotune_report(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


def _traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/hbm_traffic_counters.txt: FETCH_SIZE and WRITE_SIZE runs of
    rocprofv3, scaled by a plain copy of known size), or None when there is
    none or when one of the kernel's source files changed since the counters
    were taken (the SHA-256 of their concatenation is recorded beside the
    figures)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_counters.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("kernel="):
            continue
        kv = dict(t.split("=", 1) for t in line.strip().split(" | "))
        if kv.get("kernel") != kernel:
            continue
        # the SHA-256 of the listed sources' bytes, concatenated in the order listed
        h = hashlib.sha256()
        for rel in kv["source"].split(","):
            src = os.path.join(ROOT, rel)
            if not os.path.exists(src):
                return None
            h.update(open(src, "rb").read())
        if h.hexdigest() != kv["source_sha256"]:
            return None
        return float(kv["hbm_bytes_per_launch"])
    return None


def _cpu_baseline(cfg, w, fr):
    """The oracle (float64, as it stands) on one frame of the same workload:
    network forward, factors, then PCG with the chain apply to 1e-6."""
    import torch
    from oracle import hmatrix, network, pcg
    from oracle import grid
    nthreads = torch.get_num_threads()
    t0 = time.perf_counter()
    fs = network.FrameSys(fr.nx, fr.ny, fr.nz, fr.rho.astype(np.float32).astype(np.float64), cfg.leaf, cfg.rank)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    with torch.no_grad():
        f = network.forward(cfg, {k: np.asarray(v, np.float64) for k, v in w.items()}, fs)
    G = hmatrix.gram(f["F"]).numpy()
    Bm = hmatrix.coupling(f["U"], f["V"]).numpy()
    Ut, Vt, lam = f["Ut"].numpy(), f["Vt"].numpy(), f["lam"].numpy()
    t_inf = time.perf_counter() - t0
    b = fr.b.astype(np.float32).astype(np.float64)[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    M = lambda v: hmatrix.apply(fs.part, G, Bm, Ut, Vt, lam, fs.diagA, v)
    t0 = time.perf_counter()
    x, k, fl, _ = pcg.pcg(fs.A, b, M, tol=TOL)
    t_pcg = time.perf_counter() - t0
    ms = (t_inf + t_pcg) * 1e3
    return {"value": round(ms, 2), "unit": "ms/frame", "cores": int(nthreads), "kind": "oracle",
            "sample": f"1 frame (seed 2000) of the same workload: float64 forward {t_inf * 1e3:.0f} ms + "
                      f"PCG {t_pcg * 1e3:.0f} ms ({k} iterations); system setup {t_setup * 1e3:.0f} ms not counted"}


if __name__ == "__main__":
    sys.exit(main())
