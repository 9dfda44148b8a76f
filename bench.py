"""Benchmark: ms/frame to a 1e-6 relative residual at N = 8,192 (BF16 batched
method vs FP32 plain method vs Jacobi-PCG) on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic frames:
network inference (features, encoder, both attention stacks with highways,
heads, packed factors) and PCG with the learned H-matrix preconditioner until
every frame reaches ||r|| <= 1e-6 ||b|| on a true residual, replayed as one
captured hipGraph (inference, PCG setup and first chunk of iterations; a frame
still iterating continues in chunk graphs).  Inputs (density,
right-hand side, assembled operator, weights) are resident in HBM before the
timed region; assembly is timed separately, as the paper leaves it out.

Besides the headline (20 frames of the precision workload, N = 8,192) the
JSON line carries these legs:
  * the same step on fresh frames every step (no step sees frames solved
    before), the FP32 method batched and frame by frame, Jacobi-PCG batched;
    iterations mean and standard deviation for each;
  * the largest workload (20 frames of N = 16,384): ms/frame, iterations,
    fallback rate, HBM GB/s of the PCG kernels, MFMA fraction of the GEMMs;
  * batching (64 frames of mixed N in one launch): frames/s and per-frame
    p50 / p99 latency from device-clock stamps at each frame's stop;
  * streaming: SpMV and the single-right-hand-side apply on batches whose
    algorithmic working set exceeds 1 GB (the precision frames replicated),
    in GB/s of algorithmic bytes;
  * training: one step of the training workload (32 systems of N = 4,096),
    ms per step;
  * the paper's own 2D benchmark at its five scales and rtol 1e-8: CG,
    Jacobi-PCG and the method with 2D-trained weights, ms/frame and
    iterations (the setting of the paper's Table 4);
  * cpu_baseline: the float64 oracle as it stands on the 20 headline frames,
    which also gives each GPU leg's solution error against the oracle.

Prints one JSON line.  Run with no flags for the default (1 GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_FRAMES = 20            # frames per batch (seeds 2000..2019, the precision workload)
TOL = 1e-6
PEAK_HBM_GBS = 8000.0    # MI355X HBM3E, published
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 MFMA, published


def _weights(cfg, name=None):
    from paper_2605_13343_amd import inputs
    path = os.path.join(ROOT, "paper_2605_13343_amd", "weights", name or f"trained_L{cfg.leaf}.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return {k: z[k] for k in z.files}, "trained"
    return inputs.init_weights(cfg, 7), "seeded-init"


class Inputs:
    """One batch of frames with its inputs resident in HBM."""

    def __init__(self, cfg, frames, stream, batch=None, ops=0):
        import torch
        from paper_2605_13343_amd import hp
        from paper_2605_13343_amd.train import frame_rhs
        self.frames = frames
        self.ops = ops
        self.dims = [(f.nx, f.ny, f.nz) for f in frames]
        cache = {}
        for d in self.dims:
            if d not in cache:
                cache[d] = hp.morton_order(*d)
        self.perms = [cache[d] for d in self.dims]
        self.B = batch if batch is not None else hp.Batch(cfg, self.dims, stream)
        if any(f.region is not None for f in frames):
            self.B.set_regions([f.region for f in frames])
        self.rho = torch.tensor(np.concatenate([f.rho[p] for f, p in zip(frames, self.perms)]).astype(np.float32),
                                device="cuda")
        self.b = torch.tensor(np.concatenate([frame_rhs(f, p) for f, p in zip(frames, self.perms)]).astype(np.float32),
                              device="cuda")
        self.sys = self.B.new_sys()
        self.B.assemble(self.rho, self.sys, ops)
        self.x = torch.zeros(self.B.ntot, dtype=torch.float64, device="cuda")

    def x_frames(self):
        """The solution of every frame, lexicographic cell order, float64 (host)."""
        xs = self.x.cpu().numpy()
        out = []
        for f, p in enumerate(self.perms):
            n0, n = int(self.B.n0[f]), len(p)
            v = np.empty(n)
            v[p] = xs[n0:n0 + n]
            out.append(v)
        return out


def _method_step(I, wt, fac, compute):
    """Eager form: inference, then the PCG solve (its iterations replayed from
    captured chunk graphs)."""
    from paper_2605_13343_amd import hp
    I.B.infer_factors(wt, I.rho, I.sys, fac, compute)
    I.x.zero_()
    return I.B.pcg_solve(I.sys, fac, I.b, I.x, hp.PRECOND_HMAT, fdtype=compute, tol=TOL, use_graph=True)


def _graph_step(I, wt, fac, compute):
    """One captured graph: inference, PCG setup and the first chunk of
    iterations (hp_solve_step); the same results as _method_step bit for bit.
    Needs one _method_step (or inference) of the compute type on the batch first."""
    I.x.zero_()
    return I.B.solve_step(wt, I.rho, I.sys, fac, I.b, I.x, compute, tol=TOL)


def _timed(stream, fn, steps):
    """Run fn() `steps` times between HIP events; returns (results of the
    last call, per-call ms list, mean ms)."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    res = None
    for k in range(steps):
        res = fn(k)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    return res, per, evs[0].elapsed_time(evs[-1]) / steps


def _iter_stats(res):
    it = np.array([r[0] for r in res], dtype=np.float64)
    return {"iterations_mean": round(float(it.mean()), 2), "iterations_std": round(float(it.std()), 2),
            "iterations_max": int(it.max())}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=N_FRAMES)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline, rooflines, FP32 and Jacobi legs only (no largest, batching, streaming legs)")
    ap.add_argument("--method-only", action="store_true",
                    help="time only the BF16 batched method (for counter runs under rocprofv3)")
    ap.add_argument("--streaming-only", action="store_true",
                    help="run only the streaming SpMV / apply leg (for counter runs under rocprofv3)")
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
    stream = torch.cuda.current_stream()
    wt = torch.tensor(hp.pack_weights(cfg, w), device="cuda")
    if args.calib_copy_mib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # scale the same counters of the library's kernels to HBM bytes
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.streaming_only:
        print(json.dumps({"metric": "streaming SpMV / apply (counter run)", "streaming": _streaming_leg(cfg, frames, stream)}))
        return 0

    # ---------------------------------------------------------------- batched BF16 method (headline)
    I = Inputs(cfg, frames, stream)
    B = I.B
    fac = B.new_factors(hp.HP_BF16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        B.assemble(I.rho, I.sys)
    torch.cuda.synchronize()
    assemble_ms = (time.perf_counter() - t0) / 5 * 1e3

    eager = lambda k: _method_step(I, wt, fac, hp.HP_BF16)
    step = lambda k: _graph_step(I, wt, fac, hp.HP_BF16)
    eager(0)  # tunes the GEMM tiles; the graph is captured on the first step
    for _ in range(max(args.warmup, 1)):
        step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, step_ms, ms_per_step = _timed(stream, step, args.steps)
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    x_bf16 = I.x_frames()
    iters = [r[0] for r in res]
    flags = [r[1] for r in res]
    relres = [r[2] for r in res]
    ms_frame = ms_per_step / len(frames)
    _, _, infer_ms = _timed(stream, lambda k: B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16), 3)

    if args.method_only:
        print(json.dumps({"metric": "ms/frame (BF16 batched method only; counter run)", "value": round(ms_frame, 4),
                          "unit": "ms/frame", "steps": args.steps, "iterations_mean": float(np.mean(iters)),
                          "inference_ms_per_batch": round(infer_ms, 4)}))
        return 0

    # ---------------------------------------------------------------- rooflines
    roofline = _rooflines(B, I, wt, fac, max(iters))

    # ---------------------------------------------------------------- the eager form of the step
    # the inference launched kernel by kernel on three streams, then the solve
    # (the same results bit for bit)
    eres, _, eager_ms = _timed(stream, eager, args.steps)

    # ---------------------------------------------------------------- fresh frames every step
    # the same step on a new set of frames each time (inputs uploaded and
    # assembled beforehand): no step solves frames a previous solve has seen
    # (each step copies its frames' density, right-hand side and assembled
    # system into the buffers the captured step reads: inside the timed region)
    fresh_sets = [Inputs(cfg, [inputs.make_frame("precision8192", 2100 + 20 * s + f) for f in range(len(frames))],
                         stream, batch=B) for s in range(args.steps)]
    torch.cuda.synchronize()
    fres_all = []

    def fresh_step(k):
        F = fresh_sets[k]
        I.rho.copy_(F.rho)
        I.b.copy_(F.b)
        I.sys.copy_(F.sys)
        r = _graph_step(I, wt, fac, hp.HP_BF16)
        fres_all.extend(r)
        return r

    _, _, fresh_ms = _timed(stream, fresh_step, args.steps)
    del fresh_sets

    # the headline frames back in place for the legs below
    I2 = Inputs(cfg, frames, stream, batch=B)
    I.rho.copy_(I2.rho)
    I.b.copy_(I2.b)
    I.sys.copy_(I2.sys)
    del I2

    # ---------------------------------------------------------------- FP32 method, batched
    fac32 = B.new_factors(hp.HP_F32)
    step32 = lambda k: _graph_step(I, wt, fac32, hp.HP_F32)
    _method_step(I, wt, fac32, hp.HP_F32)
    step32(0)
    res32, _, ms32 = _timed(stream, step32, 3)
    x_fp32b = I.x_frames()

    # ---------------------------------------------------------------- Jacobi-PCG, batched
    def jac_step(k):
        I.x.zero_()
        return B.pcg_solve(I.sys, None, I.b, I.x, hp.PRECOND_JACOBI, tol=TOL, use_graph=True)

    jac_step(0)
    jres, _, jac_ms = _timed(stream, jac_step, args.steps)
    x_jac = I.x_frames()

    # ---------------------------------------------------------------- FP32 plain, frame by frame
    plain, x_plain = [], []
    for f in range(len(frames)):
        I1 = Inputs(cfg, [frames[f]], stream)
        f1 = I1.B.new_factors(hp.HP_F32)
        s1 = lambda k: _graph_step(I1, wt, f1, hp.HP_F32)
        _method_step(I1, wt, f1, hp.HP_F32)
        s1(0)
        pres, _, pms = _timed(stream, s1, 3)
        plain.append((pms, pres[0][0]))
        x_plain.append(I1.x_frames()[0])
        del I1, f1
    plain_ms = float(np.mean([p[0] for p in plain]))
    plain_it = np.array([p[1] for p in plain], dtype=np.float64)

    legs = {
        "bf16_batched_ms_per_frame": round(ms_frame, 4),
        "bf16_ms_per_frame_p50_p90": [round(float(np.percentile(step_ms, q)) / len(frames), 4) for q in (50, 90)],
        "bf16_inference_ms_per_batch": round(infer_ms, 4),
        "bf16_iterations_mean": float(np.mean(iters)),
        "bf16_iterations_std": round(float(np.std(iters)), 2),
        "bf16_iterations_max": int(max(iters)),
        "bf16_converged": int(sum(1 for fl in flags if fl & hp.CONVERGED)),
        "bf16_fell_back": int(sum(1 for fl in flags if fl & hp.FELL_BACK)),
        "bf16_max_true_relres": float(max(relres)),
        "bf16_step": "one captured hipGraph per step: inference (three streams forked and joined inside the "
                     "graph), PCG setup and the first chunk of iterations (hp_solve_step)",
        "bf16_eager_ms_per_frame": round(eager_ms / len(frames), 4),
        "bf16_eager_same_results": bool([r[:2] for r in eres] == [r[:2] for r in res]),
        "bf16_fresh_frames_ms_per_frame": round(fresh_ms / len(frames), 4),
        "bf16_fresh_frames": {**_iter_stats(fres_all), "frames": len(fres_all),
                              "seeds": f"2100..{2100 + 20 * args.steps - 1}",
                              "fell_back": int(sum(1 for r in fres_all if r[1] & hp.FELL_BACK))},
        "fp32_batched_ms_per_frame": round(ms32 / len(frames), 4),
        "fp32_batched": _iter_stats(res32),
        "fp32_plain_ms_per_frame": round(plain_ms, 4),
        "fp32_plain_frames": len(plain),
        "fp32_plain_iterations_mean": round(float(plain_it.mean()), 2),
        "fp32_plain_iterations_std": round(float(plain_it.std()), 2),
        "jacobi_batched_ms_per_frame": round(jac_ms / len(frames), 4),
        "jacobi_iterations_mean": float(np.mean([r[0] for r in jres])),
        "jacobi_iterations_std": round(float(np.std([r[0] for r in jres])), 2),
        "assemble_ms_per_batch": round(assemble_ms, 4),
        "wall_ms_per_step": round(wall, 4),
    }
    autotune = B.autotune_report()
    del B, I, fac, fac32

    if not args.no_extra:
        legs["largest_16384"] = _largest_leg(cfg, wt, stream)
        legs["batching_64_mixed"] = _batching_leg(cfg, wt, stream)
        legs["streaming"] = _streaming_leg(cfg, frames, stream)
        legs["paper2d_rtol1e-8"] = _paper2d_leg(cfg, stream)
        legs["training_4096x32"] = _training_leg(cfg, stream)

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        cpu, errs = _cpu_baseline(cfg, w, frames, {"bf16_batched": x_bf16, "fp32_batched": x_fp32b,
                                                   "fp32_plain": x_plain, "jacobi_batched": x_jac})
        legs["x_error_vs_fp64_oracle"] = errs

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
        "legs": legs,
        "roofline": roofline,
        "autotune": autotune,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


def _rooflines(B, I, wt, fac, max_iters):
    """Live kernel timing (HIP events on the batch stream around every launch
    of one kernel family).  GEMMs (BF16 MFMA): every GEMM launch of one
    inference, once counting the algorithmic flops (2 M N K per launch) and
    once the algorithmic HBM bytes (X, W, bias, outputs and residual once
    each); the bound is whichever peak the work needs longer for.  PCG
    kernels (HBM): an eager 20-iteration solve with every frame active, each
    k_update_hmat / k_spmv_p launch timed, algorithmic bytes per launch as the
    library header states."""
    from paper_2605_13343_amd import hp
    B.profile_enable("gemm")
    B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16)
    n_gemm, gemm_ms, gemm_flops = B.profile_read()
    B.profile_enable("gemm_bytes")
    B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16)
    n_gemm_b, gemm_ms_b, gemm_bytes = B.profile_read()
    B.profile_enable("none")
    gemm_tf = gemm_flops / (gemm_ms * 1e-3) / 1e12
    gemm_gbs = gemm_bytes / (gemm_ms_b * 1e-3) / 1e9
    hbm_bound = gemm_bytes / (PEAK_HBM_GBS * 1e9) >= gemm_flops / (PEAK_BF16_TFLOPS * 1e12)
    gemm_kernel = "k_gemm_dl<..> / k_gemm_bt<..> / k_gemm<bf16> and k_ffn_fused (MFMA 32x32x16, FP32 accumulation)"
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
    # the fused FFN kernels alone (part of the family above; the GEMM family's
    # figures include them)
    B.profile_enable("ffn")
    B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16)
    n_ffn, ffn_ms, ffn_flops = B.profile_read()
    B.profile_enable("ffn_bytes")
    B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16)
    _, ffn_ms_b, ffn_bytes = B.profile_read()
    B.profile_enable("none")
    ffn_roof = None
    if n_ffn > 0:
        ffn_tf = ffn_flops / (ffn_ms * 1e-3) / 1e12
        ffn_gbs = ffn_bytes / (ffn_ms_b * 1e-3) / 1e9
        ffn_hbm = ffn_bytes / (PEAK_HBM_GBS * 1e9) >= ffn_flops / (PEAK_BF16_TFLOPS * 1e12)
        ffn_common = {"traffic": None, "kernel": "k_ffn_fused (FFN1 + GELU + FFN2 + residual, MFMA 32x32x16)",
                      "launches": n_ffn, "avg_launch_us": round(ffn_ms * 1e3 / n_ffn, 2),
                      "ms_per_inference": round(ffn_ms, 4), "flops_per_inference": ffn_flops,
                      "bytes_per_inference": ffn_bytes, "tflops": round(ffn_tf, 2),
                      "mfma_frac": round(ffn_tf / PEAK_BF16_TFLOPS, 4), "hbm_frac": round(ffn_gbs / PEAK_HBM_GBS, 4)}
        ffn_roof = ({"bound": "hbm", "achieved": round(ffn_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(ffn_gbs / PEAK_HBM_GBS, 4), **ffn_common} if ffn_hbm else
                    {"bound": "mfma", "achieved": round(ffn_tf, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ffn_tf / PEAK_BF16_TFLOPS, 4), **ffn_common})
    pcg_roofs = _pcg_rooflines(B, I, fac)
    # the dominant kernel of a step by time: the fused FFN (ms per inference),
    # the other GEMM launches together, or the update kernel over the step's
    # iterations
    upd_ms_step = pcg_roofs["update"]["avg_launch_us"] * 1e-3 * float(max_iters)
    for r in [gemm_roof] + list(pcg_roofs.values()):
        r["traffic"] = _traffic(r["kernel"])
    if ffn_roof:
        ffn_roof["traffic"] = _traffic(ffn_roof["kernel"])
    cands = [(upd_ms_step, pcg_roofs["update"]), (gemm_ms - (ffn_ms if ffn_roof else 0.0), gemm_roof)]
    if ffn_roof:
        cands.append((ffn_ms, ffn_roof))
    roofline = dict(max(cands, key=lambda c: c[0])[1])
    roofline["others"] = {"gemm": gemm_roof, "pcg_update": pcg_roofs["update"], "pcg_spmv": pcg_roofs["spmv"]}
    if ffn_roof:
        roofline["others"]["ffn_fused"] = ffn_roof
    roofline["others"] = {k: v for k, v in roofline["others"].items() if v["kernel"] != roofline["kernel"]}
    return roofline


def _pcg_rooflines(B, I, fac, kname_update="k_update_hmat<64, 16, bf16>"):
    from paper_2605_13343_amd import hp
    out = {}
    for fam, kname in (("update", kname_update), ("spmv", "k_spmv_p<false>")):
        I.x.zero_()
        B.profile_enable(fam)
        # one chunk of exactly 20 iterations, every frame active throughout
        B.pcg_solve(I.sys, fac, I.b, I.x, hp.PRECOND_HMAT, fdtype=hp.HP_BF16, tol=0.0, max_iter=20, fallback=False,
                    use_graph=False, chunk=20, stagnation=False, raise_on_fail=False)
        n_l, l_ms, l_bytes = B.profile_read()
        B.profile_enable("none")
        assert n_l == 20, f"{fam}: {n_l} timed launches for a 20-iteration solve"
        gbs = l_bytes / (l_ms * 1e-3) / 1e9
        out[fam] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None, "kernel": kname, "launches": n_l,
                    "avg_launch_us": round(l_ms * 1e3 / max(n_l, 1), 2), "bytes_per_launch": l_bytes / max(n_l, 1)}
    return out


def _largest_leg(cfg, wt, stream):
    """20 frames of N = 16,384 (heavy bottom half plus 16 spheres), BF16
    inference and apply, fallback enabled."""
    from paper_2605_13343_amd import hp, inputs
    frames = [inputs.make_frame("largest16384", 5000 + f) for f in range(20)]
    I = Inputs(cfg, frames, stream)
    fac = I.B.new_factors(hp.HP_BF16)
    st = lambda k: _graph_step(I, wt, fac, hp.HP_BF16)
    _method_step(I, wt, fac, hp.HP_BF16)
    st(0)
    st(0)
    res, _, ms = _timed(stream, st, 3)
    _, _, inf = _timed(stream, lambda k: I.B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16), 2)
    I.B.profile_enable("gemm")
    I.B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16)
    n_g, g_ms, g_fl = I.B.profile_read()
    I.B.profile_enable("none")
    pr = _pcg_rooflines(I.B, I, fac)
    return {"ms_per_frame": round(ms / len(frames), 4), "inference_ms_per_batch": round(inf, 4), **_iter_stats(res),
            "fallback_rate": sum(1 for r in res if r[1] & hp.FELL_BACK) / len(res),
            "converged": sum(1 for r in res if r[1] & hp.CONVERGED),
            "max_true_relres": float(max(r[2] for r in res)),
            "gemm_mfma_frac": round(g_fl / (g_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS, 4),
            "gemm_ms_per_inference": round(g_ms, 4),
            "pcg_update_gbs": pr["update"]["achieved"], "pcg_update_us": pr["update"]["avg_launch_us"],
            "pcg_spmv_gbs": pr["spmv"]["achieved"], "pcg_spmv_us": pr["spmv"]["avg_launch_us"],
            "frames": len(frames), "n": 16384, "seeds": "5000..5019"}


def _paper2d_leg(cfg, stream, scales=(1024, 2048, 4096, 8192, 16384), trunc=(2048, 8192)):
    """The paper's own benchmark (Sec. 7.1, Table 4's setting): 20 test frames
    per scale (seeds 21000..21019) of the 2D barrier generator, the zero-flux
    operator, relative residual 1e-8.  Per scale: unpreconditioned CG and
    Jacobi-PCG (no stagnation check; graph-replayed chunks) and the method
    with the 2D-trained weights (BF16 inference and apply, the captured step,
    fallback on).  ms/frame of batched solves over the 20 frames.  The
    "trunc_<N>" rows take the paper's own grid for N (W x H close to square,
    cut to the first N cells in Morton order) as padded frames in the
    smallest power-of-two box; the residual is that of the whole box, whose
    padding rows are decoupled, so the frame's own residual is at most it."""
    import torch
    from paper_2605_13343_amd import hp, inputs
    w, kind = _weights(cfg, f"trained_paper2d_L{cfg.leaf}.npz")
    wt = torch.tensor(hp.pack_weights(cfg, w), device="cuda")
    out = {"weights": kind, "rtol": 1e-8, "frames_per_scale": 20, "seeds": "21000..21019"}
    runs = [(str(n), f"paper2d_{n}") for n in scales] + [(f"trunc_{n}", f"paper2d_trunc_{n}") for n in trunc]
    for key, recipe in runs:
        frames = [inputs.make_frame(recipe, 21000 + f) for f in range(20)]
        I = Inputs(cfg, frames, stream, ops=hp.ASM_PAPER)
        row = {}
        if frames[0].region is not None:
            W, H, _, cells = frames[0].region
            row["grid"] = f"{W}x{H} cut to {cells} cells, in a {frames[0].nx}x{frames[0].ny} box"
        for name, pc in (("cg", hp.PRECOND_NONE), ("jacobi", hp.PRECOND_JACOBI)):
            def solve(k, pc=pc):
                I.x.zero_()
                return I.B.pcg_solve(I.sys, None, I.b, I.x, pc, tol=1e-8, max_iter=20000, stagnation=False,
                                     use_graph=True)
            solve(0)
            res, _, ms = _timed(stream, solve, 2)
            row[name] = {"ms_per_frame": round(ms / len(frames), 4), **_iter_stats(res),
                         "converged": sum(1 for r in res if r[1] & hp.CONVERGED)}
        fac = I.B.new_factors(hp.HP_BF16)
        I.B.infer_factors(wt, I.rho, I.sys, fac, hp.HP_BF16)

        def ours(k):
            I.x.zero_()
            return I.B.solve_step(wt, I.rho, I.sys, fac, I.b, I.x, hp.HP_BF16, tol=1e-8, max_iter=20000)
        ours(0)
        res, _, ms = _timed(stream, ours, 3)
        row["ours_bf16"] = {"ms_per_frame": round(ms / len(frames), 4), **_iter_stats(res),
                            "converged": sum(1 for r in res if r[1] & hp.CONVERGED),
                            "fell_back": sum(1 for r in res if r[1] & hp.FELL_BACK),
                            "max_true_relres": float(max(r[2] for r in res))}
        out[key] = row
        del I, fac
    return out


def _training_leg(cfg, stream, steps: int = 5):
    """One training step of the training workload (32 systems of N = 4,096,
    16 Rademacher probes each, BF16 compute, FP32 master weights, AdamW):
    hp_train_step (probe smoothing, forward with saves, cosine-Hutchinson
    loss, reverse pass with per-layer recomputation, AdamW) on resident
    inputs, ms per step over `steps` steps after one warm-up step."""
    import torch
    from paper_2605_13343_amd import hp, inputs
    frames = [inputs.make_frame("train4096", 3_000_000 + i) for i in range(32)]
    I = Inputs(cfg, frames, stream)
    w = inputs.init_weights(cfg, 7)
    flat = torch.tensor(hp.pack_weights(cfg, w), device="cuda")
    grad, m, v = torch.zeros_like(flat), torch.zeros_like(flat), torch.zeros_like(flat)
    zr = torch.tensor(np.concatenate([inputs.rademacher(4096, 16, 3_000_000 + i + 7_000_000) for i in range(32)]),
                      device="cuda")
    losses = []

    def step(k):
        lo, gn = I.B.train_step(flat, grad, m, v, I.rho, I.sys, zr, k + 1, hp.HP_BF16, lr=2e-4)
        losses.append(lo)
        return lo

    step(0)
    _, per, ms = _timed(stream, lambda k: step(k + 1), steps)
    return {"ms_per_step": round(ms, 3), "systems_per_step": 32, "n": 4096, "probes": 16,
            "ms_per_step_min": round(min(per), 3), "steps_timed": steps,
            "note": "seeded initialisation, the same batch every step; the step drains the stream for its loss"}


def _batching_leg(cfg, wt, stream):
    """64 frames with N drawn from {1,024, 2,048, 4,096, 8,192} in one batch:
    every kernel of the inference and of the PCG covers all 64 frames in one
    launch.  Per-frame latency = the frame's stop (device clock, stamped by
    the frame's lead thread) minus the step's start."""
    from paper_2605_13343_amd import hp, inputs
    frames = [inputs.make_frame("batch_mixed", 4000 + f) for f in range(64)]
    I = Inputs(cfg, frames, stream)
    fac = I.B.new_factors(hp.HP_BF16)
    st = lambda k: _graph_step(I, wt, fac, hp.HP_BF16)
    _method_step(I, wt, fac, hp.HP_BF16)
    st(0)
    st(0)
    res, per, ms = _timed(stream, st, 3)
    stop, t_solve = I.B.frame_times()
    return {"frames_per_s": round(len(frames) / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
            "latency_ms_p50": round(float(np.percentile(stop, 50)), 4),
            "latency_ms_p99": round(float(np.percentile(stop, 99)), 4),
            "latency_ms_max": round(float(stop.max()), 4), "solve_start_ms": round(t_solve, 4), **_iter_stats(res),
            "fell_back": int(sum(1 for r in res if r[1] & hp.FELL_BACK)),
            "frames_by_n": {str(n): sum(1 for f in frames if f.n == n) for n in (1024, 2048, 4096, 8192)},
            "autotune": I.B.autotune_report()}


def _streaming_leg(cfg, frames, stream):
    """SpMV (q = A p) and the single-right-hand-side apply (y = M r, BF16
    factors) on batches of the precision frames replicated until the
    algorithmic working set exceeds 1 GB (well beyond the 256 MB Infinity
    Cache).  Algorithmic bytes per node: SpMV 24 (4 coefficients, p in, q
    out); apply 208 (G 2 L^2 / L = 128, Ut and Vt 4 L_s = 64, r, y, lam and
    1/A_ii 16), BF16 factors."""
    import torch
    from paper_2605_13343_amd import hp
    out = {}
    for kind, reps, bpn in (("spmv", 256, 24.0), ("apply", 32, 208.0)):
        fr = [f for _ in range(reps) for f in frames]
        I = Inputs(cfg, fr, stream)
        n = I.B.ntot
        g = torch.Generator(device="cuda").manual_seed(3)
        p = torch.randn(n, device="cuda", generator=g)
        q = torch.empty_like(p)
        if kind == "spmv":
            fn = lambda k: I.B.spmv(I.sys, p, q)
        else:
            fac = I.B.new_factors(hp.HP_BF16)
            v = I.B.factor_views(fac, hp.HP_BF16)
            for name in ("G", "B", "Ut", "Vt"):
                v[name].copy_((torch.randn(v[name].shape, device="cuda", generator=g) * 0.05).to(torch.bfloat16))
            v["lam"].uniform_(0.2, 1.0, generator=g)
            fn = lambda k: I.B.apply(I.sys, fac, hp.HP_BF16, p, q)
        fn(0)
        torch.cuda.synchronize()
        _, per, ms = _timed(stream, fn, 10)
        work = bpn * n
        out[kind] = {"nodes": n, "frames": len(fr), "algorithmic_bytes": work,
                     "ms_per_call": round(ms, 4), "gbs": round(work / (ms * 1e-3) / 1e9, 1),
                     "frac_of_hbm_peak": round(work / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        del I, p, q
        torch.cuda.empty_cache()
    return out


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


def _cpu_baseline(cfg, w, frames, gpu_x):
    """The oracle (float64, as it stands) on the headline frames: network
    forward, factors, then PCG with the chain apply to 1e-6, timed per frame
    (system setup not counted).  The oracle's solutions then give each GPU
    leg's error: max over frames of ||x_gpu - x_oracle|| / ||x_oracle||, with
    the oracle's Jacobi-PCG as the reference of the Jacobi leg."""
    import torch
    from oracle import grid, hmatrix, network, pcg
    nthreads = torch.get_num_threads()
    t_inf = t_pcg = 0.0
    ks = []
    xo, xj = [], []
    for fr in frames:
        fs = network.FrameSys(fr.nx, fr.ny, fr.nz, fr.rho.astype(np.float32).astype(np.float64), cfg.leaf, cfg.rank)
        t0 = time.perf_counter()
        with torch.no_grad():
            f = network.forward(cfg, {k: np.asarray(v, np.float64) for k, v in w.items()}, fs)
        G = hmatrix.gram(f["F"]).numpy()
        Bm = hmatrix.coupling(f["U"], f["V"]).numpy()
        Ut, Vt, lam = f["Ut"].numpy(), f["Vt"].numpy(), f["lam"].numpy()
        t1 = time.perf_counter()
        perm = grid.morton_perm(fr.nx, fr.ny, fr.nz)
        b = fr.b.astype(np.float32).astype(np.float64)[perm]
        M = lambda v: hmatrix.apply(fs.part, G, Bm, Ut, Vt, lam, fs.diagA, v)
        x, k, fl, _ = pcg.pcg(fs.A, b, M, tol=TOL)
        t2 = time.perf_counter()
        t_inf += t1 - t0
        t_pcg += t2 - t1
        ks.append(k)
        xl = np.empty(fr.n)
        xl[perm] = x
        xo.append(xl)
        xjj, _, _, _ = pcg.pcg(fs.A, b, pcg.jacobi(fs.A), tol=TOL)
        xl = np.empty(fr.n)
        xl[perm] = xjj
        xj.append(xl)
    nf = len(frames)
    ms = (t_inf + t_pcg) * 1e3 / nf
    err = lambda xs, ref: float(max(np.linalg.norm(a - r) / np.linalg.norm(r) for a, r in zip(xs, ref)))
    errs = {k: err(v, xj if k == "jacobi_batched" else xo) for k, v in gpu_x.items()}
    errs["reference"] = ("oracle float64 method solve (same weights) to 1e-6; oracle Jacobi-PCG for the Jacobi leg; "
                         f"max over {nf} frames")
    cpu = {"value": round(ms, 2), "unit": "ms/frame", "cores": int(nthreads), "kind": "oracle",
           "sample": f"{nf} frames (seeds 2000..{2000 + nf - 1}) of the headline workload, float64 forward "
                     f"{t_inf * 1e3 / nf:.0f} ms + PCG {t_pcg * 1e3 / nf:.0f} ms per frame "
                     f"({np.mean(ks):.1f} iterations mean); system setup not counted"}
    return cpu, errs


if __name__ == "__main__":
    sys.exit(main())
