"""Benchmark: TOD samples x CG iterations per second for the PCG map-maker on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input that is already
resident in HBM: build the plan (hits, block-Jacobi blocks, excision, compaction, band
symbols), b = P^T N^-1 d, PCG to relative residual 1e-8, true-residual check, release.
value = n_samples * iterations / (seconds per step).

Default workload: the ground-like scan (256 detectors x 2^20 samples, intervals of 2^16,
512x512 patch, lambda = 8,192).  --config tiny runs the 4 x 65,536-sample raster instead,
--config satellite the long-band scan.  --config batched measures RHS solves/s for 64
right-hand sides sharing P and N^-1 (stacked enlarged-CG solve with a tuned block size,
against plain per-column PCG on the same GPU).
One GPU only: --gpus N with N > 1 exits with a message.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector

WORKLOADS = {
    "ground": "ground-like: 256 det x 2^20 samples (268,435,456), intervals 2^16, 512x512 patch, "
              "lambda 8192, f_knee U[0.1,2] Hz",
    "tiny": "tiny raster: 4 det x 65,536 samples, 64x64 patch, lambda 1024, f_knee 1 Hz",
    "satellite": "satellite-like: 32 det x 2^23 samples (268,435,456), intervals 2^20, 786,432 "
                 "pixels, HWP, lambda 32768, f_knee 0.05 Hz",
    "batched": "batched multi-RHS: ground-like 64 det x 2^20 samples (67,108,864), intervals "
               "2^16, 512x512 patch, lambda 8192, 64 right-hand sides sharing P and N^-1",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {
    "apply_fused": ("apply_fused.hip", "fft_lds.h", "wave_runs.h"),
    "toeplitz": ("toeplitz.hip", "fft_lds.h"),
    "toeplitz_long": ("toeplitz_long.hip", "fft_lds.h"),
    "unpoint": ("pointing.hip",),
    "point": ("pointing.hip", "wave_runs.h"),
}


def kernel_source_hash(kernel):
    """Hash of the sources a kernel is built from (a PMC summary is only valid for them)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2112_03370_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was taken on the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"HBM bytes per launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash(kernel):
        return None
    return float(m_bytes.group(1))


def make_workload(name):
    import synth
    if name == "ground":
        return synth.make_config("ground")
    if name == "tiny":
        return synth.make_config("tiny")
    if name == "satellite":
        return synth.make_config("satellite")
    if name == "batched":
        return synth.make_config("batched")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(prob, target_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: the first detectors (whole
    stationary intervals), plan + b once, then timed PCG iterations."""
    import oracle as O
    threads = len(os.sched_getaffinity(0))
    n_dets = len(prob.det_offset) - 1
    # enough detectors that pixels keep well-conditioned 3x3 blocks (one eighth of the focal
    # plane, at least 4 detectors)
    use = min(n_dets, max(4, n_dets // 8))
    s1 = int(prob.det_offset[use])
    sel = prob.blk_start + prob.blk_len <= s1
    plan = O.build_plan(prob.pix[:s1], prob.wq[:s1], prob.wu[:s1], prob.n_pix_global,
                        prob.blk_start[sel], prob.blk_len[sel], prob.blk_band[sel], prob.bands)
    b = O.rhs(plan, prob.d[0, :s1])
    t0 = time.perf_counter()
    res = O.pcg(plan, b, tol=1e-30, max_iter=1)
    one = time.perf_counter() - t0
    iters = int(max(1, min(50, target_s // max(one, 1e-3))))
    t0 = time.perf_counter()
    res = O.pcg(plan, b, tol=1e-30, max_iter=iters)
    dt = time.perf_counter() - t0
    # pcg performs one extra product for the true residual: iters + 1 products were timed
    rate = s1 * (iters + 1) / dt
    return {"value": rate, "unit": "TOD samples x CG iters/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {use} of {n_dets} detectors ({s1} samples), {iters} PCG iterations "
                      f"(+1 residual product) timed, {dt:.1f} s; scipy.fft workers={threads}, "
                      f"np.bincount single-threaded"}


def fft_flops_per_sample(pinfo):
    """FP32 flops per output sample of the overlap-save product: forward and inverse real FFTs
    of N points (2 x 2.5 N log2 N) plus the pointwise spectrum work, over L = N - 2 lambda."""
    n_fft = pinfo["fft_size"]
    L = n_fft - 2 * pinfo["lambda_max"]
    return (2 * 2.5 * n_fft * np.log2(n_fft) + 6 * n_fft) / L


def run_batched(args, prob, mm, torch, dev, stream):
    """Many right-hand sides sharing P and N^-1: solves/s of the stacked (enlarged-CG) solve with
    a tuned block size, against plain per-column PCG on the same GPU and inputs."""
    k = int(prob.d.shape[0])
    d = torch.from_numpy(prob.d).to(dev)
    torch.cuda.synchronize()
    log(f"[bench] {k} right-hand sides resident ({d.numel() * 4 / 2**30:.1f} GiB)")

    def step(block, timing=False):
        with torch.cuda.stream(stream):
            plan = mm.Plan(pix_d, wq_d, wu_d, prob.n_pix_global, prob.blk_start, prob.blk_len,
                           prob.blk_band, prob.bands, det_offset=prob.det_offset, stream=stream)
            if timing:
                plan.set_timing(True)
            x, infos = plan.pcg_solve(d, tol=args.tol, block=block, stream=stream)
            kt = {q: plan.kernel_time(q) for q in range(4)} if timing else None
            pinfo = plan.info
            plan.close()
        return x, infos, pinfo, kt

    pix_d = torch.from_numpy(prob.pix).to(dev)
    wq_d = torch.from_numpy(prob.wq).to(dev)
    wu_d = torch.from_numpy(prob.wu).to(dev)
    for w in range(args.warmup):
        _, infos, _, _ = step(args.block)
        log(f"[bench] warmup {w}: block sizes {sorted({i['block'] for i in infos})}, "
            f"iterations {min(i['iterations'] for i in infos)}..{max(i['iterations'] for i in infos)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kts, all_infos = [], []
    for q in range(args.steps):
        x, infos, pinfo, kt = step(args.block, timing=True)
        kts.append(kt)
        all_infos.append(infos)
        log(f"[bench] step {q}: block sizes {[i['block'] for i in infos][::8]}, iterations "
            f"{min(i['iterations'] for i in infos)}..{max(i['iterations'] for i in infos)}, "
            f"max true relres {max(i['true_relres'] for i in infos):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = k * args.steps / elapsed

    # plain per-column PCG over the same inputs (one pass, same tolerance)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xp, pinfos, _, _ = step(0)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    plain = k / plain_s
    diff = (x - xp).reshape(k, -1).norm(dim=1) / xp.reshape(k, -1).norm(dim=1).clamp_min(1e-300)
    max_diff = float(diff.max())
    log(f"[bench] batched {value:.2f} solves/s, plain {plain:.2f} solves/s "
        f"(plain iterations {min(i['iterations'] for i in pinfos)}.."
        f"{max(i['iterations'] for i in pinfos)}), max map rel diff {max_diff:.2e}")

    # dominant kernel: the multi-column fused product; launches carry varying column counts, so
    # the achieved rate is total work over total launch time
    tot = sum(kt[1][0] for kt in kts)
    cnt = sum(kt[1][1] for kt in kts)
    col_applies = sum(sum(i["iterations"] + 3 for i in infos) for infos in all_infos)
    n_s = prob.n_samples
    flops = fft_flops_per_sample(pinfo) * n_s * col_applies
    tflops = flops / (tot * 1e-3) / 1e12
    hbm = 12.0 * n_s * cnt / (tot * 1e-3) / 1e9
    roof = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
            "traffic": committed_traffic("apply_fused", "batched"),
            "kernel": "apply_fused", "launches": cnt, "column_applies": col_applies,
            "avg_launch_ms": round(tot / max(1, cnt), 4),
            "avg_ms_per_column_apply": round(tot / max(1, col_applies), 4),
            "pointing_hbm_gbs": round(hbm, 1), "pointing_hbm_frac": round(hbm / HBM_PEAK_GBS, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.time()
        base = cpu_baseline(prob)
        iters = float(np.mean([i["iterations"] for i in pinfos]))
        # one plain solve of the whole workload costs iters (+1 residual) products of n_s samples
        cpu = dict(base)
        cpu["value"] = base["value"] / (n_s * (iters + 1))
        cpu["unit"] = "RHS solves/s"
        cpu["sample"] = (base["sample"] + f"; solves/s = rate / ({n_s} samples x "
                         f"{iters + 1:.0f} products per plain solve)")
        log(f"[bench] cpu baseline {cpu['value']:.3e} solves/s in {time.time() - t0:.1f} s")

    per_rhs_iters = [i["iterations"] for i in all_infos[-1]]
    return {
        "metric": "batched solves/s at rel-res 1e-8",
        "value": value,
        "unit": "RHS solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 time-domain / f64 pixel-domain",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "n_samples": n_s, "n_rhs": k,
                   "tol": args.tol, "n_kept": pinfo["n_kept"], "fft_size": pinfo["fft_size"],
                   "block": args.block,
                   "block_sizes_used": sorted({i["block"] for i in all_infos[-1]}),
                   "iterations_min_max": [min(per_rhs_iters), max(per_rhs_iters)],
                   "parallelism": "single GPU"},
        "plain": {"solves_per_s": plain, "seconds": round(plain_s, 3),
                  "iterations_mean": float(np.mean([i["iterations"] for i in pinfos])),
                  "speedup": round(value / plain, 3), "max_map_rel_diff": max_diff,
                  "max_true_relres_batched": max(i["true_relres"] for i in all_infos[-1]),
                  "max_true_relres_plain": max(i["true_relres"] for i in pinfos)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="ground", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unfused", action="store_true",
                    help="three-kernel FFT path (gather / Toeplitz / scatter) instead of fused")
    ap.add_argument("--block", type=int, default=-1,
                    help="batched workload: right-hand sides per block (-1: tuned among 8/16/32)")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (for PMC scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_03370_amd import mapmaker as mm

    mm.load()
    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    prob = make_workload(args.config)
    log(f"[bench] generated {args.config}: {prob.n_samples} samples in {time.time() - t0:.1f} s")
    if args.config == "batched":
        stream = torch.cuda.Stream(device=dev)
        print(json.dumps(run_batched(args, prob, mm, torch, dev, stream)), flush=True)
        return
    pix = torch.from_numpy(prob.pix).to(dev)
    wq = torch.from_numpy(prob.wq).to(dev)
    wu = torch.from_numpy(prob.wu).to(dev)
    d = torch.from_numpy(prob.d[0]).to(dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()

    def step(timing=False):
        with torch.cuda.stream(stream):
            plan = mm.Plan(pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len,
                           prob.blk_band, prob.bands, det_offset=prob.det_offset,
                           flags=mm.FLAG_UNFUSED if args.unfused else 0, stream=stream)
            if timing:
                plan.set_timing(True)
            x, info = plan.pcg_solve(d, tol=args.tol, stream=stream)
            kt = None
            if timing:
                kt = {k: plan.kernel_time(k) for k in range(4)}
            pinfo = plan.info
            plan.close()
        return x, info, pinfo, kt

    for w in range(args.warmup):
        _, info, pinfo, _ = step()
        log(f"[bench] warmup {w}: {info['iterations']} iterations, {info['ms']:.1f} ms solve")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = []
    kts = []
    for k in range(args.steps):
        x, info, pinfo, kt = step(timing=True)
        infos.append(info)
        kts.append(kt)
        log(f"[bench] step {k}: {info['iterations']} it, relres {info['relres']:.2e}, "
            f"true {info['true_relres']:.2e}, solve {info['ms']:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1e3 * elapsed / args.steps
    iters = int(np.mean([i["iterations"] for i in infos]))
    value = prob.n_samples * iters / (elapsed / args.steps)

    # Dominant kernel and its roofline.
    n_s = prob.n_samples
    tot = {k: sum(kt[k][0] for kt in kts) for k in range(4)}
    cnt = {k: sum(kt[k][1] for kt in kts) for k in range(4)}
    fused = bool(pinfo["fused"])
    toep = "toeplitz_long" if pinfo["fft_size"] > (1 << 15) else "toeplitz"
    names = {0: "unpoint", 1: "apply_fused" if fused else toep, 2: "point", 3: "cg_vector"}
    dom = max(range(3), key=lambda k: tot[k])
    avg_ms = tot[dom] / max(1, cnt[dom])
    # algorithmic bytes per sample and launch (one launch covers n_samples): pointing is 12 B
    # (pixel int32 + two FP32 weights); time-domain vectors 4 B each
    if dom == 1 and fused:
        bytes_per_sample = 12                 # pointing read once; t and u never leave LDS
    else:
        bytes_per_sample = {0: 12 + 4, 1: 4 + 4, 2: 12 + 4}[dom]
    algo_bytes = bytes_per_sample * n_s
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
    traffic = committed_traffic(names[dom], args.config)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": names[dom], "avg_launch_ms": round(avg_ms, 4),
            "bytes_per_launch": algo_bytes}
    if dom == 1 and pinfo["toeplitz_algo"] == mm.TOEPLITZ_FFT:
        flops = n_s * fft_flops_per_sample(pinfo)
        roof["fp32_tflops"] = round(flops / (avg_ms * 1e-3) / 1e12, 2)
        roof["fp32_frac"] = round(flops / (avg_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)
    per_kernel = {names[k]: {"total_ms": round(tot[k], 2), "launches": cnt[k],
                             "avg_ms": round(tot[k] / max(1, cnt[k]), 4)} for k in range(4)}
    log(f"[bench] per-kernel (timed steps): {json.dumps(per_kernel)}")

    if args.copy_probe_gib > 0:
        nbytes = int(args.copy_probe_gib * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {nbytes} bytes read + {nbytes} bytes written per launch")

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.time()
        cpu = cpu_baseline(prob)
        log(f"[bench] cpu baseline {cpu['value']:.3e} in {time.time() - t0:.1f} s")

    out = {
        "metric": "TOD samples x CG iters/s at rel-res 1e-8",
        "value": value,
        "unit": "TOD samples x CG iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 time-domain / f64 pixel-domain",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "n_samples": n_s,
                   "iterations": iters, "tol": args.tol, "n_kept": pinfo["n_kept"],
                   "fft_size": pinfo["fft_size"], "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
