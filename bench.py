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
    "serving": "serving: 400 requests, Poisson arrivals at 0.8x the sequential capacity, Zipf(1.1) "
               "over 24 ground-like geometries (4-32 det x 2^16-2^18 samples, 32^2-128^2 patches, "
               "lambda 2^8-2^13), 1-4 RHS per request",
    "serving_full": "serving at full ranges: Zipf(1.1) over 100 ground-like geometries of 4-128 "
                    "det x 2^16-2^21 samples (lambda 2^8-2^13), 1-16 RHS per request, Poisson "
                    "arrivals at 0.8x the sequential capacity; geometries are contiguous ranges of "
                    "one 128 det x 2^21 sample stream, data white noise on the device; the first "
                    "--requests requests of the 2,000-request trace",
    "templates": "template map-making: ground-like 256 det x 2^20 samples (268,435,456), white "
                 "noise with per-detector sigma (diagonal weights), Legendre baselines of degree "
                 "< 3 on every 8,192-sample sweep, polynomial drifts in the data",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {
    "apply_fused": ("apply_fused.hip", "fft_lds.h", "segment_io.h", "wave_runs.h"),
    "apply_reg": ("apply_reg.hip", "fft_lds.h", "segment_io.h", "wave_runs.h"),
    "apply_long": ("toeplitz_long.hip", "fft_lds.h", "segment_io.h", "wave_runs.h"),
    "toeplitz": ("toeplitz.hip", "fft_lds.h"),
    "toeplitz_long": ("toeplitz_long.hip", "fft_lds.h"),
    "unpoint": ("pointing.hip",),
    "point": ("pointing.hip", "wave_runs.h"),
    "template_apply": ("templates.hip", "wave_runs.h"),
}


def fused_kernel(pinfo):
    """Name of the fused product kernel a plan runs: register-resident FFT (2^15-sample
    segments with at most 2^14 outputs), persistent four-step FFT (2^16 and 2^17-sample
    segments) or LDS-resident FFT."""
    return {2: "apply_reg", 3: "apply_long"}.get(pinfo["fused"], "apply_fused")


def plan_flags(args):
    from paper_2112_03370_amd import mapmaker as mm
    return (mm.FLAG_UNFUSED if getattr(args, "unfused", False) else 0) | \
        (mm.FLAG_LDS_FFT if getattr(args, "lds_fft", False) else 0)


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
    if name == "templates":
        return synth.make_templates(cfg_id=5, n_dets=256, samples_per_det=1 << 20,
                                    interval=1 << 16, side=512, dwell=16, baseline=8192,
                                    n_poly=3, name="templates")
    raise SystemExit(f"unknown workload {name}")


def plan_kwargs(args, prob):
    """Plan arguments beyond the geometry: flags, and the baselines of template workloads."""
    kw = {"flags": plan_flags(args)}
    if prob.meta.get("kind") == "templates":
        kw.update(n_poly=prob.meta["n_poly"], base_start=prob.meta["base_start"],
                  base_len=prob.meta["base_len"])
    return kw


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
    apply = None
    if prob.meta.get("kind") == "templates":
        bs, bl = prob.meta["base_start"], prob.meta["base_len"]
        keep = bs + bl <= s1
        tp = O.build_template_plan(plan, bs[keep], bl[keep], prob.meta["n_poly"])
        b = O.template_rhs(tp, prob.d[0, :s1])
        apply = lambda v: O.template_apply_A(tp, v)  # noqa: E731
    else:
        b = O.rhs(plan, prob.d[0, :s1])
    t0 = time.perf_counter()
    res = O.pcg(plan, b, tol=1e-30, max_iter=1, apply=apply)
    one = time.perf_counter() - t0
    iters = int(max(1, min(50, target_s // max(one, 1e-3))))
    t0 = time.perf_counter()
    res = O.pcg(plan, b, tol=1e-30, max_iter=iters, apply=apply)
    dt = time.perf_counter() - t0
    # pcg performs one extra product for the true residual: iters + 1 products were timed
    rate = s1 * (iters + 1) / dt
    return {"value": rate, "unit": "TOD samples x CG iters/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {use} of {n_dets} detectors ({s1} samples), {iters} PCG iterations "
                      f"(+1 residual product) timed, {dt:.1f} s; scipy.fft workers={threads}, "
                      f"np.bincount single-threaded"}


def bands_of(mm, prob):
    """The problem's band coefficients in the ABI's table layout, concatenated once per problem
    (as its pointing arrays are moved to the device once) rather than for every plan."""
    table = getattr(prob, "_abi_bands", None)
    if table is None:
        ncoef = np.array([len(b) for b in prob.bands], np.int32)
        offset = np.zeros(len(prob.bands), np.int64)
        if len(prob.bands) > 1:
            offset[1:] = np.cumsum(ncoef[:-1])
        coef = (np.concatenate([np.asarray(b, np.float32) for b in prob.bands]) if prob.bands
                else np.zeros(0, np.float32))
        table = mm.BandTable(ncoef, offset, coef)
        prob._abi_bands = table
    return table


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
                           prob.blk_band, bands_of(mm, prob), det_offset=prob.det_offset,
                           flags=plan_flags(args), stream=stream)
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

    # two-level preconditioner: deflation space from the first right-hand side (Lanczos,
    # counted in the time), then every column by PCG with M_2lvl
    two = None
    if args.defl_m > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            plan = mm.Plan(pix_d, wq_d, wu_d, prob.n_pix_global, prob.blk_start, prob.blk_len,
                           prob.blk_band, bands_of(mm, prob), det_offset=prob.det_offset,
                           flags=plan_flags(args), stream=stream)
            dinfo = plan.deflation_build(d[0], args.defl_m, stream=stream)
            x2, infos2 = plan.pcg_solve(d, tol=args.tol, precond=1, stream=stream)
            plan.close()
        torch.cuda.synchronize()
        t2 = time.perf_counter() - t0
        d2 = (x2 - xp).reshape(k, -1).norm(dim=1) / xp.reshape(k, -1).norm(dim=1).clamp_min(1e-300)
        two = {"m": args.defl_m, "rank": dinfo["rank"], "build_ms": round(dinfo["build_ms"], 1),
               "solves_per_s": k / t2, "seconds": round(t2, 3),
               "iterations_mean": float(np.mean([i["iterations"] for i in infos2])),
               "iterations_first_rhs": int(infos2[0]["iterations"]),
               "max_map_rel_diff_vs_plain": float(d2.max())}
        log(f"[bench] two-level (m={args.defl_m}): {two['solves_per_s']:.2f} solves/s, "
            f"build {two['build_ms']} ms, iterations mean {two['iterations_mean']:.1f}")
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
            "traffic": committed_traffic(fused_kernel(pinfo), "batched"),
            "kernel": fused_kernel(pinfo), "launches": cnt, "column_applies": col_applies,
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
        "two_level": two,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def run_serving(args, mm, torch, dev):
    """Continuous batching: the same request trace served by the server (n_slots solves at
    once, plans cached on the device) and by plain per-request PCG run one at a time, both
    saturated (all requests at once: capacity) and under Poisson arrivals at 0.8x the
    sequential capacity (latency from arrival to result)."""
    import threading

    import synth
    t0 = time.time()
    full = getattr(args, "config", "") == "serving_full"
    if full:
        # views of one base stream: pointing slices of one device buffer, white-noise data rows
        base, pool = synth.serving_views()
        geom, ks, gaps = synth.serving_trace(cfg_id=6, n_requests=2000, n_geoms=len(pool),
                                             k_range=(1, 16))
        n_take = min(args.requests, len(geom))
        geom, ks, gaps = geom[:n_take], ks[:n_take], gaps[:n_take]
        bpix, bwq, bwu = (torch.from_numpy(a).to(dev) for a in (base.pix, base.wq, base.wu))
        gen = torch.Generator(device=dev)
        gen.manual_seed(2112033706)
        data = torch.randn((16, base.n_samples), generator=gen, device=dev, dtype=torch.float32)
        del base
        dev_in = [dict(pix=bpix[v.s0:v.s0 + v.n_samples], wq=bwq[v.s0:v.s0 + v.n_samples],
                       wu=bwu[v.s0:v.s0 + v.n_samples], d=data[:, v.s0:v.s0 + v.n_samples])
                  for v in pool]
    else:
        pool = synth.serving_pool()
        geom, ks, gaps = synth.serving_trace()
        dev_in = []
        for p in pool:
            dev_in.append(dict(pix=torch.from_numpy(p.pix).to(dev),
                               wq=torch.from_numpy(p.wq).to(dev),
                               wu=torch.from_numpy(p.wu).to(dev), d=torch.from_numpy(p.d).to(dev)))
    n_req = len(geom)
    log(f"[bench] serving pool of {len(pool)} geometries, {n_req} requests, "
        f"generated in {time.time() - t0:.1f} s")
    used = sorted(set(int(g) for g in geom))
    # segment lengths tuned per geometry shape (the first plan of a shape times the candidates,
    # in the sizing pass below; later plans of the shape reuse the choice)
    fft = args.fft_size
    geoms = [mm.make_geometry(di["pix"], di["wq"], di["wu"], p.n_pix_global, p.blk_start,
                              p.blk_len, p.blk_band, bands_of(mm, p), p.det_offset, fft_size=fft)
             for p, di in zip(pool, dev_in)]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream(device=dev)

    # plans once, for sizes; outputs for both runs allocated up front (inputs and outputs are
    # resident before any timed region)
    n_kept = [0] * len(pool)
    for gi in used:
        p = pool[gi]
        with torch.cuda.stream(stream):
            pl = mm.Plan(dev_in[gi]["pix"], dev_in[gi]["wq"], dev_in[gi]["wu"], p.n_pix_global,
                         p.blk_start, p.blk_len, p.blk_band, bands_of(mm, p),
                         det_offset=p.det_offset, fft_size=fft, stream=stream)
        n_kept[gi] = pl.n_kept
        pl.close()
    x_seq = [torch.empty((int(ks[i]), n_kept[geom[i]], 3), dtype=torch.float64, device=dev)
             for i in range(n_req)]
    x_srv = [torch.empty_like(x) for x in x_seq]
    work = sum(pool[geom[i]].n_samples * int(ks[i]) for i in range(n_req))

    def sequential(arrivals):
        plans = {}
        lat, iters = [], 0
        t_start = time.perf_counter()
        for i in range(n_req):
            if arrivals is not None:
                t_arr = t_start + arrivals[i]
                while time.perf_counter() < t_arr:
                    time.sleep(min(1e-3, max(0.0, t_arr - time.perf_counter())))
            else:
                t_arr = t_start
            gi = int(geom[i])
            with torch.cuda.stream(stream):
                if gi not in plans:
                    p, di = pool[gi], dev_in[gi]
                    plans[gi] = mm.Plan(di["pix"], di["wq"], di["wu"], p.n_pix_global,
                                        p.blk_start, p.blk_len, p.blk_band, bands_of(mm, p),
                                        det_offset=p.det_offset, fft_size=fft, stream=stream)
                k = int(ks[i])
                _, info = plans[gi].pcg_solve(dev_in[gi]["d"][:k], x=x_seq[i], tol=args.tol,
                                              stream=stream)
            infos = info if isinstance(info, list) else [info]
            iters += sum(int(f["iterations"]) for f in infos)
            lat.append(1e3 * (time.perf_counter() - t_arr))
        total = time.perf_counter() - t_start
        for pl in plans.values():
            pl.close()
        return total, np.array(lat), iters

    def served(arrivals, n_slots, large_work=0):
        srv = mm.Server(n_slots=n_slots, large_work=large_work, large_slots=args.large_slots)
        t_arr = np.zeros(n_req)
        t_sub = np.zeros(n_req)
        tickets = [None] * n_req
        err = []
        t_start = time.perf_counter()

        def submitter():
            try:
                for i in range(n_req):
                    if arrivals is not None:
                        ta = t_start + arrivals[i]
                        while time.perf_counter() < ta:
                            time.sleep(min(1e-3, max(0.0, ta - time.perf_counter())))
                    t_arr[i] = time.perf_counter()
                    gi = int(geom[i])
                    srv.plan(gi + 1, geometry=geoms[gi][0])
                    k = int(ks[i])
                    tickets[i] = srv.submit(gi + 1, dev_in[gi]["d"][:k], x_srv[i], tol=args.tol)
                    t_sub[i] = time.perf_counter()
            except Exception as ex:  # reported by the main thread
                err.append(ex)

        th = threading.Thread(target=submitter)
        th.start()
        lat = np.zeros(n_req)
        iters = 0
        samp_iters = 0
        for i in range(n_req):
            while tickets[i] is None and not err:
                time.sleep(2e-4)
            if err:
                break
            res = srv.wait(tickets[i])
            iters += sum(int(f["iterations"]) for f in res["info"])
            # products per column: the iterations, the right-hand side and the true residual
            samp_iters += pool[geom[i]].n_samples * sum(int(f["iterations"]) + 2
                                                        for f in res["info"])
            lat[i] = 1e3 * (t_sub[i] - t_arr[i]) + res["times"]["total_ms"]
        th.join()
        if err:
            raise err[0]
        st = srv.stats()
        done_t = time.perf_counter()
        srv.close()
        return done_t - t_start, lat, iters, st, samp_iters

    # warm-up: one pass of each geometry through both paths (plan builds, graph code paths)
    for gi in used:
        with torch.cuda.stream(stream):
            p, di = pool[gi], dev_in[gi]
            pl = mm.Plan(di["pix"], di["wq"], di["wu"], p.n_pix_global, p.blk_start, p.blk_len,
                         p.blk_band, bands_of(mm, p), det_offset=p.det_offset, fft_size=fft,
                         stream=stream)
            pl.pcg_solve(di["d"][:1], tol=args.tol, stream=stream)
            pl.close()
    torch.cuda.synchronize()

    t_seq, lat_seq_sat, it_seq = sequential(None)
    cap_seq = n_req / t_seq
    log(f"[bench] sequential, saturated: {t_seq:.2f} s, {cap_seq:.1f} requests/s")
    t_srv, lat_srv_sat, it_srv, st_sat, samp_srv = served(None, args.slots, args.large_work)
    log(f"[bench] served ({args.slots} slots, large from {args.large_work} sample-RHS at most "
        f"{args.large_slots} at once), saturated: {t_srv:.2f} s, {n_req / t_srv:.1f} requests/s, "
        f"peak running {st_sat['peak_running']}, peak large {st_sat['peak_large']}")
    # same results alone and in the mix
    diffs = [float((a - b).norm() / b.norm().clamp_min(1e-300)) for a, b in zip(x_srv, x_seq)]
    max_diff = max(diffs)
    rate = args.load * cap_seq
    arrivals = np.cumsum(gaps) / rate
    t_seq_p, lat_seq, _ = sequential(arrivals)
    t_srv_p, lat_srv, _, st_p, _ = served(arrivals, args.slots, args.large_work)
    pct = lambda a, q: round(float(np.percentile(a, q)), 3)  # noqa: E731
    log(f"[bench] Poisson at {rate:.1f} requests/s: sequential p50 {pct(lat_seq, 50)} ms p99 "
        f"{pct(lat_seq, 99)} ms; served p50 {pct(lat_srv, 50)} ms p99 {pct(lat_srv, 99)} ms; "
        f"max map rel diff mix vs alone {max_diff:.2e}")
    fifo = None
    if full and args.large_work > 0:
        # the same arrivals served without size classes (one class, first come first served)
        _, lat_fifo, _, _, _ = served(arrivals, args.slots, 0)
        fifo = {"p50_ms": pct(lat_fifo, 50), "p99_ms": pct(lat_fifo, 99)}
        log(f"[bench] Poisson, served without size classes: p50 {fifo['p50_ms']} ms p99 "
            f"{fifo['p99_ms']} ms")
    n_rhs = int(ks.sum())

    cpu = None
    if not args.no_cpu_baseline and not full:
        import oracle as O
        threads = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        n_done, rhs_done = 0, 0
        refs = {}
        while n_done < n_req and time.perf_counter() - t0 < 15.0:
            gi = int(geom[n_done])
            if gi not in refs:
                refs[gi] = O.plan_from_problem(pool[gi])
            for j in range(int(ks[n_done])):
                O.pcg(refs[gi], O.rhs(refs[gi], pool[gi].d[j]), tol=args.tol)
                rhs_done += 1
            n_done += 1
        dt = time.perf_counter() - t0
        cpu = {"value": rhs_done / dt, "unit": "RHS solves/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n_done} requests of the trace ({rhs_done} RHS, plans included) "
                         f"solved one by one in {dt:.1f} s; scipy.fft workers={threads}"}
        log(f"[bench] cpu baseline {cpu['value']:.3f} RHS solves/s")

    # aggregate rate of the served saturated run against the HBM roofline: the fused product
    # reads 12 B of pointing per sample and product; kernels of several requests overlap, so
    # this is the work of the whole run over its wall time
    agg = 12.0 * samp_srv / t_srv / 1e9
    return {
        "metric": "served p50/p99 latency at rel-res 1e-8",
        "value": pct(lat_srv, 99),
        "unit": "ms (p99, arrival to result)",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(1e3 * t_srv_p, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 time-domain / f64 pixel-domain",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["serving_full" if full else "serving"],
                   "requests": n_req, "geometries_used": len(used), "rhs": n_rhs,
                   "tod_samples_x_rhs": work, "slots": args.slots, "load": args.load,
                   "arrival_rate_per_s": round(rate, 3), "tol": args.tol,
                   "fft_size": fft, "parallelism": "single GPU"},
        "served": {"p50_ms": pct(lat_srv, 50), "p99_ms": pct(lat_srv, 99),
                   "saturated_requests_per_s": round(n_req / t_srv, 3),
                   "saturated_rhs_solves_per_s": round(n_rhs / t_srv, 3),
                   "peak_running": st_sat["peak_running"], "peak_large": st_sat["peak_large"],
                   "large_work": args.large_work, "large_slots": args.large_slots,
                   "plan_hits": st_p["plan_hits"],
                   "plan_misses": st_p["plan_misses"],
                   "peak_device_bytes": st_sat["peak_bytes"]},
        "sequential": {"p50_ms": pct(lat_seq, 50), "p99_ms": pct(lat_seq, 99),
                       "saturated_requests_per_s": round(cap_seq, 3),
                       "saturated_rhs_solves_per_s": round(n_rhs / t_seq, 3)},
        "served_one_class": fifo,
        "speedup_saturated": round(t_seq / t_srv, 3),
        "max_map_rel_diff_mix_vs_alone": max_diff,
        "iterations_total": int(it_srv),
        "roofline": {"bound": "hbm", "achieved": round(agg, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(agg / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "fused products, aggregate over overlapping requests",
                     "tod_sample_products": int(samp_srv)},
        "cpu_baseline": cpu,
    }


def run_plain(args, prob, name, mm, torch, dev, steps, warmup, refine):
    """One solve per step (plan, b, PCG to recursive 1e-8, FP64 refinement when refine > 0,
    release) on one workload; TOD samples x CG iterations per second, with the dominant kernel's
    roofline and the oracle's rate on the host."""
    pix = torch.from_numpy(prob.pix).to(dev)
    wq = torch.from_numpy(prob.wq).to(dev)
    wu = torch.from_numpy(prob.wu).to(dev)
    d = torch.from_numpy(prob.d[0]).to(dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    kw = plan_kwargs(args, prob)
    phases = []

    def step(timing=False, refine_steps=refine):
        with torch.cuda.stream(stream):
            bands = bands_of(mm, prob)  # prepared once, like the resident pointing arrays
            t0 = time.perf_counter()
            plan = mm.Plan(pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len,
                           prob.blk_band, bands, det_offset=prob.det_offset, stream=stream, **kw)
            t1 = time.perf_counter()
            if timing:
                plan.set_timing(True)
            x, info = plan.pcg_solve(d, tol=args.tol, refine=refine_steps, stream=stream)
            t2 = time.perf_counter()
            kt = None
            if timing:
                kt = {k: plan.kernel_time(k) for k in range(4)}
            pinfo = plan.info
            plan.close()
            t3 = time.perf_counter()
        phases.append((t1 - t0, t2 - t1, t3 - t2))
        return x, info, pinfo, kt

    for w in range(warmup):
        _, info, pinfo, _ = step()
        log(f"[bench] {name} warmup {w}: {info['iterations']} + {info['inner_iterations']} "
            f"iterations, {info['ms']:.1f} ms solve")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = []
    kts = []
    for k in range(steps):
        x, info, pinfo, kt = step(timing=True)
        infos.append(info)
        kts.append(kt)
        log(f"[bench] {name} step {k}: {info['iterations']} + {info['inner_iterations']} it, "
            f"relres {info['relres']:.2e}, true (PCG iterate) {info['true_relres']:.2e}, FP64 true "
            f"{info['true_relres64']:.2e}, solve {info['ms']:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1e3 * elapsed / steps
    iters = float(np.mean([i["iterations"] + i["inner_iterations"] for i in infos]))
    value = prob.n_samples * iters / (elapsed / steps)

    # the same solve without refinement (outside the timed region): recursive residual only
    plain = None
    if refine > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, pi, _, _ = step(refine_steps=0)
        torch.cuda.synchronize()
        plain = {"ms_per_step": round(1e3 * (time.perf_counter() - t0), 3),
                 "iterations": pi["iterations"], "relres": pi["relres"],
                 "value": prob.n_samples * pi["iterations"] / (time.perf_counter() - t0)}

    # Dominant kernel and its roofline.
    n_s = prob.n_samples
    tot = {k: sum(kt[k][0] for kt in kts) for k in range(4)}
    cnt = {k: sum(kt[k][1] for kt in kts) for k in range(4)}
    fused = bool(pinfo["fused"])
    templates = pinfo["n_poly"] > 0
    toep = "toeplitz_long" if pinfo["fft_size"] > (1 << 15) else "toeplitz"
    names = {0: "unpoint", 1: "template_apply" if templates else (fused_kernel(pinfo) if fused else toep),
             2: "point", 3: "cg_vector"}
    dom = max(range(3), key=lambda k: tot[k])
    avg_ms = tot[dom] / max(1, cnt[dom])
    # algorithmic bytes per sample and launch (one launch covers n_samples): pointing is 12 B
    # (pixel int32 + two FP32 weights); time-domain vectors 4 B each
    if dom == 1 and (fused or templates):
        bytes_per_sample = 12                 # pointing read once; t and u stay on chip
    else:
        bytes_per_sample = {0: 12 + 4, 1: 4 + 4, 2: 12 + 4}[dom]
    algo_bytes = bytes_per_sample * n_s
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
    traffic = committed_traffic(names[dom], name) if names[dom] in KERNEL_SOURCES else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": names[dom], "avg_launch_ms": round(avg_ms, 4),
            "bytes_per_launch": algo_bytes}
    if dom == 1 and not templates and pinfo["toeplitz_algo"] == mm.TOEPLITZ_FFT:
        flops = n_s * fft_flops_per_sample(pinfo)
        roof["fp32_tflops"] = round(flops / (avg_ms * 1e-3) / 1e12, 2)
        roof["fp32_frac"] = round(flops / (avg_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)
    per_kernel = {names[k]: {"total_ms": round(tot[k], 2), "launches": cnt[k],
                             "avg_ms": round(tot[k] / max(1, cnt[k]), 4)} for k in range(4)}
    log(f"[bench] {name} per-kernel (timed steps): {json.dumps(per_kernel)}")
    ph = np.mean(np.array(phases[warmup:warmup + steps]), axis=0) * 1e3
    log(f"[bench] {name} step phases (ms): plan {ph[0]:.1f}, solve {ph[1]:.1f}, "
        f"release {ph[2]:.1f}")

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
        log(f"[bench] {name} cpu baseline {cpu['value']:.3e} in {time.time() - t0:.1f} s")

    last = infos[-1]
    return {
        "metric": "TOD samples x CG iters/s at rel-res 1e-8",
        "value": value,
        "unit": "TOD samples x CG iters/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 time-domain / f64 pixel-domain" if not templates else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[name], "n_samples": n_s,
                   "iterations": int(last["iterations"]),
                   "refine_iterations": int(last["inner_iterations"]),
                   "refine_steps": int(last["refine_steps"]), "tol": args.tol,
                   "relres_recursive": last["relres"],
                   "true_relres64": max(i["true_relres64"] for i in infos),
                   "n_kept": pinfo["n_kept"], "fft_size": pinfo["fft_size"],
                   "n_poly": pinfo["n_poly"], "parallelism": "single GPU"},
        "unrefined": plain,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def free_host():
    """Release the host arrays of a workload the caller has dropped."""
    import gc
    gc.collect()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="ground", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--refine", type=int, default=1,
                    help="FP64 refinement steps after each solve (0: recursive residual only)")
    ap.add_argument("--no-suite", action="store_true",
                    help="ground workload only: skip the satellite, template, batched and "
                         "serving sub-records")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lds-fft", action="store_true",
                    help="keep 2^15-sample segments in the LDS-resident fused kernel")
    ap.add_argument("--unfused", action="store_true",
                    help="three-kernel FFT path (gather / Toeplitz / scatter) instead of fused")
    ap.add_argument("--block", type=int, default=-1,
                    help="batched workload: right-hand sides per block (-1: tuned among 8/16/32)")
    ap.add_argument("--slots", type=int, default=8, help="serving workload: solves at once")
    ap.add_argument("--defl-m", type=int, default=64,
                    help="batched workload: Lanczos steps of the two-level preconditioner "
                         "(0: skip that comparison)")
    ap.add_argument("--fft-size", type=int, default=-1,
                    help="serving workloads: segment length of the plans (-1: tuned per shape, "
                         "0: the rule's length)")
    ap.add_argument("--large-work", type=int, default=1 << 26,
                    help="serving workloads: requests of samples x RHS from this size are large "
                         "(0: one class)")
    ap.add_argument("--large-slots", type=int, default=1,
                    help="serving workloads: large requests running at once")
    ap.add_argument("--requests", type=int, default=100,
                    help="serving_full workload: requests taken from the 2,000-request trace")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serving workload: Poisson rate as a fraction of sequential capacity")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (for PMC scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; it would shard "
              "by whole (detector, interval) blocks with one all-reduce of the pixel vector per "
              "iteration", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_03370_amd import mapmaker as mm

    mm.load()
    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    if args.config in ("serving", "serving_full"):
        print(json.dumps(run_serving(args, mm, torch, dev)), flush=True)
        return
    t0 = time.time()
    prob = make_workload(args.config)
    log(f"[bench] generated {args.config}: {prob.n_samples} samples in {time.time() - t0:.1f} s")
    if args.config == "batched":
        stream = torch.cuda.Stream(device=dev)
        print(json.dumps(run_batched(args, prob, mm, torch, dev, stream)), flush=True)
        return
    out = run_plain(args, prob, args.config, mm, torch, dev, args.steps, args.warmup, args.refine)
    del prob
    free_host()
    torch.cuda.empty_cache()

    if args.config == "ground" and not args.no_suite:
        # the other workloads, each outside the headline's timed region, with a few steps each
        sub = {}
        small = argparse.Namespace(**vars(args))
        small.steps, small.warmup = 2, 1
        for name in ("satellite", "templates"):
            t0 = time.time()
            p2 = make_workload(name)
            log(f"[bench] generated {name}: {p2.n_samples} samples in {time.time() - t0:.1f} s")
            sub[name] = run_plain(small, p2, name, mm, torch, dev, 2, 1, args.refine)
            del p2
            free_host()
            torch.cuda.empty_cache()
        t0 = time.time()
        p3 = make_workload("batched")
        log(f"[bench] generated batched: {p3.n_samples} samples x {p3.d.shape[0]} RHS in "
            f"{time.time() - t0:.1f} s")
        sub["batched"] = run_batched(small, p3, mm, torch, dev, torch.cuda.Stream(device=dev))
        del p3
        free_host()
        torch.cuda.empty_cache()
        sub["served"] = run_serving(small, mm, torch, dev)
        out["sub"] = sub
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
