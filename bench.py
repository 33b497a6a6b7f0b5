"""Throughput of the wavelet-compressed DAMAS path on one MI355X.

Headline workload (the benchmarked configuration): a 64-mic five-arm
log-spiral array of radius 0.6 m, a 41 x 41 scan grid on a 2 x 2 m plane
1.5 m away, 64 frequency bins over 1-8 kHz, 5 uncorrelated sources, CSMs
averaged over 1024 complex-Gaussian snapshots at 20 dB SNR; each bin keeps
the 20 % of grid points with the largest wavelet detail (S~ = 337) and runs
1000 Gauss-Seidel sweeps with A stored in float.  A step is one whole solve
of all 64 bins: DAS map, selection, layout, steering rows, PSF build and
sweeps, all on the GPU, with inputs already resident in HBM.

Prints one JSON line.  Beyond the throughput keys:
  latency_ms     p50 / p99 of the per-step solve time (HIP events)
  plain          the same solve as one launch per step per bin
  roofline       the sweep kernel's algorithmic A bytes over its measured
                 launch time (HIP events recorded by the library on the
                 solve's stream), against HBM peak
  cpu_baseline   the FP64 oracle on the host, on a bounded sample of bins,
                 and the GPU result's relative L2 error against it
  variants       the other workloads at their full sizes (plain FP64 on a
                 21 x 21 grid; BF16 storage with FP32 refinement on 81 x 81,
                 32 bins; uneven compressed grids over 256 bins), each with
                 throughput, latency and the roofline of its sweeps and, for
                 BF16, of the PSF build on the bf16 matrix cores; and the
                 served workload (Poisson arrivals on the request server) with
                 p50/p99 latency and updates/s at the specified and at a
                 sustainable rate.

--workload NAME measures one workload alone (compressed, plain, precision,
batched, served) and prints its record as the line; --workload copy runs one
1 GiB device-to-device copy, the calibration of the HBM byte counters.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DAMAS grid-point updates/s + p50/p99 solve latency, batched vs plain"
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP64_MFMA_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gs_traffic.json")
GS_SOURCE = os.path.join(ROOT, "paper_1608_05179_amd", "csrc", "gs.hip")


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="per-bin (plain) solves timed for the comparison; 0 skips them")
    ap.add_argument("--cpu-bins", type=int, default=64,
                    help="bins of the workload the oracle solves for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--workload", default=None,
                    choices=["compressed", "plain", "precision", "batched", "served",
                             "csm", "copy"])
    ap.add_argument("--refine", type=int, default=60,
                    help="FP32 refinement sweeps of the precision workload")
    ap.add_argument("--tune-sweeps", type=int, default=20,
                    help="sweeps per autotuner trial before a variant is timed (0: no tuning)")
    return ap.parse_args()


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def _traffic():
    """HBM bytes per sweep launch from the committed counter summary, if it
    was taken on the current sweep kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    src = hashlib.sha256(open(GS_SOURCE, "rb").read()).hexdigest()
    if t.get("gs_source_sha256") != src:
        return None
    return t.get("hbm_bytes_per_launch")


def _workload(name, refine):
    """(synthetic workload, select mode, precision, refine sweeps, label)."""
    from paper_1608_05179_amd import damas as dm
    from paper_1608_05179_amd import synth
    if name == "compressed":
        w = synth.compressed_fp32(keep_frac=0.2)
        return (w, dm.SEL_KEEP_COUNT, dm.PREC_FP32, 0,
                "compressed-fp32: M=64 spiral, 41x41 grid, 64 bins 1-8 kHz, keep 20% "
                "(S~=337), 1000 sweeps, A stored f32")
    if name == "plain":
        w = synth.plain_fp64()
        return (w, dm.SEL_KEEP_ALL, dm.PREC_FP64, 0,
                "plain-fp64: M=16 disc, 21x21 grid (S=441), 1 bin 4 kHz, exact CSM, "
                "500 sweeps, A stored f64")
    if name == "precision":
        w = synth.precision_bf16(refine_sweeps=refine)
        return (w, dm.SEL_KEEP_ALL, dm.PREC_BF16, refine,
                f"precision-bf16: M=64 spiral, 81x81 grid (S=6561), 32 bins 2-10 kHz, "
                f"keep all, 1000 sweeps: {1000 - refine} on bf16 A + {refine} on f32 A")
    w = synth.batched_fp32()
    return (w, dm.SEL_KEEP_COUNT, dm.PREC_FP32, 0,
            "batched-fp32: M=128 disc, 101x101 grid, 256 bins 0.5-12 kHz, keep "
            "U{300..4000} per bin, 2000 sweeps, A stored f32")


def measure(name, steps, warmup, plain_steps, refine=60, psf_kernel_time=False,
            tune_sweeps=0):
    """Time `steps` batched solves of a workload; returns its record."""
    import numpy as np
    import torch

    from paper_1608_05179_amd import damas as dm

    w, mode, prec, R, label = _workload(name, refine)
    dev = torch.device("cuda:0")
    I = w.iterations
    K = None
    if mode == dm.SEL_KEEP_COUNT:
        K = [int(v) for v in w.keep_counts] if w.keep_counts is not None else int(w.keep_count)
    mic = torch.tensor(w.mic, dtype=torch.float64, device=dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = torch.tensor(w.freqs, dtype=torch.float64, device=dev)
    csm = torch.view_as_real(torch.tensor(w.csm, dtype=torch.complex128)).contiguous().to(dev)
    xt = torch.float64 if prec == dm.PREC_FP64 else torch.float32
    x = torch.empty(w.n_bins, w.S, dtype=xt, device=dev)
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
    ctx = dm.Context(0)
    stream = torch.cuda.current_stream()

    def step(batched=True):
        ctx.solve(g, freq, csm, select_mode=mode, keep_count=K, iterations=I,
                  precision=prec, batched=batched, refine_sweeps=R, x_map=x, s_tilde=st,
                  idx=idx)

    tune = None
    if tune_sweeps > 0:
        # Set-up, not timed: the schedule autotuner on this problem.
        tune = ctx.autotune(g, freq, csm, select_mode=mode, keep_count=K, precision=prec,
                            trial_sweeps=tune_sweeps)
    for _ in range(warmup):
        step()
    ctx.check()
    s_tilde = st.cpu().numpy().astype(np.int64)
    updates = int(s_tilde.sum()) * I

    ctx.set_timing(True)
    ctx.phase_time(dm.PHASE_SWEEPS)
    ctx.phase_time(dm.PHASE_SYSTEM)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.check()
    gs_ms, gs_n = ctx.phase_time(dm.PHASE_SWEEPS)
    sys_ms, sys_n = ctx.phase_time(dm.PHASE_SYSTEM)
    ctx.set_timing(False)
    wg = ctx.last_workgroups()
    lat = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_step = wall * 1e3 / steps

    # Sweeps: S~^2 elements of A per sweep per bin, at the storage width
    # (bf16 bulk sweeps and f32 refinement sweeps for the precision path).
    sq = int((s_tilde * s_tilde).sum())
    if prec == dm.PREC_FP64:
        a_bytes, a_kind = sq * I * 8, "f64"
    elif prec == dm.PREC_FP32:
        a_bytes, a_kind = sq * I * 4, "f32"
    else:
        a_bytes, a_kind = sq * ((I - R) * 2 + R * 4), "bf16+f32"
    gs_avg = gs_ms / max(gs_n, 1)
    achieved = a_bytes / (gs_avg * 1e-3) / 1e9
    rec = {
        "workload": label, "bins": w.n_bins, "iterations": I,
        "s_tilde_min": int(s_tilde.min()), "s_tilde_max": int(s_tilde.max()),
        "updates_per_step": updates,
        "value": round(updates / (ms_step * 1e-3), 1), "unit": "grid-point updates/s",
        "ms_per_step": round(ms_step, 4),
        "latency_ms": {"p50": round(_pct(lat, 50), 4), "p99": round(_pct(lat, 99), 4)},
        "sweeps_ms": round(gs_avg, 4), "system_build_ms": round(sys_ms / max(sys_n, 1), 4),
        "sweep_workgroups": wg,
        "autotune": tune,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "kernel": f"gs_kernel (A {a_kind})", "kernel_avg_ms": round(gs_avg, 4),
                     "algorithmic_bytes": a_bytes},
    }

    if plain_steps > 0:
        step(batched=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            step(batched=False)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3 / plain_steps
        ctx.check()
        rec["plain"] = {"value": round(updates / (plain_ms * 1e-3), 1),
                        "ms_per_step": round(plain_ms, 3),
                        "batched_speedup": round(plain_ms / ms_step, 2)}

    if psf_kernel_time and prec == dm.PREC_BF16:
        # The bf16 PSF kernel alone (step-level call on the same kept sets),
        # timed with events on the stream it is launched on.
        mk = int(s_tilde.max())
        E16 = dm.steer_bf16(g, freq, idx, st, mk)
        off = dm.layout(st, mk)
        A16 = dm.psf_bf16(w.M, st, mk, E16, off)
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dm.psf_bf16(w.M, st, mk, E16, off, A=A16)
        e1.record(stream)
        torch.cuda.synchronize()
        psf_ms = e0.elapsed_time(e1) / reps
        ent = int(sum(v * (v + 1) // 2 for v in s_tilde))   # distinct entries
        flops = ent * 8 * w.M                                # 8M flops per entry
        wbytes = sq * 2                                      # both triangles, bf16
        tf = flops / (psf_ms * 1e-3) / 1e12
        rec["psf_bf16"] = {"bound": "mfma", "achieved": round(tf, 2),
                           "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(tf / BF16_MFMA_PEAK_TFLOPS, 4),
                           "kernel_avg_ms": round(psf_ms, 4), "algorithmic_flops": flops,
                           "write_GBs": round(wbytes / (psf_ms * 1e-3) / 1e9, 1),
                           "write_frac_of_hbm": round(wbytes / (psf_ms * 1e-3) / 1e9
                                                      / HBM_PEAK_GBS, 4)}
        del A16, E16
    elif psf_kernel_time:
        # The PSF kernel of a float or double A alone (f64 MFMA on the
        # steering rows), on the same kept sets, timed on its stream.
        mk = int(s_tilde.max())
        E = dm.steer(g, freq, idx, st, mk)
        off = dm.layout(st, mk)
        Ap = dm.psf(w.M, st, mk, prec, E, off)
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dm.psf(w.M, st, mk, prec, E, off, A=Ap)
        e1.record(stream)
        torch.cuda.synchronize()
        psf_ms = e0.elapsed_time(e1) / reps
        ent = int(sum(v * (v + 1) // 2 for v in s_tilde))   # distinct entries
        flops = ent * 8 * w.M                                # 8M flops per entry
        tf = flops / (psf_ms * 1e-3) / 1e12
        rec["psf_f64_mfma"] = {"bound": "mfma", "achieved": round(tf, 2),
                               "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4),
                               "kernel": f"psf_kernel (A {a_kind})",
                               "kernel_avg_ms": round(psf_ms, 4), "algorithmic_flops": flops}
        del Ap, E
    ctx.close()
    return rec, w, x, st


def measure_served(n_pool=24, n_trace=40, rate=200.0, n_sustained=16, slots=4):
    """The served workload: requests arrive as a Poisson process and run on
    the request server (footprint admission, PSF cache, `slots` concurrent
    streams).  Two traces: the specified arrival rate (oversubscribed, so
    latency is mostly queueing), then a sustainable rate of 0.6 x the
    completion rate the first trace measured.  Requests are drawn in turn
    from a pool of distinct synthetic scenes, so repeats can hit the cache."""
    import numpy as np

    from paper_1608_05179_amd import damas as dm
    from paper_1608_05179_amd import synth

    pool = [synth.served_request(i) for i in range(n_pool)]
    srv = dm.Server(device=0, hbm_budget=200 << 30, cache_budget=48 << 30, slots=slots,
                    max_queue=4096)

    def submit(w):
        return srv.submit(w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.freqs, w.csm,
                          select_mode=dm.SEL_KEEP_COUNT, keep_count=w.keep_count,
                          iterations=w.iterations, precision=dm.PREC_FP32)

    def trace(lam, n, seed):
        rng = np.random.default_rng(np.random.SeedSequence([5, 100 + seed]))
        arrive = np.cumsum(rng.exponential(1.0 / lam, size=n))
        t0 = time.perf_counter()
        sub = []
        for i in range(n):
            delay = t0 + arrive[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            w = pool[(seed * 7 + i) % n_pool]
            sub.append((submit(w), w))
        lat, upd, hits = [], 0, 0
        for t, w in sub:
            _, st, info = srv.wait(t)
            lat.append(info["total_ms"])
            upd += int(st.sum()) * w.iterations
            hits += info["cache_hit"]
        wall = time.perf_counter() - t0
        return {"offered_req_s": lam, "requests": n,
                "completed_req_s": round(n / wall, 3),
                "value": round(upd / wall, 1), "unit": "grid-point updates/s",
                "latency_ms": {"p50": round(_pct(lat, 50), 1), "p99": round(_pct(lat, 99), 1)},
                "cache_hits": hits, "wall_s": round(wall, 2)}

    # one warm request so library set-up is not in the first latency
    srv.wait(submit(pool[0]))
    spec = trace(rate, n_trace, 0)
    lam_s = max(0.6 * spec["completed_req_s"], 0.05)
    sus = trace(lam_s, n_sustained, 1)
    stats = srv.stats()
    srv.close()
    return {"workload": f"served: Poisson arrivals, pool of {n_pool} requests (M=64 spiral, "
                        "N 41-101, 1-64 bins of the 1-8 kHz table, K 200-6000, 1000 sweeps, "
                        f"f32), {slots} stream slots",
            "specified_rate": spec, "sustainable_rate": sus,
            "cache": {"hits": stats["cache_hits"], "misses": stats["cache_misses"]}}


def measure_csm(steps=5, warmup=1):
    """The cross-spectral-matrix step (Eq. (1)) at the batched workload's
    shape: 256 bins x 2048 snapshots x 128 microphones, FP64."""
    import torch

    from paper_1608_05179_amd import damas as dm
    nb, K, M = 256, 2048, 128
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(1608)
    snap = torch.randn(nb, K, M, 2, dtype=torch.float64, device="cuda:0", generator=gen)
    out = torch.empty(nb, M, M, dtype=torch.complex128, device="cuda:0")
    for _ in range(warmup):
        dm.csm(snap, out=out)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        dm.csm(snap, out=out)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)[steps // 2]
    # Algorithmic work: the M (M + 1) / 2 entries of the Hermitian matrix,
    # 8 real flops per complex multiply-add per snapshot.
    flops = nb * K * (M * (M + 1) // 2) * 8
    tf = flops / (ms * 1e-3) / 1e12
    del snap, out
    torch.cuda.empty_cache()
    return {"workload": f"csm-fp64: {nb} bins x {K} snapshots x {M} mics, Eq. (1) on the "
                        "FP64 matrix cores", "ms_per_step": round(ms, 4),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2),
                         "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4),
                         "kernel": "csm_kernel", "kernel_avg_ms": round(ms, 4),
                         "algorithmic_flops": flops,
                         "input_GBs": round(nb * K * M * 16 / (ms * 1e-3) / 1e9, 1)}}


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(bins shard across GPUs with no exchange, but only the one-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch  # noqa: F401

    if args.workload == "copy":
        # Counter calibration: one device-to-device copy of 1 GiB (a plain
        # copy kernel of known size; FETCH_SIZE and WRITE_SIZE should read
        # 1 GiB each).
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes": src.numel() * 4}), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(measure_served()), flush=True)
        return
    if args.workload == "csm":
        print(json.dumps(measure_csm()), flush=True)
        return
    if args.workload is not None:
        rec, _, _, _ = measure(args.workload, args.steps, args.warmup, args.plain_steps,
                               refine=args.refine, psf_kernel_time=True,
                               tune_sweeps=args.tune_sweeps)
        print(json.dumps(rec), flush=True)
        return

    rec, w, x, st = measure("compressed", args.steps, args.warmup, args.plain_steps,
                            psf_kernel_time=True)
    rec["roofline"]["traffic"] = _traffic()
    out = {
        "metric": METRIC, "value": rec["value"], "unit": rec["unit"],
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "dtype_detail": "A stored f32, partial strip sums f32; residuals, x and row updates f64",
        "config": {"workload": rec["workload"], "bins": rec["bins"],
                   "s_tilde": rec["s_tilde_max"], "iterations": rec["iterations"],
                   "a_storage": "f32", "updates_per_step": rec["updates_per_step"]},
        "latency_ms": rec["latency_ms"],
        "roofline": rec["roofline"],
    }
    if "plain" in rec:
        out["plain"] = rec["plain"]
    if "psf_f64_mfma" in rec:
        out["psf_f64_mfma"] = rec["psf_f64_mfma"]

    # ---- CPU baseline: the oracle on a bounded sample of bins ------------
    if not args.no_cpu:
        import oracle
        oracle.build()
        og = oracle.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
        nb = min(args.cpu_bins, w.n_bins)
        bins = np.linspace(0, w.n_bins - 1, nb).round().astype(int)
        xg = x.double().cpu().numpy()
        worst = 0.0
        t0 = time.perf_counter()
        refs = []
        for f in bins:
            refs.append(oracle.solve_bin(og, w.freqs[f], w.csm[f], oracle.SEL_KEEP_COUNT,
                                         keep_count=w.keep_count, iters=w.iterations))
        cpu_t = time.perf_counter() - t0
        for f, r in zip(bins, refs):
            worst = max(worst, float(np.linalg.norm(xg[f] - r["x"]) / np.linalg.norm(r["x"])))
        cpu_updates = sum(len(r["idx"]) for r in refs) * w.iterations
        out["cpu_baseline"] = {"value": round(cpu_updates / cpu_t, 1),
                               "unit": "grid-point updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"{nb} of {w.n_bins} bins, whole path per bin, "
                                         f"{cpu_t:.1f} s single-threaded FP64 C",
                               "gpu_max_rel_l2_vs_oracle": float(f"{worst:.3e}")}

    # ---- the other workloads at full size ---------------------------------
    if not args.no_variants:
        out["variants"] = {}
        for name, steps in (("plain", 5), ("precision", 2), ("batched", 2)):
            v, _, _, _ = measure(name, steps, 1, 0, refine=args.refine,
                                 psf_kernel_time=True, tune_sweeps=args.tune_sweeps)
            out["variants"][name] = v
            torch.cuda.empty_cache()
        out["variants"]["served"] = measure_served()
        out["variants"]["csm"] = measure_csm()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
