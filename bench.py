"""Throughput of the wavelet-compressed DAMAS path on one MI355X.

Headline workload (the benchmarked configuration, the metric's largest
single-GPU band): 128 microphones uniform in a 0.6 m disc, a 101 x 101 scan
grid on a 2 x 2 m plane 1.5 m away, 256 frequency bins over 0.5-12 kHz,
10 uncorrelated sources, CSMs averaged over 2048 complex-Gaussian snapshots
at 10 dB SNR; each bin keeps its K_f ~ U{300..4000} grid points of largest
wavelet detail and runs 2000 Gauss-Seidel sweeps, A stored in float with
the per-bin precision policy (bins whose kept points overlap most are
widened to float + bf16 residuals).  A step is one whole batched solve of
all 256 bins: DAS map, selection, layout, steering rows, PSF build with the
class choice, and the sweeps, all on the GPU, with inputs resident in HBM.

Prints one JSON line.  Beyond the throughput keys:
  latency_ms     p50 / p99 of the per-step solve time (HIP events)
  classes        bins per storage class chosen by the policy
  plain          one launch per step per bin, on a spread of sampled bins
                 (each solved alone), against the batched solve of the same
                 bins, and the whole band's plain time interpolated from them
  roofline       the sweep kernel's algorithmic A bytes over its measured
                 launch time (HIP events recorded by the library on the
                 solve's stream), against HBM peak
  cpu_baseline   the FP64 oracle on the host's cores (one process per bin)
                 on a bounded sample of bins, and the GPU result's relative
                 L2 error against it per sampled bin
  variants       the other workloads at their full sizes: the compressed
                 41 x 41 band (latency-bound: ns per serial row step), plain
                 FP64 on 21 x 21, the 81 x 81 precision band (policy, plus
                 the fixed bf16 setting as the precision trade-off, each with
                 its error against the oracle on sampled bins), the served
                 workload, the CSM step and the PSF build alone.

--workload NAME measures one workload alone (batched, compressed, plain,
precision, served, csm, psf) and prints its record as the line; --workload
copy runs one 1 GiB device-to-device copy, the calibration of the HBM byte
counters.
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
CLOCK_GHZ = 2.4
CSRC = os.path.join(ROOT, "paper_1608_05179_amd", "csrc")


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-bins", type=int, default=8,
                    help="bins of the band solved one launch per step (plain) for the "
                         "comparison; 0 skips it")
    ap.add_argument("--cpu-bins", type=int, default=16,
                    help="bins of the band the oracle solves for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--requests", type=int, default=40,
                    help="served workload: requests in the specified-rate trace")
    ap.add_argument("--sus-requests", type=int, default=16,
                    help="served workload: requests per sustainable-rate trial")
    ap.add_argument("--workload", default=None,
                    choices=["batched", "compressed", "compressed10", "compressed30", "plain", "precision", "served", "stream",
                             "csm", "psf", "copy"])
    ap.add_argument("--refine", type=int, default=60,
                    help="FP32 refinement sweeps of the precision workload")
    ap.add_argument("--tune-sweeps", type=int, default=20,
                    help="sweeps per autotuner trial before a workload is timed (0: no tuning)")
    ap.add_argument("--fixed", action="store_true",
                    help="every bin at the workload's stated precision (no per-bin policy)")
    ap.add_argument("--rho-wide", type=float, default=0.0,
                    help="widening threshold of the per-bin policy (0: the library default)")
    return ap.parse_args()


_T0 = time.perf_counter()


def _progress(msg):
    """One line per finished phase on stderr (stdout carries only the
    result line)."""
    print(f"bench.py: {msg} ({time.perf_counter() - _T0:.0f} s)", file=sys.stderr, flush=True)


def _histogram(s_tilde):
    """Kept counts per bin in 500-point classes: {"lo-hi": bins}."""
    import numpy as np
    top = int(np.ceil((int(s_tilde.max()) + 1) / 500.0)) * 500
    edges = np.arange(0, top + 1, 500)
    counts, _ = np.histogram(s_tilde, bins=edges)
    return {f"{int(a)}-{int(b) - 1}": int(c) for a, b, c in zip(edges[:-1], edges[1:], counts)
            if c}


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def sources_sha256():
    """One digest over the library's HIP sources (file names and contents,
    in name order): counters taken on other sources no longer apply."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _traffic(workload):
    """HBM bytes per sweep launch of a workload from its committed counter
    summary, if that was taken on the current library sources."""
    path = os.path.join(ROOT, "profiles", f"gs_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("sources_sha256") != sources_sha256():
        return None
    return t.get("hbm_bytes_per_launch")


_GENERATED = {}


def _workload(name, refine):
    """(synthetic workload, select mode, precision, refine sweeps, label);
    each workload is generated once per process and handed out as a copy."""
    import copy
    key = (name, refine)
    if key not in _GENERATED:
        _GENERATED[key] = _make_workload(name, refine)
    w, *rest = _GENERATED[key]
    return (copy.copy(w), *rest)


def _make_workload(name, refine):
    from paper_1608_05179_amd import damas as dm
    from paper_1608_05179_amd import synth
    if name.startswith("compressed"):
        # KEEP_FRAC p = 0.2 (the headline of this band), or 0.1 / 0.3
        p = {"compressed": 0.2, "compressed10": 0.1, "compressed30": 0.3}[name]
        w = synth.compressed_fp32(keep_frac=p)
        w.keep_frac = p
        return (w, dm.SEL_KEEP_FRAC, dm.PREC_FP32, 0,
                f"compressed-fp32: M=64 spiral, 41x41 grid, 64 bins 1-8 kHz, KEEP_FRAC {p:g} "
                f"(S~={w.keep_count}), 1000 sweeps, A stored f32")
    if name == "plain":
        w = synth.plain_fp64()
        return (w, dm.SEL_KEEP_ALL, dm.PREC_FP64, 0,
                "plain-fp64: M=16 disc, 21x21 grid (S=441), 1 bin 4 kHz, exact CSM, "
                "500 sweeps, A stored f64")
    if name == "precision":
        w = synth.precision_bf16(refine_sweeps=refine)
        return (w, dm.SEL_KEEP_ALL, dm.PREC_BF16, refine,
                f"precision-bf16: M=64 spiral, 81x81 grid (S=6561), 32 bins 2-10 kHz, "
                f"keep all, 1000 sweeps, bf16 bulk + {refine} f32 refinement sweeps where "
                f"the policy allows bf16")
    w = synth.batched_fp32()
    return (w, dm.SEL_KEEP_COUNT, dm.PREC_FP32, 0,
            "batched-fp32: M=128 disc, 101x101 grid, 256 bins 0.5-12 kHz, keep "
            "U{300..4000} per bin, 2000 sweeps, A stored f32 (ill-conditioned bins "
            "f32 + bf16 residual)")


class _Problem:
    """Device-resident inputs of a workload and a context solving it."""

    def __init__(self, name, refine, fixed=False, bins=None, rho_wide=0.0):
        import numpy as np
        import torch

        from paper_1608_05179_amd import damas as dm
        w, mode, prec, R, label = _workload(name, refine)
        if bins is not None:  # a subset of the band's bins
            w.freqs, w.csm = w.freqs[bins].copy(), w.csm[bins].copy()
            if w.keep_counts is not None:
                w.keep_counts = w.keep_counts[bins].copy()
        self.w, self.mode, self.prec, self.R, self.label = w, mode, prec, R, label
        self.policy = dm.POLICY_FIXED if fixed else dm.POLICY_AUTO
        self.rho_wide = rho_wide
        dev = torch.device("cuda:0")
        self.K = None
        self.frac = 0.0
        if mode == dm.SEL_KEEP_COUNT:
            self.K = ([int(v) for v in w.keep_counts] if w.keep_counts is not None
                      else int(w.keep_count))
        elif mode == dm.SEL_KEEP_FRAC:
            self.frac = float(w.keep_frac)
            self.K = int(w.keep_count)  # ceil(p N^2), for the oracle
        self.mic = torch.tensor(w.mic, dtype=torch.float64, device=dev)
        self.g = dm.geometry(self.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
        self.freq = torch.tensor(w.freqs, dtype=torch.float64, device=dev)
        self.csm = torch.view_as_real(
            torch.tensor(w.csm, dtype=torch.complex128)).contiguous().to(dev)
        xt = torch.float64 if prec == dm.PREC_FP64 else torch.float32
        self.x = torch.empty(w.n_bins, w.S, dtype=xt, device=dev)
        self.st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
        self.idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
        self.ctx = dm.Context(0)
        self.np = np

    def _sel(self):
        from paper_1608_05179_amd import damas as dm
        if self.mode == dm.SEL_KEEP_FRAC:
            return {"select_mode": self.mode, "keep_frac": self.frac}
        return {"select_mode": self.mode, "keep_count": self.K}

    def solve(self, batched=True):
        self.ctx.solve(self.g, self.freq, self.csm, **self._sel(),
                       iterations=self.w.iterations, precision=self.prec, batched=batched,
                       refine_sweeps=self.R, x_map=self.x, s_tilde=self.st, idx=self.idx,
                       policy=self.policy, rho_wide=self.rho_wide)

    def capture(self):
        """The same batched solve captured into a graph on this context (its
        cooperative schedule included); replays write self.x."""
        return self.ctx.capture(self.g, self.freq, self.csm, **self._sel(),
                                iterations=self.w.iterations,
                                precision=self.prec, refine_sweeps=self.R, x_map=self.x,
                                s_tilde=self.st, idx=self.idx, policy=self.policy,
                                rho_wide=self.rho_wide)

    def tune(self, sweeps):
        return self.ctx.autotune(self.g, self.freq, self.csm, **self._sel(),
                                 precision=self.prec, trial_sweeps=sweeps,
                                 policy=self.policy, rho_wide=self.rho_wide)

    def close(self):
        self.ctx.close()


def _time_steps(pb, steps, warmup):
    """Wall and HIP-event times of `steps` batched solves, with the
    library's per-phase event times (recorded on the solve's stream)."""
    import torch

    from paper_1608_05179_amd import damas as dm
    for _ in range(warmup):
        pb.solve()
    pb.ctx.check()
    stream = torch.cuda.current_stream()
    pb.ctx.set_timing(True)
    pb.ctx.phase_time(dm.PHASE_SWEEPS)
    pb.ctx.phase_time(dm.PHASE_SYSTEM)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        pb.solve()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pb.ctx.check()
    gs_ms, gs_n = pb.ctx.phase_time(dm.PHASE_SWEEPS)
    sys_ms, sys_n = pb.ctx.phase_time(dm.PHASE_SYSTEM)
    pb.ctx.set_timing(False)
    lat = [e0.elapsed_time(e1) for e0, e1 in ev]
    return wall * 1e3 / steps, lat, gs_ms / max(gs_n, 1), sys_ms / max(sys_n, 1)


def _time_graph(pb, steps, warmup):
    """The solve captured once (set-up, not timed), then `steps` replays:
    wall time per replay, HIP-event latencies, and the graph's sweep
    workgroups.  Each replay is the whole path on the resident inputs."""
    import torch
    graph = pb.capture()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        graph.launch(stream)
    torch.cuda.synchronize()
    pb.ctx.check()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        graph.launch(stream)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pb.ctx.check()
    lat = [e0.elapsed_time(e1) for e0, e1 in ev]
    wg = graph.workgroups()
    graph.close()
    return wall * 1e3 / steps, lat, wg


def _sweep_bytes(pb, s_tilde, cls):
    """Algorithmic A bytes of one solve's sweeps: S~_f^2 elements of A per
    sweep of bin f, at the width its class stores them (f64 8 B; f32 4 B;
    wide f32 + bf16 residual 6 B; bf16 bulk 2 B with the refinement sweeps
    on f32)."""
    from paper_1608_05179_amd import damas as dm
    I, R = pb.w.iterations, pb.R
    tot = 0
    for f, v in enumerate(s_tilde):
        sq = int(v) * int(v)
        c = int(cls[f]) if cls is not None else 0
        if pb.prec == dm.PREC_FP64:
            tot += sq * I * 8
        elif c == dm.CLASS_WIDE:
            tot += sq * I * 6
        elif pb.prec == dm.PREC_FP32 or c == dm.CLASS_FP32:
            tot += sq * I * 4
        else:
            tot += sq * ((I - R) * 2 + R * 4)
    return tot


def measure(name, steps, warmup, refine=60, tune_sweeps=0, fixed=False, rho_wide=0.0,
            graph=True):
    """Time `steps` batched solves of a workload, eager and (graph) as
    replays of one captured graph; returns (record, problem)."""
    import numpy as np

    from paper_1608_05179_amd import damas as dm
    pb = _Problem(name, refine, fixed, rho_wide=rho_wide)
    w = pb.w
    tune = pb.tune(tune_sweeps) if tune_sweeps > 0 else None  # set-up, not timed
    ms_step, lat, gs_avg, sys_avg = _time_steps(pb, steps, warmup)
    s_tilde = pb.st.cpu().numpy().astype(np.int64)
    cls = pb.ctx.classes(w.n_bins) if (pb.policy == dm.POLICY_AUTO and
                                       pb.prec != dm.PREC_FP64) else None
    updates = int(s_tilde.sum()) * w.iterations
    a_bytes = _sweep_bytes(pb, s_tilde, cls)
    achieved = a_bytes / (gs_avg * 1e-3) / 1e9
    rec = {
        "workload": pb.label + (" [fixed precision]" if fixed else ""),
        "bins": w.n_bins, "iterations": w.iterations,
        "s_tilde_min": int(s_tilde.min()), "s_tilde_max": int(s_tilde.max()),
        "s_tilde_histogram": _histogram(s_tilde),
        "updates_per_step": updates,
        "value": round(updates / (ms_step * 1e-3), 1), "unit": "grid-point updates/s",
        "ms_per_step": round(ms_step, 4),
        "latency_ms": {"p50": round(_pct(lat, 50), 4), "p99": round(_pct(lat, 99), 4)},
        "sweeps_ms": round(gs_avg, 4), "system_build_ms": round(sys_avg, 4),
        "sweep_workgroups": pb.ctx.last_workgroups(),
        "autotune": tune,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "kernel": "gs_coop_kernel / gs_kernel (the solve's sweep launches)",
                     "kernel_avg_ms": round(gs_avg, 4), "algorithmic_bytes": a_bytes},
    }
    if graph:
        g_ms, g_lat, g_wg = _time_graph(pb, steps, warmup)
        rec["graph"] = {"ms_per_step": round(g_ms, 4),
                        "value": round(updates / (g_ms * 1e-3), 1),
                        "latency_ms": {"p50": round(_pct(g_lat, 50), 4),
                                       "p99": round(_pct(g_lat, 99), 4)},
                        "sweep_workgroups": g_wg}
    if cls is not None:
        rec["classes"] = {"narrow": int((cls == dm.CLASS_NARROW).sum()),
                          "fp32": int((cls == dm.CLASS_FP32).sum()),
                          "wide": int((cls == dm.CLASS_WIDE).sum())}
    return rec, pb


def plain_sampled(name, nbins, warmup=1):
    """One launch per step per bin ("plain") on a spread of the band's bins
    (each solved alone, so its sweeps run on one workgroup), and the batched
    solve of the same bins; the band's plain time is interpolated from the
    per-bin times as a function of the kept count."""
    import numpy as np
    import torch

    full, _, _, _, _ = _workload(name, 60)
    n = full.n_bins
    kc = np.asarray(full.keep_counts) if full.keep_counts is not None else np.full(n, 1)
    order = np.argsort(kc, kind="stable")
    bins = sorted(set(int(order[i]) for i in np.linspace(0, n - 1, nbins).round().astype(int)))
    per = []
    for f in bins:
        pb = _Problem(name, 60, bins=[f])
        for _ in range(warmup):
            pb.solve(batched=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.solve(batched=False)
        pb.ctx.check()
        per.append((time.perf_counter() - t0) * 1e3)
        pb.close()
    pb = _Problem(name, 60, bins=bins)
    pb.solve()
    pb.ctx.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.solve()
    pb.ctx.check()
    batched_ms = (time.perf_counter() - t0) * 1e3
    pb.close()
    ks = kc[bins].astype(float)
    band_ms = float(np.interp(kc.astype(float), ks, np.asarray(per)).sum())
    return {"bins": bins, "kept": [int(v) for v in kc[bins]],
            "ms_per_bin": [round(v, 2) for v in per],
            "plain_ms_sampled_bins": round(sum(per), 2),
            "batched_ms_same_bins": round(batched_ms, 2),
            "batched_speedup_sampled": round(sum(per) / batched_ms, 2),
            "plain_ms_band_interpolated": round(band_ms, 1)}


def _oracle_worker(args):
    """One bin through the oracle (DAS map, Algorithm 1, PSF, sweeps)."""
    import numpy as np

    import oracle
    mic, N, ext, z0, c, freq, csm, mode, K, iters = args
    og = oracle.Geometry(mic, N, *ext, z0, c)
    t0 = time.perf_counter()
    r = oracle.solve_bin(og, freq, csm, mode, keep_count=K, iters=iters)
    return r["x"], len(r["idx"]), time.perf_counter() - t0, np.float64(r["margin"])


def _host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def oracle_check(pb, bins, cores=None, extra_maps=()):
    """The oracle on `bins` of a solved problem, one process per bin on up
    to `cores` host cores.  Returns (per-bin relative L2 of the GPU map
    against the oracle, oracle updates, wall seconds, cores used), and the
    same errors for each further GPU map of the same problem in
    `extra_maps`."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    oracle.build()
    w = pb.w
    cores = min(cores or _host_cores(), len(bins))
    xg = pb.x.double().cpu().numpy()
    jobs = []
    from paper_1608_05179_amd import damas as dm
    # KEEP_FRAC is KEEP_COUNT with K = ceil(p N^2) for the oracle
    mode = oracle.SEL_KEEP_COUNT if pb.mode == dm.SEL_KEEP_FRAC else pb.mode
    for f in bins:
        K = pb.K[f] if isinstance(pb.K, list) else (pb.K or 0)
        jobs.append((w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.c, float(w.freqs[f]),
                     w.csm[f], mode, int(K), w.iterations))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    def errors(x):
        return {int(f): float(f"{np.linalg.norm(x[f] - xr) / np.linalg.norm(xr):.3e}")
                for f, (xr, _, _, _) in zip(bins, res)}
    upd = sum(n for _, n, _, _ in res) * w.iterations
    if extra_maps:
        return errors(xg), upd, wall, cores, [errors(x) for x in extra_maps]
    return errors(xg), upd, wall, cores


def measure_latency_bound(name, steps, warmup, tune_sweeps):
    """A band whose systems stay in cache (the compressed workload: 64 bins
    of 337 kept, 29 MB of A; the plain workload: one bin of 441, 1.6 MB):
    each bin's sweeps are a chain of S~ I serial row steps on one
    workgroup, so the sweeps are reported as ns per row step against the
    step chain's floor, not against HBM."""
    rec, pb = measure(name, steps, warmup, tune_sweeps=tune_sweeps)
    w = pb.w
    steps_chain = int(rec["s_tilde_max"]) * w.iterations
    ns = rec["sweeps_ms"] * 1e6 / steps_chain
    rec["roofline"] = {"bound": "latency", "achieved": round(ns, 2),
                       "unit": "ns per serial row step",
                       "floor": round(29 / CLOCK_GHZ, 2),
                       "floor_basis": "bare min -> broadcast -> fma chain, about 29 cycles "
                                      "at 2.4 GHz",
                       "frac": round((29 / CLOCK_GHZ) / ns, 4),
                       "algorithmic_GBs": rec["roofline"]["achieved"],
                       "kernel_avg_ms": rec["sweeps_ms"]}
    pb.close()
    return rec


def measure_served(n_trace=40, rate=200.0, slots=4, max_batch=8, n_pool=48, n_sus=16,
                   fractions=(0.8, 0.5, 0.3), p99_over_p50=3.0, n_check=3,
                   compare_unbatched=True):
    """The served workload: requests arrive as a Poisson process and run on
    the request server (footprint admission, PSF cache, `slots` concurrent
    streams, the batch former merging up to `max_batch` compatible requests
    of any grid into one sweep launch).  Traces: the specified arrival rate
    (oversubscribed, so latency is mostly queueing), with and without the
    batch former; then the sustainable rate, defined as the highest offered
    rate, among `fractions` of the batched completion rate under overload,
    whose p99 latency stays within `p99_over_p50` times its p50.  Requests
    are drawn in turn from a pool of distinct synthetic scenes (repeats can
    hit the PSF cache when they run alone).  The oracle checks one bin of
    the `n_check` served requests with the fewest kept points."""
    import numpy as np

    import oracle
    from paper_1608_05179_amd import damas as dm
    from paper_1608_05179_amd import synth

    pool = [synth.served_request(i) for i in range(n_pool)]
    _progress(f"served: {n_pool} scenes generated")

    def submit(srv, w):
        return srv.submit(w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.freqs, w.csm,
                          select_mode=dm.SEL_KEEP_COUNT, keep_count=w.keep_count,
                          iterations=w.iterations, precision=dm.PREC_FP32)

    def trace(srv, lam, n, seed, keep=()):
        rng = np.random.default_rng(np.random.SeedSequence([5, 100 + seed]))
        arrive = np.cumsum(rng.exponential(1.0 / lam, size=n))
        s0 = srv.stats()
        t0 = time.perf_counter()
        sub = []
        for i in range(n):
            delay = t0 + arrive[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            k = (seed * 7 + i) % n_pool
            sub.append((submit(srv, pool[k]), k))
        lat, upd, hits, kept = [], 0, 0, {}
        for j, (t, k) in enumerate(sub):
            if j and j % 50 == 0:
                _progress(f"served: {j} of {n} requests done")
            x, st, info = srv.wait(t)
            if info["status"] != 0:
                raise RuntimeError(f"served request failed: {info}")
            lat.append(info["total_ms"])
            upd += int(st.sum()) * pool[k].iterations
            hits += info["cache_hit"]
            if k in keep:
                kept[k] = x
        wall = time.perf_counter() - t0
        s1 = srv.stats()
        rec = {"offered_req_s": round(lam, 3), "requests": n,
               "completed_req_s": round(n / wall, 3),
               "value": round(upd / wall, 1), "unit": "grid-point updates/s",
               "latency_ms": {"p50": round(_pct(lat, 50), 1), "p99": round(_pct(lat, 99), 1)},
               "cache_hits": hits, "batches": s1["batches"] - s0["batches"],
               "merged_requests": s1["merged"] - s0["merged"], "wall_s": round(wall, 2)}
        return rec, kept

    def server(mb):
        srv = dm.Server(device=0, hbm_budget=200 << 30, cache_budget=48 << 30, slots=slots,
                        max_queue=8192, max_batch=mb)
        srv.wait(submit(srv, pool[0]))  # library set-up outside the traces
        return srv

    # the requests the oracle checks: the fewest kept points in the trace
    in_trace = sorted({i % n_pool for i in range(n_trace)},
                      key=lambda k: int(pool[k].keep_count))
    check = in_trace[:n_check]
    out = {"workload": f"served: Poisson arrivals, pool of {n_pool} distinct requests (M=64 "
                       "spiral, N 41-101, 1-64 bins of the 1-8 kHz table, K 200-6000, 1000 "
                       f"sweeps, f32), {slots} stream slots, batch former up to {max_batch}"}
    srv = server(max_batch)
    try:
        spec, kept = trace(srv, rate, n_trace, 0, keep=set(check))
        out["specified_rate"] = spec
        _progress(f"served: {n_trace} requests at {rate:g} req/s, batched")
        mu = spec["completed_req_s"]
        tried = []
        for fr in fractions:
            r, _ = trace(srv, max(fr * mu, 0.05), n_sus, len(tried) + 1)
            r["meets"] = r["latency_ms"]["p99"] <= p99_over_p50 * r["latency_ms"]["p50"]
            tried.append(r)
            if r["meets"]:
                break
        _progress("served: sustainable-rate search")
        ok = [r for r in tried if r["meets"]]
        out["sustainable_rate"] = {
            "definition": f"highest offered rate among {list(fractions)} x the batched "
                          f"completion rate under overload whose p99 <= {p99_over_p50:g} x p50",
            "rate": ok[0] if ok else None, "tried": tried}
        st = srv.stats()
        out["cache"] = {"hits": st["cache_hits"], "misses": st["cache_misses"]}
    finally:
        srv.close()
    if compare_unbatched:
        srv = server(1)
        try:
            alone, _ = trace(srv, rate, n_trace, 0)
        finally:
            srv.close()
        out["specified_rate_unbatched"] = alone
        out["batch_former_speedup"] = round(spec["completed_req_s"] /
                                            alone["completed_req_s"], 3)
        _progress(f"served: {n_trace} requests at {rate:g} req/s, one request per launch")
    # the oracle on one bin (the last) of each checked request
    errs = {}
    for k in check:
        w, x = pool[k], kept[k]
        og = oracle.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
        f = w.n_bins - 1
        ref = oracle.solve_bin(og, w.freqs[f], w.csm[f], oracle.SEL_KEEP_COUNT,
                               keep_count=int(w.keep_count), iters=w.iterations)
        e = np.linalg.norm(x[f].astype(np.float64) - ref["x"]) / np.linalg.norm(ref["x"])
        errs[f"{w.name} bin {f}"] = float(f"{e:.3e}")
    out["oracle_rel_l2_sampled"] = errs
    _progress("served: oracle spot checks")
    return out


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


def measure_psf(reps=5):
    """The PSF build alone, step-level calls on the kept sets of two bands:
    the batched band's float A on the f64 matrix cores, and the precision
    band's bf16 A on the bf16 matrix cores (8 M flops per distinct entry;
    2 or 4 bytes stored per entry, both triangles)."""
    import numpy as np
    import torch

    from paper_1608_05179_amd import damas as dm
    out = {}
    for name, kind in (("batched", "f64"), ("precision", "bf16")):
        pb = _Problem(name, 60)
        w = pb.w
        dm.das_map(pb.g, pb.freq, pb.csm)  # warm
        b = dm.das_map(pb.g, pb.freq, pb.csm)
        if pb.mode == dm.SEL_KEEP_COUNT:
            kc = torch.tensor(pb.K, dtype=torch.int32, device="cuda:0")
            idx, st = dm.select(w.N, b, pb.mode, keep_count=kc)
        else:
            idx, st = dm.select(w.N, b, pb.mode)
        s_tilde = st.cpu().numpy().astype(np.int64)
        mk = int(s_tilde.max())
        stream = torch.cuda.current_stream()
        if kind == "bf16":
            E = dm.steer_bf16(pb.g, pb.freq, idx, st, mk)
            off = dm.layout(st, mk)
            A = dm.psf_bf16(w.M, st, mk, E, off)
            call = lambda: dm.psf_bf16(w.M, st, mk, E, off, A=A)  # noqa: E731
            peak, es = BF16_MFMA_PEAK_TFLOPS, 2
        else:
            E = dm.steer(pb.g, pb.freq, idx, st, mk)
            off = dm.layout(st, mk)
            A = dm.psf(w.M, st, mk, dm.PREC_FP32, E, off)
            call = lambda: dm.psf(w.M, st, mk, dm.PREC_FP32, E, off, A=A)  # noqa: E731
            peak, es = FP64_MFMA_PEAK_TFLOPS, 4
        call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ent = int(sum(v * (v + 1) // 2 for v in s_tilde))
        flops = ent * 8 * w.M
        wbytes = int((s_tilde * s_tilde).sum()) * es
        tf = flops / (ms * 1e-3) / 1e12
        out[f"{name}_{kind}"] = {
            "workload": f"PSF of the {name} band's kept sets ({w.n_bins} bins, S~ "
                        f"{int(s_tilde.min())}-{mk}, M={w.M}), A stored {kind if kind == 'bf16' else 'f32'}",
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": peak,
                         "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                         "kernel": "psf16_kernel" if kind == "bf16" else "psf_kernel<float>",
                         "kernel_avg_ms": round(ms, 4), "algorithmic_flops": flops},
            "write_GBs": round(wbytes / (ms * 1e-3) / 1e9, 1),
            "write_frac_of_hbm": round(wbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del A, E, off, idx, st, b
        pb.close()
        torch.cuda.empty_cache()
    return out


def measure_precision(steps, warmup, refine, tune_sweeps, check_bins=(0, 31),
                      r_counts=(1, 10, 50)):
    """The precision band under the policy and with the bf16 setting fixed
    (the precision trade-off), each with its error against the oracle on
    sampled bins (the oracle needs about a minute per 6561-unknown bin)."""
    rec_f, pb_f = measure("precision", steps, warmup, refine=refine,
                          tune_sweeps=tune_sweeps, fixed=True)
    x_fixed = pb_f.x.double().cpu().numpy()
    pb_f.close()
    # the refinement count: bf16 bulk + R FP32 sweeps, every bin at bf16
    import torch
    r_sweep, r_maps = {}, []
    for R in r_counts:
        pr = _Problem("precision", R, fixed=True)
        pr.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr.solve()
        pr.ctx.check()
        torch.cuda.synchronize()
        r_sweep[R] = {"ms_per_step": round((time.perf_counter() - t0) * 1e3, 1)}
        r_maps.append(pr.x.double().cpu().numpy())
        pr.close()
    _progress("precision: refinement-count solves")
    rec, pb = measure("precision", steps, warmup, refine=refine, tune_sweeps=tune_sweeps)
    errs, _, wall, cores, extra = oracle_check(pb, list(check_bins),
                                               extra_maps=(x_fixed, *r_maps))
    pb.close()
    note = f"bins {list(check_bins)}, {wall:.0f} s on {cores} cores"
    for r, e in ((rec, errs), (rec_f, extra[0])):
        r["oracle_rel_l2"] = e
        r["oracle_max_rel_l2"] = max(e.values())
        r["oracle_check"] = note
    for R, e in zip(r_counts, extra[1:]):
        r_sweep[R]["oracle_rel_l2"] = e
        r_sweep[R]["oracle_max_rel_l2"] = max(e.values())
    return {"policy": rec, "bf16_fixed": rec_f,
            "bf16_refine_sweeps": {"note": "every bin bf16 bulk + R FP32 sweeps of 1000, "
                                           "one timed solve each; " + note,
                                   "by_R": {str(k): v for k, v in r_sweep.items()}}}


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py: the solver path runs on one GPU; --gpus {args.gpus} is not supported "
              "(bins shard across GPUs with no exchange, but only the one-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

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
    if args.workload == "stream":
        # Achievable read bandwidth: torch's sum over 8 GiB of float32 (a
        # read stream; median of 5 HIP-event timed launches).
        x = torch.ones(1 << 31, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        ts = []
        for _ in range(6):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            x.sum()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts[1:])[2]
        print(json.dumps({"workload": "stream: torch.sum over 8 GiB of float32",
                          "ms": round(ms, 3), "read_GBs": round(x.numel() * 4 / ms / 1e6, 1)}),
              flush=True)
        return
    if args.workload == "served":
        # the one-request-per-launch comparison only on short traces
        print(json.dumps(measure_served(n_trace=args.requests, n_sus=args.sus_requests,
                                        compare_unbatched=args.requests <= 100)), flush=True)
        return
    if args.workload == "csm":
        print(json.dumps(measure_csm()), flush=True)
        return
    if args.workload == "psf":
        print(json.dumps(measure_psf()), flush=True)
        torch.cuda.synchronize()
        return
    if args.workload == "precision" and not args.fixed:
        print(json.dumps(measure_precision(args.steps, args.warmup, args.refine,
                                           args.tune_sweeps)), flush=True)
        return
    if args.workload in ("compressed", "compressed10", "compressed30", "plain"):
        print(json.dumps(measure_latency_bound(args.workload, args.steps, args.warmup,
                                               args.tune_sweeps)), flush=True)
        return
    if args.workload is not None:
        rec, pb = measure(args.workload, args.steps, args.warmup, refine=args.refine,
                          tune_sweeps=args.tune_sweeps, fixed=args.fixed,
                          rho_wide=args.rho_wide)
        pb.close()
        torch.cuda.synchronize()
        print(json.dumps(rec), flush=True)
        return

    # ---- headline: the batched band --------------------------------------
    rec, pb = measure("batched", args.steps, args.warmup, tune_sweeps=args.tune_sweeps,
                      fixed=args.fixed, rho_wide=args.rho_wide)
    _progress("batched band timed")
    rec["roofline"]["traffic"] = _traffic("batched")
    out = {
        "metric": METRIC, "value": rec["value"], "unit": rec["unit"],
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "dtype_detail": "A stored f32 (wide bins: f32 + bf16 residual, FP64 strip sums); "
                        "narrow bins' partial strip sums f32; residuals, x and row "
                        "updates f64",
        "config": {"workload": rec["workload"], "bins": rec["bins"],
                   "s_tilde_min": rec["s_tilde_min"], "s_tilde_max": rec["s_tilde_max"],
                   "iterations": rec["iterations"], "updates_per_step": rec["updates_per_step"],
                   "policy": "fixed" if args.fixed else "auto"},
        "latency_ms": rec["latency_ms"],
        "classes": rec.get("classes"),
        "sweeps_ms": rec["sweeps_ms"], "system_build_ms": rec["system_build_ms"],
        "sweep_workgroups": rec["sweep_workgroups"], "autotune": rec["autotune"],
        "graph": rec.get("graph"),
        "roofline": rec["roofline"],
    }
    w = pb.w
    # ---- CPU baseline and per-bin error: the oracle on sampled bins ------
    if not args.no_cpu:
        s_tilde = pb.st.cpu().numpy()
        nb = min(args.cpu_bins, w.n_bins)
        bins = sorted(set(np.linspace(0, w.n_bins - 1, nb).round().astype(int).tolist())
                      | {0, 1, 2})
        errs, upd, wall, cores = oracle_check(pb, bins)
        lscpu = ""
        try:
            import subprocess
            r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
            for line in r.stdout.splitlines():
                if line.startswith("Model name"):
                    lscpu = line.split(":", 1)[1].strip()
        except Exception:
            pass
        out["cpu_baseline"] = {
            "value": round(upd / wall, 1), "unit": "grid-point updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{len(bins)} of {w.n_bins} bins (0, 1, 2 and a spread; "
                      f"{int(sum(s_tilde[b] for b in bins))} kept in all), whole path per "
                      f"bin at 2000 sweeps, FP64 C, one process per bin on {cores} cores, "
                      f"{wall:.1f} s wall",
            "host_cpu": lscpu, "host_cores_visible": os.cpu_count()}
        out["oracle_rel_l2"] = errs
        out["oracle_max_rel_l2"] = max(errs.values())
        _progress("oracle on sampled bins done")
    pb.close()
    torch.cuda.empty_cache()
    if args.plain_bins > 0:
        out["plain"] = plain_sampled("batched", args.plain_bins)
        torch.cuda.empty_cache()
        _progress("plain per-bin launches timed")

    # ---- the other workloads at full size ---------------------------------
    if not args.no_variants:
        v = {}
        v["compressed"] = measure_latency_bound("compressed", 10, 2, args.tune_sweeps)
        for name in ("compressed10", "compressed30"):
            r = measure_latency_bound(name, 10, 2, args.tune_sweeps)
            v["compressed"][f"keep_frac_{name[-2:]}"] = {
                k: r[k] for k in ("workload", "s_tilde_max", "ms_per_step", "value", "roofline")}
        _progress("compressed variants")
        v["plain"] = measure_latency_bound("plain", 5, 1, 0)
        torch.cuda.empty_cache()
        _progress("plain variant")
        v["precision"] = measure_precision(2, 1, args.refine, args.tune_sweeps)
        torch.cuda.empty_cache()
        _progress("precision variant")
        v["served"] = measure_served()
        _progress("served variant")
        v["csm"] = measure_csm()
        v["psf"] = measure_psf()
        _progress("csm and psf variants")
        out["variants"] = v
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
