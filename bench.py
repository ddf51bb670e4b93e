#!/usr/bin/env python
"""Throughput of shifted randomized (S)T-HOSVD on one MI355X.

Prints ONE JSON line. A step is one whole solve (every mode: sketch, svd,
q shifted power steps each with its svd and shift update, sign rule, core
contraction) of a tensor already resident in HBM, replayed from a HIP graph
captured once (--eager: launched call by call).

Default workload: tucker3_1000, the largest single-GPU configuration: a
1000^3 FP32 tensor (4 GB) = a rank-(50,50,50) Tucker tensor with superdiagonal
core 1/i and Haar factors, plus Gaussian noise at 1e-4 of its norm;
ST-HOSVD, ranks (50,50,50), p = 10, q = 3, adaptive shift.
Other workloads: --workload hilbert3_400 (the 400^3 smooth-function tensor
a_ijk = 1/(i+j+k-2), FP32, ranks 30, q = 3) | tucker3_60_fp64 | tucker4_120 |
sparse_cp3_600 | serving_stream_4096. --order natural | decreasing | i,j,k
sets ST-HOSVD's processing order (sparse_cp3_600 is the 600 x 700 x 800
sparse CP tensor of the paper's order study).

serving_stream_4096: 4096 order-3 FP32 requests (mode sizes U{32..256},
Tucker ranks U{4..32}, Gaussian core x Haar factors + 1e-3 noise, p = 8,
q = 1, adaptive shift). A step is one burst of all 4096 requests through the
continuous-batching server (persistent batched kernels, graph replay, a slot
pair per width class 16 / 32 / 48 / 64 of the sketch widths); value
is approximations/s over the timed bursts. Beside it: the same burst one
request at a time (tucker_rsthosvd per request), the relative error of every
request on both paths, and p50/p99 latency at Poisson arrival rates of 0.5
and 0.9 x the measured batched capacity.

The dominant kernel's roofline figure comes from HIP events the library
records around each launch of that kernel class (tucker_timing_*) during a
second timed pass of the same K steps; achieved = summed algorithmic bytes
(or flops) / summed event time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# fp32-split: FP32 products formed as six BF16 matrix-core products of
# three-piece BF16 splits, i.e. a sixth of the dense BF16 rate per FP32 flop
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp32-split": 2500.0 / 6}
METRIC = "Tucker approximations/sec at fixed rel. error; TTM HBM GB/s; p99 latency"

CONFIGS = {
    "hilbert3_400": dict(precision="fp32", variant="st", ranks=(30, 30, 30), p=10, q=3),
    "tucker3_60_fp64": dict(precision="fp64", variant="t", ranks=(10, 10, 10), p=5, q=1),
    "tucker4_120": dict(precision="bf16", variant="st", ranks=(20, 20, 20, 20), p=10, q=2),
    "tucker3_1000": dict(precision="fp32", variant="st", ranks=(50, 50, 50), p=10, q=3),
    "sparse_cp3_600": dict(precision="fp32", variant="st", ranks=(50, 50, 50), p=10, q=1),
}
SERVING = "serving_stream_4096"
SERVING_CFG = dict(count=4096, n_lo=32, n_hi=256, r_lo=4, r_hi=32, eta=1e-3, p=8, q=1, capacity=256, lclass="auto",
                   ws_bytes=4 << 30, data_seed=0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tucker3_1000", choices=sorted(CONFIGS) + [SERVING])
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "fp32", "bf16"])
    ap.add_argument("--q", type=int, default=None)
    ap.add_argument("--shift", default="adaptive", choices=["adaptive", "none"])
    ap.add_argument("--omega", default="gaussian", choices=["gaussian", "uniform", "kr_gaussian", "kr_uniform"],
                    help="test-matrix kind (section 5's comparison of random matrices)")
    ap.add_argument("--ranks", default=None, help="Tucker ranks as a comma list (default: the workload's)")
    ap.add_argument("--order", default="natural",
                    help="processing order: natural, decreasing (by mode size) or a comma list of modes")
    ap.add_argument("--eager", action="store_true",
                    help="time K eager solves; by default one solve is captured into a HIP graph and K replays are "
                         "timed (each replay is a whole solve), where capture is supported (not for Algorithm 4, "
                         "which reads a flag on the host every step, nor the concurrent T-HOSVD)")
    ap.add_argument("--fp32-products", default="split", choices=["split", "native"],
                    help="how FP32 solves form their mode products: three-piece BF16 splits on the BF16 matrix cores "
                         "(default) or FP32 matrix-core instructions only")
    ap.add_argument("--holistic", action="store_true",
                    help="the holistic variants of Appendices A / B (range finders at width l, then a small HOSVD)")
    ap.add_argument("--pve", type=float, default=None, metavar="TOL",
                    help="Algorithm 4: power count per mode by the per-vector-error test with this tol "
                         "(--q is then q_max, default 20)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "colreduce", "rowcontract", "powerstep"],
                    help="kernel class reported in the roofline object (auto: the larger summed launch time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--burst-only", action="store_true",
                    help="serving workload: time the batched bursts only (for profiler runs)")
    ap.add_argument("--serial", action="store_true",
                    help="serving workload: one batch on the device at a time (per-phase durations as in the "
                         "launch-timing pass)")
    ap.add_argument("--timing-pass-only", action="store_true",
                    help="serving workload: run only the batches of the launch-timing pass (one burst, direct steps, "
                         "one batch at a time), e.g. under a counter run")
    return ap.parse_args()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of a kernel class from the committed counter summary
    (profiles/<kernel>_<workload>_traffic.json), or None when there is none or
    the kernel source has changed since the counters were taken."""
    from paper_2506_04840_amd.pmc_traffic import source_digest
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_digest():
        return None
    return rec["traffic_bytes_per_launch"]


def copy_bandwidth(dev, nbytes=1 << 30, reps=5):
    """HBM bandwidth of a plain device-to-device copy (GB/s, read + write
    bytes), the measured ceiling a streaming kernel is compared with."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def step_percentiles(events):
    """p10 / p50 / p90 of per-step milliseconds from consecutive event pairs."""
    import numpy as np
    ms = np.array([a.elapsed_time(b) for a, b in zip(events[:-1], events[1:])])
    return {"p10": round(float(np.percentile(ms, 10)), 4), "p50": round(float(np.percentile(ms, 50)), 4),
            "p90": round(float(np.percentile(ms, 90)), 4)}


def reconstruct_torch(G, U):
    import torch
    t = G
    for k, u in enumerate(U):
        t = torch.movedim(torch.tensordot(u, t, dims=([1], [k])), 0, k)
    return t


def _order_arg(text):
    if text in ("natural", "decreasing"):
        return None if text == "natural" else text
    return tuple(int(x) for x in text.split(","))


def cpu_baseline(workload, cfg, a_host, shift, q, pve=None, omega="gaussian", order=None, holistic=False):
    """The FP64 oracle, untuned, on the host cores: one whole solve of the same
    workload when that takes seconds, else a bounded slab scaled by work."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import rhosvd as orc

    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    a = a_host
    scale = 1.0
    sample = "one whole solve (FP64 oracle) of the same tensor"
    if a.size > 1.1e9:
        # slab along the last mode: same n_1, n_2; the work of every product scales with numel
        d = a.shape[-1]
        keep = max(1, int(d * 1e9 / a.size))
        a = np.ascontiguousarray(a[..., :keep])
        scale = d / keep
        sample = "one whole solve (FP64 oracle) of the %s slab, time scaled by %.1f (numel ratio)" % (
            "x".join(map(str, a.shape)), scale)
    a64 = a.astype(np.float64)
    # the order of the full tensor (a slab keeps every mode but the last one's size)
    oo = orc.decreasing_order(a_host.shape) if order == "decreasing" else order
    t0 = time.perf_counter()
    if pve is not None:
        res = orc.randomized_sthosvd_pve(a64, cfg["ranks"], cfg["p"], q, pve, shift=shift, seed=1,
                                         variant=cfg["variant"])
    else:
        om = None
        if omega != "gaussian":
            from oracle.philox import omega_matrix
            ranks, dims, st = cfg["ranks"], a64.shape, cfg["variant"] == "st"

            seq = list(range(len(dims))) if oo is None else list(oo)

            def om(k, m, l):
                before = seq[:seq.index(k)]
                cur = [ranks[i] if (st and i in before) else dims[i] for i in range(len(dims))]
                return omega_matrix(omega, 1, k, [cur[i] for i in range(len(dims)) if i != k], l)
        fn = orc.randomized_hosvd_holistic if holistic else orc.randomized_hosvd
        res = fn(a64, cfg["ranks"], cfg["p"], q, shift=shift, variant=cfg["variant"], seed=1, omega=om, order=oo)
    dt = (time.perf_counter() - t0) * scale
    out = {"value": 1.0 / dt, "unit": "approximations/s", "cores": int(threads), "kind": "oracle",
           "sample": sample, "seconds_per_solve": dt}
    if scale == 1.0:
        out["rel_error"] = orc.rel_error(a64, res)  # the FP64 oracle's RE on the same tensor and sketch
        if pve is not None:
            out["q_used"] = list(res.qs)
    else:
        out["rel_error_slab"] = orc.rel_error(a64, res)  # the oracle's RE on the slab (outside its timing)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.workload == SERVING:
        serving_main(args)
        return
    order = _order_arg(args.order)

    import numpy as np
    import torch

    from paper_2506_04840_amd import _lib as T
    from workloads import generators as gen

    cfg = dict(CONFIGS[args.workload])
    if args.ranks is not None:
        cfg["ranks"] = tuple(int(x) for x in args.ranks.split(","))
    prec = args.precision or cfg["precision"]
    q = cfg["q"] if args.q is None else args.q
    dev = torch.device("cuda:0")
    w = gen.WORKLOADS[args.workload]

    if args.workload in ("hilbert3_400", "tucker3_60_fp64"):
        a_host = gen.make_tensor(args.workload)
        dt = torch.float64 if prec == "fp64" else torch.float32
        A = torch.from_numpy(a_host).to(dev, dtype=dt)
        a_host_store = A.double().cpu().numpy() if prec != "fp64" else a_host
    else:
        A = gen.build_on_device(args.workload, dev)
        if prec == "fp64":
            A = A.double()
        a_host_store = None

    if args.pve is not None:
        if order is not None or args.holistic:
            raise SystemExit("--pve runs Algorithm 3 in the natural order")
        q = 20 if args.q is None else args.q
        solver = T.PveSolver(A.shape, cfg["ranks"], cfg["p"], q, args.pve, args.shift, seed=w.sketch_seed,
                             precision=prec, device=dev, sequential=(cfg["variant"] == "st"))
    else:
        solver = T.Solver(A.shape, cfg["ranks"], cfg["p"], q, args.shift, seed=w.sketch_seed, precision=prec,
                          sequential=(cfg["variant"] == "st"), device=dev, omega=args.omega, order=order,
                          holistic=args.holistic, fp32_products=args.fp32_products)
    use_graph = not args.eager and args.pve is None and (cfg["variant"] == "st" or args.holistic)
    if use_graph:
        solver.capture(A)
        step = solver.replay
    else:
        step = lambda: solver.run(A)  # noqa: E731
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole solves (events between solves give the per-step spread, no synchronisation)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    spread = step_percentiles(evs)

    # relative error of the result (measurement, outside the timed region)
    G, U = solver.G.double(), [u.double() for u in solver.U]
    Ad = A.double()
    re = float(torch.linalg.vector_norm(Ad - reconstruct_torch(G, U)) / torch.linalg.vector_norm(Ad))
    del Ad

    roof = None
    if not args.no_kernel_timing:
        # the product classes, one timing pass each; the roofline object is the
        # class with the larger summed launch time (or the one named by --kernel)
        timed = {}
        for kern in ("colreduce", "rowcontract", "powerstep"):
            T.timing_enable(kern, capacity=65536)
            torch.cuda.synchronize()
            for _ in range(args.steps):
                solver.run(A)
            torch.cuda.synchronize()
            timed[kern] = T.timing_read(kern)
            T.timing_disable()
        kern = args.kernel if args.kernel != "auto" else max(timed, key=lambda k: timed[k]["ms"])
        tk = timed[kern]
        mk = "fp32" if (prec == "bf16" and kern == "rowcontract") else prec
        if mk == "fp32" and args.fp32_products == "split" and kern in ("colreduce", "rowcontract", "powerstep"):
            mk = "fp32-split"  # the large products of this class run as six BF16 products per pair
        roof = _roof_from_timing(tk, mk)
        # the committed counters were taken on the workload's default command
        # (default precision, ranks, q, order, test matrix and FP32 product mode)
        same = prec == CONFIGS[args.workload]["precision"] and cfg["ranks"] == CONFIGS[args.workload]["ranks"] \
            and args.fp32_products == "split" and args.omega == "gaussian"
        traffic = measured_traffic(kern, args.workload) \
            if same and order is None and not args.holistic and q == CONFIGS[args.workload]["q"] else None
        roof["traffic"] = traffic
        if traffic is not None:
            roof["traffic_unit"] = "bytes/launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["kernel"] = kern
        roof["per_step_ms"] = {k: round(v["ms"] / args.steps, 4) for k, v in timed.items()}
        if roof["bound"] == "hbm":
            roof["copy_gbs"] = round(copy_bandwidth(dev), 1)
            roof["frac_of_copy"] = round(roof["achieved"] / roof["copy_gbs"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        if a_host_store is None:
            a_host_store = A.double().cpu().numpy()
        cpu = cpu_baseline(args.workload, cfg, a_host_store, args.shift, q, args.pve, args.omega, order,
                           args.holistic)
        if "rel_error" in cpu:
            cpu["rel_error_gpu_minus_oracle"] = re - cpu["rel_error"]

    value = args.steps / elapsed
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "approximations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_spread": spread,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32" if args.fp32_products == "native" else
                  "f32 (large products as bf16x3-split pairs, f32 accumulation)",
                  "bf16": "bf16-operands/f32-acc"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(A.shape), "ranks": list(cfg["ranks"]), "p": cfg["p"],
                   "q": q, "shift": args.shift, "variant": cfg["variant"], "precision": prec,
                   "rel_error": re},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if prec == "fp32":
        line["config"]["fp32_products"] = args.fp32_products
    if args.omega != "gaussian":
        line["config"]["omega"] = args.omega
    if order is not None:
        line["config"]["order"] = order if isinstance(order, str) else list(order)
    if args.holistic:
        line["config"]["algorithm"] = "holistic (Appendix B.1 / A.2 form)"
    line["config"]["launch"] = "HIP graph replay of the whole solve" if use_graph else "eager"
    if args.pve is not None:
        line["config"].update({"algorithm": "4 (per-vector-error q)" if cfg["variant"] == "st" else
                               "2-v3 (Algorithm 4's test in T-HOSVD)", "tol": args.pve, "q_max": q,
                               "q_used": solver.q_used})
    print(json.dumps(line), flush=True)


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _roof_from_timing(tk, prec="fp32"):
    sec = tk["ms"] * 1e-3
    t_mem = tk["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_flop = tk["flops"] / (PEAK_TFLOPS[prec] * 1e12)
    if t_flop > t_mem:
        achieved = tk["flops"] / sec / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[prec], 4)}
    else:
        achieved = tk["bytes"] / sec / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof.update({"traffic": None, "launches": tk["launches"],
                 "avg_launch_us": round(1e3 * tk["ms"] / max(tk["launches"], 1), 3),
                 "alg_bytes_per_launch": tk["bytes"] / max(tk["launches"], 1),
                 "alg_flops_per_launch": tk["flops"] / max(tk["launches"], 1), "total_ms": tk["ms"]})
    return roof


def serving_main(args):
    """Continuous-batching burst throughput, one-at-a-time reference, RE parity and Poisson latency."""
    import numpy as np
    import torch

    from paper_2506_04840_amd import _lib as T
    from paper_2506_04840_amd import serve
    from workloads import generators as gen

    c = SERVING_CFG
    dev = torch.device("cuda:0")
    reqs = gen.request_stream(c["count"], 0.0, seed=c["data_seed"], n_lo=c["n_lo"], n_hi=c["n_hi"], r_lo=c["r_lo"],
                              r_hi=c["r_hi"])
    tensors = []
    for i, r in enumerate(reqs):
        tensors.append(gen.request_tensor_device(r, dev, c["eta"]))
        if (i + 1) % 1024 == 0:
            _log("built %d request tensors" % (i + 1))
    torch.cuda.synchronize()

    def jobs(arrivals=None):
        out = []
        for i, r in enumerate(reqs):
            out.append(serve.Job(r.rid, tensors[i], r.ranks, r.seed, 0.0 if arrivals is None else arrivals[i])
                       .prepare(c["p"], c["q"]))
        return out

    def timing_server():
        # the launch-timing pass: direct steps (no graphs), one batch on the device at a time
        return serve.BatchServer(capacity=c["capacity"], q=c["q"], p=c["p"], lclass=c["lclass"],
                                 ws_bytes=c["ws_bytes"], device=dev, use_graphs=False, overlap=False)

    if args.timing_pass_only:
        jt = jobs()
        srv_t = timing_server()
        srv_t.run(jt, t0=time.perf_counter())
        torch.cuda.synchronize()
        print(json.dumps({"workload": SERVING, "timing_pass_only": True, "batches": len(srv_t.batch_sizes)}),
              flush=True)
        return

    srv = serve.BatchServer(capacity=c["capacity"], q=c["q"], p=c["p"], lclass=c["lclass"], ws_bytes=c["ws_bytes"],
                            device=dev, overlap=not args.serial)
    jb = jobs()
    srv.ensure_slots(jb)
    for _ in range(args.warmup):
        srv.run(jb[:2 * c["capacity"]])
    torch.cuda.synchronize()
    _log("warm")

    # timed region: K bursts of every request through the batching server
    srv.batch_sizes, srv.inflight = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        srv.run(jb, t0=time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cap = args.steps * len(jb) / elapsed
    mean_batch = float(np.mean(srv.batch_sizes))
    mean_inflight = float(np.mean(srv.inflight))
    _log("batched burst: %.1f approximations/s" % cap)
    if args.burst_only:
        print(json.dumps({"metric": METRIC, "value": round(cap, 2), "unit": "approximations/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
                          "config": {"workload": SERVING, "burst_only": True, "serial": bool(args.serial)}}),
              flush=True)
        return

    # one request at a time, same requests, same burst
    single = serve.SingleServer(p=c["p"], q=c["q"], ws_bytes=64 << 20, device=dev)
    js = jobs()
    single.run(js[:64])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    single.run(js, t0=t1)
    torch.cuda.synchronize()
    single_rate = len(js) / (time.perf_counter() - t1)
    _log("one-at-a-time burst: %.1f approximations/s" % single_rate)

    # relative error of every request on both paths (FP64 reconstruction, outside the timed regions)
    re_b, re_s = [], []
    for a, x, y in zip(tensors, jb, js):
        ad = a.double()
        na = torch.linalg.vector_norm(ad)
        re_b.append(float(torch.linalg.vector_norm(ad - reconstruct_torch(x.G.double(), [u.double() for u in x.U])) / na))
        re_s.append(float(torch.linalg.vector_norm(ad - reconstruct_torch(y.G.double(), [u.double() for u in y.U])) / na))
    re_b, re_s = np.array(re_b), np.array(re_s)
    _log("relative errors done")

    # Poisson arrivals at 0.5 and 0.9 x the measured batched capacity
    poisson = []
    for frac in (0.5, 0.9):
        rate = frac * cap
        arr = gen.poisson_arrivals(len(reqs), rate, seed=c["data_seed"])
        jp = jobs(arr)
        srv.batch_sizes, srv.inflight = [], []
        torch.cuda.synchronize()
        out = srv.run(jp, t0=time.perf_counter())
        st = serve.latency_stats(out)
        st.update({"rate_per_s": round(rate, 1), "load": frac, "mean_batch": round(float(np.mean(srv.batch_sizes)), 2),
                   "batches": len(srv.batch_sizes), "mean_inflight_requests": round(float(np.mean(srv.inflight)), 1)})
        poisson.append({k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()})
        _log("poisson %.1f/s: p50 %.2f ms p99 %.2f ms" % (rate, st["p50_ms"], st["p99_ms"]))

    # dominant product kernel of the batched path: HIP events around each batched phase (direct steps, one
    # batch on the device at a time so that a phase's events time that phase alone)
    roof = None
    if not args.no_kernel_timing:
        timed = {}
        srv_t = timing_server()
        for kern in ("colreduce", "rowcontract"):
            T.timing_enable(kern, capacity=65536)
            torch.cuda.synchronize()
            srv_t.run(jb, t0=time.perf_counter())
            torch.cuda.synchronize()
            timed[kern] = T.timing_read(kern)
            T.timing_disable()
        kern = max(timed, key=lambda k: timed[k]["ms"])
        roof = _roof_from_timing(timed[kern])
        roof["kernel"] = "batched " + kern
        if roof["bound"] == "hbm":
            roof["copy_gbs"] = round(copy_bandwidth(dev), 1)
            roof["frac_of_copy"] = round(roof["achieved"] / roof["copy_gbs"], 4)
        roof["traffic"] = measured_traffic("batched_" + kern, SERVING)
        if roof["traffic"] is not None:
            roof["traffic_unit"] = "bytes/launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["burst_share"] = round(timed[kern]["ms"] * 1e-3 / (len(jb) / cap), 4)
        del srv_t

    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import rhosvd as orc
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        done, tsum = 0, 0.0
        for i, r in enumerate(reqs):
            a64 = tensors[i].double().cpu().numpy()
            t2 = time.perf_counter()
            orc.randomized_hosvd(a64, r.ranks, c["p"], c["q"], shift="adaptive", variant="st", seed=r.seed)
            tsum += time.perf_counter() - t2
            done += 1
            if tsum > 15.0:
                break
        cpu = {"value": round(done / tsum, 3), "unit": "approximations/s", "cores": int(threads), "kind": "oracle",
               "sample": "the first %d requests of the stream, one after another (FP64 oracle)" % done}

    line = {
        "metric": METRIC,
        "value": round(cap, 2),
        "unit": "approximations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": SERVING, "requests": c["count"], "dims": "U{%d..%d} per mode" % (c["n_lo"], c["n_hi"]),
                   "ranks": "U{%d..%d}" % (c["r_lo"], c["r_hi"]), "noise": c["eta"], "p": c["p"], "q": c["q"],
                   "shift": "adaptive", "variant": "st", "precision": "fp32", "capacity": c["capacity"],
                   "lclass": c["lclass"], "ws_bytes_per_slot": c["ws_bytes"]},
        "serving": {
            "batched_approx_per_s": round(cap, 2),
            "single_approx_per_s": round(single_rate, 2),
            "speedup": round(cap / single_rate, 3),
            "burst_mean_batch": round(mean_batch, 2),
            "burst_mean_inflight_requests": round(mean_inflight, 1),
            "rel_error_batched": {"mean": float(re_b.mean()), "max": float(re_b.max())},
            "rel_error_single": {"mean": float(re_s.mean()), "max": float(re_s.max())},
            "rel_error_max_abs_diff": float(np.max(np.abs(re_b - re_s))),
            "poisson": poisson,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
