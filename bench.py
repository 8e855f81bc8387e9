#!/usr/bin/env python3
"""Benchmark: batched LQ KKT solves/s on one MI355X, mixed precision vs float64 at equal residual.

Workload (the metric's configuration): 4096 independent time-varying LQ problems, N = 50,
nx = 12, nu = 4, synthetic seeded inputs (A = I + 0.05 G, B = 0.5 G, Q = M M^T + 0.1 I,
R = 0.1 I + diag(U(0,1)), q, r, x0 ~ N(0,1)), resident in HBM before timing.

One step = lq_factor + lq_solve for the whole batch (factor sweep, right-hand-side sweeps,
forward rollout, float64 KKT residual of every instance, refinement).  Both paths must reach
max rel_res <= 1e-10 (the float64 path certifies with one residual pass, the mixed path refines
until it gets there).  `value` is the mixed path's solves/s; the float64 path is reported beside
it.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LQ KKT solves/s, batch 4096 nx=12 nu=4 N=50: mixed vs FP64 at equal residual"
BATCH, N, NX, NU = 4096, 50, 12, 4
TOL = 1e-10
HBM_PEAK_GBS = 8000.0


def stage_sizes(nx, nu):
    """Elements per stage: input data read by a factor or residual pass, packed factor block."""
    data = nx * nx + nx * nu + nx * nx + nu * nu + nx + nu      # A, B, Q_k, R, q_k, r
    fac = nu * (nu + 1) // 2 + nu + nx * nu + nx * (nx + 1) // 2 + nx
    return data, fac


def algorithmic_bytes_factor(batch, N, nx, nu, fbytes):
    """Minimum HBM bytes of one factor launch: read the stage data once; write the packed
    factors (L^R, L^S, L^Q lower triangles + inverse diagonals) in the storage precision and the
    float64 backward-sweep vectors rbar_k, p_k."""
    data, fac = stage_sizes(nx, nu)
    return batch * N * (8 * data + fbytes * fac + 8 * (nu + nx))


def algorithmic_bytes_solve(N, nx, nu, fbytes, iters=None):
    """Algorithmic HBM bytes of one solve launch per instance: ONE forward rollout with the float64
    KKT residual fused in (read the factors in their storage precision, the stage data A, B, Q_k,
    R, q_k, r and the sweep vectors rbar_k, p_k; write x, u, lam).  Refinement passes are
    implementation bytes of this design, counted by `refinement_bytes`, never here."""
    data, fac = stage_sizes(nx, nu)
    z = 2 * nx + nu
    n_inst = 1 if iters is None else len(iters)
    return int(n_inst * N * (8 * data + fbytes * fac + 8 * (nu + nx) + 8 * z))


def refinement_bytes(N, nx, nu, fbytes, iters):
    """Implementation bytes the refinement adds to a solve launch, summed over instances (iters =
    per-instance refinement iterations).  Per stage and iteration: the residual store of the pass
    before it; a backward correction pass (read factors, A, B and the stored residual, write the
    correction sweep vectors); a forward correction pass with the residual (read factors, stage
    data, sweep vectors, the iterate and the dynamics residual; write the iterate)."""
    data, fac = stage_sizes(nx, nu)
    z = 2 * nx + nu
    total = 0
    for it in np.asarray(iters, dtype=np.int64):
        if it <= 0:
            continue
        bwd = fbytes * fac + 8 * (nx * nx + nx * nu) + 8 * z + 8 * (nu + nx)
        fwd1 = 8 * data + fbytes * fac + 8 * (nu + nx) + 8 * nx + 16 * z
        total += 8 * z + it * (bwd + fwd1) + (it - 1) * 8 * z
    return int(total) * N


def measure_copy_bandwidth():
    """HBM bandwidth of a plain device-to-device copy of 1 GiB (read + write bytes / time, median of
    five copies timed with events): the measured peak the roofline fraction is also given against."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    return 2 * n * 8 / (float(np.median(ts)) * 1e-3) / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def hbm_roofline(kernel, nbytes, ms, copy_gbs, traffic=None, extra=None):
    a = nbytes / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": kernel, "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": a / HBM_PEAK_GBS, "traffic": traffic, "peak_measured_copy": copy_gbs,
         "frac_measured_copy": a / copy_gbs if copy_gbs else None,
         "algorithmic_bytes_per_launch": nbytes, "ms_per_launch": ms}
    if extra:
        r.update(extra)
    return r


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counters, if the kernel
    source is unchanged since they were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"] or kernel not in rec["kernels"]:
        return None
    k = rec["kernels"][kernel]
    return k["read_bytes"] + k["write_bytes"]


def oracle_worker(args):
    import synth
    from oracle import riccati
    start, count = args
    probs = [synth.make_instance(2, i) for i in range(start, start + count)]
    t0 = time.perf_counter()
    for p in probs:
        riccati.solve(p)
    return time.perf_counter() - t0


def cpu_baseline(sample=2048, workers=None):
    """The oracle's textbook Riccati route (numpy float64) over a sample of the workload: each
    process generates its instances, then times their solves; throughput = sample / slowest
    process's solve time."""
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    workers = workers or min(os.cpu_count() or 1, 16)
    per = max(1, sample // workers)
    jobs = [(w * per, per) for w in range(workers)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        times = pool.map(oracle_worker, jobs)
    n = per * workers
    t = max(times)
    return {"value": n / t, "unit": "solves/s", "cores": workers, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n} instances of the workload (same generator), textbook Riccati route "
                      f"(numpy float64, 1 BLAS thread per process), {workers} processes, slowest {t:.1f} s"}


def run_path(mode, data, steps, warmup, max_it):
    import torch
    import paper_2512_09058_amd as L
    plan = L.Plan(N, NX, NU, batch=BATCH, mode=mode)
    ws = plan.workspace()
    info = torch.zeros(BATCH, dtype=torch.int32, device="cuda")
    rel = torch.zeros(BATCH, dtype=torch.float64, device="cuda")
    its = torch.zeros(BATCH, dtype=torch.int32, device="cuda")
    x, u, lam = plan.empty_outputs()
    stream = torch.cuda.current_stream()

    def step():
        L.factor(plan, data, ws, info, stream=stream)
        L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=TOL, max_it=max_it, check_res=True, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel durations with HIP events on the stream the library launches on
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for s in range(steps):
        ev[s][0].record(stream)
        L.factor(plan, data, ws, info, stream=stream)
        ev[s][1].record(stream)
        L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=TOL, max_it=max_it, check_res=True, stream=stream)
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    tf = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    ts = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    return {"plan": plan, "ms_per_step": 1e3 * wall / steps, "ms_factor": tf, "ms_solve": ts,
            "rel": rel.cpu().numpy(), "iters": its.cpu().numpy(), "info": info.cpu().numpy(),
            "x": x, "u": u, "lam": lam}


def bench_uneven(args):
    """The uneven workload (2048 instances, nx 6..64, nu 2..16, N 10..200): one persistent,
    longest-first launch per call, launch shape chosen by the autotuner; float64 and mixed."""
    import torch
    import synth
    import paper_2512_09058_amd as L
    from paper_2512_09058_amd import tune
    insts = synth.make_ragged(2048)
    sols = {}
    data = L.pack(insts)
    Ns, nxs, nus = [p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts]
    out = {"metric": "LQ KKT solves/s, uneven batch 2048 (nx 6..64, nu 2..16, N 10..200)", "unit": "solves/s",
           "n_gpus": 1, "data": "synthetic (seeded generators of the workload)"}
    for mode, max_it in (("f64", 0), ("mixed_f32", args.max_it)):
        plan = L.Plan(Ns, nxs, nus, mode=mode)
        choice = tune.tune(plan, data, max_it=max_it, reps=1)
        ws = plan.workspace()
        info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
        rel = torch.zeros(plan.batch, dtype=torch.float64, device="cuda")
        its = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
        x, u, lam = plan.empty_outputs()
        g = L.api.capture(plan, data, ws, x, u, lam, rel, its, info, tol=TOL, max_it=max_it)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        # per-kernel launch times (events on the library's stream, outside the graph)
        stream = torch.cuda.current_stream()
        kt = []
        for _ in range(3):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            L.factor(plan, data, ws, info, stream=stream)
            e[1].record(stream)
            L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=TOL, max_it=max_it, check_res=True, stream=stream)
            e[2].record(stream)
            kt.append(e)
        torch.cuda.synchronize()
        tf = float(np.median([e[0].elapsed_time(e[1]) for e in kt]))
        tsv = float(np.median([e[1].elapsed_time(e[2]) for e in kt]))
        relh = rel.cpu().numpy()
        itsh = its.cpu().numpy()
        sols[mode] = _host_solutions(plan, x, u, lam)
        fb = 8 if mode == "f64" else 4
        fbytes = sum(algorithmic_bytes_factor(1, p.N, p.nx, p.nu, fb) for p in insts)
        sbytes = sum(algorithmic_bytes_solve(p.N, p.nx, p.nu, fb, [itsh[i]]) for i, p in enumerate(insts))
        kern = {"factor": (tf, fbytes), "solve": (tsv, sbytes)}
        dom = max(kern, key=lambda k_: kern[k_][0])
        ach = kern[dom][1] / (kern[dom][0] * 1e-3) / 1e9
        out[mode] = {"value": 2048 / (ms * 1e-3), "ms_per_step": ms, "variant": choice["variant"],
                     "launch": choice["launch"],
                     "max_rel_res": float(relh.max()), "iters_max": int(itsh.max()),
                     "info_ok": bool((info == 0).all().item()), "ms_factor": tf, "ms_solve": tsv,
                     "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": ach / HBM_PEAK_GBS, "traffic": None,
                                  "algorithmic_bytes_per_launch": kern[dom][1], "ms_per_launch": kern[dom][0]},
                     "buckets": _bucket_report(insts, relh, itsh)}
        print(f"[bench] uneven {mode}: {ms:.2f} ms/step, variant {choice['variant']}, launch {choice['launch']}, "
              f"max rel_res {relh.max():.2e}",
              file=sys.stderr, flush=True)
    # per nx bucket: deviation of the mixed path from the float64 GPU solution (every instance)
    for lo, hi in NX_BUCKETS:
        idx = [i for i, p in enumerate(insts) if lo <= p.nx <= hi]
        dev = max(_fwd_err(sols["mixed_f32"][i], sols["f64"][i]) for i in idx)
        out["mixed_f32"]["buckets"][f"nx {lo}-{hi}"]["max_fwd_err_vs_f64_gpu"] = dev
        print(f"[bench] uneven bucket nx {lo}-{hi}: {len(idx)} instances, mixed vs f64 {dev:.1e}",
              file=sys.stderr, flush=True)
    m = out["mixed_f32"]
    out.update({"value": m["value"], "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32 stage products + f64 Cholesky/residual/refinement",
                "config": {"workload": "uneven batch of 2048 LQ problems, nx 6..64, nu 2..16, N 10..200, "
                                       "hipGraph replay", "batch": 2048, "tol": TOL, "max_it": args.max_it},
                "roofline": m["roofline"],
                "cpu_baseline": None if args.no_cpu else _cpu_uneven(insts, sols)})
    print(json.dumps(out))


NX_BUCKETS = ((6, 16), (17, 32), (33, 48), (49, 64))


def _host_solutions(plan, x, u, lam):
    """(x, u, lam) of every instance as host arrays (one copy of each output array)."""
    out = []
    arrs = {n: t.cpu().numpy() for n, t in (("x", x), ("u", u), ("lam", lam))}
    for i in range(plan.batch):
        N, nx, nu = int(plan.N[i]), int(plan.nx[i]), int(plan.nu[i])
        blk = []
        for n, d in (("x", nx), ("u", nu), ("lam", nx)):
            o = int(plan.offsets[n][i])
            blk.append(arrs[n][o:o + N * d].reshape(N, d))
        out.append(tuple(blk))
    return out


def _fwd_err(sol, ref):
    return float(max(np.abs(a - b).max() for a, b in zip(sol, ref)) / max(np.abs(b).max() for b in ref))


def _uneven_oracle_worker(chunk):
    from oracle import riccati
    t0 = time.perf_counter()
    for p in chunk:
        riccati.solve(p)
    return time.perf_counter() - t0


def _cpu_uneven(insts, sols, per_bucket=None, workers=16):
    """The CPU leg of the uneven workload: the oracle's textbook Riccati route timed on the batch
    (or on per_bucket instances of each nx bucket; 16 processes, one BLAS thread each); then, per
    bucket, the oracle's residual of the GPU solutions and their forward error against the
    oracle's solution on three sampled instances."""
    from oracle import kkt, riccati
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    sample = []
    for lo, hi in NX_BUCKETS:
        sample += [p for p in insts if lo <= p.nx <= hi][:per_bucket]
    chunks = [sample[w::workers] for w in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        times = pool.map(_uneven_oracle_worker, chunks)
    t = max(times)
    check = {}
    for lo, hi in NX_BUCKETS:
        idx = [i for i, p in enumerate(insts) if lo <= p.nx <= hi]
        pick = idx[:: max(1, len(idx) // 3)][:3]
        ref = {i: riccati.solve(insts[i]) for i in pick}
        check[f"nx {lo}-{hi}"] = {
            mode: {"oracle_rel_res": max(kkt.residual(insts[i], *sols[mode][i])[1] for i in pick),
                   "fwd_err_vs_oracle": max(_fwd_err(sols[mode][i], ref[i]) for i in pick)}
            for mode in sols}
    return {"value": len(sample) / t, "unit": "solves/s", "cores": workers, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{len(sample)} instances ({per_bucket or 'all'} per nx bucket), textbook Riccati route (numpy float64, "
                      f"1 BLAS thread per process), {workers} processes, slowest {t:.1f} s",
            "gpu_vs_oracle_sampled": check}


def _bucket_report(insts, rel, its):
    """Per nx bucket: instance count, largest library rel_res, refinement iterations."""
    rep = {}
    for lo, hi in NX_BUCKETS:
        idx = [i for i, p in enumerate(insts) if lo <= p.nx <= hi]
        rep[f"nx {lo}-{hi}"] = {"instances": len(idx), "max_rel_res": float(rel[idx].max()),
                                "iters_max": int(its[idx].max()), "iters_mean": float(its[idx].mean())}
    return rep


def _gen_worker(args):
    import synth
    cfg, i = args
    p = synth.make_instance(cfg, i)
    return i, {k: getattr(p, k) for k in ("A", "B", "Q", "R", "q", "r", "x0")}


def _gen_uniform(cfg, count, workers=16, distinct=0):
    """`count` instances of workload `cfg`, generated in parallel processes, as the packed device
    arrays of the library (uniform batch: instance blocks back to back).  distinct > 0: only that
    many instances, generated in this process and repeated cyclically (same shapes and value
    distributions; for short profiled runs)."""
    import torch
    import synth
    first = synth.make_instance(cfg, 0)
    host = {k: np.empty((count,) + getattr(first, k).shape) for k in ("A", "B", "Q", "R", "q", "r", "x0")}
    if distinct > 0:
        print(f"[bench] generating {distinct} distinct instances, repeated to {count}", file=sys.stderr, flush=True)
        insts = [first] + [synth.make_instance(cfg, i) for i in range(1, min(distinct, count))]
        for i in range(count):
            for k in host:
                host[k][i] = getattr(insts[i % len(insts)], k)
        return {k: torch.from_numpy(v.reshape(-1)).to("cuda") for k, v in host.items()}
    print(f"[bench] generating {count} instances in {min(workers, count)} processes", file=sys.stderr, flush=True)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"  # one BLAS thread per worker process
    ctx = mp.get_context("spawn")
    done = 0
    with ctx.Pool(min(workers, count)) as pool:
        for i, d in pool.imap_unordered(_gen_worker, [(cfg, i) for i in range(count)]):
            for k, v in d.items():
                host[k][i] = v
            done += 1
            if done % 8 == 0:
                print(f"[bench] generated {done}/{count} instances", file=sys.stderr, flush=True)
    return {k: torch.from_numpy(v.reshape(-1)).to("cuda") for k, v in host.items()}


def _oracle_time_worker(args):
    import synth
    from oracle import adjoint, kkt, riccati
    cfg, start, count, adj = args
    probs = [synth.make_instance(cfg, i) for i in range(start, start + count)]
    t0 = time.perf_counter()
    for p in probs:
        if adj:
            x, u, _ = kkt.solve_dense(p)
            _, gx, gu = adjoint.quad_loss(x, u)
            adjoint.adjoint_grad(p, gx, gu)
        else:
            riccati.solve(p)
    return time.perf_counter() - t0


def _cpu_uniform(cfg, per, workers, adj, what):
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        times = pool.map(_oracle_time_worker, [(cfg, w * per, per, adj) for w in range(workers)])
    n, t = per * workers, max(times)
    return {"value": n / t, "unit": "solves/s", "cores": workers, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n} instances of the workload, {what} (numpy float64, 1 BLAS thread per process), "
                      f"{workers} processes, slowest {t:.1f} s"}


def _cpu_large(sols0):
    """The CPU leg of the large workload: the oracle timed on 8 instances (one per process), and the
    forward error of every path's solution of instance 0 against the oracle's."""
    from oracle import riccati
    cpu = _cpu_uniform(4, 1, 8, False, "textbook Riccati route")
    ref = riccati.solve(synthetic_instance(4, 0))
    cpu["gpu_vs_oracle_inst0"] = {m: _fwd_err(s_, ref) for m, s_ in sols0.items()}
    return cpu


def _roofline(ms, nbytes, flops, peak_flops_tf):
    """Roofline entry of one launch: HBM-bound if its arithmetic intensity (algorithmic flops per
    algorithmic byte) is below the ridge point of the given matrix-core peak, else compute-bound."""
    ai = flops / nbytes
    if ai < peak_flops_tf * 1e12 / (HBM_PEAK_GBS * 1e9):
        a = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
                "traffic": None, "algorithmic_bytes_per_launch": nbytes, "ms_per_launch": ms}
    a = flops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": a, "peak": peak_flops_tf, "unit": "TFLOP/s", "frac": a / peak_flops_tf,
            "traffic": None, "algorithmic_flops_per_launch": flops, "ms_per_launch": ms}


def factor_flops(batch, N, nx, nu):
    """Operation count of the factor sweep (FMA = 2 flops): trmm 1/2 nux nx^2 + syrk 1/2 nux^2 nx +
    potrf nux^3/6 per stage."""
    ux = nx + nu
    return 2.0 * batch * N * (0.5 * ux * nx * nx + 0.5 * ux * ux * nx + ux ** 3 / 6.0)


def pit_factor_flops(batch, N, nx, nu, P):
    """Operation count of the parallel-in-time factorisation (FMA = 2 flops), summed over every
    interval (the paper's eq. flop gives the same terms per interval on the critical path): per
    stage potrf 1/6 nux^3, trsm 1/2 nx nu^2, gemm nx^2 nu, M^fwd syrk 1/2 nu nx^2; per stage but the
    interval's first trmm 1/2 nux nx^2, syrk 1/2 nux^2 nx and the propagation gemm nux nx^2;
    per interval 1/2 nx^3 (L^A) + 4/3 nx^3 (Schur blocks); cyclic reduction about 3 nx^3 per block."""
    ux = nx + nu
    n = N / P
    per = (n * (ux ** 3 / 6 + 0.5 * nx * nu * nu + nx * nx * nu + 0.5 * nu * nx * nx)
           + (n - 1) * (1.5 * ux * nx * nx + 0.5 * ux * ux * nx) + 0.5 * nx ** 3 + 4.0 / 3.0 * nx ** 3 + 3 * nx ** 3)
    return 2.0 * batch * P * per


def bench_large(args):
    """The large workload: 64 instances, N = 1000, nx = 128, nu = 32 (A = 0.99 Haar + 0.01 G,
    B = G / sqrt(nx), Q = M M^T + I, R = I); bf16 matrix-core stage products with float64
    Cholesky and refinement (the reported path), float32 products and plain float64 beside it."""
    import torch
    import paper_2512_09058_amd as L
    b, Nn, nx, nu = 64, 1000, 128, 32
    t0 = time.perf_counter()
    data = _gen_uniform(4, b, distinct=args.distinct)
    torch.cuda.synchronize()
    print(f"[bench] generated and uploaded the large workload in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    res, sols0 = {}, {}
    for mode, mi in (("f64", 0), ("mixed_f32", args.max_it), ("mixed_bf16", max(args.max_it, 20))):
        plan = L.Plan(Nn, nx, nu, batch=b, mode=mode)
        plan.set_launch(threads=512)
        ws = plan.workspace()
        info = torch.zeros(b, dtype=torch.int32, device="cuda")
        rel = torch.zeros(b, dtype=torch.float64, device="cuda")
        its = torch.zeros(b, dtype=torch.int32, device="cuda")
        x, u, lam = plan.empty_outputs()
        stream = torch.cuda.current_stream()
        ev = []
        for s_ in range(args.warmup + args.steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            L.factor(plan, data, ws, info, stream=stream)
            e[1].record(stream)
            L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=TOL, max_it=mi, check_res=True, stream=stream)
            e[2].record(stream)
            if s_ >= args.warmup:
                ev.append(e)
        torch.cuda.synchronize()
        tf = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        tsv = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        relh = rel.cpu().numpy()
        r = {"value": b / ((tf + tsv) * 1e-3), "ms_per_step": tf + tsv, "ms_factor": tf, "ms_solve": tsv,
             "max_rel_res": float(relh.max()), "iters_max": int(its.max().item()),
             "info_ok": bool((info == 0).all().item()), "variant": plan.variant}
        sols0[mode] = [L.unpack(plan, n, t, 0) for n, t in (("x", x), ("u", u), ("lam", lam))]
        fb = 8 if mode == "f64" else 4
        r["factor_roofline"] = _roofline(tf, algorithmic_bytes_factor(b, Nn, nx, nu, fb), factor_flops(b, Nn, nx, nu),
                                         78.6)
        r["solve_GBps_algorithmic"] = algorithmic_bytes_solve(Nn, nx, nu, fb, its.cpu().numpy()) / (tsv * 1e-3) / 1e9
        res[mode] = r
        print(f"[bench] large {mode}: factor {tf:.1f} ms, solve {tsv:.1f} ms, max rel_res {relh.max():.2e}, "
              f"iterations {r['iters_max']}", file=sys.stderr, flush=True)
    # the parallel-in-time path (FP64): each instance's horizon in P intervals factored at once
    from paper_2512_09058_amd import pit
    for P in args.pit_intervals:
        plan = pit.PitPlan(b, Nn, nx, nu, P)
        ws = plan.workspace()
        info = torch.zeros(b, dtype=torch.int32, device="cuda")
        rel = torch.zeros(b, dtype=torch.float64, device="cuda")
        x, u, lam = plan.empty_outputs()
        stream = torch.cuda.current_stream()
        ev = []
        for s_ in range(args.warmup + args.steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            pit.factor(plan, data, ws, info, stream=stream)
            e[1].record(stream)
            pit.solve(plan, data, ws, x, u, lam, rel, info, stream=stream)
            e[2].record(stream)
            if s_ >= args.warmup:
                ev.append(e)
        torch.cuda.synchronize()
        tf = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        tsv = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        relh = rel.cpu().numpy()
        sol = [t_.view(b, Nn, -1)[0].cpu().numpy() for t_ in (x, u, lam)]
        fl = pit_factor_flops(b, Nn, nx, nu, P)
        res[f"pit_P{P}"] = {"value": b / ((tf + tsv) * 1e-3), "ms_per_step": tf + tsv, "ms_factor": tf, "ms_solve": tsv,
                            "max_rel_res": float(relh.max()), "info_ok": bool((info == 0).all().item()),
                            "workgroups_factor": b * P, "fwd_err_vs_serial_f64_inst0": _fwd_err(sol, sols0["f64"]),
                            "factor_roofline": {"bound": "alu", "achieved": fl / (tf * 1e-3) / 1e12,
                                                "peak": 78.6, "unit": "TFLOP/s",
                                                "frac": fl / (tf * 1e-3) / 1e12 / 78.6,
                                                "algorithmic_flops_per_launch": fl, "ms_per_launch": tf}}
        sols0[f"pit_P{P}"] = sol
        print(f"[bench] large pit P={P}: factor {tf:.1f} ms, solve {tsv:.1f} ms, max rel_res {relh.max():.2e}",
              file=sys.stderr, flush=True)
        del ws
    m = res["mixed_bf16"]
    dom_solve = m["ms_solve"] >= m["ms_factor"]
    out = {"metric": "LQ KKT solves/s, batch 64 nx=128 nu=32 N=1000: bf16 products + f64 refinement vs FP64",
           "value": m["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16 stage products (f32 accumulate) + f64 Cholesky/residual/refinement",
           "data": "synthetic (seeded generators of the workload)",
           "config": {"workload": "batch 64 LQ problems, N=1000, nx=128, nu=32", "batch": b, "N": Nn, "nx": nx,
                      "nu": nu, "tol": TOL},
           "paths": res,
           "roofline": (m["factor_roofline"] if not dom_solve else
                        {"bound": "hbm", "kernel": "solve", "achieved": m["solve_GBps_algorithmic"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": m["solve_GBps_algorithmic"] / HBM_PEAK_GBS,
                         "traffic": None, "ms_per_launch": m["ms_solve"]}),
           "cpu_baseline": None if args.no_cpu else _cpu_large(sols0)}
    print(json.dumps(out))


def synthetic_instance(cfg, i):
    import synth
    return synth.make_instance(cfg, i)


def bench_adjoint(args):
    """The adjoint workload: 1024 instances, N = 100, nx = 32, nu = 8 (generators of the batch-4096
    workload); one step = factor + solve + lq_solve_backward for the loss 1/2 sum(|x_k|^2 + |u_k|^2)
    (upstream gradients x, u), float32 products with float64 Cholesky and refinement, factors
    checkpointed every 10 stages (the reported path); without checkpoints and in float64 (with and
    without checkpoints) beside it."""
    import torch
    import synth
    import paper_2512_09058_amd as L
    b = 1024
    prob = synth.make_batch(5)
    data = L.pack(prob)
    Nn, nx, nu = prob.N, prob.nx, prob.nu
    res = {}
    for mode, ckpt, mi in (("mixed_f32", 10, args.max_it), ("mixed_f32", 0, args.max_it), ("f64", 10, 0), ("f64", 0, 0)):
        plan = L.Plan(Nn, nx, nu, batch=b, mode=mode, ckpt_stride=ckpt)
        ws = plan.workspace()
        info = torch.zeros(b, dtype=torch.int32, device="cuda")
        rel = torch.zeros(b, dtype=torch.float64, device="cuda")
        relb = torch.zeros(b, dtype=torch.float64, device="cuda")
        its = torch.zeros(b, dtype=torch.int32, device="cuda")
        x, u, lam = plan.empty_outputs()
        g = {k: torch.empty(plan.totals[k], dtype=torch.float64, device="cuda")
             for k in ("A", "B", "Q", "R", "q", "r", "x0")}
        stream = torch.cuda.current_stream()
        ev = []
        for s_ in range(args.warmup + args.steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
            L.factor(plan, data, ws, info, stream=stream)
            e[1].record(stream)
            L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=TOL, max_it=mi, check_res=True, stream=stream)
            e[2].record(stream)
            L.solve_backward(plan, data, ws, x, u, lam, x, u, g, relb, None, info, tol=TOL, max_it=mi,
                             stream=stream)
            e[3].record(stream)
            if s_ >= args.warmup:
                ev.append(e)
        torch.cuda.synchronize()
        t = [float(np.mean([e[i].elapsed_time(e[i + 1]) for e in ev])) for i in range(3)]
        key = f"{mode}" + (f"_ckpt{ckpt}" if ckpt else "")
        res[key] = {"value": b / (sum(t) * 1e-3), "ms_per_step": sum(t), "ms_factor": t[0], "ms_solve": t[1],
                    "ms_backward": t[2], "max_rel_res": float(rel.max().item()),
                    "max_rel_res_adjoint": float(relb.max().item()), "info_ok": bool((info == 0).all().item()),
                    "variant": plan.variant, "workspace_bytes": plan.workspace_bytes,
                    "iters_max": int(its.max().item())}
        fb = 8 if mode == "f64" else 4
        sbytes = algorithmic_bytes_solve(Nn, nx, nu, fb, its.cpu().numpy())
        res[key]["solve_roofline"] = {"bound": "hbm", "kernel": "solve", "achieved": sbytes / (t[1] * 1e-3) / 1e9,
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": sbytes / (t[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                                      "algorithmic_bytes_per_launch": sbytes, "ms_per_launch": t[1]}
        print(f"[bench] adjoint {key}: factor {t[0]:.2f} ms, solve {t[1]:.2f} ms, backward {t[2]:.2f} ms, "
              f"rel {rel.max().item():.1e} / {relb.max().item():.1e}", file=sys.stderr, flush=True)
    m = res["mixed_f32_ckpt10"]
    out = {"metric": "LQ KKT forward+adjoint solves/s, batch 1024 nx=32 nu=8 N=100, factors checkpointed every 10",
           "value": m["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 stage products + f64 Cholesky/residual/refinement",
           "data": "synthetic (seeded generators of the workload)",
           "config": {"workload": "batch 1024 LQ problems, N=100, nx=32, nu=8, forward + adjoint", "batch": b,
                      "N": Nn, "nx": nx, "nu": nu, "tol": TOL, "ckpt_stride": 10},
           "paths": res, "roofline": m["solve_roofline"],
           "cpu_baseline": None if args.no_cpu else _cpu_uniform(5, 1, 16, True,
                                                                 "dense KKT solve + dense adjoint solve")}
    print(json.dumps(out))


def bench_single(args):
    """The single-problem workload (N = 20, nx = 4, nu = 2, float64): latency of one factor + solve
    on the GPU (each call timed with events, and as a replayed hipGraph), beside the oracle's
    dense KKT solve and textbook Riccati route on one host core, with the GPU result checked
    against the oracle."""
    import torch
    import synth
    import paper_2512_09058_amd as L
    from oracle import kkt, riccati
    p = synth.make_instance(1, 0)
    plan = L.Plan([p.N], [p.nx], [p.nu], mode="f64")
    data = L.pack([p])
    ws = plan.workspace()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rel = torch.zeros(1, dtype=torch.float64, device="cuda")
    x, u, lam = plan.empty_outputs()
    stream = torch.cuda.current_stream()
    reps = max(args.steps, 200)
    for _ in range(args.warmup + 10):
        L.factor(plan, data, ws, info, stream=stream)
        L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=TOL, max_it=0, stream=stream)
    torch.cuda.synchronize()
    us = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        L.factor(plan, data, ws, info, stream=stream)
        L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=TOL, max_it=0, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us.append(1e3 * e0.elapsed_time(e1))
    t0 = time.perf_counter()
    for _ in range(reps):
        L.factor(plan, data, ws, info, stream=stream)
        L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=TOL, max_it=0, stream=stream)
        torch.cuda.synchronize()
    wall_us = 1e6 * (time.perf_counter() - t0) / reps
    g = L.api.capture(plan, data, ws, x, u, lam, rel, None, info, tol=TOL, max_it=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    graph_us = 1e6 * (time.perf_counter() - t0) / reps
    sol = [L.unpack(plan, n, t_, 0) for n, t_ in (("x", x), ("u", u), ("lam", lam))]
    ref = kkt.solve_dense(p)
    out_cpu = None
    if not args.no_cpu:
        for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[v] = "1"
        tc = {}
        for name, fn in (("dense_kkt", kkt.solve_dense), ("textbook_riccati", riccati.solve)):
            n, t0 = 0, time.perf_counter()
            while time.perf_counter() - t0 < 2.0:
                fn(p)
                n += 1
            tc[name] = 1e6 * (time.perf_counter() - t0) / n
        out_cpu = {"value": tc["textbook_riccati"], "unit": "us/solve", "cores": 1, "kind": "oracle",
                   "cpu_model": cpu_model(),
                   "sample": "the one instance, solved repeatedly for 2 s per route in this process "
                             "(numpy float64; BLAS threads as numpy was loaded)",
                   "dense_kkt_us": tc["dense_kkt"], "textbook_riccati_us": tc["textbook_riccati"]}
    med = float(np.median(us))
    out = {"metric": "us per LQ KKT solve, single problem N=20 nx=4 nu=2, FP64", "value": med, "unit": "us/solve",
           "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": med * 1e-3,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded generators of the workload)",
           "config": {"workload": "single LQ problem, N=20, nx=4, nu=2, FP64 factor + solve", "batch": 1,
                      "variant": plan.variant},
           "gpu_event_us_median": med, "gpu_event_us_min": float(np.min(us)),
           "host_wall_us_with_sync": wall_us, "graph_replay_us": graph_us,
           "rel_res": float(rel.item()), "info": int(info.item()),
           "oracle_rel_res_of_gpu_solution": float(kkt.residual(p, *sol)[1]),
           "fwd_err_vs_oracle": _fwd_err(sol, ref),
           "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": "us", "frac": None,
                        "traffic": None},
           "cpu_baseline": out_cpu}
    print(f"[bench] single: GPU {med:.1f} us (events), {wall_us:.1f} us host wall with sync, graph "
          f"{graph_us:.1f} us", file=sys.stderr, flush=True)
    print(json.dumps(out))


def bench_shapes(args):
    """Size-specialised shapes at the batch-4096 workload's size (4096 instances, N = 50, its
    generators): shapes without a kernel of their own run padded to a compiled one (plan variant
    small_padded), beside the same plans on the tile kernels and the compiled (12, 4).  Factor +
    solve per step, HIP events; every instance's library residual; the oracle (textbook Riccati) on
    sampled instances in the CPU leg."""
    import torch
    import synth
    import paper_2512_09058_amd as L
    from oracle import riccati
    shapes = [(12, 4), (11, 4), (12, 3), (9, 5)]
    res, stream = {}, torch.cuda.current_stream()
    for nx, nu in shapes:
        b = synth.make_batch(2, 4096, N=50, nx=nx, nu=nu)
        data = L.pack(b)
        for mode, mi in (("f64", 0), ("mixed_f32", args.max_it)):
            for variant in (None, "tile"):
                plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode)
                if variant:
                    plan.set_variant(variant)
                ws = plan.workspace()
                info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
                rel = torch.zeros(plan.batch, dtype=torch.float64, device="cuda")
                x, u, lam = plan.empty_outputs()
                for _ in range(args.warmup):
                    L.factor(plan, data, ws, info, stream=stream)
                    L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=TOL, max_it=mi, stream=stream)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    L.factor(plan, data, ws, info, stream=stream)
                    L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=TOL, max_it=mi, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                key = f"{nx}x{nu}_{mode}_{plan.variant}"
                r = {"nx": nx, "nu": nu, "mode": mode, "variant": plan.variant, "ms_per_step": ms,
                     "solves_per_s": b.batch / (ms * 1e-3), "max_rel_res": float(rel.max().item()),
                     "info_ok": bool((info == 0).all().item())}
                if not args.no_cpu and variant is None and mode == "f64":
                    errs = []
                    for i in (0, 2047, 4095):
                        p = b.instance(i)
                        sol = [L.unpack(plan, n, t_, i) for n, t_ in (("x", x), ("u", u), ("lam", lam))]
                        errs.append(_fwd_err(sol, riccati.solve(p)))
                    r["fwd_err_vs_oracle_sampled"] = max(errs)
                res[key] = r
                print(f"[bench] shapes {key}: {ms:.3f} ms, max rel_res {r['max_rel_res']:.1e}", file=sys.stderr,
                      flush=True)
    out_cpu = None
    if not args.no_cpu:
        p = synth.make_batch(2, 1, N=50, nx=11, nu=4).instance(0)
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 2.0:
            riccati.solve(p)
            n += 1
        out_cpu = {"value": n / (time.perf_counter() - t0), "unit": "solves/s", "cores": 1, "kind": "oracle",
                   "cpu_model": cpu_model(),
                   "sample": "one nx = 11, nu = 4, N = 50 instance solved repeatedly for 2 s by the oracle's textbook "
                             "Riccati route in this process"}
    head = res["11x4_f64_small_padded"]
    out = {"metric": "LQ KKT solves/s, batch 4096 N=50, size-specialised shapes without their own kernel (padded)",
           "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generators of the workload)",
           "config": {"workload": "4096 x N=50, nx=11, nu=4 padded to the compiled (11, 5); also (12, 3) padded "
                                  "to (12, 4), (9, 5) padded to (9, 7), the compiled (12, 4) and the tile kernels", "batch": 4096, "N": 50},
           "shapes": res,
           "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": "ms", "frac": None,
                        "traffic": None},
           "cpu_baseline": out_cpu}
    print(json.dumps(out))


def bench_blocktri(args):
    """Batched block-tridiagonal systems (64 systems of 64 blocks of 128: the Schur complement
    shape of a 64-interval split of the large workload): cyclic-reduction factorisation and solve,
    parallel cyclic reduction, PCG with the stair preconditioner; the oracle's written-out CR
    recursion and dense solve timed on the host."""
    import torch
    import synth
    from paper_2512_09058_amd import blocktri as btl
    from oracle import blocktri as obt
    batch, Nb, n = 64, 64, 128
    M, K, b = synth.random_blocktri(1, batch, Nb, n)
    Md, Kd, bd = (torch.from_numpy(a).to("cuda") for a in (M, K, b))
    ws = btl.workspace(batch, Nb, n, "cr")
    info = torch.zeros(batch, dtype=torch.int32, device="cuda")
    x = torch.empty_like(bd)
    stream = torch.cuda.current_stream()
    t = {"cr_factor": [], "cr_solve": [], "pcr": [], "pcg_stair": []}
    wsp = btl.workspace(batch, Nb, n, "pcr")
    wsg = btl.workspace(batch, Nb, n, "pcg")
    xp = torch.empty_like(bd)
    xg = torch.empty_like(bd)
    its = torch.zeros(batch, dtype=torch.int32, device="cuda")
    relg = torch.zeros(batch, dtype=torch.float64, device="cuda")
    infog = torch.zeros(batch, dtype=torch.int32, device="cuda")
    for s_ in range(args.warmup + args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record(stream)
        btl.cr_factor(Md, Kd, ws, info, stream=stream)
        e[1].record(stream)
        btl.cr_solve(batch, Nb, n, ws, bd, x, stream=stream)
        e[2].record(stream)
        btl.pcr_solve(Md, Kd, bd, xp, wsp, info, stream=stream)
        e[3].record(stream)
        btl.pcg(Md, Kd, bd, "stair", 1e-12, 200, xg, wsg, its, relg, infog, stream=stream)
        e[4].record(stream)
        if s_ >= args.warmup:
            for i, k in enumerate(t):
                t[k].append(e)
    torch.cuda.synchronize()
    ms = {k: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in v])) for i, (k, v) in enumerate(t.items())}
    xh, xph, xgh = x.cpu().numpy(), xp.cpu().numpy(), xg.cpu().numpy()
    errs = {}
    for sidx in (0, 63):
        ref = obt.cr_recursive(M[sidx], K[sidx], b[sidx])
        for name, arr in (("cr", xh), ("pcr", xph), ("pcg", xgh)):
            errs[name] = max(errs.get(name, 0.0), float(np.abs(arr[sidx] - ref).max() / np.abs(ref).max()))
    fl = 2.0 * batch * Nb * (7.0 / 6.0 + 2.0) * n ** 3  # eliminations + updates of the remaining rows
    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        cnt = 0
        while time.perf_counter() - t0 < 10.0 and cnt < batch:
            obt.cr_recursive(M[cnt], K[cnt], b[cnt])
            cnt += 1
        tc = (time.perf_counter() - t0) / cnt
        cpu = {"value": 1.0 / tc, "unit": "systems/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{cnt} systems through the oracle's written-out cyclic-reduction recursion (numpy float64, "
                         f"one process; numpy's BLAS threads as loaded), {tc * 1e3:.0f} ms per system"}
    out = {"metric": "batched block-tridiagonal solves/s, 64 systems x 64 blocks of 128 (CR factor + solve)",
           "value": batch / ((ms["cr_factor"] + ms["cr_solve"]) * 1e-3), "unit": "systems/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms["cr_factor"] + ms["cr_solve"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded SPD block-tridiagonal systems)",
           "config": {"workload": "64 systems, Nb=64 blocks of n=128", "batch": batch, "Nb": Nb, "n": n},
           "ms": ms, "pcg_iters_max": int(its.max().item()), "rel_err_vs_oracle_sampled": errs,
           "info_ok": bool((info == 0).all().item()),
           "roofline": {"bound": "alu", "kernel": "cr_factor (k_cr_elim + k_cr_update)",
                        "achieved": fl / (ms["cr_factor"] * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                        "frac": fl / (ms["cr_factor"] * 1e-3) / 1e12 / 78.6, "traffic": None,
                        "algorithmic_flops_per_launch": fl, "ms_per_launch": ms["cr_factor"]},
           "cpu_baseline": cpu}
    print(f"[bench] blocktri: {ms}", file=sys.stderr, flush=True)
    print(json.dumps(out))


def update_flops(dsig, N, nx, nu):
    """Algorithmic float64 flops of one factor update (hyperbolic Householder steps and the products
    forming Upsilon) from the per-stage counts of nonzero rows: with W_k the nonzero rows of stages
    k..N, stage N's L^Q step and stage k's input and state steps cost 4 W per row per pivot, the
    products for stage k-1 2 (nx + nu) nx W_k."""
    nux = nx + nu
    nz = (dsig != 0).sum(axis=-1)                       # [batch, N+1]
    W = np.cumsum(nz[:, ::-1], axis=1)[:, ::-1]         # W[:, k] = rows of stages k..N
    rows_u = sum(nux - i for i in range(nu))
    rows_x = sum(nx - i for i in range(nx))
    fl = 4.0 * W[:, N] * rows_x + 2.0 * nux * nx * W[:, N]
    fl = fl + (4.0 * W[:, :N] * rows_u).sum(axis=1)
    fl = fl + (4.0 * W[:, 1:N] * rows_x + 2.0 * nux * nx * W[:, 1:N]).sum(axis=1)
    return float(fl.sum())


UPDATE_SHAPES = {"update4096": (4096, 50, 12, 4, 0.08), "update1024x60": (1024, 64, 60, 15, 0.06)}


def bench_update(args):
    """Factorisation updates, float64: every instance gets a few active-set changes per step (box
    rows, two per stage, each changed with a probability chosen for about 8 changes per instance),
    applied as penalty updates and, on the next step, removed again (downdates).  Timed per step:
    the data modification, the factor update and a solve, beside a refactorisation of the same
    modified data and the same solve.  Shapes: the batch-4096 workload (N = 50, nx = 12, nu = 4),
    where the rank of the change is close to nx, and a mass-spring-sized state (1024 instances,
    N = 64, nx = 60, nu = 15: 30 masses, a quarter of them actuated), where it is far below."""
    import torch
    import synth
    import paper_2512_09058_amd as L
    from paper_2512_09058_amd import update as U
    from oracle import riccati, update as oupd
    batch, N, nx, nu, density = UPDATE_SHAPES[args.workload]
    m = 2
    prob = synth.make_batch(2) if args.workload == "update4096" else synth.make_batch(2, batch, N=N, nx=nx, nu=nu)
    data = L.pack(prob)
    plan = L.Plan(N, nx, nu, batch=batch, mode="f64")
    data["S"] = torch.zeros(plan.totals["S"], dtype=torch.float64, device="cuda")
    ws = plan.workspace()
    info = torch.zeros(batch, dtype=torch.int32, device="cuda")
    x, u, lam = plan.empty_outputs()
    rel = torch.zeros(batch, dtype=torch.float64, device="cuda")
    C, D, dsig = synth.random_update_rows(31, batch, N, nx, nu, m, density=density)
    rows = [U.pack_rows(C, D, dsig), U.pack_rows(C, D, -dsig)]
    uws = U.workspace(plan)
    L.factor(plan, data, ws, info)
    stream = torch.cuda.current_stream()
    keys = ["update_data", "factor_update", "solve_after_update", "factor", "solve_after_factor"]
    t = {k: [] for k in keys}
    bad = 0
    for s_ in range(args.warmup + args.steps):
        rw = rows[s_ % 2]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        e[0].record(stream)
        U.update_data(plan, rw, data, stream=stream)
        e[1].record(stream)
        U.factor_update(plan, data, rw, ws, info, uws, stream=stream)
        e[2].record(stream)
        L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=1e-10, max_it=0, check_res=True, stream=stream)
        e[3].record(stream)
        L.factor(plan, data, ws, info, stream=stream)
        e[4].record(stream)
        L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=1e-10, max_it=0, check_res=True, stream=stream)
        e[5].record(stream)
        if s_ >= args.warmup:
            for i, k in enumerate(keys):
                t[k].append((e[i], e[i + 1]))
        if s_ == args.warmup + args.steps - 1:
            torch.cuda.synchronize()
            bad = int((info != 0).sum().item())
    torch.cuda.synchronize()
    ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in t.items()}
    ms_upd = ms["update_data"] + ms["factor_update"]
    # the last step's state: modified when the step count is odd
    modified = (args.warmup + args.steps) % 2 == 1
    errs = []
    for i in (0, batch - 1):
        p = prob.instance(i)
        q = oupd.modified_problem(p, C[i], D[i], dsig[i]) if modified else p
        ref = riccati.solve(q)
        sol = tuple(L.unpack(plan, n_, a_, i) for n_, a_ in (("x", x), ("u", u), ("lam", lam)))
        errs.append(max(np.abs(a - b).max() for a, b in zip(sol, ref)) / max(np.abs(b).max() for b in ref))
    fl = update_flops(dsig, N, nx, nu)
    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        cnt = 0
        while time.perf_counter() - t0 < 10.0 and cnt < batch:
            q = oupd.modified_problem(prob.instance(cnt), C[cnt], D[cnt], dsig[cnt])
            riccati.solve(q)
            cnt += 1
        tc = (time.perf_counter() - t0) / cnt
        cpu = {"value": 1.0 / tc, "unit": "solves/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{cnt} instances: the oracle's modified problem and its Riccati solve (numpy float64, one "
                         f"process), {tc * 1e6:.0f} us per instance"}
    nz = (dsig != 0).sum(axis=(1, 2))
    out = {"metric": f"LQ KKT solves/s after a low-rank active-set change, batch {batch} nx={nx} nu={nu} N={N} "
                     "(factor update + solve)",
           "value": batch / ((ms_upd + ms["solve_after_update"]) * 1e-3), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_upd + ms["solve_after_update"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (workload-2 generators; seeded box-constraint rows, penalty changes U(0.5, 2))",
           "config": {"workload": f"batch {batch}, N={N}, nx={nx}, nu={nu}, update rows m={m} per stage, "
                                  f"density {density}",
                      "batch": batch, "N": N, "nx": nx, "nu": nu, "rows_per_instance_mean": float(nz.mean()),
                      "rows_per_instance_max": int(nz.max()), "max_columns": U.max_columns(plan)},
           "ms": ms, "refactor_solves_per_s": batch / ((ms["factor"] + ms["solve_after_factor"]) * 1e-3),
           "update_over_refactor_factorisation_speedup": ms["factor"] / ms_upd,
           "info_nonzero": bad, "fwd_err_vs_oracle_sampled": max(errs),
           "roofline": {"bound": "alu", "kernel": "k_factor_update", "achieved": fl / (ms["factor_update"] * 1e-3) / 1e12,
                        "peak": 78.6, "unit": "TFLOP/s", "frac": fl / (ms["factor_update"] * 1e-3) / 1e12 / 78.6,
                        "traffic": None, "algorithmic_flops_per_launch": fl, "ms_per_launch": ms["factor_update"]},
           "cpu_baseline": cpu}
    print(f"[bench] update: {ms}", file=sys.stderr, flush=True)
    print(json.dumps(out))


def bench_qp(args):
    """Box-constrained QPs of the paper's mass-spring benchmark (M = 12 masses: nx = 24, nu = 6,
    m = 30 bound rows per stage, N = 128, 150 initial states), solved by the proximal augmented
    Lagrangian / semismooth Newton path with its Newton systems on the library's factor and solve:
    cold start (zeros), then, as in the paper's warm-start experiment, the next MPC problem (the first
    input applied to each instance) started from the previous solution shifted by one stage."""
    import torch
    import synth
    import paper_2512_09058_amd as L
    from paper_2512_09058_amd import qp as Q
    from oracle import qp as oqp
    M, N, count = 12, 128, 150
    P = args.qp_intervals
    prob, C, D, bl, bu = synth.mass_spring(M, N, count, seed=0)
    nx, nu = prob.nx, prob.nu
    plan = L.Plan(N, nx, nu, batch=count, mode="f64")
    data = L.pack(prob)
    cons = Q.pack_constraints([C] * count, [D] * count, [bl] * count, [bu] * count)
    m = cons["m"]
    ws, qws = plan.workspace(), Q.workspace(plan, m, P)
    x, u, lam = plan.empty_outputs()
    y = torch.zeros(count * (N + 1) * m, dtype=torch.float64, device="cuda")
    status = torch.zeros(count, dtype=torch.int32, device="cuda")
    iters = torch.zeros(count, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(d, warm, u0=None, y0=None):
        ts = []
        for s_ in range(args.warmup + args.steps):
            if warm:
                u.copy_(u0)
                y.copy_(y0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            Q.solve(plan, d, cons, ws, qws, x, u, lam, y, status, iters, opts={"warm": int(warm), "intervals": P},
                    stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if s_ >= args.warmup:
                ts.append(e0.elapsed_time(e1))
        return float(np.mean(ts)), float(np.max(ts))

    cold_ms, cold_max = timed(data, False)
    st_cold, it_cold = status.cpu().numpy(), iters.cpu().numpy()
    uh = u.view(count, N, nu).cpu().numpy()
    yh = y.view(count, N + 1, m).cpu().numpy()
    sol0 = [L.unpack(plan, n_, t_, 0) for n_, t_ in (("x", x), ("u", u), ("lam", lam))]
    # the next MPC problem: x_init <- A x_init + B u_0; start from the solution shifted by one stage
    x1 = np.einsum("bij,bj->bi", prob.A[:, 0], prob.x0) + np.einsum("bij,bj->bi", prob.B[:, 0], uh[:, 0])
    data2 = dict(data)
    data2["x0"] = torch.from_numpy(np.ascontiguousarray(x1).reshape(-1)).to("cuda")
    us = np.concatenate([uh[:, 1:], uh[:, -1:]], axis=1)
    ys = np.concatenate([yh[:, 1:], yh[:, -1:]], axis=1)
    warm_ms, warm_max = timed(data2, True, torch.from_numpy(us.reshape(-1)).to("cuda"),
                              torch.from_numpy(ys.reshape(-1)).to("cuda"))
    st_warm, it_warm = status.cpu().numpy(), iters.cpu().numpy()
    # checks: the oracle's certificate of sampled GPU results and its solution of instance 0 (cold)
    cert = []
    for i in (0, count - 1):
        p2 = prob.instance(i)
        p2.x0 = x1[i]
        xs, uu, ls = (L.unpack(plan, n_, t_, i) for n_, t_ in (("x", x), ("u", u), ("lam", lam)))
        cert.append(max(oqp.certificate(p2, C, D, bl, bu, xs, uu, ls, y.view(count, N + 1, m)[i].cpu().numpy())))
    cpu = None
    fwd = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        cnt = 0
        while time.perf_counter() - t0 < 10.0 and cnt < count:
            r = oqp.solve(prob.instance(cnt), C, D, bl, bu, linear="banded")
            if cnt == 0:
                fwd = max(np.abs(a - b).max() for a, b in zip(sol0, r[:3])) / max(np.abs(b).max() for b in r[:3])
            cnt += 1
        tc = (time.perf_counter() - t0) / cnt
        cpu = {"value": 1.0 / tc, "unit": "QPs/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{cnt} cold-start instances through the oracle's augmented-Lagrangian solver with banded "
                         f"Newton solves (numpy float64, one process), {tc:.2f} s per QP",
               "gpu_vs_oracle_inst0_fwd_err": fwd}
    out = {"metric": "box-constrained QP solves/s, mass-spring benchmark M=12 (nx=24, nu=6), N=128, 150 initial states",
           "value": count / (cold_ms * 1e-3), "unit": "QPs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": cold_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (the paper's mass-spring problem generated from its equations; seeded initial states)",
           "config": {"workload": "mass-spring M=12, N=128, 150 QPs, box bounds |pos| <= 4, |u| <= 0.5",
                      "batch": count, "N": N, "nx": nx, "nu": nu, "m": m,
                      "newton_systems": f"parallel-in-time, {P} intervals" if P > 1 else "serial plan"},
           "cold": {"ms_batch": cold_ms, "ms_batch_max": cold_max, "converged": int((st_cold == 0).sum()),
                    "inner_steps_mean": float(it_cold.mean()), "inner_steps_max": int(it_cold.max())},
           "warm": {"ms_batch": warm_ms, "ms_batch_max": warm_max, "converged": int((st_warm == 0).sum()),
                    "inner_steps_mean": float(it_warm.mean()), "inner_steps_max": int(it_warm.max()),
                    "qps_per_s": count / (warm_ms * 1e-3)},
           "certificate_max_sampled": max(cert),
           "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": "ms", "frac": None,
                        "traffic": None,
                        "note": "a chain of dependent Newton steps (factor, solve, line search) with one host "
                                "synchronisation per step; per-kernel times in the kernel trace"},
           "cpu_baseline": cpu}
    print(f"[bench] qp: cold {cold_ms:.2f} ms ({it_cold.mean():.1f} steps), warm {warm_ms:.2f} ms "
          f"({it_warm.mean():.1f} steps)", file=sys.stderr, flush=True)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-it", type=int, default=10)
    ap.add_argument("--distinct", type=int, default=0,
                    help="large / adjoint workloads: generate only this many distinct instances and repeat them "
                         "(0: all distinct)")
    ap.add_argument("--qp-intervals", type=int, default=0,
                    help="QP workload: intervals of the parallel-in-time Newton solves (0: serial plan)")
    ap.add_argument("--pit-intervals", type=int, nargs="*", default=[4, 8, 16],
                    help="large workload: interval counts of the parallel-in-time path")
    ap.add_argument("--workload", choices=["batch4096", "uneven2048", "large64", "adjoint1024", "single20", "blocktri",
                                           "update4096", "update1024x60", "qp_mass_spring", "shapes4096"],
                    default="batch4096",
                    help="measure another workload instead (its own JSON line): the 2048-instance uneven batch, "
                         "the 64-instance large-state batch, or the 1024-instance forward+adjoint batch")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (scale for HBM counters)")
    args = ap.parse_args()
    print(f"[bench] workload {args.workload}", file=sys.stderr, flush=True)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the instances of the batch are "
              "independent, so more GPUs would each run this same kernel on their own share; no multi-GPU run "
              "is built.", file=sys.stderr)
        sys.exit(2)

    import torch
    print("[bench] torch imported", file=sys.stderr, flush=True)
    if args.calibrate_copy:
        n = 1 << 27  # float64 elements = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8}))
        return

    import synth
    import paper_2512_09058_amd as L

    if args.workload == "uneven2048":
        return bench_uneven(args)
    if args.workload == "large64":
        return bench_large(args)
    if args.workload == "adjoint1024":
        return bench_adjoint(args)
    if args.workload == "single20":
        return bench_single(args)
    if args.workload == "blocktri":
        return bench_blocktri(args)
    if args.workload in UPDATE_SHAPES:
        return bench_update(args)
    if args.workload == "qp_mass_spring":
        return bench_qp(args)
    if args.workload == "shapes4096":
        return bench_shapes(args)

    t0 = time.perf_counter()
    prob = synth.make_batch(2)
    data = L.pack(prob)
    torch.cuda.synchronize()
    print(f"[bench] generated and uploaded workload in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    res = {}
    for mode, max_it in (("f64", 0), ("mixed_f32", args.max_it)):
        r = run_path(mode, data, args.steps, args.warmup, max_it)
        res[mode] = r
        print(f"[bench] {mode}: {r['ms_per_step']:.3f} ms/step (factor {r['ms_factor']:.3f} ms, solve "
              f"{r['ms_solve']:.3f} ms), max rel_res {r['rel'].max():.2e}, iters max {r['iters'].max()}, "
              f"variant {r['plan'].variant}", file=sys.stderr, flush=True)

    m, f = res["mixed_f32"], res["f64"]
    ok = all(np.all(r["info"] == 0) and r["rel"].max() <= TOL for r in res.values())
    cpu = None
    if not args.no_cpu:
        # the CPU leg: the oracle timed on a sample, and its residual routine applied to sampled GPU
        # solutions of both paths
        from oracle import kkt
        cpu = cpu_baseline(args.cpu_sample)
        cpu["gpu_vs_oracle_sampled"] = {
            mode: max(kkt.residual(prob.instance(i), *[L.unpack(r["plan"], n, r[n], i) for n in ("x", "u", "lam")])[1]
                      for i in (0, 1, 777, 2048, 4095))
            for mode, r in res.items()}

    # roofline of the dominant kernel of the reported (mixed) path: algorithmic bytes are one
    # factor sweep / one forward + residual pass; the refinement passes are reported apart
    copy_gbs = measure_copy_bandwidth()
    it_mean = float(np.mean(m["iters"]))
    names = {"factor": f"k_factor_small<{NX}, {NU}, float, float, false, false>",
             "solve": f"k_solve_small<{NX}, {NU}, float, false, false>"}
    kern = {"factor": (m["ms_factor"], algorithmic_bytes_factor(BATCH, N, NX, NU, 4)),
            "solve": (m["ms_solve"], algorithmic_bytes_solve(N, NX, NU, 4, m["iters"]))}
    dom = max(kern, key=lambda k: kern[k][0])
    ms, by = kern[dom]
    tr = profiled_traffic(names[dom]) if m["plan"].variant == "small" else None
    ref_b = refinement_bytes(N, NX, NU, 4, m["iters"])
    f64k = {"factor": {"ms": f["ms_factor"], "algorithmic_bytes": algorithmic_bytes_factor(BATCH, N, NX, NU, 8)},
            "solve": {"ms": f["ms_solve"], "algorithmic_bytes": algorithmic_bytes_solve(N, NX, NU, 8, f["iters"])}}
    for v in f64k.values():
        v["GBps"] = v["algorithmic_bytes"] / (v["ms"] * 1e-3) / 1e9
    mxk = {k: {"ms": v[0], "algorithmic_bytes": v[1], "GBps": v[1] / (v[0] * 1e-3) / 1e9} for k, v in kern.items()}
    mxk["solve"]["refinement_implementation_bytes"] = ref_b
    mxk["solve"]["GBps_with_refinement_bytes"] = (kern["solve"][1] + ref_b) / (m["ms_solve"] * 1e-3) / 1e9
    # the whole step against the fused ideal (inputs read once, x, u, lam written once)
    data_b, _ = stage_sizes(NX, NU)
    ideal = BATCH * N * (8 * data_b + 8 * (2 * NX + NU))
    step_vs_ideal = {"ideal_bytes": ideal, "ideal_ms_at_peak": ideal / (HBM_PEAK_GBS * 1e9) * 1e3,
                     "mixed_frac": ideal / (m["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "fp64_frac": ideal / (f["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    out = {
        "metric": METRIC,
        "value": BATCH / (m["ms_per_step"] * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 stage products + f64 Cholesky/residual/refinement",
        "data": "synthetic (seeded generators of the workload)",
        "config": {"workload": "batch 4096 LQ problems, N=50, nx=12, nu=4 (mixed f32 + f64 refinement)",
                   "batch": BATCH, "N": N, "nx": NX, "nu": NU, "tol": TOL, "max_it": args.max_it,
                   "variant": m["plan"].variant},
        "fp64": {"value": BATCH / (f["ms_per_step"] * 1e-3), "ms_per_step": f["ms_per_step"],
                 "max_rel_res": float(f["rel"].max()), "kernels": f64k},
        "mixed": {"max_rel_res": float(m["rel"].max()), "iters_mean": it_mean, "iters_max": int(m["iters"].max()),
                  "kernels": mxk},
        "mixed_over_fp64": f["ms_per_step"] / m["ms_per_step"],
        "equal_residual_ok": bool(ok),
        "step_vs_fused_ideal": step_vs_ideal,
        "roofline": hbm_roofline(names[dom], by, ms, copy_gbs, tr),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
