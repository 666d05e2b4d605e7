#!/usr/bin/env python
"""Throughput of singular value soft-thresholding through the polar
decomposition on one MI355X.

Workload (one step): the plain FP32 form on three 4096 x 4096 matrices
A = U diag(sigma) V^T (Haar U, V; sigma log-spaced 10 .. 1e-3), one per
threshold tau at the 10 / 50 / 90 % quantile of sigma (each gap-clamped so
every singular value sits >= 5 % from tau), 20 polar iterations, one matrix
per launch sequence.  Inputs, outputs and workspace are resident in HBM
before the timed region.

Printed: one JSON line with matrices/s, useful TFLOP/s and MFMA utilisation
against the FP32 MFMA peak, per-matrix latency p50/p99, the dominant
kernel's roofline (timed per launch with HIP events on its own stream
through the library's trace facility), and the FP64 CPU oracle timed on a
bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "bf16": 2516.6, "fp8": 5033.2}
HBM_GBS = 8000.0
METRIC = "SVT matrices/s + MFMA util (bf16 vs fp32) at rel err≤1e-2; p50/p99 latency"


def useful_flops(m, n, iters, with_p=True):
    """Flops the method must perform for one SVT (symmetric products at half):
    K (3 l s^2 + s^3) for P, l s^2 for the Gram, 3 K s^3 for S, 2 l s^2 for the
    final product."""
    s, l = min(m, n), max(m, n)
    f = l * s * s + 3 * iters * s ** 3 + 2 * l * s * s
    if with_p:
        f += iters * (3 * l * s * s + s ** 3)
    return float(f)


def kernel_source_sha():
    """Hash of the MFMA tile kernel's code (the gemm_*.hip units only
    instantiate it): a stored traffic figure is reported only while it
    matches the kernel that was measured."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2607_22484_amd", "csrc")
    h = hashlib.sha256()
    for f in ("device.h", "tile.h", "kernels.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, n):
    """HBM bytes per launch of ``kernel`` in the n x n FP32 workload, from
    its PMC summary under profiles/ (FETCH_SIZE + WRITE_SIZE, each scaled by
    a plain copy kernel's reading), or None when absent or taken from other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_svt%d_fp32.txt" % n)
    sha = kernel_source_sha()
    if not os.path.isfile(path):
        return None
    for f in (path,):
        with open(f) as fh:
            for line in fh:
                if not line.startswith("traffic "):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("source_sha") == sha:
                    return float(kv["traffic_bytes"])
    return None


def calibration_copy(torch, dev, nbytes=1 << 30):
    """One plain elementwise pass (read nbytes, write nbytes) whose PMC
    FETCH_SIZE / WRITE_SIZE readings scale the kernel's counters to bytes."""
    x = torch.ones(nbytes // 4, device=dev)
    y = torch.empty_like(x)
    torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    del x, y


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline_leg(problems, results, n_sample, checks):
    """The FP64 Jacobi oracle on the host cores: timed on a bounded sample of
    the main workload, and used for every accuracy figure of the run (the
    GPU legs hand over host copies of their outputs in ``checks``; nothing
    else in this file calls the oracle)."""
    import oracle
    from paper_2607_22484_amd import inputs

    errs = {}
    for pb, Y in zip(problems, results):
        ref = oracle.svt_from_svd(pb.U, pb.sigma, pb.V, pb.tau)
        nref = np.linalg.norm(ref)
        err = np.linalg.norm(Y - ref)
        delta = float(np.linalg.norm(pb.A.astype(np.float64) - pb.A64))  # prox is 1-Lipschitz
        errs[pb.name] = {"rel_err": float(err / nref), "rel_err_bound_fp32_input": float((err + delta) / (nref - delta))}
    failures = []
    for check in checks:
        try:
            check(oracle)
        except Exception as e:  # one failed accuracy check must not lose the rest of the line
            failures.append("%s: %s" % (getattr(check, "__qualname__", "check"), e))
            print("[bench] accuracy check failed: %s" % failures[-1], file=sys.stderr, flush=True)
    n_main = problems[0].A.shape[0]
    if n_sample >= n_main:
        sample = problems[len(problems) // 2]   # the main workload's own tau = q50 matrix
    else:
        sample = inputs.square_case(0.5, n=n_sample)
    t0 = time.perf_counter()
    oracle.svt(sample.A, sample.tau)
    dt = time.perf_counter() - t0
    scale = (n_main / sample.A.shape[0]) ** 3
    what = ("one-sided Jacobi SVD + threshold (FP64, OpenMP) of one %dx%d matrix of the main workload "
            "(tau at the 50%% quantile) in %.2f s" % (sample.A.shape[0], sample.A.shape[1], dt))
    if scale != 1.0:
        what += ", scaled by (%d/%d)^3 = %.0f to one %dx%d matrix" % (n_main, sample.A.shape[0], scale, n_main,
                                                                       n_main)
    cpu = {"value": 1.0 / (dt * scale), "unit": "matrices/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": what}
    return cpu, errs, failures


def time_calls(torch, fn, reps):
    """Average device time of fn() over reps calls (events on the current stream)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def precision_leg(psvt, torch, dev, checks, problems=None):
    """Precision form: BF16 operand iterations (18) + 2 FP32, on rank-200
    signal + noise, 8192 x 4096 and 4096 x 8192 (left-sided); beside it
    FP32, all 20 iterations in split bf16 (no FP32 refinement), the H-form,
    plain-BF16 P, and the serving schedule (6 FP8 + 12 BF16 + 2 FP32)."""
    from paper_2607_22484_amd import inputs
    out = {}
    for (m, n) in [(8192, 4096), (4096, 8192)]:
        pb = inputs.noisy_lowrank(m, n, rank=200, idx=0 if m > n else 1, norm_iters=40)
        A = torch.from_numpy(pb.A).to(dev)
        Y = torch.empty_like(A)
        row = {}
        for name, kw in [("fp32", dict()), ("bf16", dict(n_bf16=18)),
                         ("bf16_plainP", dict(n_bf16=18, flags=psvt.FLAG_PLAIN_P)),
                         ("bf16_hform", dict(n_bf16=18, flags=psvt.FLAG_HFORM)),
                         ("bf16_hform_plainS", dict(n_bf16=18, flags=psvt.FLAG_HFORM | psvt.FLAG_PLAIN_S)),
                         ("split_bf16_all", dict(n_bf16=20)),
                         ("fp8", dict(n_fp8=6, n_bf16=12)),
                         ("fp8_plainP", dict(n_fp8=6, n_bf16=12, flags=psvt.FLAG_PLAIN_P))]:
            cfg, _ = psvt.make_config(iters=20, **kw)
            ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, m, n, cfg), dtype=torch.uint8, device=dev)
            ms = time_calls(torch, lambda: psvt.svt(A, pb.tau, iters=20, out=Y, ws=ws, **kw), 3)
            psvt.trace_begin()
            psvt.svt(A, pb.tau, iters=20, out=Y, ws=ws, **kw)
            torch.cuda.synchronize()
            tr = psvt.trace_end()
            mfma = {}
            for t in tr:
                if t["flops"]:
                    d = t["name"].split("_")[1]
                    a = mfma.setdefault(d, [0.0, 0.0])
                    a[0] += t["flops"] * (3 if d == "bf16x3" else 1)
                    a[1] += t["total_ms"]
            peak = {"f32": 157.3, "bf16": 2516.6, "bf16x3": 2516.6, "fp8": 5033.2}
            row[name] = {"ms": ms, "matrices_per_s": 1e3 / ms,
                         "useful_tflops": useful_flops(m, n, 20) / (ms * 1e-3) / 1e12,
                         "mfma_util_by_dtype": {d: (f / (t * 1e-3) / 1e12) / peak[d] for d, (f, t) in mfma.items()}}
            if checks is not None:
                Yh = Y.cpu().numpy().astype(np.float64)

                def check(oracle, pb=pb, Yh=Yh, dst=row[name], memo={}):
                    if pb.name not in memo:  # certified compressed reference, once per matrix
                        memo[pb.name] = oracle.svt_gapped(pb.A, pb.tau, k=256, return_bound=True)
                    ref, cert = memo[pb.name]
                    dst["rel_err"] = oracle.rel_fro_err(Yh, ref)
                    dst["reference_certified_to"] = cert
                checks.append(check)
        out["%dx%d" % (m, n)] = row
    # the main workload (three 4096^2 constructed matrices, tau at the 10/50/90 %
    # quantiles) under the low-precision schedules
    if problems:
        As = [torch.from_numpy(pb.A).to(dev) for pb in problems]
        Y = torch.empty_like(As[0])
        row = {}
        for name, kw in [("bf16", dict(n_bf16=18)), ("split_bf16_all", dict(n_bf16=20))]:
            cfg, _ = psvt.make_config(iters=20, **kw)
            ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, *problems[0].A.shape, cfg), dtype=torch.uint8, device=dev)

            def three(kw=kw, ws=ws):
                for A, pb in zip(As, problems):
                    psvt.svt(A, pb.tau, iters=20, out=Y, ws=ws, **kw)
            ms = time_calls(torch, three, 2)
            row[name] = {"ms_per_matrix": ms / len(As), "matrices_per_s": 1e3 * len(As) / ms}
            if checks is not None:
                Ys = []
                for A, pb in zip(As, problems):
                    psvt.svt(A, pb.tau, iters=20, out=Y, ws=ws, **kw)
                    Ys.append(Y.cpu().numpy().astype(np.float64))

                def check(oracle, Ys=Ys, dst=row[name]):
                    worst = 0.0
                    for pb, Yh in zip(problems, Ys):
                        ref = oracle.svt_from_svd(pb.U, pb.sigma, pb.V, pb.tau)
                        delta = float(np.linalg.norm(pb.A.astype(np.float64) - pb.A64))
                        worst = max(worst, (np.linalg.norm(Yh - ref) + delta) / (np.linalg.norm(ref) - delta))
                    dst["worst_rel_err_bound_fp32_input"] = float(worst)
                checks.append(check)
            del ws
        out["main_workload_%dx%d" % problems[0].A.shape] = row
        del As, Y
    return out


def desc_graph(psvt, torch, As, taus, Ys, flags=0, **kw):
    """The device-described batched call (psvt_svt_batched) captured into a
    HIP graph after one eager run; returns (graph, workspace, keep-alive)."""
    cfg, keep = psvt.make_config(iters=20, flags=flags, **kw)
    max_m = max(A.shape[0] for A in As)
    max_n = max(A.shape[1] for A in As)
    dev = As[0].device
    ws = torch.empty(psvt.batched_workspace_bytes(len(As), max_m, max_n, cfg), dtype=torch.uint8, device=dev)
    desc = psvt.device_descriptors(As, taus, Ys, None, dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        psvt.svt_batched_raw(desc.data_ptr(), len(As), max_m, max_n, ws, cfg)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        psvt.svt_batched_raw(desc.data_ptr(), len(As), max_m, max_n, ws, cfg)
    return g, ws, (cfg, keep, desc)


def batched_leg(psvt, torch, dev, checks, count=512):
    """Batched form: 512 matrices, m, n log-uniform in [128, 2048].  Rows:
    the host-planned batch (psvt_batch_*: one graph of grouped launches),
    the device-described batch (psvt_svt_batched) as one graph of per-stage
    launches, and the persistent executor (PSVT_FLAG_PERSISTENT: one
    persistent launch after the setup kernels, graph-captured), per
    precision schedule."""
    from paper_2607_22484_amd import inputs
    pbs = inputs.batch_cases(count=count)
    As = [torch.from_numpy(p.A).to(dev) for p in pbs]
    taus = [p.tau for p in pbs]
    out = {"matrices": count}

    def add_check(row, Ys):
        if checks is None:
            return
        Yh = [Y.cpu().numpy() for Y in Ys]

        def check(oracle, Yh=Yh, dst=row):
            dst["worst_rel_err"] = max(
                oracle.rel_fro_err(Y.astype(np.float64), oracle.svt_from_svd(p.U, p.sigma, p.V, p.tau))
                for p, Y in zip(pbs, Yh))
        checks.append(check)

    useful = None
    for name, kw in [("fp32", dict()), ("bf16", dict(n_bf16=18)),
                     ("bf16_plainP", dict(n_bf16=18, flags=psvt.FLAG_PLAIN_P)), ("split_bf16_all", dict(n_bf16=20))]:
        b = psvt.Batch(As, taus, iters=20, **kw)
        nl, fl = b.stats()
        useful = useful or fl
        ms = time_calls(torch, b.run_graph, 3)
        row = {"ms_per_batch": ms, "matrices_per_s": count / (ms * 1e-3), "useful_tflops": fl / (ms * 1e-3) / 1e12,
               "launches_in_graph": nl}
        add_check(row, b.Ys)
        out[name] = row
        b.close()
        print("[bench] batched %s: %.0f matrices/s" % (name, row["matrices_per_s"]), file=sys.stderr, flush=True)
    # device-described: per-stage launches and the persistent executor
    for name, kw in [("fp32", dict()), ("bf16", dict(n_bf16=18)), ("split_bf16_all", dict(n_bf16=20))]:
        for form, flags in (("desc_staged", 0), ("persistent", psvt.FLAG_PERSISTENT)):
            Ys = [torch.empty_like(A) for A in As]
            g, ws, keep = desc_graph(psvt, torch, As, taus, Ys, flags=flags, **kw)
            ms = time_calls(torch, g.replay, 3)
            row = {"ms_per_batch": ms, "matrices_per_s": count / (ms * 1e-3),
                   "useful_tflops": useful / (ms * 1e-3) / 1e12}
            if flags:
                row["aborted"] = psvt.persistent_aborted(ws)
            add_check(row, Ys)
            out["%s_%s" % (form, name)] = row
            print("[bench] batched %s_%s: %.0f matrices/s" % (form, name, row["matrices_per_s"]), file=sys.stderr,
                  flush=True)
            del g, ws, keep, Ys
            torch.cuda.empty_cache()
    # the plain FP32 form on the same matrices: one matrix per launch sequence
    cfg, _ = psvt.make_config(iters=20)
    ws = torch.empty(max(psvt.workspace_bytes(psvt.OP_SVT, p.shape[0], p.shape[1], cfg) for p in pbs),
                     dtype=torch.uint8, device=dev)
    Ys = [torch.empty_like(a) for a in As]

    def single():
        for a, y, t in zip(As, Ys, taus):
            psvt.svt(a, t, iters=20, out=y, ws=ws)
    ms = time_calls(torch, single, 1)
    out["fp32_single_calls"] = {"ms_per_batch": ms, "matrices_per_s": count / (ms * 1e-3)}
    return out


def small_leg(psvt, torch, dev, checks, reps=50):
    """The small case (256 x 128 constructed, tau = 0.1, 20 FP32 iterations):
    latency of one SVT from eager launches and from a one-item batch graph
    (the same kernels, one submission)."""
    from paper_2607_22484_amd import inputs
    pb = inputs.small_case()
    A = torch.from_numpy(pb.A).to(dev)
    Y = torch.empty_like(A)
    cfg, _ = psvt.make_config(iters=20)
    ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, *pb.A.shape, cfg), dtype=torch.uint8, device=dev)
    eager_ms = time_calls(torch, lambda: psvt.svt(A, pb.tau, iters=20, out=Y, ws=ws), reps)
    b = psvt.Batch([A], [pb.tau], iters=20)
    graph_ms = time_calls(torch, b.run_graph, reps)
    nl, _ = b.stats()
    Yp = torch.empty_like(A)
    g, pws, keep = desc_graph(psvt, torch, [A], [pb.tau], [Yp], flags=psvt.FLAG_PERSISTENT)
    persist_ms = time_calls(torch, g.replay, reps)
    out = {"shape": list(pb.A.shape), "eager_us": 1e3 * eager_ms, "graph_us": 1e3 * graph_ms, "launches": nl,
           "persistent_graph_us": 1e3 * persist_ms, "persistent_aborted": psvt.persistent_aborted(pws)}
    del g, pws, keep
    if checks is not None:
        Yh = b.Ys[0].cpu().numpy().astype(np.float64)

        def check(oracle, dst=out):
            dst["rel_err"] = oracle.rel_fro_err(Yh, oracle.svt(pb.A, pb.tau))
        checks.append(check)
    b.close()
    return out


def rank_leg(psvt, torch, dev, checks, n=4096, r=256, reps=3):
    """Corollary 1 on the main workload's recipe: the best rank-r
    approximation [A]_r = A (I + S)/2 of a 4096^2 matrix (no polar factor),
    r = 256, tau between sigma_256 and sigma_257, plain FP32, 20 iterations."""
    from paper_2607_22484_amd import inputs
    pb = inputs.rank_case(r=r, n=n)
    A = torch.from_numpy(pb.A).to(dev)
    Y = torch.empty_like(A)
    cfg, _ = psvt.make_config(iters=20)
    ws = torch.empty(psvt.workspace_bytes(psvt.OP_RANK_R, n, n, cfg), dtype=torch.uint8, device=dev)
    ms = time_calls(torch, lambda: psvt.rank_r(A, pb.tau, iters=20, out=Y, ws=ws), reps)
    row = {"shape": [n, n], "r": r, "ms": ms, "matrices_per_s": 1e3 / ms,
           "useful_tflops": useful_flops(n, n, 20, with_p=False) / (ms * 1e-3) / 1e12}
    if checks is not None:
        Yh = Y.cpu().numpy().astype(np.float64)

        def check(oracle, pb=pb, Yh=Yh, dst=row):
            # the constructed factors give [A]_r exactly (Eckart-Young)
            ref = (pb.U[:, :r] * pb.sigma[:r]) @ pb.V[:, :r].T
            dst["rel_err_vs_construction"] = float(np.linalg.norm(Yh - ref) / np.linalg.norm(ref))
        checks.append(check)
    return row


def fig1_leg(psvt, torch, dev, checks, taus=(1.0, 17.0, 33.0), kmax=30):
    """Relative error against the number of polar iterations (the experiment
    of Fig. 1): one i.i.d. Gaussian 301 x 300 matrix (singular values inside
    the Marchenko-Pastur edges ~0.03 .. 34.7), tau near the bottom, middle
    and top of the spectrum, 1..kmax iterations, four schedules: FP32, BF16
    with the last 2 iterations FP32 (plain or split-bf16 P), and BF16
    throughout (as the paper's experiment).  Errors are filled in by the CPU
    oracle leg."""
    from paper_2607_22484_amd import inputs
    A = inputs.gaussian(301, 300, cfg=inputs.CFG_FIG1)
    Ad = torch.from_numpy(A).to(dev)
    plain = psvt.FLAG_PLAIN_P | psvt.FLAG_PLAIN_S
    scheds = {"fp32": lambda k: {}, "bf16_2fp32": lambda k: {"n_bf16": max(k - 2, 0)},
              "bf16_plainP_2fp32": lambda k: {"n_bf16": max(k - 2, 0), "flags": psvt.FLAG_PLAIN_P},
              "bf16_plain": lambda k: {"n_bf16": k, "flags": plain}}
    outs = {}
    t0 = time.perf_counter()
    for name, kw in scheds.items():
        for tau in taus:
            outs[(name, tau)] = [psvt.svt(Ad, tau, iters=k, **kw(k)).cpu().numpy() for k in range(1, kmax + 1)]
    torch.cuda.synchronize()
    out = {"shape": [301, 300], "taus": list(taus), "iters": list(range(1, kmax + 1)),
           "gpu_seconds_all_calls": time.perf_counter() - t0, "rel_err": {}}
    if checks is not None:
        def check(oracle, dst=out):
            U, sv, V = oracle.svd(A)
            dst["sigma_min_max"] = [float(sv[-1]), float(sv[0])]
            dst["min_rel_gap"] = {str(t): float(np.min(np.abs(sv / t - 1.0))) for t in taus}
            for (name, tau), Ys in outs.items():
                ref = oracle.svt_from_svd(U, sv, V, tau)
                dst["rel_err"].setdefault(name, {})[str(tau)] = [
                    float("%.3g" % oracle.rel_fro_err(Y.astype(np.float64), ref)) for Y in Ys]
        checks.append(check)
    return out


def fig2_leg(psvt, torch, dev, checks, sizes=(1000, 2000, 3000, 4000, 5000), draws=5, iters=25):
    """Run time against size (the experiment of Fig. 2, the polar method
    only): i.i.d. Gaussian m x (m+1) matrices (left-sided), 25 iterations,
    5 draws per size, tau = sqrt(m) (mid-spectrum: the singular values fill
    [0, 2 sqrt(m)]); FP32, the BF16 schedule with split-bf16 P and 2 FP32
    iterations, and BF16 throughout (as the paper's experiment).  Accuracy
    of the first 1000 x 1001 draw is filled in by the CPU oracle leg."""
    from paper_2607_22484_amd import inputs
    scheds = {"fp32": {}, "bf16_2fp32": {"n_bf16": iters - 2},
              "bf16_plain": {"n_bf16": iters, "flags": psvt.FLAG_PLAIN_P | psvt.FLAG_PLAIN_S}}
    out = {"iters": iters, "draws": draws, "ms_per_svt": {}}
    keep = {}
    for m in sizes:
        As = [torch.from_numpy(inputs.gaussian(m, m + 1, cfg=inputs.CFG_FIG2, idx=d)).to(dev) for d in range(draws)]
        tau = math.sqrt(m)
        Y = torch.empty_like(As[0])
        for name, kw in scheds.items():
            cfg, _ = psvt.make_config(iters=iters, **kw)
            ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, m, m + 1, cfg), dtype=torch.uint8, device=dev)
            ms = [time_calls(torch, lambda A=A: psvt.svt(A, tau, iters=iters, out=Y, ws=ws, **kw), 1) for A in As]
            out["ms_per_svt"].setdefault(name, {})[str(m)] = float(np.mean(ms))
            if m == sizes[0]:
                psvt.svt(As[0], tau, iters=iters, out=Y, ws=ws, **kw)
                keep[name] = Y.cpu().numpy().astype(np.float64)
            del ws
        if m == sizes[0]:
            keep["A"] = As[0].cpu().numpy()
            keep["tau"] = tau
        del As, Y
    if checks is not None:
        def check(oracle, dst=out):
            ref = oracle.svt(keep["A"], keep["tau"])
            dst["rel_err_%dx%d" % (sizes[0], sizes[0] + 1)] = {
                name: oracle.rel_fro_err(keep[name], ref) for name in scheds}
        checks.append(check)
    return out


def _fingerprint(torch, Y):
    """A checksum of the bits of Y (position-weighted sum of its int32 words,
    wrapping in int64): equal results give equal fingerprints."""
    v = Y.contiguous().view(torch.int32).flatten().to(torch.int64)
    w = torch.arange(1, v.numel() + 1, device=Y.device, dtype=torch.int64)
    return (int(v.sum().item()), int((v * w).sum().item()))


def serving_leg(psvt, torch, dev, checks, rates=(100, 200, 500, 1000, 2000, 5000), count=2000):
    """Serving form: Poisson arrivals at each rate, ``count`` requests per
    rate; short side s = round(exp U[ln 256, ln 4096]), square or 2:1 either
    way; rank r in {16, 64, 256} (<= s/4) signal + noise of std 0.01/sqrt(n),
    tau = 2 x 0.01 (sqrt(m) + sqrt(n)) / sqrt(n); 6 FP8 + 12 BF16 + 2 FP32
    iterations.  Accuracy: every served result is compared bit for bit with
    the single call of the same schedule on the same request (through a
    checksum of its bits), and the single calls of one request per size
    bucket are compared with the certified oracle by the CPU leg."""
    from paper_2607_22484_amd import inputs
    g = torch.Generator(device=dev)
    g.manual_seed(2607)
    shapes = inputs.serve_shapes(count, idx=0)
    reqs = []
    for (m, n, r) in shapes:
        U = torch.linalg.qr(torch.randn(m, r, device=dev, generator=g))[0]
        V = torch.linalg.qr(torch.randn(n, r, device=dev, generator=g))[0]
        s = 1.0 + 9.0 * torch.rand(r, device=dev, generator=g)
        A = ((U * s) @ V.T + torch.randn(m, n, device=dev, generator=g) * (0.01 / math.sqrt(n))).contiguous()
        reqs.append((A, 2 * 0.01 * (math.sqrt(m) + math.sqrt(n)) / math.sqrt(n)))
        del U, V
    torch.cuda.synchronize()
    print("[bench] serving: %d requests generated" % len(reqs), file=sys.stderr, flush=True)
    out = {"requests_per_rate": count, "schedule": "6 FP8 + 12 BF16 (split bf16) + 2 FP32"}
    # the plain FP32 form on the same requests, one matrix per launch sequence
    cfg, _ = psvt.make_config(iters=20)
    ws = torch.empty(max(psvt.workspace_bytes(psvt.OP_SVT, A.shape[0], A.shape[1], cfg) for A, _ in reqs),
                     dtype=torch.uint8, device=dev)
    Y1 = torch.empty(max(A.numel() for A, _ in reqs), device=dev)

    def single():
        for A, tau in reqs:
            psvt.svt(A, tau, iters=20, out=Y1[:A.numel()].view(A.shape), ws=ws)
    ms = time_calls(torch, single, 1)
    out["fp32_single_calls"] = {"requests": len(reqs), "matrices_per_s": len(reqs) / (ms * 1e-3)}
    del ws
    # the served schedule as single calls, one request at a time (no batching)
    lp = dict(n_fp8=6, n_bf16=12)
    cfg, _ = psvt.make_config(iters=20, **lp)
    ws = torch.empty(max(psvt.workspace_bytes(psvt.OP_SVT, A.shape[0], A.shape[1], cfg) for A, _ in reqs),
                     dtype=torch.uint8, device=dev)

    def single_lp():
        for A, tau in reqs:
            psvt.svt(A, tau, iters=20, out=Y1[:A.numel()].view(A.shape), ws=ws, **lp)
    ms = time_calls(torch, single_lp, 1)
    out["lp_single_calls"] = {"requests": len(reqs), "matrices_per_s": len(reqs) / (ms * 1e-3)}
    # reference fingerprints of the single calls, and the sampled results
    buckets = {}
    for i, (m, n, r) in enumerate(shapes):
        buckets.setdefault(int(math.log2(min(m, n))), i)
    sample = sorted(buckets.values())
    ref_fp, kept = [], {}
    for i, (A, tau) in enumerate(reqs):
        Y = Y1[:A.numel()].view(A.shape)
        psvt.svt(A, tau, iters=20, out=Y, ws=ws, **lp)
        ref_fp.append(_fingerprint(torch, Y))
        if i in sample:
            kept[i] = (A.cpu().numpy(), Y.cpu().numpy().astype(np.float64), tau, shapes[i])
    del ws, Y1
    torch.cuda.empty_cache()
    for rate in rates:
        srv = psvt.Server(budget_bytes=64 << 30, max_slots=64, iters=20, **lp)
        gaps = np.random.default_rng(rate).exponential(1.0 / rate, size=len(reqs))
        t = time.perf_counter()
        tickets = []
        for (A, tau), gp in zip(reqs, gaps):
            t += gp
            while time.perf_counter() < t:
                pass
            tickets.append(srv.submit(A, tau))
        srv.drain(timeout=900)
        st = srv.stats()
        same = sum(_fingerprint(torch, Y) == f for (_, Y), f in zip(tickets, ref_fp))
        out["%d_per_s" % rate] = {
            "completed": st["completed"], "failed": st["failed"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "launches": st["launches"], "matrices_per_s": st["matrices_per_s"], "queue_p99_ms": st["queue_p99_ms"],
            "peak_pool_gib": st["peak_bytes"] / 2 ** 30, "bitwise_equal_to_single_call": same}
        srv.close()
        del tickets
        torch.cuda.empty_cache()
        print("[bench] serving %d/s: %.1f matrices/s, p50 %.1f ms, p99 %.1f ms, %d/%d bitwise equal"
              % (rate, st["matrices_per_s"], st["p50_ms"], st["p99_ms"], same, len(reqs)), file=sys.stderr,
              flush=True)
    if checks is not None:
        def check(oracle, dst=out):
            rows = []
            for i in sample:
                A, Y, tau, (m, n, r) = kept[i]
                ref, cert = oracle.svt_gapped(A, tau, k=r + 64, return_bound=True)
                rows.append({"shape": [m, n], "rank": r, "rel_err": oracle.rel_fro_err(Y, ref),
                             "reference_certified_to": cert})
            dst["sampled_single_call_errors"] = rows
            dst["worst_sampled_rel_err"] = max(x["rel_err"] for x in rows)
        checks.append(check)
    del reqs
    return out


def _completion_reference(oracle, G, tau, r):
    """Reference thresholding of one completion iterate: the certified
    compressed oracle with k = r + 64, then with a wider basis and more power
    iterations; below 1300 on the short side the full Jacobi SVD when neither
    certifies to 1e-4.  Returns (reference, certified relative bound or 0 for
    the full SVD or None when uncertified, how)."""
    s = min(G.shape)
    for k, q in ((r + 64, 10), (min(s, 2 * r + 256), 16)):
        try:
            ref, cert = oracle.svt_gapped(G, tau, k=k, power_iters=q, max_rel_bound=1e-4, return_bound=True)
            return ref, cert, "compressed k=%d" % k
        except RuntimeError as e:
            print("[bench] completion reference %dx%d, k=%d: %s" % (G.shape + (k, e)), file=sys.stderr, flush=True)
    if s <= 1300:
        sv = np.linalg.svd(G.astype(np.float64), compute_uv=False)
        print("[bench] completion iterate %dx%d: %d singular values above tau=%.4g; next %s"
              % (G.shape + (int((sv > tau).sum()), tau, np.array2string(sv[(sv > tau).sum():][:4], precision=4))),
              file=sys.stderr, flush=True)
        return oracle.svt(G, tau), 0.0, "full Jacobi SVD"
    ref, cert = oracle.svt_gapped(G, tau, k=min(s, 2 * r + 256), power_iters=16, max_rel_bound=float("inf"),
                                  return_bound=True)
    return ref, None, "compressed, uncertified (bound %.3g)" % cert


def loop_leg(psvt, torch, dev, checks, rates=(100, 200, 500, 1000, 2000, 5000), count=2000, steps=20,
             lp=(("n_bf16", 18),)):
    """Serving form driven by matrix-completion proximal loops (section 2:
    thresholding as the proximal step of nuclear-norm methods).  count/steps
    loops, each ``steps`` proximal-gradient steps X <- SVT_lam(X - P_Omega(X
    - M)) whose thresholdings go to the server; loops arrive as a Poisson
    process at rate/steps per second, so requests are offered at ``rate``
    per second, and each loop submits its next step as soon as the previous
    one is back.  Shapes as the request stream (s log-uniform 256..4096,
    unrounded, square or 2:1), M = rank r in {16, 64, 256} + noise, 80 % of
    the entries observed, lam twice the sampling noise's edge.  The sign
    iteration warm starts from the loop's previous (I + S)/2 once the
    iterate has settled (change <= 5e-3 of its norm).  Per rate: p50/p99,
    matrices/s, warm steps; two recorded steps (first and last) of one loop
    per log2 size bucket are compared bit for bit with the single call on the
    same inputs (the warm start's (I + S)/2 included) and, once, with the
    certified oracle; every rate reproduces the first rate's recorded results
    bit for bit (the loops are deterministic).  18 BF16 + 2 FP32 iterations:
    tau lies inside the signal's range here, where e4m3 first iterations of
    P miss 1e-2."""
    from paper_2607_22484_amd import inputs, prox
    lp = dict(lp)
    nloops = count // steps
    g = torch.Generator(device=dev)
    g.manual_seed(2609)
    shapes = inputs.serve_shapes(nloops, idx=1)
    buckets = {}
    for i, (m, n, r) in enumerate(shapes):
        buckets.setdefault(int(math.log2(min(m, n))), i)
    sample = sorted(buckets.values())
    loops = []
    for i, (m, n, r) in enumerate(shapes):
        M_obs, mask, lam = inputs.completion_problem_device(torch, g, m, n, r)
        loops.append(prox.CompletionLoop(M_obs, mask, lam, steps, warm=True, name="loop%d" % i,
                                         record_steps=(0, steps - 1) if i in sample else ()))
    torch.cuda.synchronize()
    print("[bench] loops: %d completion problems generated" % nloops, file=sys.stderr, flush=True)
    out = {"loops_per_rate": nloops, "steps_per_loop": steps, "requests_per_rate": nloops * steps,
           "schedule": "%d FP8 + %d BF16 (split bf16) + 2 FP32; warm: 8 BF16 + 2 FP32 sign iterations"
                       % (lp.get("n_fp8", 0), lp.get("n_bf16", 0))}
    first_fp, kept = None, {}

    def one_rate(rate, warm, key):
        for L in loops:
            L.reset()
            L.warm = warm
        srv = psvt.Server(budget_bytes=64 << 30, max_slots=64, iters=20, **lp)
        arrivals = np.cumsum(np.random.default_rng(rate + 7).exponential(steps / rate, size=nloops))
        run = prox.run_loops(srv, loops, arrivals)
        srv.drain(timeout=900)
        st = srv.stats()
        srv.close()
        fp = {(i, rec[0]): _fingerprint(torch, rec[2]) for i in sample for rec in loops[i].inputs}
        row = {"completed": st["completed"], "failed": st["failed"] + run["failed"], "p50_ms": st["p50_ms"],
               "p99_ms": st["p99_ms"], "matrices_per_s": st["matrices_per_s"], "queue_p99_ms": st["queue_p99_ms"],
               "wall_s": run["wall_s"], "launches": st["launches"], "peak_pool_gib": st["peak_bytes"] / 2 ** 30,
               "warm_steps": sum(L.warm_steps for L in loops)}
        out[key] = row
        print("[bench] loops %s: %.1f matrices/s, p50 %.1f ms, p99 %.1f ms, %d warm steps of %d"
              % (key, st["matrices_per_s"], st["p50_ms"], st["p99_ms"], row["warm_steps"], run["submitted"]),
              file=sys.stderr, flush=True)
        return fp, row

    for rate in rates:
        fp, row = one_rate(rate, True, "%d_per_s" % rate)
        if first_fp is None:
            first_fp = fp
            # single calls of the recorded steps: same inputs, same schedule, same warm start
            cfg, _ = psvt.make_config(iters=20, **lp)
            same = 0
            for i in sample:
                for (k, G, Y, w, snap) in loops[i].inputs:
                    ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, G.shape[0], G.shape[1], cfg),
                                     dtype=torch.uint8, device=dev)
                    pi = torch.empty_like(loops[i].pi)
                    Y1 = psvt.svt(G, loops[i].tau, iters=20, ws=ws, warm_pi=snap, pi_out=pi, **lp)
                    same += int(_fingerprint(torch, Y1) == fp[(i, k)])
                    kept[(i, k)] = (G.cpu().numpy(), Y.cpu().numpy().astype(np.float64), loops[i].tau,
                                    tuple(G.shape), shapes[i][2], w)
                    del ws, Y1
            out["recorded_steps"] = len(kept)
            out["recorded_bitwise_equal_to_single_call"] = same
        row["recorded_bitwise_equal_to_first_rate"] = sum(fp[k] == first_fp.get(k) for k in fp)
        torch.cuda.empty_cache()
    # the warm-start saving: the saturated rate again with every step cold
    top = max(rates)
    _, cold = one_rate(top, False, "%d_per_s_cold" % top)
    warm_row = out["%d_per_s" % top]
    out["warm_start_saving"] = {
        "rate": top, "warm_matrices_per_s": warm_row["matrices_per_s"], "cold_matrices_per_s": cold["matrices_per_s"],
        "speedup": warm_row["matrices_per_s"] / cold["matrices_per_s"],
        "warm_fraction_of_steps": warm_row["warm_steps"] / float(nloops * steps),
        "sign_iterations_cold": 20, "sign_iterations_warm": 10}
    del loops
    torch.cuda.empty_cache()
    if checks is not None:
        def check(oracle, dst=out):
            rows = []
            for (i, k), (G, Y, tau, shape, r, w) in sorted(kept.items()):
                ref, cert, how = _completion_reference(oracle, G, tau, r)
                rows.append({"loop": i, "step": k, "shape": list(shape), "rank": r, "warm": w,
                             "rel_err": oracle.rel_fro_err(Y, ref), "reference_certified_to": cert,
                             "reference": how})
            dst["sampled_step_errors"] = rows
            dst["worst_sampled_rel_err"] = max(x["rel_err"] for x in rows)
            warm_errs = [x["rel_err"] for x in rows if x["warm"]]
            dst["worst_sampled_warm_rel_err"] = max(warm_errs) if warm_errs else None
        checks.append(check)
    return out


def gram_leg(psvt, torch, dev, checks, shapes=((16384, 1024, 100), (1024, 16384, 100), (8192, 1024, 100))):
    """Gram form of the polar factor (PSVT_FLAG_GRAM) against the standard
    form, l >> s: rank-r signal (sigma in [1, 10]) plus noise, tau twice the
    noise's spectral norm; time per SVT with FP32 and with the 18 BF16 + 2
    FP32 sign schedule (the Gram form's P products are FP32 either way),
    errors against the certified oracle."""
    from paper_2607_22484_amd import inputs
    out = {}
    for (m, n, r) in shapes:
        pb = inputs.noisy_lowrank(m, n, rank=r, idx=7, norm_iters=60)
        A = torch.from_numpy(pb.A).to(dev)
        Y = torch.empty_like(A)
        row = {"rank": r, "tau": pb.tau}
        for name, kw in [("fp32", dict()), ("fp32_gram", dict(flags=psvt.FLAG_GRAM)),
                         ("bf16S", dict(n_bf16=18)), ("bf16S_gram", dict(n_bf16=18, flags=psvt.FLAG_GRAM))]:
            cfg, _ = psvt.make_config(iters=20, **kw)
            ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, m, n, cfg), dtype=torch.uint8, device=dev)
            ms = time_calls(torch, lambda: psvt.svt(A, pb.tau, iters=20, out=Y, ws=ws, **kw), 3)
            row[name] = {"ms": ms}
            if checks is not None:
                Yh = Y.cpu().numpy().astype(np.float64)

                def check(oracle, pb=pb, Yh=Yh, dst=row[name], r=r, memo={}):
                    key = pb.name
                    if key not in memo:
                        memo.clear()
                        memo[key] = oracle.svt_gapped(pb.A.astype(np.float64), pb.tau, k=r + 64, return_bound=True)
                    ref, cert = memo[key]
                    dst["rel_err"] = oracle.rel_fro_err(Yh, ref)
                    dst["reference_certified_to"] = cert
                checks.append(check)
            del ws
        row["gram_speedup_fp32"] = row["fp32"]["ms"] / row["fp32_gram"]["ms"]
        row["gram_speedup_bf16S"] = row["bf16S"]["ms"] / row["bf16S_gram"]["ms"]
        out["%dx%d" % (m, n)] = row
        print("[bench] gram %dx%d: fp32 %.2f ms, gram %.2f ms; bf16S %.2f ms, gram %.2f ms"
              % (m, n, row["fp32"]["ms"], row["fp32_gram"]["ms"], row["bf16S"]["ms"], row["bf16S_gram"]["ms"]),
              file=sys.stderr, flush=True)
        del A, Y
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="size of the matrix the CPU oracle is timed on (the main workload's size: one of its "
                         "own matrices)")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision / batched / serving legs")
    ap.add_argument("--forms", default="small,rank,precision,batched,serving,loops,gram,fig1,fig2",
                    help="comma-separated subset of the small / rank / precision / batched / serving / loops / gram "
                         "/ fig1 / fig2 legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB elementwise copy first (scale reference for PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (matrices are independent, so "
              "several GPUs would each take a share of them). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_22484_amd as psvt
    from paper_2607_22484_amd import inputs

    psvt.load()
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        calibration_copy(torch, dev)
    n = args.n
    quantiles = (0.1, 0.5, 0.9)
    t_gen = time.perf_counter()
    problems = [inputs.square_case(q, n=n) for q in quantiles]
    print("[bench] inputs generated in %.1f s" % (time.perf_counter() - t_gen), file=sys.stderr, flush=True)
    A = [torch.from_numpy(pb.A).to(dev) for pb in problems]
    Y = [torch.empty_like(a) for a in A]
    cfg, _ = psvt.make_config(iters=args.iters)
    ws = torch.empty(psvt.workspace_bytes(psvt.OP_SVT, n, n, cfg), dtype=torch.uint8, device=dev)
    taus = [pb.tau for pb in problems]
    stream = torch.cuda.current_stream(dev)

    def step(lat=None):
        for a, y, tau in zip(A, Y, taus):
            if lat is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            psvt.svt(a, tau, iters=args.iters, out=y, ws=ws)
            if lat is not None:
                e1.record(stream)
                lat.append((e0, e1))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    lat = []
    psvt.trace_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(lat)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    trace = psvt.trace_end()
    lat_ms = [e0.elapsed_time(e1) for e0, e1 in lat]
    print("[bench] timed %d steps in %.3f s" % (args.steps, elapsed), file=sys.stderr, flush=True)

    n_mat = len(A) * args.steps
    ms_per_step = 1e3 * elapsed / args.steps
    flops_step = sum(useful_flops(n, n, args.iters) for _ in A)
    tflops = flops_step / (ms_per_step * 1e-3) / 1e12

    products = [t for t in trace if t["flops"] > 0]
    dom = max(products, key=lambda t: t["total_ms"])
    dom_avg_ms = dom["total_ms"] / dom["launches"]
    dom_tflops = dom["flops"] / (dom["total_ms"] * 1e-3) / 1e12
    roofline = {
        "bound": "mfma", "kernel": dom["name"], "launches": dom["launches"], "avg_launch_ms": dom_avg_ms,
        "flops_per_launch": dom["flops"] / dom["launches"],
        "achieved": dom_tflops, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
        "frac": dom_tflops / PEAK_TFLOPS["f32"], "traffic": stored_traffic(dom["name"], n),
        "kernel_source_sha": kernel_source_sha(),
    }
    kernels = [{"name": t["name"], "launches": t["launches"], "ms_per_step": t["total_ms"] / args.steps,
                "tflops": (t["flops"] / (t["total_ms"] * 1e-3) / 1e12) if t["flops"] else None,
                "gbs": (t["bytes"] / (t["total_ms"] * 1e-3) / 1e9) if t["bytes"] else None} for t in trace]

    out = {
        "metric": METRIC,
        "value": n_mat / elapsed,
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plain FP32 SVT, %dx%d, %d polar iterations, tau at the 10/50/90%% quantiles of a "
                        "log-spaced spectrum 10..1e-3 (gap-clamped), 3 matrices per step, one per launch sequence"
                        % (n, n, args.iters),
            "m": n, "n": n, "iters": args.iters, "matrices_per_step": len(A), "side": "left (square)",
        },
        "useful_tflops": tflops,
        "mfma_util": tflops / PEAK_TFLOPS["f32"],
        "latency_ms": {"p50": percentile(lat_ms, 0.5), "p99": percentile(lat_ms, 0.99)},
        "roofline": roofline,
        "kernels": kernels,
    }
    checks = None if args.no_cpu else []
    res = None if args.no_cpu else [y.cpu().numpy().astype(np.float64) for y in Y]
    if not args.no_forms:
        del A, Y, ws
        torch.cuda.empty_cache()
        forms = {}
        want = set(args.forms.split(","))
        if "small" in want:
            print("[bench] small case latency ...", file=sys.stderr, flush=True)
            forms["small_256x128"] = small_leg(psvt, torch, dev, checks)
        if "rank" in want:
            print("[bench] rank-r approximation (Corollary 1) ...", file=sys.stderr, flush=True)
            forms["rank_r_4096_r256"] = rank_leg(psvt, torch, dev, checks)
            torch.cuda.empty_cache()
        if "precision" in want:
            print("[bench] precision form ...", file=sys.stderr, flush=True)
            forms["precision"] = precision_leg(psvt, torch, dev, checks, problems)
        if "batched" in want:
            print("[bench] batched form ...", file=sys.stderr, flush=True)
            forms["batched"] = batched_leg(psvt, torch, dev, checks)
            torch.cuda.empty_cache()
        if "serving" in want:
            print("[bench] serving form ...", file=sys.stderr, flush=True)
            forms["serving"] = serving_leg(psvt, torch, dev, checks)
            torch.cuda.empty_cache()
        if "gram" in want:
            print("[bench] Gram form of P, l >> s ...", file=sys.stderr, flush=True)
            forms["gram_form"] = gram_leg(psvt, torch, dev, checks)
        if "loops" in want:
            print("[bench] serving form driven by completion loops ...", file=sys.stderr, flush=True)
            forms["serving_loops"] = loop_leg(psvt, torch, dev, checks)
            torch.cuda.empty_cache()
        if "fig1" in want:
            print("[bench] error vs iterations (Fig. 1 workload) ...", file=sys.stderr, flush=True)
            forms["fig1_error_vs_iterations"] = fig1_leg(psvt, torch, dev, checks)
        if "fig2" in want:
            print("[bench] run time vs size (Fig. 2 workload) ...", file=sys.stderr, flush=True)
            forms["fig2_time_vs_size"] = fig2_leg(psvt, torch, dev, checks)
        out["forms"] = forms
    if not args.no_cpu:
        print("[bench] cpu oracle leg (baseline timing and every accuracy figure) ...", file=sys.stderr, flush=True)
        cpu, errs, failures = cpu_baseline_leg(problems, res, args.cpu_sample, checks)
        out["cpu_baseline"] = cpu
        out["accuracy"] = errs
        out["accuracy_check_failures"] = failures
        out["rel_err_max"] = max(e["rel_err_bound_fp32_input"] for e in errs.values())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
