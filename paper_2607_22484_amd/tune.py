"""Autotuner for the MFMA tile configurations.

For every tile configuration (64, 128, 192, 256) it times the library's
product kernel, forced to that configuration, on a set of product shapes of
the method (symmetric s x s x s and s x s x l products, rectangular l x s x s
products), and fits, per configuration and kind (symmetric or full), the two
parameters (efficiency, per-wave overhead) of the library's cost model by
least squares in relative terms: the CU with the most tiles, p = ceil(tiles
/ 256), does all their flops on its MFMA units, in ceil(p / occ) waves of
blocks (occ: blocks per CU of the configuration, from its LDS), each wave
paying a fixed start and drain:

    time ~= p * tile flops / (eff * CU rate) + ceil(p / occ) * overhead

(linear in 1/eff and overhead).
It writes "id sym eff overhead_us" lines to ``tune_table.txt`` beside the
library (loaded by the Python binding; C callers use ``psvt_tune_load``) and
reports, per shape, the configuration the model picks against the fastest
measured one.

Usage (on the GPU):  python -m paper_2607_22484_amd.tune [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

# MFMA flop/s of one CU per dtype (split bf16: the useful rate, a third of bf16's)
CU_RATES = {0: 157.3e12 / 256, 1: 2516.6e12 / 256, 2: 5033.2e12 / 256, 3: 2516.6e12 / 3 / 256}
CU_RATE = CU_RATES[0]
TILES = {1: 64, 2: 128, 3: 192, 4: 256}
DTYPES = (0, 1, 2, 3)
SHAPES = [  # (M, N, K, sym)
    (256, 256, 768, True), (768, 256, 256, False), (640, 640, 1280, True), (1280, 640, 640, False),
    (512, 512, 512, True), (1024, 1024, 1024, True), (2048, 2048, 2048, True), (3072, 3072, 3072, True),
    (4096, 4096, 4096, True), (4096, 4096, 8192, True), (1024, 1024, 1024, False), (2048, 2048, 2048, False),
    (4096, 4096, 4096, False), (8192, 4096, 4096, False),
]


def tile_occ(dtype, t):
    """Blocks per CU of configuration t (tilemodel.h: tile_occ)."""
    if t >= 3:
        return 1
    if dtype == 3:
        return 2 if t == 1 else 1
    return 4 if t == 1 else 2


def per_cu_and_waves(M, N, bm, sym, dtype, t):
    per_cu = math.ceil(tile_count(M, N, bm, sym) / 256.0)
    return per_cu, math.ceil(per_cu / tile_occ(dtype, t))


def model_us(table, dtype, M, N, K, sym, t):
    """tilemodel.h: model_time_us."""
    bm = TILES[t]
    p, waves = per_cu_and_waves(M, N, bm, sym, dtype, t)
    e, o = table[(dtype, t, int(sym))]
    return p * 1e6 * bm * bm * 2.0 * K / (e * CU_RATES[dtype]) + waves * o


def model_pick(table, dtype, M, N, K, sym):
    """tilemodel.h: pick_tile (a configuration must win by 0.1 %)."""
    best, arg = 1e300, 2
    for t in TILES:
        v = model_us(table, dtype, M, N, K, sym, t)
        if v < best * 0.999:
            best, arg = v, t
    return arg


def tile_count(M, N, bm, sym):
    nbm, nbn = -(-M // bm), -(-N // bm)
    return nbm * (nbm + 1) // 2 if sym else nbm * nbn


def operands(psvt, torch, M, N, K, sym, dtype):
    dev = torch.device("cuda:0")
    A = torch.randn(M, K, device=dev)
    B = A if sym else torch.randn(N, K, device=dev)
    if dtype != 0:
        A = psvt.convert(A, dtype, scale=8.0)
        B = A if sym else psvt.convert(B, dtype, scale=8.0)
    return A, B, torch.empty(M, N, device=dev)


def measure(psvt, torch, M, N, K, sym, tile, dtype=0, reps=5):
    A, B, C = operands(psvt, torch, M, N, K, sym, dtype)
    psvt.force_tile(tile)
    try:
        psvt.gemm_nt(A, B, sym=sym, out=C, dtype=dtype)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            psvt.gemm_nt(A, B, sym=sym, out=C, dtype=dtype)
        e1.record()
        torch.cuda.synchronize()
    finally:
        psvt.force_tile(0)
    return e0.elapsed_time(e1) / reps * 1e-3


def fit(rows):
    """Least-squares (overhead_us, 1/eff) per (dtype, tile, sym) from rows."""
    import numpy as np
    table = {}
    for dt in sorted(set(int(r.get("dtype", 0)) for r in rows)):
      for t, bm in TILES.items():
        for sym in (0, 1):
            X, y = [], []
            for r in rows:
                if int(r["sym"]) != sym or int(r.get("dtype", 0)) != dt:
                    continue
                p, waves = per_cu_and_waves(r["M"], r["N"], bm, r["sym"], dt, t)
                work_us = p * 1e6 * bm * bm * 2.0 * r["K"] / CU_RATES[dt]
                X.append([waves, work_us])
                y.append(1e6 * r["times"][t])
            if not X:
                continue
            Xa, ya = np.array(X), np.array(y)
            w = 1.0 / ya  # relative errors: small and large products count alike
            coef, *_ = np.linalg.lstsq(Xa * w[:, None], ya * w, rcond=None)
            over, inv_eff = float(coef[0]), float(coef[1])
            if over < 0:  # refit through a zero overhead
                over = 0.0
                inv_eff = float(np.sum(w * w * ya * Xa[:, 1]) / np.sum((w * Xa[:, 1]) ** 2))
            if inv_eff < 1.0 and over > 0:  # an overhead that buys an efficiency above 1: refit without it
                over = 0.0
                inv_eff = float(np.sum(w * w * ya * Xa[:, 1]) / np.sum((w * Xa[:, 1]) ** 2))
            if inv_eff < 1.0:
                print("warning: dtype %d tile %d sym %d fits an efficiency above 1 (%.3f): clamped"
                      % (dt, t, sym, 1.0 / inv_eff), flush=True)
                inv_eff = 1.0
            table[(dt, t, sym)] = (1.0 / inv_eff, over)
    return table


def report_regret(rows, table, pick_of):
    """Per shape: the configuration picked against the fastest measured;
    returns the worst time ratio."""
    worst = 1.0
    for r in rows:
        pick = pick_of(r)
        best = min(r["times"], key=r["times"].get)
        worst = max(worst, r["times"][pick] / r["times"][best])
        print("dtype=%d M=%d N=%d K=%d sym=%d: model picks %d (%.3f ms), best %d (%.3f ms)"
              % (r["dtype"], r["M"], r["N"], r["K"], r["sym"], TILES[pick], r["times"][pick] * 1e3, TILES[best],
                 r["times"][best] * 1e3), flush=True)
    return worst


def write_table(path, table):
    with open(path, "w") as f:
        f.write("# dtype id sym efficiency overhead_us  (fitted by paper_2607_22484_amd.tune on one MI355X)\n")
        for key in sorted(table):
            e, o = table[key]
            f.write("%d %d %d %.4f %.2f\n" % (key + (e, o)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--json", default=None)
    ap.add_argument("--refit", default=None, help="fit a saved --json sweep instead of measuring")
    args = ap.parse_args()
    if args.refit:
        with open(args.refit) as f:
            rows = json.load(f)["rows"]
        for r in rows:
            r["times"] = {int(k): v for k, v in r["times"].items()}
        table = fit(rows)
        write_table(args.out, table)
        print("max regret %.3f" % report_regret(rows, table, lambda r: model_pick(table, r["dtype"], r["M"], r["N"],
                                                                                 r["K"], r["sym"])))
        return 0
    import torch
    import paper_2607_22484_amd as psvt
    psvt.load()
    rows = []
    for dt in DTYPES:
        for (M, N, K, sym) in SHAPES:
            times = {}
            for t, bm in TILES.items():
                sec = measure(psvt, torch, M, N, K, sym, t, dt)
                p, _ = per_cu_and_waves(M, N, bm, sym, dt, t)
                eff = p * bm * bm * 2.0 * K / (sec * CU_RATES[dt])
                times[t] = sec
                useful = (M * (M + 1) * K if sym else 2.0 * M * N * K) / sec / 1e12
                print("dtype=%d M=%d N=%d K=%d sym=%d tile=%d: %.3f ms, %.1f useful TF/s, model eff %.3f"
                      % (dt, M, N, K, sym, bm, sec * 1e3, useful, eff), flush=True)
            rows.append(dict(dtype=dt, M=M, N=N, K=K, sym=sym, times=times))
    table = fit(rows)
    out = args.out or psvt.TUNE_TABLE
    write_table(out, table)
    lib = psvt.load()
    lib.psvt_tune_load(out.encode())
    worst = report_regret(rows, table, lambda r: psvt.pick_tile(r["M"], r["N"], r["K"], r["sym"], r["dtype"]))
    print("table:", table, "max regret %.3f" % worst, flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(table={"%d_%d_%d" % k: v for k, v in table.items()}, rows=rows), f)


if __name__ == "__main__":
    sys.exit(main())
