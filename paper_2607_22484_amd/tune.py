"""Autotuner for the MFMA tile configurations.

For every tile configuration (64, 128, 192, 256) it times the library's
product kernel, forced to that configuration, on a set of product shapes of
the method (symmetric s x s x s and s x s x l products, rectangular l x s x s
products), and fits, per configuration and kind (symmetric or full), the two
parameters of the library's cost model

    time ~= ceil(tiles / 256) * (overhead + tile flops / (eff * CU rate))

by least squares (time / ceil(tiles/256) is linear in overhead and 1/eff).
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

CU_RATE = 157.3e12 / 256  # FP32 MFMA flop/s of one CU
TILES = {1: 64, 2: 128, 3: 192, 4: 256}
SHAPES = [  # (M, N, K, sym)
    (512, 512, 512, True), (1024, 1024, 1024, True), (2048, 2048, 2048, True), (3072, 3072, 3072, True),
    (4096, 4096, 4096, True), (4096, 4096, 8192, True), (1024, 1024, 1024, False), (2048, 2048, 2048, False),
    (4096, 4096, 4096, False), (8192, 4096, 4096, False),
]


def tile_count(M, N, bm, sym):
    nbm, nbn = -(-M // bm), -(-N // bm)
    return nbm * (nbm + 1) // 2 if sym else nbm * nbn


def measure(psvt, torch, M, N, K, sym, tile, reps=5):
    dev = torch.device("cuda:0")
    A = torch.randn(M, K, device=dev)
    B = A if sym else torch.randn(N, K, device=dev)
    C = torch.empty(M, N, device=dev)
    psvt.force_tile(tile)
    try:
        psvt.gemm_nt(A, B, sym=sym, out=C)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            psvt.gemm_nt(A, B, sym=sym, out=C)
        e1.record()
        torch.cuda.synchronize()
    finally:
        psvt.force_tile(0)
    return e0.elapsed_time(e1) / reps * 1e-3


def fit(rows):
    """Least-squares (overhead_us, 1/eff) per (tile, sym) from measured rows."""
    import numpy as np
    table = {}
    for t, bm in TILES.items():
        for sym in (0, 1):
            X, y = [], []
            for r in rows:
                if int(r["sym"]) != sym:
                    continue
                per_cu = math.ceil(tile_count(r["M"], r["N"], bm, r["sym"]) / 256.0)
                work_us = 1e6 * bm * bm * 2.0 * r["K"] / CU_RATE
                X.append([1.0, work_us])
                y.append(1e6 * r["times"][t] / per_cu)
            if not X:
                continue
            coef, *_ = np.linalg.lstsq(np.array(X), np.array(y), rcond=None)
            over, inv_eff = float(coef[0]), float(coef[1])
            if over < 0 or inv_eff < 1.0:  # fall back to a pure-efficiency fit
                over = max(over, 0.0)
                inv_eff = max(1.0, float(np.sum((np.array(y) - over) * np.array(X)[:, 1]) /
                                     np.sum(np.array(X)[:, 1] ** 2)))
            table[(t, sym)] = (1.0 / inv_eff, over)
    return table


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
        print(table)
        return 0
    import torch
    import paper_2607_22484_amd as psvt
    psvt.load()
    rows = []
    effs = {t: [] for t in TILES}
    for (M, N, K, sym) in SHAPES:
        times = {}
        for t, bm in TILES.items():
            sec = measure(psvt, torch, M, N, K, sym, t)
            per_cu = math.ceil(tile_count(M, N, bm, sym) / 256.0)
            eff = per_cu * bm * bm * 2.0 * K / (sec * CU_RATE)
            times[t] = sec
            effs[t].append(eff)
            useful = (M * (M + 1) * K if sym else 2.0 * M * N * K) / sec / 1e12
            print("M=%d N=%d K=%d sym=%d tile=%d: %.3f ms, %.1f useful TF/s, model eff %.3f"
                  % (M, N, K, sym, bm, sec * 1e3, useful, eff), flush=True)
        rows.append(dict(M=M, N=N, K=K, sym=sym, times=times))
    table = fit(rows)
    out = args.out or psvt.TUNE_TABLE
    write_table(out, table)
    lib = psvt.load()
    lib.psvt_tune_load(out.encode())
    regret = []
    for r in rows:
        pick = psvt.pick_tile(r["M"], r["N"], r["K"], r["sym"])
        best = min(r["times"], key=r["times"].get)
        regret.append(r["times"][pick] / r["times"][best])
        print("M=%d N=%d K=%d sym=%d: model picks %d (%.3f ms), best %d (%.3f ms)"
              % (r["M"], r["N"], r["K"], r["sym"], TILES[pick], r["times"][pick] * 1e3, TILES[best],
                 r["times"][best] * 1e3), flush=True)
    print("table:", table, "max regret %.3f" % max(regret), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(table={"%d_%d" % k: v for k, v in table.items()}, rows=rows), f)


if __name__ == "__main__":
    sys.exit(main())
