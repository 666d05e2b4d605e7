// Stage lists: the planner describes one operation as a sequence of stages
// (products, norm reductions, tiled elementwise passes).  A stage list runs
// either immediately, launch by launch on a stream (single-matrix calls),
// or is recorded and later executed for many matrices at once, stage by
// stage, with grouped launches (batched and serving forms).
#pragma once
#include <vector>

#include "kernels.h"

namespace psvt {

enum StageKind { ST_GEMM = 0, ST_NORM = 1, ST_TILE = 2 };

struct Stage {
    int kind;
    int dtype;  // operand type of a product
    GemmArgs g;
    NormOp n;
    TileOp t;
    const char *what;
};

struct Exec {
    hipStream_t st = nullptr;
    std::vector<Stage> *rec = nullptr;  // record instead of launching
    // A recorded soft-thresholding: stages [0, cut[0]) are the common prefix
    // (norm, Gram, shifted Gram), [cut[0], cut[1]) the P iterations,
    // [cut[1], cut[2]) the S iterations, the rest the final product.  With
    // `chains` set the two iteration chains touch disjoint buffers and may
    // run concurrently.
    size_t cut[3] = {0, 0, 0};
    bool chains = false;

    hipError_t gemm(const GemmArgs &g, int dt, const char *what) {
        if (g.M <= 0 || g.N <= 0) return hipSuccess;
        if (rec) {
            Stage s{};
            s.kind = ST_GEMM;
            s.dtype = dt;
            s.g = g;
            gemm_prepare(s.g, dt);
            s.what = what;
            rec->push_back(s);
            return hipSuccess;
        }
        return launch_gemm(g, dt, st);
    }
    hipError_t norm(const NormOp &op, const char *what) {
        if (rec) {
            Stage s{};
            s.kind = ST_NORM;
            s.n = op;
            s.what = what;
            rec->push_back(s);
            return hipSuccess;
        }
        return launch_norm_op(op, st);
    }
    hipError_t tile(const TileOp &op, const char *what) {
        if (op.rows <= 0 || op.cols <= 0) return hipSuccess;
        if (rec) {
            Stage s{};
            s.kind = ST_TILE;
            s.t = op;
            s.what = what;
            rec->push_back(s);
            return hipSuccess;
        }
        return launch_tile_op(op, st);
    }
};

}  // namespace psvt
