// Device bodies of the FP64 Frobenius norms and the element-wise tile
// operations, shared by their own kernels (single, grouped and batched
// launches) and the persistent batched executor.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device.h"
#include "kernels.h"

namespace psvt {

// Partial sums of squares in FP64 of one matrix: chunk b of nb sums rows
// b, b + nb, ...
__device__ __forceinline__ void fro_partial_body(const NormOp &op, int b, double *red) {
    double acc = 0.0;
    for (int64_t r = b; r < op.rows; r += op.nparts) {
        const float *p = op.X + r * op.ld;
        for (int64_t c = threadIdx.x; c < op.cols; c += 256) {
            const double v = (double)p[c];
            acc += v * v;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) op.part[b] = red[0];
}

// Fixed-order final reduction (deterministic), then the derived scalars.
__device__ __forceinline__ void fro_final_body(const NormOp &op, double *red) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < op.nparts; i += 256) acc += op.part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    Scalars *sc = op.sc;
    const double nrm = sqrt(red[0]);
    sc->d[D_NORM] = nrm;
    if (op.mode == NORM_INPUT) {
        sc->d[D_NU] = nrm;
        sc->f[F_NU] = (float)nrm;
        sc->f[F_INV_NU] = nrm > 0.0 ? (float)(1.0 / nrm) : 0.0f;
        sc->d[D_SHIFT] = nrm > 0.0 ? (op.tau / nrm) * (op.tau / nrm) : 0.0;
        sc->d[D_TAU] = nrm > 0.0 ? op.tau / nrm : 0.0;
    } else if (op.mode == NORM_THETA_P || op.mode == NORM_THETA_S) {
        // theta = sqrt(||M||_F) bounds the spectral radius of the iterate:
        // M = X^T X (or H^2) has eigenvalues mu_i >= 0 and
        // ||M||_F = sqrt(sum mu_i^2) >= mu_max = sigma_max^2.
        const double theta = sqrt(nrm) * op.safety;
        const int base = op.mode == NORM_THETA_P ? F_P1 : F_S1;
        const double it = theta > 0.0 ? 1.0 / theta : 0.0;
        sc->f[base] = (float)it;
        sc->f[base + 1] = (float)(it * it);
        sc->f[base + 2] = (float)(it * it * it * it);
        // tau / theta_P, tau in the input's units (D_TAU = tau / nu)
        if (op.mode == NORM_THETA_P) sc->f[F_TAU_P] = (float)(sc->d[D_TAU] * sc->d[D_NU] * it);
    } else if (op.mode == NORM_CONV) {
        sc->d[D_CONV] = op.scale * nrm / sqrt((double)(op.rows > 0 ? op.rows : 1));
    } else if (op.mode == NORM_STATUS) {
        uint32_t st = 0;
        if (!isfinite(sc->d[D_NU])) st |= ST_NONFINITE_INPUT;
        if (!isfinite(nrm)) st |= ST_NONFINITE_OUTPUT;
        if (op.tol >= 0.0 && !(sc->d[D_CONV] <= op.tol)) st |= ST_NOT_CONVERGED;
        if (op.status) *op.status = st;
    }
}

// 64 x 64 tiles through LDS, 256 threads, 16 elements each.  One body for
// every elementwise pass of the method:
//   TOP_SCALE_T  Y = s X, YT = s X^T (either may be NULL)
//   TOP_SHIFT    Y = X - shift I, the diagonal in FP64 (shift from sc)
//   TOP_SYMM     Y = s (X + X^T) / 2
//   TOP_CONVERT  L = lowp(s X) or lowp(s X^T), s = scale [x sc->f[i_scale]]
__device__ __forceinline__ void tile_op_body(const TileOp &op, int tile, float (*lds)[65]) {
    const int ntc = (int)((op.cols + 63) / 64);
    const int64_t r0 = (int64_t)(tile / ntc) * 64, c0 = (int64_t)(tile % ntc) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const float s = op.scale * (op.sc && op.i_scale >= 0 ? op.sc->f[op.i_scale] : 1.0f);
    if (op.kind == TOP_SYMM) {
        for (int k = ty; k < 64; k += 4) {  // mirrored tile X[c0.., r0..]
            const int64_t r = c0 + k, c = r0 + tx;
            lds[k][tx] = (r < op.rows && c < op.cols) ? op.X[r * op.ldx + c] : 0.0f;
        }
        __syncthreads();
        for (int k = ty; k < 64; k += 4) {
            const int64_t r = r0 + k, c = c0 + tx;
            if (r < op.rows && c < op.cols) op.Y[r * op.ldy + c] = 0.5f * s * (op.X[r * op.ldx + c] + lds[tx][k]);
        }
        return;
    }
    if (op.kind == TOP_WARM) {
        for (int k = ty; k < 64; k += 4) {
            const int64_t r = r0 + k, c = c0 + tx;
            if (r < op.rows && c < op.cols)
                op.Y[r * op.ldy + c] =
                    (s * op.X[r * op.ldx + c] + op.eps * (2.0f * op.Z[r * op.ldz + c] - (r == c ? 1.0f : 0.0f))) /
                    (1.0f + op.eps);
        }
        return;
    }
    const bool need_t = (op.kind == TOP_SCALE_T && op.YT) || (op.kind == TOP_CONVERT && op.ltrans);
    const double shift = op.kind == TOP_SHIFT ? op.sc->d[op.i_shift] : 0.0;
    for (int k = ty; k < 64; k += 4) {
        const int64_t r = r0 + k, c = c0 + tx;
        const bool in = r < op.rows && c < op.cols;
        float v = in ? op.X[r * op.ldx + c] : 0.0f;
        if (op.kind == TOP_SHIFT) {
            if (in) op.Y[r * op.ldy + c] = (r == c) ? (float)((double)v - shift) : v;
            continue;
        }
        v *= s;
        if (in) {
            if (op.kind == TOP_SCALE_T && op.Y) op.Y[r * op.ldy + c] = v;
            if (op.kind == TOP_CONVERT && !op.ltrans) {
                if (op.ltype == OP_F32)
                    ((float *)op.L)[r * op.ldl + c] = v;
                else
                    store_lp(op.L, op.ltype, r * op.ldl + c, v, op.lplane);
            }
        }
        if (need_t) lds[k][tx] = v;
    }
    if (!need_t) return;
    __syncthreads();
    for (int k = ty; k < 64; k += 4) {
        const int64_t c = c0 + k, r = r0 + tx;  // out[c][r] = X[r][c]
        if (c >= op.cols || r >= op.rows) continue;
        const float v = lds[tx][k];
        if (op.kind == TOP_SCALE_T) {
            op.YT[c * op.ldyt + r] = v;
        } else if (op.ltype == OP_F32) {
            ((float *)op.L)[c * op.ldl + r] = v;
        } else {
            store_lp(op.L, op.ltype, c * op.ldl + r, v, op.lplane);
        }
    }
}

}  // namespace psvt
