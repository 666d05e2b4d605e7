// Workspace layout of one operation, shared by the host planner and the
// device code of the batched entry point (which lays out each matrix's
// workspace on the device from its shape): the same function on both
// sides, so a matrix gets the same buffers either way.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace psvt {

// operation ids (the values of PSVT_OP_* in psvt.h)
enum OpId { OPID_SVT = 0, OPID_POLAR = 1, OPID_POLAR_SYM = 2, OPID_RANK_R = 3 };

// Buffers of a layout, by id (byte offsets from the workspace base), and
// the shape class of each: its row stride and its plane stride (the distance
// from the hi to the lo plane of a split-bf16 copy) follow from it.
enum BufId {
    B_SCAL, B_PART, B_X0, B_X0T, B_XP, B_XQ, B_XTP, B_XTQ, B_T, B_BM, B_H, B_R, B_S0, B_S1, B_X2, B_BS,
    B_TL, B_BL, B_XL0, B_XL1, B_XTL0, B_XTL1, B_SL0, B_SL1, B_X2L, B_BSL, B_COUNT
};
enum BufShape { SH_OTHER = 0, SH_LS = 1, SH_SL = 2, SH_SS = 3 };  // l x s (ld ldS), s x l (ld ldL), s x s (ld ldS)

__host__ __device__ inline int buf_shape(int b) {
    switch (b) {
        case B_X0: case B_XP: case B_XQ: case B_XL0: case B_XL1: return SH_LS;
        case B_X0T: case B_XTP: case B_XTQ: case B_XTL0: case B_XTL1: return SH_SL;
        case B_SCAL: case B_PART: return SH_OTHER;
        default: return SH_SS;
    }
}

__host__ __device__ inline int64_t round_up64(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

struct Layout {
    int64_t l = 0, s = 0, ldL = 0, ldS = 0;
    bool right = true;
    size_t scal = 0, part = 0;
    size_t X0 = 0, X0T = 0, Xp = 0, Xq = 0, XTp = 0, XTq = 0;
    size_t T = 0, Bm = 0;
    size_t H = 0, R = 0, S0 = 0, S1 = 0, X2 = 0, BS = 0;
    // low-precision operand copies: room for two bf16 planes per element
    // (split bf16); plane strides in elements
    bool lp = false;
    size_t XL[2] = {0, 0}, XTL[2] = {0, 0}, TL = 0, BL = 0, SL[2] = {0, 0};
    // S's copies of X^2 and B: the same buffers as P's unless the two
    // iterations run concurrently (fork)
    size_t X2L = 0, BSL = 0;
    bool fork = false;
    int64_t planeX = 0, planeXT = 0, planeS = 0;
    size_t total = 0;

    __host__ __device__ size_t offset(int b) const {
        switch (b) {
            case B_SCAL: return scal;  case B_PART: return part;  case B_X0: return X0;   case B_X0T: return X0T;
            case B_XP: return Xp;      case B_XQ: return Xq;      case B_XTP: return XTp; case B_XTQ: return XTq;
            case B_T: return T;        case B_BM: return Bm;      case B_H: return H;     case B_R: return R;
            case B_S0: return S0;      case B_S1: return S1;      case B_X2: return X2;   case B_BS: return BS;
            case B_TL: return TL;      case B_BL: return BL;      case B_XL0: return XL[0];
            case B_XL1: return XL[1];  case B_XTL0: return XTL[0]; case B_XTL1: return XTL[1];
            case B_SL0: return SL[0];  case B_SL1: return SL[1];  case B_X2L: return X2L;
            default: return BSL;
        }
    }
    // whether buffer b exists in this layout (offset 0 is the scalar block)
    __host__ __device__ bool has(int b) const { return b == B_SCAL || offset(b) != 0; }
    __host__ __device__ int64_t ld(int b) const { return buf_shape(b) == SH_SL ? ldL : ldS; }
    __host__ __device__ int64_t plane(int b) const {
        const int sh = buf_shape(b);
        return sh == SH_LS ? planeX : sh == SH_SL ? planeXT : sh == SH_SS ? planeS : 0;
    }
};

// P and S are independent once the Gram and the shifted Gram exist.  When a
// single call's products are too small to fill the device (s <= 2048), the P
// iterations run on a side stream; the layout then gives S its own
// low-precision copies of X^2 and B.
constexpr int64_t kForkMaxS = 2048;

// Buffers of operation `op` on an l x s iterate (s = the short side the
// Gram matrix is formed over); lp: low-precision copies; fork_ok: a single
// call that may run P and S concurrently.
__host__ __device__ inline Layout layout_for(int op, int64_t l, int64_t s, bool right, bool lp, bool fork_ok) {
    Layout L;
    L.right = right;
    L.l = l;
    L.s = s;
    L.ldL = round_up64(L.l, 64);
    L.ldS = round_up64(L.s, 64);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (size_t)round_up64((int64_t)bytes, 256);
        return o;
    };
    const size_t fS = sizeof(float) * (size_t)L.s * L.ldS;   // s x s
    const size_t fX = sizeof(float) * (size_t)L.l * L.ldS;   // l x s
    const size_t fXT = sizeof(float) * (size_t)L.s * L.ldL;  // s x l
    L.scal = take(sizeof(Scalars));
    L.part = take(sizeof(double) * NORM_PARTIALS);
    const bool need_P = op == OPID_SVT || op == OPID_POLAR;
    const bool need_S = op != OPID_POLAR;
    if (op != OPID_POLAR_SYM) {
        L.X0 = take(fX);
        L.X0T = take(fXT);
        L.T = take(fS);
    }
    if (need_P) {
        L.Xp = take(fX);
        L.Xq = take(fX);
        L.XTp = take(fXT);
        L.XTq = take(fXT);
        L.Bm = take(fS);
    }
    if (need_S) {
        L.H = take(fS);
        L.R = take(fS);
        L.S0 = take(fS);
        L.S1 = take(fS);
        L.X2 = take(fS);
        L.BS = take(fS);
    }
    L.lp = lp;
    if (L.lp) {
        L.TL = take(fS);
        L.BL = take(fS);
        L.X2L = L.TL;
        L.BSL = L.BL;
        if (need_P)
            for (int i = 0; i < 2; ++i) {
                L.XL[i] = take(fX);
                L.XTL[i] = take(fXT);
            }
        if (need_S)
            for (int i = 0; i < 2; ++i) L.SL[i] = take(fS);
        L.planeX = L.l * L.ldS;
        L.planeXT = L.s * L.ldL;
        L.planeS = L.s * L.ldS;
    }
    L.fork = fork_ok && op == OPID_SVT && L.s <= kForkMaxS;
    if (L.fork && L.lp) {
        L.X2L = take(fS);
        L.BSL = take(fS);
    }
    L.total = off;
    return L;
}

}  // namespace psvt
