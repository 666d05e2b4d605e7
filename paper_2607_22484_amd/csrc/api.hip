// Host side of the C ABI declared in include/psvt.h: argument checks,
// workspace layout and the launch plan of each operation.
//
// Orientation.  Every operation works on an l x s iterate X whose Gram
// matrix X^T X is s x s.  Right-sided (Proposition 1): X = A, s = n.
// Left-sided (footnote of Proposition 1): X = A^T, s = m; then
// A_tau = (A^T)_tau^T, so the left-sided formula is the right-sided one on
// the transposed matrix and only the final write is transposed.
//
// Plan of psvt_svt (all on the caller's stream, scalars stay on the device):
//   nu    = ||A||_F (FP64)                         -> scale into the unit ball
//   X0    = X/nu and X0^T (one tiled pass over A)
//   T     = X0^T X0                       (half-flop symmetric product)
//   theta_P = sqrt(||T||_F) >= sigma_max(X0)       (FP64)
//   H     = T - (tau/nu)^2 I              (diagonal shift in FP64)
//   R     = H H,  theta_S = sqrt(||R||_F) >= |lambda|_max(H)
//   P     : K odd-quintic iterations X <- X (a I + b X^T X + c (X^T X)^2)
//           (the first one applies 1/theta_P through device scalars)
//   S     : K iterations X <- a X + (b X^2 + c X^4) X on symmetric X,
//           starting from H / theta_S; the last one writes Pi = (I + S)/2
//   Y     = (nu X0 - tau P) Pi   (= (A - tau P)(I + S)/2, written transposed
//           for the left-sided case)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/psvt.h"
#include "coeffs.h"
#include "kernels.h"
#include "layout.h"
#include "plan.h"

using namespace psvt;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(PSVT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------ device check

constexpr int kMaxDevices = 64;
std::once_flag g_dev_once[kMaxDevices];
int g_dev_ok[kMaxDevices];

int check_device() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PSVT_EUNSUPPORTED, "device index %d out of range", dev);
    std::call_once(g_dev_once[dev], [dev]() {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            g_dev_ok[dev] = -1;
            return;
        }
        g_dev_ok[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    });
    if (g_dev_ok[dev] == 1) return PSVT_OK;
    return fail(PSVT_EUNSUPPORTED, "device %d is not gfx950", dev);
}

// ------------------------------------------------------------- config

struct Cfg {
    int iters;
    int n_fp8, n_bf16;
    int side;
    const double *coeffs;
    uint32_t flags;
    double safety;
    uint32_t *status;
    double status_tol;
    const float *warm_pi;
    float *pi_out;
    int64_t ld_pi;
    int warm_iters;
};

int read_cfg(const psvt_config *c, Cfg &out) {
    out.iters = 20;
    out.n_fp8 = out.n_bf16 = 0;
    out.side = PSVT_SIDE_AUTO;
    out.coeffs = nullptr;
    out.flags = 0;
    out.safety = 1.0;
    out.status = nullptr;
    out.status_tol = 1e-3;
    out.warm_pi = nullptr;
    out.pi_out = nullptr;
    out.ld_pi = 0;
    out.warm_iters = 10;
    if (!c) return PSVT_OK;
    if (c->iters < 0 || c->iters > 256) return fail(PSVT_EINVAL, "iters = %d outside 0..256", c->iters);
    if (c->iters) out.iters = c->iters;
    if (c->n_fp8 < 0 || c->n_bf16 < 0 || (int64_t)c->n_fp8 + c->n_bf16 > out.iters)
        return fail(PSVT_EINVAL, "n_fp8 = %d, n_bf16 = %d do not fit in %d iterations", c->n_fp8, c->n_bf16,
                    out.iters);
    if (c->side < 0 || c->side > 2) return fail(PSVT_EINVAL, "side = %d", c->side);
    const uint32_t known = PSVT_FLAG_SPLIT_P | PSVT_FLAG_PLAIN_S | PSVT_FLAG_PLAIN_P | PSVT_FLAG_STATUS | PSVT_FLAG_HFORM |
                           PSVT_FLAG_PERSISTENT | PSVT_FLAG_GRAM;
    if (c->flags & ~known) return fail(PSVT_EINVAL, "unknown flags 0x%x", c->flags);
    // the batched entry points take this flag off before they get here
    if (c->flags & PSVT_FLAG_PERSISTENT)
        return fail(PSVT_EINVAL, "PSVT_FLAG_PERSISTENT applies to psvt_svt_batched / psvt_rank_r_batched only");
    if ((c->flags & PSVT_FLAG_SPLIT_P) && (c->flags & PSVT_FLAG_PLAIN_P))
        return fail(PSVT_EINVAL, "PSVT_FLAG_SPLIT_P and PSVT_FLAG_PLAIN_P exclude each other");
    if ((c->flags & PSVT_FLAG_GRAM) && (c->flags & PSVT_FLAG_HFORM))
        return fail(PSVT_EINVAL, "PSVT_FLAG_GRAM and PSVT_FLAG_HFORM exclude each other");
    if (c->norm_safety != 0.0 && !(c->norm_safety >= 1.0 && c->norm_safety <= 16.0))
        return fail(PSVT_EINVAL, "norm_safety = %g outside [1, 16]", c->norm_safety);
    if (c->norm_safety != 0.0) out.safety = c->norm_safety;
    if ((c->flags & PSVT_FLAG_STATUS) && !c->status) return fail(PSVT_EINVAL, "PSVT_FLAG_STATUS with a NULL status");
    if (c->status_tol != 0.0 && !(c->status_tol > 0.0 && isfinite(c->status_tol)))
        return fail(PSVT_EINVAL, "status_tol = %g must be finite and > 0", c->status_tol);
    if (c->status_tol != 0.0) out.status_tol = c->status_tol;
    if (c->flags & PSVT_FLAG_STATUS) out.status = c->status;
    if (c->warm_iters < 0 || c->warm_iters > 64) return fail(PSVT_EINVAL, "warm_iters = %d outside 0..64", c->warm_iters);
    if (c->warm_iters) out.warm_iters = c->warm_iters;
    if (out.warm_iters < 2 && c->warm_pi) return fail(PSVT_EINVAL, "a warm start needs warm_iters >= 2");
    out.warm_pi = c->warm_pi;
    out.pi_out = c->pi_out;
    out.ld_pi = c->ld_pi;
    out.flags = c->flags;
    out.n_fp8 = c->n_fp8;
    out.n_bf16 = c->n_bf16;
    out.side = c->side;
    out.coeffs = c->coeffs;
    if (out.coeffs)
        for (int i = 0; i < 3 * out.iters; ++i)
            if (!isfinite(out.coeffs[i])) return fail(PSVT_EINVAL, "coeffs[%d] is not finite", i);
    return PSVT_OK;
}

void coef(const Cfg &c, int t, float &a, float &b, float &cc) {
    const double *p = c.coeffs ? c.coeffs + 3 * t : psvt_coeff_table[t < PSVT_COEFF_LEN ? t : PSVT_COEFF_LEN - 1];
    a = (float)p[0];
    b = (float)p[1];
    cc = (float)p[2];
}

// Operand type of polar iteration t: the first n_fp8 iterations FP8, the
// next n_bf16 BF16, the rest FP32.
int iter_dtype(const Cfg &c, int t) {
    if (t < c.n_fp8) return OP_FP8;
    if (t < c.n_fp8 + c.n_bf16) return OP_BF16;
    return OP_F32;
}

// P iterations: FP8 as scheduled; BF16 as split bf16 unless
// PSVT_FLAG_PLAIN_P (the error of P enters A_tau multiplied by
// tau / (sigma - tau), up to 20 for a 5 % gap, beyond what plain bf16
// operands can carry at 1e-2).
int iter_dtype_P(const Cfg &c, int t) {
    const int d = iter_dtype(c, t);
    return (d == OP_BF16 && !(c.flags & PSVT_FLAG_PLAIN_P)) ? OP_BF16X3 : d;
}

// S iterations work on the shifted Gram, whose spectrum is the square of A's:
// the eigenvalues that decide the sign sit far below bf16 resolution of the
// largest one (sigma_min^2 - tau^2 vs sigma_max^2).  Their low-precision
// iterations therefore use split bf16 (about 16 mantissa bits) unless
// PSVT_FLAG_PLAIN_S asks for plain operands (with the H-form, whose S
// spectrum is linear in sigma, plain operands come within about 1e-2).
int iter_dtype_S(const Cfg &c, int t) {
    const int d = iter_dtype(c, t);
    if (d == OP_F32 || (c.flags & PSVT_FLAG_PLAIN_S)) return d;
    return OP_BF16X3;
}

// FP8 operand scales of one iteration: the copies of X (and X^T), of T = X^T X
// (or X^2) and of B = b T + c T^2 are stored as e4m3(scale * value) and the
// product is multiplied back by 1 / (scale_A scale_B).  Scales are powers of
// two chosen from spectral bounds of the iterate, so that no entry exceeds
// e4m3's largest finite value (448): |entry| <= spectral norm.
struct IterScale {
    float sX, sT, sB;
};

float pow2_scale(double bound) {
    if (!(bound > 0.0)) return 1.0f;
    double s = exp2(floor(log2(448.0 / (1.1 * bound))));
    return (float)fmin(fmax(s, 0x1p-20), 0x1p20);
}

// U_t bounds the singular values entering iteration t (U_0 = 1 after the
// theta normalisation); B_t's eigenvalues are b mu + c mu^2 over
// mu in [0, U_t^2]; the quintic maps [0, U_t] into [-U_{t+1}, U_{t+1}].
// Entry t depends on the coefficients of iterations 0..t only.
void scales_from(const Cfg &c, int count, IterScale *out) {
    double U = 1.0;
    for (int t = 0; t < count; ++t) {
        float a, b, cc;
        coef(c, t, a, b, cc);
        double beta = 0.0, unext = 0.0;
        const int n = 4096;
        for (int k = 0; k <= n; ++k) {
            const double x = U * k / n, mu = x * x;
            beta = fmax(beta, fabs(b * mu + cc * mu * mu));
            unext = fmax(unext, fabs(x * (a + b * mu + cc * mu * mu)));
        }
        out[t] = IterScale{pow2_scale(U), pow2_scale(U * U), pow2_scale(beta)};
        U = fmax(unext, 1e-30);
    }
}

// Scales of the FP8 iterations (entries 0 .. n_fp8 - 1; nothing else reads
// them).  The bound takes 4097 polynomial evaluations per iteration, so the
// built-in schedule's entries are computed once and kept; a caller-supplied
// schedule is evaluated on every call.
void iteration_scales(const Cfg &c, IterScale *out) {
    const int count = c.n_fp8 < c.iters ? c.n_fp8 : c.iters;
    if (count <= 0) return;
    if (c.coeffs) {
        scales_from(c, count, out);
        return;
    }
    static std::mutex mu;
    static IterScale cache[256];
    static int have = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (have < count) {
        scales_from(c, count, cache);
        have = count;
    }
    memcpy(out, cache, sizeof(IterScale) * (size_t)count);
}

// ---------------------------------------------------------- workspace

// right-sided iff n < m in auto mode (the listing's rule; square -> left)
bool choose_right(int side, int64_t m, int64_t n) {
    if (side == PSVT_SIDE_RIGHT) return true;
    if (side == PSVT_SIDE_LEFT) return false;
    return n < m;
}

// Layout of op on an m x n input (layout.h).  single: a stand-alone call on
// its own stream, which may fork P's iterations to a side stream (not a
// batch item or a served request, whose stages are recorded and replayed in
// one stream).
Layout make_layout(int op, int64_t m, int64_t n, const Cfg &c, bool single = false) {
    bool right;
    int64_t l, s;
    if (op == PSVT_OP_POLAR_SYM) {
        right = true;
        l = s = n;
    } else if (op == PSVT_OP_POLAR) {
        // polar(A^T) = polar(A)^T: iterate on the tall orientation
        right = c.side == PSVT_SIDE_AUTO ? (m >= n) : choose_right(c.side, m, n);
        l = right ? m : n;
        s = right ? n : m;
    } else {
        right = choose_right(c.side, m, n);
        l = right ? m : n;
        s = right ? n : m;
    }
    return layout_for(op, l, s, right, c.n_fp8 + c.n_bf16 > 0, single);
}

// ------------------------------------------------------------ checks

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
    return rows <= 0 || cols <= 0 ? 0 : sizeof(float) * (size_t)((rows - 1) * ld + cols);
}

int check_matrix(const void *p, int64_t rows, int64_t cols, int64_t ld, const char *name) {
    if (rows < 0 || cols < 0) return fail(PSVT_EINVAL, "%s: negative size %lld x %lld", name, (long long)rows,
                                          (long long)cols);
    if (rows == 0 || cols == 0) return PSVT_OK;
    if (!p) return fail(PSVT_EINVAL, "%s is NULL", name);
    if (ld < cols) return fail(PSVT_EINVAL, "%s: ld = %lld < %lld columns", name, (long long)ld, (long long)cols);
    if (rows > (1LL << 30) || cols > (1LL << 30)) return fail(PSVT_EINVAL, "%s: dimension too large", name);
    return PSVT_OK;
}

// ------------------------------------------------------------- helpers

GemmArgs gemm_defaults() {
    GemmArgs g;
    memset(&g, 0, sizeof g);
    g.alpha = 1.0f;
    g.wa = 1.0f;
    g.ab_scale = 1.0f;
    g.lp_scale = 1.0f;
    g.i_alpha = g.i_beta = g.i_wa = g.i_wa2 = -1;
    return g;
}

char *at(void *ws, size_t off) { return (char *)ws + off; }
float *F(void *ws, size_t off) { return (float *)at(ws, off); }

// symmetric product C = alpha A B^T + beta D (+ diag I), A, B, C, D s x s
hipError_t syrk(const float *A, const float *B, int64_t ld, const float *D, float *C, int64_t ldc, int64_t s,
                float alpha, int i_alpha, float beta, int i_beta, float diag, const Scalars *sc, Exec &ex) {
    GemmArgs g = gemm_defaults();
    g.A = A;
    g.B = B;
    g.lda = g.ldb = ld;
    g.D = D;
    g.ldd = D ? ld : 0;
    g.C = C;
    g.ldc = ldc;
    g.M = g.N = (int)s;
    g.K = (int)s;
    g.alpha = alpha;
    g.i_alpha = i_alpha;
    g.beta = beta;
    g.i_beta = i_beta;
    g.diag = diag;
    g.sc = sc;
    g.sym = 1;
    return ex.gemm(g, OP_F32, "syrk");
}

// Gram prelude shared by svt / polar / rank_r: nu, X0, X0^T, T, theta_P.
int prelude(const float *A, int64_t m, int64_t n, int64_t lda, double tau, const Layout &L, void *ws,
            Exec &ex, bool want_theta_p, double safety) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    double *part = (double *)at(ws, L.part);
    HIP_TRY(ex.norm(make_norm_op(A, m, n, lda, part, sc, NORM_INPUT, tau), "norm of A"), "norm of A");
    float *X0 = F(ws, L.X0), *X0T = F(ws, L.X0T);
    // right: X = A -> X0 = A/nu (copy), X0T = A^T/nu; left: X = A^T -> swapped
    if (L.right)
        HIP_TRY(ex.tile(make_scale_transpose(A, m, n, lda, X0, L.ldS, X0T, L.ldL, sc, F_INV_NU), "scale A"), "scale A");
    else
        HIP_TRY(ex.tile(make_scale_transpose(A, m, n, lda, X0T, L.ldL, X0, L.ldS, sc, F_INV_NU), "scale A"), "scale A");
    // T = X0^T X0 = (X0^T)(X0^T)^T : NT product of the s x l transposed copy
    GemmArgs g = gemm_defaults();
    g.A = X0T;
    g.B = X0T;
    g.lda = g.ldb = L.ldL;
    g.C = F(ws, L.T);
    g.ldc = L.ldS;
    g.M = g.N = (int)L.s;
    g.K = (int)L.l;
    g.sc = sc;
    g.sym = 1;
    HIP_TRY(ex.gemm(g, OP_F32, "Gram"), "Gram");
    if (want_theta_p) {
        NormOp op = make_norm_op(F(ws, L.T), L.s, L.s, L.ldS, part, sc, NORM_THETA_P, 0.0);
        op.safety = safety;
        HIP_TRY(ex.norm(op, "theta_P"), "theta_P");
    }
    return PSVT_OK;
}

// Low-precision operand settings of one product: operands in `dt` with
// scales sa, sb; FP32 iterations keep every scale at 1.
void set_operand_scales(GemmArgs &g, int dt, float sa, float sb) {
    if (dt != OP_F32) g.ab_scale = 1.0f / (sa * sb);
}

// Low-precision copies that a product writes for the next consumer.
void set_lp_out(GemmArgs &g, int type, void *row, int64_t ldrow, void *trans, int64_t ldtrans, float scale,
                int64_t plane, int64_t plane_t = 0) {
    g.lp_plane = plane;
    g.lp_plane_t = plane_t;
    g.lp_type = type;
    g.Clp = row;
    g.ldclp = ldrow;
    g.CTlp = trans;
    g.ldctlp = ldtrans;
    g.lp_scale = scale;
}

// P iterations.  Result in *out_P (workspace, l x s, ld = ldS) or, when
// user_out is given, the last iteration writes straight to the caller's
// buffer (transposed when !L.right).
//
// Iteration t in operand type dt keeps the FP32 master X and reads its
// low-precision copies: T = X^T X (from the copy of X^T), B = c T^2 + b T
// (from the copy of T, with the FP32 T as the b-term), X' = a X + X B (from
// the copies of X and B, with the FP32 X as the a-term).  Each product writes
// the copies its consumer needs, in the consumer's type.
int polar_iterations(const Cfg &c, const Layout &L, void *ws, Exec &ex, float *user_out, int64_t ld_out,
                     const float **out_P, const float **out_PT = nullptr) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    IterScale scl[257];
    iteration_scales(c, scl);
    const float *curX = F(ws, L.X0), *curXT = F(ws, L.X0T);
    const void *curXlp = nullptr, *curXTlp = nullptr;
    float *bufX[2] = {F(ws, L.Xp), F(ws, L.Xq)};
    float *bufXT[2] = {F(ws, L.XTp), F(ws, L.XTq)};
    void *bufXlp[2] = {L.lp ? at(ws, L.XL[0]) : nullptr, L.lp ? at(ws, L.XL[1]) : nullptr};
    void *bufXTlp[2] = {L.lp ? at(ws, L.XTL[0]) : nullptr, L.lp ? at(ws, L.XTL[1]) : nullptr};
    float *T = F(ws, L.T), *Bm = F(ws, L.Bm);
    void *Tlp = L.lp ? at(ws, L.TL) : nullptr, *Blp = L.lp ? at(ws, L.BL) : nullptr;
    for (int t = 0; t < c.iters; ++t) {
        float a, b, cc;
        coef(c, t, a, b, cc);
        const bool first = t == 0, last = t == c.iters - 1;
        const int dt = iter_dtype_P(c, t), nd = last ? OP_F32 : iter_dtype_P(c, t + 1);
        const bool lp = dt != OP_F32;
        const float sX = dt == OP_FP8 ? scl[t].sX : 1.0f, sT = dt == OP_FP8 ? scl[t].sT : 1.0f,
                    sB = dt == OP_FP8 ? scl[t].sB : 1.0f, sXn = nd == OP_FP8 ? scl[t + 1].sX : 1.0f;
        if (first && lp) {
            // theta is folded into the first copies: X0 / theta and T / theta^2
            HIP_TRY(ex.tile(make_convert(curX, L.l, L.s, L.ldS, bufXlp[1], L.ldS, dt, sX, 0, sc, F_P1, L.planeX), "P: X0 copy"), "P: X0 copy");
            HIP_TRY(ex.tile(make_convert(T, L.s, L.s, L.ldS, Tlp, L.ldS, dt, sT, 0, sc, F_P2, L.planeS), "P: T copy"), "P: T copy");
            curXlp = bufXlp[1];
        }
        if (!first) {  // T = X^T X
            GemmArgs g = gemm_defaults();
            g.A = g.B = lp ? curXTlp : (const void *)curXT;
            g.lda = g.ldb = L.ldL;
            g.a_plane = g.b_plane = L.planeXT;
            g.C = T;
            g.ldc = L.ldS;
            g.M = g.N = (int)L.s;
            g.K = (int)L.l;
            g.sc = sc;
            g.sym = 1;
            set_operand_scales(g, dt, sX, sX);
            if (lp) set_lp_out(g, dt, Tlp, L.ldS, nullptr, 0, sT, L.planeS);
            HIP_TRY(ex.gemm(g, dt, "P: X^T X"), "P: X^T X");
        }
        {  // B = c T^2 + b T   (first iteration: theta scaling through device scalars)
            GemmArgs g = gemm_defaults();
            g.A = g.B = lp ? Tlp : (const void *)T;
            g.lda = g.ldb = L.ldS;
            g.a_plane = g.b_plane = L.planeS;
            g.D = T;
            g.ldd = L.ldS;
            g.M = g.N = g.K = (int)L.s;
            g.alpha = cc;
            g.i_alpha = (first && !lp) ? F_P4 : -1;
            g.beta = b;
            g.i_beta = first ? F_P2 : -1;
            g.sc = sc;
            g.sym = 1;
            set_operand_scales(g, dt, sT, sT);
            if (lp) {
                set_lp_out(g, dt, Blp, L.ldS, nullptr, 0, sB, L.planeS);
            } else {
                g.C = Bm;
                g.ldc = L.ldS;
            }
            HIP_TRY(ex.gemm(g, dt, "P: b T + c T^2"), "P: b T + c T^2");
        }
        {  // X' = a X + X B   (first iteration: times 1/theta)
            GemmArgs g = gemm_defaults();
            g.A = lp ? curXlp : (const void *)curX;
            g.lda = L.ldS;
            g.B = lp ? (const void *)Blp : (const void *)Bm;
            g.ldb = L.ldS;
            g.a_plane = L.planeX;
            g.b_plane = L.planeS;
            g.D = curX;
            g.ldd = L.ldS;
            g.M = (int)L.l;
            g.N = (int)L.s;
            g.K = (int)L.s;
            g.alpha = 1.0f;
            g.i_alpha = (first && !lp) ? F_P1 : -1;
            g.beta = a;
            g.i_beta = first ? F_P1 : -1;
            g.sc = sc;
            set_operand_scales(g, dt, sX, sB);
            const int k = t & 1;
            if (last && user_out) {
                if (L.right) {
                    g.C = user_out;
                    g.ldc = ld_out;
                } else {
                    g.CT = user_out;
                    g.ldct = ld_out;
                }
            } else {
                g.C = bufX[k];
                g.ldc = L.ldS;
                if (last && out_PT) {  // P^T too, for the H-form's P^T X0
                    g.CT = bufXT[k];
                    g.ldct = L.ldL;
                }
                if (!last) {
                    if (nd == OP_F32) {
                        g.CT = bufXT[k];
                        g.ldct = L.ldL;
                    } else {
                        set_lp_out(g, nd, bufXlp[k], L.ldS, bufXTlp[k], L.ldL, sXn, L.planeX, L.planeXT);
                    }
                }
            }
            HIP_TRY(ex.gemm(g, dt, "P: a X + X B"), "P: a X + X B");
            curX = bufX[k];
            curXT = bufXT[k];
            curXlp = bufXlp[k];
            curXTlp = bufXTlp[k];
        }
    }
    if (out_P) *out_P = curX;
    if (out_PT) *out_PT = curXT;
    return PSVT_OK;
}

// S iterations from H (s x s, ld = ldS) with R = H^2 and theta_S already in
// the scalar block.  want_pi: the last iteration writes (I + S)/2.  Same
// precision scheme as the P iterations, with X^2 in place of X^T X.
//
// Warm start (c.warm_pi, svt / rank_r): the iteration starts from
// X0 = (H / theta_S + eps S_prev) / (1 + eps), S_prev = 2 Pi_prev - I,
// eps = kWarmEps.  Every eigenvalue of X0 is then at least about eps away
// from 0 unless H and S_prev disagree there, so the built-in schedule
// (designed for eigenvalues from 1e-3 up) converges in c.warm_iters steps
// instead of the cold start's; H decides every direction with
// |lambda| / theta_S >> eps, so an error inherited from S_prev is damped by
// about eps theta_S / |lambda| per call instead of carried along.
constexpr float kWarmEps = 1e-3f;

int sign_iterations(const Cfg &c, const Layout &L, void *ws, Exec &ex, bool want_pi, float *user_out,
                    int64_t ld_out, const float **out_S) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    IterScale scl[257];
    iteration_scales(c, scl);
    const int64_t s = L.s, ld = L.ldS;
    const float *cur = F(ws, L.H);
    const void *curlp = nullptr;
    float *R = F(ws, L.R), *X2 = F(ws, L.X2), *BS = F(ws, L.BS);
    float *buf[2] = {F(ws, L.S0), F(ws, L.S1)};
    void *buflp[2] = {L.lp ? at(ws, L.SL[0]) : nullptr, L.lp ? at(ws, L.SL[1]) : nullptr};
    void *X2lp = L.lp ? at(ws, L.X2L) : nullptr, *BSlp = L.lp ? at(ws, L.BSL) : nullptr;
    const bool warm = c.warm_pi && want_pi;
    const int K = warm ? c.warm_iters : c.iters;
    // operand type of iteration t
    auto dtype_of = [&](int t) {
        if (!warm) return iter_dtype_S(c, t);
        if (t >= K - 2 || c.n_fp8 + c.n_bf16 == 0) return (int)OP_F32;
        return (c.flags & PSVT_FLAG_PLAIN_S) ? (int)OP_BF16 : (int)OP_BF16X3;
    };
    if (warm) {
        HIP_TRY(ex.tile(make_warm_start(F(ws, L.H), c.warm_pi, c.ld_pi, s, ld, buf[1], ld, sc, F_S1, kWarmEps),
                        "S: warm start"),
                "S: warm start");
        cur = buf[1];
    }
    for (int t = 0; t < K; ++t) {
        float a, b, cc;
        coef(c, t, a, b, cc);
        const bool first = t == 0 && !warm, last = t == K - 1;
        const int dt = dtype_of(t), nd = last ? OP_F32 : dtype_of(t + 1);
        const bool lp = dt != OP_F32;
        const bool fp8 = !warm && dt == OP_FP8;
        const float sX = fp8 ? scl[t].sX : 1.0f, sT = fp8 ? scl[t].sT : 1.0f, sB = fp8 ? scl[t].sB : 1.0f,
                    sXn = (!warm && nd == OP_FP8) ? scl[t + 1].sX : 1.0f;
        if (first && lp) {
            HIP_TRY(ex.tile(make_convert(cur, s, s, ld, buflp[1], ld, dt, sX, 0, sc, F_S1, L.planeS), "S: H copy"), "S: H copy");
            HIP_TRY(ex.tile(make_convert(R, s, s, ld, X2lp, ld, dt, sT, 0, sc, F_S2, L.planeS), "S: H^2 copy"), "S: H^2 copy");
            curlp = buflp[1];
        } else if (warm && t == 0 && lp) {
            HIP_TRY(ex.tile(make_convert(cur, s, s, ld, buflp[1], ld, dt, 1.0f, 0, sc, -1, L.planeS), "S: warm copy"),
                    "S: warm copy");
            curlp = buflp[1];
        }
        const float *sq = R;
        if (!first) {  // X^2
            GemmArgs g = gemm_defaults();
            g.A = g.B = lp ? curlp : (const void *)cur;
            g.lda = g.ldb = ld;
            g.a_plane = g.b_plane = L.planeS;
            g.C = X2;
            g.ldc = ld;
            g.M = g.N = g.K = (int)s;
            g.sc = sc;
            g.sym = 1;
            set_operand_scales(g, dt, sX, sX);
            if (lp) set_lp_out(g, dt, X2lp, ld, nullptr, 0, sT, L.planeS);
            HIP_TRY(ex.gemm(g, dt, "S: X^2"), "S: X^2");
            sq = X2;
        }
        {  // B = c X^4 + b X^2
            GemmArgs g = gemm_defaults();
            g.A = g.B = lp ? (const void *)X2lp : (const void *)sq;
            g.lda = g.ldb = ld;
            g.a_plane = g.b_plane = L.planeS;
            g.D = sq;
            g.ldd = ld;
            g.M = g.N = g.K = (int)s;
            g.alpha = cc;
            g.i_alpha = (first && !lp) ? F_S4 : -1;
            g.beta = b;
            g.i_beta = first ? F_S2 : -1;
            g.sc = sc;
            g.sym = 1;
            set_operand_scales(g, dt, sT, sT);
            if (lp) {
                set_lp_out(g, dt, BSlp, ld, nullptr, 0, sB, L.planeS);
            } else {
                g.C = BS;
                g.ldc = ld;
            }
            HIP_TRY(ex.gemm(g, dt, "S: b X^2 + c X^4"), "S: b X^2 + c X^4");
        }
        {  // X' = a X + B X  (symmetric: B and X commute)
            float alpha = 1.0f, beta = a, diag = 0.0f;
            if (last && want_pi) {
                alpha = 0.5f;
                beta = 0.5f * a;
                diag = 0.5f;
            }
            GemmArgs g = gemm_defaults();
            g.A = lp ? (const void *)BSlp : (const void *)BS;
            g.B = lp ? curlp : (const void *)cur;
            g.lda = g.ldb = ld;
            g.a_plane = g.b_plane = L.planeS;
            g.D = cur;
            g.ldd = ld;
            g.M = g.N = g.K = (int)s;
            g.alpha = alpha;
            g.i_alpha = (first && !lp) ? F_S1 : -1;
            g.beta = beta;
            g.i_beta = first ? F_S1 : -1;
            g.diag = diag;
            g.sc = sc;
            g.sym = 1;
            set_operand_scales(g, dt, sB, sX);
            const int k = t & 1;
            float *dst = (last && user_out) ? user_out : buf[k];
            g.C = dst;
            g.ldc = (last && user_out) ? ld_out : ld;
            if (!last && nd != OP_F32) set_lp_out(g, nd, buflp[k], ld, nullptr, 0, sXn, L.planeS);
            HIP_TRY(ex.gemm(g, dt, "S: a X + B X"), "S: a X + B X");
            cur = dst;
            curlp = buflp[k];
        }
    }
    if (want_pi && c.pi_out)  // this call's Pi for the next warm start
        HIP_TRY(ex.tile(make_scale_transpose(cur, s, s, ld, c.pi_out, c.ld_pi, nullptr, 0, nullptr, -1), "S: Pi out"),
                "S: Pi out");
    if (out_S) *out_S = cur;
    return PSVT_OK;
}

// H = T - (tau/nu)^2 I, R = H^2, theta_S
int shifted_gram(const Layout &L, void *ws, Exec &ex, double safety) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    double *part = (double *)at(ws, L.part);
    HIP_TRY(ex.tile(make_shift_copy(F(ws, L.T), L.s, L.ldS, F(ws, L.H), L.ldS, sc), "shift"), "shift");
    HIP_TRY(syrk(F(ws, L.H), F(ws, L.H), L.ldS, nullptr, F(ws, L.R), L.ldS, L.s, 1.0f, -1, 0.0f, -1, 0.0f, sc, ex),
            "H^2");
    NormOp op = make_norm_op(F(ws, L.R), L.s, L.s, L.ldS, part, sc, NORM_THETA_S, 0.0);
    op.safety = safety;
    HIP_TRY(ex.norm(op, "theta_S"), "theta_S");
    return PSVT_OK;
}

// H-form (the proof of Proposition 1: S = V1 V1^T - V2 V2^T = sign(P^T A -
// tau I), since P^T A = V Sigma V^T): H = P^T X0 - (tau/nu) I, R = H^2,
// theta_S.  P^T X0 is symmetric in exact arithmetic, so it is computed as
// a lower-triangle product (exactly symmetric) into T, free once P exists.
int hform_shifted(const Layout &L, void *ws, const float *PT, Exec &ex, double safety) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    double *part = (double *)at(ws, L.part);
    GemmArgs g = gemm_defaults();
    g.A = PT;
    g.B = F(ws, L.X0T);
    g.lda = g.ldb = L.ldL;
    g.C = F(ws, L.T);
    g.ldc = L.ldS;
    g.M = g.N = (int)L.s;
    g.K = (int)L.l;
    g.sc = sc;
    g.sym = 1;
    HIP_TRY(ex.gemm(g, OP_F32, "H-form: P^T X0"), "H-form: P^T X0");
    HIP_TRY(ex.tile(make_shift_copy(F(ws, L.T), L.s, L.ldS, F(ws, L.H), L.ldS, sc, D_TAU), "H-form: shift"),
            "H-form: shift");
    HIP_TRY(syrk(F(ws, L.H), F(ws, L.H), L.ldS, nullptr, F(ws, L.R), L.ldS, L.s, 1.0f, -1, 0.0f, -1, 0.0f, sc, ex),
            "H^2");
    NormOp op = make_norm_op(F(ws, L.R), L.s, L.s, L.ldS, part, sc, NORM_THETA_S, 0.0);
    op.safety = safety;
    HIP_TRY(ex.norm(op, "theta_S"), "theta_S");
    return PSVT_OK;
}

// Status word (PSVT_FLAG_STATUS), after the output is written.  sign: the
// final sign iterate as Pi = (I + S)/2 (pi = true) or S itself, s x s in
// the workspace or the caller's buffer; its convergence is measured as
// ||S^2 - I||_F / sqrt(s) (= 4 ||Pi^2 - Pi||_F / sqrt(s)) with the square
// written to the R buffer (free once the sign iterations are done).  Then
// a norm pass over the output checks it for non-finite entries and writes
// the word.
int status_stages(const Cfg &c, const Layout &L, void *ws, Exec &ex, const float *sign, int64_t ld_sign, bool pi,
                  const float *out, int64_t rows, int64_t cols, int64_t ld_out) {
    if (!c.status) return PSVT_OK;
    Scalars *sc = (Scalars *)at(ws, L.scal);
    double *part = (double *)at(ws, L.part);
    double tol = -1.0;
    if (sign) {
        GemmArgs g = gemm_defaults();
        g.A = g.B = sign;
        g.lda = g.ldb = ld_sign;
        g.C = F(ws, L.R);
        g.ldc = L.ldS;
        g.M = g.N = g.K = (int)L.s;
        g.sc = sc;
        g.sym = 1;
        if (pi) {  // Pi^2 - Pi
            g.D = sign;
            g.ldd = ld_sign;
            g.beta = -1.0f;
        } else {   // S^2 - I
            g.diag = -1.0f;
        }
        HIP_TRY(ex.gemm(g, OP_F32, "status: S^2 - I"), "status: S^2 - I");
        NormOp op = make_norm_op(F(ws, L.R), L.s, L.s, L.ldS, part, sc, NORM_CONV, 0.0);
        op.scale = pi ? 4.0 : 1.0;  // over sqrt(s): an RMS over the s eigenvalues
        HIP_TRY(ex.norm(op, "status: convergence"), "status: convergence");
        tol = c.status_tol;
    }
    NormOp op = make_norm_op(out, rows, cols, ld_out, part, sc, NORM_STATUS, 0.0);
    op.status = c.status;
    op.tol = tol;
    HIP_TRY(ex.norm(op, "status"), "status");
    return PSVT_OK;
}

// Y = (nu X0 [- tau P]) Pi, written transposed for the left-sided case.
int final_product(const Layout &L, void *ws, const float *P, double tau, const float *Pi, float *Y, int64_t ldy,
                  Exec &ex) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    GemmArgs g = gemm_defaults();
    g.A = F(ws, L.X0);
    g.lda = L.ldS;
    g.wa = 1.0f;
    g.i_wa = F_NU;
    if (P) {
        g.A2 = P;
        g.lda2 = L.ldS;
        g.wa2 = (float)(-tau);
    }
    g.B = Pi;
    g.ldb = L.ldS;
    g.M = (int)L.l;
    g.N = (int)L.s;
    g.K = (int)L.s;
    g.sc = sc;
    if (L.right) {
        g.C = Y;
        g.ldc = ldy;
    } else {
        g.CT = Y;
        g.ldct = ldy;
    }
    HIP_TRY(ex.gemm(g, OP_F32, "final product"), "final product");
    return PSVT_OK;
}

// Gram form of the polar factor (PSVT_FLAG_GRAM).  With T = X0^T X0 and
// Y0 = T / theta_P^2, every polar iterate is X_k = X0 N_k / theta_P with N_k
// a polynomial in T, and its Gram matrix Y_k = N_k Y0 N_k is one too; the
// odd-quintic step X <- X p(X^T X), p(y) = a + b y + c y^2, becomes
//   Q = p(Y_k),  N_{k+1} = N_k Q,  Y_{k+1} = Y_k Q^2
// (N_0 = I, so N_1 = p(Y0) and Y_1 = Y0 N_1^2): s x s products only, FP32.
// N_K tends to Y0^{-1/2}, so P = X0 T^{-1/2} = X0 N_K / theta_P.
// Only the directions that Pi = (I + S)/2 keeps matter, so the iteration
// runs on Y0' = Pi Y0 Pi + (I - Pi): the same on those directions, 1 on the
// others (which Pi removes again at the end).  Its spectrum lies in
// [tau^2 / theta_P^2, 1] instead of reaching down to the smallest singular
// value: N stays below theta_P / tau instead of growing like the inverse of
// the smallest one, which is what keeps the FP32 iteration stable.  The
// matrices are symmetric in exact arithmetic; each product is taken in full
// and symmetrised as (C + C^T) / 2, since the iteration amplifies an
// antisymmetric rounding part (keeping one triangle is not enough).
// Buffers: Y0' over T, Q in Bm, Pi Y0 and Y Q in Xp, Y in BS, N in Xq / X2,
// the unsymmetrised products in H (the S-side buffers other than Pi's are
// free once the sign iterations are done).
int gram_step(const float *A, const float *B, const float *D, float alpha, int i_alpha, float beta, int i_beta,
              float diag, float *dst, float *tmp, const Layout &L, const Scalars *sc, Exec &ex, const char *what) {
    GemmArgs g = gemm_defaults();
    g.A = A;
    g.B = B;
    g.lda = g.ldb = L.ldS;
    g.D = D;
    g.ldd = D ? L.ldS : 0;
    g.C = tmp;
    g.ldc = L.ldS;
    g.M = g.N = g.K = (int)L.s;
    g.alpha = alpha;
    g.i_alpha = i_alpha;
    g.beta = beta;
    g.i_beta = i_beta;
    g.diag = diag;
    g.sc = sc;
    HIP_TRY(ex.gemm(g, OP_F32, what), what);
    TileOp op = make_symmetrize_scale(tmp, L.s, L.ldS, dst, L.ldS, sc);
    op.i_scale = -1;  // (C + C^T) / 2, no scaling
    HIP_TRY(ex.tile(op, what), what);
    return PSVT_OK;
}

int gram_polar(const Cfg &c, const Layout &L, void *ws, const float *Pi, Exec &ex, const float **out_N) {
    const Scalars *sc = (const Scalars *)at(ws, L.scal);
    float *T = F(ws, L.T);
    float *Q = F(ws, L.Bm), *W = F(ws, L.Xp), *Y = F(ws, L.BS), *tmp = F(ws, L.H);
    float *Nb[2] = {F(ws, L.Xq), F(ws, L.X2)};
    // Y0' = Pi Y0 Pi + (I - Pi): W = Pi T / theta^2, then W Pi - Pi + I into T
    GemmArgs g = gemm_defaults();
    g.A = Pi;
    g.B = T;
    g.lda = g.ldb = L.ldS;
    g.C = W;
    g.ldc = L.ldS;
    g.M = g.N = g.K = (int)L.s;
    g.i_alpha = F_P2;
    g.sc = sc;
    HIP_TRY(ex.gemm(g, OP_F32, "gram Pi Y0"), "gram Pi Y0");
    int rc;
    if ((rc = gram_step(W, Pi, Pi, 1.0f, -1, -1.0f, -1, 1.0f, T, tmp, L, sc, ex, "gram Y0"))) return rc;
    const int K = c.iters;
    int cur = 0;
    for (int t = 0; t < K; ++t) {
        float a, b, cc;
        coef(c, t, a, b, cc);
        const float *Yt = t == 0 ? T : Y;
        if (t == 0) {  // N_1 = p(Y0')
            if ((rc = gram_step(T, T, T, cc, -1, b, -1, a, Nb[0], tmp, L, sc, ex, "gram N"))) return rc;
        } else {
            if ((rc = gram_step(Y, Y, Y, cc, -1, b, -1, a, Q, tmp, L, sc, ex, "gram Q"))) return rc;
            if ((rc = gram_step(Nb[cur], Q, nullptr, 1.0f, -1, 0.0f, -1, 0.0f, Nb[cur ^ 1], tmp, L, sc, ex, "gram N")))
                return rc;
            cur ^= 1;
        }
        if (t + 1 < K) {  // Y <- Y Q Q  (t = 0: Y0' N_1 N_1)
            const float *Qt = t == 0 ? Nb[0] : Q;
            if ((rc = gram_step(Yt, Qt, nullptr, 1.0f, -1, 0.0f, -1, 0.0f, W, tmp, L, sc, ex, "gram Y Q"))) return rc;
            if ((rc = gram_step(W, Qt, nullptr, 1.0f, -1, 0.0f, -1, 0.0f, Y, tmp, L, sc, ex, "gram Y"))) return rc;
        }
    }
    *out_N = Nb[cur];
    return PSVT_OK;
}

// Final product of the Gram form: A - tau P = X0 (nu I - (tau / theta_P) N),
// so A_tau = X0 F with F = (nu I - (tau / theta_P) N) Pi.  The product takes
// F^T = nu Pi - (tau / theta_P) Pi N (one s x s product, into Xp) as the
// rows of its NT operand, then Y = X0 F (transposed for the left side).
// Both weights come from the scalar block (nu, and tau / theta_P written by
// the theta_P pass), so the stage does not depend on tau itself.
int gram_final(const Layout &L, void *ws, const float *N, double tau, const float *Pi, float *Y, int64_t ldy,
               Exec &ex) {
    Scalars *sc = (Scalars *)at(ws, L.scal);
    float *Ft = F(ws, L.Xp);
    GemmArgs g = gemm_defaults();
    g.A = Pi;
    g.B = N;
    g.lda = g.ldb = L.ldS;
    g.D = Pi;
    g.ldd = L.ldS;
    g.C = Ft;
    g.ldc = L.ldS;
    g.M = g.N = g.K = (int)L.s;
    g.alpha = -1.0f;
    g.i_alpha = F_TAU_P;
    g.beta = 1.0f;
    g.i_beta = F_NU;
    g.sc = sc;
    HIP_TRY(ex.gemm(g, OP_F32, "gram F"), "gram F");
    GemmArgs h = gemm_defaults();
    h.A = F(ws, L.X0);
    h.lda = L.ldS;
    h.B = Ft;
    h.ldb = L.ldS;
    h.M = (int)L.l;
    h.N = (int)L.s;
    h.K = (int)L.s;
    h.sc = sc;
    if (L.right) {
        h.C = Y;
        h.ldc = ldy;
    } else {
        h.CT = Y;
        h.ldct = ldy;
    }
    HIP_TRY(ex.gemm(h, OP_F32, "final product"), "final product");
    return PSVT_OK;
}

// Warm-start buffers: s x s with row stride ld_pi, outside the workspace.
int check_warm(const Cfg &c, const Layout &L, const void *ws) {
    if (!c.warm_pi && !c.pi_out) return PSVT_OK;
    if (c.ld_pi < L.s) return fail(PSVT_EINVAL, "ld_pi = %lld < %lld (the Gram side)", (long long)c.ld_pi, (long long)L.s);
    const size_t pib = span_bytes(L.s, L.s, c.ld_pi);
    if ((c.warm_pi && overlaps(c.warm_pi, pib, ws, L.total)) || (c.pi_out && overlaps(c.pi_out, pib, ws, L.total)))
        return fail(PSVT_EINVAL, "warm_pi / pi_out must not overlap ws");
    return PSVT_OK;
}

int check_ws(void *ws, size_t ws_bytes, const Layout &L) {
    if (!ws) return fail(PSVT_EWORKSPACE, "workspace is NULL");
    if (ws_bytes < L.total)
        return fail(PSVT_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, L.total);
    if (((uintptr_t)ws & 255) != 0) return fail(PSVT_EINVAL, "workspace is not 256-byte aligned");
    return PSVT_OK;
}

// The stage list of svt / rank_r (Proposition 1 / Corollary 1).
// A library-owned second stream per (host thread, device) and the two events
// of a fork/join with the caller's stream.  Created on first use, kept for
// the life of the thread (default priority, non-blocking).
struct SideStream {
    hipStream_t st = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool failed = false;
};
SideStream *side_stream() {
    static thread_local SideStream sides[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    SideStream &s = sides[dev];
    if (s.failed) return nullptr;
    if (!s.st) {
        if (hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s.join, hipEventDisableTiming) != hipSuccess) {
            s.failed = true;
            return nullptr;
        }
    }
    return &s;
}

// One recorded stage, launched on `st`.
hipError_t launch_stage(const Stage &s, hipStream_t st) {
    if (s.kind == ST_GEMM) return launch_gemm(s.g, s.dtype, st);
    if (s.kind == ST_NORM) return launch_norm_op(s.n, st);
    return launch_tile_op(s.t, st);
}

int plan_svt_like(int op, const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy,
                  void *ws, const Layout &L, const Cfg &c, Exec &ex) {
    int rc;
    if ((rc = check_warm(c, L, ws))) return rc;
    if ((c.flags & PSVT_FLAG_HFORM) && op != PSVT_OP_SVT)
        return fail(PSVT_EINVAL, "PSVT_FLAG_HFORM applies to svt only (it needs the polar factor)");
    if ((c.flags & PSVT_FLAG_HFORM) && c.n_fp8 > 0)
        return fail(PSVT_EINVAL, "PSVT_FLAG_HFORM takes S from P^T A: P's e4m3 iterations are too coarse for it");
    if (c.flags & PSVT_FLAG_GRAM) {  // S as usual, then P in Gram form: s x s products only
        if (op != PSVT_OP_SVT) return fail(PSVT_EINVAL, "PSVT_FLAG_GRAM applies to svt only");
        const float *N = nullptr, *Pi = nullptr;
        if ((rc = prelude(A, m, n, lda, tau, L, ws, ex, true, c.safety))) return rc;
        if ((rc = shifted_gram(L, ws, ex, c.safety))) return rc;
        if (ex.rec) {
            ex.cut[0] = ex.cut[1] = ex.cut[2] = ex.rec->size();
            ex.chains = false;
        }
        if ((rc = sign_iterations(c, L, ws, ex, true, nullptr, 0, &Pi))) return rc;
        if ((rc = gram_polar(c, L, ws, Pi, ex, &N))) return rc;
        if ((rc = gram_final(L, ws, N, tau, Pi, Y, ldy, ex))) return rc;
        return status_stages(c, L, ws, ex, Pi, L.ldS, true, Y, m, n, ldy);
    }
    if (c.flags & PSVT_FLAG_HFORM) {  // P first, then S from P^T A (no concurrent chains)
        const float *P = nullptr, *PT = nullptr, *Pi = nullptr;
        if ((rc = prelude(A, m, n, lda, tau, L, ws, ex, true, c.safety))) return rc;
        if ((rc = polar_iterations(c, L, ws, ex, nullptr, 0, &P, &PT))) return rc;
        if ((rc = hform_shifted(L, ws, PT, ex, c.safety))) return rc;
        if (ex.rec) {
            ex.cut[0] = ex.cut[1] = ex.cut[2] = ex.rec->size();
            ex.chains = false;
        }
        if ((rc = sign_iterations(c, L, ws, ex, true, nullptr, 0, &Pi))) return rc;
        if ((rc = final_product(L, ws, P, tau, Pi, Y, ldy, ex))) return rc;
        return status_stages(c, L, ws, ex, Pi, L.ldS, true, Y, m, n, ldy);
    }
    if ((rc = prelude(A, m, n, lda, tau, L, ws, ex, op == PSVT_OP_SVT, c.safety))) return rc;
    if ((rc = shifted_gram(L, ws, ex, c.safety))) return rc;
    const float *P = nullptr, *Pi = nullptr;
    SideStream *side = nullptr;
    if (L.fork && !ex.rec && (side = side_stream())) {
        HIP_TRY(hipEventRecord(side->fork, ex.st), "fork");
        HIP_TRY(hipStreamWaitEvent(side->st, side->fork, 0), "fork");
    }
    if (side) {
        // both chains recorded first, then enqueued alternately, so that the
        // S stream has work from the start instead of after all of P's
        // launches (the host's launch rate bounds the small sizes)
        std::vector<Stage> sp, ss;
        Exec rp, rs;
        rp.rec = &sp;
        rs.rec = &ss;
        rc = polar_iterations(c, L, ws, rp, nullptr, 0, &P);
        if (!rc) rc = sign_iterations(c, L, ws, rs, true, nullptr, 0, &Pi);
        hipError_t e = hipSuccess;
        for (size_t i = 0; !rc && e == hipSuccess && (i < sp.size() || i < ss.size()); ++i) {
            if (i < sp.size()) e = launch_stage(sp[i], side->st);
            if (e == hipSuccess && i < ss.size()) e = launch_stage(ss[i], ex.st);
        }
        if (!rc && e != hipSuccess) rc = hip_fail(e, "iterations");
    } else {
        if (ex.rec) {
            ex.cut[0] = ex.rec->size();
            ex.chains = L.fork;
        }
        if (op == PSVT_OP_SVT) rc = polar_iterations(c, L, ws, ex, nullptr, 0, &P);
        if (ex.rec) ex.cut[1] = ex.rec->size();
        if (!rc) rc = sign_iterations(c, L, ws, ex, true, nullptr, 0, &Pi);
        if (ex.rec) ex.cut[2] = ex.rec->size();
    }
    if (side) {
        // joined on failure too: after an error the caller may free ws as
        // soon as its own stream is done, so no side-stream work may remain
        HIP_TRY(hipEventRecord(side->join, side->st), "join");
        HIP_TRY(hipStreamWaitEvent(ex.st, side->join, 0), "join");
    }
    if (rc) return rc;
    if ((rc = final_product(L, ws, P, tau, Pi, Y, ldy, ex))) return rc;
    return status_stages(c, L, ws, ex, Pi, L.ldS, true, Y, m, n, ldy);
}

// single: a stand-alone call that may fork P's iterations to the calling
// thread's side stream (creating it on first use); false keeps every launch
// on the caller's stream and creates nothing.
int svt_like(int op, const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy,
             void *ws, size_t ws_bytes, const psvt_config *cfg, void *stream, bool single = true) {
    g_last_error.clear();
    Cfg c;
    int rc = read_cfg(cfg, c);
    if (rc) return rc;
    if ((rc = check_matrix(A, m, n, lda, "A"))) return rc;
    if ((rc = check_matrix(Y, m, n, ldy, "Y"))) return rc;
    if (!(tau >= 0.0) || !isfinite(tau)) return fail(PSVT_EINVAL, "tau must be finite and >= 0");
    if (m == 0 || n == 0) return PSVT_OK;
    Layout L = make_layout(op, m, n, c, single);
    if ((rc = check_ws(ws, ws_bytes, L))) return rc;
    if (overlaps(Y, span_bytes(m, n, ldy), A, span_bytes(m, n, lda)) ||
        overlaps(Y, span_bytes(m, n, ldy), ws, L.total) || overlaps(A, span_bytes(m, n, lda), ws, L.total))
        return fail(PSVT_EINVAL, "Y, A and ws must not overlap");
    if ((rc = check_warm(c, L, ws))) return rc;
    if ((c.flags & PSVT_FLAG_HFORM) && (op != PSVT_OP_SVT || c.n_fp8 > 0))
        return fail(PSVT_EINVAL, "PSVT_FLAG_HFORM applies to svt without FP8 iterations");
    if ((rc = check_device())) return rc;
    Exec ex;
    ex.st = (hipStream_t)stream;
    return plan_svt_like(op, A, m, n, lda, tau, Y, ldy, ws, L, c, ex);
}

}  // namespace

namespace psvt {

int set_error(int code, const char *msg) { return fail(code, "%s", msg); }

// svt on a given workspace with every launch on `stream` (no side stream):
// the entry point without allocation runs through here.
int svt_on_workspace(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy,
                     void *ws, size_t ws_bytes, const psvt_config *cfg, void *stream) {
    return svt_like(PSVT_OP_SVT, A, m, n, lda, tau, Y, ldy, ws, ws_bytes, cfg, stream, false);
}

// Workspace of svt on an m x n input without the side-stream fork; 0 on a
// bad config (the message is set).
int svt_workspace_unforked(int64_t m, int64_t n, const psvt_config *cfg, size_t *bytes) {
    Cfg c;
    int rc = read_cfg(cfg, c);
    if (rc) return rc;
    *bytes = (m > 0 && n > 0) ? make_layout(PSVT_OP_SVT, m, n, c, false).total : 0;
    return PSVT_OK;
}

// Stage list of one batch item or served request (records, launches
// nothing).  ws == NULL: only report the workspace size.  chains != NULL (a
// served request): the layout of a single call, whose P and S iterations may
// run concurrently for short sides <= 2048, and chains[0..2] = the plan's
// chain boundaries (the whole plan as one prefix when they may not).
int plan_request(int op, const psvt_batch_item &it, void *ws, const psvt_config *cfg, std::vector<Stage> &out,
                 size_t *ws_bytes, bool check_dev, size_t *chains) {
    psvt_config local{};
    if (cfg) local = *cfg;
    local.warm_pi = it.warm_pi;  // per item
    local.pi_out = it.pi_out;
    local.ld_pi = it.ld_pi;
    Cfg c;
    int rc = read_cfg(&local, c);
    if (rc) return rc;
    if (c.status)
        return fail(PSVT_EINVAL, "PSVT_FLAG_STATUS names one status word per call: not for batch items or served "
                                 "requests (psvt_svt_batched takes one per descriptor)");
    Layout L = make_layout(op, it.m, it.n, c, chains != nullptr);
    *ws_bytes = L.total;
    if (!ws) return PSVT_OK;
    if (check_dev && (rc = check_device())) return rc;
    Exec ex;
    ex.rec = &out;
    if ((rc = plan_svt_like(op, it.A, it.m, it.n, it.lda, it.tau, it.Y, it.ldy, ws, L, c, ex))) return rc;
    if (chains)
        for (int i = 0; i < 3; ++i) chains[i] = ex.chains ? ex.cut[i] : out.size();
    return PSVT_OK;
}

// Stage list of one matrix of a device-described batch (no fork; with
// PSVT_FLAG_STATUS the status stages write to `status`), and its layout.
int plan_batched_matrix(int op, const psvt_batch_item &it, void *ws, const psvt_config *cfg, uint32_t *status,
                        std::vector<Stage> &out, Layout *layout) {
    psvt_config local{};
    if (cfg) local = *cfg;
    local.flags &= ~PSVT_FLAG_PERSISTENT;  // how the batch runs, not how a matrix is planned
    if (local.warm_pi || local.pi_out)
        return fail(PSVT_EINVAL, "warm starts are per matrix: not in psvt_config for psvt_svt_batched");
    if (local.flags & PSVT_FLAG_STATUS) local.status = status;
    Cfg c;
    int rc = read_cfg(&local, c);
    if (rc) return rc;
    const Layout L = make_layout(op, it.m, it.n, c, false);
    if (layout) *layout = L;
    if (!ws) return PSVT_OK;
    Exec ex;
    ex.rec = &out;
    return plan_svt_like(op, it.A, it.m, it.n, it.lda, it.tau, it.Y, it.ldy, ws, L, c, ex);
}

// Side and low-precision layout flag of a batched call's configuration.
int batched_cfg(const psvt_config *cfg, int *side, int *lp, int *persistent) {
    psvt_config local{};
    if (cfg) local = *cfg;
    *persistent = (local.flags & PSVT_FLAG_PERSISTENT) != 0;
    local.flags &= ~(PSVT_FLAG_STATUS | PSVT_FLAG_PERSISTENT);
    Cfg c;
    int rc = read_cfg(&local, c);
    if (rc) return rc;
    *side = c.side;
    *lp = c.n_fp8 + c.n_bf16 > 0;
    return PSVT_OK;
}

int batch_plan_one(int op, const psvt_batch_item &it, void *ws, const psvt_config *cfg, std::vector<Stage> &out,
                   size_t *ws_bytes) {
    return plan_request(op, it, ws, cfg, out, ws_bytes, true, nullptr);
}

}  // namespace psvt

extern "C" {

int psvt_workspace_bytes(int op, int64_t m, int64_t n, const psvt_config *cfg, size_t *bytes) {
    g_last_error.clear();
    if (!bytes) return fail(PSVT_EINVAL, "bytes is NULL");
    if (op < PSVT_OP_SVT || op > PSVT_OP_RANK_R) return fail(PSVT_EINVAL, "unknown op %d", op);
    if (m < 0 || n < 0) return fail(PSVT_EINVAL, "negative size");
    if (op == PSVT_OP_POLAR_SYM && m != n) return fail(PSVT_EINVAL, "polar_sym needs m == n");
    Cfg c;
    int rc = read_cfg(cfg, c);
    if (rc) return rc;
    if (m == 0 || n == 0) {
        *bytes = 0;
        return PSVT_OK;
    }
    *bytes = make_layout(op, m, n, c, true).total;
    return PSVT_OK;
}

int psvt_svt(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy, void *ws,
             size_t ws_bytes, const psvt_config *cfg, void *stream) {
    return svt_like(PSVT_OP_SVT, A, m, n, lda, tau, Y, ldy, ws, ws_bytes, cfg, stream);
}

int psvt_rank_r(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy, void *ws,
                size_t ws_bytes, const psvt_config *cfg, void *stream) {
    return svt_like(PSVT_OP_RANK_R, A, m, n, lda, tau, Y, ldy, ws, ws_bytes, cfg, stream);
}

int psvt_polar(const float *A, int64_t m, int64_t n, int64_t lda, float *P, int64_t ldp, void *ws, size_t ws_bytes,
               const psvt_config *cfg, void *stream) {
    g_last_error.clear();
    Cfg c;
    int rc = read_cfg(cfg, c);
    if (rc) return rc;
    if (c.flags & (PSVT_FLAG_HFORM | PSVT_FLAG_GRAM))
        return fail(PSVT_EINVAL, "PSVT_FLAG_HFORM and PSVT_FLAG_GRAM apply to svt only");
    if ((rc = check_matrix(A, m, n, lda, "A"))) return rc;
    if ((rc = check_matrix(P, m, n, ldp, "P"))) return rc;
    if (m == 0 || n == 0) return PSVT_OK;
    Layout L = make_layout(PSVT_OP_POLAR, m, n, c);
    if ((rc = check_ws(ws, ws_bytes, L))) return rc;
    if (overlaps(P, span_bytes(m, n, ldp), A, span_bytes(m, n, lda)) ||
        overlaps(P, span_bytes(m, n, ldp), ws, L.total) || overlaps(A, span_bytes(m, n, lda), ws, L.total))
        return fail(PSVT_EINVAL, "P, A and ws must not overlap");
    if ((rc = check_device())) return rc;
    Exec ex;
    ex.st = (hipStream_t)stream;
    if ((rc = prelude(A, m, n, lda, 0.0, L, ws, ex, true, c.safety))) return rc;
    if ((rc = polar_iterations(c, L, ws, ex, P, ldp, nullptr))) return rc;
    return status_stages(c, L, ws, ex, nullptr, 0, false, P, m, n, ldp);
}

int psvt_polar_sym(const float *G, int64_t n, int64_t ldg, float *S, int64_t lds, void *ws, size_t ws_bytes,
                   const psvt_config *cfg, void *stream) {
    g_last_error.clear();
    Cfg c;
    int rc = read_cfg(cfg, c);
    if (rc) return rc;
    if (c.flags & (PSVT_FLAG_HFORM | PSVT_FLAG_GRAM))
        return fail(PSVT_EINVAL, "PSVT_FLAG_HFORM and PSVT_FLAG_GRAM apply to svt only");
    if (c.warm_pi || c.pi_out) return fail(PSVT_EINVAL, "warm starts apply to svt and rank_r");
    if ((rc = check_matrix(G, n, n, ldg, "G"))) return rc;
    if ((rc = check_matrix(S, n, n, lds, "S"))) return rc;
    if (n == 0) return PSVT_OK;
    Layout L = make_layout(PSVT_OP_POLAR_SYM, n, n, c);
    if ((rc = check_ws(ws, ws_bytes, L))) return rc;
    if (overlaps(S, span_bytes(n, n, lds), G, span_bytes(n, n, ldg)) ||
        overlaps(S, span_bytes(n, n, lds), ws, L.total) || overlaps(G, span_bytes(n, n, ldg), ws, L.total))
        return fail(PSVT_EINVAL, "S, G and ws must not overlap");
    if ((rc = check_device())) return rc;
    Exec ex;
    ex.st = (hipStream_t)stream;
    Scalars *sc = (Scalars *)at(ws, L.scal);
    double *part = (double *)at(ws, L.part);
    HIP_TRY(ex.norm(make_norm_op(G, n, n, ldg, part, sc, NORM_INPUT, 0.0), "norm of G"), "norm of G");
    HIP_TRY(ex.tile(make_symmetrize_scale(G, n, ldg, F(ws, L.H), L.ldS, sc), "symmetrize"), "symmetrize");
    HIP_TRY(syrk(F(ws, L.H), F(ws, L.H), L.ldS, nullptr, F(ws, L.R), L.ldS, n, 1.0f, -1, 0.0f, -1, 0.0f, sc, ex),
            "G^2");
    NormOp th = make_norm_op(F(ws, L.R), n, n, L.ldS, part, sc, NORM_THETA_S, 0.0);
    th.safety = c.safety;
    HIP_TRY(ex.norm(th, "theta_S"), "theta_S");
    if ((rc = sign_iterations(c, L, ws, ex, false, S, lds, nullptr))) return rc;
    return status_stages(c, L, ws, ex, S, lds, false, S, n, n, lds);
}

int psvt_gemm_nt(int dtype, const void *A, int64_t lda, const void *B, int64_t ldb, const float *D, int64_t ldd,
                 float *C, int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta, int sym,
                 void *stream) {
    g_last_error.clear();
    if (dtype < 0 || dtype > 3) return fail(PSVT_EINVAL, "bad dtype %d", dtype);
    if (M < 0 || N < 0 || K < 0) return fail(PSVT_EINVAL, "negative size");
    if (M == 0 || N == 0) return PSVT_OK;
    if (M > (1LL << 30) || N > (1LL << 30) || K > (1LL << 30)) return fail(PSVT_EINVAL, "size too large");
    if (!C) return fail(PSVT_EINVAL, "C is NULL");
    if (K > 0 && (!A || !B)) return fail(PSVT_EINVAL, "A or B is NULL");
    if (ldc < N || (K > 0 && (lda < K || ldb < K)) || (D && ldd < N)) return fail(PSVT_EINVAL, "bad leading dimension");
    if (sym && M != N) return fail(PSVT_EINVAL, "sym needs M == N");
    const int esz = dtype == PSVT_DTYPE_F32 ? 4 : (dtype == PSVT_DTYPE_FP8 ? 1 : 2);
    auto al16 = [](const void *p, int64_t ldbytes) { return p == nullptr || (((uintptr_t)p & 15) == 0 && ldbytes % 16 == 0); };
    if (!al16(A, lda * esz) || !al16(B, ldb * esz) || !al16(C, ldc * 4) || !al16(D, ldd * 4))
        return fail(PSVT_EINVAL, "operands must be 16-byte aligned with 16-byte-multiple row strides");
    int rc = check_device();
    if (rc) return rc;
    GemmArgs g = gemm_defaults();
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.D = D;
    g.ldd = ldd;
    g.C = C;
    g.ldc = ldc;
    g.M = (int)M;
    g.N = (int)N;
    g.K = (int)K;
    g.alpha = alpha;
    g.beta = beta;
    g.sym = sym ? 1 : 0;
    g.a_plane = M * lda;  // split bf16: the lo plane follows the hi plane
    g.b_plane = N * ldb;
    HIP_TRY(launch_gemm(g, dtype, (hipStream_t)stream), "gemm");
    return PSVT_OK;
}

int psvt_convert(int dtype, const float *X, int64_t rows, int64_t cols, int64_t ldx, void *Y, int64_t ldy,
                 float scale, int transpose, void *stream) {
    g_last_error.clear();
    if (dtype < 0 || dtype > 3) return fail(PSVT_EINVAL, "bad dtype %d", dtype);
    if (rows < 0 || cols < 0) return fail(PSVT_EINVAL, "negative size");
    if (rows == 0 || cols == 0) return PSVT_OK;
    if (!X || !Y) return fail(PSVT_EINVAL, "NULL buffer");
    if (ldx < cols || ldy < (transpose ? rows : cols)) return fail(PSVT_EINVAL, "bad leading dimension");
    if (!isfinite(scale)) return fail(PSVT_EINVAL, "scale must be finite");
    int rc = check_device();
    if (rc) return rc;
    const int64_t plane = (transpose ? cols : rows) * ldy;  // split bf16: lo plane after the hi plane
    HIP_TRY(launch_convert(X, rows, cols, ldx, Y, ldy, dtype, scale, transpose ? 1 : 0, (hipStream_t)stream, nullptr,
                           -1, plane),
            "convert");
    return PSVT_OK;
}

int psvt_tune_force_tile(int tile) {
    if (tile < 0 || tile > 4) return fail(PSVT_EINVAL, "tile id %d outside 0..4", tile);
    tune_force_tile(tile);
    return PSVT_OK;
}

int psvt_tune_persistent_tiles(int on) {
    if (on != 0 && on != 1) return fail(PSVT_EINVAL, "on must be 0 or 1");
    tune_persistent_tiles(on);
    return PSVT_OK;
}

int psvt_tune_spin_limit(int64_t polls) {
    if (polls < 0 || polls > (1LL << 40)) return fail(PSVT_EINVAL, "spin limit %lld outside 0..2^40", (long long)polls);
    set_persist_spin_limit(polls);
    return PSVT_OK;
}

int psvt_tune_set(int dtype, int tile, int sym, double efficiency, double overhead_us) {
    if (tune_set_model(dtype, tile, sym, (float)efficiency, (float)overhead_us) != 0)
        return fail(PSVT_EINVAL, "bad tuning entry %d %d %d %g %g", dtype, tile, sym, efficiency, overhead_us);
    return PSVT_OK;
}

int psvt_tune_load(const char *path) {
    if (!path) return fail(PSVT_EINVAL, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(PSVT_EINVAL, "cannot open %s", path);
    struct Entry {
        int type, id, sym;
        double e, o;
    } ent[64];
    char line[256];
    int n = 0, lineno = 0;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        char *hash = strchr(line, '#');
        if (hash) *hash = 0;
        Entry e;
        char extra[8];
        const int got = sscanf(line, "%d %d %d %lf %lf %7s", &e.type, &e.id, &e.sym, &e.e, &e.o, extra);
        if (got <= 0) continue;  // blank or comment
        if (got != 5 || e.type < 0 || e.type > 3 || e.id < 1 || e.id > 4 || (e.sym != 0 && e.sym != 1) ||
            !(e.e > 0.0 && e.e <= 1.0) || !(e.o >= 0.0 && e.o < 1e6) || n >= 64) {
            fclose(f);
            return fail(PSVT_EINVAL, "%s:%d: expected 'dtype id sym efficiency overhead_us'", path, lineno);
        }
        ent[n++] = e;
    }
    fclose(f);
    for (int i = 0; i < n; ++i) tune_set_model(ent[i].type, ent[i].id, ent[i].sym, (float)ent[i].e, (float)ent[i].o);
    return PSVT_OK;
}

int psvt_tune_pick(int dtype, int64_t M, int64_t N, int64_t K, int sym) {
    if (dtype < 0 || dtype > 3) return fail(PSVT_EINVAL, "bad dtype %d", dtype);
    if (M <= 0 || N <= 0 || K < 0 || M > (1LL << 30) || N > (1LL << 30) || K > (1LL << 30))
        return fail(PSVT_EINVAL, "bad size");
    return tune_pick(dtype, (int)M, (int)N, (int)K, sym ? 1 : 0);
}

const char *psvt_strerror(int code) {
    switch (code) {
        case PSVT_OK: return "success";
        case PSVT_EINVAL: return "invalid argument";
        case PSVT_EWORKSPACE: return "workspace missing or too small";
        case PSVT_EUNSUPPORTED: return "unsupported device or option";
        case PSVT_EHIP: return "HIP runtime error";
        default: return "unknown error";
    }
}

const char *psvt_last_error(void) { return g_last_error.c_str(); }

const char *psvt_version(void) { return "psvt 0.1 (gfx950)"; }

}  // extern "C"
