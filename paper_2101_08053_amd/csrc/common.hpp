// Shared device helpers of the gfx950 library: error plumbing, B-spline
// evaluation, Gauss-Legendre tables and scans. Host and device code of the
// library only; nothing here is shared with the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/iga_trim.h"

#define IGA_MAXP 8
#define IGA_MAX_GAUSS 64  // largest Gauss-Legendre rule kept in the table

namespace iga {

void set_error(const std::string& msg);

struct Error {
    int code;
    std::string msg;
};

#define HIPX(expr)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::iga::Error{IGA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define IGA_REQUIRE(cond, code, msg)                    \
    do {                                                \
        if (!(cond)) throw ::iga::Error{(code), (msg)}; \
    } while (0)

// Offset of the n-point rule in the packed Gauss table (rules 1..IGA_MAX_GAUSS).
__host__ __device__ inline int gauss_off(int n) { return n * (n - 1) / 2; }

// First weighted-quadrature point of element e in one direction (layout of
// the WQ points: p+1 points in the first and the last element, 2 in every
// other one); wq_pt0(N, N, p) is the number of points Q.
__host__ __device__ inline int wq_pt0(int e, int N, int p) {
    if (e <= 0) return 0;
    if (e >= N) return (N == 1) ? p + 1 : 2 * (p + 1) + 2 * (N - 2);
    return (p + 1) + 2 * (e - 1);
}

// -------------------------------------------------------------------------
// B-spline values on one element by the triangular Cox-de Boor scheme.
// span = index of the knot at the element's left end (p + e for open knot
// vectors with simple interior knots). N[0..p] receives B_{span-p..span}(x).
// -------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void basis_eval(const double* __restrict__ knots, int span, double x, double* N) {
    double left[P + 1], right[P + 1];
    N[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        left[j] = x - knots[span + 1 - j];
        right[j] = knots[span + j] - x;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

// The triangular scheme's denominators right[r+1] + left[j-r] do not depend
// on x: knots[span+r+1] - knots[span+1-j+r]. basis_rec<P> tabulates their
// reciprocals for one span (index j(j-1)/2 + r, j = 1..P, r < j) so that many
// points of one element are evaluated without divisions.
template <int P>
__device__ __forceinline__ double basis_rec(const double* __restrict__ knots, int span, int idx) {
    int j = 1;
    while (j * (j + 1) / 2 <= idx) ++j;
    const int r = idx - j * (j - 1) / 2;
    return 1.0 / (knots[span + r + 1] - knots[span + 1 - j + r]);
}

template <int P>
__device__ __forceinline__ void basis_eval_rec(const double* __restrict__ knots, int span,
                                               const double* __restrict__ rinv, double x, double* N) {
    double left[P + 1], right[P + 1];
    N[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        left[j] = x - knots[span + 1 - j];
        right[j] = knots[span + j] - x;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            const double tmp = N[r] * rinv[j * (j - 1) / 2 + r];
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

// Values and first derivatives from the span's reciprocal table (as
// basis_eval_rec): dN_a = P (N^{P-1}_{a-1} / (t_{i+P} - t_i) - N^{P-1}_a /
// (t_{i+P+1} - t_{i+1})), i = span - P + a, whose reciprocals are the
// table's last level.
template <int P>
__device__ __forceinline__ void basis_eval_rec_d(const double* __restrict__ knots, int span,
                                                 const double* __restrict__ rinv, double x, double* N, double* dN) {
    double left[P + 1], right[P + 1], low[P + 1];
    N[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        if (j == P) {
#pragma unroll
            for (int r = 0; r < P; ++r) low[r] = N[r];
        }
        left[j] = x - knots[span + 1 - j];
        right[j] = knots[span + j] - x;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            const double tmp = N[r] * rinv[j * (j - 1) / 2 + r];
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
    constexpr int b = P * (P - 1) / 2;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double v = 0.0;
        if (a >= 1) v += P * (low[a - 1] * rinv[b + a - 1]);
        if (a <= P - 1) v -= P * (low[a] * rinv[b + a]);
        dN[a] = v;
    }
}

// Values and first derivatives, compile-time degree.
template <int P>
__device__ __forceinline__ void basis_eval_d(const double* __restrict__ knots, int span, double x, double* N,
                                             double* dN) {
    double left[P + 1], right[P + 1], low[P + 1];
    N[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        if (j == P) {
#pragma unroll
            for (int r = 0; r < P; ++r) low[r] = N[r];
        }
        left[j] = x - knots[span + 1 - j];
        right[j] = knots[span + j] - x;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        int i = span - P + a;
        double v = 0.0;
        if (a >= 1) v += P * low[a - 1] / (knots[i + P] - knots[i]);
        if (a <= P - 1) v -= P * low[a] / (knots[i + P + 1] - knots[i + 1]);
        dN[a] = v;
    }
}

// Runtime-degree variant (p <= IGA_MAXP); also returns first derivatives if dN != nullptr.
__device__ __forceinline__ void basis_eval_rt(const double* __restrict__ knots, int p, int span, double x,
                                              double* N, double* dN) {
    double left[IGA_MAXP + 1], right[IGA_MAXP + 1];
    double low[IGA_MAXP + 1];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        if (j == p) {
            for (int r = 0; r < p; ++r) low[r] = N[r];
        }
        left[j] = x - knots[span + 1 - j];
        right[j] = knots[span + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
    if (dN) {
        if (p == 0) {
            dN[0] = 0.0;
            return;
        }
        // derivative of B_{span-p+a, p}: p/(k[i+p]-k[i]) low_i - p/(k[i+p+1]-k[i+1]) low_{i+1}
        for (int a = 0; a <= p; ++a) {
            int i = span - p + a;
            double v = 0.0;
            if (a >= 1) v += p * low[a - 1] / (knots[i + p] - knots[i]);
            if (a <= p - 1) v -= p * low[a] / (knots[i + p + 1] - knots[i + 1]);
            dN[a] = v;
        }
    }
}

// ------------------------------------------------------------------ scans
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; returns the block total.
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int& total) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int nw = blockDim.x >> 6;
    int inc = wave_incl_scan(v, lane);
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int t = (lane < nw) ? sh[lane] : 0;
        int ti = wave_incl_scan(t, lane);
        if (lane < nw) sh[lane] = ti - t;
        if (lane == nw - 1) sh[nw] = ti;
    }
    __syncthreads();
    int res = inc - v + sh[wid];
    total = sh[nw];
    __syncthreads();
    return res;
}

// -------------------------------------------------------------------------
// Minimum 2-norm solution of a small under-determined system A w = b on one
// wavefront (Eq. (5) and its refined variants). Lane l holds row l of A^T
// (one quadrature point) in a[0..m); lanes >= q hold zeros. Householder QR
// of A^T = Q R, then w = Q R^{-T} b. bcol(c) returns b[c] (uniform across
// the wave). On return y is the weight of the lane's point (0 for lanes >=
// q); singular is set if a pivot of R vanishes; the result is checked by the
// caller.
// -------------------------------------------------------------------------
// A double moved across lanes of a row of 16 by a DPP control (the two
// 32-bit halves); no LDS round trip.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes, the same value in every lane (all lanes active):
// pairs inside quads, quads inside half rows, half rows inside rows of 16
// (DPP moves), then the four row sums read as scalars.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_move<0x141>(v);  // row_half_mirror: the other quad of the half row
    v += dpp_move<0x140>(v);  // row_mirror: the other half of the row
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Integer sum over the 64 lanes (every lane active), by the same moves.
__device__ __forceinline__ int wave_sum_i(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

// -------------------------------------------------------------------------
// Minimum 2-norm solution of a small under-determined system A w = b on one
// quad of lanes (four lanes per system, sixteen systems per wavefront): row
// k of A^T (point k) sits in lane k % 4 of the quad as A[k / 4][0..m), the
// quad's lanes hold b (for c < m) alike. Householder QR of A^T (q x m) with
// reductions inside the quad (DPP moves), R^T z = b solved as the columns
// come, y = Q [z; 0]. On return y[i] is the weight of point 4 i + (lane % 4)
// (0 past q); A holds R and the reflectors; singular is set if a pivot
// vanishes (the caller checks the residual). Every lane of the quad must run
// it (quads may differ in q and m).
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_move<0xB1>(v);  // lane ^ 1
    v += dpp_move<0x4E>(v);  // lane ^ 2
    return v;
}
// Lane j's value in every lane of the quad (j is a constant after unrolling: one DPP move).
__device__ __forceinline__ double quad_bcast(double v, int j) {
    switch (j & 3) {
        case 0: return dpp_move<0x00>(v);
        case 1: return dpp_move<0x55>(v);
        case 2: return dpp_move<0xAA>(v);
        default: return dpp_move<0xFF>(v);
    }
}

template <int M, int RPL>
__device__ __forceinline__ void quad_min_norm(double (&A)[RPL][M], int q, int m, const double (&b)[M],
                                              double (&y)[RPL], bool& singular) {
    const int g = threadIdx.x & 3;
    double tauv[M], z[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        tauv[c] = 0.0;
        z[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c < m) {
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int k = 4 * i + g;
                part += (k >= c && k < q) ? A[i][c] * A[i][c] : 0.0;
            }
            const double nrm2 = quad_sum(part);
            const double xc = quad_bcast(A[c >> 2][c], c);
            double alpha = 0.0, tau = 0.0, inv = 0.0;
            if (nrm2 > 0.0) {
                alpha = (xc >= 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
                const double uc = xc - alpha;
                tau = -uc / alpha;
                inv = 1.0 / uc;
            } else {
                singular = true;
            }
            double vv[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int k = 4 * i + g;
                vv[i] = (k == c) ? 1.0 : ((k > c && k < q) ? A[i][c] * inv : 0.0);
                A[i][c] = (k == c) ? alpha : ((k > c && k < q) ? vv[i] : A[i][c]);
            }
            tauv[c] = tau;
#pragma unroll
            for (int c2 = c + 1; c2 < M; ++c2) {
                if (c2 < m) {
                    double dp = 0.0;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) dp += vv[i] * A[i][c2];
                    const double f = tau * quad_sum(dp);
#pragma unroll
                    for (int i = 0; i < RPL; ++i) A[i][c2] -= f * vv[i];
                }
            }
            // z_c = (b_c - sum_{i<c} R_ic z_i) / R_cc
            double acc = b[c];
#pragma unroll
            for (int i = 0; i < c; ++i) acc -= quad_bcast(A[i >> 2][c], i) * z[i];
            z[c] = (alpha != 0.0) ? acc / alpha : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        double v = 0.0;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg)
            if (4 * i + gg < M) v = (g == gg) ? z[(4 * i + gg < M) ? 4 * i + gg : 0] : v;
        y[i] = v;
    }
#pragma unroll
    for (int j = M - 1; j >= 0; --j) {
        if (j < m) {
            double vv[RPL], dp = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int k = 4 * i + g;
                vv[i] = (k == j) ? 1.0 : ((k > j && k < q) ? A[i][j] : 0.0);
                dp += vv[i] * y[i];
            }
            const double f = tauv[j] * quad_sum(dp);
#pragma unroll
            for (int i = 0; i < RPL; ++i) y[i] -= f * vv[i];
        }
    }
}

template <int M, typename BCol>
__device__ __forceinline__ double wave_min_norm(double (&a)[M], int q, int m, BCol bcol, bool& singular) {
    const int lane = threadIdx.x & 63;
    double v[M], vn[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        v[c] = 0.0;
        vn[c] = 0.0;
    }
    singular = false;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c >= m) break;
        double x = (lane >= c && lane < q) ? a[c] : 0.0;
        double nrm2 = wave_sum(x * x);
        double xc = read_lane(a[c], c);
        double alpha = (xc >= 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        double vl = (lane == c) ? x - alpha : x;
        double vv = 2.0 * (nrm2 - alpha * xc);
        v[c] = vl;
        vn[c] = vv;
        if (vv > 0.0) {
#pragma unroll
            for (int j = c + 1; j < M; ++j) {
                if (j >= m) break;
                double d = wave_sum(vl * ((lane >= c) ? a[j] : 0.0));
                if (lane >= c) a[j] -= 2.0 * vl * d / vv;
            }
        }
        if (lane == c) a[c] = (vv > 0.0) ? alpha : xc;
        else if (lane > c) a[c] = 0.0;
        double rcc = read_lane(a[c], c);
        if (!(fabs(rcc) > 0.0)) singular = true;
    }
    // forward substitution R^T z = b (R[k][c] sits in lane k, column c)
    double zl = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c >= m) break;
        double bc = bcol(c);
        double sacc = wave_sum((lane < c) ? a[c] * zl : 0.0);
        double rcc = read_lane(a[c], c);
        double zc = (bc - sacc) / rcc;
        if (lane == c) zl = zc;
    }
    // w = H_0 ... H_{m-1} [z; 0]
    double y = (lane < m) ? zl : 0.0;
#pragma unroll
    for (int c = M - 1; c >= 0; --c) {
        if (c >= m || !(vn[c] > 0.0)) continue;
        double d = wave_sum(v[c] * y);
        y -= 2.0 * v[c] * d / vn[c];
    }
    return (lane < q) ? y : 0.0;
}

}  // namespace iga
