// Univariate tables (Sect. 2.1): Gauss-Legendre rules, the weighted-quadrature
// point layout, basis values at every rule point, the univariate mass matrix
// and the weighted-quadrature weights of Eq. (5), one system per test function.
#include "form_body.hpp"

namespace iga {

// ----------------------------------------------------------- Gauss-Legendre
// Node i (ascending) of the n-point rule by Newton's method on the Legendre
// three-term recurrence, started from the asymptotic root estimate.
__global__ void k_gauss_table(double* __restrict__ gx, double* __restrict__ gw) {
    int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= gauss_off(IGA_MAX_GAUSS + 1)) return;
    int n = 1;
    while (gauss_off(n + 1) <= tid) ++n;
    int i = tid - gauss_off(n);
    double x = -cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    bool last = false;
    for (int it = 0; it < 60; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 1; k < n; ++k) {
            double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
            p0 = p1;
            p1 = p2;
        }
        dp = (n == 1) ? 1.0 : n * (x * p1 - p0) / (x * x - 1.0);
        if (last) break;            // dp at the converged node
        double dx = p1 / dp;
        x -= dx;
        if (fabs(dx) <= 1e-14) last = true;  // quadratic convergence: one more step is exact
        if (n == 1) break;
    }
    if (n == 1) dp = 1.0;
    gx[tid] = x;
    gw[tid] = 2.0 / ((1.0 - x * x) * dp * dp);
}

void launch_gauss_table(Plan& P, hipStream_t s) {
    int tot = gauss_off(IGA_MAX_GAUSS + 1);
    klaunch(P, "k_gauss_table", k_gauss_table, dim3((tot + 255) / 256), dim3(256), 0, s, P.gauss_x, P.gauss_w);
}

// ------------------------------------------------------- direction tables
// Both directions in one launch. Per direction the thread range covers the
// breakpoints and first-point offsets (N+1), the WQ points with their basis
// values and derivatives (Q; p+1 points in the first and last element, 2
// elsewhere, uniformly inside each element, never on a knot) and the (p+1)
// Gauss points of every element with theirs.
template <int P>
__device__ __forceinline__ void dir_table_entry(const DirDev& D, int t, const double* __restrict__ gx,
                                                const double* __restrict__ gw) {
    const int N = D.N;
    if (t <= N) {
        D.bp[t] = D.knots[P + t];
        D.pt0[t] = wq_pt0(t, N, P);
        return;
    }
    t -= N + 1;
    if (t < D.Q) {
        // element of point t: inverse of wq_pt0
        int e;
        if (N == 1 || t < P + 1) e = 0;
        else if (t >= D.Q - (P + 1)) e = N - 1;
        else e = 1 + (t - (P + 1)) / 2;
        const int ne = (e == 0 || e == N - 1) ? P + 1 : 2;
        const int k = t - wq_pt0(e, N, P) + 1;
        const double a = D.knots[P + e], b = D.knots[P + e + 1];
        const double x = a + (b - a) * k / (ne + 1);
        D.xq[t] = x;
        D.eq[t] = e;
        double Nv[P + 1], dN[P + 1];
        basis_eval_d<P>(D.knots, P + e, x, Nv, dN);
#pragma unroll
        for (int c = 0; c <= P; ++c) {
            D.Bq[(size_t)t * (P + 1) + c] = Nv[c];
            D.dBq[(size_t)t * (P + 1) + c] = dN[c];
        }
        return;
    }
    t -= D.Q;
    if (t < N * (P + 1)) {
        const int e = t / (P + 1), g = t % (P + 1);
        const double a = D.knots[P + e], b = D.knots[P + e + 1];
        const double x = a + (b - a) * (gx[gauss_off(P + 1) + g] + 1.0) * 0.5;
        D.xg[t] = x;
        D.wg[t] = gw[gauss_off(P + 1) + g] * (b - a) * 0.5;
        double Nv[P + 1], dN[P + 1];
        basis_eval_d<P>(D.knots, P + e, x, Nv, dN);
#pragma unroll
        for (int c = 0; c <= P; ++c) {
            D.Bg[(size_t)t * (P + 1) + c] = Nv[c];
            D.dBg[(size_t)t * (P + 1) + c] = dN[c];
        }
    }
}

__host__ __device__ inline int dir_table_count(const DirDev& D, int p) { return D.N + 1 + D.Q + D.N * (p + 1); }

template <int P>
__global__ void __launch_bounds__(256) k_dir_tables(DirDev D1, DirDev D2, const double* __restrict__ gx,
                                                    const double* __restrict__ gw) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n1 = dir_table_count(D1, P);
    if (t < n1) dir_table_entry<P>(D1, t, gx, gw);
    else if (t < n1 + dir_table_count(D2, P)) dir_table_entry<P>(D2, t - n1, gx, gw);
}

void launch_dir_tables(Plan& P, hipStream_t s) {
    const int n = dir_table_count(P.dir[0], P.p) + dir_table_count(P.dir[1], P.p);
    dim3 g((n + 255) / 256), b(256);
    switch (P.p) {
#define CASE(PP) \
    case PP: klaunch(P, "k_dir_tables<" #PP ">", k_dir_tables<PP>, g, b, 0, s, P.dir[0], P.dir[1], P.gauss_x, P.gauss_w); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

// ---------------------------------------------------------- WQ weights (5)
// One wavefront per test function i (both directions in one launch: blocks
// [0, n1) direction 1, then direction 2). The band of the univariate mass
// matrix, b_j = int B_j B_i (exact with p+1 Gauss points per element), is
// summed over the wavefront's (element, Gauss point) pairs. Lane l owns
// row l of A^T (point k0 + l of supp B_i), A[j][k] = B_j(x_k) for |j - i| <= p;
// the minimum-norm solution of A w = b (Householder QR of A^T) is checked
// by its residual, then written with the row's test-side factors
// WB[i][q][b] = w_q B_{i+b-p}(x_q).
template <int P>
__device__ __forceinline__ void wq_weights_body(const DirDev& D1, const DirDev& D2, const double* __restrict__ gx,
                                                const double* __restrict__ gw, int* __restrict__ status, int blk) {
    constexpr int M = 2 * P + 1;
    int i = blk;
    const bool second = i >= D1.n;
    const DirDev& D = second ? D2 : D1;
    if (second) i -= D1.n;
    if (i >= D.n) return;
    const int lane = threadIdx.x;
    const int elo = max(0, i - P), ehi = min(D.N - 1, i);
    const int k0 = wq_pt0(elo, D.N, P), q = wq_pt0(ehi + 1, D.N, P) - k0;
    const int jlo = max(0, i - P), jhi = min(D.n - 1, i + P);
    const int m = jhi - jlo + 1;

    // univariate mass band of row i
    double mom[M];
#pragma unroll
    for (int c = 0; c < M; ++c) mom[c] = 0.0;
    for (int pg = lane; pg < (ehi - elo + 1) * (P + 1); pg += 64) {
        const int e = elo + pg / (P + 1), g = pg % (P + 1);
        const double a = D.knots[P + e], b = D.knots[P + e + 1];
        const double x = a + (b - a) * (gx[gauss_off(P + 1) + g] + 1.0) * 0.5;
        const double w = gw[gauss_off(P + 1) + g] * (b - a) * 0.5;
        double Nv[P + 1];
        basis_eval<P>(D.knots, P + e, x, Nv);
        const double bi = w * Nv[i - e];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int j = i + c - P;
            if (j >= e && j <= e + P) mom[c] += bi * Nv[j - e];
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) mom[c] = wave_sum(mom[c]);
    if (lane < M) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c)
            if (c == lane) v = mom[c];
        D.M1[(size_t)i * M + lane] = v;
    }

    double a[M], a0[M];
#pragma unroll
    for (int c = 0; c < M; ++c) a[c] = 0.0;
    int e_l = 0;
    if (lane < q) {
        const int k = k0 + lane;
        e_l = D.eq[k];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int j = jlo + c;
            if (c < m && j >= e_l && j <= e_l + P) a[c] = D.Bq[(size_t)k * (P + 1) + (j - e_l)];
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) a0[c] = a[c];
    bool singular = false;
    const int off = jlo - i + P;  // band column of trial function jlo
    const double y = wave_min_norm<M>(a, q, m, [&](int c) {
        double v = 0.0;
#pragma unroll
        for (int cc = 0; cc < M; ++cc)
            if (cc == c + off) v = mom[cc];
        return v;
    }, singular);
    // residual of Eq. (5)
    double rmax = 0.0, bmax = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c >= m) break;
        const double r = wave_sum(a0[c] * y);
        double bc = 0.0;
#pragma unroll
        for (int cc = 0; cc < M; ++cc)
            if (cc == c + off) bc = mom[cc];
        rmax = fmax(rmax, fabs(r - bc));
        bmax = fmax(bmax, fabs(bc));
    }
    if (lane < D.qmax) {
        D.W[(size_t)i * D.qmax + lane] = y;
        if (lane < 2 * P + 2) D.WT[(size_t)lane * D.n + i] = (lane < q) ? y : 0.0;
        // WB row q = lane: w_q B_{i+b-p}(x_q), zero where B_{i+b-p} vanishes on the point's element
        double* wb = D.WB + ((size_t)i * D.qmax + lane) * M;
#pragma unroll
        for (int bb = 0; bb < M; ++bb) {
            const int j = i + bb - P;
            double v = 0.0;
            if (lane < q && j >= e_l && j <= e_l + P && j >= jlo && j <= jhi) {
#pragma unroll
                for (int c = 0; c < M; ++c)
                    if (c == j - jlo) v = y * a0[c];
            }
            wb[bb] = v;
            const int al = bb - (lane >> 1);  // the banded copy, rows contiguous (points of a regular row)
            if (lane < 2 * P + 2 && al >= 0 && al <= P) D.WBT[((size_t)lane * (P + 1) + al) * D.n + i] = v;
        }
    }
    if (lane == 0 && (singular || !(rmax <= 1e-12 * bmax))) atomicExch(status, IGA_E_SINGULAR_WEIGHTS);
}

template <int P>
__global__ void __launch_bounds__(64) k_wq_weights(DirDev D1, DirDev D2, const double* __restrict__ gx,
                                                   const double* __restrict__ gw, int* __restrict__ status) {
    wq_weights_body<P>(D1, D2, gx, gw, status, blockIdx.x);
}

// The weights of both directions and c = |det J| on the WQ grid in one launch:
// workgroups below nw solve one weight system each, the others take 64 grid
// points each. Both read only the univariate tables, and the weight systems
// (one wavefront each, two per CU) leave the GPU mostly idle, so the grid's
// coefficient runs in their shadow instead of after them.
template <int P>
__global__ void __launch_bounds__(64) k_weights_coef(DirDev D1, DirDev D2, const double* __restrict__ gx,
                                                     const double* __restrict__ gw, int* __restrict__ status, int nw,
                                                     CoefArgs C, int64_t t1) {
    if ((int)blockIdx.x < nw) {
        wq_weights_body<P>(D1, D2, gx, gw, status, blockIdx.x);
        return;
    }
    const int64_t t = (int64_t)(blockIdx.x - nw) * 64 + threadIdx.x;
    if (t < t1) coef_point<P>(C, t);
}

// Test-side factors of the weighted-quadrature rows, WB[i][q][b] =
// w_{k0(i)+q, i} B_{i+b-p}(x_{k0(i)+q}), zero where B_{i+b-p} vanishes.
__global__ void k_wb_table(DirDev D, int p) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int W = 2 * p + 1;
    if (t >= D.n * D.qmax * W) return;
    int i = t / (D.qmax * W), q = (t / W) % D.qmax, b = t % W;
    int k0 = D.pt0[max(0, i - p)], q_i = D.pt0[min(D.N - 1, i) + 1] - k0;
    double v = 0.0;
    if (q < q_i) {
        int k = k0 + q, loc = i + b - p - D.eq[k];
        if (loc >= 0 && loc <= p) v = D.W[(size_t)i * D.qmax + q] * D.Bq[(size_t)k * (p + 1) + loc];
    }
    D.WB[t] = v;
    if (b == 0 && q < 2 * p + 2) D.WT[(size_t)q * D.n + i] = (q < q_i) ? D.W[(size_t)i * D.qmax + q] : 0.0;
    const int al = b - (q >> 1);  // the banded copy, rows contiguous (points of a regular row)
    if (q < 2 * p + 2 && al >= 0 && al <= p) D.WBT[((size_t)q * (p + 1) + al) * D.n + i] = v;
}

void launch_wb_table(Plan& P, int d, hipStream_t s) {
    DirDev& D = P.dir[d];
    int n = D.n * D.qmax * (2 * P.p + 1);
    klaunch(P, "k_wb_table", k_wb_table, dim3((n + 255) / 256), dim3(256), 0, s, D, P.p);
}

void launch_weights_coef(Plan& P, const iga_coeff& c, hipStream_t s, bool with_points) {
    CoefArgs C = coef_args(P, c);
    if (with_points) C.xy = P.pts_xy;
    const int nw = P.dir[0].n + P.dir[1].n;
    const int64_t t1 = C.nq;
    dim3 g((unsigned)(nw + (t1 + 63) / 64)), b(64);
    switch (P.p) {
#define CASE(PP)                                                                                                 \
    case PP:                                                                                                     \
        klaunch(P, "k_weights_coef<" #PP ">", k_weights_coef<PP>, g, b, 0, s, P.dir[0], P.dir[1], P.gauss_x,      \
                P.gauss_w, P.status, nw, C, t1);                                                                  \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

void launch_wq_weights(Plan& P, hipStream_t s) {
    dim3 g(P.dir[0].n + P.dir[1].n), b(64);
    switch (P.p) {
#define CASE(PP)                                                                                                 \
    case PP:                                                                                                     \
        klaunch(P, "k_wq_weights<" #PP ">", k_wq_weights<PP>, g, b, 0, s, P.dir[0], P.dir[1], P.gauss_x, P.gauss_w,  \
                P.status);                                                                                        \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

}  // namespace iga
