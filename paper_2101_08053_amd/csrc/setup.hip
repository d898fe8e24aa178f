// Univariate tables (Sect. 2.1): Gauss-Legendre rules, the weighted-quadrature
// point layout, basis values at every rule point, the univariate mass matrix
// and the weighted-quadrature weights of Eq. (5), one system per test function.
#include "plan.hpp"

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
    hipLaunchKernelGGL(k_gauss_table, dim3((tot + 255) / 256), dim3(256), 0, s, P.gauss_x, P.gauss_w);
}

// ------------------------------------------------------- WQ point layout
// p+1 points in the first and last element, 2 elsewhere, uniformly inside
// each element (never on a knot).
__global__ void k_layout(DirDev D, int p) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > D.N) return;
    D.bp[e] = D.knots[p + e];
    if (e == D.N) {
        D.pt0[D.N] = wq_pt0(D.N, D.N, p);
        return;
    }
    int ne = (e == 0 || e == D.N - 1) ? p + 1 : 2;
    int off = wq_pt0(e, D.N, p);
    D.pt0[e] = off;
    double a = D.knots[p + e], b = D.knots[p + e + 1];
    for (int k = 1; k <= ne; ++k) {
        D.xq[off + k - 1] = a + (b - a) * k / (ne + 1);
        D.eq[off + k - 1] = e;
    }
}

__global__ void k_basis_points(DirDev D, int p) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= D.Q) return;
    int e = D.eq[k];
    double N[IGA_MAXP + 1], dN[IGA_MAXP + 1];
    basis_eval_rt(D.knots, p, p + e, D.xq[k], N, dN);
    for (int a = 0; a <= p; ++a) {
        D.Bq[k * (p + 1) + a] = N[a];
        D.dBq[k * (p + 1) + a] = dN[a];
    }
}

__global__ void k_gauss_dir(DirDev D, int p, const double* __restrict__ gx, const double* __restrict__ gw) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int ng = p + 1;
    if (t >= D.N * ng) return;
    int e = t / ng, g = t % ng;
    double a = D.knots[p + e], b = D.knots[p + e + 1];
    double x = a + (b - a) * (gx[gauss_off(ng) + g] + 1.0) * 0.5;
    D.xg[t] = x;
    D.wg[t] = gw[gauss_off(ng) + g] * (b - a) * 0.5;
    double N[IGA_MAXP + 1], dN[IGA_MAXP + 1];
    basis_eval_rt(D.knots, p, p + e, x, N, dN);
    for (int c = 0; c <= p; ++c) {
        D.Bg[t * ng + c] = N[c];
        D.dBg[t * ng + c] = dN[c];
    }
}

// Univariate mass band M1[i][j-i+p] = int B_i B_j, exact with p+1 Gauss points per element.
__global__ void k_mass1d(DirDev D, int p) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int w = 2 * p + 1;
    if (t >= D.n * w) return;
    int i = t / w, j = i + t % w - p;
    double s = 0.0;
    if (j >= 0 && j < D.n) {
        int elo = max(max(i, j) - p, 0), ehi = min(min(i, j), D.N - 1);
        for (int e = elo; e <= ehi; ++e)
            for (int g = 0; g <= p; ++g) {
                int r = (e * (p + 1) + g) * (p + 1);
                s += D.wg[e * (p + 1) + g] * D.Bg[r + i - e] * D.Bg[r + j - e];
            }
    }
    D.M1[t] = s;
}

void launch_dir_tables(Plan& P, int d, hipStream_t s) {
    DirDev& D = P.dir[d];
    int p = P.p;
    hipLaunchKernelGGL(k_layout, dim3((D.N + 1 + 127) / 128), dim3(128), 0, s, D, p);
    hipLaunchKernelGGL(k_basis_points, dim3((D.Q + 127) / 128), dim3(128), 0, s, D, p);
    hipLaunchKernelGGL(k_gauss_dir, dim3((D.N * (p + 1) + 127) / 128), dim3(128), 0, s, D, p, P.gauss_x,
                       P.gauss_w);
    hipLaunchKernelGGL(k_mass1d, dim3((D.n * (2 * p + 1) + 127) / 128), dim3(128), 0, s, D, p);
}

// ---------------------------------------------------------- WQ weights (5)
// One wavefront per test function i. Lane l owns row l of A^T (point
// k0 + l of supp B_i); A[j][k] = B_j(x_k) for the trial functions j with
// |j - i| <= p. Householder QR of A^T = Q R gives the minimum-norm solution
// w = Q R^{-T} b of A w = b, b_j = int B_j B_i.
template <int P>
__global__ void __launch_bounds__(64) k_wq_weights(DirDev D, int* __restrict__ status) {
    constexpr int M = 2 * P + 1;
    int i = blockIdx.x;
    if (i >= D.n) return;
    int lane = threadIdx.x;
    int elo = max(0, i - P), ehi = min(D.N - 1, i);
    int k0 = D.pt0[elo], q = D.pt0[ehi + 1] - k0;
    int jlo = max(0, i - P), jhi = min(D.n - 1, i + P);
    int m = jhi - jlo + 1;

    double a[M];
#pragma unroll
    for (int c = 0; c < M; ++c) a[c] = 0.0;
    if (lane < q) {
        int k = k0 + lane, e = D.eq[k];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            int j = jlo + c;
            if (c < m && j >= e && j <= e + P) a[c] = D.Bq[k * (P + 1) + (j - e)];
        }
    }
    bool singular = false;
    double y = wave_min_norm<M>(a, q, m, [&](int c) { return D.M1[i * M + (jlo + c - i + P)]; }, singular);
    // residual of Eq. (5)
    double rmax = 0.0, bmax = 0.0;
    {
        int k = k0 + lane, e = (lane < q) ? D.eq[k] : 0;
        for (int c = 0; c < m; ++c) {
            int j = jlo + c;
            double ajk = (lane < q && j >= e && j <= e + P) ? D.Bq[k * (P + 1) + (j - e)] : 0.0;
            double r = wave_sum(ajk * y);
            double bc = D.M1[i * M + (j - i + P)];
            rmax = fmax(rmax, fabs(r - bc));
            bmax = fmax(bmax, fabs(bc));
        }
    }
    if (lane < D.qmax) D.W[(size_t)i * D.qmax + lane] = y;
    if (lane == 0 && (singular || !(rmax <= 1e-12 * bmax))) atomicExch(status, IGA_E_SINGULAR_WEIGHTS);
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
}

void launch_wb_table(Plan& P, int d, hipStream_t s) {
    DirDev& D = P.dir[d];
    int n = D.n * D.qmax * (2 * P.p + 1);
    hipLaunchKernelGGL(k_wb_table, dim3((n + 255) / 256), dim3(256), 0, s, D, P.p);
}

void launch_wq_weights(Plan& P, int d, hipStream_t s) {
    DirDev& D = P.dir[d];
    dim3 g(D.n), b(64);
    switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_wq_weights<PP>, g, b, 0, s, D, P.status); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
    launch_wb_table(P, d, s);
}

}  // namespace iga
