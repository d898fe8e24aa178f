// L2 projection (Sect. 4.2): right-hand side b_i = row i's own rule applied
// to g c, then Jacobi-preconditioned CG on A = (M + M^T)/2 in the band layout.
// The rule of each row is the one its mass-matrix row uses: weighted
// quadrature for interior rows, element Gauss + cut rule for rows formed
// element-wise. Reductions are block partials summed in a fixed order by one
// workgroup, so every run is bitwise reproducible.
#include <cmath>
#include <vector>

#include "plan.hpp"

namespace iga {

// g at a parameter point: target of the projection at the physical point
__device__ __forceinline__ double target_eval(const iga_target& g, double x, double y) {
    if (g.kind == IGA_TARGET_SINCOS) return sin(g.w[0] * x + g.w[1]) * cos(g.w[2] * y + g.w[3]);
    // monomial
    return pow(x, (double)(int)g.w[0]) * pow(y, (double)(int)g.w[1]);
}

// physical coordinates of a point of element (e1, e2) from its local basis values
__device__ __forceinline__ void map_local(const double* __restrict__ cp, int n1, int p, int e1, int e2,
                                          const double* B1, const double* B2, double& X, double& Y) {
    X = 0.0;
    Y = 0.0;
    for (int a2 = 0; a2 <= p; ++a2) {
        const double* row = cp + 2 * ((size_t)(e2 + a2) * n1 + e1);
        double sx = 0, sy = 0;
        for (int a1 = 0; a1 <= p; ++a1) {
            sx += B1[a1] * row[2 * a1];
            sy += B1[a1] * row[2 * a1 + 1];
        }
        X += B2[a2] * sx;
        Y += B2[a2] * sy;
    }
}

struct GcArgs {
    DirDev d1, d2;
    int p;
    iga_target g;
    const double* geom;   // control points or nullptr (identity map)
    int n1;
    const double* gpts;   // AT_POINTS values or nullptr
    // coefficient
    int c_const;
    double c_value;
    const double* c_wq;
    const double* c_band;
    const double* c_cut;
    // point sets
    const int* band_list;
    int n_band;
    const int* cut_list;
    const int* node_el;
    const double *nx, *ny;
    int n_nodes;
    double* out;          // n_points values of g c, iga_plan_points order
};

__global__ void k_gc(GcArgs A) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int p = A.p;
    int nq = A.d1.Q * A.d2.Q;
    int ng = (p + 1) * (p + 1);
    int nb = A.n_band * ng;
    if (t >= nq + nb + A.n_nodes) return;
    double x, y, c;
    int e1, e2;
    double B1[IGA_MAXP + 1], B2[IGA_MAXP + 1];
    if (t < nq) {
        int k1 = t % A.d1.Q, k2 = t / A.d1.Q;
        x = A.d1.xq[k1];
        y = A.d2.xq[k2];
        e1 = A.d1.eq[k1];
        e2 = A.d2.eq[k2];
        for (int a = 0; a <= p; ++a) {
            B1[a] = A.d1.Bq[k1 * (p + 1) + a];
            B2[a] = A.d2.Bq[k2 * (p + 1) + a];
        }
        c = A.c_const ? A.c_value : A.c_wq[t];
    } else if (t < nq + nb) {
        int u = t - nq, b = u / ng, g = u % ng, g1 = g % (p + 1), g2 = g / (p + 1);
        int e = A.band_list[b];
        e1 = e % A.d1.N;
        e2 = e / A.d1.N;
        x = A.d1.xg[e1 * (p + 1) + g1];
        y = A.d2.xg[e2 * (p + 1) + g2];
        for (int a = 0; a <= p; ++a) {
            B1[a] = A.d1.Bg[(e1 * (p + 1) + g1) * (p + 1) + a];
            B2[a] = A.d2.Bg[(e2 * (p + 1) + g2) * (p + 1) + a];
        }
        c = A.c_const ? A.c_value : A.c_band[u];
    } else {
        int n = t - nq - nb;
        int e = A.cut_list[A.node_el[n]];
        e1 = e % A.d1.N;
        e2 = e / A.d1.N;
        x = A.nx[n];
        y = A.ny[n];
        basis_eval_rt(A.d1.knots, p, p + e1, x, B1, nullptr);
        basis_eval_rt(A.d2.knots, p, p + e2, y, B2, nullptr);
        c = A.c_const ? A.c_value : A.c_cut[n];
    }
    double gv;
    if (A.gpts) {
        gv = A.gpts[t];
    } else {
        double X = x, Y = y;
        if (A.geom) map_local(A.geom, A.n1, p, e1, e2, B1, B2, X, Y);
        gv = target_eval(A.g, X, Y);
    }
    A.out[t] = gv * c;
}

// b for interior rows (weighted quadrature) -- one thread per row.
__global__ void k_rhs_wq(DirDev D1, DirDev D2, int p, const int8_t* __restrict__ fcls, int all_active,
                         const int* __restrict__ fn_of, int n_act, const double* __restrict__ gc_wq,
                         double* __restrict__ b) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_act) return;
    int f = fn_of[r];
    int8_t cls = fcls[f];
    if (!(all_active || cls == FN_INTERIOR)) return;
    int i1 = f % D1.n, i2 = f / D1.n;
    int k1 = D1.pt0[max(0, i1 - p)], q1 = D1.pt0[min(D1.N - 1, i1) + 1] - k1;
    int k2 = D2.pt0[max(0, i2 - p)], q2 = D2.pt0[min(D2.N - 1, i2) + 1] - k2;
    double s = 0.0;
    for (int a = 0; a < q1; ++a) {
        double in = 0.0;
        for (int c = 0; c < q2; ++c) in += D2.W[(size_t)i2 * D2.qmax + c] * gc_wq[(size_t)(k2 + c) * D1.Q + k1 + a];
        s += D1.W[(size_t)i1 * D1.qmax + a] * in;
    }
    b[r] = s;
}

// Element vectors F_e[l] = sum_g w_g (g c)_g B_l(x_g) of band (Gauss) and cut elements.
template <int P>
__global__ void __launch_bounds__(64) k_rhs_elem(DirDev D1, DirDev D2, const int* __restrict__ band_list, int n_band,
                                                 const int* __restrict__ cut_list, const int* __restrict__ node_off,
                                                 const double* __restrict__ nx, const double* __restrict__ ny,
                                                 const double* __restrict__ nw, const double* __restrict__ gc,
                                                 int gc_band_off, int gc_cut_off, double* __restrict__ F) {
    constexpr int L = (P + 1) * (P + 1);
    __shared__ double sPhi[64][L];
    __shared__ double sT[64];
    int re = blockIdx.x;
    bool is_cut = re >= n_band;
    int e = is_cut ? cut_list[re - n_band] : band_list[re];
    int e1 = e % D1.N, e2 = e / D1.N;
    int nb, ne;
    if (is_cut) {
        nb = node_off[re - n_band];
        ne = node_off[re - n_band + 1];
    } else {
        nb = 0;
        ne = L;
    }
    double acc[(L + 63) / 64];
#pragma unroll
    for (int k = 0; k < (L + 63) / 64; ++k) acc[k] = 0.0;
    for (int base = nb; base < ne; base += 64) {
        __syncthreads();
        int n = base + threadIdx.x;
        if (n < ne) {
            double B1[P + 1], B2[P + 1], w, gcv;
            if (is_cut) {
                basis_eval<P>(D1.knots, P + e1, nx[n], B1);
                basis_eval<P>(D2.knots, P + e2, ny[n], B2);
                w = nw[n];
                gcv = gc[gc_cut_off + n];
            } else {
                int g1 = n % (P + 1), g2 = n / (P + 1);
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    B1[a] = D1.Bg[(e1 * (P + 1) + g1) * (P + 1) + a];
                    B2[a] = D2.Bg[(e2 * (P + 1) + g2) * (P + 1) + a];
                }
                w = D1.wg[e1 * (P + 1) + g1] * D2.wg[e2 * (P + 1) + g2];
                gcv = gc[gc_band_off + re * L + n];
            }
#pragma unroll
            for (int a2 = 0; a2 <= P; ++a2)
#pragma unroll
                for (int a1 = 0; a1 <= P; ++a1) sPhi[threadIdx.x][a2 * (P + 1) + a1] = B1[a1] * B2[a2];
            sT[threadIdx.x] = w * gcv;
        }
        __syncthreads();
        int cnt = min(64, ne - base);
#pragma unroll
        for (int k = 0; k < (L + 63) / 64; ++k) {
            int l = threadIdx.x + 64 * k;
            if (l < L)
                for (int m = 0; m < cnt; ++m) acc[k] += sT[m] * sPhi[m][l];
        }
    }
#pragma unroll
    for (int k = 0; k < (L + 63) / 64; ++k) {
        int l = threadIdx.x + 64 * k;
        if (l < L) F[(size_t)re * L + l] = acc[k];
    }
}

// b for element-formed rows: gather F_e over the support elements.
__global__ void k_rhs_gather(int p, int N1, int N2, int n1, const int* __restrict__ rows, int n_rows,
                             const int* __restrict__ fn_of, const int8_t* __restrict__ ecls,
                             const int* __restrict__ band_id, const int* __restrict__ cut_id, int n_band,
                             const double* __restrict__ F, double* __restrict__ b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows) return;
    int r = rows[t], f = fn_of[r], i1 = f % n1, i2 = f / n1;
    int L = (p + 1) * (p + 1);
    double s = 0.0;
    for (int e2 = max(0, i2 - p); e2 <= min(N2 - 1, i2); ++e2)
        for (int e1 = max(0, i1 - p); e1 <= min(N1 - 1, i1); ++e1) {
            int e = e2 * N1 + e1;
            int8_t c = ecls[e];
            if (c == EL_OUTSIDE) continue;
            int re = (c == EL_CUT) ? n_band + cut_id[e] : band_id[e];
            s += F[(size_t)re * L + (i2 - e2) * (p + 1) + (i1 - e1)];
        }
    b[r] = s;
}

// ------------------------------------------------------------------- PCG
// A = (M + M^T)/2: slot (a, b) of row r pairs with slot (-a, -b) of its column's row.
__global__ void k_symmetrize(int p, int n1, const int* __restrict__ fn_of, const int* __restrict__ act_of,
                             int n2, int n_act, const double* __restrict__ M, double* __restrict__ A) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int W = 2 * p + 1;
    if (t >= (int64_t)W * W * n_act) return;
    int s = (int)(t / n_act), r = (int)(t % n_act);
    int a = s / W - p, b = s % W - p;
    int f = fn_of[r], j1 = f % n1 + a, j2 = f / n1 + b;
    double v = 0.0;
    if (j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2) {
        int c = act_of[j2 * n1 + j1];
        if (c >= 0) {
            int sm = (W * W - 1) - s;  // slot of (-a, -b)
            v = 0.5 * (M[(size_t)s * n_act + r] + M[(size_t)sm * n_act + c]);
        }
    }
    A[t] = v;
}

constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    __syncthreads();
    return s;  // valid in thread 0
}

struct SpArgs {
    int p, n1, n2, n_act;
    const int* fn_of;
    const int* act_of;
    const double* A;
    const int* cols;  // [(2p+1)^2][n_act] compact column of each slot, -1 if none (PCG iterations)
};

// Compact column of every slot of the band (once per solve).
__global__ void k_cols(SpArgs S, int* __restrict__ cols) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = 2 * S.p + 1;
    if (t >= (int64_t)W * W * S.n_act) return;
    const int sl = (int)(t / S.n_act), r = (int)(t % S.n_act);
    const int f = S.fn_of[r], j1 = f % S.n1 + sl / W - S.p, j2 = f / S.n1 + sl % W - S.p;
    cols[t] = (j1 >= 0 && j1 < S.n1 && j2 >= 0 && j2 < S.n2) ? S.act_of[j2 * S.n1 + j1] : -1;
}

// Row r of A x from the column table, slots in the order (b outer, a inner),
// every load of the row issued before the sums.
template <int P>
__device__ __forceinline__ double spmv_row_cols(const SpArgs& S, const double* __restrict__ x, int r) {
    constexpr int W = 2 * P + 1;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < W; ++b) {
        int c[W];
        double v[W], xv[W];
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const size_t o = (size_t)(a * W + b) * S.n_act + r;
            c[a] = S.cols[o];
            v[a] = S.A[o];
        }
#pragma unroll
        for (int a = 0; a < W; ++a) xv[a] = x[max(c[a], 0)];
#pragma unroll
        for (int a = 0; a < W; ++a)
            if (c[a] >= 0) s += v[a] * xv[a];
    }
    return s;
}

// Sum of a kernel's block partials, the same in every block (thread 0 holds it).
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, int nv, int v, double* sh);

__device__ __forceinline__ double spmv_row(const SpArgs& S, const double* __restrict__ x, int r) {
    int W = 2 * S.p + 1;
    int f = S.fn_of[r], i1 = f % S.n1, i2 = f / S.n1;
    double s = 0.0;
    for (int b = -S.p; b <= S.p; ++b) {
        int j2 = i2 + b;
        if (j2 < 0 || j2 >= S.n2) continue;
        for (int a = -S.p; a <= S.p; ++a) {
            int j1 = i1 + a;
            if (j1 < 0 || j1 >= S.n1) continue;
            int c = S.act_of[j2 * S.n1 + j1];
            if (c < 0) continue;
            s += S.A[(size_t)((a + S.p) * W + (b + S.p)) * S.n_act + r] * x[c];
        }
    }
    return s;
}

// scal layout: 0 rz (initial), 2 rr, 3 bb, 6 / 7 rz of even / odd iterations
// r = b - A x, z = r/d, p = z; partials of (r.z), (r.r), (b.b)
__global__ void __launch_bounds__(kRedThreads) k_cg_init(SpArgs S, const double* __restrict__ bvec,
                                                         const double* __restrict__ x, double* __restrict__ rv,
                                                         double* __restrict__ zv, double* __restrict__ pv,
                                                         double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0, rr = 0, bb = 0;
    if (r < S.n_act) {
        int W = 2 * S.p + 1;
        double d = S.A[(size_t)(S.p * W + S.p) * S.n_act + r];
        double res = bvec[r] - spmv_row(S, x, r);
        double z = res / d;
        rv[r] = res;
        zv[r] = z;
        pv[r] = z;
        rz = res * z;
        rr = res * res;
        bb = bvec[r] * bvec[r];
    }
    double s0 = block_sum(rz, sh), s1 = block_sum(rr, sh), s2 = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0;
        part[3 * blockIdx.x + 1] = s1;
        part[3 * blockIdx.x + 2] = s2;
    }
}

// The initial (r.z), (r.r), (b.b) from the block partials (one workgroup).
__global__ void __launch_bounds__(kRedThreads) k_reduce(const double* __restrict__ part, int nblk, int nv,
                                                        double* __restrict__ scal) {
    __shared__ double sh[kRedThreads / 64];
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += part[nv * k + v];
        double tot = block_sum(s, sh);
        if (threadIdx.x == 0) {
            scal[v == 0 ? 0 : (v == 1 ? 2 : 3)] = tot;
            if (v == 0) scal[6] = tot;  // (r.z) of the first iteration
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, int nv, int v, double* sh) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += part[nv * k + v];
    return block_sum(s, sh);
}

// The iteration in three launches: every block of the update and direction
// kernels sums the previous kernel's block partials itself (same order in
// every block, so the same scalars), instead of a one-block reduction launch
// in between. (r.z) alternates between scal[par] and scal[1 - par], so the
// direction kernel's block 0 can store the new value while other blocks
// still read the old one.
template <int P>
__global__ void __launch_bounds__(kRedThreads) k_cg_spmv_c(SpArgs S, const double* __restrict__ pv,
                                                           double* __restrict__ qv, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    double pq = 0.0;
    if (r < S.n_act) {
        double q = spmv_row_cols<P>(S, pv, r);
        qv[r] = q;
        pq = pv[r] * q;
    }
    double s = block_sum(pq, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) k_cg_update_c(SpArgs S, double* __restrict__ scal, int par, int nblk,
                                                             const double* __restrict__ part_pq, double* __restrict__ x,
                                                             double* __restrict__ rv, double* __restrict__ zv,
                                                             const double* __restrict__ pv,
                                                             const double* __restrict__ qv, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_alpha;
    const double pq = sum_partials(part_pq, nblk, 1, 0, sh);
    // the host reads convergence every few iterations, so iterations may run on after
    // the residual has vanished: then p.q = 0 and the step is zero, not 0/0
    if (threadIdx.x == 0) s_alpha = (pq != 0.0) ? scal[6 + par] / pq : 0.0;
    __syncthreads();
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0, rr = 0;
    if (r < S.n_act) {
        double alpha = s_alpha;
        int W = 2 * S.p + 1;
        double d = S.A[(size_t)(S.p * W + S.p) * S.n_act + r];
        x[r] += alpha * pv[r];
        double res = rv[r] - alpha * qv[r];
        double z = res / d;
        rv[r] = res;
        zv[r] = z;
        rz = res * z;
        rr = res * res;
    }
    double s0 = block_sum(rz, sh), s1 = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0;
        part[2 * blockIdx.x + 1] = s1;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_cg_dir_c(int n, double* __restrict__ scal, int par, int nblk,
                                                          const double* __restrict__ part,
                                                          const double* __restrict__ zv, double* __restrict__ pv) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_beta;
    const double rz = sum_partials(part, nblk, 2, 0, sh);
    const double rr = sum_partials(part, nblk, 2, 1, sh);
    if (threadIdx.x == 0) {
        s_beta = (scal[6 + par] != 0.0) ? rz / scal[6 + par] : 0.0;  // a vanished residual keeps p = z
        if (blockIdx.x == 0) {
            scal[6 + (1 - par)] = rz;
            scal[2] = rr;
        }
    }
    __syncthreads();
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) pv[r] = zv[r] + s_beta * pv[r];
}

}  // namespace iga

using namespace iga;

namespace iga {

void compute_gc(Plan& P, const iga_coeff& c, const iga_target& g, double* out, hipStream_t s) {
    CoefView cv = coef_view(P, c);
    GcArgs A;
    A.d1 = P.dir[0];
    A.d2 = P.dir[1];
    A.p = P.p;
    A.g = g;
    A.geom = (c.kind == IGA_COEF_GEOM_DETJ) ? c.geom_cp : nullptr;
    A.n1 = P.n1;
    A.gpts = (g.kind == IGA_TARGET_AT_POINTS) ? g.g_points : nullptr;
    A.c_const = cv.is_const;
    A.c_value = cv.value;
    A.c_wq = cv.wq;
    A.c_band = cv.band;
    A.c_cut = cv.cut;
    A.band_list = P.band_list;
    A.n_band = (int)P.n_band;
    A.cut_list = P.cut_list;
    A.node_el = P.node_el;
    A.nx = P.node_x;
    A.ny = P.node_y;
    A.n_nodes = (int)P.n_nodes;
    A.out = out;
    int64_t n = P.n_points;
    hipLaunchKernelGGL(k_gc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A);
}

void rhs(Plan& P, const iga_coeff& c, const iga_target& g, double* b, hipStream_t s) {
    SolveWork& W = P.sw;
    size_t L = (size_t)(P.p + 1) * (P.p + 1);
    if (!W.gc) W.gc = P.alloc<double>(P.n_points);
    if (!W.F) W.F = P.alloc<double>(std::max<int64_t>(1, P.n_band + P.n_cut_el) * L);
    if (c.kind == IGA_COEF_GEOM_DETJ) launch_coef(P, c, s);
    compute_gc(P, c, g, W.gc, s);
    int n = (int)P.n_act;
    hipLaunchKernelGGL(k_rhs_wq, dim3((n + 255) / 256), dim3(256), 0, s, P.dir[0], P.dir[1], P.p, P.fcls,
                       (int)(P.method == IGA_NAIVE_WQ), P.fn_of, n, W.gc, b);
    if (P.method == IGA_NAIVE_WQ || P.n_form_rows == 0) return;
    int nre = (int)(P.n_band + P.n_cut_el);
    int nq = P.dir[0].Q * P.dir[1].Q;
    if (nre > 0) {
        switch (P.p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        hipLaunchKernelGGL(k_rhs_elem<PP>, dim3(nre), dim3(64), 0, s, P.dir[0], P.dir[1], P.band_list,          \
                           (int)P.n_band, P.cut_list, P.node_off, P.node_x, P.node_y, P.node_w, W.gc, nq,        \
                           (int)(nq + P.n_band * L), W.F);                                                        \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
    }
    int nr = (int)P.n_form_rows;
    hipLaunchKernelGGL(k_rhs_gather, dim3((nr + 255) / 256), dim3(256), 0, s, P.p, P.N1, P.N2, P.n1, P.form_rows,
                       nr, P.fn_of, P.ecls, P.band_id, P.cut_id, (int)P.n_band, W.F, b);
}
}  // namespace iga

#define API_BEGIN try {
#define API_END                       \
    }                                 \
    catch (const Error& e) {          \
        set_error(e.msg);             \
        return e.code;                \
    }                                 \
    catch (const std::exception& e) { \
        set_error(e.what());          \
        return IGA_E_INVALID;         \
    }                                 \
    return IGA_OK;

extern "C" {

int iga_trim_rhs(iga_plan* plan, const iga_coeff* c, const iga_target* g, double* b, void* stream) {
    API_BEGIN
    Plan* P = plan;
    IGA_REQUIRE(P && c && g && b, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(g->kind >= IGA_TARGET_SINCOS && g->kind <= IGA_TARGET_AT_POINTS, IGA_E_UNSUPPORTED, "target kind");
    IGA_REQUIRE(g->kind != IGA_TARGET_AT_POINTS || g->g_points, IGA_E_INVALID, "target values missing");
    IGA_REQUIRE(P->method == IGA_HYBRID_GAUSS || P->method == IGA_GAUSS_REF, IGA_E_UNSUPPORTED,
                "right-hand side is built for hybrid Gauss and the reference rules");
    rhs(*P, *c, *g, b, (hipStream_t)stream);
    HIPX(hipGetLastError());
    API_END
}

int iga_trim_l2_project(iga_plan* plan, const iga_coeff* c, const double* vals, const iga_target* g, double rtol,
                        int32_t maxit, double* u, iga_solve_info* info, void* stream) {
    API_BEGIN
    Plan* P = plan;
    IGA_REQUIRE(P && c && vals && g && u, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(rtol > 0 && maxit > 0, IGA_E_INVALID, "rtol and maxit must be positive");
    IGA_REQUIRE(P->method == IGA_HYBRID_GAUSS || P->method == IGA_GAUSS_REF, IGA_E_UNSUPPORTED,
                "right-hand side is built for hybrid Gauss and the reference rules");
    hipStream_t s = (hipStream_t)stream;
    SolveWork& W = P->sw;
    int n = (int)P->n_act;
    int W2 = (2 * P->p + 1) * (2 * P->p + 1);
    int nblk = (n + kRedThreads - 1) / kRedThreads;
    if (!W.A) {
        W.A = P->alloc<double>((size_t)W2 * n);
        W.r = P->alloc<double>(n);
        W.z = P->alloc<double>(n);
        W.pv = P->alloc<double>(n);
        W.q = P->alloc<double>(n);
        W.b = P->alloc<double>(n);
        W.part = P->alloc<double>(3 * (size_t)nblk);
        W.scal = P->alloc<double>(8);
        W.cols = P->alloc<int>((size_t)W2 * n);
        HIPX(hipHostMalloc((void**)&W.h_scal, 8 * sizeof(double), hipHostMallocDefault));
    }
    rhs(*P, *c, *g, W.b, s);
    int64_t tot = (int64_t)W2 * n;
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, P->p, P->n1, P->fn_of,
                       P->act_of, P->n2, n, vals, W.A);
    SpArgs S{P->p, P->n1, P->n2, n, P->fn_of, P->act_of, W.A, nullptr};
    hipLaunchKernelGGL(k_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S, W.cols);
    S.cols = W.cols;
    hipLaunchKernelGGL(k_cg_init, dim3(nblk), dim3(kRedThreads), 0, s, S, W.b, u, W.r, W.z, W.pv, W.part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, W.part, nblk, 3, W.scal);
    auto read = [&]() {
        HIPX(hipMemcpyAsync(W.h_scal, W.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
    };
    read();
    double bnorm = std::sqrt(W.h_scal[3]);
    double rel = (bnorm > 0) ? std::sqrt(W.h_scal[2]) / bnorm : 0.0;
    int it = 0;
    const int chunk = 16;
    bool conv = rel <= rtol;
    while (!conv && it < maxit) {
        int m = std::min(chunk, maxit - it);
        for (int k = 0; k < m; ++k) {
            const int par = (it + k) & 1;
            double* part2 = W.part + nblk;
            switch (P->p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_cg_spmv_c<PP>, dim3(nblk), dim3(kRedThreads), 0, s, S, W.pv, W.q, W.part); break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
            }
            hipLaunchKernelGGL(k_cg_update_c, dim3(nblk), dim3(kRedThreads), 0, s, S, W.scal, par, nblk,
                               (const double*)W.part, u, W.r, W.z, (const double*)W.pv, (const double*)W.q, part2);
            hipLaunchKernelGGL(k_cg_dir_c, dim3(nblk), dim3(kRedThreads), 0, s, n, W.scal, par, nblk,
                               (const double*)part2, (const double*)W.z, W.pv);
        }
        it += m;
        read();
        rel = (bnorm > 0) ? std::sqrt(W.h_scal[2]) / bnorm : 0.0;
        conv = rel <= rtol;
    }
    if (info) {
        info->iterations = it;
        info->converged = conv;
        info->rel_residual = rel;
    }
    HIPX(hipGetLastError());
    if (!conv) {
        set_error("PCG did not reach the tolerance");
        return IGA_E_NOCONV;
    }
    API_END
}

}  // extern "C"
