// Matrix-free product y = M(c) u and its adjoint.
//
// With c given at every rule point, the rows of M are
//   y_i = sum_k w_hat_{k,i} c_k U_k,   U_k = sum_j B_j(x_k) u_j,
// where w_hat_{k,i} is row i's test-side weight at point k: w1 w2 for rows
// formed by weighted quadrature (interior rows), w_g B_i(x_g) for rows formed
// element-wise (hybrid Gauss cut rows: element Gauss points and cut nodes).
// For L(u, c) with dL/dy = r the adjoint is
//   du_j = sum_k B_j(x_k) c_k R_k,   dc_k = U_k R_k,   R_k = sum_i w_hat_{k,i} r_i.
// Basis values come from the per-direction tables or are recomputed at cut
// nodes; U and R are never stored per row.
#include <mutex>
#include <string>

#include "plan.hpp"

namespace iga {

struct MfArgs {
    DirDev d1, d2;
    int p, n1, n2, N1, N2;
    int method;
    const int8_t* fcls;
    const int8_t* ecls;
    const int* act_of;
    const int* fn_of;
    const int* band_list;
    const int* cut_list;
    const int* band_id;
    const int* cut_id;
    const int* node_off;
    const double *nx, *ny, *nw;
    int n_band, n_cut, n_act;
    const double* c;   // n_points, plan point order
    int nq, nb;        // point offsets: band points start at nq, cut nodes at nq + nb
    const double* WA;  // [Q1][p+1]: w1[e1(k1) + a][k1 - k0(e1(k1) + a)], 0 past the last function
    const double* BR;  // [4p+2][n1]: B_j1(x_{k0(j1) + q}), 0 past the row's points
};

__device__ __forceinline__ bool wq_row(const MfArgs& A, int8_t cls) {
    return A.method != IGA_GAUSS_REF && cls == FN_INTERIOR;
}

// The weighted-quadrature part as banded one-dimensional contractions (sum
// factorisation), fast index along xi_1:
//   V[j2][k1] = sum_a B1[k1][a] u(e1(k1) + a, j2)              (u on the xi_1 points; k_mf_v)
//   G[k2][k1] = c_k sum_a B2[k2][a] V[e2(k2) + a][k1]          (c U along grid row k2, in LDS; k_mf_gh)
//   H[k2][i1] = sum_q w1[i1][q] G[k2][k0(i1) + q]              (test rows along xi_1; k_mf_gh)
//   y(i1, i2) = sum_q w2[i2][q] H[k0(i2) + q][i1]              (interior rows; k_mf_y)
// and, transposed, for the adjoint
//   H[k2][i1] = sum_{i2 : k2 in supp} w2[i2][k2 - k0(i2)] r(i1, i2)                    (k_mf_hadj)
//   R[k2][k1] = sum_{i1 : k1 in supp} w1[i1][k1 - k0(i1)] H[k2][i1],  dc = U R, c R      (k_mf_rd, per row)
//   D[k2][j1] = sum_{k1 in supp j1} B1[k1][j1 - e1(k1)] c R[k2][k1]                    (k_mf_rd)
//   du(j1, j2) += sum_{k2 in supp j2} B2[k2][j2 - e2(k2)] D[k2][j1]                    (k_mf_gather)
// G, U, R and c R never leave their workgroup.
template <int P>
__global__ void __launch_bounds__(256) k_mf_v(MfArgs A, const double* __restrict__ u, double* __restrict__ V) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int Q1 = A.d1.Q;
    if (t >= (int64_t)A.n2 * Q1) return;
    const int k1 = (int)(t % Q1), j2 = (int)(t / Q1);
    const int e1 = A.d1.eq[k1];
    const int* act = A.act_of + (size_t)j2 * A.n1 + e1;
    int cid[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) cid[a] = act[a];
    double s = 0.0;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        const double uv = u[max(cid[a], 0)];
        s += A.d1.Bq[(size_t)k1 * (P + 1) + a] * (cid[a] >= 0 ? uv : 0.0);
    }
    V[t] = s;
}

template <int P>
__global__ void __launch_bounds__(256) k_mf_y(MfArgs A, const double* __restrict__ H, double* __restrict__ y) {
    constexpr int QM = 4 * P + 2;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int n1 = A.n1;
    if (t >= (int64_t)n1 * A.n2) return;
    if (!wq_row(A, A.fcls[t])) return;
    const int i1 = (int)(t % n1), i2 = (int)(t / n1);
    const int k0 = A.d2.pt0[max(0, i2 - P)], q2 = A.d2.pt0[min(A.N2 - 1, i2) + 1] - k0;
    const double* w = A.d2.W + (size_t)i2 * A.d2.qmax;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        if (q >= q2) break;
        s += w[q] * H[(size_t)(k0 + q) * n1 + i1];
    }
    y[A.act_of[t]] = s;
}

template <int P>
__global__ void __launch_bounds__(256) k_mf_hadj(MfArgs A, const double* __restrict__ r, double* __restrict__ H) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int n1 = A.n1;
    if (t >= (int64_t)A.d2.Q * n1) return;
    const int i1 = (int)(t % n1), k2 = (int)(t / n1);
    const int e2 = A.d2.eq[k2];
    double s = 0.0;
#pragma unroll
    for (int b = 0; b <= P; ++b) {
        const int i2 = e2 + b;
        if (i2 >= A.n2) break;
        const int f = i2 * n1 + i1;
        const int cid = A.act_of[f];
        const bool use = cid >= 0 && wq_row(A, A.fcls[f]);
        const double rv = r[max(cid, 0)];
        const double w2 = A.d2.W[(size_t)i2 * A.d2.qmax + (k2 - A.d2.pt0[max(0, i2 - P)])];
        s += use ? w2 * rv : 0.0;
    }
    H[t] = s;
}

// Per-point and per-function views of the xi_1 tables that the grid-row
// kernels read at every row: the test weights that meet at a point (WA) and
// a function's basis values at its support points (BR, functions contiguous).
template <int P>
__global__ void __launch_bounds__(256) k_mf_tables(DirDev D, int n1, double* __restrict__ WA, double* __restrict__ BR) {
    constexpr int QM = 4 * P + 2;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < D.Q * (P + 1)) {
        const int k1 = t / (P + 1), a = t % (P + 1), i1 = D.eq[k1] + a;
        WA[t] = (i1 < n1) ? D.W[(size_t)i1 * D.qmax + (k1 - D.pt0[max(0, i1 - P)])] : 0.0;
    }
    if (t < QM * n1) {
        const int q = t / n1, j1 = t % n1;
        const int k0 = D.pt0[max(0, j1 - P)], q1 = D.pt0[min(D.N - 1, j1) + 1] - k0;
        BR[t] = (q < q1) ? D.Bq[(size_t)(k0 + q) * (P + 1) + (j1 - D.eq[k0 + q])] : 0.0;
    }
}

// Forward, one workgroup per grid row k2: G = c U along the row in LDS, then
// the row's xi_1 test sums H[k2][i1] (G never leaves the workgroup). Each
// thread takes four points (or functions) at a time, loads first.
template <int P>
__global__ void __launch_bounds__(256) k_mf_gh(MfArgs A, const double* __restrict__ V, double* __restrict__ H) {
    extern __shared__ double sG[];  // Q1
    constexpr int QM = 4 * P + 2, NB = 4;
    const int k2 = blockIdx.x, Q1 = A.d1.Q, n1 = A.n1;
    const int e2 = A.d2.eq[k2];
    double b2[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) b2[a] = A.d2.Bq[(size_t)k2 * (P + 1) + a];
    const double* Vr = V + (size_t)e2 * Q1;
    const double* cr = A.c + (size_t)k2 * Q1;
#pragma unroll 1
    for (int kb = threadIdx.x; kb < Q1; kb += 256 * NB) {
        double v[NB][P + 1], cv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k1 = min(kb + 256 * j, Q1 - 1);
#pragma unroll
            for (int a = 0; a <= P; ++a) v[j][a] = Vr[(size_t)a * Q1 + k1];
            cv[j] = cr[k1];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) s += b2[a] * v[j][a];
            if (kb + 256 * j < Q1) sG[kb + 256 * j] = cv[j] * s;
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int i1 = threadIdx.x; i1 < n1; i1 += 256) {
        const int k0 = A.d1.pt0[max(0, i1 - P)], q1 = A.d1.pt0[min(A.N1 - 1, i1) + 1] - k0;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            if (q >= q1) break;
            const double w = (q < 2 * P + 2) ? A.d1.WT[(size_t)q * n1 + i1] : A.d1.W[(size_t)i1 * A.d1.qmax + q];
            s += w * sG[k0 + q];
        }
        H[(size_t)k2 * n1 + i1] = s;
    }
}

// Adjoint, one workgroup per grid row k2: the row's w2-weighted residual sums
// (H, staged in LDS), R along the row, dc = U R with U from V, c R in LDS,
// then the row's xi_1 basis sums D[k2][j1], written over H's row.
template <int P>
__global__ void __launch_bounds__(256) k_mf_rd(MfArgs A, const double* __restrict__ V, double* __restrict__ HD,
                                               double* __restrict__ dc) {
    extern __shared__ double sm[];  // n1 (H row), then Q1 (c R)
    constexpr int QM = 4 * P + 2, NB = 4;
    const int k2 = blockIdx.x, Q1 = A.d1.Q, n1 = A.n1;
    double* sH = sm;
    double* sCR = sm + n1;
    for (int i1 = threadIdx.x; i1 < n1; i1 += 256) sH[i1] = HD[(size_t)k2 * n1 + i1];
    const int e2 = A.d2.eq[k2];
    double b2[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) b2[a] = A.d2.Bq[(size_t)k2 * (P + 1) + a];
    const double* Vr = V + (size_t)e2 * Q1;
    const double* cr = A.c + (size_t)k2 * Q1;
    __syncthreads();
#pragma unroll 1
    for (int kb = threadIdx.x; kb < Q1; kb += 256 * NB) {
        double v[NB][P + 1], wa[NB][P + 1], cv[NB];
        int e1[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k1 = min(kb + 256 * j, Q1 - 1);
            e1[j] = A.d1.eq[k1];
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                v[j][a] = Vr[(size_t)a * Q1 + k1];
                wa[j][a] = A.WA[(size_t)k1 * (P + 1) + a];
            }
            cv[j] = cr[k1];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double U = 0.0, R = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                U += b2[a] * v[j][a];
                R += wa[j][a] * sH[min(e1[j] + a, n1 - 1)];  // 0 weight past the last function
            }
            const int k1 = kb + 256 * j;
            if (k1 < Q1) {
                dc[(size_t)k2 * Q1 + k1] = U * R;
                sCR[k1] = cv[j] * R;
            }
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int j1 = threadIdx.x; j1 < n1; j1 += 256) {
        const int k0 = A.d1.pt0[max(0, j1 - P)];
        double br[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) br[q] = A.BR[(size_t)q * n1 + j1];
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q) s += br[q] * sCR[min(k0 + q, Q1 - 1)];  // 0 past the row's points
        HD[(size_t)k2 * n1 + j1] = s;
    }
}

// Element part: per band / cut element, forward Y_e[l] = sum_g w_g c_g U_g B_l(x_g),
// adjoint D_e[l] = sum_g c_g R_g B_l(x_g) with R_g = w_g sum_l B_l r_l over the
// element-formed rows, and dc_g = U_g R_g.
template <int P>
__global__ void __launch_bounds__(64) k_mf_elem(MfArgs A, const double* __restrict__ u, const double* __restrict__ r,
                                                double* __restrict__ Ye, double* __restrict__ dc) {
    constexpr int L = (P + 1) * (P + 1);
    constexpr int PER = (L + 63) / 64;
    __shared__ double sPhi[64][L];
    __shared__ double sT[64];
    __shared__ double sU[L], sR[L];
    int re = blockIdx.x;
    bool is_cut = re >= A.n_band;
    int e = is_cut ? A.cut_list[re - A.n_band] : A.band_list[re];
    int e1 = e % A.N1, e2 = e / A.N1;
    for (int l = threadIdx.x; l < L; l += 64) {
        int j1 = e1 + l % (P + 1), j2 = e2 + l / (P + 1);
        int f = j2 * A.n1 + j1;
        int cid = A.act_of[f];
        sU[l] = (cid >= 0) ? u[cid] : 0.0;
        // rows formed element-wise: cut rows (hybrid) or every row (reference)
        bool erow = cid >= 0 && !wq_row(A, A.fcls[f]);
        sR[l] = (r && erow) ? r[cid] : 0.0;
    }
    int nb, ne, pbase;
    if (is_cut) {
        nb = A.node_off[re - A.n_band];
        ne = A.node_off[re - A.n_band + 1];
        pbase = A.nq + A.nb;
    } else {
        nb = 0;
        ne = L;
        pbase = A.nq + re * L;
    }
    double acc[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) acc[k] = 0.0;
    for (int base = nb; base < ne; base += 64) {
        __syncthreads();
        int n = base + threadIdx.x;
        if (n < ne) {
            double B1[P + 1], B2[P + 1], w;
            if (is_cut) {
                basis_eval<P>(A.d1.knots, P + e1, A.nx[n], B1);
                basis_eval<P>(A.d2.knots, P + e2, A.ny[n], B2);
                w = A.nw[n];
            } else {
                int g1 = n % (P + 1), g2 = n / (P + 1);
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    B1[a] = A.d1.Bg[(e1 * (P + 1) + g1) * (P + 1) + a];
                    B2[a] = A.d2.Bg[(e2 * (P + 1) + g2) * (P + 1) + a];
                }
                w = A.d1.wg[e1 * (P + 1) + g1] * A.d2.wg[e2 * (P + 1) + g2];
            }
            double Ug = 0.0, Rg = 0.0;
#pragma unroll
            for (int a2 = 0; a2 <= P; ++a2)
#pragma unroll
                for (int a1 = 0; a1 <= P; ++a1) {
                    double phi = B1[a1] * B2[a2];
                    sPhi[threadIdx.x][a2 * (P + 1) + a1] = phi;
                    Ug += phi * sU[a2 * (P + 1) + a1];
                    Rg += phi * sR[a2 * (P + 1) + a1];
                }
            double cg = A.c[pbase + n];
            if (r) {
                Rg *= w;
                dc[pbase + n] = Ug * Rg;
                sT[threadIdx.x] = cg * Rg;
            } else {
                sT[threadIdx.x] = w * cg * Ug;
            }
        }
        __syncthreads();
        int cnt = min(64, ne - base);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            int l = threadIdx.x + 64 * k;
            if (l < L)
                for (int m = 0; m < cnt; ++m) acc[k] += sT[m] * sPhi[m][l];
        }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int l = threadIdx.x + 64 * k;
        if (l < L) Ye[(size_t)re * L + l] = acc[k];
    }
}

// Sum of the element vectors over the band / cut elements of supp B_j,
// for the rows formed element-wise (forward) or every active function (adjoint),
// plus (adjoint) the WQ-grid part sum_k B_j(x_k) CR_k from its xi_1 sums D.
__global__ void k_mf_gather(MfArgs A, const double* __restrict__ Ye, const double* __restrict__ CR,
                            double* __restrict__ out, int adjoint) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= A.n_act) return;
    int f = A.fn_of[r];
    int p = A.p;
    int8_t cls = A.fcls[f];
    if (!adjoint && wq_row(A, cls)) return;
    int i1 = f % A.n1, i2 = f / A.n1;
    int L = (p + 1) * (p + 1);
    double s = 0.0;
    for (int e2 = max(0, i2 - p); e2 <= min(A.N2 - 1, i2); ++e2)
        for (int e1 = max(0, i1 - p); e1 <= min(A.N1 - 1, i1); ++e1) {
            int e = e2 * A.N1 + e1;
            int8_t c = A.ecls[e];
            if (c == EL_OUTSIDE) continue;
            int re = (c == EL_CUT) ? A.n_band + A.cut_id[e] : A.band_id[e];
            if (re < 0) continue;  // inside element used by no element-formed row
            s += Ye[(size_t)re * L + (i2 - e2) * (p + 1) + (i1 - e1)];
        }
    if (adjoint && A.method != IGA_GAUSS_REF) {  // the grid part, sum_k2 B2 D[k2][i1]
        int k2 = A.d2.pt0[max(0, i2 - p)], q2 = A.d2.pt0[min(A.N2 - 1, i2) + 1] - k2;
        double g = 0.0;
        for (int b = 0; b < q2; ++b) {
            int kk2 = k2 + b, m2 = A.d2.eq[kk2];
            g += A.d2.Bq[kk2 * (p + 1) + (i2 - m2)] * CR[(size_t)kk2 * A.n1 + i1];
        }
        s += g;
    }
    out[r] = s;
}

static MfArgs mf_args(Plan& P, const double* c) {
    MfArgs A;
    A.d1 = P.dir[0];
    A.d2 = P.dir[1];
    A.p = P.p;
    A.n1 = P.n1;
    A.n2 = P.n2;
    A.N1 = P.N1;
    A.N2 = P.N2;
    A.method = P.method;
    A.fcls = P.fcls;
    A.ecls = P.ecls;
    A.act_of = P.act_of;
    A.fn_of = P.fn_of;
    A.band_list = P.band_list;
    A.cut_list = P.cut_list;
    A.band_id = P.band_id;
    A.cut_id = P.cut_id;
    A.node_off = P.node_off;
    A.nx = P.node_x;
    A.ny = P.node_y;
    A.nw = P.node_w;
    A.n_band = (int)P.n_band;
    A.n_cut = (int)P.n_cut_el;
    A.n_act = (int)P.n_act;
    A.c = c;
    A.nq = P.dir[0].Q * P.dir[1].Q;
    A.nb = (int)P.n_band * (P.p + 1) * (P.p + 1);
    A.WA = P.sw.WA;
    A.BR = P.sw.BR;
    return A;
}

// one grid row of xi_1 points and one row of functions in LDS
static void mf_check(const Plan& P) {
    IGA_REQUIRE(sizeof(double) * ((size_t)P.dir[0].Q + P.n1) <= 65536, IGA_E_UNSUPPORTED,
                "matrix-free product: more than 2700 elements along xi_1");
}

static void mf_buffers(Plan& P) {
    size_t L = (size_t)(P.p + 1) * (P.p + 1);
    mf_check(P);
    if (!P.sw.V) P.sw.V = P.alloc<double>((size_t)P.n2 * P.dir[0].Q);
    if (!P.sw.H) P.sw.H = P.alloc<double>((size_t)P.dir[1].Q * P.n1);
    if (!P.sw.Ue) P.sw.Ue = P.alloc<double>(std::max<int64_t>(1, P.n_band + P.n_cut_el) * L);
    if (!P.sw.WA) P.sw.WA = P.alloc<double>((size_t)P.dir[0].Q * (P.p + 1));
    if (!P.sw.BR) P.sw.BR = P.alloc<double>((size_t)(4 * P.p + 2) * P.n1);
}

static dim3 grid256(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

static void launch_elem(Plan& P, const MfArgs& A, const double* u, const double* r, double* Ye, double* dc,
                        hipStream_t s) {
    int nre = (int)(P.n_band + P.n_cut_el);
    if (nre == 0) return;
    switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_mf_elem<PP>, dim3(nre), dim3(64), 0, s, A, u, r, Ye, dc); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
}

template <int P>
static void launch_wq_forward(Plan& Pl, const MfArgs& A, const double* u, double* y, double* V, double* H,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_mf_v<P>, grid256((int64_t)Pl.n2 * A.d1.Q), dim3(256), 0, s, A, u, V);
    hipLaunchKernelGGL(k_mf_gh<P>, dim3(A.d2.Q), dim3(256), sizeof(double) * A.d1.Q, s, A, (const double*)V, H);
    hipLaunchKernelGGL(k_mf_y<P>, grid256((int64_t)Pl.n1 * Pl.n2), dim3(256), 0, s, A, (const double*)H, y);
}

template <int P>
static void launch_wq_adjoint(Plan& Pl, const MfArgs& A, const double* u, const double* r, double* dc,
                              hipStream_t s) {
    const int nt = std::max(A.d1.Q * (P + 1), (4 * P + 2) * Pl.n1);  // the weights may have been injected
    hipLaunchKernelGGL(k_mf_tables<P>, grid256(nt), dim3(256), 0, s, A.d1, Pl.n1, Pl.sw.WA, Pl.sw.BR);
    hipLaunchKernelGGL(k_mf_v<P>, grid256((int64_t)Pl.n2 * A.d1.Q), dim3(256), 0, s, A, u, Pl.sw.V);
    hipLaunchKernelGGL(k_mf_hadj<P>, grid256((int64_t)A.d2.Q * Pl.n1), dim3(256), 0, s, A, r, Pl.sw.H);
    hipLaunchKernelGGL(k_mf_rd<P>, dim3(A.d2.Q), dim3(256), sizeof(double) * (A.d1.Q + Pl.n1), s, A,
                       (const double*)Pl.sw.V, Pl.sw.H, dc);  // D over H
}

// The forward product with its three intermediate arrays given: V [n2][Q1],
// H [Q2][n1], Ue [n_band + n_cut][(p+1)^2]. Every entry of them is written
// before it is read, so they need no clearing.
// The element part (element vectors, then the rows formed element-wise) runs
// on the plan's second stream beside the weighted-quadrature part: the two
// write disjoint rows of y.
static void mf_apply_into(Plan& P, const double* c, const double* u, double* y, double* V, double* H, double* Ue,
                          hipStream_t s) {
    MfArgs A = mf_args(P, c);
    int n = (int)P.n_act;
    HIPX(hipEventRecord(P.ev_mf_fork, s));
    HIPX(hipStreamWaitEvent(P.aux, P.ev_mf_fork, 0));
    launch_elem(P, A, u, nullptr, Ue, nullptr, P.aux);
    hipLaunchKernelGGL(k_mf_gather, dim3((n + 255) / 256), dim3(256), 0, P.aux, A, (const double*)Ue,
                       (const double*)nullptr, y, 0);
    HIPX(hipEventRecord(P.ev_mf_join, P.aux));
    if (P.method != IGA_GAUSS_REF) {
        switch (P.p) {
#define CASE(PP) \
    case PP: launch_wq_forward<PP>(P, A, u, y, V, H, s); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
    }
    HIPX(hipStreamWaitEvent(s, P.ev_mf_join, 0));
}

void mf_apply(Plan& P, const double* c, const double* u, double* y, hipStream_t s) {
    mf_buffers(P);
    mf_apply_into(P, c, u, y, P.sw.V, P.sw.H, P.sw.Ue, s);
}

// ------------------------------------------------- allocation-free product
// The intermediate arrays of iga_mf_apply_noalloc live in one array of
// device memory that the library holds for the life of the process (one copy
// per device, at its own address). Every call on a device shares that
// device's copy: calls that overlap on one device race.
constexpr size_t kMfScratchDoubles = (size_t)8 << 20;  // 64 MiB
static __device__ __align__(256) double scratch[kMfScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with the device current; the array's name is no device address in host code).
void mf_scratch_init(int device) {
    IGA_REQUIRE(device >= 0 && device < kMaxDevices, IGA_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    int cur = -1;
    HIPX(hipGetDevice(&cur));
    IGA_REQUIRE(cur == device, IGA_E_INVALID, "scratch set-up needs its device current");
    void* ptr = nullptr;
    HIPX(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    IGA_REQUIRE(ptr != nullptr, IGA_E_HIP, "no device address for the scratch array");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
}

static size_t round256(size_t n_doubles) { return (n_doubles + 31) & ~(size_t)31; }  // 32 doubles = 256 B

static void mf_apply_noalloc(Plan& P, const double* c, const double* u, double* y, hipStream_t s) {
    mf_check(P);
    const size_t L = (size_t)(P.p + 1) * (P.p + 1);
    const size_t nV = round256((size_t)P.n2 * P.dir[0].Q), nH = round256((size_t)P.dir[1].Q * P.n1);
    const size_t nU = round256((size_t)std::max<int64_t>(1, P.n_band + P.n_cut_el) * L);
    const size_t need = nV + nH + nU;
    IGA_REQUIRE(need <= kMfScratchDoubles, IGA_E_CAPACITY,
                "allocation-free matrix-free product: the patch needs " + std::to_string(need * sizeof(double)) +
                    " bytes of intermediate arrays, more than the " +
                    std::to_string(kMfScratchDoubles * sizeof(double)) + "-byte scratch array");
    int dev = -1;
    HIPX(hipGetDevice(&dev));
    IGA_REQUIRE(dev == P.device, IGA_E_INVALID, "the plan's device must be current");
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[dev];
    }
    if (!base) {  // plan creation looks it up; a first call on a device that skipped it does so here
        mf_scratch_init(dev);
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[dev];
    }
    mf_apply_into(P, c, u, y, base, base + nV, base + nV + nH, s);
}

void mf_adjoint(Plan& P, const double* c, const double* u, const double* r, double* du, double* dc, hipStream_t s) {
    mf_buffers(P);
    MfArgs A = mf_args(P, c);
    int n = (int)P.n_act;
    // the element vectors (and dc at band Gauss points and cut nodes) on the second stream,
    // beside the grid part; the gather needs both
    HIPX(hipEventRecord(P.ev_mf_fork, s));
    HIPX(hipStreamWaitEvent(P.aux, P.ev_mf_fork, 0));
    launch_elem(P, A, u, r, P.sw.Ue, dc, P.aux);
    HIPX(hipEventRecord(P.ev_mf_join, P.aux));
    if (P.method != IGA_GAUSS_REF) {
        switch (P.p) {
#define CASE(PP) \
    case PP: launch_wq_adjoint<PP>(P, A, u, r, dc, s); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
    } else {
        HIPX(hipMemsetAsync(dc, 0, sizeof(double) * (size_t)A.nq, s));
    }
    HIPX(hipStreamWaitEvent(s, P.ev_mf_join, 0));
    // the grid part of du reads D (held in H) through the CR argument
    hipLaunchKernelGGL(k_mf_gather, dim3((n + 255) / 256), dim3(256), 0, s, A, (const double*)P.sw.Ue,
                       (const double*)P.sw.H, du, 1);
}

}  // namespace iga

using namespace iga;

extern "C" {

int iga_mf_apply(iga_plan* plan, const double* c_points, const double* u, double* y, void* stream) {
    try {
        IGA_REQUIRE(plan && c_points && u && y, IGA_E_INVALID, "null argument");
        IGA_REQUIRE(plan->method == IGA_HYBRID_GAUSS || plan->method == IGA_GAUSS_REF, IGA_E_UNSUPPORTED,
                    "matrix-free product is built for hybrid Gauss and the reference rules");
        mf_apply(*plan, c_points, u, y, (hipStream_t)stream);
        HIPX(hipGetLastError());
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    }
    return IGA_OK;
}

int iga_mf_apply_noalloc(iga_plan* plan, const double* c_points, const double* u, double* y, void* stream) {
    try {
        IGA_REQUIRE(plan && c_points && u && y, IGA_E_INVALID, "null argument");
        IGA_REQUIRE(plan->method == IGA_HYBRID_GAUSS || plan->method == IGA_GAUSS_REF, IGA_E_UNSUPPORTED,
                    "matrix-free product is built for hybrid Gauss and the reference rules");
        mf_apply_noalloc(*plan, c_points, u, y, (hipStream_t)stream);
        HIPX(hipGetLastError());
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    }
    return IGA_OK;
}

int iga_mf_adjoint(iga_plan* plan, const double* c_points, const double* u, const double* gy, double* du, double* dc,
                   void* stream) {
    try {
        IGA_REQUIRE(plan && c_points && u && gy && du && dc, IGA_E_INVALID, "null argument");
        IGA_REQUIRE(plan->method == IGA_HYBRID_GAUSS || plan->method == IGA_GAUSS_REF, IGA_E_UNSUPPORTED,
                    "matrix-free adjoint is built for hybrid Gauss and the reference rules");
        mf_adjoint(*plan, c_points, u, gy, du, dc, (hipStream_t)stream);
        HIPX(hipGetLastError());
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    }
    return IGA_OK;
}

}  // extern "C"
