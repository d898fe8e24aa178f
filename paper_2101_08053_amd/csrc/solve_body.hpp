// Device bodies of the L2 projection (Sect. 4.2), shared by the one-patch
// kernels (solve.hip) and the batched ones (batch_solve.hip): the same
// arithmetic in the same order, so a batched projection reproduces the
// one-patch projection of each patch bit for bit.
//
//  * right-hand side b_i = row i's own rule applied to g c: weighted
//    quadrature for interior rows (Eq. (5) weights in both directions),
//    element Gauss and the cut-element rule for rows formed element-wise
//    (element vectors, then a gather over the support in a fixed order);
//  * A = (M + M^T)/2 in the band layout and the compact column of each slot;
//  * the steps of Jacobi-preconditioned CG, with block partials of the dot
//    products summed in a fixed order.
#pragma once

#include "dwq_body.hpp"
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

// g c at rule point t (iga_plan_points order): the WQ grid, the band Gauss
// points, the cut nodes.
__device__ __forceinline__ void gc_point(const GcArgs& A, int t) {
    const int p = A.p;
    const int nq = A.d1.Q * A.d2.Q;
    const int ng = (p + 1) * (p + 1);
    const int nb = A.n_band * ng;
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

// b of compact row r if it is an interior row (weighted quadrature); rows
// formed element-wise are left to the gather.
__device__ __forceinline__ void rhs_wq_row(const DirDev& D1, const DirDev& D2, int p, const int8_t* __restrict__ fcls,
                                           int all_active, const int* __restrict__ fn_of, int r,
                                           const double* __restrict__ gc_wq, double* __restrict__ b) {
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

// Element vectors F_e[l] = sum_g w_g (g c)_g B_l(x_g) of the band (Gauss) and
// cut elements; one 64-thread workgroup per element re (band elements first).
template <int P>
struct RhsElemSmem {
    double phi[64][(P + 1) * (P + 1)];
    double t[64];
};

struct RhsElemArgs {
    DirDev d1, d2;
    const int* band_list;
    int n_band;
    const int* cut_list;
    const int* node_off;
    const double *nx, *ny, *nw;
    const double* gc;   // g c in rule-point order
    int gc_band_off, gc_cut_off;
    double* F;          // [n_band + n_cut][(p+1)^2]
};

template <int P>
__device__ __forceinline__ void rhs_elem_body(const RhsElemArgs& A, int re, RhsElemSmem<P>& S) {
    constexpr int L = (P + 1) * (P + 1);
    const DirDev &D1 = A.d1, &D2 = A.d2;
    bool is_cut = re >= A.n_band;
    int e = is_cut ? A.cut_list[re - A.n_band] : A.band_list[re];
    int e1 = e % D1.N, e2 = e / D1.N;
    int nb, ne;
    if (is_cut) {
        nb = A.node_off[re - A.n_band];
        ne = A.node_off[re - A.n_band + 1];
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
                basis_eval<P>(D1.knots, P + e1, A.nx[n], B1);
                basis_eval<P>(D2.knots, P + e2, A.ny[n], B2);
                w = A.nw[n];
                gcv = A.gc[A.gc_cut_off + n];
            } else {
                int g1 = n % (P + 1), g2 = n / (P + 1);
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    B1[a] = D1.Bg[(e1 * (P + 1) + g1) * (P + 1) + a];
                    B2[a] = D2.Bg[(e2 * (P + 1) + g2) * (P + 1) + a];
                }
                w = D1.wg[e1 * (P + 1) + g1] * D2.wg[e2 * (P + 1) + g2];
                gcv = A.gc[A.gc_band_off + re * L + n];
            }
#pragma unroll
            for (int a2 = 0; a2 <= P; ++a2)
#pragma unroll
                for (int a1 = 0; a1 <= P; ++a1) S.phi[threadIdx.x][a2 * (P + 1) + a1] = B1[a1] * B2[a2];
            S.t[threadIdx.x] = w * gcv;
        }
        __syncthreads();
        int cnt = min(64, ne - base);
#pragma unroll
        for (int k = 0; k < (L + 63) / 64; ++k) {
            int l = threadIdx.x + 64 * k;
            if (l < L)
                for (int m = 0; m < cnt; ++m) acc[k] += S.t[m] * S.phi[m][l];
        }
    }
#pragma unroll
    for (int k = 0; k < (L + 63) / 64; ++k) {
        int l = threadIdx.x + 64 * k;
        if (l < L) A.F[(size_t)re * L + l] = acc[k];
    }
}

// b of element-formed row rows[t]: F_e gathered over the support elements.
struct RhsGatherArgs {
    int p, N1, N2, n1;
    const int* rows;
    int n_rows;
    const int* fn_of;
    const int8_t* ecls;
    const int* band_id;
    const int* cut_id;
    int n_band;
    const double* F;
    double* b;
    const int* region;    // DWQ: [n_rows][8] boxes; support elements inside a row's box are skipped (nullptr: none)
};

__device__ __forceinline__ void rhs_gather_row(const RhsGatherArgs& A, int t) {
    const int p = A.p;
    int r = A.rows[t], f = A.fn_of[r], i1 = f % A.n1, i2 = f / A.n1;
    int L = (p + 1) * (p + 1);
    int bx0 = 1, bx1 = 0, by0 = 1, by1 = 0;   // box (empty by default)
    if (A.region && A.region[(size_t)t * 8] >= 0) {
        bx0 = A.region[(size_t)t * 8];
        bx1 = A.region[(size_t)t * 8 + 1];
        by0 = A.region[(size_t)t * 8 + 4];
        by1 = A.region[(size_t)t * 8 + 5];
    }
    double s = 0.0;
    for (int e2 = max(0, i2 - p); e2 <= min(A.N2 - 1, i2); ++e2)
        for (int e1 = max(0, i1 - p); e1 <= min(A.N1 - 1, i1); ++e1) {
            int e = e2 * A.N1 + e1;
            int8_t c = A.ecls[e];
            if (c == EL_OUTSIDE || (e1 >= bx0 && e1 <= bx1 && e2 >= by0 && e2 <= by1)) continue;
            int re = (c == EL_CUT) ? A.n_band + A.cut_id[e] : A.band_id[e];
            s += A.F[(size_t)re * L + (i2 - e2) * (p + 1) + (i1 - e1)];
        }
    A.b[r] = s;
}

// Sum over the workgroup in a fixed order (valid in thread 0).
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

// Box part of the right-hand side of a DWQ row (Sect. 3.3 with B_j -> g):
// the row's two 1-D rules restricted to its box (dwq_rule_point) and
// sum_k sum_l w1_k w2_l (g c)(x1_k, x2_l), added to b of the row (the gather
// has written the element part outside the box). g c comes from the WQ grid
// values where both coordinates are WQ points, and is evaluated otherwise
// (nested points): g at the mapped point, c = |det J| or the constant.
struct DwqRhsArgs {
    DirDev d1, d2;
    iga_target g;
    const double* geom;   // control points or nullptr (identity map); c = |det J| when set
    int n1;
    int c_const;
    double c_value;
    const double* gc_wq;  // g c on the WQ grid
    const int* rows;
    int n_rows;
    const int* fn_of;
    const int* region;
    double* b;
};

constexpr int kDwqRhsThreads = 128;

template <int P>
__device__ __forceinline__ void dwq_rhs_body(const DwqRhsArgs& A, int r) {
    constexpr int KQ = 64;
    __shared__ double sX[2][KQ], sW[2][KQ];
    __shared__ int sE[2][KQ], sK[2][KQ], sN[2];
    __shared__ double sh[kDwqRhsThreads / 64];
    if (r >= A.n_rows) return;
    const int* reg = A.region + (size_t)r * 8;
    if (reg[0] < 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = A.rows[r];
    const int f = A.fn_of[row];
    const int i1 = f % A.d1.n, i2 = f / A.d1.n;
    if (wave < 2) {
        const int d = wave;
        double x, w;
        int e, k;
        const bool ok = dwq_rule_point<P>(d ? A.d2 : A.d1, d ? i2 : i1, reg + 4 * d, lane, x, w, e, k);
        const unsigned long long msk = __ballot(ok);
        const int pos = __popcll(msk & ((1ull << lane) - 1ull));
        if (ok) {
            sX[d][pos] = x;
            sW[d][pos] = w;
            sE[d][pos] = e;
            sK[d][pos] = k;
        }
        if (lane == 0) sN[d] = __popcll(msk);
    }
    __syncthreads();
    const int n1q = sN[0], n2q = sN[1];
    double acc = 0.0;
    for (int tt = tid; tt < n1q * n2q; tt += kDwqRhsThreads) {
        const int q1 = tt % n1q, q2 = tt / n1q;
        double gc;
        if (sK[0][q1] >= 0 && sK[1][q2] >= 0) {
            gc = A.gc_wq[(size_t)sK[1][q2] * A.d1.Q + sK[0][q1]];
        } else {
            const int e1 = sE[0][q1], e2 = sE[1][q2];
            const double x = sX[0][q1], y = sX[1][q2];
            double B1[P + 1], dB1[P + 1], B2[P + 1], dB2[P + 1];
            basis_eval_d<P>(A.d1.knots, P + e1, x, B1, dB1);
            basis_eval_d<P>(A.d2.knots, P + e2, y, B2, dB2);
            double X = x, Y = y, c = A.c_value;
            if (A.geom) map_local(A.geom, A.n1, P, e1, e2, B1, B2, X, Y);
            if (!A.c_const) c = detj_local(A.geom, A.n1, P, e1, e2, B1, dB1, B2, dB2);
            gc = target_eval(A.g, X, Y) * c;
        }
        acc += sW[0][q1] * sW[1][q2] * gc;
    }
    acc = block_sum(acc, sh);
    if (tid == 0) A.b[row] += acc;
}

// Argument blocks of one plan (solve.hip).
GcArgs gc_args(Plan& P, const iga_coeff& c, const iga_target& g, double* out);
RhsElemArgs rhs_elem_args(Plan& P, const double* gc, double* F);
RhsGatherArgs rhs_gather_args(Plan& P, const double* F, double* b);
DwqRhsArgs dwq_rhs_args(Plan& P, const iga_coeff& c, const iga_target& g, const double* gc, double* b);
// Throws unless the plan's method has a right-hand side for this target and coefficient.
void rhs_check(const Plan& P, const iga_coeff& c, const iga_target& g);
// b (device, n_act) = row rules applied to g c, on stream s
void rhs(Plan& P, const iga_coeff& c, const iga_target& g, double* b, hipStream_t s);


// ------------------------------------------------------------------- PCG
// A = (M + M^T)/2: slot (a, b) of row r pairs with slot (-a, -b) of its
// column's row. Entry t = s * n_act + r of the band.
__device__ __forceinline__ void symmetrize_entry(int p, int n1, int n2, const int* __restrict__ fn_of,
                                                 const int* __restrict__ act_of, int n_act,
                                                 const double* __restrict__ M, double* __restrict__ A, int64_t t) {
    int W = 2 * p + 1;
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
constexpr int kCgCheck = 16;  // iterations between two convergence checks

struct SpArgs {
    int p, n1, n2, n_act;
    const int* fn_of;
    const int* act_of;
    const double* A;
    const int* cols;  // [(2p+1)^2][n_act] compact column of each slot, -1 if none (PCG iterations)
    const double* dg = nullptr;  // preconditioner diagonal when given, else A's own
};

// Compact column of band entry t = s * n_act + r.
__device__ __forceinline__ int col_entry(const SpArgs& S, int64_t t) {
    const int W = 2 * S.p + 1;
    const int sl = (int)(t / S.n_act), r = (int)(t % S.n_act);
    const int f = S.fn_of[r], j1 = f % S.n1 + sl / W - S.p, j2 = f / S.n1 + sl % W - S.p;
    return (j1 >= 0 && j1 < S.n1 && j2 >= 0 && j2 < S.n2) ? S.act_of[j2 * S.n1 + j1] : -1;
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

// Row r of A x from the index maps (same order of terms as spmv_row_cols).
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

// Sum of a kernel's block partials, the same in every block (thread 0 holds it).
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, int nv, int v, double* sh) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += part[nv * k + v];
    return block_sum(s, sh);
}

// Diagonal of the Jacobi preconditioner at row r: A's own, or the one given.
__device__ __forceinline__ double diag_of(const SpArgs& S, int r) {
    const int W = 2 * S.p + 1;
    return S.dg ? S.dg[r] : S.A[(size_t)(S.p * W + S.p) * S.n_act + r];
}

// ---- the steps of the iteration, for one workgroup of kRedThreads rows: lb
// is the workgroup's block within its patch, vectors and partials start at the
// patch's first row and first block, scal holds the patch's scalars
// (0: initial (r.z), 2: (r.r), 3: (b.b), 6 / 7: (r.z) of even / odd iterations).

// r = b - A x, z = r/d, p = z; partials of (r.z), (r.r), (b.b) at part[3 lb ..]
__device__ __forceinline__ void cg_init_block(const SpArgs& S, int lb, const double* __restrict__ bvec,
                                              const double* __restrict__ x, double* __restrict__ rv,
                                              double* __restrict__ zv, double* __restrict__ pv,
                                              double* __restrict__ part, double* sh) {
    int r = lb * kRedThreads + threadIdx.x;
    double rz = 0, rr = 0, bb = 0;
    if (r < S.n_act) {
        double d = diag_of(S, r);
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
        part[3 * lb] = s0;
        part[3 * lb + 1] = s1;
        part[3 * lb + 2] = s2;
    }
}

// The initial (r.z), (r.r), (b.b) from the block partials (one workgroup).
__device__ __forceinline__ void cg_reduce0(const double* __restrict__ part, int nblk, double* __restrict__ scal,
                                           double* sh) {
    for (int v = 0; v < 3; ++v) {
        double s = 0.0;
        for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += part[3 * k + v];
        double tot = block_sum(s, sh);
        if (threadIdx.x == 0) {
            scal[v == 0 ? 0 : (v == 1 ? 2 : 3)] = tot;
            if (v == 0) scal[6] = tot;  // (r.z) of the first iteration
        }
        __syncthreads();
    }
}

// q = A p; partial of (p.q) at part[lb]
template <int P>
__device__ __forceinline__ void cg_spmv_block(const SpArgs& S, int lb, const double* __restrict__ pv,
                                              double* __restrict__ qv, double* __restrict__ part, double* sh) {
    int r = lb * kRedThreads + threadIdx.x;
    double pq = 0.0;
    if (r < S.n_act) {
        double q = spmv_row_cols<P>(S, pv, r);
        qv[r] = q;
        pq = pv[r] * q;
    }
    double s = block_sum(pq, sh);
    if (threadIdx.x == 0) part[lb] = s;
}

// alpha = (r.z) / (p.q) from the spmv kernel's partials (summed by every
// block in the same order); x += alpha p, r -= alpha q, z = r/d; partials of
// (r.z), (r.r) at part[2 lb ..]. Iterations may run on after the residual
// has vanished (convergence is read every few iterations): then p.q = 0 and
// the step is zero, not 0/0.
__device__ __forceinline__ void cg_update_block(const SpArgs& S, int lb, const double* __restrict__ scal, int par,
                                                int nblk, const double* __restrict__ part_pq, double* __restrict__ x,
                                                double* __restrict__ rv, double* __restrict__ zv,
                                                const double* __restrict__ pv, const double* __restrict__ qv,
                                                double* __restrict__ part, double* sh, double* s_alpha) {
    const double pq = sum_partials(part_pq, nblk, 1, 0, sh);
    if (threadIdx.x == 0) *s_alpha = (pq != 0.0) ? scal[6 + par] / pq : 0.0;
    __syncthreads();
    int r = lb * kRedThreads + threadIdx.x;
    double rz = 0, rr = 0;
    if (r < S.n_act) {
        double alpha = *s_alpha;
        double d = diag_of(S, r);
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
        part[2 * lb] = s0;
        part[2 * lb + 1] = s1;
    }
}

// beta = (r.z)_new / (r.z)_old; p = z + beta p. Block 0 stores the new (r.z)
// in the other parity slot and (r.r) (other blocks still read the old (r.z)).
// Returns (r.r) in thread 0.
__device__ __forceinline__ double cg_dir_block(int n, int lb, double* __restrict__ scal, int par, int nblk,
                                               const double* __restrict__ part, const double* __restrict__ zv,
                                               double* __restrict__ pv, double* sh, double* s_beta) {
    const double rz = sum_partials(part, nblk, 2, 0, sh);
    const double rr = sum_partials(part, nblk, 2, 1, sh);
    if (threadIdx.x == 0) {
        *s_beta = (scal[6 + par] != 0.0) ? rz / scal[6 + par] : 0.0;  // a vanished residual keeps p = z
        if (lb == 0) {
            scal[6 + (1 - par)] = rz;
            scal[2] = rr;
        }
    }
    __syncthreads();
    int r = lb * kRedThreads + threadIdx.x;
    if (r < n) pv[r] = zv[r] + *s_beta * pv[r];
    return rr;
}

// PCG buffers of the plan (first call allocates)
void solve_buffers(Plan& P);
// A = (M + M^T)/2 and the slot columns from vals; the operator's arguments
SpArgs solve_operator(Plan& P, const double* vals, hipStream_t s);

}  // namespace iga
