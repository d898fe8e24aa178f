// Formation of the trimmed mass matrix (Eqs. (6)-(7), Sects. 3.1-3.2).
//
//  * k_interior: rows of interior test functions by weighted quadrature and
//    sum factorisation. A workgroup owns a tile of 64 consecutive i1 (one
//    per lane) and tile2 consecutive i2. For each i2 it first contracts the
//    xi_2 direction for every xi_1 point of the tile,
//        T[b][k1] = sum_{k2 in Q_i2} w2_{k2,i2} B_{i2+b}(x_k2) c(x_k1, x_k2),
//    into LDS, then each lane contracts xi_1 for its own row,
//        M[a][b] = sum_{k1 in Q_i1} w1_{k1,i1} B_{i1+a}(x_k1) T[b][k1],
//    and writes the (2p+1)^2 band of the row slot-major (coalesced across
//    lanes, no atomics).
//  * k_cut_elem: local matrices sum_g w_g c_g B_l B_m of each cut element
//    from its cut-rule nodes (one workgroup per element).
//  * k_cut_rows: rows formed element-wise (hybrid Gauss, Sect. 3.2: cut
//    rows; the reference: every row): element Gauss on inside elements of
//    the support, the cut element matrices on cut elements. One workgroup per
//    row, one thread per band slot.
#include "plan.hpp"

namespace iga {

// ------------------------------------------------------------ points
__global__ void k_points_wq(DirDev D1, DirDev D2, double* __restrict__ xy) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= D1.Q * D2.Q) return;
    int k1 = k % D1.Q, k2 = k / D1.Q;
    xy[2 * k] = D1.xq[k1];
    xy[2 * k + 1] = D2.xq[k2];
}

__global__ void k_points_band(DirDev D1, DirDev D2, int p, const int* __restrict__ band_list, int n_band,
                              double* __restrict__ xy) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int ng = (p + 1) * (p + 1);
    if (t >= n_band * ng) return;
    int b = t / ng, g = t % ng, g1 = g % (p + 1), g2 = g / (p + 1);
    int e = band_list[b], e1 = e % D1.N, e2 = e / D1.N;
    xy[2 * t] = D1.xg[e1 * (p + 1) + g1];
    xy[2 * t + 1] = D2.xg[e2 * (p + 1) + g2];
}

__global__ void k_points_cut(const double* __restrict__ nx, const double* __restrict__ ny, int n,
                             double* __restrict__ xy) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    xy[2 * t] = nx[t];
    xy[2 * t + 1] = ny[t];
}

void launch_points(Plan& P, hipStream_t s) {
    DirDev &D1 = P.dir[0], &D2 = P.dir[1];
    int nq = D1.Q * D2.Q;
    hipLaunchKernelGGL(k_points_wq, dim3((nq + 255) / 256), dim3(256), 0, s, D1, D2, P.pts_xy);
    int nb = (int)P.n_band * (P.p + 1) * (P.p + 1);
    if (nb > 0)
        hipLaunchKernelGGL(k_points_band, dim3((nb + 255) / 256), dim3(256), 0, s, D1, D2, P.p, P.band_list,
                           (int)P.n_band, P.pts_xy + 2 * (size_t)nq);
    if (P.n_nodes > 0)
        hipLaunchKernelGGL(k_points_cut, dim3((P.n_nodes + 255) / 256), dim3(256), 0, s, P.node_x, P.node_y,
                           (int)P.n_nodes, P.pts_xy + 2 * ((size_t)nq + nb));
}

// ------------------------------------------------------- coefficient
// |det DF| at a point from per-direction values/derivatives of the local
// functions and the (p+1)^2 control points of element (e1, e2).
__device__ __forceinline__ double detj_local(const double* __restrict__ cp, int n1, int p, int e1, int e2,
                                             const double* B1, const double* dB1, const double* B2,
                                             const double* dB2) {
    double x1 = 0, x2 = 0, y1 = 0, y2 = 0;
    for (int a2 = 0; a2 <= p; ++a2) {
        double sx1 = 0, sx = 0, sy1 = 0, sy = 0;
        const double* row = cp + 2 * ((size_t)(e2 + a2) * n1 + e1);
        for (int a1 = 0; a1 <= p; ++a1) {
            double px = row[2 * a1], py = row[2 * a1 + 1];
            sx1 += dB1[a1] * px;
            sx += B1[a1] * px;
            sy1 += dB1[a1] * py;
            sy += B1[a1] * py;
        }
        x1 += B2[a2] * sx1;
        y1 += B2[a2] * sy1;
        x2 += dB2[a2] * sx;
        y2 += dB2[a2] * sy;
    }
    return fabs(x1 * y2 - x2 * y1);
}

__global__ void k_coef_wq(DirDev D1, DirDev D2, int p, const double* __restrict__ cp, int n1, double* __restrict__ c) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= D1.Q * D2.Q) return;
    int k1 = k % D1.Q, k2 = k / D1.Q;
    c[k] = detj_local(cp, n1, p, D1.eq[k1], D2.eq[k2], D1.Bq + k1 * (p + 1), D1.dBq + k1 * (p + 1),
                      D2.Bq + k2 * (p + 1), D2.dBq + k2 * (p + 1));
}

__global__ void k_coef_band(DirDev D1, DirDev D2, int p, const double* __restrict__ cp, int n1,
                            const int* __restrict__ band_list, int n_band, double* __restrict__ c) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int ng = (p + 1) * (p + 1);
    if (t >= n_band * ng) return;
    int b = t / ng, g = t % ng, g1 = g % (p + 1), g2 = g / (p + 1);
    int e = band_list[b], e1 = e % D1.N, e2 = e / D1.N;
    int r1 = (e1 * (p + 1) + g1) * (p + 1), r2 = (e2 * (p + 1) + g2) * (p + 1);
    c[t] = detj_local(cp, n1, p, e1, e2, D1.Bg + r1, D1.dBg + r1, D2.Bg + r2, D2.dBg + r2);
}

__global__ void k_coef_cut(DirDev D1, DirDev D2, int p, const double* __restrict__ cp, int n1,
                           const int* __restrict__ cut_list, const int* __restrict__ node_el,
                           const double* __restrict__ nx, const double* __restrict__ ny, int n,
                           double* __restrict__ c) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int e = cut_list[node_el[t]], e1 = e % D1.N, e2 = e / D1.N;
    double B1[IGA_MAXP + 1], dB1[IGA_MAXP + 1], B2[IGA_MAXP + 1], dB2[IGA_MAXP + 1];
    basis_eval_rt(D1.knots, p, p + e1, nx[t], B1, dB1);
    basis_eval_rt(D2.knots, p, p + e2, ny[t], B2, dB2);
    c[t] = detj_local(cp, n1, p, e1, e2, B1, dB1, B2, dB2);
}

CoefView coef_view(Plan& P, const iga_coeff& c) {
    CoefView v{0, 1.0, nullptr, nullptr, nullptr};
    size_t nq = (size_t)P.dir[0].Q * P.dir[1].Q;
    size_t nb = (size_t)P.n_band * (P.p + 1) * (P.p + 1);
    if (c.kind == IGA_COEF_CONST) {
        v.is_const = 1;
        v.value = c.value;
    } else if (c.kind == IGA_COEF_GEOM_DETJ) {
        v.wq = P.c_wq;
        v.band = P.c_band;
        v.cut = P.c_cut;
    } else {
        v.wq = c.c_points;
        v.band = c.c_points + nq;
        v.cut = c.c_points + nq + nb;
    }
    return v;
}

void launch_coef(Plan& P, const iga_coeff& c, hipStream_t s) {
    if (c.kind != IGA_COEF_GEOM_DETJ) return;
    DirDev &D1 = P.dir[0], &D2 = P.dir[1];
    int p = P.p;
    int nq = D1.Q * D2.Q;
    hipLaunchKernelGGL(k_coef_wq, dim3((nq + 255) / 256), dim3(256), 0, s, D1, D2, p, c.geom_cp, P.n1, P.c_wq);
    int nb = (int)P.n_band * (p + 1) * (p + 1);
    if (nb > 0)
        hipLaunchKernelGGL(k_coef_band, dim3((nb + 255) / 256), dim3(256), 0, s, D1, D2, p, c.geom_cp, P.n1,
                           P.band_list, (int)P.n_band, P.c_band);
    if (P.n_nodes > 0)
        hipLaunchKernelGGL(k_coef_cut, dim3((P.n_nodes + 255) / 256), dim3(256), 0, s, D1, D2, p, c.geom_cp, P.n1,
                           P.cut_list, P.node_el, P.node_x, P.node_y, (int)P.n_nodes, P.c_cut);
}

// ------------------------------------------------------- interior rows
struct IntArgs {
    DirDev d1, d2;
    CoefView c;
    const double* cwq;       // coefficient on the WQ grid (nullptr -> constant c.value)
    const int8_t* fcls;
    const int* act_of;
    int all_active;          // 1: every active row (naive WQ), 0: interior rows only
    double* vals;
    int64_t n_act;
    int tile2;
};

template <int P>
struct IntShape {
    static constexpr int W = 2 * P + 1;          // band width
    static constexpr int QM = 4 * P + 2;         // max WQ points in one support
    static constexpr int KS = 2 * (64 + P) + 2 * P + 2;  // max xi_1 points of a tile
};

template <int P>
__global__ void __launch_bounds__(256) k_interior(IntArgs A) {
    using S = IntShape<P>;
    constexpr int W = S::W, QM = S::QM, KS = S::KS;
    __shared__ double sT[W][KS];          // T[b][k1 - k1lo]
    __shared__ double sB1[KS][P + 1];     // B values at the tile's xi_1 points
    __shared__ double sW1[64][QM + 1];    // weights of each lane's test function
    __shared__ double sWB2[QM][W];        // w2 * B for the current i2
    __shared__ int sPt0[64 + P + 2];

    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int I1 = blockIdx.x * 64;
    int I2 = blockIdx.y * A.tile2;
    int elo = max(0, I1 - P), ehi = min(D1.N - 1, I1 + 63);
    int k1lo = D1.pt0[elo], k1hi = D1.pt0[ehi + 1];
    int ks = k1hi - k1lo;

    for (int t = tid; t < ehi - elo + 2; t += 256) sPt0[t] = D1.pt0[elo + t] - k1lo;
    for (int t = tid; t < ks * (P + 1); t += 256) sB1[t / (P + 1)][t % (P + 1)] = D1.Bq[(size_t)k1lo * (P + 1) + t];
    for (int t = tid; t < 64 * QM; t += 256) {
        int l = t / QM, q = t % QM;
        int i1 = I1 + l;
        sW1[l][q] = (i1 < D1.n && q < D1.qmax) ? D1.W[(size_t)i1 * D1.qmax + q] : 0.0;
    }
    int i1 = I1 + lane;
    int k0_1 = (i1 < D1.n) ? D1.pt0[max(0, i1 - P)] - k1lo : 0;

    for (int r = 0; r < A.tile2; ++r) {
        int i2 = I2 + r;
        if (i2 >= D2.n) break;
        int e2lo = max(0, i2 - P), e2hi = min(D2.N - 1, i2);
        int k2lo = D2.pt0[e2lo], q2 = D2.pt0[e2hi + 1] - k2lo;
        __syncthreads();
        // w2_{k2,i2} B_{i2+b}(x_k2) for the current i2
        for (int t = tid; t < QM * W; t += 256) {
            int q = t / W, b = t % W;
            double v = 0.0;
            if (q < q2) {
                int k2 = k2lo + q, e = D2.eq[k2];
                int loc = i2 + b - P - e;
                if (loc >= 0 && loc <= P) v = D2.W[(size_t)i2 * D2.qmax + q] * D2.Bq[(size_t)k2 * (P + 1) + loc];
            }
            sWB2[q][b] = v;
        }
        __syncthreads();
        // stage 1: contract xi_2
        for (int t = tid; t < ks; t += 256) {
            double cv[QM];
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                cv[q] = 0.0;
                if (q < q2) cv[q] = A.cwq ? A.cwq[(size_t)(k2lo + q) * D1.Q + k1lo + t] : A.c.value;
            }
#pragma unroll
            for (int b = 0; b < W; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < QM; ++q) acc += sWB2[q][b] * cv[q];
                sT[b][t] = acc;
            }
        }
        __syncthreads();
        // stage 2: contract xi_1, one row per lane
        bool live = false;
        int64_t cid = -1;
        if (i1 < D1.n) {
            int f = i2 * D1.n + i1;
            int8_t cls = A.fcls[f];
            live = A.all_active ? (cls != FN_EXTERIOR) : (cls == FN_INTERIOR);
            if (live) cid = A.act_of[f];
        }
        for (int b = wave; b < W; b += 4) {
            double acc[W];
#pragma unroll
            for (int a = 0; a < W; ++a) acc[a] = 0.0;
            if (live) {
#pragma unroll
                for (int m = 0; m <= P; ++m) {
                    int e = i1 - P + m;
                    if (e < 0 || e >= D1.N) continue;
                    int kb = sPt0[e - elo], ke = sPt0[e - elo + 1];
                    for (int k = kb; k < ke; ++k) {
                        double wt = sW1[lane][k - k0_1] * sT[b][k];
#pragma unroll
                        for (int al = 0; al <= P; ++al) acc[m + al] += wt * sB1[k][al];
                    }
                }
#pragma unroll
                for (int a = 0; a < W; ++a) A.vals[(size_t)(a * W + b) * A.n_act + cid] = acc[a];
            }
        }
    }
}

void launch_interior_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s) {
    if (P.method == IGA_GAUSS_REF) return;
    IntArgs A;
    A.d1 = P.dir[0];
    A.d2 = P.dir[1];
    A.c = coef_view(P, c);
    A.cwq = A.c.is_const ? nullptr : A.c.wq;
    if (P.method == IGA_NAIVE_WQ) A.cwq = P.c_wq_masked;
    A.fcls = P.fcls;
    A.act_of = P.act_of;
    A.all_active = (P.method == IGA_NAIVE_WQ);
    A.vals = vals;
    A.n_act = P.n_act;
    A.tile2 = P.tile2;
    dim3 g((P.n1 + 63) / 64, (P.n2 + P.tile2 - 1) / P.tile2), b(256);
    switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_interior<PP>, g, b, 0, s, A); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

// -------------------------------------------------- cut element matrices
struct CutEArgs {
    DirDev d1, d2;
    CoefView c;
    const int* cut_list;
    const int* node_off;
    const double *nx, *ny, *nw;
    double* E;
    int n_cut;
};

template <int P>
__global__ void __launch_bounds__(256) k_cut_elem(CutEArgs A) {
    constexpr int L = (P + 1) * (P + 1);
    constexpr int NE = L * (L + 1) / 2;
    constexpr int PER = (NE + 255) / 256;
    constexpr int CH = 64;
    __shared__ double sPhi[CH][L];
    __shared__ double sWc[CH];
    int c = blockIdx.x;
    if (c >= A.n_cut) return;
    int e = A.cut_list[c], e1 = e % A.d1.N, e2 = e / A.d1.N;
    int nb = A.node_off[c], ne = A.node_off[c + 1];
    double acc[PER];
    int el[PER], em[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        acc[k] = 0.0;
        int t = threadIdx.x + 256 * k;
        int l = 0, rem = t;
        while (l < L && rem >= L - l) { rem -= L - l; ++l; }   // upper-triangle enumeration
        el[k] = (t < NE) ? l : -1;
        em[k] = (t < NE) ? l + rem : -1;
    }
    for (int base = nb; base < ne; base += CH) {
        __syncthreads();
        if (threadIdx.x < CH) {
            int n = base + threadIdx.x;
            if (n < ne) {
                double B1[P + 1], B2[P + 1];
                basis_eval<P>(A.d1.knots, P + e1, A.nx[n], B1);
                basis_eval<P>(A.d2.knots, P + e2, A.ny[n], B2);
#pragma unroll
                for (int a2 = 0; a2 <= P; ++a2)
#pragma unroll
                    for (int a1 = 0; a1 <= P; ++a1) sPhi[threadIdx.x][a2 * (P + 1) + a1] = B1[a1] * B2[a2];
                sWc[threadIdx.x] = A.nw[n] * (A.c.is_const ? A.c.value : A.c.cut[n]);
            } else {
                sWc[threadIdx.x] = 0.0;
#pragma unroll
                for (int l = 0; l < L; ++l) sPhi[threadIdx.x][l] = 0.0;
            }
        }
        __syncthreads();
        int cnt = min(CH, ne - base);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (el[k] < 0) continue;
            double s = 0.0;
            for (int n = 0; n < cnt; ++n) s += sWc[n] * sPhi[n][el[k]] * sPhi[n][em[k]];
            acc[k] += s;
        }
    }
    double* E = A.E + (size_t)c * L * L;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (el[k] < 0) continue;
        E[el[k] * L + em[k]] = acc[k];
        E[em[k] * L + el[k]] = acc[k];
    }
}

// ------------------------------------------------------------ cut rows
struct CutRowArgs {
    DirDev d1, d2;
    CoefView c;
    const int* rows;        // compact ids of the rows formed here
    int n_rows;
    const int* fn_of;
    const int* act_of;
    const int8_t* ecls;
    const int* cut_id;
    const int* band_id;
    const double* E;
    double* vals;
    int64_t n_act;
};

template <int P>
__global__ void k_cut_rows(CutRowArgs A) {
    constexpr int W = 2 * P + 1, L = (P + 1) * (P + 1);
    int r = blockIdx.x;
    if (r >= A.n_rows) return;
    int s = threadIdx.x;
    if (s >= W * W) return;
    int row = A.rows[r];
    int f = A.fn_of[row];
    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    int i1 = f % D1.n, i2 = f / D1.n;
    int a = s / W - P, b = s % W - P;
    int j1 = i1 + a, j2 = i2 + b;
    double val = 0.0;
    if (j1 >= 0 && j1 < D1.n && j2 >= 0 && j2 < D2.n && A.act_of[j2 * D1.n + j1] >= 0) {
        int e1lo = max(max(i1, j1) - P, 0), e1hi = min(min(i1, j1), D1.N - 1);
        int e2lo = max(max(i2, j2) - P, 0), e2hi = min(min(i2, j2), D2.N - 1);
        for (int e2 = e2lo; e2 <= e2hi; ++e2)
            for (int e1 = e1lo; e1 <= e1hi; ++e1) {
                int e = e2 * D1.N + e1;
                int8_t cls = A.ecls[e];
                if (cls == EL_OUTSIDE) continue;
                if (cls == EL_CUT) {
                    int li = (i2 - e2) * (P + 1) + (i1 - e1), lj = (j2 - e2) * (P + 1) + (j1 - e1);
                    val += A.E[(size_t)A.cut_id[e] * L * L + li * L + lj];
                    continue;
                }
                const double* cb = A.c.is_const ? nullptr : A.c.band + (size_t)A.band_id[e] * (P + 1) * (P + 1);
                double sum = 0.0;
#pragma unroll
                for (int g2 = 0; g2 <= P; ++g2) {
                    int r2 = (e2 * (P + 1) + g2) * (P + 1);
                    double f2 = D2.wg[e2 * (P + 1) + g2] * D2.Bg[r2 + i2 - e2] * D2.Bg[r2 + j2 - e2];
                    double in = 0.0;
#pragma unroll
                    for (int g1 = 0; g1 <= P; ++g1) {
                        int r1 = (e1 * (P + 1) + g1) * (P + 1);
                        double cv = cb ? cb[g2 * (P + 1) + g1] : A.c.value;
                        in += D1.wg[e1 * (P + 1) + g1] * D1.Bg[r1 + i1 - e1] * D1.Bg[r1 + j1 - e1] * cv;
                    }
                    sum += f2 * in;
                }
                val += sum;
            }
    }
    A.vals[(size_t)s * A.n_act + row] = val;
}

void launch_cut_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s) {
    if (P.method == IGA_NAIVE_WQ) return;
    CoefView cv = coef_view(P, c);
    if (P.n_cut_el > 0) {
        CutEArgs A{P.dir[0], P.dir[1], cv, P.cut_list, P.node_off, P.node_x, P.node_y, P.node_w, P.cutE,
                   (int)P.n_cut_el};
        dim3 g((unsigned)P.n_cut_el), b(256);
        switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_cut_elem<PP>, g, b, 0, s, A); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
            default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
        }
    }
    if (P.n_form_rows > 0) {
        CutRowArgs A{P.dir[0], P.dir[1], cv, P.form_rows, (int)P.n_form_rows, P.fn_of, P.act_of, P.ecls,
                     P.cut_id, P.band_id, P.cutE, vals, P.n_act};
        int W = 2 * P.p + 1;
        dim3 g((unsigned)P.n_form_rows), b(((W * W + 63) / 64) * 64);
        switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_cut_rows<PP>, g, b, 0, s, A); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
            default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
        }
    }
}

}  // namespace iga
