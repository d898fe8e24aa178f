// Device bodies of the formation kernels, shared by the one-patch kernels
// (form.hip) and the batched persistent kernel (batch.hip). Each body forms
// one work item with 256 threads on LDS the caller provides.
#pragma once

#include "bounds.hpp"
#include "plan.hpp"

namespace iga {

// ------------------------------------------------------------ coefficient
struct CoefArgs {
    DirDev d1, d2;
    const double* cp;         // geometry control points [n2][n1][2]
    int n1;
    const int* band_list;
    int n_band;
    const int* cut_list;
    const int* node_el;
    const double *nx, *ny;
    int n_nodes;
    double *c_wq, *c_band, *c_cut;
    int64_t nq, nb;           // WQ grid points, band Gauss points
    double* xy;               // if set: the grid and band points' coordinates go to the rule-point table too
};

CoefArgs coef_args(Plan& P, const iga_coeff& c);

// |det J| at rule point t of the concatenation WQ grid | band Gauss points | cut nodes.
template <int P>
__device__ __forceinline__ void coef_point(const CoefArgs& A, int64_t t) {
    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    if (t < A.nq) {
        const int k1 = (int)(t % D1.Q), k2 = (int)(t / D1.Q);
        A.c_wq[t] = detj_local(A.cp, A.n1, P, D1.eq[k1], D2.eq[k2], D1.Bq + k1 * (P + 1), D1.dBq + k1 * (P + 1),
                               D2.Bq + k2 * (P + 1), D2.dBq + k2 * (P + 1));
        if (A.xy) {
            A.xy[2 * t] = D1.xq[k1];
            A.xy[2 * t + 1] = D2.xq[k2];
        }
    } else if (t < A.nq + A.nb) {
        constexpr int ng = (P + 1) * (P + 1);
        const int64_t u = t - A.nq;
        const int b = (int)(u / ng), g = (int)(u % ng), g1 = g % (P + 1), g2 = g / (P + 1);
        const int e = A.band_list[b], e1 = e % D1.N, e2 = e / D1.N;
        const int r1 = (e1 * (P + 1) + g1) * (P + 1), r2 = (e2 * (P + 1) + g2) * (P + 1);
        A.c_band[u] = detj_local(A.cp, A.n1, P, e1, e2, D1.Bg + r1, D1.dBg + r1, D2.Bg + r2, D2.dBg + r2);
        if (A.xy) {
            A.xy[2 * t] = D1.xg[e1 * (P + 1) + g1];
            A.xy[2 * t + 1] = D2.xg[e2 * (P + 1) + g2];
        }
    } else if (t < A.nq + A.nb + A.n_nodes) {
        const int64_t u = t - A.nq - A.nb;
        const int e = A.cut_list[A.node_el[u]], e1 = e % D1.N, e2 = e / D1.N;
        double B1[P + 1], dB1[P + 1], B2[P + 1], dB2[P + 1];
        basis_eval_d<P>(D1.knots, P + e1, A.nx[u], B1, dB1);
        basis_eval_d<P>(D2.knots, P + e2, A.ny[u], B2, dB2);
        A.c_cut[u] = detj_local(A.cp, A.n1, P, e1, e2, B1, dB1, B2, dB2);
    }
}

// |det J| on the WQ grid, sum-factorised. A tile is a strip of kCgPts
// points along xi_1 (one per thread, one wavefront) by a band of kCgBand
// elements along xi_2. The band's control rows (for the strip's columns) and
// its grid rows' B2, dB2 are staged in LDS with all loads in flight at once;
// each thread then contracts every control row once with its point's B1 and
// dB1 (x, y and their xi_1 derivatives along the row), keeps the p+1 rows of
// the current element in registers, and forms the four partial derivatives
// at each grid row of the element with B2, dB2: 4(p+1) multiply-adds per
// point instead of 4(p+1)^2, and the same sums in the same order as
// detj_local.
constexpr int kCgPts = 64;    // points (threads) per tile along xi_1
constexpr int kCgBand = 8;    // elements per tile along xi_2
constexpr int kCgCols = kCgPts / 2 + IGA_MAXP + 2;          // control columns of a strip, at most
constexpr int kCgCrows = kCgBand + IGA_MAXP;                // control rows of a band, at most
constexpr int kCgRows = 2 * kCgBand + 2 * IGA_MAXP;         // grid rows of a band, at most

__host__ __device__ inline int coef_grid_tiles(int Q1, int N2) {
    return ((Q1 + kCgPts - 1) / kCgPts) * ((N2 + kCgBand - 1) / kCgBand);
}

template <int P>
struct CoefGridSmem {
    double sP[kCgBand + P][2 * kCgCols];
    double sB2[kCgRows][P + 1], sdB2[kCgRows][P + 1];
};

template <int P>
__device__ __forceinline__ void coef_grid_body(const CoefArgs& A, int tile, CoefGridSmem<P>& S) {
    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    const int nsx = (D1.Q + kCgPts - 1) / kCgPts;
    const int sx = tile % nsx, bz = tile / nsx;
    const int E0 = bz * kCgBand, E1 = min(D2.N, E0 + kCgBand);
    const int t = threadIdx.x, nt = blockDim.x;
    const int kfirst = sx * kCgPts, klast = min(D1.Q, kfirst + kCgPts) - 1;
    const bool on = kfirst + t <= klast;
    const int k1 = on ? kfirst + t : klast;
    const int jA = D1.eq[kfirst], ncol = D1.eq[klast] + P + 1 - jA;
    const int e1l = D1.eq[k1] - jA;
    double B1[P + 1], dB1[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        B1[a] = D1.Bq[(size_t)k1 * (P + 1) + a];
        dB1[a] = D1.dBq[(size_t)k1 * (P + 1) + a];
    }
    const int KA2 = D2.pt0[E0], KB2 = D2.pt0[E1];
    for (int r = t; r < (KB2 - KA2) * (P + 1); r += nt) {
        const int k2 = KA2 + r / (P + 1), b = r % (P + 1);
        S.sB2[r / (P + 1)][b] = D2.Bq[(size_t)k2 * (P + 1) + b];
        S.sdB2[r / (P + 1)][b] = D2.dBq[(size_t)k2 * (P + 1) + b];
    }
    // control rows E0 .. E1+p-1, columns jA .. jA+ncol-1 (x and y interleaved)
    const int nrow = E1 - E0 + P;
    for (int c = t; c < nrow * 2 * ncol; c += nt) {
        const int j = c / (2 * ncol), q = c % (2 * ncol);
        S.sP[j][q] = A.cp[2 * ((size_t)(E0 + j) * A.n1 + jA) + q];
    }
    __syncthreads();
    // (sum_a1 B1 x, B1 y, dB1 x, dB1 y) of control row E0 + j
    auto t_row = [&](int j, double (&o)[4]) {
        double sx = 0.0, sy = 0.0, sx1 = 0.0, sy1 = 0.0;
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            const double px = S.sP[j][2 * (e1l + a)], py = S.sP[j][2 * (e1l + a) + 1];
            sx1 += dB1[a] * px;
            sx += B1[a] * px;
            sy1 += dB1[a] * py;
            sy += B1[a] * py;
        }
        o[0] = sx;
        o[1] = sy;
        o[2] = sx1;
        o[3] = sy1;
    };
    double T[P + 1][4];   // control rows e2 .. e2+p of the current element
#pragma unroll
    for (int j = 0; j < P; ++j) t_row(j, T[j]);
    for (int e2 = E0; e2 < E1; ++e2) {
        t_row(e2 - E0 + P, T[P]);
        for (int k2 = D2.pt0[e2]; k2 < D2.pt0[e2 + 1]; ++k2) {
            const int r = k2 - KA2;
            double x1 = 0.0, y1 = 0.0, x2 = 0.0, y2 = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                x1 += S.sB2[r][b] * T[b][2];
                y1 += S.sB2[r][b] * T[b][3];
                x2 += S.sdB2[r][b] * T[b][0];
                y2 += S.sdB2[r][b] * T[b][1];
            }
            if (on) {
                const size_t pt = (size_t)k2 * D1.Q + k1;
                A.c_wq[pt] = fabs(x1 * y2 - x2 * y1);
                if (A.xy) {
                    A.xy[2 * pt] = D1.xq[k1];
                    A.xy[2 * pt + 1] = D2.xq[k2];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < P; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) T[b][q] = T[b + 1][q];
    }
}

// ------------------------------------------------------------ interior rows
struct IntArgs {
    DirDev d1, d2;
    CoefView c;
    const double* cwq;       // coefficient on the WQ grid (nullptr -> constant c.value)
    const int8_t* fcls;
    const int* act_of;
    int all_active;          // 1: every active row (naive WQ), 0: interior rows only
    double* vals;
    int64_t n_act;
    int ntx;                 // tiles along xi_1 (interior2_ntx)
};

// Workgroups are handed to the XCDs round-robin; renumber them so that each
// XCD works on a contiguous range of rows (neighbouring rows share most of
// their coefficient points, which then stay in that XCD's L2).
__device__ __forceinline__ int xcd_block(int bid, int nb) {
    const int q = nb >> 3, r = nb & 7, x = bid & 7;
    return x * q + min(x, r) + (bid >> 3);
}

// One column b of one interior row. Tk points at T[b] for the row's
// first support point. A row touching no end element: 2p+2 points, two per
// element m, factors wbf(q, al) = (w1 B1) at point q for column m + al.
template <int P, typename WBF>
__device__ __forceinline__ void interior_col_reg(WBF wbf, const double* Tk, double* acc) {
#pragma unroll
    for (int a = 0; a < 2 * P + 1; ++a) acc[a] = 0.0;
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        const double t0 = Tk[2 * m], t1 = Tk[2 * m + 1];
#pragma unroll
        for (int al = 0; al <= P; ++al) acc[m + al] += wbf(2 * m, al) * t0 + wbf(2 * m + 1, al) * t1;
    }
}

// A row touching the first or last element: its q1 support points, full
// factor rows wb[q][a] = (w1 B1) at point q for column a.
// The factors are read a few points at a time before they are used (they
// may come from global memory); the sums run over q in order either way.
template <int P>
__device__ __forceinline__ void interior_col_end(const double* wb, const double* Tk, int q1, double* acc) {
    constexpr int W = 2 * P + 1, QB = 2;
#pragma unroll
    for (int a = 0; a < W; ++a) acc[a] = 0.0;
#pragma unroll 1
    for (int q0 = 0; q0 < q1; q0 += QB) {
        double f[QB][W], t[QB];
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int q = min(q0 + u, q1 - 1);
            t[u] = Tk[q];
#pragma unroll
            for (int a = 0; a < W; ++a) f[u][a] = wb[q * W + a];
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            if (q0 + u >= q1) break;
#pragma unroll
            for (int a = 0; a < W; ++a) acc[a] += f[u][a] * t[u];
        }
    }
}

// Interior rows (the one-patch kernel and the batched launches). Per test row i2: tiles of up to R
// consecutive "regular" test rows i1 (p+1 <= i1 <= N1-2, two WQ points in
// every support element), each row's 2p+1 columns b dealt round-robin to NB
// threads (R * NB threads per workgroup: enough waves in flight to cover the
// memory latency), and one workgroup for the 2(p+1) end rows (supports
// touching the first or last element, p+1 points there), one thread per
// (end row, column b). Stage 1 contracts xi_2 for every xi_1
// point of the workgroup's window into T[b][k] (LDS); stage 2 contracts xi_1,
// M[a][b] = sum_k (w1 B1)[i1][k][a] T[b][k], per column. A regular row's
// banded w1 B1 factors are loaded into
// registers (p <= 5) together with every other global load of the
// workgroup, before stage 1; the end rows' full factor rows go to LDS.
// For p >= 6 the factors do not fit in registers: each is formed where it
// is used, from the row's weights (registers) and the window's basis values
// (LDS), the same product as the precomputed table.
// Rows per tile and column groups per row, measured: whole rows per thread
// are fastest for p <= 5; for p >= 6 the columns of a row dealt to four
// threads.
__host__ __device__ constexpr int interior2_rows(int p) { return p <= 5 ? 128 : 64; }
__host__ __device__ constexpr int interior2_groups(int p) { return p <= 5 ? 1 : 4; }
template <int P>
struct Int2Cfg {
    static constexpr int W = 2 * P + 1;                  // band width
    static constexpr int QM = 4 * P + 2;                 // max WQ points in one support
    static constexpr int NR = 2 * P + 2;                 // support points of a regular function
    static constexpr int R = interior2_rows(P);          // rows per tile
    static constexpr int NB = interior2_groups(P);       // column groups: the row's columns b = g, g+NB, ...
    static constexpr int NT = R * NB;                    // threads per workgroup
    static constexpr int KS = 2 * (R + P) + 2 * P + 2;   // max xi_1 points of a tile window
    static constexpr int NJ = (KS + NT - 1) / NT;        // window points per thread
    static constexpr int NG = P + 1;                     // end rows at each end
    static constexpr bool PRE = (P <= 5);                // factors and coefficients preloaded in registers
};

// A regular tile's window, or the end-row workgroup's two short windows
// (at most 6p+2 points) with the end rows' factor rows: they share LDS.
template <int P>
struct Int2Smem {
    using C = Int2Cfg<P>;
    static constexpr int KSE = 6 * P + 2;
    union {
        struct {
            double sT[C::W][C::KS];
            double sB[C::KS * (P + 1)];  // basis values B[k][al] at the window's points
        } r;
        struct {
            double sT[C::W][KSE];
            double sG[2 * C::NG][C::QM][C::W];  // w1 B1 rows of the end rows
        } e;
    };
    double sWB2[C::QM][C::W];
};

// Workgroups per test row i2: the regular tiles, then the end-row workgroup.
__host__ __device__ inline int interior2_nreg(int N1, int p) {
    const int R = interior2_rows(p);
    return (N1 >= p + 3) ? ((N1 - 2) - (p + 1) + 1 + R - 1) / R : 0;
}
__host__ __device__ inline int interior2_ntx(int N1, int p) { return interior2_nreg(N1, p) + 1; }

// End row g of a test row (first p+1 rows, then the rows from N1-1 on; -1 if none).
template <int P>
__device__ __forceinline__ int interior_end_row(int g, int N1, int n1) {
    if (g < P + 1) return (g < n1) ? g : -1;
    const int r = N1 - 1 + (g - (P + 1));
    return (r < n1 && r > P) ? r : -1;
}

template <int P>
__device__ __forceinline__ void interior_rows_block(const IntArgs& A, int tx, int i2, Int2Smem<P>& S) {
    using C = Int2Cfg<P>;
    constexpr int W = C::W, QM = C::QM, NR = C::NR, R = C::R, NB = C::NB, NT = C::NT, NJ = C::NJ, NG = C::NG;
    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    const int tid = threadIdx.x;
    const int rl = tid % R, grp = tid / R;  // the thread's row in the tile and column group
    if (i2 >= D2.n) return;
    const int nreg = interior2_nreg(D1.N, P);
    const bool endtile = tx >= nreg;
    const int k2lo = wq_pt0(max(0, i2 - P), D2.N, P);
    const int q2 = wq_pt0(min(D2.N - 1, i2) + 1, D2.N, P) - k2lo;
    const bool reg_row = (i2 >= P + 1) && (i2 <= D2.N - 2);  // q2 == NR, two points per element

    // ---- the workgroup's window of xi_1 points: one range, or (end rows) two
    int I1 = 0, nlive = 0, wlo1 = 0, whi1 = 0, wlo2 = 0, whi2 = 0;
    if (!endtile) {
        I1 = (P + 1) + tx * R;
        nlive = min(R, (D1.N - 2) - I1 + 1);
        wlo1 = wq_pt0(I1 - P, D1.N, P);
        whi1 = wq_pt0(I1 + nlive - 1 + 1, D1.N, P);
    } else {
        whi1 = wq_pt0(min(P + 1, D1.N), D1.N, P);
        wlo2 = wq_pt0(max(0, D1.N - 1 - P), D1.N, P);
        whi2 = D1.Q;
        if (wlo2 <= whi1) {  // the two ranges meet: one window
            whi1 = D1.Q;
            wlo2 = whi2 = D1.Q;
        }
    }
    const int ks = (whi1 - wlo1) + (whi2 - wlo2);
    auto kglob = [&](int k) { return (k < whi1 - wlo1) ? wlo1 + k : wlo2 + (k - (whi1 - wlo1)); };
    auto kloc = [&](int kg) { return (kg < whi1) ? kg - wlo1 : (whi1 - wlo1) + (kg - wlo2); };

    // ---- loads: row identity, xi_2 factors, coefficient columns, the rows' w1 B1 factors
    auto formed = [&](int8_t cls) { return A.all_active ? (cls != FN_EXTERIOR) : (cls == FN_INTERIOR); };
    int i1 = -1;
    bool live = false;
    int64_t cid = 0;
    if (!endtile) {
        if (rl < nlive) {
            i1 = I1 + rl;
            const int f = i2 * D1.n + i1;
            const int8_t cls = A.fcls[f];
            cid = A.act_of[f];
            live = formed(cls);
        }
    } else {  // any of this thread's (end row, column) pairs formed here
        for (int t = tid; t < 2 * NG * W; t += NT) {
            const int ie = interior_end_row<P>(t / W, D1.N, D1.n);
            if (ie >= 0 && formed(A.fcls[i2 * D1.n + ie])) live = true;
        }
    }
    // (loads are unconditional, at clamped in-range addresses, and selected
    // afterwards: one batch of independent loads instead of a branch each)
    constexpr int NWB = (QM * W + NT - 1) / NT;
    double wb2[NWB];
#pragma unroll
    for (int u = 0; u < NWB; ++u) {
        const int t = tid + NT * u;
        const double v = D2.WB[(size_t)i2 * D2.qmax * W + min(t, q2 * W - 1)];
        wb2[u] = (t < q2 * W) ? v : 0.0;
    }
    double cv[C::PRE ? NJ : 1][NR];
    if (C::PRE && reg_row) {
        if (A.cwq) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int kg = kglob(min(tid + NT * j, ks - 1));
#pragma unroll
                for (int q = 0; q < NR; ++q) cv[C::PRE ? j : 0][q] = A.cwq[(size_t)(k2lo + q) * D1.Q + kg];
            }
        } else {
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int q = 0; q < NR; ++q) cv[C::PRE ? j : 0][q] = A.c.value;
        }
    }
    // A regular row's factors w1 B1 (the banded copy's values) are formed
    // in registers from its weights (rows contiguous) and the window's basis
    // values (staged once per workgroup): one product each, as in the table.
    double wt[NR];
    if (!endtile && i1 >= 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q) wt[q] = D1.WT[(size_t)q * D1.n + i1];
    }
    constexpr int NBQ = (C::KS * (P + 1) + NT - 1) / NT;
    double bq[NBQ];
    const int nbq = ks * (P + 1);
    if (!endtile) {
#pragma unroll
        for (int u = 0; u < NBQ; ++u) bq[u] = D1.Bq[(size_t)wlo1 * (P + 1) + min(tid + NT * u, nbq - 1)];
    }
    if (endtile) {  // the end rows' full w1 B1 rows, in batches of independent loads
        constexpr int NGT = 2 * NG * QM * W, NBAT = 16;
        double* sg = &S.e.sG[0][0][0];
#pragma unroll 1
        for (int t0 = 0; t0 < NGT; t0 += NT * NBAT) {
            double gv[NBAT];
#pragma unroll
            for (int u = 0; u < NBAT; ++u) {
                const int t = t0 + tid + NT * u;
                const int g = t / (QM * W), q = (t / W) % QM, a = t % W;
                const int ie = (t < NGT) ? interior_end_row<P>(g, D1.N, D1.n) : -1;
                const double v = D1.WB[((size_t)max(ie, 0) * D1.qmax + min(q, D1.qmax - 1)) * W + a];
                gv[u] = (ie >= 0 && q < D1.qmax) ? v : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NBAT; ++u) {
                const int t = t0 + tid + NT * u;
                if (t < NGT) sg[t] = gv[u];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NWB; ++u) {
        const int t = tid + NT * u;
        if (t < QM * W) S.sWB2[t / W][t % W] = wb2[u];
    }
    if (!endtile) {
#pragma unroll
        for (int u = 0; u < NBQ; ++u)
            if (tid + NT * u < nbq) S.r.sB[tid + NT * u] = bq[u];
    }
    if (!__syncthreads_or(live)) return;  // no row of the workgroup is formed here

    // ---- stage 1: contract xi_2 for every xi_1 point of the window
    double* sTb = endtile ? &S.e.sT[0][0] : &S.r.sT[0][0];
    const int kst = endtile ? Int2Smem<P>::KSE : C::KS;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = tid + NT * j;
        if (k >= ks) break;
        const int kg = kglob(k);
        if (reg_row) {
            double cr[C::PRE ? 1 : NR];
            if (!C::PRE) {
                if (A.cwq) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) cr[C::PRE ? 0 : q] = A.cwq[(size_t)(k2lo + q) * D1.Q + kg];
                } else {
#pragma unroll
                    for (int q = 0; q < NR; ++q) cr[C::PRE ? 0 : q] = A.c.value;
                }
            }
            double T[W];
#pragma unroll
            for (int b = 0; b < W; ++b) T[b] = 0.0;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const int m2 = q >> 1;
                const double cq = C::PRE ? cv[C::PRE ? j : 0][q] : cr[C::PRE ? 0 : q];
#pragma unroll
                for (int bl = 0; bl <= P; ++bl) T[m2 + bl] += S.sWB2[q][m2 + bl] * cq;
            }
#pragma unroll
            for (int b = 0; b < W; ++b) sTb[b * kst + k] = T[b];
        } else {
            double c[QM];
            if (A.cwq) {
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    const double v = A.cwq[(size_t)(k2lo + min(q, q2 - 1)) * D1.Q + kg];
                    c[q] = (q < q2) ? v : 0.0;
                }
            } else {
#pragma unroll
                for (int q = 0; q < QM; ++q) c[q] = (q < q2) ? A.c.value : 0.0;
            }
#pragma unroll 1
            for (int b = 0; b < W; ++b) {
                double Tb = 0.0;
#pragma unroll
                for (int q = 0; q < QM; ++q) Tb += S.sWB2[q][b] * c[q];
                sTb[b * kst + k] = Tb;
            }
        }
    }
    __syncthreads();
    if (!live) return;

    // ---- stage 2: contract xi_1
    if (!endtile) {  // this thread's columns of its row
        const int k0 = kloc(wq_pt0(max(0, i1 - P), D1.N, P));  // the row's first support point
        double wb[C::PRE ? NR : 1][P + 1];
        if (C::PRE) {
#pragma unroll
            for (int q = 0; q < NR; ++q)
#pragma unroll
                for (int al = 0; al <= P; ++al)
                    wb[C::PRE ? q : 0][al] = wt[q] * S.r.sB[(k0 + q) * (P + 1) + al];
        }
#pragma unroll 1
        for (int b = grp; b < W; b += NB) {
            double acc[W];
            if constexpr (C::PRE)
                interior_col_reg<P>([&](int q, int al) { return wb[q][al]; }, &S.r.sT[b][k0], acc);
            else
                interior_col_reg<P>([&](int q, int al) { return wt[q] * S.r.sB[(k0 + q) * (P + 1) + al]; },
                                    &S.r.sT[b][k0], acc);
#pragma unroll
            for (int a = 0; a < W; ++a) A.vals[band_index(a * W + b, W * W, cid, A.n_act)] = acc[a];
        }
    } else {  // one column of an end row per pair
        for (int t = tid; t < 2 * NG * W; t += NT) {
            const int g = t / W, bcol = t % W;
            const int ie = interior_end_row<P>(g, D1.N, D1.n);
            if (ie < 0) continue;
            const int f = i2 * D1.n + ie;
            if (!formed(A.fcls[f])) continue;
            const int64_t cide = A.act_of[f];
            const int kg0 = wq_pt0(max(0, ie - P), D1.N, P);
            const int q1 = wq_pt0(min(D1.N - 1, ie) + 1, D1.N, P) - kg0;
            double acc[W];
            interior_col_end<P>(&S.e.sG[g][0][0], &S.e.sT[bcol][kloc(kg0)], q1, acc);
#pragma unroll
            for (int a = 0; a < W; ++a) A.vals[band_index(a * W + bcol, W * W, cide, A.n_act)] = acc[a];
        }
    }
}

// ------------------------------------------------------------ cut element matrices
struct CutEArgs {
    DirDev d1, d2;
    CoefView c;
    const int* cut_list;  // flat id of each cut element (as the cut-rule kernel found it)
    const int* node_off;
    const double *nx, *ny, *nw;
    double* E;
    int n_cut;
    // c = |det J| of the geometry map: evaluated at the nodes here (and stored in c_cut)
    int detj;
    const double* geom_cp;
    int n1;
    double* c_cut;
};

template <int P>
struct CutECfg {
    static constexpr int L = (P + 1) * (P + 1);
    static constexpr int CH = (P == 1) ? 256 : ((P <= 6) ? 128 : 64);  // nodes staged at a time (LDS kept small)
    static constexpr int NR = P * (P + 1) / 2;                          // reciprocal denominators per direction
    static constexpr int T = (L + 15) / 16;                             // 16-wide blocks of the local basis
    static constexpr int NT = T * (T + 1) / 2;                          // 16 x 16 tiles of the upper triangle
    static constexpr int KS = (NT == 1) ? 4 : 1;                        // wavefronts sharing one tile's nodes
    static constexpr int TPW = (NT + 3) / 4;                            // tiles per wavefront (KS == 1)
};

template <int P>
struct CutESmem {
    double sPhi[CutECfg<P>::CH][CutECfg<P>::L];
    double sWc[CutECfg<P>::CH];
    double sRec[2][CutECfg<P>::NR + 1];
    double sCp[(P + 1) * (P + 1)][2];  // the element's geometry control points (c = |det J|)
};

typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

// Upper-triangle tile t -> block row I <= block column J (row-major).
__device__ __forceinline__ void tile_ij(int t, int T, int& I, int& J) {
    I = 0;
    while (t >= T - I) {
        t -= T - I;
        ++I;
    }
    J = I + t;
}

// Local matrix of cut element c (256 threads): E = sum_n w_n c_n phi_n phi_n^T
// over the element's nodes, a Gram product contracted on the matrix cores.
// With c = |det J| the node's thread evaluates c too, from the element's
// control points staged in LDS, and stores it in the rule-point table.
// Nodes are staged CH at a time with their basis products (one node per
// thread, the element's reciprocal knot differences shared, so no divisions
// per node). The L x L result is cut into 16 x 16 tiles of its upper
// triangle; each MFMA step (v_mfma_f64_16x16x4) takes four nodes, lane l
// holding phi at node l / 16 for basis 16 I + l % 16 (times w c for the row
// operand) and basis 16 J + l % 16 for the column operand. With one tile
// (p <= 3) the four wavefronts split the nodes and add their partial tiles
// in a fixed order; otherwise the wavefronts split the tiles. The lower
// triangle is the mirror of the upper one.
template <int P>
__device__ __forceinline__ void cut_elem_body(const CutEArgs& A, int c, CutESmem<P>& S) {
    using C = CutECfg<P>;
    constexpr int L = C::L, CH = C::CH, NR = C::NR, T = C::T, NT = C::NT, KS = C::KS, TPW = C::TPW;
    static_assert(CH % 4 == 0, "nodes are contracted four at a time");
    static_assert(KS == 1 || sizeof(S.sPhi) >= 4 * 256 * sizeof(double), "partial tiles reuse the node stage");
    auto& sPhi = S.sPhi;
    auto& sWc = S.sWc;
    if (c >= A.n_cut) return;
    const int e = A.cut_list[c], e1 = e % A.d1.N, e2 = e / A.d1.N;
    const int nb = A.node_off[c], ne = A.node_off[c + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, col = lane & 15;      // node within a step, basis within a block
    int tI[TPW], tJ[TPW];
    bool tOn[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = (KS == 1) ? wave + 4 * u : 0;
        tOn[u] = t < NT;
        tile_ij(tOn[u] ? t : 0, T, tI[u], tJ[u]);
    }
    mfma_f64x4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};

    __syncthreads();  // LDS of the previous work item is free
    if (threadIdx.x < 2 * NR) {
        const int d = threadIdx.x / NR, idx = threadIdx.x % NR;
        S.sRec[d][idx] = basis_rec<P>(d ? A.d2.knots : A.d1.knots, P + (d ? e2 : e1), idx);
    } else if (A.detj && threadIdx.x < 2 * NR + (P + 1) * (P + 1)) {
        const int t = threadIdx.x - 2 * NR, a2 = t / (P + 1), a1 = t % (P + 1);
        const double* q = A.geom_cp + 2 * ((size_t)(e2 + a2) * A.n1 + e1 + a1);
        S.sCp[t][0] = q[0];
        S.sCp[t][1] = q[1];
    }
    // this thread's node of the next chunk, loaded while the current chunk is contracted
    double nxv = 0.0, nyv = 0.0, nwv = 0.0, ncv = 0.0;
    auto prefetch = [&](int base) {
        const int n = base + threadIdx.x;
        if (threadIdx.x < CH && n < ne) {
            nxv = A.nx[n];
            nyv = A.ny[n];
            nwv = A.nw[n];
            if (!A.detj && !A.c.is_const) ncv = A.c.cut[n];
        }
    };
    prefetch(nb);
    for (int base = nb; base < ne; base += CH) {
        __syncthreads();
        if (threadIdx.x < CH) {
            const int n = base + threadIdx.x;
            if (n < ne) {
                const double x = nxv, y = nyv, w = nwv;
                double cv;
                double B1[P + 1], B2[P + 1];
                if (A.detj) {  // |det J| from the staged control points (the sums of detj_local)
                    double dB1[P + 1], dB2[P + 1];
                    basis_eval_rec_d<P>(A.d1.knots, P + e1, S.sRec[0], x, B1, dB1);
                    basis_eval_rec_d<P>(A.d2.knots, P + e2, S.sRec[1], y, B2, dB2);
                    double x1 = 0.0, x2 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll
                    for (int a2 = 0; a2 <= P; ++a2) {
                        double sx1 = 0.0, sx = 0.0, sy1 = 0.0, sy = 0.0;
#pragma unroll
                        for (int a1 = 0; a1 <= P; ++a1) {
                            const double px = S.sCp[a2 * (P + 1) + a1][0], py = S.sCp[a2 * (P + 1) + a1][1];
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
                    cv = fabs(x1 * y2 - x2 * y1);
                    A.c_cut[n] = cv;
                } else {
                    cv = A.c.is_const ? A.c.value : ncv;
                    basis_eval_rec<P>(A.d1.knots, P + e1, S.sRec[0], x, B1);
                    basis_eval_rec<P>(A.d2.knots, P + e2, S.sRec[1], y, B2);
                }
#pragma unroll
                for (int a2 = 0; a2 <= P; ++a2)
#pragma unroll
                    for (int a1 = 0; a1 <= P; ++a1) sPhi[threadIdx.x][a2 * (P + 1) + a1] = B1[a1] * B2[a2];
                sWc[threadIdx.x] = w * cv;
            } else {  // rows past the last node contribute zero
                sWc[threadIdx.x] = 0.0;
#pragma unroll
                for (int l = 0; l < L; ++l) sPhi[threadIdx.x][l] = 0.0;
            }
        }
        __syncthreads();
        prefetch(base + CH);
        if (KS == 1 && wave >= NT) continue;
        const int nsteps = (min(CH, ne - base) + 3) >> 2;
        for (int k = (KS == 1) ? 0 : wave; k < nsteps; k += KS) {
            const int n = 4 * k + kq;
            const double wc = sWc[n];
            double ph[T];
#pragma unroll
            for (int J = 0; J < T; ++J) {
                const int l = 16 * J + col;
                const double v = sPhi[n][l < L ? l : 0];
                ph[J] = (l < L) ? v : 0.0;
            }
#pragma unroll
            for (int u = 0; u < TPW; ++u)
                if (tOn[u]) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc * ph[tI[u]], ph[tJ[u]], acc[u], 0, 0, 0);
        }
    }
    double* E = A.E + (size_t)c * L * L;
    if constexpr (KS == 1) {
        // accumulator element v of lane l is row l / 16 + 4 v, column l % 16 of the tile
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (!tOn[u]) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * tI[u] + kq + 4 * v, q = 16 * tJ[u] + col;
                if (r < L && q < L && r <= q) {
                    E[r * L + q] = acc[u][v];
                    E[q * L + r] = acc[u][v];
                }
            }
        }
    } else {
        double (*sRed)[256] = reinterpret_cast<double (*)[256]>(&sPhi[0][0]);
        __syncthreads();  // every wavefront is done with the node stage
#pragma unroll
        for (int v = 0; v < 4; ++v) sRed[wave][lane * 4 + v] = acc[0][v];
        __syncthreads();
        const int ln = threadIdx.x >> 2, v = threadIdx.x & 3;
        const int r = (ln >> 4) + 4 * v, q = ln & 15;
        if (r < L && q < L && r <= q) {
            const double sum = ((sRed[0][threadIdx.x] + sRed[1][threadIdx.x]) + sRed[2][threadIdx.x]) + sRed[3][threadIdx.x];
            E[r * L + q] = sum;
            E[q * L + r] = sum;
        }
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
    const int* region;      // DWQ: box of inside elements left to k_dwq_rows (nullptr: none)
    double* vals;
    int64_t n_act;
    double* part;           // two-launch form: [n_rows][(2p+1)^2] inside sums, row r's slots contiguous
    const double* boxp = nullptr;  // cut-entry launch of a DWQ plan: [n_rows][(2p+1)^2] box parts, added last
};

// One workgroup per row; the row's per-direction Gauss factors
// F1[m1][g1][a] = w_g1 B_i1 B_{i1+a-p} (element e1 = i1-p+m1), F2 likewise,
// the element classes, and per support element either c at its Gauss points
// (inside) or the row's line of its local matrix (cut) are staged in LDS.
// Inside elements are summed in two contractions: the workgroup first forms
// U[m2][g2][a] (direction 1, summed over the element columns m1), then thread
// (a, b) contracts U with F2 and adds its column's entries of the cut element
// matrices. The row can also be formed in two launches with the same
// arithmetic: the inside sum (to a scratch array, the row's slots side by
// side), then the cut entries (added, and the row written to the band
// layout). A row's slots lie n_act apart in the band layout, so the scratch
// array spares the second launch a read of one cache line per slot. A DWQ
// row's box part, formed into a second scratch array beforehand, is added
// last there, as the box launch would add it to the written row.
enum : int { ROW_FUSED = 0, ROW_INSIDE = 1, ROW_CUT = 2 };

template <int P>
struct CutRSmem {
    double sF1[P + 1][P + 1][2 * P + 1];
    double sF2[P + 1][P + 1][2 * P + 1];
    double sXE[P + 1][P + 1][(P + 1) * (P + 1)];  // inside: c at its Gauss points; cut: its local matrix line
    double sU[P + 1][P + 1][2 * P + 1];           // direction-1 contraction, summed over m1
    int sCls[P + 1][P + 1];
    int sId[P + 1][P + 1];
};

template <int P, int MODE>
__device__ __forceinline__ void cut_row_body_m(const CutRowArgs& A, int r, CutRSmem<P>& S) {
    constexpr int W = 2 * P + 1, L = (P + 1) * (P + 1), NP = P + 1;
    constexpr bool INS = (MODE != ROW_CUT), CUT = (MODE != ROW_INSIDE);
    auto& sF1 = S.sF1;
    auto& sF2 = S.sF2;
    auto& sXE = S.sXE;
    auto& sCls = S.sCls;
    auto& sId = S.sId;
    if (r >= A.n_rows) return;
    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int row = A.rows[r];
    const int f = A.fn_of[row];
    const int i1 = f % D1.n, i2 = f / D1.n;
    int bx0 = 1, bx1 = 0, by0 = 1, by1 = 0;   // DWQ box (empty by default)
    if (INS && A.region && A.region[(size_t)r * 8] >= 0) {
        bx0 = A.region[(size_t)r * 8];
        bx1 = A.region[(size_t)r * 8 + 1];
        by0 = A.region[(size_t)r * 8 + 4];
        by1 = A.region[(size_t)r * 8 + 5];
    }
    if (INS) {
        for (int t = tid; t < NP * NP * W; t += nt) {
            int m = t / (NP * W), g = (t / W) % NP, a = t % W;
            // direction 1
            int e1 = i1 - P + m, j1 = i1 + a - P;
            double v = 0.0;
            if (e1 >= 0 && e1 < D1.N && j1 - e1 >= 0 && j1 - e1 <= P) {
                int rr = (e1 * NP + g) * NP;
                v = D1.wg[e1 * NP + g] * D1.Bg[rr + i1 - e1] * D1.Bg[rr + j1 - e1];
            }
            sF1[m][g][a] = v;
            int e2 = i2 - P + m, j2 = i2 + a - P;
            v = 0.0;
            if (e2 >= 0 && e2 < D2.N && j2 - e2 >= 0 && j2 - e2 <= P) {
                int rr = (e2 * NP + g) * NP;
                v = D2.wg[e2 * NP + g] * D2.Bg[rr + i2 - e2] * D2.Bg[rr + j2 - e2];
            }
            sF2[m][g][a] = v;
        }
    }
    for (int t = tid; t < NP * NP; t += nt) {
        int m2 = t / NP, m1 = t % NP;
        int e1 = i1 - P + m1, e2 = i2 - P + m2;
        int cls = -1, id = -1;
        if (e1 >= 0 && e1 < D1.N && e2 >= 0 && e2 < D2.N && !(e1 >= bx0 && e1 <= bx1 && e2 >= by0 && e2 <= by1)) {
            // every inside element of a formed row's support is a band element
            const int e = e2 * D1.N + e1;
            const int ci = A.cut_id[e], bi = A.band_id[e];
            cls = (ci >= 0) ? EL_CUT : (bi >= 0 ? EL_INSIDE : -1);
            id = (ci >= 0) ? ci : bi;
        }
        sCls[m2][m1] = cls;
        sId[m2][m1] = id;
    }
    __syncthreads();
    // per support element: c at its Gauss points (inside) or line i of its local matrix (cut)
    for (int t = tid; t < NP * NP * L; t += nt) {
        const int m2 = t / (NP * L), m1 = (t / L) % NP, g = t % L;
        const int cls = sCls[m2][m1];
        double v = 0.0;
        if (INS && cls == EL_INSIDE) v = A.c.is_const ? A.c.value : A.c.band[(size_t)sId[m2][m1] * L + g];
        else if (CUT && cls == EL_CUT) v = A.E[((size_t)sId[m2][m1] * L + (P - m2) * NP + (P - m1)) * L + g];
        sXE[m2][m1][g] = v;
    }
    __syncthreads();
    if (INS) {
        // inside elements, sum-factorised: F2 does not depend on m1, so the direction-1 contraction is
        // summed over the element columns first, U[m2][g2][a] = sum_m1 sum_g1 F1[m1][g1][a] X[m2][m1][g2][g1]
        for (int t = tid; t < NP * NP * W; t += nt) {
            const int m2 = t / (NP * W), g2 = (t / W) % NP, a = t % W;
            double u = 0.0;
#pragma unroll 1
            for (int m1 = 0; m1 <= P; ++m1) {
                const bool in = sCls[m2][m1] == EL_INSIDE;
#pragma unroll
                for (int g1 = 0; g1 < NP; ++g1) u += in ? sF1[m1][g1][a] * sXE[m2][m1][g2 * NP + g1] : 0.0;
            }
            S.sU[m2][g2][a] = u;
        }
        __syncthreads();
    }
    const int s = tid;
    if (s >= W * W) return;
    const int a = s / W, b = s % W;          // column offsets a-p, b-p
    const int j1 = i1 + a - P, j2 = i2 + b - P;
    double* out = A.vals + band_index(s, W * W, row, A.n_act);
    double val = 0.0;
    if (j1 >= 0 && j1 < D1.n && j2 >= 0 && j2 < D2.n && A.act_of[j2 * D1.n + j1] >= 0) {
        if (INS) {
#pragma unroll
            for (int m2 = 0; m2 <= P; ++m2)
#pragma unroll
                for (int g2 = 0; g2 < NP; ++g2) val += sF2[m2][g2][b] * S.sU[m2][g2][a];
        } else {
            val = A.part[band_index(r, A.n_rows, s, W * W)];   // the inside sum, written by the first launch
        }
        if (CUT) {
            // cut elements: the column's entry of the staged line, zero where the element is not cut
            // or does not overlap the column's support
#pragma unroll 1
            for (int m2 = 0; m2 <= P; ++m2) {
                const int l2 = j2 - (i2 - P + m2);
#pragma unroll
                for (int m1 = 0; m1 <= P; ++m1) {
                    const int l1 = j1 - (i1 - P + m1);
                    const bool ov = (l1 >= 0 && l1 <= P && l2 >= 0 && l2 <= P) && sCls[m2][m1] == EL_CUT;
                    const double ev = sXE[m2][m1][ov ? l2 * NP + l1 : 0];
                    val += ov ? ev : 0.0;
                }
            }
        }
        if (MODE == ROW_CUT && A.boxp && A.region[(size_t)r * 8] >= 0) val += A.boxp[(size_t)r * (W * W) + s];
    }
    if (MODE == ROW_INSIDE)
        A.part[band_index(r, A.n_rows, s, W * W)] = val;
    else
        *out = val;
}

template <int P>
__device__ __forceinline__ void cut_row_body(const CutRowArgs& A, int r, CutRSmem<P>& S) {
    cut_row_body_m<P, ROW_FUSED>(A, r, S);
}


IntArgs int_args(Plan& P, const iga_coeff& c, double* vals);
CutEArgs cute_args(Plan& P, const iga_coeff& c);
CutRowArgs cutr_args(Plan& P, const iga_coeff& c, double* vals);

}  // namespace iga
