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
};

__device__ __forceinline__ bool wq_row(const MfArgs& A, int8_t cls) {
    return A.method != IGA_GAUSS_REF && cls == FN_INTERIOR;
}

// The weighted-quadrature part as banded one-dimensional contractions (sum
// factorisation), fast index along xi_1:
//   V[j2][k1] = sum_a B1[k1][a] u(e1(k1) + a, j2)              (u on the xi_1 points)
//   G[k2][k1] = c_k sum_a B2[k2][a] V[e2(k2) + a][k1]          (c U along grid row k2)
//   H[k2][i1] = sum_q w1[i1][q] G[k2][k0(i1) + q]              (test rows along xi_1)
//   y(i1, i2) = sum_q w2[i2][q] H[k0(i2) + q][i1]              (interior rows)
// all four in one pass over the grid (k_mf_fwd), and, transposed, for the adjoint
//   Hr[k2][i1] = sum_{i2 : k2 in supp} w2[i2][k2 - k0(i2)] r(i1, i2)
//   R[k2][k1] = sum_{i1 : k1 in supp} w1[i1][k1 - k0(i1)] Hr[k2][i1],  dc = U R, c R
//   D[k2][j1] = sum_{k1 in supp j1} B1[k1][j1 - e1(k1)] c R[k2][k1]
//   du(j1, j2) += sum_{k2 in supp j2} B2[k2][j2 - e2(k2)] D[k2][j1]
// in one pass as well (k_mf_adj). None of V, G, H, U, R, c R or D leaves its workgroup.
// Forward weighted-quadrature part in one pass over the grid. A workgroup
// takes a strip of test columns i1 (one per thread) and a band of elements
// e2 (at least p+1 of them) and walks the band's grid rows k2 in order:
//   V[j2][k1] for a new u row (once per element; p+1 rows in a ring in LDS),
//   G[k1] = c_k sum_b B2[k2][b] V[e2(k2)+b][k1]   (the strip's points of row k2, LDS),
//   H(i1) = sum_q w1[i1][q] G[k0(i1)+q]            (registers),
//   acc[i2] += w2[i2][k2 - k0(i2)] H(i1)           for the p+1 rows i2 = e2..e2+p.
// Rows go two at a time with two barriers per pair: each element's rows
// take an even number of slots (a padding slot has B2 = w2 = 0), and the
// next element's V row is formed in the last pair of the current one, after
// its second barrier (its ring slot held row e2, which that pair's G was the
// last to read). When element e2 ends, row e2 has all of this band's terms:
// it is written to y if its support lies in the band (or starts at the patch
// edge), otherwise as the band's head part of that row; the p rows after the
// band are written as its tail part, and k_mf_fix adds a band's head to the
// previous band's tail. The point layout is the closed form of the WQ rule
// (p+1 points in the first and last element, 2 elsewhere), so the slot table
// needs no loads; c rows are loaded two pairs ahead and u rows one element
// ahead (their active ids two), and no load in the loop waits on a later-
// issued one. c is read once; V and H never leave the workgroup.
constexpr int kMfThreads = 128;  // threads = test columns per strip (at most)
constexpr int kMfNpt = 2;        // xi_1 points per thread (a strip has at most 2 (cols + p) + 2 (p - 1))
constexpr int kMfUpt = 2;        // u columns per thread (cols + 2p)
constexpr int kMfBand = 8;       // elements per band, at least p+1 (the last band takes the remainder)
constexpr int kMfBandMax = kMfBand > IGA_MAXP + 1 ? kMfBand : IGA_MAXP + 1;
// slots of a band: its rows, one padding slot per end element of odd row count, padding to 4 slots
constexpr int kMfSlots = 2 * (2 * kMfBandMax - 1) + 2 * IGA_MAXP + 2 + 4;

struct MfFwdArgs {
    int cols;     // test columns per strip
    int band;     // elements per band (the last band takes the remainder)
    int nstrip, nband;
    double* head; // [nband][p][n1]
    double* tail; // [nband][p][n1]
};

// LDS of one forward workgroup of the grid part.
template <int P>
struct MfFwdSmem {
    static constexpr int NP = kMfThreads * kMfNpt, QM = 4 * P + 2, NU = kMfThreads * kMfUpt;
    static constexpr int NG = NP + QM;   // the column sums read up to 4p+1 points past a strip's last one
    // G of a row with even and odd points apart: the column sums read points k0(i1) + q, and k0
    // steps by 2 from one column to the next, so each half is read with unit stride (no bank conflicts)
    static constexpr int NGH = (NG + 1) / 2;
    double sU[P + 1][NU];  // the first p+1 u rows; then rows alternate in sU[0], sU[1]
    double sV[P + 1][NP];
    double sG[2][2 * NGH];
    double sB2[kMfSlots][P + 1], sW2[kMfSlots][P + 1];
    int sK2[kMfSlots];
};

// Workgroup blk (strip blk % nstrip, band blk / nstrip) of the forward grid part.
template <int P>
__device__ __forceinline__ void mf_fwd_body(const MfArgs& A, const MfFwdArgs& F, int blk,
                                            const double* __restrict__ u, double* __restrict__ y, MfFwdSmem<P>& SM) {
    constexpr int NP = MfFwdSmem<P>::NP, NW = 2 * P + 2, QM = MfFwdSmem<P>::QM, NU = MfFwdSmem<P>::NU;
    constexpr int NG = MfFwdSmem<P>::NG, NGH = MfFwdSmem<P>::NGH;
    auto gi = [](int k) { return (k & 1) * NGH + (k >> 1); };
    auto& sU = SM.sU;
    auto& sV = SM.sV;
    auto& sG = SM.sG;
    auto& sB2 = SM.sB2;
    auto& sW2 = SM.sW2;
    auto& sK2 = SM.sK2;
    const int tid = threadIdx.x;
    const int strip = blk % F.nstrip, bnd = blk / F.nstrip;
    const int n1 = A.n1, N1 = A.N1, N2 = A.N2, Q1 = A.d1.Q;
    const int c0 = strip * F.cols, c1 = min(n1, c0 + F.cols);
    const int E0 = bnd * F.band, E1 = (bnd == F.nband - 1) ? N2 : E0 + F.band, NE = E1 - E0;
    const int jA = max(0, c0 - P), jB = min(N1 - 1, c1 - 1) + P + 1;
    // Every load in the loop is unconditional (clamped address) and its value
    // is selected where it is used: a load under a branch, or a select next to
    // the load, makes the wave wait for it there -- and, the memory counter
    // being in order, for every load issued before it.
    bool ucol[kMfUpt];
#pragma unroll
    for (int v = 0; v < kMfUpt; ++v) ucol[v] = jA + tid + kMfThreads * v < jB;
    auto u_ids = [&](int j2, int (&id)[kMfUpt]) {   // rows past the last are never used
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v)
            id[v] = A.act_of[(size_t)min(j2, A.n2 - 1) * n1 + min(jA + tid + kMfThreads * v, jB - 1)];
    };
    auto u_vals = [&](const int (&id)[kMfUpt], double (&val)[kMfUpt]) {
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v) val[v] = u[max(id[v], 0)];
    };
    auto u_ok = [&](const int (&id)[kMfUpt], bool (&ok)[kMfUpt]) {
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v) ok[v] = ucol[v] && id[v] >= 0;
    };
    // the ids of u rows E0 .. E0+p+2 first (they need nothing else)
    int idp[P + 3][kMfUpt];
#pragma unroll
    for (int j = 0; j < P + 3; ++j) u_ids(E0 + j, idp[j]);
    // the band's slots: element e (from E0) starts at slot es(e), its rows at wq_pt0(E0 + e)
    auto es = [&](int e) {   // sum over the band's elements before e of round-up-even(rows)
        int s = wq_pt0(E0 + e, N2, P) - wq_pt0(E0, N2, P);
        if ((P + 1) & 1) {   // p+1 rows (odd) in the patch's first and last element
            if (E0 == 0 && e > 0) ++s;
            if (N2 >= 2 && E0 + e >= N2) ++s;
        }
        return s;
    };
    const int S = es(NE), S4 = (S + 3) & ~3;
    const int KA2 = wq_pt0(E0, N2, P);
    for (int t = tid; t < S4 * (P + 1); t += kMfThreads) {
        const int s = t / (P + 1), b = t % (P + 1);
        int e = 0;
        while (e + 1 < NE && es(e + 1) <= s) ++e;
        const int ke = wq_pt0(E0 + e, N2, P), n = wq_pt0(E0 + e + 1, N2, P) - ke;
        const bool in = s < S && s - es(e) < n;
        const int k2 = in ? ke + (s - es(e)) : ke;
        const int i2 = E0 + e + b;
        const double bq = A.d2.Bq[(size_t)k2 * (P + 1) + b];
        const double wq = A.d2.W[(size_t)i2 * A.d2.qmax + (k2 - wq_pt0(max(0, i2 - P), N2, P))];
        sB2[s][b] = in ? bq : 0.0;
        sW2[s][b] = in ? wq : 0.0;
        if (b == 0) sK2[s] = k2;   // padding slots read a real row of c (weight 0)
    }
    const int kA = wq_pt0(max(0, c0 - P), N1, P), kB = wq_pt0(min(N1 - 1, c1 - 1) + 1, N1, P);
    // the thread's points: basis values and local element
    double B1[kMfNpt][P + 1];
    int le1[kMfNpt];
    bool pv[kMfNpt];
#pragma unroll
    for (int m = 0; m < kMfNpt; ++m) {
        const int k1 = kA + tid + kMfThreads * m;
        pv[m] = k1 < kB;
        const int kk = pv[m] ? k1 : kA;
        le1[m] = A.d1.eq[kk] - jA;
#pragma unroll
        for (int a = 0; a <= P; ++a) B1[m][a] = A.d1.Bq[(size_t)kk * (P + 1) + a];
    }
    // the thread's test column: all its weights in registers (0 past its points)
    const int i1 = c0 + tid;
    const bool has_col = i1 < c1;
    const int ic = has_col ? i1 : c0;
    const int k0l = wq_pt0(max(0, ic - P), N1, P) - kA;
    const int nq1 = wq_pt0(min(N1 - 1, ic) + 1, N1, P) - wq_pt0(max(0, ic - P), N1, P);
    double w1[QM];
#pragma unroll
    for (int q = 0; q < NW; ++q) w1[q] = A.d1.WT[(size_t)q * n1 + ic];
#pragma unroll
    for (int q = NW; q < QM; ++q) w1[q] = (q < nq1) ? A.d1.W[(size_t)ic * A.d1.qmax + q] : 0.0;
    const bool wide = nq1 > NW;   // a column next to a patch end
    // points past the strip's last one are read with weight 0: keep them finite
    for (int k = (kB - kA) + tid; k < NG; k += kMfThreads) {
        sG[0][gi(k)] = 0.0;
        sG[1][gi(k)] = 0.0;
    }
    // u values of rows E0 .. E0+p+1; rows E0 .. E0+p into the V ring
    double up[P + 2][kMfUpt];
    bool okp[P + 2][kMfUpt];
#pragma unroll
    for (int j = 0; j <= P + 1; ++j) {
        u_vals(idp[j], up[j]);
        u_ok(idp[j], okp[j]);
    }
#pragma unroll
    for (int j = 0; j <= P; ++j)
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v) sU[j][tid + kMfThreads * v] = okp[j][v] ? up[j][v] : 0.0;
    __syncthreads();
    // V of u row j2 from the values in su into its ring slot
    auto v_row = [&](int j2, const double* su) {
        double* dst = sV[j2 % (P + 1)];
#pragma unroll
        for (int m = 0; m < kMfNpt; ++m) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) s += B1[m][a] * su[le1[m] + a];
            if (pv[m]) dst[tid + kMfThreads * m] = s;
        }
    };
#pragma unroll
    for (int j = 0; j <= P; ++j) v_row(E0 + j, sU[j]);
    int idb[kMfUpt];
    double uv[kMfUpt];
    bool uok[kMfUpt];
#pragma unroll
    for (int v = 0; v < kMfUpt; ++v) {
        uv[v] = up[P + 1][v];      // row E0+p+1 (the second element's new row)
        uok[v] = okp[P + 1][v];
        idb[v] = idp[P + 2][v];    // ids of row E0+p+2
    }
    // c of a pair of slots, two pairs ahead, in two buffers (no copies: a copy of a loaded value waits for it)
    auto c_pair = [&](int s, double (&dst)[2][kMfNpt]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k2 = sK2[min(s + h, S4 - 1)];
#pragma unroll
            for (int m = 0; m < kMfNpt; ++m) dst[h][m] = A.c[(size_t)k2 * Q1 + min(kA + tid + kMfThreads * m, kB - 1)];
        }
    };
    double ca[2][kMfNpt], cb[2][kMfNpt];
    c_pair(0, ca);
    c_pair(2, cb);
    double acc[P + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) acc[b] = 0.0;
    int e2 = E0, send = es(1);
    int yid = A.act_of[(size_t)E0 * n1 + ic];
    int8_t ycls = A.fcls[(size_t)E0 * n1 + ic];
    // slots s, s+1 of element e2 with their c values in cbuf; cbuf then takes slots s+4, s+5
    auto pair = [&](int s, double (&cbuf)[2][kMfNpt]) {
        const bool last = s + 2 == send, next = last && e2 + 1 < E1;
        __syncthreads();  // the V row of the element; sG read by the last pair
#pragma unroll
        for (int m = 0; m < kMfNpt; ++m) {
            const int k = tid + kMfThreads * m;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                const double v = sV[(e2 + b) % (P + 1)][k];
                s0 += sB2[s][b] * v;
                s1 += sB2[s + 1][b] * v;
            }
            if (pv[m]) {
                sG[0][gi(k)] = cbuf[0][m] * s0;
                sG[1][gi(k)] = cbuf[1][m] * s1;
            }
        }
        c_pair(s + 4, cbuf);
        double* su = sU[(e2 + 1 + P) & 1];
        if (next) {   // u row e2+1+p for the next element's V row (after the barrier)
#pragma unroll
            for (int v = 0; v < kMfUpt; ++v) su[tid + kMfThreads * v] = uok[v] ? uv[v] : 0.0;
        }
        __syncthreads();
        double h0 = 0.0, h1 = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            h0 += w1[q] * sG[0][gi(k0l + q)];
            h1 += w1[q] * sG[1][gi(k0l + q)];
        }
        if (wide) {
#pragma unroll
            for (int q = NW; q < QM; ++q) {
                h0 += w1[q] * sG[0][gi(k0l + q)];
                h1 += w1[q] * sG[1][gi(k0l + q)];
            }
        }
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            acc[b] += sW2[s][b] * h0;
            acc[b] += sW2[s + 1][b] * h1;
        }
        if (last) {   // element e2 ends: row e2 has all of the band's terms
            if (next) {
                v_row(e2 + 1 + P, su);       // into row e2's ring slot, read by no later pair
                u_vals(idb, uv);            // row e2+p+2
                u_ok(idb, uok);
                u_ids(e2 + P + 3, idb);     // ids of row e2+p+3
            }
            if (has_col) {
                if (E0 == 0 || e2 - P >= E0) {
                    if (yid >= 0 && wq_row(A, ycls)) y[yid] = acc[0];
                } else {
                    F.head[((size_t)bnd * P + (e2 - E0)) * n1 + i1] = acc[0];
                }
            }
#pragma unroll
            for (int b = 0; b < P; ++b) acc[b] = acc[b + 1];
            acc[P] = 0.0;
            ++e2;
            if (e2 < E1) {
                const size_t f = (size_t)e2 * n1 + ic;
                yid = A.act_of[f];
                ycls = A.fcls[f];
                send = es(e2 - E0 + 1);
            }
        }
    };
    for (int s = 0; s < S4; s += 4) {  // every pair unconditional: a skipped one would make the waits conservative
        pair(s, ca);
        pair(s + 2, cb);
    }
    if (!has_col) return;
#pragma unroll
    for (int b = 0; b < P; ++b) {  // rows E1 .. E1+p-1
        const int i2 = E1 + b;
        if (E1 == N2) {
            const size_t f = (size_t)i2 * n1 + i1;
            const int id = A.act_of[f];
            if (id >= 0 && wq_row(A, A.fcls[f])) y[id] = acc[b];
        } else {
            F.tail[((size_t)bnd * P + b) * n1 + i1] = acc[b];
        }
    }
}

// Adjoint weighted-quadrature part in one pass over the grid, the forward
// pass transposed. A workgroup takes a strip of output columns j1 (lane t)
// and the test columns c0-p+t around them (lane t, their r rows in
// registers), and a band of elements, and walks the band's grid rows:
//   Hr(k2, i1) = sum_b w2[e2+b][k2 - k0(e2+b)] r(i1, e2+b)          (registers -> LDS)
//   R(k2, k1) = sum_a w1[e1+a][k1 - k0(e1+a)] Hr(k2, e1(k1)+a)      (the strip's points)
//   dc = U R with U from the V ring as in the forward pass,  CR = c R  (LDS)
//   D(k2, j1) = sum_q B_j1(x_{k0(j1)+q}) CR(k2, k0(j1)+q)
//   acc[j2] += B2[k2][j2 - e2] D(k2, j1)                             for j2 = e2..e2+p
// r counts on rows formed by weighted quadrature only; du rows are
// written for every active function (head, tail and k_mf_fix as forward),
// the element part is added afterwards.
// LDS of one adjoint workgroup of the grid part.
template <int P>
struct MfAdjSmem {
    static constexpr int NP = kMfThreads * kMfNpt, QM = 4 * P + 2, NU = kMfThreads * kMfUpt;
    static constexpr int NG = NP + QM;
    static constexpr int NGH = (NG + 1) / 2;   // CR rows with even and odd points apart (unit-stride column sums)
    double sU[P + 1][NU];
    double sV[P + 1][NP];
    double sH[2][kMfThreads];
    double sC[2][2 * NGH];
    double sB2[kMfSlots][P + 1], sW2[kMfSlots][P + 1];
    int sK2[kMfSlots];
};

// Workgroup blk of the adjoint grid part.
template <int P>
__device__ __forceinline__ void mf_adj_body(const MfArgs& A, const MfFwdArgs& F, int blk,
                                            const double* __restrict__ u, const double* __restrict__ r,
                                            double* __restrict__ du, double* __restrict__ dc, MfAdjSmem<P>& SM) {
    constexpr int NP = MfAdjSmem<P>::NP, NW = 2 * P + 2, QM = MfAdjSmem<P>::QM, NU = MfAdjSmem<P>::NU;
    constexpr int NG = MfAdjSmem<P>::NG, NGH = MfAdjSmem<P>::NGH;
    auto gi = [](int k) { return (k & 1) * NGH + (k >> 1); };
    auto& sU = SM.sU;
    auto& sV = SM.sV;
    auto& sH = SM.sH;
    auto& sC = SM.sC;
    auto& sB2 = SM.sB2;
    auto& sW2 = SM.sW2;
    auto& sK2 = SM.sK2;
    const int tid = threadIdx.x;
    const int strip = blk % F.nstrip, bnd = blk / F.nstrip;
    const int n1 = A.n1, N1 = A.N1, N2 = A.N2, Q1 = A.d1.Q;
    const int c0 = strip * F.cols, c1 = min(n1, c0 + F.cols);
    const int E0 = bnd * F.band, E1 = (bnd == F.nband - 1) ? N2 : E0 + F.band, NE = E1 - E0;
    const int jA = max(0, c0 - P), jB = min(N1 - 1, c1 - 1) + P + 1;
    bool ucol[kMfUpt];
#pragma unroll
    for (int v = 0; v < kMfUpt; ++v) ucol[v] = jA + tid + kMfThreads * v < jB;
    auto u_ids = [&](int j2, int (&id)[kMfUpt]) {
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v)
            id[v] = A.act_of[(size_t)min(j2, A.n2 - 1) * n1 + min(jA + tid + kMfThreads * v, jB - 1)];
    };
    auto u_vals = [&](const int (&id)[kMfUpt], double (&val)[kMfUpt]) {
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v) val[v] = u[max(id[v], 0)];
    };
    auto u_ok = [&](const int (&id)[kMfUpt], bool (&ok)[kMfUpt]) {
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v) ok[v] = ucol[v] && id[v] >= 0;
    };
    // the lane's test column for Hr and its r rows (0 off the weighted-quadrature rows)
    const int hc = c0 - P + tid;
    const bool hcol = hc >= 0 && hc < n1 && hc < c1 + P;
    const int hcc = min(max(hc, 0), n1 - 1);
    auto r_id = [&](int i2) {   // active id of (hc, i2) if it is a weighted-quadrature row, else -1
        const size_t f = (size_t)min(i2, A.n2 - 1) * n1 + hcc;
        const int id = A.act_of[f];
        const int8_t cls = A.fcls[f];
        return (hcol && i2 < A.n2 && id >= 0 && wq_row(A, cls)) ? id : -1;
    };
    int ida[P + 3][kMfUpt];
#pragma unroll
    for (int j = 0; j < P + 3; ++j) u_ids(E0 + j, ida[j]);
    int rid[P + 2];
#pragma unroll
    for (int j = 0; j < P + 2; ++j) rid[j] = r_id(E0 + j);
    auto es = [&](int e) {
        int s = wq_pt0(E0 + e, N2, P) - wq_pt0(E0, N2, P);
        if ((P + 1) & 1) {
            if (E0 == 0 && e > 0) ++s;
            if (N2 >= 2 && E0 + e >= N2) ++s;
        }
        return s;
    };
    const int S = es(NE), S4 = (S + 3) & ~3;
    for (int t = tid; t < S4 * (P + 1); t += kMfThreads) {
        const int s = t / (P + 1), b = t % (P + 1);
        int e = 0;
        while (e + 1 < NE && es(e + 1) <= s) ++e;
        const int ke = wq_pt0(E0 + e, N2, P), n = wq_pt0(E0 + e + 1, N2, P) - ke;
        const bool in = s < S && s - es(e) < n;
        const int k2 = in ? ke + (s - es(e)) : ke;
        const int i2 = E0 + e + b;
        const double bq = A.d2.Bq[(size_t)k2 * (P + 1) + b];
        const double wq = A.d2.W[(size_t)i2 * A.d2.qmax + (k2 - wq_pt0(max(0, i2 - P), N2, P))];
        sB2[s][b] = in ? bq : 0.0;
        sW2[s][b] = in ? wq : 0.0;
        if (b == 0) sK2[s] = in ? k2 : -1;
    }
    const int kA = wq_pt0(max(0, c0 - P), N1, P), kB = wq_pt0(min(N1 - 1, c1 - 1) + 1, N1, P);
    // the lane's points: basis values, local element and the test weights meeting there
    double B1[kMfNpt][P + 1], WA[kMfNpt][P + 1];
    int le1[kMfNpt];
    bool pv[kMfNpt];
#pragma unroll
    for (int m = 0; m < kMfNpt; ++m) {
        const int k1 = kA + tid + kMfThreads * m;
        pv[m] = k1 < kB;
        const int kk = pv[m] ? k1 : kA;
        const int e1 = A.d1.eq[kk];
        le1[m] = e1 - jA;
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            B1[m][a] = A.d1.Bq[(size_t)kk * (P + 1) + a];
            const int i1 = min(e1 + a, n1 - 1);
            const double w = A.d1.W[(size_t)i1 * A.d1.qmax + (kk - wq_pt0(max(0, i1 - P), N1, P))];
            WA[m][a] = (e1 + a < n1) ? w : 0.0;
        }
    }
    // the lane's output column: its basis values at its support points (0 past them)
    const int j1 = c0 + tid;
    const bool has_col = j1 < c1;
    const int jc = has_col ? j1 : c0;
    const int k0l = wq_pt0(max(0, jc - P), N1, P) - kA;
    const int nq1 = wq_pt0(min(N1 - 1, jc) + 1, N1, P) - wq_pt0(max(0, jc - P), N1, P);
    double bj[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int k = min(kA + k0l + q, Q1 - 1);
        const int a = jc - A.d1.eq[k];
        const double v = A.d1.Bq[(size_t)k * (P + 1) + min(max(a, 0), P)];
        bj[q] = (q < nq1 && a >= 0 && a <= P) ? v : 0.0;
    }
    const bool wide = nq1 > NW;
    for (int k = (kB - kA) + tid; k < NG; k += kMfThreads) {
        sC[0][gi(k)] = 0.0;
        sC[1][gi(k)] = 0.0;
    }
    // u rows E0 .. E0+p into the V ring, r rows E0 .. E0+p into registers
    double up[P + 2][kMfUpt];
    bool okp[P + 2][kMfUpt];
#pragma unroll
    for (int j = 0; j <= P + 1; ++j) {
        u_vals(ida[j], up[j]);
        u_ok(ida[j], okp[j]);
    }
    double rr[P + 1], rnext;
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        const double t = r[max(rid[j], 0)];
        rr[j] = rid[j] >= 0 ? t : 0.0;
    }
    rnext = r[max(rid[P + 1], 0)];    // row E0+p+1 (selected when it enters the ring)
    int rnid = rid[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j)
#pragma unroll
        for (int v = 0; v < kMfUpt; ++v) sU[j][tid + kMfThreads * v] = okp[j][v] ? up[j][v] : 0.0;
    __syncthreads();
    auto v_row = [&](int j2, const double* su) {
        double* dst = sV[j2 % (P + 1)];
#pragma unroll
        for (int m = 0; m < kMfNpt; ++m) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) s += B1[m][a] * su[le1[m] + a];
            if (pv[m]) dst[tid + kMfThreads * m] = s;
        }
    };
#pragma unroll
    for (int j = 0; j <= P; ++j) v_row(E0 + j, sU[j]);
    int idb[kMfUpt];
    double uv[kMfUpt];
    bool uok[kMfUpt];
#pragma unroll
    for (int v = 0; v < kMfUpt; ++v) {
        uv[v] = up[P + 1][v];
        uok[v] = okp[P + 1][v];
        idb[v] = ida[P + 2][v];
    }
    int rnid2 = r_id(E0 + P + 2);   // the r row after next
    auto c_pair = [&](int s, double (&dst)[2][kMfNpt]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k2 = max(sK2[min(s + h, S4 - 1)], 0);
#pragma unroll
            for (int m = 0; m < kMfNpt; ++m) dst[h][m] = A.c[(size_t)k2 * Q1 + min(kA + tid + kMfThreads * m, kB - 1)];
        }
    };
    double ca[2][kMfNpt], cb[2][kMfNpt];
    c_pair(0, ca);
    c_pair(2, cb);
    double acc[P + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) acc[b] = 0.0;
    int e2 = E0, send = es(1);
    int yid = A.act_of[(size_t)E0 * n1 + jc];
    auto pair = [&](int s, double (&cbuf)[2][kMfNpt]) {
        const bool last = s + 2 == send, next = last && e2 + 1 < E1;
        // the lane's Hr of both rows
        double h0 = 0.0, h1 = 0.0;
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            h0 += sW2[s][b] * rr[b];
            h1 += sW2[s + 1][b] * rr[b];
        }
        __syncthreads();  // V row of the element; sH and sC read by the last pair
        sH[0][tid] = h0;
        sH[1][tid] = h1;
        __syncthreads();
        const int ka = sK2[s], kb = sK2[s + 1];
#pragma unroll
        for (int m = 0; m < kMfNpt; ++m) {
            const int k = tid + kMfThreads * m;
            double u0 = 0.0, u1 = 0.0, r0 = 0.0, r1 = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                const double v = sV[(e2 + b) % (P + 1)][k];
                u0 += sB2[s][b] * v;
                u1 += sB2[s + 1][b] * v;
            }
#pragma unroll
            for (int a = 0; a <= P; ++a) {   // Hr columns e1+a: local index e1 + a - (c0 - p)
                const int hi = min(le1[m] + a + (jA - (c0 - P)), kMfThreads - 1);
                r0 += WA[m][a] * sH[0][hi];
                r1 += WA[m][a] * sH[1][hi];
            }
            if (pv[m]) {
                const int k1 = kA + k;
                if (le1[m] + jA >= c0) {   // the point's element is the strip's (the previous strip writes the halo)
                    if (ka >= 0) dc[(size_t)ka * Q1 + k1] = u0 * r0;
                    if (kb >= 0) dc[(size_t)kb * Q1 + k1] = u1 * r1;
                }
                sC[0][gi(k)] = cbuf[0][m] * r0;
                sC[1][gi(k)] = cbuf[1][m] * r1;
            }
        }
        c_pair(s + 4, cbuf);
        double* su = sU[(e2 + 1 + P) & 1];
        if (next) {
#pragma unroll
            for (int v = 0; v < kMfUpt; ++v) su[tid + kMfThreads * v] = uok[v] ? uv[v] : 0.0;
        }
        __syncthreads();
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            d0 += bj[q] * sC[0][gi(k0l + q)];
            d1 += bj[q] * sC[1][gi(k0l + q)];
        }
        if (wide) {
#pragma unroll
            for (int q = NW; q < QM; ++q) {
                d0 += bj[q] * sC[0][gi(k0l + q)];
                d1 += bj[q] * sC[1][gi(k0l + q)];
            }
        }
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            acc[b] += sB2[s][b] * d0;
            acc[b] += sB2[s + 1][b] * d1;
        }
        if (last) {   // element e2 ends: du row e2 has all of the band's grid terms
            if (next) {
                v_row(e2 + 1 + P, su);
                u_vals(idb, uv);
                u_ok(idb, uok);
                u_ids(e2 + P + 3, idb);
            }
            if (has_col) {
                if (E0 == 0 || e2 - P >= E0) {
                    if (yid >= 0) du[yid] = acc[0];
                } else {
                    F.head[((size_t)bnd * P + (e2 - E0)) * n1 + j1] = acc[0];
                }
            }
#pragma unroll
            for (int b = 0; b < P; ++b) {
                acc[b] = acc[b + 1];
                rr[b] = rr[b + 1];
            }
            acc[P] = 0.0;
            rr[P] = rnid >= 0 ? rnext : 0.0;   // r row e2+1+p
            rnext = r[max(rnid2, 0)];
            rnid = rnid2;
            rnid2 = r_id(e2 + P + 3);
            ++e2;
            if (e2 < E1) {
                yid = A.act_of[(size_t)e2 * n1 + jc];
                send = es(e2 - E0 + 1);
            }
        }
    };
    for (int s = 0; s < S4; s += 4) {
        pair(s, ca);
        pair(s + 2, cb);
    }
    if (!has_col) return;
#pragma unroll
    for (int b = 0; b < P; ++b) {  // rows E1 .. E1+p-1
        const int i2 = E1 + b;
        if (E1 == N2) {
            const int id = A.act_of[(size_t)i2 * n1 + j1];
            if (id >= 0) du[id] = acc[b];
        } else {
            F.tail[((size_t)bnd * P + b) * n1 + j1] = acc[b];
        }
    }
}

// Rows whose support spans two bands: the band's head plus the previous band's tail.
// (all_rows: every active row, as the adjoint's du; else the weighted-quadrature rows)
template <int P>
__device__ __forceinline__ void mf_fix_at(const MfArgs& A, const MfFwdArgs& F, double* __restrict__ y, int all_rows,
                                          int64_t t) {
    const int n1 = A.n1;
    if (t >= (int64_t)(F.nband - 1) * P * n1) return;
    const int bnd = 1 + (int)(t / ((int64_t)P * n1)), r = (int)((t / n1) % P), i1 = (int)(t % n1);
    const int i2 = bnd * F.band + r;
    const size_t f = (size_t)i2 * n1 + i1;
    const int id = A.act_of[f];
    if (id < 0 || !(all_rows || wq_row(A, A.fcls[f]))) return;
    y[id] = F.tail[((size_t)(bnd - 1) * P + r) * n1 + i1] + F.head[((size_t)bnd * P + r) * n1 + i1];
}

template <int P>
__global__ void __launch_bounds__(256) k_mf_fix(MfArgs A, MfFwdArgs F, double* __restrict__ y, int all_rows) {
    mf_fix_at<P>(A, F, y, all_rows, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Band elements (inside elements of the rows formed element-wise; a tensor
// Gauss rule of (p+1)^2 points): several elements per workgroup of NT threads,
// thread (element, l) taking local function l for u, point l for U, and
// output l, the element's basis tables shared in LDS:
//   U_g = sum_a2 B2[g2][a2] sum_a1 B1[g1][a1] u_a,  Y_l = sum_g2 B2[g2][l2] sum_g1 B1[g1][l1] w_g c_g U_g
// (adjoint: R_g from r alike, dc_g = U_g w_g R_g, D_l from c_g w_g R_g).
template <int P, int NT>
struct MfBandSmem {
    static constexpr int NP1 = P + 1, L = NP1 * NP1, EPW = NT / L;
    double sU[EPW][L], sR[EPW][L], sT[EPW][L];
    double sB1[EPW][NP1][NP1], sB2[EPW][NP1][NP1];
};

template <int P, int NT>
__device__ __forceinline__ void mf_band_body(const MfArgs& A, int blk, const double* __restrict__ u,
                                             const double* __restrict__ r, double* __restrict__ Ye,
                                             double* __restrict__ dc, MfBandSmem<P, NT>& S) {
    constexpr int NP1 = P + 1, L = NP1 * NP1, EPW = NT / L;
    static_assert(EPW >= 1, "an element's functions must fit the workgroup");
    auto& sU = S.sU;
    auto& sR = S.sR;
    auto& sT = S.sT;
    auto& sB1 = S.sB1;
    auto& sB2 = S.sB2;
    const int el = threadIdx.x / L, l = threadIdx.x % L;
    const int re = blk * EPW + el;
    const bool on = el < EPW && re < A.n_band;
    const int e = A.band_list[on ? re : 0];
    const int e1 = e % A.N1, e2 = e / A.N1;
    const int l1 = l % NP1, l2 = l / NP1;   // local function, point (g1, g2) and output alike
    double B1[NP1], B2[NP1];
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        B1[a] = A.d1.Bg[(e1 * NP1 + l1) * NP1 + a];
        B2[a] = A.d2.Bg[(e2 * NP1 + l2) * NP1 + a];
    }
    const double w = A.d1.wg[e1 * NP1 + l1] * A.d2.wg[e2 * NP1 + l2];
    const size_t pt = (size_t)A.nq + (size_t)(on ? re : 0) * L + l;
    const double cg = A.c[pt];
    const int f = (e2 + l2) * A.n1 + (e1 + l1);
    const int cid = A.act_of[f];
    if (on) {
        sU[el][l] = (cid >= 0) ? u[cid] : 0.0;
        // rows formed element-wise: cut rows (hybrid) or every row (reference)
        const bool erow = cid >= 0 && !wq_row(A, A.fcls[f]);
        sR[el][l] = (r && erow) ? r[cid] : 0.0;
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            if (l2 == 0) sB1[el][l1][a] = B1[a];
            if (l1 == 0) sB2[el][l2][a] = B2[a];
        }
    }
    __syncthreads();
    if (on) {
        double Ug = 0.0, Rg = 0.0;
#pragma unroll
        for (int a2 = 0; a2 <= P; ++a2) {
            double su = 0.0, sr = 0.0;
#pragma unroll
            for (int a1 = 0; a1 <= P; ++a1) {
                su += B1[a1] * sU[el][a2 * NP1 + a1];
                sr += B1[a1] * sR[el][a2 * NP1 + a1];
            }
            Ug += B2[a2] * su;
            Rg += B2[a2] * sr;
        }
        if (r) {
            Rg *= w;
            dc[pt] = Ug * Rg;
            sT[el][l] = cg * Rg;
        } else {
            sT[el][l] = w * cg * Ug;
        }
    }
    __syncthreads();
    if (!on) return;
    double y = 0.0;
#pragma unroll
    for (int g2 = 0; g2 <= P; ++g2) {
        double s = 0.0;
#pragma unroll
        for (int g1 = 0; g1 <= P; ++g1) s += sB1[el][g1][l1] * sT[el][g2 * NP1 + g1];
        y += sB2[el][g2][l2] * s;
    }
    Ye[(size_t)re * L + l] = y;
}

// Cut elements, one workgroup of NT threads each: per chunk of NT nodes, node
// n's basis rows (from the element's reciprocal table: no divisions), U_n and
// the weight term T_n in LDS; then the (p+1)^2 outputs are split over
// G = max(1, NT / (p+1)^2) lane groups, group g summing the chunk's nodes
// m = g (mod G), and the groups' sums are added in order at the end.
template <int P, int NT>
struct MfElemSmem {
    static constexpr int NP1 = P + 1, L = NP1 * NP1;
    static constexpr int G = L >= NT ? 1 : NT / L;  // lane groups of the accumulation
    static constexpr int NR = P * (P + 1) / 2;       // reciprocals of one span
    double sB1[NT][NP1], sB2[NT][NP1];
    double sT[NT];
    double sU[L], sR[L];
    double sRec[2][NR + 1];
    double sAcc[G][L];
};

template <int P, int NT>
__device__ __forceinline__ void mf_elem_body(const MfArgs& A, int re, const double* __restrict__ u,
                                             const double* __restrict__ r, double* __restrict__ Ye,
                                             double* __restrict__ dc, MfElemSmem<P, NT>& S) {
    constexpr int NP1 = P + 1, L = NP1 * NP1;
    constexpr int G = MfElemSmem<P, NT>::G;      // lane groups of the accumulation
    constexpr int PER = (L + NT - 1) / NT;       // outputs per lane when G = 1
    constexpr int NR = MfElemSmem<P, NT>::NR;    // reciprocals of one span
    auto& sB1 = S.sB1;
    auto& sB2 = S.sB2;
    auto& sT = S.sT;
    auto& sU = S.sU;
    auto& sR = S.sR;
    auto& sRec = S.sRec;
    auto& sAcc = S.sAcc;
    const int tid = threadIdx.x;
    const bool is_cut = re >= A.n_band;
    const int e = is_cut ? A.cut_list[re - A.n_band] : A.band_list[re];
    const int e1 = e % A.N1, e2 = e / A.N1;
    for (int l = tid; l < L; l += NT) {
        int j1 = e1 + l % NP1, j2 = e2 + l / NP1;
        int f = j2 * A.n1 + j1;
        int cid = A.act_of[f];
        sU[l] = (cid >= 0) ? u[cid] : 0.0;
        // rows formed element-wise: cut rows (hybrid) or every row (reference)
        bool erow = cid >= 0 && !wq_row(A, A.fcls[f]);
        sR[l] = (r && erow) ? r[cid] : 0.0;
    }
    for (int t = tid; t < 2 * NR; t += NT) {
        const int d = t / NR, idx = t % NR;
        sRec[d][idx] = basis_rec<P>(d ? A.d2.knots : A.d1.knots, P + (d ? e2 : e1), idx);
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
    // this lane's outputs: group grp, local functions l = li + NT k (G = 1) or li (G > 1)
    const int grp = (G > 1) ? tid / L : 0, li = (G > 1) ? tid % L : tid;
    const bool acc_on = (G > 1) ? grp < G : true;
    double acc[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) acc[k] = 0.0;
    for (int base = nb; base < ne; base += NT) {
        __syncthreads();
        int n = base + tid;
        if (n < ne) {
            double B1[NP1], B2[NP1], w;
            if (is_cut) {
                basis_eval_rec<P>(A.d1.knots, P + e1, sRec[0], A.nx[n], B1);
                basis_eval_rec<P>(A.d2.knots, P + e2, sRec[1], A.ny[n], B2);
                w = A.nw[n];
            } else {
                int g1 = n % NP1, g2 = n / NP1;
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    B1[a] = A.d1.Bg[(e1 * NP1 + g1) * NP1 + a];
                    B2[a] = A.d2.Bg[(e2 * NP1 + g2) * NP1 + a];
                }
                w = A.d1.wg[e1 * NP1 + g1] * A.d2.wg[e2 * NP1 + g2];
            }
            double Ug = 0.0, Rg = 0.0;
#pragma unroll
            for (int a2 = 0; a2 <= P; ++a2) {
                double su = 0.0, sr = 0.0;
#pragma unroll
                for (int a1 = 0; a1 <= P; ++a1) {
                    su += B1[a1] * sU[a2 * NP1 + a1];
                    sr += B1[a1] * sR[a2 * NP1 + a1];
                }
                Ug += B2[a2] * su;
                Rg += B2[a2] * sr;
            }
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                sB1[tid][a] = B1[a];
                sB2[tid][a] = B2[a];
            }
            double cg = A.c[pbase + n];
            if (r) {
                Rg *= w;
                dc[pbase + n] = Ug * Rg;
                sT[tid] = cg * Rg;
            } else {
                sT[tid] = w * cg * Ug;
            }
        }
        __syncthreads();
        const int cnt = min(NT, ne - base);
        if (acc_on) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int l = li + NT * k;
                if (l < L) {
                    const int a1 = l % NP1, a2 = l / NP1;
                    for (int m = grp; m < cnt; m += G) acc[k] += sT[m] * sB1[m][a1] * sB2[m][a2];
                }
            }
        }
    }
    if (G > 1) {
        if (acc_on) sAcc[grp][li] = acc[0];
        __syncthreads();
        if (tid < L) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) s += sAcc[g][tid];
            Ye[(size_t)re * L + tid] = s;
        }
    } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int l = li + NT * k;
            if (l < L) Ye[(size_t)re * L + l] = acc[k];
        }
    }
}

// Forward rows formed element-wise: the element vectors of the band and cut
// elements of the row's support, summed in a fixed order. Four lanes per row
// of the plan's element-formed list, each taking every fourth support element
// (classes, then element ids, then vector entries loaded together), the four
// partial sums added in the quad.
template <int P>
__device__ __forceinline__ void mf_gather_at(const MfArgs& A, const int* __restrict__ rows, int n_rows,
                                             const double* __restrict__ Ye, double* __restrict__ y, int t) {
    constexpr int L = (P + 1) * (P + 1), PER = (L + 3) / 4;
    const int ri = t >> 2, part = t & 3;
    const bool ok = ri < n_rows;   // lanes past the list still take part in the quad sum
    const int r = rows[min(ri, n_rows - 1)], f = A.fn_of[r];
    const int i1 = f % A.n1, i2 = f / A.n1;
    int8_t cls[PER];
    // slot idx of the (p+1)^2 support elements; the last quad's slots past them are
    // clamped onto the last element (an outside class, so they add nothing)
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = min(part + 4 * k, L - 1), b = idx / (P + 1), a = idx % (P + 1);
        const int e1 = i1 - P + a, e2 = i2 - P + b;
        const bool in = part + 4 * k < L && e1 >= 0 && e1 < A.N1 && e2 >= 0 && e2 < A.N2;
        cls[k] = in ? A.ecls[(size_t)e2 * A.N1 + e1] : (int8_t)EL_OUTSIDE;
    }
    int re[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = min(part + 4 * k, L - 1), b = idx / (P + 1), a = idx % (P + 1);
        const int e = (i2 - P + b) * A.N1 + (i1 - P + a);
        const int8_t c = cls[k];
        re[k] = (c == EL_CUT) ? A.n_band + A.cut_id[e] : (c == EL_OUTSIDE ? -1 : A.band_id[e]);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        // element (i1-p+a, i2-p+b): the row is its local function (p-a, p-b)
        const int idx = min(part + 4 * k, L - 1), b = idx / (P + 1), a = idx % (P + 1);
        const int kk = re[k];
        const double v = Ye[(size_t)max(kk, 0) * L + (P - b) * (P + 1) + (P - a)];
        s += (kk >= 0) ? v : 0.0;
    }
    s = quad_sum(s);
    if (ok && part == 0 && !wq_row(A, A.fcls[f])) y[r] = s;
}

// The forward's row fix-ups in one launch: blocks below nfix add band heads
// to tails (k_mf_fix's rows), the others gather the element vectors of the
// rows formed element-wise (disjoint rows of y).
template <int P>
__global__ void __launch_bounds__(256) k_mf_rows(MfArgs A, MfFwdArgs F, int nfix, const int* __restrict__ rows,
                                                 int n_rows, const double* __restrict__ Ye, double* __restrict__ y) {
    if ((int)blockIdx.x < nfix)
        mf_fix_at<P>(A, F, y, 0, (int64_t)blockIdx.x * 256 + threadIdx.x);
    else
        mf_gather_at<P>(A, rows, n_rows, Ye, y, ((int)blockIdx.x - nfix) * 256 + threadIdx.x);
}

// The forward in one launch: the first workgroups take the weighted-
// quadrature grid part, the next ncut the cut elements and the last
// nband_blk the band elements (their element vectors). The grid part's
// workgroups come first: the element workgroups, latency-bound, then fill
// the CUs as the grid part frees them (0.048 against 0.053 ms the other way
// round at 1024^2). All roles share one LDS allocation.
template <int P>
__global__ void __launch_bounds__(kMfThreads) k_mf_fwd(MfArgs A, MfFwdArgs F, int ncut, int nband_blk,
                                                       const double* __restrict__ u, double* __restrict__ y,
                                                       double* __restrict__ Ye) {
    __shared__ union {
        MfFwdSmem<P> f;
        MfElemSmem<P, kMfThreads> e;
        MfBandSmem<P, kMfThreads> b;
    } S;
    const int ngrid = (int)gridDim.x - ncut - nband_blk;
    const int blk = blockIdx.x;
    if (blk < ngrid)
        mf_fwd_body<P>(A, F, blk, u, y, S.f);
    else if (blk - ngrid < ncut)
        mf_elem_body<P, kMfThreads>(A, A.n_band + blk - ngrid, u, nullptr, Ye, nullptr, S.e);
    else
        mf_band_body<P, kMfThreads>(A, blk - ngrid - ncut, u, nullptr, Ye, nullptr, S.b);
}

// The adjoint's grid part and its element vectors (and dc at band Gauss
// points and cut nodes) in one launch, laid out as the forward's.
template <int P>
__global__ void __launch_bounds__(kMfThreads) k_mf_adj(MfArgs A, MfFwdArgs F, int ncut, int nband_blk,
                                                       const double* __restrict__ u, const double* __restrict__ r,
                                                       double* __restrict__ du, double* __restrict__ dc,
                                                       double* __restrict__ Ye) {
    __shared__ union {
        MfAdjSmem<P> a;
        MfElemSmem<P, kMfThreads> e;
        MfBandSmem<P, kMfThreads> b;
    } S;
    const int ngrid = (int)gridDim.x - ncut - nband_blk;
    const int blk = blockIdx.x;
    if (blk < ngrid)
        mf_adj_body<P>(A, F, blk, u, r, du, dc, S.a);
    else if (blk - ngrid < ncut)
        mf_elem_body<P, kMfThreads>(A, A.n_band + blk - ngrid, u, r, Ye, dc, S.e);
    else
        mf_band_body<P, kMfThreads>(A, blk - ngrid - ncut, u, r, Ye, dc, S.b);
}

// Adjoint: the element vectors of the band and cut elements of each listed
// row's support added to du (after the grid part), four lanes per row as in
// the forward gather.
template <int P>
__global__ void __launch_bounds__(256) k_mf_gather_add(MfArgs A, const int* __restrict__ rows, int n_rows,
                                                       const double* __restrict__ Ye, double* __restrict__ du) {
    constexpr int L = (P + 1) * (P + 1), PER = (L + 3) / 4;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int ri = t >> 2, part = t & 3;
    const bool ok = ri < n_rows;
    const int r = rows[min(ri, n_rows - 1)], f = A.fn_of[r];
    const int i1 = f % A.n1, i2 = f / A.n1;
    int8_t cls[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = min(part + 4 * k, L - 1), b = idx / (P + 1), a = idx % (P + 1);
        const int e1 = i1 - P + a, e2 = i2 - P + b;
        const bool in = part + 4 * k < L && e1 >= 0 && e1 < A.N1 && e2 >= 0 && e2 < A.N2;
        cls[k] = in ? A.ecls[(size_t)e2 * A.N1 + e1] : (int8_t)EL_OUTSIDE;
    }
    int re[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = min(part + 4 * k, L - 1), b = idx / (P + 1), a = idx % (P + 1);
        const int e = (i2 - P + b) * A.N1 + (i1 - P + a);
        const int8_t c = cls[k];
        re[k] = (c == EL_CUT) ? A.n_band + A.cut_id[e] : (c == EL_OUTSIDE ? -1 : A.band_id[e]);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = min(part + 4 * k, L - 1), b = idx / (P + 1), a = idx % (P + 1);
        const int kk = re[k];
        const double v = Ye[(size_t)max(kk, 0) * L + (P - b) * (P + 1) + (P - a)];
        s += (kk >= 0) ? v : 0.0;
    }
    s = quad_sum(s);
    if (ok && part == 0) du[r] += s;
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
    return A;
}


// Strips of test columns and bands of elements of the one-pass forward.
// adjoint: the lanes also hold the test columns p either side of the strip's
static MfFwdArgs mf_fwd_shape(const Plan& P, bool adjoint = false) {
    MfFwdArgs F{};
    int cmax = std::min(kMfThreads, (kMfThreads * kMfNpt - 2 * (P.p - 1)) / 2 - P.p);  // 2 (cols + p) + 2 (p - 1) points
    if (adjoint) cmax = std::min(cmax, kMfThreads - 2 * P.p);
    const int ns = (P.n1 + cmax - 1) / cmax;
    F.cols = (P.n1 + ns - 1) / ns;
    F.nstrip = (P.n1 + F.cols - 1) / F.cols;
    F.band = std::max(kMfBand, P.p + 1);
    IGA_REQUIRE(F.band <= kMfBandMax, IGA_E_UNSUPPORTED, "matrix-free product: band size");
    F.nband = std::max(1, P.N2 / F.band);
    for (int st = 0; st < F.nstrip; ++st) {  // points of every strip within the workgroup's share
        const int c0 = st * F.cols, c1 = std::min(P.n1, c0 + F.cols);
        const int np = wq_pt0(std::min(P.N1 - 1, c1 - 1) + 1, P.N1, P.p) - wq_pt0(std::max(0, c0 - P.p), P.N1, P.p);
        IGA_REQUIRE(np <= kMfThreads * kMfNpt, IGA_E_UNSUPPORTED, "matrix-free product: strip point count");
    }
    return F;
}

static size_t mf_part_doubles(const Plan& P, const MfFwdArgs& F) { return 2 * (size_t)F.nband * P.p * P.n1; }

static void mf_buffers(Plan& P) {
    size_t L = (size_t)(P.p + 1) * (P.p + 1);
    if (!P.sw.Ue) P.sw.Ue = P.alloc<double>(std::max<int64_t>(1, P.n_band + P.n_cut_el) * L);
    if (!P.sw.mfpart) P.sw.mfpart = P.alloc<double>(mf_part_doubles(P, mf_fwd_shape(P)));
}

// The rows that receive element vectors in the adjoint: every active row
// with a band or cut element in its support (built on the host once per plan).
static void mf_adj_rows(Plan& P, hipStream_t s) {
    if (P.sw.adj_rows) return;
    const int n = (int)P.n_act, ne = P.N1 * P.N2, p = P.p;
    std::vector<int> fn(n), bid(ne), cid(ne), rows;
    std::vector<int8_t> cls(ne);
    HIPX(hipMemcpyAsync(fn.data(), P.fn_of, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    HIPX(hipMemcpyAsync(cls.data(), P.ecls, ne, hipMemcpyDeviceToHost, s));
    HIPX(hipMemcpyAsync(bid.data(), P.band_id, sizeof(int) * ne, hipMemcpyDeviceToHost, s));
    HIPX(hipMemcpyAsync(cid.data(), P.cut_id, sizeof(int) * ne, hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    for (int r = 0; r < n; ++r) {
        const int i1 = fn[r] % P.n1, i2 = fn[r] / P.n1;
        bool hit = false;
        for (int e2 = std::max(0, i2 - p); e2 <= std::min(P.N2 - 1, i2) && !hit; ++e2)
            for (int e1 = std::max(0, i1 - p); e1 <= std::min(P.N1 - 1, i1) && !hit; ++e1) {
                const int e = e2 * P.N1 + e1;
                hit = (cls[e] == EL_CUT && cid[e] >= 0) || (cls[e] == EL_INSIDE && bid[e] >= 0);
            }
        if (hit) rows.push_back(r);
    }
    P.sw.n_adj_rows = (int)rows.size();
    P.sw.adj_rows = P.alloc<int>(std::max<size_t>(1, rows.size()));
    if (!rows.empty())
        HIPX(hipMemcpyAsync(P.sw.adj_rows, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, s));
    HIPX(hipStreamSynchronize(s));
}

static dim3 grid256(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// Element workgroups of the one-launch forward and adjoint: the cut elements
// one each, the band elements kMfThreads / (p+1)^2 to a workgroup.
static void elem_blocks(const Plan& P, int& ncut, int& nband_blk) {
    const int epw = kMfThreads / ((P.p + 1) * (P.p + 1));
    ncut = (int)P.n_cut_el;
    nband_blk = (int)((P.n_band + epw - 1) / epw);
}

static const char* const kMfFwdNames[] = {"", "k_mf_fwd<1>", "k_mf_fwd<2>", "k_mf_fwd<3>", "k_mf_fwd<4>",
                                          "k_mf_fwd<5>", "k_mf_fwd<6>", "k_mf_fwd<7>", "k_mf_fwd<8>"};
static const char* const kMfAdjNames[] = {"", "k_mf_adj<1>", "k_mf_adj<2>", "k_mf_adj<3>", "k_mf_adj<4>",
                                          "k_mf_adj<5>", "k_mf_adj<6>", "k_mf_adj<7>", "k_mf_adj<8>"};
static const char* const kMfFixNames[] = {"", "k_mf_fix<1>", "k_mf_fix<2>", "k_mf_fix<3>", "k_mf_fix<4>",
                                          "k_mf_fix<5>", "k_mf_fix<6>", "k_mf_fix<7>", "k_mf_fix<8>"};
static const char* const kMfRowsNames[] = {"", "k_mf_rows<1>", "k_mf_rows<2>", "k_mf_rows<3>", "k_mf_rows<4>",
                                           "k_mf_rows<5>", "k_mf_rows<6>", "k_mf_rows<7>", "k_mf_rows<8>"};

// Forward: element vectors and the grid part in one launch, then the row
// fix-ups (band heads added to tails, element vectors gathered) in another.
// The reference rules have no grid part: every row is formed element-wise.
template <int P>
static void launch_forward(Plan& Pl, const MfArgs& A, const double* u, double* y, double* part, double* Ue,
                           hipStream_t s) {
    const bool wq = Pl.method != IGA_GAUSS_REF;
    MfFwdArgs F{};
    if (wq) {
        F = mf_fwd_shape(Pl);
        F.head = part;
        F.tail = part + (size_t)F.nband * P * Pl.n1;
    }
    int ncut = 0, nbb = 0;
    elem_blocks(Pl, ncut, nbb);
    const int64_t nblk = (int64_t)ncut + nbb + (wq ? (int64_t)F.nstrip * F.nband : 0);
    if (nblk > 0)
        klaunch(Pl, kMfFwdNames[P], k_mf_fwd<P>, dim3((unsigned)nblk), dim3(kMfThreads), 0, s, A, F, ncut, nbb, u, y,
                Ue);
    const int nfix = (wq && F.nband > 1) ? (int)grid256((int64_t)(F.nband - 1) * P * Pl.n1).x : 0;
    const int nr = (int)Pl.n_form_rows;
    const int ngat = nr > 0 ? (int)grid256(4 * (int64_t)nr).x : 0;
    if (nfix + ngat > 0)
        klaunch(Pl, kMfRowsNames[P], k_mf_rows<P>, dim3(nfix + ngat), dim3(256), 0, s, A, F, nfix,
                (const int*)Pl.form_rows, nr, (const double*)Ue, y);
}

// Adjoint: element vectors (with dc at their points) and the grid part (every
// active row of du) in one launch, then the band heads added to tails.
template <int P>
static void launch_adjoint(Plan& Pl, const MfArgs& A, const double* u, const double* r, double* du, double* dc,
                           double* part, double* Ue, hipStream_t s) {
    const bool wq = Pl.method != IGA_GAUSS_REF;
    MfFwdArgs F{};
    if (wq) {
        F = mf_fwd_shape(Pl, true);
        F.head = part;
        F.tail = part + (size_t)F.nband * P * Pl.n1;
    }
    int ncut = 0, nbb = 0;
    elem_blocks(Pl, ncut, nbb);
    const int64_t nblk = (int64_t)ncut + nbb + (wq ? (int64_t)F.nstrip * F.nband : 0);
    if (nblk > 0)
        klaunch(Pl, kMfAdjNames[P], k_mf_adj<P>, dim3((unsigned)nblk), dim3(kMfThreads), 0, s, A, F, ncut, nbb, u, r,
                du, dc, Ue);
    if (wq && F.nband > 1)
        klaunch(Pl, kMfFixNames[P], k_mf_fix<P>, grid256((int64_t)(F.nband - 1) * P * Pl.n1), dim3(256), 0, s, A, F, du,
                1);
}

// The forward product with its two intermediate arrays given: the bands'
// head and tail rows [2][nband][p][n1] and Ue [n_band + n_cut][(p+1)^2].
// Every entry of them is written before it is read, so they need no clearing.
// Two launches on the caller's stream: the element vectors beside the
// weighted-quadrature grid part (workgroups of one launch, so they overlap;
// a second stream measured no overlap here, its queue starting some 16 us
// after the fork's kernels had ended), then the rows' fix-ups.
static void mf_apply_into(Plan& P, const double* c, const double* u, double* y, double* part, double* Ue,
                          hipStream_t s) {
    MfArgs A = mf_args(P, c);
    switch (P.p) {
#define CASE(PP) \
    case PP: launch_forward<PP>(P, A, u, y, part, Ue, s); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
}

void mf_apply(Plan& P, const double* c, const double* u, double* y, hipStream_t s) {
    mf_buffers(P);
    mf_apply_into(P, c, u, y, P.sw.mfpart, P.sw.Ue, s);
}

// ------------------------------------------------- allocation-free product
// The intermediate arrays of iga_mf_apply_noalloc live in one array of
// device memory that the library holds for the life of the process (one copy
// per device, at its own address). Every call on a device shares that
// device's copy: calls that overlap on one device race.
constexpr size_t kMfScratchDoubles = (size_t)2 << 20;  // 16 MiB
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
    const size_t L = (size_t)(P.p + 1) * (P.p + 1);
    const size_t nP = round256(mf_part_doubles(P, mf_fwd_shape(P)));
    const size_t nU = round256((size_t)std::max<int64_t>(1, P.n_band + P.n_cut_el) * L);
    const size_t need = nP + nU;
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
    mf_apply_into(P, c, u, y, base, base + nP, s);
}

// The adjoint: the element vectors (and dc at band Gauss points and cut
// nodes) beside the grid part of du and dc (every active row of du written),
// in one launch, then the element vectors added to the rows they touch.
void mf_adjoint(Plan& P, const double* c, const double* u, const double* r, double* du, double* dc, hipStream_t s) {
    mf_buffers(P);
    mf_adj_rows(P, s);
    MfArgs A = mf_args(P, c);
    switch (P.p) {
#define CASE(PP) \
    case PP: launch_adjoint<PP>(P, A, u, r, du, dc, P.sw.mfpart, P.sw.Ue, s); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
    if (P.method == IGA_GAUSS_REF) {
        HIPX(hipMemsetAsync(dc, 0, sizeof(double) * (size_t)A.nq, s));
        HIPX(hipMemsetAsync(du, 0, sizeof(double) * (size_t)P.n_act, s));
    }
    const int nr = P.sw.n_adj_rows;
    if (nr == 0) return;
    switch (P.p) {
#define CASE(PP)                                                                                            \
    case PP:                                                                                                \
        klaunch(P, "k_mf_gather_add<" #PP ">", k_mf_gather_add<PP>, grid256(4 * (int64_t)nr), dim3(256), 0, s, A,   \
                (const int*)P.sw.adj_rows, nr, (const double*)P.sw.Ue, du);                                 \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
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
