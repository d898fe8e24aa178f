// Device bodies of the formation kernels, shared by the one-patch kernels
// (form.hip) and the batched persistent kernel (batch.hip). Each body forms
// one work item with 256 threads on LDS the caller provides.
#pragma once

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
    } else if (t < A.nq + A.nb) {
        constexpr int ng = (P + 1) * (P + 1);
        const int64_t u = t - A.nq;
        const int b = (int)(u / ng), g = (int)(u % ng), g1 = g % (P + 1), g2 = g / (P + 1);
        const int e = A.band_list[b], e1 = e % D1.N, e2 = e / D1.N;
        const int r1 = (e1 * (P + 1) + g1) * (P + 1), r2 = (e2 * (P + 1) + g2) * (P + 1);
        A.c_band[u] = detj_local(A.cp, A.n1, P, e1, e2, D1.Bg + r1, D1.dBg + r1, D2.Bg + r2, D2.dBg + r2);
    } else if (t < A.nq + A.nb + A.n_nodes) {
        const int64_t u = t - A.nq - A.nb;
        const int e = A.cut_list[A.node_el[u]], e1 = e % D1.N, e2 = e / D1.N;
        double B1[P + 1], dB1[P + 1], B2[P + 1], dB2[P + 1];
        basis_eval_d<P>(D1.knots, P + e1, A.nx[u], B1, dB1);
        basis_eval_d<P>(D2.knots, P + e2, A.ny[u], B2, dB2);
        A.c_cut[u] = detj_local(A.cp, A.n1, P, e1, e2, B1, dB1, B2, dB2);
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
    int tile2;
    int ntx;                 // tiles along xi_1
};

template <int P>
struct IntCfg {
    static constexpr int W = 2 * P + 1;                  // band width
    static constexpr int QM = 4 * P + 2;                 // max WQ points in one support
    static constexpr int NR = 2 * P + 2;                 // support points of a regular function
    static constexpr int KS = 2 * (64 + P) + 2 * P + 2;  // max xi_1 points of a tile window
    static constexpr int KG = 4 * P + 2;                 // max xi_1 points of a boundary tile
    static constexpr bool WBREG = (P <= 5);              // w1 * B1 of each lane held in registers
};

// Tiles along xi_1: for N1 >= p+3, tile 0 holds the p+1 functions whose
// support touches the first element, the last tile those touching the last
// element (their elements carry p+1 points), and the tiles in between hold
// 64 "regular" functions each (2 points in every support element). Smaller
// patches use one generic tile.
__device__ __forceinline__ void tile_of(int tx, int ntx, int N1, int n1, int p, int& I1, int& nlive, bool& generic) {
    if (N1 < p + 3) {
        I1 = 0;
        nlive = n1;
        generic = true;
    } else if (tx == 0) {
        I1 = 0;
        nlive = p + 1;
        generic = true;
    } else if (tx == ntx - 1) {
        I1 = N1 - 1;
        nlive = p + 1;
        generic = true;
    } else {
        I1 = p + 1 + 64 * (tx - 1);
        nlive = min(64, (N1 - 2) - I1 + 1);
        generic = false;
    }
}

// Workgroups are handed to the XCDs round-robin; renumber them so that each
// XCD works on a contiguous range of rows (neighbouring rows share most of
// their coefficient points, which then stay in that XCD's L2).
__device__ __forceinline__ int xcd_block(int bid, int nb) {
    const int q = nb >> 3, r = nb & 7, x = bid & 7;
    return x * q + min(x, r) + (bid >> 3);
}

template <int P>
struct IntSmem {
    static constexpr int W = IntCfg<P>::W, QM = IntCfg<P>::QM, KS = IntCfg<P>::KS, KG = IntCfg<P>::KG;
    double sT[W][KS];                              // T[b][k - k1lo]
    double sWB2[QM][W];                            // w2 * B2 of the row
    double sB1[IntCfg<P>::WBREG ? KG : KS][P + 1]; // B1 at the window's points
    double sW1[64][QM + 1];                        // boundary tiles: w1 per lane
};

// One work item = one test-function row i2 and a tile tx of (up to) 64
// rows i1 (256 threads). Stage 1
// contracts xi_2 for every xi_1 point k of the tile's window,
//   T[b][k] = sum_q (w2 B2)[i2][q][b] c(k, k2lo + q),
// one point per thread; stage 2 contracts xi_1, one row i1 per lane,
//   M[a][b] = sum_k (w1 B1)[i1][k][a] T[b][k],
// the four wavefronts sharing the 2p+1 columns b. Every global load of a
// stage is issued before the first one is used.
template <int P>
__device__ __forceinline__ void interior_block(const IntArgs& A, int tx, int i2, IntSmem<P>& S) {
    using C = IntCfg<P>;
    constexpr int W = C::W, QM = C::QM, NR = C::NR, KG = C::KG;
    auto& sT = S.sT;
    auto& sWB2 = S.sWB2;
    auto& sB1 = S.sB1;
    auto& sW1 = S.sW1;

    const DirDev& D1 = A.d1;
    const DirDev& D2 = A.d2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int I1, nlive;
    bool generic;
    tile_of(tx, A.ntx, D1.N, D1.n, P, I1, nlive, generic);
    const int elo = max(0, I1 - P), ehi = min(D1.N - 1, I1 + nlive - 1);
    const int k1lo = wq_pt0(elo, D1.N, P);
    const int ks = wq_pt0(ehi + 1, D1.N, P) - k1lo;
    const int i1 = I1 + lane;

    // ---- tile tables (independent of the row)
    __syncthreads();   // LDS of the previous work item is free
    if (!generic && !C::WBREG) {
        for (int t = tid; t < ks * (P + 1); t += 256) sB1[t / (P + 1)][t % (P + 1)] = D1.Bq[(size_t)k1lo * (P + 1) + t];
    }
    if (generic) {
        constexpr int NGB = (KG * (P + 1) + 255) / 256;
        double gb[NGB];
#pragma unroll
        for (int u = 0; u < NGB; ++u) {
            const int t = tid + 256 * u;
            gb[u] = (t < ks * (P + 1)) ? D1.Bq[(size_t)k1lo * (P + 1) + t] : 0.0;
        }
        for (int t = tid; t < 64 * QM; t += 256) {
            const int l = t / QM, q = t % QM;
            sW1[l][q] = (l < nlive && q < D1.qmax) ? D1.W[(size_t)(I1 + l) * D1.qmax + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NGB; ++u) {
            const int t = tid + 256 * u;
            if (t < ks * (P + 1)) sB1[t / (P + 1)][t % (P + 1)] = gb[u];
        }
    }

    {
        if (i2 >= D2.n) return;
        const int k2lo = wq_pt0(max(0, i2 - P), D2.N, P);
        const int q2 = wq_pt0(min(D2.N - 1, i2) + 1, D2.N, P) - k2lo;
        const bool reg_row = (i2 >= P + 1) && (i2 <= D2.N - 2);  // q2 == NR, two points per element

        // ---- loads: row identity, xi_2 factors, coefficient column
        bool live = false;
        int64_t cid = 0;
        if (lane < nlive) {
            const int f = i2 * D1.n + i1;
            const int8_t cls = A.fcls[f];
            const int id = A.act_of[f];
            live = A.all_active ? (cls != FN_EXTERIOR) : (cls == FN_INTERIOR);
            cid = id;
        }
        double wb2 = 0.0;
        if (tid < QM * W) {
            const int q = tid / W;
            if (q < q2) wb2 = D2.WB[((size_t)i2 * D2.qmax) * W + tid];
        }
        const int kk = min(tid, ks - 1);
        double cv[QM];
        if (reg_row) {
            if (A.cwq) {
                const double* cc = A.cwq + (size_t)k2lo * D1.Q + k1lo + kk;
#pragma unroll
                for (int q = 0; q < NR; ++q) cv[q] = cc[(size_t)q * D1.Q];
            } else {
#pragma unroll
                for (int q = 0; q < NR; ++q) cv[q] = A.c.value;
            }
        } else {
            if (A.cwq) {
                const double* cc = A.cwq + (size_t)k2lo * D1.Q + k1lo + kk;
#pragma unroll
                for (int q = 0; q < QM; ++q) cv[q] = (q < q2) ? cc[(size_t)q * D1.Q] : 0.0;
            } else {
#pragma unroll
                for (int q = 0; q < QM; ++q) cv[q] = (q < q2) ? A.c.value : 0.0;
            }
        }
        if (tid < QM * W) sWB2[tid / W][tid % W] = wb2;
        if (!__syncthreads_or(live)) return;   // no row of the tile is formed here

        // ---- stage 1: contract xi_2 for every xi_1 point of the window
        if (tid < ks) {
            if (reg_row) {
                double T[W];
#pragma unroll
                for (int b = 0; b < W; ++b) T[b] = 0.0;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const int m2 = q >> 1;
#pragma unroll
                    for (int bl = 0; bl <= P; ++bl) T[m2 + bl] += sWB2[q][m2 + bl] * cv[q];
                }
#pragma unroll
                for (int b = 0; b < W; ++b) sT[b][tid] = T[b];
            } else {
#pragma unroll 1
                for (int b = 0; b < W; ++b) {
                    double Tb = 0.0;
#pragma unroll
                    for (int q = 0; q < QM; ++q) Tb += sWB2[q][b] * cv[q];
                    sT[b][tid] = Tb;
                }
            }
        }
        // regular lanes: w1 * B1 (or w1) at the 2p+2 support points, loaded while stage 1 finishes
        double wb[C::WBREG ? NR : 1][C::WBREG ? P + 1 : 1];
        double w1[C::WBREG ? 1 : NR];
        if (!generic) {
            const int i1c = min(i1, D1.n - 1);
            if constexpr (C::WBREG) {
                const double* row = D1.WB + (size_t)i1c * D1.qmax * W;
#pragma unroll
                for (int q = 0; q < NR; ++q)
#pragma unroll
                    for (int al = 0; al <= P; ++al) wb[q][al] = row[q * W + (q >> 1) + al];
            } else {
#pragma unroll
                for (int q = 0; q < NR; ++q) w1[q] = D1.W[(size_t)i1c * D1.qmax + q];
            }
        }
        __syncthreads();

        // ---- stage 2: contract xi_1, one row per lane, columns b shared by the wavefronts
        if (!generic) {
            // regular lane: support points 2*lane .. 2*lane + 2p+1 of the window, two per element
#pragma unroll 1
            for (int b = wave; b < W; b += 4) {
                double acc[W];
#pragma unroll
                for (int a = 0; a < W; ++a) acc[a] = 0.0;
#pragma unroll
                for (int m = 0; m <= P; ++m) {
                    const int k = 2 * lane + 2 * m;
                    const double2 t2 = *reinterpret_cast<const double2*>(&sT[b][k]);
                    if constexpr (C::WBREG) {
#pragma unroll
                        for (int al = 0; al <= P; ++al) acc[m + al] += wb[2 * m][al] * t2.x + wb[2 * m + 1][al] * t2.y;
                    } else {
                        const double wa = w1[2 * m] * t2.x, wc = w1[2 * m + 1] * t2.y;
#pragma unroll
                        for (int al = 0; al <= P; ++al) acc[m + al] += wa * sB1[k][al] + wc * sB1[k + 1][al];
                    }
                }
                if (live)
#pragma unroll
                    for (int a = 0; a < W; ++a) A.vals[(size_t)(a * W + b) * A.n_act + cid] = acc[a];
            }
        } else if (live) {
            const int k0_1 = wq_pt0(max(0, i1 - P), D1.N, P) - k1lo;
#pragma unroll 1
            for (int b = wave; b < W; b += 4) {
                double acc[W];
#pragma unroll
                for (int a = 0; a < W; ++a) acc[a] = 0.0;
#pragma unroll
                for (int m = 0; m <= P; ++m) {
                    const int e = i1 - P + m;
                    if (e < 0 || e >= D1.N) continue;
                    const int kb = wq_pt0(e, D1.N, P) - k1lo, ke = wq_pt0(e + 1, D1.N, P) - k1lo;
                    for (int k = kb; k < ke; ++k) {
                        const double wt = sW1[lane][k - k0_1] * sT[b][k];
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

// Tiles along xi_1 of a patch with N1 elements.
__host__ __device__ inline int interior_ntx(int N1, int p) {
    return (N1 < p + 3) ? 1 : 2 + ((N1 - 2) - (p + 1) + 1 + 63) / 64;
}

// ------------------------------------------------------------ cut element matrices
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
struct CutECfg {
    static constexpr int L = (P + 1) * (P + 1);
    static constexpr int CH = (P <= 4) ? 256 : ((P <= 6) ? 128 : 64);  // nodes staged at a time
    static constexpr int NR = P * (P + 1) / 2;                          // reciprocal denominators per direction
};

template <int P>
struct CutESmem {
    double sPhi[CutECfg<P>::CH][CutECfg<P>::L];
    double sWc[CutECfg<P>::CH];
    double sRec[2][CutECfg<P>::NR + 1];
};

// Local matrix of cut element c (256 threads): the element's nodes are
// staged CH at a time with their basis products (one node per thread, the
// element's reciprocal knot differences shared, so no divisions per node);
// thread t owns entries of the upper triangle and mirrors them.
template <int P>
__device__ __forceinline__ void cut_elem_body(const CutEArgs& A, int c, CutESmem<P>& S) {
    using C = CutECfg<P>;
    constexpr int L = C::L, CH = C::CH, NR = C::NR;
    constexpr int NE = L * (L + 1) / 2;
    constexpr int PER = (NE + 255) / 256;
    auto& sPhi = S.sPhi;
    auto& sWc = S.sWc;
    if (c >= A.n_cut) return;
    const int e = A.cut_list[c], e1 = e % A.d1.N, e2 = e / A.d1.N;
    const int nb = A.node_off[c], ne = A.node_off[c + 1];
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
    int elc[PER], emc[PER];  // clamped: threads past the triangle accumulate a discarded entry
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        elc[k] = max(el[k], 0);
        emc[k] = max(em[k], 0);
    }
    __syncthreads();  // LDS of the previous work item is free
    if (threadIdx.x < 2 * NR) {
        const int d = threadIdx.x / NR, idx = threadIdx.x % NR;
        S.sRec[d][idx] = basis_rec<P>(d ? A.d2.knots : A.d1.knots, P + (d ? e2 : e1), idx);
    }
    for (int base = nb; base < ne; base += CH) {
        __syncthreads();
        if (threadIdx.x < CH) {
            const int n = base + threadIdx.x;
            if (n < ne) {
                const double x = A.nx[n], y = A.ny[n], w = A.nw[n];
                const double cv = A.c.is_const ? A.c.value : A.c.cut[n];
                double B1[P + 1], B2[P + 1];
                basis_eval_rec<P>(A.d1.knots, P + e1, S.sRec[0], x, B1);
                basis_eval_rec<P>(A.d2.knots, P + e2, S.sRec[1], y, B2);
#pragma unroll
                for (int a2 = 0; a2 <= P; ++a2)
#pragma unroll
                    for (int a1 = 0; a1 <= P; ++a1) sPhi[threadIdx.x][a2 * (P + 1) + a1] = B1[a1] * B2[a2];
                sWc[threadIdx.x] = w * cv;
            } else {
                sWc[threadIdx.x] = 0.0;
#pragma unroll
                for (int l = 0; l < L; ++l) sPhi[threadIdx.x][l] = 0.0;
            }
        }
        __syncthreads();
        const int cnt = min(CH, ne - base);
        // no branch in the loop body, so the LDS reads of several nodes are issued ahead
#pragma unroll 8
        for (int n = 0; n < cnt; ++n) {
            const double wc = sWc[n];
#pragma unroll
            for (int k = 0; k < PER; ++k) acc[k] += wc * sPhi[n][elc[k]] * sPhi[n][emc[k]];
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
    const int* region;      // DWQ: box of inside elements left to k_dwq_rows (nullptr: none)
    double* vals;
    int64_t n_act;
};

// One workgroup per row; the row's per-direction Gauss factors
// F1[m1][g1][a] = w_g1 B_i1 B_{i1+a-p} (element e1 = i1-p+m1), F2 likewise,
// the element classes and c at the Gauss points of its support elements are
// staged in LDS; thread (a, b) then sums over the elements shared with its
// column: Gauss on inside elements (sum-factorised), the cut element matrix
// on cut elements.
template <int P>
struct CutRSmem {
    double sF1[P + 1][P + 1][2 * P + 1];
    double sF2[P + 1][P + 1][2 * P + 1];
    double sX[P + 1][P + 1][(P + 1) * (P + 1)];  // inside element: c at its Gauss points (else 0)
    double sE[P + 1][P + 1][(P + 1) * (P + 1)];  // cut element: row i of its local matrix (else 0)
    int sCls[P + 1][P + 1];
    int sId[P + 1][P + 1];
};

template <int P>
__device__ __forceinline__ void cut_row_body(const CutRowArgs& A, int r, CutRSmem<P>& S) {
    constexpr int W = 2 * P + 1, L = (P + 1) * (P + 1), NP = P + 1;
    auto& sF1 = S.sF1;
    auto& sF2 = S.sF2;
    auto& sX = S.sX;
    auto& sE = S.sE;
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
    if (A.region && A.region[(size_t)r * 8] >= 0) {
        bx0 = A.region[(size_t)r * 8];
        bx1 = A.region[(size_t)r * 8 + 1];
        by0 = A.region[(size_t)r * 8 + 4];
        by1 = A.region[(size_t)r * 8 + 5];
    }
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
    // per support element: c at its Gauss points (inside) or row i of its local matrix (cut)
    for (int t = tid; t < NP * NP * L; t += nt) {
        const int m2 = t / (NP * L), m1 = (t / L) % NP, g = t % L;
        const int cls = sCls[m2][m1];
        double v = 0.0, w = 0.0;
        if (cls == EL_INSIDE) v = A.c.is_const ? A.c.value : A.c.band[(size_t)sId[m2][m1] * L + g];
        else if (cls == EL_CUT) w = A.E[((size_t)sId[m2][m1] * L + (P - m2) * NP + (P - m1)) * L + g];
        sX[m2][m1][g] = v;
        sE[m2][m1][g] = w;
    }
    __syncthreads();
    const int s = tid;
    if (s >= W * W) return;
    const int a = s / W, b = s % W;          // column offsets a-p, b-p
    const int j1 = i1 + a - P, j2 = i2 + b - P;
    double val = 0.0;
    if (j1 >= 0 && j1 < D1.n && j2 >= 0 && j2 < D2.n && A.act_of[j2 * D1.n + j1] >= 0) {
        // every support element, without branches: the Gauss factors F vanish off the column's
        // overlap and sX / sE hold zeros where the element is not inside / cut
#pragma unroll
        for (int m2 = 0; m2 <= P; ++m2) {
            const int l2 = j2 - (i2 - P + m2);  // column's local index in the element, direction 2
#pragma unroll
            for (int m1 = 0; m1 <= P; ++m1) {
                const int l1 = j1 - (i1 - P + m1);
                double sum = 0.0;
#pragma unroll
                for (int g2 = 0; g2 < NP; ++g2) {
                    double in = 0.0;
#pragma unroll
                    for (int g1 = 0; g1 < NP; ++g1) in += sF1[m1][g1][a] * sX[m2][m1][g2 * NP + g1];
                    sum += sF2[m2][g2][b] * in;
                }
                const bool ov = (l1 >= 0 && l1 <= P && l2 >= 0 && l2 <= P);
                const double ev = sE[m2][m1][ov ? l2 * NP + l1 : 0];
                val += sum + (ov ? ev : 0.0);
            }
        }
    }
    A.vals[(size_t)s * A.n_act + row] = val;
}


IntArgs int_args(Plan& P, const iga_coeff& c, double* vals);
CutEArgs cute_args(Plan& P, const iga_coeff& c);
CutRowArgs cutr_args(Plan& P, const iga_coeff& c, double* vals);

}  // namespace iga
