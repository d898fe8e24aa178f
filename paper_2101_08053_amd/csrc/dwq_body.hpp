// Device bodies of discontinuous weighted quadrature (Sect. 3.3, Eqs. (9)-(10)),
// shared by the one-patch kernels (dwq.hip) and the batched launches
// (batch.hip): the side rules of a group of (direction, interior knot, side)
// slots and the box contribution of one element-formed row.
#pragma once

#include "bounds.hpp"
#include "plan.hpp"

namespace iga {

template <int P>
struct DwqCfg {
    static constexpr int KQ = 4 * P + 2;  // points of one side list / of one support
    static constexpr int NK = 3 * P + 2;  // local refined knots used
    static constexpr int M = 2 * P + 1;   // trial functions of a refined system
};

// One (direction, interior knot, side) slot per 128-thread workgroup: the
// body of k_dwq_sides and of the batched side launches.
// ------------------------------------------------ side rules, four lanes per system
// For every (direction, interior knot t = bp[s], side) slot: the side's
// first element gets p+1 points (the two WQ points plus nested ones, placed
// round robin from t in the three equal gaps); t is inserted p times (Eq.
// (10)) giving S with B_c = sum_r S[r][c] B~_r; the minimum-norm systems
// (5) of the p+1 refined functions touching that element are solved, and
// w^_{.,i} = sum_r S[r][i] w~_{.,r}. Both sides are built in the local
// coordinate u = |x - t|, so the low side is the mirror image of the high
// one.
//
// A workgroup of 256 threads takes SPW slots; each refined system (at most
// 4p points x (2p+1) trial functions) is solved by a quad of lanes holding
// its A^T row-distributed in registers (row k in lane k % 4), by Householder
// QR with quad reductions (DPP moves inside the quad): the systems are far
// too small to spread over a wavefront. The slot's points and refined knots
// are found by one lane, S by p lanes, and the quads of a slot then combine
// the refined solutions into the rules of its p local functions.
template <int P>
struct DwqQuadCfg {
    static constexpr int KQ = 4 * P + 2;   // point capacity of a side list (output layout)
    static constexpr int QS = 4 * P;       // points of one system at most
    static constexpr int RPL = P;          // rows of A^T per lane (QS / 4)
    static constexpr int NK = 3 * P + 2;   // local refined knots used
    static constexpr int M = 2 * P + 1;    // trial functions of a refined system
    static constexpr int SPW = 64 / (P + 1);  // slots per workgroup (64 quads)
    static constexpr int NSYS = SPW * (P + 1);
};
__host__ __device__ constexpr int dwq_side_spw(int p) { return 64 / (p + 1); }
constexpr int kDwqSideThreads = 256;

template <int P>
__device__ __forceinline__ void dwq_sides_body(const DirDev& D1, const DirDev& D2, const double* __restrict__ gx,
                                               const double* __restrict__ gw, int* __restrict__ status, int blk) {
    using C = DwqQuadCfg<P>;
    constexpr int KQ = C::KQ, QS = C::QS, RPL = C::RPL, NK = C::NK, M = C::M, SPW = C::SPW, NSYS = C::NSYS;
    __shared__ double sY[NSYS * QS];     // [system][k]: the minimum-norm solutions, local order
    __shared__ double sRK[SPW][NK];      // refined local knots: 0 (p+1 times), then the side's knots
    __shared__ double sU[SPW][QS];       // local coordinate of each point, local order
    __shared__ int sEl[SPW][QS];         // local element of each point
    __shared__ double sX[SPW][QS];       // coordinates, increasing x
    __shared__ int sOel[SPW][QS], sOk[SPW][QS];
    __shared__ int sCnt[SPW][P + 2];     // points in local elements < k
    __shared__ double sS[SPW][P + 1][P]; // B_c = sum_r S[r][c] B~_r on the side (local c)
    __shared__ int sInfo[SPW][3];

    const int tid = threadIdx.x, g = tid & 3, sys = tid >> 2;
    const int sl = sys / (P + 1), r = sys - sl * (P + 1);
    const int nslot1 = 2 * (D1.N - 1), nslot = nslot1 + 2 * (D2.N - 1);
    const int gs = blk * SPW + sl;
    const bool on = sys < NSYS && gs < nslot;
    int slot = gs, d = 0;
    if (slot >= nslot1) {
        slot -= nslot1;
        d = 1;
    }
    const DirDev& D = d ? D2 : D1;
    const int N = D.N;
    const int s = slot / 2 + 1;
    const bool high = (slot & 1) != 0;
    const int nk = N + 2 * P + 1;
    const double t = on ? D.knots[P + s] : 0.0;

    if (on && r == 0 && g == 0) {  // the slot's points and refined knots
        const int nE = high ? N - s : s;
        const int nEl = min(nE, P + 1);
        const int nRK = high ? nk - s : s + 2 * P + 1;
        for (int m = 0; m < NK; ++m) {
            double v = 0.0;
            if (m > P) {
                const int kk = min(m, nRK - 1) - P - 1;
                v = high ? D.knots[s + P + 1 + kk] - t : t - D.knots[s + P - 1 - kk];
            }
            sRK[sl][m] = v;
        }
        int np = 0;
        const int e_lo = high ? s : s - nEl, e_hi = high ? s + nEl - 1 : s - 1, e_adj = high ? s : s - 1;
        for (int e = e_lo; e <= e_hi; ++e) {
            const int ne = (e == 0 || e == N - 1) ? P + 1 : 2;
            const double a = D.knots[P + e], b = D.knots[P + e + 1];
            const int k0 = wq_pt0(e, N, P);
            const int nadd = (e == e_adj) ? max(0, P + 1 - ne) : 0;
            if (nadd == 0) {
                for (int j = 1; j <= ne; ++j) {
                    sX[sl][np] = a + (b - a) * j / (ne + 1);
                    sOel[sl][np] = e;
                    sOk[sl][np] = k0 + j - 1;
                    ++np;
                }
            } else {
                const double E[4] = {a, a + (b - a) * 1 / 3, a + (b - a) * 2 / 3, b};
                for (int gg = 0; gg < 3; ++gg) {
                    const int mg = high ? (nadd + 2 - gg) / 3 : (nadd + gg) / 3;
                    for (int j = 1; j <= mg; ++j) {
                        sX[sl][np] = E[gg] + (E[gg + 1] - E[gg]) * j / (mg + 1);
                        sOel[sl][np] = e;
                        sOk[sl][np] = -1;
                        ++np;
                    }
                    if (gg < 2) {
                        sX[sl][np] = E[gg + 1];
                        sOel[sl][np] = e;
                        sOk[sl][np] = k0 + gg;
                        ++np;
                    }
                }
            }
        }
        for (int k = 0; k <= P + 1; ++k) sCnt[sl][k] = 0;
        for (int q = 0; q < np; ++q) {
            const int qo = high ? q : np - 1 - q;
            sU[sl][q] = high ? sX[sl][qo] - t : t - sX[sl][qo];
            sEl[sl][q] = high ? sOel[sl][qo] - s : s - 1 - sOel[sl][qo];
            sCnt[sl][sEl[sl][q] + 1]++;
        }
        for (int k = 1; k <= P + 1; ++k) sCnt[sl][k] += sCnt[sl][k - 1];
        sInfo[sl][0] = np;
        sInfo[sl][1] = nRK - P - 1;  // refined functions on the side
        sInfo[sl][2] = nEl;
    }
    if (on && r < P && g == 1) {
        // Eq. (10) p times on the local coarse knots, for the unit vector of local function c = r
        const int c = r;
        double K[3 * P + 2], Pc[2 * P + 1], Qn[2 * P + 1];
        int L = 2 * P + 2, nf = P + 1;
        for (int m = 0; m < L; ++m) K[m] = high ? D.knots[s + m] - t : t - D.knots[s + 2 * P - m];
        for (int j = 0; j < 2 * P + 1; ++j) Pc[j] = (j == c) ? 1.0 : 0.0;
        for (int ins = 0; ins < P; ++ins) {
            int k = 0;
            while (k + 1 < L && K[k + 1] <= 0.0) ++k;  // span of the inserted knot
            for (int j = 0; j <= nf; ++j) {
                double al;
                if (j <= k - P) al = 1.0;
                else if (j <= k) al = (0.0 - K[j]) / (K[j + P] - K[j]);
                else al = 0.0;
                const double pj = (j < nf) ? Pc[j] : 0.0, pm = (j >= 1) ? Pc[j - 1] : 0.0;
                Qn[j] = al * pj + (1.0 - al) * pm;
            }
            for (int j = 0; j <= nf; ++j) Pc[j] = Qn[j];
            for (int m = L; m > k + 1; --m) K[m] = K[m - 1];
            K[k + 1] = 0.0;
            ++L;
            ++nf;
        }
        for (int rr = 0; rr <= P; ++rr) sS[sl][rr][c] = Pc[P + rr];
    }
    __syncthreads();

    // ---- the quad's refined system: A[c][k] = B~_c(u_k), b[c] = int B~_c B~_r. Every lane
    // runs it (the quad reductions need all lanes); quads without a system solve zeros.
    const int np = on ? sInfo[sl][0] : 0, n_fun = on ? sInfo[sl][1] : 0, nEl = on ? sInfo[sl][2] : 1;
    const bool solve = on && r < n_fun;
    const int slc = on ? sl : 0;
    const double* rk = sRK[slc];
    const int kr = min(r, nEl - 1);                         // last local element of supp B~_r
    const int q = solve ? sCnt[slc][kr + 1] : 0;            // its points
    const int m = solve ? min(r + P, n_fun - 1) + 1 : 0;    // trial functions 0..m-1
    // (register arrays take compile-time indices only, selected by comparison)
    double A[RPL][M];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int k = 4 * i + g;
        double Nv[P + 1];
        int el = 0;
        if (k < q) {
            el = sEl[slc][k];
            basis_eval<P>(rk, P + el, sU[slc][k], Nv);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double v = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) v = (k < q && c < m && c == el + a) ? Nv[a] : v;
            A[i][c] = v;
        }
    }
    // moments over the elements of supp B~_r, (p+1)-point Gauss, the points dealt to the quad's lanes
    double mom[M];
#pragma unroll
    for (int c = 0; c < M; ++c) mom[c] = 0.0;
    for (int pg = g; pg < (solve ? (kr + 1) * (P + 1) : 0); pg += 4) {
        const int k = pg / (P + 1), gp = pg - k * (P + 1);
        const double ua = rk[P + k], ub = rk[P + k + 1];
        const double xg = ua + (ub - ua) * (gx[gauss_off(P + 1) + gp] + 1.0) * 0.5;
        const double wgt = gw[gauss_off(P + 1) + gp] * (ub - ua) * 0.5;
        double Nv[P + 1];
        basis_eval<P>(rk, P + k, xg, Nv);
        double br = 0.0;
#pragma unroll
        for (int a = 0; a <= P; ++a) br = (r == k + a) ? Nv[a] : br;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double nc = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) nc = (c == k + a) ? Nv[a] : nc;
            mom[c] += wgt * nc * br;
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) mom[c] = quad_sum(mom[c]);

    bool singular = false;
    double y[RPL];
    quad_min_norm<M, RPL>(A, q, m, mom, y, singular);
    // residual of the moment equations, A rebuilt at the lane's points
    double res[M];
#pragma unroll
    for (int c = 0; c < M; ++c) res[c] = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int k = 4 * i + g;
        if (k < q) {
            const int el = sEl[slc][k];
            double Nv[P + 1];
            basis_eval<P>(rk, P + el, sU[slc][k], Nv);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double nc = 0.0;
#pragma unroll
                for (int a = 0; a <= P; ++a) nc = (c == el + a) ? Nv[a] : nc;
                res[c] += nc * y[i];
            }
        }
    }
    double rmax = 0.0, bmax = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double rc = quad_sum(res[c]);
        if (c < m) {
            rmax = fmax(rmax, fabs(rc - mom[c]));
            bmax = fmax(bmax, fabs(mom[c]));
        }
    }
    if (solve && g == 0 && (singular || !(rmax <= 1e-12 * bmax))) atomicExch(status, IGA_E_SINGULAR_WEIGHTS);
    if (sys < NSYS) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) sY[sys * QS + 4 * i + g] = solve ? y[i] : 0.0;
    }
    __syncthreads();

    // ---- the slot's p rules on its points (lanes of the slot's quads), and its point list
    if (!on) return;
    const int sys0 = sl * (P + 1), lane_in = tid - 4 * sys0, nlane = 4 * (P + 1);
    const int nr = min(P + 1, n_fun);
    for (int o = lane_in; o < P * KQ; o += nlane) {
        const int ii = o / KQ, qo = o - ii * KQ;
        const int c = high ? ii : P - 1 - ii;
        double v = 0.0;
        if (qo < np) {
            const int ql = high ? qo : np - 1 - qo;
            for (int rr = 0; rr < nr; ++rr) v += sS[sl][rr][c] * sY[(sys0 + rr) * QS + ql];
        }
        D.dq_w[((size_t)slot * P + ii) * KQ + qo] = v;
    }
    for (int qo = lane_in; qo < KQ; qo += nlane) {
        D.dq_x[(size_t)slot * KQ + qo] = (qo < np) ? sX[sl][qo] : 0.0;
        D.dq_el[(size_t)slot * KQ + qo] = (qo < np) ? sOel[sl][qo] : -1;
        D.dq_k[(size_t)slot * KQ + qo] = (qo < np) ? sOk[sl][qo] : -1;
    }
    if (lane_in == 0) D.dq_n[slot] = np;
}

// ------------------------------------------------------------ box rows
struct DwqRowArgs {
    DirDev d1, d2;
    CoefView c;
    const double* geom_cp;
    const int* rows;
    int n_rows;
    const int* fn_of;
    const int* act_of;
    const int* region;
    double* vals;
    int64_t n_act;
    double* boxp = nullptr;  // if set: box parts to boxp[r][(2p+1)^2] (a later launch adds them) instead of vals
};

// One workgroup per formed row with a box: the two 1-D rules restricted to
// the box (coarse WQ rule on a whole range, the side list otherwise) are
// staged in LDS with the band's basis values, c on the tensor points (the WQ
// grid where both coordinates are WQ points, |det J| evaluated otherwise),
// then T[b][q1] = sum_q2 w2 B2 c and M[a][b] = sum_q1 w1 B1 T[b][q1] is added
// to the row.
// Point `lane` of row i's 1-D rule in one direction restricted to the box
// range reg = {lo, hi, s, side}: the coarse WQ rule on a whole range of
// elements (s < 0; lanes count the WQ points of elements lo..hi), the side
// list of interior knot s otherwise (lanes count its points; those outside
// lo..hi are dropped). k is the point's WQ index, -1 for a nested point.
template <int P>
__device__ __forceinline__ bool dwq_rule_point(const DirDev& D, int i, const int* __restrict__ reg, int lane,
                                               double& x, double& w, int& e, int& k) {
    constexpr int KQ = DwqCfg<P>::KQ;
    const int lo = reg[0], hi = reg[1], s = reg[2], sd = reg[3];
    x = 0.0;
    w = 0.0;
    e = 0;
    k = -1;
    if (s < 0) {
        const int k0 = wq_pt0(max(0, i - P), D.N, P);
        const int kb = wq_pt0(lo, D.N, P), ke = wq_pt0(hi + 1, D.N, P);
        const int kk = kb + lane;
        if (kk >= ke) return false;
        x = D.xq[kk];
        e = D.eq[kk];
        k = kk;
        w = D.W[(size_t)i * D.qmax + (kk - k0)];
        return true;
    }
    const int slot = 2 * (s - 1) + sd;
    if (lane >= D.dq_n[slot]) return false;
    e = D.dq_el[(size_t)slot * KQ + lane];
    x = D.dq_x[(size_t)slot * KQ + lane];
    k = D.dq_k[(size_t)slot * KQ + lane];
    w = D.dq_w[((size_t)slot * P + (i - s)) * KQ + lane];
    return e >= lo && e <= hi;
}

template <int P>
__device__ __forceinline__ void dwq_rows_body(const DwqRowArgs& A, int r) {
    constexpr int W = 2 * P + 1, KQ = DwqCfg<P>::KQ;
    __shared__ double sX[2][KQ], sWt[2][KQ];
    __shared__ int sE[2][KQ], sK[2][KQ], sNq[2];
    __shared__ double sB[2][KQ][W];
    __shared__ double sC[KQ][KQ + 1];
    __shared__ double sT[W][KQ];
    if (r >= A.n_rows) return;
    const int* reg = A.region + (size_t)r * 8;
    if (reg[0] < 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = A.rows[r];
    const int f = A.fn_of[row];
    const int i1 = f % A.d1.n, i2 = f / A.d1.n;
    if (wave < 2) {
        const int d = wave;
        const DirDev& D = d ? A.d2 : A.d1;
        const int i = d ? i2 : i1;
        double x, w;
        int e, k;
        const bool ok = dwq_rule_point<P>(D, i, reg + 4 * d, lane, x, w, e, k);
        const unsigned long long msk = __ballot(ok);
        const int pos = __popcll(msk & ((1ull << lane) - 1ull));
        if (ok) {
            sX[d][pos] = x;
            sE[d][pos] = e;
            sK[d][pos] = k;
            sWt[d][pos] = w;
            double Nv[P + 1];
            basis_eval<P>(D.knots, P + e, x, Nv);
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const int j = i + b - P;
                sB[d][pos][b] = (j >= e && j <= e + P) ? Nv[j - e] : 0.0;
            }
        }
        if (lane == 0) sNq[d] = __popcll(msk);
    }
    __syncthreads();
    const int n1q = sNq[0], n2q = sNq[1];
    for (int tt = tid; tt < n1q * n2q; tt += 256) {
        const int q1 = tt % n1q, q2 = tt / n1q;
        double cv;
        if (A.c.is_const) {
            cv = A.c.value;
        } else if (sK[0][q1] >= 0 && sK[1][q2] >= 0) {
            cv = A.c.wq[(size_t)sK[1][q2] * A.d1.Q + sK[0][q1]];
        } else {  // a nested coordinate: |det J| of the geometry there
            const int e1 = sE[0][q1], e2 = sE[1][q2];
            double B1[P + 1], dB1[P + 1], B2[P + 1], dB2[P + 1];
            basis_eval_d<P>(A.d1.knots, P + e1, sX[0][q1], B1, dB1);
            basis_eval_d<P>(A.d2.knots, P + e2, sX[1][q2], B2, dB2);
            cv = detj_local(A.geom_cp, A.d1.n, P, e1, e2, B1, dB1, B2, dB2);
        }
        sC[q1][q2] = cv;
    }
    __syncthreads();
    for (int tt = tid; tt < W * n1q; tt += 256) {
        const int b = tt / n1q, q1 = tt % n1q;
        double acc = 0.0;
        for (int q2 = 0; q2 < n2q; ++q2) acc += sWt[1][q2] * sB[1][q2][b] * sC[q1][q2];
        sT[b][q1] = acc;
    }
    __syncthreads();
    for (int t = tid; t < W * W; t += 256) {  // (2p+1)^2 slots: more than 256 at p = 8
        const int a = t / W, b = t % W;
        const int j1 = i1 + a - P, j2 = i2 + b - P;
        if (j1 >= 0 && j1 < A.d1.n && j2 >= 0 && j2 < A.d2.n && A.act_of[j2 * A.d1.n + j1] >= 0) {
            double acc = 0.0;
            for (int q1 = 0; q1 < n1q; ++q1) acc += sWt[0][q1] * sB[0][q1][a] * sT[b][q1];
            if (A.boxp)
                A.boxp[band_index(r, A.n_rows, t, W * W)] = acc;
            else
                A.vals[band_index(t, W * W, row, A.n_act)] += acc;
        }
    }
}

}  // namespace iga
