// Formation of the trimmed mass matrix (Eqs. (6)-(7), Sects. 3.1-3.2).
//
//  * k_interior: rows of interior test functions by weighted quadrature and
//    sum factorisation. A workgroup owns one i2 and a tile of 128
//    consecutive i1 (one per thread). It first contracts the xi_2 direction
//    for every xi_1 point of the tile,
//        T[b][k1] = sum_{k2 in Q_i2} w2_{k2,i2} B_{i2+b}(x_k2) c(x_k1, x_k2),
//    into LDS, then each thread contracts xi_1 for its own row,
//        M[a][b] = sum_{k1 in Q_i1} w1_{k1,i1} B_{i1+a}(x_k1) T[b][k1],
//    and writes the (2p+1)^2 band of the row slot-major (coalesced across
//    lanes, no atomics).
//  * k_cut_elem: local matrices sum_g w_g c_g B_l B_m of each cut element
//    from its cut-rule nodes (one workgroup per element).
//  * k_cut_rows: rows formed element-wise (hybrid Gauss, Sect. 3.2: cut
//    rows; the reference: every row): element Gauss on inside elements of
//    the support, the cut element matrices on cut elements. One workgroup per
//    row, one thread per band slot.
#include <hip/hip_ext.h>

#include "form_body.hpp"

namespace iga {

// ------------------------------------------------------------ points
// Coordinates of the WQ grid and band Gauss points in the rule-point table,
// and of the cut nodes if given (the set-up's node kernel writes those itself).
__global__ void k_points(DirDev D1, DirDev D2, int p, const int* __restrict__ band_list, int nb,
                         const double* __restrict__ nx, const double* __restrict__ ny, int nn,
                         double* __restrict__ xy) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = (int64_t)D1.Q * D2.Q;
    double x, y;
    if (t < nq) {
        x = D1.xq[t % D1.Q];
        y = D2.xq[t / D1.Q];
    } else if (t < nq + nb) {
        const int ng = (p + 1) * (p + 1);
        const int u = (int)(t - nq), b = u / ng, g = u % ng, g1 = g % (p + 1), g2 = g / (p + 1);
        const int e = band_list[b], e1 = e % D1.N, e2 = e / D1.N;
        x = D1.xg[e1 * (p + 1) + g1];
        y = D2.xg[e2 * (p + 1) + g2];
    } else if (t < nq + nb + nn) {
        const int u = (int)(t - nq - nb);
        x = nx[u];
        y = ny[u];
    } else {
        return;
    }
    xy[2 * t] = x;
    xy[2 * t + 1] = y;
}

void launch_points(Plan& P, hipStream_t s, bool with_nodes) {
    DirDev &D1 = P.dir[0], &D2 = P.dir[1];
    const int64_t nq = (int64_t)D1.Q * D2.Q;
    const int nb = (int)P.n_band * (P.p + 1) * (P.p + 1);
    const int nn = with_nodes ? (int)P.n_nodes : 0;
    const int64_t n = nq + nb + nn;
    klaunch(P, "k_points", k_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D1, D2, P.p, P.band_list, nb,
                       P.node_x, P.node_y, nn, P.pts_xy);
}

// ------------------------------------------------------- coefficient
template <int P>
__global__ void __launch_bounds__(256) k_coef(CoefArgs A, int64_t t0, int64_t t1) {
    const int64_t t = t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < t1) coef_point<P>(A, t);
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

CoefArgs coef_args(Plan& P, const iga_coeff& c) {
    return CoefArgs{P.dir[0], P.dir[1], c.geom_cp, P.n1, P.band_list, (int)P.n_band, P.cut_list, P.node_el,
                    P.node_x, P.node_y, (int)P.n_nodes, P.c_wq, P.c_band, P.c_cut,
                    (int64_t)P.dir[0].Q * P.dir[1].Q, (int64_t)P.n_band * (P.p + 1) * (P.p + 1), nullptr};
}

void launch_coef(Plan& P, const iga_coeff& c, hipStream_t s, int part, bool with_points) {
    if (c.kind != IGA_COEF_GEOM_DETJ) return;
    CoefArgs A = coef_args(P, c);
    if (with_points) A.xy = P.pts_xy;
    // part 0: every rule point; 1: the WQ grid; 2: band Gauss points and cut nodes; 3: band; 4: cut nodes.
    // One point per thread: on one patch (about 10^5 - 10^6 grid points) the per-point launch fills the
    // GPU beside the trimming chain better than the sum-factorised grid tiles the batch uses (measured
    // 9 vs 19 us at 256^2, p = 4, in the two-stream formation).
    const int64_t t0 = (part == 2 || part == 3) ? A.nq : (part == 4 ? A.nq + A.nb : 0);
    const int64_t t1 = (part == 1) ? A.nq : (part == 3 ? A.nq + A.nb : A.nq + A.nb + A.n_nodes);
    if (t1 <= t0) return;
    dim3 g((unsigned)((t1 - t0 + 255) / 256)), b(256);
    switch (P.p) {
#define CASE(PP) \
    case PP: klaunch(P, "k_coef<" #PP ">", k_coef<PP>, g, b, 0, s, A, t0, t1); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

// ------------------------------------------------------- interior rows
template <int P>
__global__ void __launch_bounds__(Int2Cfg<P>::NT) k_interior(IntArgs A) {
    __shared__ __align__(16) Int2Smem<P> S;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int i2 = blk / A.ntx;
    interior_rows_block<P>(A, blk - i2 * A.ntx, i2, S);
}

// The interior rows and c = |det J| at the band Gauss points in one launch
// (the inside sums of the rows formed element-wise read those next): the
// first ncb workgroups take NT points each, the others the interior tiles.
// ncb is a multiple of 8, so the tiles' XCD renumbering sees the same
// round-robin as in the launch of their own.
template <int P>
__global__ void __launch_bounds__(Int2Cfg<P>::NT) k_interior_coef(IntArgs A, CoefArgs C, int ncb, int64_t t0,
                                                                  int64_t t1) {
    __shared__ __align__(16) Int2Smem<P> S;
    if ((int)blockIdx.x < ncb) {
        const int64_t t = t0 + (int64_t)blockIdx.x * Int2Cfg<P>::NT + threadIdx.x;
        if (t < t1) coef_point<P>(C, t);
        return;
    }
    const int blk = xcd_block((int)blockIdx.x - ncb, (int)gridDim.x - ncb);
    const int i2 = blk / A.ntx;
    interior_rows_block<P>(A, blk - i2 * A.ntx, i2, S);
}

static const char* const kInteriorNames[IGA_MAXP + 1] = {"", "k_interior<1>", "k_interior<2>", "k_interior<3>",
                                                          "k_interior<4>", "k_interior<5>", "k_interior<6>",
                                                          "k_interior<7>", "k_interior<8>"};

template <int P>
static void launch_interior_p(Plan& Pl, IntArgs A, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    A.ntx = interior2_ntx(Pl.N1, P);
    const int nb = A.ntx * Pl.n2;
    const dim3 blk(Int2Cfg<P>::NT);
    if (t0) hipExtLaunchKernelGGL(k_interior<P>, dim3(nb), blk, 0, s, t0, t1, 0, A);  // events bracket the dispatch
    else klaunch(Pl, kInteriorNames[P], k_interior<P>, dim3(nb), blk, 0, s, A);
}

template <int P>
static void launch_interior_coef_p(Plan& Pl, IntArgs A, CoefArgs C, hipStream_t s) {
    A.ntx = interior2_ntx(Pl.N1, P);
    const int nb = A.ntx * Pl.n2;
    const int64_t t0 = C.nq, t1 = C.nq + C.nb;
    const int ncb = (int)(((t1 - t0 + Int2Cfg<P>::NT - 1) / Int2Cfg<P>::NT + 7) / 8 * 8);
    klaunch(Pl, kInteriorNames[P], k_interior_coef<P>, dim3(nb + ncb), dim3(Int2Cfg<P>::NT), 0, s, A, C, ncb, t0, t1);
}

IntArgs int_args(Plan& P, const iga_coeff& c, double* vals) {
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
    A.ntx = interior2_ntx(P.N1, P.p);
    return A;
}

CutEArgs cute_args(Plan& P, const iga_coeff& c) {
    return CutEArgs{P.dir[0], P.dir[1], coef_view(P, c), P.cut_e, P.node_off, P.node_x, P.node_y, P.node_w,
                    P.cutE, (int)P.n_cut_el, c.kind == IGA_COEF_GEOM_DETJ, c.geom_cp, P.n1, P.c_cut};
}

CutRowArgs cutr_args(Plan& P, const iga_coeff& c, double* vals) {
    return CutRowArgs{P.dir[0], P.dir[1], coef_view(P, c), P.form_rows, (int)P.n_form_rows, P.fn_of, P.act_of,
                      P.ecls, P.cut_id, P.band_id, P.cutE, P.method == IGA_DWQ ? P.dwq_region : nullptr, vals,
                      P.n_act, P.cut_part};
}

void launch_interior_coef(Plan& P, const iga_coeff& c, double* vals, hipStream_t s, bool with_points) {
    IGA_REQUIRE(P.method != IGA_GAUSS_REF && c.kind == IGA_COEF_GEOM_DETJ, IGA_E_INVALID,
                "interior rows with the band coefficient: |det J| and a method with interior rows");
    IntArgs A = int_args(P, c, vals);
    CoefArgs C = coef_args(P, c);
    if (with_points) C.xy = P.pts_xy;
    switch (P.p) {
#define CASE(PP) \
    case PP: launch_interior_coef_p<PP>(P, A, C, s); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

void launch_interior_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (P.method == IGA_GAUSS_REF) return;
    IntArgs A = int_args(P, c, vals);
    switch (P.p) {
        case 1: launch_interior_p<1>(P, A, s, t0, t1); break;
        case 2: launch_interior_p<2>(P, A, s, t0, t1); break;
        case 3: launch_interior_p<3>(P, A, s, t0, t1); break;
        case 4: launch_interior_p<4>(P, A, s, t0, t1); break;
        case 5: launch_interior_p<5>(P, A, s, t0, t1); break;
        case 6: launch_interior_p<6>(P, A, s, t0, t1); break;
        case 7: launch_interior_p<7>(P, A, s, t0, t1); break;
        case 8: launch_interior_p<8>(P, A, s, t0, t1); break;
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

// -------------------------------------------------- cut element matrices / rows
template <int P>
__global__ void __launch_bounds__(256) k_cut_elem(CutEArgs A) {
    __shared__ CutESmem<P> S;
    cut_elem_body<P>(A, blockIdx.x, S);
}

template <int P, int MODE>
__global__ void __launch_bounds__((((2 * P + 1) * (2 * P + 1) + 63) / 64) * 64) k_cut_rows(CutRowArgs A) {
    __shared__ CutRSmem<P> S;
    cut_row_body_m<P, MODE>(A, blockIdx.x, S);
}

void launch_cut_elems(Plan& P, const iga_coeff& c, hipStream_t s) {
    if (P.method == IGA_NAIVE_WQ || P.n_cut_el == 0) return;
    CutEArgs A = cute_args(P, c);
    dim3 g((unsigned)P.n_cut_el), b(256);
    switch (P.p) {
#define CASE(PP) \
    case PP: klaunch(P, "k_cut_elem<" #PP ">", k_cut_elem<PP>, g, b, 0, s, A); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

// mode: ROW_FUSED (after the cut element matrices), ROW_INSIDE (the inside sums, to the plan's
// scratch array; needs no cut element matrix), ROW_CUT (adds the cut element matrices' entries to the
// inside sums and writes the rows)
void launch_cut_rows_mode(Plan& P, const iga_coeff& c, double* vals, hipStream_t s, int mode) {
    if (P.method == IGA_NAIVE_WQ || P.n_form_rows == 0) return;
    CutRowArgs A = cutr_args(P, c, vals);
    int W = 2 * P.p + 1;
    if (mode == ROW_CUT && P.method == IGA_DWQ) A.boxp = P.cut_part + (size_t)P.n_form_rows * W * W;
    dim3 g((unsigned)P.n_form_rows), b(((W * W + 63) / 64) * 64);
    switch (P.p * 4 + mode) {
#define CASE(PP)                                                                            \
    case PP * 4 + ROW_FUSED: klaunch(P, "k_cut_rows<" #PP ",fused>", k_cut_rows<PP, ROW_FUSED>, g, b, 0, s, A); break;    \
    case PP * 4 + ROW_INSIDE: klaunch(P, "k_cut_rows<" #PP ",inside>", k_cut_rows<PP, ROW_INSIDE>, g, b, 0, s, A); break; \
    case PP * 4 + ROW_CUT: klaunch(P, "k_cut_rows<" #PP ",cut>", k_cut_rows<PP, ROW_CUT>, g, b, 0, s, A); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

void launch_cut_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s) {
    launch_cut_elems(P, c, s);
    launch_cut_rows_mode(P, c, vals, s, ROW_FUSED);
}

}  // namespace iga
