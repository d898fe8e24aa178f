// Discontinuous weighted quadrature (Sect. 3.3, Eqs. (9)-(10)).
//
//  * k_dwq_sides: for every interior knot t = bp[s] of each direction and
//    each side of it, the 1-D rules w^_{.,i} of the p functions whose
//    support contains t. The side's first element gets p+1 points (the two
//    WQ points plus nested ones, placed round robin from t in the three
//    equal gaps); t is inserted p times (Eq. (10)), the minimum-norm systems
//    (5) of the p+1 refined functions touching that element are solved, one
//    quad of lanes each (several slots per workgroup), and
//    w^_{.,i} = sum_r S[r][i] w~_{.,r}. Both sides are
//    built in the local coordinate u = |x - t|, so the low side is the
//    mirror image of the high one.
//  * k_dwq_choose: per cut row, the box R = I1 x I2 of inside elements of
//    its support that is integrated by sum factorisation (largest box, then
//    fewer discontinuities, then first in the enumeration order: whole range,
//    above s ascending, below s descending; direction-1 options outer).
//  * k_dwq_rows: adds the box's contribution to a row that k_cut_rows formed
//    element-wise over the rest of the support.
#include "dwq_body.hpp"
#include "form_body.hpp"

namespace iga {

template <int P>
__global__ void __launch_bounds__(kDwqSideThreads) k_dwq_sides(DirDev D1, DirDev D2, const double* __restrict__ gx,
                                                               const double* __restrict__ gw,
                                                               int* __restrict__ status) {
    dwq_sides_body<P>(D1, D2, gx, gw, status, blockIdx.x);
}

// A full formation of a DWQ plan: the side rules (they read the knots only)
// and the cut element matrices in one launch, the side rules' workgroups
// first (they take the longest), instead of the side rules after the cut
// element matrices on the caller's stream.
template <int P>
__global__ void __launch_bounds__(kDwqSideThreads) k_cut_elem_sides(CutEArgs A, DirDev D1, DirDev D2,
                                                                    const double* __restrict__ gx,
                                                                    const double* __restrict__ gw,
                                                                    int* __restrict__ status, int nside) {
    __shared__ CutESmem<P> S;
    if ((int)blockIdx.x < nside) {
        dwq_sides_body<P>(D1, D2, gx, gw, status, blockIdx.x);
        return;
    }
    cut_elem_body<P>(A, (int)blockIdx.x - nside, S);
}

// ------------------------------------------------------------ box choice
__device__ __forceinline__ void dwq_option(int k, int lo, int hi, int& a, int& b, int& s, int& side) {
    const int w = hi - lo;
    if (k == 0) {
        a = lo;
        b = hi;
        s = -1;
        side = -1;
    } else if (k <= w) {
        s = lo + k;
        a = s;
        b = hi;
        side = 1;
    } else {
        s = hi - (k - w) + 1;
        a = lo;
        b = s - 1;
        side = 0;
    }
}

// One wavefront per row: lanes test the (I1, I2) options in parallel; the
// choice -- largest box, then fewer discontinuities, then first option in
// the enumeration order -- is a maximum of one 64-bit key over the lanes.
template <int P>
__global__ void __launch_bounds__(64) k_dwq_choose(int N1, int N2, int n1, const int* __restrict__ rows, int n_rows,
                                                   const int* __restrict__ fn_of, const int8_t* __restrict__ ecls,
                                                   int* __restrict__ region) {
    __shared__ unsigned s_rowm[P + 1];
    const int t = blockIdx.x, lane = threadIdx.x;
    if (t >= n_rows) return;
    const int f = fn_of[rows[t]];
    const int i1 = f % n1, i2 = f / n1;
    const int lo1 = max(0, i1 - P), hi1 = min(N1 - 1, i1), lo2 = max(0, i2 - P), hi2 = min(N2 - 1, i2);
    if (lane <= P) {  // inside elements of support row lo2 + lane, one bit per column
        unsigned v = 0;
        if (lo2 + lane <= hi2) {
            int8_t c[P + 1];
#pragma unroll
            for (int m1 = 0; m1 <= P; ++m1) c[m1] = ecls[(size_t)(lo2 + lane) * N1 + min(lo1 + m1, hi1)];
#pragma unroll
            for (int m1 = 0; m1 <= P; ++m1)
                if (m1 <= hi1 - lo1 && c[m1] == EL_INSIDE) v |= 1u << m1;
        }
        s_rowm[lane] = v;
    }
    __syncthreads();
    const int no1 = 1 + 2 * (hi1 - lo1), no2 = 1 + 2 * (hi2 - lo2);
    unsigned long long best = 0ull;  // (box size, 3 - discontinuities, 65535 - option), 0: none
    for (int o = lane; o < no1 * no2; o += 64) {
        const int k1 = o / no2, k2 = o % no2;
        int a1, b1, s1, d1, a2, b2, s2, d2;
        dwq_option(k1, lo1, hi1, a1, b1, s1, d1);
        dwq_option(k2, lo2, hi2, a2, b2, s2, d2);
        const unsigned cm = ((1u << (b1 - a1 + 1)) - 1u) << (a1 - lo1);
        bool ok = true;
        for (int e2 = a2; e2 <= b2; ++e2) ok = ok && (s_rowm[e2 - lo2] & cm) == cm;
        if (!ok) continue;
        const unsigned long long nel = (unsigned long long)((b1 - a1 + 1) * (b2 - a2 + 1));
        const int nd = (s1 >= 0) + (s2 >= 0);
        const unsigned long long key = (nel << 32) | ((unsigned long long)(3 - nd) << 16) | (unsigned)(65535 - o);
        best = key > best ? key : best;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long other = __shfl_xor(best, off, 64);
        best = other > best ? other : best;
    }
    if (lane < 8) {
        int R = -1;
        if (best != 0ull) {
            const int o = 65535 - (int)(best & 0xffffu);
            int a1, b1, s1, d1, a2, b2, s2, d2;
            dwq_option(o / no2, lo1, hi1, a1, b1, s1, d1);
            dwq_option(o % no2, lo2, hi2, a2, b2, s2, d2);
            const int v[8] = {a1, b1, s1, d1, a2, b2, s2, d2};
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k == lane) R = v[k];
        }
        region[(size_t)t * 8 + lane] = R;
    }
}

// ------------------------------------------------------------ box rows
template <int P>
__global__ void __launch_bounds__(256) k_dwq_rows(DwqRowArgs A) {
    dwq_rows_body<P>(A, blockIdx.x);
}

// ------------------------------------------------------------ launchers
void launch_dwq_sides(Plan& P, hipStream_t s) {
    if (P.method != IGA_DWQ) return;
    const int nslot = 2 * (P.dir[0].N - 1) + 2 * (P.dir[1].N - 1);
    if (nslot <= 0) return;
    const int spw = dwq_side_spw(P.p);
    dim3 g((nslot + spw - 1) / spw), b(kDwqSideThreads);
    switch (P.p) {
#define CASE(PP) \
    case PP: klaunch(P, "k_dwq_sides<" #PP ">", k_dwq_sides<PP>, g, b, 0, s, P.dir[0], P.dir[1], P.gauss_x, P.gauss_w, P.status); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

void launch_cut_elems_sides(Plan& P, const iga_coeff& c, hipStream_t s) {
    IGA_REQUIRE(P.method == IGA_DWQ, IGA_E_INVALID, "side rules belong to DWQ plans");
    const int nslot = 2 * (P.dir[0].N - 1) + 2 * (P.dir[1].N - 1);
    const int spw = dwq_side_spw(P.p);
    const int nside = nslot > 0 ? (nslot + spw - 1) / spw : 0;
    const int ncut = (int)P.n_cut_el;
    if (nside + ncut == 0) return;
    const CutEArgs A = cute_args(P, c);
    dim3 g((unsigned)(nside + ncut)), b(kDwqSideThreads);
    static_assert(kDwqSideThreads == 256, "the cut element matrices' workgroups have 256 threads");
    switch (P.p) {
#define CASE(PP)                                                                                                   \
    case PP:                                                                                                       \
        klaunch(P, "k_cut_elem_sides<" #PP ">", k_cut_elem_sides<PP>, g, b, 0, s, A, P.dir[0], P.dir[1], P.gauss_x, \
                P.gauss_w, P.status, nside);                                                                        \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

void launch_dwq_choose(Plan& P, hipStream_t s) {
    if (P.method != IGA_DWQ || P.n_form_rows == 0) return;
    dim3 g((unsigned)P.n_form_rows), b(64);
    switch (P.p) {
#define CASE(PP)                                                                                                 \
    case PP:                                                                                                     \
        klaunch(P, "k_dwq_choose<" #PP ">", k_dwq_choose<PP>, g, b, 0, s, P.N1, P.N2, P.n1, P.form_rows,      \
                (int)P.n_form_rows, P.fn_of, P.ecls, P.dwq_region);                                              \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

// The box parts of a DWQ plan's rows into the plan's second row scratch
// array (the cut-entry launch adds them), so they can be formed before the
// rows themselves.
void launch_dwq_box_parts(Plan& P, const iga_coeff& c, hipStream_t s) {
    if (P.method != IGA_DWQ || P.n_form_rows == 0) return;
    const int W = 2 * P.p + 1;
    DwqRowArgs A{P.dir[0], P.dir[1], coef_view(P, c), c.geom_cp, P.form_rows, (int)P.n_form_rows, P.fn_of,
                 P.act_of, P.dwq_region, nullptr, P.n_act, P.cut_part + (size_t)P.n_form_rows * W * W};
    dim3 g((unsigned)P.n_form_rows), b(256);
    switch (P.p) {
#define CASE(PP) \
    case PP: klaunch(P, "k_dwq_rows<" #PP ">", k_dwq_rows<PP>, g, b, 0, s, A); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

void launch_dwq_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s) {
    if (P.method != IGA_DWQ || P.n_form_rows == 0) return;
    DwqRowArgs A{P.dir[0], P.dir[1], coef_view(P, c), c.geom_cp, P.form_rows, (int)P.n_form_rows, P.fn_of,
                 P.act_of, P.dwq_region, vals, P.n_act};
    dim3 g((unsigned)P.n_form_rows), b(256);
    switch (P.p) {
#define CASE(PP) \
    case PP: klaunch(P, "k_dwq_rows<" #PP ">", k_dwq_rows<PP>, g, b, 0, s, A); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error{IGA_E_UNSUPPORTED, "degree outside 1..8"};
    }
}

}  // namespace iga
