// L2 projection (Sect. 4.2): right-hand side b_i = row i's own rule applied
// to g c, then Jacobi-preconditioned CG on A = (M + M^T)/2 in the band layout.
// The rule of each row is the one its mass-matrix row uses: weighted
// quadrature for interior rows, element Gauss + cut rule for rows formed
// element-wise, and for DWQ rows with a box the refined rules on the box
// plus element rules on the rest of the support. Reductions are block partials summed in a fixed order by one
// workgroup, so every run is bitwise reproducible.
#include <cmath>
#include <vector>

#include "solve_body.hpp"

namespace iga {

__global__ void k_gc(GcArgs A) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    gc_point(A, t);
}

// b for interior rows (weighted quadrature) -- one thread per row.
__global__ void k_rhs_wq(DirDev D1, DirDev D2, int p, const int8_t* __restrict__ fcls, int all_active,
                         const int* __restrict__ fn_of, int n_act, const double* __restrict__ gc_wq,
                         double* __restrict__ b) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_act) rhs_wq_row(D1, D2, p, fcls, all_active, fn_of, r, gc_wq, b);
}

// Element vectors of band (Gauss) and cut elements, one workgroup each.
template <int P>
__global__ void __launch_bounds__(64) k_rhs_elem(RhsElemArgs A) {
    __shared__ RhsElemSmem<P> S;
    rhs_elem_body<P>(A, blockIdx.x, S);
}

// b for element-formed rows: gather F_e over the support elements.
__global__ void k_rhs_gather(RhsGatherArgs A) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < A.n_rows) rhs_gather_row(A, t);
}

// DWQ rows with a box: the box part, one workgroup per element-formed row.
template <int P>
__global__ void __launch_bounds__(kDwqRhsThreads) k_rhs_dwq(DwqRhsArgs A) {
    dwq_rhs_body<P>(A, blockIdx.x);
}

// ------------------------------------------------------------------- PCG
__global__ void k_symmetrize(int p, int n1, const int* __restrict__ fn_of, const int* __restrict__ act_of,
                             int n2, int n_act, const double* __restrict__ M, double* __restrict__ A) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int W = 2 * p + 1;
    if (t < (int64_t)W * W * n_act) symmetrize_entry(p, n1, n2, fn_of, act_of, n_act, M, A, t);
}

// Compact column of every slot of the band (once per solve).
__global__ void k_cols(SpArgs S, int* __restrict__ cols) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = 2 * S.p + 1;
    if (t < (int64_t)W * W * S.n_act) cols[t] = col_entry(S, t);
}

__global__ void __launch_bounds__(kRedThreads) k_cg_init(SpArgs S, const double* __restrict__ bvec,
                                                         const double* __restrict__ x, double* __restrict__ rv,
                                                         double* __restrict__ zv, double* __restrict__ pv,
                                                         double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    cg_init_block(S, blockIdx.x, bvec, x, rv, zv, pv, part, sh);
}

__global__ void __launch_bounds__(kRedThreads) k_reduce(const double* __restrict__ part, int nblk,
                                                        double* __restrict__ scal) {
    __shared__ double sh[kRedThreads / 64];
    cg_reduce0(part, nblk, scal, sh);
}

// The iteration in three launches: every block of the update and direction
// kernels sums the previous kernel's block partials itself (same order in
// every block, so the same scalars), instead of a one-block reduction launch
// in between. (r.z) alternates between scal[6 + par] and scal[7 - par], so the
// direction kernel's block 0 can store the new value while other blocks
// still read the old one.
template <int P>
__global__ void __launch_bounds__(kRedThreads) k_cg_spmv_c(SpArgs S, const double* __restrict__ pv,
                                                           double* __restrict__ qv, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    cg_spmv_block<P>(S, blockIdx.x, pv, qv, part, sh);
}

__global__ void __launch_bounds__(kRedThreads) k_cg_update_c(SpArgs S, double* __restrict__ scal, int par, int nblk,
                                                             const double* __restrict__ part_pq, double* __restrict__ x,
                                                             double* __restrict__ rv, double* __restrict__ zv,
                                                             const double* __restrict__ pv,
                                                             const double* __restrict__ qv, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_alpha;
    cg_update_block(S, blockIdx.x, scal, par, nblk, part_pq, x, rv, zv, pv, qv, part, sh, &s_alpha);
}

__global__ void __launch_bounds__(kRedThreads) k_cg_dir_c(int n, double* __restrict__ scal, int par, int nblk,
                                                          const double* __restrict__ part,
                                                          const double* __restrict__ zv, double* __restrict__ pv) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_beta;
    cg_dir_block(n, blockIdx.x, scal, par, nblk, part, zv, pv, sh, &s_beta);
}

}  // namespace iga

using namespace iga;

namespace iga {

GcArgs gc_args(Plan& P, const iga_coeff& c, const iga_target& g, double* out) {
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
    return A;
}

RhsElemArgs rhs_elem_args(Plan& P, const double* gc, double* F) {
    const int L = (P.p + 1) * (P.p + 1);
    const int nq = P.dir[0].Q * P.dir[1].Q;
    return RhsElemArgs{P.dir[0], P.dir[1], P.band_list, (int)P.n_band, P.cut_list, P.node_off, P.node_x, P.node_y,
                       P.node_w, gc, nq, (int)(nq + P.n_band * L), F};
}

RhsGatherArgs rhs_gather_args(Plan& P, const double* F, double* b) {
    return RhsGatherArgs{P.p, P.N1, P.N2, P.n1, P.form_rows, (int)P.n_form_rows, P.fn_of, P.ecls, P.band_id,
                         P.cut_id, (int)P.n_band, F, b, P.method == IGA_DWQ ? P.dwq_region : nullptr};
}

DwqRhsArgs dwq_rhs_args(Plan& P, const iga_coeff& c, const iga_target& g, const double* gc, double* b) {
    const CoefView cv = coef_view(P, c);
    return DwqRhsArgs{P.dir[0], P.dir[1], g, (c.kind == IGA_COEF_GEOM_DETJ) ? c.geom_cp : nullptr, P.n1,
                      cv.is_const, cv.value, gc, P.form_rows, (int)P.n_form_rows, P.fn_of, P.dwq_region, b};
}

void rhs(Plan& P, const iga_coeff& c, const iga_target& g, double* b, hipStream_t s) {
    SolveWork& W = P.sw;
    size_t L = (size_t)(P.p + 1) * (P.p + 1);
    if (!W.gc) W.gc = P.alloc<double>(P.n_points);
    if (!W.F) W.F = P.alloc<double>(std::max<int64_t>(1, P.n_band + P.n_cut_el) * L);
    if (c.kind == IGA_COEF_GEOM_DETJ) launch_coef(P, c, s);
    const int64_t npts = P.n_points;
    hipLaunchKernelGGL(k_gc, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, gc_args(P, c, g, W.gc));
    int n = (int)P.n_act;
    hipLaunchKernelGGL(k_rhs_wq, dim3((n + 255) / 256), dim3(256), 0, s, P.dir[0], P.dir[1], P.p, P.fcls,
                       (int)(P.method == IGA_NAIVE_WQ), P.fn_of, n, W.gc, b);
    if (P.method == IGA_NAIVE_WQ || P.n_form_rows == 0) return;
    int nre = (int)(P.n_band + P.n_cut_el);
    if (nre > 0) {
        const RhsElemArgs A = rhs_elem_args(P, W.gc, W.F);
        switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_rhs_elem<PP>, dim3(nre), dim3(64), 0, s, A); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
    }
    int nr = (int)P.n_form_rows;
    hipLaunchKernelGGL(k_rhs_gather, dim3((nr + 255) / 256), dim3(256), 0, s, rhs_gather_args(P, W.F, b));
    if (P.method == IGA_DWQ) {
        const DwqRhsArgs A = dwq_rhs_args(P, c, g, W.gc, b);
        switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_rhs_dwq<PP>, dim3(nr), dim3(kDwqRhsThreads), 0, s, A); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        }
    }
}

void solve_buffers(Plan& P) {
    SolveWork& W = P.sw;
    if (W.A) return;
    const int n = (int)P.n_act;
    const int W2 = (2 * P.p + 1) * (2 * P.p + 1);
    const int nblk = (n + kRedThreads - 1) / kRedThreads;
    W.A = P.alloc<double>((size_t)W2 * n);
    W.r = P.alloc<double>(n);
    W.z = P.alloc<double>(n);
    W.pv = P.alloc<double>(n);
    W.q = P.alloc<double>(n);
    W.b = P.alloc<double>(n);
    W.part = P.alloc<double>(3 * (size_t)nblk);
    W.scal = P.alloc<double>(8);
    W.cols = P.alloc<int>((size_t)W2 * n);
    HIPX(hipHostMalloc((void**)&W.h_scal, 8 * sizeof(double), hipHostMallocDefault));
}

SpArgs solve_operator(Plan& P, const double* vals, hipStream_t s) {
    SolveWork& W = P.sw;
    const int n = (int)P.n_act;
    const int64_t tot = (int64_t)(2 * P.p + 1) * (2 * P.p + 1) * n;
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, P.p, P.n1, P.fn_of,
                       P.act_of, P.n2, n, vals, W.A);
    SpArgs S{P.p, P.n1, P.n2, n, P.fn_of, P.act_of, W.A, nullptr};
    hipLaunchKernelGGL(k_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, S, W.cols);
    S.cols = W.cols;
    return S;
}

// The rules each method's right-hand side takes g c at: DWQ boxes also need
// it at their nested points, so values given only at the plan's rule points
// (and a coefficient given there) cannot serve DWQ plans.
void rhs_check(const Plan& P, const iga_coeff& c, const iga_target& g) {
    IGA_REQUIRE(g.kind >= IGA_TARGET_SINCOS && g.kind <= IGA_TARGET_AT_POINTS, IGA_E_UNSUPPORTED, "target kind");
    IGA_REQUIRE(g.kind != IGA_TARGET_AT_POINTS || g.g_points, IGA_E_INVALID, "target values missing");
    IGA_REQUIRE(P.method == IGA_HYBRID_GAUSS || P.method == IGA_GAUSS_REF || P.method == IGA_DWQ,
                IGA_E_UNSUPPORTED, "right-hand side is built for hybrid Gauss, DWQ and the reference rules");
    IGA_REQUIRE(P.method != IGA_DWQ || (g.kind != IGA_TARGET_AT_POINTS && c.kind != IGA_COEF_AT_POINTS),
                IGA_E_UNSUPPORTED, "DWQ right-hand side needs g and c at its nested points: no AT_POINTS values");
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
    rhs_check(*P, *c, *g);
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
    rhs_check(*P, *c, *g);
    hipStream_t s = (hipStream_t)stream;
    SolveWork& W = P->sw;
    int n = (int)P->n_act;
    int nblk = (n + kRedThreads - 1) / kRedThreads;
    solve_buffers(*P);
    rhs(*P, *c, *g, W.b, s);
    const SpArgs S = solve_operator(*P, vals, s);
    hipLaunchKernelGGL(k_cg_init, dim3(nblk), dim3(kRedThreads), 0, s, S, W.b, u, W.r, W.z, W.pv, W.part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, W.part, nblk, W.scal);
    auto read = [&]() {
        HIPX(hipMemcpyAsync(W.h_scal, W.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
    };
    read();
    double bnorm = std::sqrt(W.h_scal[3]);
    double rel = (bnorm > 0) ? std::sqrt(W.h_scal[2]) / bnorm : 0.0;
    int it = 0;
    const int chunk = kCgCheck;
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
