// Batched L2 projection (Sect. 4.2) of the patches of a batch: every patch's
// right-hand side by its own rows' rules and a Jacobi-preconditioned CG on
// its (M + M^T)/2, all patches in the same launches.
//
// Rows of all patches are laid end to end in one set of vectors, each patch
// starting on a workgroup boundary, so every workgroup of kRedThreads rows
// belongs to one patch; a block table maps workgroups to patches. Each
// patch keeps its own scalars: a workgroup sums its own patch's block
// partials (in the one-patch kernels' order), so each patch's step sizes,
// and hence its iterates, are those of the one-patch solver. Convergence is
// tested per patch at the same iterations as the one-patch solver (every
// kCgCheck iterations and at the iteration limit); a converged patch is
// frozen (its workgroups return at once) while the others go on. The PCG
// kernels dispatch on the patch's degree inside the kernel (degree is
// uniform per workgroup), so one launch covers every degree.
#include <algorithm>
#include <cmath>
#include <vector>

#include "form_body.hpp"
#include "solve_body.hpp"

namespace iga {

// segmented launches: workgroup -> patch tables
enum : int { SEG_ROWS = 0, SEG_ENT = 1, SEG_PTS = 2, SEG_GATHER = 3, SEG_N = 4 };
constexpr int kBsMaxP = 6;

struct BsPatch {
    SpArgs S;              // band (A, cols) and index maps of the patch
    int row0;              // first row in the concatenated vectors (a multiple of kRedThreads)
    int blk0;              // first workgroup of the patch in SEG_ROWS (= row0 / kRedThreads)
    int nblk;              // its workgroups of rows
    int seg0[SEG_N];       // first workgroup of the patch in each segmented launch
    int64_t n_ent;         // band entries (2p+1)^2 n_act
    const double* M;       // formed matrix (borrowed)
    double* u;             // solution (caller's, set per call)
    int all_active;        // naive WQ rows (not batched; 0)
    const int8_t* fcls;
    GcArgs gc;             // g c of the patch; out = its slice of the concatenated values
    RhsElemArgs ea;        // element vectors; F = its slice
    RhsGatherArgs ga;      // element-formed rows; F, b = its slices
    DwqRhsArgs dq;         // DWQ plans: box parts of the element-formed rows (set per call)
    CoefArgs co;           // |det J| at every rule point (GEOM_DETJ patches)
    int64_t n_pts;         // rule points
    int detj;              // 1: c = |det J| (recomputed at every rule point first)
};

struct BsItem {
    int patch, unit;
};

struct BatchSolve {
    int n = 0;
    std::vector<BsPatch> hp;
    BsPatch* d_p = nullptr;
    int* d_seg[SEG_N] = {};
    int seg_n[SEG_N] = {};
    BsItem* d_elem = nullptr;   // element vectors, grouped by degree
    int elem_off[kBsMaxP] = {}, elem_n[kBsMaxP] = {};
    BsItem* d_coef = nullptr;   // |det J| point chunks (kRedThreads points), grouped by degree
    int coef_off[kBsMaxP] = {}, coef_n[kBsMaxP] = {};
    BsItem* d_dwq = nullptr;    // element-formed rows of DWQ plans, grouped by degree
    int dwq_off[kBsMaxP] = {}, dwq_n[kBsMaxP] = {};
    int rows = 0;               // concatenated (padded) rows
    double *b = nullptr, *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr;
    double *part0 = nullptr, *part1 = nullptr, *part2 = nullptr;  // init (3/blk), p.q (1/blk), update (2/blk)
    double* scal = nullptr;     // [n][8]
    int* state = nullptr;       // [n][2]: converged, iterations
    double* A = nullptr;        // concatenated (M + M^T)/2
    int* cols = nullptr;
    double* gc = nullptr;
    double* F = nullptr;
    std::vector<void*> mem;
    template <typename T>
    T* alloc(size_t n_) {
        void* ptr = nullptr;
        if (hipMalloc(&ptr, std::max<size_t>(1, n_) * sizeof(T) + 16) != hipSuccess)
            throw Error{IGA_E_NOMEM, "hipMalloc of the batched projection's buffers failed"};
        mem.push_back(ptr);
        return static_cast<T*>(ptr);
    }
    ~BatchSolve() {
        for (void* m : mem) hipFree(m);
    }
};

void batch_solve_free(BatchSolve* bs) { delete bs; }

// ----------------------------------------------------------------- kernels
__device__ __forceinline__ const BsPatch& bs_patch(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                   int& k) {
    k = __builtin_amdgcn_readfirstlane(seg[blockIdx.x]);
    return P[k];
}

// |det J| at every rule point of the patches of degree DEG (the one-patch
// coefficient kernel's body), kRedThreads points per item.
template <int DEG>
__global__ void __launch_bounds__(kRedThreads) k_bs_coef(const BsPatch* __restrict__ P, const BsItem* __restrict__ items) {
    const BsItem it = items[blockIdx.x];
    const BsPatch& B = P[__builtin_amdgcn_readfirstlane(it.patch)];
    const int64_t t = (int64_t)it.unit * kRedThreads + threadIdx.x;
    if (t < B.n_pts) coef_point<DEG>(B.co, t);
}

__global__ void __launch_bounds__(kRedThreads) k_bs_gc(const BsPatch* __restrict__ P, const int* __restrict__ seg) {
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    const int t = (blockIdx.x - B.seg0[SEG_PTS]) * kRedThreads + threadIdx.x;
    gc_point(B.gc, t);
}

__global__ void __launch_bounds__(kRedThreads) k_bs_rhs_wq(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                           double* __restrict__ b) {
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    const int r = (blockIdx.x - B.blk0) * kRedThreads + threadIdx.x;
    if (r < B.S.n_act) rhs_wq_row(B.gc.d1, B.gc.d2, B.S.p, B.fcls, B.all_active, B.S.fn_of, r, B.gc.out, b + B.row0);
}

template <int DEG>
__global__ void __launch_bounds__(64) k_bs_rhs_elem(const BsPatch* __restrict__ P, const BsItem* __restrict__ items) {
    __shared__ RhsElemSmem<DEG> S;
    const BsItem it = items[blockIdx.x];
    rhs_elem_body<DEG>(P[__builtin_amdgcn_readfirstlane(it.patch)].ea, it.unit, S);
}

__global__ void __launch_bounds__(kRedThreads) k_bs_gather(const BsPatch* __restrict__ P, const int* __restrict__ seg) {
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    const int t = (blockIdx.x - B.seg0[SEG_GATHER]) * kRedThreads + threadIdx.x;
    if (t < B.ga.n_rows) rhs_gather_row(B.ga, t);
}

template <int DEG>
__global__ void __launch_bounds__(kDwqRhsThreads) k_bs_rhs_dwq(const BsPatch* __restrict__ P,
                                                               const BsItem* __restrict__ items) {
    const BsItem it = items[blockIdx.x];
    dwq_rhs_body<DEG>(P[__builtin_amdgcn_readfirstlane(it.patch)].dq, it.unit);
}

// (M + M^T)/2 and the compact column of every band entry.
__global__ void __launch_bounds__(kRedThreads) k_bs_sym(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                        double* __restrict__ A, int* __restrict__ cols) {
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    const int64_t t = (int64_t)(blockIdx.x - B.seg0[SEG_ENT]) * kRedThreads + threadIdx.x;
    if (t >= B.n_ent) return;
    const SpArgs& S = B.S;
    symmetrize_entry(S.p, S.n1, S.n2, S.fn_of, S.act_of, S.n_act, B.M, const_cast<double*>(S.A), t);
    const_cast<int*>(S.cols)[t] = col_entry(S, t);
}

__global__ void __launch_bounds__(kRedThreads) k_bs_init(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                         const double* __restrict__ b, double* __restrict__ rv,
                                                         double* __restrict__ zv, double* __restrict__ pv,
                                                         double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    cg_init_block(B.S, blockIdx.x - B.blk0, b + B.row0, B.u, rv + B.row0, zv + B.row0, pv + B.row0,
                  part + 3 * (size_t)B.blk0, sh);
}

// relative residual test of the one-patch solver: sqrt(r.r) / sqrt(b.b) <= rtol
__device__ __forceinline__ bool bs_converged(double rr, double bb, double rtol) {
    const double bnorm = sqrt(bb);
    const double rel = (bnorm > 0) ? sqrt(rr) / bnorm : 0.0;
    return rel <= rtol;
}

// One workgroup per patch: the initial scalars, and patches converged at the start.
__global__ void __launch_bounds__(kRedThreads) k_bs_reduce0(const BsPatch* __restrict__ P,
                                                            const double* __restrict__ part, double* __restrict__ scal,
                                                            int* __restrict__ state, double rtol) {
    __shared__ double sh[kRedThreads / 64];
    const BsPatch& B = P[blockIdx.x];
    double* sc = scal + 8 * (size_t)blockIdx.x;
    cg_reduce0(part + 3 * (size_t)B.blk0, B.nblk, sc, sh);
    if (threadIdx.x == 0) {
        state[2 * blockIdx.x] = bs_converged(sc[2], sc[3], rtol) ? 1 : 0;
        state[2 * blockIdx.x + 1] = 0;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_bs_spmv(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                         const int* __restrict__ state, const double* __restrict__ pv,
                                                         double* __restrict__ qv, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    if (state[2 * k]) return;  // converged: frozen
    const int lb = blockIdx.x - B.blk0;
    const double* p_ = pv + B.row0;
    double* q_ = qv + B.row0;
    double* pt = part + B.blk0;
    switch (B.S.p) {
        case 1: cg_spmv_block<1>(B.S, lb, p_, q_, pt, sh); break;
        case 2: cg_spmv_block<2>(B.S, lb, p_, q_, pt, sh); break;
        case 3: cg_spmv_block<3>(B.S, lb, p_, q_, pt, sh); break;
        case 4: cg_spmv_block<4>(B.S, lb, p_, q_, pt, sh); break;
        case 5: cg_spmv_block<5>(B.S, lb, p_, q_, pt, sh); break;
        case 6: cg_spmv_block<6>(B.S, lb, p_, q_, pt, sh); break;
        default: break;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_bs_update(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                           const int* __restrict__ state, const double* __restrict__ scal,
                                                           int par, const double* __restrict__ part_pq,
                                                           double* __restrict__ rv, double* __restrict__ zv,
                                                           const double* __restrict__ pv, const double* __restrict__ qv,
                                                           double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_alpha;
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    if (state[2 * k]) return;
    cg_update_block(B.S, blockIdx.x - B.blk0, scal + 8 * (size_t)k, par, B.nblk, part_pq + B.blk0, B.u, rv + B.row0,
                    zv + B.row0, pv + B.row0, qv + B.row0, part + 2 * (size_t)B.blk0, sh, &s_alpha);
}

// Direction update; at a check iteration the patch's first workgroup tests
// convergence and freezes the patch (its iterates stay those after this
// iteration's update).
__global__ void __launch_bounds__(kRedThreads) k_bs_dir(const BsPatch* __restrict__ P, const int* __restrict__ seg,
                                                        int* __restrict__ state, double* __restrict__ scal, int par,
                                                        const double* __restrict__ part, const double* __restrict__ zv,
                                                        double* __restrict__ pv, int iter, int check, double rtol) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_beta;
    int k;
    const BsPatch& B = bs_patch(P, seg, k);
    if (state[2 * k]) return;
    const int lb = blockIdx.x - B.blk0;
    double* sc = scal + 8 * (size_t)k;
    const double rr = cg_dir_block(B.S.n_act, lb, sc, par, B.nblk, part + 2 * (size_t)B.blk0, zv + B.row0,
                                   pv + B.row0, sh, &s_beta);
    if (lb == 0 && threadIdx.x == 0) {
        state[2 * k + 1] = iter + 1;
        // every workgroup of this iteration has read the state already: the flag takes effect from the next
        if (check && bs_converged(rr, sc[3], rtol)) state[2 * k] = 1;
    }
}

// ------------------------------------------------------------------- host
static inline int cdiv(int64_t a, int b) { return (int)((a + b - 1) / b); }

static BatchSolve* bs_create(const BatchView& V) {
    auto* bs = new BatchSolve();
    try {
        bs->n = V.n;
        bs->hp.resize(V.n);
        std::vector<int> segtab[SEG_N];
        std::vector<BsItem> elems[kBsMaxP], coefs[kBsMaxP], dwqs[kBsMaxP];
        int64_t ent = 0, pts = 0, fel = 0;
        std::vector<int64_t> ent0(V.n), pts0(V.n), fel0(V.n);  // offsets into the concatenated buffers
        int rows = 0;
        for (int k = 0; k < V.n; ++k) {
            Plan& P = *V.plans[k];
            IGA_REQUIRE(P.p <= kBsMaxP, IGA_E_UNSUPPORTED, "batched projection handles degrees up to 6");
            IGA_REQUIRE(P.method == IGA_HYBRID_GAUSS || P.method == IGA_GAUSS_REF || P.method == IGA_DWQ,
                        IGA_E_UNSUPPORTED, "batched projection handles hybrid Gauss, DWQ and element Gauss plans");
            BsPatch& B = bs->hp[k];
            const int W = 2 * P.p + 1, L = (P.p + 1) * (P.p + 1);
            B.S = SpArgs{P.p, P.n1, P.n2, (int)P.n_act, P.fn_of, P.act_of, nullptr, nullptr};
            B.row0 = rows;
            B.blk0 = rows / kRedThreads;
            B.nblk = cdiv(P.n_act, kRedThreads);
            rows += B.nblk * kRedThreads;
            B.n_ent = (int64_t)W * W * P.n_act;
            B.M = V.outs[k];
            B.u = nullptr;
            B.all_active = 0;
            B.fcls = P.fcls;
            B.n_pts = P.n_points;
            B.detj = V.coeffs[k].kind == IGA_COEF_GEOM_DETJ;
            B.co = coef_args(P, V.coeffs[k]);
            const int counts[SEG_N] = {B.nblk, cdiv(B.n_ent, kRedThreads), cdiv(P.n_points, kRedThreads),
                                       cdiv(P.n_form_rows, kRedThreads)};
            for (int sgi = 0; sgi < SEG_N; ++sgi) {
                B.seg0[sgi] = (int)segtab[sgi].size();
                segtab[sgi].insert(segtab[sgi].end(), counts[sgi], k);
            }
            ent0[k] = ent;
            pts0[k] = pts;
            fel0[k] = fel;
            ent += B.n_ent;
            pts += P.n_points;
            const int nre = (int)(P.n_band + P.n_cut_el);
            if (P.n_form_rows > 0)
                for (int u = 0; u < nre; ++u) elems[P.p - 1].push_back(BsItem{k, u});
            fel += (int64_t)std::max(1, nre) * L;
            if (B.detj)
                for (int u = 0; u < cdiv(P.n_points, kRedThreads); ++u) coefs[P.p - 1].push_back(BsItem{k, u});
            if (P.method == IGA_DWQ)
                for (int u = 0; u < (int)P.n_form_rows; ++u) dwqs[P.p - 1].push_back(BsItem{k, u});
        }
        bs->rows = rows;
        const int nblk = rows / kRedThreads;
        bs->b = bs->alloc<double>(rows);
        bs->r = bs->alloc<double>(rows);
        bs->z = bs->alloc<double>(rows);
        bs->pv = bs->alloc<double>(rows);
        bs->q = bs->alloc<double>(rows);
        bs->part0 = bs->alloc<double>(3 * (size_t)nblk);
        bs->part1 = bs->alloc<double>(nblk);
        bs->part2 = bs->alloc<double>(2 * (size_t)nblk);
        bs->scal = bs->alloc<double>(8 * (size_t)V.n);
        bs->state = bs->alloc<int>(2 * (size_t)V.n);
        bs->A = bs->alloc<double>(ent);
        bs->cols = bs->alloc<int>(ent);
        bs->gc = bs->alloc<double>(pts);
        bs->F = bs->alloc<double>(fel);
        for (int k = 0; k < V.n; ++k) {
            Plan& P = *V.plans[k];
            BsPatch& B = bs->hp[k];
            B.S.A = bs->A + ent0[k];
            B.S.cols = bs->cols + ent0[k];
            double* gcs = bs->gc + pts0[k];
            double* Fs = bs->F + fel0[k];
            B.ea = rhs_elem_args(P, gcs, Fs);
            B.ga = rhs_gather_args(P, Fs, bs->b + B.row0);
            B.gc.out = gcs;  // the rest of gc is set per call (target)
        }
        for (int sgi = 0; sgi < SEG_N; ++sgi) {
            bs->seg_n[sgi] = (int)segtab[sgi].size();
            bs->d_seg[sgi] = bs->alloc<int>(segtab[sgi].size());
            if (!segtab[sgi].empty())
                HIPX(hipMemcpy(bs->d_seg[sgi], segtab[sgi].data(), sizeof(int) * segtab[sgi].size(),
                               hipMemcpyHostToDevice));
        }
        std::vector<BsItem> e_all, c_all, d_all;
        for (int g = 0; g < kBsMaxP; ++g) {
            bs->dwq_off[g] = (int)d_all.size();
            bs->dwq_n[g] = (int)dwqs[g].size();
            d_all.insert(d_all.end(), dwqs[g].begin(), dwqs[g].end());
            bs->elem_off[g] = (int)e_all.size();
            bs->elem_n[g] = (int)elems[g].size();
            e_all.insert(e_all.end(), elems[g].begin(), elems[g].end());
            bs->coef_off[g] = (int)c_all.size();
            bs->coef_n[g] = (int)coefs[g].size();
            c_all.insert(c_all.end(), coefs[g].begin(), coefs[g].end());
        }
        bs->d_elem = bs->alloc<BsItem>(e_all.size());
        bs->d_coef = bs->alloc<BsItem>(c_all.size());
        bs->d_dwq = bs->alloc<BsItem>(d_all.size());
        if (!d_all.empty())
            HIPX(hipMemcpy(bs->d_dwq, d_all.data(), sizeof(BsItem) * d_all.size(), hipMemcpyHostToDevice));
        if (!e_all.empty())
            HIPX(hipMemcpy(bs->d_elem, e_all.data(), sizeof(BsItem) * e_all.size(), hipMemcpyHostToDevice));
        if (!c_all.empty())
            HIPX(hipMemcpy(bs->d_coef, c_all.data(), sizeof(BsItem) * c_all.size(), hipMemcpyHostToDevice));
        bs->d_p = bs->alloc<BsPatch>(V.n);
    } catch (...) {
        delete bs;
        throw;
    }
    return bs;
}

// Right-hand sides, symmetrised bands and the start of PCG, all patches.
static void bs_prepare(BatchSolve& bs, const BatchView& V, const iga_target* gs, double* const* u, double rtol,
                       hipStream_t s) {
    for (int k = 0; k < V.n; ++k) {
        BsPatch& B = bs.hp[k];
        double* out = B.gc.out;
        B.gc = gc_args(*V.plans[k], V.coeffs[k], gs[k], out);
        if (V.plans[k]->method == IGA_DWQ) B.dq = dwq_rhs_args(*V.plans[k], V.coeffs[k], gs[k], out, B.ga.b);
        B.u = u[k];
    }
    HIPX(hipMemcpyAsync(bs.d_p, bs.hp.data(), sizeof(BsPatch) * V.n, hipMemcpyHostToDevice, s));
    for (int g = 0; g < kBsMaxP; ++g) {
        if (bs.coef_n[g] == 0) continue;
        const BsItem* it = bs.d_coef + bs.coef_off[g];
        const dim3 grid((unsigned)bs.coef_n[g]);
        switch (g + 1) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_bs_coef<PP>, grid, dim3(kRedThreads), 0, s, bs.d_p, it); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
            default: break;
        }
    }
    const dim3 blk(kRedThreads);
    if (bs.seg_n[SEG_PTS]) hipLaunchKernelGGL(k_bs_gc, dim3(bs.seg_n[SEG_PTS]), blk, 0, s, bs.d_p, bs.d_seg[SEG_PTS]);
    hipLaunchKernelGGL(k_bs_rhs_wq, dim3(bs.seg_n[SEG_ROWS]), blk, 0, s, bs.d_p, bs.d_seg[SEG_ROWS], bs.b);
    for (int g = 0; g < kBsMaxP; ++g) {
        if (bs.elem_n[g] == 0) continue;
        const BsItem* it = bs.d_elem + bs.elem_off[g];
        const dim3 grid((unsigned)bs.elem_n[g]);
        switch (g + 1) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_bs_rhs_elem<PP>, grid, dim3(64), 0, s, bs.d_p, it); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
            default: break;
        }
    }
    if (bs.seg_n[SEG_GATHER])
        hipLaunchKernelGGL(k_bs_gather, dim3(bs.seg_n[SEG_GATHER]), blk, 0, s, bs.d_p, bs.d_seg[SEG_GATHER]);
    for (int g = 0; g < kBsMaxP; ++g) {   // DWQ box parts, added after the gather
        if (bs.dwq_n[g] == 0) continue;
        const BsItem* it = bs.d_dwq + bs.dwq_off[g];
        const dim3 grid((unsigned)bs.dwq_n[g]);
        switch (g + 1) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_bs_rhs_dwq<PP>, grid, dim3(kDwqRhsThreads), 0, s, bs.d_p, it); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
            default: break;
        }
    }
    hipLaunchKernelGGL(k_bs_sym, dim3(bs.seg_n[SEG_ENT]), blk, 0, s, bs.d_p, bs.d_seg[SEG_ENT], bs.A, bs.cols);
    hipLaunchKernelGGL(k_bs_init, dim3(bs.seg_n[SEG_ROWS]), blk, 0, s, bs.d_p, bs.d_seg[SEG_ROWS], bs.b, bs.r, bs.z,
                       bs.pv, bs.part0);
    hipLaunchKernelGGL(k_bs_reduce0, dim3(V.n), blk, 0, s, bs.d_p, bs.part0, bs.scal, bs.state, rtol);
}

// One iteration of every unconverged patch (iteration number it, 0-based).
static void bs_iterate(BatchSolve& bs, int it, int check, double rtol, hipStream_t s) {
    const int par = it & 1;
    const dim3 grid(bs.seg_n[SEG_ROWS]), blk(kRedThreads);
    const int* seg = bs.d_seg[SEG_ROWS];
    hipLaunchKernelGGL(k_bs_spmv, grid, blk, 0, s, bs.d_p, seg, bs.state, bs.pv, bs.q, bs.part1);
    hipLaunchKernelGGL(k_bs_update, grid, blk, 0, s, bs.d_p, seg, bs.state, bs.scal, par, bs.part1, bs.r, bs.z,
                       bs.pv, bs.q, bs.part2);
    hipLaunchKernelGGL(k_bs_dir, grid, blk, 0, s, bs.d_p, seg, bs.state, bs.scal, par, bs.part2, bs.z, bs.pv, it,
                       check, rtol);
}

static int bs_project(iga_batch* batch, const iga_target* gs, double rtol, int maxit, double* const* u,
                      iga_solve_info* infos, hipStream_t s) {
    BatchView V = batch_view(batch);
    for (int k = 0; k < V.n; ++k) {
        IGA_REQUIRE(u[k], IGA_E_INVALID, "solution buffer missing");
        rhs_check(*V.plans[k], V.coeffs[k], gs[k]);
    }
    if (!*V.solve) *V.solve = bs_create(V);
    BatchSolve& bs = **V.solve;
    bs_prepare(bs, V, gs, u, rtol, s);
    std::vector<int> st(2 * (size_t)V.n);
    auto all_converged = [&]() {
        HIPX(hipMemcpyAsync(st.data(), bs.state, sizeof(int) * st.size(), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        for (int k = 0; k < V.n; ++k)
            if (!st[2 * k]) return false;
        return true;
    };
    int it = 0;
    bool done = all_converged();
    while (!done && it < maxit) {
        const int m = std::min(kCgCheck, maxit - it);
        for (int j = 0; j < m; ++j) bs_iterate(bs, it + j, j == m - 1, rtol, s);
        it += m;
        done = all_converged();
    }
    std::vector<double> sc(8 * (size_t)V.n);
    HIPX(hipMemcpyAsync(sc.data(), bs.scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    HIPX(hipGetLastError());
    bool all = true;
    for (int k = 0; k < V.n; ++k) {
        const double bnorm = std::sqrt(sc[8 * k + 3]);
        const double rel = (bnorm > 0) ? std::sqrt(sc[8 * k + 2]) / bnorm : 0.0;
        const bool conv = st[2 * k] != 0;
        all = all && conv;
        if (infos) {
            infos[k].iterations = st[2 * k + 1];
            infos[k].converged = conv;
            infos[k].rel_residual = rel;
        }
    }
    if (!all) {
        set_error("PCG did not reach the tolerance on every patch of the batch");
        return IGA_E_NOCONV;
    }
    return IGA_OK;
}

}  // namespace iga

using namespace iga;

extern "C" {

int iga_batch_project(iga_batch* batch, const iga_target* gs, double rtol, int32_t maxit, double* const* u,
                      iga_solve_info* infos, void* stream) {
    try {
        IGA_REQUIRE(batch && gs && u, IGA_E_INVALID, "null argument");
        IGA_REQUIRE(rtol > 0 && maxit > 0, IGA_E_INVALID, "rtol and maxit must be positive");
        return bs_project(batch, gs, rtol, maxit, u, infos, (hipStream_t)stream);
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return IGA_E_INVALID;
    }
}

}  // extern "C"
