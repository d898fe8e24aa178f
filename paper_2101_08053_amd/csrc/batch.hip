// Batched formation of many patches in one persistent launch.
//
// The work of every patch is cut into items of four kinds: chunks of
// coefficient points (|det J| of each patch's geometry), cut-element local
// matrices, interior work items (one test-function row i2 x one tile of rows
// i1) and element-formed rows. The cut element matrices, uneven in their
// node counts, are queued by decreasing cost, one queue per degree, for the
// persistent launch (or, where the autotuner measures it faster, launched one
// workgroup each per degree). The rest is regular or latency-bound work that needs
// many workgroups in flight per CU, which the persistent kernel's registers
// and LDS (set by its largest body) do not allow, so it runs in launches of
// its own per degree: on a second stream, beside the persistent launch, the
// coefficient chunks and then the interior tiles; on the first, once the
// persistent launch and the coefficient chunks are done, one small workgroup
// per element-formed row (beside the interior tiles).
//
// The persistent launch: a fixed grid of workgroups, split over the degrees
// in proportion to their work, takes items from its degree's queue head (one
// atomic add per chunk of items; the degree is fixed per workgroup, so each
// body is compiled for its degree and the kernel's registers are those of
// the largest body). The queue keeps dependency levels (0: coefficients,
// 1: cut elements): a workgroup counts the items it finished at each level
// and publishes the counts (one agent-scope release, i.e. one L2 write-back)
// only when it takes its first item of a later level or runs out of items;
// before running an item of level l it waits (agent-scope acquire) until its
// degree's items of all lower levels are published. Every item of a lower
// level sits earlier in the queue and is held by a workgroup that publishes
// before it waits, so the waits always end; each is bounded all the same, and
// past the bound the item proceeds and the batch status records the timeout.
// With the coefficients in launches of their own the queue holds level-1
// items only, so no workgroup waits.
//
// A batch object keeps the descriptors, the item lists, the counters and,
// once asked, a HIP graph of all the launches on both streams; the autotuner
// times the persistent grid, register budget, queue chunk and item order on
// the device and keeps the fastest.
#include <algorithm>
#include <memory>
#include <vector>

#include "dwq_body.hpp"
#include "form_body.hpp"

namespace iga {

enum : int { BK_COEF = 0, BK_CUTE = 1, BK_INT = 2, BK_CUTR = 3, BK_NKIND = 4 };
constexpr int kBatchMaxP = 6;

struct BatchPlan {
    int p;
    int method;
    int need[BK_NKIND];  // items of each kind
    IntArgs ia;
    CutEArgs ce;
    CutRowArgs cr;
    CoefArgs co;
    // discontinuous weighted quadrature (method IGA_DWQ): the side rules of
    // every (direction, interior knot, side) slot and the rows' box parts
    DwqRowArgs dr;
    const double *gx, *gw;  // packed Gauss-Legendre table
    int* status;
};

struct BatchItem {
    int plan, kind, unit, pad;
};

constexpr int kBatchGroups = kBatchMaxP;  // one queue per degree 1..6

struct BatchDev {
    const BatchPlan* plans;
    const BatchItem* items;  // queue g holds items[off[g] .. off[g] + n[g])
    int* heads;              // [kBatchGroups] queue heads
    int* level_done;         // [kBatchGroups][2] published items of levels 0 and 1
    int* status;             // 1: a dependency wait hit its bound
    int spin_limit;
    int chunk;                          // consecutive items reserved per queue-head atomic
    int first_block[kBatchGroups + 1];  // workgroups [first_block[g], first_block[g+1]) serve degree g+1
    int off[kBatchGroups], n[kBatchGroups];
    int n_level[kBatchGroups][2];       // items of levels 0 and 1 per queue
};

__device__ __forceinline__ int item_level(int kind) { return kind == BK_COEF ? 0 : 1; }

// LDS of the persistent kernel's body for degree p (sized at launch for the
// largest degree in the batch, so batches of low degrees fit more workgroups).
static size_t batch_smem_bytes(int p) {
    switch (p) {
        case 1: return sizeof(CutESmem<1>);
        case 2: return sizeof(CutESmem<2>);
        case 3: return sizeof(CutESmem<3>);
        case 4: return sizeof(CutESmem<4>);
        case 5: return sizeof(CutESmem<5>);
        default: return sizeof(CutESmem<6>);
    }
}

__device__ __forceinline__ bool wait_count(int* ctr, int need, int limit) {
    int spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++spins > limit) return false;
        __builtin_amdgcn_s_sleep(4);
    }
    return true;
}

template <int P>
__device__ __forceinline__ void run_item(const BatchPlan& Bp, const BatchItem& it, unsigned char* smem) {
    if (it.kind == BK_CUTE) cut_elem_body<P>(Bp.ce, it.unit, *reinterpret_cast<CutESmem<P>*>(smem));
    // coefficient chunks and rows run in launches of their own
}

__global__ void k_batch_reset(int* counters, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) counters[t] = 0;
}

// Thread 0 of the workgroup: publish the finished lower-level items (release; every wave of
// the workgroup has fenced its own stores before), then, unless the workgroup is leaving
// (level 3), wait for the queue's lower levels to be complete (acquire).
__device__ __forceinline__ void publish_and_wait(const BatchDev& B, int g, int level, int* pend) {
    int* ld = B.level_done + 2 * g;
    for (int l = 0; l < 2; ++l)
        if (pend[l]) {
            __hip_atomic_fetch_add(ld + l, pend[l], __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            pend[l] = 0;
        }
    if (level > 2 || __hip_atomic_load(B.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    bool ok = true;
    for (int l = 0; l < level && ok; ++l) ok = wait_count(ld + l, B.n_level[g][l], B.spin_limit);
    if (!ok) atomicExch(B.status, 1);
}

template <int P>
__device__ __forceinline__ void batch_loop(const BatchDev& B, int g, unsigned char* smem, int* s_sh) {
    const BatchItem* items = B.items + B.off[g];
    const int n = B.n[g];
    int cur = 0;             // level of the items run so far (uniform)
    int pend[2] = {0, 0};    // finished, unpublished items of levels 0 and 1 (thread 0)
    int next = 0, stop = 0;  // reserved range of the queue (thread 0)
    for (;;) {
        __syncthreads();  // the previous item is done with LDS and the shared slots
        if (threadIdx.x == 0) {
            if (next >= stop) {  // reserve the next chunk: queue order is kept, one atomic per chunk
                next = atomicAdd(B.heads + g, B.chunk);
                stop = next + B.chunk;
            }
            const int idx = next < n ? next++ : n;
            const int lvl = (idx < n) ? item_level(items[idx].kind) : 3;
            s_sh[0] = idx;
            s_sh[1] = lvl;
            s_sh[2] = (lvl > cur) && (pend[0] + pend[1] > 0);
        }
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_sh[0]);
        const int lvl = __builtin_amdgcn_readfirstlane(s_sh[1]);
        if (lvl > cur) {
            if (s_sh[2]) __threadfence();   // this wave's stores of the finished items, at agent scope
            __syncthreads();
            if (threadIdx.x == 0) publish_and_wait(B, g, lvl, pend);
            __syncthreads();
            cur = lvl;
        }
        if (idx >= n) break;
        BatchItem it = items[idx];
        it.plan = __builtin_amdgcn_readfirstlane(it.plan);  // uniform: the descriptor is read once per wave
        it.kind = __builtin_amdgcn_readfirstlane(it.kind);
        it.unit = __builtin_amdgcn_readfirstlane(it.unit);
        run_item<P>(B.plans[it.plan], it, smem);
        if (threadIdx.x == 0 && lvl < 2) pend[lvl]++;
    }
}

// Two register budgets, chosen by the autotuner: MINW = 1 lets the largest
// body keep everything in registers (one workgroup per CU), MINW = 2 caps
// them at 256 so that two workgroups share a CU (a few values spill).
template <int MINW>
__global__ void __launch_bounds__(256, MINW) k_batch(BatchDev B) {
    extern __shared__ __align__(16) unsigned char smem[];  // batch_smem_bytes of the batch's largest degree
    __shared__ int s_sh[3];
    int g = 0;
    while (g < kBatchGroups - 1 && (int)blockIdx.x >= B.first_block[g + 1]) ++g;
    switch (g + 1) {
        case 1: batch_loop<1>(B, g, smem, s_sh); break;
        case 2: batch_loop<2>(B, g, smem, s_sh); break;
        case 3: batch_loop<3>(B, g, smem, s_sh); break;
        case 4: batch_loop<4>(B, g, smem, s_sh); break;
        case 5: batch_loop<5>(B, g, smem, s_sh); break;
        case 6: batch_loop<6>(B, g, smem, s_sh); break;
        default: break;
    }
}

// Cut element matrices of the batch's patches of degree P, one workgroup per
// element: the autotuner's alternative to the persistent queue.
template <int P>
__global__ void __launch_bounds__(256)
    k_batch_cut_elems(const BatchPlan* __restrict__ plans, const BatchItem* __restrict__ items) {
    __shared__ CutESmem<P> S;
    const BatchItem it = items[blockIdx.x];
    cut_elem_body<P>(plans[it.plan].ce, it.unit, S);
}

// Coefficient items of the batch's patches of degree P, one wavefront each:
// |det J| on a tile of the WQ grid (sum-factorised, the one-patch kernel's
// body), then on kCgPts band Gauss points per item (the cut element matrices
// evaluate it at their nodes themselves).
template <int P>
__global__ void __launch_bounds__(kCgPts)
    k_batch_coef(const BatchPlan* __restrict__ plans, const BatchItem* __restrict__ items) {
    __shared__ CoefGridSmem<P> S;
    const BatchItem it = items[blockIdx.x];
    const CoefArgs& co = plans[it.plan].co;
    const int ntile = coef_grid_tiles(co.d1.Q, co.d2.N);
    if (it.unit < ntile) {
        coef_grid_body<P>(co, it.unit, S);
        return;
    }
    const int64_t t = co.nq + (int64_t)(it.unit - ntile) * kCgPts + threadIdx.x;
    if (t < co.nq + co.nb) coef_point<P>(co, t);
}

// Interior tiles of the batch's patches of degree P (the one-patch kernel's
// tiles and body), after the coefficient chunks on the same stream.
template <int P>
__global__ void __launch_bounds__(Int2Cfg<P>::NT)
    k_batch_interior(const BatchPlan* __restrict__ plans, const BatchItem* __restrict__ items) {
    __shared__ __align__(16) Int2Smem<P> S;
    const BatchItem it = items[xcd_block(blockIdx.x, gridDim.x)];
    const BatchPlan& Bp = plans[it.plan];
    const int ntx = interior2_ntx(Bp.ia.d1.N, P);
    const int i2 = it.unit / ntx;
    interior_rows_block<P>(Bp.ia, it.unit - i2 * ntx, i2, S);
}

// Side rules of the batch's DWQ patches of degree P, one workgroup per group
// of (direction, interior knot, side) slots, one quad of lanes per refined system:
// the uneven refined minimum-norm solves of every patch in one launch.
template <int P>
__global__ void __launch_bounds__(kDwqSideThreads)
    k_batch_dwq_sides(const BatchPlan* __restrict__ plans, const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    const BatchPlan& Bp = plans[__builtin_amdgcn_readfirstlane(it.plan)];
    dwq_sides_body<P>(Bp.ia.d1, Bp.ia.d2, Bp.gx, Bp.gw, Bp.status, it.unit);
}

// Box parts of the DWQ patches' element-formed rows (degree P), one
// workgroup per row with a box, after the element-formed rows.
template <int P>
__global__ void __launch_bounds__(256)
    k_batch_dwq_rows(const BatchPlan* __restrict__ plans, const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    dwq_rows_body<P>(plans[__builtin_amdgcn_readfirstlane(it.plan)].dr, it.unit);
}

// Element-formed rows of the batch's patches of degree P, one workgroup per
// row, after the persistent launch and the coefficient chunks (so the
// coefficients and cut element matrices are complete): the fused body of the
// one-patch formation, so the values are the same.
constexpr int batch_cut_row_threads(int p) { return (((2 * p + 1) * (2 * p + 1) + 63) / 64) * 64; }

template <int P>
__global__ void __launch_bounds__(batch_cut_row_threads(P))
    k_batch_cut_rows(const BatchPlan* __restrict__ plans, const BatchItem* __restrict__ items) {
    __shared__ CutRSmem<P> S;
    const BatchItem it = items[blockIdx.x];
    cut_row_body<P>(plans[it.plan].cr, it.unit, S);
}

// ------------------------------------------------------------------ host
struct BatchSolve;                      // batched projection state (batch_solve.hip)
void batch_solve_free(BatchSolve* bs);

struct Batch {
    std::vector<Plan*> plans;
    std::vector<iga_coeff> coeffs;
    std::vector<double*> outs;
    std::vector<BatchItem> items_lpt, items_plan;  // two queue orders, grouped by degree
    int g_off[kBatchGroups] = {}, g_n[kBatchGroups] = {}, g_lvl[kBatchGroups][2] = {};
    double g_work[kBatchGroups] = {};
    BatchPlan* d_plans = nullptr;
    BatchItem* d_items = nullptr;
    BatchItem* d_rows = nullptr;  // coefficient chunks, interior tiles, element-formed rows, by degree
    int coef_off[kBatchGroups] = {}, coef_n[kBatchGroups] = {};
    int cute_off[kBatchGroups] = {}, cute_n[kBatchGroups] = {};
    int persistent = 1;  // 1: cut element matrices from the persistent queue, 0: one workgroup each (autotuned)
    int int_off[kBatchGroups] = {}, int_n[kBatchGroups] = {};
    int rows_off[kBatchGroups] = {}, rows_n[kBatchGroups] = {};
    int dwqs_off[kBatchGroups] = {}, dwqs_n[kBatchGroups] = {};  // DWQ side slots
    int dwqr_off[kBatchGroups] = {}, dwqr_n[kBatchGroups] = {};  // DWQ rows with a box
    int* d_counters = nullptr;  // status, heads[kBatchGroups], level counters[kBatchGroups][2]
    int n_items = 0;
    int n_cu = 256;
    int max_wg_per_cu = 16;  // largest grid the autotuner tries, in workgroups per CU
    int wg_per_cu = 2;
    int capped = 1;  // k_batch<2> (256 registers) rather than k_batch<1>
    int order = 0;  // 0 cost-sorted, 1 patch by patch
    int chunk = 16; // queue items reserved per atomic
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    hipStream_t side = nullptr;  // coefficient chunks and interior tiles, beside the persistent launch
    hipEvent_t ev_fork = nullptr, ev_coef = nullptr, ev_join = nullptr;
    int64_t nnz = 0;
    BatchSolve* solve = nullptr;  // created by the first batched projection

    ~Batch() {
        if (solve) batch_solve_free(solve);
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (cap_stream) hipStreamDestroy(cap_stream);
        if (side) hipStreamDestroy(side);
        if (ev_fork) hipEventDestroy(ev_fork);
        if (ev_join) hipEventDestroy(ev_join);
        if (ev_coef) hipEventDestroy(ev_coef);
        if (d_plans) hipFree(d_plans);
        if (d_items) hipFree(d_items);
        if (d_rows) hipFree(d_rows);
        if (d_counters) hipFree(d_counters);
    }
    void drop_graph() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    void upload_items(hipStream_t s) {
        const auto& v = order == 0 ? items_lpt : items_plan;
        HIPX(hipMemcpyAsync(d_items, v.data(), sizeof(BatchItem) * v.size(), hipMemcpyHostToDevice, s));
        HIPX(hipStreamSynchronize(s));
    }
    // workgroups per degree: proportional to the degree's work, at least one, at most its items
    void split(int* first, int& total) const {
        double wsum = 0.0;
        for (int g = 0; g < kBatchGroups; ++g) wsum += g_work[g];
        const int budget = n_cu * wg_per_cu;
        total = 0;
        for (int g = 0; g < kBatchGroups; ++g) {
            first[g] = total;
            if (g_n[g] == 0) continue;
            int w = (int)(budget * (g_work[g] / std::max(wsum, 1e-300)));
            total += std::max(1, std::min(w, g_n[g]));
        }
        first[kBatchGroups] = total;
    }
    int grid() const {
        int first[kBatchGroups + 1], total = 0;
        split(first, total);
        return std::max(1, total);
    }
    void launch(hipStream_t s) {
        const int nc = 1 + 3 * kBatchGroups;  // status, heads, level counters
        HIPX(hipEventRecord(ev_fork, s));
        HIPX(hipStreamWaitEvent(side, ev_fork, 0));
        for (int g = 0; g < kBatchGroups; ++g) {
            if (coef_n[g] == 0) continue;
            const BatchItem* it = d_rows + coef_off[g];
            const dim3 grid((unsigned)coef_n[g]);
            switch (g + 1) {
#define CASE(PP)                                                                             \
    case PP:                                                                                 \
        hipLaunchKernelGGL(k_batch_coef<PP>, grid, dim3(kCgPts), 0, side, d_plans, it); \
        break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
                default: break;
            }
        }
        HIPX(hipEventRecord(ev_coef, side));
        for (int g = 0; g < kBatchGroups; ++g) {
            if (int_n[g] == 0) continue;
            const BatchItem* it = d_rows + int_off[g];
            const dim3 grid((unsigned)int_n[g]);
            switch (g + 1) {
#define CASE(PP)                                                                                           \
    case PP:                                                                                               \
        hipLaunchKernelGGL(k_batch_interior<PP>, grid, dim3(Int2Cfg<PP>::NT), 0, side, d_plans, it); \
        break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
                default: break;
            }
        }
        HIPX(hipEventRecord(ev_join, side));
        for (int g = 0; g < kBatchGroups; ++g) {  // DWQ side rules (read the knots only)
            if (dwqs_n[g] == 0) continue;
            const BatchItem* it = d_rows + dwqs_off[g];
            const dim3 grid((unsigned)dwqs_n[g]);
            switch (g + 1) {
#define CASE(PP)                                                                                 \
    case PP:                                                                                     \
        hipLaunchKernelGGL(k_batch_dwq_sides<PP>, grid, dim3(kDwqSideThreads), 0, s, d_plans, it); \
        break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
                default: break;
            }
        }
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, d_counters, nc);
        BatchDev B{};
        B.plans = d_plans;
        B.items = d_items;
        B.status = d_counters;
        B.heads = d_counters + 1;
        B.level_done = d_counters + 1 + kBatchGroups;
        B.spin_limit = 1 << 20;
        B.chunk = chunk;
        int total = 0;
        split(B.first_block, total);
        for (int g = 0; g < kBatchGroups; ++g) {
            B.off[g] = g_off[g];
            B.n[g] = g_n[g];
            B.n_level[g][0] = g_lvl[g][0];
            B.n_level[g][1] = g_lvl[g][1];
        }
        if (!persistent) {
            total = 0;
            for (int g = 0; g < kBatchGroups; ++g) {
                if (cute_n[g] == 0) continue;
                const BatchItem* it = d_rows + cute_off[g];
                const dim3 grid((unsigned)cute_n[g]);
                switch (g + 1) {
#define CASE(PP)                                                                            \
    case PP:                                                                                \
        hipLaunchKernelGGL(k_batch_cut_elems<PP>, grid, dim3(256), 0, s, d_plans, it); \
        break;
                    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
                    default: break;
                }
            }
        }
        if (total > 0) {
            size_t lds = 0;
            for (int g = 0; g < kBatchGroups; ++g)
                if (g_n[g] > 0) lds = std::max(lds, batch_smem_bytes(g + 1));
            if (capped) hipLaunchKernelGGL(k_batch<2>, dim3(total), dim3(256), lds, s, B);
            else hipLaunchKernelGGL(k_batch<1>, dim3(total), dim3(256), lds, s, B);
        }
        HIPX(hipStreamWaitEvent(s, ev_coef, 0));
        for (int g = 0; g < kBatchGroups; ++g) {
            if (rows_n[g] == 0) continue;
            const BatchItem* it = d_rows + rows_off[g];
            const dim3 grid((unsigned)rows_n[g]);
            switch (g + 1) {
#define CASE(PP)                                                                                              \
    case PP:                                                                                                  \
        hipLaunchKernelGGL(k_batch_cut_rows<PP>, grid, dim3(batch_cut_row_threads(PP)), 0, s, d_plans, it); \
        break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
                default: break;
            }
        }
        for (int g = 0; g < kBatchGroups; ++g) {  // DWQ box parts, added to the element-formed rows
            if (dwqr_n[g] == 0) continue;
            const BatchItem* it = d_rows + dwqr_off[g];
            const dim3 grid((unsigned)dwqr_n[g]);
            switch (g + 1) {
#define CASE(PP)                                                                                \
    case PP:                                                                                    \
        hipLaunchKernelGGL(k_batch_dwq_rows<PP>, grid, dim3(256), 0, s, d_plans, it); \
        break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
                default: break;
            }
        }
        HIPX(hipStreamWaitEvent(s, ev_join, 0));
    }
};

static double item_cost(const Plan& P, int kind, int unit, const std::vector<int>& node_off) {
    const double p1 = P.p + 1.0;
    switch (kind) {
        case BK_COEF: return kCgPts * p1 * 8.0;
        case BK_CUTE: return (node_off[unit + 1] - node_off[unit]) * p1 * p1 * p1 * p1 * 0.5;
        case BK_INT: return 64.0 * p1 * p1 * p1 * 4.0;
        default: return p1 * p1 * p1 * p1 * p1;
    }
}

}  // namespace iga

struct iga_batch : public iga::Batch {};

namespace iga {

BatchView batch_view(iga_batch* b) {
    return BatchView{(int)b->plans.size(), b->plans.data(), b->coeffs.data(), b->outs.data(), &b->solve};
}

static iga_batch* batch_create(iga_plan* const* plans, int count, const iga_coeff* cs, double* const* outs) {
    IGA_REQUIRE(count > 0 && plans && cs && outs, IGA_E_INVALID, "empty batch");
    for (int k = 0; k < count; ++k) {  // every argument before any device work
        IGA_REQUIRE(plans[k], IGA_E_INVALID, "null plan in batch");
        IGA_REQUIRE(outs[k], IGA_E_INVALID, "output buffer missing");
        const Plan& P = *static_cast<const Plan*>(plans[k]);
        IGA_REQUIRE(P.p <= kBatchMaxP, IGA_E_UNSUPPORTED, "batched formation handles degrees up to 6");
        IGA_REQUIRE(P.method == IGA_HYBRID_GAUSS || P.method == IGA_GAUSS_REF || P.method == IGA_DWQ,
                    IGA_E_UNSUPPORTED, "batched formation handles hybrid Gauss, element Gauss and DWQ plans");
    }
    auto B = std::make_unique<iga_batch>();
    int dev = 0;
    HIPX(hipGetDevice(&dev));
    HIPX(hipDeviceGetAttribute(&B->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    // A grid larger than what fits at once is allowed: workgroups past the
    // resident ones start as those finish, and each degree's share of the
    // grid then keeps more of its items in flight (measured faster). Only
    // resident workgroups ever hold items, so the dependency waits still end.
    HIPX(hipStreamCreate(&B->cap_stream));
    HIPX(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&B->ev_coef, hipEventDisableTiming));
    std::vector<BatchPlan> hp(count);
    struct Cand {
        BatchItem it;
        double cost;
    };
    std::vector<Cand> all;
    std::vector<BatchItem> coefs[kBatchGroups], tiles[kBatchGroups], rows[kBatchGroups], cutes[kBatchGroups];
    std::vector<BatchItem> dwqs[kBatchGroups], dwqr[kBatchGroups];
    for (int k = 0; k < count; ++k) {
        Plan& P = *static_cast<Plan*>(plans[k]);
        const iga_coeff& c = cs[k];
        IGA_REQUIRE(!(P.method == IGA_DWQ && c.kind == IGA_COEF_AT_POINTS), IGA_E_UNSUPPORTED,
                    "discontinuous weighted quadrature needs c at nested points: constant or |det J| only");
        IGA_REQUIRE(c.kind >= IGA_COEF_CONST && c.kind <= IGA_COEF_AT_POINTS, IGA_E_UNSUPPORTED, "coefficient kind");
        IGA_REQUIRE(c.kind != IGA_COEF_GEOM_DETJ || c.geom_cp, IGA_E_INVALID, "geometry control points missing");
        IGA_REQUIRE(c.kind != IGA_COEF_AT_POINTS || c.c_points, IGA_E_INVALID, "per-point coefficient missing");
        B->plans.push_back(&P);
        B->coeffs.push_back(c);
        B->outs.push_back(outs[k]);
        B->nnz += P.nnz;
        BatchPlan& bp = hp[k];
        bp.p = P.p;
        bp.method = P.method;
        bp.ia = int_args(P, c, outs[k]);
        bp.ce = cute_args(P, c);
        bp.cr = cutr_args(P, c, outs[k]);
        bp.co = coef_args(P, c);
        bp.dr = DwqRowArgs{P.dir[0], P.dir[1], coef_view(P, c), c.geom_cp, P.form_rows, (int)P.n_form_rows,
                           P.fn_of, P.act_of, P.dwq_region, outs[k], P.n_act};
        bp.gx = P.gauss_x;
        bp.gw = P.gauss_w;
        bp.status = P.status;
        if (P.method == IGA_DWQ) {
            const int nslot = 2 * (P.N1 - 1) + 2 * (P.N2 - 1), spw = dwq_side_spw(P.p);
            for (int u = 0; u < (nslot + spw - 1) / spw; ++u) dwqs[P.p - 1].push_back(BatchItem{k, 0, u, 0});
            if (P.n_form_rows > 0) {
                std::vector<int> reg(8 * (size_t)P.n_form_rows);
                HIPX(hipMemcpy(reg.data(), P.dwq_region, sizeof(int) * reg.size(), hipMemcpyDeviceToHost));
                for (int r = 0; r < (int)P.n_form_rows; ++r)
                    if (reg[8 * (size_t)r] >= 0) dwqr[P.p - 1].push_back(BatchItem{k, 0, r, 0});
            }
        }
        std::vector<int> node_off(P.n_cut_el + 1, 0);
        if (P.n_cut_el > 0)
            HIPX(hipMemcpy(node_off.data(), P.node_off, sizeof(int) * (P.n_cut_el + 1), hipMemcpyDeviceToHost));
        const int n_coef = (c.kind == IGA_COEF_GEOM_DETJ)
                               ? coef_grid_tiles(P.dir[0].Q, P.dir[1].N) + (int)((bp.co.nb + kCgPts - 1) / kCgPts)
                               : 0;
        const int n_int = (P.method == IGA_GAUSS_REF) ? 0 : interior2_ntx(P.N1, P.p) * P.n2;
        const int n_cute = (int)P.n_cut_el, n_cutr = (int)P.n_form_rows;
        const int counts[BK_NKIND] = {n_coef, n_cute, n_int, n_cutr};
        for (int kind = 0; kind < BK_NKIND; ++kind) {
            bp.need[kind] = counts[kind];
            if (kind == BK_CUTE)  // also listed per degree, for the one-workgroup-each alternative
                for (int u = 0; u < counts[kind]; ++u) cutes[P.p - 1].push_back(BatchItem{k, kind, u, 0});
            if (kind != BK_CUTE) {  // launches of their own
                auto& dst = (kind == BK_COEF) ? coefs[P.p - 1] : (kind == BK_INT) ? tiles[P.p - 1] : rows[P.p - 1];
                for (int u = 0; u < counts[kind]; ++u) dst.push_back(BatchItem{k, kind, u, 0});
                continue;
            }
            for (int u = 0; u < counts[kind]; ++u)
                all.push_back({BatchItem{k, kind, u, 0}, item_cost(P, kind, u, node_off)});
        }
    }
    // queues by degree; inside, kinds in dependency order (coefficients, then cut elements), then
    // by decreasing cost (or patch by patch)
    auto stage = [](int kind) { return kind == BK_COEF ? 0 : (kind == BK_CUTE ? 1 : 2); };
    auto deg = [&](const Cand& a) { return hp[a.it.plan].p; };
    std::vector<Cand> lpt = all;
    std::stable_sort(lpt.begin(), lpt.end(), [&](const Cand& a, const Cand& b) {
        if (deg(a) != deg(b)) return deg(a) < deg(b);
        if (stage(a.it.kind) != stage(b.it.kind)) return stage(a.it.kind) < stage(b.it.kind);
        return a.cost > b.cost;
    });
    std::vector<Cand> pm = all;
    std::stable_sort(pm.begin(), pm.end(), [&](const Cand& a, const Cand& b) {
        if (deg(a) != deg(b)) return deg(a) < deg(b);
        if (stage(a.it.kind) != stage(b.it.kind)) return stage(a.it.kind) < stage(b.it.kind);
        return a.it.plan < b.it.plan;
    });
    for (int g = 0; g < kBatchGroups; ++g) B->g_off[g] = B->g_n[g] = 0;
    for (size_t k = 0; k < lpt.size(); ++k) {
        const int g = deg(lpt[k]) - 1;
        if (B->g_n[g] == 0) B->g_off[g] = (int)k;
        B->g_n[g]++;
        if (stage(lpt[k].it.kind) < 2) B->g_lvl[g][stage(lpt[k].it.kind)]++;
        B->g_work[g] += lpt[k].cost;
    }
    for (auto& c : lpt) B->items_lpt.push_back(c.it);
    for (auto& c : pm) B->items_plan.push_back(c.it);
    std::vector<BatchItem> rows_all;
    for (int g = 0; g < kBatchGroups; ++g) {
        B->coef_off[g] = (int)rows_all.size();
        B->coef_n[g] = (int)coefs[g].size();
        rows_all.insert(rows_all.end(), coefs[g].begin(), coefs[g].end());
    }
    for (int g = 0; g < kBatchGroups; ++g) {
        B->cute_off[g] = (int)rows_all.size();
        B->cute_n[g] = (int)cutes[g].size();
        rows_all.insert(rows_all.end(), cutes[g].begin(), cutes[g].end());
    }
    for (int g = 0; g < kBatchGroups; ++g) {
        B->int_off[g] = (int)rows_all.size();
        B->int_n[g] = (int)tiles[g].size();
        rows_all.insert(rows_all.end(), tiles[g].begin(), tiles[g].end());
    }
    for (int g = 0; g < kBatchGroups; ++g) {
        B->rows_off[g] = (int)rows_all.size();
        B->rows_n[g] = (int)rows[g].size();
        rows_all.insert(rows_all.end(), rows[g].begin(), rows[g].end());
    }
    for (int g = 0; g < kBatchGroups; ++g) {
        B->dwqs_off[g] = (int)rows_all.size();
        B->dwqs_n[g] = (int)dwqs[g].size();
        rows_all.insert(rows_all.end(), dwqs[g].begin(), dwqs[g].end());
    }
    for (int g = 0; g < kBatchGroups; ++g) {
        B->dwqr_off[g] = (int)rows_all.size();
        B->dwqr_n[g] = (int)dwqr[g].size();
        rows_all.insert(rows_all.end(), dwqr[g].begin(), dwqr[g].end());
    }
    // cut elements sit in the queue and in their per-degree list: count them once
    B->n_items = (int)(rows_all.size() + all.size());
    for (int g = 0; g < kBatchGroups; ++g) B->n_items -= B->cute_n[g];
    HIPX(hipMalloc(&B->d_plans, sizeof(BatchPlan) * count));
    HIPX(hipMemcpy(B->d_plans, hp.data(), sizeof(BatchPlan) * count, hipMemcpyHostToDevice));
    HIPX(hipMalloc(&B->d_items, sizeof(BatchItem) * std::max<size_t>(1, all.size())));
    HIPX(hipMalloc(&B->d_rows, sizeof(BatchItem) * std::max<size_t>(1, rows_all.size())));
    if (!rows_all.empty())
        HIPX(hipMemcpy(B->d_rows, rows_all.data(), sizeof(BatchItem) * rows_all.size(), hipMemcpyHostToDevice));
    HIPX(hipMalloc(&B->d_counters, sizeof(int) * (1 + 3 * kBatchGroups)));
    HIPX(hipMemset(B->d_counters, 0, sizeof(int) * (1 + 3 * kBatchGroups)));
    B->upload_items(B->cap_stream);
    return B.release();
}

static void batch_form(Batch& B, int use_graph, hipStream_t s) {
    if (!use_graph) {
        B.launch(s);
        return;
    }
    if (!B.exec) {
        HIPX(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeRelaxed));
        B.launch(B.cap_stream);
        HIPX(hipStreamEndCapture(B.cap_stream, &B.graph));
        HIPX(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    }
    HIPX(hipGraphLaunch(B.exec, s));
}

// Times every (register budget, workgroups per CU, queue chunk, item order) choice on the device,
// keeps the fastest.
static void batch_autotune(Batch& B, hipStream_t s, float* best_ms) {
    hipEvent_t a, b;
    HIPX(hipEventCreate(&a));
    HIPX(hipEventCreate(&b));
    float best = 1e30f;
    int bw = B.wg_per_cu, bo = B.order;
    int bc = B.chunk, bcap = B.capped;
    B.persistent = 1;
    for (int order = 0; order < 2; ++order) {
        B.order = order;
        B.upload_items(s);
        for (int cap = 0; cap < 2; ++cap)
        for (int cidx = 0; cidx < 3; ++cidx)
        for (int w : {1, 2, 4, 8, 12, 16}) {
            if (w > B.max_wg_per_cu) break;
            B.capped = cap;
            B.chunk = (cidx == 0) ? 4 : (cidx == 1 ? 16 : 64);
            B.wg_per_cu = w;
            B.launch(s);  // warm-up
            float t = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                HIPX(hipEventRecord(a, s));
                B.launch(s);
                HIPX(hipEventRecord(b, s));
                HIPX(hipEventSynchronize(b));
                float ms = 0.f;
                HIPX(hipEventElapsedTime(&ms, a, b));
                t = std::min(t, ms);
            }
            if (t < best) {
                best = t;
                bw = w;
                bo = order;
                bc = B.chunk;
                bcap = cap;
            }
        }
    }
    // the alternative: every cut element its own workgroup, no queue
    B.persistent = 0;
    B.launch(s);  // warm-up
    float tp = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        HIPX(hipEventRecord(a, s));
        B.launch(s);
        HIPX(hipEventRecord(b, s));
        HIPX(hipEventSynchronize(b));
        float ms = 0.f;
        HIPX(hipEventElapsedTime(&ms, a, b));
        tp = std::min(tp, ms);
    }
    B.persistent = tp < best ? 0 : 1;
    best = std::min(best, tp);
    hipEventDestroy(a);
    hipEventDestroy(b);
    B.wg_per_cu = bw;
    B.order = bo;
    B.chunk = bc;
    B.capped = bcap;
    B.upload_items(s);
    B.drop_graph();
    if (best_ms) *best_ms = best;
}

}  // namespace iga

using namespace iga;

extern "C" {

#define API_TRY try {
#define API_CATCH                             \
    }                                         \
    catch (const Error& e) {                  \
        set_error(e.msg);                     \
        return e.code;                        \
    }                                         \
    catch (const std::exception& e) {         \
        set_error(e.what());                  \
        return IGA_E_INVALID;                 \
    }                                         \
    return IGA_OK;

int iga_batch_create(iga_plan* const* plans, int32_t count, const iga_coeff* cs, double* const* vals,
                     iga_batch** out) {
    API_TRY
    IGA_REQUIRE(out, IGA_E_INVALID, "null argument");
    *out = nullptr;
    *out = batch_create(plans, count, cs, vals);
    API_CATCH
}

void iga_batch_destroy(iga_batch* b) {
    if (!b) return;
    hipDeviceSynchronize();
    delete b;
}

int iga_batch_form(iga_batch* b, int32_t use_graph, void* stream) {
    API_TRY
    IGA_REQUIRE(b, IGA_E_INVALID, "null batch");
    batch_form(*b, use_graph, (hipStream_t)stream);
    HIPX(hipGetLastError());
    API_CATCH
}

int iga_batch_autotune(iga_batch* b, void* stream, float* best_ms) {
    API_TRY
    IGA_REQUIRE(b, IGA_E_INVALID, "null batch");
    batch_autotune(*b, (hipStream_t)stream, best_ms);
    API_CATCH
}

int iga_batch_info(const iga_batch* b, iga_batch_stats* st) {
    API_TRY
    IGA_REQUIRE(b && st, IGA_E_INVALID, "null argument");
    st->n_plans = (int64_t)b->plans.size();
    st->n_items = b->n_items;
    st->nnz = b->nnz;
    st->grid = b->persistent ? b->grid() : 0;
    st->wg_per_cu = b->wg_per_cu;
    st->order = b->order;
    st->capped = b->capped;
    st->chunk = b->chunk;
    st->graph_ready = b->exec != nullptr;
    API_CATCH
}

int iga_batch_status(iga_batch* b, void* stream) {
    API_TRY
    IGA_REQUIRE(b, IGA_E_INVALID, "null batch");
    int h = 0;
    HIPX(hipMemcpyAsync(&h, b->d_counters, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPX(hipStreamSynchronize((hipStream_t)stream));
    IGA_REQUIRE(h == 0, IGA_E_INVALID, "a dependency wait of the batched kernel hit its bound");
    for (Plan* P : b->plans) {
        int st = 0;
        HIPX(hipMemcpy(&st, P->status, sizeof(int), hipMemcpyDeviceToHost));
        IGA_REQUIRE(st == 0, st, "device status of a batched plan");
    }
    API_CATCH
}

int iga_trim_mass_form_batched(iga_plan* const* plans, int32_t count, const iga_coeff* cs, double* const* vals,
                               int32_t use_graph, void* stream) {
    API_TRY
    std::unique_ptr<iga_batch> B(batch_create(plans, count, cs, vals));
    batch_form(*B, use_graph, (hipStream_t)stream);
    HIPX(hipStreamSynchronize((hipStream_t)stream));
    API_CATCH
}

}  // extern "C"
