// Internal layout of a plan: device tables of one trimmed patch.
#pragma once

#include <hip/hip_ext.h>

#include "common.hpp"

#include <vector>

namespace iga {

enum ElemClass : int8_t { EL_OUTSIDE = 0, EL_INSIDE = 1, EL_CUT = 2 };
enum FnClass : int8_t { FN_EXTERIOR = 0, FN_INTERIOR = 1, FN_CUT = 2 };

// Endpoint kinds of an arc: a piece end, a crossing of x = bp1[line], or of y = bp2[line].
enum : int32_t { END_PIECE = 0, END_VLINE = 1, END_HLINE = 2 };

constexpr int kMaxEdgeSegs = 8;     // visible segments per element edge
constexpr int kMaxEdgeCuts = 16;    // split points per element edge
constexpr int kMaxPiecesPerSeg = 5; // monotone pieces per curve segment
constexpr int kMaxIsectPerPiece = 8;
constexpr int kRowCross = 16;       // centre-line crossings kept per row of elements
constexpr int kMaxArcsPerElem = 64; // kept arcs per cut element

// Per-direction weighted-quadrature and Gauss tables (device pointers).
struct DirDev {
    int N;      // elements
    int n;      // functions
    int Q;      // WQ points
    int qmax;   // max points in one support
    const double* knots;  // p+1 repeated ends + interior (length N + 2p + 1)
    double* bp;           // N+1 breakpoints
    double* xq;           // Q
    int* eq;              // Q owning element
    int* pt0;             // N+1 first point of element
    double* Bq;           // Q*(p+1)
    double* dBq;          // Q*(p+1)
    double* M1;           // n*(2p+1) univariate mass band
    double* W;            // n*qmax weights, point k0(i)+q with k0(i) = pt0[max(0,i-p)]
    double* WB;           // n*qmax*(2p+1): W[i][q] * B_{i+b-p}(x_{k0(i)+q}) (0 off the element)
    double* WBT;          // (2p+2)*(p+1)*n: WB[i][q][(q>>1)+al] at [(q*(p+1)+al)*n + i] (the band, rows contiguous)
    double* WT;           // (2p+2)*n: W[i][q] at [q*n + i] (rows contiguous; 0 past the row's points)
    double* xg;           // N*(p+1) Gauss points
    double* wg;           // N*(p+1) Gauss weights
    double* Bg;           // N*(p+1)*(p+1) [e][g][a]
    double* dBg;          // N*(p+1)*(p+1)
    // discontinuous weighted quadrature (method IGA_DWQ), one list per side of
    // every interior knot s = 1..N-1, slot = 2 (s-1) + side (0 below, 1 above)
    int dq_KQ;            // points per list (capacity)
    int* dq_n;            // [slots] points in the list
    double* dq_x;         // [slots][KQ] coordinates, increasing
    int* dq_el;           // [slots][KQ] owning element
    int* dq_k;            // [slots][KQ] WQ point index, -1 for a nested point
    double* dq_w;         // [slots][p][KQ] weights of B_{s+ii}, ii = 0..p-1
};

struct CurveDev {
    int kind;       // IGA_CURVE_*
    int degree;
    int n_seg;      // polynomial segments (1 for ellipses)
    int seg0;       // first segment in the segment array
    double cx, cy, a, b, phi;
    double sigma;   // -1 if the native orientation is counter-clockwise
    double t_range; // parameter length of one segment (1 or 2 pi)
};

struct SegDev {
    int curve;
    int seg;        // index within its curve
    int kind;
    int pad;
    double px[4], py[4];  // power coefficients, low first (BSPLINE)
};

struct PieceDev {
    int curve, seg;      // owning curve and segment
    int pad0, pad1;
    double t0, t1;       // parameter range, t0 < t1
    double x0, y0, x1, y1;
};

struct CrossDev {
    double t;
    int kind;   // END_VLINE or END_HLINE
    int line;   // breakpoint index
};

struct ArcDev {
    int curve, gseg, piece, keep;   // gseg: index into the segment array
    double t0, t1;
    double x0, y0, x1, y1;          // curve points at t0 and t1
    int e1, e2;
    int k0, l0;   // start endpoint kind / line
    int k1, l1;   // end endpoint kind / line
};

struct CutElemDev {
    int e1, e2;
    int variant;        // 0 left, 1 right, 2 bottom, 3 top base
    int nseg[4];        // visible segments per edge: 0 left, 1 right, 2 bottom, 3 top
    int narc;           // kept arcs in the element, ascending arc index
    double seg[4][kMaxEdgeSegs][2];
    int arc[kMaxArcsPerElem];
};

// Everything the trimming kernels need, passed by value.
struct TrimDev {
    int n_curves;
    int n_segs;
    const CurveDev* curves;
    SegDev* segs;
    PieceDev* pieces;      // capacity cap_pieces
    int* n_pieces;         // device count
    int* piece_curve_off;  // n_curves+1: pieces of curve c are [off[c], off[c+1])
    PieceDev* pieces0;     // before curve-curve splits
    int* n_pieces0;
    double* isect_t;       // cap_pieces0 * kMaxIsectPerPiece
    int* isect_n;
    CrossDev* cross;       // crossings of long pieces (more than fit in LDS), arc_slot per piece
    CrossDev* merged;      // the same sorted by t
    ArcDev* arcs;          // arc_slot per piece: the arcs of piece k are k*arc_slot + j, j <= its crossings
    int cap_pieces0, cap_pieces, cap_arcs;
    int arc_slot;          // most crossings of one piece (found at plan creation) + 1
    // Per row of elements: crossings of spline pieces with the horizontal line
    // through the row's element centres (key = min(X, piece's largest x)).
    int* epoch;            // the set-up counter (device; k_trim_front advances it)
    int* row_cnt;          // N2
    double* row_key;       // N2 * kRowCross
    int* row_curve;        // N2 * kRowCross
};

// Buffers of the L2 projection and the matrix-free product (allocated on first use).
struct SolveWork {
    double* gc = nullptr;     // g c at every rule point
    double* F = nullptr;      // element vectors of band and cut elements
    double* A = nullptr;      // (M + M^T)/2
    double *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr, *part = nullptr, *scal = nullptr, *b = nullptr;
    double* h_scal = nullptr; // pinned host copy of the scalars
    int* cols = nullptr;      // compact column of each band slot (PCG)
    double* Ue = nullptr;     // matrix-free: element vectors
    double* mfpart = nullptr; // matrix-free: rows split between two bands [2][nband][p][n1]
    int* adj_rows = nullptr;  // matrix-free adjoint: rows with band or cut elements in their support
    int n_adj_rows = 0;
    // extended B-splines (first extended projection): vectors of the extended system live in the
    // compact row space, zero at outer rows
    int8_t* x_inner = nullptr;  // [n2][n1] active with an inside element in the support
    int8_t* x_ok = nullptr;     // [n2-p][n1-p] block {l..l+p}^2 of inner functions only
    int* x_slot = nullptr;      // [n_act] outer slot of the row, -1 for inner rows
    int* x_cnt = nullptr;       // [n_act] outer rows tied to the row (a fill cursor after the scan)
    int* x_off = nullptr;       // [n_act + 1] start of the row's list of outer rows
    int* x_misc = nullptr;      // [2] outer rows, error
    int* x_row = nullptr;       // [x_cap] compact row of each outer slot
    int* x_fid = nullptr;       // [x_cap][(p+1)^2] block members (compact)
    double* x_fw = nullptr;     // [x_cap][(p+1)^2] their weights
    int* x_tj = nullptr;        // per inner row, ascending: the outer rows tied to it
    double* x_tw = nullptr;     // and their weights
    double *x_dg = nullptr, *x_e = nullptr, *x_z = nullptr, *x_w = nullptr, *x_b = nullptr, *x_p = nullptr;
    int x_cap = 0;
};

struct Plan {
    int device = 0;
    int p = 0;
    int method = IGA_HYBRID_GAUSS;
    int n_r = 0, n_q_override = 0, n_s = 0;
    int N1 = 0, N2 = 0, n1 = 0, n2 = 0;

    // raw inputs (device)
    double* knots[2] = {nullptr, nullptr};
    std::vector<double> h_knots[2];
    std::vector<CurveDev> h_curves;
    std::vector<SegDev> h_segs_in;  // control points kept here for the segment build
    double* d_cp = nullptr;         // packed curve control points (x, y)
    int* d_cp_off = nullptr;        // per curve offset into d_cp

    DirDev dir[2];
    double* gauss_x = nullptr;  // packed Gauss-Legendre table
    double* gauss_w = nullptr;

    // trimming
    TrimDev trim{};
    CurveDev* d_curves = nullptr;
    int8_t* ecls = nullptr;        // N1*N2
    int* cut_id = nullptr;         // N1*N2 -> cut element id or -1
    int* band_id = nullptr;        // N1*N2 -> band element id or -1
    int8_t* fcls = nullptr;        // n1*n2
    int* act_of = nullptr;         // n1*n2
    int* fn_of = nullptr;          // n_act
    int* cut_rows = nullptr;       // compact ids of cut rows
    int* form_rows = nullptr;      // rows formed by the element/cut kernel (method dependent)
    int* dwq_region = nullptr;     // [n_form_rows][8] DWQ box of each formed row (lo1 = -1: none)
    int* emark = nullptr;          // [N1*N2] element owns a visible arc iff emark == epoch
    // [N1*N2] head of the element's list of kept arcs: (epoch << 32) | (arc + 1),
    // stale when the epoch differs; arc_next[a] is the next arc of a's element or -1
    unsigned long long* ehead = nullptr;
    int* arc_next = nullptr;
    int* d_epoch = nullptr;        // set-up counter on the device, advanced by the trimming front (marks need no clearing)
    int* cut_list = nullptr;       // flat ids of cut elements
    int* band_list = nullptr;      // flat ids of band elements
    CutElemDev* cut_el = nullptr;
    int* cut_e = nullptr;          // flat id of each cut element, written by the cut-rule kernel
    int* node_cnt = nullptr;
    int* node_off = nullptr;
    double* node_x = nullptr;      // n_cut_nodes
    double* node_y = nullptr;
    double* node_w = nullptr;
    int* node_el = nullptr;        // cut element id of each node
    double* cutE = nullptr;        // n_cut_el * (p+1)^4 local matrices
    double* cut_part = nullptr;    // n_form_rows * (2p+1)^2 inside sums of the two-launch row formation

    // scratch for scans and counts
    int* flags = nullptr;          // max(n1*n2, N1*N2) + 1
    int* list_rcnt = nullptr;      // [4][n2][tiles along xi_1] flags set per row segment of a class tile
    int* scan_tmp = nullptr;       // block sums of a scan, then compaction positions
    int scan_pos_off = 0;
    int* counts = nullptr;         // small device counter block
    int* status = nullptr;         // device status word

    // points and coefficient values (c_wq [Q2][Q1], c_band, c_cut)
    double* pts_xy = nullptr;      // n_points * 2
    double* c_wq = nullptr;
    double* c_band = nullptr;
    double* c_cut = nullptr;
    double* c_wq_masked = nullptr; // naive WQ only

    // sizes
    int64_t n_act = 0, n_interior = 0, n_cut_fn = 0, n_cut_el = 0, n_band = 0;
    int64_t n_nodes = 0, n_arcs = 0, nnz = 0, n_form_rows = 0, n_points = 0, n_dwq_rows = 0;
    int64_t bytes = 0;

    // second stream of the formation: univariate tables, weights, WQ-grid coefficient and interior
    // rows run there, beside the trimming chain (default priority; joined by events)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_iso = nullptr, ev_lists = nullptr, ev_interior = nullptr, ev_band = nullptr,
               ev_classes = nullptr;
    hipEvent_t ev_aux_lists = nullptr;  // second stream: WQ-grid c and (split formation) the lists are done

    // timing
    bool timing = false;
    // per-kernel timing: every dispatch of the formation path bracketed by events at its start and end
    bool ktiming = false;
    struct KRec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<KRec> k_records;
    std::vector<hipEvent_t> k_pool;  // events of read records, reused
    hipEvent_t kevent() {
        if (!k_pool.empty()) {
            hipEvent_t e = k_pool.back();
            k_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        HIPX(hipEventCreate(&e));
        return e;
    }
    // The formation as one HIP graph (captured on a private stream, replayed on the caller's):
    // valid while the output, coefficient and flags match the captured call.
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t fgraph = nullptr;
    hipGraphExec_t fexec = nullptr;
    double* fkey_vals = nullptr;
    iga_coeff fkey_c{};
    int fkey_flags = -1;
    double* pkey_vals = nullptr;   // the previous call run kernel by kernel
    iga_coeff pkey_c{};
    int pkey_flags = -1;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_records;
    double phase_ms[IGA_PHASE_COUNT] = {0, 0, 0, 0};
    int64_t phase_cnt[IGA_PHASE_COUNT] = {0, 0, 0, 0};

    SolveWork sw;
    std::vector<void*> allocations;
    template <typename T>
    T* alloc(size_t n) {
        void* ptr = nullptr;
        size_t bytes_ = n * sizeof(T) + 16;
        if (hipMalloc(&ptr, bytes_) != hipSuccess)
            throw Error{IGA_E_NOMEM, "hipMalloc of " + std::to_string(bytes_) + " bytes failed"};
        allocations.push_back(ptr);
        bytes += (int64_t)bytes_;
        return static_cast<T*>(ptr);
    }
    ~Plan();
};

// Launch of a formation-path kernel; with per-kernel timing on, the
// dispatch is bracketed by events recorded at its start and end.
template <typename... Params, typename... Args>
inline void klaunch(Plan& P, const char* name, void (*kernel)(Params...), dim3 grid, dim3 block, uint32_t smem,
                    hipStream_t s, Args... args) {
    if (P.ktiming) {
        hipEvent_t a = P.kevent(), b = P.kevent();
        hipExtLaunchKernelGGL(kernel, grid, block, smem, s, a, b, 0, static_cast<Params>(args)...);
        P.k_records.push_back({name, a, b});
    } else {
        hipLaunchKernelGGL(kernel, grid, block, smem, s, args...);
    }
}

// Coefficient values seen by the formation kernels.
struct CoefView {
    int is_const;
    double value;
    const double* wq;    // [Q2][Q1]
    const double* band;  // [n_band][(p+1)^2]
    const double* cut;   // [n_nodes]
};

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


// ---------------------------------------------------------------- launchers
// setup.hip
void launch_gauss_table(Plan& P, hipStream_t s);
void launch_dir_tables(Plan& P, hipStream_t s);
void launch_wq_weights(Plan& P, hipStream_t s);
// the weights and c = |det J| on the WQ grid (with_points: the grid points' coordinates too) in one launch
void launch_weights_coef(Plan& P, const iga_coeff& c, hipStream_t s, bool with_points);
void launch_wb_table(Plan& P, int d, hipStream_t s);
// scan.hip
void exclusive_scan(const int* in, int* out, int n, int* tmp, hipStream_t s);
// trim.hip
void launch_trim_curves(Plan& P, hipStream_t s);            // segments + monotone pieces (+ unions)
void launch_trim_arcs(Plan& P, hipStream_t s);              // solve, merge, arcs
int trim_max_crossings(Plan& P, hipStream_t s);             // plan creation: most grid-line crossings of one piece
void launch_trim_classes(Plan& P, hipStream_t s);           // elements, functions, flags
void launch_trim_lists(Plan& P, hipStream_t s);             // act_of, cut/band lists
// per cut element segments, variant, counts; with fuse_nodes also the nodes, at the offsets plan creation found
void launch_trim_cutprep(Plan& P, hipStream_t s, bool fuse_nodes = false);
bool trim_lists_prefix_here(const Plan& P);                  // the list kernel sums its own row offsets
void launch_trim_nodes(Plan& P, hipStream_t s);             // node coordinates and weights
void launch_naive_mask(Plan& P, const double* src, double cval, hipStream_t s);
void launch_row_nnz(Plan& P, int* cnt, int* out, hipStream_t s);
// form.hip
CoefView coef_view(Plan& P, const iga_coeff& c);
// rule-point coordinates: WQ grid and band Gauss points (and the cut nodes with with_nodes)
void launch_points(Plan& P, hipStream_t s, bool with_nodes = false);
// part 0: every rule point, 1: WQ grid, 2: band and cut nodes, 3: band, 4: cut nodes; with_points: the
// grid and band points' coordinates are written to the rule-point table as well (|det J| only)
void launch_coef(Plan& P, const iga_coeff& c, hipStream_t s, int part = 0, bool with_points = false);
// t0 / t1 (optional): events recorded at the start and end of the kernel's execution
void launch_interior_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s, hipEvent_t t0 = nullptr,
                          hipEvent_t t1 = nullptr);
// the interior rows and c = |det J| at the band Gauss points (with_points: their coordinates too) in one launch
void launch_interior_coef(Plan& P, const iga_coeff& c, double* vals, hipStream_t s, bool with_points);
void launch_cut_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s);  // matrices, then rows
void launch_cut_elems(Plan& P, const iga_coeff& c, hipStream_t s);
// rows formed element-wise in one launch (mode 0), or their inside sums (1) and the cut entries (2)
void launch_cut_rows_mode(Plan& P, const iga_coeff& c, double* vals, hipStream_t s, int mode);
// dwq.hip
void launch_dwq_sides(Plan& P, hipStream_t s);
void launch_dwq_choose(Plan& P, hipStream_t s);
void launch_dwq_rows(Plan& P, const iga_coeff& c, double* vals, hipStream_t s);

// batch.hip: the plans, coefficients and outputs a batch borrows
struct BatchSolve;
struct BatchView {
    int n;
    Plan* const* plans;
    const iga_coeff* coeffs;
    double* const* outs;
    BatchSolve** solve;
};

}  // namespace iga

// The opaque handle of the C ABI is the plan itself.
struct iga_plan : public iga::Plan {};

namespace iga {
BatchView batch_view(iga_batch* b);
}
