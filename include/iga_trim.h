/*
 * iga_trim.h -- C ABI of the gfx950 library that forms isogeometric mass
 * matrices over trimmed bivariate B-spline patches by weighted quadrature.
 *
 * Method: Marussig, "Fast formation and assembly of isogeometric Galerkin
 * matrices for trimmed patches", arXiv 2101.08053.
 *
 *   M_ij = int_{Omega_v} c B_i B_j            (Eq. (6), visible domain of Sect. 2.2)
 *
 * Interior test functions use row-based weighted quadrature with sum
 * factorisation (Sect. 2.1, Eqs. (4), (5), (7)); cut test functions use
 * hybrid Gauss (Sect. 3.2) or discontinuous weighted quadrature (Sect. 3.3);
 * cut elements use a higher-order cut-element rule (Sect. 3.1). The matrix
 * feeds an L2 projection (Sect. 4.2).
 *
 * Conventions shared by every call:
 *  - Both parametric directions have the same degree p (1 <= p <= 8) and an
 *    open knot vector on [0, 1] with simple interior knots (C^{p-1}).
 *  - Function (i1, i2) has flat index i = i2 * n1 + i1 (xi_1 fastest); the
 *    active functions (not exterior) are numbered 0..n_act-1 in increasing
 *    flat order ("compact ids").
 *  - The mass matrix is returned in a slot-major band layout:
 *      vals[s * n_act + r],  s = (a + p) * (2p+1) + (b + p),  a, b in [-p, p],
 *    holding M(row r, column (i1 + a, i2 + b)). Column ids are implicit;
 *    slots whose column is out of range or exterior hold 0.
 *  - "Device" pointers are HIP device memory of the device that was current
 *    when the plan was created; "host" pointers are ordinary memory and are
 *    only read during the call. Streams are hipStream_t passed as void*
 *    (NULL = the default stream). Stream-ordered calls return after enqueue.
 *  - Every call returns IGA_OK (0) or a negative IGA_E_* code; no exception
 *    crosses the ABI. iga_last_error() gives a message for the calling thread.
 */
#ifndef IGA_TRIM_H
#define IGA_TRIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status codes */
#define IGA_OK                   0
#define IGA_E_INVALID           -1  /* bad argument, knot vector or curve          */
#define IGA_E_UNSUPPORTED       -2  /* degree outside 1..8, unknown kind, ...      */
#define IGA_E_NOMEM             -3  /* device allocation failed                    */
#define IGA_E_HIP               -4  /* a HIP runtime call failed                   */
#define IGA_E_SINGULAR_WEIGHTS  -5  /* a weight system (Eq. (5)) is rank deficient */
#define IGA_E_TOPOLOGY          -6  /* trimming geometry outside what is handled   */
#define IGA_E_CAPACITY          -7  /* a size exceeded what the plan reserved      */
#define IGA_E_NOCONV            -8  /* PCG did not reach the tolerance             */

/* ------------------------------------------------------------------ methods */
#define IGA_GAUSS_REF     0  /* element Gauss + cut rule on every row (Sect. 4 reference)  */
#define IGA_HYBRID_GAUSS  1  /* WQ interior rows, element Gauss cut rows (Sect. 3.2)     */
#define IGA_DWQ           2  /* WQ interior rows, discontinuous WQ cut rows (Sect. 3.3)  */
#define IGA_NAIVE_WQ      3  /* WQ on every row, c = 0 outside (Table 1, third column)   */

/* ------------------------------------------------------------ curve kinds */
#define IGA_CURVE_BSPLINE 0  /* closed uniform periodic B-spline, degree 1..3 */
#define IGA_CURVE_ELLIPSE 1  /* ellipse (circle when a == b)                  */

/* ------------------------------------------------------- coefficient kinds */
#define IGA_COEF_CONST      0  /* c = value                                          */
#define IGA_COEF_GEOM_DETJ  1  /* c = |det DF| of a B-spline map of the patch's space */
#define IGA_COEF_AT_POINTS  2  /* c given at every rule point (iga_plan_points order) */

/* ------------------------------------------------------------- form flags */
#define IGA_FORM_FULL     1  /* rebuild layout, weights, trimming data and cut rules first */

/* A closed trimming curve (Sect. 2.2). The hole is its interior, whatever
 * its orientation; the visible domain is [0,1]^2 minus the union of holes. */
typedef struct iga_curve {
    int32_t kind;        /* IGA_CURVE_*                                      */
    int32_t degree;      /* BSPLINE: 1..3                                    */
    int32_t n_cp;        /* BSPLINE: control points (> degree)               */
    int32_t reserved;
    const double* cp;    /* BSPLINE, host: n_cp (x, y) pairs                 */
    double cx, cy;       /* ELLIPSE: centre                                  */
    double a, b;         /* ELLIPSE: semi-axes (> 0)                         */
    double phi;          /* ELLIPSE: rotation of the a-axis (radians)        */
} iga_curve;

/* The problem statement: knots, degree, trimming curves, method. */
typedef struct iga_patch_desc {
    int32_t degree;              /* p, both directions                        */
    int32_t method;              /* IGA_GAUSS_REF .. IGA_NAIVE_WQ             */
    int32_t n_knots[2];          /* lengths of the two knot vectors            */
    const double* knots[2];      /* host                                      */
    int32_t n_curves;            /* 0 = untrimmed                             */
    int32_t reserved;
    const iga_curve* curves;     /* host, n_curves entries                    */
} iga_patch_desc;

/* Optional cut-rule settings (NULL or 0 fields = defaults). */
typedef struct iga_opts {
    int32_t n_r;        /* inner Gauss points of the cut rule (default p+1)          */
    int32_t n_q;        /* points per boundary arc (default d(2p+1), d = 3 ellipses) */
    int32_t n_s;        /* points along straight edge pieces (default p+1)           */
    int32_t reserved[5]; /* must be zero                                             */
} iga_opts;

typedef struct iga_plan iga_plan;   /* opaque, library owned */

typedef struct iga_sizes {
    int64_t p;
    int64_t N1, N2;           /* elements per direction                          */
    int64_t n1, n2;           /* functions per direction                         */
    int64_t n_act;            /* active functions = rows                         */
    int64_t n_interior;       /* interior functions                              */
    int64_t n_cut_fn;         /* cut functions                                   */
    int64_t n_cut_el;         /* cut elements                                    */
    int64_t n_band_el;        /* inside elements in the support of a cut function */
    int64_t band;             /* (2p+1)^2 slots per row                          */
    int64_t q1, q2;           /* weighted-quadrature points per direction        */
    int64_t n_cut_nodes;      /* nodes of all cut-element rules                  */
    int64_t n_points;         /* q1*q2 + n_band_el*(p+1)^2 + n_cut_nodes        */
    int64_t nnz;              /* active-active pairs inside the band             */
    int64_t n_arcs;           /* boundary arcs of the visible domain             */
    int64_t n_dwq_rows;       /* cut rows formed with a discontinuous rule (DWQ) */
    int64_t workspace_bytes;  /* device memory the plan holds                    */
} iga_sizes;

/* The coefficient c of Eq. (6). */
typedef struct iga_coeff {
    int32_t kind;             /* IGA_COEF_*                                              */
    int32_t reserved;
    double value;             /* CONST                                                   */
    const double* geom_cp;    /* GEOM_DETJ, device: control points [n2][n1][2]           */
    const double* c_points;   /* AT_POINTS, device: n_points values, iga_plan_points order */
} iga_coeff;

/* Target g of the L2 projection (Sect. 4.2). */
#define IGA_TARGET_SINCOS    0  /* g = sin(w0 x + w1) cos(w2 y + w3), x,y physical */
#define IGA_TARGET_MONOMIAL  1  /* g = x^e0 y^e1 (e = (int)w0, (int)w1)            */
#define IGA_TARGET_AT_POINTS 2  /* g given at every rule point                     */
typedef struct iga_target {
    int32_t kind;
    int32_t reserved;
    double w[4];
    const double* g_points;   /* AT_POINTS, device: n_points values */
} iga_target;

typedef struct iga_solve_info {
    int32_t iterations;
    int32_t converged;
    double rel_residual;      /* ||b - A u|| / ||b|| with A = (M + M^T)/2 */
} iga_solve_info;

/* ---------------------------------------------------------------- calls */

/* Builds a plan for one patch (Sects. 2.1-3.3): reads the host inputs, takes
 * device memory for every table, runs the set-up kernels once (weighted-
 * quadrature layout and weights, trimming, classes, cut rules, and for DWQ
 * the discontinuous weights) and synchronises to learn the sizes.
 * opts may be NULL. On success *out owns device memory until
 * iga_plan_destroy. Errors: IGA_E_INVALID (knots not open/uniformly simple,
 * curve data), IGA_E_UNSUPPORTED (p, kinds), IGA_E_NOMEM, IGA_E_HIP,
 * IGA_E_SINGULAR_WEIGHTS, IGA_E_TOPOLOGY. */
int iga_trim_plan_create(const iga_patch_desc* desc, const iga_opts* opts, iga_plan** out);

/* Releases the plan and its device memory (NULL is accepted). */
void iga_plan_destroy(iga_plan* plan);

/* Fills *s (host). */
int iga_plan_sizes(const iga_plan* plan, iga_sizes* s);

/* Device view of the rule points, valid while the plan lives: xy[2*k],
 * xy[2*k+1] are the parameter coordinates of point k, in this order:
 * the WQ grid (k = k2*q1 + k1), then the (p+1)^2 Gauss points of each band
 * element (flat element order, g2 outer, g1 inner), then the cut-element
 * nodes (cut elements in flat order). *npts receives n_points. */
int iga_plan_points(const iga_plan* plan, const double** xy, int64_t* npts);

/* Device views of the index maps, valid while the plan lives: act_of[flat]
 * (compact id or -1) of length n1*n2, fn_of[compact] (flat index) of length
 * n_act, fn_class[flat] (0 exterior, 1 interior, 2 cut). Any output may be NULL. */
int iga_plan_index_maps(const iga_plan* plan, const int32_t** act_of, const int32_t** fn_of,
                        const int8_t** fn_class);

/* Forms the mass matrix (Eq. (6) over the visible domain) with the plan's
 * method into vals (device, band * n_act doubles, caller owned), on stream.
 * flags & IGA_FORM_FULL re-runs every set-up kernel from the plan's inputs
 * before the formation (the whole job); without it the resident tables are
 * reused. Errors found on the device (a singular weight system) are reported
 * by iga_status_get after the stream has run. With method IGA_DWQ the
 * coefficient must be IGA_COEF_CONST or IGA_COEF_GEOM_DETJ (the rule has
 * points nested between the WQ points, where no per-point value is given):
 * IGA_E_UNSUPPORTED otherwise. */
int iga_trim_mass_form(iga_plan* plan, const iga_coeff* c, double* vals, int32_t flags, void* stream);

/* Graph replay of iga_trim_mass_form (on by default). A call with the same
 * (vals, coefficient, flags) as the previous one records the formation's
 * kernels and stream joins as a HIP graph on a private stream; later calls
 * with the same three replay it on the caller's stream (one submission),
 * reading the plan's inputs (curves, weights, nodes, coefficient values) as
 * they stand then. A call unlike the previous one runs kernel by kernel.
 * Plans with per-phase timing enabled, or method IGA_NAIVE_WQ, always launch
 * kernel by kernel. enable = 0 turns replay off for the plan. */
int iga_plan_set_graph(iga_plan* plan, int32_t enable);

/* Synchronises stream and returns the device status word of the plan
 * (IGA_OK, IGA_E_SINGULAR_WEIGHTS, IGA_E_TOPOLOGY or IGA_E_CAPACITY), then
 * clears it. */
int iga_status_get(iga_plan* plan, void* stream);

/* L2 projection (Sect. 4.2): b_i by row i's own rule applied to g c, then
 * Jacobi-preconditioned CG on A = (M + M^T)/2 (M from iga_trim_mass_form
 * with the same c) until ||b - A u|| <= rtol ||b|| or maxit iterations.
 * Row rules: weighted quadrature for interior rows; element Gauss and the
 * cut rule for rows formed element-wise; with IGA_DWQ, a cut row with a box
 * takes the box part from its discontinuous weights at the box's tensor
 * points (Sect. 3.3) and the rest of its support element-wise, as its matrix
 * row does. Methods IGA_HYBRID_GAUSS, IGA_DWQ and IGA_GAUSS_REF
 * (IGA_E_UNSUPPORTED otherwise); IGA_DWQ also needs g and c away from the
 * plan's rule points, so IGA_TARGET_AT_POINTS and IGA_COEF_AT_POINTS are
 * IGA_E_UNSUPPORTED there. u (device, n_act) is caller owned and used as the
 * start vector. Synchronous: returns after the solve. Returns IGA_E_NOCONV
 * (with u the last iterate and info filled) when the tolerance was not
 * reached. */
int iga_trim_l2_project(iga_plan* plan, const iga_coeff* c, const double* vals, const iga_target* g,
                        double rtol, int32_t maxit, double* u, iga_solve_info* info, void* stream);

/* Right-hand side alone: b (device, n_act) = row rules applied to g c (the
 * rules and the errors of iga_trim_l2_project). Asynchronous on stream. */
int iga_trim_rhs(iga_plan* plan, const iga_coeff* c, const iga_target* g, double* b, void* stream);

/* L2 projection in the extended B-spline basis (Sect. 2.2, closing remarks,
 * and Sect. 4.2: the paper stabilises its projections this way, after the
 * weighted extended B-splines of the works it cites). Inner functions are
 * active with an inside element in their support; every other active
 * (outer) function j is tied to the block {l1..l1+p} x {l2..l2+p} of inner
 * functions whose centre l + p/2 is nearest to j (squared index distance;
 * ties to the smaller l2, then l1), with weights e_{i,j} = e^1 e^2 that make
 * the block reproduce j's B-spline coefficient of every polynomial of degree
 * p in each direction. With E[i, j] = 1 (j = i inner) or e_{i,j}, the call
 * solves (E A E^T) x = E b by Jacobi-preconditioned CG (exact diagonal of
 * E A E^T) and writes u = E^T x. A = (M + M^T)/2 and b as in
 * iga_trim_l2_project, with its methods, arguments and errors; the start is
 * the inner coefficients of u; info reports ||E b - E A E^T x|| / ||E b||.
 * The blocks and weights follow the plan's element classes as they stand.
 * Errors also: IGA_E_TOPOLOGY (an outer function with no all-inner block:
 * the visible domain is too small for the degree), IGA_E_CAPACITY (more
 * outer functions than the plan's non-interior rows at creation).
 * Synchronous. */
int iga_trim_l2_project_ext(iga_plan* plan, const iga_coeff* c, const double* vals, const iga_target* g,
                            double rtol, int32_t maxit, double* u, iga_solve_info* info, void* stream);

/* The extension's columns (Sect. 2.2, as in iga_trim_l2_project_ext): for
 * every compact row j, members[j*(p+1)^2 + m] (compact ids, row-major over
 * the block, m = m2 (p+1) + m1) and weights[...] of the inner functions it
 * is tied to, so that u_j = sum_m weights * x[members]; an inner row has
 * itself with weight 1, then -1 and 0. members and weights are device
 * buffers of n_act (p+1)^2 entries, caller owned. Synchronous; errors as
 * iga_trim_l2_project_ext. */
int iga_trim_extension(iga_plan* plan, int32_t* members, double* weights, void* stream);

/* Matrix-free product y = M(c) u of Eq. (7) -- the weighted-quadrature rows
 * y_i = sum_k w_{k,i} c_k sum_j B_j(x_k) u_j, and the element rules of the cut
 * rows (Sect. 3.2) -- for device vectors of length n_act, with c
 * given at every rule point (c_points, n_points values), the rows formed by
 * the plan's interior and hybrid rules, basis values recomputed on the fly.
 * The weighted-quadrature part runs sum-factorised in one pass over the WQ
 * grid (strips of test columns by bands of elements), as does its adjoint. */
int iga_mf_apply(iga_plan* plan, const double* c_points, const double* u, double* y, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or solver loops, harnesses that forbid hipMalloc):
 * iga_mf_apply with the product's intermediate arrays taken from a static
 * device array the library holds for the life of the process (16 MiB per
 * device, one copy per device; its address is looked up when the first plan
 * is created on the device) instead of the plan's workspace. Allocates
 * nothing. Same arguments, kernels and result as iga_mf_apply.
 * IGA_E_CAPACITY (nothing enqueued) when the patch needs more than 16 MiB of
 * intermediate arrays: 8 (2 nband p n1 + (n_band_el + n_cut_el)(p+1)^2)
 * bytes with nband = max(1, floor(N2 / max(8, p+1))), each part rounded up
 * to 256 bytes (about 1150^2 elements at p = 4 with a 16-point cubic hole).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (several streams or threads) race and must be ordered by the
 * caller. */
int iga_mf_apply_noalloc(iga_plan* plan, const double* c_points, const double* u, double* y, void* stream);

/* Adjoint of iga_mf_apply (the transpose of Eq. (7)'s product and its
 * derivative in c): for a cotangent gy (n_act), du = M(c)^T gy
 * (n_act) and dc[k] = (sum_j B_j(x_k) u_j) (sum_i w_hat_{k,i} gy_i)
 * (n_points), w_hat_{k,i} being row i's test-side weight at point k. The
 * first call on a plan lists, on the host, the rows that receive element
 * vectors (it synchronises the stream once and keeps the list). */
int iga_mf_adjoint(iga_plan* plan, const double* c_points, const double* u, const double* gy,
                   double* du, double* dc, void* stream);

/* Batched formation of many patches (each patch's rules as in Sects. 2-3):
 * the resident tables of count plans (set up, each plan with its own degree
 * <= 6, method hybrid Gauss, element Gauss or DWQ) are formed into vals[k]
 * (device, band_k * n_act_k doubles) with coefficient cs[k]. The uneven
 * work, the cut-element matrices of all patches (node counts differ), is one
 * persistent launch (plus a counter reset): a cost-sorted work queue per
 * degree taken by a fixed grid of workgroups -- or, when the autotuner
 * measures it faster, one launch per degree of one workgroup per element. Beside it, on a second stream,
 * the coefficient chunks and then the interior tiles run in one launch per
 * degree; once the persistent launch and the coefficient chunks are done,
 * the element-formed rows run in one launch per degree (one workgroup per
 * row). DWQ plans (coefficient constant or |det J|) also have their side
 * rules (Sect. 3.3: the refined minimum-norm solves of every interior knot
 * and side) solved again, every DWQ patch of a degree in one launch before
 * the cut elements, and their rows' box parts added after the
 * element-formed rows. The values equal the one-patch formation's bit for
 * bit.
 *
 * A batch object keeps the descriptors, the queue and, with use_graph != 0,
 * a HIP graph recorded on the first such call and replayed afterwards. The
 * plans, coefficient data and output buffers are borrowed: they must stay
 * valid and keep their addresses while the batch lives. Calls on one batch
 * must not overlap (they share its counters). iga_batch_create checks every
 * plan and buffer pointer, degree and method before it touches the device:
 * IGA_E_INVALID (count <= 0, a null array, plan or buffer),
 * IGA_E_UNSUPPORTED (degree above 6, naive WQ), IGA_E_NOMEM, IGA_E_HIP;
 * *out is NULL after a failure. */
typedef struct iga_batch iga_batch;
typedef struct iga_batch_stats {
    int64_t n_plans;
    int64_t n_items;      /* work items: queued ones and those of the other launches */
    int64_t nnz;          /* sum of the plans' structural non-zeros     */
    int32_t grid;         /* persistent workgroups; 0: the autotuner chose one workgroup per
                             cut element (per-degree launches) over the persistent queue */
    int32_t wg_per_cu;    /* workgroups per compute unit (autotuned)    */
    int32_t order;        /* 0: cost-sorted queue, 1: patch by patch    */
    int32_t graph_ready;  /* a recorded graph is cached                 */
    int32_t chunk;        /* queue items reserved per atomic (autotuned) */
    int32_t capped;       /* 1: kernel built for 256 registers (two workgroups per CU), 0: for one
                             workgroup per CU (autotuned) */
} iga_batch_stats;
int iga_batch_create(iga_plan* const* plans, int32_t count, const iga_coeff* cs, double* const* vals,
                     iga_batch** out);
void iga_batch_destroy(iga_batch* batch);
/* Enqueues the batched formation on stream (graph replay with use_graph). */
int iga_batch_form(iga_batch* batch, int32_t use_graph, void* stream);
/* Autotuner: times the persistent grid (1, 2, 4, 8, 12 or 16 workgroups per
 * compute unit, more than fit at once allowed), the kernel's register budget (two
 * builds), the queue chunk (4, 16, 64 items per atomic) and the two queue
 * orders on the device (3 timed runs each, stream synchronised), and against
 * them the cut element matrices launched one workgroup each per degree
 * instead of the persistent queue; keeps the fastest and drops a cached
 * graph; *best_ms (may be NULL) receives its time. */
int iga_batch_autotune(iga_batch* batch, void* stream, float* best_ms);
int iga_batch_info(const iga_batch* batch, iga_batch_stats* st);
/* Synchronises stream; IGA_E_INVALID if a dependency wait hit its bound
 * (the bound is sticky for the batch), else the first plan's device status. */
int iga_batch_status(iga_batch* batch, void* stream);
/* Batched L2 projection (Sect. 4.2) of the batch's patches, after
 * iga_batch_form: for every patch k, the right-hand side by its rows' own
 * rules applied to gs[k] c_k (c_k the batch's coefficient of the patch), then
 * Jacobi-preconditioned CG on (M_k + M_k^T)/2 with M_k the batch's output
 * vals[k] -- every patch in the same launches, each with its own step sizes
 * and its own convergence test ||b_k - A_k u_k|| <= rtol ||b_k||, taken every
 * 16 iterations and at maxit as in iga_trim_l2_project, so each patch's
 * iterates and iteration count are those of the one-patch call. u[k]
 * (device, n_act_k doubles, caller owned) is the start vector and receives
 * the solution; infos (host, count entries, may be NULL) receives each
 * patch's iterations, convergence flag and relative residual. Degrees up to
 * 6; hybrid Gauss, DWQ or element Gauss plans, with the right-hand side rules
 * and restrictions of iga_trim_l2_project. The first call takes device memory
 * for the batch's symmetrised bands and vectors (kept until the batch is
 * destroyed). Synchronous. IGA_E_NOCONV if some patch did not converge
 * within maxit (its u is the last iterate). */
int iga_batch_project(iga_batch* batch, const iga_target* gs, double rtol, int32_t maxit, double* const* u,
                      iga_solve_info* infos, void* stream);
/* One-shot form: create a batch, form (graph if use_graph), synchronise, destroy. */
int iga_trim_mass_form_batched(iga_plan* const* plans, int32_t count, const iga_coeff* cs,
                               double* const* vals, int32_t use_graph, void* stream);

/* Per-phase device timing of the plan's calls (hipEvents on the streams the
 * phases run on). enable = 1 starts recording (2: per-kernel timing instead,
 * below; 0: off); iga_plan_timings synchronises and returns the accumulated
 * milliseconds and counts per phase. While phase timing is on, the interior
 * rows kernel runs alone (the two streams join before and after it), so
 * IGA_PHASE_INTERIOR is that kernel's own duration. */
#define IGA_PHASE_SETUP     0  /* layout, weights, trimming, cut rules        */
#define IGA_PHASE_COEF      1  /* coefficient at rule points                  */
#define IGA_PHASE_INTERIOR  2  /* interior rows kernel, start to end of its run */
#define IGA_PHASE_CUT       3  /* cut-element matrices and cut rows           */
#define IGA_PHASE_COUNT     4
int iga_plan_set_timing(iga_plan* plan, int32_t enable);
int iga_plan_timings(iga_plan* plan, double* ms, int64_t* counts);

/* Per-kernel timing: after iga_plan_set_timing(plan, 2), every kernel of the
 * plan's formations (launched kernel by kernel) is dispatched with events
 * recorded at the start and end of its execution on the stream it runs on.
 * iga_plan_kernel_times synchronises and returns, per kernel name, the summed
 * milliseconds and dispatch count since the last call (up to cap entries in
 * out, in order of first dispatch; *n receives the number of kernels), then
 * clears them. Durations of kernels that share the GPU with the other
 * stream's kernels include that contention. */
typedef struct iga_kernel_time {
    char name[48];
    double ms;
    int64_t count;
} iga_kernel_time;
int iga_plan_kernel_times(iga_plan* plan, iga_kernel_time* out, int32_t cap, int32_t* n);

/* Read-only device views of the plan's tables (valid while the plan lives),
 * for inspection and parity checks:
 *   IGA_TABLE_WQ_POINTS   direction dir: q_dir point coordinates
 *   IGA_TABLE_WQ_WEIGHTS  direction dir: n_dir rows of `stride` weights; row i
 *                         holds w_{k,i} (Eq. (5)) for the points k = k0(i)+q of
 *                         supp B_i, k0(i) = first point of element max(0, i-p)
 *   IGA_TABLE_MASS_1D     direction dir: n_dir rows of 2p+1, int B_i B_{i+d-p}
 *   IGA_TABLE_C_WQ / C_BAND / C_CUT: c at the WQ grid, band Gauss points and
 *                         cut nodes from the last IGA_COEF_GEOM_DETJ formation
 *   IGA_TABLE_CUT_W       weights of the cut-element nodes
 *   IGA_TABLE_DWQ_X       method IGA_DWQ, direction dir: for each interior knot
 *                         t = bp[s] (s = 1..N-1) and side (slot 2(s-1)+side,
 *                         side 0 below t, 1 above), `stride` point coordinates
 *                         in increasing order (IGA_ITABLE_DWQ_NPTS of them used)
 *   IGA_TABLE_DWQ_W       method IGA_DWQ, direction dir: per slot, p rows of
 *                         `stride` weights; row ii holds the discontinuous rule
 *                         of B_{s+ii} (Sect. 3.3) on the slot's points
 * *count receives the number of doubles, *stride the row length (or 1). */
#define IGA_TABLE_WQ_POINTS   0
#define IGA_TABLE_WQ_WEIGHTS  1
#define IGA_TABLE_MASS_1D     2
#define IGA_TABLE_C_WQ        3
#define IGA_TABLE_C_BAND      4
#define IGA_TABLE_C_CUT       5
#define IGA_TABLE_CUT_W       6
#define IGA_TABLE_DWQ_X       7
#define IGA_TABLE_DWQ_W       8
int iga_plan_table(const iga_plan* plan, int32_t table, int32_t dir, const double** ptr, int64_t* count,
                   int64_t* stride);

/* Read-only device views of the plan's integer tables (valid while the plan
 * lives; NULL with *count = 0 where the method has none):
 *   IGA_ITABLE_DWQ_NPTS   direction dir: points used in each DWQ slot
 *   IGA_ITABLE_DWQ_ELEM   direction dir: element of each DWQ slot point
 *   IGA_ITABLE_DWQ_WQIDX  direction dir: WQ point index of each DWQ slot point,
 *                         -1 for a point nested between them (Sect. 3.3)
 *   IGA_ITABLE_DWQ_BOX    per row formed element-wise (IGA_ITABLE_FORM_ROWS
 *                         order), 8 ints lo1, hi1, s1, side1, lo2, hi2, s2,
 *                         side2: the box of inside elements integrated with
 *                         the direction-d rule on elements lo_d..hi_d (s_d = -1:
 *                         the WQ rule of Eq. (5), else the discontinuous rule
 *                         of side side_d of knot s_d); lo1 = -1: no box, the
 *                         row is formed element-wise only
 *   IGA_ITABLE_FORM_ROWS  compact ids of the rows formed element-wise
 * dir is ignored by the last two. */
#define IGA_ITABLE_DWQ_NPTS   0
#define IGA_ITABLE_DWQ_ELEM   1
#define IGA_ITABLE_DWQ_WQIDX  2
#define IGA_ITABLE_DWQ_BOX    3
#define IGA_ITABLE_FORM_ROWS  4
int iga_plan_int_table(const iga_plan* plan, int32_t table, int32_t dir, const int32_t** ptr, int64_t* count,
                       int64_t* stride);

/* Replaces the weighted-quadrature weights of direction dir by W (device,
 * layout of IGA_TABLE_WQ_WEIGHTS), stream ordered. Later formations without
 * IGA_FORM_FULL use them; a FULL formation recomputes them. For checking the
 * formation kernels under rules fixed from outside. */
int iga_plan_set_weights(iga_plan* plan, int32_t dir, const double* W, void* stream);

/* Replaces the discontinuous weights of direction dir (method IGA_DWQ) by w
 * (device, layout of IGA_TABLE_DWQ_W), stream ordered; the point lists are
 * kept. Later formations without IGA_FORM_FULL use them; a FULL formation
 * recomputes them. For checking the formation kernels under rules fixed from
 * outside. IGA_E_INVALID if the plan's method is not IGA_DWQ. */
int iga_plan_set_dwq_weights(iga_plan* plan, int32_t dir, const double* w, void* stream);

/* Replaces the cut-element nodes (device arrays of n coordinates and weights,
 * in the order of iga_plan_points; n must equal n_cut_nodes, else
 * IGA_E_INVALID) and refreshes the point view.
 * Later formations, right-hand sides and matrix-free products without
 * IGA_FORM_FULL use them; a FULL formation rebuilds them. For checking the
 * kernels under rules fixed from outside. */
int iga_plan_set_cut_nodes(iga_plan* plan, const double* x, const double* y, const double* w, int64_t n,
                           void* stream);

/* Copies bytes between device (or host) buffers on stream and waits for it
 * (hipMemcpyAsync with hipMemcpyDefault, then a stream synchronisation); used
 * by bindings to read the plan's device views. */
int iga_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* Measured ceilings of the current device, the denominators beside the
 * datasheet peaks in roofline fractions: a streaming copy of n doubles from
 * src to dst (both device, n >= 256 x 8 x compute units; bytes read plus
 * written over the time), a loop of independent FP64 fused multiply-adds
 * (2 flops each) and a loop of FP64 matrix-core products (16x16x4 per
 * wavefront step); each the best of reps timed runs after a warm-up (HIP
 * events on stream, synchronised). dst is overwritten. */
typedef struct iga_peaks {
    double copy_gbs;        /* GB/s, read + write */
    double fma_tflops;      /* FP64 vector FMA, TFLOP/s */
    double mfma_f64_tflops; /* FP64 matrix core, TFLOP/s */
    int32_t n_cu;
    int32_t reserved;
} iga_peaks;
int iga_measure_peaks(const double* src, double* dst, int64_t n, int32_t reps, iga_peaks* out, void* stream);

/* For test builds of the library (compiled with -DIGA_DEBUG_BOUNDS), not a
 * paper operation: every store into the band layout vals[slot * n_act + row]
 * and into the per-row scratch arrays checks its slot and row; an offset out
 * of range is counted and redirected to the array's first element, so no
 * store leaves the array. *hits (host) receives the count over all modules
 * since the last reset (the device is synchronised first); reset != 0 clears
 * it. A release build has no checks: IGA_E_UNSUPPORTED, *hits = 0. */
int iga_debug_bounds_hits(int64_t* hits, int32_t reset);

const char* iga_status_string(int code);
const char* iga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGA_TRIM_H */
