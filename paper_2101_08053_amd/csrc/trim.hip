// Trimmed parameter space on the device (Sects. 2.2, 3 and 3.1).
//
//  * The trimming curves are cut into pieces that are monotone in x and y
//    (split at segment junctions and at the zeros of X' and Y'); for a union
//    of holes the pieces are also split where they meet another curve.
//  * Each piece is cut at every grid line it crosses; the resulting arcs lie
//    in one element each. An arc belongs to the visible boundary if its
//    midpoint is inside the unit square and outside every other hole.
//  * Elements owning a kept arc are cut; the others are inside or outside by
//    a test at their centre. Functions are exterior / interior / cut by the
//    classes of their support elements (Sect. 2.2).
//  * Each cut element gets a Gauss-Green rule on the exact boundary of its
//    visible part (the cut-element rule of Sect. 3.1): arcs give
//    n_q x n_r nodes, the visible pieces of the edge opposite the chosen base
//    give a tensor rule; of the four bases the one with the least sum |w| is
//    taken. Node order: arcs by (curve, segment, t), q outer, r inner; then
//    edge pieces by increasing coordinate, s outer, r inner.
#include "plan.hpp"

namespace iga {

// ------------------------------------------------------------ evaluation
// A point and tangent of a curve.
struct CurvePt {
    double X, Y, dX, dY;
};

// Ellipse branch out of line: its sine and cosine are large, and the trimming
// kernels run few waves each, so instruction fetch rather than arithmetic
// bounds them. Arguments and result travel in registers.
__device__ __attribute__((noinline)) CurvePt ellipse_eval(double x0, double x1, double x2, double y0, double y1,
                                                          double y2, double t) {
    double s, c;
    sincos(t, &s, &c);
    return CurvePt{x0 + x1 * c + x2 * s, y0 + y1 * c + y2 * s, -x1 * s + x2 * c, -y1 * s + y2 * c};
}

__device__ __forceinline__ void seg_eval(const SegDev& S, double t, double& X, double& Y, double& dX, double& dY) {
    if (S.kind == IGA_CURVE_ELLIPSE) {
        const CurvePt q = ellipse_eval(S.px[0], S.px[1], S.px[2], S.py[0], S.py[1], S.py[2], t);
        X = q.X;
        Y = q.Y;
        dX = q.dX;
        dY = q.dY;
    } else {
        X = ((S.px[3] * t + S.px[2]) * t + S.px[1]) * t + S.px[0];
        Y = ((S.py[3] * t + S.py[2]) * t + S.py[1]) * t + S.py[0];
        dX = (3.0 * S.px[3] * t + 2.0 * S.px[2]) * t + S.px[1];
        dY = (3.0 * S.py[3] * t + 2.0 * S.py[2]) * t + S.py[1];
    }
}

__device__ __forceinline__ double seg_coord(const SegDev& S, double t, int axis, double& deriv) {
    double X, Y, dX, dY;
    seg_eval(S, t, X, Y, dX, dY);
    deriv = axis ? dY : dX;
    return axis ? Y : X;
}

// Root of coord_axis(t) = v on a monotone piece [a, b]: bracketed Newton with bisection fallback.
__device__ double solve_monotone(const SegDev& S, int axis, double v, double a, double b) {
    double d;
    double fa = seg_coord(S, a, axis, d) - v;
    double fb = seg_coord(S, b, axis, d) - v;
    if (fa == 0.0) return a;
    if (fb == 0.0) return b;
    if ((fa < 0.0) == (fb < 0.0)) return (fabs(fa) < fabs(fb)) ? a : b;
    if (fa > 0.0) {  // orient so that f(lo) < 0 < f(hi)
        double t = a; a = b; b = t;
    }
    double t = 0.5 * (a + b);
    for (int it = 0; it < 200; ++it) {
        double ft = seg_coord(S, t, axis, d) - v;
        if (ft == 0.0) return t;
        if (ft < 0.0) a = t; else b = t;
        double tn = t - ft / d;
        double lo = fmin(a, b), hi = fmax(a, b);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (a + b);
        if (tn == t || fabs(b - a) <= 4e-16 * fmax(fabs(a), fabs(b))) return tn;
        t = tn;
    }
    return t;
}

__device__ __forceinline__ double ellipse_implicit(const CurveDev& C, double x, double y) {
    double cph = cos(C.phi), sph = sin(C.phi);
    double dx = x - C.cx, dy = y - C.cy;
    double u = (cph * dx + sph * dy) / C.a;
    double w = (-sph * dx + cph * dy) / C.b;
    return u * u + w * w - 1.0;
}

// Even-odd ray test (+x direction) of point (x, y) against curve c.
__device__ bool inside_curve(const TrimDev& T, int c, double x, double y) {
    const CurveDev C = T.curves[c];
    if (C.kind == IGA_CURVE_ELLIPSE) return ellipse_implicit(C, x, y) < 0.0;
    int lo = T.piece_curve_off[c], hi = T.piece_curve_off[c + 1];
    bool in = false;
    for (int k = lo; k < hi; ++k) {
        const PieceDev Pc = T.pieces[k];
        double ymin = fmin(Pc.y0, Pc.y1), ymax = fmax(Pc.y0, Pc.y1);
        if (!(y >= ymin && y < ymax)) continue;
        if (fmax(Pc.x0, Pc.x1) <= x) continue;  // entirely left of the point
        double t = solve_monotone(T.segs[Pc.seg], 1, y, Pc.t0, Pc.t1);
        double X, Y, dX, dY;
        seg_eval(T.segs[Pc.seg], t, X, Y, dX, dY);
        if (X > x) in = !in;
    }
    return in;
}

__device__ bool in_any_hole(const TrimDev& T, double x, double y, int skip = -1) {
    for (int c = 0; c < T.n_curves; ++c)
        if (c != skip && inside_curve(T, c, x, y)) return true;
    return false;
}

__device__ __forceinline__ int upper_bound_d(const double* a, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int lower_bound_d(const double* a, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int upper_bound_i(const int* a, int n, int v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Branch-free lower / upper bound of K values at once (first index with
// a[i] >= v, resp. a[i] > v; n >= 1): the trip count depends on n only, so
// the K searches' loads overlap.
template <int K>
__device__ __forceinline__ void lower_bound_k(const double* a, int n, const double* v, int* r) {
    int base[K];
#pragma unroll
    for (int k = 0; k < K; ++k) base[k] = 0;
    for (int len = n; len > 1;) {
        const int half = len >> 1;
#pragma unroll
        for (int k = 0; k < K; ++k) base[k] = (a[base[k] + half] < v[k]) ? base[k] + half : base[k];
        len -= half;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = base[k] + (a[base[k]] < v[k]);
}

template <int K>
__device__ __forceinline__ void upper_bound_k(const double* a, int n, const double* v, int* r) {
    int base[K];
#pragma unroll
    for (int k = 0; k < K; ++k) base[k] = 0;
    for (int len = n; len > 1;) {
        const int half = len >> 1;
#pragma unroll
        for (int k = 0; k < K; ++k) base[k] = (a[base[k] + half] <= v[k]) ? base[k] + half : base[k];
        len -= half;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = base[k] + (a[base[k]] <= v[k]);
}

// ---------------------------------------------------------- segments
// Uniform B-spline blending polynomials (power basis, low first) of degree 1..3:
// rows are the functions, columns the powers.
__constant__ double kBlend1[2][2] = {{1, -1}, {0, 1}};
__constant__ double kBlend2[3][3] = {{0.5, -1, 0.5}, {0.5, 1, -1}, {0, 0, 0.5}};
__constant__ double kBlend3[4][4] = {{1.0 / 6, -0.5, 0.5, -1.0 / 6},
                                     {4.0 / 6, 0, -1, 0.5},
                                     {1.0 / 6, 0.5, 0.5, -0.5},
                                     {0, 0, 0, 1.0 / 6}};
__device__ __forceinline__ double blend(int d, int l, int pw) {
    if (d == 1) return kBlend1[l][pw];
    if (d == 2) return kBlend2[l][pw];
    return kBlend3[l][pw];
}

// Segment s (of curve c) in power form.
__device__ SegDev segment_form(const CurveDev& C, int c, const double* __restrict__ cp, const int* __restrict__ cp_off,
                               int s) {
    SegDev S;
    S.curve = c;
    S.seg = s - C.seg0;
    S.kind = C.kind;
    S.pad = 0;
    for (int k = 0; k < 4; ++k) S.px[k] = S.py[k] = 0.0;
    if (C.kind == IGA_CURVE_ELLIPSE) {
        const CurvePt q = ellipse_eval(0.0, 1.0, 0.0, 0.0, 0.0, 1.0, C.phi);  // (cos phi, sin phi)
        const double cph = q.X, sph = q.Y;
        S.px[0] = C.cx; S.px[1] = C.a * cph; S.px[2] = -C.b * sph;
        S.py[0] = C.cy; S.py[1] = C.a * sph; S.py[2] = C.b * cph;
    } else {
        // fixed trip counts (degree <= 3), so the coefficients stay in registers
        const int d = C.degree, m = C.n_seg, o = cp_off[c];
#pragma unroll
        for (int l = 0; l <= 3; ++l) {
            if (l > d) continue;
            const int idx = (S.seg + l) % m;
            const double x = cp[2 * (o + idx)], y = cp[2 * (o + idx) + 1];
#pragma unroll
            for (int pw = 0; pw <= 3; ++pw) {
                if (pw > d) continue;
                S.px[pw] += blend(d, l, pw) * x;
                S.py[pw] += blend(d, l, pw) * y;
            }
        }
    }
    return S;
}

__device__ void segment_make(const TrimDev& T, const double* __restrict__ cp, const int* __restrict__ cp_off, int s) {
    int c = 0;
    while (c + 1 < T.n_curves && T.curves[c + 1].seg0 <= s) ++c;
    T.segs[s] = segment_form(T.curves[c], c, cp, cp_off, s);
}

// Zeros of a + b t + c t^2 in (lo, hi), ascending, +inf where absent.
__device__ __forceinline__ void quad_roots(double a, double b, double c, double lo, double hi, double& r0, double& r1) {
    const double inf = __builtin_inf();
    r0 = r1 = inf;
    double scale = fabs(a) + fabs(b) + fabs(c);
    if (scale == 0.0) return;
    if (fabs(c) <= 1e-14 * scale) {
        if (fabs(b) > 1e-14 * scale) {
            double t = -a / b;
            if (t > lo && t < hi) r0 = t;
        }
        return;
    }
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return;
    double q = -0.5 * (b + copysign(sqrt(disc), b));
    double t1 = q / c, t2 = (q != 0.0) ? a / q : t1;
    if (t1 > t2) { double t = t1; t1 = t2; t2 = t; }
    if (t1 > lo && t1 < hi) r0 = t1;
    if (t2 > lo && t2 < hi && t2 != t1) r1 = t2;
}

// Zeros of X' and Y' of an ellipse segment in (0, hi) (+inf where outside), out of line.
__device__ __attribute__((noinline)) CurvePt ellipse_splits(double x1, double x2, double y1, double y2, double hi) {
    const double tp = 2.0 * M_PI, lo = 0.0, inf = __builtin_inf();
    const double c[4] = {atan2(x2, x1), atan2(x2, x1) + M_PI, atan2(y2, y1), atan2(y2, y1) + M_PI};
    double r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double t = fmod(c[k], tp);
        if (t < 0.0) t += tp;
        r[k] = (t > lo && t < hi) ? t : inf;
    }
    return CurvePt{r[0], r[1], r[2], r[3]};
}

__device__ __forceinline__ void sort2(double& a, double& b) {
    const double lo = fmin(a, b), hi = fmax(a, b);
    a = lo;
    b = hi;
}

// Interior split parameters of a segment (the zeros of X' and Y' in (0, hi)),
// ascending, +inf where absent. The monotone pieces run between 0, every
// split above the last one used, and hi.
__device__ __forceinline__ void segment_splits(const SegDev& S, double hi, double r[4]) {
    const double lo = 0.0, inf = __builtin_inf();
    if (S.kind == IGA_CURVE_ELLIPSE) {
        const CurvePt q = ellipse_splits(S.px[1], S.px[2], S.py[1], S.py[2], hi);
        r[0] = q.X;
        r[1] = q.Y;
        r[2] = q.dX;
        r[3] = q.dY;
    } else {
        quad_roots(S.px[1], 2.0 * S.px[2], 3.0 * S.px[3], lo, hi, r[0], r[1]);
        quad_roots(S.py[1], 2.0 * S.py[2], 3.0 * S.py[3], lo, hi, r[2], r[3]);
    }
    sort2(r[0], r[1]);
    sort2(r[2], r[3]);
    sort2(r[0], r[2]);
    sort2(r[1], r[3]);
    sort2(r[1], r[2]);
}

// Monotone pieces of a segment: candidate k of {r[0..3], hi} closes a piece
// if it is below hi (or is hi itself) and above the last bound used. Fixed
// slots, so the arrays stay in registers.
struct SegPieces {
    double t0[5], t1[5];
    bool use[5];
    int n;
};

__device__ __forceinline__ SegPieces segment_pieces(double hi, const double r[4]) {
    SegPieces P;
    double last = 0.0;
    P.n = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double nxt = (k < 4) ? r[k] : hi;
        const bool use = (k < 4) ? (nxt < hi && nxt > last) : true;
        P.use[k] = use;
        P.t0[k] = last;
        P.t1[k] = nxt;
        if (use) {
            last = nxt;
            ++P.n;
        }
    }
    return P;
}

__device__ __forceinline__ PieceDev make_piece(const SegDev& S, int s, double t0, double t1) {
    PieceDev Pc;
    Pc.curve = S.curve;
    Pc.seg = s;
    Pc.pad0 = Pc.pad1 = 0;
    Pc.t0 = t0;
    Pc.t1 = t1;
    double dX, dY;
    seg_eval(S, t0, Pc.x0, Pc.y0, dX, dY);
    seg_eval(S, t1, Pc.x1, Pc.y1, dX, dY);
    return Pc;
}

__device__ int block_scan_carry(int v, int* sh, int& total);

// Single block: monotone pieces of every segment (already in T.segs),
// compacted in segment order.
__device__ void pieces_build(const TrimDev& T, PieceDev* __restrict__ out, int* __restrict__ count,
                             int* __restrict__ curve_off) {
    __shared__ int sh[1024 / 64 + 1];
    int carry = 0;
    for (int base = 0; base < T.n_segs; base += blockDim.x) {
        const int s = base + threadIdx.x;
        SegDev S;
        SegPieces sp;
        sp.n = 0;
        if (s < T.n_segs) {
            S = T.segs[s];
            double r[4];
            const double hi = T.curves[S.curve].t_range;
            segment_splits(S, hi, r);
            sp = segment_pieces(hi, r);
        }
        int total;
        const int off = block_scan_carry(sp.n, sh, total) + carry;
        if (s < T.n_segs) {
            int q = 0;
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (sp.use[k]) out[off + q++] = make_piece(S, s, sp.t0[k], sp.t1[k]);
            if (S.seg == 0) curve_off[S.curve] = off;
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        *count = carry;
        curve_off[T.n_curves] = carry;
    }
}

__device__ int block_scan_carry(int v, int* sh, int& total) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int nw = blockDim.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int t = (lane < nw) ? sh[lane] : 0, ti = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int u = __shfl_up(ti, o, 64);
            if (lane >= o) ti += u;
        }
        if (lane < nw) sh[lane] = ti - t;
        if (lane == nw - 1) sh[nw] = ti;
    }
    __syncthreads();
    int res = inc - v + sh[wid];
    total = sh[nw];
    __syncthreads();
    return res;
}

// Union of holes: where does piece k (of pieces0) meet another curve? One
// wavefront per piece samples the other ellipse's implicit function at 257
// points and refines each sign change by bisection.
__global__ void __launch_bounds__(64) k_piece_isect(TrimDev T, int* __restrict__ status) {
    int k = blockIdx.x;
    if (k >= *T.n_pieces0) return;
    const PieceDev Pc = T.pieces0[k];
    const SegDev S = T.segs[Pc.seg];
    int lane = threadIdx.x;
    double found[kMaxIsectPerPiece];
    int nf = 0;
    for (int o = 0; o < T.n_curves; ++o) {
        if (o == Pc.curve) continue;
        const CurveDev C = T.curves[o];
        double rx = sqrt(C.a * C.a * cos(C.phi) * cos(C.phi) + C.b * C.b * sin(C.phi) * sin(C.phi));
        double ry = sqrt(C.a * C.a * sin(C.phi) * sin(C.phi) + C.b * C.b * cos(C.phi) * cos(C.phi));
        if (fmax(Pc.x0, Pc.x1) < C.cx - rx || fmin(Pc.x0, Pc.x1) > C.cx + rx) continue;
        if (fmax(Pc.y0, Pc.y1) < C.cy - ry || fmin(Pc.y0, Pc.y1) > C.cy + ry) continue;
        // samples j = 4 lane + q, q = 0..3, plus j = 256 from lane 63
        double g[5];
        for (int q = 0; q < 5; ++q) {
            int j = 4 * lane + q;
            double t = Pc.t0 + (Pc.t1 - Pc.t0) * (double)j / 256.0;
            double X, Y, dX, dY;
            seg_eval(S, t, X, Y, dX, dY);
            g[q] = ellipse_implicit(C, X, Y);
        }
        for (int q = 0; q < 4; ++q) {
            int j = 4 * lane + q;
            bool change = (g[q] < 0.0) != (g[q + 1] < 0.0);
            unsigned long long m = __ballot(change);
            // process sign changes in ascending j across the wave
            while (m) {
                int src = __ffsll((long long)m) - 1;
                m &= m - 1;
                int js = __shfl(j, src, 64);
                double ga = __shfl(g[q], src, 64);
                double a = Pc.t0 + (Pc.t1 - Pc.t0) * (double)js / 256.0;
                double b = Pc.t0 + (Pc.t1 - Pc.t0) * (double)(js + 1) / 256.0;
                // 64-section: lane l tests a + (b - a)(l + 1)/64; the bracket becomes the first
                // sub-interval whose right end has changed sign (about 9 rounds to adjacent doubles)
                for (int it = 0; it < 24; ++it) {
                    const double tl = (lane == 63) ? b : a + (b - a) * (double)(lane + 1) / 64.0;
                    double X, Y, dX, dY;
                    seg_eval(S, tl, X, Y, dX, dY);
                    const bool flip = (ellipse_implicit(C, X, Y) < 0.0) != (ga < 0.0);
                    const unsigned long long fm = __ballot(flip && tl > a);
                    const int l = fm ? __ffsll((long long)fm) - 1 : 63;
                    const double nb = __shfl(tl, l, 64);
                    const double na = (l == 0) ? a : __shfl(tl, max(l - 1, 0), 64);
                    const bool done = !(na > a || nb < b);  // no progress: a and b are adjacent
                    a = na;
                    b = nb;
                    if (done) break;
                }
                if (nf < kMaxIsectPerPiece) found[nf] = 0.5 * (a + b);
                ++nf;
            }
        }
    }
    if (lane == 0) {
        if (nf > kMaxIsectPerPiece) {
            atomicExch(status, IGA_E_TOPOLOGY);
            nf = kMaxIsectPerPiece;
        }
        for (int a = 1; a < nf; ++a) {
            double v = found[a];
            int b = a - 1;
            while (b >= 0 && found[b] > v) { found[b + 1] = found[b]; --b; }
            found[b + 1] = v;
        }
        for (int q = 0; q < nf; ++q) T.isect_t[k * kMaxIsectPerPiece + q] = found[q];
        T.isect_n[k] = nf;
    }
}

__device__ void pieces_split(const TrimDev& T) {
    __shared__ int sh[1024 / 64 + 1];
    int carry = 0;
    int n0 = *T.n_pieces0;
    for (int base = 0; base < n0; base += blockDim.x) {
        int k = base + threadIdx.x;
        int ns = (k < n0) ? T.isect_n[k] + 1 : 0;
        int total;
        int off = block_scan_carry(ns, sh, total) + carry;
        if (k < n0) {
            const PieceDev Pc = T.pieces0[k];
            const SegDev S = T.segs[Pc.seg];
            double a = Pc.t0;
            for (int q = 0; q < ns; ++q) {
                double b = (q == ns - 1) ? Pc.t1 : T.isect_t[k * kMaxIsectPerPiece + q];
                T.pieces[off + q] = make_piece(S, Pc.seg, a, b);
                a = b;
            }
            if (k == 0 || T.pieces0[k - 1].curve != Pc.curve) T.piece_curve_off[Pc.curve] = off;
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        *T.n_pieces = carry;
        T.piece_curve_off[T.n_curves] = carry;
    }
}

// ------------------------------------------------------------ crossings
struct GridDev {
    const double* bp1;
    const double* bp2;
    int N1, N2;
};

// Breakpoints of both directions, staged in LDS by the single-workgroup and
// per-piece kernels when they fit (the global arrays otherwise).
constexpr int kLdsBp = 4096;
struct BpView {
    const double* b1;
    const double* b2;
};

__device__ __forceinline__ BpView stage_bp(const GridDev& G, double* sbp) {
    const int n1 = G.N1 + 1, n2 = G.N2 + 1;
    if (n1 + n2 > kLdsBp) return {G.bp1, G.bp2};
    for (int i = threadIdx.x; i < n1 + n2; i += blockDim.x) sbp[i] = (i < n1) ? G.bp1[i] : G.bp2[i - n1];
    return {sbp, sbp + n1};  // the caller synchronises before use
}

// Union of holes (one workgroup, after the curve-curve splits):
// orientation of every curve (sign of its enclosed area by Gauss on each
// segment; a hole traversed with the visible domain on its left is
// clockwise).
__device__ void curves_orient(const TrimDev& T, CurveDev* __restrict__ curves, const double* __restrict__ gx,
                              const double* __restrict__ gw) {
    __shared__ double sh_area[1024 / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nt = blockDim.x;
    constexpr int ng = 8;
    for (int c = 0; c < T.n_curves; ++c) {
        const CurveDev C = curves[c];
        double area = 0.0;
        for (int u = tid; u < C.n_seg * ng; u += nt) {
            const SegDev S = T.segs[C.seg0 + u / ng];
            const int g = u % ng;
            const double tt = C.t_range * (gx[gauss_off(ng) + g] + 1.0) * 0.5;
            const double w = gw[gauss_off(ng) + g] * C.t_range * 0.5;
            double X, Y, dX, dY;
            seg_eval(S, tt, X, Y, dX, dY);
            area += 0.5 * w * (X * dY - Y * dX);
        }
        area = wave_sum(area);
        if (lane == 0) sh_area[wid] = area;
        __syncthreads();
        if (tid == 0) {
            double a = 0.0;
            for (int w = 0; w < nt / 64; ++w) a += sh_area[w];
            curves[c].sigma = (a > 0.0) ? -1.0 : 1.0;
        }
        __syncthreads();
    }
}

// One curve, one workgroup: each thread forms its segment and splits it into
// monotone pieces, in registers; a block scan places the pieces. The
// segment's 8-point Gauss share of the enclosed area gives the orientation.
__device__ void front_one_curve(const TrimDev& T, const double* __restrict__ cp, const int* __restrict__ cp_off,
                                CurveDev* __restrict__ curves, const double* __restrict__ gx,
                                const double* __restrict__ gw) {
    __shared__ int sh[1024 / 64 + 1];
    __shared__ double sh_area[1024 / 64];
    constexpr int ng = 8;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nt = blockDim.x;
    const CurveDev C = curves[0];
    double gxv[ng], gwv[ng];
#pragma unroll
    for (int g = 0; g < ng; ++g) {
        gxv[g] = gx[gauss_off(ng) + g];
        gwv[g] = gw[gauss_off(ng) + g];
    }
    int carry_p = 0;
    double area = 0.0;
    for (int base = 0; base < T.n_segs; base += nt) {
        const int s = base + tid;
        const bool valid = s < T.n_segs;
        SegDev S;
        SegPieces sp;
        sp.n = 0;
        if (valid) {
            S = segment_form(C, 0, cp, cp_off, s);
            T.segs[s] = S;
            double r[4];
            segment_splits(S, C.t_range, r);
            sp = segment_pieces(C.t_range, r);
#pragma unroll 1
            for (int g = 0; g < ng; ++g) {
                const double tt = C.t_range * (gxv[g] + 1.0) * 0.5;
                const double w = gwv[g] * C.t_range * 0.5;
                double X, Y, dX, dY;
                seg_eval(S, tt, X, Y, dX, dY);
                area += 0.5 * w * (X * dY - Y * dX);
            }
        }
        int tot_p;
        const int offp = block_scan_carry(sp.n, sh, tot_p) + carry_p;
        if (valid) {
            int q = offp;
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (sp.use[k]) T.pieces[q++] = make_piece(S, s, sp.t0[k], sp.t1[k]);
            if (S.seg == 0) T.piece_curve_off[0] = offp;
        }
        carry_p += tot_p;
    }
    area = wave_sum(area);
    if (lane == 0) sh_area[wid] = area;
    __syncthreads();
    if (tid == 0) {
        *T.n_pieces = carry_p;
        T.piece_curve_off[1] = carry_p;
        double a = 0.0;
        for (int w = 0; w < nt / 64; ++w) a += sh_area[w];
        curves[0].sigma = (a > 0.0) ? -1.0 : 1.0;
    }
}

// Front of the trimming set-up in one workgroup (256 threads). One curve:
// segments, pieces, orientation (front_one_curve). A union of holes:
// segments and the unsplit pieces only. Both clear the per-row centre-line
// crossing counts that the arc kernel fills.
__global__ void __launch_bounds__(256) k_trim_front(TrimDev T, const double* __restrict__ cp,
                                                     const int* __restrict__ cp_off, CurveDev* __restrict__ curves,
                                                     GridDev G, const double* __restrict__ gx,
                                                     const double* __restrict__ gw) {
    if (threadIdx.x == 0) *T.epoch += 1;  // a new set-up: marks and lists of earlier ones become stale
    for (int r = threadIdx.x; r < G.N2; r += blockDim.x) T.row_cnt[r] = 0;
    if (T.n_curves == 1) {
        front_one_curve(T, cp, cp_off, curves, gx, gw);
    } else {
        for (int s = threadIdx.x; s < T.n_segs; s += blockDim.x) segment_make(T, cp, cp_off, s);
        __syncthreads();
        pieces_build(T, T.pieces0, T.n_pieces0, T.piece_curve_off);
    }
}

// Union of holes: split the pieces where they meet another curve, then
// orientation. 256 threads: a workgroup that fits beside the other stream's
// kernels (a 1024-thread one waited for a whole free CU).
__global__ void __launch_bounds__(256) k_trim_split(TrimDev T, CurveDev* __restrict__ curves,
                                                     const double* __restrict__ gx, const double* __restrict__ gw) {
    pieces_split(T);
    __syncthreads();
    curves_orient(T, curves, gx, gw);
}

void launch_trim_curves(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    if (T.n_curves == 0) return;
    GridDev G{P.dir[0].knots + P.p, P.dir[1].knots + P.p, P.N1, P.N2};  // breakpoints
    klaunch(P, "k_trim_front", k_trim_front, dim3(1), dim3(256), 0, s, T, P.d_cp, P.d_cp_off, P.d_curves, G, P.gauss_x,
                       P.gauss_w);
    if (T.n_curves > 1) {
        klaunch(P, "k_piece_isect", k_piece_isect, dim3(T.cap_pieces0), dim3(64), 0, s, T, P.status);
        klaunch(P, "k_trim_split", k_trim_split, dim3(1), dim3(256), 0, s, T, P.d_curves, P.gauss_x, P.gauss_w);
    }
}

// One workgroup per piece: solve its crossings, order them along the piece
// (own rank plus the crossings of the other family before it, vertical first
// on ties), cut the piece into arcs, keep the visible ones and mark their
// elements cut (mark = this set-up's epoch) and push each kept arc onto its
// element's list (a head per element tagged with the epoch, so nothing is
// cleared between set-ups). Spline pieces also record where they cross the
// horizontal line through each row's element centres, for the centre test of
// the other elements. Breakpoints and (short pieces') crossings live in LDS.
constexpr int kArcLds = 512;

__global__ void __launch_bounds__(256) k_piece_arcs(TrimDev T, GridDev G, int* __restrict__ emark,
                                                    unsigned long long* __restrict__ ehead, int* __restrict__ arc_next,
                                                    int* __restrict__ status) {
    __shared__ double sbp[kLdsBp];
    __shared__ CrossDev sCross[kArcLds], sMerged[kArcLds];
    const int k = blockIdx.x;
    const int np = *T.n_pieces;
    const int tid = threadIdx.x;
    if (k >= np) return;
    const BpView bp = stage_bp(G, sbp);
    const int epoch = *T.epoch;
    const PieceDev Pc = T.pieces[k];
    const SegDev S = T.segs[Pc.seg];
    const CurveDev C = T.curves[Pc.curve];
    __syncthreads();
    // crossings with the vertical (then horizontal) grid lines in the piece's box, counted
    // half-open so that a crossing at a shared end belongs to one piece
    const double xmin = fmin(Pc.x0, Pc.x1), xmax = fmax(Pc.x0, Pc.x1);
    const double ymin = fmin(Pc.y0, Pc.y1), ymax = fmax(Pc.y0, Pc.y1);
    int lv[2], lh[2];
    {
        const double vx[2] = {xmin, xmax}, vy[2] = {ymin, ymax};
        lower_bound_k<2>(bp.b1, G.N1 + 1, vx, lv);
        lower_bound_k<2>(bp.b2, G.N2 + 1, vy, lh);
    }
    const int lv0 = lv[0], lh0 = lh[0], nv = lv[1] - lv[0], n = nv + (lh[1] - lh[0]);
    if (n + 1 > T.arc_slot) {  // more crossings than at plan creation: the geometry is not the plan's
        if (tid == 0) atomicExch(status, IGA_E_TOPOLOGY);
        return;
    }
    const int base = k * T.arc_slot;  // this piece's arcs are base + j, j = 0..n
    CrossDev* cross = (n <= kArcLds) ? sCross : T.cross + base;
    CrossDev* merged = (n <= kArcLds) ? sMerged : T.merged + base;
    // spline pieces: rows whose centre y lies in [ymin, ymax) (centres are non-decreasing in
    // the row): branch-free lower bounds of ymin and ymax over the row centres, in lockstep
    int r0 = 0, r1 = 0;
    if (C.kind != IGA_CURVE_ELLIPSE) {
        int b0 = 0, b1 = 0;
        for (int len = G.N2; len > 1;) {
            const int half = len >> 1;
            b0 = (0.5 * (bp.b2[b0 + half] + bp.b2[b0 + half + 1]) < ymin) ? b0 + half : b0;
            b1 = (0.5 * (bp.b2[b1 + half] + bp.b2[b1 + half + 1]) < ymax) ? b1 + half : b1;
            len -= half;
        }
        r0 = b0 + (0.5 * (bp.b2[b0] + bp.b2[b0 + 1]) < ymin);
        r1 = b1 + (0.5 * (bp.b2[b1] + bp.b2[b1 + 1]) < ymax);
    }
    // grid-line crossings (j < n) and centre-line crossings (j >= n) in one pass
    for (int j = tid; j < n + (r1 - r0); j += 256) {
        if (j < n) {
            CrossDev X;
            if (j < nv) {
                X.kind = END_VLINE;
                X.line = lv0 + j;
                X.t = solve_monotone(S, 0, bp.b1[X.line], Pc.t0, Pc.t1);
            } else {
                X.kind = END_HLINE;
                X.line = lh0 + (j - nv);
                X.t = solve_monotone(S, 1, bp.b2[X.line], Pc.t0, Pc.t1);
            }
            cross[j] = X;
        } else {
            const int r = r0 + (j - n);
            const double y = 0.5 * (bp.b2[r] + bp.b2[r + 1]);
            const double t = solve_monotone(S, 1, y, Pc.t0, Pc.t1);
            double X, Y, dX, dY;
            seg_eval(S, t, X, Y, dX, dY);
            const int slot = atomicAdd(&T.row_cnt[r], 1);
            if (slot < kRowCross) {
                T.row_key[(size_t)r * kRowCross + slot] = fmin(X, xmax);
                T.row_curve[(size_t)r * kRowCross + slot] = Pc.curve;
            }
        }
    }
    __syncthreads();
    const int nh = n - nv;
    const bool incx = Pc.x1 > Pc.x0, incy = Pc.y1 > Pc.y0;
    for (int j = tid; j < n; j += 256) {
        const CrossDev X = cross[j];
        int own, other;
        if (j < nv) {
            own = incx ? j : nv - 1 - j;
            int lo = 0, hi = nh;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int idx = incy ? mid : nh - 1 - mid;
                if (cross[nv + idx].t < X.t) lo = mid + 1; else hi = mid;
            }
            other = lo;
        } else {
            const int jh = j - nv;
            own = incy ? jh : nh - 1 - jh;
            int lo = 0, hi = nv;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int idx = incx ? mid : nv - 1 - mid;
                if (cross[idx].t <= X.t) lo = mid + 1; else hi = mid;
            }
            other = lo;
        }
        merged[own + other] = X;
    }
    __syncthreads();
    for (int j = tid; j <= n; j += 256) {
        ArcDev A;
        A.curve = Pc.curve;
        A.gseg = Pc.seg;
        A.piece = k;
        if (j == 0) { A.t0 = Pc.t0; A.k0 = END_PIECE; A.l0 = -1; }
        else { const CrossDev X = merged[j - 1]; A.t0 = X.t; A.k0 = X.kind; A.l0 = X.line; }
        if (j == n) { A.t1 = Pc.t1; A.k1 = END_PIECE; A.l1 = -1; }
        else { const CrossDev X = merged[j]; A.t1 = X.t; A.k1 = X.kind; A.l1 = X.line; }
        double X, Y, dX, dY;
        seg_eval(S, A.t0, A.x0, A.y0, dX, dY);
        seg_eval(S, A.t1, A.x1, A.y1, dX, dY);
        seg_eval(S, 0.5 * (A.t0 + A.t1), X, Y, dX, dY);
        int keep = (A.t1 - A.t0 > 1e-13 * C.t_range);
        keep = keep && X > bp.b1[0] && X < bp.b1[G.N1] && Y > bp.b2[0] && Y < bp.b2[G.N2];
        if (keep && T.n_curves > 1) keep = !in_any_hole(T, X, Y, Pc.curve);
        A.keep = keep;
        int u1, u2;
        upper_bound_k<1>(bp.b1, G.N1 + 1, &X, &u1);
        upper_bound_k<1>(bp.b2, G.N2 + 1, &Y, &u2);
        A.e1 = min(max(u1 - 1, 0), G.N1 - 1);
        A.e2 = min(max(u2 - 1, 0), G.N2 - 1);
        const int idx = base + j;
        T.arcs[idx] = A;
        if (keep) {  // push onto the element's list (order fixed later by arc index)
            const int e = A.e2 * G.N1 + A.e1;
            emark[e] = epoch;
            const unsigned long long old =
                atomicExch(&ehead[e], ((unsigned long long)(unsigned)epoch << 32) | (unsigned)(idx + 1));
            arc_next[idx] = ((int)(old >> 32) == epoch) ? (int)(old & 0xffffffffull) - 1 : -1;
        }
    }
}

// Plan creation: the largest number of grid-line crossings of one piece.
__global__ void k_piece_maxcross(TrimDev T, GridDev G, int* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *T.n_pieces) return;
    const PieceDev Pc = T.pieces[k];
    const double vx[2] = {fmin(Pc.x0, Pc.x1), fmax(Pc.x0, Pc.x1)}, vy[2] = {fmin(Pc.y0, Pc.y1), fmax(Pc.y0, Pc.y1)};
    int lv[2], lh[2];
    lower_bound_k<2>(G.bp1, G.N1 + 1, vx, lv);
    lower_bound_k<2>(G.bp2, G.N2 + 1, vy, lh);
    atomicMax(out, (lv[1] - lv[0]) + (lh[1] - lh[0]));
}

int trim_max_crossings(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    GridDev G{P.dir[0].knots + P.p, P.dir[1].knots + P.p, P.N1, P.N2};  // breakpoints
    HIPX(hipMemsetAsync(P.counts + 8, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_piece_maxcross, dim3((std::max(T.cap_pieces, 1) + 127) / 128), dim3(128), 0, s, T, G,
                       P.counts + 8);
    int m = 0;
    HIPX(hipMemcpyAsync(&m, P.counts + 8, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    return m;
}

void launch_trim_arcs(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    if (T.n_curves == 0) return;
    GridDev G{P.dir[0].knots + P.p, P.dir[1].knots + P.p, P.N1, P.N2};  // breakpoints
    klaunch(P, "k_piece_arcs", k_piece_arcs, dim3(std::max(T.cap_pieces, 1)), dim3(256), 0, s, T, G, P.emark, P.ehead,
                       P.arc_next, P.status);
}

// -------------------------------------------------------------- classes
// Element classes: cut if it owns a visible arc (marked with this set-up's
// epoch), otherwise inside / outside by the even-odd test at its centre. For
// spline curves the test counts the crossings the arc kernel recorded on the
// row's centre line right of the centre (a crossing counts when both it and
// its piece's largest x lie right of the point, as in inside_curve); ellipses
// use their implicit function. Rows with more crossings than recorded fall
// back to the direct test.
struct ClassArgs {
    int p, N1, N2, n1, n2, method;
    TrimDev T;
    GridDev G;
    const int* emark;
    int* rcnt;  // [4][n2][tiles along x]: flags set per row segment of a tile (f_active, f_cut, e_cut, e_band)
    int8_t* ecls;
    int8_t* fcls;
    int* f_active;   // n1*n2 flags
    int* f_cut;      // n1*n2 flags
    int* e_cut;      // N1*N2 flags
    int* e_band;     // N1*N2 flags
};

// Function classes and element flags on 16 x 16 tiles of elements. The
// tile's element classes with a halo of p on each side are found in LDS
// (each workgroup classifies its halo too, and writes its own elements');
// from them the classes of the functions [x0, x0 + 16 + p) x [y0, ...)
// (Sect. 2.2: exterior if every support element is outside, interior if
// every one is inside, cut otherwise), and from those the tile's element
// flags: cut, and "band" -- an inside element in the support of a cut
// function, whose Gauss points some row formed element-wise uses. The last
// tile of each direction also owns the p functions past the last element.
constexpr int kClsTile = 16;
constexpr int8_t kElPending = -2;  // element class still to be found by the direct test

__global__ void __launch_bounds__(256) k_classes(ClassArgs A) {
    constexpr int WE = kClsTile + 2 * IGA_MAXP, WF = kClsTile + IGA_MAXP;
    __shared__ int8_t sE[WE][WE];
    __shared__ int8_t sF[WF][WF];
    const int p = A.p, tid = threadIdx.x;
    const int x0 = blockIdx.x * kClsTile, y0 = blockIdx.y * kClsTile;
    const int we = kClsTile + 2 * p, wf = kClsTile + p;
    // the window's element centres and its rows' centre-line crossings, staged once
    __shared__ double sX[WE], sY[WE], sKey[WE][kRowCross];
    __shared__ int sCnt[WE];
    __shared__ int8_t sCur[WE][kRowCross];
    const TrimDev& T = A.T;
    const int epoch = *T.epoch;
    __shared__ int sRC[4][WF];  // flags set per row of this tile (functions: rows v; elements: rows ty)
    for (int t = tid; t < 4 * WF; t += 256) sRC[t / WF][t % WF] = 0;
    if (tid < we) {
        const int ex = min(max(x0 - p + tid, 0), A.N1 - 1), ey = min(max(y0 - p + tid, 0), A.N2 - 1);
        sX[tid] = 0.5 * (A.G.bp1[ex] + A.G.bp1[ex + 1]);
        sY[tid] = 0.5 * (A.G.bp2[ey] + A.G.bp2[ey + 1]);
        sCnt[tid] = (T.n_curves > 0) ? T.row_cnt[ey] : 0;
    }
    if (T.n_curves > 0) {
        for (int t = tid; t < we * kRowCross; t += 256) {
            const int r = t / kRowCross, j = t % kRowCross;
            const size_t o = (size_t)min(max(y0 - p + r, 0), A.N2 - 1) * kRowCross + j;
            sKey[r][j] = T.row_key[o];
            sCur[r][j] = (int8_t)T.row_curve[o];
        }
    }
    constexpr int NIT = (WE * WE + 255) / 256;
    int mk[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {  // cut marks of this thread's elements, loaded together
        const int t = tid + 256 * it, u = t % we, v = t / we;
        const int ex = min(max(x0 - p + u, 0), A.N1 - 1), ey = min(max(y0 - p + v, 0), A.N2 - 1);
        mk[it] = A.emark[ey * A.N1 + ex];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int t = tid + 256 * it;
        if (t >= we * we) break;
        const int u = t % we, v = t / we;
        const int ex = x0 - p + u, ey = y0 - p + v;
        int8_t c = -1;
        if (ex >= 0 && ex < A.N1 && ey >= 0 && ey < A.N2) {
            if (mk[it] == epoch) {
                c = EL_CUT;
            } else {  // even-odd test at the centre, from the staged crossings
                const double x = sX[u], y = sY[v];
                bool out = false;
                c = EL_INSIDE;
                if (T.n_curves > 0) {
                    const int nc = sCnt[v];
                    if (nc > kRowCross || T.n_curves > 32) {
                        c = kElPending;  // the direct test, below
                    } else {
                        unsigned par = 0u;
                        for (int j = 0; j < nc; ++j)
                            if (sKey[v][j] > x) par ^= 1u << sCur[v][j];
                        out = par != 0u;
                        for (int cc = 0; cc < T.n_curves && !out; ++cc) {
                            const CurveDev C = T.curves[cc];
                            if (C.kind == IGA_CURVE_ELLIPSE) out = ellipse_implicit(C, x, y) < 0.0;
                        }
                    }
                }
                if (c != kElPending) c = out ? EL_OUTSIDE : EL_INSIDE;
            }
            if (c != kElPending && u >= p && u < p + kClsTile && v >= p && v < p + kClsTile)
                A.ecls[ey * A.N1 + ex] = c;
        }
        sE[v][u] = c;
    }
    __syncthreads();
    // rows with more crossings than recorded: the direct test (one copy of its code, not unrolled)
#pragma unroll 1
    for (int t = tid; t < we * we; t += 256) {
        const int u = t % we, v = t / we;
        if (sE[v][u] != kElPending) continue;
        const int ex = x0 - p + u, ey = y0 - p + v;
        const int8_t c = in_any_hole(T, sX[u], sY[v]) ? EL_OUTSIDE : EL_INSIDE;
        if (u >= p && u < p + kClsTile && v >= p && v < p + kClsTile) A.ecls[ey * A.N1 + ex] = c;
        sE[v][u] = c;
    }
    __syncthreads();
    const bool lastx = blockIdx.x == gridDim.x - 1, lasty = blockIdx.y == gridDim.y - 1;
    for (int t = tid; t < wf * wf; t += 256) {
        const int u = t % wf, v = t / wf;
        const int j1 = x0 + u, j2 = y0 + v;
        int8_t cls = FN_EXTERIOR;
        if (j1 < A.n1 && j2 < A.n2) {
            int nin = 0, nout = 0, ntot = 0;
            for (int e2 = max(0, j2 - p); e2 <= min(A.N2 - 1, j2); ++e2)
                for (int e1 = max(0, j1 - p); e1 <= min(A.N1 - 1, j1); ++e1) {
                    const int8_t c = sE[e2 - y0 + p][e1 - x0 + p];
                    nin += (c == EL_INSIDE);
                    nout += (c == EL_OUTSIDE);
                    ++ntot;
                }
            cls = (nout == ntot) ? FN_EXTERIOR : (nin == ntot ? FN_INTERIOR : FN_CUT);
            const bool own = (u < kClsTile || lastx) && (v < kClsTile || lasty);
            if (own) {
                const int f = j2 * A.n1 + j1;
                const int act = cls != FN_EXTERIOR;
                const int cut = (A.method == IGA_GAUSS_REF) ? (cls != FN_EXTERIOR) : (cls == FN_CUT);
                A.fcls[f] = cls;
                A.f_active[f] = act;
                A.f_cut[f] = cut;
                if (act) atomicAdd(&sRC[0][v], 1);
                if (cut) atomicAdd(&sRC[1][v], 1);
            }
        }
        sF[v][u] = cls;
    }
    __syncthreads();
    const int tx = tid % kClsTile, ty = tid / kClsTile;
    const int e1 = x0 + tx, e2 = y0 + ty;
    if (e1 < A.N1 && e2 < A.N2) {
        const int8_t c = sE[ty + p][tx + p];
        int band = 0;
        if (c == EL_INSIDE && A.method != IGA_NAIVE_WQ) {
            if (A.method == IGA_GAUSS_REF) band = 1;
            else
                for (int d2 = 0; d2 <= p; ++d2)
                    for (int d1 = 0; d1 <= p; ++d1) band |= (sF[ty + d2][tx + d1] == FN_CUT);
        }
        const int e = e2 * A.N1 + e1;
        A.e_cut[e] = (c == EL_CUT);
        A.e_band[e] = band;
        if (c == EL_CUT) atomicAdd(&sRC[2][ty], 1);
        if (band) atomicAdd(&sRC[3][ty], 1);
    }
    __syncthreads();
    // the tile's row-segment counts, for the row-wise list writer's offsets
    const int ntx = gridDim.x, bx = blockIdx.x;
    if (tid < wf) {  // function rows this tile owns
        const int j2 = y0 + tid;
        if ((tid < kClsTile || lasty) && j2 < A.n2) {
            A.rcnt[(size_t)(0 * A.n2 + j2) * ntx + bx] = sRC[0][tid];
            A.rcnt[(size_t)(1 * A.n2 + j2) * ntx + bx] = sRC[1][tid];
        }
    } else if (tid >= 64 && tid < 64 + kClsTile) {  // element rows
        const int r = tid - 64, er = y0 + r;
        if (er < A.N2) {
            A.rcnt[(size_t)(2 * A.n2 + er) * ntx + bx] = sRC[2][r];
            A.rcnt[(size_t)(3 * A.n2 + er) * ntx + bx] = sRC[3][r];
        }
    }
}

void launch_trim_classes(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    GridDev G{P.dir[0].knots + P.p, P.dir[1].knots + P.p, P.N1, P.N2};  // breakpoints
    int ne = P.N1 * P.N2;
    int nf = P.n1 * P.n2;
    int* f_active = P.flags;
    int* f_cut = P.flags + (nf + 1);
    int* e_cut = P.flags + 2 * (nf + 1);
    int* e_band = e_cut + (ne + 1);
    ClassArgs A{P.p,     P.N1,    P.N2,  P.n1,     P.n2,  P.method, T,     G,
                P.emark, P.list_rcnt, P.ecls, P.fcls, f_active, f_cut, e_cut, e_band};
    dim3 g((P.N1 + kClsTile - 1) / kClsTile, (P.N2 + kClsTile - 1) / kClsTile);
    klaunch(P, "k_classes", k_classes, g, dim3(256), 0, s, A);
}

// --------------------------------------------------------------- lists
// The four compactions of the classes -- active functions (act_of, fn_of),
// rows formed element-wise (their compact ids), cut elements and band
// elements (id map and list) -- in one launch of one workgroup per row of
// functions (and of elements): the class kernel left, per row and tile
// column, how many flags of each kind it set; a row's offset is the sum of
// those counts over the rows before it (summed by the row's workgroup, or
// scanned by a separate launch for very large patches). Lists come out in
// increasing flat order.
struct ListArgs {
    const int* flag[4];  // f_active, f_cut (functions), e_cut, e_band (elements)
    int rows[4], len[4]; // rows and row length of each flag array (n2 x n1 or N2 x N1)
    int* map[4];         // act_of, -, cut_id, band_id
    int* list[4];        // fn_of, form_rows (compact ids), cut_list, band_list
    int* bsum;           // [4][n2][ntx] row-segment counts (scanned in place when not prefix_here)
    int n2, ntx;
    int* counts;         // [4] totals
    int prefix_here;     // 1: each workgroup sums the counts of the rows before it
};

__device__ __forceinline__ int block_sum256(int v, int* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum_i(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    const int tot = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return tot;
}

// Very large patches: exclusive scan of the row-segment counts, one
// workgroup of 256 per list; each pass, every thread loads 16 consecutive
// counts (all loads issued together), scans them in registers and offsets
// them by a block scan of the thread totals.
constexpr int kListScanPer = 16;
__global__ void __launch_bounds__(256) k_list_scan(ListArgs A) {
    __shared__ int sh[256 / 64 + 1];
    const int a = blockIdx.x, nt = A.n2 * A.ntx;
    const int m = A.rows[a] * A.ntx;  // element rows past N2 hold nothing
    int* v = A.bsum + (size_t)a * nt;
    int carry = 0;
#pragma unroll 1
    for (int t0 = 0; t0 < m; t0 += 256 * kListScanPer) {
        const int i0 = t0 + (int)threadIdx.x * kListScanPer;
        int x[kListScanPer];
#pragma unroll
        for (int k = 0; k < kListScanPer; ++k) x[k] = v[min(i0 + k, m - 1)];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kListScanPer; ++k) {
            const int xv = (i0 + k < m) ? x[k] : 0;
            x[k] = sum;  // exclusive within the thread
            sum += xv;
        }
        int total;
        const int ex = block_excl_scan(sum, sh, total) + carry;
#pragma unroll
        for (int k = 0; k < kListScanPer; ++k)
            if (i0 + k < m) v[i0 + k] = ex + x[k];
        carry += total;
    }
}

// One workgroup per row r: function row r of arrays 0 and 1, element row r of 2 and 3.
__global__ void __launch_bounds__(256) k_list_rows(ListArgs A) {
    __shared__ int sh[256 / 64 + 1];
    __shared__ int s_off[4];
    const int r = blockIdx.x, nt = A.n2 * A.ntx;
    if (A.prefix_here) {
        // the counts of the rows before r, four per thread and array per pass, loaded together
        const int m = r * A.ntx;
        int v[4] = {0, 0, 0, 0};
#pragma unroll 1
        for (int t0 = 0; t0 < m; t0 += 1024) {
            int x[4][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int t = min(t0 + (int)threadIdx.x + 256 * k, m - 1);
#pragma unroll
                for (int a = 0; a < 4; ++a) x[a][k] = A.bsum[a * nt + t];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (t0 + (int)threadIdx.x + 256 * k < m)
#pragma unroll
                    for (int a = 0; a < 4; ++a) v[a] += x[a][k];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int tot = block_sum256(r <= A.rows[a] ? v[a] : 0, sh);
            if (threadIdx.x == 0) s_off[a] = tot;
        }
    } else if (threadIdx.x < 4) {
        const int a = threadIdx.x;
        s_off[a] = (r < A.rows[a]) ? A.bsum[a * nt + r * A.ntx] : 0;
    }
    __syncthreads();
#pragma unroll 1
    for (int pair = 0; pair < 2; ++pair) {  // (active functions, element-formed rows), (cut, band elements)
        const int a0 = 2 * pair;
        if (r >= A.rows[a0]) continue;
        const int len = A.len[a0];
        const int base = r * len;
        int pos0[2] = {s_off[a0], s_off[a0 + 1]};
#pragma unroll 1
        for (int c0 = 0; c0 < len; c0 += 1024) {
            const int i0 = c0 + threadIdx.x * 4;
            int fl[2][4];
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int f = A.flag[a0 + k][base + min(i0 + j, len - 1)];
                    fl[k][j] = (i0 + j < len) ? (f != 0) : 0;
                }
            int actpos[4] = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int a = a0 + k;
                const int v = fl[k][0] + fl[k][1] + fl[k][2] + fl[k][3];
                int total;
                int pos = block_excl_scan(v, sh, total) + pos0[k];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (i0 + j >= len) continue;
                    const int i = base + i0 + j;
                    if (a == 0) actpos[j] = pos;
                    if (A.map[a]) A.map[a][i] = fl[k][j] ? pos : -1;
                    if (fl[k][j]) A.list[a][pos] = (a == 1) ? actpos[j] : i;
                    pos += fl[k][j];
                }
                pos0[k] += total;
            }
        }
        if (r == A.rows[a0] - 1 && threadIdx.x == 0) {
            A.counts[a0] = pos0[0];
            A.counts[a0 + 1] = pos0[1];
        }
    }
}

bool trim_lists_prefix_here(const Plan& P) {
    return (int64_t)P.n2 * ((P.N1 + kClsTile - 1) / kClsTile) <= 8192;
}

void launch_trim_lists(Plan& P, hipStream_t s) {
    const int nf = P.n1 * P.n2, ne = P.N1 * P.N2;
    int* f_active = P.flags;
    int* f_cut = P.flags + (nf + 1);
    int* e_cut = P.flags + 2 * (nf + 1);
    int* e_band = e_cut + (ne + 1);
    ListArgs A;
    A.flag[0] = f_active; A.flag[1] = f_cut; A.flag[2] = e_cut; A.flag[3] = e_band;
    A.rows[0] = A.rows[1] = P.n2; A.rows[2] = A.rows[3] = P.N2;
    A.len[0] = A.len[1] = P.n1; A.len[2] = A.len[3] = P.N1;
    A.map[0] = P.act_of; A.map[1] = nullptr; A.map[2] = P.cut_id; A.map[3] = P.band_id;
    A.list[0] = P.fn_of; A.list[1] = P.form_rows; A.list[2] = P.cut_list; A.list[3] = P.band_list;
    A.n2 = P.n2;
    A.ntx = (P.N1 + kClsTile - 1) / kClsTile;
    A.bsum = P.list_rcnt;
    A.counts = P.counts;
    A.prefix_here = trim_lists_prefix_here(P);
    if (!A.prefix_here) klaunch(P, "k_list_scan", k_list_scan, dim3(4), dim3(256), 0, s, A);
    klaunch(P, "k_list_rows", k_list_rows, dim3(P.n2), dim3(256), 0, s, A);
}

// ------------------------------------------------------ cut-element rules
struct CutArgs {
    TrimDev T;
    GridDev G;
    int n_cut;
    const int* cut_list;
    const unsigned long long* ehead;  // element lists of kept arcs (k_piece_arcs)
    const int* arc_next;
    CutElemDev* cut_el;
    int* node_cnt;
    int n_r, n_q_override, n_s, p;
    const double* gx;
    const double* gw;
    int* status;
    int* node_off;      // exclusive scan of node_cnt (written by k_cut_nodes)
    int stage_pieces, stage_segs;  // k_cutprep: pieces / segments its LDS holds (0: read them from memory)
    // k_cutprep with fuse_nodes: also writes the element's nodes, at the offsets plan creation found
    int fuse_nodes;
    double *nx, *ny, *nw;
    int* nel;
    double* xy;         // the cut nodes' entries of the rule-point table
    // locate: each workgroup finds its element from the class kernel's counts of cut
    // elements per element row and tile column (loc_m of them, row-major) and the flags
    int locate, loc_m, ntx;
    const int* loc_cnt;
    const int* e_cut;
    int* cut_e;         // the element's flat id, for the element-matrix kernel
};

__device__ __forceinline__ int arc_nq(const CutArgs& A, const CurveDev& C) {
    if (A.n_q_override > 0) return A.n_q_override;
    int d = (C.kind == IGA_CURVE_ELLIPSE) ? 3 : C.degree;
    return d * (2 * A.p + 1);
}

// Pieces as the even-odd test reads them, staged in LDS by k_cutprep.
constexpr int kPrepPieces = 256;
struct PieceBox {
    double ymin, ymax, xmin, xmax, t0, t1;
    int seg, curve;
};

// in_any_hole with the pieces' boxes (and, if staged, the segments) read
// from LDS: same tests, same order.
constexpr int kPrepSegs = 128;
__device__ bool in_any_hole_lds(const TrimDev& T, const PieceBox* sp, const int* scoff, const SegDev* sseg, double x,
                                double y) {
    for (int c = 0; c < T.n_curves; ++c) {
        const CurveDev C = T.curves[c];
        if (C.kind == IGA_CURVE_ELLIPSE) {
            if (ellipse_implicit(C, x, y) < 0.0) return true;
            continue;
        }
        // eight boxes per step, so their LDS reads overlap; the (few) hits are solved after.
        // Pieces are monotone in x and y, so one whose box lies right of the point (by more
        // than the rounding of its end points) crosses the ray right of it without a solve.
        bool in = false;
        const int k1 = scoff[c + 1];
        for (int kb = scoff[c]; kb < k1; kb += 8) {
            unsigned hit = 0u, right = 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = min(kb + u, k1 - 1);
                const PieceBox& B = sp[k];
                const bool h = (kb + u < k1) && (y >= B.ymin && y < B.ymax) && !(B.xmax <= x);
                const bool r = B.xmin - x > 1e-13 * (1.0 + fabs(x));
                hit |= ((h && !r) ? 1u : 0u) << u;
                right |= ((h && r) ? 1u : 0u) << u;
            }
            if (__builtin_popcount(right) & 1) in = !in;
            while (hit) {
                const int u = __builtin_ctz(hit);
                hit &= hit - 1u;
                const PieceBox& B = sp[kb + u];
                const SegDev S = sseg ? sseg[B.seg] : T.segs[B.seg];
                const double t = solve_monotone(S, 1, y, B.t0, B.t1);
                double X, Y, dX, dY;
                seg_eval(S, t, X, Y, dX, dY);
                if (X > x) in = !in;
            }
        }
        if (in) return true;
    }
    return false;
}

// The flat id of the c-th cut element (flat order, as the list kernel
// orders them), from the per-segment counts: the counts are summed in
// groups of 256 (a wavefront sum each, 16 groups per batch of loads) until
// the group holding element c; a scan over the lanes of that group finds the
// segment (element row, tile column); the segment's flags give the column.
// All 64 lanes; -1 if there are fewer cut elements than c + 1.
__device__ int locate_cut_element(const CutArgs& A, int c) {
    const int lane = threadIdx.x, m = A.loc_m;
    constexpr int GB = 16;
    int before = 0, kf = -1;
    int vf[4] = {0, 0, 0, 0};
#pragma unroll 1
    for (int k0 = 0; k0 * 256 < m && kf < 0; k0 += GB) {
        int v[GB][4];
#pragma unroll
        for (int g = 0; g < GB; ++g)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = (k0 + g) * 256 + 4 * lane + j;
                const int x = A.loc_cnt[min(t, m - 1)];
                v[g][j] = (t < m) ? x : 0;
            }
#pragma unroll
        for (int g = 0; g < GB; ++g) {
            const int tot = wave_sum_i(v[g][0] + v[g][1] + v[g][2] + v[g][3]);
            if (kf < 0) {
                if (before + tot > c) {
                    kf = k0 + g;
#pragma unroll
                    for (int j = 0; j < 4; ++j) vf[j] = v[g][j];
                } else {
                    before += tot;
                }
            }
        }
    }
    if (kf < 0) return -1;
    const int mine = vf[0] + vf[1] + vf[2] + vf[3];
    int inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    const int ex = before + inc - mine;
    const unsigned long long hit = __ballot(ex <= c && c < ex + mine);
    const int L = __ffsll((long long)hit) - 1;
    int need = c - ex, j = 0;
    while (j < 3 && need >= vf[j]) {
        need -= vf[j];
        ++j;
    }
    const int t = __builtin_amdgcn_readlane(kf * 256 + 4 * lane + j, L);
    need = __builtin_amdgcn_readlane(need, L);
    const int N1 = A.G.N1, row = t / A.ntx, col0 = (t % A.ntx) * 16, col = col0 + lane;
    const bool f = lane < 16 && col < N1 && A.e_cut[(size_t)row * N1 + min(col, N1 - 1)] != 0;
    unsigned long long fm = __ballot(f);
    for (int k = 0; k < need; ++k) fm &= fm - 1ull;
    if (fm == 0ull) return -1;
    return row * N1 + col0 + __ffsll((long long)fm) - 1;
}

// The nodes write_cut_nodes writes, from what k_cutprep holds in LDS (the
// element's arcs, their Gauss point offsets and the merged edge pieces), with
// the same expressions, so the values are the same; (arc, Gauss point) and
// (piece, node) pairs are spread over the lanes.
__device__ __forceinline__ void write_cut_nodes_staged(const CutArgs& A, int c, int pos, int na, int npts, int var,
                                                       double xa, double xb, double ya, double yb,
                                                       const double (*sT)[2], const SegDev* sArcSeg, const int* sNq,
                                                       const int* sNqOff, const double* sSig, const int* sNseg,
                                                       const double (*sSeg)[kMaxEdgeSegs][2]) {
    const int lane = threadIdx.x;
    const bool vert = var < 2;
    const double b0 = (var == 0) ? xa : (var == 1) ? xb : (var == 2) ? ya : yb;
    const double b1 = (var == 0) ? xb : (var == 1) ? xa : (var == 2) ? yb : ya;
    const int nr = A.n_r;
    const double* rx = A.gx + gauss_off(nr);
    const double* rw = A.gw + gauss_off(nr);
    for (int u = lane; u < npts; u += 64) {
        int q = 0;
        while (q + 1 < na && sNqOff[q + 1] <= u) ++q;
        const int nq = sNq[q], g = u - sNqOff[q];
        const double t0 = sT[q][0], t1 = sT[q][1];
        const double tq = t0 + (t1 - t0) * (A.gx[gauss_off(nq) + g] + 1.0) * 0.5;
        const double wt = A.gw[gauss_off(nq) + g] * (t1 - t0) * 0.5;
        const double sg = sSig[q];
        double X, Y, dX, dY;
        seg_eval(sArcSeg[q], tq, X, Y, dX, dY);
        for (int r = 0; r < nr; ++r) {
            const int o = pos + u * nr + r;
            const double f = (rx[r] + 1.0) * 0.5;
            const double x = vert ? b0 + (X - b0) * f : X, y = vert ? Y : b0 + (Y - b0) * f;
            A.nx[o] = x;
            A.ny[o] = y;
            A.nw[o] = vert ? sg * wt * dY * rw[r] * (X - b0) * 0.5 : -sg * wt * dX * rw[r] * (Y - b0) * 0.5;
            A.nel[o] = c;
            A.xy[2 * o] = x;
            A.xy[2 * o + 1] = y;
        }
    }
    pos += npts * nr;
    const int edge = var ^ 1;  // the edge opposite the base
    const int ns = A.n_s, nsr = ns * nr;
    const double* sx = A.gx + gauss_off(ns);
    const double* sw = A.gw + gauss_off(ns);
    for (int u = lane; u < sNseg[edge] * nsr; u += 64) {
        const int k = u / nsr, t = u - k * nsr;
        const double a = sSeg[edge][k][0], b = sSeg[edge][k][1];
        const int si = t / nr, r = t % nr;
        const double v = a + (b - a) * (sx[si] + 1.0) * 0.5;
        const double wu = sw[si] * (b - a) * 0.5;
        const double inner = b0 + (b1 - b0) * (rx[r] + 1.0) * 0.5;
        const int o = pos + u;
        A.nx[o] = vert ? inner : v;
        A.ny[o] = vert ? v : inner;
        A.nw[o] = wu * rw[r] * fabs(b1 - b0) * 0.5;
        A.nel[o] = c;
        A.xy[2 * o] = vert ? inner : v;
        A.xy[2 * o + 1] = vert ? v : inner;
    }
}

// One wavefront per cut element. (0) lane 0 walks the element's list of kept
// arcs and sorts it by arc index, while the lanes stage the pieces for the
// hole tests in LDS; (1) one lane per arc of the element loads the
// arc, its piece and segment and evaluates its ends; (2) lanes 0..3, one per
// edge (0 left, 1 right, 2 bottom, 3 top), collect the arc ends lying on the
// edge -- crossings of that grid line, and piece ends (extrema or segment
// junctions) that lie on it -- sort them and list the sub-intervals between;
// (3) all lanes test the sub-intervals' midpoints against the holes; (4) lanes
// 0..3 merge the visible sub-intervals; (5) every lane adds its share of
// sum |w| of the four bases over the arcs' Gauss points; lane 0 picks the base
// and the node count.
__global__ void __launch_bounds__(64) k_cutprep(CutArgs A) {
    const int c = blockIdx.x;
    if (c >= A.n_cut) return;
    const TrimDev& T = A.T;
    const int lane = threadIdx.x;
    __shared__ double sEnd[kMaxArcsPerElem][2][2];   // (X, Y) at t0, t1
    __shared__ int sKind[kMaxArcsPerElem][2][2];     // (kind, line) at t0, t1
    __shared__ double sT[kMaxArcsPerElem][2];        // t0, t1
    __shared__ double sIv[4][kMaxEdgeCuts + 1][2];   // sub-intervals per edge
    __shared__ int sIvOk[4][kMaxEdgeCuts + 1];        // -1 too short, 0 in a hole, 1 visible
    __shared__ int sNiv[4];
    __shared__ double sLen[4];
    __shared__ int sOverflow;
    __shared__ int sArc[kMaxArcsPerElem];
    __shared__ int sNa;
    __shared__ int sCoff[33];
    extern __shared__ __align__(16) unsigned char sDyn[];  // pieces' boxes, then segments (sized at launch)
    PieceBox* sP = reinterpret_cast<PieceBox*>(sDyn);
    SegDev* sSegAll = reinterpret_cast<SegDev*>(sDyn + (size_t)A.stage_pieces * sizeof(PieceBox));
    __shared__ SegDev sArcSeg[kMaxArcsPerElem];
    __shared__ int sNq[kMaxArcsPerElem], sNqOff[kMaxArcsPerElem + 1];
    __shared__ double sSig[kMaxArcsPerElem];            // the arcs' curve orientation signs
    __shared__ double sSeg[4][kMaxEdgeSegs][2];          // merged visible pieces per edge
    __shared__ int sNseg[4], sVar, sCnt;
    // node offsets for the fused node writes, loaded while the rule is found
    const int off0 = A.fuse_nodes ? A.node_off[c] : 0, off1 = A.fuse_nodes ? A.node_off[c + 1] : 0;
    const int e = A.locate ? locate_cut_element(A, c) : A.cut_list[c];
    if (e < 0) {  // fewer cut elements than at plan creation
        if (lane == 0) atomicExch(A.status, IGA_E_CAPACITY);
        return;
    }
    if (lane == 0) A.cut_e[c] = e;
    const int e1 = e % A.G.N1, e2 = e / A.G.N1;
    const double xa = A.G.bp1[e1], xb = A.G.bp1[e1 + 1], ya = A.G.bp2[e2], yb = A.G.bp2[e2 + 1];
    CutElemDev& out = A.cut_el[c];
    // (0) the pieces for the hole tests, and the element's kept arcs in ascending order
    const int npc = *T.n_pieces;
    const bool staged = npc <= A.stage_pieces && T.n_curves <= 32;
    if (staged) {
        for (int k = lane; k < npc; k += 64) {
            const PieceDev Pc = T.pieces[k];
            sP[k] = PieceBox{fmin(Pc.y0, Pc.y1), fmax(Pc.y0, Pc.y1), fmin(Pc.x0, Pc.x1), fmax(Pc.x0, Pc.x1),
                             Pc.t0, Pc.t1, Pc.seg, Pc.curve};
        }
        for (int k = lane; k <= T.n_curves; k += 64) sCoff[k] = T.piece_curve_off[k];
    }
    const bool segs_staged = staged && T.n_segs <= A.stage_segs;
    if (segs_staged)
        for (int k = lane; k < T.n_segs; k += 64) sSegAll[k] = T.segs[k];
    if (lane == 0) {
        const unsigned long long h = A.ehead[e];
        int a = ((int)(h >> 32) == *T.epoch) ? (int)(h & 0xffffffffull) - 1 : -1;
        int n = 0;
        for (int it = 0; a >= 0 && it <= kMaxArcsPerElem; ++it) {
            if (n < kMaxArcsPerElem) sArc[n++] = a;
            a = A.arc_next[a];
        }
        sOverflow = a >= 0;
        for (int i = 1; i < n; ++i) {
            const int v = sArc[i];
            int j = i - 1;
            while (j >= 0 && sArc[j] > v) { sArc[j + 1] = sArc[j]; --j; }
            sArc[j + 1] = v;
        }
        sNa = n;
        out.narc = n;
    }
    __syncthreads();
    const int na = sNa;
    // (1) arcs, one lane each
    for (int q = lane; q < na; q += 64) {
        out.arc[q] = sArc[q];
        const ArcDev R = T.arcs[sArc[q]];
        sArcSeg[q] = T.segs[R.gseg];
        const CurveDev Cv = T.curves[R.curve];
        sNq[q] = arc_nq(A, Cv);
        sSig[q] = Cv.sigma;
        sEnd[q][0][0] = R.x0;
        sEnd[q][0][1] = R.y0;
        sEnd[q][1][0] = R.x1;
        sEnd[q][1][1] = R.y1;
        sKind[q][0][0] = R.k0;
        sKind[q][0][1] = R.l0;
        sKind[q][1][0] = R.k1;
        sKind[q][1][1] = R.l1;
        sT[q][0] = R.t0;
        sT[q][1] = R.t1;
    }
    __syncthreads();
    // (2) edge cut points and sub-intervals
    if (lane < 4) {
        const int edge = lane;
        double cuts[kMaxEdgeCuts];
        int n = 0;
        bool overflow = false;
        const double ref = (edge == 0) ? xa : (edge == 1) ? xb : (edge == 2) ? ya : yb;
        const double h = (edge < 2) ? xb - xa : yb - ya;
        for (int q = 0; q < na; ++q) {
            for (int end = 0; end < 2; ++end) {
                const int kind = sKind[q][end][0], line = sKind[q][end][1];
                const double X = sEnd[q][end][0], Y = sEnd[q][end][1];
                bool on = false;
                if (kind == END_VLINE) on = (line == e1 + (edge == 1)) && edge < 2;
                else if (kind == END_HLINE) on = (line == e2 + (edge == 3)) && edge >= 2;
                // a piece end (extremum or segment junction) on a grid line: the half-open
                // crossing count gives that crossing to the neighbouring piece only
                else on = fabs(((edge < 2) ? X : Y) - ref) <= 1e-12 * h;
                if (!on) continue;
                if (n < kMaxEdgeCuts) cuts[n++] = (edge < 2) ? Y : X;
                else overflow = true;
            }
        }
        for (int a = 1; a < n; ++a) {
            const double v = cuts[a];
            int b = a - 1;
            while (b >= 0 && cuts[b] > v) { cuts[b + 1] = cuts[b]; --b; }
            cuts[b + 1] = v;
        }
        const double lo = (edge < 2) ? ya : xa, hi = (edge < 2) ? yb : xb;
        const double tol = 1e-13 * (hi - lo);
        double prev = lo;
        for (int q = 0; q <= n; ++q) {
            const double a = prev;
            const double b = (q == n) ? hi : fmin(fmax(cuts[q], lo), hi);
            prev = b;
            sIv[edge][q][0] = a;
            sIv[edge][q][1] = b;
            sIvOk[edge][q] = (b - a <= tol) ? -1 : 0;
        }
        sNiv[edge] = n + 1;
        if (overflow) sOverflow = 1;
    } else if (lane == 4) {  // offsets of the arcs' Gauss points
        int off = 0;
        for (int q = 0; q < na; ++q) {
            sNqOff[q] = off;
            off += sNq[q];
        }
        sNqOff[na] = off;
    }
    __syncthreads();
    // (3) hole tests of the sub-intervals' midpoints, all lanes
    for (int u = lane; u < 4 * (kMaxEdgeCuts + 1); u += 64) {
        const int edge = u / (kMaxEdgeCuts + 1), q = u % (kMaxEdgeCuts + 1);
        if (q >= sNiv[edge] || sIvOk[edge][q] < 0) continue;
        const double fixed = (edge == 0) ? xa : (edge == 1) ? xb : (edge == 2) ? ya : yb;
        const double m = 0.5 * (sIv[edge][q][0] + sIv[edge][q][1]);
        const double x = (edge < 2) ? fixed : m, y = (edge < 2) ? m : fixed;
        sIvOk[edge][q] = (staged ? in_any_hole_lds(T, sP, sCoff, segs_staged ? sSegAll : nullptr, x, y)
                                 : in_any_hole(T, x, y))
                             ? 0
                             : 1;
    }
    __syncthreads();
    // (4) merge the visible sub-intervals
    if (lane < 4) {
        const int edge = lane;
        const double lo = (edge < 2) ? ya : xa, hi = (edge < 2) ? yb : xb;
        const double tol = 1e-13 * (hi - lo);
        int ns = 0;
        bool overflow = false;
        double len = 0.0, last_hi = 0.0;
        for (int q = 0; q < sNiv[edge]; ++q) {
            if (sIvOk[edge][q] != 1) continue;
            const double a = sIv[edge][q][0], b = sIv[edge][q][1];
            if (ns > 0 && fabs(last_hi - a) <= tol) {
                out.seg[edge][ns - 1][1] = b;
                sSeg[edge][ns - 1][1] = b;
            } else if (ns < kMaxEdgeSegs) {
                out.seg[edge][ns][0] = a;
                out.seg[edge][ns][1] = b;
                sSeg[edge][ns][0] = a;
                sSeg[edge][ns][1] = b;
                ++ns;
            } else {
                overflow = true;
                continue;
            }
            last_hi = b;
            len += b - a;
        }
        out.nseg[edge] = ns;
        sNseg[edge] = ns;
        sLen[edge] = len;
        if (overflow) sOverflow = 1;
    }
    // (5) sum |w| of the four bases over the arcs' Gauss points, one (arc, point) pair per lane
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int npts = sNqOff[na];
    const int narc_nodes = npts * A.n_r;
    for (int u = lane; u < npts; u += 64) {
        int q = 0;
        while (q + 1 < na && sNqOff[q + 1] <= u) ++q;
        const int nq = sNq[q], g = u - sNqOff[q];
        const double t0 = sT[q][0], t1 = sT[q][1];
        const double tq = t0 + (t1 - t0) * (A.gx[gauss_off(nq) + g] + 1.0) * 0.5;
        const double wt = A.gw[gauss_off(nq) + g] * (t1 - t0) * 0.5;
        double X, Y, dX, dY;
        seg_eval(sArcSeg[q], tq, X, Y, dX, dY);
        s0 += wt * fabs(dY) * fabs(X - xa);
        s1 += wt * fabs(dY) * fabs(X - xb);
        s2 += wt * fabs(dX) * fabs(Y - ya);
        s3 += wt * fabs(dX) * fabs(Y - yb);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    __syncthreads();
    if (lane == 0) {
        double sums[4] = {s0 + sLen[1] * (xb - xa), s1 + sLen[0] * (xb - xa), s2 + sLen[3] * (yb - ya),
                          s3 + sLen[2] * (yb - ya)};
        double mn = fmin(fmin(sums[0], sums[1]), fmin(sums[2], sums[3]));
        int var = 0;
        while (var < 3 && !(sums[var] <= mn * (1.0 + 1e-9))) ++var;
        const int opp = var ^ 1;
        out.e1 = e1;
        out.e2 = e2;
        out.variant = var;
        const int cnt = narc_nodes + sNseg[opp] * A.n_s * A.n_r;
        A.node_cnt[c] = cnt;
        sVar = var;
        sCnt = cnt;
        if (sOverflow) atomicExch(A.status, IGA_E_TOPOLOGY);
    }
    if (A.fuse_nodes) {
        // the same inputs as at plan creation give the same node counts, so
        // the offsets found then hold; a different count is reported, not written
        __syncthreads();
        if (sCnt == off1 - off0) {
            write_cut_nodes_staged(A, c, off0, na, npts, sVar, xa, xb, ya, yb, sT, sArcSeg, sNq, sNqOff, sSig,
                                   sNseg, sSeg);
        } else if (lane == 0) {
            atomicExch(A.status, IGA_E_CAPACITY);
        }
    }
}

void launch_trim_cutprep(Plan& P, hipStream_t s, bool fuse_nodes) {
    TrimDev& T = P.trim;
    int nc = (int)P.n_cut_el;
    if (T.n_curves == 0 || nc == 0) return;
    GridDev G{P.dir[0].knots + P.p, P.dir[1].knots + P.p, P.N1, P.N2};  // breakpoints
    CutArgs A{T, G, nc, P.cut_list, P.ehead, P.arc_next, P.cut_el, P.node_cnt,
              P.n_r, P.n_q_override, P.n_s, P.p, P.gauss_x, P.gauss_w, P.status, P.node_off, 0, 0};
    if (fuse_nodes) {
        const size_t cut0 = (size_t)P.dir[0].Q * P.dir[1].Q + (size_t)P.n_band * (P.p + 1) * (P.p + 1);
        A.fuse_nodes = 1;
        A.nx = P.node_x;
        A.ny = P.node_y;
        A.nw = P.node_w;
        A.nel = P.node_el;
        A.xy = P.pts_xy + 2 * cut0;
    }
    A.cut_e = P.cut_e;
    A.locate = trim_lists_prefix_here(P);
    if (A.locate) {  // the element counts of the class kernel's tile-row segments
        const int nf = P.n1 * P.n2;
        A.ntx = (P.N1 + kClsTile - 1) / kClsTile;
        A.loc_m = P.N2 * A.ntx;
        A.loc_cnt = P.list_rcnt + (size_t)2 * P.n2 * A.ntx;
        A.e_cut = P.flags + 2 * (nf + 1);
    }
    A.stage_pieces = (T.cap_pieces <= kPrepPieces) ? T.cap_pieces : 0;
    A.stage_segs = (A.stage_pieces > 0 && T.n_segs <= kPrepSegs) ? T.n_segs : 0;
    const size_t lds = (size_t)A.stage_pieces * sizeof(PieceBox) + (size_t)A.stage_segs * sizeof(SegDev);
    klaunch(P, "k_cutprep", k_cutprep, dim3(nc), dim3(64), (uint32_t)lds, s, A);
}

// One wavefront per cut element writes its nodes (and their entries of the
// rule-point table), at the offset the counts before it add up to.
constexpr int kNodePrefixMax = 8192;  // up to this many cut elements each workgroup sums the counts before it

// The element's nodes and weights (arcs first, then the straight pieces of
// the edge opposite the base), from offset pos on.
__device__ void write_cut_nodes(const CutArgs& A, int c, int pos, double* __restrict__ nx, double* __restrict__ ny,
                                double* __restrict__ nw, int* __restrict__ nel, double* __restrict__ xy) {
    const TrimDev& T = A.T;
    const CutElemDev& E = A.cut_el[c];
    double xa = A.G.bp1[E.e1], xb = A.G.bp1[E.e1 + 1], ya = A.G.bp2[E.e2], yb = A.G.bp2[E.e2 + 1];
    int var = E.variant;
    bool vert = var < 2;
    double b0 = (var == 0) ? xa : (var == 1) ? xb : (var == 2) ? ya : yb;
    double b1 = (var == 0) ? xb : (var == 1) ? xa : (var == 2) ? yb : ya;
    int nr = A.n_r;
    const double* rx = A.gx + gauss_off(nr);
    const double* rw = A.gw + gauss_off(nr);
    for (int q = 0; q < E.narc; ++q) {
        const ArcDev R = T.arcs[E.arc[q]];
        const SegDev S = T.segs[R.gseg];
        const CurveDev C = T.curves[R.curve];
        int nq = arc_nq(A, C);
        for (int g = threadIdx.x; g < nq; g += 64) {
            double tq = R.t0 + (R.t1 - R.t0) * (A.gx[gauss_off(nq) + g] + 1.0) * 0.5;
            double wt = A.gw[gauss_off(nq) + g] * (R.t1 - R.t0) * 0.5;
            double X, Y, dX, dY;
            seg_eval(S, tq, X, Y, dX, dY);
            for (int r = 0; r < nr; ++r) {
                int o = pos + g * nr + r;
                double f = (rx[r] + 1.0) * 0.5;
                const double x = vert ? b0 + (X - b0) * f : X, y = vert ? Y : b0 + (Y - b0) * f;
                nx[o] = x;
                ny[o] = y;
                nw[o] = vert ? C.sigma * wt * dY * rw[r] * (X - b0) * 0.5 : -C.sigma * wt * dX * rw[r] * (Y - b0) * 0.5;
                nel[o] = c;
                xy[2 * o] = x;
                xy[2 * o + 1] = y;
            }
        }
        pos += nq * nr;
    }
    const int opp[4] = {1, 0, 3, 2};
    int edge = opp[var];
    int ns = A.n_s;
    const double* sx = A.gx + gauss_off(ns);
    const double* sw = A.gw + gauss_off(ns);
    for (int k = 0; k < E.nseg[edge]; ++k) {
        double a = E.seg[edge][k][0], b = E.seg[edge][k][1];
        for (int t = threadIdx.x; t < ns * nr; t += 64) {
            int si = t / nr, r = t % nr;
            double u = a + (b - a) * (sx[si] + 1.0) * 0.5;
            double wu = sw[si] * (b - a) * 0.5;
            double inner = b0 + (b1 - b0) * (rx[r] + 1.0) * 0.5;
            int o = pos + t;
            nx[o] = vert ? inner : u;
            ny[o] = vert ? u : inner;
            nw[o] = wu * rw[r] * fabs(b1 - b0) * 0.5;
            nel[o] = c;
            xy[2 * o] = vert ? inner : u;
            xy[2 * o + 1] = vert ? u : inner;
        }
        pos += ns * nr;
    }
}

__global__ void __launch_bounds__(64) k_cut_nodes(CutArgs A, int prefix_here, double* __restrict__ nx,
                                                  double* __restrict__ ny, double* __restrict__ nw,
                                                  int* __restrict__ nel, double* __restrict__ xy) {
    int c = blockIdx.x;
    if (c >= A.n_cut) return;
    // this element's first node: the sum of the counts before it (or the scanned offsets)
    int pos;
    if (prefix_here) {
        int sum = 0;
        for (int i0 = 0; i0 < c; i0 += 64 * 8) {
            int v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = i0 + threadIdx.x + 64 * j;
                v[j] = (i < c) ? A.node_cnt[i] : 0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) sum += v[j];
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
        pos = sum;
        if (threadIdx.x == 0) {
            A.node_off[c] = pos;
            if (c == A.n_cut - 1) A.node_off[A.n_cut] = pos + A.node_cnt[c];
        }
    } else {
        pos = A.node_off[c];
    }
    write_cut_nodes(A, c, pos, nx, ny, nw, nel, xy);
}

void launch_trim_nodes(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    int nc = (int)P.n_cut_el;
    if (T.n_curves == 0 || nc == 0) return;
    GridDev G{P.dir[0].knots + P.p, P.dir[1].knots + P.p, P.N1, P.N2};  // breakpoints
    CutArgs A{T, G, nc, P.cut_list, P.ehead, P.arc_next, P.cut_el, P.node_cnt,
              P.n_r, P.n_q_override, P.n_s, P.p, P.gauss_x, P.gauss_w, P.status, P.node_off, 0, 0};
    const size_t cut0 = (size_t)P.dir[0].Q * P.dir[1].Q + (size_t)P.n_band * (P.p + 1) * (P.p + 1);
    const int prefix_here = nc <= kNodePrefixMax;
    if (!prefix_here) exclusive_scan(P.node_cnt, P.node_off, nc, P.scan_tmp, s);
    klaunch(P, "k_cut_nodes", k_cut_nodes, dim3(nc), dim3(64), 0, s, A, prefix_here, P.node_x, P.node_y, P.node_w,
                       P.node_el, P.pts_xy + 2 * cut0);
}

}  // namespace iga

namespace iga {

// Naive weighted quadrature (Table 1): c set to zero at WQ points in a hole.
__global__ void k_naive_mask(TrimDev T, DirDev D1, DirDev D2, const double* __restrict__ src, double cval,
                             double* __restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= D1.Q * D2.Q) return;
    int k1 = k % D1.Q, k2 = k / D1.Q;
    double c = src ? src[k] : cval;
    out[k] = in_any_hole(T, D1.xq[k1], D2.xq[k2]) ? 0.0 : c;
}

void launch_naive_mask(Plan& P, const double* src, double cval, hipStream_t s) {
    int nq = P.dir[0].Q * P.dir[1].Q;
    klaunch(P, "k_naive_mask", k_naive_mask, dim3((nq + 255) / 256), dim3(256), 0, s, P.trim, P.dir[0], P.dir[1], src, cval,
                       P.c_wq_masked);
}

// Structural nonzeros: active columns inside the band of each active row.
__global__ void k_row_nnz(int p, int n1, int n2, const int* __restrict__ fn_of, const int* __restrict__ act_of,
                          int n_act, int* __restrict__ cnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_act) return;
    int f = fn_of[r], i1 = f % n1, i2 = f / n1;
    int c = 0;
    for (int j2 = max(0, i2 - p); j2 <= min(n2 - 1, i2 + p); ++j2)
        for (int j1 = max(0, i1 - p); j1 <= min(n1 - 1, i1 + p); ++j1) c += act_of[j2 * n1 + j1] >= 0;
    cnt[r] = c;
}

void launch_row_nnz(Plan& P, int* cnt, int* out, hipStream_t s) {
    int n = (int)P.n_act;
    hipLaunchKernelGGL(k_row_nnz, dim3((n + 255) / 256), dim3(256), 0, s, P.p, P.n1, P.n2, P.fn_of, P.act_of, n, cnt);
    exclusive_scan(cnt, out, n, P.scan_tmp, s);
}

}  // namespace iga
