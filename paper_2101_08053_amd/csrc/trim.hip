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
__device__ __forceinline__ void seg_eval(const SegDev& S, double t, double& X, double& Y, double& dX, double& dY) {
    if (S.kind == IGA_CURVE_ELLIPSE) {
        double c = cos(t), s = sin(t);
        X = S.px[0] + S.px[1] * c + S.px[2] * s;
        Y = S.py[0] + S.py[1] * c + S.py[2] * s;
        dX = -S.px[1] * s + S.px[2] * c;
        dY = -S.py[1] * s + S.py[2] * c;
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

// ---------------------------------------------------------- segments
// Uniform B-spline blending polynomials (power basis, low first) of degree 1..3.
__device__ __forceinline__ double blend(int d, int l, int pw) {
    // rows: function l, columns: power
    const double b1[2][2] = {{1, -1}, {0, 1}};
    const double b2[3][3] = {{0.5, -1, 0.5}, {0.5, 1, -1}, {0, 0, 0.5}};
    const double b3[4][4] = {{1.0 / 6, -0.5, 0.5, -1.0 / 6},
                             {4.0 / 6, 0, -1, 0.5},
                             {1.0 / 6, 0.5, 0.5, -0.5},
                             {0, 0, 0, 1.0 / 6}};
    if (d == 1) return b1[l][pw];
    if (d == 2) return b2[l][pw];
    return b3[l][pw];
}

__global__ void k_segments(TrimDev T, const double* __restrict__ cp, const int* __restrict__ cp_off) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T.n_segs) return;
    int c = 0;
    while (c + 1 < T.n_curves && T.curves[c + 1].seg0 <= s) ++c;
    const CurveDev C = T.curves[c];
    SegDev S;
    S.curve = c;
    S.seg = s - C.seg0;
    S.kind = C.kind;
    S.pad = 0;
    for (int k = 0; k < 4; ++k) S.px[k] = S.py[k] = 0.0;
    if (C.kind == IGA_CURVE_ELLIPSE) {
        double cph = cos(C.phi), sph = sin(C.phi);
        S.px[0] = C.cx; S.px[1] = C.a * cph; S.px[2] = -C.b * sph;
        S.py[0] = C.cy; S.py[1] = C.a * sph; S.py[2] = C.b * cph;
    } else {
        int d = C.degree, m = C.n_seg;
        for (int l = 0; l <= d; ++l) {
            int idx = (S.seg + l) % m;
            double x = cp[2 * (cp_off[c] + idx)], y = cp[2 * (cp_off[c] + idx) + 1];
            for (int pw = 0; pw <= d; ++pw) {
                S.px[pw] += blend(d, l, pw) * x;
                S.py[pw] += blend(d, l, pw) * y;
            }
        }
    }
    T.segs[s] = S;
}

// Zeros of a + b t + c t^2 in (lo, hi), ascending.
__device__ int quad_roots(double a, double b, double c, double lo, double hi, double* r) {
    int n = 0;
    double scale = fabs(a) + fabs(b) + fabs(c);
    if (scale == 0.0) return 0;
    if (fabs(c) <= 1e-14 * scale) {
        if (fabs(b) > 1e-14 * scale) {
            double t = -a / b;
            if (t > lo && t < hi) r[n++] = t;
        }
        return n;
    }
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return 0;
    double q = -0.5 * (b + copysign(sqrt(disc), b));
    double t1 = q / c, t2 = (q != 0.0) ? a / q : t1;
    if (t1 > t2) { double t = t1; t1 = t2; t2 = t; }
    if (t1 > lo && t1 < hi) r[n++] = t1;
    if (t2 > lo && t2 < hi && t2 != t1) r[n++] = t2;
    return n;
}

// Split parameters of segment s (x- and y-extrema), sorted, plus the ends.
__device__ int segment_splits(const TrimDev& T, int s, double* ts) {
    const SegDev S = T.segs[s];
    const CurveDev C = T.curves[S.curve];
    int n = 0;
    double lo = 0.0, hi = C.t_range;
    ts[n++] = lo;
    double r[8];
    int nr = 0;
    if (S.kind == IGA_CURVE_ELLIPSE) {
        const double tp = 2.0 * M_PI;
        double c[4] = {atan2(S.px[2], S.px[1]), atan2(S.px[2], S.px[1]) + M_PI, atan2(S.py[2], S.py[1]),
                       atan2(S.py[2], S.py[1]) + M_PI};
        for (int k = 0; k < 4; ++k) {
            double t = fmod(c[k], tp);
            if (t < 0.0) t += tp;
            if (t > lo && t < hi) r[nr++] = t;
        }
    } else {
        nr += quad_roots(S.px[1], 2.0 * S.px[2], 3.0 * S.px[3], lo, hi, r + nr);
        nr += quad_roots(S.py[1], 2.0 * S.py[2], 3.0 * S.py[3], lo, hi, r + nr);
    }
    for (int a = 1; a < nr; ++a) {  // insertion sort
        double v = r[a];
        int b = a - 1;
        while (b >= 0 && r[b] > v) { r[b + 1] = r[b]; --b; }
        r[b + 1] = v;
    }
    for (int k = 0; k < nr; ++k)
        if (r[k] > ts[n - 1]) ts[n++] = r[k];
    ts[n++] = hi;
    return n;
}

__device__ __forceinline__ PieceDev make_piece(const TrimDev& T, int s, double t0, double t1) {
    const SegDev S = T.segs[s];
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

// Single block: monotone pieces of every segment, compacted in segment order.
__global__ void __launch_bounds__(1024) k_pieces(TrimDev T, PieceDev* __restrict__ out, int* __restrict__ count,
                                                 int* __restrict__ curve_off) {
    __shared__ int sh[1024 / 64 + 1];
    int carry = 0;
    for (int base = 0; base < T.n_segs; base += blockDim.x) {
        int s = base + threadIdx.x;
        double ts[12];
        int nt = 0;
        if (s < T.n_segs) nt = segment_splits(T, s, ts);
        int np = (nt > 1) ? nt - 1 : 0;
        int total;
        int off = block_scan_carry(np, sh, total) + carry;
        if (s < T.n_segs) {
            for (int k = 0; k < np; ++k) out[off + k] = make_piece(T, s, ts[k], ts[k + 1]);
            const SegDev S = T.segs[s];
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
                for (int it = 0; it < 200; ++it) {
                    double mid = 0.5 * (a + b);
                    if (mid == a || mid == b) break;
                    double X, Y, dX, dY;
                    seg_eval(S, mid, X, Y, dX, dY);
                    double gm = ellipse_implicit(C, X, Y);
                    if ((gm < 0.0) == (ga < 0.0)) a = mid; else b = mid;
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

__global__ void __launch_bounds__(1024) k_split_pieces(TrimDev T) {
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
            double a = Pc.t0;
            for (int q = 0; q < ns; ++q) {
                double b = (q == ns - 1) ? Pc.t1 : T.isect_t[k * kMaxIsectPerPiece + q];
                T.pieces[off + q] = make_piece(T, Pc.seg, a, b);
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

void launch_trim_curves(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    if (T.n_curves == 0) return;
    hipLaunchKernelGGL(k_segments, dim3((T.n_segs + 63) / 64), dim3(64), 0, s, T, P.d_cp, P.d_cp_off);
    if (T.n_curves == 1) {
        hipLaunchKernelGGL(k_pieces, dim3(1), dim3(1024), 0, s, T, T.pieces, T.n_pieces, T.piece_curve_off);
    } else {
        hipLaunchKernelGGL(k_pieces, dim3(1), dim3(1024), 0, s, T, T.pieces0, T.n_pieces0, T.piece_curve_off);
        hipLaunchKernelGGL(k_piece_isect, dim3(T.cap_pieces0), dim3(64), 0, s, T, P.status);
        hipLaunchKernelGGL(k_split_pieces, dim3(1), dim3(1024), 0, s, T);
    }
}

// ------------------------------------------------------------ crossings
struct GridDev {
    const double* bp1;
    const double* bp2;
    int N1, N2;
};

__global__ void k_cross_count(TrimDev T, GridDev G) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= T.cap_pieces) return;
    int np = *T.n_pieces;
    if (k >= np) {
        T.cross_cnt[k] = 0;
        T.nv[k] = 0;
        return;
    }
    const PieceDev Pc = T.pieces[k];
    double xmin = fmin(Pc.x0, Pc.x1), xmax = fmax(Pc.x0, Pc.x1);
    double ymin = fmin(Pc.y0, Pc.y1), ymax = fmax(Pc.y0, Pc.y1);
    int nv = lower_bound_d(G.bp1, G.N1 + 1, xmax) - lower_bound_d(G.bp1, G.N1 + 1, xmin);
    int nh = lower_bound_d(G.bp2, G.N2 + 1, ymax) - lower_bound_d(G.bp2, G.N2 + 1, ymin);
    T.nv[k] = nv;
    T.cross_cnt[k] = nv + nh;
}

void launch_trim_crossings(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    if (T.n_curves == 0) return;
    GridDev G{P.dir[0].bp, P.dir[1].bp, P.N1, P.N2};
    hipLaunchKernelGGL(k_cross_count, dim3((T.cap_pieces + 127) / 128), dim3(128), 0, s, T, G);
    exclusive_scan(T.cross_cnt, T.cross_off, T.cap_pieces, P.scan_tmp, s);
}

__global__ void k_cross_solve(TrimDev T, GridDev G) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int np = *T.n_pieces;
    if (c >= T.cross_off[np]) return;
    int k = upper_bound_i(T.cross_off, np + 1, c) - 1;
    int j = c - T.cross_off[k];
    const PieceDev Pc = T.pieces[k];
    const SegDev S = T.segs[Pc.seg];
    CrossDev X;
    int nv = T.nv[k];
    if (j < nv) {
        int line = lower_bound_d(G.bp1, G.N1 + 1, fmin(Pc.x0, Pc.x1)) + j;
        X.kind = END_VLINE;
        X.line = line;
        X.t = solve_monotone(S, 0, G.bp1[line], Pc.t0, Pc.t1);
    } else {
        int line = lower_bound_d(G.bp2, G.N2 + 1, fmin(Pc.y0, Pc.y1)) + (j - nv);
        X.kind = END_HLINE;
        X.line = line;
        X.t = solve_monotone(S, 1, G.bp2[line], Pc.t0, Pc.t1);
    }
    T.cross[c] = X;
}

// Rank of each crossing in its piece's t order: own rank plus the number of
// crossings of the other family before it (vertical first on ties).
__global__ void k_cross_merge(TrimDev T) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int np = *T.n_pieces;
    if (c >= T.cross_off[np]) return;
    int k = upper_bound_i(T.cross_off, np + 1, c) - 1;
    int base = T.cross_off[k];
    int j = c - base;
    int nv = T.nv[k], nh = T.cross_cnt[k] - nv;
    const PieceDev Pc = T.pieces[k];
    bool incx = Pc.x1 > Pc.x0, incy = Pc.y1 > Pc.y0;
    double t = T.cross[c].t;
    int own, other = 0;
    if (j < nv) {
        own = incx ? j : nv - 1 - j;
        // horizontal crossings with t' < t
        int lo = 0, hi = nh;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            int idx = incy ? mid : nh - 1 - mid;
            if (T.cross[base + nv + idx].t < t) lo = mid + 1; else hi = mid;
        }
        other = lo;
    } else {
        int jh = j - nv;
        own = incy ? jh : nh - 1 - jh;
        int lo = 0, hi = nv;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            int idx = incx ? mid : nv - 1 - mid;
            if (T.cross[base + idx].t <= t) lo = mid + 1; else hi = mid;
        }
        other = lo;
    }
    T.merged[base + own + other] = T.cross[c];
}

__global__ void k_arcs(TrimDev T, GridDev G) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int np = *T.n_pieces;
    int n_arcs = T.cross_off[np] + np;
    if (a >= T.cap_arcs) return;
    if (a >= n_arcs) {
        T.arcs[a].keep = 0;
        return;
    }
    // arcs of piece k start at cross_off[k] + k
    int lo = 0, hi = np;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (T.cross_off[mid] + mid <= a) lo = mid + 1; else hi = mid;
    }
    int k = lo - 1;
    int base = T.cross_off[k];
    int j = a - base - k;
    int n = T.cross_cnt[k];
    const PieceDev Pc = T.pieces[k];
    const SegDev S = T.segs[Pc.seg];
    const CurveDev C = T.curves[Pc.curve];
    ArcDev A;
    A.curve = Pc.curve;
    A.seg = S.seg;
    A.piece = k;
    if (j == 0) { A.t0 = Pc.t0; A.k0 = END_PIECE; A.l0 = -1; }
    else { CrossDev X = T.merged[base + j - 1]; A.t0 = X.t; A.k0 = X.kind; A.l0 = X.line; }
    if (j == n) { A.t1 = Pc.t1; A.k1 = END_PIECE; A.l1 = -1; }
    else { CrossDev X = T.merged[base + j]; A.t1 = X.t; A.k1 = X.kind; A.l1 = X.line; }
    double X, Y, dX, dY;
    seg_eval(S, 0.5 * (A.t0 + A.t1), X, Y, dX, dY);
    int keep = (A.t1 - A.t0 > 1e-13 * C.t_range);
    keep = keep && X > G.bp1[0] && X < G.bp1[G.N1] && Y > G.bp2[0] && Y < G.bp2[G.N2];
    if (keep && T.n_curves > 1) keep = !in_any_hole(T, X, Y, Pc.curve);
    A.keep = keep;
    A.e1 = min(max(upper_bound_d(G.bp1, G.N1 + 1, X) - 1, 0), G.N1 - 1);
    A.e2 = min(max(upper_bound_d(G.bp2, G.N2 + 1, Y) - 1, 0), G.N2 - 1);
    T.arcs[a] = A;
}

void launch_trim_arcs(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    if (T.n_curves == 0) return;
    GridDev G{P.dir[0].bp, P.dir[1].bp, P.N1, P.N2};
    int nc = T.cap_cross > 0 ? T.cap_cross : 1;
    hipLaunchKernelGGL(k_cross_solve, dim3((nc + 127) / 128), dim3(128), 0, s, T, G);
    hipLaunchKernelGGL(k_cross_merge, dim3((nc + 127) / 128), dim3(128), 0, s, T);
    hipLaunchKernelGGL(k_arcs, dim3((T.cap_arcs + 127) / 128), dim3(128), 0, s, T, G);
}

// -------------------------------------------------------------- classes
__global__ void k_elem_centre(TrimDev T, GridDev G, int8_t* __restrict__ ecls) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G.N1 * G.N2) return;
    int e1 = e % G.N1, e2 = e / G.N1;
    double x = 0.5 * (G.bp1[e1] + G.bp1[e1 + 1]), y = 0.5 * (G.bp2[e2] + G.bp2[e2 + 1]);
    ecls[e] = in_any_hole(T, x, y) ? EL_OUTSIDE : EL_INSIDE;
}

__global__ void k_mark_cut(TrimDev T, int N1, int8_t* __restrict__ ecls) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= T.cap_arcs) return;
    const ArcDev A = T.arcs[a];
    if (A.keep) ecls[A.e2 * N1 + A.e1] = EL_CUT;
}

struct ClassArgs {
    int p, N1, N2, n1, n2, method;
    const int8_t* ecls;
    int8_t* fcls;
    int* f_active;   // n1*n2 flags
    int* f_cut;      // n1*n2 flags
    int* e_cut;      // N1*N2 flags
    int* e_band;     // N1*N2 flags
};

__global__ void k_fn_class(ClassArgs A) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= A.n1 * A.n2) return;
    int i1 = f % A.n1, i2 = f / A.n1;
    int nin = 0, nout = 0, ntot = 0;
    for (int e2 = max(0, i2 - A.p); e2 <= min(A.N2 - 1, i2); ++e2)
        for (int e1 = max(0, i1 - A.p); e1 <= min(A.N1 - 1, i1); ++e1) {
            int8_t c = A.ecls[e2 * A.N1 + e1];
            nin += (c == EL_INSIDE);
            nout += (c == EL_OUTSIDE);
            ++ntot;
        }
    int8_t cls = (nout == ntot) ? FN_EXTERIOR : (nin == ntot ? FN_INTERIOR : FN_CUT);
    A.fcls[f] = cls;
    A.f_active[f] = cls != FN_EXTERIOR;
    A.f_cut[f] = (A.method == IGA_GAUSS_REF) ? (cls != FN_EXTERIOR) : (cls == FN_CUT);
}

// Element flags: cut elements, and "band" elements -- inside elements whose
// Gauss points are used by some row formed element-wise.
__global__ void k_elem_flags(ClassArgs A) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.N1 * A.N2) return;
    int e1 = e % A.N1, e2 = e / A.N1;
    int8_t c = A.ecls[e];
    A.e_cut[e] = (c == EL_CUT);
    int band = 0;
    if (c == EL_INSIDE && A.method != IGA_NAIVE_WQ) {
        if (A.method == IGA_GAUSS_REF) band = 1;
        else
            for (int j2 = e2; j2 <= e2 + A.p && !band; ++j2)
                for (int j1 = e1; j1 <= e1 + A.p; ++j1)
                    if (A.fcls[j2 * A.n1 + j1] == FN_CUT) { band = 1; break; }
    }
    A.e_band[e] = band;
}

void launch_trim_classes(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    GridDev G{P.dir[0].bp, P.dir[1].bp, P.N1, P.N2};
    int ne = P.N1 * P.N2;
    hipLaunchKernelGGL(k_elem_centre, dim3((ne + 127) / 128), dim3(128), 0, s, T, G, P.ecls);
    if (T.n_curves > 0)
        hipLaunchKernelGGL(k_mark_cut, dim3((T.cap_arcs + 127) / 128), dim3(128), 0, s, T, P.N1, P.ecls);
    int nf = P.n1 * P.n2;
    int* f_active = P.flags;
    int* f_cut = P.flags + (nf + 1);
    int* e_cut = P.flags + 2 * (nf + 1);
    int* e_band = e_cut + (ne + 1);
    ClassArgs A{P.p, P.N1, P.N2, P.n1, P.n2, P.method, P.ecls, P.fcls, f_active, f_cut, e_cut, e_band};
    hipLaunchKernelGGL(k_fn_class, dim3((nf + 127) / 128), dim3(128), 0, s, A);
    hipLaunchKernelGGL(k_elem_flags, dim3((ne + 127) / 128), dim3(128), 0, s, A);
}

// --------------------------------------------------------------- lists
// The four compactions of the classes -- active functions (act_of, fn_of),
// rows formed element-wise (their compact ids), cut elements and band
// elements (id map and list) -- in one pass of three launches: per-tile
// counts of all four flag arrays, one scan of the tile counts, and per-tile
// positions with the writes. Lists come out in increasing flat order.
constexpr int kListTile = 1024;  // 256 threads x 4 items

struct ListArgs {
    const int* flag[4];  // f_active, f_cut (functions), e_cut, e_band (elements)
    int n[4];
    int* map[4];         // act_of, -, cut_id, band_id
    int* list[4];        // fn_of, form_rows (compact ids), cut_list, band_list
    int* bsum;           // [4][ntiles] tile counts, then tile offsets
    int ntiles;
    int* counts;         // [4] totals
};

__device__ __forceinline__ int block_sum256(int v, int* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    const int tot = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return tot;
}

__global__ void __launch_bounds__(256) k_list_count(ListArgs A) {
    __shared__ int sh[4];
    const int b = blockIdx.x, base = b * kListTile + threadIdx.x * 4;
    int c[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        c[a] = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) c[a] += (base + j < A.n[a]) ? (A.flag[a][base + j] != 0) : 0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int tot = block_sum256(c[a], sh);
        if (threadIdx.x == 0) A.bsum[a * A.ntiles + b] = tot;
    }
}

__global__ void __launch_bounds__(1024) k_list_scan(ListArgs A) {
    __shared__ int sh[1024 / 64 + 1];
    for (int a = 0; a < 4; ++a) {
        int carry = 0;
        for (int base = 0; base < A.ntiles; base += 1024) {
            const int idx = base + threadIdx.x;
            const int v = (idx < A.ntiles) ? A.bsum[a * A.ntiles + idx] : 0;
            int total;
            const int ex = block_excl_scan(v, sh, total);
            if (idx < A.ntiles) A.bsum[a * A.ntiles + idx] = ex + carry;
            carry += total;
        }
        if (threadIdx.x == 0) A.counts[a] = carry;
    }
}

__global__ void __launch_bounds__(256) k_list_write(ListArgs A) {
    __shared__ int sh[256 / 64 + 1];
    const int b = blockIdx.x, base = b * kListTile + threadIdx.x * 4;
    int fl[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j) fl[a][j] = (base + j < A.n[a]) ? (A.flag[a][base + j] != 0) : 0;
    int actpos[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int v = fl[a][0] + fl[a][1] + fl[a][2] + fl[a][3];
        int total;
        int pos = block_excl_scan(v, sh, total) + A.bsum[a * A.ntiles + b];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = base + j;
            if (i >= A.n[a]) continue;
            if (a == 0) actpos[j] = pos;
            if (A.map[a]) A.map[a][i] = fl[a][j] ? pos : -1;
            if (fl[a][j]) A.list[a][pos] = (a == 1) ? actpos[j] : i;
            pos += fl[a][j];
        }
    }
}

void launch_trim_lists(Plan& P, hipStream_t s) {
    const int nf = P.n1 * P.n2, ne = P.N1 * P.N2;
    int* f_active = P.flags;
    int* f_cut = P.flags + (nf + 1);
    int* e_cut = P.flags + 2 * (nf + 1);
    int* e_band = e_cut + (ne + 1);
    ListArgs A;
    A.flag[0] = f_active; A.flag[1] = f_cut; A.flag[2] = e_cut; A.flag[3] = e_band;
    A.n[0] = nf; A.n[1] = nf; A.n[2] = ne; A.n[3] = ne;
    A.map[0] = P.act_of; A.map[1] = nullptr; A.map[2] = P.cut_id; A.map[3] = P.band_id;
    A.list[0] = P.fn_of; A.list[1] = P.form_rows; A.list[2] = P.cut_list; A.list[3] = P.band_list;
    A.ntiles = (std::max(nf, ne) + kListTile - 1) / kListTile;
    A.bsum = P.scan_tmp + P.scan_pos_off;  // 4 * ntiles <= the position region
    A.counts = P.counts;
    hipLaunchKernelGGL(k_list_count, dim3(A.ntiles), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, s, A);
    hipLaunchKernelGGL(k_list_write, dim3(A.ntiles), dim3(256), 0, s, A);
}

// ------------------------------------------------------ arcs per element
__global__ void k_arc_count(TrimDev T, int N1, const int* __restrict__ cut_id, int* __restrict__ cnt) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= T.cap_arcs) return;
    const ArcDev A = T.arcs[a];
    if (A.keep) atomicAdd(&cnt[cut_id[A.e2 * N1 + A.e1]], 1);
}

__global__ void k_arc_fill(TrimDev T, int N1, const int* __restrict__ cut_id, const int* __restrict__ off,
                           int* __restrict__ fill, int* __restrict__ list) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= T.cap_arcs) return;
    const ArcDev A = T.arcs[a];
    if (!A.keep) return;
    int c = cut_id[A.e2 * N1 + A.e1];
    int slot = atomicAdd(&fill[c], 1);
    list[off[c] + slot] = a;
}

// Arc indices are already in (curve, segment, t) order; sort each element's list by index.
__global__ void k_arc_sort(int n_cut, const int* __restrict__ off, int* __restrict__ list) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cut) return;
    int lo = off[c], hi = off[c + 1];
    for (int a = lo + 1; a < hi; ++a) {
        int v = list[a], b = a - 1;
        while (b >= lo && list[b] > v) { list[b + 1] = list[b]; --b; }
        list[b + 1] = v;
    }
}

__global__ void k_zero_int(int* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_zero_int2(int* a, int* b, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        a[i] = 0;
        b[i] = 0;
    }
}

struct CutArgs {
    TrimDev T;
    GridDev G;
    int n_cut;
    const int* cut_list;
    const int* arc_off;
    const int* arc_list;
    CutElemDev* cut_el;
    int* node_cnt;
    int n_r, n_q_override, n_s, p;
    const double* gx;
    const double* gw;
    int* status;
};

__device__ __forceinline__ int arc_nq(const CutArgs& A, const CurveDev& C) {
    if (A.n_q_override > 0) return A.n_q_override;
    int d = (C.kind == IGA_CURVE_ELLIPSE) ? 3 : C.degree;
    return d * (2 * A.p + 1);
}

// One wavefront per cut element: lanes 0..3 build the visible pieces of the
// four edges; every lane adds its share of sum |w| of the four bases over the
// arcs' Gauss points; lane 0 picks the base and the node count.
__global__ void __launch_bounds__(64) k_cutprep(CutArgs A) {
    const int c = blockIdx.x;
    if (c >= A.n_cut) return;
    const TrimDev& T = A.T;
    const int lane = threadIdx.x;
    __shared__ double sLen[4];
    __shared__ int sOverflow;
    const int e = A.cut_list[c];
    const int e1 = e % A.G.N1, e2 = e / A.G.N1;
    const double xa = A.G.bp1[e1], xb = A.G.bp1[e1 + 1], ya = A.G.bp2[e2], yb = A.G.bp2[e2 + 1];
    const int alo = A.arc_off[c], ahi = A.arc_off[c + 1];
    CutElemDev& out = A.cut_el[c];
    if (lane == 0) sOverflow = 0;
    __syncthreads();
    if (lane < 4) {
        const int edge = lane;
        double cuts[kMaxEdgeCuts];
        int n = 0;
        bool overflow = false;
        for (int q = alo; q < ahi; ++q) {
            const ArcDev R = T.arcs[A.arc_list[q]];
            const SegDev S = T.segs[T.pieces[R.piece].seg];
            for (int end = 0; end < 2; ++end) {
                int kind = end ? R.k1 : R.k0, line = end ? R.l1 : R.l0;
                double X, Y, dX, dY;
                seg_eval(S, end ? R.t1 : R.t0, X, Y, dX, dY);
                bool on = false;
                if (kind == END_VLINE) on = (line == e1 + (edge == 1)) && edge < 2;
                else if (kind == END_HLINE) on = (line == e2 + (edge == 3)) && edge >= 2;
                else {
                    // a piece end (extremum or segment junction) that lies on a grid line: the
                    // half-open crossing count gives that crossing to the neighbouring piece only
                    const double ref = (edge == 0) ? xa : (edge == 1) ? xb : (edge == 2) ? ya : yb;
                    const double h = (edge < 2) ? xb - xa : yb - ya;
                    on = fabs(((edge < 2) ? X : Y) - ref) <= 1e-12 * h;
                }
                if (!on) continue;
                if (n < kMaxEdgeCuts) cuts[n++] = (edge < 2) ? Y : X;
                else overflow = true;
            }
        }
        for (int a = 1; a < n; ++a) {
            double v = cuts[a];
            int b = a - 1;
            while (b >= 0 && cuts[b] > v) { cuts[b + 1] = cuts[b]; --b; }
            cuts[b + 1] = v;
        }
        const double lo = (edge < 2) ? ya : xa, hi = (edge < 2) ? yb : xb;
        const double fixed = (edge == 0) ? xa : (edge == 1) ? xb : (edge == 2) ? ya : yb;
        const double tol = 1e-13 * (hi - lo);
        int ns = 0;
        double prev = lo, len = 0.0, last_hi = 0.0;
        for (int q = 0; q <= n; ++q) {
            double a = prev;
            double b = (q == n) ? hi : fmin(fmax(cuts[q], lo), hi);
            prev = b;
            if (b - a <= tol) continue;
            double m = 0.5 * (a + b);
            double x = (edge < 2) ? fixed : m, y = (edge < 2) ? m : fixed;
            if (in_any_hole(T, x, y)) continue;
            if (ns > 0 && fabs(last_hi - a) <= tol) {
                out.seg[edge][ns - 1][1] = b;
            } else if (ns < kMaxEdgeSegs) {
                out.seg[edge][ns][0] = a;
                out.seg[edge][ns][1] = b;
                ++ns;
            } else {
                overflow = true;
                continue;
            }
            last_hi = b;
            len += b - a;
        }
        out.nseg[edge] = ns;
        sLen[edge] = len;
        if (overflow) sOverflow = 1;
    }
    // sum |w| of the four bases over the arcs' Gauss points
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int narc_nodes = 0;
    for (int q = alo; q < ahi; ++q) {
        const ArcDev R = T.arcs[A.arc_list[q]];
        const SegDev S = T.segs[T.pieces[R.piece].seg];
        const int nq = arc_nq(A, T.curves[R.curve]);
        narc_nodes += nq * A.n_r;
        for (int g = lane; g < nq; g += 64) {
            double tq = R.t0 + (R.t1 - R.t0) * (A.gx[gauss_off(nq) + g] + 1.0) * 0.5;
            double wt = A.gw[gauss_off(nq) + g] * (R.t1 - R.t0) * 0.5;
            double X, Y, dX, dY;
            seg_eval(S, tq, X, Y, dX, dY);
            s0 += wt * fabs(dY) * fabs(X - xa);
            s1 += wt * fabs(dY) * fabs(X - xb);
            s2 += wt * fabs(dX) * fabs(Y - ya);
            s3 += wt * fabs(dX) * fabs(Y - yb);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
        s3 += __shfl_xor(s3, o, 64);
    }
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
        A.node_cnt[c] = narc_nodes + out.nseg[opp] * A.n_s * A.n_r;
        if (sOverflow) atomicExch(A.status, IGA_E_TOPOLOGY);
    }
}

void launch_trim_cutprep(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    int nc = (int)P.n_cut_el;
    if (T.n_curves == 0 || nc == 0) return;
    GridDev G{P.dir[0].bp, P.dir[1].bp, P.N1, P.N2};
    hipLaunchKernelGGL(k_zero_int2, dim3((nc + 1 + 127) / 128), dim3(128), 0, s, P.arc_cnt, P.arc_fill, nc + 1);
    hipLaunchKernelGGL(k_arc_count, dim3((T.cap_arcs + 127) / 128), dim3(128), 0, s, T, P.N1, P.cut_id, P.arc_cnt);
    exclusive_scan(P.arc_cnt, P.arc_off, nc, P.scan_tmp, s);
    hipLaunchKernelGGL(k_arc_fill, dim3((T.cap_arcs + 127) / 128), dim3(128), 0, s, T, P.N1, P.cut_id, P.arc_off,
                       P.arc_fill, P.arc_list);
    hipLaunchKernelGGL(k_arc_sort, dim3((nc + 127) / 128), dim3(128), 0, s, nc, P.arc_off, P.arc_list);
    CutArgs A{T, G, nc, P.cut_list, P.arc_off, P.arc_list, P.cut_el, P.node_cnt,
              P.n_r, P.n_q_override, P.n_s, P.p, P.gauss_x, P.gauss_w, P.status};
    hipLaunchKernelGGL(k_cutprep, dim3(nc), dim3(64), 0, s, A);
    exclusive_scan(P.node_cnt, P.node_off, nc, P.scan_tmp, s);
}

// One wavefront per cut element writes its nodes.
__global__ void __launch_bounds__(64) k_cut_nodes(CutArgs A, const int* __restrict__ node_off, double* __restrict__ nx,
                                                  double* __restrict__ ny, double* __restrict__ nw,
                                                  int* __restrict__ nel) {
    int c = blockIdx.x;
    if (c >= A.n_cut) return;
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
    int pos = node_off[c];
    for (int q = A.arc_off[c]; q < A.arc_off[c + 1]; ++q) {
        const ArcDev R = T.arcs[A.arc_list[q]];
        const SegDev S = T.segs[T.pieces[R.piece].seg];
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
                if (vert) {
                    nx[o] = b0 + (X - b0) * f;
                    ny[o] = Y;
                    nw[o] = C.sigma * wt * dY * rw[r] * (X - b0) * 0.5;
                } else {
                    nx[o] = X;
                    ny[o] = b0 + (Y - b0) * f;
                    nw[o] = -C.sigma * wt * dX * rw[r] * (Y - b0) * 0.5;
                }
                nel[o] = c;
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
        }
        pos += ns * nr;
    }
}

void launch_trim_nodes(Plan& P, hipStream_t s) {
    TrimDev& T = P.trim;
    int nc = (int)P.n_cut_el;
    if (T.n_curves == 0 || nc == 0) return;
    GridDev G{P.dir[0].bp, P.dir[1].bp, P.N1, P.N2};
    CutArgs A{T, G, nc, P.cut_list, P.arc_off, P.arc_list, P.cut_el, P.node_cnt,
              P.n_r, P.n_q_override, P.n_s, P.p, P.gauss_x, P.gauss_w, P.status};
    hipLaunchKernelGGL(k_cut_nodes, dim3(nc), dim3(64), 0, s, A, P.node_off, P.node_x, P.node_y, P.node_w, P.node_el);
}

}  // namespace iga

namespace iga {

// Orientation of each curve: sign of (1/2) closed integral of (x dy - y dx),
// exact by Gauss on each polynomial segment; a hole traversed with the
// visible domain on its left is clockwise, so sigma = -1 for a
// counter-clockwise native orientation.
__global__ void __launch_bounds__(64) k_orientation(TrimDev T, CurveDev* __restrict__ curves,
                                                    const double* __restrict__ gx, const double* __restrict__ gw) {
    int c = blockIdx.x;
    if (c >= T.n_curves) return;
    CurveDev C = curves[c];
    double area = 0.0;
    const int ng = 8;
    for (int s = threadIdx.x; s < C.n_seg; s += 64) {
        const SegDev S = T.segs[C.seg0 + s];
        for (int g = 0; g < ng; ++g) {
            double t = C.t_range * (gx[gauss_off(ng) + g] + 1.0) * 0.5;
            double w = gw[gauss_off(ng) + g] * C.t_range * 0.5;
            double X, Y, dX, dY;
            seg_eval(S, t, X, Y, dX, dY);
            area += 0.5 * w * (X * dY - Y * dX);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) area += __shfl_xor(area, o, 64);
    if (threadIdx.x == 0) curves[c].sigma = (area > 0.0) ? -1.0 : 1.0;
}

void launch_orientation(Plan& P, hipStream_t s) {
    if (P.trim.n_curves == 0) return;
    hipLaunchKernelGGL(k_orientation, dim3(P.trim.n_curves), dim3(64), 0, s, P.trim, P.d_curves, P.gauss_x,
                       P.gauss_w);
}

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
    hipLaunchKernelGGL(k_naive_mask, dim3((nq + 255) / 256), dim3(256), 0, s, P.trim, P.dir[0], P.dir[1], src, cval,
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
