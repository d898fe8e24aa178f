// Extended B-spline stabilisation of the trimmed basis, applied to the L2
// projection (Sect. 2.2, closing remarks, and Sect. 4.2: the paper takes the
// construction from the weighted extended B-splines of the works it cites).
//
//  * inner functions are active with an inside element in their support; the
//    others (outer) see cut elements only, and can be cut to a sliver;
//  * each outer function j is tied to the block {l1..l1+p} x {l2..l2+p} of
//    inner functions whose centre l + p/2 is nearest to j (squared index
//    distance, ties to the smaller l2, then the smaller l1);
//  * per direction the block's weights reproduce j's B-spline coefficient of
//    every polynomial of degree p; the coefficient is the polynomial's blossom
//    at j's knot window, so the weights are the blossoms of the block
//    functions' polynomial pieces on their common element (de Boor's
//    algorithm with the window as arguments);
//  * E[i, j] = 1 (j = i inner) or e_{i,j} = e^1 e^2 (j outer, i in its block);
//    the projection solves (E A E^T) x = E b, A = (M + M^T)/2, by
//    Jacobi-preconditioned CG and returns u = E^T x.
//
// The extended vectors live in the compact row space with zeros at the outer
// rows, so the band operator, the reductions and the CG steps are those of
// the plain projection. E^T is a gather over each outer row's block, E a
// gather over each inner row's list of the outer rows tied to it; the lists
// are sorted, so every sum runs in a fixed order and a solve is bitwise
// reproducible. An iteration is three launches, as in the plain solver: the
// band product of z = E^T p with the partials of p.q = z.(A z); the update,
// which forms q = E (A z) row by row; the direction, which also forms E^T of
// the new direction (from E^T z and E^T of the old one).
#include <cmath>

#include "solve_body.hpp"

namespace iga {

namespace {

enum : int { kExtNoBlock = 1, kExtSingular = 2, kExtCapacity = 3 };

struct ExtArgs {
    int p, n1, n2, n_act, cap;
    const int* fn_of;
    const int* act_of;
    const double* t1;   // knot vectors
    const double* t2;
    int8_t* inner;
    int8_t* ok;
    int* slot;
    int* cnt;
    int* off;
    int* misc;
    int* row;
    int* fid;
    double* fw;
    int* tj;
    double* tw;
};

// Inner flag of every function; resets the per-row tables of the active rows.
__global__ void k_ext_mark(ExtArgs X, int N1, int N2, const int8_t* __restrict__ ecls) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) {
        X.misc[0] = 0;
        X.misc[1] = 0;
    }
    if (f >= X.n1 * X.n2) return;
    const int p = X.p, i1 = f % X.n1, i2 = f / X.n1, a = X.act_of[f];
    bool in = false;
    if (a >= 0) {
        for (int e2 = max(0, i2 - p); e2 <= min(N2 - 1, i2); ++e2)
            for (int e1 = max(0, i1 - p); e1 <= min(N1 - 1, i1); ++e1) in |= ecls[e2 * N1 + e1] == EL_INSIDE;
        X.slot[a] = -1;
        X.cnt[a] = 0;
    }
    X.inner[f] = in;
}

// Blocks whose (p+1)^2 functions are all inner.
__global__ void k_ext_blocks(ExtArgs X) {
    const int nb1 = X.n1 - X.p, nb2 = X.n2 - X.p;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb1 * nb2) return;
    const int l1 = t % nb1, l2 = t / nb1;
    bool all = true;
    for (int m2 = 0; m2 <= X.p; ++m2)
        for (int m1 = 0; m1 <= X.p; ++m1) all &= X.inner[(l2 + m2) * X.n1 + l1 + m1] != 0;
    X.ok[t] = all;
}

// The all-inner block nearest to j, searched in windows of the blocks whose
// centre is within R of j per coordinate: once the best of a window is within
// R, no block outside it is as near. Scanning l2, then l1, upwards and taking
// only strictly nearer blocks keeps the tie rule. False if there is none.
__device__ bool nearest_block(const int8_t* __restrict__ ok, int nb1, int nb2, int p, int j1, int j2, int& l1o,
                              int& l2o) {
    for (int R = p;;) {
        long long best = -1;
        const int lo2 = max(0, j2 - R - p), hi2 = min(nb2 - 1, j2 + R);
        const int lo1 = max(0, j1 - R - p), hi1 = min(nb1 - 1, j1 + R);
        for (int l2 = lo2; l2 <= hi2; ++l2) {
            const int d2 = 2 * l2 + p - 2 * j2;
            if (d2 > 2 * R || d2 < -2 * R) continue;
            for (int l1 = lo1; l1 <= hi1; ++l1) {
                const int d1 = 2 * l1 + p - 2 * j1;
                if (d1 > 2 * R || d1 < -2 * R || !ok[l2 * nb1 + l1]) continue;
                const long long d = (long long)d1 * d1 + (long long)d2 * d2;
                if (best < 0 || d < best) {
                    best = d;
                    l1o = l1;
                    l2o = l2;
                }
            }
        }
        if (best >= 0 && best <= 4LL * R * R) return true;
        if (best < 0) {
            const bool all1 = 2 * R >= max(abs(p - 2 * j1), abs(2 * (nb1 - 1) + p - 2 * j1));
            const bool all2 = 2 * R >= max(abs(p - 2 * j2), abs(2 * (nb2 - 1) + p - 2 * j2));
            if (all1 && all2) return false;
            R *= 2;
        } else {
            int r = (int)sqrt((double)best) / 2;
            while (4LL * r * r < best) ++r;
            R = max(2 * R, r);
        }
    }
}

// Weights e_0..e_P of the functions l..l+P that reproduce B_j's coefficient of
// every polynomial of degree P. The B-spline coefficient of a polynomial is its
// blossom at the function's knot window (t_{j+1}, ..., t_{j+P}); the functions
// l..l+P are all nonzero on the element [t_{l+P}, t_{l+P+1}], where their
// polynomial pieces q_0..q_P have de Boor points e_0..e_P (unit vectors), and
// each q_n has coefficient 1 on B_{l+n} and 0 on the block's other functions,
// so e_n = lambda_j(q_n) = blossom of q_n at j's window: de Boor's algorithm on
// the unit vectors with argument t_{j+r} at level r. The same weights as the
// reproduction conditions solved exactly, without their conditioning (which
// reaches 1e7 at P = 8 even on scaled monomials): the steps are affine
// combinations, extrapolating only as far as j lies from the element.
template <int P>
__device__ bool ext_weights(const double* __restrict__ t, int j, int l, double* e) {
    double d[P + 1][P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
#pragma unroll
        for (int n = 0; n <= P; ++n) d[i][n] = (i == n) ? 1.0 : 0.0;
    for (int r = 1; r <= P; ++r) {
        const double u = t[j + r];
        for (int i = P; i >= r; --i) {   // descending: d[i - 1] still holds level r - 1
            const double lo = t[l + i], hi = t[l + i + P + 1 - r];
            if (!(hi > lo)) return false;
            const double a = (u - lo) / (hi - lo);
#pragma unroll
            for (int n = 0; n <= P; ++n) d[i][n] = (1.0 - a) * d[i - 1][n] + a * d[i][n];
        }
    }
#pragma unroll
    for (int n = 0; n <= P; ++n) e[n] = d[P][n];
    return true;
}

// Block and weights of every outer row (one thread per compact row); counts
// the outer rows tied to each inner row.
template <int P>
__global__ void k_ext_fwd(ExtArgs X) {
    constexpr int L = (P + 1) * (P + 1);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= X.n_act) return;
    const int f = X.fn_of[r];
    if (X.inner[f]) return;
    const int j1 = f % X.n1, j2 = f / X.n1;
    int l1 = 0, l2 = 0;
    if (!nearest_block(X.ok, X.n1 - P, X.n2 - P, P, j1, j2, l1, l2)) {
        atomicExch(X.misc + 1, kExtNoBlock);
        return;
    }
    double w1[P + 1], w2[P + 1];
    if (!ext_weights<P>(X.t1, j1, l1, w1) || !ext_weights<P>(X.t2, j2, l2, w2)) {
        atomicExch(X.misc + 1, kExtSingular);
        return;
    }
    const int s = atomicAdd(X.misc, 1);
    if (s >= X.cap) {
        atomicExch(X.misc + 1, kExtCapacity);
        return;
    }
    X.slot[r] = s;
    X.row[s] = r;
    for (int m2 = 0; m2 <= P; ++m2)
        for (int m1 = 0; m1 <= P; ++m1) {
            const int id = X.act_of[(l2 + m2) * X.n1 + l1 + m1];
            const size_t o = (size_t)s * L + m2 * (P + 1) + m1;
            X.fid[o] = id;
            X.fw[o] = w1[m1] * w2[m2];
            atomicAdd(X.cnt + id, 1);
        }
}

// Lists of the outer rows tied to each inner row (positions from the counts,
// which run back to zero).
__global__ void k_ext_fill(ExtArgs X) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= min(X.cap, X.misc[0])) return;
    const int L = (X.p + 1) * (X.p + 1), r = X.row[s];
    for (int m = 0; m < L; ++m) {
        const int id = X.fid[(size_t)s * L + m];
        const int pos = X.off[id] + atomicSub(X.cnt + id, 1) - 1;
        X.tj[pos] = r;
        X.tw[pos] = X.fw[(size_t)s * L + m];
    }
}

// Each inner row's list in ascending order of the outer rows.
__global__ void k_ext_sort(ExtArgs X) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= X.n_act || X.slot[r] >= 0) return;
    const int b = X.off[r], e = X.off[r + 1];
    for (int k = b + 1; k < e; ++k) {
        const int key = X.tj[k];
        const double w = X.tw[k];
        int m = k - 1;
        while (m >= b && X.tj[m] > key) {
            X.tj[m + 1] = X.tj[m];
            X.tw[m + 1] = X.tw[m];
            --m;
        }
        X.tj[m + 1] = key;
        X.tw[m + 1] = w;
    }
}

// Diagonal of E A E^T: row i's terms e_x e_y A_xy over x, y in {i} and its
// list (1 at outer rows, whose unknowns stay zero).
__global__ void k_ext_diag(ExtArgs X, SpArgs S, double* __restrict__ dg) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= X.n_act) return;
    if (X.slot[r] >= 0) {
        dg[r] = 1.0;
        return;
    }
    const int p = X.p, W = 2 * p + 1, b = X.off[r], e = X.off[r + 1];
    double d = 0.0;
    for (int x = b - 1; x < e; ++x) {
        const int cx = (x < b) ? r : X.tj[x];
        const double ex = (x < b) ? 1.0 : X.tw[x];
        const int fx = X.fn_of[cx], x1 = fx % X.n1, x2 = fx / X.n1;
        double s = 0.0;
        for (int y = b - 1; y < e; ++y) {
            const int cy = (y < b) ? r : X.tj[y];
            const double ey = (y < b) ? 1.0 : X.tw[y];
            const int fy = X.fn_of[cy], da = fy % X.n1 - x1, db = fy / X.n1 - x2;
            if (da >= -p && da <= p && db >= -p && db <= p)
                s += ey * S.A[(size_t)((da + p) * W + (db + p)) * X.n_act + cx];
        }
        d += ex * s;
    }
    dg[r] = d;
}

// Columns of E, row by row of E^T: members[r][m], weights[r][m] (inner rows:
// the row itself with weight 1, then -1 / 0).
__global__ void k_ext_export(ExtArgs X, int32_t* __restrict__ members, double* __restrict__ weights) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= X.n_act) return;
    const int L = (X.p + 1) * (X.p + 1), s = X.slot[r];
    for (int m = 0; m < L; ++m) {
        const size_t o = (size_t)r * L + m;
        if (s < 0) {
            members[o] = m == 0 ? r : -1;
            weights[o] = m == 0 ? 1.0 : 0.0;
        } else {
            members[o] = X.fid[(size_t)s * L + m];
            weights[o] = X.fw[(size_t)s * L + m];
        }
    }
}

// Start of the extended unknowns: the start vector's inner coefficients.
__global__ void k_ext_start(ExtArgs X, const double* __restrict__ u, double* __restrict__ x) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < X.n_act) x[r] = X.slot[r] < 0 ? u[r] : 0.0;
}

// z = E^T x: inner rows copy, outer rows gather their block.
__global__ void k_ext_t(ExtArgs X, const double* __restrict__ x, double* __restrict__ z) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= X.n_act) return;
    const int s = X.slot[r];
    if (s < 0) {
        z[r] = x[r];
        return;
    }
    const int L = (X.p + 1) * (X.p + 1);
    double v = 0.0;
    for (int m = 0; m < L; ++m) v += X.fw[(size_t)s * L + m] * x[X.fid[(size_t)s * L + m]];
    z[r] = v;
}

// w = A z; with part, the block partial of (z . w) at part[block] (z = E^T p: p.q of the extended system).
template <int P>
__global__ void __launch_bounds__(kRedThreads) k_ext_spmv(SpArgs S, const double* __restrict__ z,
                                                          double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    const int r = blockIdx.x * kRedThreads + threadIdx.x;
    double zw = 0.0;
    if (r < S.n_act) {
        const double v = spmv_row_cols<P>(S, z, r);
        w[r] = v;
        zw = z[r] * v;
    }
    if (part) {
        const double s = block_sum(zw, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

// Row r of E w (zero at outer rows). The list is read eight entries at a
// time, every load of a chunk issued before its sums (padding adds zeros).
__device__ __forceinline__ double ext_e_row(const ExtArgs& X, const double* __restrict__ w, int r) {
    if (X.slot[r] >= 0) return 0.0;
    double v = w[r];
    const int b = X.off[r], e = X.off[r + 1];
    for (int k0 = b; k0 < e; k0 += 8) {
        int j[8];
        double t[8], wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = min(k0 + u, e - 1);
            j[u] = X.tj[k];
            t[u] = (k0 + u < e) ? X.tw[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) wv[u] = w[j[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u] * wv[u];
    }
    return v;
}

// q = E w.
__global__ void k_ext_e(ExtArgs X, const double* __restrict__ w, double* __restrict__ q) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < X.n_act) q[r] = ext_e_row(X, w, r);
}

// r = b - q (q = E A E^T x), z = r/d, p = z; partials of (r.z), (r.r), (b.b).
__global__ void __launch_bounds__(kRedThreads) k_ext_init(SpArgs S, const double* __restrict__ bvec,
                                                          const double* __restrict__ q, double* __restrict__ rv,
                                                          double* __restrict__ zv, double* __restrict__ pv,
                                                          double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    const int r = blockIdx.x * kRedThreads + threadIdx.x;
    double rz = 0, rr = 0, bb = 0;
    if (r < S.n_act) {
        const double res = bvec[r] - q[r];
        const double z = res / diag_of(S, r);
        rv[r] = res;
        zv[r] = z;
        pv[r] = z;
        rz = res * z;
        rr = res * res;
        bb = bvec[r] * bvec[r];
    }
    const double s0 = block_sum(rz, sh), s1 = block_sum(rr, sh), s2 = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0;
        part[3 * blockIdx.x + 1] = s1;
        part[3 * blockIdx.x + 2] = s2;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_ext_reduce(const double* __restrict__ part, int nblk,
                                                            double* __restrict__ scal) {
    __shared__ double sh[kRedThreads / 64];
    cg_reduce0(part, nblk, scal, sh);
}

// alpha = (r.z) / (p.q) from the product's partials (summed by every block in
// the same order); q = E w, x += alpha p, r -= alpha q, z = r/d; partials of
// (r.z), (r.r) at part[2 block ..]. The row's loads, E w among them, do not
// depend on alpha and are issued before the partials are summed.
__global__ void __launch_bounds__(kRedThreads) k_ext_update(ExtArgs X, SpArgs S, const double* __restrict__ scal,
                                                            int par, int nblk, const double* __restrict__ part_pq,
                                                            const double* __restrict__ w, double* __restrict__ x,
                                                            double* __restrict__ rv, double* __restrict__ zv,
                                                            const double* __restrict__ pv, double* __restrict__ part) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_alpha;
    const int r = blockIdx.x * kRedThreads + threadIdx.x;
    const bool act = r < X.n_act;
    double pp = 0.0;  // this thread's share of the partials, loaded first
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) pp += part_pq[k];
    double q = 0.0, pr = 0.0, rr0 = 0.0, xr = 0.0, d = 1.0;
    if (act) {
        q = ext_e_row(X, w, r);
        pr = pv[r];
        rr0 = rv[r];
        xr = x[r];
        d = diag_of(S, r);
    }
    const double pq = block_sum(pp, sh);
    if (threadIdx.x == 0) s_alpha = (pq != 0.0) ? scal[6 + par] / pq : 0.0;
    __syncthreads();
    double rz = 0, rr = 0;
    if (act) {
        const double alpha = s_alpha;
        x[r] = xr + alpha * pr;
        const double res = rr0 - alpha * q;
        const double z = res / d;
        rv[r] = res;
        zv[r] = z;
        rz = res * z;
        rr = res * res;
    }
    const double s0 = block_sum(rz, sh), s1 = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0;
        part[2 * blockIdx.x + 1] = s1;
    }
}

// beta = (r.z)_new / (r.z)_old; p_new = z + beta p_old (into the other buffer)
// and zp = E^T p_new, at an outer row as (E^T z) + beta (E^T p_old): both sums
// are read before beta is known, with the row's own loads, while the partials
// are summed. Block 0 stores the new (r.z) and (r.r).
template <int P>
__global__ void __launch_bounds__(kRedThreads) k_ext_dir(ExtArgs X, double* __restrict__ scal, int par, int nblk,
                                                         const double* __restrict__ part,
                                                         const double* __restrict__ zv,
                                                         const double* __restrict__ p_old, double* __restrict__ p_new,
                                                         double* __restrict__ zp) {
    __shared__ double sh[kRedThreads / 64];
    __shared__ double s_beta;
    constexpr int L = (P + 1) * (P + 1);
    const int r = blockIdx.x * kRedThreads + threadIdx.x;
    const bool act = r < X.n_act;
    double prz = 0.0, prr = 0.0;  // this thread's share of the partials, loaded first
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
        prz += part[2 * k];
        prr += part[2 * k + 1];
    }
    int s = -1;
    double zr = 0.0, pr = 0.0, ez = 0.0, ep = 0.0;
    if (act) {
        zr = zv[r];
        pr = p_old[r];
        s = X.slot[r];
        if (s >= 0) {
#pragma unroll
            for (int m0 = 0; m0 < L; m0 += P + 1) {
                int id[P + 1];
                double wv[P + 1];
#pragma unroll
                for (int m = 0; m <= P; ++m) {
                    id[m] = X.fid[(size_t)s * L + m0 + m];
                    wv[m] = X.fw[(size_t)s * L + m0 + m];
                }
#pragma unroll
                for (int m = 0; m <= P; ++m) {
                    ez += wv[m] * zv[id[m]];
                    ep += wv[m] * p_old[id[m]];
                }
            }
        }
    }
    const double rz = block_sum(prz, sh);
    const double rr = block_sum(prr, sh);
    if (threadIdx.x == 0) {
        s_beta = (scal[6 + par] != 0.0) ? rz / scal[6 + par] : 0.0;
        if (blockIdx.x == 0) {
            scal[6 + (1 - par)] = rz;
            scal[2] = rr;
        }
    }
    __syncthreads();
    if (!act) return;
    const double beta = s_beta;
    const double pn = zr + beta * pr;
    p_new[r] = pn;
    zp[r] = (s < 0) ? pn : ez + beta * ep;
}

inline dim3 grid_of(int64_t n, int threads) { return dim3((unsigned)std::max<int64_t>(1, (n + threads - 1) / threads)); }

void ext_buffers(Plan& P) {
    SolveWork& W = P.sw;
    if (W.x_inner) return;
    const int n = (int)P.n_act, nf = P.n1 * P.n2, L = (P.p + 1) * (P.p + 1);
    W.x_cap = (int)std::max<int64_t>(1, P.n_act - P.n_interior);
    W.x_inner = P.alloc<int8_t>(nf);
    W.x_ok = P.alloc<int8_t>((size_t)(P.n1 - P.p) * (P.n2 - P.p));
    W.x_slot = P.alloc<int>(n);
    W.x_cnt = P.alloc<int>(n + 1);
    W.x_off = P.alloc<int>(n + 1);
    W.x_misc = P.alloc<int>(2);
    W.x_row = P.alloc<int>(W.x_cap);
    W.x_fid = P.alloc<int>((size_t)W.x_cap * L);
    W.x_fw = P.alloc<double>((size_t)W.x_cap * L);
    W.x_tj = P.alloc<int>((size_t)W.x_cap * L);
    W.x_tw = P.alloc<double>((size_t)W.x_cap * L);
    W.x_dg = P.alloc<double>(n);
    W.x_e = P.alloc<double>(n);
    W.x_z = P.alloc<double>(n);
    W.x_w = P.alloc<double>(n);
    W.x_b = P.alloc<double>(n);
    W.x_p = P.alloc<double>(n);
}

ExtArgs ext_args(Plan& P) {
    SolveWork& W = P.sw;
    return ExtArgs{P.p,      P.n1,     P.n2,     (int)P.n_act, W.x_cap, P.fn_of,  P.act_of,
                   P.dir[0].knots, P.dir[1].knots, W.x_inner, W.x_ok, W.x_slot, W.x_cnt, W.x_off,
                   W.x_misc, W.x_row, W.x_fid, W.x_fw, W.x_tj, W.x_tw};
}

// Blocks and weights of the outer rows from the plan's element classes as
// they stand (the last set-up), and with `lists` each inner row's sorted list.
void ext_build(Plan& P, const ExtArgs& X, bool lists, hipStream_t s) {
    const int nf = P.n1 * P.n2, n = (int)P.n_act;
    hipLaunchKernelGGL(k_ext_mark, grid_of(nf, 256), dim3(256), 0, s, X, P.N1, P.N2, (const int8_t*)P.ecls);
    hipLaunchKernelGGL(k_ext_blocks, grid_of((int64_t)(P.n1 - P.p) * (P.n2 - P.p), 256), dim3(256), 0, s, X);
    switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_ext_fwd<PP>, grid_of(n, 128), dim3(128), 0, s, X); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
    if (!lists) return;
    exclusive_scan(X.cnt, X.off, n, P.scan_tmp, s);
    hipLaunchKernelGGL(k_ext_fill, grid_of(X.cap, 256), dim3(256), 0, s, X);
    hipLaunchKernelGGL(k_ext_sort, grid_of(n, 256), dim3(256), 0, s, X);
}

void ext_spmv(Plan& P, const SpArgs& S, const double* z, double* w, double* part, hipStream_t s) {
    switch (P.p) {
#define CASE(PP) \
    case PP: hipLaunchKernelGGL(k_ext_spmv<PP>, grid_of(S.n_act, kRedThreads), dim3(kRedThreads), 0, s, S, z, w, part); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
}

void ext_check(int err) {
    if (err == kExtNoBlock)
        throw Error{IGA_E_TOPOLOGY, "an outer function has no block of (p+1)^2 inner functions"};
    if (err == kExtSingular) throw Error{IGA_E_SINGULAR_WEIGHTS, "an extension weight system is singular"};
    if (err == kExtCapacity) throw Error{IGA_E_CAPACITY, "more outer functions than the plan reserved"};
}

// out = E A E^T in (extended vectors).
void ext_apply(Plan& P, const ExtArgs& X, const SpArgs& S, const double* in, double* out, hipStream_t s) {
    SolveWork& W = P.sw;
    const int n = (int)P.n_act;
    hipLaunchKernelGGL(k_ext_t, grid_of(n, 256), dim3(256), 0, s, X, in, W.x_z);
    ext_spmv(P, S, W.x_z, W.x_w, nullptr, s);
    hipLaunchKernelGGL(k_ext_e, grid_of(n, 256), dim3(256), 0, s, X, (const double*)W.x_w, out);
}

}  // namespace
}  // namespace iga

using namespace iga;

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

int iga_trim_extension(iga_plan* plan, int32_t* members, double* weights, void* stream) {
    API_BEGIN
    Plan* P = plan;
    IGA_REQUIRE(P && members && weights, IGA_E_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    ext_buffers(*P);
    const ExtArgs X = ext_args(*P);
    ext_build(*P, X, false, s);
    hipLaunchKernelGGL(k_ext_export, grid_of(P->n_act, 256), dim3(256), 0, s, X, members, weights);
    int err = 0;
    HIPX(hipMemcpyAsync(&err, X.misc + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    HIPX(hipGetLastError());
    ext_check(err);
    API_END
}

int iga_trim_l2_project_ext(iga_plan* plan, const iga_coeff* c, const double* vals, const iga_target* g, double rtol,
                            int32_t maxit, double* u, iga_solve_info* info, void* stream) {
    API_BEGIN
    Plan* P = plan;
    IGA_REQUIRE(P && c && vals && g && u, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(rtol > 0 && maxit > 0, IGA_E_INVALID, "rtol and maxit must be positive");
    rhs_check(*P, *c, *g);
    hipStream_t s = (hipStream_t)stream;
    SolveWork& W = P->sw;
    const int n = (int)P->n_act;
    const int nblk = (n + kRedThreads - 1) / kRedThreads;
    solve_buffers(*P);
    ext_buffers(*P);
    rhs(*P, *c, *g, W.b, s);
    SpArgs S = solve_operator(*P, vals, s);
    const ExtArgs X = ext_args(*P);
    ext_build(*P, X, true, s);
    hipLaunchKernelGGL(k_ext_diag, grid_of(n, 256), dim3(256), 0, s, X, S, W.x_dg);
    S.dg = W.x_dg;
    hipLaunchKernelGGL(k_ext_start, grid_of(n, 256), dim3(256), 0, s, X, (const double*)u, W.x_e);
    ext_apply(*P, X, S, W.x_e, W.q, s);
    hipLaunchKernelGGL(k_ext_e, grid_of(n, 256), dim3(256), 0, s, X, (const double*)W.b, W.x_b);
    hipLaunchKernelGGL(k_ext_init, grid_of(n, kRedThreads), dim3(kRedThreads), 0, s, S, (const double*)W.x_b,
                       (const double*)W.q, W.r, W.z, W.pv, W.part);
    hipLaunchKernelGGL(k_ext_reduce, dim3(1), dim3(kRedThreads), 0, s, (const double*)W.part, nblk, W.scal);
    hipLaunchKernelGGL(k_ext_t, grid_of(n, 256), dim3(256), 0, s, X, (const double*)W.pv, W.x_z);
    int err = 0;
    auto read = [&]() {
        HIPX(hipMemcpyAsync(W.h_scal, W.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
    };
    HIPX(hipMemcpyAsync(&err, X.misc + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    read();
    ext_check(err);
    const double bnorm = std::sqrt(W.h_scal[3]);
    double rel = (bnorm > 0) ? std::sqrt(W.h_scal[2]) / bnorm : 0.0;
    int it = 0;
    bool conv = rel <= rtol;
    // directions alternate between two buffers: iteration k reads pbuf[k & 1], writes pbuf[1 - (k & 1)]
    double* pbuf[2] = {W.pv, W.x_p};
    while (!conv && it < maxit) {
        const int m = std::min(kCgCheck, maxit - it);
        for (int k = 0; k < m; ++k) {
            const int par = (it + k) & 1;
            double* part2 = W.part + nblk;
            ext_spmv(*P, S, W.x_z, W.x_w, W.part, s);
            hipLaunchKernelGGL(k_ext_update, dim3(nblk), dim3(kRedThreads), 0, s, X, S, (const double*)W.scal, par,
                               nblk, (const double*)W.part, (const double*)W.x_w, W.x_e, W.r, W.z,
                               (const double*)pbuf[par], part2);
            switch (P->p) {
#define CASE(PP)                                                                                                \
    case PP:                                                                                                    \
        hipLaunchKernelGGL(k_ext_dir<PP>, dim3(nblk), dim3(kRedThreads), 0, s, X, W.scal, par, nblk,           \
                           (const double*)part2, (const double*)W.z, (const double*)pbuf[par], pbuf[1 - par], \
                           W.x_z);                                                                              \
        break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
            }
        }
        it += m;
        read();
        rel = (bnorm > 0) ? std::sqrt(W.h_scal[2]) / bnorm : 0.0;
        conv = rel <= rtol;
    }
    hipLaunchKernelGGL(k_ext_t, grid_of(n, 256), dim3(256), 0, s, X, (const double*)W.x_e, u);
    if (info) {
        info->iterations = it;
        info->converged = conv;
        info->rel_residual = rel;
    }
    HIPX(hipStreamSynchronize(s));
    HIPX(hipGetLastError());
    if (!conv) {
        set_error("PCG did not reach the tolerance");
        return IGA_E_NOCONV;
    }
    API_END
}

}  // extern "C"
