// getBasis (Section 4.1, Eqs. SRRQR1-2) as a batched interpolative
// decomposition, and the bottom-up nested-basis pass of Algorithm 2.
//
// For node i the rows of A = kappa(Xbar_i, Y_i^*) are the candidate points and
// the columns the farfield representor points.  Householder QR with column
// pivoting runs on M = A^T (s x m, stored row-major so that a wavefront reads
// 64 consecutive columns of one row), and with M P = Q [R11 R12; 0 R22] the
// interpolation matrix is T = R11^{-1} R12, U_i = P [I; T^T], and the
// skeleton Xhat_i is the first k pivoted rows.
//
// Rules (identical to the oracle's): pivot = lowest index whose partial norm
// is within a factor (1 - 2^-40) of the largest; norms down-dated with the
// LAWN 176 safeguard (recompute once a down-date has lost half the digits);
// stop before step j when |R_jj| <= tol |R_00| for the column it would pivot
// in, leaving the columns in place (or j = min(s, m)).
//
// One workgroup per node; lane c owns columns c, c+256, ...  Each lane runs
// its columns' dot products, updates and squared tail sums sequentially in row
// order, and the tail sum doubles as the next |R_jj|^2 and as the down-date
// recomputation.  With the reflector norm in closed form this reproduces the
// oracle's operation order exactly, so pivots, ranks and T agree bit for bit
// whenever the kernel entries do.  Compiled with -ffp-contract=off.
#include "common.h"
#include "kappa.h"

namespace h2 {
namespace {

constexpr int TB = 256;

__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int wave_min_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
template <int NT>
__device__ inline double block_max(double v, double* sh)
{
    v = wave_max(v);
    if (NT == 64) return v;
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < NT / 64; ++q) r = fmax(r, sh[q]);
    __syncthreads();
    return r;
}
template <int NT>
__device__ inline int block_min_i(int v, int* sh)
{
    v = wave_min_i(v);
    if (NT == 64) return v;
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    int r = sh[0];
    for (int q = 1; q < NT / 64; ++q) r = min(r, sh[q]);
    __syncthreads();
    return r;
}


// Sequential row loops of one column with the loads issued ahead in batches
// of 8: the arithmetic runs in exactly the order of a plain loop (so the
// result is the oracle's, bit for bit), only the memory latency overlaps.
constexpr int LB = 8;

// acc + sum_{r=r0}^{r1-1} a[r] * x[r*ld], accumulated in row order
__device__ __forceinline__ double dot_rows(const double* __restrict__ a, const double* x, int64_t ld, int r0,
                                           int r1, double acc)
{
    int r = r0;
    for (; r + LB <= r1; r += LB) {
        double xv[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) xv[q] = x[(int64_t)(r + q) * ld];
#pragma unroll
        for (int q = 0; q < LB; ++q) acc = acc + a[r + q] * xv[q];
    }
    for (; r < r1; ++r) acc = acc + a[r] * x[(int64_t)r * ld];
    return acc;
}

// acc + sum_{r=r0}^{r1-1} x[r*ld]^2, in row order
__device__ __forceinline__ double sumsq_rows(const double* x, int64_t ld, int r0, int r1, double acc)
{
    int r = r0;
    for (; r + LB <= r1; r += LB) {
        double xv[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) xv[q] = x[(int64_t)(r + q) * ld];
#pragma unroll
        for (int q = 0; q < LB; ++q) acc = acc + xv[q] * xv[q];
    }
    for (; r < r1; ++r) acc = acc + x[(int64_t)r * ld] * x[(int64_t)r * ld];
    return acc;
}

// x[r] <- x[r] - f v[r] for r in [r0, r1); returns the sum of the new x[r]^2
// over r in [r0+1, r1) in row order (the next step's tail norm)
__device__ __forceinline__ double axpy_rows(const double* __restrict__ v, double f, double* x, int64_t ld, int r0,
                                            int r1)
{
    {
        double y = x[(int64_t)r0 * ld] - f * v[r0];
        x[(int64_t)r0 * ld] = y;
    }
    double tail = 0.0;
    int r = r0 + 1;
    for (; r + LB <= r1; r += LB) {
        double xv[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) xv[q] = x[(int64_t)(r + q) * ld];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            double y = xv[q] - f * v[r + q];
            x[(int64_t)(r + q) * ld] = y;
            tail = tail + y * y;
        }
    }
    for (; r < r1; ++r) {
        double y = x[(int64_t)r * ld] - f * v[r];
        x[(int64_t)r * ld] = y;
        tail = tail + y * y;
    }
    return tail;
}

// NT = 64 (one wavefront, for row sets of at most 64 points) or 256 lanes.
// LDSM: the s x m block lives in LDS (dynamic shared memory after the
// reflector), otherwise in the global workspace.  The arithmetic is the same.
// Compression (s > m): the s x m block is streamed in blocks of BR rows and
// folded into the m x m upper triangle R (LDS or global) by Householder
// reflectors that each zero one column of the block against the diagonal
// entry of R (TSQR).  Lane l owns columns l, l + NT, ... (CPL of them) and
// keeps their BR block entries in registers, evaluating them itself; the
// column that step j eliminates is published in a double-buffered LDS slot
// by its owner at the end of step j - 1, so one barrier per step suffices.
// The R entries of the next row are loaded a step ahead.  (This part
// accumulates with fused multiply-adds; it is not the oracle's operation
// order, and need not be: pivots and T are fixed up to rounding.)
template <int NT, int CPL, int BR>
__device__ void tsqr_fold(const IdTask& tk, int m, int s0, double* R, double* colbuf, double* nubuf, double* scr)
{
    const double* pts = tk.pts;
    const int64_t ld = tk.ld;
    const int* xi = tk.x_idx;
    const int* yi = tk.y_idx;
    const int d = tk.d, kid = tk.kid;
    const double prm = tk.prm;
    const int lane = threadIdx.x;
    for (int64_t e = lane; e < (int64_t)m * m; e += NT) R[e] = 0.0;
    __syncthreads();
    double bc[CPL][BR], tail[CPL];
    for (int r0 = 0; r0 < s0; r0 += BR) {
        const int nb = min(BR, s0 - r0);
        // this lane's block entries (evaluated through a lane-private LDS
        // slice, scr[r * NT + lane]) and their squared sums
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = lane + t * NT;
            if (c < m) {
                const int xc = xi[c];
                for (int r = 0; r < nb; ++r)
                    scr[r * NT + lane] = kappa_r2(kid, prm, dist2(pts, ld, xc, pts, ld, yi[r0 + r], d));
            }
            tail[t] = 0.0;
#pragma unroll
            for (int r = 0; r < BR; ++r) {
                const double v = (c < m && r < nb) ? scr[r * NT + lane] : 0.0;
                bc[t][r] = v;
                tail[t] = __builtin_fma(v, v, tail[t]);
            }
        }
        // publish column 0
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < BR; ++r) colbuf[r] = bc[0][r];
            nubuf[0] = tail[0];
        }
        double rn[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = lane + t * NT;
            rn[t] = c < m ? R[c] : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < m; ++j) {
            const double* cj = colbuf + (j & 1) * BR;
            const double nub = nubuf[j & 1];
            double rc[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                rc[t] = rn[t];
                const int c = lane + t * NT;
                rn[t] = (c < m && j + 1 < m) ? R[(int64_t)(j + 1) * m + c] : 0.0;
            }
            if (nub != 0.0) {
                const double x0 = R[(int64_t)j * m + j];
                const double alpha = x0 >= 0.0 ? -sqrt(x0 * x0 + nub) : sqrt(x0 * x0 + nub);
                const double v0 = x0 - alpha;
                const double vtv = 2.0 * fabs(alpha) * (fabs(alpha) + fabs(x0));
                double cjr[BR];
#pragma unroll
                for (int r = 0; r < BR; ++r) cjr[r] = cj[r];
#pragma unroll
                for (int t = 0; t < CPL; ++t) {
                    const int c = lane + t * NT;
                    if (c > j && c < m) {
                        double w = v0 * rc[t];
#pragma unroll
                        for (int r = 0; r < BR; ++r) w = __builtin_fma(cjr[r], bc[t][r], w);
                        const double f = 2.0 * w / vtv;
                        R[(int64_t)j * m + c] = rc[t] - f * v0;
                        double ts = 0.0;
#pragma unroll
                        for (int r = 0; r < BR; ++r) {
                            bc[t][r] = __builtin_fma(-f, cjr[r], bc[t][r]);
                            ts = __builtin_fma(bc[t][r], bc[t][r], ts);
                        }
                        tail[t] = ts;
                    }
                }
                if (lane == j % NT) R[(int64_t)j * m + j] = alpha;
            }
            // the owner of column j + 1 publishes it for the next step
            if (j + 1 < m && lane == (j + 1) % NT) {
                const int t1 = (j + 1) / NT;
                double* nb1 = colbuf + ((j + 1) & 1) * BR;
#pragma unroll
                for (int t = 0; t < CPL; ++t)
                    if (t == t1) {
#pragma unroll
                        for (int r = 0; r < BR; ++r) nb1[r] = bc[t][r];
                        nubuf[(j + 1) & 1] = tail[t];
                    }
            }
            __syncthreads();
        }
    }
}

// NT = 64 (one wavefront; the matrix in LDS) or 256 lanes (global matrix).
// LDSM: the matrix the pivoted QR runs on lives in LDS (dynamic shared
// memory after the reflector), otherwise in the global workspace.  With
// s > m the s x m kernel block is first compressed to its m x m R factor
// (tsqr_fold): column pivoting sees only the partial column norms, which a
// left orthogonal factor does not change, so the pivots, |R_jj| and T are
// those of the s x m block up to rounding.
template <int NT, bool LDSM>
__global__ __launch_bounds__(NT) void k_batched_id(const IdTask* __restrict__ tasks, const int* __restrict__ order,
                                                   int bmax)
{
    extern __shared__ double dyn[];
    __shared__ double redd[4];
    __shared__ int redi[4];
    __shared__ double sh_alpha;

    const IdTask& tk = tasks[order[blockIdx.x]];
    const int m = tk.m, s0 = tk.s, d = tk.d, kid = tk.kid;
    const double prm = tk.prm, tol = tk.tol;
    int* piv = tk.piv;
    for (int c = threadIdx.x; c < m; c += NT) piv[c] = c;
    if (m == 0 || s0 == 0) {
        if (threadIdx.x == 0) *tk.rank = 0;
        return;
    }
    const bool comp = s0 > m && m <= (NT == 64 ? 64 : 4 * NT);
    const int s = comp ? m : s0;  // rows of the matrix the pivoted QR runs on
    double* v = dyn;
    double* M = LDSM ? dyn + s : tk.M;
    double* nu = tk.nu;
    double* nu0 = nu + m;
    double* ss = nu + 2 * m;
    const int* xi = tk.x_idx;
    const int* yi = tk.y_idx;

    if (comp) {
        // the published column lives after the LDS matrix, or over the (not
        // yet used) reflector space
        double* cb = LDSM ? dyn + s + (int64_t)s * m : dyn;
        if constexpr (NT == 64)
            tsqr_fold<NT, 1, 16>(tk, m, s0, M, cb, cb + 32, cb + 34);
        else
            tsqr_fold<NT, 4, 16>(tk, m, s0, M, cb, cb + 32, cb + 34);
    } else {
        // kernel block: M[r][c] = kappa(x_c, y_r)
        for (int64_t e = threadIdx.x; e < (int64_t)s * m; e += NT) {
            int r = (int)(e / m), c = (int)(e - (int64_t)r * m);
            double r2 = dist2(tk.pts, tk.ld, xi[c], tk.pts, tk.ld, yi[r], d);
            M[e] = kappa_r2(kid, prm, r2);
        }
        __syncthreads();
    }
    for (int c = threadIdx.x; c < m; c += NT) {
        double acc = sumsq_rows(M + c, m, 0, s, 0.0);
        ss[c] = acc;
        nu[c] = sqrt(acc);
        nu0[c] = nu[c];
    }
    __syncthreads();

    const double tol3z = sqrt(2.220446049250313e-16);
    const double window = 1.0 - 0x1.0p-40;
    const int kmax = m < s ? m : s;
    double r00 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        // pivot: lowest index within the window of the largest partial norm
        double mx = 0.0;
        for (int c = j + threadIdx.x; c < m; c += NT) mx = fmax(mx, nu[c]);
        mx = block_max<NT>(mx, redd);
        int cand = 0x7fffffff;
        for (int c = j + threadIdx.x; c < m; c += NT)
            if (nu[c] >= window * mx) {
                cand = c;
                break;
            }
        int pc = block_min_i<NT>(cand, redi);
        // |R_jj| of the candidate; the step that stops swaps nothing
        if (threadIdx.x == 0) sh_alpha = sqrt(ss[pc]);
        __syncthreads();
        const double alpha = sh_alpha;
        if (j == 0) r00 = alpha;
        if (alpha == 0.0 || alpha <= tol * r00) break;
        if (pc != j) {
            for (int r = threadIdx.x; r < s; r += NT) {
                double t = M[(int64_t)r * m + j];
                M[(int64_t)r * m + j] = M[(int64_t)r * m + pc];
                M[(int64_t)r * m + pc] = t;
            }
            if (threadIdx.x == 0) {
                double t = nu[j]; nu[j] = nu[pc]; nu[pc] = t;
                t = nu0[j]; nu0[j] = nu0[pc]; nu0[pc] = t;
                t = ss[j]; ss[j] = ss[pc]; ss[pc] = t;
                int ti = piv[j]; piv[j] = piv[pc]; piv[pc] = ti;
            }
        }
        __syncthreads();
        const double xj = M[(int64_t)j * m + j];
        const double beta = xj >= 0.0 ? -alpha : alpha;
        for (int r = j + threadIdx.x; r < s; r += NT) v[r] = M[(int64_t)r * m + j];
        __syncthreads();
        if (threadIdx.x == 0) v[j] = v[j] - beta;
        __syncthreads();
        const double vtv = 2.0 * alpha * (alpha + fabs(xj));
        for (int c = j + 1 + threadIdx.x; c < m; c += NT) {
            double w = dot_rows(v, M + c, m, j, s, 0.0);
            double f = 2.0 * w / vtv;
            double tail = axpy_rows(v, f, M + c, m, j, s);
            ss[c] = tail;
            if (nu[c] != 0.0) {
                double t = fabs(M[(int64_t)j * m + c]) / nu[c];
                t = (1.0 + t) * (1.0 - t);
                if (t < 0.0) t = 0.0;
                double rat = nu[c] / nu0[c];
                double t2 = t * rat * rat;
                if (t2 <= tol3z) {
                    nu[c] = sqrt(tail);
                    nu0[c] = nu[c];
                } else {
                    nu[c] = nu[c] * sqrt(t);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) M[(int64_t)j * m + j] = beta;
        __syncthreads();
        k = j + 1;
    }
    // T = R11^{-1} R12 by back substitution, one column of R12 per lane
    const int nr = m - k;
    double* T = tk.T;
    for (int u = threadIdx.x; u < nr; u += NT) {
        for (int t = k - 1; t >= 0; --t) {
            double acc = M[(int64_t)t * m + (k + u)];
            const double* Rt = M + (int64_t)t * m;
            int l = t + 1;
            for (; l + LB <= k; l += LB) {
                double rv[LB], tv[LB];
#pragma unroll
                for (int q = 0; q < LB; ++q) {
                    rv[q] = Rt[l + q];
                    tv[q] = T[(int64_t)(l + q) * nr + u];
                }
#pragma unroll
                for (int q = 0; q < LB; ++q) acc = acc - rv[q] * tv[q];
            }
            for (; l < k; ++l) acc = acc - Rt[l] * T[(int64_t)l * nr + u];
            T[(int64_t)t * nr + u] = acc / M[(int64_t)t * m + t];
        }
    }
    for (int t = threadIdx.x; t < k; t += NT) tk.skel[t] = xi[piv[t]];
    if (threadIdx.x == 0) *tk.rank = k;
}

// Row set of every node of a level: the leaf's points, or the children's
// skeletons concatenated in child order.
__global__ __launch_bounds__(TB) void k_xbar_fill(int lo, const int* __restrict__ nchild,
                                                  const int* __restrict__ first_child, const int* __restrict__ start,
                                                  const int* __restrict__ count, const int* __restrict__ rank,
                                                  const int* __restrict__ skel, int skel_stride,
                                                  const int64_t* __restrict__ off, int* __restrict__ out)
{
    int t = blockIdx.x;
    int i = lo + t;
    int* o = out + off[t];
    if (nchild[i] == 0) {
        for (int q = threadIdx.x; q < count[i]; q += TB) o[q] = start[i] + q;
        return;
    }
    int64_t w = 0;
    for (int c = first_child[i]; c < first_child[i] + nchild[i]; ++c) {
        int kc = rank[c];
        for (int q = threadIdx.x; q < kc; q += TB) o[w + q] = skel[(int64_t)c * skel_stride + q];
        w += kc;
    }
}

}  // namespace

void batched_id(const std::vector<IdTask>& tasks, hipStream_t s)
{
    const int np = (int)tasks.size();
    if (np <= 0) return;
    // class 0 / 3: one wavefront, matrix (and the compression's row block)
    // in LDS; 1: one wavefront, global matrix; 2: four wavefronts, global
    // matrix (the compression's row block in LDS)
    const int BROWS = 64;                 // compression row block (at most)
    const size_t LDS_CAP = 80 * 1024;     // bytes per workgroup
    auto lds_need = [&](const IdTask& t, int c) -> size_t {
        const bool comp = t.s > t.m && t.m <= (c == 2 ? 4 * TB : 64);
        const int sr = comp ? t.m : t.s;
        // published column (2 x 16) + its two norms + the lanes' evaluation slices
        const size_t pub = comp ? 34 + (size_t)16 * (c == 2 ? TB : 64) : 0;
        if (c == 0) return ((size_t)sr + (size_t)sr * t.m + pub) * sizeof(double);
        return std::max((size_t)sr, pub) * sizeof(double);
    };
    // class 0 is split by LDS size (0: up to 32 KiB, 3: more) so that small
    // problems are not limited to the occupancy of the largest
    std::vector<int> cls(np);
    for (int p = 0; p < np; ++p) {
        if (tasks[p].m > 64) {
            cls[p] = 2;
        } else {
            const size_t need = lds_need(tasks[p], 0);
            cls[p] = need <= 32 * 1024 ? 0 : (need <= LDS_CAP ? 3 : 1);
        }
    }
    std::vector<int> order;
    order.reserve(np);
    int cnt[4] = {0, 0, 0, 0};
    size_t lds[4] = {8, 8, 8, 8};
    for (int c = 0; c < 4; ++c)
        for (int p = 0; p < np; ++p)
            if (cls[p] == c) {
                order.push_back(p);
                ++cnt[c];
                lds[c] = std::max(lds[c], lds_need(tasks[p], c == 3 ? 0 : c));
            }
    DBuf<IdTask> d_tasks;
    DBuf<int> d_order;
    d_tasks.ensure(tasks.size(), s);
    d_order.ensure(order.size(), s);
    H2_HIP(hipMemcpyAsync(d_tasks.p, tasks.data(), tasks.size() * sizeof(IdTask), hipMemcpyHostToDevice, s));
    H2_HIP(hipMemcpyAsync(d_order.p, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, s));
    int o = 0;
    if (cnt[0] > 0) {
        k_batched_id<64, true><<<cnt[0], 64, lds[0], s>>>(d_tasks.p, d_order.p + o, BROWS);
        H2_LAUNCH_CHECK();
    }
    o += cnt[0];
    if (cnt[1] > 0) {
        k_batched_id<64, false><<<cnt[1], 64, lds[1], s>>>(d_tasks.p, d_order.p + o, BROWS);
        H2_LAUNCH_CHECK();
    }
    o += cnt[1];
    if (cnt[2] > 0) {
        k_batched_id<TB, false><<<cnt[2], TB, lds[2], s>>>(d_tasks.p, d_order.p + o, BROWS);
        H2_LAUNCH_CHECK();
    }
    o += cnt[2];
    if (cnt[3] > 0) {
        k_batched_id<64, true><<<cnt[3], 64, lds[3], s>>>(d_tasks.p, d_order.p + o, BROWS);
        H2_LAUNCH_CHECK();
    }
    H2_HIP(hipStreamSynchronize(s));
}

template <class T>
static void upload(DBuf<T>& dst, const std::vector<T>& src, hipStream_t s)
{
    dst.ensure(src.size(), s);
    if (!src.empty())
        H2_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Nested bases of several independent problems at once: round t handles
// depth maxdepth - t of every problem (a node's children were done in the
// round before), and all nodes of a round go into one batched ID launch
// (several only when the workspace cap splits it).  piv and T offsets are
// assigned per problem in processing order (deepest level first).
void build_bases_multi(const std::vector<Handle*>& hs, hipStream_t s)
{
    struct St {
        std::vector<int> ys_cnt;
        int64_t piv_total = 0, T_total = 0;
    };
    const int np = (int)hs.size();
    std::vector<St> st(np);
    int maxd = 0;
    for (int p = 0; p < np; ++p) {
        Handle& h = *hs[p];
        const int nn = h.nnode;
        h.rank.ensure((size_t)nn, s);
        h.mbar.ensure((size_t)nn, s);
        h.skel.ensure((size_t)nn * h.ys_stride, s);
        h.piv_off.ensure((size_t)nn + 1, s);
        h.T_off.ensure((size_t)nn + 1, s);
        H2_HIP(hipMemsetAsync(h.rank.p, 0, sizeof(int) * nn, s));
        H2_HIP(hipMemsetAsync(h.mbar.p, 0, sizeof(int) * nn, s));
        st[p].ys_cnt = read_vec(h.ys_cnt.p, nn, s);
        h.h_rank.assign(nn, 0);
        h.h_mbar.assign(nn, 0);
        h.h_piv_off.assign((size_t)nn + 1, 0);
        h.h_T_off.assign((size_t)nn + 1, 0);
        maxd = std::max(maxd, h.maxdepth);
    }
    const int64_t WS_CAP = (int64_t)1 << 28;  // doubles of ID workspace per launch
    DBuf<int> d_xidx;
    DBuf<int64_t> d_xoff;
    DBuf<double> Mws, nuws;
    for (int t = 0; t < maxd; ++t) {
        // problems and levels of this round; grow piv / T first (the task
        // pointers must see the final buffers)
        std::vector<int> lvl(np, 0);
        int64_t xtot = 0;
        std::vector<int64_t> xbase(np, 0);
        for (int p = 0; p < np; ++p) {
            Handle& h = *hs[p];
            const int L = h.maxdepth - t;
            lvl[p] = L;
            if (L < 1) continue;
            xbase[p] = xtot;
            const int64_t keep_piv = st[p].piv_total, keep_T = st[p].T_total;
            for (int i = h.lvl_ptr[L]; i < h.lvl_ptr[L + 1]; ++i) {
                int m = 0;
                if (h.h_nchild[i] == 0)
                    m = h.h_count[i];
                else
                    for (int c = h.h_first_child[i]; c < h.h_first_child[i] + h.h_nchild[i]; ++c) m += h.h_rank[c];
                h.h_mbar[i] = m;
                h.h_piv_off[i] = st[p].piv_total;
                h.h_T_off[i] = st[p].T_total;
                st[p].piv_total += m;
                st[p].T_total += (int64_t)m * std::min(m, st[p].ys_cnt[i]);
                xtot += m;
            }
            h.piv.grow_keep((size_t)std::max<int64_t>(st[p].piv_total, 1), (size_t)keep_piv, s);
            h.T.grow_keep((size_t)std::max<int64_t>(st[p].T_total, 1), (size_t)keep_T, s);
        }
        if (xtot == 0) continue;
        // row sets of the round
        d_xidx.ensure((size_t)xtot, s);
        for (int p = 0; p < np; ++p) {
            Handle& h = *hs[p];
            const int L = lvl[p];
            if (L < 1) continue;
            const int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
            std::vector<int64_t> xo((size_t)nl + 1, 0);
            for (int q = 0; q < nl; ++q) xo[q + 1] = xo[q] + h.h_mbar[lo + q];
            for (auto& v : xo) v += xbase[p];
            d_xoff.ensure(xo.size(), s);
            H2_HIP(hipMemcpyAsync(d_xoff.p, xo.data(), xo.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
            k_xbar_fill<<<nl, TB, 0, s>>>(lo, h.nchild.p, h.first_child.p, h.start.p, h.count.p, h.rank.p, h.skel.p,
                                          h.ys_stride, d_xoff.p, d_xidx.p);
            H2_LAUNCH_CHECK();
            H2_HIP(hipStreamSynchronize(s));  // d_xoff is reused by the next problem
        }
        // tasks, launched in chunks of bounded workspace
        std::vector<IdTask> tasks;
        std::vector<int64_t> Moff, nuoff;
        int64_t ws = 0, no = 0;
        auto flush = [&]() {
            if (tasks.empty()) return;
            Mws.ensure((size_t)std::max<int64_t>(ws, 1), s);
            nuws.ensure((size_t)std::max<int64_t>(no, 1), s);
            for (size_t q = 0; q < tasks.size(); ++q) {
                tasks[q].M = Mws.p + Moff[q];
                tasks[q].nu = nuws.p + nuoff[q];
            }
            batched_id(tasks, s);
            tasks.clear();
            Moff.clear();
            nuoff.clear();
            ws = 0;
            no = 0;
        };
        for (int p = 0; p < np; ++p) {
            Handle& h = *hs[p];
            const int L = lvl[p];
            if (L < 1) continue;
            int64_t xo = xbase[p];
            for (int i = h.lvl_ptr[L]; i < h.lvl_ptr[L + 1]; ++i) {
                const int m = h.h_mbar[i], sy = st[p].ys_cnt[i];
                const int64_t need = (int64_t)m * sy;
                if (!tasks.empty() && ws + need > WS_CAP) flush();
                IdTask tk;
                tk.pts = h.pts.p;
                tk.ld = h.n;
                tk.x_idx = d_xidx.p + xo;
                tk.y_idx = h.ys_idx.p + (int64_t)i * h.ys_stride;
                tk.piv = h.piv.p + h.h_piv_off[i];
                tk.T = h.T.p + h.h_T_off[i];
                tk.skel = h.skel.p + (int64_t)i * h.ys_stride;
                tk.rank = h.rank.p + i;
                tk.prm = h.prm;
                tk.tol = h.tol_int;
                tk.m = m;
                tk.s = sy;
                tk.d = h.d;
                tk.kid = h.kid;
                tasks.push_back(tk);
                Moff.push_back(ws);
                nuoff.push_back(no);
                ws += need;
                no += 3 * (int64_t)m;
                xo += m;
            }
        }
        flush();
        for (int p = 0; p < np; ++p) {
            Handle& h = *hs[p];
            const int L = lvl[p];
            if (L < 1) continue;
            const int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
            std::vector<int> rk = read_vec(h.rank.p + lo, nl, s);
            for (int q = 0; q < nl; ++q) h.h_rank[lo + q] = rk[q];
        }
    }
    for (int p = 0; p < np; ++p) {
        Handle& h = *hs[p];
        const int nn = h.nnode;
        h.h_piv_off[nn] = st[p].piv_total;
        h.h_T_off[nn] = st[p].T_total;
        upload(h.mbar, h.h_mbar, s);
        upload(h.piv_off, h.h_piv_off, s);
        upload(h.T_off, h.h_T_off, s);
        h.sum_rank = 0;
        for (int i = 0; i < nn; ++i) h.sum_rank += h.h_rank[i];
        h.bytes_T = st[p].T_total * (int64_t)sizeof(double);
    }
    H2_HIP(hipStreamSynchronize(s));
}

void build_bases(Handle& h) { build_bases_multi({&h}, h.stream); }

}  // namespace h2
