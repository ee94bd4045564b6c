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
template <int NT, bool LDSM>
__global__ __launch_bounds__(NT) void k_batched_id(IdBatch b, const int* __restrict__ order, int d, int kid,
                                                   double prm)
{
    extern __shared__ double dyn[];
    __shared__ double redd[4];
    __shared__ int redi[4];
    __shared__ double sh_alpha;

    const int p = order[blockIdx.x];
    const int m = b.m[p], s = b.s[p];
    int* piv = b.piv_out + b.piv_off[p];
    for (int c = threadIdx.x; c < m; c += NT) piv[c] = c;
    if (m == 0 || s == 0) {
        if (threadIdx.x == 0) b.rank_out[p] = 0;
        return;
    }
    double* v = dyn;
    double* M = LDSM ? dyn + s : b.M + b.M_off[p];
    double* nu = b.nu + b.nu_off[p];
    double* nu0 = nu + m;
    double* ss = nu + 2 * m;
    const int* xi = b.x_idx + b.x_off[p];
    const int* yi = b.y_idx + b.y_off[p];

    // kernel block: M[r][c] = kappa(x_c, y_r)
    for (int64_t e = threadIdx.x; e < (int64_t)s * m; e += NT) {
        int r = (int)(e / m), c = (int)(e - (int64_t)r * m);
        double r2 = dist2(b.xpts, b.xld, xi[c], b.ypts, b.yld, yi[r], d);
        M[e] = kappa_r2(kid, prm, r2);
    }
    __syncthreads();
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
        if (alpha == 0.0 || alpha <= b.tol * r00) break;
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
    double* T = b.T_out + b.T_off[p];
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
    for (int t = threadIdx.x; t < k; t += NT) b.skel_out[(int64_t)p * b.skel_stride + t] = xi[piv[t]];
    if (threadIdx.x == 0) b.rank_out[p] = k;
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

void batched_id(const IdBatch& b, const std::vector<int>& m_host, const std::vector<int>& s_host, int d, int kid,
                double prm, hipStream_t s)
{
    if (b.nprob <= 0) return;
    // class 0: one wavefront, block in LDS; 1: one wavefront, global block;
    // 2: four wavefronts, global block
    const int LDS_DOUBLES = 8192;  // 64 KiB per workgroup
    std::vector<int> cls(b.nprob);
    for (int p = 0; p < b.nprob; ++p) {
        int64_t need = (int64_t)s_host[p] * (m_host[p] + 1);
        cls[p] = m_host[p] <= 64 ? (need <= LDS_DOUBLES ? 0 : 1) : 2;
    }
    std::vector<int> order;
    order.reserve(b.nprob);
    int cnt[3] = {0, 0, 0};
    size_t lds[3] = {8, 8, 8};
    for (int c = 0; c < 3; ++c)
        for (int p = 0; p < b.nprob; ++p)
            if (cls[p] == c) {
                order.push_back(p);
                ++cnt[c];
                size_t need = (size_t)s_host[p] * (c == 0 ? m_host[p] + 1 : 1) * sizeof(double);
                lds[c] = std::max(lds[c], need);
            }
    DBuf<int> d_order;
    d_order.ensure(order.size(), s);
    H2_HIP(hipMemcpyAsync(d_order.p, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, s));
    int o = 0;
    if (cnt[0] > 0) {
        k_batched_id<64, true><<<cnt[0], 64, lds[0], s>>>(b, d_order.p + o, d, kid, prm);
        H2_LAUNCH_CHECK();
    }
    o += cnt[0];
    if (cnt[1] > 0) {
        k_batched_id<64, false><<<cnt[1], 64, lds[1], s>>>(b, d_order.p + o, d, kid, prm);
        H2_LAUNCH_CHECK();
    }
    o += cnt[1];
    if (cnt[2] > 0) {
        k_batched_id<TB, false><<<cnt[2], TB, lds[2], s>>>(b, d_order.p + o, d, kid, prm);
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

void build_bases(Handle& h)
{
    hipStream_t s = h.stream;
    const int nn = h.nnode;
    h.rank.ensure((size_t)nn, s);
    h.mbar.ensure((size_t)nn, s);
    h.skel.ensure((size_t)nn * h.ys_stride, s);
    h.piv_off.ensure((size_t)nn + 1, s);
    h.T_off.ensure((size_t)nn + 1, s);
    H2_HIP(hipMemsetAsync(h.rank.p, 0, sizeof(int) * nn, s));
    H2_HIP(hipMemsetAsync(h.mbar.p, 0, sizeof(int) * nn, s));
    std::vector<int> ys_cnt = read_vec(h.ys_cnt.p, nn, s);
    h.h_rank.assign(nn, 0);
    h.h_mbar.assign(nn, 0);
    h.h_piv_off.assign((size_t)nn + 1, 0);
    h.h_T_off.assign((size_t)nn + 1, 0);

    // piv and T offsets for all nodes need the ranks of the level below, so
    // they are assigned level by level; nodes are laid out in id order, with
    // the root (never compressed) at offset 0 with size 0.
    int64_t piv_total = 0, T_total = 0;
    std::vector<int> mv, sv;
    std::vector<int64_t> xoff, yoff, Moff, nuoff, pivoff, Toff;
    DBuf<int> d_m, d_s, d_xidx;
    DBuf<int64_t> d_xoff, d_yoff, d_Moff, d_nuoff, d_pivoff, d_Toff;
    DBuf<double> Mws, nuws;
    const int64_t WS_CAP = (int64_t)1 << 28;  // doubles of ID workspace per launch

    // offsets of deeper levels come first in memory; compute per level
    for (int L = h.maxdepth; L >= 1; --L) {
        const int lo = h.lvl_ptr[L], hi = h.lvl_ptr[L + 1];
        int c0 = lo;
        while (c0 < hi) {
            // chunk [c0, c1) with bounded workspace
            int c1 = c0;
            int64_t ws = 0;
            mv.clear(); sv.clear(); xoff.clear(); yoff.clear(); Moff.clear(); nuoff.clear();
            pivoff.clear(); Toff.clear();
            int64_t xo = 0, no = 0;
            while (c1 < hi) {
                int i = c1;
                int m = 0;
                if (h.h_nchild[i] == 0)
                    m = h.h_count[i];
                else
                    for (int c = h.h_first_child[i]; c < h.h_first_child[i] + h.h_nchild[i]; ++c) m += h.h_rank[c];
                int sy = ys_cnt[i];
                int64_t need = (int64_t)m * sy;
                if (c1 > c0 && ws + need > WS_CAP) break;
                mv.push_back(m);
                sv.push_back(sy);
                xoff.push_back(xo);
                yoff.push_back((int64_t)i * h.ys_stride);
                Moff.push_back(ws);
                nuoff.push_back(no);
                pivoff.push_back(piv_total);
                Toff.push_back(T_total);
                h.h_piv_off[i] = piv_total;
                h.h_T_off[i] = T_total;
                h.h_mbar[i] = m;
                xo += m;
                no += 3 * (int64_t)m;
                ws += need;
                piv_total += m;
                T_total += (int64_t)m * std::min(m, sy);
                ++c1;
            }
            int np = c1 - c0;
            xoff.push_back(xo);
            h.piv.grow_keep((size_t)std::max<int64_t>(piv_total, 1), (size_t)(piv_total - xo), s);
            h.T.grow_keep((size_t)std::max<int64_t>(T_total, 1), (size_t)Toff[0], s);
            upload(d_m, mv, s);
            upload(d_s, sv, s);
            upload(d_xoff, xoff, s);
            upload(d_yoff, yoff, s);
            upload(d_Moff, Moff, s);
            upload(d_nuoff, nuoff, s);
            upload(d_pivoff, pivoff, s);
            upload(d_Toff, Toff, s);
            d_xidx.ensure((size_t)std::max<int64_t>(xo, 1), s);
            Mws.ensure((size_t)std::max<int64_t>(ws, 1), s);
            nuws.ensure((size_t)std::max<int64_t>(no, 1), s);
            k_xbar_fill<<<np, TB, 0, s>>>(c0, h.nchild.p, h.first_child.p, h.start.p, h.count.p, h.rank.p, h.skel.p,
                                          h.ys_stride, d_xoff.p, d_xidx.p);
            H2_LAUNCH_CHECK();
            IdBatch b;
            b.nprob = np;
            b.m = d_m.p;
            b.s = d_s.p;
            b.x_off = d_xoff.p;
            b.x_idx = d_xidx.p;
            b.y_off = d_yoff.p;
            b.y_idx = h.ys_idx.p;
            b.xpts = h.pts.p;
            b.xld = h.n;
            b.ypts = h.pts.p;
            b.yld = h.n;
            b.M_off = d_Moff.p;
            b.M = Mws.p;
            b.nu = nuws.p;
            b.nu_off = d_nuoff.p;
            b.tol = h.tol_int;
            b.rank_out = h.rank.p + c0;
            b.piv_out = h.piv.p;
            b.piv_off = d_pivoff.p;
            b.T_out = h.T.p;
            b.T_off = d_Toff.p;
            b.skel_out = h.skel.p + (int64_t)c0 * h.ys_stride;
            b.skel_stride = h.ys_stride;
            batched_id(b, mv, sv, h.d, h.kid, h.prm, s);
            std::vector<int> rk = read_vec(h.rank.p + c0, np, s);
            for (int t = 0; t < np; ++t) h.h_rank[c0 + t] = rk[t];
            c0 = c1;
        }
    }
    h.h_piv_off[nn] = piv_total;
    h.h_T_off[nn] = T_total;
    upload(h.mbar, h.h_mbar, s);
    upload(h.piv_off, h.h_piv_off, s);
    upload(h.T_off, h.h_T_off, s);
    h.sum_rank = 0;
    for (int i = 0; i < nn; ++i) h.sum_rank += h.h_rank[i];
    h.bytes_T = T_total * (int64_t)sizeof(double);
    H2_HIP(hipStreamSynchronize(s));
}

}  // namespace h2
