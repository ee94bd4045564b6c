// H^2 matrix-vector product y = Ktilde x (the O(n) apply of Section 2.1).
//
// Vectors live in tree order as [n][nrhs] (right-hand sides fastest); the
// node coefficients xhat_i, yhat_i as [rank_i][nrhs] blocks laid out in node
// id order, so the children of a node (consecutive ids) own one contiguous
// block: the input rows z_p of a parent's interpolation step are exactly its
// children's xhat concatenated, as in the row set Xbar_p of Algorithm 2.
//
//   gather    x_t = x[perm]
//   upward    xhat_i = U_i^T z_i, z_i = x_t(X_i) (leaf) or children's xhat;
//             U_i = P [I; T^T] so xhat[t] = z[piv t] + sum_u T[t,u] z[piv(k+u)]
//   coupling  yhat_i = sum_{j in IL(i)} B_ij xhat_j
//   downward  children's yhat += U_p yhat_p   (depth 1 first)
//   leaves    y_t(X_i) = U_i yhat_i + sum_{j in near(i)} D_ij x_t(X_j)
//   scatter   y[perm] = y_t
// Every output element has exactly one writer; there are no atomics.
#include "common.h"

namespace h2 {
namespace {

constexpr int TB = 256;

__global__ __launch_bounds__(TB) void k_gather(const double* __restrict__ x, int64_t n, int nrhs,
                                               const int* __restrict__ perm, double* __restrict__ xt)
{
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= n * nrhs) return;
    int64_t i = q / nrhs;
    int r = (int)(q - i * nrhs);
    xt[q] = x[(int64_t)r * n + perm[i]];
}

__global__ __launch_bounds__(TB) void k_scatter(const double* __restrict__ yt, int64_t n, int nrhs,
                                                const int* __restrict__ perm, double* __restrict__ y)
{
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= n * nrhs) return;
    int64_t i = q / nrhs;
    int r = (int)(q - i * nrhs);
    y[(int64_t)r * n + perm[i]] = yt[q];
}

__global__ __launch_bounds__(TB) void k_upward(int lo, int nrhs, const int* __restrict__ nchild,
                                               const int* __restrict__ first_child, const int* __restrict__ start,
                                               const int* __restrict__ rank, const int* __restrict__ mbar,
                                               const int64_t* __restrict__ piv_off, const int* __restrict__ piv,
                                               const int64_t* __restrict__ T_off, const double* __restrict__ T,
                                               const int64_t* __restrict__ xh_off, const double* __restrict__ xt,
                                               double* __restrict__ xh)
{
    const int i = lo + blockIdx.x;
    const int k = rank[i];
    if (k == 0) return;
    const int m = mbar[i], nr = m - k;
    const double* z = nchild[i] == 0 ? xt + (int64_t)start[i] * nrhs : xh + xh_off[first_child[i]] * nrhs;
    const int* pv = piv + piv_off[i];
    const double* Ti = T + T_off[i];
    double* o = xh + xh_off[i] * nrhs;
    for (int q = threadIdx.x; q < k * nrhs; q += TB) {
        int t = q / nrhs, r = q - t * nrhs;
        double acc = z[(int64_t)pv[t] * nrhs + r];
        const double* Tr = Ti + (int64_t)t * nr;
        for (int u = 0; u < nr; ++u) acc += Tr[u] * z[(int64_t)pv[k + u] * nrhs + r];
        o[q] = acc;
    }
}

__global__ __launch_bounds__(TB) void k_coupling_mv(int nrhs, const int* __restrict__ il_ptr,
                                                    const int* __restrict__ il_col, const int* __restrict__ rank,
                                                    const int64_t* __restrict__ B_off, const double* __restrict__ B,
                                                    const int64_t* __restrict__ xh_off, const double* __restrict__ xh,
                                                    double* __restrict__ yh)
{
    const int i = blockIdx.x;
    const int ki = rank[i];
    if (ki == 0) return;
    double* o = yh + xh_off[i] * nrhs;
    for (int q = threadIdx.x; q < ki * nrhs; q += TB) {
        int t = q / nrhs, r = q - t * nrhs;
        double acc = 0.0;
        for (int e = il_ptr[i]; e < il_ptr[i + 1]; ++e) {
            const int j = il_col[e];
            const int kj = rank[j];
            const double* Bt = B + B_off[e] + (int64_t)t * kj;
            const double* xj = xh + xh_off[j] * nrhs + r;
            for (int u = 0; u < kj; ++u) acc += Bt[u] * xj[(int64_t)u * nrhs];
        }
        o[q] = acc;
    }
}

// w[piv pos] (+)= (U yhat)[pos]: pos < k -> yhat[pos]; else sum_t T[t, pos-k] yhat[t]
__device__ inline double u_times(int pos, int k, int nr, int r, int nrhs, const double* __restrict__ Ti,
                                 const double* __restrict__ yhat)
{
    if (pos < k) return yhat[(int64_t)pos * nrhs + r];
    int u = pos - k;
    double acc = 0.0;
    for (int t = 0; t < k; ++t) acc += Ti[(int64_t)t * nr + u] * yhat[(int64_t)t * nrhs + r];
    return acc;
}

__global__ __launch_bounds__(TB) void k_downward(int lo, int nrhs, const int* __restrict__ nchild,
                                                 const int* __restrict__ first_child, const int* __restrict__ rank,
                                                 const int* __restrict__ mbar, const int64_t* __restrict__ piv_off,
                                                 const int* __restrict__ piv, const int64_t* __restrict__ T_off,
                                                 const double* __restrict__ T, const int64_t* __restrict__ xh_off,
                                                 double* __restrict__ yh)
{
    const int i = lo + blockIdx.x;
    const int k = rank[i];
    if (k == 0 || nchild[i] == 0) return;
    const int m = mbar[i], nr = m - k;
    const int* pv = piv + piv_off[i];
    const double* Ti = T + T_off[i];
    const double* yi = yh + xh_off[i] * nrhs;
    double* yc = yh + xh_off[first_child[i]] * nrhs;
    for (int q = threadIdx.x; q < m * nrhs; q += TB) {
        int pos = q / nrhs, r = q - pos * nrhs;
        yc[(int64_t)pv[pos] * nrhs + r] += u_times(pos, k, nr, r, nrhs, Ti, yi);
    }
}

__global__ __launch_bounds__(TB) void k_leaves(int nrhs, const int* __restrict__ leaves, const int* __restrict__ start,
                                               const int* __restrict__ count, const int* __restrict__ rank,
                                               const int64_t* __restrict__ piv_off, const int* __restrict__ piv,
                                               const int64_t* __restrict__ T_off, const double* __restrict__ T,
                                               const int64_t* __restrict__ xh_off, const double* __restrict__ yh,
                                               const int* __restrict__ nr_ptr, const int* __restrict__ nr_col,
                                               const int64_t* __restrict__ D_off, const double* __restrict__ D,
                                               const double* __restrict__ xt, double* __restrict__ yt)
{
    const int i = leaves[blockIdx.x];
    const int k = rank[i];
    const int m = count[i], nr = m - k;
    double* yo = yt + (int64_t)start[i] * nrhs;
    if (k > 0) {
        const int* pv = piv + piv_off[i];
        const double* Ti = T + T_off[i];
        const double* yi = yh + xh_off[i] * nrhs;
        for (int q = threadIdx.x; q < m * nrhs; q += TB) {
            int pos = q / nrhs, r = q - pos * nrhs;
            yo[(int64_t)pv[pos] * nrhs + r] = u_times(pos, k, nr, r, nrhs, Ti, yi);
        }
    } else {
        for (int q = threadIdx.x; q < m * nrhs; q += TB) yo[q] = 0.0;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < m * nrhs; q += TB) {
        int t = q / nrhs, r = q - t * nrhs;
        double acc = 0.0;
        for (int e = nr_ptr[i]; e < nr_ptr[i + 1]; ++e) {
            const int j = nr_col[e];
            const int cj = count[j];
            const double* Dt = D + D_off[e] + (int64_t)t * cj;
            const double* xj = xt + (int64_t)start[j] * nrhs + r;
            for (int u = 0; u < cj; ++u) acc += Dt[u] * xj[(int64_t)u * nrhs];
        }
        yo[q] += acc;
    }
}

}  // namespace

void matvec(Handle& h, const double* x, double* y, int nrhs, hipStream_t s)
{
    const int64_t n = h.n;
    if (nrhs > h.mv_nrhs) {
        H2_HIP(hipStreamSynchronize(s));
        h.xt.ensure((size_t)n * nrhs, s);
        h.yt.ensure((size_t)n * nrhs, s);
        h.xh.ensure((size_t)std::max<int64_t>(h.sum_rank, 1) * nrhs, s);
        h.yh.ensure((size_t)std::max<int64_t>(h.sum_rank, 1) * nrhs, s);
        h.mv_nrhs = nrhs;
    }
    const bool prof = h.profile != 0;
    auto mark = [&](int e) {
        if (prof) H2_HIP(hipEventRecord(h.ev[e], s));
    };
    if (prof && !h.ev[0])
        for (auto& e : h.ev) H2_HIP(hipEventCreate(&e));
    mark(0);
    k_gather<<<blocks_for(n * nrhs, TB), TB, 0, s>>>(x, n, nrhs, h.perm.p, h.xt.p);
    H2_LAUNCH_CHECK();
    mark(1);
    for (int L = h.maxdepth; L >= 1; --L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_upward<<<nl, TB, 0, s>>>(lo, nrhs, h.nchild.p, h.first_child.p, h.start.p, h.rank.p, h.mbar.p,
                                   h.piv_off.p, h.piv.p, h.T_off.p, h.T.p, h.xh_off.p, h.xt.p, h.xh.p);
        H2_LAUNCH_CHECK();
    }
    mark(2);
    k_coupling_mv<<<h.nnode, TB, 0, s>>>(nrhs, h.il_ptr.p, h.il_col.p, h.rank.p, h.B_off.p, h.B.p, h.xh_off.p,
                                         h.xh.p, h.yh.p);
    H2_LAUNCH_CHECK();
    mark(3);
    for (int L = 1; L < h.maxdepth; ++L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_downward<<<nl, TB, 0, s>>>(lo, nrhs, h.nchild.p, h.first_child.p, h.rank.p, h.mbar.p, h.piv_off.p,
                                     h.piv.p, h.T_off.p, h.T.p, h.xh_off.p, h.yh.p);
        H2_LAUNCH_CHECK();
    }
    mark(4);
    k_leaves<<<(unsigned)h.leaves.n, TB, 0, s>>>(nrhs, h.leaves.p, h.start.p, h.count.p, h.rank.p, h.piv_off.p,
                                                 h.piv.p, h.T_off.p, h.T.p, h.xh_off.p, h.yh.p, h.nr_ptr.p,
                                                 h.nr_col.p, h.D_off.p, h.D.p, h.xt.p, h.yt.p);
    H2_LAUNCH_CHECK();
    mark(5);
    k_scatter<<<blocks_for(n * nrhs, TB), TB, 0, s>>>(h.yt.p, n, nrhs, h.perm.p, y);
    H2_LAUNCH_CHECK();
    mark(6);
    if (prof) {
        h.prof_valid = true;
        h.prof_nrhs = nrhs;
    }
}

}  // namespace h2
