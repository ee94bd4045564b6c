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

typedef double double4_t __attribute__((ext_vector_type(4)));

// Batched block products Y[rows of i] (+)= sum_{e in row i} Blk_e X[rows of j_e]
// for the coupling sweep (Blk = B, X = xhat, Y = yhat) and the nearfield
// sweep (Blk = D, X = x_t, Y = y_t).  One wavefront per task (node i, 32-row
// chunk): MT 16-row tiles x 2 16-column tiles of v_mfma_f64_16x16x4f64, the
// K loop walking the list entries four rows of X at a time.  Operand layout
// of the instruction: A lane l = A[l%16][l/16], B lane l = B[l/16][l%16],
// result lane l register r = D[4r + l/16][l%16].  Blocks are column-major,
// so each 16-lane group of an A load reads 128 contiguous bytes, and X rows
// are nrhs-contiguous, so B loads are 128-byte rows as well.  Workgroup ids
// are remapped so that each XCD (ids round-robin over 8) runs a contiguous
// range of tasks, keeping the shared X rows of neighbouring nodes in one L2.
template <int MT>
__global__ __launch_bounds__(64) void k_blockgemm(int ntask, const int* __restrict__ task_node,
                                                  const int* __restrict__ task_r0, const int* __restrict__ ptr,
                                                  const int* __restrict__ col, const int* __restrict__ krow,
                                                  const int64_t* __restrict__ blk_off, const double* __restrict__ blk,
                                                  const int64_t* __restrict__ in_off, const double* __restrict__ X,
                                                  const int64_t* __restrict__ out_off, double* __restrict__ Y,
                                                  int nrhs, int accumulate)
{
    const int per = (ntask + 7) / 8;
    const int task = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (task >= ntask) return;
    const int i = task_node[task], r0 = task_r0[task];
    const int ki = krow[i];
    const int lane = threadIdx.x, l16 = lane & 15, k4 = lane >> 4;
    const int e0 = ptr[i], e1 = ptr[i + 1];
    for (int c0 = 0; c0 < nrhs; c0 += 32) {
        double4_t acc[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = (double4_t){0.0, 0.0, 0.0, 0.0};
        for (int e = e0; e < e1; ++e) {
            const int j = col[e];
            const int kj = krow[j];
            const double* Bb = blk + blk_off[e];
            const double* Xj = X + in_off[j] * nrhs;
            for (int u0 = 0; u0 < kj; u0 += 4) {
                const int u = u0 + k4;
                const bool uv = u < kj;
                double av[MT], bv[2];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int t = r0 + 16 * mt + l16;
                    av[mt] = (uv && t < ki) ? Bb[(int64_t)u * ki + t] : 0.0;
                }
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int c = c0 + 16 * nt + l16;
                    bv[nt] = (uv && c < nrhs) ? Xj[(int64_t)u * nrhs + c] : 0.0;
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
            }
        }
        double* Yi = Y + out_off[i] * nrhs;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + 16 * mt + 4 * r + k4;
                    const int c = c0 + 16 * nt + l16;
                    if (row < ki && c < nrhs) {
                        double* dst = Yi + (int64_t)row * nrhs + c;
                        *dst = accumulate ? *dst + acc[mt][nt][r] : acc[mt][nt][r];
                    }
                }
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

// Far part of the leaves: y_t(X_i) = U_i yhat_i (zero when the leaf has no
// farfield); the nearfield sweep then accumulates into the same rows.
__global__ __launch_bounds__(TB) void k_leaves_far(int nrhs, const int* __restrict__ leaves,
                                                   const int* __restrict__ start, const int* __restrict__ count,
                                                   const int* __restrict__ rank, const int64_t* __restrict__ piv_off,
                                                   const int* __restrict__ piv, const int64_t* __restrict__ T_off,
                                                   const double* __restrict__ T, const int64_t* __restrict__ xh_off,
                                                   const double* __restrict__ yh, double* __restrict__ yt)
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
}

void launch_gemm(const Handle::Tasks& t1, const Handle::Tasks& t2, const int* ptr, const int* col, const int* krow,
                 const int64_t* blk_off, const double* blk, const int64_t* in_off, const double* X,
                 const int64_t* out_off, double* Y, int nrhs, int accumulate, hipStream_t s)
{
    if (t1.n > 0) {
        unsigned grid = (unsigned)(8 * ((t1.n + 7) / 8));
        k_blockgemm<1><<<grid, 64, 0, s>>>(t1.n, t1.node.p, t1.r0.p, ptr, col, krow, blk_off, blk, in_off, X, out_off,
                                           Y, nrhs, accumulate);
        H2_LAUNCH_CHECK();
    }
    if (t2.n > 0) {
        unsigned grid = (unsigned)(8 * ((t2.n + 7) / 8));
        k_blockgemm<2><<<grid, 64, 0, s>>>(t2.n, t2.node.p, t2.r0.p, ptr, col, krow, blk_off, blk, in_off, X, out_off,
                                           Y, nrhs, accumulate);
        H2_LAUNCH_CHECK();
    }
}

}  // namespace

// Task lists of the two block sweeps, built once per handle.
void prepare_apply(Handle& h)
{
    hipStream_t s = h.stream;
    auto make = [&](const std::vector<int>& rows_of, const std::vector<int>& ptr, bool need_rank,
                    Handle::Tasks& t1, Handle::Tasks& t2) {
        std::vector<int> n1, r1, n2, r2;
        for (int i = 0; i < h.nnode; ++i) {
            int rows = rows_of[i];
            if (rows == 0) continue;
            if (!need_rank && ptr[i + 1] == ptr[i]) continue;
            for (int r0 = 0; r0 < rows; r0 += 32) {
                if (rows - r0 > 16) {
                    n2.push_back(i);
                    r2.push_back(r0);
                } else {
                    n1.push_back(i);
                    r1.push_back(r0);
                }
            }
        }
        auto up = [&](DBuf<int>& d, const std::vector<int>& v) {
            d.ensure(std::max<size_t>(v.size(), 1), s);
            if (!v.empty()) H2_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s));
        };
        up(t1.node, n1);
        up(t1.r0, r1);
        up(t2.node, n2);
        up(t2.r0, r2);
        t1.n = (int)n1.size();
        t2.n = (int)n2.size();
        H2_HIP(hipStreamSynchronize(s));
    };
    // coupling: every node with a basis writes its yhat (zero without IL)
    make(h.h_rank, h.h_il_ptr, true, h.cp_t1, h.cp_t2);
    // nearfield: leaves with near entries (a leaf's own block is one)
    std::vector<int> leaf_rows(h.nnode, 0);
    for (int i = 0; i < h.nnode; ++i)
        if (h.h_nchild[i] == 0) leaf_rows[i] = h.h_count[i];
    make(leaf_rows, h.h_nr_ptr, false, h.nr_t1, h.nr_t2);
    std::vector<int64_t> st(h.h_start.begin(), h.h_start.end());
    h.start64.ensure(std::max<size_t>(st.size(), 1), s);
    H2_HIP(hipMemcpyAsync(h.start64.p, st.data(), st.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    H2_HIP(hipStreamSynchronize(s));
}

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
    launch_gemm(h.cp_t1, h.cp_t2, h.il_ptr.p, h.il_col.p, h.rank.p, h.B_off.p, h.B.p, h.xh_off.p, h.xh.p,
                h.xh_off.p, h.yh.p, nrhs, 0, s);
    mark(3);
    for (int L = 1; L < h.maxdepth; ++L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_downward<<<nl, TB, 0, s>>>(lo, nrhs, h.nchild.p, h.first_child.p, h.rank.p, h.mbar.p, h.piv_off.p,
                                     h.piv.p, h.T_off.p, h.T.p, h.xh_off.p, h.yh.p);
        H2_LAUNCH_CHECK();
    }
    mark(4);
    k_leaves_far<<<(unsigned)h.leaves.n, TB, 0, s>>>(nrhs, h.leaves.p, h.start.p, h.count.p, h.rank.p, h.piv_off.p,
                                                     h.piv.p, h.T_off.p, h.T.p, h.xh_off.p, h.yh.p, h.yt.p);
    H2_LAUNCH_CHECK();
    launch_gemm(h.nr_t1, h.nr_t2, h.nr_ptr.p, h.nr_col.p, h.count.p, h.D_off.p, h.D.p, h.start64.p, h.xt.p,
                h.start64.p, h.yt.p, nrhs, 1, s);
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
