// H^2 matrix-vector product y = Ktilde x (the O(n) apply of Section 2.1),
// in FP64 or, in the precision mode, FP32 blocks and vectors with FP32
// matrix-core products per block, compensated (Kahan) accumulation of the
// block products and FP64 accumulation of the interpolation sums.
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

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step per value type.  Operand layout (both types):
// A lane l = A[l%16][l/16], B lane l = B[l/16][l%16].  Result register r of
// lane l holds row 4r + l/16 (FP64) or 4(l/16) + r (FP32) of column l%16.
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double4_t V;
    __device__ static V step(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int r, int k4) { return 4 * r + k4; }
};
template <>
struct Mfma<float> {
    typedef float4_t V;
    __device__ static V step(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int r, int k4) { return 4 * k4 + r; }
};

template <class T>
__global__ __launch_bounds__(TB) void k_gather(const T* __restrict__ x, int64_t n, int nrhs, const int* __restrict__ perm,
                                               T* __restrict__ xt)
{
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= n * nrhs) return;
    int64_t i = q / nrhs;
    int r = (int)(q - i * nrhs);
    xt[q] = x[(int64_t)r * n + perm[i]];
}

template <class T>
__global__ __launch_bounds__(TB) void k_scatter(const T* __restrict__ yt, int64_t n, int nrhs,
                                                const int* __restrict__ perm, T* __restrict__ y)
{
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= n * nrhs) return;
    int64_t i = q / nrhs;
    int r = (int)(q - i * nrhs);
    y[(int64_t)r * n + perm[i]] = yt[q];
}

template <class T>
__global__ __launch_bounds__(TB) void k_upward(int lo, int nrhs, const int* __restrict__ nchild,
                                               const int* __restrict__ first_child, const int* __restrict__ start,
                                               const int* __restrict__ rank, const int* __restrict__ mbar,
                                               const int64_t* __restrict__ piv_off, const int* __restrict__ piv,
                                               const int64_t* __restrict__ T_off, const T* __restrict__ Tm,
                                               const int64_t* __restrict__ xh_off, const T* __restrict__ xt,
                                               T* __restrict__ xh)
{
    const int i = lo + blockIdx.x;
    const int k = rank[i];
    if (k == 0) return;
    const int m = mbar[i], nr = m - k;
    const T* z = nchild[i] == 0 ? xt + (int64_t)start[i] * nrhs : xh + xh_off[first_child[i]] * nrhs;
    const int* pv = piv + piv_off[i];
    const T* Ti = Tm + T_off[i];
    T* o = xh + xh_off[i] * nrhs;
    for (int q = threadIdx.x; q < k * nrhs; q += TB) {
        int t = q / nrhs, r = q - t * nrhs;
        double acc = z[(int64_t)pv[t] * nrhs + r];
        const T* Tr = Ti + (int64_t)t * nr;
        for (int u = 0; u < nr; ++u) acc += (double)Tr[u] * (double)z[(int64_t)pv[k + u] * nrhs + r];
        o[q] = (T)acc;
    }
}

// Batched block products Y[rows of i] (+)= sum_{e in row i} Blk_e X[rows of j_e]
// for the coupling sweep (Blk = B, X = xhat, Y = yhat) and the nearfield
// sweep (Blk = D, X = x_t, Y = y_t).  One wavefront per task (node i, 32-row
// chunk): MT 16-row tiles x 2 16-column tiles of 16x16x4 matrix-core steps,
// the K loop walking the list entries four rows of X at a time.  Blocks are
// column-major, so each 16-lane group of an A load reads 16 contiguous
// values, and X rows are nrhs-contiguous, so B loads are contiguous as well.
// The operands of the next K step are loaded before the current step's
// matrix-core instructions issue.  Workgroup ids are remapped so that each
// XCD (ids round-robin over 8) runs a contiguous range of tasks, keeping the
// shared X rows of neighbouring nodes in one L2.
// COMP: every block's product is formed on its own and added to the running
// sum with Kahan compensation (precision mode).
template <int MT, class T, bool COMP>
__global__ __launch_bounds__(64) void k_blockgemm(int ntask, const int* __restrict__ task_node,
                                                  const int* __restrict__ task_r0, const int* __restrict__ ptr,
                                                  const int* __restrict__ col, const int* __restrict__ krow,
                                                  const int64_t* __restrict__ blk_off, const T* __restrict__ blk,
                                                  const int64_t* __restrict__ in_off, const T* __restrict__ X,
                                                  const int64_t* __restrict__ out_off, T* __restrict__ Y, int nrhs,
                                                  int accumulate)
{
    typedef typename Mfma<T>::V V;
    const int per = (ntask + 7) / 8;
    const int task = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (task >= ntask) return;
    const int i = task_node[task], r0 = task_r0[task];
    const int ki = krow[i];
    const int lane = threadIdx.x, l16 = lane & 15, k4 = lane >> 4;
    const int e0 = ptr[i], e1 = ptr[i + 1];
    for (int c0 = 0; c0 < nrhs; c0 += 32) {
        V acc[MT][2], cmp[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                acc[mt][nt] = (V){0, 0, 0, 0};
                cmp[mt][nt] = (V){0, 0, 0, 0};
            }
        for (int e = e0; e < e1; ++e) {
            const int j = col[e];
            const int kj = krow[j];
            const T* Bb = blk + blk_off[e];
            const T* Xj = X + in_off[j] * nrhs;
            V blkacc[MT][2];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) blkacc[mt][nt] = COMP ? (V){0, 0, 0, 0} : acc[mt][nt];
            T av[MT], bv[2];
            auto load = [&](int u0) {
                const int u = u0 + k4;
                const bool uv = u < kj;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int t = r0 + 16 * mt + l16;
                    av[mt] = (uv && t < ki) ? Bb[(int64_t)u * ki + t] : (T)0;
                }
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int c = c0 + 16 * nt + l16;
                    bv[nt] = (uv && c < nrhs) ? Xj[(int64_t)u * nrhs + c] : (T)0;
                }
            };
            load(0);
            for (int u0 = 0; u0 < kj; u0 += 4) {
                T a_cur[MT], b_cur[2];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a_cur[mt] = av[mt];
                b_cur[0] = bv[0];
                b_cur[1] = bv[1];
                if (u0 + 4 < kj) load(u0 + 4);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) blkacc[mt][nt] = Mfma<T>::step(a_cur[mt], b_cur[nt], blkacc[mt][nt]);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    if (COMP) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            T yk = blkacc[mt][nt][r] - cmp[mt][nt][r];
                            T tk = acc[mt][nt][r] + yk;
                            cmp[mt][nt][r] = (tk - acc[mt][nt][r]) - yk;
                            acc[mt][nt][r] = tk;
                        }
                    } else {
                        acc[mt][nt] = blkacc[mt][nt];
                    }
                }
        }
        T* Yi = Y + out_off[i] * nrhs;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + 16 * mt + Mfma<T>::row(r, k4);
                    const int c = c0 + 16 * nt + l16;
                    if (row < ki && c < nrhs) {
                        T* dst = Yi + (int64_t)row * nrhs + c;
                        T v = COMP ? acc[mt][nt][r] - cmp[mt][nt][r] : acc[mt][nt][r];
                        *dst = accumulate ? *dst + v : v;
                    }
                }
    }
}

// The interpolation sums (up to a few hundred terms) accumulate in FP64 in
// both modes; the FP32 mode stores and loads FP32 operands only.
// w[piv pos] (+)= (U yhat)[pos]: pos < k -> yhat[pos]; else sum_t T[t, pos-k] yhat[t]
template <class T>
__device__ inline T u_times(int pos, int k, int nr, int r, int nrhs, const T* __restrict__ Ti,
                            const T* __restrict__ yhat)
{
    if (pos < k) return yhat[(int64_t)pos * nrhs + r];
    int u = pos - k;
    double acc = 0;
    for (int t = 0; t < k; ++t) acc += (double)Ti[(int64_t)t * nr + u] * (double)yhat[(int64_t)t * nrhs + r];
    return (T)acc;
}

template <class T>
__global__ __launch_bounds__(TB) void k_downward(int lo, int nrhs, const int* __restrict__ nchild,
                                                 const int* __restrict__ first_child, const int* __restrict__ rank,
                                                 const int* __restrict__ mbar, const int64_t* __restrict__ piv_off,
                                                 const int* __restrict__ piv, const int64_t* __restrict__ T_off,
                                                 const T* __restrict__ Tm, const int64_t* __restrict__ xh_off,
                                                 T* __restrict__ yh)
{
    const int i = lo + blockIdx.x;
    const int k = rank[i];
    if (k == 0 || nchild[i] == 0) return;
    const int m = mbar[i], nr = m - k;
    const int* pv = piv + piv_off[i];
    const T* Ti = Tm + T_off[i];
    const T* yi = yh + xh_off[i] * nrhs;
    T* yc = yh + xh_off[first_child[i]] * nrhs;
    for (int q = threadIdx.x; q < m * nrhs; q += TB) {
        int pos = q / nrhs, r = q - pos * nrhs;
        yc[(int64_t)pv[pos] * nrhs + r] += u_times(pos, k, nr, r, nrhs, Ti, yi);
    }
}

// Far part of the leaves: y_t(X_i) = U_i yhat_i (zero when the leaf has no
// farfield); the nearfield sweep then accumulates into the same rows.
template <class T>
__global__ __launch_bounds__(TB) void k_leaves_far(int nrhs, const int* __restrict__ leaves,
                                                   const int* __restrict__ start, const int* __restrict__ count,
                                                   const int* __restrict__ rank, const int64_t* __restrict__ piv_off,
                                                   const int* __restrict__ piv, const int64_t* __restrict__ T_off,
                                                   const T* __restrict__ Tm, const int64_t* __restrict__ xh_off,
                                                   const T* __restrict__ yh, T* __restrict__ yt)
{
    const int i = leaves[blockIdx.x];
    const int k = rank[i];
    const int m = count[i], nr = m - k;
    T* yo = yt + (int64_t)start[i] * nrhs;
    if (k > 0) {
        const int* pv = piv + piv_off[i];
        const T* Ti = Tm + T_off[i];
        const T* yi = yh + xh_off[i] * nrhs;
        for (int q = threadIdx.x; q < m * nrhs; q += TB) {
            int pos = q / nrhs, r = q - pos * nrhs;
            yo[(int64_t)pv[pos] * nrhs + r] = u_times(pos, k, nr, r, nrhs, Ti, yi);
        }
    } else {
        for (int q = threadIdx.x; q < m * nrhs; q += TB) yo[q] = (T)0;
    }
}

__global__ __launch_bounds__(TB) void k_to_f32(const double* __restrict__ a, int64_t n, float* __restrict__ b)
{
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q < n) b[q] = (float)a[q];
}

template <class T, bool COMP>
void launch_gemm(const Handle::Tasks& t1, const Handle::Tasks& t2, const int* ptr, const int* col, const int* krow,
                 const int64_t* blk_off, const T* blk, const int64_t* in_off, const T* X, const int64_t* out_off,
                 T* Y, int nrhs, int accumulate, hipStream_t s)
{
    if (t1.n > 0) {
        unsigned grid = (unsigned)(8 * ((t1.n + 7) / 8));
        k_blockgemm<1, T, COMP><<<grid, 64, 0, s>>>(t1.n, t1.node.p, t1.r0.p, ptr, col, krow, blk_off, blk, in_off,
                                                    X, out_off, Y, nrhs, accumulate);
        H2_LAUNCH_CHECK();
    }
    if (t2.n > 0) {
        unsigned grid = (unsigned)(8 * ((t2.n + 7) / 8));
        k_blockgemm<2, T, COMP><<<grid, 64, 0, s>>>(t2.n, t2.node.p, t2.r0.p, ptr, col, krow, blk_off, blk, in_off,
                                                    X, out_off, Y, nrhs, accumulate);
        H2_LAUNCH_CHECK();
    }
}

template <class T>
struct ApplyBufs;
template <>
struct ApplyBufs<double> {
    static DBuf<double>& xt(Handle& h) { return h.xt; }
    static DBuf<double>& yt(Handle& h) { return h.yt; }
    static DBuf<double>& xh(Handle& h) { return h.xh; }
    static DBuf<double>& yh(Handle& h) { return h.yh; }
    static const double* B(Handle& h) { return h.B.p; }
    static const double* D(Handle& h) { return h.D.p; }
    static const double* Tm(Handle& h) { return h.T.p; }
};
template <>
struct ApplyBufs<float> {
    static DBuf<float>& xt(Handle& h) { return h.xtf; }
    static DBuf<float>& yt(Handle& h) { return h.ytf; }
    static DBuf<float>& xh(Handle& h) { return h.xhf; }
    static DBuf<float>& yh(Handle& h) { return h.yhf; }
    static const float* B(Handle& h) { return h.Bf.p; }
    static const float* D(Handle& h) { return h.Df.p; }
    static const float* Tm(Handle& h) { return h.Tf.p; }
};

template <class T>
void matvec_t(Handle& h, const T* x, T* y, int nrhs, hipStream_t s)
{
    typedef ApplyBufs<T> AB;
    const int64_t n = h.n;
    if (nrhs > h.mv_nrhs) {
        H2_HIP(hipStreamSynchronize(s));
        AB::xt(h).ensure((size_t)n * nrhs, s);
        AB::yt(h).ensure((size_t)n * nrhs, s);
        AB::xh(h).ensure((size_t)std::max<int64_t>(h.sum_rank, 1) * nrhs, s);
        AB::yh(h).ensure((size_t)std::max<int64_t>(h.sum_rank, 1) * nrhs, s);
        h.mv_nrhs = nrhs;
    }
    T* xt = AB::xt(h).p;
    T* yt = AB::yt(h).p;
    T* xh = AB::xh(h).p;
    T* yh = AB::yh(h).p;
    const T* Tm = AB::Tm(h);
    const bool prof = h.profile != 0;
    auto mark = [&](int e) {
        if (prof) H2_HIP(hipEventRecord(h.ev[e], s));
    };
    if (prof && !h.ev[0])
        for (auto& e : h.ev) H2_HIP(hipEventCreate(&e));
    mark(0);
    k_gather<T><<<blocks_for(n * nrhs, TB), TB, 0, s>>>(x, n, nrhs, h.perm.p, xt);
    H2_LAUNCH_CHECK();
    mark(1);
    for (int L = h.maxdepth; L >= 1; --L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_upward<T><<<nl, TB, 0, s>>>(lo, nrhs, h.nchild.p, h.first_child.p, h.start.p, h.rank.p, h.mbar.p,
                                      h.piv_off.p, h.piv.p, h.T_off.p, Tm, h.xh_off.p, xt, xh);
        H2_LAUNCH_CHECK();
    }
    mark(2);
    // the precision mode adds each block product (one interaction) to the
    // row sums with compensation: FP32 recursion over the ~10^4 terms of an
    // interaction list would lose about sqrt(10^4) ulps
    launch_gemm<T, sizeof(T) == 4>(h.cp_t1, h.cp_t2, h.il_ptr.p, h.il_col.p, h.rank.p, h.B_off.p, AB::B(h), h.xh_off.p, xh,
                          h.xh_off.p, yh, nrhs, 0, s);
    mark(3);
    for (int L = 1; L < h.maxdepth; ++L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_downward<T><<<nl, TB, 0, s>>>(lo, nrhs, h.nchild.p, h.first_child.p, h.rank.p, h.mbar.p, h.piv_off.p,
                                        h.piv.p, h.T_off.p, Tm, h.xh_off.p, yh);
        H2_LAUNCH_CHECK();
    }
    mark(4);
    k_leaves_far<T><<<(unsigned)h.leaves.n, TB, 0, s>>>(nrhs, h.leaves.p, h.start.p, h.count.p, h.rank.p,
                                                        h.piv_off.p, h.piv.p, h.T_off.p, Tm, h.xh_off.p, yh, yt);
    H2_LAUNCH_CHECK();
    // the precision mode accumulates the nearfield blocks with compensation
    launch_gemm<T, sizeof(T) == 4>(h.nr_t1, h.nr_t2, h.nr_ptr.p, h.nr_col.p, h.count.p, h.D_off.p, AB::D(h),
                                   h.start64.p, xt, h.start64.p, yt, nrhs, 1, s);
    mark(5);
    k_scatter<T><<<blocks_for(n * nrhs, TB), TB, 0, s>>>(yt, n, nrhs, h.perm.p, y);
    H2_LAUNCH_CHECK();
    mark(6);
    if (prof) {
        h.prof_valid = true;
        h.prof_nrhs = nrhs;
    }
}

}  // namespace

// Task lists of the two block sweeps, built once per handle; in the
// precision mode also the FP32 copy of the interpolation matrices.
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
    if (h.precision == 32) {
        const int64_t nt = std::max<int64_t>(h.h_T_off[h.nnode], 1);
        h.Tf.ensure((size_t)nt, s);
        k_to_f32<<<blocks_for(nt, TB), TB, 0, s>>>(h.T.p, nt, h.Tf.p);
        H2_LAUNCH_CHECK();
    }
    H2_HIP(hipStreamSynchronize(s));
}

void matvec(Handle& h, const void* x, void* y, int nrhs, hipStream_t s)
{
    if (h.precision == 32)
        matvec_t<float>(h, (const float*)x, (float*)y, nrhs, s);
    else
        matvec_t<double>(h, (const double*)x, (double*)y, nrhs, s);
}

}  // namespace h2
