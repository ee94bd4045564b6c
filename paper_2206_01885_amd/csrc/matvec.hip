// H^2 matrix-vector product y = Ktilde x (the O(n) apply of Section 2.1),
// in FP64 or, in the precision mode, FP32 blocks and vectors with FP32
// matrix-core products per block, compensated (Kahan) accumulation of the
// block products and FP64 accumulation of the interpolation sums.
//
// Vectors live in tree order as [n][ld] (right-hand sides fastest, ld =
// nrhs rounded up to 32); the node coefficients xhat_i, yhat_i as
// [rank_i][ld] blocks laid out in node id order, so the children of a node
// (consecutive ids) own one contiguous block: the input rows z_p of a
// parent's interpolation step are exactly its children's xhat concatenated,
// as in the row set Xbar_p of Algorithm 2.  Columns nrhs .. ld-1 are never
// initialised: every product below is column-independent, so whatever they
// hold reaches only columns nrhs .. ld-1 of the results, which are never read.
//
//   gather    x_t = x[perm]
//   upward    xhat_i = U_i^T z_i, z_i = x_t(X_i) (leaf) or children's xhat;
//             U_i = P [I; T^T] so xhat[t] = z[piv t] + sum_u T[t,u] z[piv(k+u)]
//   coupling  yhat_i = sum_{j in IL(i)} B_ij xhat_j
//   downward  children's yhat += U_p yhat_p   (depth 1 first)
//   leaves    y_t(X_i) = U_i yhat_i + sum_{j in near(i)} D_ij x_t(X_j)
//   scatter   y[perm] = y_t
// Every output element has exactly one writer; there are no atomics.
#include <mutex>
#include <string>

#include "common.h"
#include "kappa.h"
#include "mfma.h"

namespace h2 {
namespace {

constexpr int TB = 256;

// n contiguous values loaded as one (unaligned) vector access
template <class T, int N>
struct Vec {
    T v[N];
};
template <class T, int N>
__device__ __forceinline__ Vec<T, N> vload(const T* p)
{
    Vec<T, N> r;
    __builtin_memcpy(&r, p, sizeof(r));
    return r;
}

// Caller order (x, y: nrhs rows of n) <-> tree order (xt, yt: ld values per
// point), through a tile of 64 consecutive caller-order points x 32 RHS in
// LDS: a row of x / y is read / written as 64 contiguous values and a
// point's RHS as one contiguous run; iperm[j] is the tree position of the
// caller's point j.  Grid (ceil(n / 64), ceil(nrhs / 32)), TB threads.
template <class T>
__global__ __launch_bounds__(TB) void k_gather(const T* __restrict__ x, int64_t n, int nrhs, int ld,
                                               const int* __restrict__ iperm, T* __restrict__ xt)
{
    __shared__ T tile[64][33];
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 32, nr = min(32, nrhs - c0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (j0 + lane < n)
        for (int r = wv; r < nr; r += TB / 64) tile[lane][r] = x[(int64_t)(c0 + r) * n + j0 + lane];
    __syncthreads();
    const int rr = threadIdx.x & 31;
    for (int p = threadIdx.x >> 5; p < 64; p += TB / 32)
        if (j0 + p < n && rr < nr) xt[(int64_t)iperm[j0 + p] * ld + c0 + rr] = tile[p][rr];
}

template <class T>
__global__ __launch_bounds__(TB) void k_scatter(const T* __restrict__ yt, int64_t n, int nrhs, int ld,
                                                const int* __restrict__ iperm, T* __restrict__ y)
{
    __shared__ T tile[64][33];
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 32, nr = min(32, nrhs - c0);
    const int rr = threadIdx.x & 31;
    for (int p = threadIdx.x >> 5; p < 64; p += TB / 32)
        if (j0 + p < n && rr < nr) tile[p][rr] = yt[(int64_t)iperm[j0 + p] * ld + c0 + rr];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (j0 + lane < n)
        for (int r = wv; r < nr; r += TB / 64) y[(int64_t)(c0 + r) * n + j0 + lane] = tile[lane][r];
}

// Inverse of the tree permutation: iperm[perm[i]] = i.
__global__ __launch_bounds__(TB) void k_invert_perm(int64_t n, const int* __restrict__ perm, int* __restrict__ iperm)
{
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < n) iperm[perm[i]] = (int)i;
}

// The interpolation sums (up to a few hundred terms) accumulate in FP64 in
// both modes; the FP32 mode stores and loads FP32 operands only.
template <class T>
__global__ __launch_bounds__(TB) void k_upward(int lo, int nrhs, int ld, const int* __restrict__ nchild,
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
    const T* z = nchild[i] == 0 ? xt + (int64_t)start[i] * ld : xh + xh_off[first_child[i]] * ld;
    const int* pv = piv + piv_off[i];
    const T* Ti = Tm + T_off[i];
    T* o = xh + xh_off[i] * ld;
    for (int q = threadIdx.x; q < k * nrhs; q += TB) {
        int t = q / nrhs, r = q - t * nrhs;
        double acc = z[(int64_t)pv[t] * ld + r];
        const T* Tr = Ti + (int64_t)t * nr;
        // unrolled so that the loads run ahead of the (in-order) sum
#pragma unroll 8
        for (int u = 0; u < nr; ++u) acc += (double)Tr[u] * (double)z[(int64_t)pv[k + u] * ld + r];
        o[(int64_t)t * ld + r] = (T)acc;
    }
}

// Batched block products Y[rows of i] (+)= sum_{e in row i} Blk_e X[rows of j_e]
// for the coupling sweep (Blk = B, X = xhat, Y = yhat) and the nearfield
// sweep (Blk = D, X = x_t, Y = y_t).  The blocks of one list row are stored
// back to back, each column-major with leading dimension rows_i, so row i's
// blocks together are one rows_i x (sum of columns) column-major matrix and
// the sweep over a row is one long K loop.
//
// Row i's entries are [ptr_b[i], ptr_e[i]).
// One wavefront per task (node i, rows r0 .. r0 + 16 MT - 1, 32 columns of
// X per pass): MT 16-row tiles x 2 16-column tiles of 16x16x4 matrix-core
// steps, four columns of the row matrix (four rows of X) per step.  The
// tiles are interleaved so that every lane's operands are contiguous: lane
// (q, g) = (l%16, l/16) loads rows r0 + MT q .. r0 + MT q + MT - 1 of column
// g of the step (tile mt takes row MT q + mt) and columns 2q, 2q+1 of row g
// of X (tile nt takes column 2q + nt), each as one vector access.  Rows past
// the block (the last tile of a node) compute values that are never stored;
// columns past a block's last column (its last step) read zeros from `zero`.
// The addresses move by one scalar offset per step.  Loads run P steps ahead
// of the matrix-core instructions through a register ring, across block
// boundaries; the next entry's metadata (columns, first input row) is read
// one entry ahead.  The loop runs a multiple of P steps; the surplus steps
// read zeros.  Workgroup ids are remapped so that each XCD (ids round-robin
// over 8) runs a contiguous range of tasks, keeping the X rows shared by
// neighbouring nodes in one L2.
// COMP: every block's product is formed on its own and added to the running
// sum with Kahan compensation (precision mode).
template <int MT, class T, bool COMP, int P>
__global__ __launch_bounds__(64) void k_sweep(int ntask, const int* __restrict__ task_node,
                                              const int* __restrict__ task_r0, const int* __restrict__ ptr_b,
                                              const int* __restrict__ ptr_e,
                                              const int* __restrict__ ek, const int64_t* __restrict__ ex,
                                              const int* __restrict__ nsteps, const int* __restrict__ krow,
                                              const int64_t* __restrict__ blk_off, const T* __restrict__ blk,
                                              const T* __restrict__ X, const int64_t* __restrict__ out_off,
                                              T* __restrict__ Y, int nchunk, int ld, int accumulate,
                                              const T* __restrict__ zero)
{
    typedef typename Mfma<T>::V V;
    const int per = (ntask + 7) / 8;
    const int task = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (task >= ntask) return;
    const int i = task_node[task], r0 = task_r0[task];
    const int ki = krow[i];
    const int lane = threadIdx.x, q = lane & 15, g = lane >> 4;
    const int e0 = ptr_b[i], e1 = ptr_e[i];
    const int S = nsteps[i];
    const int SP = (S + P - 1) / P * P;
    // lane bases: column g of the row matrix at row r0 + MT q; row g of X
    const T* baseA = blk + (e0 < e1 ? blk_off[e0] : 0) + (int64_t)g * ki + r0 + MT * q;
    for (int c = 0; c < nchunk; ++c) {
        const T* baseX = X + (int64_t)g * ld + 32 * c + 2 * q;
        V acc[MT][2], cmp[MT][2], bacc[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                acc[mt][nt] = (V){0, 0, 0, 0};
                cmp[mt][nt] = (V){0, 0, 0, 0};
                bacc[mt][nt] = (V){0, 0, 0, 0};
            }
        // loader state (wave-uniform): entry le, column lu within it, its
        // column count lk and first input row lx, first column lkst of the
        // entry in the row matrix; nk, nx: metadata of entry le + 1.  An entry
        // without columns (a partner of rank 0) takes one all-zero step.
        int le = e0, lu = 0, lk = 0, nk = 0;
        int64_t lx = 0, nx = 0, lkst = 0;
        if (e0 < e1) {
            lk = ek[e0];
            lx = ex[e0];
        }
        if (e0 + 1 < e1) {
            nk = ek[e0 + 1];
            nx = ex[e0 + 1];
        }
        Vec<T, MT> av[P];
        Vec<T, 2> bv[P];
        bool last[P];
        auto load = [&](Vec<T, MT>& a, Vec<T, 2>& b, bool& lst) {
            const bool uv = lu + g < lk;
            const T* pa = baseA + (lkst + lu) * ki;
            const T* px = baseX + (lx + lu) * ld;
            a = vload<T, MT>(uv ? pa : zero);
            b = vload<T, 2>(uv ? px : zero);
            lu += 4;
            lst = le < e1 && lu >= lk;
            if (lst) {
                lkst += lk;
                lu = 0;
                ++le;
                lk = nk;
                lx = nx;
                if (le + 1 < e1) {
                    nk = ek[le + 1];
                    nx = ex[le + 1];
                } else {
                    nk = 0;
                }
            }
        };
#pragma unroll
        for (int p = 0; p < P; ++p) load(av[p], bv[p], last[p]);
        for (int s0 = 0; s0 < SP; s0 += P) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                // consume slot p, then refill it (the old operands die at
                // their matrix-core instructions, so the refill reuses their
                // registers)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) {
                        if (COMP)
                            bacc[mt][nt] = Mfma<T>::step(av[p].v[mt], bv[p].v[nt], bacc[mt][nt]);
                        else
                            acc[mt][nt] = Mfma<T>::step(av[p].v[mt], bv[p].v[nt], acc[mt][nt]);
                    }
                const bool lst = last[p];
                load(av[p], bv[p], last[p]);
                if (COMP && lst) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                T yk = bacc[mt][nt][r] - cmp[mt][nt][r];
                                T tk = acc[mt][nt][r] + yk;
                                cmp[mt][nt][r] = (tk - acc[mt][nt][r]) - yk;
                                acc[mt][nt][r] = tk;
                            }
                            bacc[mt][nt] = (V){0, 0, 0, 0};
                        }
                }
            }
        }
        // tile (mt, nt) row w, column q = node row r0 + MT w + mt, column 2q + nt
        T* Yi = Y + out_off[i] * ld + 32 * c + 2 * q;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + MT * Mfma<T>::row(r, g) + mt;
                if (row < ki) {
                    Vec<T, 2> v;
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        v.v[nt] = COMP ? acc[mt][nt][r] - cmp[mt][nt][r] : acc[mt][nt][r];
                    T* dst = Yi + (int64_t)row * ld;
                    if (accumulate) {
                        const Vec<T, 2> o = vload<T, 2>(dst);
                        v.v[0] += o.v[0];
                        v.v[1] += o.v[1];
                    }
                    __builtin_memcpy(dst, &v, sizeof(v));
                }
            }
    }
}

// Coupling sweep without stored blocks (store_coupling = 0, FP64):
// yhat_i = sum_{j in IL(i)} K(Xhat_i^(row), Xhat_j^(col)) xhat_j with every
// block entry evaluated where it is used.  One wavefront per (node, 64-row
// chunk): lane t holds skeleton point t of node i and 32 accumulators (one
// 32-column slice of the right-hand sides at a time); the partner's
// skeleton points and xhat rows are staged in LDS 32 columns at a time and
// read as broadcasts (faster here than scalar-register operands read through
// the scalar cache).  Entries are summed in list order, columns ascending.
template <int FAM>
__global__ __launch_bounds__(64) void k_coupling_otf(int ntask, const int* __restrict__ task_node,
                                                     const int* __restrict__ task_r0, const int* __restrict__ ptr,
                                                     const int* __restrict__ col, const int* __restrict__ krow,
                                                     const int* __restrict__ kcol, const double* __restrict__ sr,
                                                     int64_t ldr, const int64_t* __restrict__ offr,
                                                     const double* __restrict__ sc, int64_t ldc,
                                                     const int64_t* __restrict__ offc, int d, int kid, double prm,
                                                     const double* __restrict__ X, double* __restrict__ Y, int ld)
{
    constexpr int UC = 32;
    __shared__ double sy[3][UC];
    __shared__ double sx[UC * 32];
    const int per = (ntask + 7) / 8;
    const int task = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (task >= ntask) return;
    const int i = task_node[task], r0 = task_r0[task];
    const int ki = krow[i];
    const int lane = threadIdx.x;
    const int t = r0 + lane;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (t < ki) {
        x0 = sr[offr[i] + t];
        if (d > 1) x1 = sr[ldr + offr[i] + t];
        if (d > 2) x2 = sr[2 * ldr + offr[i] + t];
    }
    const int e0 = ptr[i], e1 = ptr[i + 1];
    for (int c = 0; c < ld; c += 32) {
        double acc[32];
#pragma unroll
        for (int r = 0; r < 32; ++r) acc[r] = 0.0;
        for (int e = e0; e < e1; ++e) {
            const int j = col[e];
            const int kj = kcol[j];
            const int64_t oj = offc[j];
            for (int u0 = 0; u0 < kj; u0 += UC) {
                const int uc = min(UC, kj - u0);
                __syncthreads();  // the previous pass has read the slices
                if (lane < uc) {
                    sy[0][lane] = sc[oj + u0 + lane];
                    if (d > 1) sy[1][lane] = sc[ldc + oj + u0 + lane];
                    if (d > 2) sy[2][lane] = sc[2 * ldc + oj + u0 + lane];
                }
                for (int q = lane; q < uc * 32; q += 64) sx[q] = X[(oj + u0 + (q >> 5)) * (int64_t)ld + c + (q & 31)];
                __syncthreads();
                for (int u = 0; u < uc; ++u) {
                    const double s0 = sy[0][u];
                    const double s1 = d > 1 ? sy[1][u] : 0.0;
                    const double s2 = d > 2 ? sy[2][u] : 0.0;
                    double r2 = 0.0, xy = 0.0;
                    // (fused multiply-adds written out, as in the block
                    // evaluation of the stored path)
                    if constexpr (FAM == FAM_COSINE) {
                        xy = x0 * s0;
                        if (d > 1) xy = __builtin_fma(x1, s1, xy);
                        if (d > 2) xy = __builtin_fma(x2, s2, xy);
                    } else {
                        const double a0 = s0 - x0;
                        r2 = a0 * a0;
                        if (d > 1) {
                            const double a1 = s1 - x1;
                            r2 = __builtin_fma(a1, a1, r2);
                        }
                        if (d > 2) {
                            const double a2 = s2 - x2;
                            r2 = __builtin_fma(a2, a2, r2);
                        }
                    }
                    const double kv = kappa_store<double, FAM>(kid, prm, r2, xy, x0 - s0);
#pragma unroll
                    for (int r = 0; r < 32; ++r) acc[r] += kv * sx[u * 32 + r];
                }
            }
        }
        if (t < ki) {
            double* yr = Y + (offr[i] + t) * (int64_t)ld + c;
#pragma unroll
            for (int r = 0; r < 32; ++r) yr[r] = acc[r];
        }
    }
}

// Transposed coupling sweep of a symmetric kernel's stored blocks:
// Y[rows of i] += sum_{e in [ptr_b[i], ptr_e[i])} B_e^T X[rows of j_e],
// where B_e (blk + blk_off[e]) is the stored k_j x k_i block B_ji,
// column-major with leading dimension k_j, so row a of B_ij = B_ji^T is its
// column a, k_j contiguous values.  Same task and tile layout as k_sweep
// (lane (q, g), rows r0 + MT q + mt, columns 2q + nt of a 32-column pass),
// but the K loop goes 16 columns of B_ij at a time: lane group g takes
// columns 16 b + 4 g .. 16 b + 4 g + 3, one vector load per row tile, and the
// four matrix-core steps of the block pair them with X rows 16 b + 4 g + t
// (t = 0..3) -- a reordering of the sum over the block's columns.  X rows
// past k_j read zeros, so the A values loaded past a column's end (the next
// column's first entries, or the zero padding after the last block) add
// nothing; rows past k_i read zeros.  Loads run P blocks ahead through a
// register ring, across entries.  COMP: Kahan accumulation of the block
// products, as in k_sweep.
template <int MT, class T, bool COMP, int P>
__global__ __launch_bounds__(64) void k_sweep_t(int ntask, const int* __restrict__ task_node,
                                                const int* __restrict__ task_r0, const int* __restrict__ ptr_b,
                                                const int* __restrict__ ptr_e, const int* __restrict__ ek,
                                                const int64_t* __restrict__ ex, const int* __restrict__ nblk,
                                                const int* __restrict__ krow, const int64_t* __restrict__ blk_off,
                                                const T* __restrict__ blk, const T* __restrict__ X,
                                                const int64_t* __restrict__ out_off, T* __restrict__ Y, int nchunk,
                                                int ld, const T* __restrict__ zero)
{
    typedef typename Mfma<T>::V V;
    const int per = (ntask + 7) / 8;
    const int task = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (task >= ntask) return;
    const int i = task_node[task], r0 = task_r0[task];
    const int ki = krow[i];
    const int lane = threadIdx.x, q = lane & 15, g = lane >> 4;
    const int e0 = ptr_b[i], e1 = ptr_e[i];
    const int S = nblk[i];
    const int SP = (S + P - 1) / P * P;
    bool rv[MT];  // rows of this lane inside the block
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) rv[mt] = r0 + MT * q + mt < ki;
    for (int c = 0; c < nchunk; ++c) {
        const T* baseX = X + 32 * c + 2 * q;
        V acc[MT][2], cmp[MT][2], bacc[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                acc[mt][nt] = (V){0, 0, 0, 0};
                cmp[mt][nt] = (V){0, 0, 0, 0};
                bacc[mt][nt] = (V){0, 0, 0, 0};
            }
        // loader state (wave-uniform): entry le, first column lu of the next
        // 16-column block, the entry's columns lk, first input row lx and
        // block offset lo; nk, nx, no: the same for entry le + 1 (read one
        // entry ahead); an entry without columns takes one all-zero block
        int le = e0, lu = 0, lk = 0, nk = 0;
        int64_t lx = 0, lo = 0, nx = 0, no = 0;
        if (e0 < e1) {
            lk = ek[e0];
            lx = ex[e0];
            lo = blk_off[e0];
        }
        if (e0 + 1 < e1) {
            nk = ek[e0 + 1];
            nx = ex[e0 + 1];
            no = blk_off[e0 + 1];
        }
        Vec<T, 4> av[P][MT];
        Vec<T, 2> xv[P][4];
        bool last[P];
        auto load = [&](Vec<T, 4>* a, Vec<T, 2>* x, bool& lst) {
            const int k0 = lu + 4 * g;
            const bool kv = le < e1 && k0 < lk;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const T* pa = blk + lo + (int64_t)(r0 + MT * q + mt) * lk + k0;
                a[mt] = vload<T, 4>(kv && rv[mt] ? pa : zero);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T* px = baseX + (lx + k0 + t) * ld;
                x[t] = vload<T, 2>(le < e1 && k0 + t < lk ? px : zero);
            }
            lu += 16;
            lst = le < e1 && lu >= lk;
            if (lst) {
                lu = 0;
                ++le;
                lk = nk;
                lx = nx;
                lo = no;
                if (le + 1 < e1) {
                    nk = ek[le + 1];
                    nx = ex[le + 1];
                    no = blk_off[le + 1];
                } else {
                    nk = 0;
                }
            }
        };
#pragma unroll
        for (int p = 0; p < P; ++p) load(av[p], xv[p], last[p]);
        for (int s0 = 0; s0 < SP; s0 += P) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) {
                            if (COMP)
                                bacc[mt][nt] = Mfma<T>::step(av[p][mt].v[t], xv[p][t].v[nt], bacc[mt][nt]);
                            else
                                acc[mt][nt] = Mfma<T>::step(av[p][mt].v[t], xv[p][t].v[nt], acc[mt][nt]);
                        }
                const bool lst = last[p];
                load(av[p], xv[p], last[p]);
                if (COMP && lst) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                T yk = bacc[mt][nt][r] - cmp[mt][nt][r];
                                T tk = acc[mt][nt][r] + yk;
                                cmp[mt][nt][r] = (tk - acc[mt][nt][r]) - yk;
                                acc[mt][nt][r] = tk;
                            }
                            bacc[mt][nt] = (V){0, 0, 0, 0};
                        }
                }
            }
        }
        // added to the rows the upper sweep wrote
        T* Yi = Y + out_off[i] * ld + 32 * c + 2 * q;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + MT * Mfma<T>::row(r, g) + mt;
                if (row < ki) {
                    T* dst = Yi + (int64_t)row * ld;
                    Vec<T, 2> v = vload<T, 2>(dst);
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) v.v[nt] += COMP ? acc[mt][nt][r] - cmp[mt][nt][r] : acc[mt][nt][r];
                    __builtin_memcpy(dst, &v, sizeof(v));
                }
            }
    }
}

// Per-entry metadata of a list (columns, first input row), for every entry.
__global__ __launch_bounds__(TB) void k_entry_meta(int nrow, const int* __restrict__ ptr, const int* __restrict__ col,
                                                   const int* __restrict__ kcol, const int64_t* __restrict__ in_off,
                                                   int* __restrict__ ek, int64_t* __restrict__ ex)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
        const int j = col[e];
        ek[e] = kcol[j];
        ex[e] = in_off[j];
    }
}

// Per-node counts of the K-loop units over entries [ptr_b[i], ptr_e[i]):
// units of `width` columns, at least one per entry.
__global__ __launch_bounds__(TB) void k_range_units(int nrow, const int* __restrict__ ptr_b,
                                                    const int* __restrict__ ptr_e, const int* __restrict__ ek, int width,
                                                    int* __restrict__ units)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    int st = 0;
    for (int e = ptr_b[i]; e < ptr_e[i]; ++e) {
        const int k = ek[e];
        st += k > 0 ? (k + width - 1) / width : 1;
    }
    units[i] = st;
}

// Per-entry metadata of a list (columns, first input row) and per-node
// step counts of the sweep (an entry without columns takes one step).
__global__ __launch_bounds__(TB) void k_sweep_meta(int nrow, const int* __restrict__ ptr, const int* __restrict__ col,
                                                   const int* __restrict__ kcol, const int64_t* __restrict__ in_off,
                                                   int* __restrict__ ek, int64_t* __restrict__ ex,
                                                   int* __restrict__ nsteps)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    int st = 0;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
        const int j = col[e];
        const int k = kcol[j];
        ek[e] = k;
        ex[e] = in_off[j];
        st += k > 0 ? (k + 3) / 4 : 1;
    }
    nsteps[i] = st;
}

// w[piv pos] (+)= (U yhat)[pos]: pos < k -> yhat[pos]; else sum_t T[t, pos-k] yhat[t]
template <class T>
__device__ inline T u_times(int pos, int k, int nr, int r, int ld, const T* __restrict__ Ti,
                            const T* __restrict__ yhat)
{
    if (pos < k) return yhat[(int64_t)pos * ld + r];
    int u = pos - k;
    double acc = 0;
#pragma unroll 8
    for (int t = 0; t < k; ++t) acc += (double)Ti[(int64_t)t * nr + u] * (double)yhat[(int64_t)t * ld + r];
    return (T)acc;
}

template <class T>
__global__ __launch_bounds__(TB) void k_downward(int lo, int nrhs, int ld, const int* __restrict__ nchild,
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
    const T* yi = yh + xh_off[i] * ld;
    T* yc = yh + xh_off[first_child[i]] * ld;
    for (int q = threadIdx.x; q < m * nrhs; q += TB) {
        int pos = q / nrhs, r = q - pos * nrhs;
        yc[(int64_t)pv[pos] * ld + r] += u_times(pos, k, nr, r, ld, Ti, yi);
    }
}

// Far part of the leaves: y_t(X_i) = U_i yhat_i (zero when the leaf has no
// farfield); the nearfield sweep then accumulates into the same rows.
template <class T>
__global__ __launch_bounds__(TB) void k_leaves_far(int nrhs, int ld, const int* __restrict__ leaves,
                                                   const int* __restrict__ start, const int* __restrict__ count,
                                                   const int* __restrict__ rank, const int64_t* __restrict__ piv_off,
                                                   const int* __restrict__ piv, const int64_t* __restrict__ T_off,
                                                   const T* __restrict__ Tm, const int64_t* __restrict__ xh_off,
                                                   const T* __restrict__ yh, T* __restrict__ yt)
{
    const int i = leaves[blockIdx.x];
    const int k = rank[i];
    const int m = count[i], nr = m - k;
    T* yo = yt + (int64_t)start[i] * ld;
    if (k > 0) {
        const int* pv = piv + piv_off[i];
        const T* Ti = Tm + T_off[i];
        const T* yi = yh + xh_off[i] * ld;
        for (int q = threadIdx.x; q < m * nrhs; q += TB) {
            int pos = q / nrhs, r = q - pos * nrhs;
            yo[(int64_t)pv[pos] * ld + r] = u_times(pos, k, nr, r, ld, Ti, yi);
        }
    } else {
        for (int q = threadIdx.x; q < m * nrhs; q += TB) {
            int pos = q / nrhs, r = q - pos * nrhs;
            yo[(int64_t)pos * ld + r] = (T)0;
        }
    }
}

__global__ __launch_bounds__(TB) void k_to_f32(const double* __restrict__ a, int64_t n, float* __restrict__ b)
{
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q < n) b[q] = (float)a[q];
}

template <int MT, class T, bool COMP>
void launch_sweep_mt(const Handle::Sweep& w, const int* ptr_b, const int* ptr_e, const int* krow,
                     const int64_t* blk_off, const T* blk, const T* X, const int64_t* out_off, T* Y, int ld,
                     int accumulate, const T* zero, hipStream_t s)
{
    const int nt = w.n[MT - 1];
    if (nt == 0) return;
    constexpr int P = MT <= 2 ? 4 : 3;
    const unsigned grid = (unsigned)(8 * ((nt + 7) / 8));
    k_sweep<MT, T, COMP, P><<<grid, 64, 0, s>>>(nt, w.node[MT - 1].p, w.r0[MT - 1].p, ptr_b, ptr_e, w.ek.p, w.ex.p,
                                                w.steps.p, krow, blk_off, blk, X, out_off, Y, ld / 32, ld,
                                                accumulate, zero);
    H2_LAUNCH_CHECK();
}

// Row i's entries are [ptr_b[i], ptr_e[i]) (a CSR list: ptr_e = ptr_b + 1).
template <class T, bool COMP>
void launch_sweep(const Handle::Sweep& w, const int* ptr_b, const int* ptr_e, const int* krow,
                  const int64_t* blk_off, const T* blk, const T* X, const int64_t* out_off, T* Y, int ld,
                  int accumulate, const T* zero, hipStream_t s)
{
    launch_sweep_mt<4, T, COMP>(w, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, accumulate, zero, s);
    launch_sweep_mt<3, T, COMP>(w, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, accumulate, zero, s);
    launch_sweep_mt<2, T, COMP>(w, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, accumulate, zero, s);
    launch_sweep_mt<1, T, COMP>(w, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, accumulate, zero, s);
}

// tasks and block counts from w, entry metadata (ek, ex) shared with the
// upper sweep
template <int MT, class T, bool COMP>
void launch_sweep_t_mt(const Handle::Sweep& w, const int* ek, const int64_t* ex, const int* ptr_b, const int* ptr_e,
                       const int* krow, const int64_t* blk_off, const T* blk, const T* X, const int64_t* out_off,
                       T* Y, int ld, const T* zero, hipStream_t s)
{
    const int nt = w.n[MT - 1];
    if (nt == 0) return;
    constexpr int P = H2_TUNE_SWEEP_T_P;  // blocks of 16 columns loaded ahead
    const unsigned grid = (unsigned)(8 * ((nt + 7) / 8));
    k_sweep_t<MT, T, COMP, P><<<grid, 64, 0, s>>>(nt, w.node[MT - 1].p, w.r0[MT - 1].p, ptr_b, ptr_e, ek, ex,
                                                  w.steps.p, krow, blk_off, blk, X, out_off, Y, ld / 32, ld, zero);
    H2_LAUNCH_CHECK();
}

template <class T, bool COMP>
void launch_sweep_t(const Handle::Sweep& w, const int* ek, const int64_t* ex, const int* ptr_b, const int* ptr_e,
                    const int* krow, const int64_t* blk_off, const T* blk, const T* X, const int64_t* out_off, T* Y,
                    int ld, const T* zero, hipStream_t s)
{
    launch_sweep_t_mt<4, T, COMP>(w, ek, ex, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, zero, s);
    launch_sweep_t_mt<3, T, COMP>(w, ek, ex, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, zero, s);
    launch_sweep_t_mt<2, T, COMP>(w, ek, ex, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, zero, s);
    launch_sweep_t_mt<1, T, COMP>(w, ek, ex, ptr_b, ptr_e, krow, blk_off, blk, X, out_off, Y, ld, zero, s);
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
    static const double* Tm(const Basis& b) { return b.T.p; }
};
template <>
struct ApplyBufs<float> {
    static DBuf<float>& xt(Handle& h) { return h.xtf; }
    static DBuf<float>& yt(Handle& h) { return h.ytf; }
    static DBuf<float>& xh(Handle& h) { return h.xhf; }
    static DBuf<float>& yh(Handle& h) { return h.yhf; }
    static const float* B(Handle& h) { return h.Bf.p; }
    static const float* D(Handle& h) { return h.Df.p; }
    static const float* Tm(const Basis& b) { return b.Tf.p; }
};

// The apply's work vectors: x and y in tree order ([n][ld]) and the node
// coefficients xhat ([sum of column ranks][ld]) and yhat ([sum of row
// ranks][ld]).
template <class T>
struct ApplyWork {
    T *xt, *yt, *xh, *yh;
};

// One apply y = Ktilde x on work vectors w (column stride ld); prof: record
// the sweeps' events (creates them on first use).
template <class T>
void apply_t(Handle& h, const T* x, T* y, int nrhs, int ld, const ApplyWork<T>& w, bool prof, hipStream_t s)
{
    typedef ApplyBufs<T> AB;
    const int64_t n = h.n;
    T* xt = w.xt;
    T* yt = w.yt;
    T* xh = w.xh;
    T* yh = w.yh;
    // upward through V, W (the column basis), downward through U, R
    const Basis& bv = h.col();
    const T* Tm = AB::Tm(h.bu);
    const T* Tv = AB::Tm(bv);
    const T* zero = (const T*)h.zeros.p;
    auto mark = [&](int e) {
        if (prof) H2_HIP(hipEventRecord(h.ev[e], s));
    };
    if (prof && !h.ev[0])
        for (auto& e : h.ev) H2_HIP(hipEventCreate(&e));
    mark(0);
    const dim3 tiles((unsigned)((n + 63) / 64), (unsigned)((nrhs + 31) / 32));
    k_gather<T><<<tiles, TB, 0, s>>>(x, n, nrhs, ld, h.iperm.p, xt);
    H2_LAUNCH_CHECK();
    mark(1);
    for (int L = h.maxdepth; L >= 1; --L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_upward<T><<<nl, TB, 0, s>>>(lo, nrhs, ld, h.nchild.p, h.first_child.p, h.start.p, bv.rank.p, bv.mbar.p,
                                      bv.piv_off.p, bv.piv.p, bv.T_off.p, Tv, bv.xh_off.p, xt, xh);
        H2_LAUNCH_CHECK();
    }
    mark(2);
    // the precision mode adds each block product (one interaction) to the
    // row sums with compensation: FP32 recursion over the ~10^4 terms of an
    // interaction list would lose about sqrt(10^4) ulps
    if (h.store_coupling == 0) {
        if constexpr (std::is_same_v<T, double>) {
            const Basis& bu = h.bu;
            const unsigned grid = (unsigned)(8 * ((h.n_otf + 7) / 8));
            auto go = [&](auto fam) {
                constexpr int F = decltype(fam)::value;
                if (h.n_otf > 0)
                    k_coupling_otf<F><<<grid, 64, 0, s>>>(h.n_otf, h.otf_node.p, h.otf_r0.p, h.il_ptr.p, h.il_col.p,
                                                          bu.rank.p, bv.rank.p, h.skc_u.p, h.skc_ld_u, bu.xh_off.p,
                                                          h.nonsym ? h.skc_v.p : h.skc_u.p, h.skc_ld_v, bv.xh_off.p,
                                                          h.d, h.kid, h.prm, xh, yh, ld);
            };
            switch (kernel_family(h.kid)) {
            case FAM_COSINE: go(std::integral_constant<int, FAM_COSINE>()); break;
            case FAM_ADVECTION: go(std::integral_constant<int, FAM_ADVECTION>()); break;
            default: go(std::integral_constant<int, FAM_RADIAL>());
            }
            H2_LAUNCH_CHECK();
        } else {
            fail(H2_EINTERNAL, "coupling evaluated in the apply needs precision 64");
        }
    } else if (h.B_upper) {
        // the stored blocks of the entries j > i, then those of j < i read
        // transposed (added to the rows the first sweep wrote)
        launch_sweep<T, sizeof(T) == 4>(h.cp, h.il_split.p, h.il_ptr.p + 1, h.bu.rank.p, h.B_off.p, AB::B(h), xh,
                                        h.bu.xh_off.p, yh, ld, 0, zero, s);
        launch_sweep_t<T, sizeof(T) == 4>(h.cpt, h.cp.ek.p, h.cp.ex.p, h.il_ptr.p, h.il_split.p, h.bu.rank.p,
                                          h.B_off.p, AB::B(h), xh, h.bu.xh_off.p, yh, ld, zero, s);
    } else {
        launch_sweep<T, sizeof(T) == 4>(h.cp, h.il_ptr.p, h.il_ptr.p + 1, h.bu.rank.p, h.B_off.p, AB::B(h), xh,
                                        h.bu.xh_off.p, yh, ld, 0, zero, s);
    }
    mark(3);
    for (int L = 1; L < h.maxdepth; ++L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        k_downward<T><<<nl, TB, 0, s>>>(lo, nrhs, ld, h.nchild.p, h.first_child.p, h.bu.rank.p, h.bu.mbar.p,
                                        h.bu.piv_off.p, h.bu.piv.p, h.bu.T_off.p, Tm, h.bu.xh_off.p, yh);
        H2_LAUNCH_CHECK();
    }
    mark(4);
    k_leaves_far<T><<<(unsigned)h.leaves.n, TB, 0, s>>>(nrhs, ld, h.leaves.p, h.start.p, h.count.p, h.bu.rank.p,
                                                        h.bu.piv_off.p, h.bu.piv.p, h.bu.T_off.p, Tm, h.bu.xh_off.p, yh, yt);
    H2_LAUNCH_CHECK();
    launch_sweep<T, sizeof(T) == 4>(h.nr, h.nr_ptr.p, h.nr_ptr.p + 1, h.count.p, h.D_off.p, AB::D(h), xt,
                                    h.start64.p, yt, ld, 1, zero, s);
    mark(5);
    k_scatter<T><<<tiles, TB, 0, s>>>(yt, n, nrhs, ld, h.iperm.p, y);
    H2_LAUNCH_CHECK();
    mark(6);
    if (prof) {
        h.prof_valid = true;
        h.prof_nrhs = nrhs;
    }
}

// The apply with the handle's work vectors, grown (after synchronising s) when
// nrhs needs a wider column stride than any earlier apply.
template <class T>
void matvec_t(Handle& h, const T* x, T* y, int nrhs, hipStream_t s)
{
    typedef ApplyBufs<T> AB;
    const int64_t n = h.n;
    const int ld = (nrhs + 31) / 32 * 32;
    if (ld > h.mv_ld) {
        H2_HIP(hipStreamSynchronize(s));
        AB::xt(h).ensure((size_t)n * ld, s);
        AB::yt(h).ensure((size_t)n * ld, s);
        AB::xh(h).ensure((size_t)std::max<int64_t>(h.col().sum_rank, 1) * ld, s);
        AB::yh(h).ensure((size_t)std::max<int64_t>(h.bu.sum_rank, 1) * ld, s);
        h.mv_ld = ld;
    }
    apply_t<T>(h, x, y, nrhs, ld, ApplyWork<T>{AB::xt(h).p, AB::yt(h).p, AB::xh(h).p, AB::yh(h).p}, h.profile != 0,
               s);
}

// Work vectors of the apply that allocates nothing: one array per device,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; kernels get the device address from hipGetSymbolAddress.
constexpr int64_t SCRATCH_BYTES = H2_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
unsigned char* scratch_on_current_device()
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static unsigned char* ptr[MAXDEV] = {};
    int dev = 0;
    H2_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAXDEV) fail(H2_EDEVICE, "device index beyond the no-allocation apply's table");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(H2_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        ptr[dev] = (unsigned char*)p;
    }
    return ptr[dev];
}

// The apply on work vectors carved from `scratch` (each start rounded up to
// 256 bytes); no allocation, no events.
template <class T>
void matvec_noalloc_t(Handle& h, const T* x, T* y, int nrhs, hipStream_t s)
{
    const int ld = (nrhs + 31) / 32 * 32;
    auto bytes = [](int64_t elems) { return (elems * (int64_t)sizeof(T) + 255) / 256 * 256; };
    const int64_t bx = bytes(h.n * ld);
    const int64_t bv = bytes(std::max<int64_t>(h.col().sum_rank, 1) * ld);
    const int64_t bu = bytes(std::max<int64_t>(h.bu.sum_rank, 1) * ld);
    const int64_t need = 2 * bx + bv + bu;
    if (need > SCRATCH_BYTES)
        fail(H2_EUNSUPPORTED, "h2_matvec_noalloc: this handle and nrhs need " + std::to_string(need) +
                                  " bytes of work vectors, more than its " + std::to_string(SCRATCH_BYTES) +
                                  "-byte scratch array");
    unsigned char* base = scratch_on_current_device();
    const ApplyWork<T> w{(T*)base, (T*)(base + bx), (T*)(base + 2 * bx), (T*)(base + 2 * bx + bv)};
    apply_t<T>(h, x, y, nrhs, ld, w, false, s);
}

}  // namespace

// Task lists and list metadata of the two block sweeps, built once per
// handle; in the precision mode also the FP32 copy of the interpolation
// matrices.  A node's rows are cut into chunks of at most 64 rows (4 tiles).
void prepare_apply(Handle& h)
{
    hipStream_t s = h.stream;
    auto make = [&](const std::vector<int>& rows_of, const std::vector<int>& ptr, bool need_rank, Handle::Sweep& w) {
        std::vector<int> nd[4], rr[4];
        for (int i = 0; i < h.nnode; ++i) {
            const int rows = rows_of[i];
            if (rows == 0) continue;
            if (!need_rank && ptr[i + 1] == ptr[i]) continue;
            for (int r0 = 0; r0 < rows; r0 += 64) {
                const int mt = (std::min(64, rows - r0) + 15) / 16;
                nd[mt - 1].push_back(i);
                rr[mt - 1].push_back(r0);
            }
        }
        auto up = [&](DBuf<int>& d, const std::vector<int>& v) {
            d.ensure(std::max<size_t>(v.size(), 1), s);
            if (!v.empty()) H2_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s));
        };
        for (int c = 0; c < 4; ++c) {
            up(w.node[c], nd[c]);
            up(w.r0[c], rr[c]);
            w.n[c] = (int)nd[c].size();
        }
        H2_HIP(hipStreamSynchronize(s));
    };
    // zero source of the masked lanes of the block sweeps (FP64 and FP32)
    h.zeros.ensure(64, s);
    H2_HIP(hipMemsetAsync(h.zeros.p, 0, 64 * sizeof(double), s));
    std::vector<int64_t> st(h.h_start.begin(), h.h_start.end());
    h.start64.ensure(std::max<size_t>(st.size(), 1), s);
    H2_HIP(hipMemcpyAsync(h.start64.p, st.data(), st.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    h.iperm.ensure((size_t)std::max<int64_t>(h.n, 1), s);
    k_invert_perm<<<blocks_for(h.n, TB), TB, 0, s>>>(h.n, h.perm.p, h.iperm.p);
    H2_LAUNCH_CHECK();
    // coupling evaluated in the apply: (node, first row) of every 64-row
    // chunk of a node with a basis (zero yhat without IL)
    if (h.store_coupling == 0) {
        std::vector<int> nd, rr;
        for (int i = 0; i < h.nnode; ++i)
            for (int r0 = 0; r0 < h.bu.h_rank[i]; r0 += 64) {
                nd.push_back(i);
                rr.push_back(r0);
            }
        h.n_otf = (int)nd.size();
        h.otf_node.ensure(std::max<size_t>(nd.size(), 1), s);
        h.otf_r0.ensure(std::max<size_t>(rr.size(), 1), s);
        if (!nd.empty()) {
            H2_HIP(hipMemcpyAsync(h.otf_node.p, nd.data(), nd.size() * sizeof(int), hipMemcpyHostToDevice, s));
            H2_HIP(hipMemcpyAsync(h.otf_r0.p, rr.data(), rr.size() * sizeof(int), hipMemcpyHostToDevice, s));
        }
        H2_HIP(hipStreamSynchronize(s));
    }
    // coupling: every node with a basis writes its yhat (zero without IL);
    // block rows follow the row ranks, block columns (and the xhat they
    // read) the column ranks
    make(h.bu.h_rank, h.h_il_ptr, true, h.cp);
    h.cp.ek.ensure(std::max<int64_t>(h.nil, 1), s);
    h.cp.ex.ensure(std::max<int64_t>(h.nil, 1), s);
    h.cp.steps.ensure(std::max(h.nnode, 1), s);
    if (h.B_upper) {
        // the stored (j > i) entries in steps of 4 columns; the transposed
        // (j < i) entries in blocks of 16, for the nodes that have them
        k_entry_meta<<<blocks_for(h.nnode, TB), TB, 0, s>>>(h.nnode, h.il_ptr.p, h.il_col.p, h.col().rank.p,
                                                            h.col().xh_off.p, h.cp.ek.p, h.cp.ex.p);
        H2_LAUNCH_CHECK();
        k_range_units<<<blocks_for(h.nnode, TB), TB, 0, s>>>(h.nnode, h.il_split.p, h.il_ptr.p + 1, h.cp.ek.p, 4,
                                                             h.cp.steps.p);
        H2_LAUNCH_CHECK();
        std::vector<int> rows_l(h.nnode, 0);
        for (int i = 0; i < h.nnode; ++i)
            if (h.h_il_split[i] > h.h_il_ptr[i]) rows_l[i] = h.bu.h_rank[i];
        make(rows_l, h.h_il_ptr, true, h.cpt);
        h.cpt.steps.ensure(std::max(h.nnode, 1), s);
        k_range_units<<<blocks_for(h.nnode, TB), TB, 0, s>>>(h.nnode, h.il_ptr.p, h.il_split.p, h.cp.ek.p, 16,
                                                             h.cpt.steps.p);
        H2_LAUNCH_CHECK();
    } else {
        k_sweep_meta<<<blocks_for(h.nnode, TB), TB, 0, s>>>(h.nnode, h.il_ptr.p, h.il_col.p, h.col().rank.p,
                                                            h.col().xh_off.p, h.cp.ek.p, h.cp.ex.p, h.cp.steps.p);
        H2_LAUNCH_CHECK();
    }
    // nearfield: leaves with near entries (a leaf's own block is one)
    std::vector<int> leaf_rows(h.nnode, 0);
    for (int i = 0; i < h.nnode; ++i)
        if (h.h_nchild[i] == 0) leaf_rows[i] = h.h_count[i];
    make(leaf_rows, h.h_nr_ptr, false, h.nr);
    h.nr.ek.ensure(std::max<int64_t>(h.nnear, 1), s);
    h.nr.ex.ensure(std::max<int64_t>(h.nnear, 1), s);
    h.nr.steps.ensure(std::max(h.nnode, 1), s);
    k_sweep_meta<<<blocks_for(h.nnode, TB), TB, 0, s>>>(h.nnode, h.nr_ptr.p, h.nr_col.p, h.count.p, h.start64.p,
                                                        h.nr.ek.p, h.nr.ex.p, h.nr.steps.p);
    H2_LAUNCH_CHECK();
    if (h.precision == 32)
        for (Basis* b : {&h.bu, &h.bv}) {
            if (b == &h.bv && !h.nonsym) break;
            const int64_t nt = std::max<int64_t>(b->h_T_off[h.nnode], 1);
            b->Tf.ensure((size_t)nt, s);
            k_to_f32<<<blocks_for(nt, TB), TB, 0, s>>>(b->T.p, nt, b->Tf.p);
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

void matvec_noalloc(Handle& h, const void* x, void* y, int nrhs, hipStream_t s)
{
    if (h.precision == 32)
        matvec_noalloc_t<float>(h, (const float*)x, (float*)y, nrhs, s);
    else
        matvec_noalloc_t<double>(h, (const double*)x, (double*)y, nrhs, s);
}

}  // namespace h2
