// Coupling and nearfield blocks of Algorithm 2:
//   B_ij = K(Xhat_i^(row), Xhat_j^(col))   for (i, j) in the interaction lists,
//   D_ij = K(X_i, X_j)                     for (i, j) in the near lists (leaf pairs);
// the row and column skeletons coincide for a symmetric kernel.
// Blocks are stored column-major (rank_i x rank_j, resp. count_i x count_j)
// in CSR order of the lists; offsets come from a device scan over the block
// sizes.  For a symmetric kernel (V = U, so B_ji = B_ij^T) only the blocks of
// the entries with j > i are stored -- the interaction lists are symmetric,
// so every unordered pair once -- and the offset of an entry with j < i
// points at the stored B_ji, which the apply reads transposed.  These
// entries feed only the apply, so they use the fast kernel evaluation (an ulp
// or two from the correctly rounded form that the ID uses).
#include "common.h"
#include "kappa.h"

namespace h2 {
namespace {

constexpr int TB = 256;

// Block sizes per list entry; with `upper` set only the entries with j > i
// get a block (the others 0).
__global__ __launch_bounds__(TB) void k_block_sizes(int nrow, const int* __restrict__ ptr, const int* __restrict__ col,
                                                    const int* __restrict__ sz_row, const int* __restrict__ sz_col,
                                                    int upper, int64_t* __restrict__ out)
{
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    int64_t a = sz_row[i];
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) out[e] = (upper && col[e] < i) ? 0 : a * sz_col[col[e]];
}

// First entry of every row with column > i (rows sorted ascending; an
// interaction list never holds i itself).
__global__ __launch_bounds__(TB) void k_row_split(int nrow, const int* __restrict__ ptr, const int* __restrict__ col,
                                                  int* __restrict__ split)
{
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    int lo = ptr[i], hi = ptr[i + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < i)
            lo = mid + 1;
        else
            hi = mid;
    }
    split[i] = lo;
}

// Entries (i, j) with j < i take the offset of the stored block of (j, i),
// found by a binary search in row j's upper part.
__global__ __launch_bounds__(TB) void k_lower_offsets(int nrow, const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const int* __restrict__ split, int64_t* __restrict__ off)
{
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    for (int e = ptr[i]; e < split[i]; ++e) {
        const int j = col[e];
        int lo = split[j], hi = ptr[j + 1] - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (col[mid] < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        off[e] = off[lo];
    }
}

// Skeleton coordinates gathered into node order (SoA [d][sum k]) so that a
// block's column points are one coalesced load.
__global__ __launch_bounds__(TB) void k_skel_coords(int nn, const double* __restrict__ pts, int64_t n, int d,
                                                    const int* __restrict__ rank, const int* __restrict__ skel,
                                                    int stride, const int64_t* __restrict__ xoff, int64_t sumk,
                                                    double* __restrict__ skc)
{
    const int i = blockIdx.x;
    const int k = rank[i];
    for (int t = threadIdx.x; t < k; t += TB) {
        const int p = skel[(int64_t)i * stride + t];
        for (int a = 0; a < d; ++a) skc[a * sumk + xoff[i] + t] = pts[a * n + p];
    }
}

// Row of every list entry (CSR expansion).
__global__ __launch_bounds__(TB) void k_entry_rows(int nrow, const int* __restrict__ ptr, int* __restrict__ row)
{
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) row[e] = i;
}

// Row and column point sets of the blocks: node i's points are cnt[i]
// consecutive entries of the SoA array xs ([d][ld]) from xo[i].
struct PtSet {
    const double* xs;
    int64_t ld;
    const int64_t* xo;
    const int* cnt;
};

// One wavefront per block (list entry e = (i, j)), four blocks per
// workgroup.  Row points (rows_i of them, from the row set) and column points
// (cols_j, from the column set) are loaded once, one per lane, and the column
// point of each block column is broadcast with a lane shuffle.  The block is
// column-major (entry (t,u) at u*rows_i + t); with rows_i <= 32 the two
// half-waves fill two columns per pass.  The dimension D and the kernel id
// KID are compile-time constants of the loop (the kernel's switch over the
// kernel id sits outside it), so an entry costs its distance, the kernel
// function and one store.
template <class OutT, int FAM, int D, int KID>
__device__ __forceinline__ void blocks_eval_one(int lane, int ki, int kj, const double* __restrict__ xs, int64_t ld,
                                                int64_t bi, const double* __restrict__ ys, int64_t lc, int64_t bj,
                                                double prm, OutT* __restrict__ o)
{
    for (int t0 = 0; t0 < ki; t0 += 64) {
        const bool half = ki - t0 <= 32;  // two columns per pass
        const int t = half ? t0 + (lane & 31) : t0 + lane;
        const int du = half ? (lane >> 5) : 0;
        const int su = half ? 2 : 1;
        double xi[3] = {0.0, 0.0, 0.0};
        if (t < ki)
#pragma unroll
            for (int a = 0; a < D; ++a) xi[a] = xs[a * ld + bi + t];
        for (int u0 = 0; u0 < kj; u0 += 64) {
            const int uc = min(64, kj - u0);
            double y[3] = {0.0, 0.0, 0.0};
            if (lane < uc)
#pragma unroll
                for (int a = 0; a < D; ++a) y[a] = ys[a * lc + bj + u0 + lane];
            OutT* op = o + (int64_t)(u0 + du) * ki + t;
            const int64_t step = (int64_t)su * ki;
            // wave-uniform trip count: every lane takes part in every shuffle
            for (int ub = 0; ub < uc; ub += su, op += step) {
                const int uu = ub + du;
                const int src = uu < uc ? uu : uc - 1;
                double sc[3];
#pragma unroll
                for (int a = 0; a < D; ++a) sc[a] = __shfl(y[a], src, 64);
                double r2 = 0.0, xy = 0.0;  // xy: the cosine kernel's inner product
                // (fused multiply-adds written out, as in the apply's
                // evaluation of the same entries)
                if constexpr (FAM == FAM_COSINE) {
                    xy = xi[0] * sc[0];
#pragma unroll
                    for (int a = 1; a < D; ++a) xy = __builtin_fma(xi[a], sc[a], xy);
                } else {
                    const double a0 = sc[0] - xi[0];
                    r2 = a0 * a0;
#pragma unroll
                    for (int a = 1; a < D; ++a) {
                        const double aa = sc[a] - xi[a];
                        r2 = __builtin_fma(aa, aa, r2);
                    }
                }
                if (t < ki && uu < uc) *op = kappa_store<OutT, FAM>(KID, prm, r2, xy, xi[0] - sc[0]);
            }
        }
    }
}

// Blocks with at most FLAT_MAX rows and columns: the row and column points
// are staged in the wavefront's LDS slice sp ([2][3][FLAT_MAX]: rows, then
// columns) and lane l forms entries l, l + 64, ... of the column-major block,
// so that every store is 64 consecutive entries whatever k_i (the entries
// and their arithmetic are those of blocks_eval_one).
constexpr int FLAT_MAX = 128;
template <class OutT, int FAM, int D, int KID>
__device__ __forceinline__ void blocks_eval_flat(int lane, int ki, int kj, const double (*sp)[3][FLAT_MAX],
                                                 double prm, OutT* __restrict__ o)
{
    const int64_t tot = (int64_t)ki * kj;
    int t = lane % ki, u = lane / ki;
    const int dt = 64 % ki, du = 64 / ki;
    for (int64_t e0 = 0; e0 < tot; e0 += 64) {
        if (e0 + lane < tot) {
            double xi[3], sc[3];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                xi[a] = sp[0][a][t];
                sc[a] = sp[1][a][u];
            }
            double r2 = 0.0, xy = 0.0;
            if constexpr (FAM == FAM_COSINE) {
                xy = xi[0] * sc[0];
#pragma unroll
                for (int a = 1; a < D; ++a) xy = __builtin_fma(xi[a], sc[a], xy);
            } else {
                const double a0 = sc[0] - xi[0];
                r2 = a0 * a0;
#pragma unroll
                for (int a = 1; a < D; ++a) {
                    const double aa = sc[a] - xi[a];
                    r2 = __builtin_fma(aa, aa, r2);
                }
            }
            o[e0 + lane] = kappa_store<OutT, FAM>(KID, prm, r2, xy, xi[0] - sc[0]);
        }
        t += dt;
        u += du;
        if (t >= ki) {
            t -= ki;
            ++u;
        }
    }
}

template <class OutT, int FAM, int D>
__global__ __launch_bounds__(TB) void k_blocks_eval(int64_t nent, const int* __restrict__ erow,
                                                    const int* __restrict__ col, PtSet rs, PtSet cs, int kid,
                                                    double prm, const int64_t* __restrict__ off, int upper,
                                                    OutT* __restrict__ out)
{
    __shared__ double sp[TB / 64][2][3][FLAT_MAX];
    const int64_t e = (int64_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    bool run = e < nent;
    int i = 0, j = 0, ki = 0, kj = 0;
    if (run) {
        i = erow[e];
        j = col[e];
        if (upper && j < i) run = false;  // stored with the entry (j, i)
    }
    if (run) {
        ki = rs.cnt[i];
        kj = cs.cnt[j];
        run = ki > 0 && kj > 0;
    }
    const int64_t bi = run ? rs.xo[i] : 0, bj = run ? cs.xo[j] : 0;
    const bool flat = run && ki <= FLAT_MAX && kj <= FLAT_MAX;
    if (flat) {
        for (int q = lane; q < ki; q += 64)
#pragma unroll
            for (int a = 0; a < D; ++a) sp[wv][0][a][q] = rs.xs[a * rs.ld + bi + q];
        for (int q = lane; q < kj; q += 64)
#pragma unroll
            for (int a = 0; a < D; ++a) sp[wv][1][a][q] = cs.xs[a * cs.ld + bj + q];
    }
    __syncthreads();  // every wavefront of the workgroup reaches it once
    if (!run) return;
    OutT* o = out + off[e];
    if (flat) {
        if constexpr (FAM == FAM_RADIAL) {
            switch (kid) {
            case H2_COULOMB: blocks_eval_flat<OutT, FAM, D, H2_COULOMB>(lane, ki, kj, sp[wv], prm, o); break;
            case H2_GAUSSIAN: blocks_eval_flat<OutT, FAM, D, H2_GAUSSIAN>(lane, ki, kj, sp[wv], prm, o); break;
            case H2_EXPONENTIAL:
                blocks_eval_flat<OutT, FAM, D, H2_EXPONENTIAL>(lane, ki, kj, sp[wv], prm, o);
                break;
            case H2_BUMP: blocks_eval_flat<OutT, FAM, D, H2_BUMP>(lane, ki, kj, sp[wv], prm, o); break;
            default: blocks_eval_flat<OutT, FAM, D, H2_MATERN32>(lane, ki, kj, sp[wv], prm, o);
            }
        } else {
            blocks_eval_flat<OutT, FAM, D, 0>(lane, ki, kj, sp[wv], prm, o);
        }
        return;
    }
    if constexpr (FAM == FAM_RADIAL) {
        switch (kid) {
        case H2_COULOMB:
            blocks_eval_one<OutT, FAM, D, H2_COULOMB>(lane, ki, kj, rs.xs, rs.ld, bi, cs.xs, cs.ld, bj, prm, o);
            break;
        case H2_GAUSSIAN:
            blocks_eval_one<OutT, FAM, D, H2_GAUSSIAN>(lane, ki, kj, rs.xs, rs.ld, bi, cs.xs, cs.ld, bj, prm, o);
            break;
        case H2_EXPONENTIAL:
            blocks_eval_one<OutT, FAM, D, H2_EXPONENTIAL>(lane, ki, kj, rs.xs, rs.ld, bi, cs.xs, cs.ld, bj, prm, o);
            break;
        case H2_BUMP:
            blocks_eval_one<OutT, FAM, D, H2_BUMP>(lane, ki, kj, rs.xs, rs.ld, bi, cs.xs, cs.ld, bj, prm, o);
            break;
        default:
            blocks_eval_one<OutT, FAM, D, H2_MATERN32>(lane, ki, kj, rs.xs, rs.ld, bi, cs.xs, cs.ld, bj, prm, o);
        }
    } else {
        blocks_eval_one<OutT, FAM, D, 0>(lane, ki, kj, rs.xs, rs.ld, bi, cs.xs, cs.ld, bj, prm, o);
    }
}

// Each kernel family's blocks come from their own instance (see kappa_fam),
// one per dimension.
template <class OutT, int FAM>
void launch_blocks_eval_d(unsigned nb, int64_t nent, const int* erow, const int* col, const PtSet& rs,
                          const PtSet& cs, int d, int kid, double prm, const int64_t* off, int upper, OutT* out,
                          hipStream_t s)
{
    switch (d) {
    case 1: k_blocks_eval<OutT, FAM, 1><<<nb, TB, 0, s>>>(nent, erow, col, rs, cs, kid, prm, off, upper, out); break;
    case 2: k_blocks_eval<OutT, FAM, 2><<<nb, TB, 0, s>>>(nent, erow, col, rs, cs, kid, prm, off, upper, out); break;
    default: k_blocks_eval<OutT, FAM, 3><<<nb, TB, 0, s>>>(nent, erow, col, rs, cs, kid, prm, off, upper, out);
    }
}

template <class OutT>
void launch_blocks_eval(int64_t nent, const int* erow, const int* col, const PtSet& rs, const PtSet& cs, int d,
                        int kid, double prm, const int64_t* off, int upper, OutT* out, hipStream_t s)
{
    const unsigned nb = (unsigned)blocks_for(nent, TB / 64);
    switch (kernel_family(kid)) {
    case FAM_COSINE:
        launch_blocks_eval_d<OutT, FAM_COSINE>(nb, nent, erow, col, rs, cs, d, kid, prm, off, upper, out, s);
        break;
    case FAM_ADVECTION:
        launch_blocks_eval_d<OutT, FAM_ADVECTION>(nb, nent, erow, col, rs, cs, d, kid, prm, off, upper, out, s);
        break;
    default:
        launch_blocks_eval_d<OutT, FAM_RADIAL>(nb, nent, erow, col, rs, cs, d, kid, prm, off, upper, out, s);
    }
    H2_LAUNCH_CHECK();
}

// Nearfield blocks D_ij = K(X_i, X_j) of every near-list entry; sz and
// erow are scratch of at least nnear entries.
void near_blocks(Handle& h, DBuf<int64_t>& sz, DBuf<int>& erow)
{
    hipStream_t s = h.stream;
    const int nn = h.nnode;
    const bool f32 = h.precision == 32;
    // the leaves' points are contiguous in tree order
    k_block_sizes<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.nr_ptr.p, h.nr_col.p, h.count.p, h.count.p, 0, sz.p);
    H2_LAUNCH_CHECK();
    scan_excl_i64(sz.p, h.D_off.p, h.nnear, h.tmp_i64, s);
    int64_t nD = read_scalar(h.D_off.p + h.nnear, s);
    if (f32) {
        h.Df.ensure((size_t)(nD + BLK_PAD), s);
        H2_HIP(hipMemsetAsync(h.Df.p + nD, 0, BLK_PAD * sizeof(float), s));
    } else {
        h.D.ensure((size_t)(nD + BLK_PAD), s);
        H2_HIP(hipMemsetAsync(h.D.p + nD, 0, BLK_PAD * sizeof(double), s));
    }
    h.bytes_D = nD * (int64_t)(f32 ? sizeof(float) : sizeof(double));
    if (h.nnear > 0) {
        std::vector<int64_t> st(h.h_start.begin(), h.h_start.end());
        DBuf<int64_t> d_st;
        d_st.ensure(st.size(), s);
        H2_HIP(hipMemcpyAsync(d_st.p, st.data(), st.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        k_entry_rows<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.nr_ptr.p, erow.p);
        H2_LAUNCH_CHECK();
        const PtSet ps{h.pts.p, h.n, d_st.p, h.count.p};
        if (f32)
            launch_blocks_eval(h.nnear, erow.p, h.nr_col.p, ps, ps, h.d, h.kid, h.prm, h.D_off.p, 0, h.Df.p, s);
        else
            launch_blocks_eval(h.nnear, erow.p, h.nr_col.p, ps, ps, h.d, h.kid, h.prm, h.D_off.p, 0, h.D.p, s);
        H2_HIP(hipStreamSynchronize(s));
    }
    H2_HIP(hipStreamSynchronize(s));
}

}  // namespace

void build_blocks(Handle& h)
{
    hipStream_t s = h.stream;
    const int nn = h.nnode;
    h.B_upper = false;
    h.B_off.ensure((size_t)h.nil + 1, s);
    h.D_off.ensure((size_t)h.nnear + 1, s);
    DBuf<int64_t> sz;
    DBuf<int> erow;
    const int64_t nmax = std::max<int64_t>(std::max(h.nil, h.nnear), 1);
    sz.ensure((size_t)nmax, s);
    erow.ensure((size_t)nmax, s);
    // skeleton coordinates in node order: the row skeletons, and the column
    // skeletons of a non-symmetric kernel (kept in the handle when the apply
    // evaluates the coupling blocks itself)
    DBuf<int64_t> d_xo[2];
    DBuf<double> skc_local[2];
    DBuf<double>* skc[2] = {&skc_local[0], &skc_local[1]};
    if (h.store_coupling == 0) {
        skc[0] = &h.skc_u;
        skc[1] = &h.skc_v;
    }
    int64_t skc_ld[2] = {1, 1};
    auto skel_set = [&](const Basis& b, int w) -> PtSet {
        std::vector<int64_t> xo((size_t)nn + 1, 0);
        for (int i = 0; i < nn; ++i) xo[i + 1] = xo[i] + b.h_rank[i];
        const int64_t sumk = std::max<int64_t>(xo[nn], 1);
        d_xo[w].ensure(xo.size(), s);
        H2_HIP(hipMemcpyAsync(d_xo[w].p, xo.data(), xo.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        skc[w]->ensure((size_t)h.d * sumk, s);
        k_skel_coords<<<nn, TB, 0, s>>>(nn, h.pts.p, h.n, h.d, b.rank.p, b.skel.p, h.ys_stride, d_xo[w].p, sumk,
                                        skc[w]->p);
        H2_LAUNCH_CHECK();
        H2_HIP(hipStreamSynchronize(s));  // xo (host) is read by the copy
        skc_ld[w] = sumk;
        return PtSet{skc[w]->p, sumk, d_xo[w].p, b.rank.p};
    };
    const PtSet rs = skel_set(h.bu, 0);
    const PtSet cs = h.nonsym ? skel_set(h.bv, 1) : rs;
    h.skc_ld_u = skc_ld[0];
    h.skc_ld_v = h.nonsym ? skc_ld[1] : skc_ld[0];
    if (h.store_coupling == 0) {
        // the coupling blocks are evaluated by the apply; only the nearfield
        // blocks are stored
        h.B.release();
        h.Bf.release();
        h.bytes_B = 0;
        near_blocks(h, sz, erow);
        return;
    }
    // coupling: for a symmetric kernel the blocks of the entries j > i only
    const int upper = h.nonsym ? 0 : 1;
    h.B_upper = upper != 0;
    h.il_split.ensure((size_t)std::max(nn, 1), s);
    k_row_split<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.il_ptr.p, h.il_col.p, h.il_split.p);
    H2_LAUNCH_CHECK();
    k_block_sizes<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.il_ptr.p, h.il_col.p, h.bu.rank.p, h.col().rank.p, upper,
                                                    sz.p);
    H2_LAUNCH_CHECK();
    scan_excl_i64(sz.p, h.B_off.p, h.nil, h.tmp_i64, s);
    int64_t nB = read_scalar(h.B_off.p + h.nil, s);
    if (upper) {
        k_lower_offsets<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.il_ptr.p, h.il_col.p, h.il_split.p, h.B_off.p);
        H2_LAUNCH_CHECK();
    }
    h.h_il_split = read_vec(h.il_split.p, (size_t)nn, s);
    const bool f32 = h.precision == 32;
    // BLK_PAD zeros after the last block (read by row tiles of the apply
    // that run past a block's last row)
    if (f32) {
        h.Bf.ensure((size_t)(nB + BLK_PAD), s);
        H2_HIP(hipMemsetAsync(h.Bf.p + nB, 0, BLK_PAD * sizeof(float), s));
    } else {
        h.B.ensure((size_t)(nB + BLK_PAD), s);
        H2_HIP(hipMemsetAsync(h.B.p + nB, 0, BLK_PAD * sizeof(double), s));
    }
    h.bytes_B = nB * (int64_t)(f32 ? sizeof(float) : sizeof(double));
    if (h.nil > 0) {
        k_entry_rows<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.il_ptr.p, erow.p);
        H2_LAUNCH_CHECK();
        if (f32)
            launch_blocks_eval(h.nil, erow.p, h.il_col.p, rs, cs, h.d, h.kid, h.prm, h.B_off.p, upper, h.Bf.p, s);
        else
            launch_blocks_eval(h.nil, erow.p, h.il_col.p, rs, cs, h.d, h.kid, h.prm, h.B_off.p, upper, h.B.p, s);
    }
    near_blocks(h, sz, erow);
}

}  // namespace h2
