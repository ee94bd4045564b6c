// Coupling and nearfield blocks of Algorithm 2:
//   B_ij = K(Xhat_i, Xhat_j)   for (i, j) in the interaction lists,
//   D_ij = K(X_i, X_j)         for (i, j) in the near lists (leaf pairs).
// Blocks are stored row-major (rank_i x rank_j, resp. count_i x count_j) in
// CSR order of the lists; offsets come from a device scan over the block
// sizes.  One workgroup per row i; consecutive lanes write consecutive
// entries of a block row.
#include "common.h"
#include "kappa.h"

namespace h2 {
namespace {

constexpr int TB = 256;

__global__ __launch_bounds__(TB) void k_block_sizes(int nrow, const int* __restrict__ ptr, const int* __restrict__ col,
                                                    const int* __restrict__ sz_node, int64_t* __restrict__ out)
{
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nrow) return;
    int64_t a = sz_node[i];
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) out[e] = a * sz_node[col[e]];
}

// Coupling blocks: rows/cols are skeleton points (tree positions) skel[i*stride + t].
__global__ __launch_bounds__(TB) void k_coupling(const double* __restrict__ pts, int64_t n, int d, int kid,
                                                 double prm, const int* __restrict__ ptr, const int* __restrict__ col,
                                                 const int* __restrict__ rank, const int* __restrict__ skel,
                                                 int stride, const int64_t* __restrict__ off, double* __restrict__ B)
{
    const int i = blockIdx.x;
    const int ki = rank[i];
    if (ki == 0) return;
    const int* si = skel + (int64_t)i * stride;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
        const int j = col[e];
        const int kj = rank[j];
        const int* sj = skel + (int64_t)j * stride;
        double* o = B + off[e];
        const int64_t tot = (int64_t)ki * kj;
        for (int64_t q = threadIdx.x; q < tot; q += TB) {
            int t = (int)(q / kj), u = (int)(q - (int64_t)t * kj);
            o[q] = kappa_r2(kid, prm, dist2(pts, n, si[t], pts, n, sj[u], d));
        }
    }
}

// Nearfield blocks between leaves: rows/cols are the leaves' points.
__global__ __launch_bounds__(TB) void k_near(const double* __restrict__ pts, int64_t n, int d, int kid, double prm,
                                             const int* __restrict__ ptr, const int* __restrict__ col,
                                             const int* __restrict__ start, const int* __restrict__ count,
                                             const int64_t* __restrict__ off, double* __restrict__ D)
{
    const int i = blockIdx.x;
    const int ci = count[i], s0 = start[i];
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
        const int j = col[e];
        const int cj = count[j], s1 = start[j];
        double* o = D + off[e];
        const int64_t tot = (int64_t)ci * cj;
        for (int64_t q = threadIdx.x; q < tot; q += TB) {
            int t = (int)(q / cj), u = (int)(q - (int64_t)t * cj);
            o[q] = kappa_r2(kid, prm, dist2(pts, n, s0 + t, pts, n, s1 + u, d));
        }
    }
}

}  // namespace

void build_blocks(Handle& h)
{
    hipStream_t s = h.stream;
    const int nn = h.nnode;
    h.B_off.ensure((size_t)h.nil + 1, s);
    h.D_off.ensure((size_t)h.nnear + 1, s);
    DBuf<int64_t> sz;
    sz.ensure((size_t)std::max<int64_t>(std::max(h.nil, h.nnear), 1), s);
    // coupling
    k_block_sizes<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.il_ptr.p, h.il_col.p, h.rank.p, sz.p);
    H2_LAUNCH_CHECK();
    scan_excl_i64(sz.p, h.B_off.p, h.nil, h.tmp_i64, s);
    int64_t nB = read_scalar(h.B_off.p + h.nil, s);
    h.B.ensure((size_t)std::max<int64_t>(nB, 1), s);
    h.bytes_B = nB * (int64_t)sizeof(double);
    k_coupling<<<nn, TB, 0, s>>>(h.pts.p, h.n, h.d, h.kid, h.prm, h.il_ptr.p, h.il_col.p, h.rank.p, h.skel.p, h.r2,
                                 h.B_off.p, h.B.p);
    H2_LAUNCH_CHECK();
    // nearfield
    k_block_sizes<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.nr_ptr.p, h.nr_col.p, h.count.p, sz.p);
    H2_LAUNCH_CHECK();
    scan_excl_i64(sz.p, h.D_off.p, h.nnear, h.tmp_i64, s);
    int64_t nD = read_scalar(h.D_off.p + h.nnear, s);
    h.D.ensure((size_t)std::max<int64_t>(nD, 1), s);
    h.bytes_D = nD * (int64_t)sizeof(double);
    k_near<<<nn, TB, 0, s>>>(h.pts.p, h.n, h.d, h.kid, h.prm, h.nr_ptr.p, h.nr_col.p, h.start.p, h.count.p,
                             h.D_off.p, h.D.p);
    H2_LAUNCH_CHECK();
    H2_HIP(hipStreamSynchronize(s));
}

}  // namespace h2
