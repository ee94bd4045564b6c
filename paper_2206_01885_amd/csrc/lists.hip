// Admissibility (Eq. separation) and the interaction / near lists
// (Section 2.1), built by a level-synchronous dual traversal on the device.
//
// Reading of the interaction list: the paper's worked example (IL(4) =
// {6,7}, IL(10) = {8,12,13} on a 1-D binary tree) is reproduced by the pair
// rule -- (i,j) is in the list when (i,j) is admissible and the pair of their
// parents is not.  Starting from (root, root), every inadmissible pair with a
// non-leaf side is refined (both non-leaf: all child pairs; one side a leaf:
// the children of the other side); each new pair is admissible (interaction
// list), a pair of leaves (near list, (i,i) included) or refined further.
//
// Admissibility reads diam(X_i) as the box diagonal side*sqrt(d) and a_i as
// the box centre, squared to avoid a square root:
//     d (s_i + s_j)^2 <= 4 tau^2 |a_i - a_j|^2.
// Compiled with -ffp-contract=off: the decision is bit-for-bit the oracle's.
#include "common.h"

namespace h2 {
namespace {

constexpr int TB = 256;
constexpr int SORT_MAX = 4096;  // rows up to this length are sorted in LDS

__device__ inline bool admissible(const double* __restrict__ center, const double* __restrict__ side, int d,
                                  double tau, int i, int j)
{
    double dist2 = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = center[(int64_t)i * d + a] - center[(int64_t)j * d + a];
        dist2 = dist2 + t * t;
    }
    double ss = side[i] + side[j];
    double lhs = (double)d * (ss * ss);
    double rhs = 4.0 * tau * tau * dist2;
    return lhs <= rhs;
}

__global__ __launch_bounds__(TB) void k_pair_count(const int* __restrict__ fi, const int* __restrict__ fj, int64_t nf,
                                                   const int* __restrict__ nchild, int* __restrict__ cnt)
{
    int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (e >= nf) return;
    int ni = nchild[fi[e]], nj = nchild[fj[e]];
    cnt[e] = (ni ? ni : 1) * (nj ? nj : 1);
}

// type: 0 admissible (interaction list), 1 pair of leaves (near), 2 refine
__global__ __launch_bounds__(TB) void k_pair_expand(const int* __restrict__ fi, const int* __restrict__ fj, int64_t nf,
                                                    const int* __restrict__ off, const int* __restrict__ nchild,
                                                    const int* __restrict__ first_child,
                                                    const double* __restrict__ center, const double* __restrict__ side,
                                                    int d, double tau, int* __restrict__ ci_out,
                                                    int* __restrict__ cj_out, int* __restrict__ flags, int64_t nc)
{
    int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (e >= nf) return;
    int i = fi[e], j = fj[e];
    int ni = nchild[i], nj = nchild[j];
    int ai = ni ? ni : 1, aj = nj ? nj : 1;
    int64_t o = off[e];
    for (int a = 0; a < ai; ++a)
        for (int b = 0; b < aj; ++b) {
            int ci = ni ? first_child[i] + a : i;
            int cj = nj ? first_child[j] + b : j;
            int type;
            if (admissible(center, side, d, tau, ci, cj))
                type = 0;
            else if (nchild[ci] == 0 && nchild[cj] == 0)
                type = 1;
            else
                type = 2;
            int64_t p = o + a * aj + b;
            ci_out[p] = ci;
            cj_out[p] = cj;
            flags[p] = type == 0;
            flags[nc + p] = type == 1;
            flags[2 * nc + p] = type == 2;
        }
}

__global__ __launch_bounds__(TB) void k_compact(const int* __restrict__ ci, const int* __restrict__ cj, int64_t nc,
                                                const int* __restrict__ flags, const int* __restrict__ pos,
                                                int* __restrict__ oi, int* __restrict__ oj, int64_t base)
{
    int64_t p = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (p >= nc || !flags[p]) return;
    oi[base + pos[p]] = ci[p];
    oj[base + pos[p]] = cj[p];
}

__global__ __launch_bounds__(TB) void k_row_count(const int* __restrict__ pi, int64_t np, int* __restrict__ rowcnt)
{
    int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (e < np) atomicAdd(&rowcnt[pi[e]], 1);
}

__global__ __launch_bounds__(TB) void k_row_fill(const int* __restrict__ pi, const int* __restrict__ pj, int64_t np,
                                                 const int* __restrict__ ptr, int* __restrict__ fill,
                                                 int* __restrict__ col)
{
    int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (e >= np) return;
    int i = pi[e];
    int slot = atomicAdd(&fill[i], 1);
    col[ptr[i] + slot] = pj[e];
}

// Sort the columns of every row ascending (bitonic sort in LDS; long rows
// fall back to a single-lane shell sort).
__global__ __launch_bounds__(TB) void k_row_sort(const int* __restrict__ ptr, int* __restrict__ col, int nrow)
{
    __shared__ int sh[SORT_MAX];
    int i = blockIdx.x;
    if (i >= nrow) return;
    int b = ptr[i], len = ptr[i + 1] - b;
    if (len <= 1) return;
    if (len > SORT_MAX) {
        if (threadIdx.x == 0) {
            int gaps[] = {1750, 701, 301, 132, 57, 23, 10, 4, 1};
            for (int g : gaps)
                for (int x = g; x < len; ++x) {
                    int v = col[b + x];
                    int y = x;
                    for (; y >= g && col[b + y - g] > v; y -= g) col[b + y] = col[b + y - g];
                    col[b + y] = v;
                }
        }
        return;
    }
    int P = 1;
    while (P < len) P <<= 1;
    for (int x = threadIdx.x; x < P; x += TB) sh[x] = x < len ? col[b + x] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int x = threadIdx.x; x < P; x += TB) {
                int y = x ^ jj;
                if (y > x) {
                    bool up = (x & k) == 0;
                    int a = sh[x], c = sh[y];
                    if ((a > c) == up) {
                        sh[x] = c;
                        sh[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int x = threadIdx.x; x < len; x += TB) col[b + x] = sh[x];
}

struct PairList {
    DBuf<int> i, j;
    int64_t n = 0;
    void append_reserve(int64_t extra, hipStream_t s)
    {
        i.grow_keep((size_t)(n + extra), (size_t)n, s);
        j.grow_keep((size_t)(n + extra), (size_t)n, s);
    }
};

void to_csr(Handle& h, PairList& pl, DBuf<int>& ptr, DBuf<int>& col)
{
    hipStream_t s = h.stream;
    int nn = h.nnode;
    DBuf<int> rowcnt;
    rowcnt.ensure((size_t)nn, s);
    H2_HIP(hipMemsetAsync(rowcnt.p, 0, sizeof(int) * nn, s));
    if (pl.n) k_row_count<<<blocks_for(pl.n, TB), TB, 0, s>>>(pl.i.p, pl.n, rowcnt.p);
    H2_LAUNCH_CHECK();
    ptr.ensure((size_t)nn + 1, s);
    scan_excl_i32(rowcnt.p, ptr.p, nn, h.tmp_i32, s);
    col.ensure((size_t)std::max<int64_t>(pl.n, 1), s);
    H2_HIP(hipMemsetAsync(rowcnt.p, 0, sizeof(int) * nn, s));
    if (pl.n) k_row_fill<<<blocks_for(pl.n, TB), TB, 0, s>>>(pl.i.p, pl.j.p, pl.n, ptr.p, rowcnt.p, col.p);
    H2_LAUNCH_CHECK();
    k_row_sort<<<nn, TB, 0, s>>>(ptr.p, col.p, nn);
    H2_LAUNCH_CHECK();
}

}  // namespace

void build_lists(Handle& h)
{
    hipStream_t s = h.stream;
    PairList il, nr, fr, fr2;
    int root_leaf = h.h_nchild[0] == 0;
    int zero2[2] = {0, 0};
    if (root_leaf) {
        nr.append_reserve(1, s);
        H2_HIP(hipMemcpyAsync(nr.i.p, zero2, sizeof(int), hipMemcpyHostToDevice, s));
        H2_HIP(hipMemcpyAsync(nr.j.p, zero2, sizeof(int), hipMemcpyHostToDevice, s));
        nr.n = 1;
    } else {
        fr.append_reserve(1, s);
        H2_HIP(hipMemcpyAsync(fr.i.p, zero2, sizeof(int), hipMemcpyHostToDevice, s));
        H2_HIP(hipMemcpyAsync(fr.j.p, zero2, sizeof(int), hipMemcpyHostToDevice, s));
        fr.n = 1;
    }
    H2_HIP(hipStreamSynchronize(s));
    DBuf<int> cnt, off, ci, cj, flags, pos;
    while (fr.n > 0) {
        int64_t nf = fr.n;
        cnt.ensure((size_t)nf, s);
        off.ensure((size_t)nf + 1, s);
        k_pair_count<<<blocks_for(nf, TB), TB, 0, s>>>(fr.i.p, fr.j.p, nf, h.nchild.p, cnt.p);
        H2_LAUNCH_CHECK();
        scan_excl_i32(cnt.p, off.p, nf, h.tmp_i32, s);
        int64_t nc = read_scalar(off.p + nf, s);
        ci.ensure((size_t)nc, s);
        cj.ensure((size_t)nc, s);
        flags.ensure((size_t)nc * 3, s);
        pos.ensure((size_t)nc * 3 + 3, s);
        k_pair_expand<<<blocks_for(nf, TB), TB, 0, s>>>(fr.i.p, fr.j.p, nf, off.p, h.nchild.p, h.first_child.p,
                                                        h.center.p, h.side.p, h.d, h.tau, ci.p, cj.p, flags.p, nc);
        H2_LAUNCH_CHECK();
        int64_t tot[3];
        for (int t = 0; t < 3; ++t) {
            scan_excl_i32(flags.p + t * nc, pos.p + t * (nc + 1), nc, h.tmp_i32, s);
            tot[t] = read_scalar(pos.p + t * (nc + 1) + nc, s);
        }
        PairList* dst[3] = {&il, &nr, &fr2};
        fr2.n = 0;
        for (int t = 0; t < 3; ++t) {
            if (!tot[t]) continue;
            dst[t]->append_reserve(tot[t], s);
            k_compact<<<blocks_for(nc, TB), TB, 0, s>>>(ci.p, cj.p, nc, flags.p + t * nc, pos.p + t * (nc + 1),
                                                        dst[t]->i.p, dst[t]->j.p, dst[t]->n);
            H2_LAUNCH_CHECK();
            dst[t]->n += tot[t];
        }
        std::swap(fr.i.p, fr2.i.p);
        std::swap(fr.i.n, fr2.i.n);
        std::swap(fr.j.p, fr2.j.p);
        std::swap(fr.j.n, fr2.j.n);
        fr.n = fr2.n;
    }
    if (il.n > INT32_MAX || nr.n > INT32_MAX) fail(H2_EUNSUPPORTED, "list sizes exceed 2^31 entries");
    to_csr(h, il, h.il_ptr, h.il_col);
    to_csr(h, nr, h.nr_ptr, h.nr_col);
    h.nil = il.n;
    h.nnear = nr.n;
    h.h_il_ptr = read_vec(h.il_ptr.p, (size_t)h.nnode + 1, s);
    h.h_nr_ptr = read_vec(h.nr_ptr.p, (size_t)h.nnode + 1, s);
}

}  // namespace h2
