// Hierarchical data reduction (HiDR, Section 3.1 / Algorithm 1) with the
// volume-based DataReduct of Section 3.3, on the device.
//
// DataReduct(X, k) reading (identical to the oracle's):
//   |X| <= k            -> X unchanged;
//   otherwise           -> Q = cell centres of the g^d tensor grid over the
//                          bounding box of X (g the largest integer with
//                          g^d <= k, dimension 0 fastest); for every q the
//                          point of X at the smallest squared distance, ties to
//                          the earliest position in X; X* = the distinct picks
//                          in grid order of first occurrence.
// A list may come in parts; the reference set then holds one such grid per
// non-empty part (over that part's bounding box), each reference point taking
// its nearest point of the whole list.  The farfield list T_i of HiDR has two
// parts (Y_p^* and the interaction-list representors).
// One workgroup reduces one list.  Each lane owns up to QPT reference points
// and scans the list in LDS tiles of 256 points in list order, so the strict
// `<` keeps the earliest position.  Duplicated picks are removed with a
// bitonic sort of (pick, reference index) keys and the survivors compacted in
// reference-set order.
//
// HiDR: bottom-up (deepest level first) S_i = X_i for a leaf or the
// children's X_c^* concatenated, X_i^* = DataReduct(S_i, r1), each level's
// lists materialised with one scan and one gather; top-down T_i = Y_p^*
// followed by X_j^* for j in IL(i) ascending, Y_i^* = DataReduct(T_i, r2),
// reduced in place by an exact box-pruned search (k_datareduct_down).
//
// Compiled with -ffp-contract=off: distances round exactly as in the oracle,
// so the picks are bit-identical.
#include "common.h"

namespace h2 {
namespace {

constexpr int TB = 256;
constexpr int MAXQ_ALL = 4096;  // largest reference set: two grids of r <= 2048

__device__ inline double block_min(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = TB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ inline double block_max(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = TB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

template <int MAXQ>
__global__ __launch_bounds__(TB) void k_datareduct(const double* __restrict__ pts, int64_t ld, int d,
                                                   const int64_t* __restrict__ list_off,
                                                   const int* __restrict__ list_idx,
                                                   const int* __restrict__ split, int k, int* __restrict__ out,
                                                   int out_stride, int* __restrict__ out_cnt)
{
    __shared__ double sx[3][TB];
    __shared__ double red[TB];
    __shared__ int pick[MAXQ];
    __shared__ long long keys[MAXQ];
    __shared__ int scan_sh[TB];
    constexpr int QPT = MAXQ / TB;

    const int l = blockIdx.x;
    const int64_t b0 = list_off[l];
    const int64_t L = list_off[l + 1] - b0;
    const int* lst = list_idx + b0;
    int* o = out + (int64_t)l * out_stride;
    if (L <= k) {
        for (int64_t p = threadIdx.x; p < L; p += TB) o[p] = lst[p];
        if (threadIdx.x == 0) out_cnt[l] = (int)L;
        return;
    }
    // segments: [0, sp) and [sp, L); empty ones carry no grid
    const int64_t sp = split ? (int64_t)split[l] : L;
    int64_t seg_lo[2], seg_hi[2];
    int nseg = 0;
    if (sp > 0) {
        seg_lo[nseg] = 0;
        seg_hi[nseg++] = sp;
    }
    if (sp < L) {
        seg_lo[nseg] = sp;
        seg_hi[nseg++] = L;
    }
    // bounding box of every segment
    double lo[2][3], hi[2][3];
    for (int sg = 0; sg < nseg; ++sg)
        for (int a = 0; a < d; ++a) {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t p = seg_lo[sg] + threadIdx.x; p < seg_hi[sg]; p += TB) {
                double v = pts[a * ld + lst[p]];
                mn = fmin(mn, v);
                mx = fmax(mx, v);
            }
            lo[sg][a] = block_min(mn, red);
            hi[sg][a] = block_max(mx, red);
        }
    int g = 1;
    for (;;) {
        long long nx = 1;
        for (int a = 0; a < d; ++a) nx *= (long long)(g + 1);
        if (nx > k) break;
        ++g;
    }
    int nq1 = 1;
    for (int a = 0; a < d; ++a) nq1 *= g;
    const int nq = nq1 * nseg;

    // grid points owned by this lane: t = threadIdx.x + u*TB, in reference-set
    // order (segment 0's grid first)
    double qx[QPT][3];
    double best[QPT];
    int bi[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        int t = threadIdx.x + u * TB;
        best[u] = INFINITY;
        bi[u] = 0;
        int sg = t / nq1;
        if (sg > nseg - 1) sg = nseg - 1;
        int rem = t - sg * nq1;
        for (int a = 0; a < d; ++a) {
            int ta = rem % g;
            rem /= g;
            double w = (double)(2 * ta + 1) / (double)(2 * g);
            qx[u][a] = lo[sg][a] + (hi[sg][a] - lo[sg][a]) * w;
        }
    }
    const int nown = (nq - (int)threadIdx.x + TB - 1) / TB;  // reference points of this lane
    for (int64_t base = 0; base < L; base += TB) {
        int64_t p = base + threadIdx.x;
        if (p < L) {
            int id = lst[p];
            for (int a = 0; a < d; ++a) sx[a][threadIdx.x] = pts[a * ld + id];
        }
        __syncthreads();
        int nt = (int)min<int64_t>(TB, L - base);
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            if (u >= nown) break;
            double bu = best[u];
            int iu = bi[u];
            if (d == 3) {
                for (int e = 0; e < nt; ++e) {
                    double e0 = qx[u][0] - sx[0][e];
                    double e1 = qx[u][1] - sx[1][e];
                    double e2 = qx[u][2] - sx[2][e];
                    double dd = e0 * e0;
                    dd = dd + e1 * e1;
                    dd = dd + e2 * e2;
                    if (dd < bu) {
                        bu = dd;
                        iu = (int)base + e;
                    }
                }
            } else {
                for (int e = 0; e < nt; ++e) {
                    double dd = 0.0;
                    for (int a = 0; a < d; ++a) {
                        double ea = qx[u][a] - sx[a][e];
                        dd = dd + ea * ea;
                    }
                    if (dd < bu) {
                        bu = dd;
                        iu = (int)base + e;
                    }
                }
            }
            best[u] = bu;
            bi[u] = iu;
        }
        __syncthreads();
    }
    // (pick, grid index) keys; padding sorts last
    int P = 1;
    while (P < nq) P <<= 1;
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        int t = threadIdx.x + u * TB;
        if (t < nq) {
            pick[t] = bi[u];
            keys[t] = ((long long)bi[u] << 13) | t;
        } else if (t < P) {
            keys[t] = 0x7fffffffffffffffLL;
        }
    }
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int x = threadIdx.x; x < P; x += TB) {
                int y = x ^ jj;
                if (y > x) {
                    bool up = (x & kk) == 0;
                    long long a = keys[x], c = keys[y];
                    if ((a > c) == up) {
                        keys[x] = c;
                        keys[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    // first occurrence of every pick (smallest grid index): mark in pick[] by
    // negating the losers' entries -> flag array reuses `red` space via scan
    for (int x = threadIdx.x; x < nq; x += TB) {
        bool first = x == 0 || (keys[x - 1] >> 13) != (keys[x] >> 13);
        int t = (int)(keys[x] & 8191);
        if (!first) pick[t] = -1 - pick[t];
    }
    __syncthreads();
    // compaction in grid order: lane handles a contiguous run of grid indices
    const int per = (nq + TB - 1) / TB;
    int t0 = threadIdx.x * per;
    int c = 0;
    for (int t = t0; t < min(nq, t0 + per); ++t) c += pick[t] >= 0;
    scan_sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < TB; off <<= 1) {
        int a = (int)threadIdx.x >= off ? scan_sh[threadIdx.x - off] : 0;
        __syncthreads();
        scan_sh[threadIdx.x] += a;
        __syncthreads();
    }
    int w = scan_sh[threadIdx.x] - c;
    for (int t = t0; t < min(nq, t0 + per); ++t)
        if (pick[t] >= 0) o[w++] = lst[pick[t]];
    if (threadIdx.x == TB - 1) out_cnt[l] = scan_sh[TB - 1];
}


// Top-down DataReduct of T_i = Y_p^* ++ X_j^* (j in IL(i) ascending) without
// materialising T_i.  Same reference set, distances, tie rule and output as
// k_datareduct, but the nearest point of each reference point is found with
// exact pruning: every X_j^* lies in node j's (closed) box, so the box's
// squared distance lb_j bounds the distance of all its points from below; a
// box with lb_j (1 - 1e-12) > best cannot hold a point at distance <= best
// (the margin covers the rounding of lb_j and of the point distances), and
// the remaining candidates are scanned in list order with a strict `<`,
// which keeps the earliest position among equal distances.
template <int MAXQ>
__global__ __launch_bounds__(TB) void k_datareduct_down(
    int lo_node, const double* __restrict__ pts, int64_t ld, int d, const int* __restrict__ parent,
    const int* __restrict__ il_ptr, const int* __restrict__ il_col, const double* __restrict__ center,
    const double* __restrict__ side, const int* __restrict__ xs_cnt, const int* __restrict__ xs_idx, int r1,
    int* __restrict__ ys_cnt, int* __restrict__ ys_idx, int ys_stride, int k)
{
    __shared__ double red[TB];
    __shared__ long long keys[MAXQ];
    __shared__ int pick[MAXQ];
    __shared__ int scan_sh[TB];
    __shared__ long long lsum[TB];
    constexpr int QPT = MAXQ / TB;

    const int i = lo_node + blockIdx.x;
    const int p = parent[i];
    const int np_ = p > 0 ? ys_cnt[p] : 0;
    const int* yp = ys_idx + (int64_t)(p > 0 ? p : 0) * ys_stride;
    const int e0 = il_ptr[i], e1 = il_ptr[i + 1];
    int* o = ys_idx + (int64_t)i * ys_stride;

    long long part = 0;
    for (int e = e0 + threadIdx.x; e < e1; e += TB) part += xs_cnt[il_col[e]];
    lsum[threadIdx.x] = part;
    __syncthreads();
    for (int off = TB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) lsum[threadIdx.x] += lsum[threadIdx.x + off];
        __syncthreads();
    }
    const long long L = np_ + lsum[0];
    __syncthreads();
    if (L == 0) {
        if (threadIdx.x == 0) ys_cnt[i] = 0;
        return;
    }
    if (L <= k) {
        for (int q = threadIdx.x; q < np_; q += TB) o[q] = yp[q];
        int w = np_;
        for (int e = e0; e < e1; ++e) {
            const int j = il_col[e];
            const int c = xs_cnt[j];
            for (int q = threadIdx.x; q < c; q += TB) o[w + q] = xs_idx[(int64_t)j * r1 + q];
            w += c;
        }
        if (threadIdx.x == 0) ys_cnt[i] = (int)L;
        return;
    }
    // segments: 0 = Y_p^* (if any), 1 = the interaction-list part (if any)
    int nseg = 0;
    double lo[2][3], hi[2][3];
    if (np_ > 0) {
        for (int a = 0; a < d; ++a) {
            double mn = INFINITY, mx = -INFINITY;
            for (int q = threadIdx.x; q < np_; q += TB) {
                double v = pts[a * ld + yp[q]];
                mn = fmin(mn, v);
                mx = fmax(mx, v);
            }
            lo[nseg][a] = block_min(mn, red);
            hi[nseg][a] = block_max(mx, red);
        }
        ++nseg;
    }
    if (L > np_) {
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int e = e0; e < e1; ++e) {
            const int j = il_col[e];
            const int c = xs_cnt[j];
            for (int q = threadIdx.x; q < c; q += TB) {
                const int id = xs_idx[(int64_t)j * r1 + q];
                for (int a = 0; a < d; ++a) {
                    double v = pts[a * ld + id];
                    mn[a] = fmin(mn[a], v);
                    mx[a] = fmax(mx[a], v);
                }
            }
        }
        for (int a = 0; a < d; ++a) {
            lo[nseg][a] = block_min(mn[a], red);
            hi[nseg][a] = block_max(mx[a], red);
        }
        ++nseg;
    }
    int g = 1;
    for (;;) {
        long long nx = 1;
        for (int a = 0; a < d; ++a) nx *= (long long)(g + 1);
        if (nx > k) break;
        ++g;
    }
    int nq1 = 1;
    for (int a = 0; a < d; ++a) nq1 *= g;
    const int nq = nq1 * nseg;

    for (int u = 0; u < QPT; ++u) {
        const int t = threadIdx.x + u * TB;
        if (t >= nq) break;
        const int sg = t / nq1;
        int rem = t - sg * nq1;
        double q[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d; ++a) {
            int ta = rem % g;
            rem /= g;
            double w = (double)(2 * ta + 1) / (double)(2 * g);
            q[a] = lo[sg][a] + (hi[sg][a] - lo[sg][a]) * w;
        }
        double best = INFINITY;
        int bidx = -1;
        for (int c = 0; c < np_; ++c) {
            const int id = yp[c];
            double dd = 0.0;
            for (int a = 0; a < d; ++a) {
                double ea = q[a] - pts[a * ld + id];
                dd = dd + ea * ea;
            }
            if (dd < best) {
                best = dd;
                bidx = id;
            }
        }
        for (int e = e0; e < e1; ++e) {
            const int j = il_col[e];
            const double hs = 0.5 * side[j];
            double lb = 0.0;
            for (int a = 0; a < d; ++a) {
                double ex = fabs(q[a] - center[(int64_t)j * d + a]) - hs;
                if (ex > 0.0) lb = lb + ex * ex;
            }
            if (lb * (1.0 - 1e-12) > best) continue;
            const int c = xs_cnt[j];
            const int* xj = xs_idx + (int64_t)j * r1;
            for (int m = 0; m < c; ++m) {
                const int id = xj[m];
                double dd = 0.0;
                for (int a = 0; a < d; ++a) {
                    double ea = q[a] - pts[a * ld + id];
                    dd = dd + ea * ea;
                }
                if (dd < best) {
                    best = dd;
                    bidx = id;
                }
            }
        }
        pick[t] = bidx;
        keys[t] = ((long long)bidx << 13) | t;
    }
    int P = 1;
    while (P < nq) P <<= 1;
    for (int t = nq + threadIdx.x; t < P; t += TB) keys[t] = 0x7fffffffffffffffLL;
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int x = threadIdx.x; x < P; x += TB) {
                int y = x ^ jj;
                if (y > x) {
                    bool up = (x & kk) == 0;
                    long long a = keys[x], c = keys[y];
                    if ((a > c) == up) {
                        keys[x] = c;
                        keys[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int x = threadIdx.x; x < nq; x += TB) {
        bool first = x == 0 || (keys[x - 1] >> 13) != (keys[x] >> 13);
        int t = (int)(keys[x] & 8191);
        if (!first) pick[t] = -1;
    }
    __syncthreads();
    const int per = (nq + TB - 1) / TB;
    const int t0 = threadIdx.x * per;
    int c = 0;
    for (int t = t0; t < min(nq, t0 + per); ++t) c += pick[t] >= 0;
    scan_sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < TB; off <<= 1) {
        int a = (int)threadIdx.x >= off ? scan_sh[threadIdx.x - off] : 0;
        __syncthreads();
        scan_sh[threadIdx.x] += a;
        __syncthreads();
    }
    int w = scan_sh[threadIdx.x] - c;
    for (int t = t0; t < min(nq, t0 + per); ++t)
        if (pick[t] >= 0) o[w++] = pick[t];
    if (threadIdx.x == TB - 1) ys_cnt[i] = scan_sh[TB - 1];
}

// ---- list materialisation for one level of HiDR
__global__ __launch_bounds__(TB) void k_up_sizes(int lo, int nl, const int* __restrict__ nchild,
                                                 const int* __restrict__ first_child, const int* __restrict__ count,
                                                 const int* __restrict__ xs_cnt, int64_t* __restrict__ sz)
{
    int t = blockIdx.x * TB + threadIdx.x;
    if (t >= nl) return;
    int i = lo + t;
    int64_t v = 0;
    if (nchild[i] == 0)
        v = count[i];
    else
        for (int c = first_child[i]; c < first_child[i] + nchild[i]; ++c) v += xs_cnt[c];
    sz[t] = v;
}

__global__ __launch_bounds__(TB) void k_up_fill(int lo, const int* __restrict__ nchild,
                                                const int* __restrict__ first_child, const int* __restrict__ start,
                                                const int* __restrict__ count, const int* __restrict__ xs_cnt,
                                                const int* __restrict__ xs_idx, int r1, const int64_t* __restrict__ off,
                                                int* __restrict__ list)
{
    int t = blockIdx.x;
    int i = lo + t;
    int* o = list + off[t];
    if (nchild[i] == 0) {
        for (int p = threadIdx.x; p < count[i]; p += TB) o[p] = start[i] + p;
        return;
    }
    int64_t w = 0;
    for (int c = first_child[i]; c < first_child[i] + nchild[i]; ++c) {
        int cc = xs_cnt[c];
        for (int p = threadIdx.x; p < cc; p += TB) o[w + p] = xs_idx[(int64_t)c * r1 + p];
        w += cc;
    }
}

}  // namespace

void datareduct_lists(const double* pts, int64_t ld, int d, const int64_t* list_off, const int* list_idx,
                      const int* split, int nlist, int k, int* out, int out_stride, int* out_cnt, hipStream_t s)
{
    if (nlist <= 0) return;
    if (k < 1 || k > MAXQ_ALL / 2) fail(H2_EUNSUPPORTED, "DataReduct size must be in [1, 2048]");
    if (k <= 512)
        k_datareduct<1024><<<nlist, TB, 0, s>>>(pts, ld, d, list_off, list_idx, split, k, out, out_stride, out_cnt);
    else
        k_datareduct<MAXQ_ALL>
            <<<nlist, TB, 0, s>>>(pts, ld, d, list_off, list_idx, split, k, out, out_stride, out_cnt);
    H2_LAUNCH_CHECK();
}

void run_hidr(Handle& h)
{
    hipStream_t s = h.stream;
    const int nn = h.nnode;
    h.xs_cnt.ensure((size_t)nn, s);
    h.ys_cnt.ensure((size_t)nn, s);
    h.xs_idx.ensure((size_t)nn * h.r1, s);
    h.ys_stride = 2 * h.r2;
    h.ys_idx.ensure((size_t)nn * h.ys_stride, s);
    H2_HIP(hipMemsetAsync(h.xs_cnt.p, 0, sizeof(int) * nn, s));
    H2_HIP(hipMemsetAsync(h.ys_cnt.p, 0, sizeof(int) * nn, s));
    DBuf<int64_t> sz, off;
    DBuf<int> list;
    for (int L = h.maxdepth; L >= 1; --L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        sz.ensure((size_t)nl, s);
        off.ensure((size_t)nl + 1, s);
        k_up_sizes<<<blocks_for(nl, TB), TB, 0, s>>>(lo, nl, h.nchild.p, h.first_child.p, h.count.p, h.xs_cnt.p,
                                                     sz.p);
        H2_LAUNCH_CHECK();
        scan_excl_i64(sz.p, off.p, nl, h.tmp_i64, s);
        int64_t tot = read_scalar(off.p + nl, s);
        list.ensure((size_t)std::max<int64_t>(tot, 1), s);
        k_up_fill<<<nl, TB, 0, s>>>(lo, h.nchild.p, h.first_child.p, h.start.p, h.count.p, h.xs_cnt.p, h.xs_idx.p,
                                    h.r1, off.p, list.p);
        H2_LAUNCH_CHECK();
        datareduct_lists(h.pts.p, h.n, h.d, off.p, list.p, nullptr, nl, h.r1, h.xs_idx.p + (int64_t)lo * h.r1,
                         h.r1, h.xs_cnt.p + lo, s);
    }
    if (h.r2 < 1 || h.r2 > MAXQ_ALL / 2) fail(H2_EUNSUPPORTED, "r2 must be in [1, 2048]");
    for (int L = 1; L <= h.maxdepth; ++L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        if (h.r2 <= 512)
            k_datareduct_down<1024><<<nl, TB, 0, s>>>(lo, h.pts.p, h.n, h.d, h.parent.p, h.il_ptr.p, h.il_col.p,
                                                      h.center.p, h.side.p, h.xs_cnt.p, h.xs_idx.p, h.r1,
                                                      h.ys_cnt.p, h.ys_idx.p, h.ys_stride, h.r2);
        else
            k_datareduct_down<MAXQ_ALL><<<nl, TB, 0, s>>>(lo, h.pts.p, h.n, h.d, h.parent.p, h.il_ptr.p,
                                                          h.il_col.p, h.center.p, h.side.p, h.xs_cnt.p, h.xs_idx.p,
                                                          h.r1, h.ys_cnt.p, h.ys_idx.p, h.ys_stride, h.r2);
        H2_LAUNCH_CHECK();
    }
    H2_HIP(hipStreamSynchronize(s));
}

}  // namespace h2
