// Adaptive 2^d partition tree (Section 2.1 of the paper; Algorithm 2 step 1),
// built level-synchronously on the device.
//
// Readings (identical to the oracle's): the root box is the cube of side
// L = max_k (max x_k - min x_k) anchored at the per-axis minimum; a node
// splits iff it holds more than q points, its depth is below 48 and its side
// is positive; child code b = sum_k [x_k >= c_k] 2^k; empty children are
// dropped; points keep their relative order inside each child (stable).
// Node ids are BFS: depth, then parent id, then child code.
//
// One level is a handful of launches: per-point child codes, 2^d exclusive
// scans of the code indicator vectors (stable ranks), per-node child counts,
// a scan over the level's nodes to number the children, child creation and a
// scatter of the points.  Only the next level's node count is read back.
//
// This file is compiled with -ffp-contract=off so that every box centre,
// side and comparison rounds exactly as written.
#include "common.h"

namespace h2 {
namespace {

constexpr int MAXDEPTH = 48;
constexpr int TB = 256;

__global__ __launch_bounds__(TB) void k_bbox(const double* __restrict__ pts, int64_t n, int d,
                                             double* __restrict__ part, int* __restrict__ bad)
{
    __shared__ double smin[3][TB], smax[3][TB];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nonfinite = 0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        for (int a = 0; a < d; ++a) {
            double v = pts[a * n + i];
            if (!isfinite(v)) nonfinite = 1;
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    if (nonfinite) atomicOr(bad, 1);
    for (int a = 0; a < d; ++a) {
        smin[a][threadIdx.x] = lo[a];
        smax[a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int off = TB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int a = 0; a < d; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + off]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < d; ++a) {
            part[blockIdx.x * 6 + a] = smin[a][0];
            part[blockIdx.x * 6 + 3 + a] = smax[a][0];
        }
}

// Root node from the partial boxes (one thread; min/max are exact so the
// order of the partial reduction does not matter).
__global__ void k_root(const double* __restrict__ part, int nblk, int d, int64_t n, int* parent, int* first_child,
                       int* nchild, int* start, int* count, int* depth, double* center, double* side)
{
    double lo[3], hi[3];
    for (int a = 0; a < d; ++a) {
        lo[a] = part[a];
        hi[a] = part[3 + a];
    }
    for (int b = 1; b < nblk; ++b)
        for (int a = 0; a < d; ++a) {
            lo[a] = fmin(lo[a], part[b * 6 + a]);
            hi[a] = fmax(hi[a], part[b * 6 + 3 + a]);
        }
    double L = 0.0;
    for (int a = 0; a < d; ++a)
        if (hi[a] - lo[a] > L) L = hi[a] - lo[a];
    parent[0] = -1;
    first_child[0] = -1;
    nchild[0] = 0;
    start[0] = 0;
    count[0] = (int)n;
    depth[0] = 0;
    side[0] = L;
    for (int a = 0; a < d; ++a) center[a] = lo[a] + 0.5 * L;
}

__global__ __launch_bounds__(TB) void k_permute_in(const double* __restrict__ in, int64_t n, int d,
                                                   double* __restrict__ pts, int* __restrict__ perm,
                                                   int* __restrict__ pt_node)
{
    int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < d; ++a) pts[a * n + i] = in[a * n + i];
    perm[i] = (int)i;
    pt_node[i] = 0;
}

__device__ inline bool splits(int cnt, int dep, double s, int q) { return cnt > q && dep < MAXDEPTH && s > 0.0; }

// Child code of every point of a splitting node of the current level; -1
// for points whose node is a leaf or not on this level.  Writes the 2^d
// indicator vectors used for the stable ranks.
__global__ __launch_bounds__(TB) void k_codes(const double* __restrict__ pts, int64_t n, int d,
                                              const int* __restrict__ pt_node, int lo_node, int hi_node,
                                              const int* __restrict__ count, const int* __restrict__ depth,
                                              const double* __restrict__ side, const double* __restrict__ center,
                                              int q, int* __restrict__ code, int* __restrict__ flags)
{
    int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    int nd = pt_node[i];
    int c = -1;
    if (nd >= lo_node && nd < hi_node && splits(count[nd], depth[nd], side[nd], q)) {
        c = 0;
        for (int a = 0; a < d; ++a)
            if (pts[a * n + i] >= center[(int64_t)nd * d + a]) c |= 1 << a;
    }
    code[i] = c;
    int nb = 1 << d;
    for (int b = 0; b < nb; ++b) flags[(int64_t)b * n + i] = (c == b) ? 1 : 0;
}

// Per node of the level: child counts from the scanned indicators and the
// number of non-empty children.
__global__ __launch_bounds__(TB) void k_child_counts(int lo_node, int nl, int d, int64_t n, const int* __restrict__ start,
                                                     const int* __restrict__ count, const int* __restrict__ depth,
                                                     const double* __restrict__ side, int q,
                                                     const int* __restrict__ pre, int* __restrict__ ccnt,
                                                     int* __restrict__ nch)
{
    int t = blockIdx.x * TB + threadIdx.x;
    if (t >= nl) return;
    int nd = lo_node + t;
    int nb = 1 << d;
    int k = 0;
    bool sp = splits(count[nd], depth[nd], side[nd], q);
    for (int b = 0; b < nb; ++b) {
        int c = 0;
        if (sp) {
            const int* pb = pre + (int64_t)b * (n + 1);
            c = pb[start[nd] + count[nd]] - pb[start[nd]];
        }
        ccnt[t * 8 + b] = c;
        k += c > 0;
    }
    nch[t] = k;
}

__global__ __launch_bounds__(TB) void k_make_children(int lo_node, int nl, int d, int next_base,
                                                      const int* __restrict__ nch_off, const int* __restrict__ ccnt,
                                                      int* parent, int* first_child, int* nchild, int* start,
                                                      int* count, int* depth, double* center, double* side,
                                                      int* __restrict__ coff, int* __restrict__ cid)
{
    int t = blockIdx.x * TB + threadIdx.x;
    if (t >= nl) return;
    int nd = lo_node + t;
    int nb = 1 << d;
    int base = next_base + nch_off[t];
    int k = 0, off = 0;
    double s = side[nd];
    double qs = s * 0.25;
    for (int b = 0; b < nb; ++b) {
        int c = ccnt[t * 8 + b];
        coff[t * 8 + b] = off;
        cid[t * 8 + b] = -1;
        if (c == 0) continue;
        int ch = base + k;
        cid[t * 8 + b] = ch;
        parent[ch] = nd;
        first_child[ch] = -1;
        nchild[ch] = 0;
        start[ch] = start[nd] + off;
        count[ch] = c;
        depth[ch] = depth[nd] + 1;
        side[ch] = s * 0.5;
        for (int a = 0; a < d; ++a) {
            double ca = center[(int64_t)nd * d + a];
            center[(int64_t)ch * d + a] = ((b >> a) & 1) ? ca + qs : ca - qs;
        }
        ++k;
        off += c;
    }
    if (k > 0) {
        first_child[nd] = base;
        nchild[nd] = k;
    }
}

__global__ __launch_bounds__(TB) void k_scatter(const double* __restrict__ pts, int64_t n, int d,
                                                const int* __restrict__ perm, const int* __restrict__ pt_node,
                                                const int* __restrict__ code, const int* __restrict__ pre,
                                                int lo_node, const int* __restrict__ start,
                                                const int* __restrict__ coff, const int* __restrict__ cid,
                                                double* __restrict__ pts2, int* __restrict__ perm2,
                                                int* __restrict__ pt_node2)
{
    int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    int c = code[i];
    int nd = pt_node[i];
    int64_t dst = i;
    int nn = nd;
    if (c >= 0) {
        int t = nd - lo_node;
        const int* pb = pre + (int64_t)c * (n + 1);
        dst = (int64_t)start[nd] + coff[t * 8 + c] + (pb[i] - pb[start[nd]]);
        nn = cid[t * 8 + c];
    }
    for (int a = 0; a < d; ++a) pts2[a * n + dst] = pts[a * n + i];
    perm2[dst] = perm[i];
    pt_node2[dst] = nn;
}

}  // namespace

void build_tree(Handle& h, const double* pts_in)
{
    hipStream_t s = h.stream;
    const int64_t n = h.n;
    const int d = h.d;
    const int nb = 1 << d;

    h.pts.ensure((size_t)d * n, s);
    h.perm.ensure((size_t)n, s);
    DBuf<double> pts2;
    pts2.ensure((size_t)d * n, s);
    DBuf<int> perm2, node_a, node_b, code, flags, pre;
    perm2.ensure((size_t)n, s);
    node_a.ensure((size_t)n, s);
    node_b.ensure((size_t)n, s);
    code.ensure((size_t)n, s);
    flags.ensure((size_t)nb * n, s);
    pre.ensure((size_t)nb * (n + 1), s);

    // node arrays, grown as levels are added
    size_t cap = 1024;
    auto grow_nodes = [&](size_t need, size_t keep) {
        if (need <= cap && h.parent.p) return;
        size_t nc = cap;
        while (nc < need) nc *= 2;
        h.parent.grow_keep(nc, keep, s);
        h.first_child.grow_keep(nc, keep, s);
        h.nchild.grow_keep(nc, keep, s);
        h.start.grow_keep(nc, keep, s);
        h.count.grow_keep(nc, keep, s);
        h.depth.grow_keep(nc, keep, s);
        h.side.grow_keep(nc, keep, s);
        h.center.grow_keep(nc * d, keep * d, s);
        cap = nc;
    };
    grow_nodes(cap, 0);

    // root box and finiteness check
    int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + TB - 1) / TB));
    DBuf<double> part;
    part.ensure((size_t)nblk * 6, s);
    DBuf<int> bad;
    bad.ensure(1, s);
    H2_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    k_bbox<<<nblk, TB, 0, s>>>(pts_in, n, d, part.p, bad.p);
    H2_LAUNCH_CHECK();
    if (read_scalar(bad.p, s)) fail(H2_EINVAL, "points contain non-finite coordinates");
    k_root<<<1, 1, 0, s>>>(part.p, nblk, d, n, h.parent.p, h.first_child.p, h.nchild.p, h.start.p, h.count.p,
                          h.depth.p, h.center.p, h.side.p);
    H2_LAUNCH_CHECK();
    k_permute_in<<<blocks_for(n, TB), TB, 0, s>>>(pts_in, n, d, h.pts.p, h.perm.p, node_a.p);
    H2_LAUNCH_CHECK();

    h.lvl_ptr.assign(1, 0);
    int lo_node = 0, hi_node = 1;
    DBuf<int> ccnt, nch, nch_off, coff, cid;
    while (lo_node < hi_node) {
        h.lvl_ptr.push_back(hi_node);
        int nl = hi_node - lo_node;
        k_codes<<<blocks_for(n, TB), TB, 0, s>>>(h.pts.p, n, d, node_a.p, lo_node, hi_node, h.count.p, h.depth.p,
                                                 h.side.p, h.center.p, h.q, code.p, flags.p);
        H2_LAUNCH_CHECK();
        for (int b = 0; b < nb; ++b)
            scan_excl_i32(flags.p + (int64_t)b * n, pre.p + (int64_t)b * (n + 1), n, h.tmp_i32, s);
        ccnt.ensure((size_t)nl * 8, s);
        nch.ensure((size_t)nl, s);
        nch_off.ensure((size_t)nl + 1, s);
        coff.ensure((size_t)nl * 8, s);
        cid.ensure((size_t)nl * 8, s);
        k_child_counts<<<blocks_for(nl, TB), TB, 0, s>>>(lo_node, nl, d, n, h.start.p, h.count.p, h.depth.p,
                                                         h.side.p, h.q, pre.p, ccnt.p, nch.p);
        H2_LAUNCH_CHECK();
        scan_excl_i32(nch.p, nch_off.p, nl, h.tmp_i32, s);
        int nnew = read_scalar(nch_off.p + nl, s);
        if (nnew == 0) break;
        grow_nodes((size_t)hi_node + nnew, (size_t)hi_node);
        k_make_children<<<blocks_for(nl, TB), TB, 0, s>>>(lo_node, nl, d, hi_node, nch_off.p, ccnt.p, h.parent.p,
                                                          h.first_child.p, h.nchild.p, h.start.p, h.count.p,
                                                          h.depth.p, h.center.p, h.side.p, coff.p, cid.p);
        H2_LAUNCH_CHECK();
        k_scatter<<<blocks_for(n, TB), TB, 0, s>>>(h.pts.p, n, d, h.perm.p, node_a.p, code.p, pre.p, lo_node,
                                                   h.start.p, coff.p, cid.p, pts2.p, perm2.p, node_b.p);
        H2_LAUNCH_CHECK();
        std::swap(h.pts.p, pts2.p);
        std::swap(h.perm.p, perm2.p);
        std::swap(node_a.p, node_b.p);
        lo_node = hi_node;
        hi_node += nnew;
    }
    h.nnode = hi_node;
    h.maxdepth = (int)h.lvl_ptr.size() - 2;
    h.h_nchild = read_vec(h.nchild.p, h.nnode, s);
    h.h_first_child = read_vec(h.first_child.p, h.nnode, s);
    h.h_start = read_vec(h.start.p, h.nnode, s);
    h.h_count = read_vec(h.count.p, h.nnode, s);
    h.h_parent = read_vec(h.parent.p, h.nnode, s);
}

}  // namespace h2
