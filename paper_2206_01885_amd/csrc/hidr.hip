// Hierarchical data reduction (HiDR, Section 3.1 / Algorithm 1) with the
// volume-based DataReduct of Section 3.3, on the device; the surface-based
// method and farthest point sampling of the same section as options.
//
// DataReduct(X, k) reading (identical to the oracle's), k the maximum size
// of X* (Algorithm 1's r1 for X_i^*, r2 for Y_i^*):
//   |X| <= k            -> X unchanged;
//   otherwise           -> Q = cell centres of the g^d tensor grid over the
//                          bounding box of X (g the largest integer with
//                          g^d <= k, dimension 0 fastest); for every q the
//                          point of X at the smallest squared distance, ties to
//                          the earliest position in X; X* = the distinct picks
//                          in grid order of first occurrence.
// A list may come in two parts; the reference set then holds one such grid
// per non-empty part (over that part's bounding box, g^d <= k/2), each
// reference point taking its nearest point of the whole list, so |X*| <= k.
// The farfield list T_i of HiDR has two parts (Y_p^* and the
// interaction-list representors).
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
#include <cmath>
#include <type_traits>

#include "common.h"

namespace h2 {
namespace {

constexpr int TB = 256;
constexpr int MAXQ_ALL = 4096;  // largest reference set: r2 <= 4096 (two grids of r2/2)
constexpr int MAXR1 = 2048;     // largest r1 (the options are checked against it)

template <int NTH = TB>
__device__ inline double block_min(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = NTH / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
template <int NTH = TB>
__device__ inline double block_max(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = NTH / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// The surface method (method = H2_DR_SURFACE) differs only in its reference
// set: per part, with box [lo, hi], widths w = hi - lo and centre
// c = lo + 0.5 w, the points c + (gamma w) u_j on the ellipsoids gamma = 0.3,
// 0.6, 1.2 for the mdir unit directions u_j of `dirs` ([mdir][d]), in the
// order gamma, then j, the first kp of them (kp = the part's share of k).
template <int MAXQ>
__global__ __launch_bounds__(TB) void k_datareduct(const double* __restrict__ pts, int64_t ld, int d,
                                                   const int64_t* __restrict__ list_off,
                                                   const int* __restrict__ list_idx,
                                                   const int* __restrict__ split, int k, int* __restrict__ out,
                                                   int out_stride, int* __restrict__ out_cnt, int method,
                                                   const double* __restrict__ dirs, int mdir)
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
    const bool surf = method == H2_DR_SURFACE;
    const int kp = split ? max(1, k / 2) : k;  // grid budget of one part
    int g = 1;
    for (;;) {
        long long nx = 1;
        for (int a = 0; a < d; ++a) nx *= (long long)(g + 1);
        if (nx > kp) break;
        ++g;
    }
    int nq1 = 1;
    for (int a = 0; a < d; ++a) nq1 *= g;
    if (surf) nq1 = min(kp, 3 * mdir);
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
        if (surf) {
            const int e = rem / mdir, j = rem % mdir;
            const double gm = e == 0 ? 0.3 : (e == 1 ? 0.6 : 1.2);
            for (int a = 0; a < d; ++a) {
                const double w = hi[sg][a] - lo[sg][a];
                const double c = lo[sg][a] + 0.5 * w;
                qx[u][a] = c + (gm * w) * dirs[j * d + a];
            }
        } else {
            for (int a = 0; a < d; ++a) {
                int ta = rem % g;
                rem /= g;
                double w = (double)(2 * ta + 1) / (double)(2 * g);
                qx[u][a] = lo[sg][a] + (hi[sg][a] - lo[sg][a]) * w;
            }
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


// Coordinates of the list entries in list order, SoA [d][tot].
__global__ __launch_bounds__(TB) void k_list_coords(const double* __restrict__ pts, int64_t ld, int d,
                                                    const int* __restrict__ list_idx, int64_t tot,
                                                    double* __restrict__ cw)
{
    const int64_t p = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (p >= tot) return;
    const int id = list_idx[p];
    for (int a = 0; a < d; ++a) cw[a * tot + p] = pts[a * ld + id];
}

// Farthest point sampling of a list, one workgroup per list: S = {first
// point}; then repeatedly every lane lowers the squared distance to S of its
// points (md, in list order, distances in coordinate order as the oracle
// forms them) by the last pick and the workgroup takes the largest, the
// earliest position among equal ones, until |S| = k or the largest is 0.
// |X| <= k: X unchanged.  The picks are written in selection order.
// Lists of up to FPS_TMAX tiles of TB consecutive entries keep per tile its
// bounding box and the largest md with its earliest position; a pick leaves
// a tile alone when the squared distance from the pick to the tile's box
// (formed like the entries' distances, so by monotone rounding never above
// any of them) is not below the tile's largest md, as no entry can then get
// closer.  The picks are those of the full pass.
constexpr int FPS_TMAX = 512;
__global__ __launch_bounds__(TB) void k_datareduct_fps(const double* __restrict__ cw, int64_t tot, int d,
                                                       const int64_t* __restrict__ list_off,
                                                       const int* __restrict__ list_idx, int k,
                                                       int* __restrict__ out, int out_stride,
                                                       int* __restrict__ out_cnt, double* __restrict__ md_ws)
{
    __shared__ double rv[TB];
    __shared__ int rp[TB];
    __shared__ double tlo[3][FPS_TMAX], thi[3][FPS_TMAX], tmx[FPS_TMAX];
    __shared__ int tps[FPS_TMAX];
    const int l = blockIdx.x;
    const int64_t b0 = list_off[l];
    const int L = (int)(list_off[l + 1] - b0);
    const int* lst = list_idx + b0;
    int* o = out + (int64_t)l * out_stride;
    const int tid = threadIdx.x;
    if (L <= k) {
        for (int p = tid; p < L; p += TB) o[p] = lst[p];
        if (tid == 0) out_cnt[l] = L;
        return;
    }
    const double* x0 = cw + b0;
    const double* x1 = cw + tot + b0;
    const double* x2 = cw + 2 * tot + b0;
    double* md = md_ws + b0;  // each entry read and written by its own lane only
    const int nt = (L + TB - 1) / TB;
    if (nt <= FPS_TMAX) {
        // wave w owns the tiles t = w mod 4, lane l the entries t TB + 64 q + l
        constexpr int NW = TB / 64;
        const int w = tid >> 6, lane = tid & 63;
        for (int t = w; t < nt; t += NW) {
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int q = 0; q < NW; ++q) {
                const int p = t * TB + 64 * q + lane;
                if (p < L) {
                    md[p] = INFINITY;
                    const double v[3] = {x0[p], d > 1 ? x1[p] : 0.0, d > 2 ? x2[p] : 0.0};
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = fmin(lo[a], v[a]);
                        hi[a] = fmax(hi[a], v[a]);
                    }
                }
            }
            for (int off = 32; off > 0; off >>= 1)
                for (int a = 0; a < 3; ++a) {
                    lo[a] = fmin(lo[a], __shfl_xor(lo[a], off, 64));
                    hi[a] = fmax(hi[a], __shfl_xor(hi[a], off, 64));
                }
            if (lane == 0) {
                for (int a = 0; a < 3; ++a) {
                    tlo[a][t] = lo[a];
                    thi[a][t] = hi[a];
                }
                tmx[t] = INFINITY;
                tps[t] = t * TB;
            }
        }
        __syncthreads();
        int cur = 0, cnt = 0;
        for (;;) {
            if (tid == 0) o[cnt] = lst[cur];
            ++cnt;
            if (cnt == k) break;
            const double c0 = x0[cur];
            const double c1 = d > 1 ? x1[cur] : 0.0;
            const double c2 = d > 2 ? x2[cur] : 0.0;
            for (int t = w; t < nt; t += NW) {
                double e = fmax(fmax(tlo[0][t] - c0, c0 - thi[0][t]), 0.0);
                double lb = e * e;
                if (d > 1) {
                    e = fmax(fmax(tlo[1][t] - c1, c1 - thi[1][t]), 0.0);
                    lb = lb + e * e;
                }
                if (d > 2) {
                    e = fmax(fmax(tlo[2][t] - c2, c2 - thi[2][t]), 0.0);
                    lb = lb + e * e;
                }
                if (!(lb < tmx[t])) continue;  // wave-uniform
                double bv = -1.0;
                int bp = 0x7fffffff;
                for (int q = 0; q < NW; ++q) {
                    const int p = t * TB + 64 * q + lane;
                    if (p < L) {
                        const double e0 = x0[p] - c0;
                        double dd = e0 * e0;
                        if (d > 1) {
                            const double e1 = x1[p] - c1;
                            dd = dd + e1 * e1;
                        }
                        if (d > 2) {
                            const double e2 = x2[p] - c2;
                            dd = dd + e2 * e2;
                        }
                        double mv = md[p];
                        if (dd < mv) {
                            mv = dd;
                            md[p] = mv;
                        }
                        if (mv > bv) {
                            bv = mv;
                            bp = p;
                        }
                    }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const double v2 = __shfl_xor(bv, off, 64);
                    const int p2 = __shfl_xor(bp, off, 64);
                    if (v2 > bv || (v2 == bv && p2 < bp)) {
                        bv = v2;
                        bp = p2;
                    }
                }
                if (lane == 0) {
                    tmx[t] = bv;
                    tps[t] = bp;
                }
            }
            __syncthreads();
            double bv = -1.0;
            int bp = 0x7fffffff;
            for (int t = tid; t < nt; t += TB)
                if (tmx[t] > bv || (tmx[t] == bv && tps[t] < bp)) {
                    bv = tmx[t];
                    bp = tps[t];
                }
            rv[tid] = bv;
            rp[tid] = bp;
            __syncthreads();
            for (int off = TB / 2; off > 0; off >>= 1) {
                if (tid < off) {
                    const double v2 = rv[tid + off];
                    const int p2 = rp[tid + off];
                    if (v2 > rv[tid] || (v2 == rv[tid] && p2 < rp[tid])) {
                        rv[tid] = v2;
                        rp[tid] = p2;
                    }
                }
                __syncthreads();
            }
            const double best = rv[0];
            const int bpos = rp[0];
            __syncthreads();
            if (!(best > 0.0)) break;
            cur = bpos;
        }
        if (tid == 0) out_cnt[l] = cnt;
        return;
    }
    for (int p = tid; p < L; p += TB) md[p] = INFINITY;
    int cur = 0, cnt = 0;
    for (;;) {
        if (tid == 0) o[cnt] = lst[cur];
        ++cnt;
        if (cnt == k) break;
        const double c0 = x0[cur];
        const double c1 = d > 1 ? x1[cur] : 0.0;
        const double c2 = d > 2 ? x2[cur] : 0.0;
        double bv = -1.0;
        int bp = 0x7fffffff;
        for (int p = tid; p < L; p += TB) {
            const double e0 = x0[p] - c0;
            double dd = e0 * e0;
            if (d > 1) {
                const double e1 = x1[p] - c1;
                dd = dd + e1 * e1;
            }
            if (d > 2) {
                const double e2 = x2[p] - c2;
                dd = dd + e2 * e2;
            }
            double mv = md[p];
            if (dd < mv) {
                mv = dd;
                md[p] = mv;
            }
            if (mv > bv) {  // strict: a lane's earliest position among equal values
                bv = mv;
                bp = p;
            }
        }
        rv[tid] = bv;
        rp[tid] = bp;
        __syncthreads();
        for (int off = TB / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double v2 = rv[tid + off];
                const int p2 = rp[tid + off];
                if (v2 > rv[tid] || (v2 == rv[tid] && p2 < rp[tid])) {
                    rv[tid] = v2;
                    rp[tid] = p2;
                }
            }
            __syncthreads();
        }
        const double best = rv[0];
        const int bpos = rp[0];
        __syncthreads();
        if (!(best > 0.0)) break;
        cur = bpos;
    }
    if (tid == 0) out_cnt[l] = cnt;
}

// Top-down DataReduct of T_i = Y_p^* ++ X_j^* (j in IL(i) ascending) without
// materialising T_i.  Same reference set, distances, tie rule and output as
// k_datareduct, but the nearest point of each reference point is found with
// exact pruning: every X_j^* lies in node j's (closed) box, so the box's
// squared distance lb_j bounds the distance of all its points from below; a
// box with lb_j (1 - 1e-12) > best cannot hold a point at distance <= best
// (the margin covers the rounding of lb_j and of the point distances).  The
// candidates are compared by (distance, list position), which yields the
// sequential scan's answer -- smallest distance, earliest position among
// equal ones -- whatever the scan order; the box nearest to q is scanned
// first so that the bound prunes well.
// The staged Y_p^* is searched the same way, by runs of YCH points with
// their bounding boxes, after the nearest box has set a first bound.
// The interaction-list table (box centre, half side, count, list offset) and
// (up to YCAP points) the coordinates of Y_p^* are staged in LDS; nodes with
// more than ILCAP interaction-list entries are skipped here and reduced from
// their materialised T_i by k_datareduct (same reference set, distances, tie
// rule and output).
constexpr int ILCAP = 640;  // interaction-list entries staged per node
constexpr int YCAP = 768;   // Y_p^* points staged per node
constexpr int PB = 8;       // candidate loads issued ahead
constexpr int NCO = 9;      // child offsets per node in the grouped copy of X_i^* (2^d + 1)
constexpr int SPLIT_MIN = H2_TUNE_SPLIT_MIN;  // boxes with more candidates are searched child by child
constexpr int YCH = 16;        // staged Y_p^* points per bounding box of the search

__device__ __forceinline__ int seg_of(const int* __restrict__ off, int n, int p)
{
    // last e with off[e] <= p (off ascending, off[0] = 0)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int D, int MAXQ, int NTH>
__global__ __launch_bounds__(NTH) void k_datareduct_down(
    int lo_node, const double* __restrict__ pts, int64_t ld, const int* __restrict__ parent,
    const int* __restrict__ il_ptr, const int* __restrict__ il_col, const double* __restrict__ center,
    const double* __restrict__ side, const int* __restrict__ xs_cnt, const int* __restrict__ xs_idx,
    const double* __restrict__ xs_pts, const int* __restrict__ xs_pos, const int* __restrict__ xs_coff,
    const int* __restrict__ nchild, const int* __restrict__ first_child, int r1, int* __restrict__ ys_cnt,
    int* __restrict__ ys_idx, int ys_stride, int k, int nl, int method, const double* __restrict__ dirs, int mdir)
{
    __shared__ double red[NTH];
    __shared__ int scan_sh[NTH];
    // box table in FP32, rounded outward (centre to nearest, half side up by
    // the centre's rounding and one more ulp): every box it describes contains
    // the true box, so its distance stays a lower bound and the pruning exact
    __shared__ float bx[3][ILCAP];
    __shared__ float bh[ILCAP];
    __shared__ int bj[ILCAP], bcnt[ILCAP], boff[ILCAP + 1];
    __shared__ double yc[3][YCAP];
    // the sort keys and picks reuse the staged Y_p^* once the searches are
    // done (when they fit), which keeps three workgroups per CU
    constexpr bool ALIAS = 3 * YCAP * sizeof(double) >= MAXQ * (sizeof(long long) + sizeof(int));
    __shared__ long long keys_own[ALIAS ? 1 : MAXQ];
    __shared__ int pick_own[ALIAS ? 1 : MAXQ];
    long long* keys = ALIAS ? (long long*)&yc[0][0] : keys_own;
    int* pick = ALIAS ? (int*)((long long*)&yc[0][0] + MAXQ) : pick_own;
    constexpr int QPT = MAXQ / NTH;
    constexpr int d = D;

    // workgroup ids go round-robin over the 8 XCDs: each XCD takes a
    // contiguous range of the level's nodes, so that the boxes shared by
    // neighbouring nodes' interaction lists are read through one L2
    const int xper = (nl + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * xper + (int)(blockIdx.x / 8);
    if (t >= nl) return;
    const int i = lo_node + t;
    const int p = parent[i];
    const int np_ = p > 0 ? ys_cnt[p] : 0;
    const int* yp = ys_idx + (int64_t)(p > 0 ? p : 0) * ys_stride;
    const int e0 = il_ptr[i], ne = il_ptr[i + 1] - e0;
    if (ne > ILCAP) return;  // handled by the materialised path
    int* o = ys_idx + (int64_t)i * ys_stride;

    // interaction-list table and its exclusive prefix of counts
    for (int e = threadIdx.x; e < ne; e += NTH) {
        const int j = il_col[e0 + e];
        bj[e] = j;
        bcnt[e] = xs_cnt[j];
        double err = 0.0;
        for (int a = 0; a < d; ++a) {
            const double c = center[(int64_t)j * d + a];
            const float cf = (float)c;
            bx[a][e] = cf;
            err = fmax(err, fabs(c - (double)cf));
        }
        const double hh = 0.5 * side[j] + err;
        float hf = (float)hh;
        if ((double)hf < hh) hf = nextafterf(hf, INFINITY);
        bh[e] = nextafterf(hf, INFINITY);
    }
    const bool stage_y = np_ <= YCAP;
    if (stage_y)
        for (int q = threadIdx.x; q < np_; q += NTH)
            for (int a = 0; a < d; ++a) yc[a][q] = pts[a * ld + yp[q]];
    __syncthreads();
    // bounding boxes of the staged Y_p^* in runs of YCH points, in FP32
    // rounded outward (they contain every point of their run)
    __shared__ float ylo[3][YCAP / YCH], yhi[3][YCAP / YCH];
    const int nych = stage_y ? (np_ + YCH - 1) / YCH : 0;
    for (int w = threadIdx.x; w < nych * D; w += NTH) {
        const int ch = w / D, a = w - ch * D;
        double mn = INFINITY, mx = -INFINITY;
        for (int q = ch * YCH; q < min(np_, ch * YCH + YCH); ++q) {
            mn = fmin(mn, yc[a][q]);
            mx = fmax(mx, yc[a][q]);
        }
        float fl = (float)mn, fh = (float)mx;
        if ((double)fl > mn) fl = nextafterf(fl, -INFINITY);
        if ((double)fh < mx) fh = nextafterf(fh, INFINITY);
        ylo[a][ch] = fl;
        yhi[a][ch] = fh;
    }
    {
        // block scan over ne <= ILCAP counts: each lane sums a run of entries
        const int per = (ne + NTH - 1) / NTH;
        const int q0 = threadIdx.x * per;
        int c = 0;
        for (int e = q0; e < min(ne, q0 + per); ++e) c += bcnt[e];
        scan_sh[threadIdx.x] = c;
        __syncthreads();
        for (int off = 1; off < NTH; off <<= 1) {
            int a = (int)threadIdx.x >= off ? scan_sh[threadIdx.x - off] : 0;
            __syncthreads();
            scan_sh[threadIdx.x] += a;
            __syncthreads();
        }
        int w = scan_sh[threadIdx.x] - c;
        for (int e = q0; e < min(ne, q0 + per); ++e) {
            boff[e] = w;
            w += bcnt[e];
        }
        if (threadIdx.x == NTH - 1) boff[ne] = scan_sh[NTH - 1];
        __syncthreads();
    }
    const int Lil = boff[ne];
    const int L = np_ + Lil;
    if (L == 0) {
        if (threadIdx.x == 0) ys_cnt[i] = 0;
        return;
    }
    if (L <= k) {
        for (int q = threadIdx.x; q < np_; q += NTH) o[q] = yp[q];
        for (int q = threadIdx.x; q < Lil; q += NTH) {
            const int e = seg_of(boff, ne, q);
            o[np_ + q] = xs_idx[(int64_t)bj[e] * r1 + (q - boff[e])];
        }
        if (threadIdx.x == 0) ys_cnt[i] = L;
        return;
    }
    // segments: 0 = Y_p^* (if any), 1 = the interaction-list part (if any);
    // their boxes live in LDS so that the per-lane segment choice is a plain
    // LDS read
    __shared__ double lo[2][3], hi[2][3];
    int nseg = 0;
    if (np_ > 0) {
        for (int a = 0; a < d; ++a) {
            double mn = INFINITY, mx = -INFINITY;
            for (int q = threadIdx.x; q < np_; q += NTH) {
                const double v = stage_y ? yc[a][q] : pts[a * ld + yp[q]];
                mn = fmin(mn, v);
                mx = fmax(mx, v);
            }
            const double l0 = block_min<NTH>(mn, red), h0 = block_max<NTH>(mx, red);
            if (threadIdx.x == 0) {
                lo[nseg][a] = l0;
                hi[nseg][a] = h0;
            }
        }
        ++nseg;
    }
    if (Lil > 0) {
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int q = threadIdx.x; q < Lil; q += NTH) {
            const int e = seg_of(boff, ne, q);
            const int id = xs_idx[(int64_t)bj[e] * r1 + (q - boff[e])];
            for (int a = 0; a < d; ++a) {
                double v = pts[a * ld + id];
                mn[a] = fmin(mn[a], v);
                mx[a] = fmax(mx[a], v);
            }
        }
        for (int a = 0; a < d; ++a) {
            const double l0 = block_min<NTH>(mn[a], red), h0 = block_max<NTH>(mx[a], red);
            if (threadIdx.x == 0) {
                lo[nseg][a] = l0;
                hi[nseg][a] = h0;
            }
        }
        ++nseg;
    }
    __syncthreads();
    const int kp = max(1, k / 2);  // grid budget of each part of T_i
    int g = 1;
    for (;;) {
        long long nx = 1;
        for (int a = 0; a < d; ++a) nx *= (long long)(g + 1);
        if (nx > kp) break;
        ++g;
    }
    int nq1 = 1;
    for (int a = 0; a < d; ++a) nq1 *= g;
    // the surface method's reference set (k_datareduct's): per part, the
    // points c + (gamma w) u_j on the ellipsoids gamma = 0.3, 0.6, 1.2
    const bool surf = method == H2_DR_SURFACE;
    if (surf) nq1 = min(kp, 3 * mdir);
    const int nq = nq1 * nseg;

    // A lane's reference points (t = lane + NTH u) go through every phase
    // together, so each candidate and each box is read once per lane.
    double qv[QPT][D];
    double best[QPT];
    int bpos[QPT];
    bool act[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        const int t = threadIdx.x + u * NTH;
        act[u] = t < nq;
        const int tq = act[u] ? t : 0;
        const int sg = tq / nq1;
        int rem = tq - sg * nq1;
        if (surf) {
            const int e = rem / mdir, j = rem % mdir;
            const double gm = e == 0 ? 0.3 : (e == 1 ? 0.6 : 1.2);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double w = hi[sg][a] - lo[sg][a];
                const double c = lo[sg][a] + 0.5 * w;
                qv[u][a] = c + (gm * w) * dirs[j * D + a];
            }
        } else {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                int ta = rem % g;
                rem /= g;
                double w = (double)(2 * ta + 1) / (double)(2 * g);
                qv[u][a] = lo[sg][a] + (hi[sg][a] - lo[sg][a]) * w;
            }
        }
        best[u] = INFINITY;
        bpos[u] = 0x7fffffff;
    }
    // (distance, position) minimum: the sequential scan's answer in any
    // order; the point index is looked up from the position at the end
    auto consider = [&](int u, double dd, int pos) {
        if (dd < best[u] || (dd == best[u] && pos < bpos[u])) {
            best[u] = dd;
            bpos[u] = pos;
        }
    };
    auto dist = [&](int u, const double* c3) {
        double dd = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double ea = qv[u][a] - c3[a];
            dd = dd + ea * ea;
        }
        return dd;
    };
    auto box_lb = [&](int u, const double* bc, double h) {
        double lb = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double ex = fabs(qv[u][a] - bc[a]) - h;
            if (ex > 0.0) lb = lb + ex * ex;
        }
        return lb;
    };
    // grouped positions m0 .. m1 - 1 of box e for the reference points in
    // mask (bit u); X_j^* coordinates are read from their contiguous per-node
    // copy (grouped by child), each with its position in X_j^* (the grouped
    // order of a leaf's X_j^* is its own: ID = true reads no positions)
    auto scan_range = [&](auto id_order, int e, int m0, int m1, unsigned mask) {
        constexpr bool ID = decltype(id_order)::value;
        const double* xj = xs_pts + (int64_t)bj[e] * D * r1;
        const int* pj = xs_pos + (int64_t)bj[e] * r1;
        const int pos0 = np_ + boff[e];
        int m = m0;
        for (; m + PB <= m1; m += PB) {
            double cx[PB][D];
            int pz[PB];
#pragma unroll
            for (int z = 0; z < PB; ++z) {
#pragma unroll
                for (int a = 0; a < D; ++a) cx[z][a] = xj[a * r1 + m + z];
                pz[z] = pos0 + (ID ? m + z : pj[m + z]);
            }
#pragma unroll
            for (int u = 0; u < QPT; ++u)
                if (mask & (1u << u))
#pragma unroll
                    for (int z = 0; z < PB; ++z) consider(u, dist(u, cx[z]), pz[z]);
        }
        for (; m < m1; ++m) {
            double cx[D];
#pragma unroll
            for (int a = 0; a < D; ++a) cx[a] = xj[a * r1 + m];
            const int pz = pos0 + (ID ? m : pj[m]);
#pragma unroll
            for (int u = 0; u < QPT; ++u)
                if (mask & (1u << u)) consider(u, dist(u, cx), pz);
        }
    };
    // each reference point's nearest box first (it prunes best), then every
    // box its bound admits
    int e_first[QPT];
    double lb_first[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        e_first[u] = -1;
        lb_first[u] = INFINITY;
    }
    for (int e = 0; e < ne; ++e) {
        double bc[D];
#pragma unroll
        for (int a = 0; a < D; ++a) bc[a] = (double)bx[a][e];
        const double h = (double)bh[e];
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const double lb = box_lb(u, bc, h);
            if (lb < lb_first[u]) {
                lb_first[u] = lb;
                e_first[u] = e;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < QPT; ++u)
        if (act[u] && e_first[u] >= 0 && lb_first[u] * (1.0 - 1e-12) <= best[u])
            scan_range(std::false_type(), e_first[u], 0, bcnt[e_first[u]], 1u << u);
    // Y_p^*, run by run where staged (a run whose box bound exceeds a
    // reference point's best distance cannot hold its nearest point)
    auto scan_y = [&](int c0, int c1, unsigned mask) {
        for (int c = c0; c < c1; ++c) {
            double cy[D];
#pragma unroll
            for (int a = 0; a < D; ++a) cy[a] = stage_y ? yc[a][c] : pts[a * ld + yp[c]];
#pragma unroll
            for (int u = 0; u < QPT; ++u)
                if (mask & (1u << u)) consider(u, dist(u, cy), c);
        }
    };
    if (!stage_y) {
        unsigned am = 0;
#pragma unroll
        for (int u = 0; u < QPT; ++u)
            if (act[u]) am |= 1u << u;
        scan_y(0, np_, am);
    }
    for (int ch = 0; ch < nych; ++ch) {
        unsigned mask = 0;
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            double lb = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double ex = fmax((double)ylo[a][ch] - qv[u][a], qv[u][a] - (double)yhi[a][ch]);
                if (ex > 0.0) lb = lb + ex * ex;
            }
            if (act[u] && lb * (1.0 - 1e-12) <= best[u]) mask |= 1u << u;
        }
        if (mask) scan_y(ch * YCH, min(np_, ch * YCH + YCH), mask);
    }
    for (int e = 0; e < ne; ++e) {
        double bc[D];
#pragma unroll
        for (int a = 0; a < D; ++a) bc[a] = (double)bx[a][e];
        const double h = (double)bh[e];
        unsigned mask = 0;
#pragma unroll
        for (int u = 0; u < QPT; ++u)
            if (act[u] && e != e_first[u] && box_lb(u, bc, h) * (1.0 - 1e-12) <= best[u]) mask |= 1u << u;
        if (!mask) continue;
        // an admitted box with more than SPLIT_MIN candidates is searched
        // child by child: the points of X_j^* in child c lie in c's box (its
        // half side padded by 1e-13 of its extent for the rounding of the
        // tree's centres), whose distance bounds them from below in the same
        // way
        const int j = bj[e];
        const int nc = nchild[j];
        if (nc == 0) {
            scan_range(std::true_type(), e, 0, bcnt[e], mask);
            continue;
        }
        if (bcnt[e] <= SPLIT_MIN) {
            scan_range(std::false_type(), e, 0, bcnt[e], mask);
            continue;
        }
        const int* co = xs_coff + (int64_t)j * NCO;
        const int fc = first_child[j];
        for (int kc = 0; kc < nc; ++kc) {
            const int m0 = co[kc], m1 = co[kc + 1];
            if (m0 == m1) continue;
            double cc[D];
            double cm = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                cc[a] = center[(int64_t)(fc + kc) * D + a];
                cm = fmax(cm, fabs(cc[a]));
            }
            const double sc = side[fc + kc];
            const double hc = 0.5 * sc + 1e-13 * (cm + sc);
            unsigned cmask = 0;
#pragma unroll
            for (int u = 0; u < QPT; ++u)
                if ((mask & (1u << u)) && box_lb(u, cc, hc) * (1.0 - 1e-12) <= best[u]) cmask |= 1u << u;
            if (cmask) scan_range(std::false_type(), e, m0, m1, cmask);
        }
    }
    __syncthreads();  // every lane is done with Y_p^* (keys and picks reuse it)
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        if (!act[u]) continue;
        const int t = threadIdx.x + u * NTH;
        int bidx;
        if (bpos[u] < np_) {
            bidx = yp[bpos[u]];
        } else {
            const int qq = bpos[u] - np_;
            const int e = seg_of(boff, ne, qq);
            bidx = xs_idx[(int64_t)bj[e] * r1 + (qq - boff[e])];
        }
        pick[t] = bidx;
        keys[t] = ((long long)bidx << 13) | t;
    }
    int P = 1;
    while (P < nq) P <<= 1;
    for (int t = nq + threadIdx.x; t < P; t += NTH) keys[t] = 0x7fffffffffffffffLL;
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int x = threadIdx.x; x < P; x += NTH) {
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
    for (int x = threadIdx.x; x < nq; x += NTH) {
        bool first = x == 0 || (keys[x - 1] >> 13) != (keys[x] >> 13);
        int t = (int)(keys[x] & 8191);
        if (!first) pick[t] = -1;
    }
    __syncthreads();
    const int per = (nq + NTH - 1) / NTH;
    const int t0 = threadIdx.x * per;
    int c = 0;
    for (int t = t0; t < min(nq, t0 + per); ++t) c += pick[t] >= 0;
    scan_sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < NTH; off <<= 1) {
        int a = (int)threadIdx.x >= off ? scan_sh[threadIdx.x - off] : 0;
        __syncthreads();
        scan_sh[threadIdx.x] += a;
        __syncthreads();
    }
    int w = scan_sh[threadIdx.x] - c;
    for (int t = t0; t < min(nq, t0 + per); ++t)
        if (pick[t] >= 0) o[w++] = pick[t];
    if (threadIdx.x == NTH - 1) ys_cnt[i] = scan_sh[NTH - 1];
}

// ---- T_i = Y_p^* ++ X_j^* (j in IL(i)) materialised for the nodes with long
// interaction lists; split = |Y_p^*| marks the two parts
__global__ __launch_bounds__(TB) void k_down_sizes(int nl, const int* __restrict__ nodes, const int* __restrict__ parent,
                                                   const int* __restrict__ il_ptr, const int* __restrict__ il_col,
                                                   const int* __restrict__ xs_cnt, const int* __restrict__ ys_cnt,
                                                   int64_t* __restrict__ sz, int* __restrict__ split)
{
    int t = blockIdx.x * TB + threadIdx.x;
    if (t >= nl) return;
    const int i = nodes[t], p = parent[i];
    const int np_ = p > 0 ? ys_cnt[p] : 0;
    int64_t v = np_;
    for (int e = il_ptr[i]; e < il_ptr[i + 1]; ++e) v += xs_cnt[il_col[e]];
    sz[t] = v;
    split[t] = np_;
}

__global__ __launch_bounds__(TB) void k_down_fill(const int* __restrict__ nodes, const int* __restrict__ parent,
                                                  const int* __restrict__ il_ptr, const int* __restrict__ il_col,
                                                  const int* __restrict__ xs_cnt, const int* __restrict__ xs_idx,
                                                  int r1, const int* __restrict__ ys_cnt,
                                                  const int* __restrict__ ys_idx, int ys_stride,
                                                  const int64_t* __restrict__ off, int* __restrict__ list)
{
    const int t = blockIdx.x;
    const int i = nodes[t], p = parent[i];
    int* o = list + off[t];
    int64_t w = 0;
    if (p > 0) {
        const int np_ = ys_cnt[p];
        for (int q = threadIdx.x; q < np_; q += TB) o[q] = ys_idx[(int64_t)p * ys_stride + q];
        w = np_;
    }
    for (int e = il_ptr[i]; e < il_ptr[i + 1]; ++e) {
        const int j = il_col[e], c = xs_cnt[j];
        for (int q = threadIdx.x; q < c; q += TB) o[w + q] = xs_idx[(int64_t)j * r1 + q];
        w += c;
    }
}

__global__ __launch_bounds__(TB) void k_rows_scatter(const int* __restrict__ nodes, const int* __restrict__ cnt,
                                                     const int* __restrict__ src, int stride, int* __restrict__ dst_cnt,
                                                     int* __restrict__ dst)
{
    const int t = blockIdx.x, i = nodes[t], c = cnt[t];
    for (int q = threadIdx.x; q < c; q += TB) dst[(int64_t)i * stride + q] = src[(int64_t)t * stride + q];
    if (threadIdx.x == 0) dst_cnt[i] = c;
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

// Levels with fewer than h.down_wide_nodes nodes run 1024 lanes per node (one
// reference point per lane): the 4x more wavefronts hide the latency of the
// searches where a level has too few nodes to fill the CUs.  The result does
// not depend on the workgroup size.

// the grouped copy of every node's X_i^* (k_xs_grouped)
struct XsGrouped {
    const double* pts;
    const int* pos;
    const int* coff;
    const double* dirs;  // the surface method's directions (mdir of them)
    int mdir;
};

template <int D, int MAXQ, int NTH>
void launch_down_k(Handle& h, int lo, int nl, const XsGrouped& xg, hipStream_t s)
{
    const unsigned grid = 8u * (unsigned)((nl + 7) / 8);
    k_datareduct_down<D, MAXQ, NTH><<<grid, NTH, 0, s>>>(lo, h.pts.p, h.n, h.parent.p, h.il_ptr.p, h.il_col.p,
                                                         h.center.p, h.side.p, h.xs_cnt.p, h.xs_idx.p, xg.pts,
                                                         xg.pos, xg.coff, h.nchild.p, h.first_child.p, h.r1,
                                                         h.ys_cnt.p, h.ys_idx.p, h.ys_stride, h.r2, nl, h.dr, xg.dirs,
                                                         xg.mdir);
}

template <int D>
void launch_down_d(Handle& h, int lo, int nl, const XsGrouped& xg, hipStream_t s)
{
    if (h.r2 > 1024)
        launch_down_k<D, MAXQ_ALL, TB>(h, lo, nl, xg, s);
    else if (nl < h.down_wide_nodes)
        launch_down_k<D, 1024, 1024>(h, lo, nl, xg, s);
    else
        launch_down_k<D, 1024, TB>(h, lo, nl, xg, s);
}

void launch_down(Handle& h, int lo, int nl, const XsGrouped& xg, hipStream_t s)
{
    if (h.d == 1)
        launch_down_d<1>(h, lo, nl, xg, s);
    else if (h.d == 2)
        launch_down_d<2>(h, lo, nl, xg, s);
    else
        launch_down_d<3>(h, lo, nl, xg, s);
}

// |T_i| for the nodes the top-down kernel reduces (interaction lists of at
// most ILCAP entries; 0 for the others), and the squared distances the
// definition of DataReduct evaluates for them (every reference point against
// every candidate: |T_i| times gd points per non-empty part when |T_i| > k),
// for the profile; gd is the grid size of one part.
__global__ __launch_bounds__(TB) void k_down_len(int nn, const int* __restrict__ parent, const int* __restrict__ il_ptr,
                                                 const int* __restrict__ il_col, const int* __restrict__ xs_cnt,
                                                 const int* __restrict__ ys_cnt, int k, int gd,
                                                 int64_t* __restrict__ len, int64_t* __restrict__ evals)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= nn) return;
    const int e0 = il_ptr[i], ne = il_ptr[i + 1] - e0;
    int64_t l = 0, lp = 0;
    if (i > 0 && ne <= ILCAP) {
        lp = parent[i] > 0 ? ys_cnt[parent[i]] : 0;
        l = lp;
        for (int e = 0; e < ne; ++e) l += xs_cnt[il_col[e0 + e]];
    }
    len[i] = l;
    const int nseg = (lp > 0) + (l > lp);
    evals[i] = l > k ? l * nseg * gd : 0;
}

// Coordinates of every node's X_i^* in a contiguous copy grouped by the child
// of i whose point range holds each point (a leaf: one group), in order of
// position within a group: xs_pts[(i * d + a) * r1 + m'] is coordinate a of
// the point at grouped position m', xs_pos[i * r1 + m'] its position in
// X_i^*, and grouped positions xs_coff[i * NCO + k] .. xs_coff[i * NCO + k + 1]
// - 1 belong to child k.
__global__ __launch_bounds__(TB) void k_xs_grouped(const double* __restrict__ pts, int64_t ld, int d,
                                                   const int* __restrict__ xs_cnt, const int* __restrict__ xs_idx,
                                                   int r1, const int* __restrict__ nchild,
                                                   const int* __restrict__ first_child, const int* __restrict__ start,
                                                   const int* __restrict__ count, double* __restrict__ xs_pts,
                                                   int* __restrict__ xs_pos, int* __restrict__ xs_coff)
{
    __shared__ unsigned char grp[MAXR1];
    __shared__ int gcnt[NCO];
    const int i = blockIdx.x;
    const int c = xs_cnt[i];
    const int nc = nchild[i], fc = first_child[i];
    const int ng = nc > 0 ? nc : 1;
    for (int m = threadIdx.x; m < c; m += TB) {
        int g = 0;
        if (nc > 0) {
            const int id = xs_idx[(int64_t)i * r1 + m];
            for (int k = 0; k < nc; ++k)
                if (id >= start[fc + k] && id < start[fc + k] + count[fc + k]) g = k;
        }
        grp[m] = (unsigned char)g;
    }
    __syncthreads();
    if ((int)threadIdx.x < ng) {
        int w = 0;
        for (int m = 0; m < c; ++m) w += grp[m] == (int)threadIdx.x;
        gcnt[threadIdx.x] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int w = 0;
        for (int k = 0; k < ng; ++k) {
            xs_coff[(int64_t)i * NCO + k] = w;
            w += gcnt[k];
        }
        xs_coff[(int64_t)i * NCO + ng] = w;
    }
    for (int m = threadIdx.x; m < c; m += TB) {
        const int g = grp[m];
        int w = 0;
        for (int k = 0; k < g; ++k) w += gcnt[k];
        for (int q = 0; q < m; ++q) w += grp[q] == g;
        const int id = xs_idx[(int64_t)i * r1 + m];
        xs_pos[(int64_t)i * r1 + w] = m;
        for (int a = 0; a < d; ++a) xs_pts[((int64_t)i * d + a) * r1 + w] = pts[a * ld + id];
    }
}

}  // namespace

void datareduct_lists(const double* pts, int64_t ld, int d, const int64_t* list_off, const int* list_idx,
                      const int* split, int nlist, int k, int* out, int out_stride, int* out_cnt, hipStream_t s)
{
    datareduct_lists_method(H2_DR_VOLUME, pts, ld, d, list_off, list_idx, split, nlist, k, out, out_stride, out_cnt,
                            s);
}

// Unit direction j of m on the reference surfaces of the surface method
// (3-D: the golden-angle spiral z = 1 - (2j+1)/m, rho = sqrt(1 - z^2),
// phi = j pi (3 - sqrt 5); 2-D: the angles 2 pi (j + 1/2) / m; 1-D: -1, +1).
static void surface_dirs(int d, int m, std::vector<double>& u)
{
    const double pi = 3.14159265358979323846;
    u.assign((size_t)m * d, 0.0);
    for (int j = 0; j < m; ++j) {
        double* v = u.data() + (size_t)j * d;
        if (d == 1) {
            v[0] = j == 0 ? -1.0 : 1.0;
        } else if (d == 2) {
            const double th = 2.0 * pi * ((double)j + 0.5) / (double)m;
            v[0] = std::cos(th);
            v[1] = std::sin(th);
        } else {
            const double z = 1.0 - (double)(2 * j + 1) / (double)m;
            const double rho = std::sqrt(1.0 - z * z);
            const double phi = (double)j * (pi * (3.0 - std::sqrt(5.0)));
            v[0] = rho * std::cos(phi);
            v[1] = rho * std::sin(phi);
            v[2] = z;
        }
    }
}

void datareduct_lists_method(int method, const double* pts, int64_t ld, int d, const int64_t* list_off,
                             const int* list_idx, const int* split, int nlist, int k, int* out, int out_stride,
                             int* out_cnt, hipStream_t s)
{
    if (nlist <= 0) return;
    if (k < 1 || k > MAXQ_ALL) fail(H2_EUNSUPPORTED, "DataReduct size must be in [1, 4096]");
    if (method == H2_DR_FPS) {
        const int64_t tot = read_scalar(list_off + nlist, s);
        if (tot > (int64_t)INT32_MAX) fail(H2_EUNSUPPORTED, "lists longer than 2^31 entries");
        DBuf<double> md, cw;
        md.ensure((size_t)std::max<int64_t>(tot, 1), s);
        cw.ensure((size_t)std::max<int64_t>(tot, 1) * d, s);
        if (tot > 0) {
            k_list_coords<<<blocks_for(tot, TB), TB, 0, s>>>(pts, ld, d, list_idx, tot, cw.p);
            H2_LAUNCH_CHECK();
        }
        k_datareduct_fps<<<nlist, TB, 0, s>>>(cw.p, tot, d, list_off, list_idx, k, out, out_stride, out_cnt, md.p);
        H2_LAUNCH_CHECK();
        H2_HIP(hipStreamSynchronize(s));
        return;
    }
    DBuf<double> dirs;
    int mdir = 0;
    if (method == H2_DR_SURFACE) {
        const int kp = split ? std::max(1, k / 2) : k;
        mdir = std::max(1, kp / 3);
        if (d == 1) mdir = std::min(mdir, 2);
        std::vector<double> u;
        surface_dirs(d, mdir, u);
        dirs.ensure(u.size(), s);
        H2_HIP(hipMemcpyAsync(dirs.p, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (k <= 1024)
        k_datareduct<1024><<<nlist, TB, 0, s>>>(pts, ld, d, list_off, list_idx, split, k, out, out_stride, out_cnt,
                                                method, dirs.p, mdir);
    else
        k_datareduct<MAXQ_ALL><<<nlist, TB, 0, s>>>(pts, ld, d, list_off, list_idx, split, k, out, out_stride,
                                                    out_cnt, method, dirs.p, mdir);
    H2_LAUNCH_CHECK();
    if (method == H2_DR_SURFACE) H2_HIP(hipStreamSynchronize(s));  // the direction table's lifetime
}

void run_hidr(Handle& h)
{
    hipStream_t s = h.stream;
    const int nn = h.nnode;
    h.xs_cnt.ensure((size_t)nn, s);
    h.ys_cnt.ensure((size_t)nn, s);
    h.xs_idx.ensure((size_t)nn * h.r1, s);
    h.ys_stride = h.r2;
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
        datareduct_lists_method(h.dr, h.pts.p, h.n, h.d, off.p, list.p, nullptr, nl, h.r1,
                                h.xs_idx.p + (int64_t)lo * h.r1, h.r1, h.xs_cnt.p + lo, s);
    }
    if (h.r2 < 2 || h.r2 > MAXQ_ALL) fail(H2_EUNSUPPORTED, "r2 must be in [2, 4096]");
    DBuf<double> xs_pts;
    DBuf<int> xs_pos, xs_coff;
    xs_pts.ensure((size_t)nn * h.d * h.r1, s);
    xs_pos.ensure((size_t)nn * h.r1, s);
    xs_coff.ensure((size_t)nn * NCO, s);
    k_xs_grouped<<<nn, TB, 0, s>>>(h.pts.p, h.n, h.d, h.xs_cnt.p, h.xs_idx.p, h.r1, h.nchild.p, h.first_child.p,
                                   h.start.p, h.count.p, xs_pts.p, xs_pos.p, xs_coff.p);
    // the surface method's directions, as datareduct_lists_method forms them
    // for a two-part T_i
    DBuf<double> dirs;
    std::vector<double> dir_h;
    int mdir = 0;
    if (h.dr == H2_DR_SURFACE) {
        mdir = std::max(1, std::max(1, h.r2 / 2) / 3);
        if (h.d == 1) mdir = std::min(mdir, 2);
        surface_dirs(h.d, mdir, dir_h);
        dirs.ensure(dir_h.size(), s);
        H2_HIP(hipMemcpyAsync(dirs.p, dir_h.data(), dir_h.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    const XsGrouped xg{xs_pts.p, xs_pos.p, xs_coff.p, dirs.p, mdir};
    H2_LAUNCH_CHECK();
    DBuf<int> lnodes, split, tmp, tmp_cnt;
    std::vector<hipEvent_t> ev;  // around each level's launch (profile)
    if (h.profile) {
        ev.resize(2 * (size_t)(h.maxdepth + 1));
        for (auto& e : ev) H2_HIP(hipEventCreate(&e));
    }
    for (int L = 1; L <= h.maxdepth; ++L) {
        int lo = h.lvl_ptr[L], nl = h.lvl_ptr[L + 1] - lo;
        if (h.profile) H2_HIP(hipEventRecord(ev[2 * L], s));
        // the box-pruned kernel serves the volume and surface methods; FPS
        // reduces every node's materialised T_i
        const bool pruned = h.dr == H2_DR_VOLUME || h.dr == H2_DR_SURFACE;
        if (pruned) launch_down(h, lo, nl, xg, s);
        if (h.profile) H2_HIP(hipEventRecord(ev[2 * L + 1], s));
        H2_LAUNCH_CHECK();
        std::vector<int> longn;
        for (int i = lo; i < lo + nl; ++i)
            if (!pruned || h.h_il_ptr[i + 1] - h.h_il_ptr[i] > ILCAP) longn.push_back(i);
        if (longn.empty()) continue;
        const int nlong = (int)longn.size();
        lnodes.ensure((size_t)nlong, s);
        H2_HIP(hipMemcpyAsync(lnodes.p, longn.data(), sizeof(int) * nlong, hipMemcpyHostToDevice, s));
        sz.ensure((size_t)nlong, s);
        off.ensure((size_t)nlong + 1, s);
        split.ensure((size_t)nlong, s);
        k_down_sizes<<<blocks_for(nlong, TB), TB, 0, s>>>(nlong, lnodes.p, h.parent.p, h.il_ptr.p, h.il_col.p,
                                                          h.xs_cnt.p, h.ys_cnt.p, sz.p, split.p);
        H2_LAUNCH_CHECK();
        scan_excl_i64(sz.p, off.p, nlong, h.tmp_i64, s);
        int64_t tot = read_scalar(off.p + nlong, s);
        list.ensure((size_t)std::max<int64_t>(tot, 1), s);
        k_down_fill<<<nlong, TB, 0, s>>>(lnodes.p, h.parent.p, h.il_ptr.p, h.il_col.p, h.xs_cnt.p, h.xs_idx.p, h.r1,
                                         h.ys_cnt.p, h.ys_idx.p, h.ys_stride, off.p, list.p);
        H2_LAUNCH_CHECK();
        tmp.ensure((size_t)nlong * h.ys_stride, s);
        tmp_cnt.ensure((size_t)nlong, s);
        datareduct_lists_method(h.dr, h.pts.p, h.n, h.d, off.p, list.p, split.p, nlong, h.r2, tmp.p, h.ys_stride,
                                tmp_cnt.p, s);
        k_rows_scatter<<<nlong, TB, 0, s>>>(lnodes.p, tmp_cnt.p, tmp.p, h.ys_stride, h.ys_cnt.p, h.ys_idx.p);
        H2_LAUNCH_CHECK();
    }
    h.hidr_down_ms = h.hidr_down_bytes = h.hidr_down_evals = 0;
    if (h.profile && h.dr == H2_DR_VOLUME) {
        // candidate bytes of the nodes the top-down kernel reduced:
        // |T_i| = |Y_p^*| + sum over IL(i) of |X_j^*| coordinates of d doubles
        int g = 1;
        for (;;) {
            long long nx = 1;
            for (int a = 0; a < h.d; ++a) nx *= g + 1;
            if (nx > h.r2 / 2) break;
            ++g;
        }
        int gd = 1;
        for (int a = 0; a < h.d; ++a) gd *= g;
        DBuf<int64_t> len, ev_n;
        len.ensure((size_t)nn, s);
        ev_n.ensure((size_t)nn, s);
        k_down_len<<<blocks_for(nn, TB), TB, 0, s>>>(nn, h.parent.p, h.il_ptr.p, h.il_col.p, h.xs_cnt.p, h.ys_cnt.p,
                                                     h.r2, gd, len.p, ev_n.p);
        H2_LAUNCH_CHECK();
        std::vector<int64_t> hl((size_t)nn), he((size_t)nn);
        H2_HIP(hipMemcpyAsync(hl.data(), len.p, sizeof(int64_t) * nn, hipMemcpyDeviceToHost, s));
        H2_HIP(hipMemcpyAsync(he.data(), ev_n.p, sizeof(int64_t) * nn, hipMemcpyDeviceToHost, s));
        H2_HIP(hipStreamSynchronize(s));
        double tot = 0, tev = 0;
        for (int64_t v : hl) tot += (double)v;
        for (int64_t v : he) tev += (double)v;
        h.hidr_down_bytes = tot * h.d * sizeof(double);
        h.hidr_down_evals = tev;
        h.hidr_down_ms = 0;
        for (int L = 1; L <= h.maxdepth; ++L) {
            float ms = 0.f;
            H2_HIP(hipEventElapsedTime(&ms, ev[2 * L], ev[2 * L + 1]));
            h.hidr_down_ms += ms;
        }
    }
    H2_HIP(hipStreamSynchronize(s));
    for (auto& e : ev) H2_HIP(hipEventDestroy(e));
}

}  // namespace h2
