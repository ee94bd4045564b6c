// getBasis (Section 4.1, Eqs. SRRQR1-2) as a batched interpolative
// decomposition, and the bottom-up nested-basis pass of Algorithm 2.
//
// For node i the rows of A = kappa(Xbar_i, Y_i^*) are the candidate points and
// the columns the farfield representor points.  Householder QR with column
// pivoting runs on M = A^T (s x m, stored row-major so that a wavefront reads
// 64 consecutive columns of one row), and with M P = Q [R11 R12; 0 R22] the
// interpolation matrix is T = R11^{-1} R12, U_i = P [I; T^T], and the
// skeleton Xhat_i is the first k pivoted rows.
//
// Rules (identical to the oracle's): pivot = lowest index whose partial norm
// is within a factor (1 - 2^-40) of the largest; norms down-dated with the
// LAWN 176 safeguard (recompute once a down-date has lost half the digits);
// stop before step j when |R_jj| <= tol |R_00| for the column it would pivot
// in, leaving the columns in place (or j = min(s, m)).
//
// One workgroup per node; lane c owns columns c, c+256, ...  Each lane runs
// its columns' dot products, updates and squared tail sums sequentially in row
// order, and the tail sum doubles as the next |R_jj|^2 and as the down-date
// recomputation.  With the reflector norm in closed form this reproduces the
// oracle's operation order exactly, so pivots, ranks and T agree bit for bit
// whenever the kernel entries do.  Compiled with -ffp-contract=off.
#include <type_traits>

#include <algorithm>

#include "common.h"
#include "kappa.h"

namespace h2 {
namespace {

constexpr int TB = 256;

__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int wave_min_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
template <int NT>
__device__ inline double block_max(double v, double* sh)
{
    v = wave_max(v);
    if (NT == 64) return v;
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < NT / 64; ++q) r = fmax(r, sh[q]);
    __syncthreads();
    return r;
}
template <int NT>
__device__ inline int block_min_i(int v, int* sh)
{
    v = wave_min_i(v);
    if (NT == 64) return v;
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    int r = sh[0];
    for (int q = 1; q < NT / 64; ++q) r = min(r, sh[q]);
    __syncthreads();
    return r;
}


// Device buffers reached through pointers loaded from memory would be
// accessed with flat instructions, which also count against the LDS wait
// counter: a wait for an LDS value would then drain every global load in
// flight.  Global buffers are therefore addressed through the global address
// space.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) int gint;
template <class ET>
using gptr = __attribute__((address_space(1))) ET*;

// Kernel entries of the interpolative decompositions: FP64 correctly rounded
// (compared with the oracle bit for bit), or, for the precision mode's FP32
// decompositions, the kernel function evaluated in FP32.
template <class ET, int FAM>
__device__ __forceinline__ ET kappa_id(int kid, double prm, double r2, double xy, double d0)
{
    if constexpr (std::is_same_v<ET, float>)
        return kappa_store<float, FAM>(kid, prm, r2, xy, d0);
    else
        return kappa_fam<FAM>(kid, prm, r2, xy, d0);
}

// Barrier that orders LDS accesses only: global loads and stores of a lane
// stay in flight across it.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sequential row loops of one column (x: LDS or gdouble pointer) with the
// loads issued ahead: batches of LB rows, the next batch in flight while the
// current one is used.  The arithmetic runs in exactly the order of a plain
// loop (so the result is the oracle's, bit for bit); only the memory latency
// overlaps.
constexpr int LB = 8;

// A norm down-date is trusted while the squared remainder it leaves is
// above the square root of the matrix type's machine epsilon (LAWN 176);
// FP32 data makes it unreliable far earlier than FP64 data.
template <class ET>
__device__ __forceinline__ double down_tol()
{
    return std::is_same_v<ET, float> ? 3.4526698300124393e-04 /* sqrt(2^-23) */
                                     : sqrt(2.220446049250313e-16);
}

__device__ __forceinline__ double fma_e(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_e(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// acc + sum_{r=r0}^{r1-1} a[r] * x[r*ld], accumulated in row order in the
// type of a (FP64, or FP32 in the precision mode's decompositions)
template <int BATCH = LB, class AT, class XP>
__device__ __forceinline__ AT dot_rows(const AT* __restrict__ a, XP x, int64_t ld, int r0, int r1, AT acc)
{
    int r = r0;
    if (r + BATCH <= r1) {
        AT cur[BATCH];
#pragma unroll
        for (int q = 0; q < BATCH; ++q) cur[q] = x[(int64_t)(r + q) * ld];
        for (; r + 2 * BATCH <= r1; r += BATCH) {
            AT nxt[BATCH];
#pragma unroll
            for (int q = 0; q < BATCH; ++q) nxt[q] = x[(int64_t)(r + BATCH + q) * ld];
#pragma unroll
            for (int q = 0; q < BATCH; ++q) acc = acc + a[r + q] * cur[q];
#pragma unroll
            for (int q = 0; q < BATCH; ++q) cur[q] = nxt[q];
        }
#pragma unroll
        for (int q = 0; q < BATCH; ++q) acc = acc + a[r + q] * cur[q];
        r += BATCH;
    }
    for (; r < r1; ++r) acc = acc + a[r] * x[(int64_t)r * ld];
    return acc;
}

// acc + sum_{r=r0}^{r1-1} x[r*ld]^2, in row order, in FP64
template <class XP>
__device__ __forceinline__ double sumsq_rows(XP x, int64_t ld, int r0, int r1, double acc)
{
    int r = r0;
    if (r + LB <= r1) {
        double cur[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) cur[q] = x[(int64_t)(r + q) * ld];
        for (; r + 2 * LB <= r1; r += LB) {
            double nxt[LB];
#pragma unroll
            for (int q = 0; q < LB; ++q) nxt[q] = x[(int64_t)(r + LB + q) * ld];
#pragma unroll
            for (int q = 0; q < LB; ++q) acc = acc + cur[q] * cur[q];
#pragma unroll
            for (int q = 0; q < LB; ++q) cur[q] = nxt[q];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) acc = acc + cur[q] * cur[q];
        r += LB;
    }
    for (; r < r1; ++r) acc = acc + x[(int64_t)r * ld] * x[(int64_t)r * ld];
    return acc;
}

// x[r] <- x[r] - f v[r] for r in [r0, r1) in the type of v; returns the sum
// of the new x[r]^2 over r in [r0+1, r1) in row order, in FP64 (the next
// step's tail norm)
template <class AT, class XP>
__device__ __forceinline__ double axpy_rows(const AT* __restrict__ v, AT f, XP x, int64_t ld, int r0, int r1)
{
    {
        AT y = x[(int64_t)r0 * ld] - f * v[r0];
        x[(int64_t)r0 * ld] = y;
    }
    double tail = 0.0;
    int r = r0 + 1;
    if (r + LB <= r1) {
        AT cur[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) cur[q] = x[(int64_t)(r + q) * ld];
        for (; r + 2 * LB <= r1; r += LB) {
            AT nxt[LB];
#pragma unroll
            for (int q = 0; q < LB; ++q) nxt[q] = x[(int64_t)(r + LB + q) * ld];
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                AT y = cur[q] - f * v[r + q];
                x[(int64_t)(r + q) * ld] = y;
                tail = tail + (double)y * (double)y;
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) cur[q] = nxt[q];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            AT y = cur[q] - f * v[r + q];
            x[(int64_t)(r + q) * ld] = y;
            tail = tail + (double)y * (double)y;
        }
        r += LB;
    }
    for (; r < r1; ++r) {
        AT y = x[(int64_t)r * ld] - f * v[r];
        x[(int64_t)r * ld] = y;
        tail = tail + (double)y * (double)y;
    }
    return tail;
}

// Coordinates of a lane's columns (c = lane + nt t) for the block
// evaluation: held in registers when the lane owns one column, otherwise
// read from global memory at each use.
template <int CPL>
struct XCoords {
    const gdouble* p;
    int64_t ld;
    int idx[CPL];
    __device__ XCoords(const double* pts, int64_t ld_, const int* xi, int lane, int nt, int m, int d) : ld(ld_)
    {
        (void)d;
        p = (const gdouble*)pts;
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = lane + t * nt;
            idx[t] = c < m ? xi[c] : 0;
        }
    }
    __device__ double get(int t, int a) const { return p[a * ld + idx[t]]; }
};
template <>
struct XCoords<1> {
    double x[3];
    __device__ XCoords(const double* pts, int64_t ld, const int* xi, int lane, int nt, int m, int d)
    {
        (void)nt;
        const int c = lane;
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = (c < m && a < d) ? pts[a * ld + xi[c]] : 0.0;
    }
    // selects instead of an index, so that x stays in registers
    __device__ double get(int, int a) const { return a == 0 ? x[0] : (a == 1 ? x[1] : x[2]); }
};

// Compression of a tall block (TSQR): the s x m block is streamed in blocks
// of BR rows and folded into the m x m upper triangle R (LDS or global) by
// Householder reflectors that each zero one column of the block against the
// diagonal entry of R.  Lane l owns columns l, l + NT, ... (CPL of them) and
// keeps their BR block entries in registers, evaluating them itself; the
// column that step j eliminates, its squared norm and the diagonal entry
// R[j][j] are published in a double-buffered LDS slot by the column's owner
// at the end of step j - 1, so one barrier per step suffices.  The R entries
// of the next row are loaded a step ahead.  (This part accumulates with fused
// multiply-adds; it is not the oracle's operation order, and need not be:
// pivots and T are fixed up to rounding.)  R is an LDS pointer or a gdouble
// pointer.  Every R entry is read and written by the lane that owns its
// column only (the diagonal entry reaches the other lanes through LDS), so
// the steps need LDS barriers only.
template <int NT, int CPL, int BR, int FAM, class ET, class RPtr>
__device__ void tsqr_fold(const IdTask& tk, int m, int s0, RPtr R, double* colbuf_d, double* nubuf_d, double* scr_d)
{
    // ET buffers at the places of the FP64 ones (an FP32 fold uses half)
    ET* colbuf = (ET*)colbuf_d;
    ET* nubuf = (ET*)nubuf_d;
    ET* x0buf = (ET*)(nubuf_d + 2);
    ET* scr = (ET*)scr_d;
    const double* pts = tk.pts;
    const int64_t ld = tk.ld;
    const int* xi = tk.x_idx;
    const int* yi = tk.y_idx;
    const int d = tk.d, kid = tk.kid;
    const double prm = tk.prm;
    const double dsgn = tk.swap ? -1.0 : 1.0;  // column side: kappa(y, x)
    const int lane = threadIdx.x;
    constexpr int SL = 8;              // rows per evaluation slice
    static_assert(BR % SL == 0, "row block");
    double* ycrd = scr_d + SL * NT;  // 3 x BR: the row block's points
    for (int64_t e = lane; e < (int64_t)m * m; e += NT) R[e] = 0.0;
    // this lane's column points: in registers for one column per lane,
    // otherwise read where needed (L1 hits; registers kept for occupancy)
    XCoords<CPL> xr(pts, ld, xi, lane, NT, m, d);
    __syncthreads();
    ET bc[CPL][BR];
    // squared norm of a column's block part, in row order (formed by the
    // column's owner when it publishes the column)
    auto sumsq = [](const ET* b) {
        ET ts = ET(0);
#pragma unroll
        for (int r = 0; r < BR; ++r) ts = fma_e(b[r], b[r], ts);
        return ts;
    };
    for (int r0 = 0; r0 < s0; r0 += BR) {
        const int nb = min(BR, s0 - r0);
        // the row block's points, staged once in LDS for all lanes
        if (lane < nb)
            for (int a = 0; a < d; ++a) ycrd[a * BR + lane] = pts[a * ld + yi[r0 + lane]];
        lds_barrier();
        // this lane's block entries (evaluated SL rows at a time through a
        // lane-private LDS slice, scr[r * NT + lane]; squared distances
        // accumulated in coordinate order as dist2 does)
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = lane + t * NT;
#pragma unroll
            for (int k0 = 0; k0 < BR; k0 += SL) {
                if (c < m)
                    for (int r = 0; r < SL && k0 + r < nb; ++r) {
                        double r2 = 0.0, xy = 0.0, e0 = 0.0;
                        if constexpr (FAM == FAM_COSINE)
                            for (int a = 0; a < d; ++a) xy = xy + xr.get(t, a) * ycrd[a * BR + k0 + r];
                        else
                            for (int a = 0; a < d; ++a) {
                                const double ea = xr.get(t, a) - ycrd[a * BR + k0 + r];
                                if (a == 0) e0 = ea;
                                r2 = r2 + ea * ea;
                            }
                        scr[r * NT + lane] = kappa_id<ET, FAM>(kid, prm, r2, xy, dsgn * e0);
                    }
#pragma unroll
                for (int r = 0; r < SL; ++r) bc[t][k0 + r] = (c < m && k0 + r < nb) ? scr[r * NT + lane] : ET(0);
            }
        }
        ET rn[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = lane + t * NT;
            rn[t] = c < m ? R[c] : ET(0);
        }
        // publish column 0
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < BR; ++r) colbuf[r] = bc[0][r];
            nubuf[0] = sumsq(bc[0]);
            x0buf[0] = rn[0];
        }
        lds_barrier();
        for (int j = 0; j < m; ++j) {
            const ET* cj = colbuf + (j & 1) * BR;
            const ET nub = nubuf[j & 1];
            const ET x0 = x0buf[j & 1];
            ET rc[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                rc[t] = rn[t];
                const int c = lane + t * NT;
                rn[t] = (c < m && j + 1 < m) ? R[(int64_t)(j + 1) * m + c] : ET(0);
            }
            if (nub != ET(0)) {
                const ET alpha = x0 >= ET(0) ? -sqrt(x0 * x0 + nub) : sqrt(x0 * x0 + nub);
                const ET v0 = x0 - alpha;
                const ET vtv = ET(2) * fabs(alpha) * (fabs(alpha) + fabs(x0));
#pragma unroll
                for (int t = 0; t < CPL; ++t) {
                    const int c = lane + t * NT;
                    if (c > j && c < m) {
                        // the published column is read from LDS (broadcast)
                        // in chunks of 8, once for the dot product and once
                        // for the update: holding it in registers between
                        // them would cost 2 BR registers and occupancy
                        ET w = v0 * rc[t];
#pragma unroll
                        for (int r0 = 0; r0 < BR; r0 += 8) {
                            ET cv[8];
#pragma unroll
                            for (int r = 0; r < 8; ++r) cv[r] = cj[r0 + r];
#pragma unroll
                            for (int r = 0; r < 8; ++r) w = fma_e(cv[r], bc[t][r0 + r], w);
                        }
                        const ET f = ET(2) * w / vtv;
                        R[(int64_t)j * m + c] = rc[t] - f * v0;
                        __asm__ __volatile__("" ::: "memory");  // re-read, do not keep
#pragma unroll
                        for (int r0 = 0; r0 < BR; r0 += 8) {
                            ET cv[8];
#pragma unroll
                            for (int r = 0; r < 8; ++r) cv[r] = cj[r0 + r];
#pragma unroll
                            for (int r = 0; r < 8; ++r) bc[t][r0 + r] = fma_e(-f, cv[r], bc[t][r0 + r]);
                        }
                    }
                }
                if (lane == j % NT) R[(int64_t)j * m + j] = alpha;
            }
            // the owner of column j + 1 publishes it (entries, squared norm,
            // diagonal entry of R from the row loaded ahead) for the next step
            if (j + 1 < m && lane == (j + 1) % NT) {
                const int t1 = (j + 1) / NT;
                ET* nb1 = colbuf + ((j + 1) & 1) * BR;
#pragma unroll
                for (int t = 0; t < CPL; ++t)
                    if (t == t1) {
#pragma unroll
                        for (int r = 0; r < BR; ++r) nb1[r] = bc[t][r];
                        nubuf[(j + 1) & 1] = sumsq(bc[t]);
                        x0buf[(j + 1) & 1] = rn[t];
                    }
            }
            lds_barrier();
        }
    }
    __syncthreads();  // R complete and visible to every lane
}

template <int NT>
__device__ inline double block_sum(double v, double* sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (NT == 64) return v;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < NT / 64; ++q) r = r + sh[q];
    __syncthreads();
    return r;
}

// LDS doubles of cpqr_blocked: the reflector (s), the norms (2 m), the
// panel's reflectors (s x nb) and scratch
__host__ __device__ constexpr int64_t cpqr_blocked_lds(int64_t s, int64_t m, int nt, int nb)
{
    return s + 2 * m + s * nb + 4 * nb + (nt / 64) * nb + 2 * (nt / 64) + 2;
}
// The blocked form runs when the lanes can hold the F rows of their columns
// and the panel fits the LDS budget.
constexpr int64_t QR_LDS_MAX = 80 * 1024;
__host__ __device__ inline bool use_blocked(int64_t s, int64_t m, int cols, int nt, int nb)
{
    return m <= cols && cpqr_blocked_lds(s, m, nt, nb) * 8 <= QR_LDS_MAX;
}

// Pivoted QR with delayed updates (the blocked form of LAPACK's QP3) of the
// s x m matrix M (global, row-major).  Within a panel of NB steps only the
// pivot column and the pivot row are brought up to date, from the panel's
// Householder vectors V (kept below the diagonal of the factored columns)
// and F, F[c][b] = 2 v_b^T a_c^(b) / (v_b^T v_b) (a_c^(b): column c after
// the panel's first b reflectors), whose row c lives in the registers of the
// lane that owns column c (c = lane + NT t); the trailing matrix is updated
// once per panel.  That is one read pass over the trailing matrix per step
// where the unblocked loop makes three.  Pivot rule, stopping rule and norm
// downdates are those of the unblocked loop; a norm that has to be
// recomputed is formed from the up-to-date column, its panel update applied
// on the fly (LAPACK ends the panel instead; with the fast-decaying spectra
// of kernel blocks that would end nearly every panel).  Returns the rank;
// the pivot order is in piv and R in the upper triangle of M.
template <int NT, int CPL, int NB, class ET>
__device__ __forceinline__ int cpqr_blocked(gptr<ET> M, int m, int s, double tol, gint* piv, double* lds)
{
    constexpr int W = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // LDS laid out in FP64 slots; the matrix-typed (ET) arrays start at their
    // slots (an FP32 decomposition fills half of each)
    double* nu = lds + s;       // m: partial column norms (FP64)
    double* nu0 = nu + m;       // m: their reference values
    double* Vl_d = nu0 + m;
    double* fp_d = Vl_d + (int64_t)s * NB;
    double* fj_d = fp_d + NB;
    double* vj_d = fj_d + NB;
    double* red_d = vj_d + NB;
    double* redd = red_d + W * NB;  // W
    int* redi = (int*)(redd + W);   // W
    ET* v = (ET*)lds;           // s: the reflector of the step
    ET* Vl = (ET*)Vl_d;         // s x NB: the panel's reflectors, Vl[r * NB + b]
    ET* fp = (ET*)fp_d;         // NB: F row of the pivot column
    ET* fj = (ET*)fj_d;         // NB: F row of column j
    ET* vj = (ET*)vj_d;         // NB: row j of V
    ET* red = (ET*)red_d;       // W x NB partial sums
    for (int t = 0; t < CPL; ++t) {
        const int c = tid + t * NT;
        if (c < m) {
            const double a = sumsq_rows(M + c, m, 0, s, 0.0);
            nu[c] = sqrt(a);
            nu0[c] = nu[c];
        }
    }
    __syncthreads();
    const double tol3z = down_tol<ET>();
    const double window = 1.0 - 0x1.0p-40;
    const int kmax = m < s ? m : s;
    ET F[CPL][NB];
#pragma unroll
    for (int t = 0; t < CPL; ++t)
#pragma unroll
        for (int b = 0; b < NB; ++b) F[t][b] = ET(0);
    double r00 = 0.0;
    int k = 0, j0 = 0;
    for (int j = 0; j < kmax; ++j) {
        const int jb = j - j0;
        // pivot: lowest index within the window of the largest partial norm
        double mx = 0.0;
        for (int c = j + tid; c < m; c += NT) mx = fmax(mx, nu[c]);
        mx = block_max<NT>(mx, redd);
        int cand = 0x7fffffff;
        for (int c = j + tid; c < m; c += NT)
            if (nu[c] >= window * mx) {
                cand = c;
                break;
            }
        const int pc = block_min_i<NT>(cand, redi);
        // no admissible pivot (non-finite norms, e.g. a kernel that
        // overflowed): stop, as at the rank threshold
        if (pc >= m) break;
        // F rows of the pivot column and of column j (their owners)
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = tid + t * NT;
            if (c == pc)
#pragma unroll
                for (int b = 0; b < NB; ++b) fp[b] = F[t][b];
            if (c == j)
#pragma unroll
                for (int b = 0; b < NB; ++b) fj[b] = F[t][b];
        }
        __syncthreads();
        // the pivot column brought up to date (rows >= j) and its norm, |R_jj|;
        // row r >= j is handled by thread (r - j) mod NT in this step
        double a2 = 0.0;
        for (int r = j + tid; r < s; r += NT) {
            ET x = M[(int64_t)r * m + pc];
            const ET* Vr = Vl + (int64_t)r * NB;
            for (int b = 0; b < jb; ++b) x = x - Vr[b] * fp[b];
            v[r] = x;
            a2 = a2 + (double)x * (double)x;
        }
        a2 = block_sum<NT>(a2, redd);
        const double alpha = sqrt(a2);
        if (j == 0) r00 = alpha;
        // the step that stops swaps nothing
        if (alpha == 0.0 || alpha <= tol * r00) break;
        const ET xj = v[j];
        const ET beta = xj >= ET(0) ? ET(-alpha) : ET(alpha);
        const ET vd = xj - beta;  // first entry of the Householder vector
        const ET vtv = ET(2.0 * alpha * (alpha + fabs((double)xj)));
        // swap columns j and pc (every row), F rows and norms; the reflector
        // below the diagonal of column j, R_jj
        for (int r = j + tid; r < s; r += NT) {
            if (pc != j) M[(int64_t)r * m + pc] = M[(int64_t)r * m + j];
            M[(int64_t)r * m + j] = r == j ? beta : v[r];
            if (r > j) Vl[(int64_t)r * NB + jb] = v[r];
        }
        if (pc != j) {
            for (int r = tid; r < j; r += NT) {
                const ET a = M[(int64_t)r * m + j];
                M[(int64_t)r * m + j] = M[(int64_t)r * m + pc];
                M[(int64_t)r * m + pc] = a;
            }
#pragma unroll
            for (int t = 0; t < CPL; ++t)
                if (tid + t * NT == pc)
#pragma unroll
                    for (int b = 0; b < NB; ++b) F[t][b] = fj[b];
            if (tid == 0) {
                double tmp = nu[j]; nu[j] = nu[pc]; nu[pc] = tmp;
                tmp = nu0[j]; nu0[j] = nu0[pc]; nu0[pc] = tmp;
                const int ti = piv[j]; piv[j] = piv[pc]; piv[pc] = ti;
            }
        }
        // y_b = v^T v_b over rows >= j (b < jb), row j of V
        ET yp[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) yp[b] = ET(0);
        for (int r = j + tid; r < s; r += NT) {
            const ET vr = r == j ? vd : v[r];
            const ET* Vr = Vl + (int64_t)r * NB;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < jb) yp[b] = yp[b] + vr * Vr[b];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            for (int off = 32; off > 0; off >>= 1) yp[b] += __shfl_xor(yp[b], off, 64);
            if (lane == 0) red[wv * NB + b] = yp[b];
        }
        if (tid < jb) vj[tid] = Vl[(int64_t)j * NB + tid];
        if (tid == 0) {
            v[j] = vd;
            vj[jb] = vd;
        }
        __syncthreads();
        ET yb[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            ET a = ET(0);
            for (int q = 0; q < W; ++q) a = a + red[q * NB + b];
            yb[b] = a;
        }
        // this lane's columns c > j: F column jb, the pivot row, norm downdate
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = tid + t * NT;
            if (c > j && c < m) {
                const ET w = dot_rows<16>(v, M + c, m, j, s, ET(0));
                ET corr = ET(0);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (b < jb) corr = corr + yb[b] * F[t][b];
                const ET fn = ET(2) * (w - corr) / vtv;
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (b == jb) F[t][b] = fn;
                ET rj = M[(int64_t)j * m + c];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (b <= jb) rj = rj - vj[b] * F[t][b];
                M[(int64_t)j * m + c] = rj;
                if (nu[c] != 0.0) {
                    double tt = fabs((double)rj) / nu[c];
                    tt = (1.0 + tt) * (1.0 - tt);
                    if (tt < 0.0) tt = 0.0;
                    const double rat = nu[c] / nu0[c];
                    if (tt * rat * rat <= tol3z) {
                        // recomputed from the up-to-date column (rows > j),
                        // formed on the fly from the panel's reflectors
                        double a = 0.0;
                        constexpr int RB = 8;
                        int r = j + 1;
                        for (; r + RB <= s; r += RB) {
                            ET x[RB];
#pragma unroll
                            for (int q = 0; q < RB; ++q) x[q] = M[(int64_t)(r + q) * m + c];
#pragma unroll
                            for (int q = 0; q < RB; ++q) {
                                const ET* Vr = Vl + (int64_t)(r + q) * NB;
#pragma unroll
                                for (int b = 0; b < NB; ++b)
                                    if (b <= jb) x[q] = x[q] - Vr[b] * F[t][b];
                                a = a + (double)x[q] * (double)x[q];
                            }
                        }
                        for (; r < s; ++r) {
                            ET x = M[(int64_t)r * m + c];
                            const ET* Vr = Vl + (int64_t)r * NB;
#pragma unroll
                            for (int b = 0; b < NB; ++b)
                                if (b <= jb) x = x - Vr[b] * F[t][b];
                            a = a + (double)x * (double)x;
                        }
                        nu[c] = sqrt(a);
                        nu0[c] = nu[c];
                    } else {
                        nu[c] = nu[c] * sqrt(tt);
                    }
                }
            }
        }
        __syncthreads();
        k = j + 1;
        if (jb + 1 == NB && k < kmax) {
            // panel update of the trailing matrix (rows > j, this lane's
            // columns > j)
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = tid + t * NT;
                if (c > j && c < m) {
                    constexpr int RB = 8;
                    int r = j + 1;
                    for (; r + RB <= s; r += RB) {
                        ET x[RB];
#pragma unroll
                        for (int q = 0; q < RB; ++q) x[q] = M[(int64_t)(r + q) * m + c];
#pragma unroll
                        for (int q = 0; q < RB; ++q) {
                            const ET* Vr = Vl + (int64_t)(r + q) * NB;
#pragma unroll
                            for (int b = 0; b < NB; ++b)
                                if (b <= jb) x[q] = x[q] - Vr[b] * F[t][b];
                            M[(int64_t)(r + q) * m + c] = x[q];
                        }
                    }
                    for (; r < s; ++r) {
                        ET x = M[(int64_t)r * m + c];
                        const ET* Vr = Vl + (int64_t)r * NB;
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            if (b <= jb) x = x - Vr[b] * F[t][b];
                        M[(int64_t)r * m + c] = x;
                    }
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) F[t][b] = ET(0);
            }
            j0 = j + 1;
            __syncthreads();
        }
    }
    return k;
}

constexpr int QR_NB = 8;  // steps per panel of the blocked pivoted QR
constexpr int WNT = 512;  // lanes per wide task

// The s x m block is compressed to its R factor when that removes a good
// share of the rows (s > 1.5 m) and the lanes can hold its columns (m <= cap).
__host__ __device__ inline bool compress_rows(int s, int m, int cap)
{
    return 2 * (int64_t)s > 3 * (int64_t)m && m <= cap;
}

// One node per workgroup of NT lanes (64: one wavefront; 256 or 512 for
// the wide nodes).  LDSM: the matrix the pivoted QR runs on lives in LDS
// (dynamic shared memory after the reflector), otherwise in the global
// workspace, where the blocked form runs when it fits.  When compress_rows
// holds, the s x m kernel block is first compressed to its m x m R factor
// (tsqr_fold; PRE: k_id_fold already did it): column pivoting sees only the
// partial column norms, which a left orthogonal factor does not change, so
// the pivots, |R_jj| and T are those of the s x m block up to rounding.
template <int NT, bool LDSM, int CPL, int BR, bool PRE, int FAM, class ET>
__global__ __launch_bounds__(NT) void k_batched_id(const IdTask* __restrict__ tasks, const int* __restrict__ order)
{
    extern __shared__ double dyn[];
    __shared__ double redd[NT / 64];
    __shared__ int redi[NT / 64];
    __shared__ double sh_alpha;

    const IdTask& tk = tasks[order[blockIdx.x]];
    const int m = tk.m, s0 = tk.s, d = tk.d, kid = tk.kid;
    const double prm = tk.prm, tol = tk.tol;
    gint* piv = (gint*)tk.piv;
    for (int c = threadIdx.x; c < m; c += NT) piv[c] = c;
    if (m == 0 || s0 == 0) {
        if (threadIdx.x == 0) *tk.rank = 0;
        return;
    }
    // PRE: the block was compressed to its m x m R factor by k_id_fold
    const bool comp = !PRE && compress_rows(s0, m, CPL * NT);
    const int s = (comp || PRE) ? m : s0;  // rows of the matrix the pivoted QR runs on
    ET* v = (ET*)dyn;  // in the FP64 slots of dyn, like everything below
    using MPtr = std::conditional_t<LDSM, ET*, gptr<ET>>;
    MPtr M;
    if constexpr (LDSM)
        M = (ET*)(dyn + s);
    else
        M = (gptr<ET>)tk.M;
    gdouble* nu = (gdouble*)tk.nu;
    gdouble* nu0 = nu + m;
    gdouble* ss = nu + 2 * m;
    const int* xi = tk.x_idx;
    const int* yi = tk.y_idx;

    if constexpr (PRE) {
    } else if (comp) {
        // the published column lives after the LDS matrix, or over the (not
        // yet used) reflector space
        double* cb = LDSM ? dyn + s + (int64_t)s * m : dyn;
        tsqr_fold<NT, CPL, BR, FAM, ET>(tk, m, s0, M, cb, cb + 2 * BR, cb + 2 * BR + 4);
    } else {
        // kernel block: M[r][c] = kappa(x_c, y_r), a row per wavefront at a
        // time (its point read once), the columns across the lanes
        constexpr int W = NT / 64;
        const int lane = threadIdx.x & 63;
        const gdouble* gp = (const gdouble*)tk.pts;
        const int64_t ld = tk.ld;
        for (int r = threadIdx.x >> 6; r < s; r += W) {
            const int yr = yi[r];
            double yc[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < d; ++a) yc[a] = gp[a * ld + yr];
            for (int c = lane; c < m; c += 64) {
                const int xc = xi[c];
                double r2 = 0.0, xy = 0.0, e0 = 0.0;  // coordinate order, as dist2
                for (int a = 0; a < d; ++a) {
                    const double xa = gp[a * ld + xc];
                    const double ya = a == 0 ? yc[0] : (a == 1 ? yc[1] : yc[2]);
                    if constexpr (FAM == FAM_COSINE) {
                        xy = xy + xa * ya;
                    } else {
                        const double t = xa - ya;
                        if (a == 0) e0 = t;
                        r2 = r2 + t * t;
                    }
                }
                M[(int64_t)r * m + c] = kappa_id<ET, FAM>(kid, prm, r2, xy, tk.swap ? -e0 : e0);
            }
        }
        __syncthreads();
    }
    int k = 0;
    bool blocked = false;
    if constexpr (!LDSM) {
        // global matrix: the blocked form when the lanes can hold the F rows
        if (use_blocked(s, m, CPL * NT, NT, QR_NB)) {
            k = cpqr_blocked<NT, CPL, QR_NB, ET>(M, m, s, tol, piv, dyn);
            blocked = true;
        }
    }
    if (!blocked) {
    for (int c = threadIdx.x; c < m; c += NT) {
        double acc = sumsq_rows(M + c, m, 0, s, 0.0);
        ss[c] = acc;
        nu[c] = sqrt(acc);
        nu0[c] = nu[c];
    }
    __syncthreads();

    const double tol3z = down_tol<ET>();
    const double window = 1.0 - 0x1.0p-40;
    const int kmax = m < s ? m : s;
    double r00 = 0.0;
    for (int j = 0; j < kmax; ++j) {
        // pivot: lowest index within the window of the largest partial norm
        double mx = 0.0;
        for (int c = j + threadIdx.x; c < m; c += NT) mx = fmax(mx, nu[c]);
        mx = block_max<NT>(mx, redd);
        int cand = 0x7fffffff;
        for (int c = j + threadIdx.x; c < m; c += NT)
            if (nu[c] >= window * mx) {
                cand = c;
                break;
            }
        int pc = block_min_i<NT>(cand, redi);
        // no admissible pivot (non-finite norms, e.g. a kernel that
        // overflowed): stop, as at the rank threshold
        if (pc >= m) break;
        // |R_jj| of the candidate; the step that stops swaps nothing
        if (threadIdx.x == 0) sh_alpha = sqrt(ss[pc]);
        __syncthreads();
        const double alpha = sh_alpha;
        if (j == 0) r00 = alpha;
        if (alpha == 0.0 || alpha <= tol * r00) break;
        if (pc != j) {
            for (int r = threadIdx.x; r < s; r += NT) {
                ET t = M[(int64_t)r * m + j];
                M[(int64_t)r * m + j] = M[(int64_t)r * m + pc];
                M[(int64_t)r * m + pc] = t;
            }
            if (threadIdx.x == 0) {
                double t = nu[j]; nu[j] = nu[pc]; nu[pc] = t;
                t = nu0[j]; nu0[j] = nu0[pc]; nu0[pc] = t;
                t = ss[j]; ss[j] = ss[pc]; ss[pc] = t;
                int ti = piv[j]; piv[j] = piv[pc]; piv[pc] = ti;
            }
        }
        __syncthreads();
        const ET xj = M[(int64_t)j * m + j];
        const ET beta = xj >= ET(0) ? ET(-alpha) : ET(alpha);
        for (int r = j + threadIdx.x; r < s; r += NT) v[r] = M[(int64_t)r * m + j];
        __syncthreads();
        if (threadIdx.x == 0) v[j] = v[j] - beta;
        __syncthreads();
        const ET vtv = ET(2.0 * alpha * (alpha + fabs((double)xj)));
        for (int c = j + 1 + threadIdx.x; c < m; c += NT) {
            ET w = dot_rows(v, M + c, m, j, s, ET(0));
            ET f = ET(2) * w / vtv;
            double tail = axpy_rows(v, f, M + c, m, j, s);
            ss[c] = tail;
            if (nu[c] != 0.0) {
                double t = fabs((double)M[(int64_t)j * m + c]) / nu[c];
                t = (1.0 + t) * (1.0 - t);
                if (t < 0.0) t = 0.0;
                double rat = nu[c] / nu0[c];
                double t2 = t * rat * rat;
                if (t2 <= tol3z) {
                    nu[c] = sqrt(tail);
                    nu0[c] = nu[c];
                } else {
                    nu[c] = nu[c] * sqrt(t);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) M[(int64_t)j * m + j] = beta;
        __syncthreads();
        k = j + 1;
    }
    }
    __syncthreads();
    // T = R11^{-1} R12 by back substitution, one column of R12 per lane
    const int nr = m - k;
    gdouble* T = (gdouble*)tk.T;
    for (int u = threadIdx.x; u < nr; u += NT) {
        for (int t = k - 1; t >= 0; --t) {
            double acc = M[(int64_t)t * m + (k + u)];
            const MPtr Rt = M + (int64_t)t * m;
            int l = t + 1;
            for (; l + LB <= k; l += LB) {
                double rv[LB], tv[LB];
#pragma unroll
                for (int q = 0; q < LB; ++q) {
                    rv[q] = Rt[l + q];
                    tv[q] = T[(int64_t)(l + q) * nr + u];
                }
#pragma unroll
                for (int q = 0; q < LB; ++q) acc = acc - rv[q] * tv[q];
            }
            for (; l < k; ++l) acc = acc - Rt[l] * T[(int64_t)l * nr + u];
            T[(int64_t)t * nr + u] = acc / M[(int64_t)t * m + t];
        }
    }
    for (int t = threadIdx.x; t < k; t += NT) tk.skel[t] = xi[piv[t]];
    if (threadIdx.x == 0) *tk.rank = k;
}

// Strong rank-revealing swaps after the ID of a task with srrqr_f = f > 1
// (Eq. SRRQR1 bounds the interpolation matrix by a constant), one workgroup
// per task, T (k x (m-k), row-major) in place: while the largest |T_tu|
// (the first in row-major order among equal ones) exceeds f, skeleton t and
// non-skeleton u trade places by a Gauss-Jordan pivot on p = T_tu:
//   row t:       T_tu' <- T_tu' / p,   T_tu <- 1 / p
//   rows l != t: T_lu' <- T_lu' - T_lu (T_tu' / p),   T_lu <- -T_lu / p
// and piv[t] <-> piv[k + u]; at most 8k swaps.  The skeleton is rewritten
// from the final pivots.  Dynamic LDS: the pivot column (k doubles).
__global__ __launch_bounds__(TB) void k_srrqr(const IdTask* __restrict__ tasks, int ntask)
{
    extern __shared__ double cbuf[];
    __shared__ double rv[TB];
    __shared__ int ri[TB];
    if ((int)blockIdx.x >= ntask) return;
    const IdTask& tk = tasks[blockIdx.x];
    const double f = tk.srrqr_f;
    const int m = tk.m;
    const int k = *tk.rank;
    const int nr = m - k;
    const int tid = threadIdx.x;
    if (!(f > 1.0) || k <= 0 || nr <= 0) return;
    gdouble* T = (gdouble*)tk.T;
    int* piv = tk.piv;
    const int ne = k * nr;
    for (int nsw = 0; nsw < 8 * k; ++nsw) {
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int e = tid; e < ne; e += TB) {
            const double a = fabs(T[e]);
            if (a > bv) {
                bv = a;
                bi = e;
            }
        }
        rv[tid] = bv;
        ri[tid] = bi;
        __syncthreads();
        for (int off = TB / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double v2 = rv[tid + off];
                const int i2 = ri[tid + off];
                if (v2 > rv[tid] || (v2 == rv[tid] && i2 < ri[tid])) {
                    rv[tid] = v2;
                    ri[tid] = i2;
                }
            }
            __syncthreads();
        }
        const double best = rv[0];
        const int bidx = ri[0];
        __syncthreads();
        if (!(best > f)) break;
        const int bt = bidx / nr, bu = bidx - bt * nr;
        const double p = T[bidx];
        for (int l = tid; l < k; l += TB) cbuf[l] = T[(int64_t)l * nr + bu];
        __syncthreads();
        for (int u = tid; u < nr; u += TB) {
            const int64_t e = (int64_t)bt * nr + u;
            T[e] = u == bu ? 1.0 / p : T[e] / p;
        }
        __syncthreads();
        for (int e = tid; e < ne; e += TB) {
            const int l = e / nr, u = e - l * nr;
            if (l == bt) continue;
            T[e] = u == bu ? -cbuf[l] / p : T[e] - cbuf[l] * T[(int64_t)bt * nr + u];
        }
        if (tid == 0) {
            const int x = piv[bt];
            piv[bt] = piv[k + bu];
            piv[k + bu] = x;
        }
        __syncthreads();
    }
    for (int t = tid; t < k; t += TB) tk.skel[t] = tk.x_idx[piv[t]];
}

// Row set of every node of a level: the leaf's points, or the children's
// skeletons concatenated in child order.
__global__ __launch_bounds__(TB) void k_xbar_fill(int lo, const int* __restrict__ nchild,
                                                  const int* __restrict__ first_child, const int* __restrict__ start,
                                                  const int* __restrict__ count, const int* __restrict__ rank,
                                                  const int* __restrict__ skel, int skel_stride,
                                                  const int64_t* __restrict__ off, int* __restrict__ out)
{
    int t = blockIdx.x;
    int i = lo + t;
    int* o = out + off[t];
    if (nchild[i] == 0) {
        for (int q = threadIdx.x; q < count[i]; q += TB) o[q] = start[i] + q;
        return;
    }
    int64_t w = 0;
    for (int c = first_child[i]; c < first_child[i] + nchild[i]; ++c) {
        int kc = rank[c];
        for (int q = threadIdx.x; q < kc; q += TB) o[w + q] = skel[(int64_t)c * skel_stride + q];
        w += kc;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Wide nodes (m > 64) run as two launches: the compression of tall blocks
// (k_id_fold) and the pivoted QR (k_id_qr).
//
// k_id_fold: the s x m block (s > m) is folded into its m x m R factor in the
// task's workspace with the reflectors of tsqr_fold.  Lane l owns columns
// l, l + 256, ... (CPL of them) and is the only lane to touch their R
// entries, so a step synchronises through LDS only; the R rows a lane needs
// are loaded D steps ahead into a register ring, and the block entries are
// evaluated SL rows at a time through a lane-private LDS slice.
template <int CPL, int BR, int D, int FAM, class ET, bool REREAD = false>
__global__ __launch_bounds__(256) void k_id_fold(const IdTask* __restrict__ tasks, const int* __restrict__ order)
{
    constexpr int NT = 256, SL = 8;
    static_assert(BR % SL == 0 && BR % 4 == 0, "row block");
    extern __shared__ double dyn[];
    // FP64 slots; the ET arrays start at theirs
    ET* colbuf = (ET*)dyn;                   // 2 x BR: the column step j eliminates
    ET* nubuf = (ET*)(dyn + 2 * BR);         // 2: its squared norm
    ET* x0buf = (ET*)(dyn + 2 * BR + 2);     // 2: the diagonal entry R[j][j]
    ET* scr = (ET*)(dyn + 2 * BR + 4);       // SL x NT evaluation slices
    double* ycrd = dyn + 2 * BR + 4 + SL * NT;  // 3 x BR: the row block's points
    const IdTask& tk = tasks[order[blockIdx.x]];
    const int m = tk.m, s0 = tk.s, d = tk.d, kid = tk.kid;
    const double prm = tk.prm;
    const double dsgn = tk.swap ? -1.0 : 1.0;  // column side: kappa(y, x)
    const double* pts = tk.pts;
    const int64_t ld = tk.ld;
    const int* yi = tk.y_idx;
    gptr<ET> R = (gptr<ET>)tk.M;
    const int lane = threadIdx.x;
    for (int64_t e = lane; e < (int64_t)m * m; e += NT) R[e] = 0.0;
    // this lane's column points: in registers for one column per lane,
    // otherwise read where needed (L1 hits; registers kept for occupancy)
    XCoords<CPL> xr(pts, ld, tk.x_idx, lane, NT, m, d);
    __syncthreads();
    ET bc[CPL][BR], rn[D][CPL];
    // squared norm of a column's block part (formed by the column's owner
    // when it publishes the column)
    auto sumsq = [](const ET* b) {
        ET t4[4] = {ET(0), ET(0), ET(0), ET(0)};
#pragma unroll
        for (int r = 0; r < BR; ++r) t4[r & 3] = fma_e(b[r], b[r], t4[r & 3]);
        return (t4[0] + t4[1]) + (t4[2] + t4[3]);
    };
    for (int r0 = 0; r0 < s0; r0 += BR) {
        const int nb = min(BR, s0 - r0);
        // the row block's points, staged once in LDS for all lanes
        if (lane < nb)
            for (int a = 0; a < d; ++a) ycrd[a * BR + lane] = pts[a * ld + yi[r0 + lane]];
        lds_barrier();
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = lane + t * NT;
#pragma unroll
            for (int k0 = 0; k0 < BR; k0 += SL) {
                if (c < m)
                    for (int r = 0; r < SL && k0 + r < nb; ++r) {
                        // squared distance in coordinate order, as dist2
                        double r2 = 0.0, xy = 0.0, e0 = 0.0;
                        if constexpr (FAM == FAM_COSINE)
                            for (int a = 0; a < d; ++a) xy = xy + xr.get(t, a) * ycrd[a * BR + k0 + r];
                        else
                            for (int a = 0; a < d; ++a) {
                                const double ea = xr.get(t, a) - ycrd[a * BR + k0 + r];
                                if (a == 0) e0 = ea;
                                r2 = r2 + ea * ea;
                            }
                        scr[r * NT + lane] = kappa_id<ET, FAM>(kid, prm, r2, xy, dsgn * e0);
                    }
#pragma unroll
                for (int r = 0; r < SL; ++r) bc[t][k0 + r] = (c < m && k0 + r < nb) ? scr[r * NT + lane] : ET(0);
            }
        }
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = lane + t * NT;
                rn[q][t] = (c < m && q < m) ? R[(int64_t)q * m + c] : ET(0);
            }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < BR; ++r) colbuf[r] = bc[0][r];
            nubuf[0] = sumsq(bc[0]);
            x0buf[0] = rn[0][0];
        }
        lds_barrier();
        for (int j0 = 0; j0 < m; j0 += D) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const int j = j0 + q;
                if (j < m) {
                    const ET* cj = colbuf + (j & 1) * BR;
                    const ET nub = nubuf[j & 1];
                    const ET x0 = x0buf[j & 1];
                    ET rc[CPL];
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        rc[t] = rn[q][t];
                        const int c = lane + t * NT;
                        rn[q][t] = (c < m && j + D < m) ? R[(int64_t)(j + D) * m + c] : ET(0);
                    }
                    if (nub != ET(0)) {
                        const ET alpha = x0 >= ET(0) ? -sqrt(x0 * x0 + nub) : sqrt(x0 * x0 + nub);
                        const ET v0 = x0 - alpha;
                        const ET vtv = ET(2) * fabs(alpha) * (fabs(alpha) + fabs(x0));
#pragma unroll
                        for (int t = 0; t < CPL; ++t) {
                            const int c = lane + t * NT;
                            // chunks wholly at or left of column j, or past m, are skipped
                            if (t * NT + NT - 1 > j && t * NT < m && c > j && c < m) {
                                // the published column is read from LDS in chunks of 8
                                ET w4[4] = {v0 * rc[t], ET(0), ET(0), ET(0)};
#pragma unroll
                                for (int r0 = 0; r0 < BR; r0 += 8) {
                                    ET cv[8];
#pragma unroll
                                    for (int r = 0; r < 8; ++r) cv[r] = cj[r0 + r];
#pragma unroll
                                    for (int r = 0; r < 8; ++r)
                                        w4[r & 3] = fma_e(cv[r], bc[t][r0 + r], w4[r & 3]);
                                }
                                const ET f = ET(2) * ((w4[0] + w4[1]) + (w4[2] + w4[3])) / vtv;
                                R[(int64_t)j * m + c] = rc[t] - f * v0;
                                // REREAD: the published column is read again for the
                                // update instead of being held (2 BR registers)
                                if constexpr (REREAD) __asm__ __volatile__("" ::: "memory");
#pragma unroll
                                for (int r0 = 0; r0 < BR; r0 += 8) {
                                    ET cv[8];
#pragma unroll
                                    for (int r = 0; r < 8; ++r) cv[r] = cj[r0 + r];
#pragma unroll
                                    for (int r = 0; r < 8; ++r) bc[t][r0 + r] = fma_e(-f, cv[r], bc[t][r0 + r]);
                                }
                            }
                        }
                        if (lane == j % NT) R[(int64_t)j * m + j] = alpha;
                    }
                    // the owner of column j + 1 publishes it for the next step
                    if (j + 1 < m && lane == (j + 1) % NT) {
                        const int t1 = (j + 1) / NT;
                        ET* nb1 = colbuf + ((j + 1) & 1) * BR;
#pragma unroll
                        for (int t = 0; t < CPL; ++t)
                            if (t == t1) {
#pragma unroll
                                for (int r = 0; r < BR; ++r) nb1[r] = bc[t][r];
                                nubuf[(j + 1) & 1] = sumsq(bc[t]);
                                x0buf[(j + 1) & 1] = rn[(q + 1) % D][t];
                            }
                    }
                    lds_barrier();
                }
            }
        }
    }
}

namespace {

template <int FAM, class ET>
void batched_id_family(const std::vector<IdTask>& tasks_in, hipStream_t s, IdProf* prof)
{
    const int np = (int)tasks_in.size();
    if (np <= 0) return;
    std::vector<IdTask> tasks(tasks_in);
    // Launch classes (lanes per task, where the matrix lives, columns per lane
    // and rows per block of the compression):
    //   0      64 lanes, matrix in LDS, m <= 64 (one launch per LDS bin)
    //   1      64 lanes, global matrix, m <= 64
    //   4 / 5  64 < m <= 1024 and s > 1.5 m: compression by k_id_fold (many
    //          tasks per CU), then the blocked pivoted QR of the m x m
    //          factor on 512 lanes, or 256 when m <= 256 (two tasks per CU)
    //   2      512 lanes, global matrix, the other wide nodes
    struct Cls {
        int nt, cpl, br;
    };
    const Cls CL[6] = {{64, 1, 32}, {64, 1, 16}, {WNT, 2, 16}, {64, 1, 32}, {WNT, 2, 16}, {256, 1, 16}};  // 3: unused
    const size_t LDS_CAP = 80 * 1024;     // bytes per workgroup
    auto lds_need = [&](const IdTask& t, int c) -> size_t {
        const Cls& k = CL[c];
        const bool comp = c == 4 || c == 5 || compress_rows(t.s, t.m, k.cpl * k.nt);
        const int sr = comp ? t.m : t.s;
        // the blocked pivoted QR keeps the norms and panel scratch in LDS
        const size_t qr = use_blocked(sr, t.m, k.cpl * k.nt, k.nt, QR_NB) ? cpqr_blocked_lds(sr, t.m, k.nt, QR_NB) : 0;
        if (c == 4 || c == 5) return std::max((size_t)sr, qr) * sizeof(double);
        // published column (2 x BR), its norms and diagonal entries (2 x 2),
        // the lanes' evaluation slices, the row block's points (3 x BR)
        const size_t pub = comp ? 2 * k.br + 4 + (size_t)8 * k.nt + 3 * k.br : 0;
        if (c == 0 || c == 3) return ((size_t)sr + (size_t)sr * t.m + pub) * sizeof(double);
        return std::max(std::max((size_t)sr, qr), pub) * sizeof(double);
    };
    // The narrow nodes in LDS go out in one launch per size bin of their LDS
    // need (a launch reserves its largest need for every workgroup), so that
    // the bulk of the leaves is not held to the occupancy of the largest.
    constexpr int NBIN = 12;
    const size_t BIN_CAP[NBIN] = {12 << 10, 14 << 10, 16 << 10, 18 << 10, 20 << 10, 24 << 10,
                                  28 << 10, 32 << 10, 40 << 10, 48 << 10, 64 << 10, 80 << 10};
    static_assert(80 << 10 == LDS_CAP, "last bin");
    std::vector<int> cls(np), bin(np, -1);
    for (int p = 0; p < np; ++p) {
        const IdTask& t = tasks[p];
        if (t.m > 64) {
            const bool comp = compress_rows(t.s, t.m, 4 * TB);
            cls[p] = comp ? (t.m <= 256 ? 5 : 4) : 2;
            tasks[p].folded = comp ? 1 : 0;
        } else {
            const size_t need = lds_need(t, 0);
            cls[p] = need <= LDS_CAP ? 0 : 1;
            if (cls[p] == 0)
                for (int b = NBIN - 1; b >= 0 && need <= BIN_CAP[b]; --b) bin[p] = b;
        }
    }
    // A bin of fewer than BIN_MIN tasks joins the next smaller non-empty bin
    // (whose launch then reserves the larger need): a launch of a few
    // workgroups lasts a whole task, which the larger launch hides.  A launch
    // starts its tasks of the largest bins first.
    constexpr int BIN_MIN = H2_TUNE_BIN_MIN;
    std::vector<int> bin0(bin);
    {
        int nb[NBIN] = {};
        for (int p = 0; p < np; ++p)
            if (bin[p] >= 0) ++nb[bin[p]];
        for (int b = NBIN - 1; b > 0; --b) {
            if (nb[b] == 0 || nb[b] >= BIN_MIN) continue;
            int to = b - 1;
            while (to >= 0 && nb[to] == 0) --to;
            if (to < 0) break;
            for (int p = 0; p < np; ++p)
                if (bin[p] == b) bin[p] = to;
            nb[to] += nb[b];
            nb[b] = 0;
        }
    }
    // narrow classes first (the LDS bins, then the global one), then the
    // wide ones (timed together)
    std::vector<int> order;
    order.reserve(np);
    int bcnt[NBIN] = {}, boff[NBIN] = {};
    size_t blds[NBIN] = {};
    {
        std::vector<int> nar;
        for (int p = 0; p < np; ++p)
            if (bin[p] >= 0) nar.push_back(p);
        std::stable_sort(nar.begin(), nar.end(),
                         [&](int x, int y) { return bin[x] != bin[y] ? bin[x] < bin[y] : bin0[x] > bin0[y]; });
        for (int b = 0; b < NBIN; ++b) blds[b] = 8;
        for (int p : nar) {
            const int b = bin[p];
            if (bcnt[b] == 0) boff[b] = (int)order.size();
            order.push_back(p);
            ++bcnt[b];
            blds[b] = std::max(blds[b], lds_need(tasks[p], 0));
        }
    }
    const int ORD[4] = {1, 5, 4, 2};
    int cnt[6] = {0, 0, 0, 0, 0, 0}, off[6] = {0, 0, 0, 0, 0, 0};
    size_t lds[6] = {8, 8, 8, 8, 8, 8};
    for (int c : ORD) {
        off[c] = (int)order.size();
        for (int p = 0; p < np; ++p)
            if (cls[p] == c) {
                order.push_back(p);
                ++cnt[c];
                lds[c] = std::max(lds[c], lds_need(tasks[p], c));
            }
    }
    // the tall wide blocks to compress, grouped by columns per lane
    std::vector<int> fold[3];
    for (int p = 0; p < np; ++p) {
        const IdTask& t = tasks[p];
        if (t.folded) fold[t.m <= 256 ? 0 : (t.m <= 512 ? 1 : 2)].push_back(p);
    }
    int foff[3] = {0, 0, 0}, nfold = 0;
    for (int g = 0; g < 3; ++g) {
        foff[g] = (int)order.size() + nfold;
        nfold += (int)fold[g].size();
    }
    std::vector<int> order_all(order);
    for (auto& v : fold) order_all.insert(order_all.end(), v.begin(), v.end());
    DBuf<IdTask> d_tasks;
    DBuf<int> d_order;
    d_tasks.ensure(tasks.size(), s);
    d_order.ensure(order_all.size(), s);
    H2_HIP(hipMemcpyAsync(d_tasks.p, tasks.data(), tasks.size() * sizeof(IdTask), hipMemcpyHostToDevice, s));
    H2_HIP(hipMemcpyAsync(d_order.p, order_all.data(), order_all.size() * sizeof(int), hipMemcpyHostToDevice, s));
    hipEvent_t ev[4] = {};
    if (prof)
        for (auto& e : ev) H2_HIP(hipEventCreate(&e));
    if (prof) H2_HIP(hipEventRecord(ev[0], s));
    auto launch = [&](int c) {
        if (cnt[c] == 0) return;
        const int* ord = d_order.p + off[c];
        switch (c) {
        case 1: k_batched_id<64, false, 1, 16, false, FAM, ET><<<cnt[c], 64, lds[c], s>>>(d_tasks.p, ord); break;
        case 4: k_batched_id<WNT, false, 2, 16, true, FAM, ET><<<cnt[c], WNT, lds[c], s>>>(d_tasks.p, ord); break;
        case 5: k_batched_id<256, false, 1, 16, true, FAM, ET><<<cnt[c], 256, lds[c], s>>>(d_tasks.p, ord); break;
        default: k_batched_id<WNT, false, 2, 16, false, FAM, ET><<<cnt[c], WNT, lds[c], s>>>(d_tasks.p, ord); break;
        }
        H2_LAUNCH_CHECK();
    };
    for (int b = 0; b < NBIN; ++b)
        if (bcnt[b] > 0) {
            k_batched_id<64, true, 1, 32, false, FAM, ET><<<bcnt[b], 64, blds[b], s>>>(d_tasks.p, d_order.p + boff[b]);
            H2_LAUNCH_CHECK();
        }
    launch(1);
    if (prof) H2_HIP(hipEventRecord(ev[1], s));
    if (!fold[0].empty())
        k_id_fold<1, 32, 1, FAM, ET><<<(unsigned)fold[0].size(), 256, (2 * 32 + 4 + 8 * 256 + 3 * 32) * sizeof(double), s>>>(
            d_tasks.p, d_order.p + foff[0]);
    if (!fold[1].empty())
        k_id_fold<2, 32, 1, FAM, ET, true><<<(unsigned)fold[1].size(), 256, (2 * 32 + 4 + 8 * 256 + 3 * 32) * sizeof(double), s>>>(
            d_tasks.p, d_order.p + foff[1]);
    if (!fold[2].empty())
        k_id_fold<4, 8, 1, FAM, ET><<<(unsigned)fold[2].size(), 256, (2 * 8 + 4 + 8 * 256 + 3 * 8) * sizeof(double), s>>>(
            d_tasks.p, d_order.p + foff[2]);
    H2_LAUNCH_CHECK();
    launch(5);
    launch(4);
    launch(2);
    if (prof) H2_HIP(hipEventRecord(ev[2], s));
    if (prof) H2_HIP(hipEventRecord(ev[3], s));
    H2_HIP(hipStreamSynchronize(s));
    if (prof) {
        float a = 0.f, w = 0.f;
        H2_HIP(hipEventElapsedTime(&a, ev[0], ev[3]));
        H2_HIP(hipEventElapsedTime(&w, ev[1], ev[2]));
        prof->ms_all += a;
        prof->ms_wide += w;
        for (auto& e : ev) H2_HIP(hipEventDestroy(e));
    }
}

}  // namespace

// The ID tasks of each kernel family and arithmetic (FP64, or FP32 for the
// precision mode) run through their own instances of the launches (a
// batched build may mix them).
void batched_id(const std::vector<IdTask>& tasks, hipStream_t s, IdProf* prof)
{
    std::vector<IdTask> fam[2][3];
    for (const IdTask& t : tasks) fam[t.f32 ? 1 : 0][kernel_family(t.kid)].push_back(t);
    batched_id_family<FAM_RADIAL, double>(fam[0][FAM_RADIAL], s, prof);
    batched_id_family<FAM_COSINE, double>(fam[0][FAM_COSINE], s, prof);
    batched_id_family<FAM_ADVECTION, double>(fam[0][FAM_ADVECTION], s, prof);
    batched_id_family<FAM_RADIAL, float>(fam[1][FAM_RADIAL], s, prof);
    batched_id_family<FAM_COSINE, float>(fam[1][FAM_COSINE], s, prof);
    batched_id_family<FAM_ADVECTION, float>(fam[1][FAM_ADVECTION], s, prof);
}

template <class T>
static void upload(DBuf<T>& dst, const std::vector<T>& src, hipStream_t s)
{
    dst.ensure(src.size(), s);
    if (!src.empty())
        H2_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Nested bases of several independent problems at once: round t handles
// depth maxdepth - t of every problem (a node's children were done in the
// round before), and all nodes of a round go into one batched ID launch
// (several only when the workspace cap splits it).  piv and T offsets are
// assigned per problem in processing order (deepest level first).
// Floating-point operations of the pivoted-QR interpolative decomposition of
// an s x m block stopped at rank k (Section 3.2): the initial column norms,
// each Householder vector and its application to the remaining columns, and
// the triangular solve for T.  (The compression of tall blocks and the norm
// downdates are not counted: this is the method's own work.)
static double id_flop_count(int64_t s, int64_t m, int64_t k)
{
    double f = 2.0 * (double)s * (double)m;
    for (int64_t j = 0; j < k; ++j) f += 2.0 * (double)(s - j) * (1.0 + 2.0 * (double)(m - j - 1));
    return f + (double)k * (double)k * (double)(m - k);
}

// Nested bases of every problem of `hs`, level by level from the deepest,
// all problems' nodes of a round in one batched ID.  A non-symmetric kernel
// adds the column side: the same steps on K(Y_i*, Xbar_i)^T with row sets
// from the column skeletons, in the same launches.
void build_bases_multi(const std::vector<Handle*>& hs, hipStream_t s)
{
    // one unit per (problem, side)
    struct Unit {
        Handle* h;
        Basis* b;
        int swap;
        const std::vector<int>* ys_cnt;
        int64_t piv_total = 0, T_total = 0, xbase = 0;
        int L = 0;
    };
    const int np = (int)hs.size();
    std::vector<std::vector<int>> ys_cnt(np);
    std::vector<Unit> units;
    int maxd = 0;
    for (int p = 0; p < np; ++p) {
        Handle& h = *hs[p];
        const int nn = h.nnode;
        ys_cnt[p] = read_vec(h.ys_cnt.p, nn, s);
        for (int side = 0; side < (h.nonsym ? 2 : 1); ++side) {
            Basis& b = side == 0 ? h.bu : h.bv;
            b.rank.ensure((size_t)nn, s);
            b.mbar.ensure((size_t)nn, s);
            b.skel.ensure((size_t)nn * h.ys_stride, s);
            b.piv_off.ensure((size_t)nn + 1, s);
            b.T_off.ensure((size_t)nn + 1, s);
            H2_HIP(hipMemsetAsync(b.rank.p, 0, sizeof(int) * nn, s));
            H2_HIP(hipMemsetAsync(b.mbar.p, 0, sizeof(int) * nn, s));
            b.h_rank.assign(nn, 0);
            b.h_mbar.assign(nn, 0);
            b.h_piv_off.assign((size_t)nn + 1, 0);
            b.h_T_off.assign((size_t)nn + 1, 0);
            Unit u;
            u.h = &h;
            u.b = &b;
            u.swap = side;
            u.ys_cnt = &ys_cnt[p];
            units.push_back(u);
        }
        maxd = std::max(maxd, h.maxdepth);
    }
    bool prof_on = false;
    for (auto* h : hs) prof_on = prof_on || h->profile != 0;
    IdProf prof;
    // doubles of ID workspace per launch (8 GiB): a whole level of a 2^20-point
    // problem fits, so each launch class fills the chip in one grid
    const int64_t WS_CAP = (int64_t)1 << 30;
    DBuf<int> d_xidx;
    DBuf<int64_t> d_xoff;
    DBuf<double> Mws, nuws;
    DBuf<IdTask> d_sw;
    for (int t = 0; t < maxd; ++t) {
        // units and levels of this round; grow piv / T first (the task
        // pointers must see the final buffers)
        int64_t xtot = 0;
        for (Unit& u : units) {
            Handle& h = *u.h;
            Basis& b = *u.b;
            u.L = h.maxdepth - t;
            if (u.L < 1) continue;
            u.xbase = xtot;
            const int64_t keep_piv = u.piv_total, keep_T = u.T_total;
            for (int i = h.lvl_ptr[u.L]; i < h.lvl_ptr[u.L + 1]; ++i) {
                int m = 0;
                if (h.h_nchild[i] == 0)
                    m = h.h_count[i];
                else
                    for (int c = h.h_first_child[i]; c < h.h_first_child[i] + h.h_nchild[i]; ++c) m += b.h_rank[c];
                b.h_mbar[i] = m;
                b.h_piv_off[i] = u.piv_total;
                b.h_T_off[i] = u.T_total;
                u.piv_total += m;
                u.T_total += (int64_t)m * std::min(m, (*u.ys_cnt)[i]);
                xtot += m;
            }
            b.piv.grow_keep((size_t)std::max<int64_t>(u.piv_total, 1), (size_t)keep_piv, s);
            b.T.grow_keep((size_t)std::max<int64_t>(u.T_total, 1), (size_t)keep_T, s);
        }
        if (xtot == 0) continue;
        // row sets of the round
        d_xidx.ensure((size_t)xtot, s);
        for (Unit& u : units) {
            Handle& h = *u.h;
            Basis& b = *u.b;
            if (u.L < 1) continue;
            const int lo = h.lvl_ptr[u.L], nl = h.lvl_ptr[u.L + 1] - lo;
            std::vector<int64_t> xo((size_t)nl + 1, 0);
            for (int q = 0; q < nl; ++q) xo[q + 1] = xo[q] + b.h_mbar[lo + q];
            for (auto& v : xo) v += u.xbase;
            d_xoff.ensure(xo.size(), s);
            H2_HIP(hipMemcpyAsync(d_xoff.p, xo.data(), xo.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
            k_xbar_fill<<<nl, TB, 0, s>>>(lo, h.nchild.p, h.first_child.p, h.start.p, h.count.p, b.rank.p, b.skel.p,
                                          h.ys_stride, d_xoff.p, d_xidx.p);
            H2_LAUNCH_CHECK();
            H2_HIP(hipStreamSynchronize(s));  // d_xoff is reused by the next unit
        }
        // tasks, launched in chunks of bounded workspace
        std::vector<IdTask> tasks;
        std::vector<int64_t> Moff, nuoff;
        int64_t ws = 0, no = 0;
        // workspace sizes rounded up to a power of two, so that builds of
        // different sizes reuse the same cached device blocks
        auto pow2 = [](int64_t v) {
            size_t c = 1;
            while (c < (size_t)v) c <<= 1;
            return c;
        };
        auto flush = [&]() {
            if (tasks.empty()) return;
            Mws.ensure(pow2(ws), s);
            nuws.ensure(pow2(no), s);
            for (size_t q = 0; q < tasks.size(); ++q) {
                tasks[q].M = Mws.p + Moff[q];
                tasks[q].nu = nuws.p + nuoff[q];
            }
            batched_id(tasks, s, prof_on ? &prof : nullptr);
            // strong rank-revealing swaps where a problem asks for them
            std::vector<IdTask> sw;
            size_t kmax = 1;
            for (const IdTask& t : tasks)
                if (t.srrqr_f > 1.0) {
                    sw.push_back(t);
                    kmax = std::max(kmax, (size_t)std::min(t.m, t.s));
                }
            if (!sw.empty()) {
                d_sw.ensure(sw.size(), s);
                H2_HIP(hipMemcpyAsync(d_sw.p, sw.data(), sw.size() * sizeof(IdTask), hipMemcpyHostToDevice, s));
                k_srrqr<<<(unsigned)sw.size(), TB, kmax * sizeof(double), s>>>(d_sw.p, (int)sw.size());
                H2_LAUNCH_CHECK();
                H2_HIP(hipStreamSynchronize(s));  // sw (host) is read by the copy
            }
            tasks.clear();
            Moff.clear();
            nuoff.clear();
            ws = 0;
            no = 0;
        };
        for (Unit& u : units) {
            Handle& h = *u.h;
            Basis& b = *u.b;
            if (u.L < 1) continue;
            int64_t xo = u.xbase;
            for (int i = h.lvl_ptr[u.L]; i < h.lvl_ptr[u.L + 1]; ++i) {
                const int m = b.h_mbar[i], sy = (*u.ys_cnt)[i];
                const int64_t need = (int64_t)m * sy;
                if (!tasks.empty() && ws + need > WS_CAP) flush();
                IdTask tk;
                tk.pts = h.pts.p;
                tk.ld = h.n;
                tk.x_idx = d_xidx.p + xo;
                tk.y_idx = h.ys_idx.p + (int64_t)i * h.ys_stride;
                tk.piv = b.piv.p + b.h_piv_off[i];
                tk.T = b.T.p + b.h_T_off[i];
                tk.skel = b.skel.p + (int64_t)i * h.ys_stride;
                tk.rank = b.rank.p + i;
                tk.prm = h.prm;
                tk.tol = h.tol_int;
                tk.m = m;
                tk.s = sy;
                tk.d = h.d;
                tk.kid = h.kid;
                tk.swap = u.swap;
                tk.srrqr_f = h.srrqr_f;
                tk.f32 = id_f32(h) ? 1 : 0;
                tasks.push_back(tk);
                Moff.push_back(ws);
                nuoff.push_back(no);
                ws += need;
                no += 3 * (int64_t)m;
                xo += m;
            }
        }
        flush();
        for (Unit& u : units) {
            Handle& h = *u.h;
            Basis& b = *u.b;
            if (u.L < 1) continue;
            const int lo = h.lvl_ptr[u.L], nl = h.lvl_ptr[u.L + 1] - lo;
            std::vector<int> rk = read_vec(b.rank.p + lo, nl, s);
            for (int q = 0; q < nl; ++q) b.h_rank[lo + q] = rk[q];
            if (prof_on)
                for (int q = 0; q < nl; ++q) {
                    const int i = lo + q;
                    const double f = id_flop_count((*u.ys_cnt)[i], b.h_mbar[i], rk[q]);
                    h.id_flops += f;
                    if (b.h_mbar[i] > 64) h.id_wide_flops += f;
                }
        }
    }
    for (Unit& u : units) {
        Handle& h = *u.h;
        Basis& b = *u.b;
        const int nn = h.nnode;
        b.h_piv_off[nn] = u.piv_total;
        b.h_T_off[nn] = u.T_total;
        upload(b.mbar, b.h_mbar, s);
        upload(b.piv_off, b.h_piv_off, s);
        upload(b.T_off, b.h_T_off, s);
        b.sum_rank = 0;
        for (int i = 0; i < nn; ++i) b.sum_rank += b.h_rank[i];
        b.bytes_T = u.T_total * (int64_t)sizeof(double);
        h.id_ms = prof.ms_all;  // launches shared by all problems of the call
        h.id_wide_ms = prof.ms_wide;
    }
    H2_HIP(hipStreamSynchronize(s));
}

void build_bases(Handle& h) { build_bases_multi({&h}, h.stream); }

}  // namespace h2
