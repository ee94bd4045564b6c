// Internal declarations shared by the HIP sources of the H^2 library.
// Nothing here is part of the public C ABI (see include/h2.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/h2.h"
#include "tuning.h"

namespace h2 {

// ------------------------------------------------------------------ errors
struct Error {
    int code;
    std::string msg;
};

#define H2_HIP(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::h2::Error{H2_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define H2_LAUNCH_CHECK() H2_HIP(hipGetLastError())

inline void fail(int code, const std::string& m) { throw Error{code, m}; }

// ------------------------------------------------------------------ device memory
// Device allocations go through a caching layer (alloc.hip): released
// blocks are kept and handed out again (small ones per power-of-two class,
// large ones to a request of a similar size), so that repeated builds pay
// neither for mapping ~100 GB of HBM nor for the device-wide
// synchronisation of hipFree.  A block reused on another stream than the one
// that released it is ordered after that stream's work by an event.  On
// allocation failure the cache is emptied and the allocation retried once; a
// second failure surfaces as H2_ENOMEM.  `s` is the stream that will use the
// block.
void* dev_alloc(size_t bytes, hipStream_t s);
// Returns a block; `s` is the stream whose work may still use it (waited for
// before the block can be handed out again).
void dev_free(void* p, size_t bytes, hipStream_t s);
// Releases every cached block back to the runtime.
void dev_cache_trim();
// While an IdleFree object lives on this thread, dev_free takes the released
// blocks as idle (the caller has waited for all work on them): they are
// reused without ordering against the stream that allocated them.
struct IdleFree {
    IdleFree();
    ~IdleFree();
};

// A plain owning device buffer.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) dev_free(p, n * sizeof(T), s);
        p = nullptr;
        n = 0;
    }
    // (Re)allocate to hold at least cnt elements; contents are not kept.
    void ensure(size_t cnt, hipStream_t stream = nullptr)
    {
        if (cnt <= n && p) return;
        release();
        s = stream;
        size_t c = cnt ? cnt : 1;
        p = (T*)dev_alloc(c * sizeof(T), stream);
        n = c;
    }
    // Grow to at least cnt elements keeping the first `keep` elements.
    void grow_keep(size_t cnt, size_t keep, hipStream_t stream)
    {
        if (cnt <= n && p) return;
        size_t nc = n ? n : 16;
        while (nc < cnt) nc *= 2;
        T* q = (T*)dev_alloc(nc * sizeof(T), stream);
        if (p && keep) H2_HIP(hipMemcpyAsync(q, p, keep * sizeof(T), hipMemcpyDeviceToDevice, stream));
        H2_HIP(hipStreamSynchronize(stream));
        release();
        s = stream;
        p = q;
        n = nc;
    }
};

template <class T>
inline T read_scalar(const T* dptr, hipStream_t s)
{
    T v;
    H2_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
    return v;
}

template <class T>
inline std::vector<T> read_vec(const T* dptr, size_t cnt, hipStream_t s)
{
    std::vector<T> v(cnt);
    if (cnt) {
        H2_HIP(hipMemcpyAsync(v.data(), dptr, cnt * sizeof(T), hipMemcpyDeviceToHost, s));
        H2_HIP(hipStreamSynchronize(s));
    }
    return v;
}

// Host vector -> device buffer (resized as needed); synchronises s, so the
// host vector may go out of scope on return.
template <class T>
inline void upload_vec(DBuf<T>& dst, const std::vector<T>& src, hipStream_t s)
{
    dst.ensure(src.size(), s);
    if (!src.empty())
        H2_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    H2_HIP(hipStreamSynchronize(s));
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ scan (scan.hip)
// Exclusive prefix sums.  out has cnt+1 entries; out[cnt] is the total.
// `tmp` is scratch resized as needed.  Deterministic (integer arithmetic).
void scan_excl_i32(const int* in, int* out, int64_t cnt, DBuf<int>& tmp, hipStream_t s);
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t cnt, DBuf<int64_t>& tmp, hipStream_t s);

// ------------------------------------------------------------------ handle
// Elements kept (zeroed) after the last coupling / nearfield block: a row
// tile of the apply reads up to 15 elements past the end of a block column.
constexpr int64_t BLK_PAD = 64;

// One side of the nested bases of Algorithm 2: per node the rank k, the row
// count m of its block (the points X_i of a leaf, else the children's
// skeletons), the pivots and T of the ID (U_i = P [I; T^T]), the skeleton
// points, and the offsets of the node's coefficients in xhat / yhat.
struct Basis {
    DBuf<int> rank, mbar;
    std::vector<int> h_rank, h_mbar;
    DBuf<int> skel;         // stride ys_stride: skeleton tree positions in pivot order
    DBuf<int64_t> piv_off;  // per node offset into piv
    DBuf<int> piv;          // per node m_i entries
    DBuf<int64_t> T_off;    // per node offset into T (row-major k x (m-k))
    DBuf<double> T;
    DBuf<float> Tf;         // precision mode: T in FP32
    std::vector<int64_t> h_piv_off, h_T_off;
    DBuf<int64_t> xh_off;   // per node offset (in units of rank) into xhat / yhat
    int64_t sum_rank = 0, bytes_T = 0;
};

struct Handle {
    // problem
    int64_t n = 0;
    int d = 0, kid = 0;
    double prm = 1.0;
    double tol = 1e-6;      // user tolerance eps
    double tol_int = 5e-7;  // construction tolerance eps' = eps / 2
    double tau = 0.7;
    int q = 64;
    int r1 = 0, r2 = 0, r_min = 0;
    int dr = H2_DR_VOLUME;  // DataReduct method of HiDR
    double srrqr_f = 0.0;   // > 1: strong rank-revealing swaps after every ID
    int precision = 64;
    int store_coupling = 1;
    uint64_t calib_seed = 0x5EED;
    // top-down DataReduct: levels with fewer nodes than this take 1024 lanes
    // per node; 0 for the problems below 2^18 points of a batched build,
    // which fill the device together
    int down_wide_nodes = H2_TUNE_DOWN_WIDE;
    hipStream_t stream = nullptr;

    // tree: nodes in BFS order (depth, parent, child code)
    int nnode = 0, maxdepth = 0;
    std::vector<int> lvl_ptr;  // host copy: nodes of depth L are lvl_ptr[L]..lvl_ptr[L+1]-1
    DBuf<int> parent, first_child, nchild, start, count, depth;
    DBuf<double> center;  // [cap][d]
    DBuf<double> side;
    DBuf<double> pts;  // [d][n] SoA, tree order
    DBuf<int> perm;    // tree position -> original index
    DBuf<int> iperm;   // original index -> tree position (the apply's gather and scatter)
    std::vector<int> h_nchild, h_first_child, h_start, h_count, h_parent;  // host mirrors (small)

    // lists (CSR, columns ascending)
    int64_t nil = 0, nnear = 0;
    DBuf<int> il_ptr, il_col, nr_ptr, nr_col;
    std::vector<int> h_il_ptr, h_nr_ptr;

    // HiDR representor sets, fixed stride per node
    DBuf<int> xs_cnt, xs_idx;  // stride r1
    DBuf<int> ys_cnt, ys_idx;  // stride ys_stride = r2 (the maximum size of Y_i^*)
    int ys_stride = 0;
    std::vector<int> calib_r;
    std::vector<double> calib_err;

    // bases: bu holds U and R (row side, the ID of K(Xbar_i, Y_i*)); for a
    // non-symmetric kernel bv holds V and W (column side, the ID of
    // K(Y_i*, Xbar_i)^T), otherwise V = U and bu serves both sides
    bool nonsym = false;
    Basis bu, bv;
    Basis& col() { return nonsym ? bv : bu; }

    // coupling and nearfield blocks
    DBuf<int64_t> B_off;  // per IL entry (CSR order), size nil+1
    // B_upper (symmetric kernel): blocks stored for the entries j > i only;
    // B_off of an entry j < i points at the stored B_ji (read transposed).
    // il_split[i]: first entry of row i with column > i.
    bool B_upper = false;
    DBuf<int> il_split;
    std::vector<int> h_il_split;
    DBuf<double> B;
    DBuf<int64_t> D_off;  // per near entry, size nnear+1
    DBuf<double> D;
    DBuf<float> Bf, Df;  // precision mode: FP32 blocks
    // skeleton coordinates (SoA [d][skc_ld], node offsets = the bases'
    // xh_off) and the apply's tasks (node, first row) when the apply
    // evaluates the coupling blocks itself (store_coupling = 0)
    DBuf<double> skc_u, skc_v;
    int64_t skc_ld_u = 1, skc_ld_v = 1;
    DBuf<int> otf_node, otf_r0;
    int n_otf = 0;
    DBuf<int> leaves;    // leaf node ids

    // apply task lists: (node, first row) of every 32-row chunk of a block
    // row, split by whether the chunk holds one or two 16-row tiles
    // A block sweep of the apply: tasks (node, first row) grouped by their
    // number of 16-row tiles (1..4), and per-entry metadata of the list.
    struct Sweep {
        DBuf<int> node[4], r0[4];
        int n[4] = {0, 0, 0, 0};
        DBuf<int> ek;       // per list entry: columns of the block
        DBuf<int64_t> ex;   // per list entry: first input row of the block
        DBuf<int> steps;    // per node: sum over its entries of max(1, ceil(columns / 4))
    };
    Sweep cp, nr;
    Sweep cpt;  // B_upper: the transposed (j < i) coupling entries
    DBuf<double> zeros;     // 64 zeros, read by masked lanes of the sweeps
    DBuf<int64_t> start64;  // start[] widened, row offsets of the leaves in x_t / y_t

    // matvec workspace (sized for the largest nrhs seen)
    int mv_ld = 0;  // column stride the apply buffers are sized for
    bool ready = true;  // false while (or after a failed) h2_rebuild
    hipEvent_t mv_done = nullptr;  // recorded after every apply (waited for at destroy)
    DBuf<double> xt, yt, xh, yh;
    DBuf<float> xtf, ytf, xhf, yhf;

    // optional per-sweep events of the last apply
    int profile = 0;
    bool prof_valid = false;
    int prof_nrhs = 0;
    hipEvent_t ev[7] = {};

    // diagnostics
    double t_tree = 0, t_lists = 0, t_calib = 0, t_hidr = 0, t_basis = 0, t_blocks = 0;
    int64_t bytes_B = 0, bytes_D = 0;
    // interpolative decompositions of the build (profile = 1): launch times
    // (ms) and the algorithmic floating-point operations of the IDs
    double id_ms = 0, id_wide_ms = 0, id_flops = 0, id_wide_flops = 0;
    // top-down DataReduct launches (profile = 1): time (ms) and the bytes of
    // the candidate coordinates they reduce (each T_i read once)
    double hidr_down_ms = 0, hidr_down_bytes = 0, hidr_down_evals = 0;

    // scratch
    DBuf<int> tmp_i32;
    DBuf<int64_t> tmp_i64;
};

// ------------------------------------------------------------------ phases
void build_tree(Handle& h, const double* pts_in);                // tree.hip
void build_lists(Handle& h);                                      // lists.hip
void run_calibration(Handle& h);                                  // calib.hip
void run_calibration_multi(const std::vector<Handle*>& hs, hipStream_t s);  // calib.hip
void run_hidr(Handle& h);                                         // hidr.hip
void build_bases(Handle& h);                                      // basis.hip
void build_bases_multi(const std::vector<Handle*>& hs, hipStream_t s);  // basis.hip
void build_blocks(Handle& h);                                     // blocks.hip
void prepare_apply(Handle& h);                                   // matvec.hip
void matvec(Handle& h, const void* x, void* y, int nrhs, hipStream_t s);  // matvec.hip
// The same apply on the library's per-device scratch array (no allocation;
// H2_EUNSUPPORTED when the work vectors exceed H2_NOALLOC_SCRATCH_BYTES).
void matvec_noalloc(Handle& h, const void* x, void* y, int nrhs, hipStream_t s);  // matvec.hip

// DataReduct over materialised index lists (hidr.hip); used by HiDR and by
// the calibration.  For each of `nlist` lists (indices into the SoA point
// array pts with leading dimension ld), writes up to k selected indices to
// out[list * out_stride ...] and the count to out_cnt[list].
// `split` (may be NULL) gives, per list, the length of its first part: the
// reference set then holds one grid per non-empty part.
void datareduct_lists(const double* pts, int64_t ld, int d, const int64_t* list_off, const int* list_idx,
                      const int* split, int nlist, int k, int* out, int out_stride, int* out_cnt, hipStream_t s);
// The same with the DataReduct method of Section 3.3 (H2_DR_*): the volume
// method as above, farthest point sampling (split ignored: the list is taken
// whole) or the surface method (one reference set per part).
void datareduct_lists_method(int method, const double* pts, int64_t ld, int d, const int64_t* list_off,
                             const int* list_idx, const int* split, int nlist, int k, int* out, int out_stride,
                             int* out_cnt, hipStream_t s);

// Batched ID (basis.hip): one problem per entry.  Problem p has rows X
// (m_p indices into pts) and columns Y (s_p indices into pts2); the kernel
// matrix is evaluated and compressed with the column-pivoted QR rule.
// One ID problem (a node of a level, or a calibration set): the candidate
// points x_idx[0..m) and reference points y_idx[0..s) index the SoA point
// array pts ([d][ld]); outputs go to absolute device addresses, so one batch
// may hold nodes of many independent problems.
struct IdTask {
    const double* pts = nullptr;
    int64_t ld = 0;
    const int* x_idx = nullptr;  // m entries
    const int* y_idx = nullptr;  // s entries
    double* M = nullptr;         // workspace, s*m doubles (unless the block fits LDS)
    double* nu = nullptr;        // workspace, 3*m doubles
    int* piv = nullptr;          // m entries
    double* T = nullptr;         // k*(m-k) entries
    int* skel = nullptr;         // k entries (x indices)
    int* rank = nullptr;         // 1 entry
    double prm = 1.0, tol = 0.0;
    double srrqr_f = 0.0;  // > 1: swaps bounding max |T| by it after the ID
    int m = 0, s = 0, d = 0, kid = 0;
    int swap = 0;    // 1: column side, entries kappa(y_r, x_c) instead of kappa(x_c, y_r)
    int f32 = 0;     // 1: FP32 kernel entries and Householder updates (FP64 norms and T)
    int folded = 0;  // set by batched_id: M holds the m x m R factor of the block
};
// HIP-event time (ms) of batched_id's launches: all classes, and the class of
// the wide nodes (m > 64), accumulated over calls.
// The precision mode's decompositions run in FP32 (kernel entries,
// Householder updates; FP64 column norms, down-dates and T) when the
// tolerance leaves room for FP32 rounding: eps >= 1e-5.  Each Householder
// step rounds every updated entry to FP32, and over the hundreds of steps of
// a wide block that noise reaches the truncation level of eps = 1e-6 (there
// the n = 2^20 Coulomb product came out 1.2e-6 from the dense one, against
// 0.6e-6 with FP64 decompositions); below 1e-5 the decompositions stay FP64.
inline bool id_f32(const Handle& h) { return h.precision == 32 && h.tol >= 1e-5; }

struct IdProf {
    double ms_all = 0, ms_wide = 0;
};
void batched_id(const std::vector<IdTask>& tasks, hipStream_t s, IdProf* prof = nullptr);

}  // namespace h2
