// C ABI (include/h2.h): argument checks, the build pipeline of Algorithm 2
// (tree -> lists -> r1/r2 -> HiDR -> nested bases -> coupling/near blocks),
// the apply, queries and exports.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <thread>

#include "common.h"

struct h2_handle_s {
    h2::Handle h;
};

namespace {

thread_local std::string g_last_error;

h2_status set_err(int code, const std::string& msg)
{
    g_last_error = msg;
    return (h2_status)code;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}



// Worker streams of the batched build: created once, kept for the life of
// the process (buffers allocated on them remember them), default priority,
// not synchronising with the null stream.
constexpr int NWORK = 8;
hipStream_t worker_stream(int w)
{
    static std::mutex mu;
    static hipStream_t st[NWORK] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (!st[w]) H2_HIP(hipStreamCreateWithFlags(&st[w], hipStreamNonBlocking));
    return st[w];
}

// Argument checks and the handle's problem parameters (h2_build_ex and
// h2_build_batched).
h2_status check_and_init(h2::Handle& h, const double* points, int64_t n, int dim, int kernel_id,
                         const double* params, double tol, int leaf_size, const h2_options& opt, hipStream_t s)
{
    if (!points) return set_err(H2_EINVAL, "points is NULL");
    if (n < 1 || n > (int64_t)INT32_MAX) return set_err(H2_EINVAL, "n must be in [1, 2^31)");
    if (dim < 1 || dim > 3) return set_err(H2_EINVAL, "dim must be 1, 2 or 3");
    if (kernel_id < H2_COULOMB || kernel_id > H2_ADVECTION) return set_err(H2_EINVAL, "unknown kernel_id");
    if (!(tol > 0.0 && tol < 1.0)) return set_err(H2_EINVAL, "tol must be in (0, 1)");
    if (leaf_size < 1) return set_err(H2_EINVAL, "leaf_size must be >= 1");
    if (!(opt.tau > 0.0 && opt.tau < 1.0)) return set_err(H2_EINVAL, "tau must be in (0, 1)");
    if (opt.r1 < 0 || opt.r1 > 2048) return set_err(H2_EINVAL, "r1 must be in [0, 2048]");
    if (opt.r2 < 0 || opt.r2 == 1 || opt.r2 > 4096) return set_err(H2_EINVAL, "r2 must be 0 or in [2, 4096]");
    if (opt.precision != 64 && opt.precision != 32) return set_err(H2_EINVAL, "precision must be 64 or 32");
    if (opt.r_min < 0 || opt.r_min > 2048) return set_err(H2_EINVAL, "r_min must be in [0, 2048]");
    if (opt.datareduct < H2_DR_VOLUME || opt.datareduct > H2_DR_SURFACE)
        return set_err(H2_EINVAL, "unknown DataReduct method");
    if (opt.srrqr_f != 0.0 && !(opt.srrqr_f > 1.0 && opt.srrqr_f <= 1e6))
        return set_err(H2_EINVAL, "srrqr_f must be 0 or in (1, 1e6]");
    if (opt.store_coupling != 0 && opt.store_coupling != 1) return set_err(H2_EINVAL, "store_coupling must be 0 or 1");
    if (opt.store_coupling == 0 && opt.precision != 64)
        return set_err(H2_EUNSUPPORTED, "coupling blocks evaluated in the apply need precision 64");
    if ((kernel_id == H2_COSINE || kernel_id == H2_ADVECTION) && (opt.r1 == 0 || opt.r2 == 0))
        return set_err(H2_EINVAL, "the cosine and advection kernels need options.r1 and options.r2 (no calibration)");
    double prm = 1.0;
    if (kernel_id != H2_COULOMB) {
        if (!params) return set_err(H2_EINVAL, "params is NULL");
        prm = params[0];
        if (!(std::isfinite(prm) && prm > 0.0)) return set_err(H2_EINVAL, "params[0] must be finite and > 0");
    }
    h.n = n;
    h.d = dim;
    h.kid = kernel_id;
    h.nonsym = kernel_id == H2_ADVECTION;
    h.prm = prm;
    h.tol = tol;
    h.tol_int = 0.5 * tol;  // eps' = eps/2 for truncation and calibration
    h.tau = opt.tau;
    h.q = leaf_size;
    h.r1 = opt.r1;
    h.r2 = opt.r2;
    h.precision = opt.precision;
    h.store_coupling = opt.store_coupling;
    h.calib_seed = opt.calib_seed;
    h.profile = opt.profile;
    h.r_min = opt.r_min;
    h.dr = opt.datareduct;
    h.srrqr_f = opt.srrqr_f;
    h.stream = s;
    return H2_OK;
}

// Algorithm 2, first steps: tree and lists.
void build_tree_lists(h2::Handle& h, const double* points)
{
    double t0 = now_s();
    h2::build_tree(h, points);
    H2_HIP(hipStreamSynchronize(h.stream));
    double t1 = now_s();
    h2::build_lists(h);
    H2_HIP(hipStreamSynchronize(h.stream));
    double t2 = now_s();
    h.t_tree = t1 - t0;
    h.t_lists = t2 - t1;
}

// HiDR (after r1, r2 are known).
void build_hidr(h2::Handle& h)
{
    double t0 = now_s();
    h2::run_hidr(h);
    h.t_hidr = now_s() - t0;
}

// After the nested bases: coupling and nearfield blocks, apply preparation.
void build_back(h2::Handle& h)
{
    double t5 = now_s();
    h2::build_blocks(h);
    double t6 = now_s();
    std::vector<int> leaves;
    for (int i = 0; i < h.nnode; ++i)
        if (h.h_nchild[i] == 0) leaves.push_back(i);
    upload_vec(h.leaves, leaves, h.stream);
    for (h2::Basis* b : {&h.bu, &h.bv}) {
        if (b == &h.bv && !h.nonsym) break;
        std::vector<int64_t> xo((size_t)h.nnode + 1, 0);
        for (int i = 0; i < h.nnode; ++i) xo[i + 1] = xo[i] + b->h_rank[i];
        upload_vec(b->xh_off, xo, h.stream);
    }
    h2::prepare_apply(h);
    // marks the end of the last apply (h2_destroy and h2_rebuild wait for it)
    if (!h.mv_done) H2_HIP(hipEventCreateWithFlags(&h.mv_done, hipEventDisableTiming));
    h.t_blocks = t6 - t5;
}

}  // namespace

extern "C" {

void h2_options_default(h2_options* opt)
{
    if (!opt) return;
    opt->tau = 0.7;
    opt->r1 = 0;
    opt->r2 = 0;
    opt->precision = 64;
    opt->store_coupling = 1;
    opt->calib_seed = 0x5EED;
    opt->profile = 0;
    opt->r_min = 0;
    opt->datareduct = H2_DR_VOLUME;
    opt->srrqr_f = 0.0;
}

const char* h2_last_error(void) { return g_last_error.c_str(); }

h2_status h2_build(const double* points, int64_t n, int dim, int kernel_id, const double* params, double tol,
                   int leaf_size, h2_handle* out)
{
    return h2_build_ex(points, n, dim, kernel_id, params, tol, leaf_size, nullptr, nullptr, out);
}

h2_status h2_build_ex(const double* points, int64_t n, int dim, int kernel_id, const double* params, double tol,
                      int leaf_size, const h2_options* opt_in, void* hip_stream, h2_handle* out)
{
    if (!out) return set_err(H2_EINVAL, "out is NULL");
    *out = nullptr;
    h2_options opt;
    h2_options_default(&opt);
    if (opt_in) opt = *opt_in;
    h2_handle_s* hs = new (std::nothrow) h2_handle_s();
    if (!hs) return set_err(H2_ENOMEM, "host allocation failed");
    h2::Handle& h = hs->h;
    h2_status st = check_and_init(h, points, n, dim, kernel_id, params, tol, leaf_size, opt, (hipStream_t)hip_stream);
    if (st != H2_OK) {
        delete hs;
        return st;
    }
    try {
        // The scale-invariant Coulomb kernel is calibrated at side 1 whatever
        // the points: that calibration runs from a second host thread on a
        // worker stream while the tree and the lists are built.
        if (h.kid == H2_COULOMB && !(h.r1 > 0 && h.r2 > 0)) {
            h2::Handle c;
            c.d = h.d;
            c.kid = h.kid;
            c.prm = h.prm;
            c.tol = h.tol;
            c.tol_int = h.tol_int;
            c.tau = h.tau;
            c.r1 = h.r1;
            c.r2 = h.r2;
            c.r_min = h.r_min;
            c.calib_seed = h.calib_seed;
            int dev = 0;
            H2_HIP(hipGetDevice(&dev));
            std::exception_ptr cerr;
            double tc = 0.0;
            std::thread th([&]() {
                try {
                    H2_HIP(hipSetDevice(dev));
                    const double t0 = now_s();
                    h2::run_calibration_multi({&c}, worker_stream(0));
                    tc = now_s() - t0;
                } catch (...) {
                    cerr = std::current_exception();
                }
            });
            try {
                build_tree_lists(h, points);
            } catch (...) {
                th.join();
                throw;
            }
            th.join();
            if (cerr) std::rethrow_exception(cerr);
            h.calib_r.assign((size_t)h.maxdepth + 1, c.calib_r[0]);
            h.calib_err.assign((size_t)h.maxdepth + 1, c.calib_err[0]);
            h.r1 = c.r1;
            h.r2 = c.r2;
            h.t_calib = tc;
        } else {
            build_tree_lists(h, points);
            double t0 = now_s();
            h2::run_calibration(h);
            h.t_calib = now_s() - t0;
        }
        build_hidr(h);
        const double t0 = now_s();
        h2::build_bases(h);
        h.t_basis = now_s() - t0;
        build_back(h);
    } catch (const h2::Error& e) {
        delete hs;
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        delete hs;
        return set_err(H2_ENOMEM, "host allocation failed");
    }
    *out = hs;
    return H2_OK;
}

h2_status h2_rebuild(h2_handle hd, int kernel_id, const double* params, double tol)
{
    if (!hd) return set_err(H2_EINVAL, "handle is NULL");
    if (kernel_id < H2_COULOMB || kernel_id > H2_ADVECTION) return set_err(H2_EINVAL, "unknown kernel_id");
    if (!(tol > 0.0 && tol < 1.0)) return set_err(H2_EINVAL, "tol must be in (0, 1)");
    double prm = 1.0;
    if (kernel_id != H2_COULOMB) {
        if (!params) return set_err(H2_EINVAL, "params is NULL");
        prm = params[0];
        if (!(std::isfinite(prm) && prm > 0.0)) return set_err(H2_EINVAL, "params[0] must be finite and > 0");
    }
    h2::Handle& h = hd->h;
    try {
        // the buffers an apply in flight reads are about to be replaced
        if (h.mv_done) H2_HIP(hipEventSynchronize(h.mv_done));
        H2_HIP(hipStreamSynchronize(h.stream));
        h.ready = false;
        h.kid = kernel_id;
        h.nonsym = kernel_id == H2_ADVECTION;
        h.prm = prm;
        h.tol = tol;
        h.tol_int = 0.5 * tol;
        h.mv_ld = 0;  // the apply workspace follows the new ranks
        h.prof_valid = false;
        h.id_ms = h.id_wide_ms = h.id_flops = h.id_wide_flops = 0;
        double t0 = now_s();
        h2::build_bases(h);
        h.t_basis = now_s() - t0;
        build_back(h);
        h.ready = true;
    } catch (const h2::Error& e) {
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return set_err(H2_ENOMEM, "host allocation failed");
    }
    return H2_OK;
}

h2_status h2_build_batched(int nprob, const double* const* points, const int64_t* n, const int* dim,
                           const int* kernel_id, const double* params, const double* tol, const int* leaf_size,
                           const h2_options* opt_in, void* hip_stream, h2_handle* out)
{
    if (!out) return set_err(H2_EINVAL, "out is NULL");
    if (nprob < 1) return set_err(H2_EINVAL, "nprob must be >= 1");
    for (int p = 0; p < nprob; ++p) out[p] = nullptr;
    if (!points || !n || !dim || !kernel_id || !params || !tol || !leaf_size)
        return set_err(H2_EINVAL, "an argument array is NULL");
    h2_options opt;
    h2_options_default(&opt);
    if (opt_in) opt = *opt_in;
    std::vector<h2_handle_s*> hs(nprob, nullptr);
    auto cleanup = [&]() {
        for (auto* x : hs) delete x;
    };
    for (int p = 0; p < nprob; ++p) {
        hs[p] = new (std::nothrow) h2_handle_s();
        if (!hs[p]) {
            cleanup();
            return set_err(H2_ENOMEM, "host allocation failed");
        }
        h2_status st = check_and_init(hs[p]->h, points[p], n[p], dim[p], kernel_id[p], params + p, tol[p],
                                      leaf_size[p], opt, (hipStream_t)hip_stream);
        if (st != H2_OK) {
            std::string msg = "problem " + std::to_string(p) + ": " + g_last_error;
            cleanup();
            return set_err(st, msg);
        }
    }
    try {
        const hipStream_t us = (hipStream_t)hip_stream;
        std::vector<h2::Handle*> hv(nprob);
        for (int p = 0; p < nprob; ++p) {
            hv[p] = &hs[p]->h;
            // small problems fill the device together: their top-down
            // DataReduct keeps 256 lanes per node at every level
            if (n[p] < (int64_t)1 << 18) hv[p]->down_wide_nodes = 0;
        }
        // the per-problem steps (many small launches and read-backs each) run
        // concurrently: problem p on worker p % W, each worker with its own
        // stream, ordered after the caller's stream; the shared steps run on
        // the caller's stream after all workers finished
        const int W = std::min(nprob, NWORK);
        std::vector<hipStream_t> ws(W);
        for (int w = 0; w < W; ++w) ws[w] = worker_stream(w);
        hipEvent_t ready = nullptr;
        H2_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        H2_HIP(hipEventRecord(ready, us));
        for (int w = 0; w < W; ++w) H2_HIP(hipStreamWaitEvent(ws[w], ready, 0));
        H2_HIP(hipEventSynchronize(ready));
        (void)hipEventDestroy(ready);
        auto parallel = [&](auto&& fn) {
            int dev = 0;
            H2_HIP(hipGetDevice(&dev));
            std::vector<std::exception_ptr> errs(W);
            std::vector<std::thread> th;
            for (int w = 0; w < W; ++w)
                th.emplace_back([&, w]() {
                    try {
                        H2_HIP(hipSetDevice(dev));
                        for (int p = w; p < nprob; p += W) {
                            hv[p]->stream = ws[w];
                            fn(p);
                        }
                        H2_HIP(hipStreamSynchronize(ws[w]));
                    } catch (...) {
                        errs[w] = std::current_exception();
                    }
                });
            for (auto& t : th) t.join();
            for (int p = 0; p < nprob; ++p) hv[p]->stream = us;
            for (auto& e : errs)
                if (e) std::rethrow_exception(e);
        };
        parallel([&](int p) { build_tree_lists(*hv[p], points[p]); });
        double t0 = now_s();
        h2::run_calibration_multi(hv, us);
        const double tc = now_s() - t0;
        parallel([&](int p) {
            hv[p]->t_calib = tc;
            build_hidr(*hv[p]);
        });
        t0 = now_s();
        h2::build_bases_multi(hv, us);
        const double tb = now_s() - t0;
        parallel([&](int p) {
            hv[p]->t_basis = tb;
            build_back(*hv[p]);
        });
    } catch (const h2::Error& e) {
        cleanup();
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        cleanup();
        return set_err(H2_ENOMEM, "host allocation failed");
    }
    for (int p = 0; p < nprob; ++p) out[p] = hs[p];
    return H2_OK;
}

h2_status h2_matvec(h2_handle hd, const void* x, void* y, int nrhs)
{
    return h2_matvec_ex(hd, x, y, nrhs, hd ? (void*)hd->h.stream : nullptr);
}

// Checks shared by the apply entry points.
static h2_status check_apply(h2_handle hd, const void* x, const void* y, int nrhs)
{
    if (!hd) return set_err(H2_EINVAL, "handle is NULL");
    if (!x || !y) return set_err(H2_EINVAL, "x or y is NULL");
    if (!hd->h.ready) return set_err(H2_EINVAL, "the handle holds no representation (a rebuild failed)");
    if (nrhs < 1 || nrhs > 256) return set_err(H2_EINVAL, "nrhs must be in [1, 256]");
    const h2::Handle& h = hd->h;
    const size_t bytes = (size_t)h.n * nrhs * (h.precision == 32 ? sizeof(float) : sizeof(double));
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + bytes <= yb || yb + bytes <= xb)) return set_err(H2_EINVAL, "x and y overlap");
    return H2_OK;
}

h2_status h2_matvec_noalloc(h2_handle hd, const void* x, void* y, int nrhs, void* hip_stream)
{
    const h2_status st = check_apply(hd, x, y, nrhs);
    if (st != H2_OK) return st;
    h2::Handle& h = hd->h;
    try {
        hipStream_t ms = (hipStream_t)hip_stream;
        h2::matvec_noalloc(h, x, y, nrhs, ms);
        // created with the handle, so recording allocates nothing
        if (h.mv_done) H2_HIP(hipEventRecord(h.mv_done, ms));
    } catch (const h2::Error& e) {
        return set_err(e.code, e.msg);
    }
    return H2_OK;
}

h2_status h2_matvec_ex(h2_handle hd, const void* x, void* y, int nrhs, void* hip_stream)
{
    const h2_status st = check_apply(hd, x, y, nrhs);
    if (st != H2_OK) return st;
    h2::Handle& h = hd->h;
    try {
        hipStream_t ms = (hipStream_t)hip_stream;
        h2::matvec(h, x, y, nrhs, ms);
        if (!h.mv_done) H2_HIP(hipEventCreateWithFlags(&h.mv_done, hipEventDisableTiming));
        H2_HIP(hipEventRecord(h.mv_done, ms));
    } catch (const h2::Error& e) {
        return set_err(e.code, e.msg);
    }
    return H2_OK;
}

h2_status h2_query(h2_handle hd, h2_info* info)
{
    if (!hd || !info) return set_err(H2_EINVAL, "NULL argument");
    h2::Handle& h = hd->h;
    std::memset(info, 0, sizeof(*info));
    info->n = h.n;
    info->dim = h.d;
    info->kernel_id = h.kid;
    info->nnode = h.nnode;
    info->maxdepth = h.maxdepth;
    int nleaf = 0, maxr = 0;
    for (int i = 0; i < h.nnode; ++i) {
        nleaf += h.h_nchild[i] == 0;
        maxr = std::max(maxr, h.bu.h_rank[i]);
    }
    info->nleaf = nleaf;
    info->r1 = h.r1;
    info->r2 = h.r2;
    info->nnz_il = h.nil;
    info->nnz_near = h.nnear;
    info->max_rank = maxr;
    info->sum_rank = h.bu.sum_rank;
    info->bytes_U = h.bu.bytes_T;
    info->nonsymmetric = h.nonsym ? 1 : 0;
    for (int i = 0; i < h.nnode; ++i) info->max_rank_v = std::max(info->max_rank_v, h.col().h_rank[i]);
    info->sum_rank_v = h.col().sum_rank;
    info->bytes_V = h.nonsym ? h.bv.bytes_T : 0;
    info->bytes_B = h.bytes_B;
    info->bytes_D = h.bytes_D;
    info->precision = h.precision;
    info->t_tree = h.t_tree;
    info->t_lists = h.t_lists;
    info->t_calib = h.t_calib;
    info->t_hidr = h.t_hidr;
    info->t_basis = h.t_basis;
    info->t_blocks = h.t_blocks;
    if (h.prof_valid) {
        float ms[6];
        if (hipEventSynchronize(h.ev[6]) != hipSuccess) return set_err(H2_EDEVICE, "event wait failed");
        for (int e = 0; e < 6; ++e)
            if (hipEventElapsedTime(&ms[e], h.ev[e], h.ev[e + 1]) != hipSuccess)
                return set_err(H2_EDEVICE, "event timing failed");
        info->mv_gather = ms[0];
        info->mv_upward = ms[1];
        info->mv_coupling = ms[2];
        info->mv_downward = ms[3];
        info->mv_leaves = ms[4];
        info->mv_scatter = ms[5];
        info->mv_nrhs = h.prof_nrhs;
    }
    info->id_ms = h.id_ms;
    info->id_wide_ms = h.id_wide_ms;
    info->id_flops = h.id_flops;
    info->id_wide_flops = h.id_wide_flops;
    info->hidr_down_ms = h.hidr_down_ms;
    info->hidr_down_bytes = h.hidr_down_bytes;
    info->hidr_down_evals = h.hidr_down_evals;
    return H2_OK;
}

h2_status h2_export(h2_handle hd, int what, int node, void* host_buf, size_t bytes, int64_t* count)
{
    if (!hd) return set_err(H2_EINVAL, "handle is NULL");
    h2::Handle& h = hd->h;
    hipStream_t s = h.stream;
    const void* src = nullptr;
    int64_t cnt = 0;
    size_t esz = 4;
    std::vector<int> tmp_i;
    auto node_ok = [&]() { return node >= 0 && node < h.nnode; };
    try {
        switch (what) {
        case H2_EXP_PERM: src = h.perm.p; cnt = h.n; break;
        case H2_EXP_PARENT: src = h.parent.p; cnt = h.nnode; break;
        case H2_EXP_FIRST_CHILD: src = h.first_child.p; cnt = h.nnode; break;
        case H2_EXP_NCHILD: src = h.nchild.p; cnt = h.nnode; break;
        case H2_EXP_START: src = h.start.p; cnt = h.nnode; break;
        case H2_EXP_COUNT: src = h.count.p; cnt = h.nnode; break;
        case H2_EXP_DEPTH: src = h.depth.p; cnt = h.nnode; break;
        case H2_EXP_CENTER: src = h.center.p; cnt = (int64_t)h.nnode * h.d; esz = 8; break;
        case H2_EXP_SIDE: src = h.side.p; cnt = h.nnode; esz = 8; break;
        case H2_EXP_IL_PTR: src = h.il_ptr.p; cnt = h.nnode + 1; break;
        case H2_EXP_IL_COL: src = h.il_col.p; cnt = h.nil; break;
        case H2_EXP_NEAR_PTR: src = h.nr_ptr.p; cnt = h.nnode + 1; break;
        case H2_EXP_NEAR_COL: src = h.nr_col.p; cnt = h.nnear; break;
        case H2_EXP_XSTAR:
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            cnt = h2::read_scalar(h.xs_cnt.p + node, s);
            src = h.xs_idx.p + (int64_t)node * h.r1;
            break;
        case H2_EXP_YSTAR:
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            cnt = h2::read_scalar(h.ys_cnt.p + node, s);
            src = h.ys_idx.p + (int64_t)node * h.ys_stride;
            break;
        case H2_EXP_RANK:
        case H2_EXP_RANK_V: src = (what == H2_EXP_RANK ? h.bu : h.col()).rank.p; cnt = h.nnode; break;
        case H2_EXP_MBAR:
        case H2_EXP_MBAR_V: src = (what == H2_EXP_MBAR ? h.bu : h.col()).mbar.p; cnt = h.nnode; break;
        case H2_EXP_PIV:
        case H2_EXP_PIV_V: {
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            const h2::Basis& b = what == H2_EXP_PIV ? h.bu : h.col();
            cnt = b.h_mbar[node];
            src = b.piv.p + b.h_piv_off[node];
            break;
        }
        case H2_EXP_SKEL:
        case H2_EXP_SKEL_V: {
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            const h2::Basis& b = what == H2_EXP_SKEL ? h.bu : h.col();
            cnt = b.h_rank[node];
            src = b.skel.p + (int64_t)node * h.ys_stride;
            break;
        }
        case H2_EXP_T:
        case H2_EXP_T_V: {
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            const h2::Basis& b = what == H2_EXP_T ? h.bu : h.col();
            cnt = (int64_t)b.h_rank[node] * (b.h_mbar[node] - b.h_rank[node]);
            src = b.T.p + b.h_T_off[node];
            esz = 8;
            break;
        }
        case H2_EXP_POINTS: src = h.pts.p; cnt = h.n * h.d; esz = 8; break;
        case H2_EXP_B: {
            if (node < 0 || node >= h.nil) return set_err(H2_EINVAL, "IL entry out of range");
            if (h.precision != 64) return set_err(H2_EUNSUPPORTED, "B export needs precision 64");
            if (h.store_coupling == 0) return set_err(H2_EUNSUPPORTED, "coupling blocks are not stored");
            // B_ij of entry e = (i, j), rank_i x rank_j column-major; an entry
            // j < i of a symmetric kernel reads the stored B_ji transposed
            const int i = (int)(std::upper_bound(h.h_il_ptr.begin(), h.h_il_ptr.end(), (int)node) -
                                h.h_il_ptr.begin()) - 1;
            int j = 0;
            int64_t o = 0;
            H2_HIP(hipMemcpy(&j, h.il_col.p + node, sizeof(int), hipMemcpyDeviceToHost));
            H2_HIP(hipMemcpy(&o, h.B_off.p + node, sizeof(int64_t), hipMemcpyDeviceToHost));
            const int ki = h.bu.h_rank[i], kj = h.col().h_rank[j];
            cnt = (int64_t)ki * kj;
            if (count) *count = cnt;
            if (!host_buf) return H2_OK;
            if (bytes < (size_t)cnt * 8) return set_err(H2_EINVAL, "buffer too small");
            if (cnt == 0) return H2_OK;
            H2_HIP(hipStreamSynchronize(s));
            std::vector<double> blk((size_t)cnt);
            H2_HIP(hipMemcpy(blk.data(), h.B.p + o, (size_t)cnt * 8, hipMemcpyDeviceToHost));
            double* outp = (double*)host_buf;
            if (h.B_upper && j < i) {
                for (int u = 0; u < kj; ++u)
                    for (int t = 0; t < ki; ++t) outp[(size_t)u * ki + t] = blk[(size_t)t * kj + u];
            } else {
                std::memcpy(outp, blk.data(), (size_t)cnt * 8);
            }
            return H2_OK;
        }
        case H2_EXP_CALIB_R:
            cnt = (int64_t)h.calib_r.size();
            if (count) *count = cnt;
            if (!host_buf) return H2_OK;
            if (bytes < (size_t)cnt * 4) return set_err(H2_EINVAL, "buffer too small");
            std::memcpy(host_buf, h.calib_r.data(), (size_t)cnt * 4);
            return H2_OK;
        default: return set_err(H2_EINVAL, "unknown export id");
        }
        if (count) *count = cnt;
        if (!host_buf) return H2_OK;
        if (bytes < (size_t)cnt * esz) return set_err(H2_EINVAL, "buffer too small");
        if (cnt > 0) {
            H2_HIP(hipStreamSynchronize(s));
            H2_HIP(hipMemcpy(host_buf, src, (size_t)cnt * esz, hipMemcpyDeviceToHost));
        }
    } catch (const h2::Error& e) {
        return set_err(e.code, e.msg);
    }
    return H2_OK;
}

h2_status h2_destroy(h2_handle hd)
{
    if (!hd) return H2_OK;
    // the build finished before it returned; wait for the last apply only
    // (not for whatever else its stream is running), then release the
    // buffers as idle
    if (hd->h.mv_done) (void)hipEventSynchronize(hd->h.mv_done);
    for (auto& e : hd->h.ev)
        if (e) (void)hipEventDestroy(e);
    hipEvent_t md = hd->h.mv_done;
    {
        h2::IdleFree idle;
        delete hd;
    }
    if (md) (void)hipEventDestroy(md);
    return H2_OK;
}

}  // extern "C"
