// C ABI (include/h2.h): argument checks, the build pipeline of Algorithm 2
// (tree -> lists -> r1/r2 -> HiDR -> nested bases -> coupling/near blocks),
// the apply, queries and exports.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

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

template <class T>
void upload_vec(h2::DBuf<T>& dst, const std::vector<T>& src, hipStream_t s)
{
    dst.ensure(src.size(), s);
    if (!src.empty())
        H2_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    H2_HIP(hipStreamSynchronize(s));
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
    if (!points) return set_err(H2_EINVAL, "points is NULL");
    if (n < 1 || n > (int64_t)INT32_MAX) return set_err(H2_EINVAL, "n must be in [1, 2^31)");
    if (dim < 1 || dim > 3) return set_err(H2_EINVAL, "dim must be 1, 2 or 3");
    if (kernel_id < H2_COULOMB || kernel_id > H2_MATERN32) return set_err(H2_EINVAL, "unknown kernel_id");
    if (!(tol > 0.0 && tol < 1.0)) return set_err(H2_EINVAL, "tol must be in (0, 1)");
    if (leaf_size < 1) return set_err(H2_EINVAL, "leaf_size must be >= 1");
    if (!(opt.tau > 0.0 && opt.tau < 1.0)) return set_err(H2_EINVAL, "tau must be in (0, 1)");
    if (opt.r1 < 0 || opt.r2 < 0 || opt.r1 > 2048 || opt.r2 > 2048)
        return set_err(H2_EINVAL, "r1, r2 must be in [0, 2048]");
    if (opt.precision != 64 && opt.precision != 32) return set_err(H2_EINVAL, "precision must be 64 or 32");
    if (opt.r_min < 0 || opt.r_min > 2048) return set_err(H2_EINVAL, "r_min must be in [0, 2048]");
    if (opt.store_coupling != 1) return set_err(H2_EUNSUPPORTED, "only stored coupling blocks are implemented");
    double prm = 1.0;
    if (kernel_id != H2_COULOMB) {
        if (!params) return set_err(H2_EINVAL, "params is NULL");
        prm = params[0];
        if (!(std::isfinite(prm) && prm > 0.0)) return set_err(H2_EINVAL, "params[0] must be finite and > 0");
    }
    h2_handle_s* hs = new (std::nothrow) h2_handle_s();
    if (!hs) return set_err(H2_ENOMEM, "host allocation failed");
    h2::Handle& h = hs->h;
    h.n = n;
    h.d = dim;
    h.kid = kernel_id;
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
    h.stream = (hipStream_t)hip_stream;
    try {
        double t0 = now_s();
        h2::build_tree(h, points);
        H2_HIP(hipStreamSynchronize(h.stream));
        double t1 = now_s();
        h2::build_lists(h);
        H2_HIP(hipStreamSynchronize(h.stream));
        double t2 = now_s();
        h2::run_calibration(h);
        double t3 = now_s();
        h2::run_hidr(h);
        double t4 = now_s();
        h2::build_bases(h);
        double t5 = now_s();
        h2::build_blocks(h);
        double t6 = now_s();
        // leaves and coefficient offsets for the apply
        std::vector<int> leaves;
        for (int i = 0; i < h.nnode; ++i)
            if (h.h_nchild[i] == 0) leaves.push_back(i);
        upload_vec(h.leaves, leaves, h.stream);
        std::vector<int64_t> xo((size_t)h.nnode + 1, 0);
        for (int i = 0; i < h.nnode; ++i) xo[i + 1] = xo[i] + h.h_rank[i];
        upload_vec(h.xh_off, xo, h.stream);
        h2::prepare_apply(h);
        h.t_tree = t1 - t0;
        h.t_lists = t2 - t1;
        h.t_calib = t3 - t2;
        h.t_hidr = t4 - t3;
        h.t_basis = t5 - t4;
        h.t_blocks = t6 - t5;
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

h2_status h2_matvec(h2_handle hd, const void* x, void* y, int nrhs)
{
    return h2_matvec_ex(hd, x, y, nrhs, hd ? (void*)hd->h.stream : nullptr);
}

h2_status h2_matvec_ex(h2_handle hd, const void* x, void* y, int nrhs, void* hip_stream)
{
    if (!hd) return set_err(H2_EINVAL, "handle is NULL");
    if (!x || !y) return set_err(H2_EINVAL, "x or y is NULL");
    if (nrhs < 1 || nrhs > 256) return set_err(H2_EINVAL, "nrhs must be in [1, 256]");
    h2::Handle& h = hd->h;
    const size_t bytes = (size_t)h.n * nrhs * (h.precision == 32 ? sizeof(float) : sizeof(double));
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + bytes <= yb || yb + bytes <= xb)) return set_err(H2_EINVAL, "x and y overlap");
    try {
        h2::matvec(h, x, y, nrhs, (hipStream_t)hip_stream);
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
        maxr = std::max(maxr, h.h_rank[i]);
    }
    info->nleaf = nleaf;
    info->r1 = h.r1;
    info->r2 = h.r2;
    info->nnz_il = h.nil;
    info->nnz_near = h.nnear;
    info->max_rank = maxr;
    info->sum_rank = h.sum_rank;
    info->bytes_U = h.bytes_T;
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
        case H2_EXP_RANK: src = h.rank.p; cnt = h.nnode; break;
        case H2_EXP_MBAR: src = h.mbar.p; cnt = h.nnode; break;
        case H2_EXP_PIV:
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            cnt = h.h_mbar[node];
            src = h.piv.p + h.h_piv_off[node];
            break;
        case H2_EXP_SKEL:
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            cnt = h.h_rank[node];
            src = h.skel.p + (int64_t)node * h.ys_stride;
            break;
        case H2_EXP_T:
            if (!node_ok()) return set_err(H2_EINVAL, "node out of range");
            cnt = (int64_t)h.h_rank[node] * (h.h_mbar[node] - h.h_rank[node]);
            src = h.T.p + h.h_T_off[node];
            esz = 8;
            break;
        case H2_EXP_POINTS: src = h.pts.p; cnt = h.n * h.d; esz = 8; break;
        case H2_EXP_B: {
            if (node < 0 || node >= h.nil) return set_err(H2_EINVAL, "IL entry out of range");
            if (h.precision != 64) return set_err(H2_EUNSUPPORTED, "B export needs precision 64");
            int64_t o[2];
            H2_HIP(hipMemcpy(o, h.B_off.p + node, 2 * sizeof(int64_t), hipMemcpyDeviceToHost));
            cnt = o[1] - o[0];
            src = h.B.p + o[0];
            esz = 8;
            break;
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
    (void)hipStreamSynchronize(hd->h.stream);
    for (auto& e : hd->h.ev)
        if (e) (void)hipEventDestroy(e);
    delete hd;
    return H2_OK;
}

}  // extern "C"
