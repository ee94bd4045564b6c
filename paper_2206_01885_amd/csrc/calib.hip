// Choice of r1, r2 from the tolerance (Section 4.2; Algorithm 2 step 2).
//
// The paper grows r1 = r2 from 1 until the ID built on the reduced set
// approximates an artificial well-separated block K(Z1, Z2) to better than
// 1e-2 eps.  Readings (identical to the oracle's): r steps over g^d, g = 1,
// 2, ..., capped at 512 (3-D), 484 (2-D) or 64 (1-D); Z1, Z2 hold 512
// points each, uniform in cubes of side s whose centres lie s sqrt(d)/tau
// apart along axis 0; coordinates are SplitMix64 values (Z1 first, then Z2,
// coordinate fastest); the ID inside uses tolerance 1e-3 eps; the error is the
// relative Frobenius norm of K(Z1,Z2) - U K(Zhat, Z2).  The scale-invariant
// Coulomb kernel is calibrated once (s = 1); the others at the box side of
// every depth holding interaction-list pairs, taking r = the maximum.
//
// Every candidate round runs on the device: point generation, DataReduct,
// the batched ID and the error reduction; all still-open depths of a round
// share one launch of each.
#include "common.h"
#include "kappa.h"

namespace h2 {
namespace {

constexpr int TB = 256;
constexpr int NZ = 512;

__device__ inline double splitmix_u01(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

// Sets are laid out as [Z1 (512) | Z2 (512)] per set, SoA with ld = nset*1024.
__global__ __launch_bounds__(TB) void k_points(int nset, const double* __restrict__ sides, int d, double tau,
                                               uint64_t seed, double* __restrict__ Z)
{
    int64_t ld = (int64_t)nset * 2 * NZ;
    int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= ld) return;
    int set = (int)(q / (2 * NZ));
    int w = (int)(q - (int64_t)set * 2 * NZ);
    double s = sides[set];
    double sep = s * sqrt((double)d) / tau;
    bool second = w >= NZ;
    int i = second ? w - NZ : w;
    for (int a = 0; a < d; ++a) {
        uint64_t ctr = (second ? (uint64_t)NZ * d : 0) + (uint64_t)i * d + a;
        double u = splitmix_u01(seed, ctr);
        Z[a * ld + q] = second ? s * (u - 0.5) + (a == 0 ? sep : 0.0) : s * (u - 0.5);
    }
}

__global__ void k_lists(int nprob, const int* __restrict__ set_of, int64_t* __restrict__ zoff,
                        int* __restrict__ z2idx, int* __restrict__ z1idx, int64_t* __restrict__ xoff,
                        int* __restrict__ mm)
{
    int p = blockIdx.x;
    int base = set_of[p] * 2 * NZ;
    for (int i = threadIdx.x; i < NZ; i += blockDim.x) {
        z2idx[(int64_t)p * NZ + i] = base + NZ + i;
        z1idx[(int64_t)p * NZ + i] = base + i;
    }
    if (threadIdx.x == 0) {
        zoff[p] = (int64_t)p * NZ;
        xoff[p] = (int64_t)p * NZ;
        mm[p] = NZ;
        if (p == nprob - 1) {
            zoff[nprob] = (int64_t)nprob * NZ;
            xoff[nprob] = (int64_t)nprob * NZ;
        }
    }
}

// Squared Frobenius norms for the calibration error, spread over the grid:
// workgroup (p, cb) owns 8 columns c of Z2; it stages K(Zhat, c) in LDS and
// each lane forms rows u of K(Z1 rest, c) - T^T K(Zhat, c).  Partial sums go
// to part[(p*64 + cb)*2 + {0,1}] (residual, full norm) and are reduced in a
// fixed order by k_err_final, so the result does not depend on scheduling.
constexpr int ECOLS = 8;
constexpr int ECB = NZ / ECOLS;
__global__ __launch_bounds__(TB) void k_err_part(const double* __restrict__ Z, int64_t ld, int d, int kid,
                                                 double prm, const int* __restrict__ set_of,
                                                 const int* __restrict__ rank, const int* __restrict__ piv,
                                                 const double* __restrict__ T, int64_t T_stride,
                                                 double* __restrict__ part)
{
    __shared__ double ks[NZ * ECOLS];  // K(Zhat_t, c) for t < k <= 512
    __shared__ double red_r[TB], red_f[TB];
    const int p = blockIdx.x / ECB, cb = blockIdx.x % ECB;
    const int base = set_of[p] * 2 * NZ;
    const int k = rank[p], nr = NZ - k;
    const int* pv = piv + (int64_t)p * NZ;
    const double* Tp = T + (int64_t)p * T_stride;
    const int cl = threadIdx.x % ECOLS, ul = threadIdx.x / ECOLS;  // 8 columns x 32 row lanes
    const int c = cb * ECOLS + cl;
    for (int t = ul; t < k; t += TB / ECOLS)
        ks[t * ECOLS + cl] = kappa_r2(kid, prm, dist2(Z, ld, base + pv[t], Z, ld, base + NZ + c, d));
    __syncthreads();
    double res = 0.0, fro = 0.0;
    for (int i = ul; i < NZ; i += TB / ECOLS) {
        double kv = kappa_r2(kid, prm, dist2(Z, ld, base + i, Z, ld, base + NZ + c, d));
        fro += kv * kv;
    }
    for (int u = ul; u < nr; u += TB / ECOLS) {
        double approx = 0.0;
        for (int t = 0; t < k; ++t) approx = approx + Tp[(int64_t)t * nr + u] * ks[t * ECOLS + cl];
        double e = kappa_r2(kid, prm, dist2(Z, ld, base + pv[k + u], Z, ld, base + NZ + c, d)) - approx;
        res += e * e;
    }
    red_r[threadIdx.x] = res;
    red_f[threadIdx.x] = fro;
    __syncthreads();
    for (int off = TB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red_r[threadIdx.x] += red_r[threadIdx.x + off];
            red_f[threadIdx.x] += red_f[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * 2] = red_r[0];
        part[(int64_t)blockIdx.x * 2 + 1] = red_f[0];
    }
}

__global__ void k_err_final(int np, const double* __restrict__ part, double* __restrict__ err)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double r = 0.0, f = 0.0;
    for (int cb = 0; cb < ECB; ++cb) {
        r += part[((int64_t)p * ECB + cb) * 2];
        f += part[((int64_t)p * ECB + cb) * 2 + 1];
    }
    err[p] = f > 0.0 ? sqrt(r) / sqrt(f) : 0.0;
}

}  // namespace

static int r_cap(int d) { return d == 3 ? 512 : (d == 2 ? 484 : 64); }

void run_calibration(Handle& h)
{
    hipStream_t s = h.stream;
    const int d = h.d;
    const double eps = h.tol_int;
    const int cap = r_cap(d);
    h.calib_r.assign((size_t)h.maxdepth + 1, 0);
    h.calib_err.assign((size_t)h.maxdepth + 1, 0.0);
    if (h.r1 > 0 && h.r2 > 0) return;

    // the calibration sets: (depth, side)
    std::vector<int> depths;
    std::vector<double> sides;
    std::vector<double> hside = read_vec(h.side.p, (size_t)h.nnode, s);
    if (h.kid == H2_COULOMB) {
        depths.push_back(-1);
        sides.push_back(1.0);
    } else {
        for (int L = 1; L <= h.maxdepth; ++L) {
            bool has = false;
            for (int i = h.lvl_ptr[L]; i < h.lvl_ptr[L + 1] && !has; ++i) has = h.h_il_ptr[i + 1] > h.h_il_ptr[i];
            if (!has) continue;
            depths.push_back(L);
            sides.push_back(hside[h.lvl_ptr[L]]);
        }
    }
    const int nset = (int)depths.size();
    int rmax = 1;
    if (nset > 0) {
        DBuf<double> dsides, Z;
        dsides.ensure(nset, s);
        H2_HIP(hipMemcpyAsync(dsides.p, sides.data(), sizeof(double) * nset, hipMemcpyHostToDevice, s));
        const int64_t ld = (int64_t)nset * 2 * NZ;
        Z.ensure((size_t)d * ld, s);
        k_points<<<blocks_for(ld, TB), TB, 0, s>>>(nset, dsides.p, d, h.tau, h.calib_seed, Z.p);
        H2_LAUNCH_CHECK();

        std::vector<int> open(nset, 1), result(nset, cap);
        std::vector<double> result_err(nset, 0.0);
        DBuf<int> set_of, z2idx, z1idx, mm, ycnt, yidx, rank, piv, skel;
        DBuf<int64_t> zoff, xoff, yoff, Moff, nuoff, pivoff, Toff;
        DBuf<double> M, nu, T, err, part;
        for (int g = 1;; ++g) {
            long long rr = 1;
            for (int a = 0; a < d; ++a) rr *= g;
            const int r = rr > cap ? cap : (int)rr;
            std::vector<int> sets;
            for (int t = 0; t < nset; ++t)
                if (open[t]) sets.push_back(t);
            if (sets.empty()) break;
            const int np = (int)sets.size();
            set_of.ensure(np, s);
            H2_HIP(hipMemcpyAsync(set_of.p, sets.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
            z2idx.ensure((size_t)np * NZ, s);
            z1idx.ensure((size_t)np * NZ, s);
            zoff.ensure((size_t)np + 1, s);
            xoff.ensure((size_t)np + 1, s);
            mm.ensure(np, s);
            k_lists<<<np, TB, 0, s>>>(np, set_of.p, zoff.p, z2idx.p, z1idx.p, xoff.p, mm.p);
            H2_LAUNCH_CHECK();
            const int rs = std::min(r, NZ);  // |Y*| <= min(r, 512)
            ycnt.ensure(np, s);
            yidx.ensure((size_t)np * rs, s);
            datareduct_lists(Z.p, ld, d, zoff.p, z2idx.p, nullptr, np, r, yidx.p, rs, ycnt.p, s);
            // ID workspaces
            std::vector<int64_t> h_yoff(np), h_Moff(np), h_nuoff(np), h_pivoff(np), h_Toff(np);
            for (int p = 0; p < np; ++p) {
                h_yoff[p] = (int64_t)p * rs;
                h_Moff[p] = (int64_t)p * rs * NZ;
                h_nuoff[p] = (int64_t)p * 3 * NZ;
                h_pivoff[p] = (int64_t)p * NZ;
                h_Toff[p] = (int64_t)p * rs * NZ;
            }
            auto up = [&](DBuf<int64_t>& dst, const std::vector<int64_t>& src) {
                dst.ensure(src.size(), s);
                H2_HIP(hipMemcpyAsync(dst.p, src.data(), sizeof(int64_t) * src.size(), hipMemcpyHostToDevice, s));
            };
            up(yoff, h_yoff);
            up(Moff, h_Moff);
            up(nuoff, h_nuoff);
            up(pivoff, h_pivoff);
            up(Toff, h_Toff);
            M.ensure((size_t)np * rs * NZ, s);
            nu.ensure((size_t)np * 3 * NZ, s);
            T.ensure((size_t)np * rs * NZ, s);
            rank.ensure(np, s);
            piv.ensure((size_t)np * NZ, s);
            skel.ensure((size_t)np * rs, s);
            err.ensure(np, s);
            IdBatch b;
            b.nprob = np;
            b.m = mm.p;
            b.s = ycnt.p;
            b.x_off = xoff.p;
            b.x_idx = z1idx.p;
            b.y_off = yoff.p;
            b.y_idx = yidx.p;
            b.xpts = Z.p;
            b.xld = ld;
            b.ypts = Z.p;
            b.yld = ld;
            b.M_off = Moff.p;
            b.M = M.p;
            b.nu = nu.p;
            b.nu_off = nuoff.p;
            b.tol = 1e-3 * eps;
            b.rank_out = rank.p;
            b.piv_out = piv.p;
            b.piv_off = pivoff.p;
            b.T_out = T.p;
            b.T_off = Toff.p;
            b.skel_out = skel.p;
            b.skel_stride = rs;
            std::vector<int> ys_h = read_vec(ycnt.p, np, s);
            batched_id(b, std::vector<int>(np, NZ), ys_h, d, h.kid, h.prm, s);
            part.ensure((size_t)np * ECB * 2, s);
            k_err_part<<<np * ECB, TB, 0, s>>>(Z.p, ld, d, h.kid, h.prm, set_of.p, rank.p, piv.p, T.p,
                                               (int64_t)rs * NZ, part.p);
            H2_LAUNCH_CHECK();
            k_err_final<<<blocks_for(np, 64), 64, 0, s>>>(np, part.p, err.p);
            H2_LAUNCH_CHECK();
            std::vector<double> e = read_vec(err.p, np, s);
            for (int p = 0; p < np; ++p) {
                int t = sets[p];
                if (e[p] < 1e-2 * eps) {
                    result[t] = r;
                    result_err[t] = e[p];
                    open[t] = 0;
                } else if (r >= cap) {
                    result[t] = cap;
                    result_err[t] = e[p];
                    open[t] = 0;
                }
            }
        }
        for (int t = 0; t < nset; ++t) {
            rmax = std::max(rmax, result[t]);
            if (depths[t] < 0) {
                for (int L = 0; L <= h.maxdepth; ++L) {
                    h.calib_r[L] = result[t];
                    h.calib_err[L] = result_err[t];
                }
            } else {
                h.calib_r[depths[t]] = result[t];
                h.calib_err[depths[t]] = result_err[t];
            }
        }
    }
    if (h.r1 <= 0) h.r1 = std::max(rmax, h.r_min);
    if (h.r2 <= 0) h.r2 = std::max(rmax, h.r_min);
}

}  // namespace h2
