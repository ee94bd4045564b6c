// Choice of r1, r2 from the tolerance (Section 4.2; Algorithm 2 step 2).
//
// The paper grows r1 = r2 from 1 until the ID built on the reduced set
// approximates an artificial block K(Z1, Z2) of well-separated point sets to
// better than 1e-2 eps.  Readings (identical to the oracle's): r steps over
// g^d, g = 1, 2, ..., capped at 512 (3-D), 484 (2-D) or 64 (1-D), and gives
// r1 = r, r2 = 2 r (Y_i^* samples the two parts of T_i with r points each);
// Z1 holds 512 points uniform in the box [0, s)^d; Z2 holds 4096 points, each
// uniform in a box drawn uniformly from the interaction list of Z1's box in
// the uniform tree of boxes of side s (the pair rule: admissible to the box,
// parent cell floor(o/2) not admissible to the parent [0, 2s)^d; listed with
// dimension 0 fastest, coordinates ascending); coordinates are SplitMix64
// values: i d + a for Z1, 512 d + j (d + 1) for the box of Z2 point j and the
// d values after it for its place in the box; the ID inside is built on
// DataReduct(Z2, r) with tolerance 1e-3 eps' (eps' = eps/2); the error is the
// relative Frobenius norm of K(Z1,Z2) - U K(Zhat, Z2) over all of Z2.  The
// scale-invariant Coulomb kernel is calibrated once (s = 1); the others at
// the box side of every depth holding interaction-list pairs, taking r = the
// maximum.
//
// Every step runs on the device: point generation, DataReduct, the batched
// ID and the error reduction, for every candidate r below the cap of every
// set at once (one launch of each, one read-back), then for the cap only for
// the sets none of those met; each set takes its first candidate below the
// target, which is what trying them in turn would give.
#include <map>
#include <tuple>

#include "common.h"
#include "kappa.h"

namespace h2 {
namespace {

constexpr int TB = 256;
constexpr int NZ = 512;    // Z1: the candidate rows of the ID
constexpr int NZ2 = 4096;  // Z2: the farfield sample
constexpr int NS = NZ + NZ2;

__device__ inline double splitmix_u01(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

// Sets are laid out as [Z1 (512) | Z2 (4096)] per set, SoA with
// ld = nset * NS; shell ([nb][d]) holds the cell offsets of Z2's boxes.
__global__ __launch_bounds__(TB) void k_points(int nset, const double* __restrict__ sides, int d,
                                               const int* __restrict__ shell, int nb, uint64_t seed,
                                               double* __restrict__ Z)
{
    const int64_t ld = (int64_t)nset * NS;
    const int64_t q = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (q >= ld) return;
    const int set = (int)(q / NS);
    const int w = (int)(q - (int64_t)set * NS);
    const double s = sides[set];
    if (w < NZ) {
        for (int a = 0; a < d; ++a) Z[a * ld + q] = s * splitmix_u01(seed, (uint64_t)w * d + a);
        return;
    }
    const uint64_t c = (uint64_t)NZ * d + (uint64_t)(w - NZ) * (d + 1);
    int b = (int)(splitmix_u01(seed, c) * (double)nb);
    if (b > nb - 1) b = nb - 1;
    for (int a = 0; a < d; ++a)
        Z[a * ld + q] = s * ((double)shell[b * d + a] + splitmix_u01(seed, c + 1 + a));
}

__global__ void k_lists(int nprob, const int* __restrict__ set_of, int64_t* __restrict__ zoff,
                        int* __restrict__ z2idx, int* __restrict__ z1idx, int64_t* __restrict__ xoff,
                        int* __restrict__ mm)
{
    int p = blockIdx.x;
    int base = set_of[p] * NS;
    for (int i = threadIdx.x; i < NZ2; i += blockDim.x) z2idx[(int64_t)p * NZ2 + i] = base + NZ + i;
    for (int i = threadIdx.x; i < NZ; i += blockDim.x) z1idx[(int64_t)p * NZ + i] = base + i;
    if (threadIdx.x == 0) {
        zoff[p] = (int64_t)p * NZ2;
        xoff[p] = (int64_t)p * NZ;
        mm[p] = NZ;
        if (p == nprob - 1) {
            zoff[nprob] = (int64_t)nprob * NZ2;
            xoff[nprob] = (int64_t)nprob * NZ;
        }
    }
}

// Squared Frobenius norms for the calibration error, spread over the grid:
// workgroup (p, cb) owns 8 columns c of Z2; it stages K(Zhat, c) in LDS and
// each lane forms rows u of K(Z1 rest, c) - T^T K(Zhat, c).  Partial sums go
// to part[(p*ECB + cb)*2 + {0,1}] (residual, full norm) and are reduced in a
// fixed order by k_err_final, so the result does not depend on scheduling.
constexpr int ECOLS = 8;
constexpr int ECB = NZ2 / ECOLS;
__global__ __launch_bounds__(TB) void k_err_part(const double* __restrict__ Z, int64_t ld, int d,
                                                 const int* __restrict__ set_kid, const double* __restrict__ set_prm,
                                                 const int* __restrict__ set_of,
                                                 const int* __restrict__ rank, const int* __restrict__ piv,
                                                 const double* __restrict__ T, const int64_t* __restrict__ T_off,
                                                 double* __restrict__ part)
{
    __shared__ double ks[NZ * ECOLS];  // K(Zhat_t, c) for t < k <= 512
    __shared__ double red_r[TB], red_f[TB];
    const int p = blockIdx.x / ECB, cb = blockIdx.x % ECB;
    const int base = set_of[p] * NS;
    const int kid = set_kid[set_of[p]];
    const double prm = set_prm[set_of[p]];
    const int k = rank[p], nr = NZ - k;
    const int* pv = piv + (int64_t)p * NZ;
    const double* Tp = T + T_off[p];
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

// Cell offsets of the interaction list of the box [0, 1)^d in the uniform
// tree of unit boxes (pair rule, Eq. separation with box diagonals and
// centres): cell o is admissible to the box and its parent cell floor(o/2)
// (side 2) is not admissible to the box's parent [0, 2)^d.  Dimension 0
// varies fastest, coordinates ascending.
static std::vector<int> shell_cells(int d, double tau)
{
    const int R = (int)std::ceil(2.0 * std::sqrt((double)d) / tau) + 1;  // |o_a| < 2 sqrt(d)/tau + 1
    const int w = 2 * R + 1;
    int64_t tot = 1;
    for (int a = 0; a < d; ++a) tot *= w;
    std::vector<int> out;
    for (int64_t t = 0; t < tot; ++t) {
        int o[3];
        int64_t rem = t;
        double dc = 0.0, dp = 0.0;
        for (int a = 0; a < d; ++a) {
            o[a] = (int)(rem % w) - R;
            rem /= w;
            const int po = (o[a] >= 0) ? o[a] / 2 : -((1 - o[a]) / 2);  // floor(o/2)
            const double ec = (double)o[a], ep = 2.0 * (double)po;    // centre offsets
            dc = dc + ec * ec;
            dp = dp + ep * ep;
        }
        const bool adm = (double)d * 4.0 <= 4.0 * tau * tau * dc;
        const bool adm_parent = (double)d * 16.0 <= 4.0 * tau * tau * dp;
        if (adm && !adm_parent)
            for (int a = 0; a < d; ++a) out.push_back(o[a]);
    }
    return out;
}

// Calibration of a list of sets that share d, tau and the seed; set t has
// kernel kid[t] with parameter prm[t], box side side[t] and tolerance eps[t].
// Returns, per set, the first r = g^d whose error is below 1e-2 eps (or the
// cap) and that error.
static void calibrate_sets(int d, double tau, uint64_t seed, const std::vector<double>& sides,
                           const std::vector<int>& kids, const std::vector<double>& prms,
                           const std::vector<double>& epss, int cap, std::vector<int>& result,
                           std::vector<double>& result_err, hipStream_t s)
{
    const int nset = (int)sides.size();
    result.assign(nset, cap);
    result_err.assign(nset, 0.0);
    if (nset == 0) return;
    DBuf<double> dsides, Z, dprm;
    DBuf<int> dkid;
    dsides.ensure(nset, s);
    dprm.ensure(nset, s);
    dkid.ensure(nset, s);
    H2_HIP(hipMemcpyAsync(dsides.p, sides.data(), sizeof(double) * nset, hipMemcpyHostToDevice, s));
    H2_HIP(hipMemcpyAsync(dprm.p, prms.data(), sizeof(double) * nset, hipMemcpyHostToDevice, s));
    H2_HIP(hipMemcpyAsync(dkid.p, kids.data(), sizeof(int) * nset, hipMemcpyHostToDevice, s));
    const int64_t ld = (int64_t)nset * NS;
    Z.ensure((size_t)d * ld, s);
    const std::vector<int> shell = shell_cells(d, tau);
    const int nb = (int)shell.size() / d;
    if (nb < 1) fail(H2_EINTERNAL, "calibration: empty interaction list");
    DBuf<int> dshell;
    upload_vec(dshell, shell, s);
    k_points<<<blocks_for(ld, TB), TB, 0, s>>>(nset, dsides.p, d, dshell.p, nb, seed, Z.p);
    H2_LAUNCH_CHECK();
    // candidate sizes r = g^d (g = 1, 2, ... up to the cap)
    std::vector<int> rs_of;
    for (int g = 1;; ++g) {
        long long rr = 1;
        for (int a = 0; a < d; ++a) rr *= g;
        rs_of.push_back(rr > cap ? cap : (int)rr);
        if (rr >= cap) break;
    }
    const int ng = (int)rs_of.size();
    // The errors of candidates G (indices into rs_of) of sets S, all in one
    // round: task p = (G[gi], S[si]), p = gi |S| + si (tasks grouped by
    // candidate size); returns e[p].
    auto run = [&](const std::vector<int>& G, const std::vector<int>& S) {
        const int nS = (int)S.size(), np = (int)G.size() * nS;
        std::vector<int> sets(np);
        std::vector<int64_t> y_off(np + 1, 0), mt_off(np + 1, 0);
        for (int gi = 0; gi < (int)G.size(); ++gi)
            for (int si = 0; si < nS; ++si) {
                const int p = gi * nS + si;
                sets[p] = S[si];
                y_off[p + 1] = y_off[p] + rs_of[G[gi]];
                mt_off[p + 1] = mt_off[p] + (int64_t)rs_of[G[gi]] * NZ;
            }
        DBuf<int> set_of, z2idx, z1idx, mm, ycnt, yidx, rank, piv, skel;
        DBuf<int64_t> zoff, xoff, d_mt_off;
        DBuf<double> M, nu, T, err, part;
        upload_vec(set_of, sets, s);
        upload_vec(d_mt_off, mt_off, s);
        z2idx.ensure((size_t)np * NZ2, s);
        z1idx.ensure((size_t)np * NZ, s);
        zoff.ensure((size_t)np + 1, s);
        xoff.ensure((size_t)np + 1, s);
        mm.ensure(np, s);
        k_lists<<<np, TB, 0, s>>>(np, set_of.p, zoff.p, z2idx.p, z1idx.p, xoff.p, mm.p);
        H2_LAUNCH_CHECK();
        ycnt.ensure(np, s);
        yidx.ensure((size_t)y_off[np], s);
        for (int gi = 0; gi < (int)G.size(); ++gi) {  // |Y*| <= r <= the cap (512)
            const int r = rs_of[G[gi]];
            datareduct_lists(Z.p, ld, d, zoff.p + (int64_t)gi * nS, z2idx.p, nullptr, nS, r,
                             yidx.p + y_off[(size_t)gi * nS], r, ycnt.p + (int64_t)gi * nS, s);
        }
        M.ensure((size_t)mt_off[np], s);
        nu.ensure((size_t)np * 3 * NZ, s);
        T.ensure((size_t)mt_off[np], s);
        rank.ensure(np, s);
        piv.ensure((size_t)np * NZ, s);
        skel.ensure((size_t)y_off[np], s);
        err.ensure(np, s);
        std::vector<int> ys_h = read_vec(ycnt.p, np, s);
        std::vector<IdTask> tasks(np);
        for (int p = 0; p < np; ++p) {
            IdTask& t = tasks[p];
            t.pts = Z.p;
            t.ld = ld;
            t.x_idx = z1idx.p + (int64_t)p * NZ;
            t.y_idx = yidx.p + y_off[p];
            t.M = M.p + mt_off[p];
            t.nu = nu.p + (int64_t)p * 3 * NZ;
            t.piv = piv.p + (int64_t)p * NZ;
            t.T = T.p + mt_off[p];
            t.skel = skel.p + y_off[p];
            t.rank = rank.p + p;
            t.prm = prms[sets[p]];
            t.tol = 1e-3 * (0.5 * epss[sets[p]]);  // 1e-3 eps'
            t.m = NZ;
            t.s = ys_h[p];
            t.d = d;
            t.kid = kids[sets[p]];
        }
        batched_id(tasks, s);
        part.ensure((size_t)np * ECB * 2, s);
        k_err_part<<<np * ECB, TB, 0, s>>>(Z.p, ld, d, dkid.p, dprm.p, set_of.p, rank.p, piv.p, T.p, d_mt_off.p,
                                           part.p);
        H2_LAUNCH_CHECK();
        k_err_final<<<blocks_for(np, 64), 64, 0, s>>>(np, part.p, err.p);
        H2_LAUNCH_CHECK();
        return read_vec(err.p, np, s);
    };
    // Each set takes its first candidate below the target, as if they were
    // tried in turn.  The candidates below the cap run together; the cap (the
    // largest and slowest ID) only for the sets none of them satisfied.
    std::vector<int> all(nset), G1;
    for (int t = 0; t < nset; ++t) all[t] = t;
    for (int g = 0; g + 1 < ng; ++g) G1.push_back(g);
    std::vector<int> rest;
    if (!G1.empty()) {
        const std::vector<double> e = run(G1, all);
        for (int t = 0; t < nset; ++t) {
            bool found = false;
            for (int gi = 0; gi < (int)G1.size() && !found; ++gi)
                if (e[(size_t)gi * nset + t] < 1e-2 * epss[t]) {
                    result[t] = rs_of[G1[gi]];
                    result_err[t] = e[(size_t)gi * nset + t];
                    found = true;
                }
            if (!found) rest.push_back(t);
        }
    } else {
        rest = all;
    }
    if (!rest.empty()) {
        const std::vector<double> e = run({ng - 1}, rest);
        for (size_t q = 0; q < rest.size(); ++q) {
            result[rest[q]] = rs_of[ng - 1];  // the cap, met or not
            result_err[rest[q]] = e[q];
        }
    }
}

// r1, r2 of several problems at once.  Each problem's sets (Coulomb: one set
// of side 1; otherwise one per depth holding interaction-list pairs) are
// pooled; identical sets (same d, tau, seed, kernel, parameter, side and
// tolerance: e.g. every Coulomb problem at one tolerance) are calibrated once,
// and all sets of one (d, tau, seed) share each round's launches.  Each
// problem gets exactly the r it would get alone.
void run_calibration_multi(const std::vector<Handle*>& hs, hipStream_t s)
{
    struct Key {
        int d, kid;
        double tau, prm, side, eps;
        uint64_t seed;
        bool operator<(const Key& o) const
        {
            return std::tie(d, tau, seed, kid, prm, side, eps) <
                   std::tie(o.d, o.tau, o.seed, o.kid, o.prm, o.side, o.eps);
        }
    };
    std::map<Key, int> uniq;
    std::vector<Key> keys;
    std::vector<std::vector<std::pair<int, int>>> uses;  // (depth, set) per problem
    uses.resize(hs.size());
    for (size_t p = 0; p < hs.size(); ++p) {
        Handle& h = *hs[p];
        h.calib_r.assign((size_t)h.maxdepth + 1, 0);
        h.calib_err.assign((size_t)h.maxdepth + 1, 0.0);
        if (h.r1 > 0 && h.r2 > 0) continue;
        std::vector<std::pair<int, double>> ds;
        if (h.kid == H2_COULOMB) {
            ds.push_back({-1, 1.0});
        } else {
            std::vector<double> hside = read_vec(h.side.p, (size_t)h.nnode, s);
            for (int L = 1; L <= h.maxdepth; ++L) {
                bool has = false;
                for (int i = h.lvl_ptr[L]; i < h.lvl_ptr[L + 1] && !has; ++i)
                    has = h.h_il_ptr[i + 1] > h.h_il_ptr[i];
                if (has) ds.push_back({L, hside[h.lvl_ptr[L]]});
            }
        }
        for (auto& x : ds) {
            Key k{h.d, h.kid, h.tau, h.kid == H2_COULOMB ? 1.0 : h.prm, x.second, h.tol, h.calib_seed};
            auto it = uniq.find(k);
            int id;
            if (it == uniq.end()) {
                id = (int)keys.size();
                uniq[k] = id;
                keys.push_back(k);
            } else {
                id = it->second;
            }
            uses[p].push_back({x.first, id});
        }
    }
    std::vector<int> res(keys.size(), 0);
    std::vector<double> res_err(keys.size(), 0.0);
    // one calibration per (d, tau, seed) group
    std::vector<int> done(keys.size(), 0);
    for (size_t t0 = 0; t0 < keys.size(); ++t0) {
        if (done[t0]) continue;
        std::vector<int> grp;
        for (size_t t = t0; t < keys.size(); ++t)
            if (!done[t] && keys[t].d == keys[t0].d && keys[t].tau == keys[t0].tau && keys[t].seed == keys[t0].seed) {
                grp.push_back((int)t);
                done[t] = 1;
            }
        std::vector<double> sides, prms, epss;
        std::vector<int> kids;
        for (int t : grp) {
            sides.push_back(keys[t].side);
            prms.push_back(keys[t].prm);
            epss.push_back(keys[t].eps);
            kids.push_back(keys[t].kid);
        }
        std::vector<int> r;
        std::vector<double> e;
        calibrate_sets(keys[t0].d, keys[t0].tau, keys[t0].seed, sides, kids, prms, epss, r_cap(keys[t0].d), r, e,
                       s);
        for (size_t q = 0; q < grp.size(); ++q) {
            res[grp[q]] = r[q];
            res_err[grp[q]] = e[q];
        }
    }
    for (size_t p = 0; p < hs.size(); ++p) {
        Handle& h = *hs[p];
        if (h.r1 > 0 && h.r2 > 0) continue;
        int rmax = 1;
        for (auto& u : uses[p]) {
            const int r = res[u.second];
            rmax = std::max(rmax, r);
            if (u.first < 0) {
                for (int L = 0; L <= h.maxdepth; ++L) {
                    h.calib_r[L] = r;
                    h.calib_err[L] = res_err[u.second];
                }
            } else {
                h.calib_r[u.first] = r;
                h.calib_err[u.first] = res_err[u.second];
            }
        }
        const int r = std::max(rmax, h.r_min);
        if (h.r1 <= 0) h.r1 = r;
        if (h.r2 <= 0) h.r2 = 2 * r;
    }
}

void run_calibration(Handle& h) { run_calibration_multi({&h}, h.stream); }

}  // namespace h2
