// Device-wide exclusive prefix sums over int32 / int64 arrays.
// Three passes: per-tile totals, a scan of the tile totals (one workgroup
// looping over them), and the per-tile scan with the tile offset added.
// Integer arithmetic, so the result is independent of the schedule.
#include "common.h"

namespace h2 {
namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_PER = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_PER;

template <class T>
__device__ T block_excl_scan(T v, T* sh, T* total)
{
    // Hillis-Steele over the 256 lanes of the workgroup through LDS.
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        T a = t >= off ? sh[t - off] : T(0);
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    T incl = sh[t];
    if (total) *total = sh[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

template <class T>
__global__ __launch_bounds__(SCAN_BLOCK) void tile_sums(const T* __restrict__ in, int64_t n, T* __restrict__ sums)
{
    __shared__ T sh[SCAN_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
    for (int e = 0; e < SCAN_PER; ++e) {
        int64_t i = base + (int64_t)e * SCAN_BLOCK + threadIdx.x;
        if (i < n) acc += in[i];
    }
    T tot;
    block_excl_scan<T>(acc, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(SCAN_BLOCK) void scan_sums(T* __restrict__ sums, int64_t nt, T* __restrict__ grand)
{
    __shared__ T sh[SCAN_BLOCK];
    T carry = 0;
    for (int64_t base = 0; base < nt; base += SCAN_BLOCK) {
        int64_t i = base + threadIdx.x;
        T v = i < nt ? sums[i] : T(0);
        T tot;
        T ex = block_excl_scan<T>(v, sh, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

template <class T>
__global__ __launch_bounds__(SCAN_BLOCK) void tile_scan(const T* __restrict__ in, int64_t n, const T* __restrict__ sums,
                                                        T* __restrict__ out)
{
    __shared__ T sh[SCAN_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    T v[SCAN_PER];
    T acc = 0;
    for (int e = 0; e < SCAN_PER; ++e) {
        int64_t i = base + e;
        v[e] = i < n ? in[i] : T(0);
        acc += v[e];
    }
    T ex = block_excl_scan<T>(acc, sh, nullptr) + sums[blockIdx.x];
    for (int e = 0; e < SCAN_PER; ++e) {
        int64_t i = base + e;
        if (i < n) out[i] = ex;
        ex += v[e];
    }
}

template <class T>
void scan_impl(const T* in, T* out, int64_t cnt, DBuf<T>& tmp, hipStream_t s)
{
    int64_t nt = (cnt + SCAN_TILE - 1) / SCAN_TILE;
    if (nt == 0) {
        H2_HIP(hipMemsetAsync(out, 0, sizeof(T), s));
        return;
    }
    tmp.ensure((size_t)nt + 1, s);
    tile_sums<T><<<(unsigned)nt, SCAN_BLOCK, 0, s>>>(in, cnt, tmp.p);
    H2_LAUNCH_CHECK();
    scan_sums<T><<<1, SCAN_BLOCK, 0, s>>>(tmp.p, nt, out + cnt);
    H2_LAUNCH_CHECK();
    tile_scan<T><<<(unsigned)nt, SCAN_BLOCK, 0, s>>>(in, cnt, tmp.p, out);
    H2_LAUNCH_CHECK();
}

}  // namespace

void scan_excl_i32(const int* in, int* out, int64_t cnt, DBuf<int>& tmp, hipStream_t s)
{
    scan_impl<int>(in, out, cnt, tmp, s);
}
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t cnt, DBuf<int64_t>& tmp, hipStream_t s)
{
    scan_impl<int64_t>(in, out, cnt, tmp, s);
}

}  // namespace h2
