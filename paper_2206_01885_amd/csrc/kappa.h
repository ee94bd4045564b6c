// Kernel functions kappa(x, y) of the paper (Section 2, Table 1) as device
// functions.  prm is the bandwidth h or the length scale l.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace h2 {

// kappa from the squared distance r2 = |x - y|^2.
__device__ __forceinline__ double kappa_r2(int kid, double prm, double r2)
{
    switch (kid) {
    case H2_COULOMB:
        return r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    case H2_GAUSSIAN:
        return exp(-r2 / (prm * prm));
    case H2_EXPONENTIAL:
        return exp(-sqrt(r2) / prm);
    case H2_BUMP:
        return exp(-1.0 / (1.0 - prm * r2));
    default: {  // H2_MATERN32
        double t = sqrt(3.0) * sqrt(r2) / prm;
        return (1.0 + t) * exp(-t);
    }
    }
}

// Kernel families.  The kernels that evaluate kappa are compiled once per
// family, so that the radial kernels' code (functions of r2 = |x - y|^2)
// carries neither the register cost of cos nor the drift term:
//   FAM_RADIAL     Coulomb, Gaussian, exponential, Matern-3/2, bump
//   FAM_COSINE     kappa_3 of Table 1, a function of xy = x.y
//   FAM_ADVECTION  the advection-diffusion kernel, a function of r2 and of
//                  d0 = (x - y)_0; not symmetric
enum { FAM_RADIAL = 0, FAM_COSINE = 1, FAM_ADVECTION = 2 };
inline int kernel_family(int kid)
{
    return kid == H2_COSINE ? FAM_COSINE : (kid == H2_ADVECTION ? FAM_ADVECTION : FAM_RADIAL);
}

// exp(a (d0 - r)) / r with r = sqrt(r2), 0 at r2 = 0 (a = prm): the Green's
// function of steady advection-diffusion with the drift along axis 0.
__device__ __forceinline__ double kappa_advection(double prm, double r2, double d0)
{
    if (!(r2 > 0.0)) return 0.0;
    const double r = sqrt(r2);
    return exp(prm * (d0 - r)) / r;
}

template <int FAM>
__device__ __forceinline__ double kappa_fam(int kid, double prm, double r2, double xy, double d0)
{
    if constexpr (FAM == FAM_COSINE)
        return cos(prm * xy);
    else if constexpr (FAM == FAM_ADVECTION)
        return kappa_advection(prm, r2, d0);
    else
        return kappa_r2(kid, prm, r2);
}

// 1/sqrt(r2) for r2 > 0: the hardware estimate refined by two Newton steps
// y <- y (3 - r2 y^2) / 2 (each roughly doubles the correct bits).
// (Fused multiply-adds written out, so that every kernel that evaluates
// entries forms them alike, whatever the contraction mode of its file.)
__device__ __forceinline__ double rsqrt_nr(double r2)
{
    double y = __builtin_amdgcn_rsq(r2);
    const double h = 0.5 * r2;
    y = y * __builtin_fma(-(h * y), y, 1.5);
    y = y * __builtin_fma(-(h * y), y, 1.5);
    return y;
}

// Same functions with the refined reciprocal square root (an ulp or two);
// used where the entries are not compared bit for bit.
__device__ __forceinline__ double kappa_fast(int kid, double prm, double r2)
{
    switch (kid) {
    case H2_COULOMB:
        return r2 > 0.0 ? rsqrt_nr(r2) : 0.0;
    case H2_GAUSSIAN:
        return exp(-r2 / (prm * prm));
    case H2_EXPONENTIAL:
        return exp(-sqrt(r2) / prm);
    case H2_BUMP:
        return exp(-1.0 / (1.0 - prm * r2));
    default: {
        double t = sqrt(3.0) * sqrt(r2) / prm;
        return (1.0 + t) * exp(-t);
    }
    }
}

// FP32 evaluation from an FP64 squared distance (precision mode): the
// distance is formed in FP64 (differences of nearby points keep their
// digits), the kernel function in FP32.
__device__ __forceinline__ float kappa_f32(int kid, float prm, double r2d)
{
    const float r2 = (float)r2d;
    switch (kid) {
    case H2_COULOMB:
        return r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
    case H2_GAUSSIAN:
        return __expf(-r2 / (prm * prm));
    case H2_EXPONENTIAL:
        return __expf(-sqrtf(r2) / prm);
    case H2_BUMP:
        return __expf(-1.0f / (1.0f - prm * r2));
    default: {
        float t = 1.7320508075688772f * sqrtf(r2) / prm;
        return (1.0f + t) * __expf(-t);
    }
    }
}

template <class T, int FAM>
__device__ __forceinline__ T kappa_store(int kid, double prm, double r2, double xy, double d0)
{
    if constexpr (FAM != FAM_RADIAL)
        return (T)kappa_fam<FAM>(kid, prm, r2, xy, d0);
    else if constexpr (std::is_same_v<T, float>)
        return kappa_f32(kid, (float)prm, r2);
    else
        return kappa_fast(kid, prm, r2);
}

// Squared distance accumulated in coordinate order from 0 (as the oracle does).
__device__ __forceinline__ double dist2(const double* __restrict__ xa, int64_t xld, int64_t xi,
                                        const double* __restrict__ ya, int64_t yld, int64_t yi, int d)
{
    double r2 = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = xa[a * xld + xi] - ya[a * yld + yi];
        r2 = r2 + t * t;
    }
    return r2;
}

}  // namespace h2
