// Kernel functions kappa(x, y) of the paper (Section 2, Table 1) as device
// functions.  prm is the bandwidth h or the length scale l.
#pragma once

#include <hip/hip_runtime.h>

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
    default: {  // H2_MATERN32
        double t = sqrt(3.0) * sqrt(r2) / prm;
        return (1.0 + t) * exp(-t);
    }
    }
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
