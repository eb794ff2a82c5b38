// bb_sigma.hip -- singular values of the upper bidiagonal B = bidiag(d, e) on the
// GPU, the step that follows the reduction (the paper hands B to a CPU solver,
// Sec. V-A).
//
// sigma(B) are the n non-negative eigenvalues of the 2n x 2n Golub-Kahan
// tridiagonal T: zero diagonal, off-diagonal b = (d0, e0, d1, e1, ..., d_{n-1}),
// spectrum {+-sigma_i}.  The number of eigenvalues of T below x is the number of
// negative pivots of the LDL^T factorisation of T - x I (Sylvester's law of
// inertia):
//   q_0 = -x,   q_i = -x - b_{i-1}^2 / q_{i-1}   (i = 1 .. 2n-1),
// where a pivot smaller in magnitude than pivmin = DBL_MIN * max(1, max b^2) is
// replaced by -pivmin, the usual safeguard of bisection for symmetric
// tridiagonals.  A group of kSect lanes finds sigma_j of the descending order --
// the eigenvalue of T with index t = 2n-1-j in ascending order -- by
// multisection of [0, Gershgorin bound]: each lane evaluates the count at one of
// kSect equally spaced interior points, and the group keeps the subinterval with
// count(lo) <= t < count(hi), so every step divides the interval by kSect + 1
// (about 26 steps instead of 62 bisections), until it is below 4 eps of its
// upper end or 2^-60 of the bound.  The count is a serial chain of divisions;
// more lanes per value also give each SIMD more waves to hide its latency.
// Every lane walks the same entries in the same order, so the loads of d and e
// are wave-uniform.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bbk {

constexpr int kWaveSize = 64;

__device__ __forceinline__ int tgk_count_below(const double* __restrict__ d, const double* __restrict__ e, int n,
                                               double x, double pivmin) {
    double q = -x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 0; i < n; ++i) {
        q = -x - (d[i] * d[i]) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        if (i + 1 < n) {
            q = -x - (e[i] * e[i]) / q;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
    }
    return cnt;
}

constexpr int kSect = 4;  // lanes per singular value (divides the wave size; 4 measured fastest)

__global__ void bb_tgk_bisect(const double* __restrict__ d, const double* __restrict__ e, int n,
                              double* __restrict__ sigma) {
    // Gershgorin bound of T (|lambda| <= |b_{i-1}| + |b_i|) and the pivot floor
    double bound = 0.0, bmax2 = 0.0, prev = 0.0;
    for (int i = 0; i < 2 * n - 1; ++i) {
        const double b = fabs((i & 1) ? e[i >> 1] : d[i >> 1]);
        bound = fmax(bound, prev + b);
        bmax2 = fmax(bmax2, b * b);
        prev = b;
    }
    bound = fmax(bound, prev);
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = (int)(gid / kSect), k = (int)(gid % kSect);
    if (j >= n) return;  // the kSect lanes of a value leave together
    const int t = 2 * n - 1 - j;  // ascending index of sigma_j among the eigenvalues of T
    const double eps = 2.220446049250313e-16;
    double lo = 0.0;
    double hi = bound * (1.0 + 4.0 * eps) + pivmin;
    const double floor_width = bound * 0x1p-60;
    // lo and hi are equal on the group's lanes, so the loop is uniform per group
    for (int it = 0; it < 128 && hi - lo > fmax(4.0 * eps * hi, floor_width); ++it) {
        const double x = lo + (hi - lo) * (double)(k + 1) / (double)(kSect + 1);
        const bool above = tgk_count_below(d, e, n, x, pivmin) > t;
        double nh = above ? x : hi, nl = above ? lo : x;
#pragma unroll
        for (int o = 1; o < kSect; o <<= 1) {
            nh = fmin(nh, __shfl_xor(nh, o, kWaveSize));
            nl = fmax(nl, __shfl_xor(nl, o, kWaveSize));
        }
        lo = fmin(nl, nh);  // a count that is not monotone in x cannot invert the interval
        hi = fmax(nl, nh);
    }
    if (k == 0) sigma[j] = 0.5 * (lo + hi);
}

hipError_t launch_bidiag_sigma(const double* d, const double* e, int64_t n, double* sigma, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int threads = 64;  // one wave per workgroup spreads the values over more CUs
    const int64_t lanes = n * kSect;
    const int grid = (int)((lanes + threads - 1) / threads);
    hipLaunchKernelGGL(bb_tgk_bisect, dim3(grid), dim3(threads), 0, st, d, e, (int)n, sigma);
    return hipGetLastError();
}

}  // namespace bbk
