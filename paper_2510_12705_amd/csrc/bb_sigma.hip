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
// multisection of [0, Gershgorin bound]: each lane evaluates the count at kPts
// of the kSect * kPts equally spaced interior points (two independent division
// chains in flight per lane), and the group keeps the subinterval with
// count(lo) <= t < count(hi), so every step divides the interval by
// kSect * kPts + 1 (about 19 steps instead of 62 bisections), until it is below
// 4 eps of its upper end or 2^-60 of the bound.  The quotient b^2 / q is formed
// from the hardware reciprocal refined by one Newton step (relative error a few
// ulps instead of a correctly rounded division): a Sturm count only needs each
// pivot to small relative accuracy, the premise of its backward error bound.
// The Gershgorin bound and the pivot floor are reduced once per wave (each lane
// strides over the entries), not recomputed by every lane.  Every lane walks the
// same entries in the same order, so the loads of d and e are wave-uniform.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bbk {

constexpr int kWaveSize = 64;

// b2 / q for |q| >= pivmin (a normal number): reciprocal plus one Newton step
__device__ __forceinline__ double quot(double b2, double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    return b2 * r;
}

__device__ __forceinline__ double pivot(double x, double b2, double q, double pivmin) {
    q = -x - quot(b2, q);
    return fabs(q) < pivmin ? -pivmin : q;
}

constexpr int kSect = 4;  // lanes per singular value (divides the wave size)
constexpr int kPts = 2;   // count evaluations per lane and step (independent chains)

// Sturm counts of T - x_p I for the kPts points x[p], walked together.
__device__ __forceinline__ void tgk_counts_below(const double* __restrict__ d, const double* __restrict__ e, int n,
                                                 const double (&x)[kPts], double pivmin, int (&cnt)[kPts]) {
    double q[kPts];
#pragma unroll
    for (int p = 0; p < kPts; ++p) {
        q[p] = -x[p];
        if (fabs(q[p]) < pivmin) q[p] = -pivmin;
        cnt[p] = q[p] < 0.0;
    }
    for (int i = 0; i < n; ++i) {
        const double d2 = d[i] * d[i];
#pragma unroll
        for (int p = 0; p < kPts; ++p) {
            q[p] = pivot(x[p], d2, q[p], pivmin);
            cnt[p] += q[p] < 0.0;
        }
        if (i + 1 < n) {
            const double e2 = e[i] * e[i];
#pragma unroll
            for (int p = 0; p < kPts; ++p) {
                q[p] = pivot(x[p], e2, q[p], pivmin);
                cnt[p] += q[p] < 0.0;
            }
        }
    }
}

__global__ void bb_tgk_bisect(const double* __restrict__ d, const double* __restrict__ e, int n,
                              double* __restrict__ sigma) {
    // Gershgorin bound of T (|lambda| <= |b_{i-1}| + |b_i|, b_{-1} = b_{2n-1} = 0) and
    // the pivot floor, reduced over the wave: lane l takes i = l, l + 64, ...
    const int lane = threadIdx.x & (kWaveSize - 1);
    auto offd = [&](int i) { return (i < 0 || i > 2 * n - 2) ? 0.0 : fabs((i & 1) ? e[i >> 1] : d[i >> 1]); };
    double bound = 0.0, bmax2 = 0.0;
    for (int i = lane; i < 2 * n; i += kWaveSize) {
        const double b = offd(i);
        bound = fmax(bound, offd(i - 1) + b);
        bmax2 = fmax(bmax2, b * b);
    }
    for (int o = kWaveSize / 2; o >= 1; o >>= 1) {
        bound = fmax(bound, __shfl_xor(bound, o, kWaveSize));
        bmax2 = fmax(bmax2, __shfl_xor(bmax2, o, kWaveSize));
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = (int)(gid / kSect), k = (int)(gid % kSect);
    if (j >= n) return;  // the kSect lanes of a value leave together
    const int t = 2 * n - 1 - j;  // ascending index of sigma_j among the eigenvalues of T
    const double eps = 2.220446049250313e-16;
    double lo = 0.0;
    double hi = bound * (1.0 + 4.0 * eps) + pivmin;
    const double floor_width = bound * 0x1p-60;
    constexpr int kDiv = kSect * kPts + 1;
    // lo and hi are equal on the group's lanes, so the loop is uniform per group
    for (int it = 0; it < 128 && hi - lo > fmax(4.0 * eps * hi, floor_width); ++it) {
        double x[kPts];
        int cnt[kPts];
#pragma unroll
        for (int p = 0; p < kPts; ++p) x[p] = lo + (hi - lo) * (double)(k * kPts + p + 1) / (double)kDiv;
        tgk_counts_below(d, e, n, x, pivmin, cnt);
        double nh = hi, nl = lo;
#pragma unroll
        for (int p = 0; p < kPts; ++p) {
            if (cnt[p] > t) nh = fmin(nh, x[p]);
            else nl = fmax(nl, x[p]);
        }
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
