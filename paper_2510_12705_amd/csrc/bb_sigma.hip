// bb_sigma.hip -- singular values of the upper bidiagonal B = bidiag(d, e) on the
// GPU, the step that follows the reduction (the paper hands B to a CPU solver,
// Sec. V-A).
//
// sigma(B) are the n non-negative eigenvalues of the 2n x 2n Golub-Kahan
// tridiagonal T: zero diagonal, off-diagonal b = (d0, e0, d1, e1, ..., d_{n-1}),
// spectrum {+-sigma_i}.  The number of eigenvalues of T below x is the number of
// sign changes in the sequence of leading principal minors of T - x I (Sturm):
//   p_{-1} = 1,  p_0 = -x,  p_k = -x p_{k-1} - b_{k-1}^2 p_{k-2}   (k = 1 .. 2n-1),
// each sign change being a negative pivot p_k / p_{k-1} of the LDL^T
// factorisation.  Evaluated this way a step costs one multiply and one fused
// multiply-add per point, with no division; the price is the range of the minors,
// which is kept in check by working on the matrix scaled by a power of two so
// that max |b| lies in [1/2, 1) (exact), and by rescaling the pair
// (p_{k-1}, p_{k-2}) by a power of two every four steps (exact, and the signs and
// the ratio -- the pivot -- are unchanged).  With |x| <= 2 and |b| < 1 a step
// grows the pair by at most 1 + sqrt(2), so four steps cannot overflow.  The
// rounding of one step, p_k = (-x p_{k-1} (1+d1) - b^2 p_{k-2} (1+d2)) (1+d3),
// is that of the pivot recurrence q_k = -x - b^2 / q_{k-1} with x and b^2
// perturbed in their last bits, the premise of the backward error bound of a
// Sturm count.
//
// A group of kSect lanes finds sigma_j of the descending order -- the eigenvalue
// of T with index t = 2n-1-j in ascending order -- by multisection of
// [0, Gershgorin bound]: each lane evaluates the count at kPts of the
// kSect * kPts equally spaced interior points (independent chains in flight per
// lane), and the group keeps the subinterval with count(lo) <= t < count(hi), so
// every step divides the interval by kSect * kPts + 1, until it is below 4 eps of
// its upper end or 2^-60 of the bound.  The Gershgorin bound and the scale are
// reduced once per wave (each lane strides over the entries).  Every lane walks
// the same entries in the same order, so the loads of d and e are wave-uniform.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bbk {

constexpr int kWaveSize = 64;
#ifndef BB_SIGMA_SECT
#define BB_SIGMA_SECT 4
#endif
#ifndef BB_SIGMA_PTS
#define BB_SIGMA_PTS 2
#endif
constexpr int kSect = BB_SIGMA_SECT;  // lanes per singular value (divides the wave size)
constexpr int kPts = BB_SIGMA_PTS;    // count evaluations per lane and step (independent chains)

__device__ __forceinline__ unsigned sign_bit(double v) { return (unsigned)__double2hiint(v) >> 31; }

// Sturm counts of T - x_p I for the P points x[p] (scaled units; bs = the
// power of two that scales the entries).
template <int P>
__device__ __forceinline__ void tgk_counts_below(const double* __restrict__ d, const double* __restrict__ e, int n,
                                                 double bs, const double (&x)[P], int (&cnt)[P]) {
    constexpr int kPts = P;
    double p1[kPts], p2[kPts];  // p_{k-1}, p_{k-2}
    unsigned c[kPts];
#pragma unroll
    for (int p = 0; p < kPts; ++p) {
        p2[p] = 1.0;
        p1[p] = -x[p];
        c[p] = sign_bit(p1[p]);  // p_{-1} = 1 > 0
    }
    auto step = [&](double b) {
        const double s = b * bs, b2 = s * s;
#pragma unroll
        for (int p = 0; p < kPts; ++p) {
            const double pn = fma(-x[p], p1[p], -(b2 * p2[p]));
            c[p] += ((unsigned)__double2hiint(pn) ^ (unsigned)__double2hiint(p1[p])) >> 31;
            p2[p] = p1[p];
            p1[p] = pn;
        }
    };
    auto rescale = [&]() {
#pragma unroll
        for (int p = 0; p < kPts; ++p) {
            const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(p1[p]), fabs(p2[p])));
            p1[p] = __builtin_amdgcn_ldexp(p1[p], -ex);
            p2[p] = __builtin_amdgcn_ldexp(p2[p], -ex);
        }
    };
    int i = 0;
    if (n >= 3) {
        // couplings d_i, e_i, d_{i+1}, e_{i+1}; the next four are loaded one
        // iteration ahead (indices clamped into range on the last iteration)
        double d0 = d[0], e0 = e[0], d1 = d[1], e1 = e[1];
        for (; i + 2 < n; i += 2) {
            const double a0 = d0, a1 = e0, a2 = d1, a3 = e1;
            d0 = d[min(i + 2, n - 1)];
            e0 = e[min(i + 2, n - 2)];
            d1 = d[min(i + 3, n - 1)];
            e1 = e[min(i + 3, n - 2)];
            step(a0);
            step(a1);
            step(a2);
            step(a3);
            rescale();
        }
    }
    if (i + 1 < n) {  // i = n-2: d_{n-2}, e_{n-2}, d_{n-1}
        step(d[i]);
        step(e[i]);
        step(d[i + 1]);
    } else if (i < n) {  // i = n-1: d_{n-1}
        step(d[i]);
    }
#pragma unroll
    for (int p = 0; p < kPts; ++p) cnt[p] = (int)c[p];
}

// The scaling and the Gershgorin bound, reduced over the wave (lane l takes
// entries l, l + 64, ...); every lane of the wave must be active.
struct TgkFrame {
    int ex;        // max |b| * 2^-ex in [1/2, 1)
    double bs;     // 2^-ex
    double hi0;    // Gershgorin bound of the scaled T, widened by 4 eps: above every eigenvalue
    bool nan_in;   // a NaN or infinite entry
    bool zero;     // B = 0
};

__device__ __forceinline__ TgkFrame tgk_frame(const double* __restrict__ d, const double* __restrict__ e, int n) {
    // |lambda| <= |b_{i-1}| + |b_i| with b_{-1} = b_{2n-1} = 0
    const int lane = threadIdx.x & (kWaveSize - 1);
    auto offd = [&](int i) { return (i < 0 || i > 2 * n - 2) ? 0.0 : fabs((i & 1) ? e[i >> 1] : d[i >> 1]); };
    double bmax = 0.0, gersh = 0.0;
    bool nan_in = false;
    for (int i = lane; i < 2 * n - 1; i += kWaveSize) {
        const double b = offd(i);
        nan_in |= !(b <= 1.7976931348623157e308);  // NaN or infinite
        bmax = fmax(bmax, b);
        gersh = fmax(gersh, offd(i - 1) + b);
    }
    gersh = fmax(gersh, offd(2 * n - 2));  // the last row: |b_{2n-2}| + 0
    for (int o = kWaveSize / 2; o >= 1; o >>= 1) {
        bmax = fmax(bmax, __shfl_xor(bmax, o, kWaveSize));
        gersh = fmax(gersh, __shfl_xor(gersh, o, kWaveSize));
        nan_in |= __shfl_xor((int)nan_in, o, kWaveSize) != 0;
    }
    TgkFrame f;
    f.nan_in = nan_in;
    f.zero = bmax == 0.0;
    // scaling by 2^-ex is exact for every entry that stays a normal number
    f.ex = __builtin_amdgcn_frexp_exp(bmax);
    f.bs = __builtin_amdgcn_ldexp(1.0, -f.ex);
    f.hi0 = __builtin_amdgcn_ldexp(gersh, -f.ex) * (1.0 + 4.0 * 2.220446049250313e-16);  // <= 2
    return f;
}

// Point m (0 <= m < M) of the coarse grid over (0, hi0]; the same expression in
// both kernels, so both see the same points.
__device__ __forceinline__ double grid_point(double hi0, int64_t m, int64_t M) {
    return hi0 * (double)(m + 1) / (double)M;
}

// Coarse pass: the counts at M = kCells * (lanes) grid points, from which every
// value gets the grid cell (x_{m-1}, x_m] that holds it (x_{-1} = 0), written
// into its output slot as the number m.  Lane g owns cells g*kCells ..
// g*kCells + kCells - 1 and evaluates the count at their upper ends and at the
// upper end of the cell before (counts are deterministic in x, so a point that
// two lanes evaluate has one count).  Value t (ascending index among the
// eigenvalues of T, n <= t < 2n) lies in cell m when C[m-1] <= t < C[m], with
// C[-1] = n (the n eigenvalues -sigma_i <= 0 lie below every grid point) and
// C[M-1] = 2n (every eigenvalue lies below hi0).  Those ranges cover [n, 2n)
// even where rounding makes the counts non-monotone (the first m with C[m] > t
// has C[m-1] <= t), so every slot is written; where they overlap, a value may
// get either of two cells, and both contain a point where the count passes t.
constexpr int kCells = 3;

__global__ void bb_tgk_grid(const double* __restrict__ d, const double* __restrict__ e, int n,
                            double* __restrict__ sigma, int64_t lanes) {
    const TgkFrame f = tgk_frame(d, e, n);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= lanes || f.nan_in || f.zero) return;
    const int64_t M = kCells * lanes, m0 = g * kCells;
    double x[kCells + 1];
    int cnt[kCells + 1];
#pragma unroll
    for (int q = 0; q <= kCells; ++q) x[q] = grid_point(f.hi0, m0 - 1 + q, M);  // m0 - 1 = -1: x = 0, unused
    tgk_counts_below(d, e, n, f.bs, x, cnt);
    if (m0 == 0) cnt[0] = n;
    if (m0 + kCells == M) cnt[kCells] = 2 * n;
    for (int q = 1; q <= kCells; ++q) {
        const int t0 = max(cnt[q - 1], n), t1 = min(cnt[q], 2 * n);  // a count below n: rounding near 0
        for (int t = t0; t < t1; ++t) sigma[2 * n - 1 - t] = (double)(m0 + q - 1);
    }
}

// Fine pass: a group of kSect lanes finds sigma_j -- the eigenvalue of T with
// ascending index t = 2n-1-j -- by multisection of the cell the coarse pass left
// in its slot, until the interval is below 4 eps of its upper end or 2^-60 of
// the bound.  Each lane reads and writes only its own value's slot.
__global__ void bb_tgk_bisect(const double* __restrict__ d, const double* __restrict__ e, int n,
                              double* __restrict__ sigma, int64_t grid_lanes) {
    const TgkFrame f = tgk_frame(d, e, n);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = (int)(gid / kSect), k = (int)(gid % kSect);
    if (j >= n) return;  // the kSect lanes of a value leave together
    if (f.nan_in || f.zero) {
        if (k == 0) sigma[j] = f.nan_in ? __builtin_nan("") : 0.0;
        return;
    }
    const int t = 2 * n - 1 - j;
    const int64_t M = kCells * grid_lanes;
    const int64_t m = (int64_t)sigma[j];  // written by the coarse pass, read before the group writes it
    const double eps = 2.220446049250313e-16;
    double lo = m == 0 ? 0.0 : grid_point(f.hi0, m - 1, M);
    double hi = grid_point(f.hi0, m, M);
    const double floor_width = f.hi0 * 0x1p-60;
    constexpr int kDiv = kSect * kPts + 1;
    // lo and hi are equal on the group's lanes, so the loop is uniform per group
    for (int it = 0; it < 128 && hi - lo > fmax(4.0 * eps * hi, floor_width); ++it) {
        double x[kPts];
        int cnt[kPts];
#pragma unroll
        for (int p = 0; p < kPts; ++p) x[p] = lo + (hi - lo) * (double)(k * kPts + p + 1) / (double)kDiv;
        tgk_counts_below(d, e, n, f.bs, x, cnt);
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
    // the group's lanes share a wave, which loaded the slot before this store
    if (k == 0) sigma[j] = __builtin_amdgcn_ldexp(0.5 * (lo + hi), f.ex);
}

hipError_t launch_bidiag_sigma(const double* d, const double* e, int64_t n, double* sigma, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int threads = 64;  // one wave per workgroup spreads the work over more CUs
    const int64_t glanes = n;  // coarse pass: 3n cells
    hipLaunchKernelGGL(bb_tgk_grid, dim3((unsigned)((glanes + threads - 1) / threads)), dim3(threads), 0, st, d, e,
                       (int)n, sigma, glanes);
    const int64_t lanes = n * kSect;
    hipLaunchKernelGGL(bb_tgk_bisect, dim3((unsigned)((lanes + threads - 1) / threads)), dim3(threads), 0, st, d, e,
                       (int)n, sigma, glanes);
    return hipGetLastError();
}

}  // namespace bbk
